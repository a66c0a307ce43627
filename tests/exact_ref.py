"""Exact rational references used to pin the oracle and the HIP predicates.

Test-only.  These restate the definitions with ``fractions.Fraction`` in a
formulation that differs from both implementations under test: the hit test
here solves for the plane crossing point and checks its barycentric
coordinates, while the oracle and the library use orientation signs only.
"""
from fractions import Fraction as Fr

import numpy as np


def fr3(p):
    return [Fr(float(v)) for v in p]


def sub(a, b):
    return [a[0] - b[0], a[1] - b[1], a[2] - b[2]]


def cross(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def orient_exact(a, b, c, p):
    """det[b-a, c-a, p-a] as an exact rational."""
    a, b, c, p = fr3(a), fr3(b), fr3(c), fr3(p)
    return dot(cross(sub(b, a), sub(c, a)), sub(p, a))


def sign(x):
    return (x > 0) - (x < 0)


def ef_hit_parametric(p, q, a, b, c):
    """0 no hit; 1 hit with p behind; 2 hit with q behind (crossing-point form).

    The segment crosses the plane strictly between its endpoints; the
    crossing point X = p + t (q - p) must lie in the closed triangle, i.e.
    all three barycentric coordinates (signed sub-areas along the normal)
    are >= 0.  A zero-area triangle never hits.
    """
    P, Q, A, B, C = fr3(p), fr3(q), fr3(a), fr3(b), fr3(c)
    N = cross(sub(B, A), sub(C, A))
    nn = dot(N, N)
    if nn == 0:
        return 0
    sp = dot(N, sub(P, A))
    sq = dot(N, sub(Q, A))
    if not ((sp < 0 < sq) or (sq < 0 < sp)):
        return 0
    t = sp / (sp - sq)
    X = [P[i] + t * (Q[i] - P[i]) for i in range(3)]
    la = dot(N, cross(sub(B, X), sub(C, X)))
    lb = dot(N, cross(sub(C, X), sub(A, X)))
    lc = dot(N, cross(sub(A, X), sub(B, X)))
    if la >= 0 and lb >= 0 and lc >= 0:
        return 1 if sp < 0 else 2
    return 0


def brute_force_hits(pos_e, edges_e, pos_f, tri_f):
    """All (edge index, face index, x0) by exact rational tests of every pair."""
    out = []
    for ei, (u, v) in enumerate(edges_e):
        p, q = pos_e[u], pos_e[v]
        lo = np.minimum(p, q)
        hi = np.maximum(p, q)
        for f, (i, j, k) in enumerate(tri_f):
            a, b, c = pos_f[i], pos_f[j], pos_f[k]
            flo = np.minimum(np.minimum(a, b), c)
            fhi = np.maximum(np.maximum(a, b), c)
            if np.any(flo > hi) or np.any(fhi < lo):
                continue
            h = ef_hit_parametric(p, q, a, b, c)
            if h:
                out.append((ei, f, int(u if h == 1 else v)))
    return np.array(out, dtype=np.int64).reshape(-1, 3)


def adversarial_points(rng, n):
    """Quadruples (a, b, c, p) built to sit on or next to degeneracies."""
    pts = []
    for i in range(n):
        kind = i % 6
        a, b, c = rng.integers(-8, 9, (3, 3)).astype(float) / 8.0
        if kind == 0:  # p exactly coplanar (integer combination on a dyadic grid)
            s, t = rng.integers(-4, 5, 2) / 4.0
            p = a + s * (b - a) + t * (c - a)
        elif kind == 1:  # coplanar, then nudged by one ulp
            s, t = rng.integers(-4, 5, 2) / 4.0
            p = a + s * (b - a) + t * (c - a)
            step = rng.choice([-1.0, 1.0], 3)
            # one ulp for nonzero coordinates; an exact zero moves to +-2^-100,
            # the inputs' domain being 0 or magnitudes in [2^-200, 2^200]
            p = np.where(p != 0, np.nextafter(p, p + step), step * 2.0 ** -100)
        elif kind == 2:  # large offset: differences lose bits in floating point
            off = rng.uniform(1e6, 1e8, 3)
            s, t = rng.integers(-4, 5, 2) / 4.0
            p = a + s * (b - a) + t * (c - a)
            a, b, c, p = a + off, b + off, c + off, p + off
            p = p + rng.choice([0.0, 1.0]) * np.spacing(p)
        elif kind == 3:  # collinear triangle (zero area)
            c = a + rng.integers(-3, 4) / 2.0 * (b - a)
            p = rng.normal(size=3)
        elif kind == 4:  # random generic
            a, b, c, p = rng.normal(size=(4, 3))
        else:  # float32-representable near-coplanar
            a, b, c = (rng.normal(size=(3, 3))).astype(np.float32).astype(float)
            s, t = rng.uniform(-1, 1, 2)
            p = (a + s * (b - a) + t * (c - a)).astype(np.float32).astype(float)
        pts.append(np.stack([a, b, c, p]))
    pts = np.array(pts)
    mag = np.abs(pts)
    assert np.all((mag == 0) | ((mag >= 2.0 ** -200) & (mag <= 2.0 ** 200)))
    return pts
