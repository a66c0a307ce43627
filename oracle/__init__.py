"""CPU oracle for the history-free two-mesh collision pipeline.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plainly written
reference that the HIP library is checked against.  It shares no code with
``paper_1409_2081_amd`` (no kernels, headers, helpers or tables) and the
library never imports it; only ``tests/``, the smoke check and the
benchmark's CPU-baseline leg may call it.

It follows J. Ye, "History-free Collision Response for Deformable Surfaces"
(arXiv 1409.2081):

  * DCD (Sections 1 and 3): every E-F intersection between the edges of one
    mesh and the triangles of the other (the exact test lives in
    ``hfcr_oracle.c``);
  * penetration stencils (Section 4, Fig. 3): the back-side endpoint x0 of an
    intersecting edge plus the three vertices of the oriented face, with
    duplicates merged and no stencil for an un-oriented face;
  * constraints (Eq. 1, Eq. 2): D = n . [x0 - (x1 + x2 + x3)/3] with the unit
    face normal n, gradient (n, -n/3, -n/3, -n/3);
  * impact zones (Section 4, "Implementation"): stencils that share a vertex,
    closed transitively; one system per zone;
  * minimizer (Eq. 3 - Eq. 8): x' = x - M^-1 grad(D)^T lambda with
    grad(D) M^-1 grad(D)^T lambda = grad(D) x - d;
  * repair loop (Section 3): detect, relocate, repeat until no E-F
    intersection remains.

Readings of points the paper leaves open:
  * the normal n is unit length, so D is a signed distance and d a distance;
  * orientation is given by winding: counter-clockwise (right-hand) = front;
  * when both meshes are oriented the roles alternate between rounds: round r
    treats mesh B's faces as the oriented ones when r is even and mesh A's
    when r is odd; if that direction has no hit the other one is used, and
    the loop ends when neither has one;
  * lambda is not clamped to be non-negative (the paper relaxes the sign);
  * a singular zone system is solved in the least-squares minimum-norm sense
    (pseudo-inverse with relative eigenvalue cut 1e-12); x' does not depend
    on the choice among least-squares solutions;
  * normals are recomputed from each round's positions; float32 storage is
    rounded to nearest after every round;
  * the diffusion of displacements (Section 5) is not part of this path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import scipy.sparse as sp

from . import build as _build

ORIENT_B = 0
ORIENT_A = 1
ORIENT_BOTH = 2
MODE_ALTERNATE = 0
MODE_SIMULTANEOUS = 1

_LIB = None


def lib():
    """Load the oracle's C part, compiling it first if it is not built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        lp = ctypes.POINTER(ctypes.c_int64)
        for name in ("ora_orient_sign", "ora_orient_sign_exact"):
            f = getattr(L, name)
            f.argtypes = [dp, dp, dp, dp]
            f.restype = ctypes.c_int
        L.ora_ef_hit.argtypes = [dp, dp, dp, dp, dp]
        L.ora_ef_hit.restype = ctypes.c_int
        L.ora_dcd.argtypes = [dp, ip, ctypes.c_int64, dp, ip, ctypes.c_int64,
                              ip, ctypes.c_int64, lp, ctypes.c_int]
        L.ora_dcd.restype = ctypes.c_int64
        L.ora_dcd_edges.argtypes = [dp, ip, lp, ctypes.c_int64, dp, ip, ctypes.c_int64,
                                    ip, ctypes.c_int64, lp, ctypes.c_int]
        L.ora_dcd_edges.restype = ctypes.c_int64
        L.ora_max_threads.argtypes = []
        L.ora_max_threads.restype = ctypes.c_int
        _LIB = L
    return _LIB


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _lptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _vec(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3))


# --------------------------------------------------------------- predicates

def orient_sign(a, b, c, p) -> int:
    """Exact sign of det[b-a, c-a, p-a] (+1: p on the front side of CCW (a,b,c))."""
    a, b, c, p = map(_vec, (a, b, c, p))
    return lib().ora_orient_sign(_dptr(a), _dptr(b), _dptr(c), _dptr(p))


def orient_sign_exact(a, b, c, p) -> int:
    """Same sign, always through the exact expansion (no floating-point filter)."""
    a, b, c, p = map(_vec, (a, b, c, p))
    return lib().ora_orient_sign_exact(_dptr(a), _dptr(b), _dptr(c), _dptr(p))


def ef_hit(p, q, a, b, c) -> int:
    """0: no hit; 1: edge pq crosses triangle abc with p behind; 2: with q behind."""
    p, q, a, b, c = map(_vec, (p, q, a, b, c))
    return lib().ora_ef_hit(_dptr(p), _dptr(q), _dptr(a), _dptr(b), _dptr(c))


# --------------------------------------------------------------------- DCD

def edges(tri) -> np.ndarray:
    """Unique undirected edges {u, v}, u < v, of a triangle mesh, sorted."""
    tri = np.asarray(tri, dtype=np.int64).reshape(-1, 3)
    if len(tri) == 0:
        return np.zeros((0, 2), dtype=np.int32)
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e = np.sort(e, axis=1)
    e = e[e[:, 0] != e[:, 1]]
    return np.unique(e, axis=0).astype(np.int32)


def dcd(pos_e, edges_e, pos_f, tri_f, nthreads: int = 1, edge_ids=None):
    """All E-F hits of the edges of one mesh against the faces of the other.

    Returns (hits [H,3] int32 of (edge index, face index, x0), candidate count)
    in (edge, face) order.  With ``edge_ids`` only those edges are tested.
    """
    pe = np.ascontiguousarray(pos_e, dtype=np.float64).reshape(-1, 3)
    pf = np.ascontiguousarray(pos_f, dtype=np.float64).reshape(-1, 3)
    ee = np.ascontiguousarray(edges_e, dtype=np.int32).reshape(-1, 2)
    tf = np.ascontiguousarray(tri_f, dtype=np.int32).reshape(-1, 3)
    L = lib()
    cap = 1024
    while True:
        out = np.zeros((cap, 3), dtype=np.int32)
        cand = np.zeros(1, dtype=np.int64)
        if edge_ids is None:
            n = L.ora_dcd(_dptr(pe), _iptr(ee), len(ee), _dptr(pf), _iptr(tf), len(tf),
                          _iptr(out), cap, _lptr(cand), int(nthreads))
        else:
            ids = np.ascontiguousarray(edge_ids, dtype=np.int64)
            n = L.ora_dcd_edges(_dptr(pe), _iptr(ee), _lptr(ids), len(ids), _dptr(pf),
                                _iptr(tf), len(tf), _iptr(out), cap, _lptr(cand), int(nthreads))
        if n <= cap:
            return out[:n].copy(), int(cand[0])
        cap = int(n)


def _sort_rows(a: np.ndarray) -> np.ndarray:
    if len(a) == 0:
        return a
    order = np.lexsort(a.T[::-1])
    return a[order]


def detect(xa, ea, ta, xb, eb, tb, direction: int, nthreads: int = 1):
    """Hit records (dir, u, v, f, x0) for one direction, sorted.

    direction 0: edges of mesh A against the faces of mesh B (B oriented);
    direction 1: edges of mesh B against the faces of mesh A (A oriented).
    Vertex and face indices are local to their own mesh.
    """
    if direction == 0:
        h, cand = dcd(xa, ea, xb, tb, nthreads)
        e = ea
    else:
        h, cand = dcd(xb, eb, xa, ta, nthreads)
        e = eb
    rec = np.zeros((len(h), 5), dtype=np.int32)
    rec[:, 0] = direction
    rec[:, 1:3] = e[h[:, 0]] if len(h) else np.zeros((0, 2), np.int32)
    rec[:, 3] = h[:, 1]
    rec[:, 4] = h[:, 2]
    return _sort_rows(rec), cand


# ---------------------------------------------------------------- stencils

def stencils(hits: np.ndarray) -> np.ndarray:
    """Unique penetration stencils (dir, x0, f), sorted (Section 4, Fig. 3).

    Two E-F hits with the same back-side vertex and the same oriented face
    give the same stencil and are merged.
    """
    hits = np.asarray(hits, dtype=np.int32).reshape(-1, 5)
    if len(hits) == 0:
        return np.zeros((0, 3), dtype=np.int32)
    st = hits[:, [0, 4, 3]]
    return np.unique(st, axis=0).astype(np.int32)


def constraints(st, xa, ta, xb, tb, d):
    """Per stencil: global vertex ids (x0, x1, x2, x3), unit normal n, D and r = D - d.

    Eq. 1: D = n . [x0 - (x1 + x2 + x3)/3], n the unit normal of the face
    (x1, x2, x3) taken in index order; Eq. 8: right-hand side D - d.
    Global ids: mesh A's vertices first, then mesh B's (offset by |V_A|).
    """
    st = np.asarray(st, dtype=np.int64).reshape(-1, 3)
    na = len(xa)
    S = len(st)
    verts = np.zeros((S, 4), dtype=np.int64)
    P = np.zeros((S, 4, 3))
    for i, (dr, x0, f) in enumerate(st):
        if dr == 0:
            face = tb[f].astype(np.int64)
            verts[i] = [x0, na + face[0], na + face[1], na + face[2]]
            P[i, 0] = xa[x0]
            P[i, 1:] = xb[face]
        else:
            face = ta[f].astype(np.int64)
            verts[i] = [na + x0, face[0], face[1], face[2]]
            P[i, 0] = xb[x0]
            P[i, 1:] = xa[face]
    cr = np.cross(P[:, 2] - P[:, 1], P[:, 3] - P[:, 1])
    ln = np.linalg.norm(cr, axis=1)
    n = np.divide(cr, ln[:, None], out=np.zeros_like(cr), where=ln[:, None] > 0)
    centroid = (P[:, 1] + P[:, 2] + P[:, 3]) / 3.0
    D = np.einsum("ij,ij->i", n, P[:, 0] - centroid)
    return {"verts": verts, "n": n, "D": D, "r": D - d}


COEF = np.array([1.0, -1.0 / 3.0, -1.0 / 3.0, -1.0 / 3.0])  # Eq. 2, alpha = 1/3


def impact_zones(verts: np.ndarray):
    """Connected components of stencils that share at least one vertex.

    Returns a list of index arrays (ascending), ordered by their first index.
    """
    S = len(verts)
    parent = list(range(S))

    def find(i):
        while parent[i] != i:
            parent[i] = parent[parent[i]]
            i = parent[i]
        return i

    owner = {}
    for i in range(S):
        for v in verts[i]:
            v = int(v)
            if v in owner:
                ri, rj = find(i), find(owner[v])
                if ri != rj:
                    parent[max(ri, rj)] = min(ri, rj)
            else:
                owner[v] = i
    groups = {}
    for i in range(S):
        groups.setdefault(find(i), []).append(i)
    zones = [np.array(g, dtype=np.int64) for g in groups.values()]
    zones.sort(key=lambda z: int(z[0]))
    return zones


def zone_system(idx, verts, n, w):
    """The zone's gradient G (rows grad D_i over the zone's vertices) and A = G W G^T."""
    zv = np.unique(verts[idx].ravel())
    col = {int(v): j for j, v in enumerate(zv)}
    rows, cols, vals = [], [], []
    for li, i in enumerate(idx):
        for s in range(4):
            j = col[int(verts[i, s])]
            for k in range(3):
                rows.append(li)
                cols.append(3 * j + k)
                vals.append(COEF[s] * n[i, k])
    G = sp.csr_matrix((vals, (rows, cols)), shape=(len(idx), 3 * len(zv)))
    wdiag = sp.diags(np.repeat(w[zv], 3))
    A = (G @ wdiag @ G.T).toarray()
    return zv, G, wdiag, A


def solve_min_norm(A, r, rcut: float = 1e-12):
    """lambda = A^+ r via the symmetric eigendecomposition, relative cut rcut."""
    mu, V = np.linalg.eigh(A)
    top = float(np.max(np.abs(mu))) if len(mu) else 0.0
    keep = mu > rcut * top if top > 0 else np.zeros_like(mu, dtype=bool)
    inv = np.zeros_like(mu)
    inv[keep] = 1.0 / mu[keep]
    lam = V @ (inv * (V.T @ r))
    return lam, int(np.count_nonzero(~keep))


class ZoneLimit(Exception):
    """An impact zone larger than the caller's limit (no position was changed)."""


def respond(xa, xb, ta, tb, st, d, wa=None, wb=None, max_zone=None):
    """One response: relocate the stencil vertices (Eq. 3 - Eq. 8), per impact zone.

    Returns (new xa, new xb, info) with positions in float64 (no storage rounding).
    Raises ZoneLimit, before moving anything, if a zone has more than
    ``max_zone`` stencils.
    """
    xa = np.array(xa, dtype=np.float64)
    xb = np.array(xb, dtype=np.float64)
    na = len(xa)
    w = np.concatenate([np.ones(na) if wa is None else np.asarray(wa, dtype=np.float64),
                        np.ones(len(xb)) if wb is None else np.asarray(wb, dtype=np.float64)])
    con = constraints(st, xa, ta, xb, tb, d)
    X = np.concatenate([xa, xb])
    Xn = X.copy()
    zones = impact_zones(con["verts"])
    if max_zone is not None and max(len(z) for z in zones) > max_zone:
        raise ZoneLimit(max(len(z) for z in zones))
    lam_all = np.full(len(st), np.nan)
    n_cut = 0
    for idx in zones:
        zv, G, wdiag, A = zone_system(idx, con["verts"], con["n"], w)
        r = con["r"][idx]
        if len(idx) <= 3 * len(zv):
            lam, cut = solve_min_norm(A, r)
            lam_all[idx] = lam
            dx = -(wdiag @ (G.T @ lam))  # Eq. 5: x' = x - M^-1 grad(D)^T lambda
        else:
            # More constraints than coordinates: the same displacement through
            # the smaller Gram matrix.  With B = G W^1/2 (so A = B B^T),
            # W G^T A^+ r = W^1/2 B^+ r and B^+ = (B^T B)^+ B^T; B^T B has the
            # same nonzero eigenvalues as A, so the same relative cut applies.
            B = G @ wdiag.sqrt()
            y, cut = solve_min_norm((B.T @ B).toarray(), B.T @ r)
            dx = -(wdiag.sqrt() @ y)
        n_cut += cut
        Xn[zv] = X[zv] + dx.reshape(-1, 3)
    info = {"zones": len(zones), "max_k": max((len(z) for z in zones), default=0),
            "lambda": lam_all, "rank_cut": n_cut, "con": con}
    return Xn[:na], Xn[na:], info


# ------------------------------------------------------------------- loop

def resolve(pos_a, tri_a, pos_b, tri_b, orientation: int = ORIENT_B, d: float = 1e-3,
            dtype: str = "f64", max_rounds: int = 256, mode: int = MODE_ALTERNATE,
            inv_mass_a=None, inv_mass_b=None, nthreads: int = 1, record: bool = False,
            round_offset: int = 0, max_zone: int | None = None):
    """The repair loop of Section 3: detect, relocate, repeat until no E-F hit.

    ``round_offset`` shifts the round numbering that decides, when both meshes
    are oriented, which one plays the oriented role first (round r uses mesh
    B's faces when r + round_offset is even).  With ``max_zone``, a round whose
    largest impact zone exceeds it ends the loop (status "zone_limit") with
    the positions from before that round.

    At most ``max_rounds`` responses are made; the loop then reports
    ``converged = False`` with the residual hit count.  Returns a dict with
    the final positions (storage dtype), the round-0 hit list and stencils
    over every oriented direction, and per-round counts.
    """
    ta = np.asarray(tri_a, dtype=np.int32).reshape(-1, 3)
    tb = np.asarray(tri_b, dtype=np.int32).reshape(-1, 3)
    ea, eb = edges(ta), edges(tb)
    xa = np.array(pos_a, dtype=np.float64).reshape(-1, 3)
    xb = np.array(pos_b, dtype=np.float64).reshape(-1, 3)
    oriented = {ORIENT_B: [0], ORIENT_A: [1], ORIENT_BOTH: [0, 1]}[orientation]
    cand_total = 0
    rounds = []
    hits0 = np.zeros((0, 5), np.int32)
    converged = False
    status = "not_converged"
    residual_now = 0
    r = 0

    def det(direction):
        nonlocal cand_total
        h, c = detect(xa, ea, ta, xb, eb, tb, direction, nthreads)
        cand_total += c
        return h

    for r in range(max_rounds + 1):
        if orientation == ORIENT_BOTH and mode == MODE_ALTERNATE:
            first = (r + round_offset) % 2
            h1 = det(first)
            h2 = det(1 - first) if (r == 0 or len(h1) == 0) else np.zeros((0, 5), np.int32)
            if r == 0:
                hits0 = _sort_rows(np.concatenate([h1, h2]))
            active = h1 if len(h1) else h2
        else:
            hs = [det(dr) for dr in oriented]
            active = _sort_rows(np.concatenate(hs))
            if r == 0:
                hits0 = active
        if len(active) == 0:
            converged = True
            break
        if r == max_rounds:
            # residual over every oriented direction, reusing this round's detections
            if orientation == ORIENT_BOTH and mode == MODE_ALTERNATE:
                residual_now = len(h1) + (len(h2) if (r == 0 or len(h1) == 0) else len(det(1 - first)))
            else:
                residual_now = len(active)
            break
        st = stencils(active)
        try:
            xa_new, xb_new, info = respond(xa, xb, ta, tb, st, d, inv_mass_a, inv_mass_b, max_zone)
        except ZoneLimit:
            status = "zone_limit"
            break
        if dtype == "f32":
            xa_new = xa_new.astype(np.float32).astype(np.float64)
            xb_new = xb_new.astype(np.float32).astype(np.float64)
        rec = {"dir": int(active[0, 0]) if len(np.unique(active[:, 0])) == 1 else -1,
               "hits": len(active), "stencils": len(st), "zones": info["zones"],
               "max_k": info["max_k"], "rank_cut": info["rank_cut"]}
        if record:
            rec["active"] = active
            rec["stencil_list"] = st
            rec["x_before"] = (xa, xb)
            rec["x_after"] = (xa_new, xb_new)
        rounds.append(rec)
        xa, xb = xa_new, xb_new
    residual = 0
    if converged:
        status = "ok"
    elif status != "zone_limit":
        residual = residual_now
    out_t = np.float32 if dtype == "f32" else np.float64
    return {
        "pos_a": xa.astype(out_t), "pos_b": xb.astype(out_t),
        "hits0": hits0, "stencils0": stencils(hits0),
        "rounds": len(rounds), "converged": converged, "residual": residual, "status": status,
        "per_round": rounds, "candidates": cand_total,
    }


def resolve_pair(pair, **kw):
    """``resolve`` on a ``meshgen.Pair``."""
    return resolve(pair.pos_a, pair.tri_a, pair.pos_b, pair.tri_b, pair.orientation,
                   pair.d, pair.dtype, **kw)
