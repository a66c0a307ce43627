"""Seeded synthetic mesh pairs for the two-mesh collision pipeline.

This module only builds inputs: vertex positions, triangle index arrays and
the run parameters of each workload.  It holds none of the method's
arithmetic (no orientation predicates, no constraints, no solves), so both
the CPU oracle and the HIP path can consume its output without sharing any
of the computation under test.

Conventions shared by every generator:
  * positions are float64 arrays of shape [nv, 3] (cast by the caller or by
    ``Pair.cast`` to the workload's storage type);
  * triangles are int32 arrays of shape [nt, 3]; on an oriented (closed)
    surface the vertex order is counter-clockwise seen from outside, so the
    right-hand normal (b - a) x (c - a) points to the front (outside);
  * ``orientation`` is one of ORIENT_B (only mesh B is oriented), ORIENT_A
    (only mesh A) or ORIENT_BOTH.

The paper's own models (the spike and sheet, the 576-vertex tori, the dummy
and its garment) are not available; the workloads below stand in for them
with the shapes of the paper's experiments (Section 6).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ORIENT_B = 0
ORIENT_A = 1
ORIENT_BOTH = 2

F32 = "f32"
F64 = "f64"


@dataclasses.dataclass
class Pair:
    """One resolve request: edge-side mesh A, face-side mesh B and parameters."""

    name: str
    pos_a: np.ndarray
    tri_a: np.ndarray
    pos_b: np.ndarray
    tri_b: np.ndarray
    orientation: int = ORIENT_B
    d: float = 1e-3
    dtype: str = F64
    tier: int = 1  # 0: FP32 filter first, 1: FP64 filter first

    def cast(self) -> "Pair":
        """Round positions to the storage type (RNE) and return self."""
        if self.dtype == F32:
            self.pos_a = np.ascontiguousarray(self.pos_a, dtype=np.float32)
            self.pos_b = np.ascontiguousarray(self.pos_b, dtype=np.float32)
        else:
            self.pos_a = np.ascontiguousarray(self.pos_a, dtype=np.float64)
            self.pos_b = np.ascontiguousarray(self.pos_b, dtype=np.float64)
        self.tri_a = np.ascontiguousarray(self.tri_a, dtype=np.int32)
        self.tri_b = np.ascontiguousarray(self.tri_b, dtype=np.int32)
        return self

    @property
    def sizes(self) -> dict:
        return {
            "nv_a": int(len(self.pos_a)), "nt_a": int(len(self.tri_a)),
            "nv_b": int(len(self.pos_b)), "nt_b": int(len(self.tri_b)),
        }


# --------------------------------------------------------------------------
# primitive surfaces
# --------------------------------------------------------------------------

def signed_volume(pos: np.ndarray, tri: np.ndarray) -> float:
    """Signed enclosed volume; positive for a closed, outward-wound mesh."""
    p = np.asarray(pos, dtype=np.float64)
    a, b, c = p[tri[:, 0]], p[tri[:, 1]], p[tri[:, 2]]
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def _orient_outward(pos: np.ndarray, tri: np.ndarray) -> np.ndarray:
    if signed_volume(pos, tri) < 0:
        tri = tri[:, [0, 2, 1]]
    return np.ascontiguousarray(tri, dtype=np.int32)


def icosphere(subdiv: int, radius: float = 1.0):
    """Subdivided icosahedron: 10*4^s+2 vertices, 20*4^s triangles, outward CCW."""
    phi = (1.0 + math.sqrt(5.0)) / 2.0
    v = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v.append((0.0, s1, s2 * phi))
            v.append((s1, s2 * phi, 0.0))
            v.append((s2 * phi, 0.0, s1))
    verts = [np.array(x) / np.linalg.norm(x) for x in v]
    # faces of the icosahedron: triples of mutually adjacent vertices
    # (adjacent = at the minimum pairwise distance)
    P = np.array(verts)
    dist = np.linalg.norm(P[:, None, :] - P[None, :, :], axis=2)
    edge_len = np.min(dist[dist > 1e-9])
    adj = np.abs(dist - edge_len) < 1e-6
    faces = []
    for i in range(12):
        for j in range(i + 1, 12):
            if not adj[i, j]:
                continue
            for k in range(j + 1, 12):
                if adj[i, k] and adj[j, k]:
                    a, b, c = P[i], P[j], P[k]
                    if np.dot(np.cross(b - a, c - a), a + b + c) < 0:
                        faces.append((i, k, j))
                    else:
                        faces.append((i, j, k))
    assert len(faces) == 20
    for _ in range(subdiv):
        cache = {}
        new_faces = []

        def mid(i, j):
            key = (min(i, j), max(i, j))
            if key not in cache:
                m = verts[i] + verts[j]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        for (a, b, c) in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        faces = new_faces
    pos = np.array(verts) * radius
    tri = np.array(faces, dtype=np.int32)
    return pos, _orient_outward(pos, tri)


def uv_sphere(n_rings: int, n_seg: int, radius: float = 1.0):
    """Latitude/longitude sphere with poles; 2*n_seg*(n_rings-1) triangles."""
    th = math.pi * np.arange(1, n_rings) / n_rings
    ph = 2.0 * math.pi * np.arange(n_seg) / n_seg
    T, PH = np.meshgrid(th, ph, indexing="ij")
    ring_pts = np.stack([radius * np.sin(T) * np.cos(PH), radius * np.sin(T) * np.sin(PH),
                         radius * np.cos(T)], axis=-1).reshape(-1, 3)
    pos = np.concatenate([[[0.0, 0.0, radius]], ring_pts, [[0.0, 0.0, -radius]]]).astype(np.float64)
    south = len(pos) - 1

    def ring(i, j):
        return 1 + (i - 1) * n_seg + (j % n_seg)

    j = np.arange(n_seg)
    north = np.stack([np.zeros(n_seg, np.int64), ring(1, j), ring(1, j + 1)], -1)
    ii, jj = np.meshgrid(np.arange(1, n_rings - 1), j, indexing="ij")
    a, b = ring(ii, jj), ring(ii, jj + 1)
    c, d = ring(ii + 1, jj), ring(ii + 1, jj + 1)
    mid = np.stack([np.stack([a, c, d], -1), np.stack([a, d, b], -1)], axis=2).reshape(-1, 3)
    southf = np.stack([np.full(n_seg, south), ring(n_rings - 1, j + 1), ring(n_rings - 1, j)], -1)
    faces = np.concatenate([north, mid, southf]).astype(np.int32)
    return pos, _orient_outward(pos, faces)


def grid_sheet(nx: int, ny: int, side: float, z: float = 0.0):
    """Flat nx-by-ny vertex grid on [-side/2, side/2]^2 at height z.

    Each cell (i, j) is split along its (i, j)-(i+1, j+1) diagonal, giving
    2*(nx-1)*(ny-1) triangles, wound counter-clockwise seen from +z.
    """
    xs = np.linspace(-side / 2, side / 2, nx)
    ys = np.linspace(-side / 2, side / 2, ny)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    pos = np.stack([X.ravel(), Y.ravel(), np.full(nx * ny, z)], axis=1)

    ii, jj = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="ij")
    a, b = ii * ny + jj, (ii + 1) * ny + jj
    c, d = (ii + 1) * ny + jj + 1, ii * ny + jj + 1
    faces = np.stack([np.stack([a, b, c], -1), np.stack([a, c, d], -1)], axis=2).reshape(-1, 3)
    return pos, faces.astype(np.int32)


def torus(nu: int, nv: int, R: float = 1.0, r: float = 0.3):
    """Torus about the z axis: nu major x nv minor segments, outward CCW."""
    i = np.arange(nu)[:, None]
    j = np.arange(nv)[None, :]
    th = 2.0 * np.pi * i / nu
    ph = 2.0 * np.pi * j / nv
    x = (R + r * np.cos(ph)) * np.cos(th)
    y = (R + r * np.cos(ph)) * np.sin(th)
    z = r * np.sin(ph) * np.ones_like(th)
    pos = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    ii, jj = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    a = ii * nv + jj
    b = ((ii + 1) % nu) * nv + jj
    c = ((ii + 1) % nu) * nv + (jj + 1) % nv
    d = ii * nv + (jj + 1) % nv
    faces = np.stack([np.stack([a, b, c], -1), np.stack([a, c, d], -1)], axis=2).reshape(-1, 3)
    return pos, _orient_outward(pos, faces.astype(np.int32))


def rot_x(deg: float) -> np.ndarray:
    t = math.radians(deg)
    c, s = math.cos(t), math.sin(t)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random proper rotation (QR of a Gaussian matrix)."""
    q, rr = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q @ np.diag(np.sign(np.diag(rr)))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def edges_of(tri: np.ndarray) -> np.ndarray:
    """Unique undirected edges (u < v), lexicographically sorted (for sizes)."""
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e = np.sort(e, axis=1)
    return np.unique(e, axis=0)


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------

def sphere_sheet(seed: int = 1, subdiv: int = 3, grid: int = 32, side: float = 2.5,
                 z: float = 0.3, sigma: float = 0.01, dtype: str = F64, tier: int = 1) -> Pair:
    """Oriented icosphere (mesh B, radius 1) pierced by a flat cloth sheet (mesh A).

    Default sizes: icosphere subdivision 3 (642 vertices, 1280 triangles) and a
    32x32 sheet of side 2.5 (1024 vertices, 1922 triangles) at z = 0.3, with
    N(0, sigma^2) jitter on every coordinate of both meshes.
    """
    rng = np.random.default_rng(seed)
    pb, tb = icosphere(subdiv, 1.0)
    pa, ta = grid_sheet(grid, grid, side, z)
    pa = pa + rng.normal(0.0, sigma, pa.shape)
    pb = pb + rng.normal(0.0, sigma, pb.shape)
    return Pair("sphere_sheet", pa, ta, pb, tb, ORIENT_B, 1e-3, dtype, tier).cast()


def linked_tori(nu: int = 128, nv: int = 64, R: float = 1.0, r: float = 0.3,
                shift: float = 1.7, dtype: str = F32, tier: int = 0) -> Pair:
    """Two oriented tori; the second is rotated 90 degrees about x, then shifted along x.

    With the defaults each torus has 8192 vertices and 16384 triangles and the
    tubes overlap to a depth of 0.3 near x = 0.7 .. 1.0.
    """
    pa, ta = torus(nu, nv, R, r)
    pb, tb = torus(nu, nv, R, r)
    pb = pb @ rot_x(90.0).T + np.array([shift, 0.0, 0.0])
    return Pair("linked_tori", pa, ta, pb, tb, ORIENT_BOTH, 1e-3, dtype, tier).cast()


def random_small_pair(seed: int, kind: str = "sphere_sheet") -> Pair:
    """Tiny randomly placed pairs (tens to a few hundred triangles) for brute-force checks."""
    rng = np.random.default_rng(seed)
    if kind == "sphere_sheet":
        pb, tb = icosphere(int(rng.integers(0, 2)), 1.0)
        n = int(rng.integers(4, 9))
        pa, ta = grid_sheet(n, n, 2.5, float(rng.uniform(-0.8, 0.8)))
        pa = pa @ random_rotation(rng).T
        pa = pa + rng.normal(0.0, 0.02, pa.shape)
        pb = pb + rng.normal(0.0, 0.02, pb.shape)
        return Pair(f"small_ss_{seed}", pa, ta, pb, tb, ORIENT_B, 1e-3, F64, 1).cast()
    nu = int(rng.integers(6, 12))
    pa, ta = torus(nu, max(3, nu // 2), 1.0, 0.3)
    pb, tb = torus(nu, max(3, nu // 2), 1.0, 0.3)
    pb = pb @ rot_x(90.0).T + np.array([float(rng.uniform(1.45, 1.75)), 0.0, 0.0])
    pa = pa + rng.normal(0.0, 0.01, pa.shape)
    pb = pb + rng.normal(0.0, 0.01, pb.shape)
    return Pair(f"small_tt_{seed}", pa, ta, pb, tb, ORIENT_BOTH, 1e-3, F32, 0).cast()


def _loguniform(rng: np.random.Generator, lo: float, hi: float) -> float:
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


def uv_sphere_f(target: float, radius: float = 1.0):
    """UV sphere with about `target` triangles (2 * n_seg * (n_rings - 1))."""
    n_rings = max(3, int(round(math.sqrt(target / 4.0))) + 1)
    n_seg = max(3, int(round(target / (2.0 * (n_rings - 1)))))
    return uv_sphere(n_rings, n_seg, radius)


def sheet_f(target: float, side: float, z: float):
    """Square sheet of the given side with about `target` triangles."""
    a = max(1, int(round(math.sqrt(target / 2.0))))
    b = max(1, int(round(target / (2.0 * a))))
    return grid_sheet(a + 1, b + 1, side, z)


def torus_f(target: float, R: float = 1.0, r: float = 0.3):
    """Torus with about `target` triangles and twice as many major as minor segments."""
    nv = max(3, int(round(math.sqrt(target / 4.0))))
    nu = max(3, int(round(target / (2.0 * nv))))
    return torus(nu, nv, R, r)


def pair_set(seed: int = 4, n: int = 256, f_lo: float = 500.0, f_hi: float = 50000.0,
             dtype: str = F32, tier: int = 0) -> list:
    """A batch of independent pairs of mixed kinds and sizes.

    Even entries are sphere-sheet pairs (UV sphere of radius 1, oriented, as
    mesh B; a square sheet of side 2.5 as mesh A in the plane at distance
    1 - depth from the sphere's centre), odd entries torus-torus pairs (both
    oriented, R = 1, r = 0.3, the second rotated 90 degrees about x and
    shifted 1.4 + depth along x).  Each mesh has a triangle count drawn
    log-uniformly from [f_lo, f_hi]; depth ~ U[0.1, 0.4]; each pair is then
    moved by one uniform random rotation and a translation ~ U[-5, 5]^3.
    Every pair draws from its own stream, SeedSequence(seed).spawn(n)[k].
    """
    pairs = []
    for k, ss in enumerate(np.random.SeedSequence(seed).spawn(n)):
        rng = np.random.default_rng(ss)
        depth = float(rng.uniform(0.1, 0.4))
        fa, fb = _loguniform(rng, f_lo, f_hi), _loguniform(rng, f_lo, f_hi)
        if k % 2 == 0:
            pb, tb = uv_sphere_f(fb)
            pa, ta = sheet_f(fa, 2.5, 1.0 - depth)
            kind, orient = "ss", ORIENT_B
        else:
            pa, ta = torus_f(fa)
            pb, tb = torus_f(fb)
            pb = pb @ rot_x(90.0).T + np.array([1.4 + depth, 0.0, 0.0])
            kind, orient = "tt", ORIENT_BOTH
        rot = random_rotation(rng)
        shift = rng.uniform(-5.0, 5.0, 3)
        pa = pa @ rot.T + shift
        pb = pb @ rot.T + shift
        pairs.append(Pair(f"set{seed}_{k}_{kind}", pa, ta, pb, tb, orient, 1e-3, dtype, tier).cast())
    return pairs


# ------------------------------------------------------------ capsule body
# 12 capsules (segment end points and radius, metres, z up): torso, pelvis
# (two spheres), neck, head, upper arms, forearms, thighs, shins.
CAPSULES = [
    ((0.0, 0.0, 0.95), (0.0, 0.0, 1.35), 0.16),
    ((0.09, 0.0, 0.92), (0.09, 0.0, 0.92), 0.14),
    ((-0.09, 0.0, 0.92), (-0.09, 0.0, 0.92), 0.14),
    ((0.0, 0.0, 1.38), (0.0, 0.0, 1.50), 0.06),
    ((0.0, 0.0, 1.58), (0.0, 0.0, 1.66), 0.11),
    ((0.20, 0.0, 1.36), (0.45, 0.0, 1.12), 0.055),
    ((-0.20, 0.0, 1.36), (-0.45, 0.0, 1.12), 0.055),
    ((0.45, 0.0, 1.12), (0.62, 0.0, 0.90), 0.045),
    ((-0.45, 0.0, 1.12), (-0.62, 0.0, 0.90), 0.045),
    ((0.10, 0.0, 0.88), (0.12, 0.0, 0.48), 0.085),
    ((-0.10, 0.0, 0.88), (-0.12, 0.0, 0.48), 0.085),
    ((0.12, 0.0, 0.48), (0.12, 0.0, 0.08), 0.06),
    ((-0.12, 0.0, 0.48), (-0.12, 0.0, 0.08), 0.06),
]


def capsule_sdf(p: np.ndarray) -> np.ndarray:
    """Signed distance to the union of CAPSULES at points p [n, 3] (negative inside)."""
    d = np.full(len(p), np.inf)
    for a, b, r in CAPSULES:
        a, b = np.asarray(a), np.asarray(b)
        ab = b - a
        L2 = float(ab @ ab)
        t = np.zeros(len(p)) if L2 == 0.0 else np.clip((p - a) @ ab / L2, 0.0, 1.0)
        d = np.minimum(d, np.linalg.norm(p - (a + t[:, None] * ab), axis=1) - r)
    return d


# Six tetrahedra per cube, all sharing the cube diagonal 0-7 (corner c = x + 2y + 4z);
# neighbouring cubes split their common faces the same way, so the surface is closed.
_KUHN = np.array([[0, 1, 3, 7], [0, 1, 5, 7], [0, 2, 3, 7], [0, 2, 6, 7], [0, 4, 5, 7], [0, 4, 6, 7]])


def marching_tetrahedra(sdf, lo, h: float, shape, level: float = 0.0):
    """Closed triangle mesh of {sdf = level} on the grid lo + h*(i, j, k), i < shape[0] ...

    ``sdf`` maps points [n, 3] to values.  Only cubes whose corner values
    straddle the level are split.  Crossing points are linear interpolants
    along tetrahedron edges (shared between neighbours by the edge's grid
    end points); triangles are wound counter-clockwise seen from outside
    (the side where sdf > level).
    """
    nx, ny, nz = shape
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    pts = np.stack([ii, jj, kk], -1).reshape(-1, 3) * h + np.asarray(lo)
    val = sdf(pts).reshape(nx, ny, nz) - level
    val[val == 0.0] = 1e-12  # no grid node exactly on the surface
    node = np.arange(nx * ny * nz).reshape(nx, ny, nz)
    c = node[:-1, :-1, :-1].ravel()
    corner_off = np.array([0, ny * nz, nz, ny * nz + nz, 1, ny * nz + 1, nz + 1, ny * nz + nz + 1])  # c = x+2y+4z
    corners = c[:, None] + corner_off[None, :]
    v = val.ravel()[corners]
    keep = (v.min(1) < 0) & (v.max(1) > 0)
    corners = corners[keep]
    tets = corners[:, _KUHN].reshape(-1, 4)
    tv = val.ravel()[tets]
    inside = tv < 0
    n_in = inside.sum(1)
    tris, ref = [], []

    def cross(u, w):  # crossing point id on grid edge (u, w)
        return np.minimum(u, w).astype(np.int64) * (nx * ny * nz) + np.maximum(u, w)

    for k in (1, 3):  # one corner separated: one triangle
        sel = n_in == k
        t, iv = tets[sel], inside[sel]
        lone = iv if k == 1 else ~iv
        a = t[lone]
        o = t[~lone].reshape(-1, 3)
        tris.append(np.stack([cross(a, o[:, 0]), cross(a, o[:, 1]), cross(a, o[:, 2])], 1))
        ref.append(np.stack([a, o[:, 0]], 1) if k == 1 else np.stack([o[:, 0], a], 1))
    sel = n_in == 2  # two and two: a quad, two triangles
    t, iv = tets[sel], inside[sel]
    i_ = t[iv].reshape(-1, 2)
    o_ = t[~iv].reshape(-1, 2)
    q = [cross(i_[:, 0], o_[:, 0]), cross(i_[:, 0], o_[:, 1]), cross(i_[:, 1], o_[:, 1]), cross(i_[:, 1], o_[:, 0])]
    tris += [np.stack([q[0], q[1], q[2]], 1), np.stack([q[0], q[2], q[3]], 1)]
    ref += [np.stack([i_[:, 0], o_[:, 0]], 1)] * 2
    tri_keys = np.concatenate(tris)
    ref = np.concatenate(ref)  # (an inside node, an outside node) of each triangle's tetrahedron
    keys, tri = np.unique(tri_keys.ravel(), return_inverse=True)
    tri = tri.reshape(-1, 3)
    u, w = keys // (nx * ny * nz), keys % (nx * ny * nz)
    fu, fw = val.ravel()[u], val.ravel()[w]
    s_ = fu / (fu - fw)
    pos = pts[u] + s_[:, None] * (pts[w] - pts[u])
    # wind counter-clockwise seen from outside
    n = np.cross(pos[tri[:, 1]] - pos[tri[:, 0]], pos[tri[:, 2]] - pos[tri[:, 0]])
    flip = np.einsum("ij,ij->i", n, pts[ref[:, 1]] - pts[ref[:, 0]]) < 0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return pos, tri.astype(np.int32)


def capsule_surface(level: float, h: float):
    """Marching-tetrahedra mesh of the capsule body's level set at grid spacing h."""
    lo = np.array([-0.75, -0.25, -0.02]) - level
    hi = np.array([0.75, 0.25, 1.80]) + level
    shape = tuple(int(x) for x in np.ceil((hi - lo) / h) + 1)
    return marching_tetrahedra(capsule_sdf, lo, h, shape, level)


def _sized_surface(level: float, target: int, h0: float):
    """capsule_surface with the grid spacing tuned to target +- 5 % triangles."""
    h = h0
    for _ in range(12):
        pos, tri = capsule_surface(level, h)
        if abs(len(tri) - target) <= 0.05 * target:
            return pos, tri
        h *= math.sqrt(len(tri) / target)
    return pos, tri


def vertex_normals(pos: np.ndarray, tri: np.ndarray) -> np.ndarray:
    """Area-weighted unit vertex normals."""
    fn = np.cross(pos[tri[:, 1]] - pos[tri[:, 0]], pos[tri[:, 2]] - pos[tri[:, 0]])
    vn = np.zeros_like(pos)
    for k in range(3):
        np.add.at(vn, tri[:, k], fn)
    return vn / np.maximum(np.linalg.norm(vn, axis=1, keepdims=True), 1e-300)


def body_garment(seed: int = 3, body_tris: int = 200000, cloth_tris: int = 100000, offset: float = 0.01,
                 frac: float = 0.05, push: float = 0.03, dtype: str = F32, tier: int = 0) -> Pair:
    """Closed oriented capsule body (mesh B) inside a cloth shell (mesh A) pushed into it.

    The body is the zero level set of the union of 12 capsules, the cloth the
    level set at `offset`, both by marching tetrahedra with grid spacings
    tuned to the triangle counts (+- 5 %).  A fraction `frac` of the cloth
    vertices (chosen with default_rng(seed)) move along minus their
    area-weighted normal by U[0, push]; those moved farther than `offset`
    penetrate the body.
    """
    rng = np.random.default_rng(seed)
    pb, tb = _sized_surface(0.0, body_tris, 0.0097 * math.sqrt(200000.0 / body_tris))
    pa, ta = _sized_surface(offset, cloth_tris, 0.0145 * math.sqrt(100000.0 / cloth_tris))
    n = vertex_normals(pa, ta)
    pick = rng.choice(len(pa), size=int(round(frac * len(pa))), replace=False)
    pa = pa.copy()
    pa[pick] -= rng.uniform(0.0, push, len(pick))[:, None] * n[pick]
    return Pair("body_garment", pa, ta, pb, tb, ORIENT_B, 1e-3, dtype, tier).cast()


def workload(name: str, **kw) -> Pair:
    if name == "sphere_sheet":
        return sphere_sheet(**kw)
    if name == "linked_tori":
        return linked_tori(**kw)
    if name == "body_garment":
        return body_garment(**kw)
    raise KeyError(name)
