"""Pins of the oracle's response (Section 4, Eq. 1 - Eq. 8).

* the single-constraint closed form, against hand-worked fractions in
  tests/golden/single_stencil.json;
* the multi-constraint minimiser, against its defining properties: every
  constraint met (Eq. 8), displacement in the range of M^-1 grad(D)^T
  (Eq. 5), no feasible perturbation is shorter in the M-norm (Eq. 3), one
  global solve equals the per-zone solves, uniform mass scaling changes
  nothing, and rank-deficient systems give the pseudo-inverse solution.
"""
import json
import os
from fractions import Fraction as Fr

import numpy as np
import pytest

import meshgen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "single_stencil.json")


def _f(v):
    return float(Fr(v))


@pytest.mark.parametrize("case", json.load(open(GOLDEN))["cases"], ids=lambda c: c["name"])
def test_single_stencil_closed_form(case):
    x0 = np.array([[_f(v) for v in case["x0"]]])
    face = np.array([[_f(v) for v in p] for p in case["face"]])
    w = [_f(v) for v in case["inv_mass"]]
    d = _f(case["d"])
    # mesh A holds x0 (edge side), mesh B the face (oriented)
    ta = np.zeros((0, 3), np.int32)
    tb = np.array([[0, 1, 2]], np.int32)
    st = np.array([[0, 0, 0]], np.int32)
    con = oracle.constraints(st, x0, ta, face, tb, d)
    assert con["D"][0] == pytest.approx(_f(case["D"]), abs=1e-15)
    xa, xb, info = oracle.respond(x0, face, ta, tb, st, d, wa=np.array(w[:1]), wb=np.array(w[1:]))
    assert info["lambda"][0] == pytest.approx(_f(case["lambda"]), abs=1e-15)
    np.testing.assert_allclose(xa[0], [_f(v) for v in case["x0_after"]], atol=1e-15)
    np.testing.assert_allclose(xb, [[_f(v) for v in p] for p in case["face_after"]], atol=1e-15)
    # post-response signed distance equals d and the normal is unchanged
    con2 = oracle.constraints(st, xa, ta, xb, tb, d)
    assert con2["D"][0] == pytest.approx(d, abs=1e-14)
    np.testing.assert_allclose(con2["n"], con["n"], atol=1e-15)


def _round0(pair):
    xa, xb = pair.pos_a.astype(float), pair.pos_b.astype(float)
    h, _ = oracle.detect(xa, oracle.edges(pair.tri_a), pair.tri_a, xb, oracle.edges(pair.tri_b), pair.tri_b, 0)
    return xa, xb, oracle.stencils(h)


def _global_gradient(con, nvt):
    S = len(con["verts"])
    G = np.zeros((S, 3 * nvt))
    for i in range(S):
        for s in range(4):
            v = con["verts"][i, s]
            G[i, 3 * v:3 * v + 3] += oracle.COEF[s] * con["n"][i]
    return G


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_multi_constraint_properties(seed):
    pair = meshgen.random_small_pair(seed, "sphere_sheet")
    xa, xb, st = _round0(pair)
    assert len(st) > 3
    d = 1e-3
    rng = np.random.default_rng(seed)
    wa = rng.uniform(0.5, 2.0, len(xa))
    wb = rng.uniform(0.5, 2.0, len(xb))
    xa2, xb2, info = oracle.respond(xa, xb, pair.tri_a, pair.tri_b, st, d, wa, wb)
    con = info["con"]
    X, X2 = np.concatenate([xa, xb]).ravel(), np.concatenate([xa2, xb2]).ravel()
    G = _global_gradient(con, len(xa) + len(xb))
    W = np.repeat(np.concatenate([wa, wb]), 3)
    assert info["rank_cut"] == 0
    # Eq. 8: grad(D) x' = d (linearised constraint with the pre-response normals)
    lin = G @ X2 - (G @ X - con["D"])  # grad(D) x' = D(x) + grad(D)(x' - x)
    np.testing.assert_allclose(lin, d, atol=1e-12)
    # Eq. 5: x' - x = -W grad(D)^T lambda
    np.testing.assert_allclose(X2 - X, -W * (G.T @ info["lambda"]), atol=1e-13)
    # Eq. 3: any feasible perturbation z (G z = 0) is no shorter in the M-norm
    _, sv, vt = np.linalg.svd(G)
    null = vt[len(sv):]
    base = np.sum((X2 - X) ** 2 / W)
    for _ in range(20):
        z = null.T @ rng.normal(size=null.shape[0]) * 1e-2
        assert np.sum((X2 + z - X) ** 2 / W) >= base - 1e-15
    # one global solve == per-zone solves (A is block diagonal over zones)
    A = G @ (W[:, None] * G.T)
    lam = np.linalg.solve(A, con["r"])
    np.testing.assert_allclose(X - W * (G.T @ lam), X2, atol=1e-12)
    # uniform mass scaling leaves x' unchanged
    xa3, xb3, _ = oracle.respond(xa, xb, pair.tri_a, pair.tri_b, st, d, 3.0 * wa, 3.0 * wb)
    np.testing.assert_allclose(np.concatenate([xa3, xb3]), np.concatenate([xa2, xb2]), atol=1e-12)


def _fan(k=6):
    """A flat fan of k triangles around vertex 0 in the plane z = 0 (front +z)."""
    ang = 2 * np.pi * np.arange(k) / k
    ring = np.stack([np.cos(ang), np.sin(ang), np.zeros(k)], axis=1)
    pos = np.concatenate([[[0.0, 0.0, 0.0]], ring])
    tri = np.array([[0, 1 + i, 1 + (i + 1) % k] for i in range(k)], np.int32)
    return pos, tri


def test_rank_deficient_matches_pseudo_inverse():
    # one vertex behind all six coplanar fan faces: the rows are dependent
    # (alternating multipliers around the fan cancel), so A is singular.
    fpos, ftri = _fan(6)
    x0 = np.array([[0.1, 0.05, -0.2]])
    st = np.array([[0, 0, f] for f in range(6)], np.int32)
    ta = np.zeros((0, 3), np.int32)
    d = 1e-3
    xa2, xb2, info = oracle.respond(x0, fpos, ta, ftri, st, d)
    assert info["rank_cut"] >= 1
    con = info["con"]
    G = _global_gradient(con, 1 + len(fpos))
    X = np.concatenate([x0, fpos]).ravel()
    lam = np.linalg.pinv(G @ G.T, rcond=1e-10) @ con["r"]
    np.testing.assert_allclose(np.concatenate([xa2, xb2]).ravel(), X - G.T @ lam, atol=1e-12)


def test_more_constraints_than_coordinates_uses_same_solution():
    # every inner vertex against every face of an octahedron: k = 40 > 3m = 33,
    # which takes the smaller Gram-matrix path; compare with the literal A-form.
    fpos = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    ftri = np.array([[0, 2, 4], [2, 1, 4], [1, 3, 4], [3, 0, 4], [2, 0, 5], [1, 2, 5], [3, 1, 5], [0, 3, 5]],
                    np.int32)
    assert meshgen.signed_volume(fpos, ftri) > 0
    rng = np.random.default_rng(9)
    xa = rng.uniform(-0.2, 0.2, (5, 3))
    st = np.array([[0, v, f] for v in range(5) for f in range(8)], np.int32)
    ta = np.zeros((0, 3), np.int32)
    wa, wb = rng.uniform(0.5, 2, 5), rng.uniform(0.5, 2, 6)
    xa2, xb2, info = oracle.respond(xa, fpos, ta, ftri, st, 1e-3, wa, wb)
    con = info["con"]
    G = _global_gradient(con, 11)
    W = np.repeat(np.concatenate([wa, wb]), 3)
    A = G @ (W[:, None] * G.T)
    mu, V = np.linalg.eigh(A)
    keep = mu > 1e-12 * mu.max()
    lam = V[:, keep] @ ((V[:, keep].T @ con["r"]) / mu[keep])
    X = np.concatenate([xa, fpos]).ravel()
    np.testing.assert_allclose(np.concatenate([xa2, xb2]).ravel(), X - W * (G.T @ lam), atol=1e-12)


def test_impact_zones_transitive():
    verts = np.array([[0, 10, 11, 12], [1, 12, 13, 14], [2, 20, 21, 22], [3, 14, 30, 31], [4, 40, 41, 42],
                      [2, 40, 50, 51]])
    zones = oracle.impact_zones(verts)
    assert [z.tolist() for z in zones] == [[0, 1, 3], [2, 4, 5]]


def test_resolve_shallow_pairs_converge_and_leave_no_hit():
    for pair in (meshgen.sphere_sheet(z=0.9), meshgen.linked_tori(nu=32, nv=16, shift=1.45)):
        r = oracle.resolve_pair(pair, nthreads=4)
        assert r["converged"] and r["residual"] == 0 and r["rounds"] >= 1
        assert len(r["hits0"]) > 0
        # termination invariant: the exact DCD finds nothing in the oriented directions
        ta, tb = pair.tri_a, pair.tri_b
        dirs = [0] if pair.orientation == meshgen.ORIENT_B else [0, 1]
        for dr in dirs:
            h, _ = oracle.detect(r["pos_a"], oracle.edges(ta), ta, r["pos_b"], oracle.edges(tb), tb, dr)
            assert len(h) == 0


def test_resolve_round_cap_reports_residual():
    pair = meshgen.sphere_sheet(z=0.9)
    r = oracle.resolve_pair(pair, max_rounds=0)
    assert not r["converged"] and r["rounds"] == 0
    assert r["residual"] == len(r["hits0"]) > 0
    np.testing.assert_array_equal(r["pos_a"], pair.pos_a)


def test_float32_storage_is_rounded_each_round():
    pair = meshgen.linked_tori(nu=32, nv=16, shift=1.45)
    r = oracle.resolve_pair(pair, nthreads=4, max_rounds=2)
    assert r["pos_a"].dtype == np.float32
    xa, xb = pair.pos_a.astype(float), pair.pos_b.astype(float)
    h, _ = oracle.detect(xa, oracle.edges(pair.tri_a), pair.tri_a, xb, oracle.edges(pair.tri_b), pair.tri_b, 0)
    xa1, xb1, _ = oracle.respond(xa, xb, pair.tri_a, pair.tri_b, oracle.stencils(h), pair.d)
    rec = oracle.resolve_pair(pair, nthreads=4, max_rounds=1, record=True)
    np.testing.assert_array_equal(rec["pos_a"], xa1.astype(np.float32))
    np.testing.assert_array_equal(rec["pos_b"], xb1.astype(np.float32))
