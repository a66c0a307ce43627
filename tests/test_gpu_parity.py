"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bars: hit lists and stencils bit-exact; displaced positions within
1e-6 x (bounding-box diagonal of the pair) -- the float64 oracle and the
library differ only in rounding order, so the observed error is ~1e-15
relative for float64 storage and at most one float32 ulp for float32
storage.  Multi-round comparisons run in lockstep: every round starts both
sides from the same positions, because a one-ulp difference can change a
later round's hit set legitimately.
"""
import dataclasses

import numpy as np
import pytest
import torch

import meshgen
import oracle
import paper_1409_2081_amd as hf
from tests.exact_ref import adversarial_points, orient_exact, sign
from tests.test_oracle_dcd import _cases as small_cases

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _np(t):
    return t.detach().cpu().numpy()


def _diag(pair):
    p = np.concatenate([pair.pos_a, pair.pos_b]).astype(float)
    return float(np.linalg.norm(p.max(0) - p.min(0)))


def _oracle_round0(pair, xa=None, xb=None):
    xa = pair.pos_a if xa is None else xa
    xb = pair.pos_b if xb is None else xb
    dirs = {0: [0], 1: [1], 2: [0, 1]}[pair.orientation]
    hs = []
    for d in dirs:
        h, _ = oracle.detect(xa, oracle.edges(pair.tri_a), pair.tri_a, xb, oracle.edges(pair.tri_b),
                             pair.tri_b, d, nthreads=8)
        hs.append(h)
    h = np.concatenate(hs)
    return h, oracle.stencils(h)


# ----------------------------------------------------------------- predicates

def test_orient_tiers_against_rationals(hfcr_ctx):
    rng = np.random.default_rng(1)
    pts = adversarial_points(rng, 3000)
    want = np.array([sign(orient_exact(*q)) for q in pts])
    got = {t: _np(hfcr_ctx.test_orient(_t(pts), t)) for t in (0, 1, 2)}
    bad = np.nonzero(got[2] != want)[0]
    assert len(bad) == 0, [(int(i), int(i % 6), int(want[i]), int(got[2][i]), pts[i].tolist()) for i in bad[:5]]
    # the float32 filter judges the points rounded to float32
    pts32 = pts.astype(np.float32).astype(np.float64)
    want32 = np.array([sign(orient_exact(*q)) for q in pts32])
    for t, ref in ((0, want32), (1, want)):
        ok = (got[t] == ref) | (got[t] == 2)
        assert ok.all(), (t, [(int(i), int(ref[i]), int(got[t][i])) for i in np.nonzero(~ok)[0][:5]])
        # exact zeros can never be certified by a filter
        assert np.all(np.abs(got[t][ref == 0]) != 1)
        # while generic (non-degenerate) quadruples are nearly always certified
        generic = np.arange(len(pts)) % 6 == 4
        assert (got[t][generic] != 2).mean() > 0.95
    assert (want == 0).sum() > 300


# ------------------------------------------------------------------- detect

def _detect_parity(ctx, pair, tier):
    ta, tb = _t(pair.tri_a), _t(pair.tri_b)
    g = ctx.detect(_t(pair.pos_a), ta, _t(pair.pos_b), tb, pair.orientation, tier=tier)
    h, st = _oracle_round0(pair)
    assert np.array_equal(_np(g["hits"]), h), pair.name
    assert np.array_equal(_np(g["stencils"]), st), pair.name
    return g


@pytest.mark.parametrize("pair", small_cases(), ids=lambda p: p.name)
def test_detect_small_and_degenerate(hfcr_ctx, pair):
    for tier in (0, 1):
        _detect_parity(hfcr_ctx, pair, tier)
    # the other orientation settings on the same geometry
    for orient in (meshgen.ORIENT_A, meshgen.ORIENT_BOTH):
        pair.orientation = orient
        _detect_parity(hfcr_ctx, pair, 1)


def test_detect_sphere_sheet_full_size(hfcr_ctx):
    pair = meshgen.sphere_sheet()
    g = _detect_parity(hfcr_ctx, pair, 1)
    assert g["stats"]["hits0"] > 100


def test_detect_linked_tori_full_size_both_tiers(hfcr_ctx):
    pair = meshgen.linked_tori()
    g0 = _detect_parity(hfcr_ctx, pair, 0)
    g1 = _detect_parity(hfcr_ctx, pair, 1)
    assert g0["stats"]["hits0"] > 100
    # the degenerate y = 0 plane makes some tests reach the exact tier
    assert g0["stats"]["exact_tests"] > 0 or g0["stats"]["f32_ambiguous"] > 0
    assert np.array_equal(_np(g0["hits"]), _np(g1["hits"]))


# ------------------------------------------------------------------ resolve

def _lockstep(ctx, pair, rounds, tier):
    """Run `rounds` single-round resolves, each from the same positions on both sides."""
    xa, xb = pair.pos_a.copy(), pair.pos_b.copy()
    ta, tb = _t(pair.tri_a), _t(pair.tri_b)
    L = _diag(pair)
    worst = 0.0
    rank_def = 0
    for r in range(rounds):
        g = ctx.resolve(_t(xa), ta, _t(xb), tb, pair.orientation, pair.d, max_rounds=1, round_offset=r,
                        tier=tier)
        o = oracle.resolve(xa, pair.tri_a, xb, pair.tri_b, pair.orientation, pair.d, pair.dtype,
                           max_rounds=1, nthreads=8, round_offset=r)
        assert np.array_equal(_np(g["hits"]), o["hits0"]), (pair.name, r)
        assert np.array_equal(_np(g["stencils"]), o["stencils0"]), (pair.name, r)
        assert g["stats"]["rounds"] == o["rounds"], (pair.name, r)
        assert g["stats"]["converged"] == o["converged"], (pair.name, r)
        ga, gb = _np(g["pos_a"]).astype(float), _np(g["pos_b"]).astype(float)
        err = max(np.abs(ga - o["pos_a"]).max(), np.abs(gb - o["pos_b"]).max()) / L
        worst = max(worst, err)
        assert err <= 1e-6, (pair.name, r, err)
        rank_def += g["stats"]["rank_deficient"]
        if o["converged"]:
            break
        xa, xb = _np(g["pos_a"]), _np(g["pos_b"])
    return worst, rank_def


def test_lockstep_sphere_sheet_float64(hfcr_ctx):
    # rounds 0-12 push one ring of the sheet per round; 13-17 already build
    # rank-deficient impact zones (min-norm least-squares path)
    worst, rank_def = _lockstep(hfcr_ctx, meshgen.sphere_sheet(), 18, tier=1)
    print("sphere_sheet max rel err", worst, "rank-deficient zones", rank_def)
    assert rank_def > 0


def test_largest_zone_round_matches_oracle(hfcr_ctx):
    # round 18 of the sphere-sheet pair builds one rank-deficient impact zone
    # of 4074 stencils, next to the dense solver's 4096 limit: matrix and
    # vectors in global scratch, tiled attempt, then the pivoted path
    pair = meshgen.sphere_sheet()
    pre = oracle.resolve_pair(pair, nthreads=8, max_rounds=18)
    xa, xb = pre["pos_a"], pre["pos_b"]
    g = hfcr_ctx.resolve(_t(xa), _t(pair.tri_a), _t(xb), _t(pair.tri_b), pair.orientation, pair.d, max_rounds=1,
                         round_offset=18, tier=1)
    o = oracle.resolve(xa, pair.tri_a, xb, pair.tri_b, pair.orientation, pair.d, pair.dtype, max_rounds=1,
                       nthreads=8, round_offset=18)
    assert o["per_round"][0]["max_k"] == 4074
    assert g["stats"]["max_zone"] == 4074 and g["stats"]["rank_deficient"] >= 1
    assert np.array_equal(_np(g["hits"]), o["hits0"])
    assert np.array_equal(_np(g["stencils"]), o["stencils0"])
    err = max(np.abs(_np(g["pos_a"]) - o["pos_a"]).max(), np.abs(_np(g["pos_b"]) - o["pos_b"]).max()) / _diag(pair)
    print("largest zone round: rel err", err)
    assert err <= 1e-6, err


def test_lockstep_linked_tori_float32(hfcr_ctx):
    worst, _ = _lockstep(hfcr_ctx, meshgen.linked_tori(), 12, tier=0)
    print("linked_tori max rel err", worst)


@pytest.mark.parametrize("which", ["sheet_cap", "tori_shallow", "tori_shallower", "tori_shallower_simultaneous"])
def test_full_resolve_matches_oracle(hfcr_ctx, which):
    if which == "sheet_cap":
        pair = meshgen.sphere_sheet(z=0.9)
    elif which == "tori_shallow":
        pair = meshgen.linked_tori(nu=64, nv=32, shift=1.5)
    else:
        pair = meshgen.linked_tori(nu=64, nv=32, shift=1.45)
    ta, tb = _t(pair.tri_a), _t(pair.tri_b)
    for mode in ((1,) if which.endswith("simultaneous") else (0,)):
        g = hfcr_ctx.resolve(_t(pair.pos_a), ta, _t(pair.pos_b), tb, pair.orientation, pair.d,
                             tier=pair.tier, both_mode=mode)
        o = oracle.resolve_pair(pair, nthreads=8, mode=mode, max_zone=hf.MAX_ZONE)
        assert g["status"] == hf.HFCR_OK and o["converged"]
        assert g["stats"]["rounds"] == o["rounds"]
        assert np.array_equal(_np(g["hits"]), o["hits0"])
        assert np.array_equal(_np(g["stencils"]), o["stencils0"])
        L = _diag(pair)
        err = max(np.abs(_np(g["pos_a"]).astype(float) - o["pos_a"]).max(),
                  np.abs(_np(g["pos_b"]).astype(float) - o["pos_b"]).max()) / L
        assert err <= 1e-6, err
        # termination invariant, checked by the oracle's exact DCD on the GPU result
        dirs = [0] if pair.orientation == meshgen.ORIENT_B else [0, 1]
        for dr in dirs:
            h, _ = oracle.detect(_np(g["pos_a"]), oracle.edges(pair.tri_a), pair.tri_a, _np(g["pos_b"]),
                                 oracle.edges(pair.tri_b), pair.tri_b, dr, nthreads=8)
            assert len(h) == 0


def test_zone_limit_stops_like_the_oracle(hfcr_ctx):
    # simultaneous responses on this overlap grow an impact zone beyond the
    # dense solver's limit.  From the oracle's state just before that round,
    # both sides must stop at once and leave the positions unchanged.
    pair = meshgen.linked_tori(nu=64, nv=32, shift=1.5)
    o = oracle.resolve_pair(pair, nthreads=8, mode=1, max_zone=hf.MAX_ZONE)
    assert o["status"] == "zone_limit" and o["rounds"] > 0
    xa, xb = o["pos_a"], o["pos_b"]
    g = hfcr_ctx.resolve(_t(xa), _t(pair.tri_a), _t(xb), _t(pair.tri_b), pair.orientation, pair.d, tier=0,
                         both_mode=1)
    assert g["status"] == hf.HFCR_E_ZONE_LIMIT and g["stats"]["rounds"] == 0
    assert "exceeds" in g["error"]
    np.testing.assert_array_equal(_np(g["pos_a"]), xa)
    np.testing.assert_array_equal(_np(g["pos_b"]), xb)


def test_inverse_masses_pinned_face_mesh(hfcr_ctx):
    pair = meshgen.sphere_sheet(z=0.9)
    wa = np.ones(len(pair.pos_a))
    wb = np.zeros(len(pair.pos_b))  # the sphere does not move
    g = hfcr_ctx.resolve(_t(pair.pos_a), _t(pair.tri_a), _t(pair.pos_b), _t(pair.tri_b), pair.orientation, pair.d,
                         tier=1, inv_mass_a=_t(wa), inv_mass_b=_t(wb))
    o = oracle.resolve_pair(pair, nthreads=8, inv_mass_a=wa, inv_mass_b=wb)
    assert g["stats"]["rounds"] == o["rounds"] and o["converged"]
    np.testing.assert_array_equal(_np(g["pos_b"]), pair.pos_b)
    assert np.abs(_np(g["pos_a"]) - o["pos_a"]).max() <= 1e-6 * _diag(pair)


def test_topology_reuse_does_not_change_results():
    # a context keeps the edge sets and BVH trees of its last call and reuses
    # them while the triangle arrays are unchanged; results must equal those
    # of a fresh context, also for new positions on the same triangles and
    # for orientations that need structures the last call did not build
    warm, fresh = hf.Context(0), hf.Context(0)
    base = meshgen.sphere_sheet(z=0.6)
    moved = dataclasses.replace(base, pos_a=base.pos_a + np.array([0.0, 0.0, 0.1]), pos_b=base.pos_b.copy())
    seq = [(base, meshgen.ORIENT_B), (base, meshgen.ORIENT_B), (moved, meshgen.ORIENT_B), (moved, meshgen.ORIENT_A),
           (moved, meshgen.ORIENT_BOTH), (meshgen.linked_tori(nu=32, nv=16, shift=1.5), meshgen.ORIENT_BOTH),
           (base, meshgen.ORIENT_BOTH)]
    for pair, orient in seq:
        args = (*hf.pair_tensors(pair), orient, pair.d)
        g = warm.resolve(*args, tier=1, max_rounds=4)
        f = fresh.resolve(*args, tier=1, max_rounds=4)
        fresh.close()
        fresh = hf.Context(0)
        assert g["status"] == f["status"], (pair.name, orient)
        for k in ("pos_a", "pos_b", "hits", "stencils"):
            assert torch.equal(g[k], f[k]), (pair.name, orient, k)
        for k in ("rounds", "hits0", "stencils0", "candidates", "residual_hits", "round_hits", "round_stencils"):
            assert g["stats"][k] == f["stats"][k], (pair.name, orient, k)
    warm.close()
    fresh.close()


def test_deterministic_bitwise(hfcr_ctx):
    pair = meshgen.linked_tori()
    args = (_t(pair.pos_a), _t(pair.tri_a), _t(pair.pos_b), _t(pair.tri_b), pair.orientation, pair.d)
    a = hfcr_ctx.resolve(*args, max_rounds=6, tier=0)
    b = hfcr_ctx.resolve(*args, max_rounds=6, tier=0)
    assert torch.equal(a["pos_a"], b["pos_a"]) and torch.equal(a["pos_b"], b["pos_b"])
    assert torch.equal(a["hits"], b["hits"]) and a["stats"]["round_hits"] == b["stats"]["round_hits"]


# --------------------------------------------------------------- edge cases

def test_no_intersection_and_round_cap(hfcr_ctx):
    pair = meshgen.sphere_sheet(z=3.0)
    g = hfcr_ctx.resolve(*hf.pair_tensors(pair), pair.orientation, pair.d, tier=1)
    assert g["status"] == hf.HFCR_OK and g["stats"]["rounds"] == 0 and len(g["hits"]) == 0
    np.testing.assert_array_equal(_np(g["pos_a"]), pair.pos_a)
    pair = meshgen.sphere_sheet(z=0.9)
    g = hfcr_ctx.resolve(*hf.pair_tensors(pair), pair.orientation, pair.d, tier=1, max_rounds=0)
    assert g["status"] == hf.HFCR_NOT_CONVERGED
    assert g["stats"]["residual_hits"] == g["stats"]["hits0"] > 0
    np.testing.assert_array_equal(_np(g["pos_a"]), pair.pos_a)


def test_empty_and_single_triangle_meshes(hfcr_ctx):
    pa, ta = meshgen.grid_sheet(3, 3, 1.0, 0.0)
    # a single triangle pierced by one sheet edge
    pb = np.array([[-0.3, -0.3, -0.2], [0.4, -0.3, 0.2], [-0.3, 0.4, 0.2]])
    tb = np.array([[0, 1, 2]], np.int32)
    g = hfcr_ctx.resolve(_t(pa), _t(ta), _t(pb), _t(tb), 0, 1e-3)
    o = oracle.resolve(pa, ta, pb, tb, 0, 1e-3, "f64", nthreads=2)
    assert np.array_equal(_np(g["hits"]), o["hits0"]) and g["stats"]["rounds"] == o["rounds"]
    # empty face mesh and empty edge mesh
    e3 = torch.zeros((0, 3), dtype=torch.int32, device=DEV)
    g = hfcr_ctx.resolve(_t(pa), _t(ta), _t(pb), e3, 0, 1e-3)
    assert g["status"] == hf.HFCR_OK and g["stats"]["hits0"] == 0
    g = hfcr_ctx.resolve(_t(pa), e3, _t(pb), _t(tb), 2, 1e-3)
    assert g["status"] == hf.HFCR_OK and g["stats"]["hits0"] == 0


def test_invalid_inputs_are_rejected(hfcr_ctx):
    pair = meshgen.sphere_sheet(z=0.9)
    pa = pair.pos_a.copy()
    pa[5, 1] = np.nan
    with pytest.raises(hf.HfcrError) as e:
        hfcr_ctx.resolve(_t(pa), _t(pair.tri_a), _t(pair.pos_b), _t(pair.tri_b), 0, 1e-3)
    assert e.value.status == hf.HFCR_E_INVALID
    tb = pair.tri_b.copy()
    tb[3, 2] = len(pair.pos_b)
    with pytest.raises(hf.HfcrError) as e:
        hfcr_ctx.resolve(_t(pair.pos_a), _t(pair.tri_a), _t(pair.pos_b), _t(tb), 0, 1e-3)
    assert e.value.status == hf.HFCR_E_INVALID
    pa = pair.pos_a.copy()
    pa[0, 0] = 1e-250  # outside the exact predicates' domain
    with pytest.raises(hf.HfcrError) as e:
        hfcr_ctx.resolve(_t(pa), _t(pair.tri_a), _t(pair.pos_b), _t(pair.tri_b), 0, 1e-3)
    assert e.value.status == hf.HFCR_E_INVALID
    # the context stays usable after errors
    g = hfcr_ctx.resolve(*hf.pair_tensors(pair), 0, 1e-3, tier=1)
    assert g["status"] == hf.HFCR_OK
