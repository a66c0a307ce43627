"""Pins of the oracle's DCD: brute force with exact rationals, relabelling,
and the expected size of a known configuration."""
import numpy as np
import pytest

import meshgen
import oracle
from tests.exact_ref import brute_force_hits


def _snap(pair, step):
    pair.pos_a = np.round(pair.pos_a / step) * step
    pair.pos_b = np.round(pair.pos_b / step) * step
    return pair


def _cases():
    out = []
    for s in range(4):
        out.append(meshgen.random_small_pair(s, "sphere_sheet"))
    for s in range(2):
        out.append(meshgen.random_small_pair(10 + s, "tori"))
    # snapped to a coarse dyadic grid: many exact coplanarities and
    # crossings through triangle edges and vertices
    out.append(_snap(meshgen.random_small_pair(20, "sphere_sheet"), 0.125))
    out.append(_snap(meshgen.random_small_pair(21, "sphere_sheet"), 0.25))
    return out


@pytest.mark.parametrize("pair", _cases(), ids=lambda p: p.name)
def test_dcd_equals_exact_brute_force(pair):
    xa, xb = pair.pos_a.astype(float), pair.pos_b.astype(float)
    ea, eb = oracle.edges(pair.tri_a), oracle.edges(pair.tri_b)
    for direction in (0, 1):
        if direction == 0:
            got, _ = oracle.dcd(xa, ea, xb, pair.tri_b)
            want = brute_force_hits(xa, ea, xb, pair.tri_b)
        else:
            got, _ = oracle.dcd(xb, eb, xa, pair.tri_a)
            want = brute_force_hits(xb, eb, xa, pair.tri_a)
        assert np.array_equal(got.astype(np.int64), want), (pair.name, direction)


def test_edges_definition():
    tri = np.array([[0, 1, 2], [2, 1, 3], [3, 3, 4]], dtype=np.int32)
    e = oracle.edges(tri)
    assert e.tolist() == [[0, 1], [0, 2], [1, 2], [1, 3], [2, 3], [3, 4]]


def test_relabel_invariance():
    pair = meshgen.random_small_pair(3, "sphere_sheet")
    rng = np.random.default_rng(5)
    xa, xb = pair.pos_a.astype(float), pair.pos_b.astype(float)
    ta, tb = pair.tri_a, pair.tri_b
    h0, _ = oracle.detect(xa, oracle.edges(ta), ta, xb, oracle.edges(tb), tb, 0)
    # permute vertices and faces of both meshes, rotate each triangle's indices
    pa, pb = rng.permutation(len(xa)), rng.permutation(len(xb))
    ia, ib = np.argsort(pa), np.argsort(pb)  # new index of old vertex v is ia[v]
    fa, fb = rng.permutation(len(ta)), rng.permutation(len(tb))
    ta2 = np.roll(ia[ta[fa]], 1, axis=1).astype(np.int32)
    tb2 = np.roll(ib[tb[fb]], 2, axis=1).astype(np.int32)
    xa2, xb2 = xa[pa], xb[pb]
    h1, _ = oracle.detect(xa2, oracle.edges(ta2), ta2, xb2, oracle.edges(tb2), tb2, 0)
    inv_fb = np.argsort(fb)
    mapped = []
    for d, u, v, f, x0 in h0:
        uu, vv = sorted((ia[u], ia[v]))
        mapped.append((d, uu, vv, inv_fb[f], ia[x0]))
    mapped = np.array(sorted(mapped))
    assert len(h0) > 0
    assert np.array_equal(mapped, h1)


def test_sphere_sheet_round0_hit_count_near_crofton_estimate():
    # The sheet's edges cut the sphere along a circle of radius ~0.954; for a
    # square grid with diagonals the expected number of crossing edges is
    # about (4 rho / h) * (1 + 1 + sqrt 2) / ... ~ 160.
    pair = meshgen.sphere_sheet()
    h, cand = oracle.detect(pair.pos_a, oracle.edges(pair.tri_a), pair.tri_a, pair.pos_b,
                            oracle.edges(pair.tri_b), pair.tri_b, 0, nthreads=4)
    assert 120 <= len(h) <= 200
    assert cand > len(h)
    assert set(np.unique(h[:, 0])) == {0}
    # every x0 is an endpoint of its edge and lies strictly inside the sphere's plane side
    assert np.all((h[:, 4] == h[:, 1]) | (h[:, 4] == h[:, 2]))


def test_dcd_threads_do_not_change_result():
    pair = meshgen.sphere_sheet()
    ea = oracle.edges(pair.tri_a)
    h1, c1 = oracle.dcd(pair.pos_a, ea, pair.pos_b, pair.tri_b, nthreads=1)
    h4, c4 = oracle.dcd(pair.pos_a, ea, pair.pos_b, pair.tri_b, nthreads=4)
    assert np.array_equal(h1, h4) and c1 == c4


def test_sampled_edges_match_full_pass():
    pair = meshgen.sphere_sheet()
    ea = oracle.edges(pair.tri_a)
    full, _ = oracle.dcd(pair.pos_a, ea, pair.pos_b, pair.tri_b, nthreads=4)
    ids = np.unique(np.concatenate([full[::3, 0], np.arange(0, len(ea), 97)]))
    part, _ = oracle.dcd(pair.pos_a, ea, pair.pos_b, pair.tri_b, nthreads=4, edge_ids=ids)
    want = full[np.isin(full[:, 0], ids)]
    assert np.array_equal(part, want)
