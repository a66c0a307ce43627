"""The seeded generators produce the workloads' stated shapes."""
import math

import numpy as np

import meshgen


def _closed_and_outward(pos, tri):
    e = np.sort(np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]]), axis=1)
    _, counts = np.unique(e, axis=0, return_counts=True)
    return bool(np.all(counts == 2)) and meshgen.signed_volume(pos, tri) > 0


def test_pair_set_sizes_kinds_and_placement():
    ps = meshgen.pair_set(seed=4, n=16)
    assert len(ps) == 16
    for k, p in enumerate(ps):
        for tri in (p.tri_a, p.tri_b):
            assert 500 * 0.9 <= len(tri) <= 50000 * 1.1, (p.name, len(tri))
        assert p.pos_a.dtype == np.float32 and p.tier == 0 and p.d == 1e-3
        if k % 2 == 0:
            assert p.orientation == meshgen.ORIENT_B
            assert _closed_and_outward(p.pos_b.astype(float), p.tri_b)
        else:
            assert p.orientation == meshgen.ORIENT_BOTH
            assert _closed_and_outward(p.pos_a.astype(float), p.tri_a)
            assert _closed_and_outward(p.pos_b.astype(float), p.tri_b)
        c = np.concatenate([p.pos_a, p.pos_b]).astype(float).mean(0)
        assert np.all(np.abs(c) < 5.0 + 2.0)
    # deterministic, and the sizes spread over the log range
    again = meshgen.pair_set(seed=4, n=16)
    assert all(np.array_equal(a.pos_a, b.pos_a) and np.array_equal(a.tri_b, b.tri_b) for a, b in zip(ps, again))
    f = np.log([len(p.tri_a) for p in meshgen.pair_set(seed=4, n=64)])
    assert f.min() < math.log(2000) and f.max() > math.log(12000)


def test_sized_primitives_hit_their_targets():
    for target in (500, 3000, 50000):
        for make in (meshgen.uv_sphere_f, meshgen.torus_f):
            pos, tri = make(target)
            assert abs(len(tri) - target) <= 0.05 * target, (make.__name__, target, len(tri))
            assert _closed_and_outward(pos, tri)
        pos, tri = meshgen.sheet_f(target, 2.5, 0.3)
        assert abs(len(tri) - target) <= 0.05 * target


def test_body_garment_is_closed_oriented_and_penetrating():
    p = meshgen.body_garment(body_tris=20000, cloth_tris=10000)
    assert abs(len(p.tri_b) - 20000) <= 1000 and abs(len(p.tri_a) - 10000) <= 500
    assert p.orientation == meshgen.ORIENT_B and p.pos_a.dtype == np.float32
    assert _closed_and_outward(p.pos_b.astype(float), p.tri_b)
    assert _closed_and_outward(p.pos_a.astype(float), p.tri_a)
    # the body surface sits on the capsules' zero level (within the linear
    # interpolation error of a ~3 cm grid), the cloth near 0.01 outside
    db = meshgen.capsule_sdf(p.pos_b.astype(float))
    assert np.abs(db).max() < 0.02 and np.median(np.abs(db)) < 2e-3
    da = meshgen.capsule_sdf(p.pos_a.astype(float))
    inside = (da < 0).sum()
    moved = int(round(0.05 * len(p.pos_a)))
    # displacements U[0, 0.03] against a 0.01 offset: about two thirds end inside
    assert 0.5 * moved < inside < 0.8 * moved
