"""Batched calls (hfcr_resolve_batch, hfcr_detect_batch) through the C ABI.

A pair's positions, hit list, stencils and per-pair stats from a batch must
be bit-identical to what hfcr_resolve / hfcr_detect give for that pair
alone (the alone path is the one checked against the oracle elsewhere),
whatever the number of pairs in flight; the batch stats must be the sums
over the pairs, and a pair that fails must not disturb the others.
"""
import dataclasses

import numpy as np
import pytest
import torch

import meshgen
import paper_1409_2081_amd as hf

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
PAIR_FIELDS = ["rounds", "converged", "residual_hits", "hits0", "stencils0", "candidates", "max_zone",
               "round_hits", "round_stencils", "round_zones", "round_max_zone"]


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _f32(pair):
    return dataclasses.replace(pair, dtype=meshgen.F32, tier=0).cast()


def _item(pair, **kw):
    it = hf.pair_item(pair, DEV)
    it.update(kw)
    return it


def _alone(ctx, it, **opt):
    w = {k: it[k] for k in ("inv_mass_a", "inv_mass_b") if it.get(k) is not None}
    return ctx.resolve(it["pos_a"], it["tri_a"], it["pos_b"], it["tri_b"], it["orientation"], it["d"],
                       raise_on_error=False, **w, **opt)


def _check_same(alone, got, name):
    assert got["status"] == alone["status"], (name, got["status_name"], alone["status_name"])
    for k in PAIR_FIELDS:
        assert got["stats"][k] == alone["stats"][k], (name, k, got["stats"][k], alone["stats"][k])
    for k in ("pos_a", "pos_b", "hits", "stencils"):
        assert torch.equal(got[k], alone[k]), (name, k)


def _sums(bst, pairs):
    for k in ("hits0", "stencils0", "candidates", "residual_hits"):
        assert bst[k] == sum(p["stats"][k] for p in pairs), k
    assert bst["rounds"] == max(p["stats"]["rounds"] for p in pairs)
    assert bst["max_zone"] == max(p["stats"]["max_zone"] for p in pairs)


def _mixed_pairs():
    ps = [_f32(meshgen.random_small_pair(s, k)) for s in range(4) for k in ("sphere_sheet", "torus")]
    ps.append(_f32(meshgen.sphere_sheet(z=0.9)))
    ps.append(meshgen.linked_tori(nu=32, nv=16, shift=1.5))
    # mesh A oriented: the sphere as A, the sheet as B
    ss = _f32(meshgen.sphere_sheet(seed=3, z=0.6))
    ps.append(dataclasses.replace(ss, pos_a=ss.pos_b, tri_a=ss.tri_b, pos_b=ss.pos_a, tri_b=ss.tri_a,
                                  orientation=meshgen.ORIENT_A))
    ps.append(_f32(meshgen.sphere_sheet(z=3.0)))  # no contact
    return ps


@pytest.mark.parametrize("workers", [1, 3, 8])
def test_batch_equals_alone_mixed(hfcr_ctx, workers):
    hfcr_ctx.set_tuning(batch_workers=workers)
    ps = _mixed_pairs()
    items = [_item(p) for p in ps]
    # one pair with inverse masses (the sphere pinned), one with an empty face mesh
    items[8]["inv_mass_b"] = _t(np.zeros(len(ps[8].pos_b)))
    items[8]["inv_mass_a"] = _t(np.full(len(ps[8].pos_a), 0.5))
    empty = _item(ps[0])
    empty["tri_b"] = torch.zeros((0, 3), dtype=torch.int32, device=DEV)
    items.append(empty)
    names = [p.name for p in ps] + ["empty_faces"]
    for mode in (hf.BOTH_ALTERNATE, hf.BOTH_SIMULTANEOUS):
        opt = dict(max_rounds=40, both_mode=mode, round_offset=1 if mode == hf.BOTH_ALTERNATE else 0)
        b = hfcr_ctx.resolve_batch(items, **opt)
        assert len(b["pairs"]) == len(items)
        for it, got, name in zip(items, b["pairs"], names):
            _check_same(_alone(hfcr_ctx, it, **opt), got, name)
        _sums(b["stats"], b["pairs"])
        assert any(p["stats"]["rounds"] > 0 for p in b["pairs"])
    hfcr_ctx.set_tuning(batch_workers=12)


def test_batch_equals_alone_pair_set_full_size(hfcr_ctx):
    # the 256-pair mixed set at full size, a few rounds
    ps = meshgen.pair_set()
    items = [_item(p) for p in ps]
    b = hfcr_ctx.resolve_batch(items, max_rounds=3, tier=0)
    print("pair set statuses", {k: sum(p["status_name"] == k for p in b["pairs"]) for k in hf.STATUS_NAMES.values()})
    for it, got, p in zip(items, b["pairs"], ps):
        _check_same(_alone(hfcr_ctx, it, max_rounds=3, tier=0), got, p.name)
    _sums(b["stats"], b["pairs"])
    assert b["stats"]["hits0"] > 0


def test_batch_failures_stay_with_their_pair(hfcr_ctx):
    good = _f32(meshgen.sphere_sheet(z=0.9))
    nan = _f32(meshgen.sphere_sheet(z=0.9))
    nan.pos_a[3, 0] = np.nan
    badidx = _f32(meshgen.random_small_pair(2, "torus"))
    badidx.tri_b[1, 1] = len(badidx.pos_b)
    negd = _item(good, d=-1.0)
    items = [_item(good), _item(nan), _item(badidx), negd, _item(meshgen.linked_tori(nu=32, nv=16, shift=1.5))]
    b = hfcr_ctx.resolve_batch(items, max_rounds=30)
    st = [p["status"] for p in b["pairs"]]
    assert st[1] == st[2] == st[3] == hf.HFCR_E_INVALID, st
    assert b["status"] == hf.HFCR_E_INVALID
    for k in (0, 4):
        _check_same(_alone(hfcr_ctx, items[k], max_rounds=30), b["pairs"][k], k)
    # pairs of different storage types mix freely
    f64 = meshgen.sphere_sheet(z=0.9)
    items = [_item(good), _item(f64)]
    b = hfcr_ctx.resolve_batch(items, max_rounds=30, tier=1)
    assert [p["status"] for p in b["pairs"]] == [hf.HFCR_OK, hf.HFCR_OK]
    _check_same(_alone(hfcr_ctx, items[1], max_rounds=30, tier=1), b["pairs"][1], "f64")


def test_batch_zone_limit_stays_with_its_pair(hfcr_ctx):
    # simultaneous responses on this overlap grow an impact zone beyond the
    # dense solver's limit; the small pair beside it must not notice
    big = _item(meshgen.linked_tori(nu=64, nv=32, shift=1.5))
    small = _item(_f32(meshgen.random_small_pair(1, "sphere_sheet")))
    alone = _alone(hfcr_ctx, big, both_mode=hf.BOTH_SIMULTANEOUS)
    assert alone["status"] == hf.HFCR_E_ZONE_LIMIT
    b = hfcr_ctx.resolve_batch([small, big], both_mode=hf.BOTH_SIMULTANEOUS)
    _check_same(alone, b["pairs"][1], "tori")
    _check_same(_alone(hfcr_ctx, small, both_mode=hf.BOTH_SIMULTANEOUS), b["pairs"][0], "small")
    assert b["pairs"][0]["status"] == hf.HFCR_OK


def test_detect_batch_equals_detect(hfcr_ctx):
    ps = _mixed_pairs()
    items = [_item(p) for p in ps]
    b = hfcr_ctx.detect_batch(items, tier=0)
    for it, got, p in zip(items, b["pairs"], ps):
        a = hfcr_ctx.detect(it["pos_a"], it["tri_a"], it["pos_b"], it["tri_b"], it["orientation"], tier=0)
        assert got["status"] == a["status"]
        assert torch.equal(got["hits"], a["hits"]) and torch.equal(got["stencils"], a["stencils"]), p.name
        for k in ("hits0", "stencils0", "candidates", "residual_hits", "converged"):
            assert got["stats"][k] == a["stats"][k], (p.name, k)


def test_empty_batch(hfcr_ctx):
    b = hfcr_ctx.resolve_batch([])
    assert b["status"] == hf.HFCR_OK and b["pairs"] == [] and b["stats"]["converged"]
