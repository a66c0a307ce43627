"""The request server (hfcr_server_*) through the C ABI.

Requests that are in flight together must give the same results as each
pair resolved alone (bit for bit: every request runs the single-pair path),
admission must respect the slot count and the memory budget, and waits,
timeouts and shutdown must behave as documented.
"""
import time

import numpy as np
import pytest
import torch

import meshgen
import paper_1409_2081_amd as hf
from tests.test_gpu_batch import PAIR_FIELDS, _alone, _f32, _item, _mixed_pairs

pytestmark = pytest.mark.gpu


def _same(alone, got, name):
    assert got["status"] == alone["status"], (name, got["status_name"], alone["status_name"])
    for k in PAIR_FIELDS:
        assert got["stats"][k] == alone["stats"][k], (name, k)
    for k in ("pos_a", "pos_b", "hits", "stencils"):
        assert torch.equal(got[k], alone[k]), (name, k)


def test_server_results_equal_alone_in_a_mix(hfcr_ctx):
    ps = _mixed_pairs() + meshgen.pair_set(seed=5, n=12, f_hi=20000.0)
    items = [_item(p) for p in ps]
    srv = hf.Server(0, slots=4)
    try:
        tickets = [srv.submit(it, max_rounds=12) for it in items]  # all in flight together
        got = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for it, g, p in zip(items, got, ps):
        assert g["latency_ms"] > 0
        _same(_alone(hfcr_ctx, it, max_rounds=12), g, p.name)


def test_server_admission_respects_slots_and_budget(hfcr_ctx):
    ps = meshgen.pair_set(seed=6, n=24, f_hi=30000.0)
    items = [_item(p) for p in ps]
    big = max(hf.Server.footprint(it) for it in items)
    budget = int(1.5 * big)
    srv = hf.Server(0, slots=8, pool_bytes=budget)
    try:
        tickets = [srv.submit(it, max_rounds=6) for it in items]
        seen_bytes, seen_running = 0, 0
        pending = list(tickets)
        results = {}
        while pending:
            c = srv.counts()
            seen_bytes = max(seen_bytes, c["admitted_bytes"])
            seen_running = max(seen_running, c["running"])
            t = pending[0]
            r = srv.wait(t, timeout_us=200)
            if r is not None:
                results[t] = r
                pending.pop(0)
        assert 0 < seen_bytes <= budget and 1 <= seen_running <= 8
        # a request larger than the whole budget is refused at once
        huge = _item(meshgen.linked_tori(nu=256, nv=128))
        assert hf.Server.footprint(huge) > budget
        with pytest.raises(hf.HfcrError) as e:
            srv.submit(huge)
        assert e.value.status == hf.HFCR_E_REJECTED
    finally:
        srv.close()
    assert srv is not None and len(results) == len(items)
    for t, it, p in list(zip(tickets, items, ps))[:6]:
        _same(_alone(hfcr_ctx, it, max_rounds=6), results[t], p.name)


def test_server_wait_timeout_and_shutdown(hfcr_ctx):
    srv = hf.Server(0, slots=1)
    tori = _item(meshgen.linked_tori())
    t0 = srv.submit(tori, max_rounds=12)
    r = srv.wait(t0, timeout_us=0)
    if r is None:  # still running: the ticket stays valid
        r = srv.wait(t0)
    assert r["status"] == hf.HFCR_NOT_CONVERGED
    with pytest.raises(hf.HfcrError):
        srv.wait(t0)  # released after its final status
    # shutdown finishes what was queued
    items = [_item(_f32(meshgen.random_small_pair(s, "sphere_sheet"))) for s in range(6)]
    for it in items:
        srv.submit(it, max_rounds=10)
    t = time.perf_counter()
    srv.close()
    assert time.perf_counter() - t < 60
