"""Body-in-garment pair at full size (about 200k body and 100k cloth triangles).

The oracle's brute-force DCD over every edge is too slow at this size, so
parity is checked on samples it computes exactly: every edge the library
reports plus random edges, each tested by the oracle against every body
face; the library's hit list restricted to those edges must equal the
oracle's.  The response is checked by a lockstep round against the oracle,
and the converged output by the library's own detection and the oracle's on
the edges that moved plus random edges.
"""
import numpy as np
import pytest
import torch

import meshgen
import oracle
import paper_1409_2081_amd as hf

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def body():
    p = meshgen.body_garment()
    return p, hf.pair_tensors(p, DEV)


def _records(h, e):
    rec = np.zeros((len(h), 5), np.int32)
    if len(h):
        rec[:, 1:3] = e[h[:, 0]]
        rec[:, 3], rec[:, 4] = h[:, 1], h[:, 2]
    order = np.lexsort(rec.T[::-1])
    return rec[order]


def _sampled_hits(pos_a, tri_a, pos_b, tri_b, edge_ids):
    ea = oracle.edges(tri_a)
    h, _ = oracle.dcd(pos_a, ea, pos_b, tri_b, nthreads=16, edge_ids=edge_ids)
    return _records(h, ea)


def _edge_index(tri_a):
    ea = oracle.edges(tri_a)
    return ea, {(int(u), int(v)): k for k, (u, v) in enumerate(ea)}


@pytest.mark.parametrize("tier", [0, 1])
def test_body_garment_detect_sampled_parity(hfcr_ctx, body, tier):
    p, t = body
    g = hfcr_ctx.detect(*t, p.orientation, tier=tier, hit_cap=1 << 18, stencil_cap=1 << 18)
    hits = g["hits"].cpu().numpy()
    print("body-garment round-0 hits", len(hits), "stencils", len(g["stencils"]))
    assert len(hits) > 1000
    ea, index = _edge_index(p.tri_a)
    rng = np.random.default_rng(0)
    reported = {index[(int(u), int(v))] for u, v in hits[:, 1:3]}
    sample = np.array(sorted(reported | set(rng.choice(len(ea), 4000, replace=False).tolist())))
    want = _sampled_hits(p.pos_a, p.tri_a, p.pos_b, p.tri_b, sample)
    assert np.array_equal(hits, want)
    assert np.array_equal(g["stencils"].cpu().numpy(), oracle.stencils(want))


def test_body_garment_one_round_lockstep(hfcr_ctx, body):
    p, t = body
    g = hfcr_ctx.resolve(*t, p.orientation, p.d, tier=0, max_rounds=1, hit_cap=1 << 18, stencil_cap=1 << 18)
    st = oracle.stencils(g["hits"].cpu().numpy())
    assert np.array_equal(st, g["stencils"].cpu().numpy())
    xa, xb, info = oracle.respond(p.pos_a.astype(float), p.pos_b.astype(float), p.tri_a, p.tri_b, st, p.d)
    xa, xb = xa.astype(np.float32), xb.astype(np.float32)
    L = float(np.linalg.norm(np.ptp(np.concatenate([p.pos_a, p.pos_b]).astype(float), axis=0)))
    err = max(np.abs(g["pos_a"].cpu().numpy().astype(float) - xa).max(),
              np.abs(g["pos_b"].cpu().numpy().astype(float) - xb).max()) / L
    print("body-garment round 1: zones", info["zones"], "largest", info["max_k"], "rel err", err)
    assert err <= 1e-6


def test_body_garment_resolves(hfcr_ctx, body):
    p, t = body
    g = hfcr_ctx.resolve(*t, p.orientation, p.d, tier=0, max_rounds=64, hit_cap=1 << 18, stencil_cap=1 << 18)
    s = g["stats"]
    print("body-garment resolve:", g["status_name"], "rounds", s["rounds"], "hits0", s["hits0"],
          "round hits", s["round_hits"][:12], "largest zone", s["max_zone"])
    assert g["status"] == hf.HFCR_OK and s["converged"] and s["residual_hits"] == 0
    pa = g["pos_a"]
    again = hfcr_ctx.detect(pa, t[1], g["pos_b"], t[3], p.orientation, tier=1)
    assert again["stats"]["hits0"] == 0
    # the oracle on every edge touching a moved vertex, plus random edges
    xa = pa.cpu().numpy()
    moved = np.nonzero(np.any(xa != p.pos_a, axis=1))[0]
    ea, _ = _edge_index(p.tri_a)
    touch = np.nonzero(np.isin(ea[:, 0], moved) | np.isin(ea[:, 1], moved))[0]
    rng = np.random.default_rng(1)
    sample = np.union1d(touch, rng.choice(len(ea), 4000, replace=False))
    assert len(_sampled_hits(xa, p.tri_a, g["pos_b"].cpu().numpy(), p.tri_b, sample)) == 0
