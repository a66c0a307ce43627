"""Python binding of libhfcr.so: history-free collision response on gfx950.

Argument marshalling only: every step of detection and response runs in the
library's HIP kernels.  PyTorch supplies device memory and the stream.  The
library must be built (``python -m paper_1409_2081_amd.build`` or
``__graft_entry__.build()``); there is no fallback path, so a missing library
or device raises.

Entry points mirror include/hfcr.h: ``Context.resolve``, ``Context.detect``,
``Context.resolve_batch``, ``Context.detect_batch`` and ``Context.test_orient``.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhfcr.so")

HFCR_OK = 0
HFCR_NOT_CONVERGED = 1
HFCR_PENDING = 2
HFCR_E_INVALID = -1
HFCR_E_CAPACITY = -2
HFCR_E_OOM = -3
HFCR_E_DEVICE = -4
HFCR_E_ZONE_LIMIT = -5
HFCR_E_REJECTED = -6
STATUS_NAMES = {0: "OK", 1: "NOT_CONVERGED", 2: "PENDING", -1: "E_INVALID", -2: "E_CAPACITY", -3: "E_OOM",
                -4: "E_DEVICE", -5: "E_ZONE_LIMIT", -6: "E_REJECTED"}

HFCR_F32 = 0
HFCR_F64 = 1
ORIENT_B = 0
ORIENT_A = 1
ORIENT_BOTH = 2
BOTH_ALTERNATE = 0
BOTH_SIMULTANEOUS = 1
FLAG_TIMING = 1
MAX_ZONE = 4096
MAX_BATCH = 65536
STAT_ROUNDS = 64
STAGES = 8
STAGE_NAMES = ["setup", "refit", "traverse", "narrow", "stencils", "zones", "solve", "update"]

EXPORTED = ["hfcr_default_opts", "hfcr_create", "hfcr_destroy", "hfcr_last_error", "hfcr_detect",
            "hfcr_resolve", "hfcr_resolve_batch", "hfcr_detect_batch", "hfcr_test_orient",
            "hfcr_get_tuning", "hfcr_set_tuning", "hfcr_server_create", "hfcr_server_destroy",
            "hfcr_server_submit", "hfcr_server_wait", "hfcr_server_counts"]


class Mesh(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("nv", ctypes.c_int32), ("nt", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("pos", ctypes.c_void_p), ("tri", ctypes.c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("max_rounds", ctypes.c_int32), ("both_mode", ctypes.c_int32),
                ("predicate_tier", ctypes.c_int32), ("round_offset", ctypes.c_int32),
                ("inv_mass_a", ctypes.c_void_p), ("inv_mass_b", ctypes.c_void_p),
                ("flags", ctypes.c_uint32), ("reserved", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("residual_hits", ctypes.c_int64), ("hits0", ctypes.c_int64),
                ("stencils0", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("exact_tests", ctypes.c_int64), ("f32_ambiguous", ctypes.c_int64),
                ("max_zone", ctypes.c_int32), ("rank_deficient", ctypes.c_int32),
                ("node_visits", ctypes.c_int64), ("pivoted_zones", ctypes.c_int32),
                ("max_query_path", ctypes.c_int32),
                ("stage_ms", ctypes.c_double * STAGES), ("stage_calls", ctypes.c_int32 * STAGES),
                ("round_hits", ctypes.c_int32 * STAT_ROUNDS),
                ("round_stencils", ctypes.c_int32 * STAT_ROUNDS),
                ("round_zones", ctypes.c_int32 * STAT_ROUNDS),
                ("round_max_zone", ctypes.c_int32 * STAT_ROUNDS)]

    def to_dict(self) -> dict:
        n = min(self.rounds + 1, STAT_ROUNDS)
        return {
            "rounds": self.rounds, "converged": bool(self.converged),
            "residual_hits": self.residual_hits, "hits0": self.hits0, "stencils0": self.stencils0,
            "candidates": self.candidates, "exact_tests": self.exact_tests,
            "f32_ambiguous": self.f32_ambiguous, "max_zone": self.max_zone,
            "rank_deficient": self.rank_deficient, "node_visits": self.node_visits,
            "pivoted_zones": self.pivoted_zones, "max_query_path": self.max_query_path,
            "stage_ms": {STAGE_NAMES[i]: self.stage_ms[i] for i in range(STAGES)},
            "stage_calls": {STAGE_NAMES[i]: self.stage_calls[i] for i in range(STAGES)},
            "round_hits": list(self.round_hits[:n]), "round_stencils": list(self.round_stencils[:n]),
            "round_zones": list(self.round_zones[:n]), "round_max_zone": list(self.round_max_zone[:n]),
        }


class Tuning(ctypes.Structure):
    _fields_ = [("trav_block", ctypes.c_int32), ("trav_warm", ctypes.c_int32),
                ("batch_workers", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Result(ctypes.Structure):
    _fields_ = [("pos_a_out", ctypes.c_void_p), ("pos_b_out", ctypes.c_void_p),
                ("hits", ctypes.c_void_p), ("hit_cap", ctypes.c_int64),
                ("stencils", ctypes.c_void_p), ("stencil_cap", ctypes.c_int64),
                ("stats", ctypes.POINTER(Stats))]


class PairDesc(ctypes.Structure):
    """hfcr_pair: one mesh pair of a batch call."""
    _fields_ = [("a", Mesh), ("b", Mesh), ("orientation", ctypes.c_int32), ("status", ctypes.c_int32),
                ("d", ctypes.c_double), ("inv_mass_a", ctypes.c_void_p), ("inv_mass_b", ctypes.c_void_p),
                ("res", Result)]


class ServerCfg(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("reserved", ctypes.c_int32), ("pool_bytes", ctypes.c_int64)]


_LIB = None


def lib():
    """Load libhfcr.so; raises if it has not been built."""
    global _LIB
    if _LIB is None:
        # load PyTorch's HIP runtime first, so that the library binds to the same
        # one (two runtimes in one process do not share devices or memory)
        _torch()
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_1409_2081_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.hfcr_default_opts.argtypes = [ctypes.POINTER(Opts)]
        L.hfcr_default_opts.restype = None
        L.hfcr_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int]
        L.hfcr_create.restype = ctypes.c_int
        L.hfcr_destroy.argtypes = [vp]
        L.hfcr_destroy.restype = None
        L.hfcr_last_error.argtypes = [vp]
        L.hfcr_last_error.restype = ctypes.c_char_p
        L.hfcr_detect.argtypes = [vp, ctypes.POINTER(Mesh), ctypes.POINTER(Mesh), ctypes.c_int32,
                                  ctypes.POINTER(Opts), ctypes.POINTER(Result), vp]
        L.hfcr_detect.restype = ctypes.c_int
        L.hfcr_resolve.argtypes = [vp, ctypes.POINTER(Mesh), ctypes.POINTER(Mesh), ctypes.c_int32,
                                   ctypes.c_double, ctypes.POINTER(Opts), ctypes.POINTER(Result), vp]
        L.hfcr_resolve.restype = ctypes.c_int
        for name in ("hfcr_resolve_batch", "hfcr_detect_batch"):
            f = getattr(L, name)
            f.argtypes = [vp, ctypes.POINTER(PairDesc), ctypes.c_int32, ctypes.POINTER(Opts),
                          ctypes.POINTER(Stats), vp]
            f.restype = ctypes.c_int
        L.hfcr_server_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.POINTER(ServerCfg)]
        L.hfcr_server_create.restype = ctypes.c_int
        L.hfcr_server_destroy.argtypes = [vp]
        L.hfcr_server_destroy.restype = None
        L.hfcr_server_submit.argtypes = [vp, ctypes.POINTER(PairDesc), ctypes.POINTER(Opts),
                                         ctypes.POINTER(ctypes.c_uint64)]
        L.hfcr_server_submit.restype = ctypes.c_int
        L.hfcr_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
        L.hfcr_server_wait.restype = ctypes.c_int
        i64p = ctypes.POINTER(ctypes.c_int64)
        L.hfcr_server_counts.argtypes = [vp, i64p, i64p, i64p, i64p]
        L.hfcr_server_counts.restype = None
        L.hfcr_test_orient.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, vp, vp]
        L.hfcr_test_orient.restype = ctypes.c_int
        L.hfcr_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.hfcr_get_tuning.restype = ctypes.c_int
        L.hfcr_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
        L.hfcr_set_tuning.restype = ctypes.c_int
        _LIB = L
    return _LIB


class HfcrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _torch():
    import torch
    return torch


def _mesh(pos, tri) -> Mesh:
    torch = _torch()
    if not (pos.is_cuda and tri.is_cuda):
        raise ValueError("positions and triangles must be device tensors")
    if pos.dtype not in (torch.float32, torch.float64) or tri.dtype != torch.int32:
        raise ValueError("positions must be float32/float64 and triangles int32")
    if pos.dim() != 2 or pos.shape[1] != 3 or tri.dim() != 2 or tri.shape[1] != 3:
        raise ValueError("positions must be [nv,3] and triangles [nt,3]")
    if not (pos.is_contiguous() and tri.is_contiguous()):
        raise ValueError("arrays must be contiguous")
    return Mesh(HFCR_F32 if pos.dtype == torch.float32 else HFCR_F64, pos.shape[0], tri.shape[0], 0,
                pos.data_ptr() if pos.numel() else None, tri.data_ptr() if tri.numel() else None)


class Context:
    """One library context on a GPU (owns the device workspace)."""

    def __init__(self, device: int = 0):
        self._L = lib()
        h = ctypes.c_void_p()
        st = self._L.hfcr_create(ctypes.byref(h), int(device))
        if st != HFCR_OK:
            raise HfcrError(st, "hfcr_create failed")
        self._h = h
        self.device = device

    def close(self):
        if getattr(self, "_h", None):
            self._L.hfcr_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_tuning(self) -> dict:
        t = Tuning()
        st = self._L.hfcr_get_tuning(self._h, ctypes.byref(t))
        if st != HFCR_OK:
            raise HfcrError(st, self.last_error())
        return {"trav_block": t.trav_block, "trav_warm": t.trav_warm, "batch_workers": t.batch_workers}

    def set_tuning(self, **kw) -> None:
        cur = self.get_tuning()
        cur.update(kw)
        t = Tuning(int(cur["trav_block"]), int(cur["trav_warm"]), int(cur["batch_workers"]), 0)
        st = self._L.hfcr_set_tuning(self._h, ctypes.byref(t))
        if st != HFCR_OK:
            raise HfcrError(st, self.last_error())

    def last_error(self) -> str:
        return self._L.hfcr_last_error(self._h).decode()

    @staticmethod
    def _opts(max_rounds=256, both_mode=BOTH_ALTERNATE, tier=0, round_offset=0, inv_mass_a=None,
              inv_mass_b=None, timing=False) -> Opts:
        o = Opts()
        lib().hfcr_default_opts(ctypes.byref(o))
        o.max_rounds = int(max_rounds)
        o.both_mode = int(both_mode)
        o.predicate_tier = int(tier)
        o.round_offset = int(round_offset)
        o.inv_mass_a = inv_mass_a.data_ptr() if inv_mass_a is not None else None
        o.inv_mass_b = inv_mass_b.data_ptr() if inv_mass_b is not None else None
        o.flags = FLAG_TIMING if timing else 0
        return o

    def resolve(self, pos_a, tri_a, pos_b, tri_b, orientation=ORIENT_B, d=1e-3, *, hit_cap=1 << 16,
                stencil_cap=1 << 16, want_lists=True, raise_on_error=True, stream=None, **opt_kw) -> dict:
        """hfcr_resolve: returns positions, round-0 hits/stencils, stats and status."""
        torch = _torch()
        ma, mb = _mesh(pos_a, tri_a), _mesh(pos_b, tri_b)
        out_a, out_b = torch.empty_like(pos_a), torch.empty_like(pos_b)
        hits = torch.empty((hit_cap, 5), dtype=torch.int32, device=pos_a.device) if want_lists else None
        sten = torch.empty((stencil_cap, 3), dtype=torch.int32, device=pos_a.device) if want_lists else None
        stats = Stats()
        res = Result(out_a.data_ptr() if out_a.numel() else None,
                     out_b.data_ptr() if out_b.numel() else None,
                     hits.data_ptr() if hits is not None else None, hit_cap,
                     sten.data_ptr() if sten is not None else None, stencil_cap,
                     ctypes.pointer(stats))
        o = self._opts(**opt_kw)
        s = stream if stream is not None else torch.cuda.current_stream(pos_a.device).cuda_stream
        st = self._L.hfcr_resolve(self._h, ctypes.byref(ma), ctypes.byref(mb), int(orientation), float(d),
                                  ctypes.byref(o), ctypes.byref(res), ctypes.c_void_p(s))
        if st == HFCR_E_CAPACITY and want_lists:
            return self.resolve(pos_a, tri_a, pos_b, tri_b, orientation, d,
                                hit_cap=max(hit_cap, stats.hits0), stencil_cap=max(stencil_cap, stats.stencils0),
                                want_lists=True, raise_on_error=raise_on_error, stream=stream, **opt_kw)
        if st < 0 and st != HFCR_E_ZONE_LIMIT and raise_on_error:
            raise HfcrError(st, self.last_error())
        out = {"status": st, "status_name": STATUS_NAMES.get(st, str(st)), "pos_a": out_a, "pos_b": out_b,
               "stats": stats.to_dict()}
        if st == HFCR_E_ZONE_LIMIT:
            out["error"] = self.last_error()
        if want_lists:
            out["hits"] = hits[: min(stats.hits0, hit_cap)]
            out["stencils"] = sten[: min(stats.stencils0, stencil_cap)]
        return out

    def detect(self, pos_a, tri_a, pos_b, tri_b, orientation=ORIENT_B, *, hit_cap=1 << 16,
               stencil_cap=1 << 16, stream=None, **opt_kw) -> dict:
        """hfcr_detect: one DCD pass; returns hits, stencils and stats."""
        torch = _torch()
        ma, mb = _mesh(pos_a, tri_a), _mesh(pos_b, tri_b)
        hits = torch.empty((hit_cap, 5), dtype=torch.int32, device=pos_a.device)
        sten = torch.empty((stencil_cap, 3), dtype=torch.int32, device=pos_a.device)
        stats = Stats()
        res = Result(None, None, hits.data_ptr(), hit_cap, sten.data_ptr(), stencil_cap, ctypes.pointer(stats))
        o = self._opts(**opt_kw)
        s = stream if stream is not None else torch.cuda.current_stream(pos_a.device).cuda_stream
        st = self._L.hfcr_detect(self._h, ctypes.byref(ma), ctypes.byref(mb), int(orientation),
                                 ctypes.byref(o), ctypes.byref(res), ctypes.c_void_p(s))
        if st == HFCR_E_CAPACITY:
            return self.detect(pos_a, tri_a, pos_b, tri_b, orientation, hit_cap=max(hit_cap, stats.hits0),
                               stencil_cap=max(stencil_cap, stats.stencils0), stream=stream, **opt_kw)
        if st < 0:
            raise HfcrError(st, self.last_error())
        return {"status": st, "hits": hits[: stats.hits0], "stencils": sten[: stats.stencils0],
                "stats": stats.to_dict()}

    def _batch(self, fn, items, detect: bool, hit_cap, stencil_cap, want_lists, stream, opt_kw):
        torch = _torch()
        n = len(items)
        arr = (PairDesc * max(n, 1))()
        keep, outs = [], []
        stats = [Stats() for _ in range(n)]
        caps_h = hit_cap if isinstance(hit_cap, (list, tuple)) else [hit_cap] * n
        caps_s = stencil_cap if isinstance(stencil_cap, (list, tuple)) else [stencil_cap] * n
        dev = None
        for i, it in enumerate(items):
            pa, ta, pb, tb = it["pos_a"], it["tri_a"], it["pos_b"], it["tri_b"]
            dev = pa.device
            q = arr[i]
            q.a, q.b = _mesh(pa, ta), _mesh(pb, tb)
            q.orientation = int(it.get("orientation", ORIENT_B))
            q.d = float(it.get("d", 1e-3))
            wa, wb = it.get("inv_mass_a"), it.get("inv_mass_b")
            q.inv_mass_a = wa.data_ptr() if wa is not None else None
            q.inv_mass_b = wb.data_ptr() if wb is not None else None
            out_a = None if detect else torch.empty_like(pa)
            out_b = None if detect else torch.empty_like(pb)
            hits = torch.empty((caps_h[i], 5), dtype=torch.int32, device=dev) if want_lists else None
            sten = torch.empty((caps_s[i], 3), dtype=torch.int32, device=dev) if want_lists else None
            q.res = Result(out_a.data_ptr() if out_a is not None and out_a.numel() else None,
                           out_b.data_ptr() if out_b is not None and out_b.numel() else None,
                           hits.data_ptr() if hits is not None else None, caps_h[i],
                           sten.data_ptr() if sten is not None else None, caps_s[i],
                           ctypes.pointer(stats[i]))
            keep.append((wa, wb))
            outs.append((out_a, out_b, hits, sten))
        bstats = Stats()
        o = self._opts(**opt_kw)
        if stream is None:
            stream = torch.cuda.current_stream(dev).cuda_stream if dev is not None else 0
        st = fn(self._h, arr, n, ctypes.byref(o), ctypes.byref(bstats), ctypes.c_void_p(stream))
        # a negative status no pair carries is a failure of the call as a whole
        if st < 0 and all(arr[i].status != st for i in range(n)):
            raise HfcrError(st, self.last_error())
        if want_lists and any(arr[i].status == HFCR_E_CAPACITY for i in range(n)):
            nh = [max(caps_h[i], stats[i].hits0) for i in range(n)]
            ns = [max(caps_s[i], stats[i].stencils0) for i in range(n)]
            return self._batch(fn, items, detect, nh, ns, want_lists, stream, opt_kw)
        res = []
        for i in range(n):
            out_a, out_b, hits, sten = outs[i]
            r = {"status": arr[i].status, "status_name": STATUS_NAMES.get(arr[i].status, str(arr[i].status)),
                 "stats": stats[i].to_dict()}
            if not detect:
                r["pos_a"], r["pos_b"] = out_a, out_b
            if want_lists:
                r["hits"] = hits[: min(stats[i].hits0, caps_h[i])]
                r["stencils"] = sten[: min(stats[i].stencils0, caps_s[i])]
            res.append(r)
        return {"status": st, "status_name": STATUS_NAMES.get(st, str(st)), "pairs": res,
                "stats": bstats.to_dict(), "error": self.last_error() if st != HFCR_OK else ""}

    def resolve_batch(self, items, *, hit_cap=4096, stencil_cap=4096, want_lists=True, stream=None,
                      **opt_kw) -> dict:
        """hfcr_resolve_batch over items: dicts with pos_a, tri_a, pos_b, tri_b and optionally
        orientation, d, inv_mass_a, inv_mass_b.  Returns per-pair results and the batch stats."""
        return self._batch(self._L.hfcr_resolve_batch, items, False, hit_cap, stencil_cap, want_lists,
                           stream, opt_kw)

    def detect_batch(self, items, *, hit_cap=4096, stencil_cap=4096, stream=None, **opt_kw) -> dict:
        """hfcr_detect_batch: one DCD pass per oriented direction for every pair."""
        return self._batch(self._L.hfcr_detect_batch, items, True, hit_cap, stencil_cap, True, stream,
                           opt_kw)

    def test_orient(self, pts, tier: int, stream=None):
        """Signs of orient for pts [n,4,3] float64 (device); 2 means unsure (tiers 0 and 1)."""
        torch = _torch()
        pts = pts.contiguous()
        out = torch.empty(pts.shape[0], dtype=torch.int32, device=pts.device)
        s = stream if stream is not None else torch.cuda.current_stream(pts.device).cuda_stream
        st = self._L.hfcr_test_orient(self._h, ctypes.c_void_p(pts.data_ptr()), pts.shape[0], int(tier),
                                      ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s))
        if st != HFCR_OK:
            raise HfcrError(st, self.last_error())
        return out


class Server:
    """hfcr_server_*: a request loop admitting resolves by slots and an HBM footprint budget."""

    def __init__(self, device: int = 0, slots: int = 8, pool_bytes: int = 0):
        self._L = lib()
        h = ctypes.c_void_p()
        cfg = ServerCfg(int(slots), 0, int(pool_bytes))
        st = self._L.hfcr_server_create(ctypes.byref(h), int(device), ctypes.byref(cfg))
        if st != HFCR_OK:
            raise HfcrError(st, "hfcr_server_create failed")
        self._h = h
        self._live = {}  # ticket -> (descriptor, tensors, stats) kept alive until waited

    def submit(self, item: dict, *, hit_cap=4096, stencil_cap=4096, want_lists=True, **opt_kw) -> int:
        """Queue one resolve (an item as for Context.resolve_batch); returns the ticket."""
        torch = _torch()
        pa, ta, pb, tb = item["pos_a"], item["tri_a"], item["pos_b"], item["tri_b"]
        q = PairDesc()
        q.a, q.b = _mesh(pa, ta), _mesh(pb, tb)
        q.orientation = int(item.get("orientation", ORIENT_B))
        q.d = float(item.get("d", 1e-3))
        wa, wb = item.get("inv_mass_a"), item.get("inv_mass_b")
        q.inv_mass_a = wa.data_ptr() if wa is not None else None
        q.inv_mass_b = wb.data_ptr() if wb is not None else None
        out_a, out_b = torch.empty_like(pa), torch.empty_like(pb)
        hits = torch.empty((hit_cap, 5), dtype=torch.int32, device=pa.device) if want_lists else None
        sten = torch.empty((stencil_cap, 3), dtype=torch.int32, device=pa.device) if want_lists else None
        stats = Stats()
        q.res = Result(out_a.data_ptr() if out_a.numel() else None, out_b.data_ptr() if out_b.numel() else None,
                       hits.data_ptr() if hits is not None else None, hit_cap,
                       sten.data_ptr() if sten is not None else None, stencil_cap, ctypes.pointer(stats))
        o = Context._opts(**opt_kw)
        torch.cuda.synchronize(pa.device)  # inputs (and the fresh outputs) are complete on the device
        t = ctypes.c_uint64()
        st = self._L.hfcr_server_submit(self._h, ctypes.byref(q), ctypes.byref(o), ctypes.byref(t))
        if st != HFCR_OK:
            raise HfcrError(st, "request rejected" if st == HFCR_E_REJECTED else "submit failed")
        self._live[t.value] = (q, o, item, out_a, out_b, hits, sten, stats, hit_cap, stencil_cap)
        return t.value

    def wait(self, ticket: int, timeout_us: int = -1):
        """The request's result dict, or None if it is still pending after timeout_us."""
        lat = ctypes.c_double()
        st = self._L.hfcr_server_wait(self._h, ctypes.c_uint64(ticket), int(timeout_us), ctypes.byref(lat))
        if st == HFCR_PENDING:
            return None
        if st == HFCR_E_INVALID and ticket not in self._live:
            raise HfcrError(st, "unknown ticket")
        q, o, item, out_a, out_b, hits, sten, stats, hcap, scap = self._live.pop(ticket)
        r = {"status": st, "status_name": STATUS_NAMES.get(st, str(st)), "latency_ms": lat.value,
             "pos_a": out_a, "pos_b": out_b, "stats": stats.to_dict()}
        if hits is not None:
            r["hits"] = hits[: min(stats.hits0, hcap)]
            r["stencils"] = sten[: min(stats.stencils0, scap)]
        return r

    def counts(self) -> dict:
        v = [ctypes.c_int64() for _ in range(4)]
        self._L.hfcr_server_counts(self._h, *[ctypes.byref(x) for x in v])
        return dict(zip(("queued", "running", "completed", "admitted_bytes"), [x.value for x in v]))

    @staticmethod
    def footprint(item: dict) -> int:
        """The server's device-footprint estimate of a request (bytes)."""
        nv = item["pos_a"].shape[0] + item["pos_b"].shape[0]
        nt = item["tri_a"].shape[0] + item["tri_b"].shape[0]
        return 512 * nv + 1024 * nt + (1 << 20)

    def close(self):
        if getattr(self, "_h", None):
            self._L.hfcr_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pair_item(pair, device="cuda") -> dict:
    """A resolve_batch item from a meshgen.Pair."""
    pa, ta, pb, tb = pair_tensors(pair, device)
    return {"pos_a": pa, "tri_a": ta, "pos_b": pb, "tri_b": tb, "orientation": pair.orientation,
            "d": pair.d}


def pair_tensors(pair, device="cuda"):
    """Device tensors (pos_a, tri_a, pos_b, tri_b) of a meshgen.Pair."""
    torch = _torch()
    return (torch.from_numpy(pair.pos_a).to(device), torch.from_numpy(pair.tri_a).to(device),
            torch.from_numpy(pair.pos_b).to(device), torch.from_numpy(pair.tri_b).to(device))
