// C ABI and host runtime: workspace management, per-call set-up (ingest,
// edges, Morton orders, BVH build), the detect / respond repair loop and
// status reporting.  Every arithmetic step runs in the kernels; the host
// only sequences launches and reads back the counts that size the next step.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hfcr.h"
#include "common.hpp"
#include "kernels.hpp"

using namespace hfcr;

namespace {

struct DBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// Counts of one detection pass, cleared together at its start; a pass that
// overflows a buffer is redone, and only the accepted pass is counted.
struct PassCount {
  uint32_t hits, amb, cand_n, pad;
  unsigned long long cand, f32_unsure, exact, visits;
};

struct Counters {
  uint32_t err;
  uint32_t maxabs[2];
  uint32_t tri_diff[2];  // triangle arrays differ from the cached topology's
  int32_t overflow;
  uint32_t total;
  uint32_t nzones;
  uint32_t maxk;      // cleared with retry_n, which must follow it
  uint32_t retry_n;   // zones the tiled solve hands to the pivoted one
  int32_t rank_def;
  int32_t pivoted;
  uint32_t max_path;
  PassCount pass[2];  // per direction
};

struct Timer {
  int stage;
  hipEvent_t a, b;
};

int bits_for(int64_t n) {  // bits to hold values 0..n-1 (at least 1)
  int b = 1;
  while (b < 62 && (1ll << b) < n) ++b;
  return b;
}

struct HipError {
  hipError_t e;
  const char *what;
};

}  // namespace

struct hfcr_ctx {
  int device = 0;
  std::string err;
  hipStream_t s = nullptr;
  // per mesh
  DBuf x64[2], x32[2], edges[2], qedges[2], leaf_tri[2], nodes[2], leaf_parent[2], counters_n[2], root_box[2],
      codes[2], scene_box[2], topo[2];
  // topology kept from the previous call (edge sets, query order, BVH tree),
  // reused while a mesh's triangle array is unchanged
  struct TopoCache {
    int nv = -1, nt = -1, ne = 0;
    bool edges = false, bvh = false;
  } topo_cache[2];
  DBuf tri_cache[2];
  // detection
  DBuf hk[2], hv[2], amb[2], cand;
  // generic sort / scan scratch
  DBuf sk0, sk1, sv0, sv1, hist, flags, pos, bsums;
  // response
  DBuf st_keys, st_out_keys, con, parent, zkeys, zvals, starts, lambda, inc_keys, solve_scratch, retry;
  DBuf ctr;
  Counters *hctr = nullptr;  // pinned
  std::vector<Timer> timers;
  std::vector<hipEvent_t> free_events;
  bool timing = false;
  hfcr_tuning tune{64, 0, 12, 0};
  // batch calls: one context and stream per concurrent worker
  std::vector<hfcr_ctx *> workers;
  std::vector<hipStream_t> wstreams;
};

namespace {

#define HIP_CHECK(x)                                   \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) throw HipError{e_, #x};      \
  } while (0)

struct StatusError {
  hfcr_status st;
  std::string msg;
};

void ensure(DBuf &b, size_t bytes, bool zero = false) {
  if (bytes == 0) bytes = 16;
  if (b.bytes >= bytes) return;
  const size_t old = b.bytes;
  if (b.p) HIP_CHECK(hipFree(b.p));
  b.p = nullptr;
  b.bytes = 0;
  size_t want = std::max(bytes, old + old / 2);
  hipError_t e = hipMalloc(&b.p, want);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    throw StatusError{HFCR_E_OOM, "device allocation of " + std::to_string(want) + " bytes failed"};
  }
  b.bytes = want;
  if (zero) HIP_CHECK(hipMemset(b.p, 0, want));
}

template <typename T>
T *ptr(DBuf &b) {
  return reinterpret_cast<T *>(b.p);
}

hipEvent_t take_event(hfcr_ctx *c) {
  if (!c->free_events.empty()) {
    hipEvent_t e = c->free_events.back();
    c->free_events.pop_back();
    return e;
  }
  hipEvent_t e;
  HIP_CHECK(hipEventCreate(&e));
  return e;
}

struct Scope {  // times the launches issued during its lifetime
  hfcr_ctx *c;
  int stage;
  hipEvent_t a = nullptr;
  Scope(hfcr_ctx *ctx, int st) : c(ctx), stage(st) {
    if (c->timing) {
      a = take_event(c);
      HIP_CHECK(hipEventRecord(a, c->s));
    }
  }
  ~Scope() {
    // never throws: a failed record only loses this interval
    if (c->timing && a) {
      hipEvent_t b = nullptr;
      if (!c->free_events.empty()) {
        b = c->free_events.back();
        c->free_events.pop_back();
      } else if (hipEventCreate(&b) != hipSuccess) {
        c->free_events.push_back(a);
        return;
      }
      if (hipEventRecord(b, c->s) == hipSuccess) {
        c->timers.push_back({stage, a, b});
      } else {
        c->free_events.push_back(a);
        c->free_events.push_back(b);
      }
    }
  }
};

void readback(hfcr_ctx *c) {
  HIP_CHECK(hipGetLastError());  // a refused launch surfaces here
  HIP_CHECK(hipMemcpyAsync(c->hctr, c->ctr.p, sizeof(Counters), hipMemcpyDeviceToHost, c->s));
  HIP_CHECK(hipStreamSynchronize(c->s));
}

// Sort (k, v) of length n in place, using the context's alternate buffers.
void sort_inplace(hfcr_ctx *c, uint64_t *k, uint32_t *v, int64_t n, int key_bits) {
  if (n <= 1) return;
  ensure(c->sk1, n * sizeof(uint64_t));
  if (v) ensure(c->sv1, n * sizeof(uint32_t));
  ensure(c->hist, radix_hist_entries(n) * sizeof(uint32_t));
  SortBufs b{k, ptr<uint64_t>(c->sk1), v, v ? ptr<uint32_t>(c->sv1) : nullptr, ptr<uint32_t>(c->hist),
             radix_hist_entries(n)};
  bool alt = false;
  sort_pairs(b, n, key_bits, c->s, alt);
  if (alt) {
    HIP_CHECK(hipMemcpyAsync(k, c->sk1.p, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, c->s));
    if (v) HIP_CHECK(hipMemcpyAsync(v, c->sv1.p, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, c->s));
  }
}

// Exclusive scan of flags[0..n) into c->pos; returns the total (synchronises).
uint32_t scan_count(hfcr_ctx *c, const uint32_t *flags, int64_t n) {
  ensure(c->pos, n * sizeof(uint32_t));
  ensure(c->bsums, scan_block_sums_entries(n) * sizeof(uint32_t));
  Counters *dc = ptr<Counters>(c->ctr);
  scan_u32(flags, ptr<uint32_t>(c->pos), n, ptr<uint32_t>(c->bsums), &dc->total, c->s);
  readback(c);
  return c->hctr->total;
}

struct Pair {
  MeshDev m[2];
  int orientation;
  int dirs[2];
  int ndirs;
  HitLayout hl;
  StencilLayout sl;
  bool tier0;
  bool dirty[2];
  bool has_edges[2], has_bvh[2];
  int64_t hit_cap[2], amb_cap[2], cand_cap[2];
  int64_t hits_n[2];
  // sums over the accepted detection passes
  int64_t cand = 0, f32_unsure = 0, exact = 0, visits = 0;
};

void check_mesh(const hfcr_mesh *m, const char *name) {
  if (!m) throw StatusError{HFCR_E_INVALID, std::string("mesh ") + name + " is NULL"};
  if (m->dtype != HFCR_F32 && m->dtype != HFCR_F64)
    throw StatusError{HFCR_E_INVALID, std::string("mesh ") + name + ": bad dtype"};
  if (m->nv < 0 || m->nt < 0) throw StatusError{HFCR_E_INVALID, std::string("mesh ") + name + ": negative count"};
  if (m->nt >= (1 << 24)) throw StatusError{HFCR_E_INVALID, std::string("mesh ") + name + ": more than 2^24-1 triangles"};
  if (m->nv >= (1 << 28)) throw StatusError{HFCR_E_INVALID, std::string("mesh ") + name + ": more than 2^28-1 vertices"};
  if ((m->nv > 0 && !m->pos) || (m->nt > 0 && !m->tri))
    throw StatusError{HFCR_E_INVALID, std::string("mesh ") + name + ": NULL array"};
}

void setup_mesh(hfcr_ctx *c, Pair &P, int i, const hfcr_mesh *src, const double *inv_mass) {
  MeshDev &m = P.m[i];
  m.nv = src->nv;
  m.nt = src->nt;
  m.ne = 0;
  m.f32 = src->dtype == HFCR_F32;
  m.pos_in = src->pos;
  m.tri_in = src->tri;
  m.inv_mass = inv_mass;
  ensure(c->x64[i], (size_t)3 * m.nv * sizeof(double));
  m.x64 = ptr<double>(c->x64[i]);
  if (m.f32) {
    ensure(c->x32[i], (size_t)3 * m.nv * sizeof(float));
    m.x32 = ptr<float>(c->x32[i]);
  } else {
    m.x32 = nullptr;
  }
  Counters *dc = ptr<Counters>(c->ctr);
  launch_ingest(m, &dc->err, &dc->maxabs[i], c->s);
}

// Points mesh i's edge fields at the context's buffers (sized for ne edges).
void bind_edges(hfcr_ctx *c, Pair &P, int i, int64_t ne) {
  MeshDev &m = P.m[i];
  m.ne = (int)ne;
  ensure(c->edges[i], std::max<int64_t>(ne, 1) * sizeof(int2));
  ensure(c->qedges[i], std::max<int64_t>(ne, 1) * sizeof(int4));
  m.edges = ptr<int2>(c->edges[i]);
  m.qedges = ptr<int4>(c->qedges[i]);
}

void build_edges(hfcr_ctx *c, Pair &P, int i) {
  MeshDev &m = P.m[i];
  const int64_t n = 3 * (int64_t)m.nt;
  if (n == 0) {
    m.ne = 0;
    return;
  }
  ensure(c->sk0, n * sizeof(uint64_t));
  ensure(c->flags, n * sizeof(uint32_t));
  uint64_t *keys = ptr<uint64_t>(c->sk0);
  launch_edge_keys(m, keys, c->s);
  sort_inplace(c, keys, nullptr, n, 32 + bits_for((int64_t)m.nv + 1));
  launch_unique_flags(keys, n, (uint64_t)m.nv << 32, ptr<uint32_t>(c->flags), c->s);
  const uint32_t ne = scan_count(c, ptr<uint32_t>(c->flags), n);
  bind_edges(c, P, i, ne);
  launch_compact_edges(keys, ptr<uint32_t>(c->flags), ptr<uint32_t>(c->pos), n, m.edges, c->s);
  if (ne == 0) return;
  // queries in Morton order of the edge midpoints
  ensure(c->scene_box[i], 6 * sizeof(float));
  launch_bounds(m, ptr<float>(c->scene_box[i]), c->s);
  ensure(c->sk0, (size_t)ne * sizeof(uint64_t));
  launch_edge_morton(m, ptr<float>(c->scene_box[i]), ptr<uint64_t>(c->sk0), c->s);
  sort_inplace(c, ptr<uint64_t>(c->sk0), nullptr, ne, -62);
  launch_make_qedges(m, ptr<uint64_t>(c->sk0), c->s);
  P.has_edges[i] = true;
}

// Points mesh i's BVH fields at the context's buffers.
void bind_bvh(hfcr_ctx *c, Pair &P, int i) {
  MeshDev &m = P.m[i];
  const int nt = m.nt;
  ensure(c->leaf_tri[i], std::max(nt, 1) * sizeof(int4));
  ensure(c->nodes[i], std::max(nt, 1) * sizeof(BvhNode));
  ensure(c->leaf_parent[i], std::max(nt, 1) * sizeof(int));
  ensure(c->counters_n[i], std::max(nt, 1) * sizeof(int), /*zero=*/true);
  ensure(c->root_box[i], 8 * sizeof(float));
  ensure(c->codes[i], std::max(nt, 1) * sizeof(uint32_t));
  ensure(c->scene_box[i], 6 * sizeof(float));
  m.leaf_tri = ptr<int4>(c->leaf_tri[i]);
  m.nodes = ptr<BvhNode>(c->nodes[i]);
  m.leaf_parent = ptr<int>(c->leaf_parent[i]);
  m.counters = ptr<int>(c->counters_n[i]);
  m.root_box = ptr<float>(c->root_box[i]);
  // range (2 ints), top_pos, top_list, top_pre per node, and the top count
  ensure(c->topo[i], ((size_t)5 * std::max(nt, 1) + 4) * sizeof(int));
  int *tb = ptr<int>(c->topo[i]);
  const size_t n1 = std::max(nt, 1);
  m.range = reinterpret_cast<int2 *>(tb);
  m.top_pos = tb + 2 * n1;
  m.top_list = tb + 3 * n1;
  m.top_pre = tb + 4 * n1;
  m.top_count = tb + 5 * n1;
}

void build_bvh(hfcr_ctx *c, Pair &P, int i) {
  MeshDev &m = P.m[i];
  const int nt = m.nt;
  bind_bvh(c, P, i);
  if (nt == 0) return;
  launch_bounds(m, ptr<float>(c->scene_box[i]), c->s);
  ensure(c->sk0, (size_t)nt * sizeof(uint64_t));
  launch_face_morton(m, ptr<float>(c->scene_box[i]), ptr<uint64_t>(c->sk0), c->s);
  sort_inplace(c, ptr<uint64_t>(c->sk0), nullptr, nt, -62);
  launch_leaf_tri(m, ptr<uint64_t>(c->sk0), ptr<uint32_t>(c->codes[i]), c->s);
  launch_build_tree(m, ptr<uint32_t>(c->codes[i]), c->s);
  P.has_bvh[i] = true;
  P.dirty[i] = true;
}

static_assert(sizeof(Counters) % 4 == 0 && sizeof(PassCount) % 4 == 0, "counters are zeroed as 32-bit words");
void reset_counters(hfcr_ctx *c) {
  launch_zero_words(ptr<uint32_t>(c->ctr), (int)(sizeof(Counters) / 4), c->s);
}

// Launches one detection pass in direction dir (refitting the face side's
// tree first if its positions changed); the counts are read back later.
void detect_launch(hfcr_ctx *c, Pair &P, int dir) {
  const int ei = dir == 0 ? 0 : 1, fi = dir == 0 ? 1 : 0;
  MeshDev &E = P.m[ei], &F = P.m[fi];
  if (P.dirty[fi]) {
    Scope t(c, 1);
    launch_refit(F, c->s);
    P.dirty[fi] = false;
  }
  Counters *dc = ptr<Counters>(c->ctr);
  ensure(c->hk[dir], P.hit_cap[dir] * sizeof(uint64_t));
  ensure(c->hv[dir], P.hit_cap[dir] * sizeof(uint32_t));
  ensure(c->amb[dir], P.amb_cap[dir] * sizeof(uint2));
  ensure(c->cand, P.cand_cap[dir] * sizeof(uint2));
  // use all of what earlier calls allocated
  P.hit_cap[dir] = std::max<int64_t>(P.hit_cap[dir], (int64_t)std::min(c->hk[dir].bytes / sizeof(uint64_t),
                                                                       c->hv[dir].bytes / sizeof(uint32_t)));
  P.amb_cap[dir] = std::max<int64_t>(P.amb_cap[dir], (int64_t)(c->amb[dir].bytes / sizeof(uint2)));
  P.cand_cap[dir] = std::max<int64_t>(P.cand_cap[dir], (int64_t)(c->cand.bytes / sizeof(uint2)));
  PassCount *pc = &dc->pass[dir];
  launch_zero_words(reinterpret_cast<uint32_t *>(pc), (int)(sizeof(PassCount) / 4), c->s);
  DcdOut out;
  out.keys = ptr<uint64_t>(c->hk[dir]);
  out.vals = ptr<uint32_t>(c->hv[dir]);
  out.count = &pc->hits;
  out.cap = P.hit_cap[dir];
  out.amb = ptr<uint2>(c->amb[dir]);
  out.amb_count = &pc->amb;
  out.amb_cap = P.amb_cap[dir];
  out.cand = &pc->cand;
  out.f32_unsure = &pc->f32_unsure;
  out.exact = &pc->exact;
  out.visits = &pc->visits;
  out.max_path = &dc->max_path;
  out.overflow = &dc->overflow;
  out.warm = c->tune.trav_warm;
  out.cand_buf = ptr<uint2>(c->cand);
  out.cand_count = &pc->cand_n;
  out.cand_cap = P.cand_cap[dir];
  {
    Scope t(c, 2);
    launch_traverse(E, F, dir, P.tier0, P.hl, out, c->tune.trav_block, c->s);
  }
  {
    Scope t(c, 3);
    launch_narrow(E, F, dir, P.tier0, P.hl, out, c->s);
    launch_exact(E, F, dir, P.hl, out, c->s);
  }
}

// After the readback that follows detect_launch: whether the pass fit its
// buffers (then its counts are added to the pair's and its hit count kept);
// otherwise the capacities grow for a redo.
bool detect_accept(hfcr_ctx *c, Pair &P, int dir) {
  if (c->hctr->overflow & 1) throw StatusError{HFCR_E_DEVICE, "BVH traversal stack overflow"};
  const PassCount &hp = c->hctr->pass[dir];
  const int64_t nh = hp.hits, na = hp.amb, nc = hp.cand_n;
  if (nc <= P.cand_cap[dir] && nh <= P.hit_cap[dir] && na <= P.amb_cap[dir]) {
    P.cand += (int64_t)hp.cand;
    P.f32_unsure += (int64_t)hp.f32_unsure;
    P.exact += (int64_t)hp.exact;
    P.visits += (int64_t)hp.visits;
    P.hits_n[dir] = nh;
    return true;
  }
  P.hit_cap[dir] = std::max<int64_t>(P.hit_cap[dir], nh + nh / 2 + 64);
  P.amb_cap[dir] = std::max<int64_t>(P.amb_cap[dir], na + na / 2 + 64);
  P.cand_cap[dir] = std::max<int64_t>(P.cand_cap[dir], nc + nc / 8 + 64);
  return false;
}

// One detection pass in direction dir; leaves the hits in hk/hv[dir], sorted
// when `sorted` (the order only matters for the returned round-0 list: the
// stencils built from later rounds are sorted and made unique anyway).
int64_t detect_dir(hfcr_ctx *c, Pair &P, int dir, bool sorted = true) {
  for (int attempt = 0; attempt < 8; ++attempt) {
    detect_launch(c, P, dir);
    readback(c);
    if (detect_accept(c, P, dir)) {
      Scope t(c, 4);
      if (sorted) sort_inplace(c, ptr<uint64_t>(c->hk[dir]), ptr<uint32_t>(c->hv[dir]), P.hits_n[dir],
                               1 + P.hl.bits_e + P.hl.bits_f);
      return P.hits_n[dir];
    }
  }
  throw StatusError{HFCR_E_DEVICE, "hit buffer did not converge"};
}

// Room for the one-launch stencil and zone stage of up to kRoundSmallHits hits.
void ensure_round_small(hfcr_ctx *c, const Pair &P) {
  ensure(c->st_keys, kRoundSmallHits * sizeof(uint64_t));
  ensure(c->con, kRoundSmallHits * sizeof(Constraint));
  ensure(c->zkeys, kRoundSmallHits * sizeof(uint64_t));
  ensure(c->zvals, kRoundSmallHits * sizeof(uint32_t));
  ensure(c->starts, (kRoundSmallHits + 1) * sizeof(uint32_t));
}

void launch_round_small(hfcr_ctx *c, Pair &P, const int *dirs, int nd, double d) {
  Counters *dc = ptr<Counters>(c->ctr);
  const int d0 = dirs[0], d1 = nd > 1 ? dirs[1] : dirs[0];
  Scope t(c, 5);
  launch_round_small(ptr<uint64_t>(c->hk[d0]), ptr<uint32_t>(c->hv[d0]), &dc->pass[d0].hits, P.hit_cap[d0],
                     ptr<uint64_t>(c->hk[d1]), ptr<uint32_t>(c->hv[d1]), nd > 1 ? &dc->pass[d1].hits : nullptr,
                     P.hit_cap[d1], P.hl, P.sl, P.m[0], P.m[1], d, ptr<uint64_t>(c->st_keys), ptr<Constraint>(c->con),
                     ptr<uint64_t>(c->zkeys), ptr<uint32_t>(c->zvals), ptr<uint32_t>(c->starts), &dc->nzones,
                     &dc->maxk, &dc->total, c->s);
}

// Detection passes of the directions dirs[0..nd) followed at once by the
// one-launch stencil and zone stage on their hits, with a single readback.
// Every pass that overflowed its buffers is redone.  Returns whether the
// stage's results stand (every pass fit the first time; the stage itself ran
// only for 1..kRoundSmallHits hits).
bool detect_and_round_small(hfcr_ctx *c, Pair &P, const int *dirs, int nd, double d) {
  for (int q = 0; q < nd; ++q) detect_launch(c, P, dirs[q]);
  ensure_round_small(c, P);
  launch_round_small(c, P, dirs, nd, d);
  readback(c);
  bool fit[2] = {true, true};
  for (int q = 0; q < nd; ++q) fit[q] = detect_accept(c, P, dirs[q]);
  bool ok = true;
  for (int q = 0; q < nd; ++q)
    if (!fit[q]) {
      detect_dir(c, P, dirs[q], false);
      ok = false;
    }
  return ok;
}

// Unique stencil keys of the hits of the listed directions into c->st_keys.
int64_t build_stencils(hfcr_ctx *c, Pair &P, const int *dirs, int nd, DBuf &dst) {
  int64_t n = 0;
  for (int q = 0; q < nd; ++q) n += P.hits_n[dirs[q]];
  if (n == 0) return 0;
  {
    const int d0 = dirs[0], d1 = nd > 1 ? dirs[1] : dirs[0];
    const int64_t n1 = nd > 1 ? P.hits_n[d1] : 0;
    ensure(dst, n * sizeof(uint64_t));
    Counters *dc = ptr<Counters>(c->ctr);
    if (launch_stencils_small(ptr<uint64_t>(c->hk[d0]), ptr<uint32_t>(c->hv[d0]), P.hits_n[d0],
                              ptr<uint64_t>(c->hk[d1]), ptr<uint32_t>(c->hv[d1]), n1, P.hl, P.sl, ptr<uint64_t>(dst),
                              &dc->total, c->s)) {
      readback(c);
      return c->hctr->total;
    }
  }
  ensure(c->sk0, n * sizeof(uint64_t));
  ensure(c->flags, n * sizeof(uint32_t));
  int64_t off = 0;
  for (int q = 0; q < nd; ++q) {
    const int dir = dirs[q];
    launch_stencil_keys(ptr<uint64_t>(c->hk[dir]), ptr<uint32_t>(c->hv[dir]), P.hits_n[dir], P.hl, P.sl,
                        ptr<uint64_t>(c->sk0) + off, c->s);
    off += P.hits_n[dir];
  }
  sort_inplace(c, ptr<uint64_t>(c->sk0), nullptr, n, 1 + P.sl.bits_v + P.sl.bits_f);
  launch_unique_flags(ptr<uint64_t>(c->sk0), n, ~0ull, ptr<uint32_t>(c->flags), c->s);
  const uint32_t S = scan_count(c, ptr<uint32_t>(c->flags), n);
  ensure(dst, std::max<int64_t>(S, 1) * sizeof(uint64_t));
  launch_compact_keys(ptr<uint64_t>(c->sk0), ptr<uint32_t>(c->flags), ptr<uint32_t>(c->pos), n, ptr<uint64_t>(dst),
                      c->s);
  return S;
}

struct RoundInfo {
  int64_t S = 0;
  int nzones = 0;
  int maxk = 0;
};

// Stencils, constraints, impact zones, solve and update of one round for the
// hits of the active directions act[0..nact).  `staged`: the one-launch
// stencil and zone stage already ran on these hits and its counts are in the
// last readback.
RoundInfo respond(hfcr_ctx *c, Pair &P, const int *act, int nact, double d, hfcr_stats *st, bool staged) {
  RoundInfo info;
  Counters *dc = ptr<Counters>(c->ctr);
  const int nvt = P.m[0].nv + P.m[1].nv;
  const int64_t nh = P.hits_n[act[0]] + (nact > 1 ? P.hits_n[act[1]] : 0);
  bool fused = staged;
  if (!staged && nh <= kRoundSmallHits) {
    // stencils, constraints and zones in one launch, and one readback for
    // their counts
    ensure_round_small(c, P);
    launch_round_small(c, P, act, nact, d);
    fused = true;
  }
  int64_t S = 0;
  if (!fused) {
    ensure(c->parent, (size_t)std::max(nvt, 1) * sizeof(int));
    S = build_stencils(c, P, act, nact, c->st_keys);
    const int bits_s = bits_for(S);
    {
      Scope t(c, 4);
      ensure(c->con, S * sizeof(Constraint));
      launch_constraints(ptr<uint64_t>(c->st_keys), S, P.sl, P.m[0], P.m[1], d, ptr<Constraint>(c->con), c->s);
    }
    Scope t(c, 5);
    ensure(c->zkeys, S * sizeof(uint64_t));
    ensure(c->zvals, S * sizeof(uint32_t));
    ensure(c->starts, (S + 1) * sizeof(uint32_t));
    if (!launch_zones_small(ptr<Constraint>(c->con), S, bits_s, ptr<uint64_t>(c->zkeys), ptr<uint32_t>(c->zvals),
                            ptr<uint32_t>(c->starts), &dc->nzones, &dc->maxk, c->s)) {
      launch_uf_init(ptr<int>(c->parent), nvt, &dc->maxk, c->s);
      launch_uf_union(ptr<Constraint>(c->con), S, ptr<int>(c->parent), c->s);
      launch_zone_keys(ptr<Constraint>(c->con), S, ptr<int>(c->parent), bits_s, ptr<uint64_t>(c->zkeys),
                       ptr<uint32_t>(c->zvals), c->s);
      sort_inplace(c, ptr<uint64_t>(c->zkeys), ptr<uint32_t>(c->zvals), S, bits_s + bits_for(nvt));
      ensure(c->flags, S * sizeof(uint32_t));
      ensure(c->pos, S * sizeof(uint32_t));
      ensure(c->bsums, scan_block_sums_entries(S) * sizeof(uint32_t));
      launch_zone_flags(ptr<uint64_t>(c->zkeys), S, bits_s, ptr<uint32_t>(c->flags), c->s);
      scan_u32(ptr<uint32_t>(c->flags), ptr<uint32_t>(c->pos), S, ptr<uint32_t>(c->bsums), nullptr, c->s);
      launch_zone_starts(ptr<uint32_t>(c->flags), ptr<uint32_t>(c->pos), S, ptr<uint32_t>(c->starts),
                         &dc->nzones, &dc->maxk, c->s);
    }
  }
  if (!staged) readback(c);
  if (fused) S = c->hctr->total;
  info.S = S;
  const int bits_s = bits_for(S);
  info.nzones = (int)c->hctr->nzones;
  info.maxk = (int)c->hctr->maxk;
  if (info.maxk > HFCR_MAX_ZONE)
    throw StatusError{HFCR_E_ZONE_LIMIT, "impact zone of " + std::to_string(info.maxk) + " stencils exceeds " +
                                             std::to_string(HFCR_MAX_ZONE)};
  {
    Scope t(c, 6);
    const int64_t stride = (int64_t)solve_slot_doubles(info.maxk);
    const int64_t budget = (int64_t)1 << 28;       // doubles (2 GiB) across slots
    int nslots = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)info.nzones, 2048, budget / stride}));
    ensure(c->solve_scratch, (size_t)nslots * stride * sizeof(double));
    ensure(c->lambda, S * sizeof(double));
    ensure(c->retry, (size_t)info.nzones * sizeof(uint32_t));
    SolveArgs a;
    a.con = ptr<Constraint>(c->con);
    a.order = ptr<uint32_t>(c->zvals);
    a.starts = ptr<uint32_t>(c->starts);
    a.nzones = info.nzones;
    a.w_a = P.m[0].inv_mass;
    a.w_b = P.m[1].inv_mass;
    a.nv_a = P.m[0].nv;
    a.lambda = ptr<double>(c->lambda);
    a.scratch = ptr<double>(c->solve_scratch);
    a.slot_stride = stride;
    a.nslots = nslots;
    a.rank_def = &dc->rank_def;
    a.pivoted = &dc->pivoted;
    a.retry = ptr<uint32_t>(c->retry);
    a.retry_n = &dc->retry_n;
    a.tau = 1e-12;
    a.maxk = info.maxk;
    launch_solve(a, c->s);
  }
  {
    Scope t(c, 7);
    if (!launch_update_small(ptr<Constraint>(c->con), S, bits_s, ptr<double>(c->lambda), P.m[0], P.m[1], c->s)) {
      ensure(c->inc_keys, 4 * S * sizeof(uint64_t));
      launch_incidence(ptr<Constraint>(c->con), S, bits_s, ptr<uint64_t>(c->inc_keys), c->s);
      sort_inplace(c, ptr<uint64_t>(c->inc_keys), nullptr, 4 * S, bits_s + 2 + bits_for(nvt));
      launch_update(ptr<uint64_t>(c->inc_keys), 4 * S, bits_s, ptr<Constraint>(c->con), ptr<double>(c->lambda),
                    P.m[0], P.m[1], c->s);
    }
  }
  P.dirty[0] = P.dirty[1] = true;
  if (st) st->max_zone = std::max(st->max_zone, info.maxk);
  return info;
}

void write_hit_outputs(hfcr_ctx *c, Pair &P, hfcr_result *res, hfcr_stats *st, bool &truncated) {
  // round-0 hits of every oriented direction, sorted (direction is the key's top bit)
  int64_t total = 0;
  for (int q = 0; q < P.ndirs; ++q) total += P.hits_n[P.dirs[q]];
  if (st) st->hits0 = total;
  if (res && res->hits && total > 0) {
    int64_t off = 0;
    for (int q = 0; q < P.ndirs; ++q) {
      const int dir = P.dirs[q];
      int64_t n = P.hits_n[dir];
      int64_t room = std::max<int64_t>(0, res->hit_cap - off);
      int64_t m = std::min(n, room);
      launch_write_hits(ptr<uint64_t>(c->hk[dir]), ptr<uint32_t>(c->hv[dir]), m, P.hl, P.m[0].edges, P.m[1].edges,
                        res->hits + 5 * off, c->s);
      off += n;
    }
    if (total > res->hit_cap) truncated = true;
  }
  const int64_t S0 = build_stencils(c, P, P.dirs, P.ndirs, c->st_out_keys);
  if (st) st->stencils0 = S0;
  if (res && res->stencils && S0 > 0) {
    launch_write_stencils(ptr<uint64_t>(c->st_out_keys), std::min<int64_t>(S0, res->stencil_cap), P.sl,
                          res->stencils, c->s);
    if (S0 > res->stencil_cap) truncated = true;
  }
}

void setup_pair(hfcr_ctx *c, Pair &P, const hfcr_mesh *a, const hfcr_mesh *b, int orientation,
                const hfcr_opts *o) {
  check_mesh(a, "A");
  check_mesh(b, "B");
  if (orientation < HFCR_ORIENT_B || orientation > HFCR_ORIENT_BOTH)
    throw StatusError{HFCR_E_INVALID, "bad orientation"};
  P.orientation = orientation;
  if (orientation == HFCR_ORIENT_B) {
    P.dirs[0] = 0;
    P.ndirs = 1;
  } else if (orientation == HFCR_ORIENT_A) {
    P.dirs[0] = 1;
    P.ndirs = 1;
  } else {
    P.dirs[0] = 0;
    P.dirs[1] = 1;
    P.ndirs = 2;
  }
  P.tier0 = o->predicate_tier == 0;
  for (int i = 0; i < 2; ++i) {
    P.dirty[i] = false;
    P.has_edges[i] = P.has_bvh[i] = false;
    P.hit_cap[i] = 4096;
    P.amb_cap[i] = 4096;
    P.cand_cap[i] = 1 << 16;
    P.hits_n[i] = 0;
  }
  ensure(c->ctr, sizeof(Counters));
  reset_counters(c);
  {
    Scope t(c, 0);
    setup_mesh(c, P, 0, a, o->inv_mass_a);
    setup_mesh(c, P, 1, b, o->inv_mass_b);
    Counters *dc = ptr<Counters>(c->ctr);
    bool cached[2];
    for (int i = 0; i < 2; ++i) {
      const hfcr_ctx::TopoCache &tc = c->topo_cache[i];
      const MeshDev &m = P.m[i];
      cached[i] = tc.nv == m.nv && tc.nt == m.nt && m.nt > 0 && (tc.edges || tc.bvh);
      if (cached[i]) launch_tri_diff(m.tri_in, ptr<int32_t>(c->tri_cache[i]), 3 * (int64_t)m.nt, &dc->tri_diff[i], c->s);
    }
    readback(c);
    if (c->hctr->err & 1u)
      throw StatusError{HFCR_E_INVALID, "non-finite or out-of-domain coordinate (|x| must be 0 or in [2^-200, 2^200])"};
    if (c->hctr->err & 2u) throw StatusError{HFCR_E_INVALID, "triangle index out of range"};
    for (int i = 0; i < 2; ++i) {
      float m;
      std::memcpy(&m, &c->hctr->maxabs[i], sizeof(float));
      P.m[i].small_coords = m <= 4294967296.0f;
    }
    // the edge sets, query orders and BVH trees of the previous call stay
    // valid while the triangle arrays are unchanged (refitting takes care of
    // the new positions; the hits do not depend on the tree's shape)
    bool built[2] = {false, false};
    for (int i = 0; i < 2; ++i)
      if (!(cached[i] && c->hctr->tri_diff[i] == 0)) c->topo_cache[i] = hfcr_ctx::TopoCache{};
    for (int q = 0; q < P.ndirs; ++q) {
      const int dir = P.dirs[q];
      const int ei = dir == 0 ? 0 : 1, fi = dir == 0 ? 1 : 0;
      if (!P.has_edges[ei]) {
        if (c->topo_cache[ei].edges) {
          bind_edges(c, P, ei, c->topo_cache[ei].ne);
          P.has_edges[ei] = true;
        } else {
          build_edges(c, P, ei);
          built[ei] = true;
          P.has_edges[ei] = true;
        }
      }
      if (!P.has_bvh[fi]) {
        if (c->topo_cache[fi].bvh) {
          bind_bvh(c, P, fi);
          P.has_bvh[fi] = true;
          P.dirty[fi] = true;
        } else {
          build_bvh(c, P, fi);
          built[fi] = true;
        }
      }
    }
    for (int i = 0; i < 2; ++i) {
      if (!built[i]) continue;
      hfcr_ctx::TopoCache &tc = c->topo_cache[i];
      if (tc.nt != P.m[i].nt || tc.nv != P.m[i].nv) {  // new content: keep a copy of the triangles
        ensure(c->tri_cache[i], std::max<int64_t>(3 * (int64_t)P.m[i].nt, 1) * sizeof(int32_t));
        HIP_CHECK(hipMemcpyAsync(c->tri_cache[i].p, P.m[i].tri_in, 3 * (size_t)P.m[i].nt * sizeof(int32_t),
                                 hipMemcpyDeviceToDevice, c->s));
      }
      tc.nv = P.m[i].nv;
      tc.nt = P.m[i].nt;
      if (P.has_edges[i]) {  // built or bound in this call; else keep what the cache holds
        tc.ne = P.m[i].ne;
        tc.edges = true;
      }
      tc.bvh = tc.bvh || P.has_bvh[i];
    }
  }
  int64_t maxe = std::max(P.m[0].ne, P.m[1].ne), maxf = std::max(P.m[0].nt, P.m[1].nt);
  int64_t maxv = std::max(P.m[0].nv, P.m[1].nv);
  P.hl.bits_f = bits_for(maxf);
  P.hl.bits_e = bits_for(maxe);
  P.sl.bits_f = P.hl.bits_f;
  P.sl.bits_v = bits_for(maxv);
}

void finish_timing(hfcr_ctx *c, hfcr_stats *st) {
  if (!c->timers.empty()) {
    HIP_CHECK(hipStreamSynchronize(c->s));
    for (auto &t : c->timers) {
      float ms = 0.f;
      HIP_CHECK(hipEventElapsedTime(&ms, t.a, t.b));
      if (st) {
        st->stage_ms[t.stage] += ms;
        st->stage_calls[t.stage] += 1;
      }
      c->free_events.push_back(t.a);
      c->free_events.push_back(t.b);
    }
    c->timers.clear();
  }
}

template <typename F>
hfcr_status guarded(hfcr_ctx *c, F &&body) {
  if (!c) return HFCR_E_INVALID;
  int prev = 0;
  (void)hipGetDevice(&prev);
  hfcr_status st = HFCR_OK;
  try {
    HIP_CHECK(hipSetDevice(c->device));
    st = body();
  } catch (const StatusError &e) {
    c->err = e.msg;
    st = e.st;
  } catch (const HipError &e) {
    c->err = std::string(e.what) + ": " + hipGetErrorString(e.e);
    st = HFCR_E_DEVICE;
  }
  // release timers on error paths too
  for (auto &t : c->timers) {
    c->free_events.push_back(t.a);
    c->free_events.push_back(t.b);
  }
  c->timers.clear();
  (void)hipSetDevice(prev);
  return st;
}

}  // namespace

extern "C" {

void hfcr_default_opts(hfcr_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->max_rounds = 256;
  o->both_mode = HFCR_BOTH_ALTERNATE;
  o->predicate_tier = 0;
  o->round_offset = 0;
}

hfcr_status hfcr_create(hfcr_ctx **out, int device) {
  if (!out) return HFCR_E_INVALID;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return HFCR_E_DEVICE;
  hfcr_ctx *c = new hfcr_ctx();
  c->device = device;
  hfcr_status st = guarded(c, [&]() -> hfcr_status {
    void *h = nullptr;
    HIP_CHECK(hipHostMalloc(&h, sizeof(Counters), hipHostMallocDefault));
    c->hctr = reinterpret_cast<Counters *>(h);
    ensure(c->ctr, sizeof(Counters), true);
    return HFCR_OK;
  });
  if (st != HFCR_OK) {
    hfcr_destroy(c);
    return st;
  }
  *out = c;
  return HFCR_OK;
}

void hfcr_destroy(hfcr_ctx *c) {
  if (!c) return;
  for (hfcr_ctx *w : c->workers) hfcr_destroy(w);
  int prev = 0;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (hipStream_t s : c->wstreams) (void)hipStreamDestroy(s);
  DBuf *all[] = {&c->sk0, &c->sk1, &c->sv0, &c->sv1, &c->hist, &c->flags, &c->pos, &c->bsums, &c->st_keys,
                 &c->st_out_keys, &c->con, &c->parent, &c->zkeys, &c->zvals, &c->starts, &c->lambda, &c->inc_keys,
                 &c->solve_scratch, &c->ctr, &c->cand, &c->retry};
  for (DBuf *b : all)
    if (b->p) (void)hipFree(b->p);
  for (int i = 0; i < 2; ++i) {
    DBuf *m[] = {&c->x64[i], &c->x32[i], &c->edges[i], &c->qedges[i], &c->leaf_tri[i], &c->nodes[i],
                 &c->leaf_parent[i], &c->counters_n[i], &c->root_box[i], &c->codes[i], &c->scene_box[i], &c->topo[i],
                 &c->hk[i], &c->hv[i], &c->amb[i], &c->tri_cache[i]};
    for (DBuf *b : m)
      if (b->p) (void)hipFree(b->p);
  }
  if (c->hctr) (void)hipHostFree(c->hctr);
  for (hipEvent_t e : c->free_events) (void)hipEventDestroy(e);
  (void)hipSetDevice(prev);
  delete c;
}

const char *hfcr_last_error(const hfcr_ctx *c) { return c ? c->err.c_str() : "null context"; }

hfcr_status hfcr_detect(hfcr_ctx *c, const hfcr_mesh *a, const hfcr_mesh *b, int32_t orientation,
                        const hfcr_opts *opts, hfcr_result *res, void *stream) {
  return guarded(c, [&]() -> hfcr_status {
    hfcr_opts o;
    hfcr_default_opts(&o);
    if (opts) o = *opts;
    c->s = (hipStream_t)stream;
    hfcr_stats *st = res ? res->stats : nullptr;
    if (st) std::memset(st, 0, sizeof(*st));
    c->timing = (o.flags & HFCR_FLAG_TIMING) != 0;
    Pair P;
    setup_pair(c, P, a, b, orientation, &o);
    for (int q = 0; q < P.ndirs; ++q) detect_dir(c, P, P.dirs[q]);
    bool truncated = false;
    write_hit_outputs(c, P, res, st, truncated);
    readback(c);
    if (st) {
      st->candidates = P.cand;
      st->exact_tests = P.exact;
      st->f32_ambiguous = P.f32_unsure;
      st->node_visits = P.visits;
      st->max_query_path = (int32_t)c->hctr->max_path;
      st->converged = st->hits0 == 0;
      st->residual_hits = st->hits0;
    }
    finish_timing(c, st);
    return truncated ? HFCR_E_CAPACITY : HFCR_OK;
  });
}

hfcr_status hfcr_resolve(hfcr_ctx *c, const hfcr_mesh *a, const hfcr_mesh *b, int32_t orientation, double d,
                         const hfcr_opts *opts, hfcr_result *res, void *stream) {
  return guarded(c, [&]() -> hfcr_status {
    hfcr_opts o;
    hfcr_default_opts(&o);
    if (opts) o = *opts;
    if (!(d >= 0.0) || !std::isfinite(d)) throw StatusError{HFCR_E_INVALID, "d must be finite and >= 0"};
    if (o.max_rounds < 0) throw StatusError{HFCR_E_INVALID, "max_rounds must be >= 0"};
    if (o.both_mode != HFCR_BOTH_ALTERNATE && o.both_mode != HFCR_BOTH_SIMULTANEOUS)
      throw StatusError{HFCR_E_INVALID, "bad both_mode"};
    c->s = (hipStream_t)stream;
    hfcr_stats *st = res ? res->stats : nullptr;
    if (st) std::memset(st, 0, sizeof(*st));
    c->timing = (o.flags & HFCR_FLAG_TIMING) != 0;
    Pair P;
    setup_pair(c, P, a, b, orientation, &o);
    const bool alternate = orientation == HFCR_ORIENT_BOTH && o.both_mode == HFCR_BOTH_ALTERNATE;
    bool converged = false, truncated = false;
    int rounds = 0;
    int64_t residual = 0;
    hfcr_status status = HFCR_OK;
    try {
      for (int r = 0; r <= o.max_rounds; ++r) {
        int act[2], nact = 0;
        int64_t nhits = 0, nf = 0, ns = 0;
        bool second_done = false;
        const int first = (int)(((int64_t)r + o.round_offset) & 1);
        // rounds after the first (and before the last) start the stencil and
        // zone stage right behind detection; it stands when the round's hits
        // fit it
        const bool speculate = r > 0 && r < o.max_rounds;
        bool fit = false, staged = false;
        if (speculate) {
          int sd[2], nsd = 0;
          if (alternate) sd[nsd++] = first;
          else
            for (int q = 0; q < P.ndirs; ++q) sd[nsd++] = P.dirs[q];
          fit = detect_and_round_small(c, P, sd, nsd, d);
        }
        if (alternate) {
          nf = speculate ? P.hits_n[first] : detect_dir(c, P, first, r == 0);
          second_done = r == 0 || nf == 0;
          if (second_done) ns = detect_dir(c, P, 1 - first, r == 0);
          else P.hits_n[1 - first] = 0;
          if (r == 0) write_hit_outputs(c, P, res, st, truncated);
          if (nf > 0) {
            act[nact++] = first;
            nhits = nf;
          } else if (ns > 0) {
            act[nact++] = 1 - first;
            nhits = ns;
          }
        } else {
          for (int q = 0; q < P.ndirs; ++q) {
            const int dir = P.dirs[q];
            const int64_t n = speculate ? P.hits_n[dir] : detect_dir(c, P, dir, r == 0);
            if (n > 0) {
              act[nact++] = dir;
              nhits += n;
            }
          }
          if (r == 0) write_hit_outputs(c, P, res, st, truncated);
        }
        // the staged results belong to the active hits only if no other
        // detection or readback came between
        staged = fit && nhits > 0 && nhits <= kRoundSmallHits && (!alternate || nf > 0);
        if (st && r < HFCR_STAT_ROUNDS) st->round_hits[r] = (int32_t)nhits;
        if (nact == 0) {
          converged = true;
          break;
        }
        if (r == o.max_rounds) {
          // residual over every oriented direction at the final positions
          residual = nhits;
          if (alternate) residual = nf + (second_done ? ns : detect_dir(c, P, 1 - first, false));
          break;
        }
        RoundInfo info = respond(c, P, act, nact, d, st, staged);
        if (st && r < HFCR_STAT_ROUNDS) {
          st->round_stencils[r] = (int32_t)info.S;
          st->round_zones[r] = info.nzones;
          st->round_max_zone[r] = info.maxk;
        }
        ++rounds;
      }
    } catch (const StatusError &e) {
      if (e.st != HFCR_E_ZONE_LIMIT) throw;
      c->err = e.msg;
      status = HFCR_E_ZONE_LIMIT;
    }
    if (res) {
      launch_write_positions(P.m[0], res->pos_a_out, c->s);
      launch_write_positions(P.m[1], res->pos_b_out, c->s);
    }
    readback(c);
    if (st) {
      st->rounds = rounds;
      st->converged = converged ? 1 : 0;
      st->residual_hits = converged ? 0 : residual;
      st->candidates = P.cand;
      st->exact_tests = P.exact;
      st->f32_ambiguous = P.f32_unsure;
      st->rank_deficient = c->hctr->rank_def;
      st->node_visits = P.visits;
      st->max_query_path = (int32_t)c->hctr->max_path;
      st->pivoted_zones = c->hctr->pivoted;
    }
    finish_timing(c, st);
    if (status != HFCR_OK) return status;
    if (truncated) return HFCR_E_CAPACITY;
    return converged ? HFCR_OK : HFCR_NOT_CONVERGED;
  });
}

}  // extern "C"

namespace {

// The per-pair entry point on a worker's context and stream.
hfcr_status run_pair(hfcr_ctx *w, hipStream_t s, hfcr_pair &q, const hfcr_opts &o, bool detect, hfcr_stats *st) {
  hfcr_opts po = o;
  po.inv_mass_a = q.inv_mass_a;
  po.inv_mass_b = q.inv_mass_b;
  hfcr_result r = q.res;
  r.stats = st;
  if (detect) {
    r.pos_a_out = r.pos_b_out = nullptr;
    return hfcr_detect(w, &q.a, &q.b, q.orientation, &po, &r, s);
  }
  return hfcr_resolve(w, &q.a, &q.b, q.orientation, q.d, &po, &r, s);
}

void add_stats(hfcr_stats &b, const hfcr_stats &s) {
  b.rounds = std::max(b.rounds, s.rounds);
  b.converged = b.converged && s.converged;
  b.residual_hits += s.residual_hits;
  b.hits0 += s.hits0;
  b.stencils0 += s.stencils0;
  b.candidates += s.candidates;
  b.exact_tests += s.exact_tests;
  b.f32_ambiguous += s.f32_ambiguous;
  b.max_zone = std::max(b.max_zone, s.max_zone);
  b.rank_deficient += s.rank_deficient;
  b.node_visits += s.node_visits;
  b.pivoted_zones += s.pivoted_zones;
  b.max_query_path = std::max(b.max_query_path, s.max_query_path);
  for (int k = 0; k < HFCR_STAGES; ++k) {
    b.stage_ms[k] += s.stage_ms[k];
    b.stage_calls[k] += s.stage_calls[k];
  }
  for (int r = 0; r < HFCR_STAT_ROUNDS; ++r) {
    b.round_hits[r] += s.round_hits[r];
    b.round_stencils[r] += s.round_stencils[r];
    b.round_zones[r] += s.round_zones[r];
    b.round_max_zone[r] = std::max(b.round_max_zone[r], s.round_max_zone[r]);
  }
}

// Batch calls: pairs are dealt dynamically to `batch_workers` host threads,
// each driving its own context and stream, so the launches and host waits of
// different pairs overlap on the device.  Every pair runs exactly the
// single-pair path, so its results do not depend on the batch.
hfcr_status run_batch(hfcr_ctx *c, hfcr_pair *pairs, int32_t n, const hfcr_opts *opts, hfcr_stats *bst,
                      hipStream_t caller, bool detect) {
  if (n < 0 || n > HFCR_MAX_BATCH) throw StatusError{HFCR_E_INVALID, "npairs must be in [0, HFCR_MAX_BATCH]"};
  if (n > 0 && !pairs) throw StatusError{HFCR_E_INVALID, "pairs is NULL"};
  hfcr_opts o;
  hfcr_default_opts(&o);
  if (opts) o = *opts;
  // inputs produced on the caller's stream are complete before the workers start
  HIP_CHECK(hipStreamSynchronize(caller));
  const int nw = std::max(1, std::min<int>(c->tune.batch_workers, n));
  while ((int)c->workers.size() < nw) {
    hfcr_ctx *w = nullptr;
    const hfcr_status st = hfcr_create(&w, c->device);
    if (st != HFCR_OK) throw StatusError{st, "worker context creation failed"};
    w->tune = c->tune;
    hipStream_t ws = nullptr;
    const hipError_t e = hipStreamCreateWithFlags(&ws, hipStreamNonBlocking);
    if (e != hipSuccess) {
      hfcr_destroy(w);
      throw HipError{e, "hipStreamCreateWithFlags"};
    }
    c->workers.push_back(w);
    c->wstreams.push_back(ws);
  }
  std::vector<hfcr_stats> st(n);
  std::vector<std::string> msg(n);
  std::atomic<int> next{0};
  auto work = [&](int wi) {
    hfcr_ctx *w = c->workers[wi];
    w->tune = c->tune;
    for (;;) {
      const int p = next.fetch_add(1);
      if (p >= n) break;
      std::memset(&st[p], 0, sizeof(hfcr_stats));
      pairs[p].status = run_pair(w, c->wstreams[wi], pairs[p], o, detect, &st[p]);
      if (pairs[p].status < 0) msg[p] = w->err;
      if (pairs[p].res.stats) *pairs[p].res.stats = st[p];
    }
  };
  std::vector<std::thread> th;
  for (int wi = 1; wi < nw; ++wi) th.emplace_back(work, wi);
  work(0);
  for (auto &t : th) t.join();
  if (bst) {
    std::memset(bst, 0, sizeof(*bst));
    bst->converged = 1;
    for (int p = 0; p < n; ++p) add_stats(*bst, st[p]);
  }
  for (int p = 0; p < n; ++p)
    if (pairs[p].status != HFCR_OK) {
      c->err = "pair " + std::to_string(p) + ": " + (msg[p].empty() ? "did not converge" : msg[p]);
      return (hfcr_status)pairs[p].status;
    }
  return HFCR_OK;
}

}  // namespace

extern "C" {

hfcr_status hfcr_resolve_batch(hfcr_ctx *c, hfcr_pair *pairs, int32_t npairs, const hfcr_opts *opts,
                               hfcr_stats *batch_stats, void *stream) {
  return guarded(c, [&]() { return run_batch(c, pairs, npairs, opts, batch_stats, (hipStream_t)stream, false); });
}

hfcr_status hfcr_detect_batch(hfcr_ctx *c, hfcr_pair *pairs, int32_t npairs, const hfcr_opts *opts,
                              hfcr_stats *batch_stats, void *stream) {
  return guarded(c, [&]() { return run_batch(c, pairs, npairs, opts, batch_stats, (hipStream_t)stream, true); });
}

hfcr_status hfcr_get_tuning(const hfcr_ctx *c, hfcr_tuning *t) {
  if (!c || !t) return HFCR_E_INVALID;
  *t = c->tune;
  return HFCR_OK;
}

hfcr_status hfcr_set_tuning(hfcr_ctx *c, const hfcr_tuning *t) {
  if (!c || !t) return HFCR_E_INVALID;
  if (t->trav_block != 64 && t->trav_block != 128 && t->trav_block != 256) {
    c->err = "trav_block must be 64, 128 or 256";
    return HFCR_E_INVALID;
  }
  if (t->trav_warm != 0 && t->trav_warm != 1) {
    c->err = "trav_warm must be 0 or 1";
    return HFCR_E_INVALID;
  }
  if (t->batch_workers < 1 || t->batch_workers > 64) {
    c->err = "batch_workers must be in [1, 64]";
    return HFCR_E_INVALID;
  }
  c->tune = *t;
  return HFCR_OK;
}

hfcr_status hfcr_test_orient(hfcr_ctx *c, const double *pts, int64_t n, int32_t tier, int32_t *out, void *stream) {
  return guarded(c, [&]() -> hfcr_status {
    if (n < 0 || tier < 0 || tier > 2 || (n > 0 && (!pts || !out)))
      throw StatusError{HFCR_E_INVALID, "bad arguments"};
    launch_test_orient(pts, n, tier, out, (hipStream_t)stream);
    HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
    return HFCR_OK;
  });
}

}  // extern "C"
