// Discrete collision detection: every E-F intersection between the edges of
// one mesh (queries, in Morton order) and the faces of the other (leaves of
// its BVH).
//
// One lane per query edge walks the face BVH depth-first; its stack lives in
// LDS (one column per lane, so lanes of a wave hit distinct banks).  Every
// leaf whose box overlaps the segment's box is a candidate; the traversal
// only queues (query, leaf) pairs, staged in LDS and written in batches, so
// its loop carries one dependent memory access per step (the node), and a
// second kernel runs the filtered narrow phase on all queued pairs at once.  Candidates, hits and undecided pairs
// are appended with one atomic per wavefront (ballot, popcount, prefix by
// mbcnt); the order is made deterministic afterwards by sorting the keys.
#include "common.hpp"
#include "kernels.hpp"
#include "predicates.hpp"

namespace hfcr {

constexpr int kStack = 64;  // tree depth <= 30 Morton bits + 24 index bits + 1

__device__ inline uint64_t lanemask_lt() {
  const unsigned lane = __lane_id();
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

// Append for the lanes where pred holds; returns the slot (or ~0u).
__device__ inline uint32_t wave_append(uint32_t *counter, bool pred) {
  const uint64_t m = __ballot(pred);
  if (m == 0) return ~0u;
  const int leader = __ffsll((unsigned long long)m) - 1;
  uint32_t base = 0;
  if ((int)__lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
  base = (uint32_t)__shfl((int)base, leader);
  return pred ? base + (uint32_t)__popcll(m & lanemask_lt()) : ~0u;
}

__device__ inline bool box_overlap(const float lo[3], const float hi[3], float l0, float l1, float l2, float h0,
                                   float h1, float h2) {
  return lo[0] <= h0 && l0 <= hi[0] && lo[1] <= h1 && l1 <= hi[1] && lo[2] <= h2 && l2 <= hi[2];
}

// Warm this XCD's L2 with the face-side data the traversal will chase:
// workgroups are dealt to the 8 XCDs round-robin, so the workgroups that
// share an XCD split the arrays between them.  The loaded words feed a
// checksum that is consumed only on an impossible branch, which keeps the
// loads alive.
constexpr int kXcds = 8;

__device__ inline unsigned warm_l2(const void *p, int64_t bytes, unsigned acc) {
  const int64_t n16 = bytes / 16;
  const int slices = (int)((gridDim.x + kXcds - 1) / kXcds);
  const int slice = (int)(blockIdx.x / kXcds);
  const int64_t per = (n16 + slices - 1) / slices;
  const int64_t lo = slice * per, hi = lo + per < n16 ? lo + per : n16;
  const uint4 *q = reinterpret_cast<const uint4 *>(p);
  constexpr int U = 8;  // independent loads in flight per thread
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += (int64_t)U * blockDim.x) {
    uint4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + (int64_t)u * blockDim.x;
      v[u] = i < hi ? q[i] : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  return acc;
}

struct TravArgs {
  const int4 *qedges;
  int ne;
  const double *ex64;
  const float *ex32;
  int env;
  const int4 *leaf_tri;
  const BvhNode *nodes;
  const float *root_box;
  int nt;
  const double *fx64;
  const float *fx32;
  int fnv;
  int dir;
  HitLayout lay;
  DcdOut out;
  int warm;  // warm the L2 with the BVH, leaves and face positions first
};

template <bool F32>
__device__ inline void load_point(const double *x64, const float *x32, int nv, int i, P3f &pf, P3d &pd) {
  pd.x = x64[i];
  pd.y = x64[(int64_t)nv + i];
  pd.z = x64[2 * (int64_t)nv + i];
  if (F32) {
    pf.x = x32[i];
    pf.y = x32[(int64_t)nv + i];
    pf.z = x32[2 * (int64_t)nv + i];
  }
}

__device__ inline P3f load_f32(const float *x32, int nv, int i) {
  return P3f{x32[i], x32[(int64_t)nv + i], x32[2 * (int64_t)nv + i]};
}

__device__ inline P3d load_f64(const double *x64, int nv, int i) {
  return P3d{x64[i], x64[(int64_t)nv + i], x64[2 * (int64_t)nv + i]};
}

// Narrow phase for one candidate: returns 0/1/2, or kHitUnsure after both filters.
// In the float32 tier the float64 coordinates are loaded only when the
// float32 filter cannot settle the test.
template <bool F32, bool TIER0>
__device__ inline int narrow(const TravArgs &A, int4 qe, P3f pf, P3f qf, int4 t, unsigned long long &unsure32) {
  if (TIER0) {
    const P3f af = load_f32(A.fx32, A.fnv, t.x), bf = load_f32(A.fx32, A.fnv, t.y), cf = load_f32(A.fx32, A.fnv, t.z);
    const int r = ef_test_f32(pf, qf, af, bf, cf);
    if (r != kHitUnsure) return r;
    ++unsure32;
  }
  const P3d pd = load_f64(A.ex64, A.env, qe.x), qd = load_f64(A.ex64, A.env, qe.y);
  const P3d ad = load_f64(A.fx64, A.fnv, t.x), bd = load_f64(A.fx64, A.fnv, t.y), cd = load_f64(A.fx64, A.fnv, t.z);
  return ef_test_f64<false>(pd, qd, ad, bd, cd);
}

// Workgroups are dealt to the XCDs round-robin (workgroup b runs on XCD
// b mod 8).  Renumbering them so that each XCD takes one contiguous run of
// workgroups gives each XCD a contiguous range of Morton-ordered queries,
// i.e. one region of space, so its L2 holds only the part of the face BVH
// that region touches.  The map is a bijection of [0, n).
__device__ inline int xcd_contiguous_block(int b, int n) {
  const int x = b % kXcds, q = n / kXcds, r = n % kXcds;
  return x * q + (x < r ? x : r) + b / kXcds;
}

// Candidates are staged per wavefront in LDS and written out in batches, so
// the step loop carries no global atomic: a batch is flushed (one atomic for
// the wavefront) when fewer than two steps' worth of slots remain, and at the
// end.
constexpr int kCandStage = 256;

template <int BLOCK>
__device__ inline void flush_candidates(const TravArgs &A, uint2 *stage, int &cn) {
  __builtin_amdgcn_wave_barrier();
  uint32_t base = 0;
  if (__lane_id() == 0) base = atomicAdd(A.out.cand_count, (uint32_t)cn);
  base = (uint32_t)__shfl((int)base, 0);
  for (int j = (int)__lane_id(); j < cn; j += kWave)
    if (base + (uint32_t)j < A.out.cand_cap) A.out.cand_buf[base + j] = stage[j];
  __builtin_amdgcn_wave_barrier();
  cn = 0;
}

// Deferred subtrees are shared within a wavefront: when a step leaves lanes
// idle (their queries finished, mostly at the root box) and other lanes
// defer a child, those children go to a LIFO in LDS with their query's box,
// and idle lanes take them.  A wavefront's step count then approaches its
// total node count / 64 plus the depth, instead of its longest query's node
// count.  Each lane still keeps a private stack (most recent entry in a
// register) for the rest.
constexpr int kWaveQueue = 256;  // shared entries per wavefront
struct TravTask {
  float lo[3], hi[3];
  int qi, node;
};

template <bool F32, bool TIER0, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_traverse(TravArgs A) {
  __shared__ int stack[kStack][BLOCK];
  __shared__ uint2 cstage[BLOCK / kWave][kCandStage];
  __shared__ TravTask wq[BLOCK / kWave][kWaveQueue];
  const int tid = threadIdx.x;
  uint2 *stage = cstage[tid / kWave];
  TravTask *queue = wq[tid / kWave];
  int cn = 0;  // candidates staged by this wavefront (wave-uniform)
  int qn = 0;  // shared entries queued by this wavefront (wave-uniform)
  int qi = xcd_contiguous_block((int)blockIdx.x, (int)gridDim.x) * BLOCK + tid;
  if (A.warm && A.nt > 1) {
    unsigned acc = warm_l2(A.nodes, (int64_t)(A.nt - 1) * sizeof(BvhNode), 0u);
    acc = warm_l2(A.leaf_tri, (int64_t)A.nt * sizeof(int4), acc);
    acc = warm_l2(F32 ? (const void *)A.fx32 : (const void *)A.fx64,
                  (int64_t)3 * A.fnv * (F32 ? sizeof(float) : sizeof(double)), acc);
    if (acc == 0x9e3779b9u && qi == -1) atomicOr(A.out.overflow, 2);  // never true for qi >= 0
  }
  const bool valid = qi < A.ne;
  unsigned long long ncand = 0, nvisit = 0;
  float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  if (valid) {
    const int4 qe = A.qedges[qi];
    if (F32) {
      const P3f pf = load_f32(A.ex32, A.env, qe.x), qf = load_f32(A.ex32, A.env, qe.y);
      lo[0] = fminf(pf.x, qf.x); hi[0] = fmaxf(pf.x, qf.x);
      lo[1] = fminf(pf.y, qf.y); hi[1] = fmaxf(pf.y, qf.y);
      lo[2] = fminf(pf.z, qf.z); hi[2] = fmaxf(pf.z, qf.z);
    } else {
      const P3d pd = load_f64(A.ex64, A.env, qe.x), qd = load_f64(A.ex64, A.env, qe.y);
      lo[0] = __double2float_rd(fmin(pd.x, qd.x)); hi[0] = __double2float_ru(fmax(pd.x, qd.x));
      lo[1] = __double2float_rd(fmin(pd.y, qd.y)); hi[1] = __double2float_ru(fmax(pd.y, qd.y));
      lo[2] = __double2float_rd(fmin(pd.z, qd.z)); hi[2] = __double2float_ru(fmax(pd.z, qd.z));
    }
  }
  const float *rb = A.root_box;
  bool alive = valid && A.nt > 0 && box_overlap(lo, hi, rb[0], rb[1], rb[2], rb[3], rb[4], rb[5]);
  // A single face has no internal node: test it directly.
  int pending_leaf = (alive && A.nt == 1) ? 0 : -1;
  if (A.nt == 1) alive = false;
  int node = 0, sp = 0, top = -1;
  unsigned steps = 0;
  const uint64_t lt = lanemask_lt();
  while (true) {
    // idle lanes take shared entries (most recent first)
    if (qn > 0) {
      const uint64_t idle = __ballot(!alive);
      const int take = min(__popcll(idle), qn);
      const int rank = __popcll(idle & lt);
      __builtin_amdgcn_wave_barrier();
      if (!alive && rank < take) {
        const TravTask t = queue[qn - 1 - rank];
        lo[0] = t.lo[0]; lo[1] = t.lo[1]; lo[2] = t.lo[2];
        hi[0] = t.hi[0]; hi[1] = t.hi[1]; hi[2] = t.hi[2];
        qi = t.qi;
        node = t.node;
        top = -1;
        sp = 0;
        alive = true;
      }
      __builtin_amdgcn_wave_barrier();
      qn -= take;
    }
    int leaf_a = pending_leaf, leaf_b = -1;
    pending_leaf = -1;
    const bool any_alive = __any(alive);
    int defer = -1;
    if (alive) {
      ++nvisit;
      const BvhNode nd = A.nodes[node];
      const bool o0 = box_overlap(lo, hi, nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y);
      const bool o1 = box_overlap(lo, hi, nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w);
      const int c0 = nd.d.x, c1 = nd.d.y;
      bool i0 = o0 && c0 >= 0, i1 = o1 && c1 >= 0;
      if (o0 && c0 < 0) leaf_a = ~c0;
      if (o1 && c1 < 0) leaf_b = ~c1;
      if (i0 && i1) {
        defer = c1;
        node = c0;
      } else if (i0) {
        node = c0;
      } else if (i1) {
        node = c1;
      } else if (top >= 0) {
        node = top;
        top = sp > 0 ? stack[--sp][tid] : -1;
      } else {
        alive = false;
      }
    }
    if (any_alive) ++steps;
    // deferred children: to the shared LIFO while lanes are idle, else to
    // the lane's own stack (the most recent one stays in a register)
    const uint64_t dm = __ballot(defer >= 0);
    if (dm) {
      const int idle_now = __popcll(__ballot(!alive));
      const int give = min(min(__popcll(dm), max(idle_now - qn, 0)), kWaveQueue - qn);
      const int drank = __popcll(dm & lt);
      __builtin_amdgcn_wave_barrier();
      if (defer >= 0) {
        if (drank < give) {
          TravTask t;
          t.lo[0] = lo[0]; t.lo[1] = lo[1]; t.lo[2] = lo[2];
          t.hi[0] = hi[0]; t.hi[1] = hi[1]; t.hi[2] = hi[2];
          t.qi = qi;
          t.node = defer;
          queue[qn + drank] = t;
        } else {
          if (top >= 0) {
            if (sp >= kStack) {
              atomicOr(A.out.overflow, 1);
              alive = false;
            } else {
              stack[sp++][tid] = top;
            }
          }
          top = defer;
        }
      }
      __builtin_amdgcn_wave_barrier();
      qn += give;
    }
    // stage up to two candidate leaves found at this step
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int leaf = k == 0 ? leaf_a : leaf_b;
      const uint64_t m = __ballot(leaf >= 0);
      if (m == 0) continue;
      if (leaf >= 0) {
        ++ncand;
        stage[cn + __popcll(m & lt)] = make_uint2((uint32_t)qi, (uint32_t)leaf);
      }
      cn += __popcll(m);
    }
    if (cn > kCandStage - 2 * kWave) flush_candidates<BLOCK>(A, stage, cn);
    if (!__any(alive) && qn == 0) break;
  }
  if (cn > 0) flush_candidates<BLOCK>(A, stage, cn);
  // one counter update per wave
  for (int off = 32; off > 0; off >>= 1) {
    ncand += __shfl_xor(ncand, off);
    nvisit += __shfl_xor(nvisit, off);
  }
  if (__lane_id() == 0) {
    if (ncand) atomicAdd(A.out.cand, ncand);
    if (nvisit) atomicAdd(A.out.visits, nvisit);
    if (steps) atomicMax(A.out.max_path, steps);
  }
}

static TravArgs make_args(const MeshDev &E, const MeshDev &F, int dir, HitLayout lay, const DcdOut &out) {
  TravArgs a;
  a.warm = out.warm;
  a.qedges = E.qedges;
  a.ne = E.ne;
  a.ex64 = E.x64;
  a.ex32 = E.x32;
  a.env = E.nv;
  a.leaf_tri = F.leaf_tri;
  a.nodes = F.nodes;
  a.root_box = F.root_box;
  a.nt = F.nt;
  a.fx64 = F.x64;
  a.fx32 = F.x32;
  a.fnv = F.nv;
  a.dir = dir;
  a.lay = lay;
  a.out = out;
  return a;
}

template <int BLOCK>
static void launch_traverse_b(const MeshDev &E, const MeshDev &F, bool tier0, const TravArgs &a, hipStream_t s) {
  const unsigned grid = grid_for(E.ne, BLOCK);
  const bool f32 = E.f32 && F.f32 && E.x32 && F.x32;
  if (f32 && tier0 && E.small_coords && F.small_coords)
    k_traverse<true, true, BLOCK><<<grid, BLOCK, 0, s>>>(a);
  else if (f32)
    k_traverse<true, false, BLOCK><<<grid, BLOCK, 0, s>>>(a);
  else
    k_traverse<false, false, BLOCK><<<grid, BLOCK, 0, s>>>(a);
}

void launch_traverse(const MeshDev &E, const MeshDev &F, int dir, bool tier0, HitLayout lay, const DcdOut &out,
                     int block, hipStream_t s) {
  if (E.ne <= 0 || F.nt <= 0) return;
  TravArgs a = make_args(E, F, dir, lay, out);
  if (block <= 64)
    launch_traverse_b<64>(E, F, tier0, a, s);
  else if (block <= 128)
    launch_traverse_b<128>(E, F, tier0, a, s);
  else
    launch_traverse_b<256>(E, F, tier0, a, s);
}

// ----------------------------------------------------------- narrow phase
// Grid-stride over the queued candidates (count read on the device).
template <bool F32, bool TIER0>
__global__ __launch_bounds__(256) void k_narrow(TravArgs A) {
  const uint32_t nc = *A.out.cand_count;
  const uint32_t n = nc < A.out.cand_cap ? nc : (uint32_t)A.out.cand_cap;
  const uint64_t dir_bits = (uint64_t)A.dir << (A.lay.bits_e + A.lay.bits_f);
  unsigned long long unsure32 = 0;
  const uint32_t stride = gridDim.x * blockDim.x;
  // every lane of a wave runs the same number of iterations (wave_append)
  const uint32_t n_round = (n + 63u) & ~63u;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_round; i += stride) {
    int res = 0;
    int4 qe = make_int4(0, 0, 0, 0), t = make_int4(0, 0, 0, 0);
    uint2 item = make_uint2(0, 0);
    if (i < n) {
      item = A.out.cand_buf[i];
      qe = A.qedges[item.x];
      t = A.leaf_tri[item.y];
      P3f pf{}, qf{};
      if (TIER0) {
        pf = load_f32(A.ex32, A.env, qe.x);
        qf = load_f32(A.ex32, A.env, qe.y);
      }
      res = narrow<F32, TIER0>(A, qe, pf, qf, t, unsure32);
    }
    const bool is_hit = res == 1 || res == 2;
    const uint32_t slot = wave_append(A.out.count, is_hit);
    if (is_hit && slot < A.out.cap) {
      A.out.keys[slot] = dir_bits | ((uint64_t)qe.z << A.lay.bits_f) | (uint32_t)t.w;
      A.out.vals[slot] = (uint32_t)(res == 1 ? qe.x : qe.y);
    }
    const bool is_amb = res == kHitUnsure;
    const uint32_t aslot = wave_append(A.out.amb_count, is_amb);
    if (is_amb && aslot < A.out.amb_cap) A.out.amb[aslot] = item;
  }
  for (int off = 32; off > 0; off >>= 1) unsure32 += __shfl_xor(unsure32, off);
  if (__lane_id() == 0 && unsure32) atomicAdd(A.out.f32_unsure, unsure32);
}

void launch_narrow(const MeshDev &E, const MeshDev &F, int dir, bool tier0, HitLayout lay, const DcdOut &out,
                   hipStream_t s) {
  if (E.ne <= 0 || F.nt <= 0) return;
  TravArgs a = make_args(E, F, dir, lay, out);
  const bool f32 = E.f32 && F.f32 && E.x32 && F.x32;
  // grid-stride, since the count is only known on the device: about two
  // candidates per query edge fill the grid once
  const unsigned grid = std::min<unsigned>(1024u, std::max<unsigned>(8u, grid_for(2 * (int64_t)E.ne, 256)));
  if (f32 && tier0 && E.small_coords && F.small_coords)
    k_narrow<true, true><<<grid, 256, 0, s>>>(a);
  else if (f32)
    k_narrow<true, false><<<grid, 256, 0, s>>>(a);
  else
    k_narrow<false, false><<<grid, 256, 0, s>>>(a);
}

// ------------------------------------------------------------ exact tier
// Grid-stride over the undecided candidates (count read on the device).
__global__ __launch_bounds__(64) void k_exact(TravArgs A) {
  const uint32_t namb = *A.out.amb_count;
  const uint32_t n = namb < A.out.amb_cap ? namb : (uint32_t)A.out.amb_cap;
  const uint64_t dir_bits = (uint64_t)A.dir << (A.lay.bits_e + A.lay.bits_f);
  unsigned long long nex = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    uint2 item = A.out.amb[i];
    int4 qe = A.qedges[item.x];
    int4 t = A.leaf_tri[item.y];
    P3f dummy;
    P3d p, q, a, b, c;
    load_point<false>(A.ex64, nullptr, A.env, qe.x, dummy, p);
    load_point<false>(A.ex64, nullptr, A.env, qe.y, dummy, q);
    load_point<false>(A.fx64, nullptr, A.fnv, t.x, dummy, a);
    load_point<false>(A.fx64, nullptr, A.fnv, t.y, dummy, b);
    load_point<false>(A.fx64, nullptr, A.fnv, t.z, dummy, c);
    int ne = 0;
    int res = ef_test_f64<true>(p, q, a, b, c, &ne);
    nex += (unsigned long long)ne;
    if (res == 1 || res == 2) {
      uint32_t slot = atomicAdd(A.out.count, 1u);
      if (slot < A.out.cap) {
        A.out.keys[slot] = dir_bits | ((uint64_t)qe.z << A.lay.bits_f) | (uint32_t)t.w;
        A.out.vals[slot] = (uint32_t)(res == 1 ? qe.x : qe.y);
      }
    }
  }
  if (nex) atomicAdd(A.out.exact, nex);
}

void launch_exact(const MeshDev &E, const MeshDev &F, int dir, HitLayout lay, const DcdOut &out, hipStream_t s) {
  if (E.ne <= 0 || F.nt <= 0) return;
  TravArgs a = make_args(E, F, dir, lay, out);
  k_exact<<<256, 64, 0, s>>>(a);
}

// ------------------------------------------------------------ hit output
__global__ void k_write_hits(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals, int64_t n,
                             HitLayout lay, const int2 *__restrict__ ea, const int2 *__restrict__ eb, int32_t *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t k = keys[i];
  int f = (int)(k & ((1ull << lay.bits_f) - 1));
  int e = (int)((k >> lay.bits_f) & ((1ull << lay.bits_e) - 1));
  int dir = (int)(k >> (lay.bits_f + lay.bits_e));
  int2 uv = dir == 0 ? ea[e] : eb[e];
  int32_t *o = out + 5 * i;
  o[0] = dir;
  o[1] = uv.x;
  o[2] = uv.y;
  o[3] = f;
  o[4] = (int32_t)vals[i];
}

void launch_write_hits(const uint64_t *keys, const uint32_t *vals, int64_t n, HitLayout lay, const int2 *ea,
                       const int2 *eb, int32_t *out, hipStream_t s) {
  if (n > 0) k_write_hits<<<grid_for(n, 256), 256, 0, s>>>(keys, vals, n, lay, ea, eb, out);
}

// ------------------------------------------------------ predicate probe
// Signs of orient(a,b,c,p) for n quadruples pts[n][4][3]: tier 0 = float32
// filter (may be kUnsure), 1 = float64 filter (may be kUnsure), 2 = exact.
__global__ void k_test_orient(const double *pts, int64_t n, int tier, int32_t *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double *q = pts + 12 * i;
  int s;
  if (tier == 0)
    s = filtered_sign_f32((float)q[0], (float)q[1], (float)q[2], (float)q[3], (float)q[4], (float)q[5],
                          (float)q[6], (float)q[7], (float)q[8], (float)q[9], (float)q[10], (float)q[11]);
  else if (tier == 1)
    s = filtered_sign_f64(q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7], q[8], q[9], q[10], q[11]);
  else
    s = exact_sign(q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7], q[8], q[9], q[10], q[11]);
  out[i] = s;
}

void launch_test_orient(const double *pts, int64_t n, int tier, int32_t *out, hipStream_t s) {
  if (n > 0) k_test_orient<<<grid_for(n, 256), 256, 0, s>>>(pts, n, tier, out);
}

}  // namespace hfcr
