// Per-mesh set-up: input ingest and validation, the unique edge set, Morton
// ordering of edge queries and faces, the linear BVH over faces (radix tree
// built from sorted Morton codes, after Karras 2012, "Maximizing parallelism
// in the construction of BVHs, octrees, and k-d trees") and its bottom-up
// refit with per-node arrival counters.
//
// Boxes are float32 and conservative: for float64 positions the lower bound
// is rounded down and the upper bound up, so a box always contains the
// exact triangle or segment (the closed-box overlap test never rejects a
// true E-F intersection, whose crossing point lies in both boxes).
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace hfcr {

// ------------------------------------------------------------------ ingest
// AoS input -> SoA float64 working copy (+ float32 copy for float32 storage),
// with validation: non-finite or out-of-domain coordinates set bit 0 of
// *err; the largest magnitude is folded into *maxabs_bits (float bits).
template <typename T>
__global__ void k_ingest(const T *__restrict__ pos, int nv, double *__restrict__ x64, float *__restrict__ x32,
                         unsigned *err, unsigned *maxabs_bits) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  float m = 0.0f;
  if (i < nv) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T v = pos[3 * (int64_t)i + k];
      double dv = (double)v;
      double a = fabs(dv);
      bool ok = isfinite(dv) && (a == 0.0 || (a >= 0x1p-200 && a <= 0x1p200));
      if (!ok) atomicOr(err, 1u);
      x64[(int64_t)k * nv + i] = dv;
      if (x32) x32[(int64_t)k * nv + i] = (float)v;
      float af = isfinite(dv) ? __double2float_ru(a) : INFINITY;
      m = fmaxf(m, af);
    }
  }
  // wave max, then one atomic per wave (positive floats order like ints)
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) atomicMax(maxabs_bits, __float_as_uint(m));
}

__global__ void k_check_tri(const int32_t *__restrict__ tri, int nt, int nv, unsigned *err) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  for (int k = 0; k < 3; ++k) {
    int v = tri[3 * (int64_t)i + k];
    if (v < 0 || v >= nv) atomicOr(err, 2u);
  }
}

// *diff |= 1 when the two index arrays differ anywhere.
__global__ void k_tri_diff(const int32_t *__restrict__ a, const int32_t *__restrict__ b, int64_t n, unsigned *diff) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool d = i < n && a[i] != b[i];
  if (__any(d) && __lane_id() == 0) atomicOr(diff, 1u);
}

void launch_tri_diff(const int32_t *a, const int32_t *b, int64_t n, unsigned *diff, hipStream_t s) {
  if (n > 0) k_tri_diff<<<grid_for(n, 256), 256, 0, s>>>(a, b, n, diff);
}

void launch_ingest(const MeshDev &m, unsigned *err, unsigned *maxabs, hipStream_t s) {
  if (m.nv > 0) {
    if (m.f32)
      k_ingest<float><<<grid_for(m.nv, 256), 256, 0, s>>>((const float *)m.pos_in, m.nv, m.x64, m.x32, err, maxabs);
    else
      k_ingest<double><<<grid_for(m.nv, 256), 256, 0, s>>>((const double *)m.pos_in, m.nv, m.x64, nullptr, err,
                                                             maxabs);
  }
  if (m.nt > 0) k_check_tri<<<grid_for(m.nt, 256), 256, 0, s>>>(m.tri_in, m.nt, m.nv, err);
}

// ------------------------------------------------------------------- edges
// Half-edge keys (min << 32 | max); a degenerate side (u == v) gets the key
// nv << 32, which sorts after every real edge and is dropped.
__global__ void k_halfedge_keys(const int32_t *__restrict__ tri, int nt, int nv, uint64_t *keys) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 3 * nt) return;
  int t = i / 3, k = i % 3;
  uint32_t u = (uint32_t)tri[3 * (int64_t)t + k];
  uint32_t v = (uint32_t)tri[3 * (int64_t)t + (k + 1) % 3];
  uint32_t lo = u < v ? u : v, hi = u < v ? v : u;
  keys[i] = (u == v) ? ((uint64_t)nv << 32) : (((uint64_t)lo << 32) | hi);
}

__global__ void k_unique_flags(const uint64_t *__restrict__ keys, int64_t n, uint64_t invalid_from,
                               uint32_t *flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t k = keys[i];
  flags[i] = (k < invalid_from && (i == 0 || keys[i - 1] != k)) ? 1u : 0u;
}

__global__ void k_compact_edges(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ flags,
                                const uint32_t *__restrict__ pos, int64_t n, int2 *edges) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flags[i]) return;
  uint64_t k = keys[i];
  edges[pos[i]] = make_int2((int)(k >> 32), (int)(k & 0xffffffffu));
}

void launch_edge_keys(const MeshDev &m, uint64_t *keys, hipStream_t s) {
  k_halfedge_keys<<<grid_for(3 * (int64_t)m.nt, 256), 256, 0, s>>>(m.tri_in, m.nt, m.nv, keys);
}

void launch_unique_flags(const uint64_t *keys, int64_t n, uint64_t invalid_from, uint32_t *flags,
                         hipStream_t s) {
  k_unique_flags<<<grid_for(n, 256), 256, 0, s>>>(keys, n, invalid_from, flags);
}

void launch_compact_edges(const uint64_t *keys, const uint32_t *flags, const uint32_t *pos, int64_t n,
                          int2 *edges, hipStream_t s) {
  k_compact_edges<<<grid_for(n, 256), 256, 0, s>>>(keys, flags, pos, n, edges);
}

// ------------------------------------------------------------------ bounds
// Scene box of a mesh's vertices (one workgroup); used only to quantise
// Morton codes, so plain float rounding is fine here.
__global__ __launch_bounds__(1024) void k_bounds(const double *__restrict__ x64, int nv, float *box) {
  __shared__ float red[6][1024];
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int i = threadIdx.x; i < nv; i += 1024)
    for (int k = 0; k < 3; ++k) {
      float v = (float)x64[(int64_t)k * nv + i];
      lo[k] = fminf(lo[k], v);
      hi[k] = fmaxf(hi[k], v);
    }
  for (int k = 0; k < 3; ++k) {
    red[k][threadIdx.x] = lo[k];
    red[3 + k][threadIdx.x] = hi[k];
  }
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = fminf(red[k][threadIdx.x], red[k][threadIdx.x + off]);
        red[3 + k][threadIdx.x] = fmaxf(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + off]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) box[threadIdx.x] = red[threadIdx.x][0];
}

void launch_bounds(const MeshDev &m, float *box, hipStream_t s) {
  k_bounds<<<1, 1024, 0, s>>>(m.x64, m.nv, box);
}

// ------------------------------------------------------------------ morton
__device__ inline uint32_t spread10(uint32_t v) {
  v &= 1023u;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

__device__ inline uint32_t morton3(float x, float y, float z, const float *box) {
  float c[3] = {x, y, z};
  uint32_t q[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    float ext = box[3 + k] - box[k];
    float t = ext > 0.0f ? (c[k] - box[k]) / ext : 0.5f;
    t = fminf(fmaxf(t, 0.0f), 1.0f);
    q[k] = (uint32_t)fminf(t * 1024.0f, 1023.0f);
  }
  return (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
}

__global__ void k_edge_morton(const int2 *__restrict__ edges, int ne, const double *__restrict__ x64, int nv,
                              const float *__restrict__ box, uint64_t *keys) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ne) return;
  int2 uv = edges[e];
  float m[3];
  for (int k = 0; k < 3; ++k)
    m[k] = (float)(0.5 * (x64[(int64_t)k * nv + uv.x] + x64[(int64_t)k * nv + uv.y]));
  keys[e] = ((uint64_t)morton3(m[0], m[1], m[2], box) << 32) | (uint32_t)e;
}

__global__ void k_make_qedges(const uint64_t *__restrict__ keys, const int2 *__restrict__ edges, int ne,
                              int4 *q) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ne) return;
  int e = (int)(keys[i] & 0xffffffffu);
  int2 uv = edges[e];
  q[i] = make_int4(uv.x, uv.y, e, 0);
}

__global__ void k_face_morton(const int32_t *__restrict__ tri, int nt, const double *__restrict__ x64, int nv,
                              const float *__restrict__ box, uint64_t *keys) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nt) return;
  float c[3];
  for (int k = 0; k < 3; ++k) {
    double s = x64[(int64_t)k * nv + tri[3 * (int64_t)f]] + x64[(int64_t)k * nv + tri[3 * (int64_t)f + 1]] +
               x64[(int64_t)k * nv + tri[3 * (int64_t)f + 2]];
    c[k] = (float)(s / 3.0);
  }
  keys[f] = ((uint64_t)morton3(c[0], c[1], c[2], box) << 32) | (uint32_t)f;
}

__global__ void k_leaf_tri(const uint64_t *__restrict__ keys, const int32_t *__restrict__ tri, int nt,
                           int4 *leaf_tri, uint32_t *codes) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nt) return;
  uint64_t k = keys[i];
  int f = (int)(k & 0xffffffffu);
  leaf_tri[i] = make_int4(tri[3 * (int64_t)f], tri[3 * (int64_t)f + 1], tri[3 * (int64_t)f + 2], f);
  codes[i] = (uint32_t)(k >> 32);
}

void launch_edge_morton(const MeshDev &m, const float *box, uint64_t *keys, hipStream_t s) {
  k_edge_morton<<<grid_for(m.ne, 256), 256, 0, s>>>(m.edges, m.ne, m.x64, m.nv, box, keys);
}
void launch_make_qedges(const MeshDev &m, const uint64_t *keys, hipStream_t s) {
  k_make_qedges<<<grid_for(m.ne, 256), 256, 0, s>>>(keys, m.edges, m.ne, m.qedges);
}
void launch_face_morton(const MeshDev &m, const float *box, uint64_t *keys, hipStream_t s) {
  k_face_morton<<<grid_for(m.nt, 256), 256, 0, s>>>(m.tri_in, m.nt, m.x64, m.nv, box, keys);
}
void launch_leaf_tri(const MeshDev &m, const uint64_t *keys, uint32_t *codes, hipStream_t s) {
  k_leaf_tri<<<grid_for(m.nt, 256), 256, 0, s>>>(keys, m.tri_in, m.nt, m.leaf_tri, codes);
}

// ------------------------------------------------------------ radix tree
// Common-prefix length of the (code, index) keys of leaves i and j; -1 when
// j is outside [0, n).  Equal codes fall back to the index bits.
__device__ inline int prefix_len(const uint32_t *__restrict__ code, int n, int i, int j) {
  if (j < 0 || j >= n) return -1;
  uint32_t a = code[i], b = code[j];
  if (a == b) return 32 + __clz((unsigned)(i ^ j));
  return __clz(a ^ b);
}

__global__ void k_build_tree(const uint32_t *__restrict__ code, int n, BvhNode *nodes, int *leaf_parent,
                             int2 *range) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  // direction of the node's range: towards the neighbour sharing more bits
  int d = (prefix_len(code, n, i, i + 1) - prefix_len(code, n, i, i - 1)) >= 0 ? 1 : -1;
  int dmin = prefix_len(code, n, i, i - d);
  int lmax = 2;
  while (prefix_len(code, n, i, i + lmax * d) > dmin) lmax <<= 1;
  int l = 0;
  for (int t = lmax >> 1; t >= 1; t >>= 1)
    if (prefix_len(code, n, i, i + (l + t) * d) > dmin) l += t;
  int j = i + l * d;
  int dnode = prefix_len(code, n, i, j);
  // split: the last position sharing more than dnode bits with i
  int s = 0;
  for (int div = 2;; div <<= 1) {
    int t = (l + div - 1) / div;
    if (prefix_len(code, n, i, i + (s + t) * d) > dnode) s += t;
    if (t <= 1) break;
  }
  int gamma = i + s * d + (d < 0 ? d : 0);
  int lo = i < j ? i : j, hi = i < j ? j : i;
  range[i] = make_int2(lo, hi);
  int left = (lo == gamma) ? ~gamma : gamma;
  int right = (hi == gamma + 1) ? ~(gamma + 1) : gamma + 1;
  nodes[i].d.x = left;
  nodes[i].d.y = right;
  if (left < 0) leaf_parent[~left] = (i << 1) | 0;
  else {
    nodes[left].d.z = i;
    nodes[left].d.w = 0;
  }
  if (right < 0) leaf_parent[~right] = (i << 1) | 1;
  else {
    nodes[right].d.z = i;
    nodes[right].d.w = 1;
  }
  if (i == 0) {
    nodes[0].d.z = -1;
    nodes[0].d.w = 0;
  }
}

// Refit chunks: each internal node covers a contiguous range of leaves (in
// Morton order) and contains one end of its range in its own index, so the
// nodes whose range lies inside chunk c have indices in that chunk.  Nodes
// whose range crosses a chunk boundary ("top" nodes) are listed here.
constexpr int kChunkBits = 10;
constexpr int kChunk = 1 << kChunkBits;

__global__ void k_mark_top(const int2 *__restrict__ range, const BvhNode *__restrict__ nodes, int n, int *top_pos,
                           int *top_list, int *top_count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n - 1) return;
  int2 r = range[i];
  if ((r.x >> kChunkBits) != (r.y >> kChunkBits)) {
    int pos = atomicAdd(top_count, 1);
    top_pos[i] = pos;
    top_list[pos] = i;
  } else {
    top_pos[i] = -1;
  }
}

__global__ void k_top_pre(const BvhNode *__restrict__ nodes, const int *__restrict__ top_pos,
                          const int *__restrict__ top_list, const int *__restrict__ top_count, int *top_pre) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= *top_count) return;
  int4 d = nodes[top_list[t]].d;
  int pre = 0;
  pre += (d.x < 0 || top_pos[d.x] < 0) ? 1 : 0;
  pre += (d.y < 0 || top_pos[d.y] < 0) ? 1 : 0;
  top_pre[t] = pre;
}

void launch_build_tree(const MeshDev &m, const uint32_t *codes, hipStream_t s) {
  if (m.nt < 2) return;
  k_build_tree<<<grid_for(m.nt - 1, 256), 256, 0, s>>>(codes, m.nt, m.nodes, m.leaf_parent, m.range);
  (void)hipMemsetAsync(m.top_count, 0, sizeof(int), s);
  k_mark_top<<<grid_for(m.nt - 1, 256), 256, 0, s>>>(m.range, m.nodes, m.nt, m.top_pos, m.top_list, m.top_count);
  k_top_pre<<<grid_for(m.nt - 1, 256), 256, 0, s>>>(m.nodes, m.top_pos, m.top_list, m.top_count, m.top_pre);
}

// -------------------------------------------------------------------- refit
__device__ inline void store_child_box(BvhNode *nd, int slot, const float lo[3], const float hi[3]) {
  float *p = reinterpret_cast<float *>(nd);
  // layout: a = lo0.xyz hi0.x ; b = hi0.yz lo1.xy ; c = lo1.z hi1.xyz
  if (slot == 0) {
    p[0] = lo[0]; p[1] = lo[1]; p[2] = lo[2];
    p[3] = hi[0]; p[4] = hi[1]; p[5] = hi[2];
  } else {
    p[6] = lo[0]; p[7] = lo[1]; p[8] = lo[2];
    p[9] = hi[0]; p[10] = hi[1]; p[11] = hi[2];
  }
}

__device__ inline float coherent_load(const float *p) {
  return __int_as_float(__hip_atomic_load(reinterpret_cast<const int *>(p), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT));
}

template <bool F32>
__global__ void k_refit(const int4 *__restrict__ leaf_tri, int nt, const double *__restrict__ x64,
                        const float *__restrict__ x32, int nv, BvhNode *nodes, const int *__restrict__ leaf_parent,
                        int *counters, float *root_box) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= nt) return;
  int4 t = leaf_tri[l];
  float lo[3], hi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (F32) {
      float a = x32[(int64_t)k * nv + t.x], b = x32[(int64_t)k * nv + t.y], c = x32[(int64_t)k * nv + t.z];
      lo[k] = fminf(a, fminf(b, c));
      hi[k] = fmaxf(a, fmaxf(b, c));
    } else {
      double a = x64[(int64_t)k * nv + t.x], b = x64[(int64_t)k * nv + t.y], c = x64[(int64_t)k * nv + t.z];
      lo[k] = __double2float_rd(fmin(a, fmin(b, c)));
      hi[k] = __double2float_ru(fmax(a, fmax(b, c)));
    }
  }
  if (nt == 1) {
    for (int k = 0; k < 3; ++k) {
      root_box[k] = lo[k];
      root_box[3 + k] = hi[k];
    }
    return;
  }
  int pp = leaf_parent[l];
  int node = pp >> 1;
  store_child_box(&nodes[node], pp & 1, lo, hi);
  while (true) {
    __threadfence();
    int old = atomicAdd(&counters[node], 1);
    if (old == 0) return;  // the sibling subtree is not finished yet
    counters[node] = 0;    // both children arrived: reset for the next refit
    __threadfence();
    const float *p = reinterpret_cast<const float *>(&nodes[node]);
    float b[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) b[k] = coherent_load(p + k);
    for (int k = 0; k < 3; ++k) {
      lo[k] = fminf(b[k], b[6 + k]);
      hi[k] = fmaxf(b[3 + k], b[9 + k]);
    }
    int parent = nodes[node].d.z;
    int slot = nodes[node].d.w;
    if (parent < 0) {
      for (int k = 0; k < 3; ++k) {
        root_box[k] = lo[k];
        root_box[3 + k] = hi[k];
      }
      return;
    }
    store_child_box(&nodes[parent], slot, lo, hi);
    node = parent;
  }
}

// Single-workgroup refit for trees whose arrival counters fit in LDS: every
// climb stays on one CU, so workgroup-scope release/acquire on the LDS
// counter orders the box stores and loads without any cache maintenance.
constexpr int kRefitBlock = 1024;
constexpr int kRefitWgMaxNodes = 38 * 1024;  // counters in LDS (152 KiB)
// Measured slower than the multi-workgroup climb for 16k-leaf trees (one
// workgroup walks 16 leaves per thread in sequence), so it is off.
constexpr bool kRefitSingleWg = false;

template <bool F32>
__global__ __launch_bounds__(kRefitBlock) void k_refit_wg(const int4 *__restrict__ leaf_tri, int nt,
                                                          const double *__restrict__ x64,
                                                          const float *__restrict__ x32, int nv, BvhNode *nodes,
                                                          const int *__restrict__ leaf_parent, float *root_box) {
  extern __shared__ int cnt[];
  for (int i = threadIdx.x; i < nt - 1; i += kRefitBlock) cnt[i] = 0;
  __syncthreads();
  for (int l = threadIdx.x; l < nt; l += kRefitBlock) {
    const int4 t = leaf_tri[l];
    float lo[3], hi[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (F32) {
        float a = x32[(int64_t)k * nv + t.x], b = x32[(int64_t)k * nv + t.y], c = x32[(int64_t)k * nv + t.z];
        lo[k] = fminf(a, fminf(b, c));
        hi[k] = fmaxf(a, fmaxf(b, c));
      } else {
        double a = x64[(int64_t)k * nv + t.x], b = x64[(int64_t)k * nv + t.y], c = x64[(int64_t)k * nv + t.z];
        lo[k] = __double2float_rd(fmin(a, fmin(b, c)));
        hi[k] = __double2float_ru(fmax(a, fmax(b, c)));
      }
    }
    const int pp = leaf_parent[l];
    int node = pp >> 1;
    store_child_box(&nodes[node], pp & 1, lo, hi);
    while (true) {
      // release our box store, acquire the sibling's (workgroup scope)
      const int old = __hip_atomic_fetch_add(&cnt[node], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (old == 0) break;
      const BvhNode nd = nodes[node];
      lo[0] = fminf(nd.a.x, nd.b.z); lo[1] = fminf(nd.a.y, nd.b.w); lo[2] = fminf(nd.a.z, nd.c.x);
      hi[0] = fmaxf(nd.a.w, nd.c.y); hi[1] = fmaxf(nd.b.x, nd.c.z); hi[2] = fmaxf(nd.b.y, nd.c.w);
      const int parent = nd.d.z;
      if (parent < 0) {
        for (int k = 0; k < 3; ++k) {
          root_box[k] = lo[k];
          root_box[3 + k] = hi[k];
        }
        break;
      }
      store_child_box(&nodes[parent], nd.d.w, lo, hi);
      node = parent;
    }
  }
}

// Two-phase refit.  Phase 1: one workgroup per chunk of kChunk leaves climbs
// through the nodes inside its chunk, with arrival counters in LDS and
// workgroup-scope release/acquire, stopping below the first top node.
// Phase 2: one workgroup climbs the top nodes, whose counters start at the
// number of children phase 1 already finished.  No step needs device-wide
// cache maintenance; the kernel boundary orders the two phases.
__device__ inline void leaf_box(const int4 t, bool f32, const double *__restrict__ x64, const float *__restrict__ x32,
                                int nv, float lo[3], float hi[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    if (f32) {
      float a = x32[(int64_t)k * nv + t.x], b = x32[(int64_t)k * nv + t.y], c = x32[(int64_t)k * nv + t.z];
      lo[k] = fminf(a, fminf(b, c));
      hi[k] = fmaxf(a, fmaxf(b, c));
    } else {
      double a = x64[(int64_t)k * nv + t.x], b = x64[(int64_t)k * nv + t.y], c = x64[(int64_t)k * nv + t.z];
      lo[k] = __double2float_rd(fmin(a, fmin(b, c)));
      hi[k] = __double2float_ru(fmax(a, fmax(b, c)));
    }
  }
}

__device__ inline void node_union(const BvhNode &nd, float lo[3], float hi[3]) {
  lo[0] = fminf(nd.a.x, nd.b.z); lo[1] = fminf(nd.a.y, nd.b.w); lo[2] = fminf(nd.a.z, nd.c.x);
  hi[0] = fmaxf(nd.a.w, nd.c.y); hi[1] = fmaxf(nd.b.x, nd.c.z); hi[2] = fmaxf(nd.b.y, nd.c.w);
}

// One workgroup per chunk of kChunk leaves.  The chunk's internal nodes
// (indices base .. base + kChunk - 1) keep a copy of their child boxes,
// parent and top flag in LDS, so a climb step is LDS work: the second thread
// to arrive at a node reads its sibling's box there.  Every child box is
// also stored to the node array, which the traversal reads; a climb stops
// at a top node (handled by k_refit_top).
template <bool F32>
__global__ __launch_bounds__(kChunk) void k_refit_chunk(const int4 *__restrict__ leaf_tri, int nt,
                                                        const double *__restrict__ x64, const float *__restrict__ x32,
                                                        int nv, BvhNode *nodes, const int *__restrict__ leaf_parent,
                                                        const int *__restrict__ top_pos, float *root_box) {
  __shared__ int cnt[kChunk];
  __shared__ float sbox[kChunk][12];  // child boxes, in the node array's layout
  __shared__ int spar[kChunk];        // parent << 1 | slot, or -1 at the root
  __shared__ unsigned char stop[kChunk];
  const int base = blockIdx.x * kChunk;
  const int tid = threadIdx.x;
  cnt[tid] = 0;
  {
    const int n = base + tid;
    if (n < nt - 1) {
      const int4 d = nodes[n].d;
      spar[tid] = d.z < 0 ? -1 : (d.z << 1) | d.w;
      stop[tid] = top_pos[n] >= 0;
    }
  }
  __syncthreads();
  const int l = base + tid;
  if (l >= nt) return;
  float lo[3], hi[3];
  leaf_box(leaf_tri[l], F32, x64, x32, nv, lo, hi);
  int pp = leaf_parent[l];
  while (true) {
    const int node = pp >> 1, slot = pp & 1;
    store_child_box(&nodes[node], slot, lo, hi);
    // a node outside the chunk's index range has a range that crosses it
    const int li = node - base;
    if (li < 0 || li >= kChunk || stop[li]) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      sbox[li][6 * slot + k] = lo[k];
      sbox[li][6 * slot + 3 + k] = hi[k];
    }
    const int old = __hip_atomic_fetch_add(&cnt[li], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (old == 0) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lo[k] = fminf(sbox[li][k], sbox[li][6 + k]);
      hi[k] = fmaxf(sbox[li][3 + k], sbox[li][9 + k]);
    }
    pp = spar[li];
    if (pp < 0) {
      for (int k = 0; k < 3; ++k) {
        root_box[k] = lo[k];
        root_box[3 + k] = hi[k];
      }
      return;
    }
  }
}

constexpr int kTopLds = 32 * 1024;  // top nodes handled by the two-phase refit
constexpr int kTopStage = 1536;     // top nodes whose boxes fit in LDS (56 B each)

// The nodes whose range crosses a chunk boundary, climbed by one workgroup.
// With at most `cap` of them, their child boxes, parents and arrival
// counters live in LDS (staged from the node array, which the chunk kernel
// has just written), so a climb step is LDS work; otherwise the boxes are
// read from the node array.  Every child box is also stored to the array.
__global__ __launch_bounds__(1024) void k_refit_top(BvhNode *nodes, const int *__restrict__ top_pos,
                                                    const int *__restrict__ top_list, const int *__restrict__ top_pre,
                                                    const int *__restrict__ top_count, float *root_box, int cap) {
  extern __shared__ int dyn[];
  const int ntop = *top_count;
  if (ntop <= cap) {
    float *tbox = reinterpret_cast<float *>(dyn);  // [cap][12]
    int *tpar = dyn + 12 * cap;                    // parent's top index << 1 | slot, or -1 at the root
    int *tcnt = tpar + cap;
    for (int t = threadIdx.x; t < ntop; t += 1024) {
      const BvhNode nd = nodes[top_list[t]];
      const float *f = reinterpret_cast<const float *>(&nd);
#pragma unroll
      for (int k = 0; k < 12; ++k) tbox[12 * t + k] = f[k];
      tpar[t] = nd.d.z < 0 ? -1 : (top_pos[nd.d.z] << 1) | nd.d.w;
      tcnt[t] = top_pre[t];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ntop; t += 1024) {
      if (top_pre[t] != 2) continue;  // a climb starts where both children are done
      int u = t;
      while (true) {
        float lo[3], hi[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          lo[k] = fminf(tbox[12 * u + k], tbox[12 * u + 6 + k]);
          hi[k] = fmaxf(tbox[12 * u + 3 + k], tbox[12 * u + 9 + k]);
        }
        const int pt = tpar[u];
        if (pt < 0) {
          for (int k = 0; k < 3; ++k) {
            root_box[k] = lo[k];
            root_box[3 + k] = hi[k];
          }
          break;
        }
        const int pu = pt >> 1, slot = pt & 1;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          tbox[12 * pu + 6 * slot + k] = lo[k];
          tbox[12 * pu + 6 * slot + 3 + k] = hi[k];
        }
        store_child_box(&nodes[top_list[pu]], slot, lo, hi);
        const int old = __hip_atomic_fetch_add(&tcnt[pu], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old != 1) break;  // the other child is not finished yet
        u = pu;
      }
    }
    return;
  }
  int *tcnt = dyn;
  for (int t = threadIdx.x; t < ntop; t += 1024) tcnt[t] = top_pre[t];
  __syncthreads();
  for (int t = threadIdx.x; t < ntop; t += 1024) {
    if (top_pre[t] != 2) continue;  // a climb starts where both children are done
    int node = top_list[t];
    while (true) {
      float lo[3], hi[3];
      const BvhNode nd = nodes[node];
      node_union(nd, lo, hi);
      const int parent = nd.d.z;
      if (parent < 0) {
        for (int k = 0; k < 3; ++k) {
          root_box[k] = lo[k];
          root_box[3 + k] = hi[k];
        }
        break;
      }
      store_child_box(&nodes[parent], nd.d.w, lo, hi);
      const int old =
          __hip_atomic_fetch_add(&tcnt[top_pos[parent]], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (old != 1) break;  // the other child is not finished yet
      node = parent;
    }
  }
}

void launch_refit(const MeshDev &m, hipStream_t s) {
  if (m.nt <= 0) return;
  const int nchunks = (m.nt + kChunk - 1) / kChunk;
  if (m.nt >= 2 && (int64_t)nchunks * 64 <= kTopLds) {
    if (m.f32)
      k_refit_chunk<true><<<nchunks, kChunk, 0, s>>>(m.leaf_tri, m.nt, m.x64, m.x32, m.nv, m.nodes, m.leaf_parent,
                                                     m.top_pos, m.root_box);
    else
      k_refit_chunk<false><<<nchunks, kChunk, 0, s>>>(m.leaf_tri, m.nt, m.x64, m.x32, m.nv, m.nodes,
                                                      m.leaf_parent, m.top_pos, m.root_box);
    if (nchunks > 1) {
      static const bool attr_set = [] {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_refit_top),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, kTopLds * (int)sizeof(int));
        return true;
      }();
      (void)attr_set;
      // at most nchunks * 64 top nodes; the LDS staging takes up to kTopStage of them
      const int64_t maxtop = std::min<int64_t>((int64_t)nchunks * 64, m.nt);
      const int cap = (int)std::min<int64_t>(maxtop, kTopStage);
      const size_t bytes = std::max<size_t>((size_t)maxtop * sizeof(int), (size_t)cap * 14 * sizeof(int));
      k_refit_top<<<1, 1024, bytes, s>>>(m.nodes, m.top_pos, m.top_list, m.top_pre, m.top_count, m.root_box, cap);
    }
    return;
  }
  if (kRefitSingleWg && m.nt >= 2 && m.nt - 1 <= kRefitWgMaxNodes) {
    const size_t bytes = (size_t)(m.nt - 1) * sizeof(int);
    static const bool attr_set = [] {
      for (const void *fn : {reinterpret_cast<const void *>(&k_refit_wg<true>),
                             reinterpret_cast<const void *>(&k_refit_wg<false>)})
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  kRefitWgMaxNodes * (int)sizeof(int));
      return true;
    }();
    (void)attr_set;
    if (m.f32)
      k_refit_wg<true><<<1, kRefitBlock, bytes, s>>>(m.leaf_tri, m.nt, m.x64, m.x32, m.nv, m.nodes, m.leaf_parent,
                                                     m.root_box);
    else
      k_refit_wg<false><<<1, kRefitBlock, bytes, s>>>(m.leaf_tri, m.nt, m.x64, m.x32, m.nv, m.nodes,
                                                      m.leaf_parent, m.root_box);
    return;
  }
  if (m.f32)
    k_refit<true><<<grid_for(m.nt, 256), 256, 0, s>>>(m.leaf_tri, m.nt, m.x64, m.x32, m.nv, m.nodes,
                                                      m.leaf_parent, m.counters, m.root_box);
  else
    k_refit<false><<<grid_for(m.nt, 256), 256, 0, s>>>(m.leaf_tri, m.nt, m.x64, m.x32, m.nv, m.nodes,
                                                       m.leaf_parent, m.counters, m.root_box);
}

}  // namespace hfcr
