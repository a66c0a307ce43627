// Response: stencils, constraints, impact zones, the per-zone minimum
// displacement solve and the position update.
//
// Stencil (Section 4, Fig. 3): the endpoint x0 of an intersecting edge that
// lies behind the oriented face, plus the face's three vertices.  Stencils
// are keyed (dir, x0, f), sorted and made unique, so two E-F hits that give
// the same stencil count once.
//
// Constraint (Eq. 1, Eq. 2, Eq. 8): D = n . [x0 - (x1 + x2 + x3)/3] with the
// face's unit normal n = (x2 - x1) x (x3 - x1) / |.|; gradient coefficients
// +1 on x0 and -1/3 on each face vertex; right-hand side r = D - d.
//
// Impact zones (Section 4, "Implementation"): stencils sharing a vertex,
// closed transitively, by a lock-free union-find on global vertex ids that
// always hooks the larger root under the smaller one (so every component's
// root is its smallest vertex id, whatever the interleaving).
//
// Zone solve (Eq. 7, Eq. 8): A lambda = r with A_ij = (n_i . n_j) *
// sum over shared vertices v of w_v c_iv c_jv.  One workgroup per zone
// factors A by Cholesky with diagonal pivoting, stopping when the largest
// remaining pivot is at most tau * max(diag A) (tau = 1e-12).  Full rank:
// two triangular solves.  Rank r < k: with the k-by-r factor L,
// lambda = L (L^T L)^-1 (L^T L)^-1 L^T r, the minimum-norm least-squares
// solution, for which x' below does not depend on the choice of lambda.
//
// Update (Eq. 5): x'_v = x_v - w_v sum_i c_iv n_i lambda_i, gathered per
// vertex over its (stencil, slot) incidences in stencil order, so the sum
// order is fixed.  Float32 storage is rounded to nearest afterwards.
#include "common.hpp"
#include "kernels.hpp"
#include "wgsort.hpp"

#pragma clang fp contract(off)

namespace hfcr {

// ---------------------------------------------------------------- stencils
__global__ void k_stencil_keys(const uint64_t *__restrict__ hk, const uint32_t *__restrict__ hv, int64_t n,
                               HitLayout hl, StencilLayout sl, uint64_t *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t k = hk[i];
  uint64_t f = k & ((1ull << hl.bits_f) - 1);
  uint64_t dir = k >> (hl.bits_e + hl.bits_f);
  out[i] = (dir << (sl.bits_v + sl.bits_f)) | ((uint64_t)hv[i] << sl.bits_f) | f;
}

void launch_stencil_keys(const uint64_t *hk, const uint32_t *hv, int64_t n, HitLayout hl, StencilLayout sl,
                         uint64_t *out, hipStream_t s) {
  if (n > 0) k_stencil_keys<<<grid_for(n, 256), 256, 0, s>>>(hk, hv, n, hl, sl, out);
}

__global__ void k_compact_keys(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ flags,
                               const uint32_t *__restrict__ pos, int64_t n, uint64_t *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flags[i]) out[pos[i]] = keys[i];
}

void launch_compact_keys(const uint64_t *keys, const uint32_t *flags, const uint32_t *pos, int64_t n,
                         uint64_t *out, hipStream_t s) {
  if (n > 0) k_compact_keys<<<grid_for(n, 256), 256, 0, s>>>(keys, flags, pos, n, out);
}

// The stencil build for at most 1024 hits in one workgroup (keys of up to two
// hit lists, sorting network, unique, compaction): the same keys, order and
// count as the multi-kernel path.  The unique keys go to out[0..count) and to
// sk[0..count); every thread gets the count.
__device__ uint32_t stencils_wg(const uint64_t *__restrict__ hk0, const uint32_t *__restrict__ hv0, int n0,
                                const uint64_t *__restrict__ hk1, const uint32_t *__restrict__ hv1, int n1,
                                HitLayout hl, StencilLayout sl, uint64_t *out, uint64_t *sk, uint32_t *sv,
                                uint32_t *wsum) {
  const int t = threadIdx.x;
  const int n = n0 + n1;
  uint64_t k = ~0ull;
  uint32_t v = 0;
  if (t < n) {
    const uint64_t hk = t < n0 ? hk0[t] : hk1[t - n0];
    const uint32_t hv = t < n0 ? hv0[t] : hv1[t - n0];
    const uint64_t f = hk & ((1ull << hl.bits_f) - 1);
    const uint64_t dir = hk >> (hl.bits_e + hl.bits_f);
    k = (dir << (sl.bits_v + sl.bits_f)) | ((uint64_t)hv << sl.bits_f) | f;
  }
  int P = 2;
  while (P < n) P <<= 1;
  wg_bitonic_1k(k, v, P, sk, sv);
  sk[t] = k;
  __syncthreads();
  const bool flag = k != ~0ull && (t == 0 || sk[t - 1] != k);
  const uint64_t m = __ballot(flag);
  const int lane = t & (kWave - 1), wave = t / kWave;
  if (lane == 0) wsum[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t before = 0, count = 0;
  for (int w = 0; w < 1024 / kWave; ++w) {
    if (w < wave) before += wsum[w];
    count += wsum[w];
  }
  const uint32_t pos = before + (uint32_t)__popcll(m & (lane ? (~0ull >> (64 - lane)) : 0ull));
  if (flag) out[pos] = k;
  __syncthreads();  // every read of sk and wsum above is done
  if (flag) sk[pos] = k;
  __syncthreads();
  return count;
}

__global__ __launch_bounds__(1024) void k_stencils_small(const uint64_t *__restrict__ hk0,
                                                         const uint32_t *__restrict__ hv0, int n0,
                                                         const uint64_t *__restrict__ hk1,
                                                         const uint32_t *__restrict__ hv1, int n1, HitLayout hl,
                                                         StencilLayout sl, uint64_t *out, uint32_t *total) {
  __shared__ uint64_t sk[1024];
  __shared__ uint32_t sv[1024];
  __shared__ uint32_t wsum[1024 / kWave];
  const uint32_t count = stencils_wg(hk0, hv0, n0, hk1, hv1, n1, hl, sl, out, sk, sv, wsum);
  if (threadIdx.x == 0) *total = count;
}

bool launch_stencils_small(const uint64_t *hk0, const uint32_t *hv0, int64_t n0, const uint64_t *hk1,
                           const uint32_t *hv1, int64_t n1, HitLayout hl, StencilLayout sl, uint64_t *out,
                           uint32_t *total, hipStream_t s) {
  if (n0 + n1 <= 0 || n0 + n1 > 1024) return false;
  k_stencils_small<<<1, 1024, 0, s>>>(hk0, hv0, (int)n0, hk1, hv1, (int)n1, hl, sl, out, total);
  return true;
}

__global__ void k_write_stencils(const uint64_t *__restrict__ keys, int64_t n, StencilLayout sl, int32_t *out) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t k = keys[i];
  out[3 * i + 0] = (int32_t)(k >> (sl.bits_v + sl.bits_f));
  out[3 * i + 1] = (int32_t)((k >> sl.bits_f) & ((1ull << sl.bits_v) - 1));
  out[3 * i + 2] = (int32_t)(k & ((1ull << sl.bits_f) - 1));
}

void launch_write_stencils(const uint64_t *keys, int64_t n, StencilLayout sl, int32_t *out, hipStream_t s) {
  if (n > 0) k_write_stencils<<<grid_for(n, 256), 256, 0, s>>>(keys, n, sl, out);
}

// ------------------------------------------------------------- constraints
struct MeshView {
  const double *x64;
  const int32_t *tri;
  int nv;
};

// Constraint of the stencil with key k (Eq. 1, Eq. 2, Eq. 8).
__device__ Constraint make_constraint(uint64_t k, StencilLayout sl, const MeshView &A, const MeshView &B,
                                      double d) {
  int dir = (int)(k >> (sl.bits_v + sl.bits_f));
  int x0 = (int)((k >> sl.bits_f) & ((1ull << sl.bits_v) - 1));
  int f = (int)(k & ((1ull << sl.bits_f) - 1));
  const MeshView &E = dir == 0 ? A : B;
  const MeshView &F = dir == 0 ? B : A;
  int t0 = F.tri[3 * (int64_t)f], t1 = F.tri[3 * (int64_t)f + 1], t2 = F.tri[3 * (int64_t)f + 2];
  double P[4][3];
  for (int c = 0; c < 3; ++c) {
    P[0][c] = E.x64[(int64_t)c * E.nv + x0];
    P[1][c] = F.x64[(int64_t)c * F.nv + t0];
    P[2][c] = F.x64[(int64_t)c * F.nv + t1];
    P[3][c] = F.x64[(int64_t)c * F.nv + t2];
  }
  double e1[3], e2[3];
  for (int c = 0; c < 3; ++c) {
    e1[c] = P[2][c] - P[1][c];
    e2[c] = P[3][c] - P[1][c];
  }
  double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  double len = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
  double n[3] = {0.0, 0.0, 0.0};
  if (len > 0.0)
    for (int c = 0; c < 3; ++c) n[c] = cr[c] / len;
  double D = 0.0;
  for (int c = 0; c < 3; ++c) {
    double centroid = (P[1][c] + P[2][c] + P[3][c]) / 3.0;
    D += n[c] * (P[0][c] - centroid);
  }
  Constraint out;
  out.n = make_double4(n[0], n[1], n[2], D - d);
  const int off_e = dir == 0 ? 0 : A.nv;  // global id offset of the edge mesh
  const int off_f = dir == 0 ? A.nv : 0;  // and of the face mesh
  out.v = make_int4(off_e + x0, off_f + t0, off_f + t1, off_f + t2);
  return out;
}

__global__ void k_constraints(const uint64_t *__restrict__ keys, int64_t S, StencilLayout sl, MeshView A,
                              MeshView B, double d, Constraint *con) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  con[i] = make_constraint(keys[i], sl, A, B, d);
}

void launch_constraints(const uint64_t *keys, int64_t S, StencilLayout sl, const MeshDev &A, const MeshDev &B,
                        double d, Constraint *con, hipStream_t s) {
  if (S <= 0) return;
  MeshView a{A.x64, A.tri_in, A.nv}, b{B.x64, B.tri_in, B.nv};
  k_constraints<<<grid_for(S, 256), 256, 0, s>>>(keys, S, sl, a, b, d, con);
}

// -------------------------------------------------------------- union-find
__device__ inline int uf_load(const int *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int uf_find(int *P, int x) {
  while (true) {
    int p = uf_load(P + x);
    if (p == x) return x;
    int gp = uf_load(P + p);
    if (gp != p) __hip_atomic_store(P + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // path halving
    x = gp;
  }
}

__device__ inline void uf_unite(int *P, int a, int b) {
  while (true) {
    a = uf_find(P, a);
    b = uf_find(P, b);
    if (a == b) return;
    if (a < b) {
      int t = a;
      a = b;
      b = t;
    }
    // hook the larger root a under the smaller root b
    if (atomicCAS(P + a, a, b) == a) return;
  }
}

__global__ void k_uf_init(int *parent, int n, uint32_t *clear) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) parent[i] = i;
  if (i < 2 && clear) clear[i] = 0u;  // the round's largest-zone and solve-retry counters
}

__global__ void k_uf_union(const Constraint *__restrict__ con, int64_t S, int *parent) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  int4 v = con[i].v;
  uf_unite(parent, v.x, v.y);
  uf_unite(parent, v.x, v.z);
  uf_unite(parent, v.x, v.w);
}

void launch_uf_init(int *parent, int n, uint32_t *clear, hipStream_t s) {
  k_uf_init<<<grid_for(n, 256), 256, 0, s>>>(parent, n, clear);
}
void launch_uf_union(const Constraint *con, int64_t S, int *parent, hipStream_t s) {
  if (S > 0) k_uf_union<<<grid_for(S, 256), 256, 0, s>>>(con, S, parent);
}

__global__ void k_zone_keys(const Constraint *__restrict__ con, int64_t S, int *parent, int bits_s,
                            uint64_t *keys, uint32_t *vals) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  int root = uf_find(parent, con[i].v.x);
  keys[i] = ((uint64_t)root << bits_s) | (uint64_t)i;
  vals[i] = (uint32_t)i;
}

void launch_zone_keys(const Constraint *con, int64_t S, const int *parent, int bits_s, uint64_t *keys,
                      uint32_t *vals, hipStream_t s) {
  if (S > 0) k_zone_keys<<<grid_for(S, 256), 256, 0, s>>>(con, S, const_cast<int *>(parent), bits_s, keys, vals);
}

__global__ void k_zone_flags(const uint64_t *__restrict__ keys, int64_t S, int bits_s, uint32_t *flags) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  flags[i] = (i == 0 || (keys[i] >> bits_s) != (keys[i - 1] >> bits_s)) ? 1u : 0u;
}

void launch_zone_flags(const uint64_t *keys, int64_t S, int bits_s, uint32_t *flags, hipStream_t s) {
  if (S > 0) k_zone_flags<<<grid_for(S, 256), 256, 0, s>>>(keys, S, bits_s, flags);
}

__global__ void k_zone_starts(const uint32_t *__restrict__ flags, const uint32_t *__restrict__ pos, int64_t S,
                              uint32_t *starts, uint32_t *nz) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  if (flags[i]) starts[pos[i]] = (uint32_t)i;
  if (i == S - 1) {
    uint32_t z = pos[i] + flags[i];
    starts[z] = (uint32_t)S;
    *nz = z;
  }
}

__global__ void k_zone_maxk(const uint32_t *__restrict__ starts, const uint32_t *__restrict__ nz, uint32_t *maxk) {
  uint32_t n = *nz;
  uint32_t m = 0;
  for (uint32_t z = blockIdx.x * blockDim.x + threadIdx.x; z < n; z += gridDim.x * blockDim.x) {
    uint32_t k = starts[z + 1] - starts[z];
    m = k > m ? k : m;
  }
  atomicMax(maxk, m);
}

void launch_zone_starts(const uint32_t *flags, const uint32_t *pos, int64_t S, uint32_t *starts, uint32_t *nz,
                        uint32_t *maxk, hipStream_t s) {
  if (S <= 0) return;
  k_zone_starts<<<grid_for(S, 256), 256, 0, s>>>(flags, pos, S, starts, nz);
  k_zone_maxk<<<64, 256, 0, s>>>(starts, nz, maxk);
}

// The whole zone stage for at most kZonesSmall stencils in one workgroup: the
// same components, keys (root, stencil), sorting network, segment flags and
// starts as the multi-kernel path, so every output is identical.  The
// union-find runs in LDS on a hash table of the stencils' vertex ids (slot =
// open addressing on the id), hooking the root with the larger vertex id under
// the other, so every root is again its component's smallest id.  clear[0]
// receives the largest zone, clear[1] (the solve's retry counter) is zeroed.
constexpr int kZonesSmall = 1024;
constexpr int kUfSlots = 8192;  // at least twice the 4 * kZonesSmall vertex ids
static_assert(kRoundSmallHits <= kZonesSmall, "the fused round uses the one-workgroup zone stage");
static_assert(kUfSlots >= 8 * kZonesSmall && (kUfSlots & (kUfSlots - 1)) == 0, "hash table size");

// Slot of vertex id v in the table (inserted if absent).  Terminates: the
// table holds at most half as many ids as slots.
__device__ inline int uf_slot(int *key, int v) {
  uint32_t h = ((uint32_t)v * 2654435761u) >> 19;  // the top 13 bits: 0 .. kUfSlots - 1
  while (true) {
    const int old = atomicCAS(key + h, -1, v);
    if (old == -1 || old == v) return (int)h;
    h = (h + 1) & (kUfSlots - 1);
  }
}

__device__ inline int lds_uf_find(int *par, int x) {
  while (true) {
    const int p = __hip_atomic_load(par + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (p == x) return x;
    const int gp = __hip_atomic_load(par + p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (gp != p) __hip_atomic_store(par + x, gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);  // path halving
    x = gp;
  }
}

__device__ inline void lds_uf_unite(int *par, const int *key, int a, int b) {
  while (true) {
    a = lds_uf_find(par, a);
    b = lds_uf_find(par, b);
    if (a == b) return;
    if (key[a] < key[b]) {
      const int t = a;
      a = b;
      b = t;
    }
    // hook root a (the larger vertex id) under root b
    if (atomicCAS(par + a, a, b) == a) return;
  }
}

// Thread t holds stencil t's vertices v (act = t < S); hkey and hpar are the
// LDS hash table (kUfSlots entries each).
__device__ void zones_wg(int4 v, bool act, int S, int bits_s, uint64_t *keys, uint32_t *vals, uint32_t *starts,
                         uint32_t *nz, uint32_t *clear, uint64_t *sk, uint32_t *sv, uint32_t *wsum, uint32_t *sst,
                         int *hkey, int *hpar) {
  const int t = threadIdx.x;
  for (int i = t; i < kUfSlots; i += blockDim.x) {
    hkey[i] = -1;
    hpar[i] = i;
  }
  __syncthreads();
  int s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  if (act) {
    s0 = uf_slot(hkey, v.x);
    s1 = uf_slot(hkey, v.y);
    s2 = uf_slot(hkey, v.z);
    s3 = uf_slot(hkey, v.w);
  }
  __syncthreads();
  if (act) {
    lds_uf_unite(hpar, hkey, s0, s1);
    lds_uf_unite(hpar, hkey, s0, s2);
    lds_uf_unite(hpar, hkey, s0, s3);
  }
  __syncthreads();
  uint64_t k = ~0ull;
  uint32_t val = 0;
  if (act) {
    k = ((uint64_t)hkey[lds_uf_find(hpar, s0)] << bits_s) | (uint64_t)t;
    val = (uint32_t)t;
  }
  int P = 2;
  while (P < S) P <<= 1;
  wg_bitonic_1k(k, val, P, sk, sv);
  if (act) {
    keys[t] = k;
    vals[t] = val;
  }
  // segment flags and their exclusive prefix (ballots per wavefront)
  sk[t] = k;
  __syncthreads();
  const bool flag = act && (t == 0 || (k >> bits_s) != (sk[t - 1] >> bits_s));
  const uint64_t m = __ballot(flag);
  const int lane = t & (kWave - 1), wave = t / kWave;
  if (lane == 0) wsum[wave] = (uint32_t)__popcll(m);
  __syncthreads();
  uint32_t before = 0, total = 0;
  for (int w = 0; w < 1024 / kWave; ++w) {
    if (w < wave) before += wsum[w];
    total += wsum[w];
  }
  const uint32_t pos = before + (uint32_t)__popcll(m & (lane ? (~0ull >> (64 - lane)) : 0ull));
  if (flag) {
    starts[pos] = (uint32_t)t;
    sst[pos] = (uint32_t)t;
  }
  if (t == 0) {
    starts[total] = (uint32_t)S;
    sst[total] = (uint32_t)S;
    *nz = total;
  }
  __syncthreads();
  // largest zone
  uint32_t kz = flag ? sst[pos + 1] - (uint32_t)t : 0u;
  for (int off = 32; off > 0; off >>= 1) kz = max(kz, (uint32_t)__shfl_xor((int)kz, off));
  __syncthreads();
  if (lane == 0) wsum[wave] = kz;
  __syncthreads();
  if (t == 0) {
    uint32_t mk = 0;
    for (int w = 0; w < 1024 / kWave; ++w) mk = max(mk, wsum[w]);
    clear[0] = mk;
    clear[1] = 0u;
  }
}

__global__ __launch_bounds__(1024) void k_zones_small(const Constraint *__restrict__ con, int S, int bits_s,
                                                      uint64_t *keys, uint32_t *vals, uint32_t *starts,
                                                      uint32_t *nz, uint32_t *clear) {
  __shared__ uint64_t sk[1024];
  __shared__ uint32_t sv[1024];
  __shared__ uint32_t wsum[1024 / kWave];
  __shared__ uint32_t sst[1024 + 1];
  __shared__ int hkey[kUfSlots];
  __shared__ int hpar[kUfSlots];
  const int t = threadIdx.x;
  const bool act = t < S;
  const int4 v = act ? con[t].v : make_int4(0, 0, 0, 0);
  zones_wg(v, act, S, bits_s, keys, vals, starts, nz, clear, sk, sv, wsum, sst, hkey, hpar);
}

bool launch_zones_small(const Constraint *con, int64_t S, int bits_s, uint64_t *keys, uint32_t *vals,
                        uint32_t *starts, uint32_t *nz, uint32_t *clear, hipStream_t s) {
  if (S <= 0 || S > kZonesSmall) return false;
  k_zones_small<<<1, 1024, 0, s>>>(con, (int)S, bits_s, keys, vals, starts, nz, clear);
  return true;
}

// Stencils, constraints and impact zones of one round for at most kZonesSmall
// hits in one workgroup: the three stages above in sequence, with the same
// outputs (stencil keys, constraints, zone keys, order, starts, counts); the
// stencil count goes to *total.  The hit counts are read from the detection
// pass's own counters (cnt1 null: no second list), so the launch can follow
// the pass before the host has seen them; a list that overflowed its buffer
// (count > cap), more than kZonesSmall hits or none leave *total = 0 and
// nothing else written.
__global__ __launch_bounds__(1024) void k_round_small(const uint64_t *__restrict__ hk0,
                                                      const uint32_t *__restrict__ hv0, const uint32_t *cnt0,
                                                      int64_t cap0, const uint64_t *__restrict__ hk1,
                                                      const uint32_t *__restrict__ hv1, const uint32_t *cnt1,
                                                      int64_t cap1, HitLayout hl, StencilLayout sl, MeshView A,
                                                      MeshView B, double d, uint64_t *st_keys, Constraint *con,
                                                      uint64_t *keys, uint32_t *vals, uint32_t *starts, uint32_t *nz,
                                                      uint32_t *clear, uint32_t *total) {
  __shared__ uint64_t sk[1024];
  __shared__ uint32_t sv[1024];
  __shared__ uint32_t wsum[1024 / kWave];
  __shared__ uint32_t sst[1024 + 1];
  __shared__ int hkey[kUfSlots];
  __shared__ int hpar[kUfSlots];
  const int t = threadIdx.x;
  const int64_t n0 = *cnt0, n1 = cnt1 ? *cnt1 : 0;
  if (n0 > cap0 || n1 > cap1 || n0 + n1 <= 0 || n0 + n1 > kRoundSmallHits) {
    if (t == 0) *total = 0u;
    return;
  }
  const int S = (int)stencils_wg(hk0, hv0, (int)n0, hk1, hv1, (int)n1, hl, sl, st_keys, sk, sv, wsum);
  const bool act = t < S;
  int4 v = make_int4(0, 0, 0, 0);
  if (act) {
    const Constraint cn = make_constraint(sk[t], sl, A, B, d);
    con[t] = cn;
    v = cn.v;
  }
  // zones_wg passes three barriers before its sorting network reuses sk
  int bits_s = 1;
  while (bits_s < 62 && (1 << bits_s) < S) ++bits_s;
  zones_wg(v, act, S, bits_s, keys, vals, starts, nz, clear, sk, sv, wsum, sst, hkey, hpar);
  if (t == 0) *total = (uint32_t)S;
}

void launch_round_small(const uint64_t *hk0, const uint32_t *hv0, const uint32_t *cnt0, int64_t cap0,
                        const uint64_t *hk1, const uint32_t *hv1, const uint32_t *cnt1, int64_t cap1, HitLayout hl,
                        StencilLayout sl, const MeshDev &A, const MeshDev &B, double d, uint64_t *st_keys,
                        Constraint *con, uint64_t *keys, uint32_t *vals, uint32_t *starts, uint32_t *nz,
                        uint32_t *clear, uint32_t *total, hipStream_t s) {
  MeshView a{A.x64, A.tri_in, A.nv}, b{B.x64, B.tri_in, B.nv};
  k_round_small<<<1, 1024, 0, s>>>(hk0, hv0, cnt0, cap0, hk1, hv1, cnt1, cap1, hl, sl, a, b, d, st_keys, con, keys,
                                   vals, starts, nz, clear, total);
}

// -------------------------------------------------------------- zone solve
// Storage: the packed lower triangle of the zone matrix, S[i(i+1)/2 + l] for
// i >= l (index order).  Pivot step j takes p = argmax of the remaining
// diagonal (ties: smaller index), stores L(i, j) = A_ip / sqrt(A_pp) where
// A_ip was kept, and updates the remaining lower triangle; the next step's
// argmax and the forward substitution L~ y = r~ are folded into that update,
// so a factorization step costs two barriers and the forward solve none.
// The remaining indices stay in increasing order (stable compaction), so
// "lower" keeps its meaning at every step.
//
// Zones of up to kZoneLds stencils keep the matrix and every vector in LDS
// (sized at launch for the largest such zone); larger zones keep the matrix
// in the workgroup's global slot (L2-resident) and the rest in LDS when it
// fits, else in the slot too.
constexpr int kSolveBlock = 256;   // pivoted path
constexpr int kTiledBlock = 1024;  // tiled path: 16 waves, four per SIMD, to hide LDS and FMA latency
constexpr int kWgBytes = 512;      // per-wave reduction slots (up to 16 waves) and a flag
constexpr int kZoneLds = 176;
constexpr int kZoneVecLds = 896;  // vectors + kWgBytes + a column of 112 tiles fit in 160 KB
constexpr int kZoneMax = 4096;  // == HFCR_MAX_ZONE

__device__ inline double inv_mass(int v, const double *wa, const double *wb, int nva) {
  if (v < nva) return wa ? wa[v] : 1.0;
  return wb ? wb[v - nva] : 1.0;
}

__device__ inline double coef(int slot) { return slot == 0 ? 1.0 : -1.0 / 3.0; }

__device__ inline int64_t tri_base(int i) { return (int64_t)i * (i + 1) / 2; }
__device__ inline int64_t lp(int i, int l) { return i >= l ? tri_base(i) + l : tri_base(l) + i; }

// (value, position, key) reduction over a wavefront: larger value, ties -> smaller key
__device__ inline void wave_argmax(double &v, int &pos, int &key) {
  for (int off = 32; off > 0; off >>= 1) {
    const double v2 = __shfl_xor(v, off);
    const int p2 = __shfl_xor(pos, off);
    const int k2 = __shfl_xor(key, off);
    if (v2 > v || (v2 == v && k2 >= 0 && (key < 0 || k2 < key))) {
      v = v2;
      pos = p2;
      key = k2;
    }
  }
}

// Per-zone arrays: 7 doubles (n.xyz, r, rhs, lcol, lam) and 8 ints
// (vertex ids x4, piv, step_of, rem x2) per stencil, plus y and 1/L_jj.
constexpr int kVecDoubles = 9;
constexpr int kVecInts = 8;

__host__ __device__ inline int round8(int k) { return (k + 7) / 8 * 8; }
__host__ __device__ inline size_t zone_vec_bytes(int k) {
  return (size_t)round8(k) * (kVecDoubles * 8 + kVecInts * 4);
}
// matrix doubles: the larger of the 8x8-tiled lower triangle and the packed one
__host__ __device__ inline size_t zone_mat_doubles(int k) {
  const size_t t = (size_t)(k + 7) / 8;
  const size_t tiled = t * (t + 1) / 2 * 64, packed = (size_t)k * (k + 1) / 2;
  return tiled > packed ? tiled : packed;
}
__host__ __device__ inline size_t zone_lds_bytes(bool mat_lds, int kcap) {
  return (mat_lds ? zone_mat_doubles(kcap) * 8 : 0) + zone_vec_bytes(kcap) + kWgBytes;
}

// ---- tiled unpivoted Cholesky (fast path) --------------------------------
// Lower tiles of 8 x 8, tile (I, J) for I >= J at (I(I+1)/2 + J) * 64.
// Inside a tile, element (r, c) sits at 8r + (c xor r): the rows are 64 B
// apart, so without the swizzle the eight rows of a column would fall on
// the same few LDS banks; with it they fall on eight different ones.  The
// matrix is padded to a multiple of 8 with diag = max diag A (so padded
// rows never trip the pivot test) and rhs 0.
constexpr int TB = 8;
typedef double mfma_d4 __attribute__((ext_vector_type(4)));  // an fp64 MFMA accumulator
__device__ inline int64_t tile_off(int I, int J) { return ((int64_t)I * (I + 1) / 2 + J) * (TB * TB); }
__device__ inline int sw(int r, int c) { return r * TB + (c ^ r); }

// Value of v in lane `lane` (a compile-time or wave-uniform index).
__device__ inline double read_lane(double v, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Returns true when every pivot exceeds thr_u; on success lam[0..k) holds the
// solution.  On failure the matrix storage is garbage (the caller reassembles).
// STAGE (matrix in global memory): each step's factored diagonal tile and
// column of tiles are also written to LDS (P: 64 + 64 (T - 1) doubles), and
// the panel and trailing update read them there, so the trailing update's
// only global accesses are the tile it updates.
template <int BLOCK, bool STAGE>
__device__ bool tiled_solve(double *M, int k, const double *nx, const double *ny, const double *nz,
                            const int *v0, const int *v1, const int *v2, const int *v3, const double *rr,
                            double *rhs, double *y, double *dinv, double *lam, const SolveArgs &a, double dmax,
                            int *flag, double *P) {
  const int tid = threadIdx.x;
  const int T = (k + TB - 1) / TB;
  const int kp = T * TB;
  // assemble the lower tiles (diagonal tiles: full, the upper half is ignored)
  const int64_t ntile_el = (int64_t)T * (T + 1) / 2 * (TB * TB);
  int I = 0;  // tile row of this thread's current element, advanced incrementally
  for (int64_t e = tid; e < ntile_el; e += BLOCK) {
    const int64_t t = e >> 6;
    const int rc = (int)(e & 63), r = rc >> 3, c = rc & 7;
    while ((int64_t)(I + 1) * (I + 2) / 2 <= t) ++I;
    const int J = (int)(t - (int64_t)I * (I + 1) / 2);
    const int i = I * TB + r, l = J * TB + c;
    double val = 0.0;
    if (i < k && l < k) {
      const int vi[4] = {v0[i], v1[i], v2[i], v3[i]};
      const int vl[4] = {v0[l], v1[l], v2[l], v3[l]};
      double acc = 0.0;
      for (int s = 0; s < 4; ++s)
        for (int u = 0; u < 4; ++u)
          if (vi[s] == vl[u]) acc += inv_mass(vi[s], a.w_a, a.w_b, a.nv_a) * coef(s) * coef(u);
      val = acc * (nx[i] * nx[l] + ny[i] * ny[l] + nz[i] * nz[l]);
    } else if (i == l) {
      val = dmax > 0.0 ? dmax : 1.0;
    }
    M[t * (TB * TB) + sw(r, c)] = val;
  }
  for (int i = tid; i < kp; i += BLOCK) rhs[i] = i < k ? rr[i] : 0.0;
  if (tid == 0) *flag = 0;
  __syncthreads();
  const double thr_u = 1e-6 * dmax;
  // (1) diagonal tile J and the forward substitution of its block: lane r < 8
  // of wave 0 holds row r of the tile, its rhs entry, y_r and 1/L_rr.
  // Column by column: the pivot is read from its lane, the column scaled and
  // the trailing lower part updated, each value computed as the serial
  // column-oriented algorithm computes it.  Values move between lanes by
  // lane reads (scalar registers), not through LDS.  Called by wave 0 only.
  auto factor_diag = [&](int J) {
    double *D = M + tile_off(J, J);
    const int r = tid;
    double row[TB];
#pragma unroll
    for (int c = 0; c < TB; ++c) row[c] = (r < TB && r >= c) ? D[sw(r, c)] : 0.0;
    double rb = r < TB ? rhs[J * TB + r] : 0.0, yv = 0.0, dv = 0.0;
    bool bad = false;
#pragma unroll
    for (int c = 0; c < TB; ++c) {
      const double piv = read_lane(row[c], c);
      bad = bad || !(piv > thr_u);
      // one reciprocal square root on the serial chain instead of a square
      // root and a division (both within an ulp or so; a failed pivot is
      // redone by the pivoted path anyway)
      const double pv = fmax(piv, 0.0), inv = rsqrt(pv), l = pv * inv;
      if (r > c) row[c] = row[c] * inv;
      if (r == c) row[c] = l;
#pragma unroll
      for (int cc = c + 1; cc < TB; ++cc) {
        const double lcc = read_lane(row[c], cc);  // L[cc][c]
        if (r >= cc) row[cc] = row[cc] - row[c] * lcc;
      }
      // forward substitution of the block's rhs
      const double yc = read_lane(rb, c) * inv;
      if (r == c) {
        yv = yc;
        dv = inv;
      }
      if (r < TB && r > c) rb = rb - row[c] * yc;
    }
    if (bad) {
      if (tid == 0) *flag = 1;
    } else if (r < TB) {
#pragma unroll
      for (int c = 0; c < TB; ++c)
        if (c <= r) {
          D[sw(r, c)] = row[c];
          if (STAGE) P[sw(r, c)] = row[c];
        }
      y[J * TB + r] = yv;
      dinv[J * TB + r] = dv;
    }
  };
  if (tid < kWave) factor_diag(0);
  __syncthreads();
  if (*flag) return false;
  for (int J = 0; J < T; ++J) {
    double *D = M + tile_off(J, J);
    // (2) panel: L_IJ = A_IJ L_JJ^-T, and the forward-substitution update
    for (int it = tid; it < (T - J - 1) * TB; it += BLOCK) {
      const int I = J + 1 + it / TB, r = it % TB;
      double *B = M + tile_off(I, J);
      const double *Dp = STAGE ? P : D;
      double x[TB];
#pragma unroll
      for (int c = 0; c < TB; ++c) x[c] = B[sw(r, c)];
#pragma unroll
      for (int c = 0; c < TB; ++c) {
        double s = x[c];
#pragma unroll
        for (int m = 0; m < c; ++m) s = s - x[m] * Dp[sw(c, m)];
        x[c] = s * dinv[J * TB + c];
      }
      double acc = 0.0;
#pragma unroll
      for (int c = 0; c < TB; ++c) {
        B[sw(r, c)] = x[c];
        if (STAGE) P[(I - J) * (TB * TB) + sw(r, c)] = x[c];
        acc = acc + x[c] * y[J * TB + c];
      }
      rhs[I * TB + r] = rhs[I * TB + r] - acc;
    }
    __syncthreads();
    // (3) trailing update: A_IK -= L_IJ L_KJ^T for J < K <= I on the fp64
    // matrix cores.  The trailing tiles are taken in 2 x 2 blocks of 16 x 16
    // (block rows and columns of two tile rows each, the last one ragged when
    // the count is odd); one wavefront per block computes
    // D = C + (-L_I) L_K^T with two 16x16x4 fp64 MFMAs (the panel's eight
    // columns, four per MFMA) and stores the tiles on or below the diagonal.
    // Lane layout of the MFMA: A row l % 16, k l / 16; B column l % 16, k
    // l / 16; D row l / 16 + 4 v, column l % 16 (v = 0..3).
    // Look-ahead: wave 0 takes block (0, 0), which holds tile (J+1, J+1),
    // and then factors that tile, while the other wavefronts update the
    // rest, so the serial diagonal factorization overlaps the update.
    {
      const int nrem = T - J - 1;
      const int nb = (nrem + 1) >> 1;
      const int nblk = nb * (nb + 1) / 2;
      const int lane = tid & 63, wave = tid >> 6;
      const int li = lane & 15, lk = lane >> 4;
      int u = 0;  // block row of this wave's current block, advanced incrementally
      for (int q = wave; q < (wave == 0 ? min(nblk, 1) : nblk); q += (wave == 0 ? 1 : BLOCK / 64 - 1)) {
        while ((u + 1) * (u + 2) / 2 <= q) ++u;
        const int v = q - u * (u + 1) / 2;
        const int I0 = J + 1 + 2 * u, K0 = J + 1 + 2 * v;
        // operands: row li of the 16 x 8 panels of block row u and block column v
        const int Ia = I0 + (li >> 3), Kb = K0 + (li >> 3), ra = li & 7;
        const double *LA = STAGE ? P + (Ia - J) * (TB * TB) : M + (Ia * (Ia + 1) / 2 + J) * (TB * TB);
        const double *LB = STAGE ? P + (Kb - J) * (TB * TB) : M + (Kb * (Kb + 1) / 2 + J) * (TB * TB);
        const double a0 = Ia < T ? -LA[sw(ra, lk)] : 0.0, a1 = Ia < T ? -LA[sw(ra, lk + 4)] : 0.0;
        const double b0 = Kb < T ? LB[sw(ra, lk)] : 0.0, b1 = Kb < T ? LB[sw(ra, lk + 4)] : 0.0;
        // accumulator: rows lk + 4 v, column li of the block
        const int Kc = K0 + (li >> 3), cc = li & 7;
        mfma_d4 acc;
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int i = lk + 4 * w, Ic = I0 + (i >> 3);
          acc[w] = (Ic < T && Kc <= Ic) ? M[(Ic * (Ic + 1) / 2 + Kc) * (TB * TB) + sw(i & 7, cc)] : 0.0;
        }
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc, 0, 0, 0);
#pragma unroll
        for (int w = 0; w < 4; ++w) {
          const int i = lk + 4 * w, Ic = I0 + (i >> 3);
          if (Ic < T && Kc <= Ic) M[(Ic * (Ic + 1) / 2 + Kc) * (TB * TB) + sw(i & 7, cc)] = acc[w];
        }
      }
      if (wave == 0 && J + 1 < T) {
        __threadfence_block();  // this wavefront's update of tile (J+1, J+1) is read by other lanes
        factor_diag(J + 1);
      }
    }
    __syncthreads();
    if (*flag) return false;
  }
  // backward: L^T lambda = y, tile by tile
  for (int J = T - 1; J >= 0; --J) {
    const double *D = M + tile_off(J, J);
    if (tid == 0) {
      double lb[TB];
#pragma unroll
      for (int c = TB - 1; c >= 0; --c) {
        double s2 = y[J * TB + c];
#pragma unroll
        for (int m = c + 1; m < TB; ++m) s2 = s2 - D[sw(m, c)] * lb[m];
        lb[c] = s2 * dinv[J * TB + c];
      }
#pragma unroll
      for (int c = 0; c < TB; ++c) lam[J * TB + c] = lb[c];
    }
    __syncthreads();
    for (int it = tid; it < J * TB; it += BLOCK) {
      const int K = it / TB, c = it % TB;
      const double *B = M + tile_off(J, K);
      double s = 0.0;
#pragma unroll
      for (int r = 0; r < TB; ++r) s = s + B[sw(r, c)] * lam[J * TB + r];
      y[K * TB + c] = y[K * TB + c] - s;
    }
    __syncthreads();
  }
  return true;
}

// Tiled path of every zone with kmin < k <= kcap; a zone whose tiled
// factorization meets a small pivot is appended to a.retry for k_solve.
template <bool MAT_LDS, bool VEC_LDS>
__global__ __launch_bounds__(kTiledBlock) void k_solve_tiled(SolveArgs a, int kmin, int kcap) {
  constexpr bool vec_lds = VEC_LDS;  // compile-time, so LDS accesses stay ds_* (never flat)
  extern __shared__ double dyn[];
  constexpr int NW = kTiledBlock / 64;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  double *S_lds = dyn;
  double *vec_lds_base = dyn + (MAT_LDS ? (int64_t)zone_mat_doubles(kcap) : 0);
  double *wv = vec_lds_base + (vec_lds ? zone_vec_bytes(kcap) / 8 : 0);
  int *flag = reinterpret_cast<int *>(wv + NW);
  constexpr bool stage = !MAT_LDS && VEC_LDS;  // global matrix, LDS to spare for a column of tiles
  double *P = wv + kWgBytes / 8;
  for (int z = blockIdx.x; z < a.nzones; z += gridDim.x) {
    const int st = (int)a.starts[z];
    const int k = (int)a.starts[z + 1] - st;
    if (k <= kmin || k > kcap) continue;
    double *slot = a.scratch + (int64_t)blockIdx.x * a.slot_stride;
    double *S = MAT_LDS ? S_lds : slot;
    double *Cm = slot + zone_mat_doubles(k);
    double *vb = vec_lds ? vec_lds_base : Cm + tri_base(k);
    const int k8 = round8(k);
    double *nx = vb, *ny = vb + k8, *nz = vb + 2 * k8, *rr = vb + 3 * k8, *rhs = vb + 4 * k8, *lam = vb + 6 * k8,
           *y = vb + 7 * k8, *dinv = vb + 8 * k8;
    int *ib = reinterpret_cast<int *>(vb + kVecDoubles * k8);
    int *v0 = ib, *v1 = ib + k8, *v2 = ib + 2 * k8, *v3 = ib + 3 * k8;
    for (int i = tid; i < k; i += kTiledBlock) {
      const Constraint c = a.con[a.order[st + i]];
      nx[i] = c.n.x;
      ny[i] = c.n.y;
      nz[i] = c.n.z;
      rr[i] = c.n.w;
      v0[i] = c.v.x;
      v1[i] = c.v.y;
      v2[i] = c.v.z;
      v3[i] = c.v.w;
    }
    __syncthreads();
    // largest diagonal entry: A_ii = (n_i . n_i) (w_x0 + (w_1 + w_2 + w_3) / 9)
    double dmax = 0.0;
    {
      double v = 0.0;
      int pos = 0, key = 0;
      for (int i = tid; i < k; i += kTiledBlock) {
        const double d = (nx[i] * nx[i] + ny[i] * ny[i] + nz[i] * nz[i]) *
                         (inv_mass(v0[i], a.w_a, a.w_b, a.nv_a) +
                          (inv_mass(v1[i], a.w_a, a.w_b, a.nv_a) + inv_mass(v2[i], a.w_a, a.w_b, a.nv_a) +
                           inv_mass(v3[i], a.w_a, a.w_b, a.nv_a)) / 9.0);
        v = fmax(v, d);
      }
      wave_argmax(v, pos, key);
      if (lane == 0) wv[wave] = v;
      __syncthreads();
      for (int w = 0; w < NW; ++w) dmax = fmax(dmax, wv[w]);
      __syncthreads();
    }
    if (tiled_solve<kTiledBlock, stage>(S, k, nx, ny, nz, v0, v1, v2, v3, rr, rhs, y, dinv, lam, a, dmax, flag, P)) {
      for (int i = tid; i < k; i += kTiledBlock) a.lambda[a.order[st + i]] = lam[i];
    } else if (tid == 0) {
      atomicAdd(a.pivoted, 1);
      a.retry[atomicAdd(a.retry_n, 1u)] = (uint32_t)z;
    }
    __syncthreads();
  }
}

// Pivoted (rank-revealing) path of the zones the tiled path handed over.
// The matrix-in-LDS class keeps 256 threads (its trailing update holds a
// row block in registers); the global-matrix classes use 1024.
template <bool MAT_LDS, bool VEC_LDS>
__global__ __launch_bounds__(MAT_LDS ? kSolveBlock : kTiledBlock) void k_solve(SolveArgs a, int kmin, int kcap) {
  constexpr int BLOCK = MAT_LDS ? kSolveBlock : kTiledBlock;
  constexpr bool vec_lds = VEC_LDS;  // compile-time, so LDS accesses stay ds_* (never flat)
  extern __shared__ double dyn[];
  constexpr int TY = 16;  // 16 x 16 tiling of the trailing update
  constexpr int NW = BLOCK / 64;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int tx = tid % TY, ty = tid / TY;
  double *S_lds = dyn;
  double *vec_lds_base = dyn + (MAT_LDS ? (int64_t)zone_mat_doubles(kcap) : 0);
  double *wv = vec_lds_base + (vec_lds ? zone_vec_bytes(kcap) / 8 : 0);
  int *wp = reinterpret_cast<int *>(wv + NW);
  int *wk = wp + NW;
  int *flag = wk + NW;
  const uint32_t nretry = *a.retry_n;
  for (uint32_t q = blockIdx.x; q < nretry; q += gridDim.x) {
    const int z = (int)a.retry[q];
    const int st = (int)a.starts[z];
    const int k = (int)a.starts[z + 1] - st;
    if (k <= kmin || k > kcap) continue;  // another class's zone
    double *slot = a.scratch + (int64_t)blockIdx.x * a.slot_stride;
    double *S = MAT_LDS ? S_lds : slot;
    double *Cm = slot + zone_mat_doubles(k);  // rank-deficient case only (packed r x r)
    double *vb = vec_lds ? vec_lds_base : Cm + tri_base(k);
    const int k8 = round8(k);
    double *nx = vb, *ny = vb + k8, *nz = vb + 2 * k8, *rr = vb + 3 * k8, *rhs = vb + 4 * k8, *lcol = vb + 5 * k8,
           *lam = vb + 6 * k8, *y = vb + 7 * k8, *dinv = vb + 8 * k8;
    int *ib = reinterpret_cast<int *>(vb + kVecDoubles * k8);
    int *v0 = ib, *v1 = ib + k8, *v2 = ib + 2 * k8, *v3 = ib + 3 * k8, *piv = ib + 4 * k8, *step_of = ib + 5 * k8,
        *rem0 = ib + 6 * k8, *rem1 = ib + 7 * k8;
    // stage the zone's constraints
    for (int i = tid; i < k; i += BLOCK) {
      const Constraint c = a.con[a.order[st + i]];
      nx[i] = c.n.x;
      ny[i] = c.n.y;
      nz[i] = c.n.z;
      rr[i] = c.n.w;
      rhs[i] = c.n.w;
      v0[i] = c.v.x;
      v1[i] = c.v.y;
      v2[i] = c.v.z;
      v3[i] = c.v.w;
      step_of[i] = k;
      rem0[i] = i;
    }
    __syncthreads();
    double dmax = 0.0;
    // Cholesky with diagonal pivoting (rank-revealing)
    for (int i = tid; i < k; i += BLOCK) {
      rhs[i] = rr[i];
      step_of[i] = k;
      rem0[i] = i;
    }
    __syncthreads();
    // assemble the packed lower triangle
    for (int i = ty; i < k; i += BLOCK / TY) {
      const int vi[4] = {v0[i], v1[i], v2[i], v3[i]};
      double wi[4];
      for (int s = 0; s < 4; ++s) wi[s] = inv_mass(vi[s], a.w_a, a.w_b, a.nv_a) * coef(s);
      const double nix = nx[i], niy = ny[i], niz = nz[i];
      const int64_t base = tri_base(i);
      for (int l = tx; l <= i; l += TY) {
        const int vl[4] = {v0[l], v1[l], v2[l], v3[l]};
        double acc = 0.0;
        for (int s = 0; s < 4; ++s)
          for (int t = 0; t < 4; ++t)
            if (vi[s] == vl[t]) acc += wi[s] * coef(t);
        S[base + l] = acc * (nix * nx[l] + niy * ny[l] + niz * nz[l]);
      }
    }
    __syncthreads();
    // first argmax (also the largest diagonal, which scales the threshold)
    {
      double v = -1.0;
      int pos = -1, key = -1;
      for (int i = tid; i < k; i += BLOCK) {
        const double d = S[tri_base(i) + i];
        if (d > v) { v = d; pos = i; key = i; }
      }
      wave_argmax(v, pos, key);
      if (lane == 0) { wv[wave] = v; wp[wave] = pos; wk[wave] = key; }
      __syncthreads();
    }
    dmax = wv[0];
    for (int w = 1; w < NW; ++w) dmax = fmax(dmax, wv[w]);
    const double thresh = a.tau * dmax;
    int rank = k;
    int *rem = rem0, *rem2 = rem1;
    for (int j = 0; j < k; ++j) {
      const int nrem = k - j;
      double best = wv[0];
      int q0 = wp[0], p = wk[0];
      for (int w = 1; w < NW; ++w) {
        const double vw = wv[w];
        const int kw = wk[w];
        if (vw > best || (vw == best && kw >= 0 && (p < 0 || kw < p))) {
          best = vw;
          q0 = wp[w];
          p = kw;
        }
      }
      if (!(best > thresh)) {
        rank = j;
        break;
      }
      const double lpp = sqrt(best);
      const double inv = 1.0 / lpp;
      const double yj = rhs[p] * inv;  // forward substitution, step j
      // B: column p of L and the stable compaction of the remaining list
      for (int q = tid; q < nrem; q += BLOCK) {
        if (q == q0) continue;
        const int i = rem[q];
        const int64_t at = lp(i, p);
        const double l = S[at] * inv;
        S[at] = l;
        const int qn = q < q0 ? q : q - 1;
        rem2[qn] = i;
        lcol[qn] = l;
      }
      if (tid == 0) {
        S[tri_base(p) + p] = lpp;
        dinv[j] = inv;
        y[j] = yj;
        piv[j] = p;
        step_of[p] = j;
      }
      __syncthreads();
      // C: trailing update, forward-substitution update, next argmax
      const int nr = nrem - 1;
      double v = -1.0;
      int pos = -1, key = -1;
      if (MAT_LDS) {
        // this thread's columns c = tx + 16 m and rows r = ty + 16 a, held in
        // registers; each row's entries are loaded before any is stored (the
        // columns of a row are distinct, so the stores cannot alias the loads)
        constexpr int MC = (kZoneLds + TY - 1) / TY;
        int cidx[MC];
        double cval[MC];
#pragma unroll
        for (int m = 0; m < MC; ++m) {
          const int c = tx + TY * m;
          cidx[m] = c < nr ? rem2[c] : 0;
          cval[m] = c < nr ? lcol[c] : 0.0;
        }
        int ridx[MC];
        double rval[MC];
#pragma unroll
        for (int a2 = 0; a2 < MC; ++a2) {
          const int r = ty + TY * a2;
          ridx[a2] = r < nr ? rem2[r] : 0;
          rval[a2] = r < nr ? lcol[r] : 0.0;
        }
#pragma unroll
        for (int a2 = 0; a2 < MC; ++a2) {
          const int r = ty + TY * a2;
          if (r >= nr) break;
          const int i = ridx[a2];
          const double li = rval[a2];
          if (tx == 0) rhs[i] = rhs[i] - li * yj;
          double *row = S + tri_base(i);
          double old[MC];
#pragma unroll
          for (int m = 0; m < MC; ++m) old[m] = (tx + TY * m <= r) ? row[cidx[m]] : 0.0;
#pragma unroll
          for (int m = 0; m < MC; ++m) {
            const int c = tx + TY * m;
            if (c <= r) {
              const double nv = old[m] - li * cval[m];
              row[cidx[m]] = nv;
              if (c == r && (nv > v || (nv == v && i < key))) { v = nv; pos = r; key = i; }
            }
          }
        }
      } else {
        constexpr int CH = 4;  // columns loaded per batch
        for (int r = ty; r < nr; r += BLOCK / TY) {
          const int i = rem2[r];
          const double li = lcol[r];
          if (tx == 0) rhs[i] = rhs[i] - li * yj;
          double *row = S + tri_base(i);
          for (int c0 = tx; c0 <= r; c0 += TY * CH) {
            int ci[CH];
            double old[CH], cv[CH];
#pragma unroll
            for (int m = 0; m < CH; ++m) {
              const int c = c0 + TY * m;
              ci[m] = c <= r ? rem2[c] : 0;
              cv[m] = c <= r ? lcol[c] : 0.0;
            }
#pragma unroll
            for (int m = 0; m < CH; ++m) old[m] = (c0 + TY * m <= r) ? row[ci[m]] : 0.0;
#pragma unroll
            for (int m = 0; m < CH; ++m) {
              const int c = c0 + TY * m;
              if (c <= r) {
                const double nv = old[m] - li * cv[m];
                row[ci[m]] = nv;
                if (c == r && (nv > v || (nv == v && i < key))) { v = nv; pos = r; key = i; }
              }
            }
          }
        }
      }
      wave_argmax(v, pos, key);
      if (lane == 0) { wv[wave] = v; wp[wave] = pos; wk[wave] = key; }
      int *t = rem;
      rem = rem2;
      rem2 = t;
      __syncthreads();
    }
    if (rank == k) {
      // backward: L~^T lambda~ = y
      if (MAT_LDS) {
        // k <= BLOCK here: thread tid owns y[tid] in a register
        const int my_p = tid < k ? piv[tid] : 0;
        double my_y = tid < k ? y[tid] : 0.0;
        for (int j = k - 1; j >= 0; --j) {
          if (tid == j) {
            const double lj = my_y * dinv[j];
            lam[my_p] = lj;
            y[j] = lj;
          }
          __syncthreads();
          const double lj = y[j];
          const int pj = piv[j];
          if (tid < j) my_y = my_y - S[lp(pj, my_p)] * lj;
        }
        __syncthreads();
      } else {
        for (int j = k - 1; j >= 0; --j) {
          const int pj = piv[j];
          const double lj = y[j] * dinv[j];
          for (int jj = tid; jj < j; jj += BLOCK) y[jj] = y[jj] - S[lp(pj, piv[jj])] * lj;
          if (tid == 0) lam[pj] = lj;
          __syncthreads();
        }
      }
    } else {
      if (tid == 0) atomicAdd(a.rank_def, 1);
      const int r = rank;
      // row order: pivots, then the never-pivoted indices (in index order)
      for (int q = tid; q < k - r; q += BLOCK) piv[r + q] = rem[q];
      __syncthreads();
#define LT(aa, jj) ((aa) < (jj) ? 0.0 : S[lp(piv[(aa)], piv[(jj)])])
      for (int j = tid; j < r; j += BLOCK) {  // y = L~^T r~
        double acc = 0.0;
        for (int aa = j; aa < k; ++aa) acc += LT(aa, j) * rr[piv[aa]];
        y[j] = acc;
      }
      for (int j1 = ty; j1 < r; j1 += BLOCK / TY)  // C = L~^T L~ (packed lower)
        for (int j2 = tx; j2 <= j1; j2 += TY) {
          double acc = 0.0;
          for (int aa = j1; aa < k; ++aa) acc += LT(aa, j1) * LT(aa, j2);
          Cm[tri_base(j1) + j2] = acc;
        }
      __syncthreads();
      for (int j = 0; j < r; ++j) {  // Cholesky of C (positive definite)
        const double cjj = sqrt(Cm[tri_base(j) + j]);
        __syncthreads();
        if (tid == 0) Cm[tri_base(j) + j] = cjj;
        for (int i = j + 1 + tid; i < r; i += BLOCK) Cm[tri_base(i) + j] = Cm[tri_base(i) + j] / cjj;
        __syncthreads();
        for (int i = j + 1 + ty; i < r; i += BLOCK / TY) {
          const double lij = Cm[tri_base(i) + j];
          for (int l = j + 1 + tx; l <= i; l += TY)
            Cm[tri_base(i) + l] = Cm[tri_base(i) + l] - lij * Cm[tri_base(l) + j];
        }
        __syncthreads();
      }
      for (int pass = 0; pass < 2; ++pass) {  // y <- C^-1 y, twice
        for (int j = 0; j < r; ++j) {
          const double yj = y[j] / Cm[tri_base(j) + j];
          __syncthreads();
          for (int i = j + 1 + tid; i < r; i += BLOCK) y[i] = y[i] - Cm[tri_base(i) + j] * yj;
          if (tid == 0) y[j] = yj;
          __syncthreads();
        }
        for (int j = r - 1; j >= 0; --j) {
          const double lj = y[j] / Cm[tri_base(j) + j];
          __syncthreads();
          for (int i = tid; i < j; i += BLOCK) y[i] = y[i] - Cm[tri_base(j) + i] * lj;
          if (tid == 0) y[j] = lj;
          __syncthreads();
        }
      }
      for (int aa = tid; aa < k; aa += BLOCK) {  // lambda~ = L~ u
        double acc = 0.0;
        const int jm = aa < r - 1 ? aa : r - 1;
        for (int j = 0; j <= jm; ++j) acc += LT(aa, j) * y[j];
        lam[piv[aa]] = acc;
      }
#undef LT
    }
    __syncthreads();
    for (int i = tid; i < k; i += BLOCK) a.lambda[a.order[st + i]] = lam[i];
    __syncthreads();
  }
}

template <bool MAT_LDS, bool VEC_LDS>
static void launch_class(const SolveArgs &a, int kmin, int kcap, int grid, hipStream_t s) {
  const size_t bytes = MAT_LDS ? zone_lds_bytes(true, kcap) : (VEC_LDS ? zone_vec_bytes(kcap) : 0) + kWgBytes;
  // the tiled kernel of the global-matrix class with LDS vectors also stages a column of tiles
  const size_t tiled_bytes = bytes + (!MAT_LDS && VEC_LDS ? (size_t)((kcap + TB - 1) / TB) * TB * TB * 8 : 0);
  // the attribute is per function; set once (thread-safe static initialisation)
  static const bool attr_set = [] {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_solve_tiled<MAT_LDS, VEC_LDS>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&k_solve<MAT_LDS, VEC_LDS>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    return true;
  }();
  (void)attr_set;
  k_solve_tiled<MAT_LDS, VEC_LDS><<<grid, kTiledBlock, tiled_bytes, s>>>(a, kmin, kcap);
  k_solve<MAT_LDS, VEC_LDS><<<grid, MAT_LDS ? kSolveBlock : kTiledBlock, bytes, s>>>(a, kmin, kcap);
}

void launch_solve(const SolveArgs &a, hipStream_t s) {
  if (a.nzones <= 0) return;
  const int grid = a.nslots < a.nzones ? a.nslots : a.nzones;
  const int kl = a.maxk < kZoneLds ? a.maxk : kZoneLds;
  launch_class<true, true>(a, 0, kl, grid, s);
  if (a.maxk > kZoneLds && a.maxk <= kZoneVecLds) launch_class<false, true>(a, kZoneLds, a.maxk, grid, s);
  if (a.maxk > kZoneVecLds) launch_class<false, false>(a, kZoneLds, a.maxk, grid, s);
}

size_t solve_slot_doubles(int maxk) {
  const int64_t k = maxk;
  // matrix (tiled or packed), C (packed), then the per-zone arrays
  return (size_t)(zone_mat_doubles(maxk) + k * (k + 1) / 2 + (int64_t)(zone_vec_bytes(maxk) / 8) + 16);
}

// ------------------------------------------------------------------ update
__global__ void k_incidence(const Constraint *__restrict__ con, int64_t S, int bits_s, uint64_t *keys) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 4 * S) return;
  int64_t s = i >> 2;
  int slot = (int)(i & 3);
  int4 v = con[s].v;
  int vert = slot == 0 ? v.x : slot == 1 ? v.y : slot == 2 ? v.z : v.w;
  keys[i] = ((uint64_t)vert << (bits_s + 2)) | (uint64_t)i;
}

void launch_incidence(const Constraint *con, int64_t S, int bits_s, uint64_t *keys, hipStream_t s) {
  if (S > 0) k_incidence<<<grid_for(4 * S, 256), 256, 0, s>>>(con, S, bits_s, keys);
}

struct MeshOut {
  double *x64;
  float *x32;
  int nv;
  const double *w;
};

__global__ void k_update(const uint64_t *__restrict__ keys, int64_t n, int bits_s, const Constraint *__restrict__ con,
                         const double *__restrict__ lambda, MeshOut A, MeshOut B) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int shift = bits_s + 2;
  const uint64_t v = keys[i] >> shift;
  if (i > 0 && (keys[i - 1] >> shift) == v) return;  // not the first incidence of v
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int64_t j = i; j < n && (keys[j] >> shift) == v; ++j) {
    const uint64_t low = keys[j] & ((1ull << shift) - 1);
    const int64_t s = (int64_t)(low >> 2);
    const int slot = (int)(low & 3);
    const double c = slot == 0 ? 1.0 : -1.0 / 3.0;
    const double4 nn = con[s].n;
    const double g = c * lambda[s];
    sx += g * nn.x;
    sy += g * nn.y;
    sz += g * nn.z;
  }
  const bool in_a = (int64_t)v < A.nv;
  MeshOut &M = in_a ? A : B;
  const int lv = in_a ? (int)v : (int)(v - A.nv);
  const double w = M.w ? M.w[lv] : 1.0;
  double x = M.x64[lv] - w * sx;
  double y = M.x64[(int64_t)M.nv + lv] - w * sy;
  double z = M.x64[2 * (int64_t)M.nv + lv] - w * sz;
  if (M.x32) {
    const float fx = (float)x, fy = (float)y, fz = (float)z;
    M.x32[lv] = fx;
    M.x32[(int64_t)M.nv + lv] = fy;
    M.x32[2 * (int64_t)M.nv + lv] = fz;
    x = fx;
    y = fy;
    z = fz;
  }
  M.x64[lv] = x;
  M.x64[(int64_t)M.nv + lv] = y;
  M.x64[2 * (int64_t)M.nv + lv] = z;
}

void launch_update(const uint64_t *keys, int64_t n, int bits_s, const Constraint *con, const double *lambda,
                   MeshDev &A, MeshDev &B, hipStream_t s) {
  if (n <= 0) return;
  MeshOut a{A.x64, A.f32 ? A.x32 : nullptr, A.nv, A.inv_mass};
  MeshOut b{B.x64, B.f32 ? B.x32 : nullptr, B.nv, B.inv_mass};
  k_update<<<grid_for(n, 256), 256, 0, s>>>(keys, n, bits_s, con, lambda, a, b);
}

// Incidence keys, sort and update for at most 256 stencils (1024
// incidences) in one workgroup; the same keys, order and sums as
// k_incidence, the sort and k_update.
__global__ __launch_bounds__(1024) void k_update_small(const Constraint *__restrict__ con, int S, int bits_s,
                                                       const double *__restrict__ lambda, MeshOut A, MeshOut B) {
  __shared__ uint64_t sk[1024];
  __shared__ uint32_t sv[1024];
  // each stencil's lambda and normal, so the per-vertex gathers below read LDS
  __shared__ double sl[256], snx[256], sny[256], snz[256];
  const int t = threadIdx.x;
  const int n = 4 * S;
  const int shift = bits_s + 2;
  uint64_t k = ~0ull;
  uint32_t unused = 0;
  if (t < n) {
    const int4 v = con[t >> 2].v;
    const int slot = t & 3;
    const int vert = slot == 0 ? v.x : slot == 1 ? v.y : slot == 2 ? v.z : v.w;
    k = ((uint64_t)vert << shift) | (uint64_t)t;
  }
  if (t < S) {
    const double4 nn = con[t].n;
    sl[t] = lambda[t];
    snx[t] = nn.x;
    sny[t] = nn.y;
    snz[t] = nn.z;
  }
  int P = 2;
  while (P < n) P <<= 1;
  wg_bitonic_1k(k, unused, P, sk, sv);  // ends with a barrier: the stencil arrays are visible
  sk[t] = k;
  __syncthreads();
  if (t >= n) return;
  const uint64_t vtx = k >> shift;
  if (t > 0 && (sk[t - 1] >> shift) == vtx) return;  // not the first incidence of this vertex
  double sx = 0.0, sy = 0.0, sz = 0.0;
  for (int j = t; j < n && (sk[j] >> shift) == vtx; ++j) {
    const uint64_t low = sk[j] & ((1ull << shift) - 1);
    const int64_t s = (int64_t)(low >> 2);
    const int slot = (int)(low & 3);
    const double c = slot == 0 ? 1.0 : -1.0 / 3.0;
    const double g = c * sl[s];
    sx += g * snx[s];
    sy += g * sny[s];
    sz += g * snz[s];
  }
  const bool in_a = (int64_t)vtx < A.nv;
  MeshOut &M = in_a ? A : B;
  const int lv = in_a ? (int)vtx : (int)(vtx - A.nv);
  const double w = M.w ? M.w[lv] : 1.0;
  double x = M.x64[lv] - w * sx;
  double y = M.x64[(int64_t)M.nv + lv] - w * sy;
  double z = M.x64[2 * (int64_t)M.nv + lv] - w * sz;
  if (M.x32) {
    const float fx = (float)x, fy = (float)y, fz = (float)z;
    M.x32[lv] = fx;
    M.x32[(int64_t)M.nv + lv] = fy;
    M.x32[2 * (int64_t)M.nv + lv] = fz;
    x = fx;
    y = fy;
    z = fz;
  }
  M.x64[lv] = x;
  M.x64[(int64_t)M.nv + lv] = y;
  M.x64[2 * (int64_t)M.nv + lv] = z;
}

bool launch_update_small(const Constraint *con, int64_t S, int bits_s, const double *lambda, MeshDev &A,
                         MeshDev &B, hipStream_t s) {
  if (S <= 0 || 4 * S > 1024) return false;  // S <= 256: the kernel's stencil arrays
  MeshOut a{A.x64, A.f32 ? A.x32 : nullptr, A.nv, A.inv_mass};
  MeshOut b{B.x64, B.f32 ? B.x32 : nullptr, B.nv, B.inv_mass};
  k_update_small<<<1, 1024, 0, s>>>(con, (int)S, bits_s, lambda, a, b);
  return true;
}

// ---------------------------------------------------------------- output
template <typename T>
__global__ void k_write_positions(const double *__restrict__ x64, int nv, T *out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nv) return;
  for (int c = 0; c < 3; ++c) out[3 * (int64_t)i + c] = (T)x64[(int64_t)c * nv + i];
}

void launch_write_positions(const MeshDev &m, void *out, hipStream_t s) {
  if (m.nv <= 0 || !out) return;
  if (m.f32)
    k_write_positions<float><<<grid_for(m.nv, 256), 256, 0, s>>>(m.x64, m.nv, (float *)out);
  else
    k_write_positions<double><<<grid_for(m.nv, 256), 256, 0, s>>>(m.x64, m.nv, (double *)out);
}

}  // namespace hfcr
