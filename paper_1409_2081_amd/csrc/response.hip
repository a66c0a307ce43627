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
// remaining pivot falls below tau * max(diag A) (tau = 1e-12).  Full rank:
// two triangular solves.  Rank r < k: with the k-by-r factor L,
// lambda = L (L^T L)^-1 (L^T L)^-1 L^T r, the minimum-norm least-squares
// solution, for which x' below does not depend on the choice of lambda.
//
// Update (Eq. 5): x'_v = x_v - w_v sum_i c_iv n_i lambda_i, gathered per
// vertex over its (stencil, slot) incidences in stencil order, so the sum
// order is fixed.  Float32 storage is rounded to nearest afterwards.
#include "common.hpp"
#include "kernels.hpp"

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

__global__ void k_constraints(const uint64_t *__restrict__ keys, int64_t S, StencilLayout sl, MeshView A,
                              MeshView B, double d, Constraint *con) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  uint64_t k = keys[i];
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
  con[i] = out;
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

__global__ void k_uf_init(int *parent, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) parent[i] = i;
}

__global__ void k_uf_union(const Constraint *__restrict__ con, int64_t S, int *parent) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= S) return;
  int4 v = con[i].v;
  uf_unite(parent, v.x, v.y);
  uf_unite(parent, v.x, v.z);
  uf_unite(parent, v.x, v.w);
}

void launch_uf_init(int *parent, int n, hipStream_t s) {
  if (n > 0) k_uf_init<<<grid_for(n, 256), 256, 0, s>>>(parent, n);
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

// -------------------------------------------------------------- zone solve
// Storage: the lower triangle of the zone matrix, S[i*k + l] for i >= l
// (index order).  Pivot step j chooses p = argmax of the remaining diagonal
// (ties: smaller index), stores L(i, j) = A_ip / sqrt(A_pp) where A_ip was
// kept (S[max(i,p)*k + min(i,p)]) and updates the remaining lower triangle.
// The remaining indices are kept in increasing order by a stable compaction,
// so "lower" keeps its meaning in index order at every step.
constexpr int kSmallZone = 64;     // zones up to this size: one wave, matrix in LDS
constexpr int kLdsCon = 512;       // zones up to this size keep constraints in LDS
constexpr int kBigBlock = 256;
constexpr int kMaxZoneLds = 4096;  // == HFCR_MAX_ZONE

__device__ inline double inv_mass(int v, const double *wa, const double *wb, int nva) {
  if (v < nva) return wa ? wa[v] : 1.0;
  return wb ? wb[v - nva] : 1.0;
}

__device__ inline double coef(int slot) { return slot == 0 ? 1.0 : -1.0 / 3.0; }

__device__ inline int64_t lidx(int i, int l, int k) {
  return i >= l ? (int64_t)i * k + l : (int64_t)l * k + i;
}

// (value, position) pair reduction over a wavefront; ties -> smaller key
__device__ inline void wave_argmax(double &v, int &pos, int &key) {
  for (int off = 32; off > 0; off >>= 1) {
    double v2 = __shfl_xor(v, off);
    int p2 = __shfl_xor(pos, off);
    int k2 = __shfl_xor(key, off);
    if (v2 > v || (v2 == v && k2 >= 0 && (key < 0 || k2 < key))) {
      v = v2;
      pos = p2;
      key = k2;
    }
  }
}

template <int BLOCK>
struct SolveShared {
  static constexpr int kCon = BLOCK == 64 ? kSmallZone : kLdsCon;
  Constraint con[kCon];
  double wv[BLOCK / 64];
  int wp[BLOCK / 64], wk[BLOCK / 64];
  int rem[2][BLOCK == 64 ? kSmallZone : kMaxZoneLds];
  double lcol[BLOCK == 64 ? kSmallZone : kMaxZoneLds];
  double s_y;
  double mat[BLOCK == 64 ? kSmallZone * kSmallZone : 1];
};

// Zones with kmin < k <= kmax; the matrix lives in LDS when BLOCK == 64.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_solve(SolveArgs a, int kmin, int kmax) {
  __shared__ SolveShared<BLOCK> sh;
  constexpr bool kLds = BLOCK == 64;
  constexpr int TY = BLOCK == 64 ? 8 : 16;  // 2-D thread tiling for the trailing update
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int tx = tid % TY, ty = tid / TY;
  for (int z = blockIdx.x; z < a.nzones; z += gridDim.x) {
    const int st = (int)a.starts[z];
    const int k = (int)a.starts[z + 1] - st;
    if (k <= kmin || k > kmax) continue;
    double *slot = a.scratch + (int64_t)blockIdx.x * a.slot_stride;
    double *S = kLds ? sh.mat : slot;
    double *Cm = slot + (int64_t)k * k;
    double *vec = slot + 2 * (int64_t)k * k;  // rhs, y, lam: 3k doubles
    double *rhs = vec, *y = vec + k, *lam = vec + 2 * k;
    int *piv = reinterpret_cast<int *>(vec + 3 * k);  // k
    int *step_of = piv + k;                           // k
    const bool con_lds = k <= SolveShared<BLOCK>::kCon;
    for (int i = tid; i < k && con_lds; i += BLOCK) sh.con[i] = a.con[a.order[st + i]];
    __syncthreads();
#define CON(i) (con_lds ? sh.con[(i)] : a.con[a.order[st + (i)]])
    // assemble the lower triangle of A
    for (int i = ty; i < k; i += BLOCK / TY) {
      const Constraint ci = CON(i);
      const int vi[4] = {ci.v.x, ci.v.y, ci.v.z, ci.v.w};
      double wi[4];
      for (int s = 0; s < 4; ++s) wi[s] = inv_mass(vi[s], a.w_a, a.w_b, a.nv_a) * coef(s);
      for (int l = tx; l <= i; l += TY) {
        const Constraint cl = CON(l);
        const int vl[4] = {cl.v.x, cl.v.y, cl.v.z, cl.v.w};
        double acc = 0.0;
        for (int s = 0; s < 4; ++s)
          for (int t = 0; t < 4; ++t)
            if (vi[s] == vl[t]) acc += wi[s] * coef(t);
        S[(int64_t)i * k + l] = acc * (ci.n.x * cl.n.x + ci.n.y * cl.n.y + ci.n.z * cl.n.z);
      }
    }
    for (int i = tid; i < k; i += BLOCK) {
      rhs[i] = CON(i).n.w;
      step_of[i] = k;
      sh.rem[0][i] = i;
    }
    __syncthreads();
    // largest diagonal entry (the pivot threshold is relative to it)
    double dmax = 0.0;
    {
      double v = -1.0;
      int pos = -1, key = -1;
      for (int i = tid; i < k; i += BLOCK) {
        const double d = S[(int64_t)i * k + i];
        if (d > v) { v = d; pos = i; key = i; }
      }
      wave_argmax(v, pos, key);
      if (lane == 0) sh.wv[wave] = v;
      __syncthreads();
      for (int w = 0; w < BLOCK / 64; ++w) dmax = fmax(dmax, sh.wv[w]);
      __syncthreads();
    }
    const double thresh = a.tau * dmax;
    int rank = k, cur = 0;
    for (int j = 0; j < k; ++j) {
      const int nrem = k - j;
      const int *rem = sh.rem[cur];
      int *rem2 = sh.rem[cur ^ 1];
      // A: argmax of the remaining diagonal
      double v = -1.0;
      int pos = -1, key = -1;
      for (int q = tid; q < nrem; q += BLOCK) {
        const int i = rem[q];
        const double d = S[(int64_t)i * k + i];
        if (d > v || (d == v && i < key)) { v = d; pos = q; key = i; }
      }
      wave_argmax(v, pos, key);
      if (lane == 0) {
        sh.wv[wave] = v;
        sh.wp[wave] = pos;
        sh.wk[wave] = key;
      }
      __syncthreads();
      double best = sh.wv[0];
      int q0 = sh.wp[0], p = sh.wk[0];
      for (int w = 1; w < BLOCK / 64; ++w) {
        const double v2 = sh.wv[w];
        const int k2 = sh.wk[w];
        if (v2 > best || (v2 == best && k2 >= 0 && (p < 0 || k2 < p))) {
          best = v2;
          q0 = sh.wp[w];
          p = k2;
        }
      }
      if (!(best > thresh)) {
        rank = j;
        break;
      }
      const double lpp = sqrt(best);
      // B: column p of L, and the stable compaction of the remaining list
      for (int q = tid; q < nrem; q += BLOCK) {
        if (q == q0) continue;
        const int i = rem[q];
        const int64_t at = lidx(i, p, k);
        const double l = S[at] / lpp;
        S[at] = l;
        const int qn = q < q0 ? q : q - 1;
        rem2[qn] = i;
        sh.lcol[qn] = l;
      }
      if (tid == 0) {
        S[(int64_t)p * k + p] = lpp;
        piv[j] = p;
        step_of[p] = j;
      }
      __syncthreads();
      // C: trailing update of the remaining lower triangle
      const int nr = nrem - 1;
      for (int r = ty; r < nr; r += BLOCK / TY) {
        const int i = rem2[r];
        const double li = sh.lcol[r];
        double *row = S + (int64_t)i * k;
        for (int c = tx; c <= r; c += TY) row[rem2[c]] = row[rem2[c]] - li * sh.lcol[c];
      }
      cur ^= 1;
      __syncthreads();
    }
    if (rank == k) {
      // forward: L~ y = r~ (rows in pivot order)
      for (int j = 0; j < k; ++j) {
        const int pj = piv[j];
        const double yj = rhs[pj] / S[(int64_t)pj * k + pj];
        for (int i = tid; i < k; i += BLOCK)
          if (step_of[i] > j) rhs[i] = rhs[i] - S[lidx(i, pj, k)] * yj;
        if (tid == 0) y[j] = yj;
        __syncthreads();
      }
      // backward: L~^T lambda~ = y
      for (int j = k - 1; j >= 0; --j) {
        const int pj = piv[j];
        const double lj = y[j] / S[(int64_t)pj * k + pj];
        for (int jj = tid; jj < j; jj += BLOCK) y[jj] = y[jj] - S[lidx(pj, piv[jj], k)] * lj;
        if (tid == 0) lam[pj] = lj;
        __syncthreads();
      }
    } else {
      if (tid == 0) atomicAdd(a.rank_def, 1);
      const int r = rank;
      // row order: pivots, then the never-pivoted indices (in index order)
      const int *rem = sh.rem[cur];
      for (int q = tid; q < k - r; q += BLOCK) piv[r + q] = rem[q];
      __syncthreads();
#define LT(aa, jj) ((aa) < (jj) ? 0.0 : S[lidx(piv[(aa)], piv[(jj)], k)])
      for (int j = tid; j < r; j += BLOCK) {  // y = L~^T r~
        double acc = 0.0;
        for (int aa = j; aa < k; ++aa) acc += LT(aa, j) * rhs[piv[aa]];
        y[j] = acc;
      }
      for (int64_t idx = tid; idx < (int64_t)r * r; idx += BLOCK) {  // C = L~^T L~ (lower)
        const int j1 = (int)(idx / r), j2 = (int)(idx % r);
        if (j2 > j1) continue;
        double acc = 0.0;
        for (int aa = j1; aa < k; ++aa) acc += LT(aa, j1) * LT(aa, j2);
        Cm[(int64_t)j1 * r + j2] = acc;
      }
      __syncthreads();
      for (int j = 0; j < r; ++j) {  // Cholesky of C (positive definite), lower
        const double cjj = sqrt(Cm[(int64_t)j * r + j]);
        __syncthreads();
        if (tid == 0) Cm[(int64_t)j * r + j] = cjj;
        for (int i = j + 1 + tid; i < r; i += BLOCK) Cm[(int64_t)i * r + j] = Cm[(int64_t)i * r + j] / cjj;
        __syncthreads();
        for (int i = j + 1 + ty; i < r; i += BLOCK / TY) {
          const double lij = Cm[(int64_t)i * r + j];
          for (int l = j + 1 + tx; l <= i; l += TY)
            Cm[(int64_t)i * r + l] = Cm[(int64_t)i * r + l] - lij * Cm[(int64_t)l * r + j];
        }
        __syncthreads();
      }
      for (int pass = 0; pass < 2; ++pass) {  // y <- C^-1 y, twice
        for (int j = 0; j < r; ++j) {
          const double yj = y[j] / Cm[(int64_t)j * r + j];
          __syncthreads();
          for (int i = j + 1 + tid; i < r; i += BLOCK) y[i] = y[i] - Cm[(int64_t)i * r + j] * yj;
          if (tid == 0) y[j] = yj;
          __syncthreads();
        }
        for (int j = r - 1; j >= 0; --j) {
          const double lj = y[j] / Cm[(int64_t)j * r + j];
          __syncthreads();
          for (int i = tid; i < j; i += BLOCK) y[i] = y[i] - Cm[(int64_t)j * r + i] * lj;
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
#undef CON
  }
}

void launch_solve(const SolveArgs &a, hipStream_t s) {
  if (a.nzones <= 0) return;
  const int grid = a.nslots < a.nzones ? a.nslots : a.nzones;
  k_solve<64><<<grid, 64, 0, s>>>(a, 0, kSmallZone);
  if (a.maxk > kSmallZone) k_solve<kBigBlock><<<grid, kBigBlock, 0, s>>>(a, kSmallZone, kMaxZoneLds);
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
