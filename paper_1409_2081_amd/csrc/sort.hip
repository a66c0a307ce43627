// Device-wide sort and scan primitives.
//
// * Short inputs (n <= kSmallSort) are sorted by one workgroup with a
//   bitonic network (keys must then be unique for a stable result; every
//   caller builds unique keys): up to 1024 in registers and lane shuffles,
//   otherwise in LDS.
// * Longer inputs use an LSD radix sort with 8-bit digits: a per-tile digit
//   histogram, one scan over all (digit, tile) counts, then a stable scatter
//   in which each key's rank among equal digits of its wavefront comes from
//   eight ballots (one per digit bit) and a popcount, and the wavefronts of
//   a tile are combined through LDS counters.
#include "common.hpp"
#include "wgsort.hpp"

namespace hfcr {

constexpr int kSmallSort = 4096;
constexpr int kRadixBlock = 256;
constexpr int kRadixItems = 8;
constexpr int kRadixTile = kRadixBlock * kRadixItems;  // keys per block
constexpr int kScanInScatter = 64;  // up to this many tiles the scatter scans the counts itself
static_assert(kRadixBlock == 256, "one thread per digit in the scatter's bucket bases");
constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

// ------------------------------------------------------------ bitonic sort
__global__ __launch_bounds__(1024) void k_bitonic(uint64_t *keys, uint32_t *vals, int n, int P) {
  __shared__ uint64_t sk[kSmallSort];
  __shared__ uint32_t sv[kSmallSort];
  const int tid = threadIdx.x;
  for (int i = tid; i < P; i += blockDim.x) {
    sk[i] = i < n ? keys[i] : ~0ull;
    sv[i] = (vals && i < n) ? vals[i] : 0u;
  }
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = tid; t < (P >> 1); t += blockDim.x) {
        int i = (t / stride) * 2 * stride + (t % stride);
        int j = i + stride;
        bool up = (i & size) == 0;
        uint64_t ki = sk[i], kj = sk[j];
        if ((ki > kj) == up) {
          sk[i] = kj;
          sk[j] = ki;
          uint32_t t0 = sv[i];
          sv[i] = sv[j];
          sv[j] = t0;
        }
      }
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += blockDim.x) {
    keys[i] = sk[i];
    if (vals) vals[i] = sv[i];
  }
}

// Up to 1024 pairs: thread t holds element t in registers (wg_bitonic_1k).
__global__ __launch_bounds__(1024) void k_bitonic_1k(uint64_t *keys, uint32_t *vals, int n, int P) {
  __shared__ uint64_t sk[1024];
  __shared__ uint32_t sv[1024];
  const int t = threadIdx.x;
  uint64_t k = t < n ? keys[t] : ~0ull;
  uint32_t v = (vals && t < n) ? vals[t] : 0u;
  wg_bitonic_1k(k, v, P, sk, sv);
  if (t < n) {
    keys[t] = k;
    if (vals) vals[t] = v;
  }
}

// ------------------------------------------------------- workgroup scans
// Exclusive scan of data[0..n) in place by one workgroup of 1024 threads;
// each thread owns a contiguous chunk.  Optionally stores the total.
__device__ void wg_exclusive_scan_1024(uint32_t *data, int64_t n, uint32_t *total) {
  __shared__ uint32_t part[1024];
  const int tid = threadIdx.x;
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t lo = tid * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  uint32_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += data[i];
  part[tid] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over 1024 partial sums
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = tid >= off ? part[tid - off] : 0u;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint32_t run = tid ? part[tid - 1] : 0u;
  for (int64_t i = lo; i < hi; ++i) {
    uint32_t v = data[i];
    data[i] = run;
    run += v;
  }
  if (total && tid == 1023) *total = part[1023];
}

__global__ __launch_bounds__(1024) void k_scan_single(uint32_t *data, int64_t n, uint32_t *total) {
  wg_exclusive_scan_1024(data, n, total);
}

// --------------------------------------------------------------- radix sort
__global__ __launch_bounds__(kRadixBlock) void k_radix_hist(const uint64_t *keys, int64_t n, int shift,
                                                            uint32_t *hist, int nblocks) {
  __shared__ uint32_t h[256];
  const int tid = threadIdx.x;
  h[tid] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
#pragma unroll
  for (int it = 0; it < kRadixItems; ++it) {
    int64_t idx = base + it * kRadixBlock + tid;
    if (idx < n) atomicAdd(&h[(unsigned)(keys[idx] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(int64_t)tid * nblocks + blockIdx.x] = h[tid];
}

// SCAN: hist holds the raw (digit, tile) counts and every workgroup derives
// its 256 bucket bases from them (all tiles' counts of each digit, and those
// of the tiles before its own): the separate scan launch is saved where the
// count table is small.  Otherwise hist holds the exclusive scan already.
template <bool SCAN>
__global__ __launch_bounds__(kRadixBlock) void k_radix_scatter(const uint64_t *kin, const uint32_t *vin,
                                                               uint64_t *kout, uint32_t *vout, int64_t n,
                                                               int shift, const uint32_t *hist,
                                                               int nblocks) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[kRadixBlock / kWave][256];
  const int tid = threadIdx.x;
  const int lane = tid & (kWave - 1);
  const int wave = tid / kWave;
  if (SCAN) {
    // digit tid: its count over all tiles and over the tiles before this one
    uint32_t tot = 0, pre = 0;
    for (int b = 0; b < nblocks; ++b) {
      const uint32_t h = hist[(int64_t)tid * nblocks + b];
      tot += h;
      pre += b < (int)blockIdx.x ? h : 0u;
    }
    // exclusive scan of the totals over the 256 digits (Hillis-Steele in LDS)
    base[tid] = tot;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const uint32_t v = tid >= off ? base[tid - off] : 0u;
      __syncthreads();
      base[tid] += v;
      __syncthreads();
    }
    const uint32_t excl = base[tid] - tot;
    __syncthreads();
    base[tid] = excl + pre;
  } else {
    base[tid] = hist[(int64_t)tid * nblocks + blockIdx.x];
  }
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
  const int64_t tile = (int64_t)blockIdx.x * kRadixTile;
  for (int it = 0; it < kRadixItems; ++it) {
#pragma unroll
    for (int w = 0; w < kRadixBlock / kWave; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const int64_t idx = tile + it * kRadixBlock + tid;
    const bool valid = idx < n;
    const uint64_t key = valid ? kin[idx] : 0ull;
    const uint32_t val = (valid && vin) ? vin[idx] : 0u;
    const unsigned digit = (unsigned)(key >> shift) & 255u;
    uint64_t match = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const bool set = (digit >> bit) & 1u;
      const uint64_t m = __ballot(set);
      match &= set ? m : ~m;
    }
    const unsigned rank = (unsigned)__popcll(match & lt_mask);
    if (valid && rank == 0) wcnt[wave][digit] = (uint32_t)__popcll(match);
    __syncthreads();
    if (valid) {
      uint32_t off = base[digit] + rank;
      for (int w = 0; w < wave; ++w) off += wcnt[w][digit];
      kout[off] = key;
      if (vout) vout[off] = val;
    }
    __syncthreads();
    uint32_t add = 0;
#pragma unroll
    for (int w = 0; w < kRadixBlock / kWave; ++w) add += wcnt[w][tid];
    base[tid] += add;
    __syncthreads();
  }
}

size_t radix_hist_entries(int64_t n) {
  int64_t nb = (n + kRadixTile - 1) / kRadixTile;
  if (nb < 1) nb = 1;
  return (size_t)nb * 256;
}

void sort_pairs(SortBufs &b, int64_t n, int key_bits, hipStream_t s, bool &in_alt) {
  in_alt = false;
  if (n <= 1) return;
  if (n <= kSmallSort) {
    int P = 2;
    while (P < n) P <<= 1;
    if (P <= 1024)
      k_bitonic_1k<<<1, 1024, 0, s>>>(b.k0, b.v0, (int)n, P);
    else
      k_bitonic<<<1, 1024, 0, s>>>(b.k0, b.v0, (int)n, P);
    return;
  }
  const int nblocks = (int)((n + kRadixTile - 1) / kRadixTile);
  uint64_t *kin = b.k0, *kout = b.k1;
  uint32_t *vin = b.v0, *vout = b.v1;
  const int lo_bit = key_bits < 0 ? 32 : 0;  // negative: low 32 bits already ordered
  const int hi_bit = key_bits < 0 ? -key_bits : key_bits;
  for (int shift = lo_bit; shift < hi_bit; shift += 8) {
    k_radix_hist<<<nblocks, kRadixBlock, 0, s>>>(kin, n, shift, b.hist, nblocks);
    if (nblocks <= kScanInScatter) {
      k_radix_scatter<true><<<nblocks, kRadixBlock, 0, s>>>(kin, vin, kout, vout, n, shift, b.hist, nblocks);
    } else {
      k_scan_single<<<1, 1024, 0, s>>>(b.hist, (int64_t)nblocks * 256, nullptr);
      k_radix_scatter<false><<<nblocks, kRadixBlock, 0, s>>>(kin, vin, kout, vout, n, shift, b.hist, nblocks);
    }
    uint64_t *tk = kin; kin = kout; kout = tk;
    uint32_t *tv = vin; vin = vout; vout = tv;
    in_alt = !in_alt;
  }
}

// -------------------------------------------------------------------- scan
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const uint32_t *in, int64_t n, uint32_t *sums) {
  __shared__ uint32_t red[kScanBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  uint32_t s = 0;
  for (int it = 0; it < kScanItems; ++it) {
    int64_t idx = base + it * kScanBlock + threadIdx.x;
    if (idx < n) s += in[idx];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int off = kScanBlock / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// Block-local exclusive scan of a tile (items owned contiguously per thread),
// offset by the tile's prefix.
__global__ __launch_bounds__(kScanBlock) void k_scan_apply(const uint32_t *in, uint32_t *out, int64_t n,
                                                           const uint32_t *sums) {
  __shared__ uint32_t part[kScanBlock];
  const int tid = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)tid * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = (base + i < n) ? in[base + i] : 0u;
    s += v[i];
  }
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < kScanBlock; off <<= 1) {
    uint32_t t = tid >= off ? part[tid - off] : 0u;
    __syncthreads();
    part[tid] += t;
    __syncthreads();
  }
  uint32_t run = (tid ? part[tid - 1] : 0u) + sums[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}

__global__ void k_copy_total(const uint32_t *sums, int nb, const uint32_t *in, const uint32_t *out,
                             int64_t n, uint32_t *total) {
  // total = last exclusive prefix + last input
  if (threadIdx.x == 0 && blockIdx.x == 0) *total = n ? out[n - 1] + in[n - 1] : 0u;
  (void)sums;
  (void)nb;
}

// One-workgroup exclusive scan of in[0..n) into out, total in *total: each
// of the 1024 threads sums a contiguous chunk, the chunk sums are scanned in
// LDS, and each chunk is written with its offset.  Used for short inputs,
// where one launch costs less than three.
constexpr int64_t kScanOneWgMax = 1 << 14;

__global__ __launch_bounds__(1024) void k_scan_one_wg(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                      int64_t n, uint32_t *total) {
  __shared__ uint32_t part[1024];
  const int tid = threadIdx.x;
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t lo = tid * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  uint32_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += in[i];
  part[tid] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = tid >= off ? part[tid - off] : 0u;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  uint32_t run = tid ? part[tid - 1] : 0u;
  for (int64_t i = lo; i < hi; ++i) {
    const uint32_t v = in[i];
    out[i] = run;
    run += v;
  }
  if (total && tid == 1023) *total = part[1023];
}

size_t scan_block_sums_entries(int64_t n) {
  int64_t nb = (n + kScanTile - 1) / kScanTile;
  return (size_t)(nb < 1 ? 1 : nb);
}

void scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *block_sums, uint32_t *total_dev,
              hipStream_t s) {
  if (n <= kScanOneWgMax) {
    k_scan_one_wg<<<1, 1024, 0, s>>>(in, out, n, total_dev);
    return;
  }
  const int nb = (int)scan_block_sums_entries(n);
  k_scan_reduce<<<nb, kScanBlock, 0, s>>>(in, n, block_sums);
  k_scan_single<<<1, 1024, 0, s>>>(block_sums, nb, nullptr);
  k_scan_apply<<<nb, kScanBlock, 0, s>>>(in, out, n, block_sums);
  if (total_dev) k_copy_total<<<1, 1, 0, s>>>(block_sums, nb, in, out, n, total_dev);
}

// Zero n 32-bit words in one launch (a runtime memset of a few dozen bytes can
// take several fill launches when the address is not 16-byte aligned).
__global__ void k_zero_words(uint32_t *p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0u;
}

void launch_zero_words(uint32_t *p, int n, hipStream_t s) {
  if (n > 0) k_zero_words<<<1, 256, 0, s>>>(p, n);
}

}  // namespace hfcr
