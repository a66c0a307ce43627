// Internal declarations shared by the library's translation units.
// Every kernel is launched through a host function declared here; no device
// code crosses translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hfcr {

constexpr int kWave = 64;

// --------------------------------------------------------------- BVH layout
// Internal node of the face BVH: the boxes of both children are stored in
// the parent so that one 64-byte fetch tests both.  Child index c >= 0 is an
// internal node, c < 0 is leaf ~c (a position in Morton order).
struct __align__(16) BvhNode {
  float4 a;  // lo0.x lo0.y lo0.z hi0.x
  float4 b;  // hi0.y hi0.z lo1.x lo1.y
  float4 c;  // lo1.z hi1.x hi1.y hi1.z
  int4 d;    // child0, child1, parent, unused
};

// Per-mesh device state for one call.
struct MeshDev {
  int nv = 0, nt = 0, ne = 0;
  bool f32 = false;          // storage type
  const void *pos_in = nullptr;
  const int32_t *tri_in = nullptr;
  double *x64 = nullptr;     // SoA working positions, 3*nv (x | y | z)
  float *x32 = nullptr;      // SoA float32 positions (float32 storage only)
  int2 *edges = nullptr;     // [ne] canonical edges (u < v), sorted
  int4 *qedges = nullptr;    // [ne] (u, v, canonical id, 0) in Morton order
  int4 *leaf_tri = nullptr;  // [nt] (a, b, c, face id) in Morton order
  BvhNode *nodes = nullptr;  // [max(nt-1,1)]
  int *leaf_parent = nullptr;// [nt] parent node of each leaf (slot in bit 31)
  int *counters = nullptr;   // [nt] refit visit counters (self-clearing)
  float *root_box = nullptr; // [6]
  int2 *range = nullptr;     // [nt] leaf range (lo, hi) of each internal node
  int *top_pos = nullptr;    // [nt] position in top_list, or -1
  int *top_list = nullptr;   // [nt] internal nodes whose range crosses a refit chunk
  int *top_pre = nullptr;    // [nt] per top node: children finished by the chunk pass
  int *top_count = nullptr;  // [1]
  const double *inv_mass = nullptr;
  bool small_coords = true;  // every |coordinate| <= 2^32 (float32 filter valid)
};

// ------------------------------------------------------------------- sorts
// Sort (key, value) pairs by key, keys < 2^key_bits.  Uses a single-workgroup
// bitonic network for short inputs and an LSD radix sort otherwise.  Returns
// the buffers holding the result (either the inputs or the alternates).
struct SortBufs {
  uint64_t *k0, *k1;
  uint32_t *v0, *v1;   // may be null for key-only sorts
  uint32_t *hist;      // radix histogram scratch
  size_t hist_cap;     // entries
};
void sort_pairs(SortBufs &b, int64_t n, int key_bits, hipStream_t s, bool &in_alt);
size_t radix_hist_entries(int64_t n);

// Exclusive scan of n uint32 flags into out (may alias? no), and total.
void scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *block_sums,
              uint32_t *total_dev, hipStream_t s);
size_t scan_block_sums_entries(int64_t n);

// ------------------------------------------------------------------ launch
inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace hfcr
