// Host-side launchers of every kernel (one translation unit each family).
#pragma once

#include "common.hpp"

namespace hfcr {

// bvh.hip
void launch_ingest(const MeshDev &m, unsigned *err, unsigned *maxabs, hipStream_t s);
// *diff |= 1 when the index arrays a[0..n) and b[0..n) differ.
void launch_tri_diff(const int32_t *a, const int32_t *b, int64_t n, unsigned *diff, hipStream_t s);
void launch_edge_keys(const MeshDev &m, uint64_t *keys, hipStream_t s);
void launch_unique_flags(const uint64_t *keys, int64_t n, uint64_t invalid_from, uint32_t *flags,
                         hipStream_t s);
void launch_compact_edges(const uint64_t *keys, const uint32_t *flags, const uint32_t *pos, int64_t n,
                          int2 *edges, hipStream_t s);
void launch_bounds(const MeshDev &m, float *box, hipStream_t s);
void launch_edge_morton(const MeshDev &m, const float *box, uint64_t *keys, hipStream_t s);
void launch_make_qedges(const MeshDev &m, const uint64_t *keys, hipStream_t s);
void launch_face_morton(const MeshDev &m, const float *box, uint64_t *keys, hipStream_t s);
void launch_leaf_tri(const MeshDev &m, const uint64_t *keys, uint32_t *codes, hipStream_t s);
void launch_build_tree(const MeshDev &m, const uint32_t *codes, hipStream_t s);
void launch_refit(const MeshDev &m, hipStream_t s);

// dcd.hip
struct HitLayout {
  int bits_f;  // face index bits
  int bits_e;  // edge index bits
};
struct DcdOut {
  uint64_t *keys;        // hit keys (dir, e, f)
  uint32_t *vals;        // x0 (local vertex id in the edge mesh)
  uint32_t *count;       // device counter
  int64_t cap;
  uint2 *amb;            // (query index, leaf index) needing the exact tier
  uint32_t *amb_count;   // device counter
  int64_t amb_cap;
  unsigned long long *cand;     // narrow-phase tests
  unsigned long long *f32_unsure;
  unsigned long long *exact;    // exact-tier tests
  unsigned long long *visits;   // BVH nodes fetched
  unsigned *max_path;           // most traversal steps of any wavefront
  int *overflow;         // traversal stack overflow flag
  int warm;              // warm the L2 before traversing
  uint2 *cand_buf;       // (query index, leaf index) pairs found by the traversal
  uint32_t *cand_count;  // device counter
  int64_t cand_cap;
};
void launch_traverse(const MeshDev &edge_mesh, const MeshDev &face_mesh, int dir, bool tier0, HitLayout lay,
                     const DcdOut &out, int block, hipStream_t s);
// Narrow phase of the candidate pairs the traversal queued (float32 filter,
// then float64 filter; undecided pairs go to the exact tier).
void launch_narrow(const MeshDev &edge_mesh, const MeshDev &face_mesh, int dir, bool tier0, HitLayout lay,
                   const DcdOut &out, hipStream_t s);
void launch_exact(const MeshDev &edge_mesh, const MeshDev &face_mesh, int dir, HitLayout lay, const DcdOut &out,
                  hipStream_t s);
void launch_write_hits(const uint64_t *keys, const uint32_t *vals, int64_t n, HitLayout lay, const int2 *edges_a,
                       const int2 *edges_b, int32_t *out, hipStream_t s);
void launch_test_orient(const double *pts, int64_t n, int tier, int32_t *out, hipStream_t s);

// response.hip
struct StencilLayout {
  int bits_f;  // face index bits
  int bits_v;  // local vertex bits
};
void launch_stencil_keys(const uint64_t *hit_keys, const uint32_t *hit_vals, int64_t n, HitLayout hl,
                         StencilLayout sl, uint64_t *out, hipStream_t s);
void launch_compact_keys(const uint64_t *keys, const uint32_t *flags, const uint32_t *pos, int64_t n,
                         uint64_t *out, hipStream_t s);
void launch_write_stencils(const uint64_t *keys, int64_t n, StencilLayout sl, int32_t *out, hipStream_t s);

struct Constraint {
  double4 n;   // unit normal (x, y, z) and r = D - d in w
  int4 v;      // global vertex ids x0, x1, x2, x3
};
void launch_constraints(const uint64_t *st_keys, int64_t S, StencilLayout sl, const MeshDev &A, const MeshDev &B,
                        double d, Constraint *con, hipStream_t s);
// Also sets *clear to 0 (may be null).
// parent[i] = i; also zeroes clear[0] and clear[1] (when clear is not null)
// p[0..n) = 0 (n 32-bit words), one launch.
void launch_zero_words(uint32_t *p, int n, hipStream_t s);
void launch_uf_init(int *parent, int n, uint32_t *clear, hipStream_t s);
void launch_uf_union(const Constraint *con, int64_t S, int *parent, hipStream_t s);
// Stencil keys of up to two hit lists, sorted and made unique, written to
// out (room for n0 + n1 keys) with their count in *total, in one launch when
// n0 + n1 <= 1024; returns false (and launches nothing) otherwise.
bool launch_stencils_small(const uint64_t *hk0, const uint32_t *hv0, int64_t n0, const uint64_t *hk1,
                           const uint32_t *hv1, int64_t n1, HitLayout hl, StencilLayout sl, uint64_t *out,
                           uint32_t *total, hipStream_t s);
void launch_zone_keys(const Constraint *con, int64_t S, const int *parent, int bits_s, uint64_t *keys,
                      uint32_t *vals, hipStream_t s);
void launch_zone_flags(const uint64_t *keys, int64_t S, int bits_s, uint32_t *flags, hipStream_t s);
void launch_zone_starts(const uint32_t *flags, const uint32_t *pos, int64_t S, uint32_t *starts,
                        uint32_t *nzones_out, uint32_t *maxk_out, hipStream_t s);
// The zone stage (uf_init .. zone_starts) in one launch when S is small
// enough; returns false (and launches nothing) otherwise.
bool launch_zones_small(const Constraint *con, int64_t S, int bits_s, uint64_t *keys, uint32_t *vals,
                        uint32_t *starts, uint32_t *nzones_out, uint32_t *clear, hipStream_t s);

// Stencils, constraints and the zone stage of one round (the three launches
// above) in one launch, for two hit lists whose counts the kernel reads from
// cnt0 and cnt1 (null: no second list).  Lists within their buffers (count <=
// cap) and 1..kRoundSmallHits hits in all: the stencil keys go to st_keys,
// their count to *total; otherwise *total = 0 and nothing else is written.
// st_keys, con, keys, vals need room for kRoundSmallHits entries, starts for
// one more.
constexpr int kRoundSmallHits = 1024;
void launch_round_small(const uint64_t *hk0, const uint32_t *hv0, const uint32_t *cnt0, int64_t cap0,
                        const uint64_t *hk1, const uint32_t *hv1, const uint32_t *cnt1, int64_t cap1, HitLayout hl,
                        StencilLayout sl, const MeshDev &A, const MeshDev &B, double d, uint64_t *st_keys,
                        Constraint *con, uint64_t *keys, uint32_t *vals, uint32_t *starts, uint32_t *nzones_out,
                        uint32_t *clear, uint32_t *total, hipStream_t s);

struct SolveArgs {
  const Constraint *con;
  const uint32_t *order;    // stencil ids grouped by zone
  const uint32_t *starts;   // [nzones + 1]
  int nzones;
  const double *w_a, *w_b;  // inverse masses or null
  int nv_a;
  double *lambda;           // [S]
  double *scratch;          // per-slot solve_slot_doubles(maxk) doubles
  int64_t slot_stride;      // doubles per slot
  int nslots;
  int *rank_def;            // count of rank-deficient zones
  int *pivoted;             // zones that needed the pivoted (rank-revealing) path
  uint32_t *retry;          // [nzones] zones handed from the tiled to the pivoted path
  uint32_t *retry_n;        // their count (zero before the solve)
  double tau;
  int maxk;                 // largest zone
};
void launch_solve(const SolveArgs &a, hipStream_t s);
size_t solve_slot_doubles(int maxk);  // scratch doubles per workgroup slot
void launch_incidence(const Constraint *con, int64_t S, int bits_s, uint64_t *keys, hipStream_t s);
void launch_update(const uint64_t *keys, int64_t n, int bits_s, const Constraint *con, const double *lambda,
                   MeshDev &A, MeshDev &B, hipStream_t s);
// launch_incidence, the sort and launch_update in one launch for S <= 256
// stencils; returns false (and launches nothing) otherwise.
bool launch_update_small(const Constraint *con, int64_t S, int bits_s, const double *lambda, MeshDev &A,
                         MeshDev &B, hipStream_t s);
void launch_write_positions(const MeshDev &m, void *out, hipStream_t s);

}  // namespace hfcr
