// Orientation and E-F intersection predicates evaluated in three tiers.
//
// orient(a,b,c,p) = det[b-a, c-a, p-a]; positive when p lies in front of the
// counter-clockwise triangle (a,b,c) (on the side of (b-a) x (c-a)).
//
// Edge {p,q} hits triangle (a,b,c) iff p and q are strictly on opposite
// sides of the plane (a touching endpoint or a coplanar edge is no hit) and
// orient(p,q,a,b), orient(p,q,b,c), orient(p,q,c,a) are all >= 0 or all
// <= 0 (the line through p and q meets the closed triangle).  A zero-area
// triangle never hits.  The endpoint behind the face is the stencil vertex.
//
// Tiers.  Each filter evaluates the determinant in one precision, with the
// differences taken from a, and returns its sign only when |det| exceeds a
// bound on the rounding error, else "unsure":
//   every monomial of the determinant passes at most eight roundings (three
//   differences, a product, a subtraction, a product, two sums), so the error
//   is below gamma_8 * P, where P is the permanent; the permanent computed in
//   the same precision is at least (1 - 8u) P, hence the bound 9 u P_computed
//   with u the unit roundoff (2^-24 in float32, 2^-53 in float64).
// The float32 filter further requires P >= 2^-60 and every coordinate of the
// scene within 2^32 in magnitude, which keeps any underflowed product's error
// far below the bound; otherwise it is unsure.  The float64 filter needs no
// such guard in the library's coordinate domain (0 or [2^-200, 2^200]).
// The exact tier forms every difference as an exact two-term expansion
// (Two-Diff), every monomial exactly from fused multiply-adds (a product and
// its rounding error), and sums all parts into a nonoverlapping expansion
// with zero elimination (expansion arithmetic after Shewchuk 1997, "Adaptive
// precision floating-point arithmetic and fast robust geometric predicates");
// the sign of that expansion is the sign of its largest component.
//
// This file must be compiled without floating-point contraction.
#pragma once

#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace hfcr {

constexpr int kUnsure = 2;     // a filtered sign that could not be certified
constexpr int kHitUnsure = 3;  // an E-F decision that needs the exact tier

__device__ inline int filtered_sign_f32(float ax, float ay, float az, float bx, float by, float bz, float cx,
                                        float cy, float cz, float px, float py, float pz) {
  float ux = bx - ax, uy = by - ay, uz = bz - az;
  float vx = cx - ax, vy = cy - ay, vz = cz - az;
  float wx = px - ax, wy = py - ay, wz = pz - az;
  float m1 = uy * vz, m2 = uz * vy;
  float m3 = uz * vx, m4 = ux * vz;
  float m5 = ux * vy, m6 = uy * vx;
  float det = wx * (m1 - m2) + wy * (m3 - m4) + wz * (m5 - m6);
  float perm = fabsf(wx) * (fabsf(m1) + fabsf(m2)) + fabsf(wy) * (fabsf(m3) + fabsf(m4)) +
               fabsf(wz) * (fabsf(m5) + fabsf(m6));
  if (!(perm >= 0x1p-60f) || !(perm < INFINITY)) return kUnsure;
  float bound = (9.0f * 0x1p-24f) * perm;
  if (det > bound) return 1;
  if (-det > bound) return -1;
  return kUnsure;
}

__device__ inline int filtered_sign_f64(double ax, double ay, double az, double bx, double by, double bz,
                                        double cx, double cy, double cz, double px, double py, double pz) {
  double ux = bx - ax, uy = by - ay, uz = bz - az;
  double vx = cx - ax, vy = cy - ay, vz = cz - az;
  double wx = px - ax, wy = py - ay, wz = pz - az;
  double m1 = uy * vz, m2 = uz * vy;
  double m3 = uz * vx, m4 = ux * vz;
  double m5 = ux * vy, m6 = uy * vx;
  double det = wx * (m1 - m2) + wy * (m3 - m4) + wz * (m5 - m6);
  double perm = fabs(wx) * (fabs(m1) + fabs(m2)) + fabs(wy) * (fabs(m3) + fabs(m4)) +
                fabs(wz) * (fabs(m5) + fabs(m6));
  if (perm == 0.0) return 0;  // every exact monomial is zero (no underflow in the domain)
  double bound = (9.0 * 0x1p-53) * perm;
  if (det > bound) return 1;
  if (-det > bound) return -1;
  return kUnsure;
}

// ---------------------------------------------------------------- exact tier
__device__ inline void xs_two_sum(double a, double b, double &s, double &e) {
  s = a + b;
  double bv = s - a;
  double av = s - bv;
  e = (a - av) + (b - bv);
}

__device__ inline void xs_two_diff(double a, double b, double &d, double &e) {
  d = a - b;
  double bv = a - d;
  double av = d + bv;
  e = (a - av) + (bv - b);
}

__device__ inline void xs_two_prod(double a, double b, double &p, double &e) {
  p = a * b;
  e = __builtin_fma(a, b, -p);
}

// Insert b into the nonoverlapping, increasing expansion h[0..n); returns n'.
__device__ inline int xs_grow(double *h, int n, double b) {
  double q = b;
  int m = 0;
  for (int i = 0; i < n; ++i) {
    double s, t;
    xs_two_sum(q, h[i], s, t);
    if (t != 0.0) h[m++] = t;
    q = s;
  }
  if (q != 0.0 || m == 0) h[m++] = q;
  return m;
}

constexpr int kExpMax = 200;

__device__ inline int exact_sign(double ax, double ay, double az, double bx, double by, double bz, double cx,
                                 double cy, double cz, double px, double py, double pz) {
  double u[3][2], v[3][2], w[3][2];
  xs_two_diff(bx, ax, u[0][0], u[0][1]);
  xs_two_diff(by, ay, u[1][0], u[1][1]);
  xs_two_diff(bz, az, u[2][0], u[2][1]);
  xs_two_diff(cx, ax, v[0][0], v[0][1]);
  xs_two_diff(cy, ay, v[1][0], v[1][1]);
  xs_two_diff(cz, az, v[2][0], v[2][1]);
  xs_two_diff(px, ax, w[0][0], w[0][1]);
  xs_two_diff(py, ay, w[1][0], w[1][1]);
  xs_two_diff(pz, az, w[2][0], w[2][1]);
  // det = sum over permutations (i,j,k) of sgn * u_i v_j w_k
  const int perm[6][3] = {{0, 1, 2}, {1, 2, 0}, {2, 0, 1}, {0, 2, 1}, {1, 0, 2}, {2, 1, 0}};
  double h[kExpMax];
  int n = 0;
  for (int t = 0; t < 6; ++t) {
    const double sg = t < 3 ? 1.0 : -1.0;
    const int i = perm[t][0], j = perm[t][1], k = perm[t][2];
    for (int a = 0; a < 2; ++a) {
      double x = u[i][a];
      if (x == 0.0) continue;
      for (int b = 0; b < 2; ++b) {
        double y = v[j][b];
        if (y == 0.0) continue;
        double p, e;
        xs_two_prod(sg * x, y, p, e);
        for (int c = 0; c < 2; ++c) {
          double z = w[k][c];
          if (z == 0.0) continue;
          double p1, e1, p2, e2;
          xs_two_prod(p, z, p1, e1);
          xs_two_prod(e, z, p2, e2);
          const double parts[4] = {e2, p2, e1, p1};
          for (int r = 0; r < 4; ++r)
            if (parts[r] != 0.0) n = xs_grow(h, n, parts[r]);
        }
      }
    }
  }
  if (n == 0) return 0;
  double top = h[n - 1];
  return (top > 0.0) - (top < 0.0);
}

// --------------------------------------------------------------- decisions
// Combine five (possibly unsure) signs into a hit decision:
// 0 no hit, 1 hit with p behind, 2 hit with q behind, kHitUnsure otherwise.
__device__ inline int ef_decide_side(int sp, int sq) {
  // returns 0: certainly no opposite strict signs, 1: certainly opposite, kUnsure
  if (sp != kUnsure && sq != kUnsure) return (sp * sq < 0) ? 1 : 0;
  if (sp == 0 || sq == 0) return 0;
  return kUnsure;
}

__device__ inline int ef_decide_line(int t1, int t2, int t3) {
  // 1: consistent (all >= 0 or all <= 0), 0: certainly inconsistent, kUnsure
  bool pos = (t1 == 1) || (t2 == 1) || (t3 == 1);
  bool neg = (t1 == -1) || (t2 == -1) || (t3 == -1);
  if (pos && neg) return 0;
  if (t1 == kUnsure || t2 == kUnsure || t3 == kUnsure) return kUnsure;
  return 1;
}

struct P3f { float x, y, z; };
struct P3d { double x, y, z; };

__device__ inline int ef_test_f32(P3f p, P3f q, P3f a, P3f b, P3f c) {
  int sp = filtered_sign_f32(a.x, a.y, a.z, b.x, b.y, b.z, c.x, c.y, c.z, p.x, p.y, p.z);
  int sq = filtered_sign_f32(a.x, a.y, a.z, b.x, b.y, b.z, c.x, c.y, c.z, q.x, q.y, q.z);
  int side = ef_decide_side(sp, sq);
  if (side == 0) return 0;
  int t1 = filtered_sign_f32(p.x, p.y, p.z, q.x, q.y, q.z, a.x, a.y, a.z, b.x, b.y, b.z);
  int t2 = filtered_sign_f32(p.x, p.y, p.z, q.x, q.y, q.z, b.x, b.y, b.z, c.x, c.y, c.z);
  int t3 = filtered_sign_f32(p.x, p.y, p.z, q.x, q.y, q.z, c.x, c.y, c.z, a.x, a.y, a.z);
  int line = ef_decide_line(t1, t2, t3);
  if (line == 0) return 0;
  if (side == kUnsure || line == kUnsure) return kHitUnsure;
  return sp < 0 ? 1 : 2;
}

template <bool EXACT>
__device__ inline int sign_f64(P3d a, P3d b, P3d c, P3d p) {
  int s = filtered_sign_f64(a.x, a.y, a.z, b.x, b.y, b.z, c.x, c.y, c.z, p.x, p.y, p.z);
  if (EXACT && s == kUnsure) s = exact_sign(a.x, a.y, a.z, b.x, b.y, b.z, c.x, c.y, c.z, p.x, p.y, p.z);
  return s;
}

// Float64 filter alone (EXACT = false) may return kHitUnsure; with EXACT = true
// every unsure sign is recomputed exactly and the result is final.
template <bool EXACT>
__device__ inline int ef_test_f64(P3d p, P3d q, P3d a, P3d b, P3d c, int *n_exact = nullptr) {
  int sp = sign_f64<false>(a, b, c, p);
  int sq = sign_f64<false>(a, b, c, q);
  if (EXACT) {
    if (sp == kUnsure) { sp = exact_sign(a.x, a.y, a.z, b.x, b.y, b.z, c.x, c.y, c.z, p.x, p.y, p.z); if (n_exact) ++*n_exact; }
    if (sq == kUnsure) { sq = exact_sign(a.x, a.y, a.z, b.x, b.y, b.z, c.x, c.y, c.z, q.x, q.y, q.z); if (n_exact) ++*n_exact; }
  }
  int side = ef_decide_side(sp, sq);
  if (side == 0) return 0;
  int t1 = sign_f64<false>(p, q, a, b);
  int t2 = sign_f64<false>(p, q, b, c);
  int t3 = sign_f64<false>(p, q, c, a);
  if (EXACT) {
    if (t1 == kUnsure) { t1 = exact_sign(p.x, p.y, p.z, q.x, q.y, q.z, a.x, a.y, a.z, b.x, b.y, b.z); if (n_exact) ++*n_exact; }
    if (t2 == kUnsure) { t2 = exact_sign(p.x, p.y, p.z, q.x, q.y, q.z, b.x, b.y, b.z, c.x, c.y, c.z); if (n_exact) ++*n_exact; }
    if (t3 == kUnsure) { t3 = exact_sign(p.x, p.y, p.z, q.x, q.y, q.z, c.x, c.y, c.z, a.x, a.y, a.z); if (n_exact) ++*n_exact; }
  }
  int line = ef_decide_line(t1, t2, t3);
  if (line == 0) return 0;
  if (side == kUnsure || line == kUnsure) return kHitUnsure;
  return sp < 0 ? 1 : 2;
}

}  // namespace hfcr
