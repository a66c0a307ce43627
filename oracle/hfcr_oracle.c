/*
 * CPU oracle, exact part: orientation predicate and brute-force edge-face
 * discrete collision detection.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker the HIP path is
 * compared against; it shares no code, header or table with the library
 * under paper_1409_2081_amd/, and the library never calls it.  Only tests,
 * the smoke check and the CPU-baseline leg of the benchmark load it.
 *
 * What is computed (paper, Section 3 and Section 4 "Penetration
 * Constraints"):
 *   The DCD step finds every edge-face (E-F) intersection between the edges
 *   of one mesh and the triangles of the other.  An F-F penetration always
 *   decomposes into E-F penetrations, so testing edges against faces finds
 *   all of them.  The vertex of an intersecting edge that lies on the back
 *   side of the oriented face is the illegal vertex x0 of a penetration
 *   stencil.
 *
 * Readings (the paper gives no formulas for the intersection test):
 *   orient(a,b,c,p) = det[b-a, c-a, p-a], evaluated EXACTLY.  A positive value
 *   means p lies on the front side, the side the right-hand normal
 *   (b-a) x (c-a) of the counter-clockwise triangle (a,b,c) points to.
 *   Edge {p,q} hits triangle (a,b,c) iff
 *     sign orient(a,b,c,p) * sign orient(a,b,c,q) < 0          (open segment)
 *   and the three signs of orient(p,q,a,b), orient(p,q,b,c), orient(p,q,c,a)
 *   are all >= 0 or all <= 0                                  (closed triangle).
 *   A touching endpoint or a coplanar edge is not a hit; a crossing through a
 *   shared triangle edge or vertex hits every incident face; a zero-area
 *   triangle never hits.
 *
 * Exactness.  The sign is first taken from a double-precision evaluation
 * whose absolute rounding error is bounded by 9*eps*permanent (eps = 2^-53):
 * every monomial of the determinant passes through at most eight roundings
 * (three differences, one product, one subtraction, one product, two sums),
 * and the permanent computed in floating point under-estimates the exact one
 * by at most a factor (1 - 8 eps).  When |det| does not exceed that bound the
 * sign is recomputed exactly: the 4x4 determinant
 *      | ax ay az 1 |
 *      | bx by bz 1 |   = -orient(a,b,c,p)
 *      | cx cy cz 1 |
 *      | px py pz 1 |
 * is expanded into its 24 Leibniz monomials, each the product of three raw
 * coordinates; each product is formed exactly as four doubles with Dekker's
 * split product, and the 96 doubles are summed exactly into a nonoverlapping
 * expansion (Shewchuk 1997, "Adaptive precision floating-point arithmetic
 * and fast robust geometric predicates": Two-Sum, Split, Two-Product and
 * Grow-Expansion with zero elimination).  The sign of such an expansion is
 * the sign of its largest component.
 *
 * Domain: every coordinate is 0 or has magnitude in [2^-200, 2^200], so that
 * no product underflows or overflows.  All finite float32 values qualify.
 *
 * Build: gcc -O2 -fPIC -shared -ffp-contract=off -fopenmp (no -ffast-math:
 * the expansion arithmetic relies on IEEE round-to-nearest without
 * contraction).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_EPS (1.1102230246251565e-16) /* 2^-53 */

/* ---------------------------------------------------------------- expansions */

static inline void ora_two_sum(double a, double b, double *s, double *e) {
  double x = a + b;
  double bv = x - a;
  double av = x - bv;
  *s = x;
  *e = (a - av) + (b - bv);
}

static inline void ora_split(double a, double *hi, double *lo) {
  double c = 134217729.0 * a; /* 2^27 + 1 */
  double big = c - a;
  *hi = c - big;
  *lo = a - *hi;
}

static inline void ora_two_product(double a, double b, double *p, double *e) {
  double x = a * b;
  double ah, al, bh, bl;
  ora_split(a, &ah, &al);
  ora_split(b, &bh, &bl);
  double err1 = x - ah * bh;
  double err2 = err1 - al * bh;
  double err3 = err2 - ah * bl;
  *p = x;
  *e = al * bl - err3;
}

/* h = e + b, e nonoverlapping with increasing magnitude; zeros dropped. */
static int ora_grow(const double *e, int n, double b, double *h) {
  double q = b;
  int m = 0;
  for (int i = 0; i < n; ++i) {
    double s, t;
    ora_two_sum(q, e[i], &s, &t);
    if (t != 0.0) h[m++] = t;
    q = s;
  }
  if (q != 0.0 || m == 0) h[m++] = q;
  return m;
}

static int ora_expansion_sign(const double *e, int n) {
  /* components are in increasing magnitude; the last one dominates */
  double top = e[n - 1];
  return (top > 0.0) - (top < 0.0);
}

/* Exact sign of orient(a,b,c,p) from the Leibniz expansion of the 4x4 form. */
int ora_orient_sign_exact(const double *a, const double *b, const double *c,
                          const double *p) {
  const double *rows[4] = {a, b, c, p};
  double acc[2][128];
  int n = 0, cur = 0;
  /* all 24 permutations sigma of {0,1,2,3}; row i takes column sigma[i] */
  for (int s0 = 0; s0 < 4; ++s0)
    for (int s1 = 0; s1 < 4; ++s1) {
      if (s1 == s0) continue;
      for (int s2 = 0; s2 < 4; ++s2) {
        if (s2 == s0 || s2 == s1) continue;
        int s3 = 6 - s0 - s1 - s2;
        int sig[4] = {s0, s1, s2, s3};
        int inv = 0;
        for (int i = 0; i < 4; ++i)
          for (int j = i + 1; j < 4; ++j)
            if (sig[i] > sig[j]) ++inv;
        double sgn = (inv & 1) ? -1.0 : 1.0;
        /* product of the three coordinate entries (column 3 holds 1) */
        double f[3];
        int k = 0;
        for (int i = 0; i < 4; ++i)
          if (sig[i] != 3) f[k++] = rows[i][sig[i]];
        double h, l, hh, hl, lh, ll;
        ora_two_product(sgn * f[0], f[1], &h, &l);
        ora_two_product(h, f[2], &hh, &hl);
        ora_two_product(l, f[2], &lh, &ll);
        double parts[4] = {hh, hl, lh, ll};
        for (int t = 0; t < 4; ++t) {
          if (parts[t] == 0.0) continue;
          n = ora_grow(acc[cur], n, parts[t], acc[cur ^ 1]);
          cur ^= 1;
        }
      }
    }
  if (n == 0) return 0;
  /* orient = -det4 */
  return -ora_expansion_sign(acc[cur], n);
}

/* Sign of orient(a,b,c,p): filtered double evaluation, exact when unsure. */
int ora_orient_sign(const double *a, const double *b, const double *c,
                    const double *p) {
  double ux = b[0] - a[0], uy = b[1] - a[1], uz = b[2] - a[2];
  double vx = c[0] - a[0], vy = c[1] - a[1], vz = c[2] - a[2];
  double wx = p[0] - a[0], wy = p[1] - a[1], wz = p[2] - a[2];
  double m1 = uy * vz, m2 = uz * vy;
  double m3 = uz * vx, m4 = ux * vz;
  double m5 = ux * vy, m6 = uy * vx;
  double det = wx * (m1 - m2) + wy * (m3 - m4) + wz * (m5 - m6);
  double perm = fabs(wx) * (fabs(m1) + fabs(m2)) +
                fabs(wy) * (fabs(m3) + fabs(m4)) +
                fabs(wz) * (fabs(m5) + fabs(m6));
  double bound = (9.0 * ORA_EPS) * perm;
  if (det > bound) return 1;
  if (-det > bound) return -1;
  return ora_orient_sign_exact(a, b, c, p);
}

/* Filter statistics are not kept: the oracle is only ever judged on signs. */

/* E-F hit test.  Returns 0 (no hit), 1 (hit, p is on the back side) or
 * 2 (hit, q is on the back side). */
int ora_ef_hit(const double *p, const double *q, const double *a,
               const double *b, const double *c) {
  int sp = ora_orient_sign(a, b, c, p);
  int sq = ora_orient_sign(a, b, c, q);
  if (sp * sq >= 0) return 0;
  int t1 = ora_orient_sign(p, q, a, b);
  int t2 = ora_orient_sign(p, q, b, c);
  int t3 = ora_orient_sign(p, q, c, a);
  int all_ge = (t1 >= 0) && (t2 >= 0) && (t3 >= 0);
  int all_le = (t1 <= 0) && (t2 <= 0) && (t3 <= 0);
  if (!(all_ge || all_le)) return 0;
  return sp < 0 ? 1 : 2;
}

/* --------------------------------------------------------------- brute force */

typedef struct {
  int32_t *rec; /* triples (edge, face, x0) */
  int64_t n, cap;
  int64_t cand;
} ora_buf;

static void ora_push(ora_buf *b, int32_t e, int32_t f, int32_t x0) {
  if (b->n == b->cap) {
    int64_t nc = b->cap ? 2 * b->cap : 256;
    int32_t *r = (int32_t *)realloc(b->rec, (size_t)nc * 3 * sizeof(int32_t));
    if (!r) abort();
    b->rec = r;
    b->cap = nc;
  }
  b->rec[3 * b->n + 0] = e;
  b->rec[3 * b->n + 1] = f;
  b->rec[3 * b->n + 2] = x0;
  b->n++;
}

/*
 * All E-F intersections between the edges of mesh E and the triangles of
 * mesh F, by testing every (edge, face) pair.  A pair whose closed axis-
 * aligned boxes do not overlap cannot intersect (the crossing point would
 * lie in both boxes), so only overlapping pairs ("candidates") are tested.
 *
 *   pe [nve][3]  positions of the edge mesh (doubles, exact copies of storage)
 *   edges [ne][2] vertex pairs of the edge mesh
 *   pf [nvf][3], tris [nf][3]  the face mesh
 *   out [cap][3] receives (edge index, face index, x0) in (edge, face) order
 *   *n_cand receives the number of candidate pairs tested
 * Returns the number of hits (which may exceed cap; then only cap are written).
 */
int64_t ora_dcd(const double *pe, const int32_t *edges, int64_t ne,
                const double *pf, const int32_t *tris, int64_t nf,
                int32_t *out, int64_t cap, int64_t *n_cand, int nthreads) {
  double *fb = (double *)malloc((size_t)(nf > 0 ? nf : 1) * 6 * sizeof(double));
  for (int64_t f = 0; f < nf; ++f) {
    const double *a = pf + 3 * (int64_t)tris[3 * f + 0];
    const double *b = pf + 3 * (int64_t)tris[3 * f + 1];
    const double *c = pf + 3 * (int64_t)tris[3 * f + 2];
    for (int k = 0; k < 3; ++k) {
      double lo = a[k], hi = a[k];
      if (b[k] < lo) lo = b[k];
      if (c[k] < lo) lo = c[k];
      if (b[k] > hi) hi = b[k];
      if (c[k] > hi) hi = c[k];
      fb[k * nf + f] = lo;       /* SoA: lo x, lo y, lo z */
      fb[(3 + k) * nf + f] = hi; /*      hi x, hi y, hi z */
    }
  }
  int nt = nthreads > 0 ? nthreads : 1;
#ifndef _OPENMP
  nt = 1;
#endif
  ora_buf *bufs = (ora_buf *)calloc((size_t)nt, sizeof(ora_buf));
#pragma omp parallel for schedule(static) num_threads(nt)
  for (int64_t e = 0; e < ne; ++e) {
    int tid = 0;
#ifdef _OPENMP
    tid = omp_get_thread_num();
#endif
    ora_buf *buf = &bufs[tid];
    const double *p = pe + 3 * (int64_t)edges[2 * e + 0];
    const double *q = pe + 3 * (int64_t)edges[2 * e + 1];
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      lo[k] = p[k] < q[k] ? p[k] : q[k];
      hi[k] = p[k] < q[k] ? q[k] : p[k];
    }
    for (int64_t f = 0; f < nf; ++f) {
      if (fb[0 * nf + f] > hi[0] || fb[3 * nf + f] < lo[0]) continue;
      if (fb[1 * nf + f] > hi[1] || fb[4 * nf + f] < lo[1]) continue;
      if (fb[2 * nf + f] > hi[2] || fb[5 * nf + f] < lo[2]) continue;
      buf->cand++;
      const double *a = pf + 3 * (int64_t)tris[3 * f + 0];
      const double *b = pf + 3 * (int64_t)tris[3 * f + 1];
      const double *c = pf + 3 * (int64_t)tris[3 * f + 2];
      int h = ora_ef_hit(p, q, a, b, c);
      if (h) ora_push(buf, (int32_t)e, (int32_t)f, h == 1 ? edges[2 * e] : edges[2 * e + 1]);
    }
  }
  /* static schedule: thread t holds a contiguous, increasing block of edges */
  int64_t total = 0, cand = 0;
  for (int t = 0; t < nt; ++t) {
    for (int64_t i = 0; i < bufs[t].n; ++i) {
      if (total < cap) memcpy(out + 3 * total, bufs[t].rec + 3 * i, 3 * sizeof(int32_t));
      total++;
    }
    cand += bufs[t].cand;
    free(bufs[t].rec);
  }
  free(bufs);
  free(fb);
  if (n_cand) *n_cand = cand;
  return total;
}

/* Hits of a given list of edges against every face (sampled checks). */
int64_t ora_dcd_edges(const double *pe, const int32_t *edges,
                      const int64_t *edge_ids, int64_t n_ids, const double *pf,
                      const int32_t *tris, int64_t nf, int32_t *out,
                      int64_t cap, int64_t *n_cand, int nthreads) {
  int32_t *sub = (int32_t *)malloc((size_t)(n_ids > 0 ? n_ids : 1) * 2 * sizeof(int32_t));
  for (int64_t i = 0; i < n_ids; ++i) {
    sub[2 * i] = edges[2 * edge_ids[i]];
    sub[2 * i + 1] = edges[2 * edge_ids[i] + 1];
  }
  int64_t n = ora_dcd(pe, sub, n_ids, pf, tris, nf, out, cap, n_cand, nthreads);
  int64_t m = n < cap ? n : cap;
  for (int64_t i = 0; i < m; ++i) out[3 * i] = (int32_t)edge_ids[out[3 * i]];
  free(sub);
  return n;
}

int ora_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
