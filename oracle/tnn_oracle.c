/*
 * CPU oracle for exact masked, scaled k-nearest-neighbour search over
 * trajectory points.  TEST INFRASTRUCTURE ONLY: tests, the smoke check and the
 * benchmark's CPU-baseline leg call it; the GPU library never does.  It shares
 * no code, header or build flag with the GPU library.
 *
 * Built with  gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC
 * so that every floating-point operation below is one IEEE-754 binary64
 * operation with round-to-nearest-even, in the order written.
 *
 * What it computes (the plain definition that the trajectory search reaches
 * exactly, Sec. 4.2 / Table "numberofcomparison": the method is exact, so its
 * neighbours equal a linear search's):
 *
 *   metric (Sec. 3.4, the scaled metric and its space/time split):
 *     d(q, i) = sx*dx^2 + sy*dy^2 + sz*dz^2 + st*dt^2,   d? = q? - p?
 *     (the paper shares one scale between x and y; four independent scales
 *     are accepted here and the workloads pass sx = sy);
 *   time mask (Sec. 3.4, masked temporal part; Sec. 3.5): point i is a
 *     candidate for query q iff t_i < t_q - t_w (strict);
 *   result: the k candidates with the smallest (d, i), ascending, i being the
 *     position in the caller's arrays; missing slots are (-1, +inf).
 *
 * Every function returns 0 on success and -1 on a bad argument.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* One scaled squared distance; each step a single rounded binary64 op. */
static double scaled_sq_dist(const double s[4], float qx, float qy, float qz,
                             float qt, float px, float py, float pz, float pt) {
  double dx = (double)qx - (double)px;
  double dy = (double)qy - (double)py;
  double dz = (double)qz - (double)pz;
  double dt = (double)qt - (double)pt;
  double a = s[0] * (dx * dx);
  double b = s[1] * (dy * dy);
  double c = s[2] * (dz * dz);
  double e = s[3] * (dt * dt);
  return ((a + b) + c) + e;
}

/*
 * Brute-force masked scaled k-NN.  Points (x, y, z, t)[n], queries
 * (qx, qy, qz, qt)[nq], scale[4], t_window >= 0, k >= 1.
 * Writes out_idx[nq*k] (int64) and out_dist[nq*k] (binary64), row-major.
 * Ties: scanning i in increasing order and inserting only on a strictly
 * smaller distance keeps the lower index first among equal distances.
 */
int oracle_knn(int64_t n, const float *x, const float *y, const float *z,
               const float *t, int64_t nq, const float *qx, const float *qy,
               const float *qz, const float *qt, const double *scale,
               double t_window, int32_t k, int64_t *out_idx, double *out_dist) {
  if (n < 0 || nq < 0 || k < 1 || !scale) return -1;
  double s[4] = {scale[0], scale[1], scale[2], scale[3]};
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t q = 0; q < nq; ++q) {
    double *bd = out_dist + q * (int64_t)k;
    int64_t *bi = out_idx + q * (int64_t)k;
    for (int32_t r = 0; r < k; ++r) {
      bd[r] = INFINITY;
      bi[r] = -1;
    }
    double thr = (double)qt[q] - t_window;
    for (int64_t i = 0; i < n; ++i) {
      if (!((double)t[i] < thr)) continue;
      double d = scaled_sq_dist(s, qx[q], qy[q], qz[q], qt[q], x[i], y[i], z[i], t[i]);
      if (!(d < bd[k - 1])) continue;
      int32_t r = k - 1;
      while (r > 0 && d < bd[r - 1]) {
        bd[r] = bd[r - 1];
        bi[r] = bi[r - 1];
        --r;
      }
      bd[r] = d;
      bi[r] = i;
    }
  }
  return 0;
}

/* The same k-NN when every query has its own scales (Sec. 3.2: the scale
 * vector may be a function of position): query q uses scale[4 q .. 4 q + 3].
 * A row with a negative or non-finite scale has no metric: every slot of
 * that query is (-1, NaN). */
int oracle_knn_qscale(int64_t n, const float *x, const float *y, const float *z,
                      const float *t, int64_t nq, const float *qx, const float *qy,
                      const float *qz, const float *qt, const double *scale,
                      double t_window, int32_t k, int64_t *out_idx, double *out_dist) {
  if (n < 0 || nq < 0 || k < 1 || (!scale && nq > 0)) return -1;
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t q = 0; q < nq; ++q) {
    double *bd = out_dist + q * (int64_t)k;
    int64_t *bi = out_idx + q * (int64_t)k;
    double s[4];
    int ok = 1;
    for (int f = 0; f < 4; ++f) {
      s[f] = scale[4 * q + f];
      if (!(s[f] >= 0.0) || !isfinite(s[f])) ok = 0;
    }
    for (int32_t r = 0; r < k; ++r) {
      bd[r] = ok ? INFINITY : NAN;
      bi[r] = -1;
    }
    if (!ok) continue;
    double thr = (double)qt[q] - t_window;
    for (int64_t i = 0; i < n; ++i) {
      if (!((double)t[i] < thr)) continue;
      double d = scaled_sq_dist(s, qx[q], qy[q], qz[q], qt[q], x[i], y[i], z[i], t[i]);
      if (!(d < bd[k - 1])) continue;
      int32_t r = k - 1;
      while (r > 0 && d < bd[r - 1]) {
        bd[r] = bd[r - 1];
        bi[r] = bi[r - 1];
        --r;
      }
      bd[r] = d;
      bi[r] = i;
    }
  }
  return 0;
}

/* Distances of explicit (query, point) pairs with the same arithmetic:
 * used to check sampled outputs at full size. */
int oracle_pair_dist(int64_t m, const int64_t *qi, const int64_t *pi,
                     const float *qx, const float *qy, const float *qz,
                     const float *qt, const float *x, const float *y,
                     const float *z, const float *t, const double *scale,
                     double *out) {
  if (m < 0 || !scale) return -1;
  double s[4] = {scale[0], scale[1], scale[2], scale[3]};
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < m; ++j) {
    int64_t a = qi[j], b = pi[j];
    out[j] = scaled_sq_dist(s, qx[a], qy[a], qz[a], qt[a], x[b], y[b], z[b], t[b]);
  }
  return 0;
}

/* The same with one scale row per query (Sec. 3.2, scales as a function of
 * position): pair j uses the metric of its query, scale[4*qi[j] .. +3]. */
int oracle_pair_dist_qscale(int64_t m, const int64_t *qi, const int64_t *pi,
                            const float *qx, const float *qy, const float *qz,
                            const float *qt, const float *x, const float *y,
                            const float *z, const float *t, const double *scale,
                            double *out) {
  if (m < 0 || !scale) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < m; ++j) {
    int64_t a = qi[j], b = pi[j];
    const double *s = scale + 4 * a;
    out[j] = scaled_sq_dist(s, qx[a], qy[a], qz[a], qt[a], x[b], y[b], z[b], t[b]);
  }
  return 0;
}

/* Number of segments that cutting every trajectory into runs of seg_len
 * consecutive points produces (the last run of a trajectory may be shorter:
 * no padding copies). */
int64_t oracle_segment_count(const int64_t *off, int64_t n_traj, int32_t seg_len) {
  if (n_traj < 0 || seg_len < 1) return -1;
  int64_t s = 0;
  for (int64_t j = 0; j < n_traj; ++j) {
    int64_t len = off[j + 1] - off[j];
    if (len < 0) return -1;
    s += (len + seg_len - 1) / seg_len;
  }
  return s;
}

/*
 * Segments of Sec. 3.4 (partition into sets of K consecutive time-sorted
 * points, each approximated by the segment from its first point A to its last
 * point B) with the approximation error of the same section, kept per axis:
 *   for every member P: u = clamp(<AP, AB> / |AB|_2^2, 0, 1)  (u = 0 when
 *   |AB| = 0), Q = A + u AB (Euclidean clamped projection, Sec. 3.4),
 *   e_f = max over members of |P_f - Q_f|,  f in {x, y, z}.
 * Also t_min / t_max over the members, start and count.
 * Arrays: start[S], count[S], a[3S], b[3S], tmin[S], tmax[S], e[3S]
 * (xyz interleaved).  Returns S, or -1.
 */
int64_t oracle_segments(const float *x, const float *y, const float *z,
                        const float *t, const int64_t *off, int64_t n_traj,
                        int32_t seg_len, int64_t cap, int64_t *start,
                        int32_t *count, double *a, double *b, double *tmin,
                        double *tmax, double *e) {
  int64_t total = oracle_segment_count(off, n_traj, seg_len);
  if (total < 0 || total > cap) return -1;
  int64_t s = 0;
  for (int64_t j = 0; j < n_traj; ++j) {
    for (int64_t p0 = off[j]; p0 < off[j + 1]; p0 += seg_len) {
      int64_t c = off[j + 1] - p0;
      if (c > seg_len) c = seg_len;
      int64_t p1 = p0 + c - 1;
      double A[3] = {x[p0], y[p0], z[p0]};
      double B[3] = {x[p1], y[p1], z[p1]};
      double AB[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
      double n2 = (AB[0] * AB[0] + AB[1] * AB[1]) + AB[2] * AB[2];
      double ex = 0.0, ey = 0.0, ez = 0.0;
      double lo = (double)t[p0], hi = (double)t[p0];
      for (int64_t i = p0; i <= p1; ++i) {
        double P[3] = {x[i], y[i], z[i]};
        double AP[3] = {P[0] - A[0], P[1] - A[1], P[2] - A[2]};
        double u = 0.0;
        if (n2 > 0.0) {
          u = ((AP[0] * AB[0] + AP[1] * AB[1]) + AP[2] * AB[2]) / n2;
          if (u < 0.0) u = 0.0;
          if (u > 1.0) u = 1.0;
        }
        double Q[3] = {A[0] + u * AB[0], A[1] + u * AB[1], A[2] + u * AB[2]};
        double dx = fabs(P[0] - Q[0]), dy = fabs(P[1] - Q[1]), dz = fabs(P[2] - Q[2]);
        if (dx > ex) ex = dx;
        if (dy > ey) ey = dy;
        if (dz > ez) ez = dz;
        if ((double)t[i] < lo) lo = (double)t[i];
        if ((double)t[i] > hi) hi = (double)t[i];
      }
      start[s] = p0;
      count[s] = (int32_t)c;
      for (int f = 0; f < 3; ++f) {
        a[3 * s + f] = A[f];
        b[3 * s + f] = B[f];
      }
      tmin[s] = lo;
      tmax[s] = hi;
      e[3 * s + 0] = ex;
      e[3 * s + 1] = ey;
      e[3 * s + 2] = ez;
      ++s;
    }
  }
  return s;
}
