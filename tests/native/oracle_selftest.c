/*
 * Self-test of the C oracle (oracle/tnn_oracle.c) under the address and
 * undefined-behaviour sanitizers, built with gcc by tests/test_sanitizers.py
 * (OpenMP off: the pragmas are ignored, the loops run serially).  Exercises
 * every entry point on small random inputs, including k > n, empty sets,
 * ragged segments and invalid per-query scales, and checks the output
 * shape: ascending (distance, index), candidates strictly earlier than
 * t_q - t_w, padding (-1, +inf) or (-1, NaN).  Prints "oracle ok".
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_knn(int64_t n, const float *x, const float *y, const float *z, const float *t,
               int64_t nq, const float *qx, const float *qy, const float *qz, const float *qt,
               const double *scale, double t_window, int32_t k, int64_t *idx, double *dist);
int oracle_knn_qscale(int64_t n, const float *x, const float *y, const float *z, const float *t,
                      int64_t nq, const float *qx, const float *qy, const float *qz,
                      const float *qt, const double *scale, double t_window, int32_t k,
                      int64_t *idx, double *dist);
int oracle_pair_dist(int64_t m, const int64_t *qi, const int64_t *pi, const float *qx,
                     const float *qy, const float *qz, const float *qt, const float *x,
                     const float *y, const float *z, const float *t, const double *scale,
                     double *out);
int oracle_pair_dist_qscale(int64_t m, const int64_t *qi, const int64_t *pi, const float *qx,
                            const float *qy, const float *qz, const float *qt, const float *x,
                            const float *y, const float *z, const float *t,
                            const double *scale, double *out);
int64_t oracle_segment_count(const int64_t *off, int64_t n_traj, int32_t seg_len);
int64_t oracle_segments(const float *x, const float *y, const float *z, const float *t,
                        const int64_t *off, int64_t n_traj, int32_t seg_len, int64_t cap,
                        int64_t *start, int32_t *count, double *a, double *b, double *tmin,
                        double *tmax, double *e);

#define CHECK(c)                                                            \
  do {                                                                      \
    if (!(c)) {                                                             \
      fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__);       \
      exit(1);                                                              \
    }                                                                       \
  } while (0)

static float frand(unsigned *s) {
  *s = *s * 1664525u + 1013904223u;
  return (float)((*s >> 8) & 0xffff) / 65536.0f;
}

static void check_rows(int64_t nq, int32_t k, const float *t, const float *qt, double tw,
                       const int64_t *idx, const double *dist, int allow_nan) {
  for (int64_t q = 0; q < nq; ++q) {
    for (int32_t r = 0; r < k; ++r) {
      const int64_t i = idx[q * k + r];
      const double d = dist[q * k + r];
      if (i < 0) {
        CHECK(isinf(d) || (allow_nan && isnan(d)));
        continue;
      }
      CHECK((double)t[i] < (double)qt[q] - tw);
      CHECK(d >= 0.0);
      if (r > 0 && idx[q * k + r - 1] >= 0) {
        const double p = dist[q * k + r - 1];
        CHECK(p < d || (p == d && idx[q * k + r - 1] < i));
      }
    }
  }
}

int main(void) {
  unsigned seed = 12345u;
  enum { N = 300, NQ = 40, K = 70 };
  float x[N], y[N], z[N], t[N], qx[NQ], qy[NQ], qz[NQ], qt[NQ];
  int64_t off[8] = {0, 40, 40, 101, 160, 220, 299, 300};
  for (int j = 0; j < 7; ++j) {
    float tt = 100.0f * frand(&seed);
    for (int64_t i = off[j]; i < off[j + 1]; ++i) {
      x[i] = 50.0f * frand(&seed);
      y[i] = 50.0f * frand(&seed);
      z[i] = 10.0f * frand(&seed);
      tt += 4.0f * frand(&seed);
      t[i] = tt;
    }
  }
  for (int q = 0; q < NQ; ++q) {
    qx[q] = 50.0f * frand(&seed);
    qy[q] = 50.0f * frand(&seed);
    qz[q] = 10.0f * frand(&seed);
    qt[q] = 400.0f * frand(&seed);
  }
  const double scale[4] = {1.0, 1.0, 10.0, 0.05};
  static int64_t idx[NQ * K];
  static double dist[NQ * K];
  const int32_t ks[] = {1, 8, K};
  const double tws[] = {0.0, 30.0};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 2; ++b) {
      CHECK(oracle_knn(N, x, y, z, t, NQ, qx, qy, qz, qt, scale, tws[b], ks[a], idx, dist) == 0);
      check_rows(NQ, ks[a], t, qt, tws[b], idx, dist, 0);
    }
  CHECK(oracle_knn(0, x, y, z, t, NQ, qx, qy, qz, qt, scale, 0.0, 4, idx, dist) == 0);
  check_rows(NQ, 4, t, qt, 0.0, idx, dist, 0);
  CHECK(oracle_knn(N, x, y, z, t, NQ, qx, qy, qz, qt, scale, 0.0, 0, idx, dist) != 0);
  static double rows[NQ * 4];
  for (int q = 0; q < NQ; ++q)
    for (int f = 0; f < 4; ++f) rows[4 * q + f] = scale[f] * (0.5 + frand(&seed));
  rows[4 * 3 + 1] = -1.0;
  rows[4 * 7 + 2] = NAN;
  CHECK(oracle_knn_qscale(N, x, y, z, t, NQ, qx, qy, qz, qt, rows, 0.0, 8, idx, dist) == 0);
  check_rows(NQ, 8, t, qt, 0.0, idx, dist, 1);
  CHECK(isnan(dist[3 * 8]) && isnan(dist[7 * 8]));
  int64_t qi[NQ * 5], pi[NQ * 5];
  double out[NQ * 5], out2[NQ * 5];
  for (int j = 0; j < NQ * 5; ++j) {
    qi[j] = j % NQ;
    pi[j] = (j * 7) % N;
  }
  CHECK(oracle_pair_dist(NQ * 5, qi, pi, qx, qy, qz, qt, x, y, z, t, scale, out) == 0);
  CHECK(oracle_pair_dist_qscale(NQ * 5, qi, pi, qx, qy, qz, qt, x, y, z, t, rows, out2) == 0);
  for (int j = 0; j < NQ * 5; ++j) CHECK(out[j] >= 0.0);
  const int32_t lens[] = {1, 7, 16, 64};
  for (int a = 0; a < 4; ++a) {
    const int64_t S = oracle_segment_count(off, 7, lens[a]);
    CHECK(S > 0);
    int64_t *start = malloc(sizeof(int64_t) * S);
    int32_t *count = malloc(sizeof(int32_t) * S);
    double *A = malloc(sizeof(double) * 3 * S), *B = malloc(sizeof(double) * 3 * S);
    double *tmin = malloc(sizeof(double) * S), *tmax = malloc(sizeof(double) * S);
    double *e = malloc(sizeof(double) * 3 * S);
    CHECK(oracle_segments(x, y, z, t, off, 7, lens[a], S, start, count, A, B, tmin, tmax, e) == S);
    CHECK(oracle_segments(x, y, z, t, off, 7, lens[a], S - 1, start, count, A, B, tmin, tmax, e) < 0);
    int64_t total = 0;
    for (int64_t s = 0; s < S; ++s) {
      CHECK(count[s] >= 1 && count[s] <= lens[a] && tmin[s] <= tmax[s]);
      CHECK(e[3 * s] >= 0.0 && e[3 * s + 1] >= 0.0 && e[3 * s + 2] >= 0.0);
      total += count[s];
    }
    CHECK(total == N);
    free(start), free(count), free(A), free(B), free(tmin), free(tmax), free(e);
  }
  CHECK(oracle_segment_count(off, 7, 0) < 0);
  printf("oracle ok\n");
  return 0;
}
