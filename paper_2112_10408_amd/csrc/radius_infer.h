// Learned k-th radius: the model's parameter layout, its feature map and the
// MFMA inference of one workgroup, shared by the radius kernels and by the
// search's per-call preparation (which predicts the radius in the same
// launch).  Not part of the paper; the prediction only seeds TNN_LEARNED
// queries.
#pragma once
#include <cmath>

#include "tnn_internal.h"
#include "wave.h"

namespace tnn {
namespace radius {

constexpr int H = TNN_RADIUS_HIDDEN;
constexpr int NI = TNN_RADIUS_INPUTS;
constexpr int G = TNN_RADIUS_GRID;
constexpr int SXY = TNN_RADIUS_START_XY;
constexpr int ST = TNN_RADIUS_START_T;
constexpr int64_t kStartCells = (int64_t)SXY * SXY * ST;
constexpr int NP = TNN_RADIUS_NPARAMS;
// offsets of the parameter tensors in params[]
constexpr int OW1 = 0, OB1 = OW1 + H * NI, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H,
              OB3 = OW3 + H;
static_assert(OB3 + 1 == NP, "parameter layout");

// Cell along one axis of a grid of n cells over [lo, hi], decided in float32
// exactly as written: min(n-1, max(0, trunc((v - lo) * (n / (hi - lo))))).
__device__ inline int cell_n(float v, float lo, float hi, int n) {
  const float span = hi - lo;
  const float cs = span > 0.0f ? (float)n / span : 0.0f;
  float c = (v - lo) * cs;
  if (!isfinite(c)) c = 0.0f;
  c = truncf(c);
  int i = (int)fminf(fmaxf(c, 0.0f), (float)(n - 1));
  return i;
}

__device__ inline int cell_of(float v, float lo, float hi) { return cell_n(v, lo, hi, G); }

__device__ inline void features(const tnn_radius_model *m, float x, float y, float z, float t,
                                float f[NI]) {
  const float v[4] = {x, y, z, t};
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const float span = m->hi[j] - m->lo[j];
    const float g = span > 0.0f ? 2.0f / span : 1.0f;
    f[j] = (v[j] - 0.5f * (m->lo[j] + m->hi[j])) * g;
  }
  const int cx = cell_of(x, m->lo[0], m->hi[0]);
  const int cy = cell_of(y, m->lo[1], m->hi[1]);
  const int ct = cell_of(t, m->lo[3], m->hi[3]);
  f[4] = 0.25f * log1pf((float)m->grid[(cx * G + cy) * G + ct]);
  // trajectory starts in the start-grid cell, its 8 spatial neighbours and
  // those 9 cells one time step earlier: summed into each cell at init
  const int sx = cell_n(x, m->lo[0], m->hi[0], SXY);
  const int sy = cell_n(y, m->lo[1], m->hi[1], SXY);
  const int stc = cell_n(t, m->lo[3], m->hi[3], ST);
  f[5] = 0.5f * log1pf((float)m->starts[((int64_t)sx * SXY + sy) * ST + stc]);
}

// Inference, one wave per tile of 32 queries.  The hidden-to-hidden layer
// (the only dense contraction: 32 queries x 64 inputs x 64 units) runs on
// the matrix cores with float32 operands, v_mfma_f32_32x32x2f32:
//   A (32 x 2): lane l holds A[l % 32][l / 32]   (query l % 32, input 2s + l / 32)
//   B (2 x 32): lane l holds B[l / 32][l % 32]   (input 2s + l / 32, unit l % 32)
//   D (32 x 32): element e of lane l is D[(e / 4) 8 + (l / 32) 4 + e % 4][l % 32]
// Two output blocks cover units 0..31 and 32..63; 32 K-steps of 2 cover the
// 64 inputs.  The first layer (6 -> 64) and the output layer run on the
// vector units; the output layer's sum over units goes through LDS.
typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kInferTile = 32;
constexpr int kInferWaves = 4;  // waves per workgroup; the weights are staged once per workgroup

// The tile loop of one workgroup of 64 * kInferWaves threads: workgroup
// `group` of `n_groups` (every thread of the workgroup calls it).
__device__ __forceinline__ void infer_tiles(const tnn_radius_model *__restrict__ m, tnn_points q,
                                            float alpha, float *__restrict__ radius2,
                                            float *__restrict__ logr, int64_t group,
                                            int64_t n_groups) {
  __shared__ float w2s[H][H + 1];  // hidden-to-hidden weights, padded rows
  __shared__ float4 w1s[H][2];     // first layer, per unit: weights 0..3 | weights 4, 5, bias
  static_assert(NI == 6, "the first layer's LDS layout holds six weights and a bias per unit");
  static_assert(H == 64, "the MFMA tiling covers 64 hidden units: two 32-unit output blocks "
                         "(c0, c1) and H / 2 K-steps of two inputs");
  __shared__ float part[kInferWaves][kInferTile][kInferTile + 1];
  const float *__restrict__ W = m->params;
  const int wv = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int col = l & 31;   // unit within an output block / query within the tile
  const int half = l >> 5;  // which of the two inputs of a K-step
  const int64_t n_tiles = (q.n + kInferTile - 1) / kInferTile;
  const int64_t tile0 = group * kInferWaves + wv;
  // the first tile's query point is requested before the weights are staged,
  // so the two latencies overlap
  float px = 0.0f, py = 0.0f, pz = 0.0f, pt = 0.0f;
  {
    const int64_t qi = tile0 * kInferTile + col;
    if (tile0 < n_tiles && qi < q.n) {
      px = q.x[qi];
      py = q.y[qi];
      pz = q.z[qi];
      pt = q.t[qi];
    }
  }
  {
    // all of a thread's loads in flight before its first LDS write (a rolled
    // loop waits out one global-load latency per element)
    constexpr int kThreads = 64 * kInferWaves, kPer = H * H / kThreads;
    static_assert(H * H % kThreads == 0, "hidden weights split evenly over the threads");
    float wv[kPer];
#pragma unroll
    for (int r = 0; r < kPer; ++r) wv[r] = W[OW2 + threadIdx.x + r * kThreads];
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
      const int i = threadIdx.x + r * kThreads;
      w2s[i / H][i % H] = wv[r];
    }
  }
  for (int k = threadIdx.x; k < H; k += blockDim.x) {
    w1s[k][0] = make_float4(W[OW1 + k * NI], W[OW1 + k * NI + 1], W[OW1 + k * NI + 2],
                            W[OW1 + k * NI + 3]);
    w1s[k][1] = make_float4(W[OW1 + k * NI + 4], W[OW1 + k * NI + 5], W[OB1 + k], 0.0f);
  }
  __syncthreads();
  const float b2_0 = W[OB2 + col], b2_1 = W[OB2 + 32 + col];
  const float w3_0 = W[OW3 + col], w3_1 = W[OW3 + 32 + col];
  const float b3 = W[OB3];
  float(*pw)[kInferTile + 1] = part[wv];
  for (int64_t tile = tile0; tile < n_tiles; tile += n_groups * kInferWaves) {
    const int64_t qi = tile * kInferTile + col;
    const bool ok = qi < q.n;
    if (tile != tile0 && ok) {
      px = q.x[qi];
      py = q.y[qi];
      pz = q.z[qi];
      pt = q.t[qi];
    }
    float f[NI] = {};
    if (ok) features(m, px, py, pz, pt, f);
    f32x16 c0, c1;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      c0[e] = b2_0;
      c1[e] = b2_1;
    }
    // per K-step: the first-layer unit this lane feeds to the matrix cores
    // and the B operands W2[unit][input], formed just before their MFMAs (a
    // wave usually answers one tile: holding all 32 steps' operands in
    // registers only limited how many waves fit on a SIMD)
#pragma unroll
    for (int st = 0; st < H / 2; ++st) {
      const float4 wa = w1s[2 * st + half][0], wb = w1s[2 * st + half][1];
      const float a =
          wb.z + wa.x * f[0] + wa.y * f[1] + wa.z * f[2] + wa.w * f[3] + wb.x * f[4] + wb.y * f[5];
      const float h1 = fmaxf(a, 0.0f);
      c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(h1, w2s[col][2 * st + half], c0, 0, 0, 0);
      c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(h1, w2s[32 + col][2 * st + half], c1, 0, 0, 0);
    }
    // output layer: per (query row, unit) terms, summed over units through
    // this wave's LDS rows
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int row = (e >> 2) * 8 + half * 4 + (e & 3);
      pw[row][col] = w3_0 * fmaxf(c0[e], 0.0f) + w3_1 * fmaxf(c1[e], 0.0f);
    }
    wave_sync();
    if (l < kInferTile && ok) {
      float out = b3;
#pragma unroll
      for (int u = 0; u < kInferTile; ++u) out += pw[l][u];
      const float r = alpha * expf(out);
      radius2[qi] = r * r;
      if (logr) logr[qi] = out;
    }
    wave_sync();
  }
}

}  // namespace radius
}  // namespace tnn
