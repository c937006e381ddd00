// Learned k-th radius: a 6-64-64-1 ReLU MLP (float32) with hand-written
// inference, forward/backward and Adam kernels.  Not part of the paper; it
// only seeds the search radius of TNN_LEARNED queries.
#include <cmath>
#include <cstring>

#include "host.h"
#include "radius_infer.h"
#include "tnn_internal.h"
#include "wave.h"

namespace tnn {
namespace {

using namespace radius;
constexpr int kTrainBlock = 64;  // samples per workgroup in the forward/backward pass

__host__ __device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

__global__ void init_kernel(tnn_radius_model *m, uint64_t seed, IndexDesc ix) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < NP) {
    int fan_in = 0;
    if (i < OB1) fan_in = NI;
    else if (i >= OW2 && i < OB2) fan_in = H;
    else if (i >= OW3 && i < OB3) fan_in = H;
    float w = 0.0f;
    if (fan_in) {
      const uint64_t r = splitmix64(seed ^ ((uint64_t)i * 0xd1b54a32d192ed03ull));
      const float u = (float)(r >> 40) * (1.0f / 16777216.0f);  // [0, 1)
      w = (2.0f * u - 1.0f) * sqrtf(6.0f / (float)fan_in);
    }
    m->params[i] = w;
  }
  if (i < 3) m->pad[i] = 0.0f;
  if (i < 4) {
    m->lo[i] = ix.lo[i];
    m->hi[i] = ix.hi[i];
  }
  if (i < G * G * G) m->grid[i] = 0;
}

__global__ void starts_zero_kernel(tnn_radius_model *m) {
  uint32_t *w = reinterpret_cast<uint32_t *>(m->starts);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < kStartCells / 2;
       i += (int64_t)gridDim.x * blockDim.x)
    w[i] = 0u;
}

// Saturating increment of a 16-bit count inside its aligned 32-bit word.
__device__ inline void add_start(tnn_radius_model *m, int64_t cell) {
  uint32_t *w = reinterpret_cast<uint32_t *>(m->starts) + (cell >> 1);
  const int shift = (int)(cell & 1) * 16;
  uint32_t old = *w;
  for (;;) {
    if (((old >> shift) & 0xffffu) == 0xffffu) return;
    const uint32_t seen = atomicCAS(w, old, old + (1u << shift));
    if (seen == old) return;
    old = seen;
  }
}

__global__ void grid_kernel(tnn_radius_model *m, IndexDesc ix) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ix.n_seg) return;
  if (ix.sfirst[s]) {
    // the trajectory's first point (A and t_min of its first segment) counts
    // for every cell whose neighbourhood holds it: the 3 x 3 spatial block
    // around its cell, at its time cell and the next
    const int sx = cell_n(ix.ax[s], m->lo[0], m->hi[0], SXY);
    const int sy = cell_n(ix.ay[s], m->lo[1], m->hi[1], SXY);
    const int stc = cell_n(ix.tmin[s], m->lo[3], m->hi[3], ST);
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dt = 0; dt <= 1; ++dt) {
          const int cx2 = sx + dx, cy2 = sy + dy, ct2 = stc + dt;
          if (cx2 >= 0 && cx2 < SXY && cy2 >= 0 && cy2 < SXY && ct2 < ST)
            add_start(m, ((int64_t)cx2 * SXY + cy2) * ST + ct2);
        }
  }
  const float mx = 0.5f * (ix.ax[s] + ix.bx[s]);
  const float my = 0.5f * (ix.ay[s] + ix.by[s]);
  const float mt = 0.5f * (ix.tmin[s] + ix.tmax[s]);
  const int cx = cell_of(mx, m->lo[0], m->hi[0]);
  const int cy = cell_of(my, m->lo[1], m->hi[1]);
  const int ct = cell_of(mt, m->lo[3], m->hi[3]);
  atomicAdd(&m->grid[(cx * G + cy) * G + ct], 1);
}

__global__ void features_kernel(const tnn_radius_model *m, tnn_points q, float *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= q.n) return;
  float f[NI];
  features(m, q.x[i], q.y[i], q.z[i], q.t[i], f);
  for (int j = 0; j < NI; ++j) out[NI * i + j] = f[j];
}

__global__ __launch_bounds__(64 * kInferWaves) void infer_kernel(
    const tnn_radius_model *__restrict__ m, tnn_points q, float alpha, float *__restrict__ radius2,
    float *__restrict__ logr) {
  infer_tiles(m, q, alpha, radius2, logr, blockIdx.x, gridDim.x);
}

// Sample b of the batch is samples[order[first + b]] (order: a permutation of
// the samples, device int32), or samples[first + b] without one.
__device__ __forceinline__ int64_t sample_of(const int32_t *order, int64_t first, int64_t b) {
  return order ? (int64_t)order[first + b] : first + b;
}

// Forward and backward over kTrainBlock samples per workgroup, one wave per
// tile of 32 samples; writes this workgroup's un-normalised gradient sum
// (2 r dout/dtheta) and its loss partials (sum r^2, count) to
// partial[blockIdx].  A tile's three dense contractions run on the matrix
// cores with float32 operands, in the lane layout of the inference
// (v_mfma_f32_32x32x2f32): the hidden layer (32 samples x 64 inputs x 64
// units), the delta through the hidden weights (32 samples x 64 units x 64
// inputs) and the hidden weights' gradient (64 units x 32 samples x 64
// inputs).  The first layer, the output layer and the biases, whose
// gradients are short sums over the workgroup's samples, run on the vector
// units from LDS.
constexpr int kTrainTile = 32;
constexpr int kTrainWaves = kTrainBlock / kTrainTile;
constexpr int kRow = H + 1;  // padded LDS row
static_assert(kTrainWaves == 2, "two tiles per workgroup: their hidden-weight gradients are "
                                "exchanged through the two activation areas");
static_assert(kTrainWaves * kTrainTile * kRow >= H * H, "an activation area holds a tile's "
                                                        "hidden-weight gradient");

__global__ __launch_bounds__(64 * kTrainWaves) void fwd_bwd_kernel(
    const tnn_radius_model *m, tnn_points smp, const double *dist, const int32_t *order, int32_t k,
    int64_t first, int64_t batch, float *partial) {
  static_assert(NI == 6 && H == 64, "the tiling covers 6 inputs and 64 hidden units");
  __shared__ float W2s[H][kRow];  // W2s[unit][input]
  __shared__ float4 W1s[H][2];    // per unit: weights 0..3 | weights 4, 5, bias
  __shared__ float H1[kTrainWaves][kTrainTile][kRow];  // h1[sample][unit]
  __shared__ float H2[kTrainWaves][kTrainTile][kRow];  // h2[sample][unit]
  __shared__ float G2[kTrainWaves][kTrainTile][kRow];  // dL/dz2
  __shared__ float G1[kTrainWaves][kTrainTile][kRow];  // output-layer terms, then dL/dz1
  __shared__ float F[kTrainWaves][kTrainTile][NI];
  __shared__ float GO[kTrainWaves][kTrainTile];  // dL/dout (un-normalised: 2 r)
  __shared__ float R2[kTrainWaves][kTrainTile];
  __shared__ float LB[kTrainWaves][kTrainTile];  // 1 for a labelled sample
  const float *__restrict__ W = m->params;
  const int wv = threadIdx.x >> 6;
  const int l = threadIdx.x & 63;
  const int col = l & 31;   // sample (A rows) or unit / input (B, D columns) within a block
  const int half = l >> 5;  // which of the two K entries of a step
  // All of a thread's hidden-weight loads are issued before the sample's
  // dependent loads and written to LDS after them, so that the latencies
  // overlap (a rolled loop waits out one load latency per element).
  constexpr int kThreads = 64 * kTrainWaves, kPer = H * H / kThreads;
  static_assert(H * H % kThreads == 0, "hidden weights split evenly over the threads");
  float w2v[kPer];
#pragma unroll
  for (int r = 0; r < kPer; ++r) w2v[r] = W[OW2 + threadIdx.x + r * kThreads];
  // the lane's sample (both halves of the wave hold the same 32 samples)
  const int64_t b = (int64_t)blockIdx.x * kTrainBlock + wv * kTrainTile + col;
  float f[NI] = {};
  bool lab = false;
  float y = 0.0f;
  if (b < batch) {
    const int64_t si = sample_of(order, first, b);
    features(m, smp.x[si], smp.y[si], smp.z[si], smp.t[si], f);
    const double dk = dist[si * k + (k - 1)];
    lab = dk > 0.0 && dk < __builtin_huge_val();
    if (lab) y = (float)(0.5 * log(dk));
  }
  // the hidden weights into LDS (their loads were issued first)
#pragma unroll
  for (int r = 0; r < kPer; ++r) {
    const int i = threadIdx.x + r * kThreads;
    W2s[i / H][i % H] = w2v[r];
  }
  for (int u = threadIdx.x; u < H; u += blockDim.x) {
    W1s[u][0] = make_float4(W[OW1 + u * NI], W[OW1 + u * NI + 1], W[OW1 + u * NI + 2],
                            W[OW1 + u * NI + 3]);
    W1s[u][1] = make_float4(W[OW1 + u * NI + 4], W[OW1 + u * NI + 5], W[OB1 + u], 0.0f);
  }
  if (half == 0)
#pragma unroll
    for (int c = 0; c < NI; ++c) F[wv][col][c] = f[c];
  __syncthreads();
  float(*h1)[kRow] = H1[wv];
  float(*h2)[kRow] = H2[wv];
  float(*g2)[kRow] = G2[wv];
  float(*g1)[kRow] = G1[wv];

  // forward: z2 = b2 + W2 h1 on the matrix cores, h1 formed per K-step
  f32x16 c0, c1;
  {
    const float b2_0 = W[OB2 + col], b2_1 = W[OB2 + 32 + col];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      c0[e] = b2_0;
      c1[e] = b2_1;
    }
  }
#pragma unroll 4
  for (int st = 0; st < H / 2; ++st) {
    const int u = 2 * st + half;
    const float4 wa = W1s[u][0], wb = W1s[u][1];
    const float a =
        wb.z + wa.x * f[0] + wa.y * f[1] + wa.z * f[2] + wa.w * f[3] + wb.x * f[4] + wb.y * f[5];
    const float hu = fmaxf(a, 0.0f);
    h1[col][u] = hu;
    c0 = __builtin_amdgcn_mfma_f32_32x32x2f32(hu, W2s[col][u], c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x2f32(hu, W2s[32 + col][u], c1, 0, 0, 0);
  }
  // output layer: per (sample, unit) terms summed over units through LDS
  const float w3_0 = W[OW3 + col], w3_1 = W[OW3 + 32 + col];
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int row = (e >> 2) * 8 + half * 4 + (e & 3);
    const float a0 = fmaxf(c0[e], 0.0f), a1 = fmaxf(c1[e], 0.0f);
    h2[row][col] = a0;
    h2[row][32 + col] = a1;
    g1[row][col] = w3_0 * a0 + w3_1 * a1;
  }
  wave_sync();
  if (l < kTrainTile) {
    float out = W[OB3];
#pragma unroll
    for (int u = 0; u < kTrainTile; ++u) out += g1[l][u];
    float go = 0.0f, r2 = 0.0f;
    if (lab) {
      const float r = out - y;
      go = 2.0f * r;
      r2 = r * r;
    }
    GO[wv][l] = go;
    R2[wv][l] = r2;
    LB[wv][l] = lab ? 1.0f : 0.0f;
  }
  wave_sync();
  // dL/dz2 = go w3 where z2 > 0
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    const int row = (e >> 2) * 8 + half * 4 + (e & 3);
    const float go = GO[wv][row];
    g2[row][col] = c0[e] > 0.0f ? go * w3_0 : 0.0f;
    g2[row][32 + col] = c1[e] > 0.0f ? go * w3_1 : 0.0f;
  }
  wave_sync();
  // dL/dz1 = (W2^T dL/dz2) where z1 > 0: A = dL/dz2 (sample x unit), B = W2
  // (unit x input)
  {
    f32x16 d0, d1;
#pragma unroll
    for (int e = 0; e < 16; ++e) d0[e] = d1[e] = 0.0f;
#pragma unroll 4
    for (int st = 0; st < H / 2; ++st) {
      const int j = 2 * st + half;
      const float a = g2[col][j];
      d0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, W2s[j][col], d0, 0, 0, 0);
      d1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, W2s[j][32 + col], d1, 0, 0, 0);
    }
    wave_sync();  // the output-layer terms in g1 have been read
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int row = (e >> 2) * 8 + half * 4 + (e & 3);
      g1[row][col] = h1[row][col] > 0.0f ? d0[e] : 0.0f;
      g1[row][32 + col] = h1[row][32 + col] > 0.0f ? d1[e] : 0.0f;
    }
  }
  // the tile's hidden-weight gradient, sum over samples of dL/dz2[s][unit]
  // h1[s][input]: A = dL/dz2^T (unit x sample), B = h1 (sample x input)
  f32x16 acc[2][2];
#pragma unroll
  for (int jb = 0; jb < 2; ++jb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[jb][cb][e] = 0.0f;
#pragma unroll 4
  for (int st = 0; st < kTrainTile / 2; ++st) {
    const int s = 2 * st + half;
    const float a0 = g2[s][col], a1 = g2[s][32 + col];
    const float b0 = h1[s][col], b1 = h1[s][32 + col];
    acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b0, acc[0][0], 0, 0, 0);
    acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, b1, acc[0][1], 0, 0, 0);
    acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b0, acc[1][0], 0, 0, 0);
    acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, b1, acc[1][1], 0, 0, 0);
  }
  __syncthreads();

  // the small gradients over the workgroup's samples, tile by tile
  float *out = partial + (size_t)blockIdx.x * (NP + 3);
  for (int q = threadIdx.x; q < NP - H * H; q += blockDim.x) {
    const int p = q < OW2 ? q : q + H * H;  // every parameter but the hidden weights
    float a = 0.0f;
    for (int w = 0; w < kTrainWaves; ++w) {
      if (p < OB1) {
        const int j = p / NI, c = p % NI;
        for (int s = 0; s < kTrainTile; ++s) a += G1[w][s][j] * F[w][s][c];
      } else if (p < OW2) {
        for (int s = 0; s < kTrainTile; ++s) a += G1[w][s][p - OB1];
      } else if (p < OW3) {
        for (int s = 0; s < kTrainTile; ++s) a += G2[w][s][p - OB2];
      } else if (p < OB3) {
        for (int s = 0; s < kTrainTile; ++s) a += GO[w][s] * H2[w][s][p - OW3];
      } else {
        for (int s = 0; s < kTrainTile; ++s) a += GO[w][s];
      }
    }
    out[p] = a;
  }
  if (threadIdx.x == 0) {
    float loss = 0.0f, cnt = 0.0f;
    for (int w = 0; w < kTrainWaves; ++w)
      for (int s = 0; s < kTrainTile; ++s) {
        loss += R2[w][s];
        cnt += LB[w][s];
      }
    out[NP] = loss;
    out[NP + 1] = cnt;
  }
  __syncthreads();
  // hidden weights: tile 0's gradient in the H1 area, tile 1's in H2, summed
  float *xg = wv == 0 ? &H1[0][0][0] : &H2[0][0][0];
#pragma unroll
  for (int jb = 0; jb < 2; ++jb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int j = jb * 32 + (e >> 2) * 8 + half * 4 + (e & 3);
        xg[j * H + cb * 32 + col] = acc[jb][cb][e];
      }
  __syncthreads();
  const float *x0 = &H1[0][0][0], *x1 = &H2[0][0][0];
  for (int i = threadIdx.x; i < H * H; i += blockDim.x) out[OW2 + i] = x0[i] + x1[i];
}

// Sum of the partials in block order (deterministic), divided by the number
// of labelled samples.
// The loops are unrolled so that 16 loads are in flight at a time (a rolled
// loop waits out one load latency per block); the sums stay in block order.
__global__ void reduce_kernel(const float *__restrict__ partial, int nblk, float *grad,
                              float *loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  float n = 0.0f;
#pragma unroll 16
  for (int b = 0; b < nblk; ++b) n += partial[(size_t)b * (NP + 3) + NP + 1];
  const float inv = 1.0f / fmaxf(n, 1.0f);
  if (p < NP) {
    float a = 0.0f;
#pragma unroll 16
    for (int b = 0; b < nblk; ++b) a += partial[(size_t)b * (NP + 3) + p];
    grad[p] = a * inv;
  }
  if (p == 0 && loss) {
    float l = 0.0f;
#pragma unroll 16
    for (int b = 0; b < nblk; ++b) l += partial[(size_t)b * (NP + 3) + NP];
    *loss = l * inv;
  }
}

__global__ void adam_kernel(float *params, float *mom, const float *grad, int step, float lr) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float g = grad[p];
  const float m = b1 * mom[p] + (1.0f - b1) * g;
  const float v = b2 * mom[NP + p] + (1.0f - b2) * g * g;
  mom[p] = m;
  mom[NP + p] = v;
  const float mh = m / (1.0f - powf(b1, (float)step));
  const float vh = v / (1.0f - powf(b2, (float)step));
  params[p] -= lr * mh / (sqrtf(vh) + eps);
}

// ---------------------------------------------------------------------------
// Training order: a permutation of [0, n) drawn from a seed, element i being
// a keyed 4-round Feistel permutation of [0, 4^h) (4^h >= n, the smallest
// such) walked along its cycle until it lands below n (cycle walking keeps
// it a bijection on [0, n)).  The round function is SplitMix64 of the seed,
// the round and the half.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t feistel(uint64_t v, int h, uint64_t seed) {
  const uint64_t mask = (1ull << h) - 1;
  uint64_t l = v >> h, r = v & mask;
#pragma unroll
  for (int round = 0; round < 4; ++round) {
    const uint64_t f = splitmix64(seed ^ ((uint64_t)(round + 1) << 56) ^ r) & mask;
    const uint64_t nl = r;
    r = l ^ f;
    l = nl;
  }
  return (l << h) | r;
}

__global__ void shuffle_kernel(int64_t n, int h, uint64_t seed, int32_t *order) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  // each step moves along the cycle of i; the first value below n ends the
  // walk (the cycle holds i itself, so the walk is finite)
  uint64_t v = (uint64_t)i;
  do {
    v = feistel(v, h, seed);
  } while (v >= (uint64_t)n);
  order[i] = (int32_t)v;
}

// ---------------------------------------------------------------------------
// Safety factor of the predicted radius: alpha = exp(x_q), x_q the quantile q
// (linear interpolation between order statistics, position (m - 1) q) of the
// log-residuals 0.5 log d_k - out over the m samples whose k-th distance is
// finite and positive and whose residual is finite.  Residuals are binary64,
// kept as order-preserving 64-bit keys; one workgroup selects the two order
// statistics by an 8-bit radix select.
// ---------------------------------------------------------------------------
constexpr unsigned long long kNoKey = ~0ull;  // above every finite value's key
constexpr int kSelectThreads = 1024;

__device__ __forceinline__ unsigned long long order_key(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | (1ull << 63));
}

__device__ __forceinline__ double key_value(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & ~(1ull << 63)) : ~k;
  return __longlong_as_double((long long)b);
}

__global__ void calib_keys_kernel(const double *dist, int32_t k, const float *logr, int64_t n,
                                  unsigned long long *keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double dk = dist[i * k + (k - 1)];
  unsigned long long key = kNoKey;
  if (dk > 0.0 && dk < __builtin_huge_val()) {
    const double r = 0.5 * log(dk) - (double)logr[i];
    if (r - r == 0.0) key = order_key(r);  // finite
  }
  keys[i] = key;
}

// The r-th smallest (0-based) of the keys other than kNoKey; every thread of
// the (single) workgroup calls it.
__device__ unsigned long long select_key(const unsigned long long *keys, int64_t n, long long r,
                                         unsigned *hist, unsigned long long *shared) {
  unsigned long long prefix = 0, mask = 0;
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
    __syncthreads();
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
      const unsigned long long key = keys[i];
      if (key != kNoKey && (key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      long long below = 0;
      int d = 0;
      for (; d < 255; ++d) {
        if (below + (long long)hist[d] > r) break;
        below += hist[d];
      }
      shared[0] = prefix | ((unsigned long long)d << shift);
      shared[1] = (unsigned long long)(r - below);
    }
    __syncthreads();
    prefix = shared[0];
    r = (long long)shared[1];
    mask |= 255ull << shift;
    __syncthreads();
  }
  return prefix;
}

__global__ __launch_bounds__(kSelectThreads) void calib_select_kernel(
    const unsigned long long *keys, int64_t n, double quantile, float *alpha) {
  __shared__ unsigned hist[256];
  __shared__ unsigned long long shared[2];
  __shared__ unsigned long long count;
  if (threadIdx.x == 0) count = 0;
  __syncthreads();
  unsigned long long mine = 0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) mine += keys[i] != kNoKey ? 1 : 0;
  atomicAdd(&count, mine);
  __syncthreads();
  const long long m = (long long)count;
  if (m == 0) {
    if (threadIdx.x == 0) *alpha = 1.0f;
    return;
  }
  const double h = (double)(m - 1) * quantile;
  const long long lo = (long long)floor(h);
  const double frac = h - (double)lo;
  const double x_lo = key_value(select_key(keys, n, lo, hist, shared));
  const double x_hi = lo + 1 < m ? key_value(select_key(keys, n, lo + 1, hist, shared)) : x_lo;
  if (threadIdx.x == 0) *alpha = (float)exp(x_lo + frac * (x_hi - x_lo));
}

size_t calib_scratch(int64_t n) {
  return align_up((size_t)n * 8) + 2 * align_up((size_t)n * 4) + 256;
}

size_t train_scratch(int64_t batch) {
  const int64_t nblk = (batch + kTrainBlock - 1) / kTrainBlock;
  return align_up((size_t)nblk * (NP + 3) * sizeof(float)) + align_up(NP * sizeof(float)) + 256;
}

const IndexDesc *desc_of(const tnn_index *index) {
  if (!index) return nullptr;
  const IndexDesc *d = reinterpret_cast<const IndexDesc *>(index);
  return d->magic == kIndexMagic ? d : nullptr;
}

bool pts_ok(const tnn_points &p) {
  return p.n >= 0 && (p.n == 0 || (p.x && p.y && p.z && p.t));
}

tnn_status launch_grad(const void *d_model, tnn_points smp, const double *d_dist,
                       const int32_t *d_order, int32_t k, int64_t first, int64_t batch,
                       float *grad, float *loss, void *scratch, size_t bytes, hipStream_t st) {
  if (!d_model || !pts_ok(smp) || !d_dist || k < 1 || k > kMaxK || first < 0 || batch < 1 ||
      first + batch > smp.n || !grad)
    return TNN_E_ARG;
  if (!scratch || bytes < train_scratch(batch)) return TNN_E_WORKSPACE;
  const int nblk = (int)((batch + kTrainBlock - 1) / kTrainBlock);
  float *partial = static_cast<float *>(scratch);
  hipLaunchKernelGGL(fwd_bwd_kernel, dim3(nblk), dim3(64 * kTrainWaves), 0, st,
                     static_cast<const tnn_radius_model *>(d_model), smp, d_dist, d_order, k,
                     first, batch, partial);
  TNN_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(reduce_kernel, dim3((NP + 255) / 256), dim3(256), 0, st, partial, nblk, grad,
                     loss);
  TNN_HIP_CHECK(hipGetLastError());
  return TNN_OK;
}

}  // namespace
}  // namespace tnn

using namespace tnn;

extern "C" {

tnn_status tnn_radius_model_bytes(size_t *bytes) {
  if (!bytes) return TNN_E_ARG;
  *bytes = sizeof(tnn_radius_model);
  return TNN_OK;
}

tnn_status tnn_radius_model_init(const tnn_index *index, void *d_model, uint64_t seed,
                                 void *stream) {
  const IndexDesc *d = desc_of(index);
  if (!d || !d_model) return TNN_E_ARG;
  hipStream_t st = static_cast<hipStream_t>(stream);
  tnn_radius_model *m = static_cast<tnn_radius_model *>(d_model);
  const int n = G * G * G > NP ? G * G * G : NP;
  hipLaunchKernelGGL(init_kernel, dim3((n + 255) / 256), dim3(256), 0, st, m, seed, *d);
  TNN_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(starts_zero_kernel, dim3(2048), dim3(256), 0, st, m);
  TNN_HIP_CHECK(hipGetLastError());
  if (d->n_seg > 0) {
    hipLaunchKernelGGL(grid_kernel, dim3((unsigned)((d->n_seg + 255) / 256)), dim3(256), 0, st, m,
                       *d);
    TNN_HIP_CHECK(hipGetLastError());
  }
  return TNN_OK;
}

tnn_status tnn_radius_train_workspace(int64_t batch, size_t *bytes) {
  if (!bytes || batch < 1) return TNN_E_ARG;
  *bytes = train_scratch(batch);
  return TNN_OK;
}

tnn_status tnn_radius_grad(const void *d_model, tnn_points samples, const double *d_dist,
                           const int32_t *d_order, int32_t k, int64_t first, int64_t batch,
                           float *d_grad, float *d_loss, void *d_scratch, size_t scratch_bytes,
                           void *stream) {
  return launch_grad(d_model, samples, d_dist, d_order, k, first, batch, d_grad, d_loss,
                     d_scratch, scratch_bytes, static_cast<hipStream_t>(stream));
}

tnn_status tnn_radius_train_step(void *d_model, float *d_adam, tnn_points samples,
                                 const double *d_dist, const int32_t *d_order, int32_t k,
                                 int64_t first, int64_t batch, int32_t step, float lr,
                                 float *d_loss, void *d_scratch, size_t scratch_bytes,
                                 void *stream) {
  if (!d_adam || step < 1 || !(lr > 0.0f) || !std::isfinite(lr)) return TNN_E_ARG;
  if (!d_scratch || scratch_bytes < train_scratch(batch > 0 ? batch : 1)) return TNN_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t nblk = (batch + kTrainBlock - 1) / kTrainBlock;
  float *grad = reinterpret_cast<float *>(static_cast<char *>(d_scratch) +
                                          align_up((size_t)nblk * (NP + 3) * sizeof(float)));
  const tnn_status s = launch_grad(d_model, samples, d_dist, d_order, k, first, batch, grad,
                                   d_loss, d_scratch, scratch_bytes, st);
  if (s != TNN_OK) return s;
  hipLaunchKernelGGL(adam_kernel, dim3((NP + 255) / 256), dim3(256), 0, st,
                     static_cast<tnn_radius_model *>(d_model)->params, d_adam, grad, step, lr);
  TNN_HIP_CHECK(hipGetLastError());
  return TNN_OK;
}

tnn_status tnn_radius_features(const void *d_model, tnn_points queries, float *d_feat,
                               void *stream) {
  if (!d_model || !pts_ok(queries) || (queries.n > 0 && !d_feat)) return TNN_E_ARG;
  if (queries.n == 0) return TNN_OK;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)((queries.n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream),
                     static_cast<const tnn_radius_model *>(d_model), queries, d_feat);
  TNN_HIP_CHECK(hipGetLastError());
  return TNN_OK;
}

tnn_status tnn_radius_infer(const void *d_model, tnn_points queries, float alpha,
                            float *d_radius2, float *d_logr, void *stream) {
  if (!d_model || !pts_ok(queries) || (queries.n > 0 && !d_radius2) || !(alpha > 0.0f) ||
      !std::isfinite(alpha))
    return TNN_E_ARG;
  if (queries.n == 0) return TNN_OK;
  const int64_t groups = (queries.n + kInferTile * kInferWaves - 1) / (kInferTile * kInferWaves);
  const int64_t grid = groups < 1024 ? groups : 1024;
  hipLaunchKernelGGL(infer_kernel, dim3((unsigned)grid), dim3(64 * kInferWaves), 0,
                     static_cast<hipStream_t>(stream),
                     static_cast<const tnn_radius_model *>(d_model), queries, alpha, d_radius2,
                     d_logr);
  TNN_HIP_CHECK(hipGetLastError());
  return TNN_OK;
}

static host::CkptDims ckpt_dims() {
  return host::CkptDims{(uint32_t)H, (uint32_t)NI, (uint32_t)G, (uint32_t)SXY, (uint32_t)ST,
                        (uint32_t)NP};
}

tnn_status tnn_radius_checkpoint_bytes(size_t *bytes) {
  if (!bytes) return TNN_E_ARG;
  *bytes = host::kCkptHeaderBytes + sizeof(tnn_radius_model);
  return TNN_OK;
}

tnn_status tnn_radius_model_save(const void *d_model, void *h_buf, size_t bytes, void *stream) {
  if (!d_model || !h_buf) return TNN_E_ARG;
  const size_t mb = sizeof(tnn_radius_model);
  if (bytes < host::kCkptHeaderBytes + mb) return TNN_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char *b = static_cast<char *>(h_buf);
  TNN_HIP_CHECK(hipMemcpyAsync(b + host::kCkptHeaderBytes, d_model, mb, hipMemcpyDeviceToHost, st));
  TNN_HIP_CHECK(hipStreamSynchronize(st));
  host::ckpt_write_header(b, mb, ckpt_dims(), host::fnv1a64(b + host::kCkptHeaderBytes, mb));
  return TNN_OK;
}

tnn_status tnn_radius_model_load(const void *h_buf, size_t bytes, void *d_model, void *stream) {
  if (!d_model || !h_buf) return TNN_E_ARG;
  const size_t mb = sizeof(tnn_radius_model);
  if (host::ckpt_check(h_buf, bytes, mb, ckpt_dims()) != 0) return TNN_E_FORMAT;
  hipStream_t st = static_cast<hipStream_t>(stream);
  TNN_HIP_CHECK(hipMemcpyAsync(d_model, static_cast<const char *>(h_buf) + host::kCkptHeaderBytes,
                               mb, hipMemcpyHostToDevice, st));
  TNN_HIP_CHECK(hipStreamSynchronize(st));
  return TNN_OK;
}

tnn_status tnn_radius_shuffle(int64_t n, uint64_t seed, int32_t *d_order, void *stream) {
  if (n < 0 || n > INT32_MAX || (n > 0 && !d_order)) return TNN_E_ARG;
  if (n == 0) return TNN_OK;
  int h = 1;
  while ((1ull << (2 * h)) < (uint64_t)n) ++h;
  hipLaunchKernelGGL(shuffle_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0,
                     static_cast<hipStream_t>(stream), n, h, seed, d_order);
  TNN_HIP_CHECK(hipGetLastError());
  return TNN_OK;
}

tnn_status tnn_radius_calibrate_workspace(int64_t n_samples, size_t *bytes) {
  if (!bytes || n_samples < 0) return TNN_E_ARG;
  *bytes = calib_scratch(n_samples);
  return TNN_OK;
}

tnn_status tnn_radius_calibrate(const void *d_model, tnn_points samples, const double *d_dist,
                                int32_t k, double quantile, float *d_alpha, void *d_scratch,
                                size_t scratch_bytes, void *stream) {
  if (!d_model || !pts_ok(samples) || (samples.n > 0 && !d_dist) || k < 1 || k > kMaxK ||
      !d_alpha || !(quantile >= 0.0 && quantile <= 1.0))
    return TNN_E_ARG;
  const int64_t n = samples.n;
  if (!d_scratch || scratch_bytes < calib_scratch(n)) return TNN_E_WORKSPACE;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char *b = static_cast<char *>(d_scratch);
  unsigned long long *keys = reinterpret_cast<unsigned long long *>(b);
  float *logr = reinterpret_cast<float *>(b + align_up((size_t)n * 8));
  float *r2 = reinterpret_cast<float *>(b + align_up((size_t)n * 8) + align_up((size_t)n * 4));
  if (n > 0) {
    const tnn_status s = tnn_radius_infer(d_model, samples, 1.0f, r2, logr, stream);
    if (s != TNN_OK) return s;
    hipLaunchKernelGGL(calib_keys_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       d_dist, k, logr, n, keys);
    TNN_HIP_CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(calib_select_kernel, dim3(1), dim3(kSelectThreads), 0, st, keys, n, quantile,
                     d_alpha);
  TNN_HIP_CHECK(hipGetLastError());
  return TNN_OK;
}

}  // extern "C"
