// The learned root (gfx950): a monotone MLP CDF trained on the sample by this
// file's own forward and backward kernels, used as the root of the RMI; and
// the equi-depth leaves that the MLP and the linear-spline roots share.
//
// The paper's CDF model is an RMI of linear models fitted to a sample of the
// keys (Section 3.1).  Here the root may instead be a small monotone network
// fitted to the same target, the sample's empirical CDF rank/S:
//   phi_k = min(1, max(code - q_k, 0) / w_k)   k = 0..7, quantile knots q_k
//   h1 = sigmoid(W1 phi + b1)    8 -> 64, FP32 (vector ALUs in training, FP32 matrix cores in evaluation)
//   h2 = sigmoid(W2 h1 + b2)     64 -> 64, bfloat16 matrix cores, FP32 accumulate
//   y  = w3 . h2 + b3            64 -> 1
// with W1, W2, w3 >= 0, so y is non-decreasing in the key.  The leaves are
// equi-depth in the sorted sample: leaf j starts at the first sample of the
// run of equal codes that holds sample floor(j S / L), and that sample's code
// is a routing boundary.  A record's leaf is the number of boundaries at or
// below its code.  The network narrows the search: a cell table over its
// output (cell floor(L y)) gives the bracket of leaves a record of that cell
// can fall in, and the router checks the bracket before searching it, so the
// leaf is exact whatever the rounding inside the matrix cores.  Each leaf's
// linear model is the same two-point spline as under the linear root.  The
// linear-spline root routes among the same boundaries through its segment
// knots instead.
#include "mlp_device.h"

namespace elsar {

// ------------------------------------------------------------------ state --
namespace {
constexpr size_t kA = 256;
inline size_t al(size_t x) { return (x + kA - 1) & ~(kA - 1); }
}  // namespace

size_t mlp_state_bytes(uint32_t L, uint32_t B) {
  return al(sizeof(MlpBlock)) + al((size_t)L * sizeof(Leaf)) + al(((size_t)L + 1) * 8) + al(((size_t)L + 1) * 4) +
         2 * al((size_t)B * 4) + al(((size_t)spline_segments(L) + 1) * 8) + al(cell_table_words(L) * 4) +
         al(((size_t)L + 1) * 4) +
         al((size_t)kMlpParams * 4) + al((size_t)kMlpParams * 8);
}

void place_mlp_state(MlpState* s, void* base, uint32_t L, uint32_t B) {
  uint8_t* b = static_cast<uint8_t*>(base);
  s->M = reinterpret_cast<MlpBlock*>(b);
  b += al(sizeof(MlpBlock));
  s->leaves = reinterpret_cast<Leaf*>(b);
  b += al((size_t)L * sizeof(Leaf));
  s->bound = reinterpret_cast<uint64_t*>(b);
  b += al(((size_t)L + 1) * 8);
  s->first = reinterpret_cast<uint32_t*>(b);
  b += al(((size_t)L + 1) * 4);
  s->hist = reinterpret_cast<uint32_t*>(b);
  b += al((size_t)B * 4);
  s->hist_net = reinterpret_cast<uint32_t*>(b);
  b += al((size_t)B * 4);
  s->knots = reinterpret_cast<uint64_t*>(b);
  b += al(((size_t)spline_segments(L) + 1) * 8);
  s->ccells = reinterpret_cast<uint32_t*>(b);
  b += al(cell_table_words(L) * 4);
  s->cells = reinterpret_cast<uint32_t*>(b);
  b += al(((size_t)L + 1) * 4);
  s->master = reinterpret_cast<float*>(b);
  b += al((size_t)kMlpParams * 4);
  s->adam = reinterpret_cast<float*>(b);
}

// ------------------------------------------------------------------ setup --
__device__ __forceinline__ float philox_unit(uint64_t i, uint32_t stream, uint64_t seed) {
  return (float)(philox_x(i, stream, 0u, seed) >> 8) * (1.0f / 16777216.0f);
}

__device__ void set_knots(const uint64_t* q9, MlpHead* h) {
  if (threadIdx.x < 9) h->q[threadIdx.x] = q9[threadIdx.x];
  if (threadIdx.x < 8) {
    const uint64_t a = q9[threadIdx.x], b = q9[threadIdx.x + 1];
    h->inv_w[threadIdx.x] = (float)(1.0 / (b > a ? (double)(b - a) : 1.0));
  }
}

// Knots q_k = e[k S / 8] (k < 8), q_8 = e[S-1]; initial weights from Philox
// draws u: W1 = u, b1 = -4u, W2 = 0.1u, b2 = -3, w3 = 0.05u, b3 = 0 (small
// positive weights, hidden units off saturation); Adam moments zero.
__global__ void mlp_setup_kernel(const uint64_t* __restrict__ e, uint64_t S, uint64_t seed,
                                 MlpBlock* __restrict__ M, float* __restrict__ master, float* __restrict__ adam) {
  __shared__ uint64_t q9[9];
  if (threadIdx.x < 9) q9[threadIdx.x] = e[threadIdx.x < 8 ? (threadIdx.x * S) / 8 : S - 1];
  __syncthreads();
  set_knots(q9, &M->h);
  for (uint32_t p = threadIdx.x; p < kMlpParams; p += blockDim.x) {
    const float u = philox_unit(p, 0x4D4C5049u /* "MLPI" */, seed);
    float v;
    if (p < kOffB1) v = u;
    else if (p < kOffW2) v = -4.0f * u;
    else if (p < kOffB2) v = 0.1f * u;
    else if (p < kOffW3) v = -3.0f;
    else if (p < kOffB3) v = 0.05f * u;
    else v = 0.0f;
    master[p] = v;
    adam[p] = 0.0f;
    adam[kMlpParams + p] = 0.0f;
  }
}

// Evaluation copy of one FP32 parameter (W2 in bfloat16, both orientations).
__device__ __forceinline__ void publish_one(uint32_t p, float v, MlpBlock* __restrict__ M) {
  if (p < kOffB1) M->h.W1[p] = v;
  else if (p < kOffW2) M->h.b1[p - kOffB1] = v;
  else if (p < kOffB2) {
    const uint32_t j = (p - kOffW2) / 64, u = (p - kOffW2) % 64;
    const uint16_t b = f32_to_bf16(v);
    M->W2bf[j * kW2S + u] = b;
    M->W2bfT[u * kW2S + j] = b;
  } else if (p < kOffW3) M->h.b2[p - kOffB2] = v;
  else if (p < kOffB3) M->h.w3[p - kOffW3] = v;
  else M->h.b3 = v;
}

__device__ void publish(const float* __restrict__ master, MlpBlock* __restrict__ M) {
  for (uint32_t p = threadIdx.x; p < kMlpParams; p += blockDim.x) publish_one(p, master[p], M);
}

__global__ void mlp_publish_kernel(const float* __restrict__ master, const uint64_t* __restrict__ q9,
                                   MlpBlock* __restrict__ M) {
  if (q9) set_knots(q9, &M->h);
  publish(master, M);
}

// --------------------------------------------------------------- training --
// One step on kMlpGradRows rows: forward, MSE gradient with targets t, backward
// into G (flat parameter order).  Block of 512 threads; wave w owns rows
// 16w .. 16w + 15 (one 16-row chunk), and output tiles w, w + 8 of dW2.  The
// 64x64 products (forward, dW2 and dh1) run on the matrix cores in bfloat16
// with FP32 accumulation; everything else is FP32.
constexpr uint32_t kTrainThreads = 512;
constexpr uint32_t kWaves = kTrainThreads / 64;
constexpr uint32_t kRows = kMlpGradRows;
constexpr uint32_t kChunks = kRows / (16 * kWaves);  // 16-row chunks per wave
static_assert(kChunks >= 1 && kRows == 16 * kChunks * kWaves, "whole chunks per wave");

// Row strides of the training arrays, padded so that the 16 lanes of a
// matrix-core fragment, which read 16 consecutive rows, fall in different
// LDS banks (unpadded, H1T and DZ2T rows are 512 and 256 bytes apart and the
// 16 reads of a fragment hit one bank).
constexpr uint32_t kH1S = kRows + 4;  // floats per H1T row
constexpr uint32_t kDzS = 64 + 4;     // bf16 per DZ2 row
constexpr uint32_t kDzTS = kRows + 4; // bf16 per DZ2T row

struct TrainLds {
  MlpBlock M;
  float H1T[64 * kH1S];        // h1 (FP32), [unit][row]
  uint16_t DZ2[kRows * kDzS];  // dL/dz2 (bf16), [row][j]
  uint16_t DZ2T[64 * kDzTS];   // dL/dz2 (bf16), [j][row]
  float PHI[kRows * 8];
  float T[kRows], DY[kRows];
  float PW1[kWaves][9 * 64];   // each wave's dW1 ([k][u], k < 8) and db1 (k = 8) over its rows
  float G[kMlpParams];
  float loss;
};

__device__ void step_grad(TrainLds& sm) {
  const uint32_t tid = threadIdx.x, w = tid >> 6, l = __lane_id(), r = l & 15u, g = l >> 4;
  const MlpHead& M = sm.M.h;
  float h2[kChunks][4][4];  // [chunk][ct][e]: row 16 kChunks w + 16c + 4g + e, column 16ct + r
  // forward
#pragma unroll
  for (uint32_t c = 0; c < kChunks; ++c) {
    const uint32_t r0 = 16 * kChunks * w + 16 * c;
    float phi[8], h1[16];
    s16x4 a[4];
#pragma unroll
    for (int k = 0; k < 8; ++k) phi[k] = sm.PHI[(r0 + r) * 8 + k];
    mlp_layer1_frags(phi, M, g, a, h1);
#pragma unroll
    for (uint32_t ks = 0; ks < 4; ++ks)
#pragma unroll
      for (uint32_t e = 0; e < 4; ++e) sm.H1T[(16 * ks + 4 * g + e) * kH1S + r0 + r] = h1[4 * ks + e];
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (uint32_t ct = 0; ct < 4; ++ct) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (uint32_t s2 = 0; s2 < 2; ++s2) {  // K-steps 2s2 and 2s2+1 as one 16x16x32 product
        const uint16_t* wr = sm.M.W2bf + (16 * ct + r) * kW2S + 32 * s2 + 4 * g;
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cat8_bf16(a[2 * s2], a[2 * s2 + 1]),
                                                      cat8_bf16(load4_bf16(wr), load4_bf16(wr + 16)), acc, 0, 0, 0);
      }
      const uint32_t col = 16 * ct + r;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float v = sigm(acc[e] + M.b2[col]);
        h2[c][ct][e] = v;
        part[e] = __builtin_fmaf(M.w3[col], v, part[e]);
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) part[e] += __shfl_xor(part[e], off);
      if (r == 0) {
        const uint32_t row = r0 + 4 * g + e;
        const float res = part[e] + M.b3 - sm.T[row];
        sm.DY[row] = 2.0f * res / (float)kRows;
        atomicAdd(&sm.loss, res * res / (float)kRows);
      }
    }
  }
  __syncthreads();
  // output layer: dw3, db2, db3 and dz2 = dy w3 h2 (1 - h2)
  {
    float gb3 = tid < kRows ? sm.DY[tid] : 0.0f;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) gb3 += __shfl_xor(gb3, off);
    if (l == 0 && tid < kRows) atomicAdd(&sm.G[kOffB3], gb3);
#pragma unroll
    for (uint32_t ct = 0; ct < 4; ++ct) {
      const uint32_t col = 16 * ct + r;
      float gw3 = 0.f, gb2 = 0.f;
#pragma unroll
      for (uint32_t c = 0; c < kChunks; ++c)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint32_t row = 16 * kChunks * w + 16 * c + 4 * g + e;
          const float dy = sm.DY[row], v = h2[c][ct][e];
          const float dz2 = dy * M.w3[col] * v * (1.0f - v);
          gw3 = __builtin_fmaf(dy, v, gw3);
          gb2 += dz2;
          const uint16_t hz = f32_to_bf16(dz2);
          sm.DZ2[row * kDzS + col] = hz;
          sm.DZ2T[col * kDzTS + row] = hz;
        }
      gw3 += __shfl_xor(gw3, 16);
      gw3 += __shfl_xor(gw3, 32);
      gb2 += __shfl_xor(gb2, 16);
      gb2 += __shfl_xor(gb2, 32);
      if (g == 0) {
        atomicAdd(&sm.G[kOffW3 + col], gw3);
        atomicAdd(&sm.G[kOffB2 + col], gb2);
      }
    }
  }
  __syncthreads();
  // dW2[j][u] = sum_t dz2[t][j] h1q[t][u]: 16 output tiles (jt, ct), wave w
  // takes tiles w, w + kWaves, ...
  for (uint32_t tile = w; tile < 16; tile += kWaves) {
    const uint32_t jt = tile & 3u, ct = tile >> 2;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (uint32_t s2 = 0; s2 < kRows / 32; ++s2) {  // rows 32s2 + 4g + e and 32s2 + 16 + 4g + e
      const uint16_t* dz = sm.DZ2T + (16 * jt + r) * kDzTS + 32 * s2 + 4 * g;
      const float* h = sm.H1T + (16 * ct + r) * kH1S + 32 * s2 + 4 * g;
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cat8_bf16(load4_bf16(dz), load4_bf16(dz + 16)),
                                                    cat8_bf16(pack4_bf16(h[0], h[1], h[2], h[3]),
                                                              pack4_bf16(h[16], h[17], h[18], h[19])),
                                                    acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) sm.G[kOffW2 + (16 * jt + 4 * g + e) * 64 + 16 * ct + r] = acc[e];
  }
  // dh1[t][u] = sum_j dz2[t][j] W2q[j][u]; dz1 = dh1 h1 (1 - h1); dW1 = dz1^T phi, db1
#pragma unroll
  for (uint32_t c = 0; c < kChunks; ++c) {
    const uint32_t r0 = 16 * kChunks * w + 16 * c;
#pragma unroll
    for (uint32_t ct = 0; ct < 4; ++ct) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (uint32_t s2 = 0; s2 < 2; ++s2) {
        const uint16_t* dz = sm.DZ2 + (r0 + r) * kDzS + 32 * s2 + 4 * g;
        const uint16_t* wt = sm.M.W2bfT + (16 * ct + r) * kW2S + 32 * s2 + 4 * g;
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cat8_bf16(load4_bf16(dz), load4_bf16(dz + 16)),
                                                      cat8_bf16(load4_bf16(wt), load4_bf16(wt + 16)), acc, 0, 0, 0);
      }
      const uint32_t u = 16 * ct + r;
      float gw[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f}, gb = 0.f;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t row = r0 + 4 * g + e;
        const float h = sm.H1T[u * kH1S + row];
        const float dz1 = acc[e] * h * (1.0f - h);
        gb += dz1;
#pragma unroll
        for (int k = 0; k < 8; ++k) gw[k] = __builtin_fmaf(dz1, sm.PHI[row * 8 + k], gw[k]);
      }
      gb += __shfl_xor(gb, 16);
      gb += __shfl_xor(gb, 32);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        gw[k] += __shfl_xor(gw[k], 16);
        gw[k] += __shfl_xor(gw[k], 32);
      }
      if (g == 0) {  // this wave's share, summed over the waves below (no contended LDS atomics)
        sm.PW1[w][8 * 64 + u] = gb;
#pragma unroll
        for (int k = 0; k < 8; ++k) sm.PW1[w][k * 64 + u] = gw[k];
      }
    }
  }
  static_assert(kChunks == 1, "one chunk per wave: each wave writes its partials once");
  __syncthreads();
  for (uint32_t t = tid; t < 9 * 64; t += kTrainThreads) {
    float v = 0.f;
#pragma unroll
    for (uint32_t ww = 0; ww < kWaves; ++ww) v += sm.PW1[ww][t];
    const uint32_t k = t / 64, u = t % 64;
    sm.G[k < 8 ? kOffW1 + u * 8 + k : kOffB1 + u] = v;
  }
  __syncthreads();
}

__device__ void load_block(const MlpBlock* __restrict__ src, MlpBlock& dst) {
  const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
  uint32_t* d = reinterpret_cast<uint32_t*>(&dst);
  for (uint32_t i = threadIdx.x; i < sizeof(MlpBlock) / 4; i += blockDim.x) d[i] = s[i];
}

__device__ void clear_grad(TrainLds& sm) {
  for (uint32_t p = threadIdx.x; p < kMlpParams; p += blockDim.x) sm.G[p] = 0.0f;
  if (threadIdx.x == 0) sm.loss = 0.0f;
}

// All training steps in one block: per step kRows sample positions drawn with
// Philox, the gradient, then Adam (beta1 0.9, beta2 0.999, eps 1e-8) with
// W1, W2, w3 projected onto >= 0, and a fresh evaluation copy.  Thread t owns
// parameters t, t + kTrainThreads, ...: their FP32 values and Adam moments stay in its
// registers for the whole fit.
constexpr uint32_t kOwn = (kMlpParams + kTrainThreads - 1) / kTrainThreads;

__device__ __forceinline__ bool mlp_nonneg(uint32_t p) {  // W1, W2 and w3 stay >= 0
  return p < kOffB1 || (p >= kOffW2 && p < kOffB2) || (p >= kOffW3 && p < kOffB3);
}

// Adam on parameter p with gradient gr: moments m1 <- 0.9 m1 + 0.1 gr and
// m2 <- 0.999 m2 + 0.001 gr^2, then v - lr (m1 c1) / (sqrt(m2 c2) + 1e-8)
// with the bias corrections c1 = 1 / (1 - 0.9^t), c2 = 1 / (1 - 0.999^t),
// projected onto >= 0 for the weights.
__device__ __forceinline__ float adam_update(uint32_t p, float v, float gr, float& m1, float& m2, float c1, float c2,
                                             float lr) {
  m1 = 0.9f * m1 + 0.1f * gr;
  m2 = 0.999f * m2 + 0.001f * gr * gr;
  float r = v - lr * (m1 * c1) / (sqrtf(m2 * c2) + 1e-8f);
  if (mlp_nonneg(p)) r = fmaxf(r, 0.0f);
  return r;
}

__global__ __launch_bounds__(kTrainThreads) void mlp_train_kernel(const uint64_t* __restrict__ e, uint64_t S,
                                                                  uint32_t steps, float lr, uint64_t seed,
                                                                  float* __restrict__ master,
                                                                  float* __restrict__ adam,
                                                                  MlpBlock* __restrict__ Mout) {
  extern __shared__ uint4 lds_raw[];
  TrainLds& sm = *reinterpret_cast<TrainLds*>(lds_raw);
  const uint32_t tid = threadIdx.x;
  load_block(Mout, sm.M);
  float pv[kOwn], a1[kOwn], a2[kOwn];
#pragma unroll
  for (uint32_t k = 0; k < kOwn; ++k) {
    const uint32_t p = tid + k * kTrainThreads;
    const bool ok = p < kMlpParams;
    pv[k] = ok ? master[p] : 0.0f;
    a1[k] = ok ? adam[p] : 0.0f;
    a2[k] = ok ? adam[kMlpParams + p] : 0.0f;
  }
  float p1 = 1.0f, p2 = 1.0f;  // beta^step
  // row tid of each step: the sample position and its code, fetched one step
  // ahead so that the load's latency overlaps the previous step
  auto pick = [&](uint32_t step) {
    const uint64_t ctr = (uint64_t)step * kRows + tid;
    return ((uint64_t)philox_x(ctr, 0x4D4C5042u /* "MLPB" */, 0u, seed) * S) >> 32;
  };
  uint64_t s_cur = tid < kRows ? pick(1) : 0, code_cur = tid < kRows ? e[s_cur] : 0;
  __syncthreads();
  for (uint32_t step = 1; step <= steps; ++step) {
    clear_grad(sm);
    uint64_t s_next = 0, code_next = 0;
    if (tid < kRows) {
      sm.T[tid] = (float)((double)s_cur / (double)S);
      float phi[8];
      mlp_features(code_cur, sm.M.h, phi);
#pragma unroll
      for (int k = 0; k < 8; ++k) sm.PHI[tid * 8 + k] = phi[k];
      if (step < steps) {
        s_next = pick(step + 1);
        code_next = e[s_next];
      }
    }
    __syncthreads();
    step_grad(sm);
    p1 *= 0.9f;
    p2 *= 0.999f;
    const float c1 = 1.0f / (1.0f - p1), c2 = 1.0f / (1.0f - p2);
#pragma unroll
    for (uint32_t k = 0; k < kOwn; ++k) {
      const uint32_t p = tid + k * kTrainThreads;
      if (p < kMlpParams) {
        pv[k] = adam_update(p, pv[k], sm.G[p], a1[k], a2[k], c1, c2, lr);
        publish_one(p, pv[k], &sm.M);
      }
    }
    __syncthreads();
    s_cur = s_next;
    code_cur = code_next;
  }
#pragma unroll
  for (uint32_t k = 0; k < kOwn; ++k) {
    const uint32_t p = tid + k * kTrainThreads;
    if (p < kMlpParams) {
      master[p] = pv[k];
      adam[p] = a1[k];
      adam[kMlpParams + p] = a2[k];
    }
  }
  // the knots were in the copy loaded at the start; write everything back
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&sm.M);
  uint32_t* d = reinterpret_cast<uint32_t*>(Mout);
  for (uint32_t i = tid; i < sizeof(MlpBlock) / 4; i += kTrainThreads) d[i] = src[i];
}

// One gradient on caller-supplied rows (codes and targets), for verification.
__global__ __launch_bounds__(kTrainThreads) void mlp_grad_kernel(const MlpBlock* __restrict__ Mg,
                                                                 const uint64_t* __restrict__ codes,
                                                                 const float* __restrict__ targets,
                                                                 float* __restrict__ grad, float* __restrict__ loss) {
  extern __shared__ uint4 lds_raw[];
  TrainLds& sm = *reinterpret_cast<TrainLds*>(lds_raw);
  const uint32_t tid = threadIdx.x;
  load_block(Mg, sm.M);
  clear_grad(sm);
  __syncthreads();
  if (tid < kRows) {
    sm.T[tid] = targets[tid];
    float phi[8];
    mlp_features(codes[tid], sm.M.h, phi);
#pragma unroll
    for (int k = 0; k < 8; ++k) sm.PHI[tid * 8 + k] = phi[k];
  }
  __syncthreads();
  step_grad(sm);
  for (uint32_t p = tid; p < kMlpParams; p += kTrainThreads) grad[p] = sm.G[p];
  if (tid == 0) *loss = sm.loss;
}

// One training step on caller-supplied rows, for verification: the gradient
// of mlp_grad_kernel, then the training kernel's Adam update at step `step`
// (the bias corrections from beta^step accumulated the way training does)
// applied to params and adam (moments m then v) in place.
__global__ __launch_bounds__(kTrainThreads) void mlp_step_kernel(const MlpBlock* __restrict__ Mg,
                                                                 float* __restrict__ params, float* __restrict__ adam,
                                                                 const uint64_t* __restrict__ codes,
                                                                 const float* __restrict__ targets, uint32_t step,
                                                                 float lr, float* __restrict__ grad,
                                                                 float* __restrict__ loss) {
  extern __shared__ uint4 lds_raw[];
  TrainLds& sm = *reinterpret_cast<TrainLds*>(lds_raw);
  const uint32_t tid = threadIdx.x;
  load_block(Mg, sm.M);
  clear_grad(sm);
  __syncthreads();
  if (tid < kRows) {
    sm.T[tid] = targets[tid];
    float phi[8];
    mlp_features(codes[tid], sm.M.h, phi);
#pragma unroll
    for (int k = 0; k < 8; ++k) sm.PHI[tid * 8 + k] = phi[k];
  }
  __syncthreads();
  step_grad(sm);
  float p1 = 1.0f, p2 = 1.0f;
  for (uint32_t t = 0; t < step; ++t) {
    p1 *= 0.9f;
    p2 *= 0.999f;
  }
  const float c1 = 1.0f / (1.0f - p1), c2 = 1.0f / (1.0f - p2);
  for (uint32_t p = tid; p < kMlpParams; p += kTrainThreads) {
    float m1 = adam[p], m2 = adam[kMlpParams + p];
    params[p] = adam_update(p, params[p], sm.G[p], m1, m2, c1, c2, lr);
    adam[p] = m1;
    adam[kMlpParams + p] = m2;
    grad[p] = sm.G[p];
  }
  if (tid == 0) *loss = sm.loss;
}

// ------------------------------------------------------- leaves and bounds --
__device__ __forceinline__ void load_head(const MlpBlock* __restrict__ Mg, MlpHead& mh) {
  for (uint32_t i = threadIdx.x; i < sizeof(MlpHead) / 4; i += blockDim.x)
    reinterpret_cast<uint32_t*>(&mh)[i] = reinterpret_cast<const uint32_t*>(&Mg->h)[i];
}

// y of n codes (64 per wave; the tail wave clamps its reads).
__global__ __launch_bounds__(256) void mlp_eval_kernel(const MlpBlock* __restrict__ Mg,
                                                       const uint64_t* __restrict__ codes, uint64_t n,
                                                       float* __restrict__ y) {
  __shared__ MlpHead mh;
  load_head(Mg, mh);
  MlpFrags w;
  mlp_load_frags(Mg, w);
  __syncthreads();
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const float v = mlp_y64(codes[i < n ? i : n - 1], mh, w);
  if (i < n) y[i] = v;
}

// Equi-depth leaves on the sorted sample: leaf j starts at the first sample
// of the run of equal codes that holds sample floor(j S / L), so a run is
// never split (its records route to one leaf); first[L] = S.  Leaves that a
// long run swallows come out empty (first[j] == first[j+1]).
__global__ __launch_bounds__(256) void quantile_first_kernel(const uint64_t* __restrict__ e, uint64_t S,
                                                             uint32_t L, uint32_t* __restrict__ first,
                                                             ModelHeader* __restrict__ hdr) {
  if (hdr->mlp_skip) return;  // the automatic choice kept the linear root
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > L) return;
  if (j == L) {
    first[L] = (uint32_t)S;
    hdr->mlp_L = L;
    hdr->spline_K = spline_segments(L);
    hdr->max_sample_run = S ? 1u : 0u;  // runs of one; longer ones are added by the sample statistics
    return;
  }
  const uint64_t q = ((uint64_t)j * S) / L;
  const uint64_t c = e[q];
  if (j > 0 && e[((uint64_t)(j - 1) * S) / L] == c) {
    // the previous leaf's start lies in the same run: that leaf takes the
    // run alone, this one starts after it (the first position past c)
    uint64_t lo = q + 1, hi = S;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (e[mid] <= c) lo = mid + 1; else hi = mid;
    }
    first[j] = (uint32_t)lo;
    return;
  }
  uint64_t lo = 0, hi = q;  // the first position holding c; e[hi] == c
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (e[mid] < c) lo = mid + 1; else hi = mid;
  }
  first[j] = (uint32_t)lo;
}

// Leaf j covers samples first[j] .. first[j+1]-1: the same two-point spline
// and bucket range as a leaf of the linear root.  bound[j] = code of the
// leaf's first sample (0 for leaf 0; past every code for leaves after the
// last sample); for a leaf that starts after a run of equal codes v (its
// start sample shares the previous leaf's run), v + 1, so that the run's own
// leaf holds exactly the code v; bound[L] is past every code.
__global__ __launch_bounds__(256) void mlp_leaf_fit_kernel(const uint64_t* __restrict__ e, uint64_t S, uint32_t L,
                                                           uint32_t B, const uint32_t* __restrict__ first,
                                                           Leaf* __restrict__ leaves, uint64_t* __restrict__ bound,
                                                           const ModelHeader* __restrict__ hdr) {
  if (hdr->mlp_skip) return;
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j == 0) bound[L] = ~0ull;
  if (j >= L) return;
  const uint64_t f = first[j], gg = first[j + 1];
  const uint64_t cq = e[((uint64_t)j * S) / L];
  const bool after_run = j > 0 && e[((uint64_t)(j - 1) * S) / L] == cq;
  bound[j] = j == 0 ? 0ull : (after_run ? cq + 1 : (f < S ? e[f] : ~0ull));
  Leaf lf;
  lf.pad[0] = lf.pad[1] = 0;
  if (f >= gg) {
    const uint32_t v = f < S ? (uint32_t)(((uint64_t)B * f) / S) : B - 1;
    lf.base = 0;
    lf.c = 0.0f;
    lf.b = (float)v;
    lf.lo = lf.hi = v;
  } else {
    const double tf = (double)B * (double)f / (double)S;
    const double tl = (double)B * (double)(gg - 1) / (double)S;
    const double span = (double)code_f32(e[gg - 1] - e[f]);
    lf.base = e[f];
    lf.c = (float)(span > 0 ? (tl - tf) / span : 0.0);
    lf.b = (float)tf;
    lf.lo = (uint32_t)(((uint64_t)B * f) / S);
    const uint64_t h = ((uint64_t)B * (gg - 1)) / S;
    lf.hi = (uint32_t)(h < B - 1 ? h : B - 1);
  }
  leaves[j] = lf;
}

// Segment knots of the spline root: knots[i] = bound[(i L) / K], i = 0..K.
__global__ __launch_bounds__(256) void spline_knots_kernel(const uint64_t* __restrict__ bound, uint32_t L,
                                                           uint32_t K, uint64_t* __restrict__ knots,
                                                           const ModelHeader* __restrict__ hdr) {
  if (hdr->mlp_skip) return;
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= K) knots[i] = bound[((uint64_t)i * L) / K];
}

// Code-cell table of the equi-depth leaves (cell_exact_leaf): ccells[c] =
// boundaries bound[1 .. L-1] in cells below c, a binary search over j since
// the cells of the sorted boundaries are non-decreasing in j.
__global__ __launch_bounds__(256) void code_cell_kernel(const uint64_t* __restrict__ bound, uint32_t L,
                                                        uint32_t* __restrict__ ccells, ModelHeader* __restrict__ hdr) {
  if (hdr->mlp_skip) return;
  const uint64_t e0 = L >= 2 ? bound[1] : 0ull, range = L >= 2 ? bound[L - 1] - e0 : 0ull;
  uint32_t shift = 0;
  const uint32_t nc = code_cells_for(L);
  while ((range >> shift) >= nc) ++shift;
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) hdr->cell_shift = shift;
  if (c > nc) return;
  uint32_t lo = 1, hi = L > 0 ? L : 1;  // first j in [1, L) whose cell is >= c (hi if none)
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (code_cell(bound[mid], e0, shift, nc) < c) lo = mid + 1;
    else hi = mid;
  }
  reinterpret_cast<uint2*>(ccells)[c] = make_uint2(lo - 1, 0u);
}

// Info words of the cells and sub-tables of the dense ones (cell_exact_leaf):
// one wave per cell; entry s (one lane each) = the boundaries below the cell +
// those of its sub-cells below s, by a binary search over the cell's
// boundaries.
__global__ __launch_bounds__(256) void code_subcell_kernel(const uint64_t* __restrict__ bound, uint32_t L,
                                                           uint32_t* __restrict__ ccells,
                                                           ModelHeader* __restrict__ hdr) {
  if (hdr->mlp_skip) return;
  const uint32_t nc = code_cells_for(L), shift = hdr->cell_shift;
  const uint32_t c = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, lane = threadIdx.x & 63u;
  if (c >= nc) return;
  uint2* cl = reinterpret_cast<uint2*>(ccells);
  const uint32_t lo = cl[c].x, hi = cl[c + 1].x;  // the cell's boundaries are bound[lo + 1 .. hi]
  uint32_t k = 1;
  while ((1u << k) < hi - lo) ++k;
  ++k;  // at least two sub-cells per boundary
  k = k < shift ? k : shift;
  k = k < 16u ? k : 16u;
  // few boundaries, or cells one code wide (nothing to split): the count
  if (hi - lo <= kCellDense || k == 0) {
    if (lane == 0) cl[c].y = (hi - lo) << 1;
    return;
  }
  const uint64_t e0 = L >= 2 ? bound[1] : 0ull;
  const uint32_t o = 4 * lo + c;
  uint32_t* sub = ccells + 2 * ((size_t)nc + 1) + o;
  for (uint32_t s = lane; s <= (1u << k); s += 64) {
    uint32_t a = lo + 1, b = hi + 1;  // first boundary of the cell in sub-cell s or above (b if none)
    while (a < b) {
      const uint32_t mid = (a + b) >> 1;
      if (code_subcell(bound[mid], e0, shift, c, k) < s) a = mid + 1;
      else b = mid;
    }
    sub[s] = a - 1;
  }
  if (lane == 0) cl[c].y = (((o << 5) | k) << 1) | 1u;
}


// Cell table of the MLP root.  Cell c of the network's output is [c/L,
// (c+1)/L); cells[c] counts the leaves j whose boundary code bound[j] lands in
// a cell below c, found by a binary search over j that evaluates the network
// at each probe (a wave-collective evaluation: every lane takes part in every
// probe, lanes past the table repeat the last entry's search).  With y
// non-decreasing in the code, a record in leaf j* with cell c satisfies
// cells[c] - 1 <= j* < cells[c + 1], so the leaf search starts from that
// bracket; the router checks the bracket against the boundaries and falls back
// to the unbracketed search if rounding ever broke the order.
__global__ __launch_bounds__(256) void mlp_cell_table_kernel(const MlpBlock* __restrict__ Mg,
                                                             const uint64_t* __restrict__ bound, uint32_t L,
                                                             uint32_t* __restrict__ cells,
                                                             const ModelHeader* __restrict__ hdr) {
  if (hdr->kind_used != 1u) return;  // only the MLP root routes through it
  __shared__ MlpHead mh;
  load_head(Mg, mh);
  MlpFrags w;
  mlp_load_frags(Mg, w);
  __syncthreads();
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t c = i < L ? i : L;  // cells[L] = L: no cell reaches L
  uint32_t lo = 0, hi = L;           // first j in [0, L] with cell(j) >= c; j = L counts as true
  uint32_t iters = 0;
  while ((1ull << iters) < (uint64_t)L + 1) ++iters;
  for (uint32_t it = 0; it < iters; ++it) {
    const uint32_t mid = (lo + hi) >> 1;  // < L while lo < hi
    const float y = mlp_y64(bound[mid < L ? mid : L - 1], mh, w);
    if (lo < hi) {
      if (mlp_leaf_guess(y, L) >= c) hi = mid; else lo = mid + 1;
    }
  }
  if (i <= L) cells[i] = lo;
}

// The sample histogram under the equi-depth leaves, and the longest run of
// equal codes (no monotone bucketing can split a run).  With one leaf per
// bucket a leaf's count is its sample range, first[j + 1] - first[j] (thread
// j); otherwise each sample finds its leaf (the last j with first[j] <= s) and
// its bucket there, with one add per run of equal buckets within a wave (the
// sample is sorted).  A run's length is found at its last sample, by a search
// for its first only when the run is longer than one; each wave adds its
// longest once, and only if it is longer than one (atomics on one address
// serialise: one per wave over 10^6 samples took 0.17 ms).
__global__ __launch_bounds__(256) void mlp_sample_stats_kernel(const uint64_t* __restrict__ e, uint64_t S,
                                                               uint32_t L, uint32_t B, const uint32_t* __restrict__ first,
                                                               const Leaf* __restrict__ leaves,
                                                               uint32_t* __restrict__ hist,
                                                               ModelHeader* __restrict__ hdr) {
  if (hdr->mlp_skip) return;
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = s < S;
  const uint64_t c = e[in ? s : S - 1];
  uint32_t run = 0;
  if (in && (s + 1 == S || e[s + 1] != c)) {
    run = 1;
    if (s > 0 && e[s - 1] == c) {
      uint64_t lo = 0, hi = s - 1;  // the first position holding c; e[hi] == c
      while (lo < hi) {
        const uint64_t mid = (lo + hi) >> 1;
        if (e[mid] < c) lo = mid + 1; else hi = mid;
      }
      run = (uint32_t)(s + 1 - lo);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t o = __shfl_xor(run, off);
    run = o > run ? o : run;
  }
  if (__lane_id() == 0 && run > 1) atomicMax(&hdr->max_sample_run, run);  // one address: only longer runs
  if (L == B) {
    if (s < L) hist[s] = first[s + 1] - first[s];
    return;
  }
  uint32_t lo = 0, hi = L;  // last j with first[j] <= s
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (first[mid] <= s) lo = mid; else hi = mid;
  }
  const uint32_t b = leaf_bucket(load_leaf(leaves, lo), c);
  const uint32_t l = __lane_id();
  const uint32_t bl = __shfl_up(b, 1), br = __shfl_down(b, 1);
  const bool start = in && (l == 0 || bl != b);
  const bool last = in && (l == 63 || br != b || s + 1 == S);
  const uint64_t starts = __ballot(start);
  if (last) {
    const uint64_t below = starts & (l == 63 ? ~0ull : ((2ull << l) - 1));  // starts at lanes <= l
    const uint32_t first_lane = 63u - (uint32_t)__clzll((long long)below);
    atomicAdd(&hist[b], l + 1 - first_lane);
  }
}

// The network's own buckets on the sorted sample: b = clamp(floor(B y), 0,
// B-1) of every sample code, counted per bucket (one add per run of equal
// buckets within a wave).  This is the MLP's acceptance statistic: it judges
// the network itself, independently of the equi-depth leaves that route the
// records once the network is accepted.  Every lane takes part in the
// evaluation; lanes past the sample repeat the last code and add nothing.
__global__ __launch_bounds__(256) void mlp_net_hist_kernel(const MlpBlock* __restrict__ Mg,
                                                           const uint64_t* __restrict__ e, uint64_t S, uint32_t B,
                                                           uint32_t* __restrict__ hist_net) {
  __shared__ MlpHead mh;
  load_head(Mg, mh);
  MlpFrags w;
  mlp_load_frags(Mg, w);
  __syncthreads();
  const uint64_t s = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = s < S;
  const float y = mlp_y64(e[in ? s : S - 1], mh, w);
  const uint32_t b = mlp_leaf_guess(y, B);
  const uint32_t l = __lane_id();
  const uint32_t bl = __shfl_up(b, 1), br = __shfl_down(b, 1);
  const bool start = in && (l == 0 || bl != b);
  const bool last = in && (l == 63 || br != b || s + 1 == S);
  const uint64_t starts = __ballot(start);
  if (last) {
    const uint64_t below = starts & (l == 63 ? ~0ull : ((2ull << l) - 1));  // starts at lanes <= l
    const uint32_t first_lane = 63u - (uint32_t)__clzll((long long)below);
    atomicAdd(&hist_net[b], l + 1 - first_lane);
  }
}

// Gate of the linear root, for every kind with equi-depth leaves: the linear
// root passes when its largest sample bucket is within accept_ratio of what a
// perfect model shows on S sample keys, lambda + sqrt(2 ln(B) lambda) + 1 with
// lambda = S/B (about the largest of B Poisson(lambda) counts).  Under the
// automatic choice a passing linear root is kept and the equi-depth leaves are
// not fitted (mlp_skip).  One block.
constexpr uint32_t kGateThreads = 1024;

__global__ __launch_bounds__(kGateThreads) void auto_gate_kernel(const uint32_t* __restrict__ hist_rmi, uint32_t B,
                                                                 uint64_t S, float accept_ratio, uint32_t kind,
                                                                 ModelHeader* __restrict__ hdr) {
  __shared__ uint32_t mr[kGateThreads / 64];
  uint32_t a = 0;
#pragma unroll 4
  for (uint32_t j = threadIdx.x; j < B; j += kGateThreads) a = hist_rmi[j] > a ? hist_rmi[j] : a;
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t x = __shfl_xor(a, off);
    a = x > a ? x : a;
  }
  if (__lane_id() == 0) mr[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t w = 1; w < kGateThreads / 64; ++w) mr[0] = mr[w] > mr[0] ? mr[w] : mr[0];
    const double lambda = (double)S / (double)B;
    const double perfect = lambda + sqrt(2.0 * log((double)B) * lambda) + 1.0;
    const bool ok = (double)mr[0] <= (double)accept_ratio * perfect;
    hdr->max_rmi = mr[0];
    hdr->perfect = (float)perfect;
    hdr->rmi_ok = ok ? 1u : 0u;
    hdr->mlp_skip = (kind == 2u && ok) ? 1u : 0u;
  }
}

// Choice of the root.  hist_eq: the sample histogram under the equi-depth
// leaves (MLP and spline roots share them); hist_net: the network's own
// buckets (kind MLP).  The ideal is max(ceil(S/B), longest equal-code run).
//  kind 1 (MLP): the network is accepted if its own largest sample bucket is
//    at most accept_ratio times the ideal; records are then routed by the
//    network into the equi-depth leaves.  Otherwise the plain model takes
//    over, as the automatic choice picks it: the linear root if it passed its
//    gate, else the spline root.
//  kind 2 (automatic): the linear root if it passed its gate, else the spline.
//  kind 4 (spline): the spline root.  Kinds 0 and 3: the linear root.
// The chosen root's sample histogram is copied to hist_used; the three
// largest sample buckets are recorded.
constexpr uint32_t kDecideThreads = 1024;

__global__ __launch_bounds__(kDecideThreads) void decide_root_kernel(const uint32_t* __restrict__ hist_rmi,
                                                                     const uint32_t* __restrict__ hist_eq,
                                                                     const uint32_t* __restrict__ hist_net, uint32_t B,
                                                                     uint64_t S, float accept_ratio, uint32_t kind,
                                                                     ModelHeader* __restrict__ hdr,
                                                                     uint32_t* __restrict__ hist_used) {
  constexpr uint32_t W = kDecideThreads / 64;
  __shared__ uint32_t mr[W], me[W], mn[W];
  __shared__ uint32_t use_eq;
  // the largest count of each histogram: four buckets a thread per step as
  // 16-byte loads (the arrays start 16-byte aligned), one loop per array and
  // no branch around the loads, so that the unrolled steps' loads are in
  // flight together (one bucket at a time they took 31-47 us on one CU)
  const uint32_t B4 = B & ~3u;
  auto hmax = [&](const uint32_t* __restrict__ h) {
    uint32_t m = 0;
#pragma unroll 4
    for (uint32_t j = 4 * threadIdx.x; j < B4; j += 4 * kDecideThreads) {
      const uint4 x = *reinterpret_cast<const uint4*>(h + j);
      const uint32_t p = x.x > x.y ? x.x : x.y, q = x.z > x.w ? x.z : x.w;
      const uint32_t r = p > q ? p : q;
      m = r > m ? r : m;
    }
    for (uint32_t j = B4 + threadIdx.x; j < B; j += kDecideThreads) m = h[j] > m ? h[j] : m;
    return m;
  };
  uint32_t a = hmax(hist_rmi), b = hist_eq ? hmax(hist_eq) : 0u, c = hist_net ? hmax(hist_net) : 0u;
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t x = __shfl_xor(a, off), y = __shfl_xor(b, off), z = __shfl_xor(c, off);
    a = x > a ? x : a;
    b = y > b ? y : b;
    c = z > c ? z : c;
  }
  if (__lane_id() == 0) {
    mr[threadIdx.x >> 6] = a;
    me[threadIdx.x >> 6] = b;
    mn[threadIdx.x >> 6] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t w = 1; w < W; ++w) {
      mr[0] = mr[w] > mr[0] ? mr[w] : mr[0];
      me[0] = me[w] > me[0] ? me[w] : me[0];
      mn[0] = mn[w] > mn[0] ? mn[w] : mn[0];
    }
    uint32_t ideal = (uint32_t)((S + B - 1) / B);
    if (hist_eq && hdr->max_sample_run > ideal) ideal = hdr->max_sample_run;
    uint32_t u = 0, rejected = 0;
    if (hist_eq) {
      if (kind == 1u) {
        const bool pass = hist_net && (double)mn[0] <= (double)accept_ratio * (double)ideal;
        rejected = pass ? 0u : 1u;
        u = pass ? 1u : (hdr->rmi_ok ? 0u : 2u);
      } else if (kind == 2u) {
        u = hdr->mlp_skip ? 0u : 2u;
      } else if (kind == 4u) {
        u = 2u;
      }
    }
    hdr->kind_used = u;
    hdr->mlp_rejected = rejected;
    hdr->max_rmi = mr[0];
    hdr->max_eq = hist_eq ? me[0] : 0u;
    hdr->max_net = hist_net ? mn[0] : 0u;
    hdr->max_sample_bucket = u ? me[0] : mr[0];
    hdr->opt_sample_bucket = ideal;
    use_eq = u;
  }
  __syncthreads();
  if (use_eq) {
#pragma unroll 4
    for (uint32_t j = 4 * threadIdx.x; j < B4; j += 4 * kDecideThreads)
      *reinterpret_cast<uint4*>(hist_used + j) = *reinterpret_cast<const uint4*>(hist_eq + j);
    for (uint32_t j = B4 + threadIdx.x; j < B; j += kDecideThreads) hist_used[j] = hist_eq[j];
  }
}

// ------------------------------------------------------------------- host --
// The training kernels' LDS exceeds the default limit; the attribute is set
// once per process (not while a stream is being captured).
static hipError_t allow_big_lds(const void* fn) {
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sizeof(TrainLds));
}

hipError_t mlp_prepare_kernels() {
  static hipError_t once = [] {
    hipError_t e = allow_big_lds(reinterpret_cast<const void*>(mlp_train_kernel));
    if (e == hipSuccess) e = allow_big_lds(reinterpret_cast<const void*>(mlp_grad_kernel));
    if (e == hipSuccess) e = allow_big_lds(reinterpret_cast<const void*>(mlp_step_kernel));
    return e;
  }();
  return once;
}

hipError_t launch_mlp_train(const uint64_t* e, uint64_t S, uint64_t seed, uint32_t steps, float lr,
                            const MlpState& ms, hipStream_t st) {
  if (S == 0) return hipSuccess;
  mlp_setup_kernel<<<1, 256, 0, st>>>(e, S, seed, ms.M, ms.master, ms.adam);
  mlp_publish_kernel<<<1, 256, 0, st>>>(ms.master, nullptr, ms.M);
  if (steps) {
    hipError_t err = mlp_prepare_kernels();
    if (err != hipSuccess) return err;
    mlp_train_kernel<<<1, kTrainThreads, sizeof(TrainLds), st>>>(e, S, steps, lr, seed, ms.master, ms.adam, ms.M);
  }
  return hipGetLastError();
}

hipError_t launch_equi_depth_leaves(const uint64_t* e, uint64_t S, uint32_t L, uint32_t B, ModelHeader* hdr,
                                    const MlpState& ms, hipStream_t st) {
  if (S == 0) return hipSuccess;
  const uint32_t K = spline_segments(L);
  quantile_first_kernel<<<(L + 1 + 255) / 256, 256, 0, st>>>(e, S, L, ms.first, hdr);
  mlp_leaf_fit_kernel<<<(L + 255) / 256, 256, 0, st>>>(e, S, L, B, ms.first, ms.leaves, ms.bound, hdr);
  spline_knots_kernel<<<(K + 1 + 255) / 256, 256, 0, st>>>(ms.bound, L, K, ms.knots, hdr);
  code_cell_kernel<<<(code_cells_for(L) + 1 + 255) / 256, 256, 0, st>>>(ms.bound, L, ms.ccells, hdr);
  code_subcell_kernel<<<(code_cells_for(L) + 3) / 4, 256, 0, st>>>(ms.bound, L, ms.ccells, hdr);
  hipError_t err = launch_fill_u32(ms.hist, B, 0u, st);
  if (err != hipSuccess) return err;
  const uint64_t threads = S > L ? S : L;
  mlp_sample_stats_kernel<<<(uint32_t)((threads + 255) / 256), 256, 0, st>>>(e, S, L, B, ms.first, ms.leaves,
                                                                              ms.hist, hdr);
  return hipGetLastError();
}

hipError_t launch_mlp_cell_table(const MlpState& ms, uint32_t L, const ModelHeader* hdr, hipStream_t st) {
  if (L == 0) return hipSuccess;
  mlp_cell_table_kernel<<<(L + 1 + 255) / 256, 256, 0, st>>>(ms.M, ms.bound, L, ms.cells, hdr);
  return hipGetLastError();
}

hipError_t launch_auto_gate(const uint32_t* hist_rmi, uint32_t B, uint64_t S, float accept_ratio, uint32_t kind,
                            ModelHeader* hdr, hipStream_t st) {
  auto_gate_kernel<<<1, kGateThreads, 0, st>>>(hist_rmi, B, S, accept_ratio, kind, hdr);
  return hipGetLastError();
}

hipError_t launch_decide_root(const uint32_t* hist_rmi, const MlpState* ms, uint32_t B, uint64_t S,
                              float accept_ratio, uint32_t kind, ModelHeader* hdr, uint32_t* hist_used,
                              hipStream_t st) {
  const uint32_t* hist_net = (ms && kind == 1u) ? ms->hist_net : nullptr;
  decide_root_kernel<<<1, kDecideThreads, 0, st>>>(hist_rmi, ms ? ms->hist : nullptr, hist_net, B, S, accept_ratio,
                                                   kind, hdr, hist_used);
  return hipGetLastError();
}

hipError_t launch_mlp_net_hist(const MlpState& ms, const uint64_t* e, uint64_t S, uint32_t B, hipStream_t st) {
  hipError_t err = launch_fill_u32(ms.hist_net, B, 0u, st);
  if (err != hipSuccess || S == 0) return err;
  mlp_net_hist_kernel<<<(uint32_t)((S + 255) / 256), 256, 0, st>>>(ms.M, e, S, B, ms.hist_net);
  return hipGetLastError();
}

hipError_t launch_mlp_step(const MlpBlock* M, float* params, float* adam, const uint64_t* codes,
                           const float* targets, uint32_t step, float lr, float* grad, float* loss, hipStream_t st) {
  hipError_t err = mlp_prepare_kernels();
  if (err != hipSuccess) return err;
  mlp_step_kernel<<<1, kTrainThreads, sizeof(TrainLds), st>>>(M, params, adam, codes, targets, step, lr, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_params_to_block(const float* d_params, const uint64_t* d_q9, MlpBlock* M, hipStream_t st) {
  mlp_publish_kernel<<<1, 256, 0, st>>>(d_params, d_q9, M);
  return hipGetLastError();
}

hipError_t launch_mlp_eval(const MlpBlock* M, const uint64_t* codes, uint64_t n, float* y, hipStream_t st) {
  if (n == 0) return hipSuccess;
  mlp_eval_kernel<<<(uint32_t)((n + 255) / 256), 256, 0, st>>>(M, codes, n, y);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpBlock* M, const uint64_t* codes, const float* targets, float* grad, float* loss,
                           hipStream_t st) {
  hipError_t err = mlp_prepare_kernels();
  if (err != hipSuccess) return err;
  mlp_grad_kernel<<<1, kTrainThreads, sizeof(TrainLds), st>>>(M, codes, targets, grad, loss);
  return hipGetLastError();
}

}  // namespace elsar
