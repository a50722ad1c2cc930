// Device-side evaluation of the monotone MLP root, shared by the fit kernels
// and the partition kernel.
//
// Matrix core layout of v_mfma_f32_16x16x16bf16_1k (one wave, 16x16x16):
// lane l holds A[l%16][4(l/16)+e], B[4(l/16)+e][l%16] and D[4(l/16)+e][l%16]
// for e = 0..3.  A wave evaluates 16 records per product: lane l computes the
// layer-1 units 16ks + 4(l/16) + e (ks, e = 0..3) of record l%16, which are
// exactly the A fragments it feeds to the four K-steps, so h1 never leaves
// registers.
#pragma once
#include "elsar_internal.h"

namespace elsar {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f32_to_bf16(float f) {  // round to nearest, ties to even (finite f)
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float sigm(float z) {  // logistic with the hardware exp2 and reciprocal
  return __builtin_amdgcn_rcpf(1.0f + __expf(-z));
}

__device__ __forceinline__ s16x4 load4_bf16(const uint16_t* p) {  // 8-byte aligned
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  s16x4 r;
  r[0] = (short)(v.x & 0xFFFFu);
  r[1] = (short)(v.x >> 16);
  r[2] = (short)(v.y & 0xFFFFu);
  r[3] = (short)(v.y >> 16);
  return r;
}

__device__ __forceinline__ s16x4 pack4_bf16(float a, float b, float c, float d) {
  s16x4 r;
  r[0] = (short)f32_to_bf16(a);
  r[1] = (short)f32_to_bf16(b);
  r[2] = (short)f32_to_bf16(c);
  r[3] = (short)f32_to_bf16(d);
  return r;
}

// phi_k = min(1, max(code - q_k, 0) / w_k): each feature non-decreasing in the code.
__device__ __forceinline__ void mlp_features(uint64_t code, const MlpHead& M, float phi[8]) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    uint64_t d = code >= M.q[k] ? code - M.q[k] : 0ull;
    phi[k] = fminf(1.0f, (float)d * M.inv_w[k]);
  }
}

// sigmoid(b1[u] + W1[u] . phi) for the 16 units this lane feeds to the matrix core.
__device__ __forceinline__ void mlp_layer1_frags(const float phi[8], const MlpHead& M, uint32_t g, s16x4 a[4],
                                                 float h1[16]) {
#pragma unroll
  for (uint32_t ks = 0; ks < 4; ++ks) {
#pragma unroll
    for (uint32_t e = 0; e < 4; ++e) {
      const uint32_t u = 16 * ks + 4 * g + e;
      float z = M.b1[u];
#pragma unroll
      for (int k = 0; k < 8; ++k) z = __builtin_fmaf(M.W1[u * 8 + k], phi[k], z);
      h1[4 * ks + e] = sigm(z);
    }
    a[ks] = pack4_bf16(h1[4 * ks], h1[4 * ks + 1], h1[4 * ks + 2], h1[4 * ks + 3]);
  }
}

// B fragments of W2 for the 4 column tiles x 4 K-steps, held for a whole kernel.
struct W2Frags {
  s16x4 f[16];  // [ct * 4 + ks]
};

__device__ __forceinline__ void mlp_load_w2(const uint16_t* __restrict__ W2bf, W2Frags& w) {
  const uint32_t l = __lane_id(), r = l & 15u, g = l >> 4;
#pragma unroll
  for (uint32_t ct = 0; ct < 4; ++ct)
#pragma unroll
    for (uint32_t ks = 0; ks < 4; ++ks) w.f[ct * 4 + ks] = load4_bf16(W2bf + (16 * ct + r) * 64 + 16 * ks + 4 * g);
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = __shfl((uint32_t)v, src), hi = __shfl((uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

// Root output y of the record whose code this lane holds; all 64 lanes of the
// wave must take part (64 records per call).
__device__ __forceinline__ float mlp_y64(uint64_t code, const MlpHead& M, const W2Frags& w) {
  const uint32_t l = __lane_id(), r = l & 15u, g = l >> 4;
  float y_own = 0.0f;
#pragma unroll 1
  for (uint32_t c = 0; c < 4; ++c) {
    // the layer-1 weights are re-read from LDS for every chunk instead of
    // being kept in registers across chunks and tiles (which costs occupancy)
    __asm__ volatile("" ::: "memory");
    const uint64_t cc = shfl_u64(code, (int)(16 * c + r));  // record 16c + r
    float phi[8], h1[16];
    s16x4 a[4];
    mlp_features(cc, M, phi);
    mlp_layer1_frags(phi, M, g, a, h1);
    float part[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (uint32_t ct = 0; ct < 4; ++ct) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (uint32_t ks = 0; ks < 4; ++ks)
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[ks], w.f[ct * 4 + ks], acc, 0, 0, 0);
      const uint32_t col = 16 * ct + r;
#pragma unroll
      for (int e = 0; e < 4; ++e) part[e] = __builtin_fmaf(M.w3[col], sigm(acc[e] + M.b2[col]), part[e]);
    }
    // sum over the 16 columns a lane group holds: rows 4g + e of this chunk
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) part[e] += __shfl_xor(part[e], off);
    // lane l's own record is row l%16 of chunk l/16: lane group r/4, slot r%4
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const float v = __shfl(part[e], (int)(16 * (r >> 2)));
      if (g == c && (r & 3u) == (uint32_t)e) y_own = v;
    }
  }
  return y_own + M.b3;
}

__device__ __forceinline__ uint32_t mlp_leaf_guess(float y, uint32_t L) {
  const float f = floorf(y * (float)L);
  if (!(f > 0.0f)) return 0;  // also NaN
  if (f > (float)(L - 1)) return L - 1;
  return (uint32_t)f;
}

// The leaf j with bound[j] <= code < bound[j+1] (bound[0] = 0, bound[L] past
// every code), by exponential search from the guess j0.
__device__ __forceinline__ uint32_t mlp_exact_leaf(const uint64_t* __restrict__ bound, uint32_t L, uint64_t code,
                                                   uint32_t j0) {
  uint32_t lo, hi;  // bound[lo] <= code < bound[hi], hi <= L
  if (bound[j0] > code) {
    hi = j0;
    uint32_t step = 1;
    for (;;) {
      if (step >= hi) { lo = 0; break; }
      lo = hi - step;
      if (bound[lo] <= code) break;
      hi = lo;
      step <<= 1;
    }
  } else {
    lo = j0;
    uint32_t step = 1;
    for (;;) {
      if (lo + step >= L) { hi = L; break; }
      hi = lo + step;
      if (bound[hi] > code) break;
      lo = hi;
      step <<= 1;
    }
  }
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (bound[mid] <= code) lo = mid; else hi = mid;
  }
  return lo;
}

}  // namespace elsar
