// Device-side code of the monotone MLP root: the training kernels' layer-1
// helper and the evaluation shared by the cell-table, forward and partition
// kernels, plus the leaf routers.
//
// Matrix-core layouts (one wave, 16x16 outputs): for gfx950's
// v_mfma_f32_16x16x32_bf16 lane l holds A[l%16][8(l/16)+e] and
// B[8(l/16)+e][l%16] for e = 0..7, and D[4(l/16)+e][l%16] for e = 0..3; for
// v_mfma_f32_16x16x4_f32 lane l holds A[l%16][l/16] and B[l/16][l%16], D as
// above.  The bfloat16 fragments are built as groups of four K-indices per
// lane, 4(l/16)+e of a 16-wide K-step, and two K-steps' groups are joined
// into the eight a 16x16x32 product takes (cat8_bf16): a contraction only
// needs A and B to list K in the same order.  Training computes records x
// units (layer-1 units of record l%16 become the A fragments of the layer-2
// product); evaluation computes units x records (mlp_y64).
#pragma once
#include "elsar_internal.h"

namespace elsar {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Two 4-element bfloat16 fragments as the 8 elements one lane gives a
// 16x16x32 product.
__device__ __forceinline__ bf16x8 cat8_bf16(s16x4 a, s16x4 b) {
  const s16x8 v = {a[0], a[1], a[2], a[3], b[0], b[1], b[2], b[3]};
  return __builtin_bit_cast(bf16x8, v);
}

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

// Matrix-core operands of the evaluation, held for a whole kernel:
// f[4ct + ks] = W2[16ct + l%16][16ks + 4(l/16) + e] (e = 0..3, bfloat16), the
// A fragments of layer 2 computed as W2 . H1^T; w1[2ks + h] = W1[16ks +
// l%16][4h + l/16], the A operands of layer 1 computed as W1 . Phi^T in FP32
// (v_mfma_f32_16x16x4_f32: lane l gives A[l%16][l/16] and B[l/16][l%16]).
struct MlpFrags {
  s16x4 f[16];
  float w1[8];
};

__device__ __forceinline__ void mlp_load_frags(const MlpBlock* __restrict__ Mg, MlpFrags& w) {
  const uint32_t l = __lane_id(), r = l & 15u, g = l >> 4;
#pragma unroll
  for (uint32_t ct = 0; ct < 4; ++ct)
#pragma unroll
    for (uint32_t ks = 0; ks < 4; ++ks)
      w.f[ct * 4 + ks] = load4_bf16(Mg->W2bf + (16 * ct + r) * kW2S + 16 * ks + 4 * g);
#pragma unroll
  for (uint32_t ks = 0; ks < 4; ++ks)
#pragma unroll
    for (uint32_t h = 0; h < 2; ++h) w.w1[2 * ks + h] = Mg->h.W1[(16 * ks + r) * 8 + 4 * h + g];
}

// Feature k of one code (as in mlp_features).
__device__ __forceinline__ float mlp_feature(uint64_t code, const MlpHead& M, uint32_t k) {
  const uint64_t d = code >= M.q[k] ? code - M.q[k] : 0ull;
  return fminf(1.0f, (float)d * M.inv_w[k]);
}

// Four values rounded to bfloat16 (nearest, ties to even) by the converter.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ s16x4 pack4_bf16_cvt(float a, float b, float c, float d) {
  const bf16x2 lo = __builtin_convertvector((f32x2){a, b}, bf16x2);
  const bf16x2 hi = __builtin_convertvector((f32x2){c, d}, bf16x2);
  const uint32_t u0 = __builtin_bit_cast(uint32_t, lo), u1 = __builtin_bit_cast(uint32_t, hi);
  s16x4 v;
  v[0] = (short)(u0 & 0xFFFFu);
  v[1] = (short)(u0 >> 16);
  v[2] = (short)(u1 & 0xFFFFu);
  v[3] = (short)(u1 >> 16);
  return v;
}

// Root output y of the record whose code this lane holds; all 64 lanes of the
// wave must take part (64 records per call, in four chunks of 16).  Both
// hidden layers run transposed, units x records, on the matrix cores: layer 1
// in FP32 from two features per lane, layer 2 in bfloat16 with FP32
// accumulation.  Lane l then holds units 16t + 4(l/16) + e of record l%16 of
// the chunk, so layer 1's output is already layer 2's B fragment, and the
// output unit is an in-lane sum over 16 units plus a sum over the four lane
// groups.  Layer 2 runs as 16x16x32 products: K-step s contracts units
// 32s .. 32s+31, lane group g giving units 32s + 4g + e and 32s + 16 + 4g +
// e (e = 0..3) -- the h1 tiles 2s and 2s+1 it holds, and the W2 fragments of
// the same units; the contraction does not depend on the order of its terms
// across lane slots, only on A and B agreeing on it.
__device__ __forceinline__ float mlp_y64(uint64_t code, const MlpHead& M, const MlpFrags& w) {
  const uint32_t l = __lane_id(), r = l & 15u, g = l >> 4;
  float y_own = 0.0f;
#pragma unroll 1
  for (uint32_t c = 0; c < 4; ++c) {
    // biases are re-read from LDS for every chunk rather than held in registers
    __asm__ volatile("" ::: "memory");
    const uint64_t cc = shfl_u64(code, (int)(16 * c + r));  // record 16c + r
    const float p0 = mlp_feature(cc, M, g), p1 = mlp_feature(cc, M, g + 4);
    s16x4 h1[4];  // units 16ks + 4g + e of record r
#pragma unroll
    for (uint32_t ks = 0; ks < 4; ++ks) {
      const uint32_t u = 16 * ks + 4 * g;
      f32x4 z = {M.b1[u], M.b1[u + 1], M.b1[u + 2], M.b1[u + 3]};
      z = __builtin_amdgcn_mfma_f32_16x16x4f32(w.w1[2 * ks], p0, z, 0, 0, 0);
      z = __builtin_amdgcn_mfma_f32_16x16x4f32(w.w1[2 * ks + 1], p1, z, 0, 0, 0);
      h1[ks] = pack4_bf16_cvt(sigm(z[0]), sigm(z[1]), sigm(z[2]), sigm(z[3]));
    }
    float part = 0.0f;
#pragma unroll
    for (uint32_t ct = 0; ct < 4; ++ct) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (uint32_t s = 0; s < 2; ++s)
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(cat8_bf16(w.f[ct * 4 + 2 * s], w.f[ct * 4 + 2 * s + 1]),
                                                      cat8_bf16(h1[2 * s], h1[2 * s + 1]), acc, 0, 0, 0);
      const uint32_t u = 16 * ct + 4 * g;
#pragma unroll
      for (int e = 0; e < 4; ++e) part = __builtin_fmaf(M.w3[u + e], sigm(acc[e] + M.b2[u + e]), part);
    }
    // the four lane groups of record r (every lane ends with the same sum)
    part += __shfl_xor(part, 16);
    part += __shfl_xor(part, 32);
    if (g == c) y_own = part;  // lane l's own record is record l%16 of chunk l/16
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

// The same leaf, searched inside the bracket that the cell table gives for
// the network's output y: cells[c] - 1 <= j < cells[c + 1] for c = floor(L y).
// The bracket is checked against the boundaries first; a bracket that does not
// hold (only possible if rounding made y decrease somewhere) falls back to the
// search from the guess, so the leaf is exact either way.
__device__ __forceinline__ uint32_t mlp_bracket_leaf(const uint64_t* __restrict__ bound,
                                                     const uint32_t* __restrict__ cells, uint32_t L, uint64_t code,
                                                     float y) {
  const uint32_t c = mlp_leaf_guess(y, L);
  const uint32_t t0 = cells[c], t1 = cells[c + 1];
  uint32_t lo = t0 ? t0 - 1u : 0u, hi = t1;  // bound[lo] <= code < bound[hi] (hi == L: past every code)
  if (hi <= lo || bound[lo] > code || (hi < L && bound[hi] <= code)) return mlp_exact_leaf(bound, L, code, c);
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (bound[mid] <= code) lo = mid; else hi = mid;
  }
  return lo;
}

}  // namespace elsar
