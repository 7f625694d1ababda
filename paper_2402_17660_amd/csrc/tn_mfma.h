// Wave-level MFMA tile products shared by the pair kernels and the node mixing kernel.
#pragma once

#include <hip/hip_runtime.h>

namespace tn {

typedef float floatx4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4 mfma4(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// mfma4 with the activation fragment a and the weight fragment b; with TR the weights are the
// instruction's first operand, so the accumulator holds the product transposed (see wave_mm_t).
template <bool TR>
__device__ __forceinline__ floatx4 mfma4_ab(float a, float b, floatx4 c) {
  return TR ? mfma4(b, a, c) : mfma4(a, b, c);
}

// BF16 operands, FP32 accumulation (v_mfma_f32_16x16x32_bf16): lane l holds
// A[l%16][8(l/16)..8(l/16)+7] and B[8(l/16)..+7][l%16]; the result layout is that of mfma4.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
constexpr int kPadB = 8;   // LDS row padding of BF16 operand tiles (elements)

__device__ __forceinline__ floatx4 mfma_bf16(const bf16x8 &a, const bf16x8 &b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Four consecutive values (16-byte aligned FP32, 8-byte aligned BF16) as one vector access.
__device__ __forceinline__ floatx4 ld4(const float *p) { return *reinterpret_cast<const floatx4 *>(p); }
__device__ __forceinline__ floatx4 ld4(const __bf16 *p) {
  const bf16x4 v = *reinterpret_cast<const bf16x4 *>(p);
  return floatx4{(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
}
__device__ __forceinline__ void st4(float *p, const floatx4 &v) { *reinterpret_cast<floatx4 *>(p) = v; }
__device__ __forceinline__ void st4(__bf16 *p, const floatx4 &v) {
  bf16x4 o;
#pragma unroll
  for (int t = 0; t < 4; ++t) o[t] = (__bf16)v[t];
  *reinterpret_cast<bf16x4 *>(p) = o;
}

// acc[rb][cb] += act_rb[16 x Kin] * Bt^T for rb < RB, where row i of block rb starts at
// act + rb*rbs + i*ld (LDS) and Bt is [ncol][Kin] in global memory (row stride Kin); this wave
// covers columns col0 .. col0 + 16*NB - 1 (v_mfma_f32_16x16x4f32).  Inside each 16-wide K
// chunk, lane group q takes k = 4q..4q+3, so one 16-byte load feeds four MFMAs for both
// operands; the weight fragments of the next chunk are loaded while the current chunk's MFMAs
// run.  Element t of acc[rb][cb] in lane l is D_rb[4*(l/16) + t][col0 + cb*16 + l%16].
template <int RB, int NB, bool TR = false>
__device__ __forceinline__ void wave_mm_rows(const float *act, int ld, int rbs, int Kin, const float *__restrict__ Bt,
                                             int col0, floatx4 (&acc)[RB][NB]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
  const float *ap = act + r * ld + 4 * q;
  const float *bp = Bt + (size_t)(col0 + r) * Kin + 4 * q;
  const size_t bstride = (size_t)16 * Kin;
  float4 bn[NB];
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) bn[cb] = *reinterpret_cast<const float4 *>(bp + cb * bstride);
  for (int k0 = 0; k0 < Kin; k0 += 16) {
    float4 b[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) b[cb] = bn[cb];
    if (k0 + 16 < Kin) {
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) bn[cb] = *reinterpret_cast<const float4 *>(bp + cb * bstride + k0 + 16);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const float4 a = *reinterpret_cast<const float4 *>(ap + rb * rbs + k0);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        acc[rb][cb] = mfma4_ab<TR>(a.x, b[cb].x, acc[rb][cb]);
        acc[rb][cb] = mfma4_ab<TR>(a.y, b[cb].y, acc[rb][cb]);
        acc[rb][cb] = mfma4_ab<TR>(a.z, b[cb].z, acc[rb][cb]);
        acc[rb][cb] = mfma4_ab<TR>(a.w, b[cb].w, acc[rb][cb]);
      }
    }
  }
}

// Row blocks stacked contiguously: block rb starts 16 rows after block rb - 1.
template <int RB, int NB>
__device__ __forceinline__ void wave_mm_rb(const float *act, int ld, int Kin, const float *__restrict__ Bt, int col0,
                                           floatx4 (&acc)[RB][NB]) {
  wave_mm_rows<RB, NB>(act, ld, 16 * ld, Kin, Bt, col0, acc);
}

// wave_mm_rb with the operands of each instruction swapped: the accumulator holds the product
// transposed.  Entry t of acc[rb][cb] in lane l is D_rb[l%16][col0 + cb*16 + 4(l/16) + t], so a
// lane holds four consecutive columns of one row, which a row-major store or load moves in one
// vector access.  Same products, same k order.
template <int RB, int NB>
__device__ __forceinline__ void wave_mm_t(const float *act, int ld, int Kin, const float *__restrict__ Bt, int col0,
                                          floatx4 (&acc)[RB][NB]) {
  wave_mm_rows<RB, NB, true>(act, ld, 16 * ld, Kin, Bt, col0, acc);
}

// The same product with this wave's weight fragments already in registers: b[kc][cb] holds
// Bt[col0 + cb*16 + l%16][16 kc + 4(l/16) .. +3] for the KC = Kin/16 chunks (TR: transposed
// accumulator, as wave_mm_t).
template <int RB, int NB, int KC, bool TR = false>
__device__ __forceinline__ void wave_mm_rows_breg(const float *act, int ld, int rbs, const float4 (&b)[KC][NB],
                                                  floatx4 (&acc)[RB][NB]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
  const float *ap = act + r * ld + 4 * q;
#pragma unroll
  for (int kc = 0; kc < KC; ++kc) {
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const float4 a = *reinterpret_cast<const float4 *>(ap + rb * rbs + 16 * kc);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        acc[rb][cb] = mfma4_ab<TR>(a.x, b[kc][cb].x, acc[rb][cb]);
        acc[rb][cb] = mfma4_ab<TR>(a.y, b[kc][cb].y, acc[rb][cb]);
        acc[rb][cb] = mfma4_ab<TR>(a.z, b[kc][cb].z, acc[rb][cb]);
        acc[rb][cb] = mfma4_ab<TR>(a.w, b[kc][cb].w, acc[rb][cb]);
      }
    }
  }
}

// Loads this wave's weight fragments for wave_mm_rows_breg.
template <int NB, int KC>
__device__ __forceinline__ void load_bfrag(const float *__restrict__ Bt, int Kin, int col0, float4 (&b)[KC][NB]) {
  const int lane = threadIdx.x & 63;
  const float *bp = Bt + (size_t)(col0 + (lane & 15)) * Kin + 4 * (lane >> 4);
#pragma unroll
  for (int kc = 0; kc < KC; ++kc)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) b[kc][cb] = *reinterpret_cast<const float4 *>(bp + (size_t)cb * 16 * Kin + 16 * kc);
}

template <int RB, int NB>
__device__ __forceinline__ void zero_acc_rb(floatx4 (&acc)[RB][NB]) {
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) acc[rb][cb] = floatx4{0.f, 0.f, 0.f, 0.f};
}

}  // namespace tn
