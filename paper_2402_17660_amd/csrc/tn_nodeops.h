// Node-level and generic kernels shared by the plain and fused paths (templated on the
// arithmetic type).  Feature layout: [atoms, 9 coordinates, F channels], see tn_device.h.
#pragma once

#include "tn_internal.h"
#include "tn_device.h"
#include "tn_mfma.h"

#include <type_traits>

namespace tn {

// ============================================================================ generic GEMM
// C[m, n] = epilogue(sum_k A[m, k] * B(k, n)),  B(k, n) = B[n*ldb + k] if transB else B[k*ldb + n].
// Epilogue: + bias[n]; store pre-activation to Z; SiLU; * rowscale[m]; * silu'(gate[m, n]);
// store or accumulate.  Rows >= min(M, *Mdev) are skipped.  blockIdx.z batches over the nine
// feature coordinates: A, C, gate shifted by z * zoff, B = Bz[part(z)] when zpart.
template <class T>
struct GemmArgs {
  const T *A = nullptr; int64_t lda = 0;
  const T *B = nullptr; int64_t ldb = 0; int transB = 0;
  T *C = nullptr; int64_t ldc = 0;
  const T *bias = nullptr;
  T *Z = nullptr; int64_t ldz = 0;
  int act = 0;
  const T *rowscale = nullptr;
  const T *gate = nullptr; int64_t ldg = 0;
  int accumulate = 0;
  int64_t M = 0, N = 0, K = 0;
  const int64_t *Mdev = nullptr;
  int64_t zoff = 0;
  int zpart = 0;
  const T *Bz[3] = {nullptr, nullptr, nullptr};
};

constexpr int GBN = 64, GBK = 32;

// The product runs on the matrix cores: BMx64 block tiles (BM = 32 or 64), each of the four
// waves computes a (BM/2)x32 part as MFMA 16x16x4 tiles (f32 or f64).  A and B chunks of 32 along K are
// staged through LDS; the next chunk's global loads are issued into registers before the
// current chunk's MFMAs, so their latency overlaps the products.  Both instructions take
// A[l%16][l/16] and B[l/16][l%16] from lane l; element t of the result in lane l is
// D[4(l/16)+t][l%16] for f32 and D[4t+l/16][l%16] for f64.
typedef float mf_f32x4 __attribute__((ext_vector_type(4)));
typedef double mf_f64x4 __attribute__((ext_vector_type(4)));
template <class T> struct MfmaVec;
template <> struct MfmaVec<float> { using type = mf_f32x4; };
template <> struct MfmaVec<double> { using type = mf_f64x4; };
__device__ __forceinline__ mf_f32x4 mfma_16x16x4(float a, float b, mf_f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ mf_f64x4 mfma_16x16x4(double a, double b, mf_f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Epilogue inputs a GEMM launch uses (bits of EP): the row scale, the gate, the old output.
// Kernels compiled for a subset hold registers only for those inputs.
constexpr int kEpScale = 1, kEpGate = 2, kEpAcc = 4, kEpAll = 7;
template <class T>
__host__ __device__ inline int gemm_ep(const GemmArgs<T> &g) {
  return (g.rowscale ? kEpScale : 0) | (g.gate ? kEpGate : 0) | (g.accumulate ? kEpAcc : 0);
}

// One BM x 64 output tile: blk is the flat (row tile, column tile) index, z the coordinate
// batch index; As [BM][GBK+1] and Bs [GBN][GBK+1] are the caller's LDS.  256 threads.
// EP: the epilogue inputs this instance may use (each still checked at run time).
template <class T, int BM, int EP = kEpAll>
__device__ __forceinline__ void gemm_tile(const GemmArgs<T> &g, int64_t blk, int z, T (*As)[GBK + 1],
                                          T (*Bs)[GBK + 1]) {
  using V = typename MfmaVec<T>::type;
  constexpr int RBW = BM / 32;                 // 16-row MFMA blocks per wave
  constexpr int PERA = BM * GBK / 256, PERB = GBN * GBK / 256;   // chunk elements per thread
  int64_t Mrows = g.M;
  if (g.Mdev) {
    const int64_t md = *g.Mdev;
    if (md < Mrows) Mrows = md;
  }
  // one flat block index over (row tile, column tile), column tiles fastest (so the blocks that
  // share a row tile run together); a flat x dimension has no 65535-block limit
  const int64_t nb = (g.N + GBN - 1) / GBN;
  const int64_t m0 = (blk / nb) * BM;
  const int64_t n0 = (blk % nb) * GBN;
  if (m0 >= Mrows) return;
  const T *__restrict__ A = g.A + z * g.zoff;
  const T *__restrict__ B = g.zpart ? g.Bz[coord_part(z)] : g.B;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * (BM / 2), wc = (wave & 1) * 32;
  const int r16 = lane & 15, q = lane >> 4;
  T ra[PERA], rb[PERB];
  auto load_chunk = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < PERA; ++e) {
      const int t = tid + 256 * e, mm_ = t / GBK, kk = t % GBK;
      const int64_t m = m0 + mm_, k = k0 + kk;
      ra[e] = (m < Mrows && k < g.K) ? A[m * g.lda + k] : T(0);
    }
#pragma unroll
    for (int e = 0; e < PERB; ++e) {
      const int t = tid + 256 * e;
      int nn, kk;
      if (g.transB) { nn = t / GBK; kk = t % GBK; } else { kk = t / GBN; nn = t % GBN; }
      const int64_t n = n0 + nn, k = k0 + kk;
      T v = T(0);
      if (n < g.N && k < g.K) v = g.transB ? B[n * g.ldb + k] : B[k * g.ldb + n];
      rb[e] = v;
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int e = 0; e < PERA; ++e) {
      const int t = tid + 256 * e;
      As[t / GBK][t % GBK] = ra[e];
    }
#pragma unroll
    for (int e = 0; e < PERB; ++e) {
      const int t = tid + 256 * e;
      int nn, kk;
      if (g.transB) { nn = t / GBK; kk = t % GBK; } else { kk = t / GBN; nn = t % GBN; }
      Bs[nn][kk] = rb[e];
    }
  };
  V acc[RBW][2];
#pragma unroll
  for (int a = 0; a < RBW; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = V{T(0), T(0), T(0), T(0)};
  load_chunk(0);
  for (int64_t k0 = 0; k0 < g.K; k0 += GBK) {
    store_chunk();
    __syncthreads();
    if (k0 + GBK < g.K) load_chunk(k0 + GBK);
#pragma unroll
    for (int s4 = 0; s4 < GBK; s4 += 4) {
      const T b0 = Bs[wc + r16][s4 + q], b1 = Bs[wc + 16 + r16][s4 + q];
#pragma unroll
      for (int a = 0; a < RBW; ++a) {
        const T av = As[wr + 16 * a + r16][s4 + q];
        acc[a][0] = mfma_16x16x4(av, b0, acc[a][0]);
        acc[a][1] = mfma_16x16x4(av, b1, acc[a][1]);
      }
    }
    __syncthreads();
  }
  T *C = g.C + z * g.zoff;
  T bias[2] = {T(0), T(0)};
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int64_t n = n0 + wc + cb * 16 + r16;
    if (g.bias && n < g.N) bias[cb] = g.bias[n];
  }
  // The epilogue's per-entry inputs (row scale, gate, old output) are all loaded before the
  // first store, so their latencies overlap.
  auto ep_m = [&](int rb_, int t) -> int64_t {
    return m0 + wr + rb_ * 16 + (sizeof(T) == 4 ? 4 * q + t : 4 * t + q);
  };
  constexpr int RS = (EP & kEpScale) ? RBW : 1, GT = (EP & kEpGate) ? RBW : 1, OL = (EP & kEpAcc) ? RBW : 1;
  T rs[RS][2][4], gt[GT][2][4], old[OL][2][4];
#pragma unroll
  for (int rb_ = 0; rb_ < RBW; ++rb_)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t m = ep_m(rb_, t), n = n0 + wc + cb * 16 + r16;
        const bool ok = m < Mrows && n < g.N;
        if constexpr ((EP & kEpScale) != 0) rs[rb_][cb][t] = (ok && g.rowscale) ? g.rowscale[m] : T(1);
        if constexpr ((EP & kEpGate) != 0) gt[rb_][cb][t] = (ok && g.gate) ? g.gate[z * g.zoff + m * g.ldg + n] : T(0);
        if constexpr ((EP & kEpAcc) != 0) old[rb_][cb][t] = (ok && g.accumulate) ? C[m * g.ldc + n] : T(0);
      }
#pragma unroll
  for (int rb_ = 0; rb_ < RBW; ++rb_)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t m = ep_m(rb_, t), n = n0 + wc + cb * 16 + r16;
        if (m >= Mrows || n >= g.N) continue;
        T v = acc[rb_][cb][t] + bias[cb];
        if (g.Z) g.Z[z * g.zoff + m * g.ldz + n] = v;
        if (g.act == 1) v = silu(v);
        if constexpr ((EP & kEpScale) != 0)
          if (g.rowscale) v *= rs[rb_][cb][t];
        if constexpr ((EP & kEpGate) != 0)
          if (g.gate) v *= silu_grad(gt[rb_][cb][t]);
        T *dst = C + m * g.ldc + n;
        if constexpr ((EP & kEpAcc) != 0) {
          if (g.accumulate) *dst = old[rb_][cb][t] + v; else *dst = v;
        } else {
          *dst = v;
        }
      }
}

// The FP64 64-row tile is held to three waves per SIMD (160 registers, no spills; the compiler
// otherwise takes 186 and leaves two): 343 -> 297 us per node-MLP product on 100k atoms.
template <class T, int BM, int EP>
__global__ void __launch_bounds__(256, (sizeof(T) == 8 && BM == 64) ? 3 : 1) k_gemm_mfma(GemmArgs<T> g) {
  __shared__ T As[BM][GBK + 1];
  __shared__ T Bs[GBN][GBK + 1];
  gemm_tile<T, BM, EP>(g, blockIdx.x, blockIdx.z, As, Bs);
}

template <class T, int BM>
inline void launch_gemm_ep(hipStream_t s, const GemmArgs<T> &g, dim3 grid) {
  switch (gemm_ep(g)) {
    case 0: hipLaunchKernelGGL((k_gemm_mfma<T, BM, 0>), grid, dim3(256), 0, s, g); break;
    case kEpScale: hipLaunchKernelGGL((k_gemm_mfma<T, BM, kEpScale>), grid, dim3(256), 0, s, g); break;
    case kEpGate: hipLaunchKernelGGL((k_gemm_mfma<T, BM, kEpGate>), grid, dim3(256), 0, s, g); break;
    case kEpAcc: hipLaunchKernelGGL((k_gemm_mfma<T, BM, kEpAcc>), grid, dim3(256), 0, s, g); break;
    default: hipLaunchKernelGGL((k_gemm_mfma<T, BM, kEpAll>), grid, dim3(256), 0, s, g); break;
  }
}

// Products with few 64-row tiles use 32-row tiles: fewer than two per compute unit in FP32,
// fewer than eight in FP64 (whose matrix instructions take twice as long, so a 64-row tile
// keeps a compute unit busy twice as long).
template <class T>
inline int gemm(hipStream_t s, const GemmArgs<T> &g, int zdim = 1) {
  if (g.M <= 0 || g.N <= 0) return TN_OK;
  const int64_t nb = (g.N + GBN - 1) / GBN;
  const int64_t tiles64 = nb * ((g.M + 63) / 64) * zdim;
  if (tiles64 < (sizeof(T) == 8 ? 2048 : 512)) {
    launch_gemm_ep<T, 32>(s, g, dim3((unsigned)(nb * ((g.M + 31) / 32)), 1, (unsigned)zdim));
  } else {
    launch_gemm_ep<T, 64>(s, g, dim3((unsigned)(nb * ((g.M + 63) / 64)), 1, (unsigned)zdim));
  }
  TN_LAUNCH_CHECK();
  return TN_OK;
}

// y = act(x W^T + b) over rows of x; W is [Nout, Kin] (torch Linear layout).
template <class T>
__host__ __device__ inline GemmArgs<T> linear_fwd_args(const T *x, int64_t M, int64_t Kin, const T *W, const T *b,
                                                       int64_t Nout, T *y, T *z_pre, int act,
                                                       const T *rowscale = nullptr, const int64_t *Mdev = nullptr) {
  GemmArgs<T> g;
  g.A = x; g.lda = Kin; g.B = W; g.ldb = Kin; g.transB = 1;
  g.C = y; g.ldc = Nout; g.bias = b; g.Z = z_pre; g.ldz = Nout; g.act = act; g.rowscale = rowscale;
  g.M = M; g.N = Nout; g.K = Kin; g.Mdev = Mdev;
  return g;
}

template <class T>
inline int linear_fwd(hipStream_t s, const T *x, int64_t M, int64_t Kin, const T *W, const T *b, int64_t Nout,
                      T *y, T *z_pre, int act, const T *rowscale = nullptr, const int64_t *Mdev = nullptr) {
  return gemm(s, linear_fwd_args(x, M, Kin, W, b, Nout, y, z_pre, act, rowscale, Mdev));
}

// dx (+)= (dy W) * silu'(gate); W is [Nout, Kin], dy [M, Nout], dx [M, Kin].
template <class T>
__host__ __device__ inline GemmArgs<T> linear_bwd_args(const T *dy, int64_t M, int64_t Nout, const T *W, int64_t Kin,
                                                       T *dx, const T *gate, int accumulate,
                                                       const int64_t *Mdev = nullptr) {
  GemmArgs<T> g;
  g.A = dy; g.lda = Nout; g.B = W; g.ldb = Kin; g.transB = 0;
  g.C = dx; g.ldc = Kin; g.gate = gate; g.ldg = Kin; g.accumulate = accumulate;
  g.M = M; g.N = Kin; g.K = Nout; g.Mdev = Mdev;
  return g;
}

template <class T>
inline int linear_bwd(hipStream_t s, const T *dy, int64_t M, int64_t Nout, const T *W, int64_t Kin, T *dx,
                      const T *gate, int accumulate, const int64_t *Mdev = nullptr) {
  return gemm(s, linear_bwd_args(dy, M, Nout, W, Kin, dx, gate, accumulate, Mdev));
}

// The mixing tiles' results from a transposed accumulator (weights as the instruction's first
// operand): lane l holds atom a0 + l%16, channels col0 + cb*16 + 4(l/16) .. +3 of coordinate
// C0 + rb, stored (or, accumulating, added to the old values, all loaded before the first
// store) as one 16-byte access per block, and as 8 bytes to the optional BF16 copy.
template <int F, int NC, int NB>
__device__ __forceinline__ void mix_epilogue(floatx4 (&acc)[NC][NB], float *__restrict__ out,
                                             __bf16 *__restrict__ out16, int64_t a0, int C0, int64_t navail,
                                             int col0, int accumulate) {
  const int lane = threadIdx.x & 63;
  const int r16 = lane & 15, q = lane >> 4;
  if (r16 >= navail) return;
  const int64_t o = ((a0 + r16) * 9 + C0) * F + col0 + 4 * q;
  if (accumulate) {
    floatx4 old[NC][NB];
#pragma unroll
    for (int rb = 0; rb < NC; ++rb)
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) old[rb][cb] = ld4(out + o + rb * F + cb * 16);
#pragma unroll
    for (int rb = 0; rb < NC; ++rb)
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) acc[rb][cb] = old[rb][cb] + acc[rb][cb];
  }
#pragma unroll
  for (int rb = 0; rb < NC; ++rb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      st4(out + o + rb * F + cb * 16, acc[rb][cb]);
      if (out16) st4(out16 + o + rb * F + cb * 16, acc[rb][cb]);
    }
}

// FP32 channel mixing on the matrix cores.  A block takes one part (I, A or S: 1, 3 or 5
// coordinates) of 16 atoms, stages those coordinates (contiguous per atom, F channels each)
// in LDS with padded rows, and computes 64*NB output channels; each of the four waves takes
// 16*NB of them for the part's coordinate rows, so one weight fragment feeds every
// coordinate of the part.  Bt[p] is the [F][F] matrix whose row n holds the input weights of
// output channel n (W_p itself for the forward mixing, its transpose for the adjoint).
// Blocks are numbered so that the column blocks and parts of the same 16 atoms are
// dispatched to the same XCD.
// Tile t of the mixing (16 atoms, one part, one block of 64 NB output channels); sA is the
// caller's LDS of 16 * 5 * (F + 4) floats.  256 threads.
template <int F, int NB>
__device__ __forceinline__ void mix_tile(const float *__restrict__ in, float *__restrict__ out, int64_t N,
                                         const float *__restrict__ B0, const float *__restrict__ B1,
                                         const float *__restrict__ B2, int accumulate, int ncb, int64_t t,
                                         float *__restrict__ sA, __bf16 *__restrict__ out16 = nullptr) {
  constexpr int LD = F + 4;
  constexpr int KC = F / 16;
  // this wave's weight fragments of its part stay in registers when they fit
  constexpr bool kBreg = KC * NB * 4 <= 64;
  const int64_t a0 = (t / (3 * ncb)) * 16;
  const int part = (int)(t % 3);
  const int cblk = (int)((t / 3) % ncb);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col0 = cblk * 64 * NB + wave * 16 * NB;
  const int64_t navail = N - a0 < 16 ? N - a0 : 16;
  const int r16 = lane & 15, q = lane >> 4;
  auto run = [&](auto c0_tag, auto nc_tag, const float *Bt) {
    constexpr int C0 = decltype(c0_tag)::value, NC = decltype(nc_tag)::value;
    float4 breg[kBreg ? KC : 1][NB];
    if constexpr (kBreg) load_bfrag<NB, KC>(Bt, F, col0, breg);   // overlaps the staging below
    // every load of the staging is issued before the first LDS write, so their latencies overlap
    const float4 *src = reinterpret_cast<const float4 *>(in + a0 * 9 * F);
    constexpr int NE = 16 * NC * (F / 4), IT = (NE + 255) / 256;
    float4 stage[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = threadIdx.x + 256 * it;
      const int row = e / (F / 4), c4 = e % (F / 4);   // row = atom * NC + coordinate
      const int at = row / NC, cc = row % NC;
      stage[it] = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < NE && at < navail) stage[it] = src[(at * 9 + C0 + cc) * (F / 4) + c4];
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = threadIdx.x + 256 * it;
      const int row = e / (F / 4), c4 = e % (F / 4);
      if (e < NE) *reinterpret_cast<float4 *>(sA + row * LD + 4 * c4) = stage[it];
    }
    __syncthreads();
    floatx4 acc[NC][NB];
    zero_acc_rb<NC, NB>(acc);
    if constexpr (kBreg)
      wave_mm_rows_breg<NC, NB, KC, true>(sA, NC * LD, LD, breg, acc);
    else
      wave_mm_rows<NC, NB, true>(sA, NC * LD, LD, F, Bt, col0, acc);
    mix_epilogue<F, NC, NB>(acc, out, out16, a0, C0, navail, col0, accumulate);
  };
  if (part == 0)
    run(std::integral_constant<int, 0>{}, std::integral_constant<int, 1>{}, B0);
  else if (part == 1)
    run(std::integral_constant<int, 1>{}, std::integral_constant<int, 3>{}, B1);
  else
    run(std::integral_constant<int, 4>{}, std::integral_constant<int, 5>{}, B2);
}

template <int F, int NB>
__global__ void __launch_bounds__(256) k_mix(const float *__restrict__ in, float *__restrict__ out, int64_t N,
                                             const float *__restrict__ B0, const float *__restrict__ B1,
                                             const float *__restrict__ B2, int accumulate, int ncb,
                                             int64_t ntiles, __bf16 *__restrict__ out16) {
  __shared__ __attribute__((aligned(16))) float sA[16 * 5 * (F + 4)];
  const int64_t per_xcd = (int64_t)gridDim.x / 8;
  const int64_t t = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (t >= ntiles) return;
  mix_tile<F, NB>(in, out, N, B0, B1, B2, accumulate, ncb, t, sA, out16);
}

template <int F, int NB>
inline int launch_mix(hipStream_t s, const float *in, float *out, int64_t N, const float *const Bt[3],
                      int accumulate, __bf16 *out16) {
  constexpr int ncb = F / (64 * NB);
  const int64_t ntiles = (N + 15) / 16 * ncb * 3;
  const int64_t grid = (ntiles + 7) / 8 * 8;
  hipLaunchKernelGGL((k_mix<F, NB>), dim3((unsigned)grid), dim3(256), 0, s, in, out, N, Bt[0], Bt[1], Bt[2],
                     accumulate, ncb, ntiles, out16);
  TN_LAUNCH_CHECK();
  return TN_OK;
}

// Four consecutive staging values of a mixing input: FP32 (float4), or BF16 (bf16x4) when the
// producer already rounded them, as the BF16 mixing would; stored to LDS as BF16.
template <class TI> struct Stage4;
template <> struct Stage4<float> {
  using type = float4;
  static __device__ __forceinline__ float4 zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
  static __device__ __forceinline__ bf16x4 to_bf16(const float4 &v) {
    bf16x4 o;
    o[0] = (__bf16)v.x;
    o[1] = (__bf16)v.y;
    o[2] = (__bf16)v.z;
    o[3] = (__bf16)v.w;
    return o;
  }
};
template <> struct Stage4<__bf16> {
  using type = bf16x4;
  static __device__ __forceinline__ bf16x4 zero() { return bf16x4{}; }
  static __device__ __forceinline__ bf16x4 to_bf16(const bf16x4 &v) { return v; }
};

// BF16 channel mixing (the BF16 precision mode): the tiles of mix_tile, with the part's
// coordinates rounded to BF16 as they are staged in LDS, BF16 weights held in registers
// (KC = F/32 fragments of 32 input channels per 16 output channels) and
// v_mfma_f32_16x16x32_bf16; FP32 accumulation, FP32 output (plus the optional BF16 copy).
// The input is FP32 or already BF16 (TI).  sA holds 16 * 5 * (F + kPadB) BF16 elements.
// 256 threads.
template <int F, int NB, class TI = float>
__device__ __forceinline__ void mix_tile_bf16(const TI *__restrict__ in, float *__restrict__ out, int64_t N,
                                              const __bf16 *__restrict__ B0, const __bf16 *__restrict__ B1,
                                              const __bf16 *__restrict__ B2, int accumulate, int ncb, int64_t t,
                                              __bf16 *__restrict__ sA, __bf16 *__restrict__ out16 = nullptr) {
  constexpr int LD = F + kPadB;
  constexpr int KC = F / 32;
  const int64_t a0 = (t / (3 * ncb)) * 16;
  const int part = (int)(t % 3);
  const int cblk = (int)((t / 3) % ncb);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col0 = cblk * 64 * NB + wave * 16 * NB;
  const int64_t navail = N - a0 < 16 ? N - a0 : 16;
  const int r16 = lane & 15, q = lane >> 4;
  auto run = [&](auto c0_tag, auto nc_tag, const __bf16 *Bt) {
    constexpr int C0 = decltype(c0_tag)::value, NC = decltype(nc_tag)::value;
    bf16x8 breg[KC][NB];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
        breg[kc][cb] = *reinterpret_cast<const bf16x8 *>(Bt + (size_t)(col0 + cb * 16 + r16) * F + 32 * kc + 8 * q);
    using S4 = Stage4<TI>;
    const typename S4::type *src = reinterpret_cast<const typename S4::type *>(in + a0 * 9 * F);
    constexpr int NE = 16 * NC * (F / 4), IT = (NE + 255) / 256;
    typename S4::type stage[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = threadIdx.x + 256 * it;
      const int row = e / (F / 4), c4 = e % (F / 4);   // row = atom * NC + coordinate
      const int at = row / NC, cc = row % NC;
      stage[it] = S4::zero();
      if (e < NE && at < navail) stage[it] = src[(at * 9 + C0 + cc) * (F / 4) + c4];
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int e = threadIdx.x + 256 * it;
      const int row = e / (F / 4), c4 = e % (F / 4);
      if (e < NE) *reinterpret_cast<bf16x4 *>(sA + row * LD + 4 * c4) = S4::to_bf16(stage[it]);
    }
    __syncthreads();
    floatx4 acc[NC][NB];
    zero_acc_rb<NC, NB>(acc);
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
      for (int rb = 0; rb < NC; ++rb) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(sA + (r16 * NC + rb) * LD + 32 * kc + 8 * q);
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) acc[rb][cb] = mfma_bf16(breg[kc][cb], a, acc[rb][cb]);
      }
    mix_epilogue<F, NC, NB>(acc, out, out16, a0, C0, navail, col0, accumulate);
  };
  if (part == 0)
    run(std::integral_constant<int, 0>{}, std::integral_constant<int, 1>{}, B0);
  else if (part == 1)
    run(std::integral_constant<int, 1>{}, std::integral_constant<int, 3>{}, B1);
  else
    run(std::integral_constant<int, 4>{}, std::integral_constant<int, 5>{}, B2);
}

template <int F, int NB, class TI>
__global__ void __launch_bounds__(256) k_mix_bf16(const TI *__restrict__ in, float *__restrict__ out, int64_t N,
                                                  const __bf16 *__restrict__ B0, const __bf16 *__restrict__ B1,
                                                  const __bf16 *__restrict__ B2, int accumulate, int ncb,
                                                  int64_t ntiles, __bf16 *__restrict__ out16) {
  __shared__ __attribute__((aligned(16))) __bf16 sA[16 * 5 * (F + kPadB)];
  const int64_t per_xcd = (int64_t)gridDim.x / 8;
  const int64_t t = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (t >= ntiles) return;
  mix_tile_bf16<F, NB, TI>(in, out, N, B0, B1, B2, accumulate, ncb, t, sA, out16);
}

// output channels per BF16 mixing workgroup: all F for F <= 128 (each staged part is read once)
template <int F>
struct MixBf16Shape {
  static constexpr int NB = F >= 128 ? 2 : 1;
  static constexpr int ncb = F / (64 * NB);
};

template <int F, class TI>
inline int launch_mix_bf16(hipStream_t s, const TI *in, float *out, int64_t N, const __bf16 *const Bt[3],
                           int accumulate, __bf16 *out16) {
  constexpr int NB = MixBf16Shape<F>::NB, ncb = MixBf16Shape<F>::ncb;
  const int64_t ntiles = (N + 15) / 16 * ncb * 3;
  const int64_t grid = (ntiles + 7) / 8 * 8;
  hipLaunchKernelGGL((k_mix_bf16<F, NB, TI>), dim3((unsigned)grid), dim3(256), 0, s, in, out, N, Bt[0], Bt[1], Bt[2],
                     accumulate, ncb, ntiles, out16);
  TN_LAUNCH_CHECK();
  return TN_OK;
}

// Persistent, software-pipelined mixing for F = 64 and 128 (all F output channels per
// workgroup): workgroup b takes one part, whose weight fragments it loads into registers once,
// and a contiguous range of 16-atom groups inside its XCD's share of the atoms; the next
// group's coordinates are loaded into registers while the current group is multiplied and
// stored.  The tiles and their arithmetic are those of mix_tile (BF = false: FP32 operands) and
// mix_tile_bf16 (BF = true: coordinates rounded to BF16 in LDS, BF16 weights), so the results
// are the same bits.  Part p gets Mp[p] workgroups per XCD (grid = 8 (Mp[0] + Mp[1] + Mp[2])),
// chosen so that every workgroup takes about the same time (mix_pipe_split).
struct MixPipeSplit {
  int Mp[3];
};
template <int F, int NB, bool BF, class TI = float>
__global__ void __launch_bounds__(256, 2) k_mix_pipe(const TI *__restrict__ in, float *__restrict__ out, int64_t N,
                                                  const void *B0, const void *B1, const void *B2, int accumulate,
                                                  MixPipeSplit sp, __bf16 *__restrict__ out16) {
  static_assert(F / (64 * NB) == 1, "one column block per workgroup");
  static_assert(BF || std::is_same<TI, float>::value, "BF16 inputs only for BF16 operands");
  using TS = typename std::conditional<BF, __bf16, float>::type;
  constexpr int LD = F + (BF ? kPadB : 4);
  __shared__ __attribute__((aligned(16))) TS sA[16 * 5 * LD];
  const int64_t G = (N + 15) / 16;
  const int xcd = blockIdx.x % 8, r = blockIdx.x / 8;
  const int part = r < sp.Mp[0] ? 0 : (r < sp.Mp[0] + sp.Mp[1] ? 1 : 2);
  const int m = part == 0 ? r : (part == 1 ? r - sp.Mp[0] : r - sp.Mp[0] - sp.Mp[1]);
  const int Mp = sp.Mp[part];   // workgroups of this part per XCD
  const int64_t gx0 = G * xcd / 8, gx1 = G * (xcd + 1) / 8;
  const int64_t g0 = gx0 + (gx1 - gx0) * m / Mp, g1 = gx0 + (gx1 - gx0) * (m + 1) / Mp;
  if (g0 >= g1) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r16 = lane & 15, q = lane >> 4;
  const int col0 = wave * 16 * NB;
  auto run = [&](auto c0_tag, auto nc_tag, const void *Bv) {
    constexpr int C0 = decltype(c0_tag)::value, NC = decltype(nc_tag)::value;
    constexpr int NE = 16 * NC * (F / 4), IT = (NE + 255) / 256;
    // this wave's weight fragments, once
    constexpr int KC = BF ? F / 32 : F / 16;
    using BFrag = typename std::conditional<BF, bf16x8, float4>::type;
    BFrag breg[KC][NB];
    if constexpr (BF) {
      const __bf16 *Bt = static_cast<const __bf16 *>(Bv);
#pragma unroll
      for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
          breg[kc][cb] = *reinterpret_cast<const bf16x8 *>(Bt + (size_t)(col0 + cb * 16 + r16) * F + 32 * kc + 8 * q);
    } else {
      load_bfrag<NB, KC>(static_cast<const float *>(Bv), F, col0, breg);
    }
    using S4 = Stage4<TI>;
    typename S4::type stage[IT];
    auto load = [&](int64_t g) {
      const int64_t a0 = g * 16;
      const int64_t navail = N - a0 < 16 ? N - a0 : 16;
      const typename S4::type *src = reinterpret_cast<const typename S4::type *>(in + a0 * 9 * F);
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int e = threadIdx.x + 256 * it;
        const int row = e / (F / 4), c4 = e % (F / 4);   // row = atom * NC + coordinate
        const int at = row / NC, cc = row % NC;
        stage[it] = S4::zero();
        if (e < NE && at < navail) stage[it] = src[(at * 9 + C0 + cc) * (F / 4) + c4];
      }
    };
    load(g0);
    for (int64_t g = g0; g < g1; ++g) {
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int e = threadIdx.x + 256 * it;
        const int row = e / (F / 4), c4 = e % (F / 4);
        if (e < NE) {
          if constexpr (BF) {
            *reinterpret_cast<bf16x4 *>(sA + row * LD + 4 * c4) = S4::to_bf16(stage[it]);
          } else {
            *reinterpret_cast<float4 *>(sA + row * LD + 4 * c4) = stage[it];
          }
        }
      }
      __syncthreads();
      if (g + 1 < g1) load(g + 1);   // in flight during this group's products and stores
      floatx4 acc[NC][NB];
      zero_acc_rb<NC, NB>(acc);
      if constexpr (BF) {
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
          for (int rb = 0; rb < NC; ++rb) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(sA + (r16 * NC + rb) * LD + 32 * kc + 8 * q);
#pragma unroll
            for (int cb = 0; cb < NB; ++cb) acc[rb][cb] = mfma_bf16(breg[kc][cb], a, acc[rb][cb]);
          }
      } else {
        wave_mm_rows_breg<NC, NB, KC, true>(sA, NC * LD, LD, breg, acc);
      }
      const int64_t a0 = g * 16;
      mix_epilogue<F, NC, NB>(acc, out, out16, a0, C0, N - a0 < 16 ? N - a0 : 16, col0, accumulate);
      __syncthreads();   // every wave has read sA before the next group is staged
    }
  };
  if (part == 0)
    run(std::integral_constant<int, 0>{}, std::integral_constant<int, 1>{}, B0);
  else if (part == 1)
    run(std::integral_constant<int, 1>{}, std::integral_constant<int, 3>{}, B1);
  else
    run(std::integral_constant<int, 4>{}, std::integral_constant<int, 5>{}, B2);
}

// k_mix_pipe's workgroups per XCD and part: 63 in all (two resident per CU, the launch bound's
// occupancy, over an XCD's 32 CUs).  A group of 16 atoms costs a fixed latency plus a time per
// coordinate (measured on a 100k-atom box at F = 128: about 0.94 + 1.84 NC us per group and
// workgroup with FP32 operands, 1.25 + 1.04 NC us with BF16), so the parts (NC = 1, 3, 5) get
// workgroups in proportion to those costs and every workgroup ends at about the same time.
// The pipelined kernel is used from 672 16-atom groups on; smaller inputs run one tile per
// workgroup (more tiles in parallel), which measured faster there (a 6000-atom box: 3.8
// against 4.1 ms per call).
inline MixPipeSplit mix_pipe_split(bool bf16) { return bf16 ? MixPipeSplit{{11, 21, 31}} : MixPipeSplit{{9, 21, 33}}; }
inline bool mix_pipe_pays(int64_t N) { return (N + 15) / 16 >= 672; }

template <int F, int NB, bool BF, class TI = float>
inline int launch_mix_pipe(hipStream_t s, const TI *in, float *out, int64_t N, const void *const Bt[3],
                           int accumulate, __bf16 *out16) {
  const MixPipeSplit sp = mix_pipe_split(BF);
  hipLaunchKernelGGL((k_mix_pipe<F, NB, BF, TI>), dim3((unsigned)(8 * (sp.Mp[0] + sp.Mp[1] + sp.Mp[2]))), dim3(256), 0, s,
                     in, out, N, Bt[0], Bt[1], Bt[2], accumulate, sp, out16);
  TN_LAUNCH_CHECK();
  return TN_OK;
}

inline bool aligned16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Per-part channel mixing of [N, 9, F] features: out[n,c,:] = W_part(c) in[n,c,:] (forward)
// or out[n,c,:] (+)= in[n,c,:] W_part(c) (adjoint).  WT holds the transposed matrices (used by
// the FP32 matrix-core kernel for the adjoint; may be null otherwise).  out16, when given (FP32
// matrix-core kernel only), receives a BF16 copy of out.
template <class T>
inline int mix(hipStream_t s, const T *in, T *out, int64_t N, int64_t F, const T *W[3], const T *WT[3], int adjoint,
               int accumulate, __bf16 *out16 = nullptr) {
  if (N <= 0) return TN_OK;
  if constexpr (sizeof(T) == 4) {
    const T *const *Bt = adjoint ? WT : W;
    bool ok = Bt != nullptr && aligned16(in) && aligned16(out);
    for (int q = 0; ok && q < 3; ++q) ok = Bt[q] != nullptr && aligned16(Bt[q]);
    const void *Bv[3] = {Bt[0], Bt[1], Bt[2]};
    const bool pipe = mix_pipe_pays(N);
    if (ok && F == 64)
      return pipe ? launch_mix_pipe<64, 1, false>(s, in, out, N, Bv, accumulate, out16)
                  : launch_mix<64, 1>(s, in, out, N, Bt, accumulate, out16);
    if (ok && F == 128)
      return pipe ? launch_mix_pipe<128, 2, false>(s, in, out, N, Bv, accumulate, out16)
                  : launch_mix<128, 2>(s, in, out, N, Bt, accumulate, out16);
    if (ok && F == 256) return launch_mix<256, 2>(s, in, out, N, Bt, accumulate, out16);
  }
  if (out16) return TN_E_UNSUPPORTED;
  GemmArgs<T> g;
  g.A = in; g.lda = 9 * F; g.C = out; g.ldc = 9 * F; g.transB = adjoint ? 0 : 1; g.ldb = F;
  g.M = N; g.N = F; g.K = F; g.zoff = F; g.zpart = 1; g.accumulate = accumulate;
  for (int q = 0; q < 3; ++q) g.Bz[q] = W[q];
  return gemm(s, g, 9);
}

// BF16 per-part channel mixing of [N, 9, F] features (see mix), FP32 or already rounded to BF16
// (TI, the same results): Bt[p] is W_p (forward) or its transpose (adjoint), BF16, 16-byte
// aligned.  F in {64, 128, 256}.
template <class TI>
inline int mix_bf16(hipStream_t s, const TI *in, float *out, int64_t N, int64_t F, const __bf16 *const Bt[3],
                    int accumulate, __bf16 *out16 = nullptr) {
  if (N <= 0) return TN_OK;
  bool ok = aligned16(in) && aligned16(out);
  for (int q = 0; ok && q < 3; ++q) ok = Bt[q] != nullptr && aligned16(Bt[q]);
  if (!ok) return TN_E_UNSUPPORTED;
  const void *Bv[3] = {Bt[0], Bt[1], Bt[2]};
  const bool pipe = mix_pipe_pays(N);
  if (F == 64)
    return pipe ? launch_mix_pipe<64, 1, true, TI>(s, in, out, N, Bv, accumulate, out16)
                : launch_mix_bf16<64, TI>(s, in, out, N, Bt, accumulate, out16);
  if (F == 128)
    return pipe ? launch_mix_pipe<128, 2, true, TI>(s, in, out, N, Bv, accumulate, out16)
                : launch_mix_bf16<128, TI>(s, in, out, N, Bt, accumulate, out16);
  if (F == 256) return launch_mix_bf16<256, TI>(s, in, out, N, Bt, accumulate, out16);
  return TN_E_UNSUPPORTED;
}

// ============================================================================ element kernels
__device__ inline bool pairs_ok(const int64_t *n_pairs, int64_t max_pairs) { return *n_pairs <= max_pairs; }

// Pairs a pair-indexed kernel works on: all of them, or none after a pair overflow (the
// neighbour search then leaves the internal pair list unwritten, so no entry may be read).
__device__ inline int64_t pair_bound(const int64_t *n_pairs, int64_t max_pairs) {
  const int64_t P = *n_pairs;
  return P <= max_pairs ? P : 0;
}

__device__ inline int clamp_z(int32_t z, int max_z) { return z < 0 ? 0 : (z >= max_z ? max_z - 1 : z); }

// Per pair: unit vector, distance, cutoff phi(d), exp-normal basis e_k(d).  Evaluated in
// FP64 from the (promoted) input positions and rounded once to T: the narrow Gaussians of
// the exp-normal basis amplify rounding in d by up to 2*alpha*beta*u*|u - mu_k|.
template <class T>
__global__ void k_geom(const int32_t *pairs, int64_t max_pairs, const int64_t *n_pairs, const T *pos, Lattice box,
                       double r_c, double r_lo, double alpha, const double *mu, const double *beta, int K, T *geo,
                       T *phi, T *rbf) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= pair_bound(n_pairs, max_pairs)) return;
  const int64_t i = pairs[p], j = pairs[max_pairs + p];
  double v[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) v[a] = (double)pos[3 * j + a] - (double)pos[3 * i + a];
  min_image(box, v[0], v[1], v[2]);
  const double d = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const double inv = 1.0 / d;
  geo[4 * p + 0] = (T)(v[0] * inv);
  geo[4 * p + 1] = (T)(v[1] * inv);
  geo[4 * p + 2] = (T)(v[2] * inv);
  geo[4 * p + 3] = (T)d;
  const double ph = 0.5 * (cos(M_PI * d / r_c) + 1.0);
  phi[p] = (T)ph;
  const double u = exp(-alpha * (d - r_lo));
  for (int k = 0; k < K; ++k) {
    const double t = u - mu[k];
    rbf[p * K + k] = (T)(ph * exp(-beta[k] * t * t));
  }
}

template <class TI, class TO>
__global__ void k_convert(int64_t n, const TI *in, TO *out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) out[t] = (TO)in[t];
}

// X_i = sum_j phi Z_ij (a 1 + b A0(u_ij) + c S0(u_ij)), one thread per (atom, channel).
template <class T>
__global__ void k_embed_gather(int64_t n, int F, const int32_t *rowptr, const int32_t *nbr, const int32_t *pid,
                               const int64_t *n_pairs, int64_t max_pairs, const int32_t *z, int max_z,
                               const T *U, const T *V, const T *geo, const T *phi, const T *f0, T *X) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F || !pairs_ok(n_pairs, max_pairs)) return;
  const int64_t i = t / F;
  const int f = (int)(t % F);
  const T ui = U[(int64_t)clamp_z(z[i], max_z) * F + f];
  T c[9] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
  for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const int32_t j = nbr[e];
    const int64_t p = pid[e];
    const T sg = (j > i) ? T(1) : T(-1);
    const T ux = sg * geo[4 * p], uy = sg * geo[4 * p + 1], uz = sg * geo[4 * p + 2];
    const T w = phi[p] * (ui + V[(int64_t)clamp_z(z[j], max_z) * F + f]);
    const T a = f0[p * 3 * F + f], b = f0[p * 3 * F + F + f], cc = f0[p * 3 * F + 2 * F + f];
    T s5[5];
    s0_coords(ux, uy, uz, s5);
    c[0] += w * a;
    c[1] += w * b * ux; c[2] += w * b * uy; c[3] += w * b * uz;
#pragma unroll
    for (int q = 0; q < 5; ++q) c[4 + q] += w * cc * s5[q];
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) X[i * 9 * F + q * F + f] = c[q];
}

template <class T>
__device__ inline void load9(const T *X, int64_t i, int F, int f, T c[9]) {
#pragma unroll
  for (int q = 0; q < 9; ++q) c[q] = X[i * 9 * F + q * F + f];
}
template <class T>
__device__ inline void store9(T *X, int64_t i, int F, int f, const T c[9]) {
#pragma unroll
  for (int q = 0; q < 9; ++q) X[i * 9 * F + q * F + f] = c[q];
}

// Norms in T of features stored as TX (the FP64 island reads FP32 features directly).
template <class T, class TX>
__device__ inline void node_norm_at(int64_t t, int F, const TX *X, T *nrm) {
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T c[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) c[q] = (T)X[i * 9 * F + q * F + f];
  nrm[i * F + f] = norm9(c);
}
template <class T, class TX = T>
__global__ void k_node_norm(int64_t n, int F, const TX *X, T *nrm) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  node_norm_at<T, TX>(t, F, X, nrm);
}

// Block-wide sum (blockDim.x threads, power of two <= 1024).
template <class T>
__device__ inline T block_sum(T v, T *lds) {
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) lds[threadIdx.x] += lds[threadIdx.x + s];
    __syncthreads();
  }
  T r = lds[0];
  __syncthreads();
  return r;
}

// Sum over the 64 lanes in the order of a 64-thread shared-memory tree (pairs at distance 32,
// then 16, ...); every lane receives the result.
template <class T>
__device__ __forceinline__ T lane_shfl_down(T v, int off) { return __shfl_down(v, off, 64); }
template <class T>
__device__ __forceinline__ T lane_shfl(T v, int src) { return __shfl(v, src, 64); }
template <class T>
__device__ __forceinline__ T wave_tree_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += lane_shfl_down(v, off);
  return lane_shfl(v, 0);
}

// LayerNorm of row r (length C; population variance, eps 1e-5, affine g/b) by one wave: lane l
// sums entries l, l + 64, ..., and the lanes' sums meet in the 64-lane tree.
template <class TA>
__device__ inline void layernorm_row_wave(int64_t r, int C, const TA *x, const TA *gmul, const TA *badd, TA *y,
                                          TA *xhat, TA *rstd) {
  const int lane = threadIdx.x & 63;
  TA s = TA(0);
  for (int k = lane; k < C; k += 64) s += x[r * C + k];
  const TA mean = wave_tree_sum(s) / TA(C);
  TA v = TA(0);
  for (int k = lane; k < C; k += 64) {
    const TA d = x[r * C + k] - mean;
    v += d * d;
  }
  const TA var = wave_tree_sum(v) / TA(C);
  const TA rs = TA(1) / dsqrt(var + TA(1e-5));
  for (int k = lane; k < C; k += 64) {
    const TA hh = (x[r * C + k] - mean) * rs;
    xhat[r * C + k] = hh;
    y[r * C + k] = hh * gmul[k] + badd[k];
  }
  if (lane == 0) rstd[r] = rs;
}

// Its adjoint: dx = rstd * (g*dy - mean(g*dy) - xhat * mean(g*dy*xhat)).
template <class TA>
__device__ inline void layernorm_bwd_row_wave(int64_t r, int C, const TA *dy, const TA *xhat, const TA *rstd,
                                              const TA *gmul, TA *dx) {
  const int lane = threadIdx.x & 63;
  TA s1 = TA(0), s2 = TA(0);
  for (int k = lane; k < C; k += 64) {
    const TA gd = gmul[k] * dy[r * C + k];
    s1 += gd;
    s2 += gd * xhat[r * C + k];
  }
  const TA m1 = wave_tree_sum(s1) / TA(C);
  const TA m2 = wave_tree_sum(s2) / TA(C);
  const TA rs = rstd[r];
  for (int k = lane; k < C; k += 64) dx[r * C + k] = rs * (gmul[k] * dy[r * C + k] - m1 - xhat[r * C + k] * m2);
}

// The grid kernels: one wave per row, four rows per 256-thread block.
template <class T>
__global__ void __launch_bounds__(256) k_layernorm(int64_t rows, int C, const T *x, const T *gmul, const T *badd,
                                                   T *y, T *xhat, T *rstd) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  layernorm_row_wave<T>(r, C, x, gmul, badd, y, xhat, rstd);
}

template <class T>
__global__ void __launch_bounds__(256) k_layernorm_bwd(int64_t rows, int C, const T *dy, const T *xhat,
                                                       const T *rstd, const T *gmul, T *dx) {
  const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= rows) return;
  layernorm_bwd_row_wave<T>(r, C, dy, xhat, rstd, gmul, dx);
}

inline unsigned layernorm_grid(int64_t rows) { return (unsigned)((rows + 3) / 4); }

// X = g_part(c) * T0 (gating), product in T, features stored as TX.
template <class T, class TX>
__device__ inline void gate_at(int64_t t, int F, const T *g, const TX *T0, TX *X) {
  const int64_t i = t / (9 * F);
  const int rem = (int)(t % (9 * F));
  const int q = rem / F, f = rem % F;
  X[t] = (TX)(g[i * 3 * F + coord_part(q) * F + f] * (T)T0[t]);
}
template <class T, class TX = T>
__global__ void k_gate(int64_t n, int F, const T *g, const TX *T0, TX *X) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * 9 * F) return;
  gate_at<T, TX>(t, F, g, T0, X);
}

// X = g_part(c) * T0 (gating) followed by the first layer's normalisation:
// nX = ||X||, Xb = X / (||X|| + 1).  One thread per (atom, channel); products in T.
template <class T, class TX>
__device__ inline void gate_normalize_at(int64_t t, int F, const T *g, const TX *T0, TX *X, TX *nX, TX *Xb) {
  const int64_t i = t / F;
  const int f = (int)(t % F);
  TX c[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int64_t o = i * 9 * F + q * F + f;
    c[q] = (TX)(g[i * 3 * F + coord_part(q) * F + f] * (T)T0[o]);
    X[o] = c[q];
  }
  const TX nn = norm9(c);
  nX[i * F + f] = nn;
  const TX sc = TX(1) / (nn + TX(1));
#pragma unroll
  for (int q = 0; q < 9; ++q) Xb[i * 9 * F + q * F + f] = c[q] * sc;
}
template <class T, class TX>
__global__ void k_gate_normalize(int64_t n, int F, const T *g, const TX *T0, TX *X, TX *nX, TX *Xb) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  gate_normalize_at<T, TX>(t, F, g, T0, X, nX, Xb);
}

template <class T>
__device__ inline void normalize_at(int64_t t, int F, const T *X, T *nX, T *Xb) {
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T c[9];
  load9(X, i, F, f, c);
  const T nn = norm9(c);
  nX[i * F + f] = nn;
  const T s = T(1) / (nn + T(1));
#pragma unroll
  for (int q = 0; q < 9; ++q) c[q] *= s;
  store9(Xb, i, F, f, c);
}
template <class T>
__global__ void k_normalize(int64_t n, int F, const T *X, T *nX, T *Xb) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  normalize_at<T>(t, F, X, nX, Xb);
}

// M_i (+)= sum_j h_part(c)(d_ij) * Y_j[c] over the CSR row of i.
template <class T>
__global__ void k_message(int64_t n, int F, const int32_t *rowptr, const int32_t *nbr, const int32_t *pid,
                          const int64_t *n_pairs, int64_t max_pairs, const T *h, const T *Y, T *M, int accumulate) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F || !pairs_ok(n_pairs, max_pairs)) return;
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T c[9] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
  for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const int64_t j = nbr[e];
    const int64_t p = pid[e];
    const T hI = h[p * 3 * F + f], hA = h[p * 3 * F + F + f], hS = h[p * 3 * F + 2 * F + f];
    const T *y = Y + j * 9 * F + f;
    c[0] += hI * y[0];
#pragma unroll
    for (int q = 1; q < 4; ++q) c[q] += hA * y[q * F];
#pragma unroll
    for (int q = 4; q < 9; ++q) c[q] += hS * y[q * F];
  }
  if (accumulate) {
#pragma unroll
    for (int q = 0; q < 9; ++q) M[i * 9 * F + q * F + f] += c[q];
  } else {
    store9(M, i, F, f, c);
  }
}

// P = Y M + M Y, Pb = P / (||P|| + 1)
template <class T>
__global__ void k_product(int64_t n, int F, const T *Y, const T *M, T *P, T *nP, T *Pb) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T yc[9], mc[9], Ym[9], Mm[9], A1[9], A2[9], pc[9];
  load9(Y, i, F, f, yc);
  load9(M, i, F, f, mc);
  rec(yc, Ym);
  rec(mc, Mm);
  mm(Ym, Mm, A1);
  mm(Mm, Ym, A2);
#pragma unroll
  for (int q = 0; q < 9; ++q) A1[q] += A2[q];
  dec(A1, pc);
  store9(P, i, F, f, pc);
  const T nn = norm9(pc);
  nP[i * F + f] = nn;
  const T s = T(1) / (nn + T(1));
#pragma unroll
  for (int q = 0; q < 9; ++q) pc[q] *= s;
  store9(Pb, i, F, f, pc);
}

// Message and product in one pass: M_i = sum_j h_part(c) * Y_j[c] over the CSR row of i,
// then P = Y M + M Y and Pb = P / (||P|| + 1).  Writes M, P, ||P|| and Pb.
template <class T>
__global__ void k_message_product(int64_t n, int F, const int32_t *rowptr, const int32_t *nbr, const int32_t *pid,
                                  const int64_t *n_pairs, int64_t max_pairs, const T *h, const T *Y, T *M, T *P,
                                  T *nP, T *Pb) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F || !pairs_ok(n_pairs, max_pairs)) return;
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T mc[9] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
  for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
    const int64_t j = nbr[e];
    const int64_t p = pid[e];
    const T hI = h[p * 3 * F + f], hA = h[p * 3 * F + F + f], hS = h[p * 3 * F + 2 * F + f];
    const T *y = Y + j * 9 * F + f;
    mc[0] += hI * y[0];
#pragma unroll
    for (int q = 1; q < 4; ++q) mc[q] += hA * y[q * F];
#pragma unroll
    for (int q = 4; q < 9; ++q) mc[q] += hS * y[q * F];
  }
  store9(M, i, F, f, mc);
  T yc[9], Ym[9], Mm[9], A1[9], A2[9], pc[9];
  load9(Y, i, F, f, yc);
  rec(yc, Ym);
  rec(mc, Mm);
  mm(Ym, Mm, A1);
  mm(Mm, Ym, A2);
#pragma unroll
  for (int q = 0; q < 9; ++q) A1[q] += A2[q];
  dec(A1, pc);
  store9(P, i, F, f, pc);
  const T nn = norm9(pc);
  nP[i * F + f] = nn;
  const T sc = T(1) / (nn + T(1));
#pragma unroll
  for (int q = 0; q < 9; ++q) pc[q] *= sc;
  store9(Pb, i, F, f, pc);
}

// X_out = Xb + D + D D, and for the next layer ||X_out|| and X_out / (||X_out|| + 1).
template <class T>
__device__ inline void residual_normalize_at(int64_t t, int F, const T *Xb, const T *D, T *Xo, T *nXo, T *Xbo) {
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T dc[9], Dm[9], Q[9], qc[9], xb[9];
  load9(D, i, F, f, dc);
  load9(Xb, i, F, f, xb);
  rec(dc, Dm);
  mm(Dm, Dm, Q);
  dec(Q, qc);
#pragma unroll
  for (int q = 0; q < 9; ++q) xb[q] += dc[q] + qc[q];
  store9(Xo, i, F, f, xb);
  const T nn = norm9(xb);
  nXo[i * F + f] = nn;
  const T sc = T(1) / (nn + T(1));
#pragma unroll
  for (int q = 0; q < 9; ++q) xb[q] *= sc;
  store9(Xbo, i, F, f, xb);
}
template <class T>
__global__ void k_residual_normalize(int64_t n, int F, const T *Xb, const T *D, T *Xo, T *nXo, T *Xbo) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  residual_normalize_at<T>(t, F, Xb, D, Xo, nXo, Xbo);
}

// X_out = Xb + D + D D
template <class T>
__device__ inline void residual_at(int64_t t, int F, const T *Xb, const T *D, T *Xo) {
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T dc[9], Dm[9], Q[9], qc[9], xb[9];
  load9(D, i, F, f, dc);
  load9(Xb, i, F, f, xb);
  rec(dc, Dm);
  mm(Dm, Dm, Q);
  dec(Q, qc);
#pragma unroll
  for (int q = 0; q < 9; ++q) xb[q] += dc[q] + qc[q];
  store9(Xo, i, F, f, xb);
}
template <class T>
__global__ void k_residual(int64_t n, int F, const T *Xb, const T *D, T *Xo) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  residual_at<T>(t, F, Xb, D, Xo);
}

template <class T, class TX>
__device__ inline void out_norms_at(int64_t t, int F, const TX *X, T *on) {
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T c[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) c[q] = (T)X[i * 9 * F + q * F + f];
  on[i * 3 * F + f] = norm_I(c);
  on[i * 3 * F + F + f] = norm_A(c);
  on[i * 3 * F + 2 * F + f] = norm_S(c);
}
template <class T, class TX = T>
__global__ void k_out_norms(int64_t n, int F, const TX *X, T *on) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  out_norms_at<T, TX>(t, F, X, on);
}

// eps_i = w . hx_i + b (final scalar of the output network)

// First index i in [0, n) with batch[i] >= key (n if none) for a sorted batch vector, found by
// the whole block: each round probes blockDim.x evenly spaced entries at once and keeps the gap
// where the comparison changes, so a few thousand atoms take two rounds of parallel loads
// instead of a dozen dependent ones.  Every thread of the block must call it.
__device__ inline int64_t block_lower_bound(const int32_t *batch, int64_t n, int32_t key) {
  int64_t a = 0, e = n;   // the answer lies in [a, e]
  while (a < e) {
    const int64_t step = (e - a + blockDim.x - 1) / blockDim.x;
    const int64_t p = a + (int64_t)threadIdx.x * step;
    const int c = __syncthreads_count(p < e && batch[p] < key);   // the true probes form a prefix
    if (c == 0) break;                                              // batch[a] >= key
    const int64_t last = a + (int64_t)(c - 1) * step;               // batch[last] < key
    const int64_t next = a + (int64_t)c * step;                     // batch[next] >= key, or past e
    a = last + 1;
    if (next < e) e = next;
  }
  return a;
}

// E_s = sum over the (contiguous) atoms of system s, in FP64; one block per system.
template <class T>
__global__ void __launch_bounds__(128) k_energy_reduce(int64_t n, const T *eps, const int32_t *batch, double *E,
                                                       int32_t *status) {
  __shared__ double lds[128];
  const int32_t s = blockIdx.x;
  const int64_t lo = block_lower_bound(batch, n, s);
  const int64_t hi = block_lower_bound(batch, n, s + 1);
  // thread t adds atoms lo + t, lo + t + 128, ... in that order; sixteen loads are issued at a
  // time (unconditionally, the index clamped in range), so a large system does not wait for
  // one load per term
  double acc = 0.0;
  for (int64_t i0 = lo + threadIdx.x; i0 < hi; i0 += 128 * 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t i = i0 + 128 * u;
      v[u] = (double)eps[i < hi ? i : hi - 1];
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (i0 + 128 * u < hi) acc += v[u];
  }
  const double tot = block_sum(acc, lds);
  if (threadIdx.x == 0) {
    E[s] = tot;
    if (!isfinite(tot)) set_status(status, TN_STATUS_NONFINITE);
  }
}

// ----------------------------------------------------------------------------- backward kernels
template <class T>
__device__ inline void out_final_bwd_at(int64_t t, int H, const T *hz, const T *w, T *dhz) {
  const int k = (int)(t % H);
  dhz[t] = w[k] * silu_grad(hz[t]);
}
template <class T>
__global__ void k_out_final_bwd(int64_t n, int H, const T *hz, const T *w, T *dhz) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * H) return;
  out_final_bwd_at<T>(t, H, hz, w, dhz);
}

// adjoint of the part norms: dX = sum_part d(norm_part) * grad(norm_part)
template <class T, class TX>
__device__ inline void out_norms_bwd_at(int64_t t, int F, const TX *X, const T *don, TX *dX) {
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T c[9], d[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) c[q] = (T)X[i * 9 * F + q * F + f];
  norm_grad_parts(c, don[i * 3 * F + f], don[i * 3 * F + F + f], don[i * 3 * F + 2 * F + f], d);
#pragma unroll
  for (int q = 0; q < 9; ++q) dX[i * 9 * F + q * F + f] = (TX)d[q];
}
template <class T, class TX = T>
__global__ void k_out_norms_bwd(int64_t n, int F, const TX *X, const T *don, TX *dX) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  out_norms_bwd_at<T, TX>(t, F, X, don, dX);
}

// X_out = Xb + D + DD:  dD = dX + rec^T(dQ D^T + D^T dQ) with dQ = dec^T(dX)
// dD in T or, for a consumer that rounds it to BF16 anyway, BF16 (TO)
template <class T, class TO = T>
__device__ inline void residual_bwd_at(int64_t t, int F, const T *D, const T *dX, TO *dD) {
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T dc[9], Dm[9], g[9], dQ[9], A1[9], A2[9], r[9];
  load9(D, i, F, f, dc);
  load9(dX, i, F, f, g);
  rec(dc, Dm);
  dec_adj(g, dQ);
  mmt(dQ, Dm, A1);
  mtm(Dm, dQ, A2);
#pragma unroll
  for (int q = 0; q < 9; ++q) A1[q] += A2[q];
  rec_adj(A1, r);
#pragma unroll
  for (int q = 0; q < 9; ++q) dD[i * 9 * F + q * F + f] = (TO)(r[q] + g[q]);
}
template <class T, class TO = T>
__global__ void k_residual_bwd(int64_t n, int F, const T *D, const T *dX, TO *dD) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  residual_bwd_at<T, TO>(t, F, D, dX, dD);
}

// P = Y M + M Y for one channel (the product of the interaction layer), from the nine
// coordinates of Y and M to those of P.
template <class T>
__device__ __forceinline__ void sym_product(const T y9[9], const T m9[9], T p9[9]) {
  T Ym[9], Mm[9], A1[9], A2[9];
  rec(y9, Ym);
  rec(m9, Mm);
  mm(Ym, Mm, A1);
  mm(Mm, Ym, A2);
#pragma unroll
  for (int q = 0; q < 9; ++q) A1[q] += A2[q];
  dec(A1, p9);
}

// Through Pb = P/(||P||+1) and P = Y M + M Y: dY (overwritten) and dM.  With P null, P and
// ||P|| are formed again from Y and M (sym_product, norm9: the forward's arithmetic) instead
// of being read.
template <class T>
__device__ inline void product_bwd_at(int64_t t, int F, const T *dPb, const T *P, const T *nP, const T *Y, const T *M, T *dY, T *dM,
                               __bf16 *dM16 = nullptr) {
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T g[9], pc[9], gn[9];
  load9(dPb, i, F, f, g);
  T pn;
  if (P) {
    load9(P, i, F, f, pc);
    pn = nP[i * F + f];
  } else {
    T y9[9], m9[9];
    load9(Y, i, F, f, y9);
    load9(M, i, F, f, m9);
    sym_product(y9, m9, pc);
    pn = norm9(pc);
  }
  const T s = T(1) / (pn + T(1));
  T dot = T(0);
#pragma unroll
  for (int q = 0; q < 9; ++q) dot += g[q] * pc[q];
  norm_grad_parts(pc, T(1), T(1), T(1), gn);
  T dp[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) dp[q] = g[q] * s - dot * s * s * gn[q];
  T dPm[9], yc[9], mc[9], Ym[9], Mm[9], A1[9], A2[9], r[9];
  dec_adj(dp, dPm);
  load9(Y, i, F, f, yc);
  load9(M, i, F, f, mc);
  rec(yc, Ym);
  rec(mc, Mm);
  // dY = dP M^T + M^T dP
  mmt(dPm, Mm, A1);
  mtm(Mm, dPm, A2);
#pragma unroll
  for (int q = 0; q < 9; ++q) A1[q] += A2[q];
  rec_adj(A1, r);
  store9(dY, i, F, f, r);
  // dM = Y^T dP + dP Y^T
  mtm(Ym, dPm, A1);
  mmt(dPm, Ym, A2);
#pragma unroll
  for (int q = 0; q < 9; ++q) A1[q] += A2[q];
  rec_adj(A1, r);
  store9(dM, i, F, f, r);
  if constexpr (std::is_same<T, float>::value) {
    if (dM16) {
#pragma unroll
      for (int q = 0; q < 9; ++q) dM16[i * 9 * F + q * F + f] = (__bf16)r[q];
    }
  }
}
// dM16, when given, receives a BF16 copy of dM.
template <class T>
__global__ void k_product_bwd(int64_t n, int F, const T *dPb, const T *P, const T *nP, const T *Y, const T *M,
                              T *dY, T *dM, __bf16 *dM16) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  product_bwd_at<T>(t, F, dPb, P, nP, Y, M, dY, dM, dM16);
}

// dh[p] from both directions of pair p = (i, j): <part(Y_j), dM_i> + <part(Y_i), dM_j> per channel.
template <class T>
__global__ void k_message_bwd_pair(const int32_t *pairs, int64_t max_pairs, const int64_t *n_pairs, int F,
                                   const T *Y, const T *dM, T *dh) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t p = t / F;
  if (p >= pair_bound(n_pairs, max_pairs)) return;
  const int f = (int)(t % F);
  const int64_t i = pairs[p], j = pairs[max_pairs + p];
  const T *yi = Y + i * 9 * F + f, *yj = Y + j * 9 * F + f;
  const T *gi = dM + i * 9 * F + f, *gj = dM + j * 9 * F + f;
  T s[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int q = 0; q < 9; ++q) s[coord_part(q)] += yj[q * F] * gi[q * F] + yi[q * F] * gj[q * F];
  dh[p * 3 * F + f] = s[0];
  dh[p * 3 * F + F + f] = s[1];
  dh[p * 3 * F + 2 * F + f] = s[2];
}

// through Xb = X/(||X||+1): dX = dXb/(n+1) - <dXb, X>/(n+1)^2 grad||X||   (in place on g)
template <class T>
__device__ inline void normalize_bwd_at(int64_t t, int F, const T *X, const T *nX, T *g) {
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T c[9], d[9], gn[9];
  load9(X, i, F, f, c);
  load9(g, i, F, f, d);
  const T s = T(1) / (nX[i * F + f] + T(1));
  T dot = T(0);
#pragma unroll
  for (int q = 0; q < 9; ++q) dot += d[q] * c[q];
  norm_grad_parts(c, T(1), T(1), T(1), gn);
#pragma unroll
  for (int q = 0; q < 9; ++q) d[q] = d[q] * s - dot * s * s * gn[q];
  store9(g, i, F, f, d);
}
template <class T>
__global__ void k_normalize_bwd(int64_t n, int F, const T *X, const T *nX, T *g) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  normalize_bwd_at<T>(t, F, X, nX, g);
}

// h = phi * silu(z3):  dz3 = dh * phi * silu'(z3);  dphi += sum dh * silu(z3).  One block per pair.
template <class T>
__global__ void __launch_bounds__(128) k_edge_bwd_top(int64_t max_pairs, const int64_t *n_pairs, int C,
                                                      const T *dh, const T *z3, const T *phi, T *dz3, T *dphi) {
  __shared__ T lds[128];
  const int64_t p = blockIdx.x;
  if (p >= pair_bound(n_pairs, max_pairs)) return;
  const T ph = phi[p];
  T acc = T(0);
  for (int k = threadIdx.x; k < C; k += 128) {
    const T zz = z3[p * C + k], g = dh[p * C + k];
    dz3[p * C + k] = g * ph * silu_grad(zz);
    acc += g * silu(zz);
  }
  const T tot = block_sum(acc, lds);
  if (threadIdx.x == 0) dphi[p] += tot;
}

// X0 = g * T0 (per part):  dg[part] = sum_{c in part} dX0_c T0_c;  dT0 = g dX0
// With ez given, dg leaves multiplied by silu'(ez) (the adjoint of the MLP's last SiLU).
// dT0 in TX or, for a consumer that rounds it to BF16 anyway, BF16 (TO)
template <class T, class TX, class TO = TX>
__device__ inline void gate_bwd_at(int64_t t, int F, const TX *dX, const TX *T0, const T *g, T *dg, TO *dT0,
                                   const T *ez) {
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T s[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int64_t o = i * 9 * F + q * F + f;
    const int pt = coord_part(q);
    s[pt] += (T)dX[o] * (T)T0[o];
    dT0[o] = (TO)(TX)(g[i * 3 * F + pt * F + f] * (T)dX[o]);
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int64_t o = i * 3 * F + q * F + f;
    dg[o] = ez ? s[q] * silu_grad(ez[o]) : s[q];
  }
}
template <class T, class TX = T, class TO = TX>
__global__ void k_gate_bwd(int64_t n, int F, const TX *dX, const TX *T0, const T *g, T *dg, TO *dT0,
                           const T *ez = nullptr) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  gate_bwd_at<T, TX, TO>(t, F, dX, T0, g, dg, dT0, ez);
}

template <class T>
__global__ void k_mul_silu_grad(int64_t n, const T *d, const T *zz, T *out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  out[t] = d[t] * silu_grad(zz[t]);
}

// dX += dn * grad||X||
template <class T, class TX>
__device__ inline void norm_bwd_add_at(int64_t t, int F, const TX *X, const T *dn, TX *dX) {
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T c[9], gn[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) c[q] = (T)X[i * 9 * F + q * F + f];
  const T s = dn[i * F + f];
  norm_grad_parts(c, s, s, s, gn);
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    TX &d = dX[i * 9 * F + q * F + f];
    d = (TX)((T)d + gn[q]);
  }
}
template <class T, class TX = T>
__global__ void k_norm_bwd_add(int64_t n, int F, const TX *X, const T *dn, TX *dX) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  norm_bwd_add_at<T, TX>(t, F, X, dn, dX);
}

// Embedding adjoint per pair (one block per pair, threads over channels):
// df0 = (da, db, dc), dphi += ..., dvhat = ...
template <class T>
__global__ void __launch_bounds__(128) k_embed_bwd_pair(const int32_t *pairs, int64_t max_pairs,
                                                        const int64_t *n_pairs, int F, const int32_t *z, int max_z,
                                                        const T *U, const T *V, const T *geo, const T *phi,
                                                        const T *f0, const T *dXr, T *df0, T *dphi, T *dvhat) {
  __shared__ T lds[128];
  const int64_t p = blockIdx.x;
  if (p >= pair_bound(n_pairs, max_pairs)) return;
  const int64_t i = pairs[p], j = pairs[max_pairs + p];
  const int zi = clamp_z(z[i], max_z), zj = clamp_z(z[j], max_z);
  const T ux = geo[4 * p], uy = geo[4 * p + 1], uz = geo[4 * p + 2];
  const T ph = phi[p];
  T s5[5];
  s0_coords(ux, uy, uz, s5);
  T aphi = T(0), av[3] = {T(0), T(0), T(0)};
  for (int f = threadIdx.x; f < F; f += 128) {
    const T Zij = U[(int64_t)zi * F + f] + V[(int64_t)zj * F + f];
    const T Zji = U[(int64_t)zj * F + f] + V[(int64_t)zi * F + f];
    const T a = f0[p * 3 * F + f], b = f0[p * 3 * F + F + f], c = f0[p * 3 * F + 2 * F + f];
    T di[9], dj[9];
    load9(dXr, i, F, f, di);
    load9(dXr, j, F, f, dj);
    const T gi0 = di[0], gj0 = dj[0];
    const T giA = di[1] * ux + di[2] * uy + di[3] * uz;
    const T gjA = -(dj[1] * ux + dj[2] * uy + dj[3] * uz);
    T giS = T(0), gjS = T(0);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      giS += di[4 + q] * s5[q];
      gjS += dj[4 + q] * s5[q];
    }
    df0[p * 3 * F + f] = ph * (Zij * gi0 + Zji * gj0);
    df0[p * 3 * F + F + f] = ph * (Zij * giA + Zji * gjA);
    df0[p * 3 * F + 2 * F + f] = ph * (Zij * giS + Zji * gjS);
    aphi += Zij * (a * gi0 + b * giA + c * giS) + Zji * (a * gj0 + b * gjA + c * gjS);
    T gsi[3], gsj[3];
    s0_dot_grad(di + 4, ux, uy, uz, gsi);
    s0_dot_grad(dj + 4, ux, uy, uz, gsj);
#pragma unroll
    for (int q = 0; q < 3; ++q)
      av[q] += ph * (b * (Zij * di[1 + q] - Zji * dj[1 + q]) + c * (Zij * gsi[q] + Zji * gsj[q]));
  }
  const T tphi = block_sum(aphi, lds);
  T tv[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) tv[q] = block_sum(av[q], lds);
  if (threadIdx.x == 0) {
    dphi[p] += tphi;
    dvhat[3 * p] = tv[0];
    dvhat[3 * p + 1] = tv[1];
    dvhat[3 * p + 2] = tv[2];
  }
}

// Per pair: g = dE/dv from dE/de_k, dE/dphi and dE/dvhat.
template <class T>
__global__ void k_geom_bwd(int64_t max_pairs, const int64_t *n_pairs, T r_c, T r_lo, T alpha, const T *mu,
                           const T *beta, int K, const T *geo, const T *de, const T *dphi, const T *dvhat, T *gpair) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= pair_bound(n_pairs, max_pairs)) return;
  const T ux = geo[4 * p], uy = geo[4 * p + 1], uz = geo[4 * p + 2], d = geo[4 * p + 3];
  const T arg = T(M_PI) * d / r_c;
  const T ph = T(0.5) * (dcos(arg) + T(1));
  const T dph = -T(0.5) * T(M_PI) / r_c * dsin(arg);
  const T u = dexp(-alpha * (d - r_lo));
  T dd = dphi[p] * dph;
  for (int k = 0; k < K; ++k) {
    const T t = u - mu[k];
    const T gk = dexp(-beta[k] * t * t);
    const T dek = dph * gk + ph * gk * T(2) * alpha * beta[k] * u * t;
    dd += de[p * K + k] * dek;
  }
  const T gx = dvhat[3 * p], gy = dvhat[3 * p + 1], gz = dvhat[3 * p + 2];
  const T proj = gx * ux + gy * uy + gz * uz;
  const T inv = T(1) / d;
  gpair[3 * p] = dd * ux + (gx - proj * ux) * inv;
  gpair[3 * p + 1] = dd * uy + (gy - proj * uy) * inv;
  gpair[3 * p + 2] = dd * uz + (gz - proj * uz) * inv;
}

// F_i = sum over the CSR row of i of +-g_pair, accumulated in FP64.
template <class T, class TO>
__global__ void k_force_gather(int64_t n, const int32_t *rowptr, const int32_t *nbr, const int32_t *pid,
                               const int64_t *n_pairs, int64_t max_pairs, const T *gpair, const int32_t *perm,
                               TO *forces) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  if (pairs_ok(n_pairs, max_pairs)) {
    for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
      const int64_t p = pid[e];
      const double sg = (nbr[e] > i) ? 1.0 : -1.0;
      fx += sg * (double)gpair[3 * p];
      fy += sg * (double)gpair[3 * p + 1];
      fz += sg * (double)gpair[3 * p + 2];
    }
  }
  const int64_t o = perm ? perm[i] : i;
  forces[3 * o] = (TO)fx;
  forces[3 * o + 1] = (TO)fy;
  forces[3 * o + 2] = (TO)fz;
}

// out[perm[i]] = in[i]  (back to the caller's atom order)
template <class T>
__global__ void k_unpermute(int64_t n, const int32_t *perm, const T *in, T *out) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[perm[i]] = in[i];
}


// ============================================================================ wave-per-atom gathers
// FP32 gathers over the CSR rows with one wave per atom: the row is wave-uniform, so its
// indices and per-pair scalars come through scalar loads, and lane l owns the V channels
// V*l .. V*l+V-1 (F = 64 V), read with one vector access per coordinate.  Four atoms per
// 256-thread block, numbered per XCD.
__device__ __forceinline__ int32_t wave_atom() {
  return __builtin_amdgcn_readfirstlane((int32_t)(xcd_block() * 4 + (threadIdx.x >> 6)));
}

inline unsigned wave_atom_grid(int64_t n) { return (unsigned)((n + 3) / 4); }

// The gathers below split an atom's channels over G waves (F = 64 V G): wave g of the atom's
// group owns channels (64 g + l) V .. +V-1.  More waves per atom keep more loads in flight
// when there are few atoms per compute unit.
template <int G>
__device__ __forceinline__ int32_t group_atom() {
  return __builtin_amdgcn_readfirstlane((int32_t)(xcd_block() * (4 / G) + (threadIdx.x >> 6) / G));
}
template <int V, int G>
__device__ __forceinline__ int group_channel() {
  return ((((int)threadIdx.x >> 6) % G) * 64 + ((int)threadIdx.x & 63)) * V;
}

// V consecutive values of a per-pair array stored as float or BF16, as floats.
template <int V>
__device__ __forceinline__ void ld_pair_row(const float *p, float (&o)[V]) {
  ldv<V>(p, o);
}
template <int V>
__device__ __forceinline__ void ld_pair_row(const __bf16 *p, float (&o)[V]) {
  if constexpr (V == 2) {   // one 4-byte access (p is 4-byte aligned: even channel offsets)
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const bf16x2 v = *reinterpret_cast<const bf16x2 *>(p);
    o[0] = (float)v[0];
    o[1] = (float)v[1];
    return;
  }
#pragma unroll
  for (int v = 0; v < V; ++v) o[v] = (float)p[v];
}

// X_i = sum_j phi Z_ij (a 1 + b A0(u_ij) + c S0(u_ij)) for this lane's channels f .. f+V-1 of
// atom i, whose CSR row is [e0, e1); f0 = (a, b, c) per pair in FP32 or BF16 (TF)
template <int V, int G, class TF>
__device__ __forceinline__ void embed_gather_wave(int32_t i, int f, int32_t e0, int32_t e1,
                                                  const int32_t *__restrict__ nbr, const int32_t *__restrict__ pid,
                                                  const int32_t *__restrict__ z, int max_z,
                                                  const float *__restrict__ U, const float *__restrict__ Vt,
                                                  const float *__restrict__ geo, const float *__restrict__ phi,
                                                  const TF *__restrict__ f0, float *__restrict__ X) {
  constexpr int F = 64 * V * G;
  float ui[V];
  ldv<V>(U + (int64_t)clamp_z(z[i], max_z) * F + f, ui);
  float c[9][V];
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int v = 0; v < V; ++v) c[q][v] = 0.f;
  for (int32_t e = e0; e < e1; ++e) {
    const int32_t j = nbr[e];
    const int64_t p = pid[e];
    const float sg = (j > i) ? 1.f : -1.f;
    const float ux = sg * geo[4 * p], uy = sg * geo[4 * p + 1], uz = sg * geo[4 * p + 2];
    const float ph = phi[p];
    float vj[V], a[V], b[V], cc[V];
    ldv<V>(Vt + (int64_t)clamp_z(z[j], max_z) * F + f, vj);
    ld_pair_row<V>(f0 + p * 3 * F + f, a);
    ld_pair_row<V>(f0 + p * 3 * F + F + f, b);
    ld_pair_row<V>(f0 + p * 3 * F + 2 * F + f, cc);
    float s5[5];
    s0_coords(ux, uy, uz, s5);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const float w = ph * (ui[v] + vj[v]);
      const float wb = w * b[v], wc = w * cc[v];
      c[0][v] += w * a[v];
      c[1][v] += wb * ux;
      c[2][v] += wb * uy;
      c[3][v] += wb * uz;
#pragma unroll
      for (int q = 0; q < 5; ++q) c[4 + q][v] += wc * s5[q];
    }
  }
  float *x = X + (int64_t)i * 9 * F + f;
#pragma unroll
  for (int q = 0; q < 9; ++q) stv<V>(x + q * F, c[q]);
}

template <int V, int G, class TF>
__global__ void __launch_bounds__(256) k_embed_gather_w(int64_t n, const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ nbr,
                                                        const int32_t *__restrict__ pid, const int64_t *n_pairs,
                                                        int64_t max_pairs, const int32_t *__restrict__ z, int max_z,
                                                        const float *__restrict__ U, const float *__restrict__ Vt,
                                                        const float *__restrict__ geo, const float *__restrict__ phi,
                                                        const TF *__restrict__ f0, float *__restrict__ X) {
  const int32_t i = group_atom<G>();
  if (i >= n || !pairs_ok(n_pairs, max_pairs)) return;
  embed_gather_wave<V, G, TF>(i, group_channel<V, G>(), rowptr[i], rowptr[i + 1], nbr, pid, z, max_z, U, Vt, geo,
                              phi, f0, X);
}

// c[q] = sum over the CSR row [e0, e1) of h_part(q)(pair) * Y_j[q]; h (TH) and the gathered
// rows Y (TY) in FP32 or BF16.  With HZ, h holds the pre-activations z3 (TH: FP32, or BF16 in
// the BF16 path) and the filter is formed here as phi silu(z3), in FP32: in FP32 the expression
// the forward pair kernel would have stored, bit for bit.  The loads of kGatherEdges edges are
// issued before the first of them is summed; the sums still run edge by edge in CSR order (on
// 100k atoms 2-3 % faster than one edge at a time; four edges gain nothing more: the gathers
// are bound by the rows' path through L2 and MALL, about 13 TB/s, not by latency).
constexpr int kGatherEdges = 2;
template <int V, int G, class TH, class TY, bool HZ = false>
__device__ __forceinline__ void gather_message(int32_t e0, int32_t e1, const int32_t *__restrict__ nbr,
                                               const int32_t *__restrict__ pid, const TH *__restrict__ h,
                                               const TY *__restrict__ Y, int f, float (&c)[9][V],
                                               const float *__restrict__ hphi = nullptr) {
  constexpr int F = 64 * V * G, U = kGatherEdges;
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int v = 0; v < V; ++v) c[q][v] = 0.f;
  auto load_edge = [&](int32_t e, float (&hh)[3][V], float (&y)[9][V]) {
    const int64_t j = nbr[e];
    const int64_t p = pid[e];
#pragma unroll
    for (int pt = 0; pt < 3; ++pt) ld_pair_row<V>(h + p * 3 * F + pt * F + f, hh[pt]);
    if constexpr (HZ) {
      const float ph = hphi[p];
#pragma unroll
      for (int pt = 0; pt < 3; ++pt)
#pragma unroll
        for (int v = 0; v < V; ++v) hh[pt][v] = ph * fast_silu(hh[pt][v]);
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) ld_pair_row<V>(Y + j * 9 * F + q * F + f, y[q]);
  };
  auto add_edge = [&](const float (&hh)[3][V], const float (&y)[9][V]) {
#pragma unroll
    for (int q = 0; q < 9; ++q)
#pragma unroll
      for (int v = 0; v < V; ++v) c[q][v] += hh[coord_part(q)][v] * y[q][v];
  };
  int32_t e = e0;
  for (; e + U <= e1; e += U) {
    float hh[U][3][V], y[U][9][V];
#pragma unroll
    for (int u = 0; u < U; ++u) load_edge(e + u, hh[u], y[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) add_edge(hh[u], y[u]);
  }
  for (; e < e1; ++e) {
    float hh[3][V], y[9][V];
    load_edge(e, hh, y);
    add_edge(hh, y);
  }
}

// V consecutive FP32 values stored as float or, rounded, as BF16 (one 4-byte access for V = 2).
template <int V>
__device__ __forceinline__ void st_vals(float *p, const float (&o)[V]) {
  stv<V>(p, o);
}
template <int V>
__device__ __forceinline__ void st_vals(__bf16 *p, const float (&o)[V]) {
  if constexpr (V == 2) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    bf16x2 v;
    v[0] = (__bf16)o[0];
    v[1] = (__bf16)o[1];
    *reinterpret_cast<bf16x2 *>(p) = v;
    return;
  }
#pragma unroll
  for (int v = 0; v < V; ++v) p[v] = (__bf16)o[v];
}

// M_i (+)= sum_j h_part(c)(d_ij) * Y_j[c]; M in FP32 or, for a consumer that rounds it to BF16
// anyway, BF16 (TO).  Accumulating, the old values are read from Mold (FP32), or from M itself
// when Mold is null (TO = float only).
template <int V, int G, class TH, class TY, class TO = float, bool HZ = false>
__device__ __forceinline__ void message_wave(int32_t i, int f, int32_t e0, int32_t e1,
                                             const int32_t *__restrict__ nbr, const int32_t *__restrict__ pid,
                                             const TH *__restrict__ h, const TY *__restrict__ Y, TO *M,
                                             int accumulate, const float *Mold = nullptr,
                                             const float *hphi = nullptr) {
  constexpr int F = 64 * V * G;
  float c[9][V];
  gather_message<V, G, TH, TY, HZ>(e0, e1, nbr, pid, h, Y, f, c, hphi);
  const int64_t base = (int64_t)i * 9 * F + f;
  const float *src = Mold;
  if constexpr (std::is_same<TO, float>::value) {
    if (!src) src = M;
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    if (accumulate) {
      float old[V];
      ldv<V>(src + base + q * F, old);
#pragma unroll
      for (int v = 0; v < V; ++v) c[q][v] += old[v];
    }
    st_vals<V>(M + base + q * F, c[q]);
  }
}

template <int V, int G, class TH, class TY, class TO, bool HZ>
__global__ void __launch_bounds__(256) k_message_w(int64_t n, const int32_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ nbr, const int32_t *__restrict__ pid,
                                                   const int64_t *n_pairs, int64_t max_pairs,
                                                   const TH *__restrict__ h, const float *__restrict__ hphi,
                                                   const TY *__restrict__ Y, TO *M, int accumulate,
                                                   const float *Mold) {
  const int32_t i = group_atom<G>();
  if (i >= n || !pairs_ok(n_pairs, max_pairs)) return;
  message_wave<V, G, TH, TY, TO, HZ>(i, group_channel<V, G>(), rowptr[i], rowptr[i + 1], nbr, pid, h, Y, M,
                                     accumulate, Mold, hphi);
}

// M_i = sum_j h_part(c) * Y_j[c]; P = Y M + M Y; Pb = P / (||P|| + 1).  Writes M, Pb and, when
// P is given, P and ||P||.
// The neighbours' rows come from Yg (TY: Y itself, or its BF16 copy), the atom's own from Y;
// Pb in FP32 or, for a consumer that rounds it to BF16 anyway, BF16 (TO).
template <int V, int G, class TH, class TY, class TO = float, bool HZ = false>
__device__ __forceinline__ void message_product_wave(int32_t i, int f, int32_t e0, int32_t e1,
                                                     const int32_t *__restrict__ nbr,
                                                     const int32_t *__restrict__ pid, const TH *__restrict__ h,
                                                     const TY *__restrict__ Yg, const float *__restrict__ Y,
                                                     float *__restrict__ M, float *__restrict__ P,
                                                     float *__restrict__ nP, TO *__restrict__ Pb,
                                                     const float *hphi = nullptr) {
  constexpr int F = 64 * V * G;
  float mc[9][V], yc[9][V];
  gather_message<V, G, TH, TY, HZ>(e0, e1, nbr, pid, h, Yg, f, mc, hphi);
  const int64_t base = (int64_t)i * 9 * F + f;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    stv<V>(M + base + q * F, mc[q]);
    ldv<V>(Y + base + q * F, yc[q]);
  }
  float pc[9][V], nn[V];
#pragma unroll
  for (int v = 0; v < V; ++v) {
    float y9[9], m9[9], p9[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      y9[q] = yc[q][v];
      m9[q] = mc[q][v];
    }
    sym_product(y9, m9, p9);
#pragma unroll
    for (int q = 0; q < 9; ++q) pc[q][v] = p9[q];
    nn[v] = norm9(p9);
  }
  if (P) {   // null: the reverse pass forms P and its norms again from Y and M
#pragma unroll
    for (int q = 0; q < 9; ++q) stv<V>(P + base + q * F, pc[q]);
    stv<V>(nP + (int64_t)i * F + f, nn);
  }
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const float sc = 1.f / (nn[v] + 1.f);
#pragma unroll
    for (int q = 0; q < 9; ++q) pc[q][v] *= sc;
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) st_vals<V>(Pb + base + q * F, pc[q]);
}

template <int V, int G, class TH, class TY, class TO, bool HZ>
__global__ void __launch_bounds__(256) k_message_product_w(int64_t n, const int32_t *__restrict__ rowptr,
                                                           const int32_t *__restrict__ nbr,
                                                           const int32_t *__restrict__ pid, const int64_t *n_pairs,
                                                           int64_t max_pairs, const TH *__restrict__ h,
                                                           const float *__restrict__ hphi, const TY *__restrict__ Yg,
                                                           TO *__restrict__ Pb, const float *__restrict__ Y,
                                                           float *__restrict__ M, float *__restrict__ P,
                                                           float *__restrict__ nP) {
  const int32_t i = group_atom<G>();
  if (i >= n || !pairs_ok(n_pairs, max_pairs)) return;
  message_product_wave<V, G, TH, TY, TO, HZ>(i, group_channel<V, G>(), rowptr[i], rowptr[i + 1], nbr, pid, h, Yg, Y,
                                             M, P, nP, Pb, hphi);
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// eps_i = w . hx_i + b, one wave per atom: lanes stride over the H hidden units, then a fixed
// butterfly sums the lanes (the output layer's per-atom dot products, FP64).
template <class T>
__device__ __forceinline__ void out_final_wave(int32_t i, int H, const T *__restrict__ hx, const T *__restrict__ w,
                                               const T *__restrict__ b, T *__restrict__ eps) {
  const int lane = threadIdx.x & 63;
  double acc = 0.0;
  for (int k = lane; k < H; k += 64) acc += w[k] * hx[(int64_t)i * H + k];
  acc = wave_sum_d(acc);
  if (lane == 0) eps[i] = acc + b[0];
}

template <class T>
__global__ void __launch_bounds__(256) k_out_final_w(int64_t n, int H, const T *__restrict__ hx,
                                                     const T *__restrict__ w, const T *__restrict__ b,
                                                     T *__restrict__ eps) {
  const int32_t i = wave_atom();
  if (i >= n) return;
  out_final_wave<T>(i, H, hx, w, b, eps);
}

// F_i = sum over the CSR row of i of +-g_pair in FP64: lanes stride over the row, then a fixed
// butterfly sums the lanes (deterministic).
// forces[o] for atom i from its CSR row [e0, e1) (rows == false: no pair list, zero force)
template <class T, class TO>
__device__ __forceinline__ void force_gather_wave(int32_t i, int64_t o, bool rows, int32_t e0, int32_t e1,
                                                  const int32_t *__restrict__ nbr, const int32_t *__restrict__ pid,
                                                  const T *__restrict__ gpair, TO *__restrict__ forces) {
  const int lane = threadIdx.x & 63;
  double fx = 0.0, fy = 0.0, fz = 0.0;
  if (rows) {
    for (int32_t e = e0 + lane; e < e1; e += 64) {
      const int64_t p = pid[e];
      const double sg = (nbr[e] > i) ? 1.0 : -1.0;
      fx += sg * (double)gpair[3 * p];
      fy += sg * (double)gpair[3 * p + 1];
      fz += sg * (double)gpair[3 * p + 2];
    }
  }
  fx = wave_sum_d(fx);
  fy = wave_sum_d(fy);
  fz = wave_sum_d(fz);
  if (lane == 0) {
    forces[3 * o] = (TO)fx;
    forces[3 * o + 1] = (TO)fy;
    forces[3 * o + 2] = (TO)fz;
  }
}

template <class T, class TO>
__global__ void __launch_bounds__(256) k_force_gather_w(int64_t n, const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ nbr,
                                                        const int32_t *__restrict__ pid, const int64_t *n_pairs,
                                                        int64_t max_pairs, const T *__restrict__ gpair,
                                                        const int32_t *__restrict__ perm, TO *__restrict__ forces) {
  const int32_t i = wave_atom();
  if (i >= n) return;
  const bool rows = pairs_ok(n_pairs, max_pairs);
  force_gather_wave<T, TO>(i, perm ? perm[i] : i, rows, rows ? rowptr[i] : 0, rows ? rowptr[i + 1] : 0, nbr, pid,
                           gpair, forces);
}

// The embedding gather: F = 64 one wave per atom; F = 128 and 256 two waves per atom with
// V = F/128 channels per lane; f0 in FP32 or BF16 (TF).
template <class TF>
inline int embed_gather_w(hipStream_t s, int64_t F, int64_t n, const int32_t *rowptr, const int32_t *nbr,
                          const int32_t *pid, const int64_t *n_pairs, int64_t max_pairs, const int32_t *z, int max_z,
                          const float *U, const float *Vt, const float *geo, const float *phi, const TF *f0,
                          float *X) {
  if (n <= 0) return TN_OK;
  const dim3 b(256);
  if (F == 64)
    hipLaunchKernelGGL((k_embed_gather_w<1, 1, TF>), dim3(wave_atom_grid(n)), b, 0, s, n, rowptr, nbr, pid, n_pairs,
                       max_pairs, z, max_z, U, Vt, geo, phi, f0, X);
  else if (F == 128 && std::is_same<TF, __bf16>::value)   // BF16 f0: two channels per lane, 4-byte loads
    hipLaunchKernelGGL((k_embed_gather_w<2, 1, TF>), dim3(wave_atom_grid(n)), b, 0, s, n, rowptr, nbr, pid, n_pairs,
                       max_pairs, z, max_z, U, Vt, geo, phi, f0, X);
  else if (F == 128)
    hipLaunchKernelGGL((k_embed_gather_w<1, 2, TF>), dim3(wave_atom_grid(2 * n)), b, 0, s, n, rowptr, nbr, pid,
                       n_pairs, max_pairs, z, max_z, U, Vt, geo, phi, f0, X);
  else if (F == 256)
    hipLaunchKernelGGL((k_embed_gather_w<2, 2, TF>), dim3(wave_atom_grid(2 * n)), b, 0, s, n, rowptr, nbr, pid,
                       n_pairs, max_pairs, z, max_z, U, Vt, geo, phi, f0, X);
  else
    return TN_E_UNSUPPORTED;
  TN_LAUNCH_CHECK();
  return TN_OK;
}

// The message gathers, with the edge filters h (TH) and the gathered atom rows (TY) in FP32 or
// BF16.  F = 128: FP32 rows over two waves per atom, one channel per lane; BF16 rows by one
// wave per atom, two channels per lane, so each load moves 4 bytes instead of 2 (on 100k
// atoms 1.51 / 1.28 ms per launch against 1.65 / 1.45; for FP32 rows the same shape is 1.3 ms
// per step slower).  Each channel's sum runs over the same edges in the same order either way.
// hphi: when given, h holds z3 and the kernels form phi silu(z3) themselves.
#define TN_MESSAGE_LAUNCH_HZ(KERNEL, VV, GG, GRID)                                                         \
  if (hphi) {                                                                                              \
    hipLaunchKernelGGL((KERNEL<VV, GG, TH, TY, TO, true>), dim3(GRID), b, 0, s, n, rowptr, nbr, pid,        \
                       n_pairs, max_pairs, h, hphi, y, o, a...);                                          \
  } else {                                                                                                 \
    hipLaunchKernelGGL((KERNEL<VV, GG, TH, TY, TO, false>), dim3(GRID), b, 0, s, n, rowptr, nbr, pid,       \
                       n_pairs, max_pairs, h, hphi, y, o, a...);                                          \
  }
#define TN_MESSAGE_LAUNCHER(NAME, KERNEL)                                                                   \
  template <class TH, class TY, class TO, class... A>                                                     \
  inline int NAME(hipStream_t s, int64_t F, int64_t n, const int32_t *rowptr, const int32_t *nbr,          \
                  const int32_t *pid, const int64_t *n_pairs, int64_t max_pairs, const TH *h,              \
                  const float *hphi, const TY *y, TO *o, A... a) {                                         \
    if (n <= 0) return TN_OK;                                                                              \
    const dim3 b(256);                                                                                     \
    if (F == 64) {                                                                                         \
      TN_MESSAGE_LAUNCH_HZ(KERNEL, 1, 1, wave_atom_grid(n))                                                \
    } else if (F == 128 && std::is_same<TY, __bf16>::value) {                                              \
      TN_MESSAGE_LAUNCH_HZ(KERNEL, 2, 1, wave_atom_grid(n))                                                \
    } else if (F == 128) {                                                                                 \
      TN_MESSAGE_LAUNCH_HZ(KERNEL, 1, 2, wave_atom_grid(2 * n))                                            \
    } else if (F == 256) {                                                                                 \
      TN_MESSAGE_LAUNCH_HZ(KERNEL, 2, 2, wave_atom_grid(2 * n))                                            \
    } else {                                                                                               \
      return TN_E_UNSUPPORTED;                                                                             \
    }                                                                                                      \
    TN_LAUNCH_CHECK();                                                                                     \
    return TN_OK;                                                                                          \
  }
TN_MESSAGE_LAUNCHER(message_w, k_message_w)
TN_MESSAGE_LAUNCHER(message_product_w, k_message_product_w)
#undef TN_MESSAGE_LAUNCHER
#undef TN_MESSAGE_LAUNCH_HZ

template <class TI, class TO>
inline int convert(hipStream_t s, const TI *in, TO *out, int64_t n) {
  if (n <= 0) return TN_OK;
  hipLaunchKernelGGL((k_convert<TI, TO>), dim3(grid_for(n, 256)), dim3(256), 0, s, n, in, out);
  TN_LAUNCH_CHECK();
  return TN_OK;
}

}  // namespace tn
