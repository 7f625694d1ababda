// Fused per-pair kernels on MFMA (FP32, v_mfma_f32_16x16x4f32).
//
// The edge filters of TensorNet (Sec. 2.1.1; exp-normal basis and SiLU of Sec. 2.4) depend
// on the pair distance only, so every layer's filter and the embedding's K -> 3F map are
// evaluated once per unordered pair, in one pass over pair tiles:
//   forward   geometry + basis (FP64) -> f0 = W0 e + b0 -> per layer
//             z1 = Wa e + ba, z2 = Wb silu(z1) + bb, z3 = Wc silu(z2) + bc, h = phi silu(z3)
//             (h stored only when asked for: the message gathers can form it from z3)
//   reverse   dE/df0, dE/dphi, dE/dvhat of the embedding and, per layer, dh from the two
//             atoms' adjoint rows (gathered in the tile's prologue), then per layer
//             dz3 = dh phi silu'(z3), dz2 = (dz3 Wc) silu'(z2), dz1 = (dz2 Wb) silu'(z1),
//             de += dz1 Wa;  de += df0 W0;  then dE/dv from de, dE/dphi, dE/dvhat (FP64)
// Tiles hold 16 RB pairs (RB = 1 to 7; see the launchers); the NW waves of a workgroup
// split the output columns, each wave covering all rows in RB 16-row MFMA blocks.
// Activations live in LDS (row padding of
// 4 floats), weights stream from L2 as 16-byte loads.  The K index inside each 16-wide
// chunk is permuted (lane group q takes k = 4q..4q+3) so that one 16-byte load feeds four
// consecutive MFMAs for both operands.  The BF16 forward kernel passes the weights as the
// instruction's first operand, so each lane ends with four consecutive output channels of one
// pair and stores them to the row-major BF16 arrays in one 8-byte access.
#pragma once

#include "tn_internal.h"
#include "tn_device.h"
#include "tn_mfma.h"

#include <type_traits>

namespace tn {

constexpr int kPad = 4;     // LDS row padding (floats)


// Visit this lane's accumulator entries: f(rb, cb, t, row, col, value).  Entry t of block
// (rb, cb) sits at row rb*16 + 4(l/16) + t and column col0 + cb*16 + l%16 (lane l).
template <int RB, int NB, class Fn>
__device__ __forceinline__ void for_acc_rc(const floatx4 (&acc)[RB][NB], int col0, Fn &&f) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t)
        f(rb, cb, t, rb * 16 + 4 * (lane >> 4) + t, col0 + cb * 16 + (lane & 15), acc[rb][cb][t]);
}

// Visit this lane's blocks of a transposed accumulator (wave_mm_t, wave_mm_bf16_t):
// f(rb, cb, row, col, v), where v (acc[rb][cb], writable) holds row `row`, columns col .. col+3.
template <int RB, int NB, class Fn>
__device__ __forceinline__ void for_acc_t(floatx4 (&acc)[RB][NB], int col0, Fn &&f) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) f(rb, cb, rb * 16 + (lane & 15), col0 + cb * 16 + 4 * (lane >> 4), acc[rb][cb]);
}

// This lane's four columns per column block of a per-column vector (bias) for a transposed
// accumulator, loaded once before the products.
template <int NB>
__device__ __forceinline__ void load_cols_t(const float *v, int col0, floatx4 (&o)[NB]) {
  const int c = col0 + 4 * ((threadIdx.x & 63) >> 4);
#pragma unroll
  for (int cb = 0; cb < NB; ++cb)
#pragma unroll
    for (int t = 0; t < 4; ++t) o[cb][t] = v[c + cb * 16 + t];
}

__device__ __forceinline__ floatx4 silu4(const floatx4 &z) {
  return floatx4{fast_silu(z[0]), fast_silu(z[1]), fast_silu(z[2]), fast_silu(z[3])};
}
__device__ __forceinline__ floatx4 silu_and_grad4(const floatx4 &z, floatx4 &g) {
  floatx4 o;
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float gt;
    o[t] = fast_silu_and_grad(z[t], gt);
    g[t] = gt;
  }
  return o;
}

// This lane's columns of a per-column vector (bias), loaded once before the products.
template <int NB>
__device__ __forceinline__ void load_cols(const float *v, int col0, float (&o)[NB]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) o[cb] = v[col0 + cb * 16 + (lane & 15)];
}

// The stored pre-activations at this lane's accumulator positions (rows past nvalid read
// row 0), issued before the product so that their latency overlaps the MFMAs.
template <int RB, int NB, class TZ>
__device__ __forceinline__ void load_acc_rows(const TZ *z, int ldz, int64_t p0, int nvalid, int col0,
                                              float (&o)[RB][NB][4]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int row = rb * 16 + 4 * (lane >> 4) + t;
      const int64_t base = (p0 + (row < nvalid ? row : 0)) * ldz + col0 + (lane & 15);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) o[rb][cb][t] = (float)z[base + cb * 16];
    }
}

// The FP32 kernels store silu'(z1) and silu'(z2) in 16-pair blocks, column-major inside a
// block: entry (p, c) of a C-column array sits at ((p / 16) * C + c) * 16 + p % 16.  The four
// rows an accumulator lane holds are then one 16-byte access, and the sixteen lanes of a row
// group cover 1 KB without gaps.  Only rows below nvalid are written; the buffers hold whole
// blocks, so the reverse kernel may read a block's unwritten rows (their values are not used).
template <int RB, int NB>
__device__ __forceinline__ void store_acc_blocked(float *z, int C, int64_t p0, int nvalid, int col0,
                                                  const floatx4 (&acc)[RB][NB]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int row = rb * 16 + 4 * q;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      float *dst = z + ((p0 / 16 + rb) * C + col0 + cb * 16 + r) * 16 + 4 * q;
      if (row + 3 < nvalid) {
        *reinterpret_cast<floatx4 *>(dst) = acc[rb][cb];
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (row + t < nvalid) dst[t] = acc[rb][cb][t];
      }
    }
  }
}

// Reads what store_acc_blocked wrote, at this lane's accumulator positions; row blocks that
// start past nvalid are not read (zeros).
template <int RB, int NB>
__device__ __forceinline__ void load_acc_blocked(const float *z, int C, int64_t p0, int nvalid, int col0,
                                                 float (&o)[RB][NB][4]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
#pragma unroll
  for (int rb = 0; rb < RB; ++rb)
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      floatx4 v = floatx4{0.f, 0.f, 0.f, 0.f};
      if (rb * 16 < nvalid) v = *reinterpret_cast<const floatx4 *>(z + ((p0 / 16 + rb) * C + col0 + cb * 16 + r) * 16 + 4 * q);
#pragma unroll
      for (int t = 0; t < 4; ++t) o[rb][cb][t] = v[t];
    }
}

// Pair geometry in FP64 from the FP32 positions: unit vector, distance, cutoff and its derivative.
struct PairGeo {
  double u[3], d, phi, dphi;
};

__device__ inline PairGeo pair_geometry(const float *pos, int64_t i, int64_t j, const Lattice &lat, double r_c) {
  PairGeo g;
  double v[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) v[a] = (double)pos[3 * j + a] - (double)pos[3 * i + a];
  min_image(lat, v[0], v[1], v[2]);
  g.d = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const double inv = 1.0 / g.d;
#pragma unroll
  for (int a = 0; a < 3; ++a) g.u[a] = v[a] * inv;
  const double arg = M_PI * g.d / r_c;
  g.phi = 0.5 * (cos(arg) + 1.0);
  g.dphi = -0.5 * M_PI / r_c * sin(arg);
  return g;
}


// The tile functions below (pair_fwd_tile, pair_bwd_tile and their BF16 twins) declare their
// LDS arrays themselves, so a kernel that calls one gets them in its static LDS; a caller that
// runs several tiles in sequence synchronises the workgroup between them.
// ============================================================================ forward
// One LDS buffer holds the tile's current activation, silu(z1) and then silu(z2); each product
// keeps its result in registers until every wave has finished reading the buffer.
template <int F, int K, int RB, int NW>
__device__ __forceinline__ void pair_fwd_tile(const PairFwdArgs &a, int64_t p0, int nvalid) {
  constexpr int TILE = 16 * RB;
  constexpr int LE = K + kPad, L1 = F + kPad, L2 = 2 * F + kPad;
  __shared__ __attribute__((aligned(16))) float sE[TILE * LE];
  __shared__ __attribute__((aligned(16))) float sA[TILE * L2];
  __shared__ double sD[TILE], sPhi[TILE];
  const int tid = threadIdx.x, wave = tid >> 6;

  if (tid < TILE) {
    double d = a.r_c, ph = 0.0;
    if (tid < nvalid) {
      const int64_t p = p0 + tid;
      const int64_t i = a.pairs[p], j = a.pairs[a.max_pairs + p];
      const PairGeo g = pair_geometry(a.pos, i, j, a.lat, a.r_c);
      d = g.d;
      ph = g.phi;
      a.geo[4 * p + 0] = (float)g.u[0];
      a.geo[4 * p + 1] = (float)g.u[1];
      a.geo[4 * p + 2] = (float)g.u[2];
      a.geo[4 * p + 3] = (float)g.d;
      a.phi[p] = (float)g.phi;
    }
    sD[tid] = exp(-a.alpha * (d - a.r_lo));   // the basis argument u, once per pair
    sPhi[tid] = ph;
  }
  __syncthreads();
  for (int t = tid; t < TILE * K; t += 64 * NW) {
    const int row = t / K, k = t % K;
    const double u = sD[row];
    const double x = u - a.mu[k];
    sE[row * LE + k] = (float)(sPhi[row] * exp(-a.beta[k] * x * x));
  }
  __syncthreads();

  // embedding map f0 = W0 e + b0  (3F outputs; wave covers 3F/NW columns)
  {
    constexpr int NB = 3 * F / (16 * NW);
    floatx4 acc[RB][NB];
    zero_acc_rb<RB, NB>(acc);
    const int col0 = wave * (3 * F / NW);
    float br[NB];
    load_cols<NB>(a.b0, col0, br);
    wave_mm_rb<RB, NB>(sE, LE, K, a.W0, col0, acc);
    for_acc_rc(acc, col0, [&](int, int cb, int, int row, int col, float v) {
      if (row < nvalid) a.f0[(p0 + row) * 3 * F + col] = v + br[cb];
    });
  }
  for (int l = 0; l < a.L; ++l) {
    {  // z1 = Wa e + ba
      constexpr int NB = F / (16 * NW);
      floatx4 acc[RB][NB];
      zero_acc_rb<RB, NB>(acc);
      const int col0 = wave * (F / NW);
      float br[NB];
      load_cols<NB>(a.ba[l], col0, br);
      wave_mm_rb<RB, NB>(sE, LE, K, a.Wa[l], col0, acc);
      __syncthreads();   // the previous layer's last product has finished reading sA
      for_acc_rc(acc, col0, [&](int rb, int cb, int t, int row, int col, float v) {
        // silu'(z1) is all the reverse pass needs of z1, so that is what is stored
        float g;
        sA[row * L1 + col] = fast_silu_and_grad(v + br[cb], g);
        acc[rb][cb][t] = g;
      });
      store_acc_blocked<RB, NB>(a.z1[l], F, p0, nvalid, col0, acc);
    }
    __syncthreads();
    {  // z2 = Wb silu(z1) + bb
      constexpr int NB = 2 * F / (16 * NW);
      floatx4 acc[RB][NB];
      zero_acc_rb<RB, NB>(acc);
      const int col0 = wave * (2 * F / NW);
      float br[NB];
      load_cols<NB>(a.bb[l], col0, br);
      wave_mm_rb<RB, NB>(sA, L1, F, a.Wb[l], col0, acc);
      __syncthreads();
      for_acc_rc(acc, col0, [&](int rb, int cb, int t, int row, int col, float v) {
        float g;
        sA[row * L2 + col] = fast_silu_and_grad(v + br[cb], g);
        acc[rb][cb][t] = g;   // stores silu'(z2)
      });
      store_acc_blocked<RB, NB>(a.z2[l], 2 * F, p0, nvalid, col0, acc);
    }
    __syncthreads();
    {  // z3 = Wc silu(z2) + bc, h = phi silu(z3)
      constexpr int NB = 3 * F / (16 * NW);
      floatx4 acc[RB][NB];
      zero_acc_rb<RB, NB>(acc);
      const int col0 = wave * (3 * F / NW);
      float br[NB];
      load_cols<NB>(a.bc[l], col0, br);
      wave_mm_rb<RB, NB>(sA, L2, 2 * F, a.Wc[l], col0, acc);
      // h is stored only when given: its consumers may instead form it from z3 and phi,
      // with this same expression
      float *z3 = a.z3[l], *h = a.h[l];
      for_acc_rc(acc, col0, [&](int, int cb, int, int row, int col, float v) {
        const float z = v + br[cb];
        if (row < nvalid) {
          z3[(p0 + row) * 3 * F + col] = z;
          if (h) h[(p0 + row) * 3 * F + col] = (float)sPhi[row] * fast_silu(z);
        }
      });
    }
  }
}

template <int F, int K, int RB, int NW, int MINB>
__global__ void __launch_bounds__(64 * NW, MINB) k_pair_fwd(PairFwdArgs a) {
  constexpr int TILE = 16 * RB;
  const int64_t P = *a.n_pairs <= a.max_pairs ? *a.n_pairs : 0;   // no pair list after an overflow
  const int64_t tile = xcd_block_of((P + TILE - 1) / TILE);
  if (tile < 0) return;
  const int64_t p0 = tile * TILE;
  pair_fwd_tile<F, K, RB, NW>(a, p0, (int)((P - p0) < TILE ? (P - p0) : TILE));
}

// ============================================================================ reverse-sweep prologues
// Both directions of a pair meet in the pair tile, so the pair-level adjoints are formed
// here from the two atoms' rows (coordinates layout [N, 9, F]) and written straight into
// LDS as the A operand of the MFMA backprop.  Each of the NW waves owns R/NW rows; lane l holds the
// V = F/64 channels V*l .. V*l+V-1 (one vector access per coordinate), and per-row scalars
// are reduced across the wave.  Rows past the tile's valid count read the tile's first pair
// and store zeros, so the row loop has no branches and its loads can overlap.

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}

// Sum over the 64 lanes of a wave, returned wave-uniform.  Inside each row of 16 lanes the
// partners are swapped by DPP (xor 1 and xor 2 inside a quad, then the mirror inside each half
// row and inside the row), so every lane of a row ends with the same row sum; the four row sums
// are then added in a fixed order.  The order does not depend on the caller, so every tile
// shape rounds alike.
__device__ __forceinline__ float wave_sum(float v) {
  v += dpp_mov<0xB1>(v);    // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);    // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);   // row_half_mirror
  v += dpp_mov<0x140>(v);   // row_mirror
  const int b = __builtin_bit_cast(int, v);
  const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 0));
  const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 16));
  const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 32));
  const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(b, 48));
  return (r0 + r1) + (r2 + r3);
}

template <class TL, int V>
__device__ __forceinline__ void st_row(TL *p, const float (&o)[V]) {
  if constexpr (std::is_same<TL, float>::value) {
    stv<V>(p, o);
  } else if constexpr (V == 2) {   // one 4-byte access (even channel offsets)
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    bf16x2 v;
    v[0] = (__bf16)o[0];
    v[1] = (__bf16)o[1];
    *reinterpret_cast<bf16x2 *>(p) = v;
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) p[v] = (TL)o[v];
  }
}

template <class TZ, int V>
__device__ __forceinline__ void ld_row(const TZ *p, float (&o)[V]) {
  if constexpr (std::is_same<TZ, float>::value) {
    ldv<V>(p, o);
  } else if constexpr (V == 2) {   // one 4-byte access (even channel offsets)
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    const bf16x2 v = *reinterpret_cast<const bf16x2 *>(p);
    o[0] = (float)v[0];
    o[1] = (float)v[1];
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = (float)p[v];
  }
}

// The pair indices of this wave's rows, read once at the start of a prologue (rows past the
// tile's valid count take the tile's first pair).
template <int rows>
__device__ __forceinline__ int64_t wave_row_pair(int64_t p0, int nvalid, int wave, int rr) {
  const int row = wave * rows + rr;
  return p0 + (row < nvalid ? row : 0);
}

template <int rows>
__device__ __forceinline__ void wave_pair_rows(const int32_t *pairs, int64_t max_pairs, int64_t p0, int nvalid,
                                               int wave, int32_t (&pi)[rows], int32_t (&pj)[rows]) {
#pragma unroll
  for (int rr = 0; rr < rows; ++rr) {
    const int64_t p = wave_row_pair<rows>(p0, nvalid, wave, rr);
    pi[rr] = pairs[p];
    pj[rr] = pairs[max_pairs + p];
  }
}

// The second atom's rows and the pair's f0 (FP32, or BF16 when TF is __bf16) for the embedding
// adjoint.  The atom rows ("near": mostly cache hits) and the pair's row ("far": written by the
// forward pass, read from HBM) can be loaded one row ahead separately.
template <int F, class TF = float>
struct EmbedRowJ {
  static constexpr int V = F / 64;
  float c[9][V], U[V], W[V], a[V], b[V], cc[V];
  __device__ __forceinline__ void load_near(const BwdGather &bg, int64_t j, int f) {
    int zj = bg.z[j];
    zj = zj < 0 ? 0 : (zj >= bg.max_z ? bg.max_z - 1 : zj);
#pragma unroll
    for (int q = 0; q < 9; ++q) ldv<V>(bg.dXr + j * 9 * F + q * F + f, c[q]);
    ldv<V>(bg.U + zj * F + f, U);
    ldv<V>(bg.V + zj * F + f, W);
  }
  __device__ __forceinline__ void load_far(const BwdGather &bg, int64_t p, int f) {
    const TF *f0;
    if constexpr (std::is_same<TF, float>::value)
      f0 = bg.f0;
    else
      f0 = bg.f016;
    ld_row<TF, V>(f0 + p * 3 * F + f, a);
    ld_row<TF, V>(f0 + p * 3 * F + F + f, b);
    ld_row<TF, V>(f0 + p * 3 * F + 2 * F + f, cc);
  }
};

// dE/df0 = (da, db, dc) for both directions of the pair -> lds[row][0..3F); returns the pair's
// dE/dphi and dE/dvhat (embedding part) through the per-row LDS arrays.
template <int F, int R, class TL, int NW = 4, int PF = 2, class TF = float>
__device__ __forceinline__ void embed_adjoint_rows(const BwdGather &bg, const int32_t *pairs, int64_t max_pairs,
                                                   int64_t p0, int nvalid, const float (*sU)[3], const float *sPhi,
                                                   TL *lds, int ld, float *sDphi, float (*sDv)[3]) {
#pragma clang fp contract(on)   // fused multiply-adds per expression only, so every tile shape rounds alike
  constexpr int V = F / 64, rows = R / NW;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int f = lane * V;
  int32_t pi[rows], pj[rows];
  wave_pair_rows<rows>(pairs, max_pairs, p0, nvalid, wave, pi, pj);
  // the first atom's rows are reloaded only when it changes (pairs sorted by (i, j)); the next
  // row's pair row (PF >= 1, 6 registers per lane) and atom rows (PF = 2, about 25 more) are
  // loaded one row ahead so that their latency overlaps a row's work
  int64_t prev_i = -1;
  float ci[9][V], Ui[V], Vi[V];
  EmbedRowJ<F, TF> nxt;
  if constexpr (PF >= 1) nxt.load_far(bg, wave_row_pair<rows>(p0, nvalid, wave, 0), f);
  if constexpr (PF >= 2) nxt.load_near(bg, pj[0], f);
#pragma unroll
  for (int rr = 0; rr < rows; ++rr) {
    const int row = wave * rows + rr;
    const bool valid = row < nvalid;
    const int64_t i = pi[rr];
    if (i != prev_i) {
      int zi = bg.z[i];
      zi = zi < 0 ? 0 : (zi >= bg.max_z ? bg.max_z - 1 : zi);
#pragma unroll
      for (int q = 0; q < 9; ++q) ldv<V>(bg.dXr + i * 9 * F + q * F + f, ci[q]);
      ldv<V>(bg.U + zi * F + f, Ui);
      ldv<V>(bg.V + zi * F + f, Vi);
      prev_i = i;
    }
    EmbedRowJ<F, TF> cur = nxt;
    if constexpr (PF < 2) cur.load_near(bg, pj[rr], f);
    if constexpr (PF < 1) cur.load_far(bg, wave_row_pair<rows>(p0, nvalid, wave, rr), f);
    if (rr + 1 < rows) {
      if constexpr (PF >= 1) nxt.load_far(bg, wave_row_pair<rows>(p0, nvalid, wave, rr + 1), f);
      if constexpr (PF >= 2) nxt.load_near(bg, pj[rr + 1], f);
    }
    const float ux = sU[row][0], uy = sU[row][1], uz = sU[row][2];
    const float ph = sPhi[row];
    float s5[5];
    s0_coords(ux, uy, uz, s5);
    float oI[V], oA[V], oS[V];
    float aphi = 0.f, av0 = 0.f, av1 = 0.f, av2 = 0.f;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const float Zij = Ui[v] + cur.W[v], Zji = cur.U[v] + Vi[v];
      const float a = cur.a[v], b = cur.b[v], c = cur.cc[v];
      float xi[9], xj[9];
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        xi[q] = ci[q][v];
        xj[q] = cur.c[q][v];
      }
      const float giA = xi[1] * ux + xi[2] * uy + xi[3] * uz;
      const float gjA = -(xj[1] * ux + xj[2] * uy + xj[3] * uz);
      float giS = 0.f, gjS = 0.f;
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        giS += xi[4 + q] * s5[q];
        gjS += xj[4 + q] * s5[q];
      }
      oI[v] = valid ? ph * (Zij * xi[0] + Zji * xj[0]) : 0.f;
      oA[v] = valid ? ph * (Zij * giA + Zji * gjA) : 0.f;
      oS[v] = valid ? ph * (Zij * giS + Zji * gjS) : 0.f;
      aphi += Zij * (a * xi[0] + b * giA + c * giS) + Zji * (a * xj[0] + b * gjA + c * gjS);
      float gsi[3], gsj[3];
      s0_dot_grad(xi + 4, ux, uy, uz, gsi);
      s0_dot_grad(xj + 4, ux, uy, uz, gsj);
      av0 += ph * (b * (Zij * xi[1] - Zji * xj[1]) + c * (Zij * gsi[0] + Zji * gsj[0]));
      av1 += ph * (b * (Zij * xi[2] - Zji * xj[2]) + c * (Zij * gsi[1] + Zji * gsj[1]));
      av2 += ph * (b * (Zij * xi[3] - Zji * xj[3]) + c * (Zij * gsi[2] + Zji * gsj[2]));
    }
    st_row<TL, V>(lds + row * ld + f, oI);
    st_row<TL, V>(lds + row * ld + F + f, oA);
    st_row<TL, V>(lds + row * ld + 2 * F + f, oS);
    aphi = wave_sum(valid ? aphi : 0.f);
    av0 = wave_sum(valid ? av0 : 0.f);
    av1 = wave_sum(valid ? av1 : 0.f);
    av2 = wave_sum(valid ? av2 : 0.f);
    if (lane == 0) {
      sDphi[row] = aphi;
      sDv[row][0] = av0;
      sDv[row][1] = av1;
      sDv[row][2] = av2;
    }
  }
}

// The second atom's rows of Y and dE/dM ("near") and the pair's stored z3 ("far") for one
// layer's filter adjoint.
template <int F, class TZ, class TY>
struct FilterRowJ {
  static constexpr int V = F / 64;
  float y[9][V], g[9][V], z[3][V];
  __device__ __forceinline__ void load_near(const TY *Y, const TY *dM, int64_t j, int f) {
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      ld_row<TY, V>(Y + j * 9 * F + q * F + f, y[q]);
      ld_row<TY, V>(dM + j * 9 * F + q * F + f, g[q]);
    }
  }
  __device__ __forceinline__ void load_far(const TZ *z3, int64_t p, int f) {
#pragma unroll
    for (int pt = 0; pt < 3; ++pt) ld_row<TZ, V>(z3 + p * 3 * F + pt * F + f, z[pt]);
  }
};

// Layer l: dh = <part(Y_j), dM_i> + <part(Y_i), dM_j> per channel; then
// lds[row][c] = dh phi silu'(z3) and dE/dphi += sum_c dh silu(z3).  The atom rows Y and dM are
// read as TY (FP32, or the BF16 copies of the BF16 path).
template <int F, int R, class TL, class TZ, int NW = 4, int PF = 2, class TY = float>
__device__ __forceinline__ void filter_adjoint_rows(const TY *Y, const TY *dM, const TZ *z3,
                                                    const int32_t *pairs, int64_t max_pairs, int64_t p0, int nvalid,
                                                    const float *sPhi, TL *lds, int ld, float *sDphi) {
#pragma clang fp contract(on)   // fused multiply-adds per expression only, so every tile shape rounds alike
  constexpr int V = F / 64, rows = R / NW;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int f = lane * V;
  int32_t pi[rows], pj[rows];
  wave_pair_rows<rows>(pairs, max_pairs, p0, nvalid, wave, pi, pj);
  // consecutive pairs mostly share their first atom (the list is sorted by (i, j)): its rows
  // are reloaded only when i changes; the next row's z3 (PF >= 1, 6 registers per lane) and atom
  // rows (PF = 2, 36 more) are loaded one row ahead
  int64_t prev_i = -1;
  float yi[9][V], gi[9][V];
  FilterRowJ<F, TZ, TY> nxt;
  if constexpr (PF >= 1) nxt.load_far(z3, wave_row_pair<rows>(p0, nvalid, wave, 0), f);
  if constexpr (PF >= 2) nxt.load_near(Y, dM, pj[0], f);
#pragma unroll
  for (int rr = 0; rr < rows; ++rr) {
    const int row = wave * rows + rr;
    const bool valid = row < nvalid;
    const int64_t i = pi[rr];
    if (i != prev_i) {
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        ld_row<TY, V>(Y + i * 9 * F + q * F + f, yi[q]);
        ld_row<TY, V>(dM + i * 9 * F + q * F + f, gi[q]);
      }
      prev_i = i;
    }
    FilterRowJ<F, TZ, TY> cur = nxt;
    if constexpr (PF < 2) cur.load_near(Y, dM, pj[rr], f);
    if constexpr (PF < 1) cur.load_far(z3, wave_row_pair<rows>(p0, nvalid, wave, rr), f);
    if (rr + 1 < rows) {
      if constexpr (PF >= 1) nxt.load_far(z3, wave_row_pair<rows>(p0, nvalid, wave, rr + 1), f);
      if constexpr (PF >= 2) nxt.load_near(Y, dM, pj[rr + 1], f);
    }
    const float ph = sPhi[row];
    float dh[3][V];
#pragma unroll
    for (int pt = 0; pt < 3; ++pt)
#pragma unroll
      for (int v = 0; v < V; ++v) dh[pt][v] = 0.f;
#pragma unroll
    for (int q = 0; q < 9; ++q)
#pragma unroll
      for (int v = 0; v < V; ++v) dh[coord_part(q)][v] += cur.y[q][v] * gi[q][v] + yi[q][v] * cur.g[q][v];
    float part = 0.f;
#pragma unroll
    for (int pt = 0; pt < 3; ++pt) {
      float o[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        o[v] = valid ? dh[pt][v] * ph * fast_silu_grad(cur.z[pt][v]) : 0.f;
        part += dh[pt][v] * fast_silu(cur.z[pt][v]);
      }
      st_row<TL, V>(lds + row * ld + pt * F + f, o);
    }
    part = wave_sum(valid ? part : 0.f);
    if (lane == 0) sDphi[row] += part;
  }
}

// dE/dv for the tile's pairs from dE/de (LDS [R][ldE]), dE/dphi and dE/dvhat (per-row LDS).
template <int K>
__device__ __forceinline__ void geometry_adjoint_rows(const PairGeo &g, const float *sDE, int ldE, float dphi,
                                                      const float *dv, double alpha, double r_lo, const double *mu,
                                                      const double *beta, float *gout) {
  const double u = exp(-alpha * (g.d - r_lo));
  double dd = (double)dphi * g.dphi;
  for (int k = 0; k < K; ++k) {
    const double x = u - mu[k];
    const double gk = exp(-beta[k] * x * x);
    const double dek = g.dphi * gk + g.phi * gk * 2.0 * alpha * beta[k] * u * x;
    dd += (double)sDE[k] * dek;
  }
  const double gx = dv[0], gy = dv[1], gz = dv[2];
  const double proj = gx * g.u[0] + gy * g.u[1] + gz * g.u[2];
  const double inv = 1.0 / g.d;
  gout[0] = (float)(dd * g.u[0] + (gx - proj * g.u[0]) * inv);
  gout[1] = (float)(dd * g.u[1] + (gy - proj * g.u[1]) * inv);
  gout[2] = (float)(dd * g.u[2] + (gz - proj * g.u[2]) * inv);
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov_d(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Sum over each aligned group of eight lanes (xor 1, xor 2 inside a quad, then the mirror
// inside the half row); every lane of the group ends with the same value.
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_mov_d<0xB1>(v);
  v += dpp_mov_d<0x4E>(v);
  v += dpp_mov_d<0x141>(v);
  return v;
}

// dE/dv for a tile's pairs from dE/de (LDS [TILE][ldE]), dE/dphi and dE/dvhat (per-row LDS) and
// the FP64 geometry (LDS).  Eight threads per pair split the K basis derivatives (thread s takes
// k = s, s + 8, ...) and add them in a fixed order, the same for every tile shape.
template <int K, int TILE, int NT>
__device__ __forceinline__ void geometry_adjoint_tile(const PairGeo *sGeo, const float *sDE, int ldE,
                                                      const float *sDphi, const float (*sDv)[3], int nvalid,
                                                      double alpha, double r_lo, const double *mu,
                                                      const double *beta, float *gout) {
  static_assert(K % 8 == 0 && NT % 64 == 0, "eight threads per pair");
  const int tid = threadIdx.x, s = tid & 7;
#pragma unroll
  for (int row0 = 0; row0 < TILE; row0 += NT / 8) {
    const int row = row0 + (tid >> 3);
    if (row < TILE) {   // whole groups of eight lanes
      const PairGeo &g = sGeo[row];
      const double u = exp(-alpha * (g.d - r_lo));
      double acc = 0.0;
#pragma unroll
      for (int m = 0; m < K / 8; ++m) {
        const int k = s + 8 * m;
        const double x = u - mu[k];
        const double gk = exp(-beta[k] * x * x);
        const double dek = g.dphi * gk + g.phi * gk * 2.0 * alpha * beta[k] * u * x;
        acc += (double)sDE[row * ldE + k] * dek;
      }
      acc = group8_sum(acc);
      if (s == 0 && row < nvalid) {
        const double dd = (double)sDphi[row] * g.dphi + acc;
        const double gx = sDv[row][0], gy = sDv[row][1], gz = sDv[row][2];
        const double proj = gx * g.u[0] + gy * g.u[1] + gz * g.u[2];
        const double inv = 1.0 / g.d;
        gout[3 * row + 0] = (float)(dd * g.u[0] + (gx - proj * g.u[0]) * inv);
        gout[3 * row + 1] = (float)(dd * g.u[1] + (gy - proj * g.u[1]) * inv);
        gout[3 * row + 2] = (float)(dd * g.u[2] + (gz - proj * g.u[2]) * inv);
      }
    }
  }
}

// ============================================================================ reverse
// One LDS buffer holds the tile's current adjoint: dE/df0, then per layer dz3, dz2, dz1, and
// finally dE/de.  Each product keeps its result in registers until every wave has finished
// reading the buffer, so the tile needs ~50 KB of LDS and two blocks share a CU.  Of z1 and z2
// the reverse pass needs only silu'(z1) and silu'(z2), which the forward pass stores in their
// place (it has the sigmoid at hand), so no transcendental is evaluated for them here.  They
// are loaded, not recomputed: recomputing z1 = Wa e + ba from the basis (8 kFLOP per pair and
// layer) made the reverse launch 0.47 ms slower on a 100,000-atom box (19.45 against 18.98 ms)
// and the forward, which then skips the store, 0.21 ms faster; recomputing f0 as well, 0.5 ms
// slower still.

// PF: how much of the next row the prologues prefetch (by the register budget of the caller's
// launch bound; 2 = pair row and atom rows, 1 = pair row, 0 = none)
template <int F, int K, int RB, int NW, int PF>
__device__ __forceinline__ void pair_bwd_tile(const PairBwdArgs &a, int64_t p0, int nvalid) {
  constexpr int TILE = 16 * RB;
  constexpr int L3 = 3 * F + kPad, L2 = 2 * F + kPad, L1 = F + kPad, LE = K + kPad;
  __shared__ __attribute__((aligned(16))) float sG[TILE * L3];
  __shared__ float sPhi[TILE], sDphi[TILE], sU[TILE][3], sDv[TILE][3];
  __shared__ PairGeo sGeo[TILE];   // FP64 geometry for the final dE/dv, kept out of registers
  const int tid = threadIdx.x, wave = tid >> 6;
  // dE/de is split into (16-row block, 16-column block) pieces dealt round-robin to the waves
  constexpr int KB = K / 16, NDE = (RB * KB + NW - 1) / NW;

  if (tid < TILE) {
    PairGeo g{};
    float ph = 0.f;
    if (tid < nvalid) {
      const int64_t p = p0 + tid;
      g = pair_geometry(a.pos, a.pairs[p], a.pairs[a.max_pairs + p], a.lat, a.r_c);
      ph = (float)g.phi;
    }
    sPhi[tid] = ph;
    sU[tid][0] = (float)g.u[0];
    sU[tid][1] = (float)g.u[1];
    sU[tid][2] = (float)g.u[2];
    sGeo[tid] = g;
  }
  __syncthreads();
  // embedding adjoint: dE/df0 -> sG, dE/dphi and dE/dvhat per pair
  embed_adjoint_rows<F, TILE, float, NW, PF>(a.g, a.pairs, a.max_pairs, p0, nvalid, sU, sPhi, sG, L3, sDphi, sDv);
  __syncthreads();
  floatx4 de[NDE][1][1];
  auto de_product = [&](const float *act, int ld, int Kin, const float *Bt) {
#pragma unroll
    for (int n = 0; n < NDE; ++n) {
      const int c = wave + NW * n;
      if (c < RB * KB) wave_mm_rows<1, 1>(act + (c / KB) * 16 * ld, ld, 16 * ld, Kin, Bt, (c % KB) * 16, de[n]);
    }
  };
#pragma unroll
  for (int n = 0; n < NDE; ++n) zero_acc_rb<1, 1>(de[n]);
  de_product(sG, L3, 3 * F, a.W0T);
  __syncthreads();

  for (int l = 0; l < a.L; ++l) {
    const float *z1 = a.z1[l], *z2 = a.z2[l];
    filter_adjoint_rows<F, TILE, float, float, NW, PF>(a.g.Y[l], a.g.dM[l], a.z3[l], a.pairs, a.max_pairs, p0, nvalid, sPhi, sG, L3,
                                  sDphi);
    __syncthreads();
    {  // dz2 = (dz3 Wc) silu'(z2)
      constexpr int NB = 2 * F / (16 * NW);
      floatx4 acc[RB][NB];
      zero_acc_rb<RB, NB>(acc);
      const int col0 = wave * (2 * F / NW);
      float zp[RB][NB][4];
      load_acc_blocked<RB, NB>(z2, 2 * F, p0, nvalid, col0, zp);
      wave_mm_rb<RB, NB>(sG, L3, 3 * F, a.WcT[l], col0, acc);
      __syncthreads();
      for_acc_rc(acc, col0, [&](int rb, int cb, int t, int row, int col, float v) {
        sG[row * L2 + col] = row < nvalid ? v * zp[rb][cb][t] : 0.f;   // zp = silu'(z2)
      });
    }
    __syncthreads();
    {  // dz1 = (dz2 Wb) silu'(z1)
      constexpr int NB = F / (16 * NW);
      floatx4 acc[RB][NB];
      zero_acc_rb<RB, NB>(acc);
      const int col0 = wave * (F / NW);
      float zp[RB][NB][4];
      load_acc_blocked<RB, NB>(z1, F, p0, nvalid, col0, zp);
      wave_mm_rb<RB, NB>(sG, L2, 2 * F, a.WbT[l], col0, acc);
      __syncthreads();
      for_acc_rc(acc, col0, [&](int rb, int cb, int t, int row, int col, float v) {
        sG[row * L1 + col] = row < nvalid ? v * zp[rb][cb][t] : 0.f;   // zp = silu'(z1)
      });
    }
    __syncthreads();
    de_product(sG, L1, F, a.WaT[l]);   // de += dz1 Wa
    __syncthreads();
  }

  float *sDE = sG;   // [TILE][K+4]
#pragma unroll
  for (int n = 0; n < NDE; ++n) {
    const int c = wave + NW * n;
    if (c < RB * KB)
      for_acc_rc(de[n], (c % KB) * 16, [&](int, int, int, int row, int col, float v) {
        sDE[((c / KB) * 16 + row) * LE + col] = v;
      });
  }
  __syncthreads();
  geometry_adjoint_tile<K, TILE, 64 * NW>(sGeo, sDE, LE, sDphi, sDv, nvalid, a.alpha, a.r_lo, a.mu, a.beta,
                                          a.gpair + 3 * p0);
}

template <int F, int K, int RB, int NW, int MINB>
__global__ void __launch_bounds__(64 * NW, MINB) k_pair_bwd(PairBwdArgs a) {
  constexpr int TILE = 16 * RB;
  // how much of the next row the prologues prefetch, by the register budget (MINB waves per SIMD)
  constexpr int PF = MINB <= 2 ? 2 : (MINB == 3 ? 1 : 0);
  const int64_t P = *a.n_pairs <= a.max_pairs ? *a.n_pairs : 0;   // no pair list after an overflow
  const int64_t tile = xcd_block_of((P + TILE - 1) / TILE);
  if (tile < 0) return;
  const int64_t p0 = tile * TILE;
  pair_bwd_tile<F, K, RB, NW, PF>(a, p0, (int)((P - p0) < TILE ? (P - p0) : TILE));
}

// ============================================================================ BF16 variant
// GEMM operands (basis, activations, adjoints and weights) in BF16, FP32 accumulation
// (v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16)..8(l/16)+7] and
// B[8(l/16)..+7][l%16]).  Tiles of 16 RB pairs (RB 16-row blocks), so every weight fragment
// read from L2 feeds RB MFMAs.  Pre-activations (and, when asked for, the filters h) are stored
// in BF16.

// acc[rb][cb] += act[16*RB x Kin] (LDS bf16, row stride ld) * Bt^T (Bt [ncol][Kin] bf16 in global
// memory); with TR the operands of each instruction are swapped and the accumulator holds the
// block transposed, as with wave_mm_t (visit it with for_acc_t).
template <int RB, int NB, bool TR = false>
__device__ __forceinline__ void wave_mm_bf16(const __bf16 *act, int ld, int Kin, const __bf16 *__restrict__ Bt,
                                             int col0, floatx4 (&acc)[RB][NB]) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
  const __bf16 *ap = act + r * ld + 8 * q;
  const __bf16 *bp = Bt + (size_t)(col0 + r) * Kin + 8 * q;
  const size_t bstride = (size_t)16 * Kin;
  const int astride = 16 * ld;
  bf16x8 bn[NB];
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) bn[cb] = *reinterpret_cast<const bf16x8 *>(bp + cb * bstride);
  for (int k0 = 0; k0 < Kin; k0 += 32) {
    bf16x8 b[NB];
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) b[cb] = bn[cb];
    if (k0 + 32 < Kin) {
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) bn[cb] = *reinterpret_cast<const bf16x8 *>(bp + cb * bstride + k0 + 32);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const bf16x8 a = *reinterpret_cast<const bf16x8 *>(ap + rb * astride + k0);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) acc[rb][cb] = TR ? mfma_bf16(b[cb], a, acc[rb][cb]) : mfma_bf16(a, b[cb], acc[rb][cb]);
    }
  }
}


// NW waves per workgroup (4 or 8): wave w computes output columns [w C / NW, (w + 1) C / NW) of
// every C-column product, so with eight waves a tile of twice the pairs reads each weight
// fragment once for twice the rows.
template <int F, int K, int RB, int NW = 4>
__device__ __forceinline__ void pair_fwd_tile_bf16(const PairFwdArgsB &a, int64_t p0, int nvalid) {
  static_assert(F % (16 * NW) == 0, "every wave takes whole 16-column blocks");
  constexpr int TILE = 16 * RB, NT = 64 * NW;
  constexpr int LE = K + kPadB, L1 = F + kPadB, L2 = 2 * F + kPadB;
  __shared__ __attribute__((aligned(16))) __bf16 sE[TILE * LE];
  __shared__ __attribute__((aligned(16))) __bf16 sA1[TILE * L1];
  __shared__ __attribute__((aligned(16))) __bf16 sA2[TILE * L2];
  __shared__ double sD[TILE], sPhi[TILE];
  const int tid = threadIdx.x, wave = tid >> 6;
  if (tid < TILE) {
    double d = a.r_c, ph = 0.0;
    if (tid < nvalid) {
      const int64_t p = p0 + tid;
      const PairGeo g = pair_geometry(a.pos, a.pairs[p], a.pairs[a.max_pairs + p], a.lat, a.r_c);
      d = g.d;
      ph = g.phi;
      a.geo[4 * p + 0] = (float)g.u[0];
      a.geo[4 * p + 1] = (float)g.u[1];
      a.geo[4 * p + 2] = (float)g.u[2];
      a.geo[4 * p + 3] = (float)g.d;
      a.phi[p] = (float)g.phi;
    }
    sD[tid] = exp(-a.alpha * (d - a.r_lo));   // the basis argument u, once per pair
    sPhi[tid] = ph;
  }
  __syncthreads();
  for (int t = tid; t < TILE * K; t += NT) {
    const int row = t / K, k = t % K;
    const double u = sD[row];
    const double x = u - a.mu[k];
    sE[row * LE + k] = (__bf16)(float)(sPhi[row] * exp(-a.beta[k] * x * x));
  }
  __syncthreads();
  {
    constexpr int NB = 3 * F / (16 * NW);
    floatx4 acc[RB][NB];
    zero_acc_rb<RB, NB>(acc);
    const int col0 = wave * (3 * F / NW);
    floatx4 br[NB];
    load_cols_t<NB>(a.b0, col0, br);
    wave_mm_bf16<RB, NB, true>(sE, LE, K, a.W0, col0, acc);
    for_acc_t(acc, col0, [&](int, int cb, int row, int col, floatx4 &v) {
      if (row < nvalid) st4(a.f0 + (p0 + row) * 3 * F + col, v + br[cb]);
    });
  }
  for (int l = 0; l < a.L; ++l) {
    {
      constexpr int NB = F / (16 * NW);
      floatx4 acc[RB][NB];
      zero_acc_rb<RB, NB>(acc);
      const int col0 = wave * (F / NW);
      floatx4 br[NB];
      load_cols_t<NB>(a.ba[l], col0, br);
      wave_mm_bf16<RB, NB, true>(sE, LE, K, a.Wa[l], col0, acc);
      __bf16 *z1 = a.z1[l];
      for_acc_t(acc, col0, [&](int, int cb, int row, int col, floatx4 &v) {
        floatx4 g;
        const floatx4 sv = silu_and_grad4(v + br[cb], g);
        if (row < nvalid) st4(z1 + (p0 + row) * F + col, g);   // silu'(z1): all the reverse pass needs of z1
        st4(sA1 + row * L1 + col, sv);
      });
    }
    __syncthreads();
    {
      constexpr int NB = 2 * F / (16 * NW);
      floatx4 acc[RB][NB];
      zero_acc_rb<RB, NB>(acc);
      const int col0 = wave * (2 * F / NW);
      floatx4 br[NB];
      load_cols_t<NB>(a.bb[l], col0, br);
      wave_mm_bf16<RB, NB, true>(sA1, L1, F, a.Wb[l], col0, acc);
      __bf16 *z2 = a.z2[l];
      for_acc_t(acc, col0, [&](int, int cb, int row, int col, floatx4 &v) {
        floatx4 g;
        const floatx4 sv = silu_and_grad4(v + br[cb], g);
        if (row < nvalid) st4(z2 + (p0 + row) * 2 * F + col, g);   // silu'(z2)
        st4(sA2 + row * L2 + col, sv);
      });
    }
    __syncthreads();
    {
      constexpr int NB = 3 * F / (16 * NW);
      floatx4 acc[RB][NB];
      zero_acc_rb<RB, NB>(acc);
      const int col0 = wave * (3 * F / NW);
      floatx4 br[NB];
      load_cols_t<NB>(a.bc[l], col0, br);
      wave_mm_bf16<RB, NB, true>(sA2, L2, 2 * F, a.Wc[l], col0, acc);
      __bf16 *z3 = a.z3[l], *h = a.h[l];   // h only when given (see pair_fwd_tile)
      for_acc_t(acc, col0, [&](int, int cb, int row, int col, floatx4 &v) {
        if (row < nvalid) {
          v += br[cb];
          st4(z3 + (p0 + row) * 3 * F + col, v);
          if (h) st4(h + (p0 + row) * 3 * F + col, (float)sPhi[row] * silu4(v));
        }
      });
    }
  }
}

template <int F, int K, int RB, int MINB, int NW = 4>
__global__ void __launch_bounds__(64 * NW, MINB) k_pair_fwd_bf16(PairFwdArgsB a) {
  constexpr int TILE = 16 * RB;
  const int64_t P = *a.n_pairs <= a.max_pairs ? *a.n_pairs : 0;   // no pair list after an overflow
  const int64_t tile = xcd_block_of((P + TILE - 1) / TILE);
  if (tile < 0) return;
  const int64_t p0 = tile * TILE;
  pair_fwd_tile_bf16<F, K, RB, NW>(a, p0, (int)((P - p0) < TILE ? (P - p0) : TILE));
}


// NW waves per workgroup (4 or 8), as pair_fwd_tile_bf16; PF: how far the prologues load ahead
// (embed_adjoint_rows, filter_adjoint_rows).
template <int F, int K, int RB, int NW = 4, int PF = 2>
__device__ __forceinline__ void pair_bwd_tile_bf16(const PairBwdArgsB &a, int64_t p0, int nvalid) {
  static_assert(F % (16 * NW) == 0 && NW >= K / 16, "every wave takes whole 16-column blocks");
  constexpr int TILE = 16 * RB;
  constexpr int L3 = 3 * F + kPadB, L2 = 2 * F + kPadB, L1 = F + kPadB, LE = K + 4;
  __shared__ __attribute__((aligned(16))) __bf16 sG[TILE * L3];   // df0, dz3, dz2, dz1
  // dE/de between its products (the embedding's and each layer's): an FP32 accumulator kept in
  // LDS instead of registers and reloaded exactly, so the sums are those of one register chain
  __shared__ float sDE[TILE * LE];
  __shared__ float sPhi[TILE], sDphi[TILE], sU[TILE][3], sDv[TILE][3];
  const int tid = threadIdx.x, wave = tid >> 6;
  constexpr int NWDE = K / 16;
  if (tid < TILE) {
    float ph = 0.f;
    PairGeo g{};
    if (tid < nvalid) {
      const int64_t p = p0 + tid;
      g = pair_geometry(a.pos, a.pairs[p], a.pairs[a.max_pairs + p], a.lat, a.r_c);
      ph = (float)g.phi;
    }
    sPhi[tid] = ph;
    sU[tid][0] = (float)g.u[0];
    sU[tid][1] = (float)g.u[1];
    sU[tid][2] = (float)g.u[2];
  }
  __syncthreads();
  embed_adjoint_rows<F, TILE, __bf16, NW, PF, __bf16>(a.g, a.pairs, a.max_pairs, p0, nvalid, sU, sPhi, sG, L3, sDphi,
                                                   sDv);
  __syncthreads();
  // de += act * Bt^T for this wave's 16 columns of dE/de (waves < NWDE), through sDE
  auto de_product = [&](const __bf16 *act, int ld, int Kin, const __bf16 *Bt, bool first) {
    if (wave >= NWDE) return;
    floatx4 de[RB][1];
    if (first) {
      zero_acc_rb<RB, 1>(de);
    } else {
      const int lane = tid & 63;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int t = 0; t < 4; ++t) de[rb][0][t] = sDE[(rb * 16 + 4 * (lane >> 4) + t) * LE + wave * 16 + (lane & 15)];
    }
    wave_mm_bf16<RB, 1>(act, ld, Kin, Bt, wave * 16, de);
    for_acc_rc(de, wave * 16, [&](int, int, int, int row, int col, float v) { sDE[row * LE + col] = v; });
  };
  de_product(sG, L3, 3 * F, a.W0T, true);
  __syncthreads();
  for (int l = 0; l < a.L; ++l) {
    const __bf16 *z1 = a.z1[l], *z2 = a.z2[l];
    filter_adjoint_rows<F, TILE, __bf16, __bf16, NW, PF, __bf16>(a.Y16[l], a.dM16[l], a.z3[l], a.pairs, a.max_pairs, p0,
                                                            nvalid, sPhi, sG, L3,
                                   sDphi);
    __syncthreads();
    {
      constexpr int NB = 2 * F / (16 * NW);
      floatx4 acc[RB][NB];
      zero_acc_rb<RB, NB>(acc);
      const int col0 = wave * (2 * F / NW);
      float zp[RB][NB][4];
      load_acc_rows<RB, NB>(z2, 2 * F, p0, nvalid, col0, zp);
      __builtin_amdgcn_sched_barrier(0);   // issue these loads before the product loop, not inside it
      wave_mm_bf16<RB, NB>(sG, L3, 3 * F, a.WcT[l], col0, acc);
      __syncthreads();
      for_acc_rc(acc, col0, [&](int rb, int cb, int t, int row, int col, float v) {
        sG[row * L2 + col] = (__bf16)(row < nvalid ? v * zp[rb][cb][t] : 0.f);   // zp = silu'(z2)
      });
    }
    __syncthreads();
    {
      constexpr int NB = F / (16 * NW);
      floatx4 acc[RB][NB];
      zero_acc_rb<RB, NB>(acc);
      const int col0 = wave * (F / NW);
      float zp[RB][NB][4];
      load_acc_rows<RB, NB>(z1, F, p0, nvalid, col0, zp);
      __builtin_amdgcn_sched_barrier(0);   // issue these loads before the product loop, not inside it
      wave_mm_bf16<RB, NB>(sG, L2, 2 * F, a.WbT[l], col0, acc);
      __syncthreads();
      for_acc_rc(acc, col0, [&](int rb, int cb, int t, int row, int col, float v) {
        sG[row * L1 + col] = (__bf16)(row < nvalid ? v * zp[rb][cb][t] : 0.f);   // zp = silu'(z1)
      });
    }
    __syncthreads();
    de_product(sG, L1, F, a.WaT[l], false);
    __syncthreads();
  }
  if (tid < nvalid) {   // the geometry again (the same arithmetic), rather than held in registers throughout
    const int64_t p = p0 + tid;
    const PairGeo g = pair_geometry(a.pos, a.pairs[p], a.pairs[a.max_pairs + p], a.lat, a.r_c);
    geometry_adjoint_rows<K>(g, sDE + tid * LE, 0, sDphi[tid], sDv[tid], a.alpha, a.r_lo, a.mu, a.beta,
                             a.gpair + 3 * p);
  }
}

template <int F, int K, int RB, int MINB, int NW = 4, int PF = 2>
__global__ void __launch_bounds__(64 * NW, MINB) k_pair_bwd_bf16(PairBwdArgsB a) {
  constexpr int TILE = 16 * RB;
  const int64_t P = *a.n_pairs <= a.max_pairs ? *a.n_pairs : 0;   // no pair list after an overflow
  const int64_t tile = xcd_block_of((P + TILE - 1) / TILE);
  if (tile < 0) return;
  const int64_t p0 = tile * TILE;
  pair_bwd_tile_bf16<F, K, RB, NW, PF>(a, p0, (int)((P - p0) < TILE ? (P - p0) : TILE));
}

}  // namespace tn
