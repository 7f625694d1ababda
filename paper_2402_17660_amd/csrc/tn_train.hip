// Training step: the energy + force loss and its gradient with respect to every weight.
//
// Force training (Sec. 2.5; the loss of Sec. 3 weighs energy and force errors) needs the
// parameter gradient of a function of the forces, which are themselves the negative
// position gradient of the energy: a second derivative through the whole network.  With
//   loss = w_E mean_s (E_s - E*_s)^2 + w_F mean_{i,a} (F_ia - F*_ia)^2,   F = -dE/dr,
//   a_s = d loss / d E_s,   W_ia = d loss / d F_ia,
// the gradient is  sum_s a_s dE_s/dtheta - D_W (d E_tot / d theta),  where D_W is the
// directional derivative along positions r + eps W.  The step computes it in two passes:
//   1. energies and forces at r (the fused path in FP32, else the plain path), the loss, a_s
//      and W;
//   2. the hand-written reverse sweep energy -> parameters, run on dual numbers whose
//      positions carry the tangent W and whose per-system seeds are (-1, a_s): the eps parts
//      of the parameter adjoints are then exactly the loss gradient (forward-over-reverse).
// Pass 2 is the plain path's forward and reverse sweep with T = Dual<S> everywhere (no
// precision islands: S is the precision asked for) plus the parameter adjoints, which the
// energy/forces sweep does not need: outer products of layer adjoints with layer inputs for
// every linear map and mixing matrix, column sums for biases and LayerNorm gains, and the
// species tables U, V (Z_ij = U[z_i] + V[z_j]) pulled back to the embedding E, W_z, b_z.
// The reverse sweep stops at the parameters: no position adjoints are formed in pass 2.
#include "tn_nodeops.h"
#include "tn_dual.h"

#include <algorithm>
#include <cmath>

namespace tn {

constexpr int kSlices = 256;     // most row slices of a parameter-adjoint outer-product reduction
constexpr int kColSlices = 256;  // row slices of a column reduction (64 rows or more each)

// Rows of a feature array: row r starts at (r / rg) * gs + (c0 + r % rg) * cs.  One row per
// pair or atom (rg = 1, gs = row length) or, for a mixing matrix, the coordinates of one part
// (rg = 1, 3 or 5 coordinates starting at c0, gs = 9F, cs = F).
struct RowMap {
  int rg = 1;
  int64_t gs = 0;
  int c0 = 0;
  int64_t cs = 0;
};
__device__ inline int64_t row_at(const RowMap &m, int64_t r) {
  if (m.rg == 1) return r * m.gs + m.c0 * m.cs;
  const uint32_t r32 = (uint32_t)r, g = r32 / (uint32_t)m.rg;   // part rows: r < 5 N < 2^31
  return (int64_t)g * m.gs + (m.c0 + (int)(r32 - g * (uint32_t)m.rg)) * m.cs;
}
inline RowMap rows_of(int64_t len) { return RowMap{1, len, 0, 0}; }
inline RowMap part_rows(int part, int64_t F) {
  const int c0 = part == 0 ? 0 : (part == 1 ? 1 : 4), nc = part == 0 ? 1 : (part == 1 ? 3 : 5);
  return RowMap{nc, 9 * F, c0, F};
}
inline int64_t part_count(int part) { return part == 0 ? 1 : (part == 1 ? 3 : 5); }

// C[o * ldc + k] += sum_z P[z][o][k], the slices summed in a fixed order: 64 outputs per
// block, four groups of slices (z = g mod 4) per output, the groups combined in order.
template <class T>
__global__ void __launch_bounds__(256) k_sum_slices(int O, int Kc, int G, const T *P, T *C, int64_t ldc) {
  __shared__ T part[4][64];
  const int l = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int64_t t = blockIdx.x * (int64_t)64 + l, n = (int64_t)O * Kc;
  T s = T(0);
  if (t < n)
    for (int z = g; z < G; z += 4) s += P[(int64_t)z * n + t];
  part[g][l] = s;
  __syncthreads();
  if (g == 0 && t < n) {
    const int o = (int)(t / Kc), k = (int)(t % Kc);
    C[o * ldc + k] += ((part[0][l] + part[1][l]) + part[2][l]) + part[3][l];
  }
}

// P[z][c] = sum over rows r < min(R, *Rdev) of slice z of rs[r] * A[r*C + c] * B[r*C + c] (rs, B = 1
// when null).
template <class T>
__global__ void k_coldot_part(const T *A, const T *B, const T *rs, int64_t R, const int64_t *Rdev, int C,
                              int64_t slice, T *P) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= C) return;
  int64_t Rn = R;
  if (Rdev) {
    const int64_t md = *Rdev;
    if (md < Rn) Rn = md;
  }
  const int64_t rb = (int64_t)blockIdx.y * slice;
  const int64_t re = rb + slice < Rn ? rb + slice : Rn;
  T s = T(0);
  for (int64_t r = rb; r < re; ++r) {
    T v = A[r * C + c];
    if (B) v *= B[r * C + c];
    if (rs) v *= rs[r];
    s += v;
  }
  P[(int64_t)blockIdx.y * C + c] = s;
}

// ---------------------------------------------------------------- dual products on the matrix cores
// C = epilogue(A B) with A dual and B real (a weight matrix: the weights carry no tangent),
// the same product and epilogue as GemmArgs / k_gemm_mfma: bias (real), pre-activation store,
// SiLU, row scale, silu'(gate) factor and accumulation, each applied in dual arithmetic.  The
// value and the eps part of A are staged as two LDS tiles and share every B fragment: two
// MFMA 16x16x4 per fragment pair instead of one.
template <class S>
struct DualGemmArgs {
  const Dual<S> *A = nullptr; int64_t lda = 0;
  const S *B = nullptr; int64_t ldb = 0; int transB = 0;
  Dual<S> *C = nullptr; int64_t ldc = 0;
  const S *bias = nullptr;
  Dual<S> *Z = nullptr; int64_t ldz = 0;
  int act = 0;
  const Dual<S> *rowscale = nullptr;
  const Dual<S> *gate = nullptr; int64_t ldg = 0;
  int accumulate = 0;
  int64_t M = 0, N = 0, K = 0;
  const int64_t *Mdev = nullptr;
  int64_t zoff = 0;
  int zpart = 0;
  const S *Bz[3] = {nullptr, nullptr, nullptr};
};

template <class S, int BM>
__global__ void __launch_bounds__(256) k_gemm_dual(DualGemmArgs<S> g) {
  using D = Dual<S>;
  using V = typename MfmaVec<S>::type;
  constexpr int RBW = BM / 32;
  constexpr int PERA = BM * GBK / 256, PERB = GBN * GBK / 256;
  __shared__ S Av[BM][GBK + 1];
  __shared__ S Ad[BM][GBK + 1];
  __shared__ S Bs[GBN][GBK + 1];
  int64_t Mrows = g.M;
  if (g.Mdev) {
    const int64_t md = *g.Mdev;
    if (md < Mrows) Mrows = md;
  }
  // one flat block index over (row tile, column tile), column tiles fastest (so the blocks that
  // share a row tile run together); a flat x dimension has no 65535-block limit
  const int64_t nb = (g.N + GBN - 1) / GBN;
  const int64_t m0 = (int64_t)(blockIdx.x / nb) * BM;
  const int64_t n0 = (int64_t)(blockIdx.x % nb) * GBN;
  if (m0 >= Mrows) return;
  const int z = blockIdx.z;
  const D *__restrict__ A = g.A + z * g.zoff;
  const S *__restrict__ B = g.zpart ? g.Bz[coord_part(z)] : g.B;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = (wave >> 1) * (BM / 2), wc = (wave & 1) * 32;
  const int r16 = lane & 15, q = lane >> 4;
  D ra[PERA];
  S rb[PERB];
  auto load_chunk = [&](int64_t k0) {
#pragma unroll
    for (int e = 0; e < PERA; ++e) {
      const int t = tid + 256 * e, mm_ = t / GBK, kk = t % GBK;
      const int64_t m = m0 + mm_, k = k0 + kk;
      ra[e] = (m < Mrows && k < g.K) ? A[m * g.lda + k] : D(S(0), S(0));
    }
#pragma unroll
    for (int e = 0; e < PERB; ++e) {
      const int t = tid + 256 * e;
      int nn, kk;
      if (g.transB) { nn = t / GBK; kk = t % GBK; } else { kk = t / GBN; nn = t % GBN; }
      const int64_t n = n0 + nn, k = k0 + kk;
      S v = S(0);
      if (n < g.N && k < g.K) v = g.transB ? B[n * g.ldb + k] : B[k * g.ldb + n];
      rb[e] = v;
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int e = 0; e < PERA; ++e) {
      const int t = tid + 256 * e;
      Av[t / GBK][t % GBK] = ra[e].v;
      Ad[t / GBK][t % GBK] = ra[e].d;
    }
#pragma unroll
    for (int e = 0; e < PERB; ++e) {
      const int t = tid + 256 * e;
      int nn, kk;
      if (g.transB) { nn = t / GBK; kk = t % GBK; } else { kk = t / GBN; nn = t % GBN; }
      Bs[nn][kk] = rb[e];
    }
  };
  V accv[RBW][2], accd[RBW][2];
#pragma unroll
  for (int a = 0; a < RBW; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      accv[a][b] = V{S(0), S(0), S(0), S(0)};
      accd[a][b] = V{S(0), S(0), S(0), S(0)};
    }
  load_chunk(0);
  for (int64_t k0 = 0; k0 < g.K; k0 += GBK) {
    store_chunk();
    __syncthreads();
    if (k0 + GBK < g.K) load_chunk(k0 + GBK);
#pragma unroll
    for (int s4 = 0; s4 < GBK; s4 += 4) {
      const S b0 = Bs[wc + r16][s4 + q], b1 = Bs[wc + 16 + r16][s4 + q];
#pragma unroll
      for (int a = 0; a < RBW; ++a) {
        const S av = Av[wr + 16 * a + r16][s4 + q], ad = Ad[wr + 16 * a + r16][s4 + q];
        accv[a][0] = mfma_16x16x4(av, b0, accv[a][0]);
        accv[a][1] = mfma_16x16x4(av, b1, accv[a][1]);
        accd[a][0] = mfma_16x16x4(ad, b0, accd[a][0]);
        accd[a][1] = mfma_16x16x4(ad, b1, accd[a][1]);
      }
    }
    __syncthreads();
  }
  D *C = g.C + z * g.zoff;
  S bias[2] = {S(0), S(0)};
#pragma unroll
  for (int cb = 0; cb < 2; ++cb) {
    const int64_t n = n0 + wc + cb * 16 + r16;
    if (g.bias && n < g.N) bias[cb] = g.bias[n];
  }
#pragma unroll
  for (int rb_ = 0; rb_ < RBW; ++rb_)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t m = m0 + wr + rb_ * 16 + (sizeof(S) == 4 ? 4 * q + t : 4 * t + q);
        const int64_t n = n0 + wc + cb * 16 + r16;
        if (m >= Mrows || n >= g.N) continue;
        D v(accv[rb_][cb][t] + bias[cb], accd[rb_][cb][t]);
        if (g.Z) g.Z[z * g.zoff + m * g.ldz + n] = v;
        if (g.act == 1) v = silu(v);
        if (g.rowscale) v *= g.rowscale[m];
        if (g.gate) v *= silu_grad(g.gate[z * g.zoff + m * g.ldg + n]);
        D *dst = C + m * g.ldc + n;
        if (g.accumulate) *dst += v; else *dst = v;
      }
}

template <class S>
inline int dgemm(hipStream_t s, const DualGemmArgs<S> &g, int zdim = 1) {
  if (g.M <= 0 || g.N <= 0) return TN_OK;
  const int64_t nb = (g.N + GBN - 1) / GBN;
  const int64_t tiles64 = nb * ((g.M + 63) / 64) * zdim;
  if (tiles64 < 512) {
    dim3 grid((unsigned)(nb * ((g.M + 31) / 32)), 1, (unsigned)zdim);
    hipLaunchKernelGGL((k_gemm_dual<S, 32>), grid, dim3(256), 0, s, g);
  } else {
    dim3 grid((unsigned)(nb * ((g.M + 63) / 64)), 1, (unsigned)zdim);
    hipLaunchKernelGGL((k_gemm_dual<S, 64>), grid, dim3(256), 0, s, g);
  }
  TN_LAUNCH_CHECK();
  return TN_OK;
}

// y = act(x W^T + b), W [Nout, Kin] real
template <class S>
inline int dlinear_fwd(hipStream_t s, const Dual<S> *x, int64_t M, int64_t Kin, const S *W, const S *b, int64_t Nout,
                       Dual<S> *y, Dual<S> *z_pre, int act, const Dual<S> *rowscale = nullptr,
                       const int64_t *Mdev = nullptr) {
  DualGemmArgs<S> g;
  g.A = x; g.lda = Kin; g.B = W; g.ldb = Kin; g.transB = 1;
  g.C = y; g.ldc = Nout; g.bias = b; g.Z = z_pre; g.ldz = Nout; g.act = act; g.rowscale = rowscale;
  g.M = M; g.N = Nout; g.K = Kin; g.Mdev = Mdev;
  return dgemm(s, g);
}

// dx (+)= (dy W) * silu'(gate)
template <class S>
inline int dlinear_bwd(hipStream_t s, const Dual<S> *dy, int64_t M, int64_t Nout, const S *W, int64_t Kin,
                       Dual<S> *dx, const Dual<S> *gate, int accumulate, const int64_t *Mdev = nullptr) {
  DualGemmArgs<S> g;
  g.A = dy; g.lda = Nout; g.B = W; g.ldb = Kin; g.transB = 0;
  g.C = dx; g.ldc = Kin; g.gate = gate; g.ldg = Kin; g.accumulate = accumulate;
  g.M = M; g.N = Kin; g.K = Nout; g.Mdev = Mdev;
  return dgemm(s, g);
}

// per-part channel mixing of [N, 9, F] dual features with real matrices (forward or adjoint)
template <class S>
inline int dmix(hipStream_t s, const Dual<S> *in, Dual<S> *out, int64_t N, int64_t F, const S *const W[3],
                int adjoint, int accumulate) {
  if (N <= 0) return TN_OK;
  DualGemmArgs<S> g;
  g.A = in; g.lda = 9 * F; g.C = out; g.ldc = 9 * F; g.transB = adjoint ? 0 : 1; g.ldb = F;
  g.M = N; g.N = F; g.K = F; g.zoff = F; g.zpart = 1; g.accumulate = accumulate;
  for (int q = 0; q < 3; ++q) g.Bz[q] = W[q];
  return dgemm(s, g, 9);
}

// Parameter adjoints on the matrix cores: P[z][o][k] = sum over the rows r of slice z of
// A(r, o) B(r, k), both dual.  Only the eps part A_d B_v + A_v B_d is formed (two MFMA per
// fragment): the loss gradient is the eps part of every weight adjoint, and nothing reads the
// value part, which is written as zero.  64x64 outputs per block, 32 rows staged per step in LDS as [row][column] tiles
// (coalesced along the feature axis); lane l of MFMA 16x16x4 supplies A(r0 + l/16, o0 + l%16)
// and B(r0 + l/16, k0 + l%16).  Every block writes its outputs.  With Q given, the blocks of
// the first column block also form the column sums of A over the slice (the bias adjoint of
// a linear map, from the tiles already in LDS): Q[z][o] = sum_r A_d(r, o) (eps part only),
// four row groups per column combined in a fixed order.
constexpr int WRC = 32;
template <class S>
__global__ void __launch_bounds__(256) k_wgrad_mfma(const Dual<S> *A, RowMap ma, const Dual<S> *B, RowMap mb,
                                                    int64_t R, const int64_t *Rdev, int O, int Kc, int64_t slice,
                                                    Dual<S> *P, Dual<S> *Q) {
  using D = Dual<S>;
  using V = typename MfmaVec<S>::type;
  __shared__ S Av[WRC][64 + 1], Ad[WRC][64 + 1], Bv[WRC][64 + 1], Bd[WRC][64 + 1];
  const bool colsum = Q != nullptr && blockIdx.x == 0;
  S qd = S(0);   // column (tid % 64), rows tid / 64 + 4 m of each staged step
  int64_t Rn = R;
  if (Rdev) {
    const int64_t md = *Rdev;
    if (md < Rn) Rn = md;
  }
  const int o0 = blockIdx.y * 64, k0 = blockIdx.x * 64;
  const int64_t rb = (int64_t)blockIdx.z * slice;
  const int64_t re = rb + slice < Rn ? rb + slice : Rn;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wo = (wave >> 1) * 32, wk = (wave & 1) * 32;
  const int r16 = lane & 15, q = lane >> 4;
  V cd[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) cd[a][b] = V{S(0), S(0), S(0), S(0)};
  constexpr int PER = WRC * 64 / 256;
  D xa[PER], xb[PER];
  auto load_rows = [&](int64_t r0) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int t = tid + 256 * e, rr = t / 64, cc = t % 64;
      const int64_t r = r0 + rr;
      xa[e] = D(S(0), S(0));
      xb[e] = D(S(0), S(0));
      if (r < re) {
        if (o0 + cc < O) xa[e] = A[row_at(ma, r) + o0 + cc];
        if (k0 + cc < Kc) xb[e] = B[row_at(mb, r) + k0 + cc];
      }
    }
  };
  // the next rows' global loads are issued before the current rows' products
  if (rb < re) load_rows(rb);
  for (int64_t r0 = rb; r0 < re; r0 += WRC) {
#pragma unroll
    for (int e = 0; e < PER; ++e) {
      const int t = tid + 256 * e, rr = t / 64, cc = t % 64;
      Av[rr][cc] = xa[e].v;
      Ad[rr][cc] = xa[e].d;
      Bv[rr][cc] = xb[e].v;
      Bd[rr][cc] = xb[e].d;
    }
    __syncthreads();
    if (r0 + WRC < re) load_rows(r0 + WRC);
    if (colsum) {
#pragma unroll
      for (int rr = tid >> 6; rr < WRC; rr += 4) qd += Ad[rr][tid & 63];
    }
#pragma unroll
    for (int s4 = 0; s4 < WRC; s4 += 4) {
      S bv[2], bd[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        bv[b] = Bv[s4 + q][wk + 16 * b + r16];
        bd[b] = Bd[s4 + q][wk + 16 * b + r16];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const S av = Av[s4 + q][wo + 16 * a + r16], ad = Ad[s4 + q][wo + 16 * a + r16];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          cd[a][b] = mfma_16x16x4(ad, bv[b], cd[a][b]);
          cd[a][b] = mfma_16x16x4(av, bd[b], cd[a][b]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int o = o0 + wo + 16 * a + (sizeof(S) == 4 ? 4 * q + t : 4 * t + q);
        const int k = k0 + wk + 16 * b + r16;
        if (o < O && k < Kc) P[((int64_t)blockIdx.z * O + o) * Kc + k] = D(S(0), cd[a][b][t]);
      }
  if (colsum) {   // reuse the A tiles (every wave is past its last read of them)
    Ad[tid >> 6][tid & 63] = qd;
    __syncthreads();
    const int o = o0 + tid;
    if (tid < 64 && o < O)
      Q[(int64_t)blockIdx.z * O + o] = D(S(0), ((Ad[0][tid] + Ad[1][tid]) + Ad[2][tid]) + Ad[3][tid]);
  }
}

template <class T>
struct Reducer {
  T *part = nullptr;
  int64_t cap = 0;   // elements of part

  // Row slices of an outer-product reduction: enough blocks to fill the chip (about eight per
  // compute unit), at least 256 rows per slice, and the partial sums within the scratch.
  int slices(int64_t R, int O, int Kc) const {
    const int64_t tiles = (int64_t)((O + 63) / 64) * ((Kc + 63) / 64);
    int64_t g = std::min<int64_t>((2048 + tiles - 1) / tiles, (R + 255) / 256);
    g = std::min<int64_t>(g, std::min<int64_t>(kSlices, cap / ((int64_t)O * (Kc + 1))));
    return (int)std::max<int64_t>(1, g);
  }
  // C[o][k] (row stride ldc) += sum_r A(r, o) B(r, k), rows r < min(R, *Rdev); with cb given
  // also cb[o] += sum_r A(r, o)
  int wgrad(hipStream_t s, const T *A, RowMap ma, const T *B, RowMap mb, int64_t R, const int64_t *Rdev, int O,
            int Kc, T *C, int64_t ldc, T *cb = nullptr) const {
    if (R <= 0 || O <= 0 || Kc <= 0) return TN_OK;
    const int G = slices(R, O, Kc);
    if ((int64_t)G * O * (Kc + 1) > cap) return TN_E_WORKSPACE;
    T *Q = cb ? part + (int64_t)G * O * Kc : nullptr;
    const int64_t slice = ((R + G - 1) / G + WRC - 1) / WRC * WRC;
    {
      TimedScope ts("train_wgrad", s);
      hipLaunchKernelGGL(k_wgrad_mfma<typename T::scalar>, dim3((unsigned)((Kc + 63) / 64),
                         (unsigned)((O + 63) / 64), (unsigned)G), dim3(256), 0, s, A, ma, B, mb, R, Rdev, O, Kc,
                         slice, part, Q);
      TN_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_sum_slices<T>, dim3(grid_for((int64_t)O * Kc, 64)), dim3(256), 0, s, O, Kc, G,
                       (const T *)part, C, ldc);
    TN_LAUNCH_CHECK();
    if (cb) {
      hipLaunchKernelGGL(k_sum_slices<T>, dim3(grid_for(O, 64)), dim3(256), 0, s, 1, O, G, (const T *)Q, cb,
                         (int64_t)O);
      TN_LAUNCH_CHECK();
    }
    return TN_OK;
  }
  // weight and bias of y = x W^T + b from the pre-activation adjoint dz
  int linear(hipStream_t s, const T *dz, const T *x, int64_t R, const int64_t *Rdev, int O, int Kin, T *dW,
             T *db) const {
    return wgrad(s, dz, rows_of(O), x, rows_of(Kin), R, Rdev, O, Kin, dW, Kin, db);
  }
  // out[c] += sum_r rs[r] A[r][c] B[r][c], rows r < min(R, *Rdev)
  int coldot(hipStream_t s, const T *A, const T *B, const T *rs, int64_t R, const int64_t *Rdev, int C,
             T *out) const {
    if (R <= 0 || C <= 0) return TN_OK;
    const int G = (int)std::max<int64_t>(1, std::min<int64_t>(kColSlices, (R + 63) / 64));
    if ((int64_t)G * C > cap) return TN_E_WORKSPACE;
    const int64_t slice = (R + G - 1) / G;
    hipLaunchKernelGGL(k_coldot_part<T>, dim3((unsigned)((C + 127) / 128), (unsigned)G), dim3(128), 0, s, A, B, rs,
                       R, Rdev, C, slice, part);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_slices<T>, dim3(grid_for(C, 64)), dim3(256), 0, s, 1, C, G, (const T *)part, out,
                       (int64_t)C);
    TN_LAUNCH_CHECK();
    return TN_OK;
  }
};

// ---------------------------------------------------------------- dual messages
// M_i (+)= sum over the CSR row of i of h_ij (per part) * Y_j on dual numbers, G waves per
// atom: lane l of wave g holds channels (64 g + l) V .. +V-1 (F = 64 V G) and the row's
// indices are wave-uniform, as in the FP32 gather kernels.
template <class T, int V, int G>
__global__ void __launch_bounds__(256) k_message_dual_w(int64_t n, const int32_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ nbr, const int32_t *__restrict__ pid,
                                                        const int64_t *n_pairs, int64_t max_pairs,
                                                        const T *__restrict__ h, const T *__restrict__ Y,
                                                        T *__restrict__ M, int accumulate) {
  constexpr int F = 64 * V * G;
  const int32_t i = group_atom<G>();
  if (i >= n || !pairs_ok(n_pairs, max_pairs)) return;
  const int f = group_channel<V, G>();
  T c[9][V];
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int v = 0; v < V; ++v) c[q][v] = T(0);
  const int32_t e1 = rowptr[i + 1];
  for (int32_t e = rowptr[i]; e < e1; ++e) {
    const int64_t j = nbr[e], p = pid[e];
    T hh[3][V];
#pragma unroll
    for (int pt = 0; pt < 3; ++pt)
#pragma unroll
      for (int v = 0; v < V; ++v) hh[pt][v] = h[p * 3 * F + pt * F + f + v];
#pragma unroll
    for (int q = 0; q < 9; ++q)
#pragma unroll
      for (int v = 0; v < V; ++v) c[q][v] += hh[coord_part(q)][v] * Y[j * 9 * F + q * F + f + v];
  }
  T *m = M + (int64_t)i * 9 * F + f;
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int v = 0; v < V; ++v) m[q * F + v] = accumulate ? m[q * F + v] + c[q][v] : c[q][v];
}

template <class T>
inline int dmessage(hipStream_t s, int64_t N, int64_t F, const int32_t *rowptr, const int32_t *nbr, const int32_t *pid,
                    const int64_t *np, int64_t MP, const T *h, const T *Y, T *M, int accumulate) {
  if (N <= 0) return TN_OK;
  if (F == 64 || F == 128 || F == 256) {
    const dim3 block(256);
    if (F == 64)
      hipLaunchKernelGGL((k_message_dual_w<T, 1, 1>), dim3(wave_atom_grid(N)), block, 0, s, N, rowptr, nbr, pid, np,
                         MP, h, Y, M, accumulate);
    else if (F == 128)
      hipLaunchKernelGGL((k_message_dual_w<T, 1, 2>), dim3(wave_atom_grid(2 * N)), block, 0, s, N, rowptr, nbr, pid,
                         np, MP, h, Y, M, accumulate);
    else
      hipLaunchKernelGGL((k_message_dual_w<T, 2, 2>), dim3(wave_atom_grid(2 * N)), block, 0, s, N, rowptr, nbr, pid,
                         np, MP, h, Y, M, accumulate);
  } else {
    hipLaunchKernelGGL(k_message<T>, dim3(grid_for(N * F, 256)), dim3(256), 0, s, N, (int)F, rowptr, nbr, pid, np,
                       MP, h, Y, M, accumulate);
  }
  TN_LAUNCH_CHECK();
  return TN_OK;
}

// ---------------------------------------------------------------- pass 1: loss and seeds
// loss = w_E/S sum_s e_s^2 + w_F/(3N) sum f^2 with e = E - E*, f = F - F*;
// seed_s = (-1, d loss/d E_s), wt = d loss / dF (caller's atom order).  One block.
template <class S>
__global__ void __launch_bounds__(256) k_loss(int64_t n, int64_t ns, const double *E, const double *Eref,
                                              const S *Fv, const double *Fref, double wE, double wF, double *loss,
                                              Dual<S> *seed, double *wt) {
  __shared__ double lds[256];
  double ae = 0.0, af = 0.0;
  const double inv_s = ns > 0 ? 1.0 / (double)ns : 0.0;
  const double inv_f = n > 0 ? 1.0 / (3.0 * (double)n) : 0.0;
  for (int64_t k = threadIdx.x; k < ns; k += 256) {
    const double e = E[k] - Eref[k];
    ae += e * e;
    seed[k] = Dual<S>(S(-1), (S)(2.0 * wE * e * inv_s));
  }
  for (int64_t k = threadIdx.x; k < 3 * n; k += 256) {
    const double f = (double)Fv[k] - Fref[k];
    af += f * f;
    wt[k] = 2.0 * wF * f * inv_f;
  }
  const double te = block_sum(ae, lds);
  const double tf = block_sum(af, lds);
  if (threadIdx.x == 0) *loss = wE * te * inv_s + wF * tf * inv_f;
}

// ---------------------------------------------------------------- pass 2 helpers
template <class S>
__global__ void k_to_dual(int64_t n, const double *w, Dual<S> *out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) out[t] = Dual<S>((S)w[t], S(0));
}

// Positions r + eps W in the internal atom order (perm maps internal -> caller index).
template <class S>
__global__ void k_pos_dual(int64_t n, const S *pos, const int32_t *perm, const double *wt, Dual<S> *posD) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t o = perm ? perm[i] : i;
#pragma unroll
  for (int a = 0; a < 3; ++a) posD[3 * i + a] = Dual<S>(pos[3 * i + a], (S)wt[3 * o + a]);
}

template <class S>
__device__ inline Dual<S> narrow(Dual<double> x) { return Dual<S>((S)x.v, (S)x.d); }

// Pair geometry and radial basis on dual positions, evaluated in Dual<double> and rounded
// once: the lattice shift of the minimum image is a constant, so it moves the value only.
template <class S>
__global__ void k_geom_dual(const int32_t *pairs, int64_t max_pairs, const int64_t *n_pairs, const Dual<S> *posD,
                            Lattice box, double r_c, double r_lo, double alpha, const double *mu, const double *beta,
                            int K, Dual<S> *geo, Dual<S> *phi, Dual<S> *rbf) {
  using DD = Dual<double>;
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= pair_bound(n_pairs, max_pairs)) return;
  const int64_t i = pairs[p], j = pairs[max_pairs + p];
  DD v[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    v[a] = DD((double)posD[3 * j + a].v - (double)posD[3 * i + a].v,
              (double)posD[3 * j + a].d - (double)posD[3 * i + a].d);
  double x = v[0].v, y = v[1].v, z = v[2].v;
  min_image(box, x, y, z);
  v[0].v = x;
  v[1].v = y;
  v[2].v = z;
  const DD d = dsqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const DD inv = DD(1.0) / d;
#pragma unroll
  for (int a = 0; a < 3; ++a) geo[4 * p + a] = narrow<S>(v[a] * inv);
  geo[4 * p + 3] = narrow<S>(d);
  const DD ph = DD(0.5) * (dcos(DD(M_PI) * d / DD(r_c)) + DD(1.0));
  phi[p] = narrow<S>(ph);
  const DD u = dexp(-DD(alpha) * (d - DD(r_lo)));
  for (int k = 0; k < K; ++k) {
    const DD t = u - DD(mu[k]);
    rbf[p * K + k] = narrow<S>(ph * dexp(-DD(beta[k]) * t * t));
  }
}

// Per-atom seed: that of the atom's system (zero for a system index outside [0, ns), which
// the neighbour search has already flagged in the status word).
template <class T>
__global__ void k_seed_atoms(int64_t n, int64_t ns, const int32_t *batch, const T *seed, T *sd) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int32_t b = batch[i];
  sd[i] = (b >= 0 && b < ns) ? seed[b] : T(0);
}

// eps_i = w . silu(hz_i) + b with seed sd_i on eps_i:  dhz = sd_i w silu'(hz)
template <class T>
__global__ void k_out_final_bwd_seed(int64_t n, int H, const T *hz, const T *w, const T *sd, T *dhz) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * H) return;
  const int64_t i = t / H;
  const int k = (int)(t % H);
  dhz[t] = sd[i] * w[k] * silu_grad(hz[t]);
}

// Adjoint of the species factor of each pair's embedding message, both directions:
// dZ[p][0][f] = d E / d Z_ij[f] (receiver i), dZ[p][1][f] = d E / d Z_ji[f] (receiver j).
template <class T>
__global__ void k_embed_dz(const int32_t *pairs, int64_t max_pairs, const int64_t *n_pairs, int F, const T *geo,
                           const T *phi, const T *f0, const T *dXr, T *dZ) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t p = t / F;
  if (p >= pair_bound(n_pairs, max_pairs)) return;
  const int f = (int)(t % F);
  const int64_t i = pairs[p], j = pairs[max_pairs + p];
  const T ux = geo[4 * p], uy = geo[4 * p + 1], uz = geo[4 * p + 2];
  T s5[5];
  s0_coords(ux, uy, uz, s5);
  const T a = f0[p * 3 * F + f], b = f0[p * 3 * F + F + f], c = f0[p * 3 * F + 2 * F + f];
  T di[9], dj[9];
  load9(dXr, i, F, f, di);
  load9(dXr, j, F, f, dj);
  const T giA = di[1] * ux + di[2] * uy + di[3] * uz;
  const T gjA = -(dj[1] * ux + dj[2] * uy + dj[3] * uz);
  T giS = T(0), gjS = T(0);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    giS += di[4 + q] * s5[q];
    gjS += dj[4 + q] * s5[q];
  }
  const T ph = phi[p];
  dZ[p * 2 * F + f] = ph * (a * di[0] + b * giA + c * giS);
  dZ[p * 2 * F + F + f] = ph * (a * dj[0] + b * gjA + c * gjS);
}

// Per atom a, the adjoints of its species rows: dUa[a] = sum of dZ over the pair directions that
// a receives, dVa[a] over those it sends.  A stored pair (i, j) has i < j, so along the CSR row of
// a a neighbour b > a means a is the pair's i.  One thread per (atom, channel).
template <class T>
__global__ void k_atom_dz(int64_t n, int F, const int32_t *rowptr, const int32_t *nbr, const int32_t *pid,
                          const int64_t *n_pairs, int64_t max_pairs, const T *dZ, T *dUa, T *dVa) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  const int64_t a = t / F;
  const int f = (int)(t % F);
  T u = T(0), v = T(0);
  if (pairs_ok(n_pairs, max_pairs)) {
    for (int32_t e = rowptr[a]; e < rowptr[a + 1]; ++e) {
      const int64_t p = pid[e];
      const T d0 = dZ[p * 2 * F + f], d1 = dZ[p * 2 * F + F + f];
      if (nbr[e] > a) { u += d0; v += d1; } else { u += d1; v += d0; }
    }
  }
  dUa[t] = u;
  dVa[t] = v;
}

// dU[s] = sum of dUa over the atoms of species s, likewise dV.  One block per (species, 64
// channels); sixteen atom groups per block, combined in a fixed order.
template <class T>
__global__ void __launch_bounds__(1024) k_species_sum(int64_t n, int F, const int32_t *z, int max_z, const T *dUa,
                                                      const T *dVa, T *dU, T *dV) {
  __shared__ T lu[16][64];
  __shared__ T lv[16][64];
  const int sp = blockIdx.x;
  const int l = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int f = blockIdx.y * 64 + l;
  T u = T(0), v = T(0);
  if (f < F) {
    for (int64_t a = grp; a < n; a += 16) {
      if (clamp_z(z[a], max_z) != sp) continue;
      u += dUa[a * F + f];
      v += dVa[a * F + f];
    }
  }
  lu[grp][l] = u;
  lv[grp][l] = v;
  __syncthreads();
  if (grp == 0 && f < F) {
    T su = T(0), sv = T(0);
#pragma unroll
    for (int g = 0; g < 16; ++g) {
      su += lu[g][l];
      sv += lv[g][l];
    }
    dU[(int64_t)sp * F + f] = su;
    dV[(int64_t)sp * F + f] = sv;
  }
}

template <class S>
__global__ void k_grad_out(int64_t n, const Dual<S> *g, double *out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t < n) out[t] = (double)g[t].d;
}

// ---------------------------------------------------------------- workspace
template <class S>
struct TrainWs {
  using D = Dual<S>;
  void *plain = nullptr;
  size_t plain_bytes = 0;
  double *wt = nullptr;
  D *seed, *sd;
  NbrWs nb;
  D *wD, *gD, *dU, *dV, *dUa, *dVa, *part, *posD;
  D *geo, *phi, *rbf, *f0, *Xr, *T0, *nrm0, *xhat0, *rstd0, *n0, *ez1, *ea1, *ez2, *g;
  std::vector<D *> X, nX, Xb, Y, z1, a1, z2, a2, z3, h, M, P, nP, Pb, Dl;
  D *on, *oxhat, *orstd, *q, *oz, *ox, *hz, *hx;
  D *dX, *dD, *dPb, *dY, *dM, *dXr, *dT0, *dg, *dez2, *dez1, *dn0, *dnrm0, *dhz, *dox, *dq, *don;
  D *dh, *dz3, *dz2, *dz1, *dphi, *dvhat, *df0, *dZ;
  int64_t part_cap = 0;
};

// The weight blob's tensors come first in the packed copy, in blob order, ending with the
// output bias (one element).
inline int64_t param_count(const tn_model *m) { return (int64_t)m->off.bout + 1; }

template <class S>
static void plan_train(WsPlan &p, const tn_model *m, int64_t N, int64_t NS, int64_t MP, const BoxInfo &bi,
                       size_t plain_bytes, TrainWs<S> *w) {
  using D = Dual<S>;
  const int64_t F = m->F, K = m->K, L = m->L, Z = m->max_z;
  w->plain = p.take<char>(plain_bytes);
  w->plain_bytes = plain_bytes;
  w->wt = p.take<double>(3 * N);
  w->seed = p.take<D>(NS);
  w->sd = p.take<D>(N);
  plan_neighbors(p, N, MP, bi, &w->nb);
  w->wD = p.take<D>(m->off.total);
  w->gD = p.take<D>(param_count(m));
  w->dU = p.take<D>(Z * F);
  w->dV = p.take<D>(Z * F);
  w->dUa = p.take<D>(N * F);
  w->dVa = p.take<D>(N * F);
  // partial sums: up to 96 slices of the largest weight matrix (3F x 2F or 3F x K) and its bias
  w->part_cap = std::max<int64_t>((int64_t)96 * (std::max<int64_t>(6 * F * F, 3 * F * K) + 3 * F), kColSlices * 3 * F);
  w->part = p.take<D>(w->part_cap);
  w->posD = p.take<D>(3 * N);
  w->geo = p.take<D>(4 * MP);
  w->phi = p.take<D>(MP);
  w->rbf = p.take<D>(MP * K);
  w->f0 = p.take<D>(MP * 3 * F);
  w->Xr = p.take<D>(N * 9 * F);
  w->T0 = p.take<D>(N * 9 * F);
  w->nrm0 = p.take<D>(N * F);
  w->xhat0 = p.take<D>(N * F);
  w->rstd0 = p.take<D>(N);
  w->n0 = p.take<D>(N * F);
  w->ez1 = p.take<D>(N * 2 * F);
  w->ea1 = p.take<D>(N * 2 * F);
  w->ez2 = p.take<D>(N * 3 * F);
  w->g = p.take<D>(N * 3 * F);
  w->X.resize(L + 1);
  for (int64_t l = 0; l <= L; ++l) w->X[l] = p.take<D>(N * 9 * F);
  auto per_layer = [&](std::vector<D *> &v, int64_t count) {
    v.resize(L);
    for (int64_t l = 0; l < L; ++l) v[l] = p.take<D>(count);
  };
  per_layer(w->nX, N * F);
  per_layer(w->Xb, N * 9 * F);
  per_layer(w->Y, N * 9 * F);
  per_layer(w->z1, MP * F);
  per_layer(w->a1, MP * F);
  per_layer(w->z2, MP * 2 * F);
  per_layer(w->a2, MP * 2 * F);
  per_layer(w->z3, MP * 3 * F);
  per_layer(w->h, MP * 3 * F);
  per_layer(w->M, N * 9 * F);
  per_layer(w->P, N * 9 * F);
  per_layer(w->nP, N * F);
  per_layer(w->Pb, N * 9 * F);
  per_layer(w->Dl, N * 9 * F);
  w->on = p.take<D>(N * 3 * F);
  w->oxhat = p.take<D>(N * 3 * F);
  w->orstd = p.take<D>(N);
  w->q = p.take<D>(N * 3 * F);
  w->oz = p.take<D>(N * F);
  w->ox = p.take<D>(N * F);
  w->hz = p.take<D>(N * (F / 2));
  w->hx = p.take<D>(N * (F / 2));
  w->dX = p.take<D>(N * 9 * F);
  w->dD = p.take<D>(N * 9 * F);
  w->dPb = p.take<D>(N * 9 * F);
  w->dY = p.take<D>(N * 9 * F);
  w->dM = p.take<D>(N * 9 * F);
  w->dXr = p.take<D>(N * 9 * F);
  w->dT0 = p.take<D>(N * 9 * F);
  w->dg = p.take<D>(N * 3 * F);
  w->dez2 = p.take<D>(N * 3 * F);
  w->dez1 = p.take<D>(N * 2 * F);
  w->dn0 = p.take<D>(N * F);
  w->dnrm0 = p.take<D>(N * F);
  w->dhz = p.take<D>(N * (F / 2));
  w->dox = p.take<D>(N * F);
  w->dq = p.take<D>(N * 3 * F);
  w->don = p.take<D>(N * 3 * F);
  w->dh = p.take<D>(MP * 3 * F);
  w->dz3 = p.take<D>(MP * 3 * F);
  w->dz2 = p.take<D>(MP * 2 * F);
  w->dz1 = p.take<D>(MP * F);
  w->dphi = p.take<D>(MP);
  w->dvhat = p.take<D>(3 * MP);
  w->df0 = p.take<D>(MP * 3 * F);
  w->dZ = p.take<D>(MP * 2 * F);
}

// Pass 1 (energies and forces) runs on the fused path in FP32 where its pair kernels cover the
// model's sizes, else on the plain path.
static bool pass1_fused(const tn_model *m, int prec) {
  return prec == TN_FP32 && pair_kernels_support(m->F, m->K, m->L, false);
}
static size_t pass1_bytes(const tn_model *m, int64_t n, int64_t ns, int64_t mp, const BoxInfo &bi, int prec) {
  return pass1_fused(m, prec) ? fused_workspace_bytes(m, n, ns, mp, bi, prec, 1)
                              : plain_workspace_bytes(m, n, ns, mp, bi, prec, 1);
}

static size_t train_bytes(const tn_model *m, int64_t n, int64_t ns, int64_t mp, const BoxInfo &bi, int prec) {
  const size_t pb = pass1_bytes(m, n, ns, mp, bi, prec);
  WsPlan p(nullptr);
  if (prec == TN_FP64) {
    TrainWs<double> w;
    plan_train(p, m, n, ns, mp, bi, pb, &w);
  } else {
    TrainWs<float> w;
    plan_train(p, m, n, ns, mp, bi, pb, &w);
  }
  return p.off;
}

// ---------------------------------------------------------------- the step
template <class S>
static int run_train(const tn_model *m, hipStream_t s, const Problem &pb, const double *Eref, const double *Fref,
                     double wE, double wF, double *loss, double *grad, void *ws, size_t ws_bytes) {
  using D = Dual<S>;
  const int64_t N = pb.n, NS = pb.S, MP = pb.max_pairs, F = m->F, K = m->K, L = m->L, Z = m->max_z;
  const int64_t H = F / 2;
  const int prec = std::is_same<S, double>::value ? TN_FP64 : TN_FP32;
  const size_t plain_bytes = pass1_bytes(m, N, NS, MP, pb.box, prec);
  WsPlan plan(ws);
  TrainWs<S> w;
  plan_train(plan, m, N, NS, MP, pb.box, plain_bytes, &w);
  if (plan.off > ws_bytes) return TN_E_WORKSPACE;
  int rc;
  const unsigned bs = 256;
  const WeightOff &o = m->off;
  const int64_t NP = param_count(m);

  // ---- pass 1: energies and forces at r, the loss, its seeds and the position tangent
  rc = pass1_fused(m, prec) ? fused_run(m, s, pb, prec, w.plain, w.plain_bytes)
                            : plain_run(m, s, pb, prec, w.plain, w.plain_bytes);
  if (rc) return rc;
  hipLaunchKernelGGL(k_loss<S>, dim3(1), dim3(256), 0, s, N, NS, pb.energy, Eref, static_cast<const S *>(pb.forces),
                     Fref, wE, wF, loss, w.seed, w.wt);
  TN_LAUNCH_CHECK();

  // ---- pass 2: dual forward
  hipLaunchKernelGGL(k_to_dual<S>, dim3(grid_for((int64_t)o.total, bs)), dim3(bs), 0, s, (int64_t)o.total, m->w64,
                     w.wD);
  TN_LAUNCH_CHECK();
  if ((rc = fill_bytes_zero(s, w.gD, NP * sizeof(D)))) return rc;
  auto W = [&](size_t off) { return static_cast<const D *>(w.wD + off); };
  auto Wr = [&](size_t off) { return wptr<S>(m, off); };   // real weights for the matrix products
  auto G = [&](size_t off) { return w.gD + off; };
  Reducer<D> red{w.part, w.part_cap};

  NbrGraph<S> gr;
  if ((rc = build_neighbors<S>(s, N, static_cast<const S *>(pb.pos), pb.z, pb.batch, pb.box, m->r_c, MP, nullptr,
                               pb.n_pairs, pb.status, w.nb, &gr, NS, m->max_z)))
    return rc;
  const int64_t *np = pb.n_pairs;
  const int32_t *rowptr = gr.rowptr, *nbr = gr.nbr, *pid = gr.pid, *zz = gr.z;
  const unsigned gN = grid_for(N, bs), gNF = grid_for(N * F, bs);
  if (N > 0) {
    hipLaunchKernelGGL(k_pos_dual<S>, dim3(gN), dim3(bs), 0, s, N, gr.pos, gr.perm, (const double *)w.wt, w.posD);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_seed_atoms<D>, dim3(gN), dim3(bs), 0, s, N, NS, gr.batch, (const D *)w.seed, w.sd);
    TN_LAUNCH_CHECK();
  }
  if (MP > 0) {
    hipLaunchKernelGGL(k_geom_dual<S>, dim3(grid_for(MP, bs)), dim3(bs), 0, s, gr.pairs, MP, np,
                       (const D *)w.posD, pb.box.lat, m->r_c, m->r_lo, m->alpha, m->w64 + o.mu, m->w64 + o.beta,
                       (int)K, w.geo, w.phi, w.rbf);
    TN_LAUNCH_CHECK();
  }
  // embedding
  if ((rc = dlinear_fwd<S>(s, w.rbf, MP, K, Wr(o.W0), Wr(o.b0), 3 * F, w.f0, nullptr, 0, nullptr, np))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_embed_gather<D>, dim3(gNF), dim3(bs), 0, s, N, (int)F, rowptr, nbr, pid, np, MP, zz,
                       m->max_z, W(o.U), W(o.V), (const D *)w.geo, (const D *)w.phi, (const D *)w.f0, w.Xr);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_node_norm<D>, dim3(gNF), dim3(bs), 0, s, N, (int)F, (const D *)w.Xr, w.nrm0);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_layernorm<D>, dim3(layernorm_grid(N)), dim3(256), 0, s, N, (int)F, (const D *)w.nrm0,
                       W(o.ln_g), W(o.ln_b), w.n0, w.xhat0, w.rstd0);
    TN_LAUNCH_CHECK();
  }
  if ((rc = dlinear_fwd<S>(s, w.n0, N, F, Wr(o.W1), Wr(o.b1), 2 * F, w.ea1, w.ez1, 1))) return rc;
  if ((rc = dlinear_fwd<S>(s, w.ea1, N, 2 * F, Wr(o.W2), Wr(o.b2), 3 * F, w.g, w.ez2, 1))) return rc;
  const S *Wemb[3] = {Wr(o.Wmix[0]), Wr(o.Wmix[1]), Wr(o.Wmix[2])};
  if ((rc = dmix<S>(s, w.Xr, w.T0, N, F, Wemb, 0, 0))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_gate<D>, dim3(grid_for(N * 9 * F, bs)), dim3(bs), 0, s, N, (int)F, (const D *)w.g,
                       (const D *)w.T0, w.X[0]);
    TN_LAUNCH_CHECK();
  }
  // interaction layers
  for (int64_t l = 0; l < L; ++l) {
    const LayerOff &lo = o.layer[l];
    if (N > 0) {
      hipLaunchKernelGGL(k_normalize<D>, dim3(gNF), dim3(bs), 0, s, N, (int)F, (const D *)w.X[l], w.nX[l], w.Xb[l]);
      TN_LAUNCH_CHECK();
    }
    const S *W1[3] = {Wr(lo.W1[0]), Wr(lo.W1[1]), Wr(lo.W1[2])};
    if ((rc = dmix<S>(s, w.Xb[l], w.Y[l], N, F, W1, 0, 0))) return rc;
    if ((rc = dlinear_fwd<S>(s, w.rbf, MP, K, Wr(lo.Wa), Wr(lo.ba), F, w.a1[l], w.z1[l], 1, nullptr, np))) return rc;
    if ((rc = dlinear_fwd<S>(s, w.a1[l], MP, F, Wr(lo.Wb), Wr(lo.bb), 2 * F, w.a2[l], w.z2[l], 1, nullptr, np)))
      return rc;
    if ((rc = dlinear_fwd<S>(s, w.a2[l], MP, 2 * F, Wr(lo.Wc), Wr(lo.bc), 3 * F, w.h[l], w.z3[l], 1, w.phi, np)))
      return rc;
    if (N > 0) {
      if ((rc = dmessage<D>(s, N, F, rowptr, nbr, pid, np, MP, w.h[l], w.Y[l], w.M[l], 0))) return rc;
      hipLaunchKernelGGL(k_product<D>, dim3(gNF), dim3(bs), 0, s, N, (int)F, (const D *)w.Y[l], (const D *)w.M[l],
                         w.P[l], w.nP[l], w.Pb[l]);
      TN_LAUNCH_CHECK();
    }
    const S *W2[3] = {Wr(lo.W2[0]), Wr(lo.W2[1]), Wr(lo.W2[2])};
    if ((rc = dmix<S>(s, w.Pb[l], w.Dl[l], N, F, W2, 0, 0))) return rc;
    if (N > 0) {
      hipLaunchKernelGGL(k_residual<D>, dim3(gNF), dim3(bs), 0, s, N, (int)F, (const D *)w.Xb[l], (const D *)w.Dl[l],
                         w.X[l + 1]);
      TN_LAUNCH_CHECK();
    }
  }
  // output network
  if (N > 0) {
    hipLaunchKernelGGL(k_out_norms<D>, dim3(gNF), dim3(bs), 0, s, N, (int)F, (const D *)w.X[L], w.on);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_layernorm<D>, dim3(layernorm_grid(N)), dim3(256), 0, s, N, (int)(3 * F), (const D *)w.on,
                       W(o.oln_g), W(o.oln_b), w.q, w.oxhat, w.orstd);
    TN_LAUNCH_CHECK();
  }
  if ((rc = dlinear_fwd<S>(s, w.q, N, 3 * F, Wr(o.Wo), Wr(o.bo), F, w.ox, w.oz, 1))) return rc;
  if ((rc = dlinear_fwd<S>(s, w.ox, N, F, Wr(o.Wh), Wr(o.bh), H, w.hx, w.hz, 1))) return rc;

  // ---- pass 2: reverse sweep to the parameters, seeds sd_i = seed_{system of i}
  if (N > 0) {
    hipLaunchKernelGGL(k_out_final_bwd_seed<D>, dim3(grid_for(N * H, bs)), dim3(bs), 0, s, N, (int)H,
                       (const D *)w.hz, W(o.wout), (const D *)w.sd, w.dhz);
    TN_LAUNCH_CHECK();
  }
  if ((rc = red.coldot(s, w.hx, nullptr, w.sd, N, nullptr, (int)H, G(o.wout)))) return rc;
  if ((rc = red.coldot(s, w.sd, nullptr, nullptr, N, nullptr, 1, G(o.bout)))) return rc;
  if ((rc = red.linear(s, w.dhz, w.ox, N, nullptr, (int)H, (int)F, G(o.Wh), G(o.bh)))) return rc;
  if ((rc = dlinear_bwd<S>(s, w.dhz, N, H, Wr(o.Wh), F, w.dox, w.oz, 0))) return rc;
  if ((rc = red.linear(s, w.dox, w.q, N, nullptr, (int)F, (int)(3 * F), G(o.Wo), G(o.bo)))) return rc;
  if ((rc = dlinear_bwd<S>(s, w.dox, N, F, Wr(o.Wo), 3 * F, w.dq, nullptr, 0))) return rc;
  if ((rc = red.coldot(s, w.dq, w.oxhat, nullptr, N, nullptr, (int)(3 * F), G(o.oln_g)))) return rc;
  if ((rc = red.coldot(s, w.dq, nullptr, nullptr, N, nullptr, (int)(3 * F), G(o.oln_b)))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_layernorm_bwd<D>, dim3(layernorm_grid(N)), dim3(256), 0, s, N, (int)(3 * F), (const D *)w.dq,
                       (const D *)w.oxhat, (const D *)w.orstd, W(o.oln_g), w.don);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_out_norms_bwd<D>, dim3(gNF), dim3(bs), 0, s, N, (int)F, (const D *)w.X[L],
                       (const D *)w.don, w.dX);
    TN_LAUNCH_CHECK();
  }
  if (MP > 0 && (rc = fill_bytes_zero(s, w.dphi, MP * sizeof(D)))) return rc;
  for (int64_t l = L - 1; l >= 0; --l) {
    const LayerOff &lo = o.layer[l];
    const S *W1[3] = {Wr(lo.W1[0]), Wr(lo.W1[1]), Wr(lo.W1[2])};
    const S *W2[3] = {Wr(lo.W2[0]), Wr(lo.W2[1]), Wr(lo.W2[2])};
    if (N > 0) {
      hipLaunchKernelGGL(k_residual_bwd<D>, dim3(gNF), dim3(bs), 0, s, N, (int)F, (const D *)w.Dl[l],
                         (const D *)w.dX, w.dD);
      TN_LAUNCH_CHECK();
    }
    for (int q = 0; q < 3; ++q)
      if ((rc = red.wgrad(s, w.dD, part_rows(q, F), w.Pb[l], part_rows(q, F), N * part_count(q), nullptr, (int)F,
                          (int)F, G(lo.W2[q]), F)))
        return rc;
    if ((rc = dmix<S>(s, w.dD, w.dPb, N, F, W2, 1, 0))) return rc;
    if (N > 0) {
      hipLaunchKernelGGL(k_product_bwd<D>, dim3(gNF), dim3(bs), 0, s, N, (int)F, (const D *)w.dPb, (const D *)w.P[l],
                         (const D *)w.nP[l], (const D *)w.Y[l], (const D *)w.M[l], w.dY, w.dM, nullptr);
      TN_LAUNCH_CHECK();
      if ((rc = dmessage<D>(s, N, F, rowptr, nbr, pid, np, MP, w.h[l], w.dM, w.dY, 1))) return rc;
    }
    if (MP > 0) {
      hipLaunchKernelGGL(k_message_bwd_pair<D>, dim3(grid_for(MP * F, bs)), dim3(bs), 0, s, gr.pairs, MP, np, (int)F,
                         (const D *)w.Y[l], (const D *)w.dM, w.dh);
      TN_LAUNCH_CHECK();
    }
    for (int q = 0; q < 3; ++q)
      if ((rc = red.wgrad(s, w.dY, part_rows(q, F), w.Xb[l], part_rows(q, F), N * part_count(q), nullptr, (int)F,
                          (int)F, G(lo.W1[q]), F)))
        return rc;
    if ((rc = dmix<S>(s, w.dY, w.dX, N, F, W1, 1, 1))) return rc;
    if (N > 0) {
      hipLaunchKernelGGL(k_normalize_bwd<D>, dim3(gNF), dim3(bs), 0, s, N, (int)F, (const D *)w.X[l],
                         (const D *)w.nX[l], w.dX);
      TN_LAUNCH_CHECK();
    }
    if (MP > 0) {
      hipLaunchKernelGGL(k_edge_bwd_top<D>, dim3((unsigned)MP), dim3(128), 0, s, MP, np, (int)(3 * F),
                         (const D *)w.dh, (const D *)w.z3[l], (const D *)w.phi, w.dz3, w.dphi);
      TN_LAUNCH_CHECK();
    }
    if ((rc = red.linear(s, w.dz3, w.a2[l], MP, np, (int)(3 * F), (int)(2 * F), G(lo.Wc), G(lo.bc)))) return rc;
    if ((rc = dlinear_bwd<S>(s, w.dz3, MP, 3 * F, Wr(lo.Wc), 2 * F, w.dz2, w.z2[l], 0, np))) return rc;
    if ((rc = red.linear(s, w.dz2, w.a1[l], MP, np, (int)(2 * F), (int)F, G(lo.Wb), G(lo.bb)))) return rc;
    if ((rc = dlinear_bwd<S>(s, w.dz2, MP, 2 * F, Wr(lo.Wb), F, w.dz1, w.z1[l], 0, np))) return rc;
    if ((rc = red.linear(s, w.dz1, w.rbf, MP, np, (int)F, (int)K, G(lo.Wa), G(lo.ba)))) return rc;
  }
  // embedding: dX holds dE/dX0
  if (N > 0) {
    hipLaunchKernelGGL(k_gate_bwd<D>, dim3(gNF), dim3(bs), 0, s, N, (int)F, (const D *)w.dX, (const D *)w.T0,
                       (const D *)w.g, w.dg, w.dT0, nullptr);
    TN_LAUNCH_CHECK();
  }
  for (int q = 0; q < 3; ++q)
    if ((rc = red.wgrad(s, w.dT0, part_rows(q, F), w.Xr, part_rows(q, F), N * part_count(q), nullptr, (int)F, (int)F,
                        G(o.Wmix[q]), F)))
      return rc;
  if ((rc = dmix<S>(s, w.dT0, w.dXr, N, F, Wemb, 1, 0))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_mul_silu_grad<D>, dim3(grid_for(N * 3 * F, bs)), dim3(bs), 0, s, N * 3 * F, (const D *)w.dg,
                       (const D *)w.ez2, w.dez2);
    TN_LAUNCH_CHECK();
  }
  if ((rc = red.linear(s, w.dez2, w.ea1, N, nullptr, (int)(3 * F), (int)(2 * F), G(o.W2), G(o.b2)))) return rc;
  if ((rc = dlinear_bwd<S>(s, w.dez2, N, 3 * F, Wr(o.W2), 2 * F, w.dez1, w.ez1, 0))) return rc;
  if ((rc = red.linear(s, w.dez1, w.n0, N, nullptr, (int)(2 * F), (int)F, G(o.W1), G(o.b1)))) return rc;
  if ((rc = dlinear_bwd<S>(s, w.dez1, N, 2 * F, Wr(o.W1), F, w.dn0, nullptr, 0))) return rc;
  if ((rc = red.coldot(s, w.dn0, w.xhat0, nullptr, N, nullptr, (int)F, G(o.ln_g)))) return rc;
  if ((rc = red.coldot(s, w.dn0, nullptr, nullptr, N, nullptr, (int)F, G(o.ln_b)))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_layernorm_bwd<D>, dim3(layernorm_grid(N)), dim3(256), 0, s, N, (int)F, (const D *)w.dn0,
                       (const D *)w.xhat0, (const D *)w.rstd0, W(o.ln_g), w.dnrm0);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_norm_bwd_add<D>, dim3(gNF), dim3(bs), 0, s, N, (int)F, (const D *)w.Xr, (const D *)w.dnrm0,
                       w.dXr);
    TN_LAUNCH_CHECK();
  }
  if (MP > 0) {
    hipLaunchKernelGGL(k_embed_bwd_pair<D>, dim3((unsigned)MP), dim3(128), 0, s, gr.pairs, MP, np, (int)F, zz,
                       m->max_z, W(o.U), W(o.V), (const D *)w.geo, (const D *)w.phi, (const D *)w.f0,
                       (const D *)w.dXr, w.df0, w.dphi, w.dvhat);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_embed_dz<D>, dim3(grid_for(MP * F, bs)), dim3(bs), 0, s, gr.pairs, MP, np, (int)F,
                       (const D *)w.geo, (const D *)w.phi, (const D *)w.f0, (const D *)w.dXr, w.dZ);
    TN_LAUNCH_CHECK();
  }
  if ((rc = red.linear(s, w.df0, w.rbf, MP, np, (int)(3 * F), (int)K, G(o.W0), G(o.b0)))) return rc;
  // species tables U = W_z[:, :F] E + b_z, V = W_z[:, F:] E  ->  E, W_z, b_z
  if (N > 0) {
    hipLaunchKernelGGL(k_atom_dz<D>, dim3(gNF), dim3(bs), 0, s, N, (int)F, rowptr, nbr, pid, np, MP,
                       (const D *)w.dZ, w.dUa, w.dVa);
    TN_LAUNCH_CHECK();
  }
  {
    hipLaunchKernelGGL(k_species_sum<D>, dim3((unsigned)Z, (unsigned)((F + 63) / 64)), dim3(1024), 0, s, N, (int)F,
                       zz, m->max_z, (const D *)w.dUa, (const D *)w.dVa, w.dU, w.dV);
    TN_LAUNCH_CHECK();
    if ((rc = red.wgrad(s, w.dU, rows_of(F), W(o.E), rows_of(F), Z, nullptr, (int)F, (int)F, G(o.Wz), 2 * F)))
      return rc;
    if ((rc = red.wgrad(s, w.dV, rows_of(F), W(o.E), rows_of(F), Z, nullptr, (int)F, (int)F, G(o.Wz) + F, 2 * F)))
      return rc;
    if ((rc = red.coldot(s, w.dU, nullptr, nullptr, Z, nullptr, (int)F, G(o.bz)))) return rc;
    for (int half = 0; half < 2; ++half) {
      DualGemmArgs<S> ga;
      ga.A = half ? w.dV : w.dU; ga.lda = F;
      ga.B = Wr(o.Wz) + half * F; ga.ldb = 2 * F; ga.transB = 0;
      ga.C = G(o.E); ga.ldc = F; ga.accumulate = 1;
      ga.M = Z; ga.N = F; ga.K = F;
      if ((rc = dgemm(s, ga))) return rc;
    }
  }
  if (NP > 0) {
    hipLaunchKernelGGL(k_grad_out<S>, dim3(grid_for(NP, bs)), dim3(bs), 0, s, NP, (const D *)w.gD, grad);
    TN_LAUNCH_CHECK();
  }
  return TN_OK;
}

}  // namespace tn

using namespace tn;

extern "C" {

int64_t tn_param_count(const tn_model *m) { return m ? param_count(m) : -1; }

size_t tn_train_workspace_bytes(const tn_model *m, int64_t n_atoms, int64_t n_systems, int64_t max_pairs,
                                const double *box, int precision) {
  if (!m || n_atoms < 0 || n_systems < 0 || max_pairs < 0) return 0;
  if (precision != TN_FP32 && precision != TN_FP64) return 0;
  BoxInfo bi;
  if (box_info(box, m->r_c, &bi)) return 0;
  return train_bytes(m, n_atoms, n_systems, max_pairs, bi, precision);
}

int tn_train_grad(const tn_model *m, void *stream, int64_t n_atoms, int64_t n_systems, const void *pos,
                  const int32_t *z, const int32_t *batch, const double *box, int64_t max_pairs, int precision,
                  const double *energy_ref, const double *forces_ref, double w_energy, double w_force, double *loss,
                  double *energy, void *forces, double *grad, int64_t *n_pairs, int32_t *status, void *ws,
                  size_t ws_bytes) {
  if (!m || n_atoms < 0 || n_systems < 0 || max_pairs < 0 || max_pairs > (int64_t(1) << 30) ||
      n_atoms >= (int64_t(1) << 31))
    return TN_E_ARG;
  if (precision != TN_FP32 && precision != TN_FP64) return TN_E_UNSUPPORTED;
  if (n_atoms > 0 && (!pos || !z || !batch || n_systems < 1 || !forces || !forces_ref)) return TN_E_ARG;
  if (n_systems > 0 && (!energy || !energy_ref)) return TN_E_ARG;
  if (!loss || !grad || !n_pairs || !status || !ws) return TN_E_ARG;
  if (!std::isfinite(w_energy) || !std::isfinite(w_force)) return TN_E_ARG;
  Problem pb;
  int rc = box_info(box, m->r_c, &pb.box);
  if (rc) return rc;
  if (hipSetDevice(m->device) != hipSuccess) return TN_E_HIP;
  pb.n = n_atoms;
  pb.S = n_systems;
  pb.max_pairs = max_pairs;
  pb.pos = pos;
  pb.z = z;
  pb.batch = batch;
  pb.energy = energy;
  pb.forces = forces;
  pb.n_pairs = n_pairs;
  pb.status = status;
  pb.want_forces = true;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((rc = fill_i32(s, status, 1, 0))) return rc;
  if (precision == TN_FP64)
    return run_train<double>(m, s, pb, energy_ref, forces_ref, w_energy, w_force, loss, grad, ws, ws_bytes);
  return run_train<float>(m, s, pb, energy_ref, forces_ref, w_energy, w_force, loss, grad, ws, ws_bytes);
}

}  // extern "C"
