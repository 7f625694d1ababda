// Plain (unfused) TensorNet path: one kernel per operation, every intermediate
// kept in device memory, templated on the arithmetic type (float or double).
// It is the baseline the fused path is measured against, and in double it is
// the GPU-side correctness anchor.  Math follows TensorNet as described in
// Sec. 2.1.1 of the paper (I/A/S decomposition, channel mixing, messages,
// symmetric matrix products, normalisation) with the settings of Sec. 2.4
// (exp-normal basis, cosine cutoff, SiLU); energies are summed per system and
// forces are the negative position gradient (Sec. 2), here by a hand-written
// reverse sweep.
#include "tn_internal.h"
#include "tn_device.h"

#include <cmath>

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

constexpr int GBM = 64, GBN = 64, GBK = 16;

template <class T>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs<T> g) {
  __shared__ T As[GBK][GBM + 1];
  __shared__ T Bs[GBK][GBN + 1];
  int64_t Mrows = g.M;
  if (g.Mdev) {
    const int64_t md = *g.Mdev;
    if (md < Mrows) Mrows = md;
  }
  const int64_t m0 = (int64_t)blockIdx.y * GBM;
  const int64_t n0 = (int64_t)blockIdx.x * GBN;
  if (m0 >= Mrows) return;
  const int z = blockIdx.z;
  const T *A = g.A + z * g.zoff;
  const T *B = g.zpart ? g.Bz[coord_part(z)] : g.B;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  T acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = T(0);
  for (int64_t k0 = 0; k0 < g.K; k0 += GBK) {
    // A tile: GBM x GBK
    for (int t = threadIdx.x; t < GBM * GBK; t += 256) {
      const int mm_ = t / GBK, kk = t % GBK;
      const int64_t m = m0 + mm_, k = k0 + kk;
      As[kk][mm_] = (m < Mrows && k < g.K) ? A[m * g.lda + k] : T(0);
    }
    for (int t = threadIdx.x; t < GBK * GBN; t += 256) {
      int kk, nn;
      if (g.transB) { nn = t / GBK; kk = t % GBK; } else { kk = t / GBN; nn = t % GBN; }
      const int64_t n = n0 + nn, k = k0 + kk;
      T v = T(0);
      if (n < g.N && k < g.K) v = g.transB ? B[n * g.ldb + k] : B[k * g.ldb + n];
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GBK; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty + 16 * r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx + 16 * c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] += a[r] * b[c];
    }
    __syncthreads();
  }
  T *C = g.C + z * g.zoff;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t m = m0 + ty + 16 * r;
    if (m >= Mrows) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int64_t n = n0 + tx + 16 * c;
      if (n >= g.N) continue;
      T v = acc[r][c];
      if (g.bias) v += g.bias[n];
      if (g.Z) g.Z[z * g.zoff + m * g.ldz + n] = v;
      if (g.act == 1) v = silu(v);
      if (g.rowscale) v *= g.rowscale[m];
      if (g.gate) v *= silu_grad(g.gate[z * g.zoff + m * g.ldg + n]);
      T *dst = C + m * g.ldc + n;
      if (g.accumulate) *dst += v; else *dst = v;
    }
  }
}

template <class T>
static int gemm(hipStream_t s, const GemmArgs<T> &g, int zdim = 1) {
  if (g.M <= 0 || g.N <= 0) return TN_OK;
  dim3 grid((unsigned)((g.N + GBN - 1) / GBN), (unsigned)((g.M + GBM - 1) / GBM), (unsigned)zdim);
  hipLaunchKernelGGL(k_gemm<T>, grid, dim3(256), 0, s, g);
  TN_LAUNCH_CHECK();
  return TN_OK;
}

// y = act(x W^T + b) over rows of x; W is [Nout, Kin] (torch Linear layout).
template <class T>
static int linear_fwd(hipStream_t s, const T *x, int64_t M, int64_t Kin, const T *W, const T *b, int64_t Nout,
                      T *y, T *z_pre, int act, const T *rowscale = nullptr, const int64_t *Mdev = nullptr) {
  GemmArgs<T> g;
  g.A = x; g.lda = Kin; g.B = W; g.ldb = Kin; g.transB = 1;
  g.C = y; g.ldc = Nout; g.bias = b; g.Z = z_pre; g.ldz = Nout; g.act = act; g.rowscale = rowscale;
  g.M = M; g.N = Nout; g.K = Kin; g.Mdev = Mdev;
  return gemm(s, g);
}

// dx (+)= (dy W) * silu'(gate); W is [Nout, Kin], dy [M, Nout], dx [M, Kin].
template <class T>
static int linear_bwd(hipStream_t s, const T *dy, int64_t M, int64_t Nout, const T *W, int64_t Kin, T *dx,
                      const T *gate, int accumulate, const int64_t *Mdev = nullptr) {
  GemmArgs<T> g;
  g.A = dy; g.lda = Nout; g.B = W; g.ldb = Kin; g.transB = 0;
  g.C = dx; g.ldc = Kin; g.gate = gate; g.ldg = Kin; g.accumulate = accumulate;
  g.M = M; g.N = Kin; g.K = Nout; g.Mdev = Mdev;
  return gemm(s, g);
}

// Per-part channel mixing of [N, 9, F] features: out[n,c,:] = W_part(c) in[n,c,:] (forward)
// or out[n,c,:] (+)= in[n,c,:] W_part(c) (adjoint).
template <class T>
static int mix(hipStream_t s, const T *in, T *out, int64_t N, int64_t F, const T *W[3], int adjoint,
               int accumulate) {
  GemmArgs<T> g;
  g.A = in; g.lda = 9 * F; g.C = out; g.ldc = 9 * F; g.transB = adjoint ? 0 : 1; g.ldb = F;
  g.M = N; g.N = F; g.K = F; g.zoff = F; g.zpart = 1; g.accumulate = accumulate;
  for (int q = 0; q < 3; ++q) g.Bz[q] = W[q];
  return gemm(s, g, 9);
}

// ============================================================================ element kernels
__device__ inline bool pairs_ok(const int64_t *n_pairs, int64_t max_pairs) { return *n_pairs <= max_pairs; }

__device__ inline int64_t pair_bound(const int64_t *n_pairs, int64_t max_pairs) {
  const int64_t P = *n_pairs;
  return P < max_pairs ? P : max_pairs;
}

struct BoxLen {
  int periodic;
  double len[3];
};

template <class T>
__global__ void k_check_inputs(const int32_t *z, const int32_t *batch, int64_t n, int64_t S, int max_z,
                               int32_t *status) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (z[i] < 0 || z[i] >= max_z) set_status(status, TN_STATUS_Z);
  if (batch[i] < 0 || batch[i] >= S) set_status(status, TN_STATUS_BATCH);
}

__device__ inline int clamp_z(int32_t z, int max_z) { return z < 0 ? 0 : (z >= max_z ? max_z - 1 : z); }

// Per pair: unit vector, distance, cutoff phi(d), exp-normal basis e_k(d).  Evaluated in
// FP64 from the (promoted) input positions and rounded once to T: the narrow Gaussians of
// the exp-normal basis amplify rounding in d by up to 2*alpha*beta*u*|u - mu_k|.
template <class T>
__global__ void k_geom(const int32_t *pairs, int64_t max_pairs, const int64_t *n_pairs, const T *pos, BoxLen box,
                       double r_c, double r_lo, double alpha, const double *mu, const double *beta, int K, T *geo,
                       T *phi, T *rbf) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= pair_bound(n_pairs, max_pairs)) return;
  const int64_t i = pairs[p], j = pairs[max_pairs + p];
  double v[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double dlt = (double)pos[3 * j + a] - (double)pos[3 * i + a];
    if (box.periodic) dlt -= box.len[a] * rint(dlt / box.len[a]);
    v[a] = dlt;
  }
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

template <class T>
__global__ void k_node_norm(int64_t n, int F, const T *X, T *nrm) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T c[9];
  load9(X, i, F, f, c);
  nrm[i * F + f] = norm9(c);
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

// LayerNorm over rows of length C (population variance, eps 1e-5, affine g/b).
template <class T>
__global__ void __launch_bounds__(128) k_layernorm(int64_t rows, int C, const T *x, const T *gmul, const T *badd,
                                                   T *y, T *xhat, T *rstd) {
  __shared__ T lds[128];
  const int64_t r = blockIdx.x;
  if (r >= rows) return;
  T s = T(0);
  for (int k = threadIdx.x; k < C; k += 128) s += x[r * C + k];
  const T mean = block_sum(s, lds) / T(C);
  T v = T(0);
  for (int k = threadIdx.x; k < C; k += 128) {
    const T d = x[r * C + k] - mean;
    v += d * d;
  }
  const T var = block_sum(v, lds) / T(C);
  const T rs = T(1) / dsqrt(var + T(1e-5));
  for (int k = threadIdx.x; k < C; k += 128) {
    const T h = (x[r * C + k] - mean) * rs;
    xhat[r * C + k] = h;
    y[r * C + k] = h * gmul[k] + badd[k];
  }
  if (threadIdx.x == 0) rstd[r] = rs;
}

// dx = rstd * (g*dy - mean(g*dy) - xhat * mean(g*dy*xhat))
template <class T>
__global__ void __launch_bounds__(128) k_layernorm_bwd(int64_t rows, int C, const T *dy, const T *xhat,
                                                       const T *rstd, const T *gmul, T *dx) {
  __shared__ T lds[128];
  const int64_t r = blockIdx.x;
  if (r >= rows) return;
  T s1 = T(0), s2 = T(0);
  for (int k = threadIdx.x; k < C; k += 128) {
    const T gd = gmul[k] * dy[r * C + k];
    s1 += gd;
    s2 += gd * xhat[r * C + k];
  }
  const T m1 = block_sum(s1, lds) / T(C);
  const T m2 = block_sum(s2, lds) / T(C);
  const T rs = rstd[r];
  for (int k = threadIdx.x; k < C; k += 128)
    dx[r * C + k] = rs * (gmul[k] * dy[r * C + k] - m1 - xhat[r * C + k] * m2);
}

template <class T>
__global__ void k_gate(int64_t n, int F, const T *g, const T *T0, T *X) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * 9 * F) return;
  const int64_t i = t / (9 * F);
  const int rem = (int)(t % (9 * F));
  const int q = rem / F, f = rem % F;
  X[t] = g[i * 3 * F + coord_part(q) * F + f] * T0[t];
}

template <class T>
__global__ void k_normalize(int64_t n, int F, const T *X, T *nX, T *Xb) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
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

// X_out = Xb + D + D D
template <class T>
__global__ void k_residual(int64_t n, int F, const T *Xb, const T *D, T *Xo) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
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
__global__ void k_out_norms(int64_t n, int F, const T *X, T *on) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T c[9];
  load9(X, i, F, f, c);
  on[i * 3 * F + f] = norm_I(c);
  on[i * 3 * F + F + f] = norm_A(c);
  on[i * 3 * F + 2 * F + f] = norm_S(c);
}

// eps_i = w . hx_i + b (final scalar of the output network)
template <class T>
__global__ void k_out_final(int64_t n, int H, const T *hx, const T *w, const T *b, T *eps) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  T s = b[0];
  for (int k = 0; k < H; ++k) s += w[k] * hx[i * H + k];
  eps[i] = s;
}

// E_s = sum over the (contiguous) atoms of system s, in FP64; one block per system.
template <class T>
__global__ void __launch_bounds__(128) k_energy_reduce(int64_t n, const T *eps, const int32_t *batch, double *E,
                                                       int32_t *status) {
  __shared__ double lds[128];
  const int32_t s = blockIdx.x;
  int64_t a = 0, e = n;
  while (a < e) {
    const int64_t m = (a + e) >> 1;
    if (batch[m] < s) a = m + 1; else e = m;
  }
  const int64_t lo = a;
  e = n;
  while (a < e) {
    const int64_t m = (a + e) >> 1;
    if (batch[m] <= s) a = m + 1; else e = m;
  }
  const int64_t hi = a;
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 128) acc += (double)eps[i];
  const double tot = block_sum(acc, lds);
  if (threadIdx.x == 0) {
    E[s] = tot;
    if (!isfinite(tot)) set_status(status, TN_STATUS_NONFINITE);
  }
}

// ----------------------------------------------------------------------------- backward kernels
template <class T>
__global__ void k_out_final_bwd(int64_t n, int H, const T *hz, const T *w, T *dhz) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * H) return;
  const int k = (int)(t % H);
  dhz[t] = w[k] * silu_grad(hz[t]);
}

// adjoint of the part norms: dX = sum_part d(norm_part) * grad(norm_part)
template <class T>
__global__ void k_out_norms_bwd(int64_t n, int F, const T *X, const T *don, T *dX) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T c[9], d[9];
  load9(X, i, F, f, c);
  norm_grad_parts(c, don[i * 3 * F + f], don[i * 3 * F + F + f], don[i * 3 * F + 2 * F + f], d);
  store9(dX, i, F, f, d);
}

// X_out = Xb + D + DD:  dD = dX + rec^T(dQ D^T + D^T dQ) with dQ = dec^T(dX)
template <class T>
__global__ void k_residual_bwd(int64_t n, int F, const T *D, const T *dX, T *dD) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
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
  for (int q = 0; q < 9; ++q) r[q] += g[q];
  store9(dD, i, F, f, r);
}

// Through Pb = P/(||P||+1) and P = Y M + M Y: dY (overwritten) and dM.
template <class T>
__global__ void k_product_bwd(int64_t n, int F, const T *dPb, const T *P, const T *nP, const T *Y, const T *M,
                              T *dY, T *dM) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T g[9], pc[9], gn[9];
  load9(dPb, i, F, f, g);
  load9(P, i, F, f, pc);
  const T s = T(1) / (nP[i * F + f] + T(1));
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
__global__ void k_normalize_bwd(int64_t n, int F, const T *X, const T *nX, T *g) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
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
template <class T>
__global__ void k_gate_bwd(int64_t n, int F, const T *dX, const T *T0, const T *g, T *dg, T *dT0) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T s[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int64_t o = i * 9 * F + q * F + f;
    const int pt = coord_part(q);
    s[pt] += dX[o] * T0[o];
    dT0[o] = g[i * 3 * F + pt * F + f] * dX[o];
  }
#pragma unroll
  for (int q = 0; q < 3; ++q) dg[i * 3 * F + q * F + f] = s[q];
}

template <class T>
__global__ void k_mul_silu_grad(int64_t n, const T *d, const T *zz, T *out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n) return;
  out[t] = d[t] * silu_grad(zz[t]);
}

// dX += dn * grad||X||
template <class T>
__global__ void k_norm_bwd_add(int64_t n, int F, const T *X, const T *dn, T *dX) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * F) return;
  const int64_t i = t / F;
  const int f = (int)(t % F);
  T c[9], gn[9];
  load9(X, i, F, f, c);
  const T s = dn[i * F + f];
  norm_grad_parts(c, s, s, s, gn);
#pragma unroll
  for (int q = 0; q < 9; ++q) dX[i * 9 * F + q * F + f] += gn[q];
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
                               const int64_t *n_pairs, int64_t max_pairs, const T *gpair, TO *forces) {
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
  forces[3 * i] = (TO)fx;
  forces[3 * i + 1] = (TO)fy;
  forces[3 * i + 2] = (TO)fz;
}

// ============================================================================ workspace
// Precision plan.  T is the path's arithmetic type.  Three short stages always run in FP64
// ("accurate islands"): the pair geometry and radial basis (inside k_geom), the embedding's
// node stage (norm, LayerNorm, the F->2F->3F MLP, mixing and gating) and the output network
// (part norms, LayerNorm, 3F->F->F/2->1).  In FP32 they are the main amplifiers of rounding:
// without them per-system energies miss a 1e-6 relative bound on 8-64 atom molecules.
using TA = double;

template <class T>
struct PlainWs {
  NbrWs nb;
  int32_t *pairs = nullptr;
  T *geo, *phi, *rbf, *f0, *Xr;
  TA *XrA, *T0, *nrm0, *xhat0, *rstd0, *n0, *ez1, *ea1, *ez2, *g, *X0A;
  std::vector<T *> X;              // L+1 layer inputs/outputs
  std::vector<T *> nX, Xb, Y, z1, a1, z2, a2, z3, h, M, P, nP, Pb, D;
  TA *XLA, *on, *oxhat, *orstd, *q, *oz, *ox, *hz, *hx, *eps;
  // backward
  T *dX = nullptr, *dD, *dPb, *dY, *dM, *dXr;
  TA *dXA, *dT0, *dXrA, *dg, *dez2, *dez1, *dn0, *dnrm0, *dhz, *dox, *dq, *don;
  T *dh, *dz3, *dz2, *dz1, *de, *dphi, *dvhat, *df0, *gpair;
};

template <class T>
static void plan_plain(WsPlan &p, const tn_model *m, int64_t N, int64_t MP, const BoxInfo &bi, bool fw,
                       PlainWs<T> *w) {
  const int64_t F = m->F, K = m->K, L = m->L;
  plan_neighbors(p, N, MP, bi, &w->nb);
  w->pairs = p.take<int32_t>(2 * MP);
  w->geo = p.take<T>(4 * MP);
  w->phi = p.take<T>(MP);
  w->rbf = p.take<T>(MP * K);
  w->f0 = p.take<T>(MP * 3 * F);
  w->Xr = p.take<T>(N * 9 * F);
  w->XrA = p.take<TA>(N * 9 * F);
  w->T0 = p.take<TA>(N * 9 * F);
  w->nrm0 = p.take<TA>(N * F);
  w->xhat0 = p.take<TA>(N * F);
  w->rstd0 = p.take<TA>(N);
  w->n0 = p.take<TA>(N * F);
  w->ez1 = p.take<TA>(N * 2 * F);
  w->ea1 = p.take<TA>(N * 2 * F);
  w->ez2 = p.take<TA>(N * 3 * F);
  w->g = p.take<TA>(N * 3 * F);
  w->X0A = p.take<TA>(N * 9 * F);
  w->X.resize(L + 1);
  for (int64_t l = 0; l <= L; ++l) w->X[l] = p.take<T>(N * 9 * F);
  auto per_layer = [&](std::vector<T *> &v, int64_t count) {
    v.resize(L);
    for (int64_t l = 0; l < L; ++l) v[l] = p.take<T>(count);
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
  per_layer(w->D, N * 9 * F);
  w->XLA = p.take<TA>(N * 9 * F);
  w->on = p.take<TA>(N * 3 * F);
  w->oxhat = p.take<TA>(N * 3 * F);
  w->orstd = p.take<TA>(N);
  w->q = p.take<TA>(N * 3 * F);
  w->oz = p.take<TA>(N * F);
  w->ox = p.take<TA>(N * F);
  w->hz = p.take<TA>(N * (F / 2));
  w->hx = p.take<TA>(N * (F / 2));
  w->eps = p.take<TA>(N);
  if (!fw) return;
  w->dX = p.take<T>(N * 9 * F);
  w->dD = p.take<T>(N * 9 * F);
  w->dPb = p.take<T>(N * 9 * F);
  w->dY = p.take<T>(N * 9 * F);
  w->dM = p.take<T>(N * 9 * F);
  w->dXr = p.take<T>(N * 9 * F);
  w->dXA = p.take<TA>(N * 9 * F);
  w->dT0 = p.take<TA>(N * 9 * F);
  w->dXrA = p.take<TA>(N * 9 * F);
  w->dg = p.take<TA>(N * 3 * F);
  w->dez2 = p.take<TA>(N * 3 * F);
  w->dez1 = p.take<TA>(N * 2 * F);
  w->dn0 = p.take<TA>(N * F);
  w->dnrm0 = p.take<TA>(N * F);
  w->dhz = p.take<TA>(N * (F / 2));
  w->dox = p.take<TA>(N * F);
  w->dq = p.take<TA>(N * 3 * F);
  w->don = p.take<TA>(N * 3 * F);
  w->dh = p.take<T>(MP * 3 * F);
  w->dz3 = p.take<T>(MP * 3 * F);
  w->dz2 = p.take<T>(MP * 2 * F);
  w->dz1 = p.take<T>(MP * F);
  w->de = p.take<T>(MP * K);
  w->dphi = p.take<T>(MP);
  w->dvhat = p.take<T>(3 * MP);
  w->df0 = p.take<T>(MP * 3 * F);
  w->gpair = p.take<T>(3 * MP);
}

size_t plain_workspace_bytes(const tn_model *m, int64_t n, int64_t S, int64_t max_pairs, const BoxInfo &bi, int prec,
                             int want_forces) {
  (void)S;
  WsPlan p(nullptr);
  if (prec == TN_FP64) {
    PlainWs<double> w;
    plan_plain(p, m, n, max_pairs, bi, want_forces != 0, &w);
  } else {
    PlainWs<float> w;
    plan_plain(p, m, n, max_pairs, bi, want_forces != 0, &w);
  }
  return p.off;
}

template <class TI, class TO>
static int convert(hipStream_t s, const TI *in, TO *out, int64_t n) {
  if (n <= 0) return TN_OK;
  hipLaunchKernelGGL((k_convert<TI, TO>), dim3(grid_for(n, 256)), dim3(256), 0, s, n, in, out);
  TN_LAUNCH_CHECK();
  return TN_OK;
}

// ============================================================================ driver
template <class T>
static int run_plain(const tn_model *m, hipStream_t s, const Problem &pb, void *ws, size_t ws_bytes) {
  const int64_t N = pb.n, MP = pb.max_pairs, F = m->F, K = m->K, L = m->L;
  WsPlan plan(ws);
  PlainWs<T> w;
  plan_plain(plan, m, N, MP, pb.box, pb.want_forces, &w);
  if (plan.off > ws_bytes) return TN_E_WORKSPACE;
  const T *pos = static_cast<const T *>(pb.pos);
  int rc;
  const unsigned bs = 256;
  auto W = [&](size_t off) { return wptr<T>(m, off); };
  auto WA = [&](size_t off) { return wptr<TA>(m, off); };
  const WeightOff &o = m->off;

  if (N > 0) {
    hipLaunchKernelGGL(k_check_inputs<T>, dim3(grid_for(N, bs)), dim3(bs), 0, s, pb.z, pb.batch, N, pb.S, m->max_z,
                       pb.status);
    TN_LAUNCH_CHECK();
  }
  if ((rc = build_neighbors<T>(s, N, pos, pb.batch, pb.box, m->r_c, MP, w.pairs, pb.n_pairs, pb.status, w.nb)))
    return rc;
  const int64_t *np = pb.n_pairs;
  const int32_t *rowptr = w.nb.deg, *nbr = w.nb.nbr, *pid = w.nb.pid;

  BoxLen bl;
  bl.periodic = pb.box.periodic;
  for (int a = 0; a < 3; ++a) bl.len[a] = pb.box.len[a];
  if (MP > 0) {
    hipLaunchKernelGGL(k_geom<T>, dim3(grid_for(MP, bs)), dim3(bs), 0, s, w.pairs, MP, np, pos, bl, m->r_c, m->r_lo,
                       m->alpha, WA(o.mu), WA(o.beta), (int)K, w.geo, w.phi, w.rbf);
    TN_LAUNCH_CHECK();
  }
  // ---- embedding: pair part in T, node part in FP64
  if ((rc = linear_fwd<T>(s, w.rbf, MP, K, W(o.W0), W(o.b0), 3 * F, w.f0, nullptr, 0, nullptr, np))) return rc;
  const unsigned gNF = grid_for(N * F, bs);
  if (N > 0) {
    hipLaunchKernelGGL(k_embed_gather<T>, dim3(gNF), dim3(bs), 0, s, N, (int)F, rowptr, nbr, pid, np, MP, pb.z,
                       m->max_z, W(o.U), W(o.V), w.geo, w.phi, w.f0, w.Xr);
    TN_LAUNCH_CHECK();
  }
  if ((rc = convert<T, TA>(s, w.Xr, w.XrA, N * 9 * F))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_node_norm<TA>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.XrA, w.nrm0);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_layernorm<TA>, dim3((unsigned)N), dim3(128), 0, s, N, (int)F, w.nrm0, WA(o.ln_g),
                       WA(o.ln_b), w.n0, w.xhat0, w.rstd0);
    TN_LAUNCH_CHECK();
  }
  if ((rc = linear_fwd<TA>(s, w.n0, N, F, WA(o.W1), WA(o.b1), 2 * F, w.ea1, w.ez1, 1))) return rc;
  if ((rc = linear_fwd<TA>(s, w.ea1, N, 2 * F, WA(o.W2), WA(o.b2), 3 * F, w.g, w.ez2, 1))) return rc;
  const TA *Wemb[3] = {WA(o.Wmix[0]), WA(o.Wmix[1]), WA(o.Wmix[2])};
  if ((rc = mix<TA>(s, w.XrA, w.T0, N, F, Wemb, 0, 0))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_gate<TA>, dim3(grid_for(N * 9 * F, bs)), dim3(bs), 0, s, N, (int)F, w.g, w.T0, w.X0A);
    TN_LAUNCH_CHECK();
  }
  if ((rc = convert<TA, T>(s, w.X0A, w.X[0], N * 9 * F))) return rc;
  // ---- interaction layers (T)
  for (int64_t l = 0; l < L; ++l) {
    const LayerOff &lo = o.layer[l];
    if (N > 0) {
      hipLaunchKernelGGL(k_normalize<T>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.X[l], w.nX[l], w.Xb[l]);
      TN_LAUNCH_CHECK();
    }
    const T *W1[3] = {W(lo.W1[0]), W(lo.W1[1]), W(lo.W1[2])};
    if ((rc = mix<T>(s, w.Xb[l], w.Y[l], N, F, W1, 0, 0))) return rc;
    if ((rc = linear_fwd<T>(s, w.rbf, MP, K, W(lo.Wa), W(lo.ba), F, w.a1[l], w.z1[l], 1, nullptr, np))) return rc;
    if ((rc = linear_fwd<T>(s, w.a1[l], MP, F, W(lo.Wb), W(lo.bb), 2 * F, w.a2[l], w.z2[l], 1, nullptr, np))) return rc;
    {
      TimedScope ts("plain_edge_gemm_c", s);   // the largest edge-filter GEMM (2F -> 3F)
      if ((rc = linear_fwd<T>(s, w.a2[l], MP, 2 * F, W(lo.Wc), W(lo.bc), 3 * F, w.h[l], w.z3[l], 1, w.phi, np)))
        return rc;
    }
    if (N > 0) {
      hipLaunchKernelGGL(k_message<T>, dim3(gNF), dim3(bs), 0, s, N, (int)F, rowptr, nbr, pid, np, MP, w.h[l],
                         w.Y[l], w.M[l], 0);
      TN_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_product<T>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.Y[l], w.M[l], w.P[l], w.nP[l], w.Pb[l]);
      TN_LAUNCH_CHECK();
    }
    const T *W2[3] = {W(lo.W2[0]), W(lo.W2[1]), W(lo.W2[2])};
    if ((rc = mix<T>(s, w.Pb[l], w.D[l], N, F, W2, 0, 0))) return rc;
    if (N > 0) {
      hipLaunchKernelGGL(k_residual<T>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.Xb[l], w.D[l], w.X[l + 1]);
      TN_LAUNCH_CHECK();
    }
  }
  // ---- output network (FP64) and energies
  const int64_t H = F / 2;
  if ((rc = convert<T, TA>(s, w.X[L], w.XLA, N * 9 * F))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_out_norms<TA>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.XLA, w.on);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_layernorm<TA>, dim3((unsigned)N), dim3(128), 0, s, N, (int)(3 * F), w.on, WA(o.oln_g),
                       WA(o.oln_b), w.q, w.oxhat, w.orstd);
    TN_LAUNCH_CHECK();
  }
  if ((rc = linear_fwd<TA>(s, w.q, N, 3 * F, WA(o.Wo), WA(o.bo), F, w.ox, w.oz, 1))) return rc;
  if ((rc = linear_fwd<TA>(s, w.ox, N, F, WA(o.Wh), WA(o.bh), H, w.hx, w.hz, 1))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_out_final<TA>, dim3(grid_for(N, bs)), dim3(bs), 0, s, N, (int)H, w.hx, WA(o.wout),
                       WA(o.bout), w.eps);
    TN_LAUNCH_CHECK();
  }
  if (pb.S > 0) {
    hipLaunchKernelGGL(k_energy_reduce<TA>, dim3((unsigned)pb.S), dim3(128), 0, s, N, w.eps, pb.batch, pb.energy,
                       pb.status);
    TN_LAUNCH_CHECK();
  }
  if (!pb.want_forces) return TN_OK;

  // ================================================================ reverse sweep
  if (N > 0) {
    hipLaunchKernelGGL(k_out_final_bwd<TA>, dim3(grid_for(N * H, bs)), dim3(bs), 0, s, N, (int)H, w.hz, WA(o.wout),
                       w.dhz);
    TN_LAUNCH_CHECK();
  }
  if ((rc = linear_bwd<TA>(s, w.dhz, N, H, WA(o.Wh), F, w.dox, w.oz, 0))) return rc;
  if ((rc = linear_bwd<TA>(s, w.dox, N, F, WA(o.Wo), 3 * F, w.dq, nullptr, 0))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_layernorm_bwd<TA>, dim3((unsigned)N), dim3(128), 0, s, N, (int)(3 * F), w.dq, w.oxhat,
                       w.orstd, WA(o.oln_g), w.don);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_out_norms_bwd<TA>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.XLA, w.don, w.dXA);
    TN_LAUNCH_CHECK();
  }
  if ((rc = convert<TA, T>(s, w.dXA, w.dX, N * 9 * F))) return rc;
  if (MP > 0) {
    if ((rc = fill_bytes_zero(s, w.dphi, MP * sizeof(T)))) return rc;
    if ((rc = fill_bytes_zero(s, w.de, MP * K * sizeof(T)))) return rc;
  }
  for (int64_t l = L - 1; l >= 0; --l) {
    const LayerOff &lo = o.layer[l];
    const T *W1[3] = {W(lo.W1[0]), W(lo.W1[1]), W(lo.W1[2])};
    const T *W2[3] = {W(lo.W2[0]), W(lo.W2[1]), W(lo.W2[2])};
    if (N > 0) {
      hipLaunchKernelGGL(k_residual_bwd<T>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.D[l], w.dX, w.dD);
      TN_LAUNCH_CHECK();
    }
    if ((rc = mix<T>(s, w.dD, w.dPb, N, F, W2, 1, 0))) return rc;
    if (N > 0) {
      hipLaunchKernelGGL(k_product_bwd<T>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.dPb, w.P[l], w.nP[l], w.Y[l],
                         w.M[l], w.dY, w.dM);
      TN_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_message<T>, dim3(gNF), dim3(bs), 0, s, N, (int)F, rowptr, nbr, pid, np, MP, w.h[l], w.dM,
                         w.dY, 1);
      TN_LAUNCH_CHECK();
    }
    if (MP > 0) {
      hipLaunchKernelGGL(k_message_bwd_pair<T>, dim3(grid_for(MP * F, bs)), dim3(bs), 0, s, w.pairs, MP, np, (int)F,
                         w.Y[l], w.dM, w.dh);
      TN_LAUNCH_CHECK();
    }
    // dXb = dX (identity branch) + mix^T(W1, dY), accumulated in place
    if ((rc = mix<T>(s, w.dY, w.dX, N, F, W1, 1, 1))) return rc;
    if (N > 0) {
      hipLaunchKernelGGL(k_normalize_bwd<T>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.X[l], w.nX[l], w.dX);
      TN_LAUNCH_CHECK();
    }
    // edge filter adjoint
    if (MP > 0) {
      hipLaunchKernelGGL(k_edge_bwd_top<T>, dim3((unsigned)MP), dim3(128), 0, s, MP, np, (int)(3 * F), w.dh, w.z3[l],
                         w.phi, w.dz3, w.dphi);
      TN_LAUNCH_CHECK();
    }
    if ((rc = linear_bwd<T>(s, w.dz3, MP, 3 * F, W(lo.Wc), 2 * F, w.dz2, w.z2[l], 0, np))) return rc;
    if ((rc = linear_bwd<T>(s, w.dz2, MP, 2 * F, W(lo.Wb), F, w.dz1, w.z1[l], 0, np))) return rc;
    if ((rc = linear_bwd<T>(s, w.dz1, MP, F, W(lo.Wa), K, w.de, nullptr, 1, np))) return rc;
  }
  // ---- embedding adjoint (dX now holds dE/dX0); node part in FP64
  if ((rc = convert<T, TA>(s, w.dX, w.dXA, N * 9 * F))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_gate_bwd<TA>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.dXA, w.T0, w.g, w.dg, w.dT0);
    TN_LAUNCH_CHECK();
  }
  if ((rc = mix<TA>(s, w.dT0, w.dXrA, N, F, Wemb, 1, 0))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_mul_silu_grad<TA>, dim3(grid_for(N * 3 * F, bs)), dim3(bs), 0, s, N * 3 * F, w.dg, w.ez2,
                       w.dez2);
    TN_LAUNCH_CHECK();
  }
  if ((rc = linear_bwd<TA>(s, w.dez2, N, 3 * F, WA(o.W2), 2 * F, w.dez1, w.ez1, 0))) return rc;
  if ((rc = linear_bwd<TA>(s, w.dez1, N, 2 * F, WA(o.W1), F, w.dn0, nullptr, 0))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_layernorm_bwd<TA>, dim3((unsigned)N), dim3(128), 0, s, N, (int)F, w.dn0, w.xhat0, w.rstd0,
                       WA(o.ln_g), w.dnrm0);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_norm_bwd_add<TA>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.XrA, w.dnrm0, w.dXrA);
    TN_LAUNCH_CHECK();
  }
  if ((rc = convert<TA, T>(s, w.dXrA, w.dXr, N * 9 * F))) return rc;
  if (MP > 0) {
    hipLaunchKernelGGL(k_embed_bwd_pair<T>, dim3((unsigned)MP), dim3(128), 0, s, w.pairs, MP, np, (int)F, pb.z,
                       m->max_z, W(o.U), W(o.V), w.geo, w.phi, w.f0, w.dXr, w.df0, w.dphi, w.dvhat);
    TN_LAUNCH_CHECK();
  }
  if ((rc = linear_bwd<T>(s, w.df0, MP, 3 * F, W(o.W0), K, w.de, nullptr, 1, np))) return rc;
  if (MP > 0) {
    hipLaunchKernelGGL(k_geom_bwd<T>, dim3(grid_for(MP, bs)), dim3(bs), 0, s, MP, np, (T)m->r_c, (T)m->r_lo,
                       (T)m->alpha, W(o.mu), W(o.beta), (int)K, w.geo, w.de, w.dphi, w.dvhat, w.gpair);
    TN_LAUNCH_CHECK();
  }
  if (N > 0) {
    hipLaunchKernelGGL((k_force_gather<T, T>), dim3(grid_for(N, bs)), dim3(bs), 0, s, N, rowptr, nbr, pid, np, MP,
                       w.gpair, static_cast<T *>(pb.forces));
    TN_LAUNCH_CHECK();
  }
  return TN_OK;
}

int plain_run(const tn_model *m, hipStream_t s, const Problem &pb, int prec, void *ws, size_t ws_bytes) {
  if (prec == TN_FP64) return run_plain<double>(m, s, pb, ws, ws_bytes);
  if (prec == TN_FP32) return run_plain<float>(m, s, pb, ws, ws_bytes);
  return TN_E_UNSUPPORTED;
}

}  // namespace tn
