// Device-side math shared by the plain and fused paths.
//
// Per-atom features are F channels of 3x3 matrices X = t*1 + A0(a) + S(s),
// stored as nine coordinates per channel in the order
//   c = 0      t          (scalar part I = t * identity)
//   c = 1..3   a_x a_y a_z (antisymmetric part, A0(a) w = a x w)
//   c = 4..8   s_xx s_yy s_xy s_xz s_yz (symmetric traceless part, s_zz = -s_xx - s_yy)
// so that the per-part channel mixing of TensorNet is one [rows, F] x [F, F]
// product per coordinate.  The helpers below convert between coordinates and
// 3x3 matrices and give the adjoints of those linear maps.
#pragma once

#include <hip/hip_runtime.h>

namespace tn {

constexpr int kCoord = 9;

__host__ __device__ inline int coord_part(int c) { return c == 0 ? 0 : (c < 4 ? 1 : 2); }

// A periodic cell given by its rows a = (ax, 0, 0), b = (bx, by, 0), c = (cx, cy, cz), lower
// triangular and reduced (|bx|, |cx| <= ax/2, |cy| <= by/2); a rectangular box has zero tilts.
struct Lattice {
  int periodic = 0;
  double ax = 0, bx = 0, by = 0, cx = 0, cy = 0, cz = 0;
};

// Minimum image of a displacement d = r_j - r_i (Sec. 2.5.1, rectangular and triclinic
// boundaries): reduce along c, then b, then a.  In a reduced cell whose heights are at least
// twice the distance of interest this is the nearest image.  Every product is rounded before
// its subtraction (no contraction), so the neighbour predicate is reproducible bit for bit.
__host__ __device__ inline void min_image(const Lattice &L, double &dx, double &dy, double &dz) {
#pragma clang fp contract(off)
  if (!L.periodic) return;
  const double kz = rint(dz / L.cz);
  dx = dx - L.cx * kz;
  dy = dy - L.cy * kz;
  dz = dz - L.cz * kz;
  const double ky = rint(dy / L.by);
  dx = dx - L.bx * ky;
  dy = dy - L.by * ky;
  const double kx = rint(dx / L.ax);
  dx = dx - L.ax * kx;
}

// Fractional coordinates s = r H^-1 (H has the rows a, b, c).
__host__ __device__ inline void fractional(const Lattice &L, double x, double y, double z, double &s0, double &s1,
                                           double &s2) {
  s2 = z / L.cz;
  s1 = (y - L.cy * s2) / L.by;
  s0 = (x - L.cx * s2 - L.bx * s1) / L.ax;
}

__device__ inline float dexp(float x) { return expf(x); }
__device__ inline double dexp(double x) { return exp(x); }
__device__ inline float dsqrt(float x) { return sqrtf(x); }
__device__ inline double dsqrt(double x) { return sqrt(x); }
__device__ inline float dcos(float x) { return cosf(x); }
__device__ inline double dcos(double x) { return cos(x); }
__device__ inline float dsin(float x) { return sinf(x); }
__device__ inline double dsin(double x) { return sin(x); }
__device__ inline float drint(float x) { return rintf(x); }
__device__ inline double drint(double x) { return rint(x); }

// FP32 SiLU for the pair kernels' epilogues: exp through the hardware exponential and the
// hardware reciprocal (1 ulp) instead of an IEEE division.  The relative error stays at a
// few ulp; the pair kernels evaluate it tens of millions of times per call.
__device__ __forceinline__ float fast_sigmoid(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }
__device__ __forceinline__ float fast_silu(float x) { return x * fast_sigmoid(x); }
__device__ __forceinline__ float fast_silu_grad(float x) {
  const float s = fast_sigmoid(x);
  return s * (1.0f + x * (1.0f - s));
}
// Both from one sigmoid: returns silu(x) and sets grad = silu'(x) (the same values as above).
__device__ __forceinline__ float fast_silu_and_grad(float x, float &grad) {
  const float s = fast_sigmoid(x);
  grad = s * (1.0f + x * (1.0f - s));
  return x * s;
}

// SiLU x*sigmoid(x) and its derivative sigmoid(x) * (1 + x * (1 - sigmoid(x))).
template <class T> __device__ inline T sigmoid(T x) { return T(1) / (T(1) + dexp(-x)); }
template <class T> __device__ inline T silu(T x) { return x * sigmoid(x); }
template <class T> __device__ inline T silu_grad(T x) {
  T s = sigmoid(x);
  return s * (T(1) + x * (T(1) - s));
}

// Coordinates -> row-major 3x3 matrix.
template <class T> __device__ inline void rec(const T c[9], T X[9]) {
  const T t = c[0], ax = c[1], ay = c[2], az = c[3];
  const T xx = c[4], yy = c[5], xy = c[6], xz = c[7], yz = c[8];
  X[0] = t + xx;  X[1] = -az + xy; X[2] = ay + xz;
  X[3] = az + xy; X[4] = t + yy;   X[5] = -ax + yz;
  X[6] = -ay + xz; X[7] = ax + yz; X[8] = t - xx - yy;
}

// 3x3 matrix -> coordinates of its I, A and S parts.
template <class T> __device__ inline void dec(const T X[9], T c[9]) {
  const T t = (X[0] + X[4] + X[8]) * (T(1) / T(3));
  c[0] = t;
  c[1] = T(0.5) * (X[7] - X[5]);
  c[2] = T(0.5) * (X[2] - X[6]);
  c[3] = T(0.5) * (X[3] - X[1]);
  c[4] = X[0] - t;
  c[5] = X[4] - t;
  c[6] = T(0.5) * (X[1] + X[3]);
  c[7] = T(0.5) * (X[2] + X[6]);
  c[8] = T(0.5) * (X[5] + X[7]);
}

// Adjoint of rec: gradient w.r.t. coordinates from a gradient w.r.t. matrix entries.
template <class T> __device__ inline void rec_adj(const T G[9], T d[9]) {
  d[0] = G[0] + G[4] + G[8];
  d[1] = G[7] - G[5];
  d[2] = G[2] - G[6];
  d[3] = G[3] - G[1];
  d[4] = G[0] - G[8];
  d[5] = G[4] - G[8];
  d[6] = G[1] + G[3];
  d[7] = G[2] + G[6];
  d[8] = G[5] + G[7];
}

// Adjoint of dec: gradient w.r.t. matrix entries from a gradient w.r.t. coordinates.
template <class T> __device__ inline void dec_adj(const T d[9], T G[9]) {
  const T t3 = d[0] * (T(1) / T(3));
  const T h = T(0.5);
  G[0] = t3 + (T(2) * d[4] - d[5]) * (T(1) / T(3));
  G[4] = t3 + (T(2) * d[5] - d[4]) * (T(1) / T(3));
  G[8] = t3 - (d[4] + d[5]) * (T(1) / T(3));
  G[1] = h * (d[6] - d[3]); G[3] = h * (d[6] + d[3]);
  G[2] = h * (d[7] + d[2]); G[6] = h * (d[7] - d[2]);
  G[5] = h * (d[8] - d[1]); G[7] = h * (d[8] + d[1]);
}

// Squared Frobenius norm of rec(c) and its parts.
template <class T> __device__ inline T norm_I(const T c[9]) { return T(3) * c[0] * c[0]; }
template <class T> __device__ inline T norm_A(const T c[9]) {
  return T(2) * (c[1] * c[1] + c[2] * c[2] + c[3] * c[3]);
}
template <class T> __device__ inline T norm_S(const T c[9]) {
  const T zz = c[4] + c[5];
  return c[4] * c[4] + c[5] * c[5] + zz * zz + T(2) * (c[6] * c[6] + c[7] * c[7] + c[8] * c[8]);
}
template <class T> __device__ inline T norm9(const T c[9]) { return norm_I(c) + norm_A(c) + norm_S(c); }

// d(norm)/dc scaled: out[k] = s_I * d norm_I/dc_k + s_A * ... + s_S * ... (s_* per part).
template <class T> __device__ inline void norm_grad_parts(const T c[9], T sI, T sA, T sS, T out[9]) {
  out[0] = sI * T(6) * c[0];
  out[1] = sA * T(4) * c[1];
  out[2] = sA * T(4) * c[2];
  out[3] = sA * T(4) * c[3];
  out[4] = sS * (T(4) * c[4] + T(2) * c[5]);
  out[5] = sS * (T(4) * c[5] + T(2) * c[4]);
  out[6] = sS * T(4) * c[6];
  out[7] = sS * T(4) * c[7];
  out[8] = sS * T(4) * c[8];
}

// 3x3 row-major products.
template <class T> __device__ inline void mm(const T A[9], const T B[9], T C[9]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) C[r * 3 + q] = A[r * 3] * B[q] + A[r * 3 + 1] * B[3 + q] + A[r * 3 + 2] * B[6 + q];
}
// C = A^T B
template <class T> __device__ inline void mtm(const T A[9], const T B[9], T C[9]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) C[r * 3 + q] = A[r] * B[q] + A[3 + r] * B[3 + q] + A[6 + r] * B[6 + q];
}
// C = A B^T
template <class T> __device__ inline void mmt(const T A[9], const T B[9], T C[9]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q) C[r * 3 + q] = A[r * 3] * B[q * 3] + A[r * 3 + 1] * B[q * 3 + 1] + A[r * 3 + 2] * B[q * 3 + 2];
}

// Coordinates of S0(u) = u u^T - 1/3 for a unit vector u.
template <class T> __device__ inline void s0_coords(T ux, T uy, T uz, T s[5]) {
  s[0] = ux * ux - T(1) / T(3);
  s[1] = uy * uy - T(1) / T(3);
  s[2] = ux * uy;
  s[3] = ux * uz;
  s[4] = uy * uz;
}

// Gradient w.r.t. u of <w, s0_coords(u)> (plain dot over the five coordinates).
template <class T> __device__ inline void s0_dot_grad(const T w[5], T ux, T uy, T uz, T g[3]) {
  g[0] = T(2) * w[0] * ux + w[2] * uy + w[3] * uz;
  g[1] = T(2) * w[1] * uy + w[2] * ux + w[4] * uz;
  g[2] = w[3] * ux + w[4] * uy;
}

// V consecutive floats through one vector access (V = 1, 2 or 4; p aligned to 4V bytes).
template <int V>
__device__ __forceinline__ void ldv(const float *p, float (&o)[V]) {
  if constexpr (V == 4) {
    const float4 t = *reinterpret_cast<const float4 *>(p);
    o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
  } else if constexpr (V == 2) {
    const float2 t = *reinterpret_cast<const float2 *>(p);
    o[0] = t.x; o[1] = t.y;
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = p[v];
  }
}
template <int V>
__device__ __forceinline__ void stv(float *p, const float (&o)[V]) {
  if constexpr (V == 4) {
    *reinterpret_cast<float4 *>(p) = make_float4(o[0], o[1], o[2], o[3]);
  } else if constexpr (V == 2) {
    *reinterpret_cast<float2 *>(p) = make_float2(o[0], o[1]);
  } else {
#pragma unroll
    for (int v = 0; v < V; ++v) p[v] = o[v];
  }
}

// Workgroups are dispatched round-robin over the eight XCDs, each with its own L2.  This
// renumbering gives every XCD one contiguous range of logical blocks, so that blocks working
// on neighbouring atoms or pairs (both are kept in spatial cell order) share an L2.
__device__ __forceinline__ int64_t xcd_block() {
  const int64_t G = gridDim.x, b = blockIdx.x;
  const int64_t q = G / 8, r = G % 8, x = b % 8;
  return x * q + (x < r ? x : r) + b / 8;
}

// The same renumbering when only the first T of the grid's blocks have work (the grid is
// sized for a static bound such as max_pairs): every XCD gets an equal contiguous share of
// the T work items, so a partly filled grid still spreads over all eight XCDs.  Returns the
// work item of this block, or -1 for a block without one.  Needs gridDim.x >= T.
__device__ __forceinline__ int64_t xcd_block_of(int64_t T) {
  const int64_t b = blockIdx.x, x = b % 8, k = b / 8;
  const int64_t q = T / 8, r = T % 8;
  const int64_t len = q + (x < r ? 1 : 0);
  return k < len ? x * q + (x < r ? x : r) + k : -1;
}

// Flag a bit in the device status word.
__device__ inline void set_status(int32_t *status, int32_t bit) {
  if (status) atomicOr(reinterpret_cast<int *>(status), bit);
}

}  // namespace tn
