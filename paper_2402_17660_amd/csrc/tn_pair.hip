// Launchers of the fused per-pair MFMA kernels (the tile code is in tn_pairtile.h).
#include "tn_pairtile.h"

namespace tn {

bool pair_kernels_support(int F, int K, int L, bool bf16) {
  const bool k_ok = bf16 ? (K == 32 || K == 64) : (K == 16 || K == 32 || K == 48 || K == 64);
  return (F == 64 || F == 128) && k_ok && L >= 0 && L <= kMaxLayers;
}

// ============================================================================ launchers
// Tile shapes: pairs per tile = 16 RB, NW waves per workgroup; MINB, the launch bound's
// minimum waves per SIMD, caps the registers at 512 / MINB per lane and so allows MINB * 4 / NW
// workgroups per compute unit (LDS permitting).  Every shape computes each pair with the same
// arithmetic in the same order, so results do not depend on the shape; tn_autotune picks the
// fastest.  Workgroups per CU:
//   FP32: 0 = 32 pairs, 4 waves, 3 per CU; 1 = 32, 4, 2; 2 = 16, 4, 4; 3 = 64, 4, 1;
//         4 = 48, 4, 2
//   BF16: 0 = 64 pairs, 4 waves, 1 per CU; 1 = 32, 4, 2; 2 = 48, 4, 2
// (FP32 eight-wave tiles, NW = 8, measured slower on the 6000-atom box: 32 pairs, and 48 pairs at
// two workgroups per CU, where the 128-register cap spills; they are not built.)
int pair_variant_count(bool bf16) { return bf16 ? 5 : 5; }

template <int TILE>
static unsigned tile_grid(int64_t max_pairs) {
  return (unsigned)((max_pairs + TILE - 1) / TILE);
}

template <int F, int K, int RB, int NW, int MINB>
static int launch_fwd_v(hipStream_t s, const PairFwdArgs &a) {
  const unsigned grid = tile_grid<16 * RB>(a.max_pairs);
  if (grid == 0) return TN_OK;
  TimedScope ts("edge_fwd", s);
  hipLaunchKernelGGL((k_pair_fwd<F, K, RB, NW, MINB>), dim3(grid), dim3(64 * NW), 0, s, a);
  TN_LAUNCH_CHECK();
  return TN_OK;
}

template <int F, int K, int RB, int NW, int MINB>
static int launch_bwd_v(hipStream_t s, const PairBwdArgs &a) {
  const unsigned grid = tile_grid<16 * RB>(a.max_pairs);
  if (grid == 0) return TN_OK;
  TimedScope ts("edge_bwd", s);
  hipLaunchKernelGGL((k_pair_bwd<F, K, RB, NW, MINB>), dim3(grid), dim3(64 * NW), 0, s, a);
  TN_LAUNCH_CHECK();
  return TN_OK;
}

template <int F, int K, int RB, int MINB, int NW = 4>
static int launch_fwd_bf16_v(hipStream_t s, const PairFwdArgsB &a) {
  const unsigned grid = tile_grid<16 * RB>(a.max_pairs);
  if (grid == 0) return TN_OK;
  TimedScope ts("edge_fwd", s);
  hipLaunchKernelGGL((k_pair_fwd_bf16<F, K, RB, MINB, NW>), dim3(grid), dim3(64 * NW), 0, s, a);
  TN_LAUNCH_CHECK();
  return TN_OK;
}

template <int F, int K, int RB, int MINB, int NW = 4, int PF = 2>
static int launch_bwd_bf16_v(hipStream_t s, const PairBwdArgsB &a) {
  const unsigned grid = tile_grid<16 * RB>(a.max_pairs);
  if (grid == 0) return TN_OK;
  TimedScope ts("edge_bwd", s);
  hipLaunchKernelGGL((k_pair_bwd_bf16<F, K, RB, MINB, NW, PF>), dim3(grid), dim3(64 * NW), 0, s, a);
  TN_LAUNCH_CHECK();
  return TN_OK;
}

template <int F, int K>
static int launch_fwd(hipStream_t s, const PairFwdArgs &a, int v) {
  switch (v) {
    case 1: return launch_fwd_v<F, K, 2, 4, 2>(s, a);
    case 2: return launch_fwd_v<F, K, 1, 4, 4>(s, a);
    case 3: return launch_fwd_v<F, K, 4, 4, 1>(s, a);
    case 4: return launch_fwd_v<F, K, 3, 4, 2>(s, a);
    default: return launch_fwd_v<F, K, 2, 4, 3>(s, a);
  }
}

template <int F, int K>
static int launch_bwd(hipStream_t s, const PairBwdArgs &a, int v) {
  switch (v) {
    case 1: return launch_bwd_v<F, K, 2, 4, 2>(s, a);
    case 2: return launch_bwd_v<F, K, 1, 4, 4>(s, a);
    case 3: return launch_bwd_v<F, K, 4, 4, 1>(s, a);
    case 4: return launch_bwd_v<F, K, 3, 4, 2>(s, a);
    default: return launch_bwd_v<F, K, 2, 4, 3>(s, a);
  }
}

// BF16 shapes 3 and 4 (F = 128): eight-wave tiles, one workgroup per CU, each weight fragment
// read once for twice (or more) the rows of the four-wave tiles: forward 96 and 112 pairs
// (4.9 against 6.0 ms per launch on 100k atoms); reverse 96 pairs, its prologues loading one row
// ahead or none (about as fast as shape 2: its gathers, not its weight reads, set its time;
// 112 pairs spill).  F = 64 takes shape 2 for them.
template <int F, int K>
static int launch_fwd_bf16(hipStream_t s, const PairFwdArgsB &a, int v) {
  if (v == 1) return launch_fwd_bf16_v<F, K, 2, 2>(s, a);
  if (v == 2) return launch_fwd_bf16_v<F, K, 3, 2>(s, a);
  if constexpr (F == 128) {
    if (v == 3) return launch_fwd_bf16_v<F, K, 6, 1, 8>(s, a);
    if (v == 4) return launch_fwd_bf16_v<F, K, 7, 1, 8>(s, a);
  }
  if (v >= 3) return launch_fwd_bf16_v<F, K, 3, 2>(s, a);
  return launch_fwd_bf16_v<F, K, 4, 1>(s, a);
}

template <int F, int K>
static int launch_bwd_bf16(hipStream_t s, const PairBwdArgsB &a, int v) {
  if (v == 1) return launch_bwd_bf16_v<F, K, 2, 2>(s, a);
  if (v == 2) return launch_bwd_bf16_v<F, K, 3, 2>(s, a);
  if constexpr (F == 128 && K <= 128) {
    if (v == 3) return launch_bwd_bf16_v<F, K, 6, 1, 8, 1>(s, a);
    if (v == 4) return launch_bwd_bf16_v<F, K, 6, 1, 8, 0>(s, a);
  }
  if (v >= 3) return launch_bwd_bf16_v<F, K, 3, 2>(s, a);
  return launch_bwd_bf16_v<F, K, 4, 1>(s, a);
}

#define TN_PAIR_DISPATCH(FN)                                         \
  switch (F * 1000 + K) {                                            \
    case 64016: return FN<64, 16>(s, a, v);                          \
    case 64032: return FN<64, 32>(s, a, v);                          \
    case 64048: return FN<64, 48>(s, a, v);                          \
    case 64064: return FN<64, 64>(s, a, v);                          \
    case 128016: return FN<128, 16>(s, a, v);                        \
    case 128032: return FN<128, 32>(s, a, v);                        \
    case 128048: return FN<128, 48>(s, a, v);                        \
    case 128064: return FN<128, 64>(s, a, v);                        \
    default: return TN_E_UNSUPPORTED;                                \
  }

#define TN_PAIR_DISPATCH_BF16(FN)                                    \
  switch (F * 1000 + K) {                                            \
    case 64032: return FN<64, 32>(s, a, v);                          \
    case 64064: return FN<64, 64>(s, a, v);                          \
    case 128032: return FN<128, 32>(s, a, v);                        \
    case 128064: return FN<128, 64>(s, a, v);                        \
    default: return TN_E_UNSUPPORTED;                                \
  }

int launch_pair_fwd(hipStream_t s, int F, int K, const PairFwdArgs &a, int v) { TN_PAIR_DISPATCH(launch_fwd) }
int launch_pair_bwd(hipStream_t s, int F, int K, const PairBwdArgs &a, int v) { TN_PAIR_DISPATCH(launch_bwd) }
int launch_pair_fwd_bf16(hipStream_t s, int F, int K, const PairFwdArgsB &a, int v) {
  TN_PAIR_DISPATCH_BF16(launch_fwd_bf16)
}
int launch_pair_bwd_bf16(hipStream_t s, int F, int K, const PairBwdArgsB &a, int v) {
  TN_PAIR_DISPATCH_BF16(launch_bwd_bf16)
}

}  // namespace tn
