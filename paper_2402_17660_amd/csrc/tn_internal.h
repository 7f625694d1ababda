// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <cstdio>
#include <array>
#include <map>
#include <vector>

#include "tensornet.h"
#include "tn_device.h"

#define TN_HIP(call)                                                   \
  do {                                                                 \
    hipError_t e_ = (call);                                            \
    if (e_ != hipSuccess) {                                            \
      std::fprintf(stderr, "tensornet: %s failed: %s (%s:%d)\n", #call, \
                   hipGetErrorString(e_), __FILE__, __LINE__);         \
      return TN_E_HIP;                                                 \
    }                                                                  \
  } while (0)

#define TN_LAUNCH_CHECK() TN_HIP(hipGetLastError())

namespace tn {

constexpr int kMaxK = 64;          // radial basis functions supported by the kernels
constexpr int kWsAlign = 256;

// ------------------------------------------------------------------ weights
struct LayerOff {
  size_t Wa, ba, Wb, bb, Wc, bc, W1[3], W2[3];
  size_t WaT, WbT, WcT;   // transposed copies [K][F], [F][2F], [2F][3F] (fused reverse sweep)
  size_t Waf, Wbf, Wcf;   // 64-element aligned copies of Wa, Wb, Wc (fused forward)
  size_t W1T[3], W2T[3];  // transposed mixing matrices, 64-element aligned (adjoint mixing)
  size_t W1f[3], W2f[3];  // 64-element aligned copies of the mixing matrices (forward mixing)
};

struct WeightOff {
  size_t E, Wz, bz, W0, b0, ln_g, ln_b, W1, b1, W2, b2, Wmix[3];
  std::vector<LayerOff> layer;
  size_t oln_g, oln_b, Wo, bo, Wh, bh, wout, bout;
  size_t W0T, W0f;  // transposed [K][3F] and aligned copy of W0
  size_t WmixT[3];  // transposed embedding mixing matrices (adjoint mixing)
  size_t Wmixf[3];  // 64-element aligned copies of the embedding mixing matrices
  size_t U, V;      // species tables [max_z, F]: Z_ij = U[z_i] + V[z_j]
  size_t mu, beta;  // radial basis constants [K]
  size_t total;     // element count of one packed copy
};

}  // namespace tn

struct tn_model {
  // Pair-kernel tile shapes [precision: 0 FP32, 1 BF16][0 forward, 1 reverse]: `pair_force`
  // (>= 0) overrides; otherwise `pair_tuned` by pair-budget class (bit length of max_pairs),
  // filled by tn_autotune; otherwise shape 0.
  int pair_force[2][2] = {{-1, -1}, {-1, -1}};
  std::map<int, std::array<int, 2>> pair_tuned[2];
  int device = 0;
  int F = 0, K = 0, L = 0, max_z = 0;
  double r_lo = 0.0, r_c = 0.0, alpha = 0.0;
  tn::WeightOff off;
  double *w64 = nullptr;           // packed FP64 weights (device)
  float *w32 = nullptr;            // packed FP32 weights (device)
  __bf16 *w16 = nullptr;           // packed BF16 weights (device)
  void *mol_const = nullptr;       // the molecule path's weight pointers (device; tn_mol.hip)
};

namespace tn {

template <class T> inline const T *wptr(const tn_model *m, size_t off);
template <> inline const double *wptr<double>(const tn_model *m, size_t off) { return m->w64 + off; }
template <> inline const float *wptr<float>(const tn_model *m, size_t off) { return m->w32 + off; }

// ------------------------------------------------------------------ workspace planning
// Bump allocator: run once with base == nullptr to size the workspace, then
// again with the caller's buffer to hand out aligned sub-buffers.
struct WsPlan {
  char *base = nullptr;
  size_t off = 0;
  __host__ __device__ explicit WsPlan(void *b) : base(static_cast<char *>(b)) {}
  template <class T> __host__ __device__ T *take(size_t count) {
    off = (off + kWsAlign - 1) / kWsAlign * kWsAlign;
    T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
    off += count * sizeof(T) + kWsAlign;   // keep a guard gap between buffers
    return p;
  }
};

// ------------------------------------------------------------------ neighbour search
struct BoxInfo {
  int periodic = 0;
  int cells = 0;   // candidates from the cell list (periodic box) rather than the system's atom range
  int tri = 0;     // nonzero tilt: cells are binned in fractional coordinates
  Lattice lat;
  double len[3] = {0, 0, 0};   // ax, by, cz
  int nc[3] = {1, 1, 1};
  double side[3] = {0, 0, 0};
};

// Validates the box; returns TN_OK, TN_E_ARG or TN_E_BOX.
int box_info(const double *box, double cutoff, BoxInfo *bi);

struct NbrWs {
  int32_t *cell_of = nullptr, *cell_count = nullptr, *cell_start = nullptr, *cell_fill = nullptr,
          *cell_atoms = nullptr;
  int32_t *deg = nullptr, *nup = nullptr;       // [N+1], scanned in place into rowptr / pair base
  int32_t *nbr = nullptr, *pid = nullptr;       // [2*max_pairs] CSR rows (sorted by neighbour)
  int32_t *scan_tmp = nullptr;                  // block sums
  int64_t *count64 = nullptr;                   // [2]: total pairs, total directed edges
  void *spos = nullptr;                         // [N,3] cell-ordered positions (periodic)
  int32_t *sz = nullptr, *sbatch = nullptr, *scell = nullptr;   // cell-ordered z, batch, cell
  int32_t *ipairs = nullptr;                    // [2, max_pairs] internal pair list
};

// The graph the model kernels consume, in the internal atom order (cell order for a
// periodic box, the caller's order otherwise; perm maps internal -> caller index).
template <class T>
struct NbrGraph {
  const T *pos = nullptr;
  const int32_t *z = nullptr, *batch = nullptr, *perm = nullptr;
  const int32_t *rowptr = nullptr, *nbr = nullptr, *pid = nullptr, *pairs = nullptr;
};

void plan_neighbors(WsPlan &p, int64_t n, int64_t max_pairs, const BoxInfo &bi, NbrWs *w);

// Builds the CSR graph and the internal pair list, *n_pairs, and (if public_pairs) the
// caller-order pair list padded with -1.  z may be null.  T is the position type.
template <class T>
int build_neighbors(hipStream_t s, int64_t n, const T *pos, const int32_t *z, const int32_t *batch,
                    const BoxInfo &bi, double cutoff, int64_t max_pairs, int32_t *public_pairs, int64_t *n_pairs,
                    int32_t *status, const NbrWs &w, NbrGraph<T> *graph,
                    int64_t n_systems = 0, int max_z = 0);

// ------------------------------------------------------------------ scans and fills
int exclusive_scan_i32(hipStream_t s, int32_t *data, int64_t n, int32_t *block_tmp, int64_t *total_out);
size_t scan_tmp_count(int64_t n);
int fill_i32(hipStream_t s, int32_t *p, int64_t n, int32_t v);
int fill_bytes_zero(hipStream_t s, void *p, size_t bytes);

// ------------------------------------------------------------------ model paths
struct Problem {
  int64_t n = 0, S = 0, max_pairs = 0;
  const void *pos = nullptr;
  const int32_t *z = nullptr, *batch = nullptr;
  BoxInfo box;
  double *energy = nullptr;
  void *forces = nullptr;
  int64_t *n_pairs = nullptr;
  int32_t *status = nullptr;
  bool want_forces = false;
};

size_t plain_workspace_bytes(const tn_model *m, int64_t n, int64_t S, int64_t max_pairs, const BoxInfo &bi, int prec,
                             int want_forces);
int plain_run(const tn_model *m, hipStream_t s, const Problem &pb, int prec, void *ws, size_t ws_bytes);

// The molecule path: one launch in which a workgroup owns each isolated system (no box).
size_t molecule_workspace_bytes(const tn_model *m, int64_t n, int64_t S, int64_t max_pairs, int prec,
                                int want_forces);
int molecule_run(const tn_model *m, hipStream_t s, const Problem &pb, int prec, void *ws, size_t ws_bytes);
bool molecule_kernels_support(int F, int K, bool bf16);
// Uploads the molecule path's table of weight pointers at model creation (m->mol_const); a
// model whose sizes the path does not support gets none.  Returns TN_OK or TN_E_HIP.
int molecule_setup(tn_model *m);

size_t fused_workspace_bytes(const tn_model *m, int64_t n, int64_t S, int64_t max_pairs, const BoxInfo &bi, int prec,
                             int want_forces);
int fused_run(const tn_model *m, hipStream_t s, const Problem &pb, int prec, void *ws, size_t ws_bytes);

// ------------------------------------------------------------------ MFMA pair kernels (fused path)
constexpr int kMaxLayers = 16;

// Whether the fused pair kernels support these sizes.
bool pair_kernels_support(int F, int K, int L, bool bf16);
// Number of tile shapes of the fused pair kernels (see tn_pair.hip).
int pair_variant_count(bool bf16);
// Pair-budget class of the tuning table: the bit length of max_pairs.
int pair_budget_class(int64_t max_pairs);
// The tile shape a fused call uses for this model, precision, budget and direction.
int pair_variant(const tn_model *m, bool bf16, int64_t max_pairs, bool reverse);

struct PairFwdArgs {
  const int32_t *pairs = nullptr;   // [2, max_pairs]
  int64_t max_pairs = 0;
  const int64_t *n_pairs = nullptr;
  const float *pos = nullptr;
  Lattice lat;   // periodic cell (lat.periodic == 0: isolated systems)
  double r_c = 0, r_lo = 0, alpha = 0;
  const double *mu = nullptr, *beta = nullptr;
  const float *W0 = nullptr, *b0 = nullptr;
  const float *Wa[kMaxLayers], *ba[kMaxLayers], *Wb[kMaxLayers], *bb[kMaxLayers], *Wc[kMaxLayers], *bc[kMaxLayers];
  int L = 0;
  float *geo = nullptr, *phi = nullptr, *f0 = nullptr;
  // per pair and layer: z1, z2 hold silu'(z1), silu'(z2) (the reverse pass's only use of them),
  // z3 the pre-activation itself, h the filters phi silu(z3) (null: not stored; the fused and
  // molecule paths form them from z3 in the message gathers)
  float *z1[kMaxLayers], *z2[kMaxLayers], *z3[kMaxLayers], *h[kMaxLayers];
};

// Per-atom rows the reverse pair kernels gather (internal atom order, [N][9][F] coordinates).
struct BwdGather {
  const int32_t *z = nullptr;
  const float *U = nullptr, *V = nullptr;
  int max_z = 0;
  const float *f0 = nullptr;
  const __bf16 *f016 = nullptr;   // f0 in BF16 (BF16 path; f0 then unused)
  const float *dXr = nullptr;
  const float *Y[kMaxLayers], *dM[kMaxLayers];
};

struct PairBwdArgs {
  const int32_t *pairs = nullptr;
  int64_t max_pairs = 0;
  const int64_t *n_pairs = nullptr;
  const float *pos = nullptr;
  Lattice lat;   // periodic cell (lat.periodic == 0: isolated systems)
  double r_c = 0, r_lo = 0, alpha = 0;
  const double *mu = nullptr, *beta = nullptr;
  const float *W0T = nullptr;
  const float *WaT[kMaxLayers], *WbT[kMaxLayers], *WcT[kMaxLayers];
  int L = 0;
  const float *z1[kMaxLayers], *z2[kMaxLayers], *z3[kMaxLayers];
  BwdGather g;
  float *gpair = nullptr;
};

int launch_pair_fwd(hipStream_t s, int F, int K, const PairFwdArgs &a, int variant);
int launch_pair_bwd(hipStream_t s, int F, int K, const PairBwdArgs &a, int variant);

// BF16-operand variants: weights, stored pre-activations and (when stored) the edge filters h in BF16;
// biases, basis constants, f0 and every other stored quantity in FP32/FP64 as above.
struct PairFwdArgsB {
  const int32_t *pairs = nullptr;
  int64_t max_pairs = 0;
  const int64_t *n_pairs = nullptr;
  const float *pos = nullptr;
  Lattice lat;   // periodic cell (lat.periodic == 0: isolated systems)
  double r_c = 0, r_lo = 0, alpha = 0;
  const double *mu = nullptr, *beta = nullptr;
  const __bf16 *W0 = nullptr;
  const float *b0 = nullptr;
  const __bf16 *Wa[kMaxLayers], *Wb[kMaxLayers], *Wc[kMaxLayers];
  const float *ba[kMaxLayers], *bb[kMaxLayers], *bc[kMaxLayers];
  int L = 0;
  float *geo = nullptr, *phi = nullptr;
  __bf16 *f0 = nullptr;   // the embedding map W0 e + b0 in BF16
  __bf16 *z1[kMaxLayers], *z2[kMaxLayers], *z3[kMaxLayers];
  __bf16 *h[kMaxLayers];   // the edge filters in BF16, or null: not stored (formed from z3 by the gathers)
};

struct PairBwdArgsB {
  const int32_t *pairs = nullptr;
  int64_t max_pairs = 0;
  const int64_t *n_pairs = nullptr;
  const float *pos = nullptr;
  Lattice lat;   // periodic cell (lat.periodic == 0: isolated systems)
  double r_c = 0, r_lo = 0, alpha = 0;
  const double *mu = nullptr, *beta = nullptr;
  const __bf16 *W0T = nullptr;
  const __bf16 *WaT[kMaxLayers], *WbT[kMaxLayers], *WcT[kMaxLayers];
  int L = 0;
  const __bf16 *z1[kMaxLayers], *z2[kMaxLayers], *z3[kMaxLayers];
  const __bf16 *Y16[kMaxLayers], *dM16[kMaxLayers];   // BF16 copies of g.Y and g.dM for the filter adjoints
  BwdGather g;
  float *gpair = nullptr;
};

int launch_pair_fwd_bf16(hipStream_t s, int F, int K, const PairFwdArgsB &a, int variant);
int launch_pair_bwd_bf16(hipStream_t s, int F, int K, const PairBwdArgsB &a, int variant);

inline unsigned grid_for(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

// Event pair around the launches of a named kernel while timing is enabled.
// Turns the timing registry on or off; returns the previous state.
bool timing_swap(bool on);

struct TimedScope {
  TimedScope(const char *name, hipStream_t s);
  ~TimedScope();
  int slot = -1;
  hipStream_t stream = nullptr;
};

}  // namespace tn
