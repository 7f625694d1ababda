// Molecule path: one launch for a batch of isolated systems of uneven sizes, in which a
// workgroup owns whole systems and runs every stage of the energy-and-forces evaluation for
// them with workgroup barriers only (Sec. 2.5: small systems are bound by launch overhead,
// which the paper removes by capturing the whole computation in one graph).  The grid is at
// most one workgroup per compute unit (the launch bound then leaves 512 registers per lane for
// the largest stage, the reverse pair tile, instead of spilling to memory); workgroup b takes
// systems b, b + grid, ...
//
// Per system (atoms [a0, a1) of the sorted batch vector), the stages are those of the fused
// path, computed by the same device code in the same order:
//   neighbour pairs (brute force over the system, FP64 predicate) -> row offsets -> sorted
//   CSR rows -> pair ids; pair tiles forward (geometry, basis, embedding map, edge filters);
//   embedding gather; FP64 node stage of the embedding; per layer mixing, message + product,
//   mixing, residual; FP64 output network and the system's energy sum; then the reverse sweep
//   and the pair tiles' reverse pass; per-atom force sums in FP64.
// A system of n atoms gets the pair slots [c(a0), c(a1)) with c(a) = max_pairs * a / N
// rounded up to a multiple of 16 (the static pair budget of the paper, split in proportion to
// the atoms); a system with more pairs sets the overflow bit and is skipped.
#include "tn_nodeops.h"
#include "tn_pairtile.h"

namespace tn {

namespace {

constexpr int kMolThreads = 256;
constexpr int kMolRB = 2;   // 32-pair tiles: little padding on molecules of a few hundred pairs

// The islands (embedding node stage, output network) run in FP64 with FP32 pair kernels and
// in FP32 with BF16 ones, as in the fused path; TA is their type.
template <class TA>
struct MolWs {
  int32_t *deg, *nup, *rowbeg, *pbase;
  int32_t *nbr, *pid, *pairs;
  float *geo, *phi, *f0, *Xr, *T0;
  TA *nrm0, *xhat0, *rstd0, *n0, *ez1, *ea1, *ez2, *g;
  float *X[kMaxLayers + 1], *nX[kMaxLayers], *Xb[kMaxLayers], *Y[kMaxLayers], *z1[kMaxLayers], *z2[kMaxLayers],
      *z3[kMaxLayers], *h[kMaxLayers], *M[kMaxLayers], *P[kMaxLayers], *nP[kMaxLayers], *Pb[kMaxLayers],
      *D[kMaxLayers], *dM[kMaxLayers];
  __bf16 *Y16[kMaxLayers], *dM16[kMaxLayers];   // BF16 copies of Y and dM for the gathers (BF16 path)
  TA *on, *oxhat, *orstd, *q, *oz, *ox, *hz, *hx, *eps;
  float *dX, *dD, *dPb, *dY, *dXr, *dT0;
  TA *dez2, *dez1, *dn0, *dnrm0, *dhz, *dox, *dq, *don;
  float *gpair;
};

// Pair capacity of the whole batch: max_pairs rounded up to whole 16-pair blocks.
__host__ __device__ inline int64_t mol_pair_capacity(int64_t max_pairs) { return (max_pairs + 15) / 16 * 16; }

template <class TA>
__host__ __device__ inline void plan_mol(WsPlan &p, int64_t F, int64_t L, int64_t N, int64_t MP, bool fw,
                                         MolWs<TA> *w) {
  w->deg = p.take<int32_t>(N);
  w->nup = p.take<int32_t>(N);
  w->rowbeg = p.take<int32_t>(N);
  w->pbase = p.take<int32_t>(N);
  w->nbr = p.take<int32_t>(2 * MP);
  w->pid = p.take<int32_t>(2 * MP);
  w->pairs = p.take<int32_t>(2 * MP);
  w->geo = p.take<float>(4 * MP);
  w->phi = p.take<float>(MP);
  w->f0 = p.take<float>(std::is_same<TA, float>::value ? MP * 3 * F / 2 : MP * 3 * F);   // BF16 in the BF16 path
  w->Xr = p.take<float>(N * 9 * F);
  w->T0 = p.take<float>(N * 9 * F);
  w->nrm0 = p.take<TA>(N * F);
  w->xhat0 = p.take<TA>(N * F);
  w->rstd0 = p.take<TA>(N);
  w->n0 = p.take<TA>(N * F);
  w->ez1 = p.take<TA>(N * 2 * F);
  w->ea1 = p.take<TA>(N * 2 * F);
  w->ez2 = p.take<TA>(N * 3 * F);
  w->g = p.take<TA>(N * 3 * F);
  for (int64_t l = 0; l <= L; ++l) w->X[l] = p.take<float>(N * 9 * F);
  for (int64_t l = 0; l < L; ++l) {
    w->nX[l] = p.take<float>(N * F);
    w->Xb[l] = p.take<float>(N * 9 * F);
    w->Y[l] = p.take<float>(N * 9 * F);
    w->z1[l] = p.take<float>(MP * F);   // MP is a multiple of 16 (whole 16-pair blocks)
    w->z2[l] = p.take<float>(MP * 2 * F);
    w->z3[l] = p.take<float>(MP * 3 * F);
    w->h[l] = nullptr;   // not stored (formed from z3 and phi where needed)
    w->M[l] = p.take<float>(N * 9 * F);
    w->P[l] = nullptr;   // formed again by the reverse pass, as in the fused path
    w->nP[l] = nullptr;
    w->Pb[l] = p.take<float>(N * 9 * F);
    w->D[l] = p.take<float>(N * 9 * F);
    w->Y16[l] = std::is_same<TA, float>::value ? p.take<__bf16>(N * 9 * F) : nullptr;
  }
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
  for (int64_t l = 0; l < L; ++l) {
    w->dM[l] = p.take<float>(N * 9 * F);
    w->dM16[l] = std::is_same<TA, float>::value ? p.take<__bf16>(N * 9 * F) : nullptr;
  }
  w->dX = p.take<float>(N * 9 * F);
  w->dD = p.take<float>(N * 9 * F);
  w->dPb = p.take<float>(N * 9 * F);
  w->dY = p.take<float>(N * 9 * F);
  w->dXr = p.take<float>(N * 9 * F);
  w->dT0 = p.take<float>(N * 9 * F);
  w->dez2 = p.take<TA>(N * 3 * F);
  w->dez1 = p.take<TA>(N * 2 * F);
  w->dn0 = p.take<TA>(N * F);
  w->dnrm0 = p.take<TA>(N * F);
  w->dhz = p.take<TA>(N * (F / 2));
  w->dox = p.take<TA>(N * F);
  w->dq = p.take<TA>(N * 3 * F);
  w->don = p.take<TA>(N * 3 * F);
  w->gpair = p.take<float>(3 * MP);
}

// Weight pointers of the model (FP32 copies for the FP32 stages, FP64 for the islands, BF16
// for the BF16 pair tiles and mixing).
template <class T>
struct IslandWeights {
  const T *ln_g, *ln_b, *W1, *b1, *W2, *b2, *oln_g, *oln_b, *Wo, *bo, *Wh, *bh, *wout, *bout;
};

struct MolWeights {
  const float *U, *V, *Wemb[3], *WembT[3];
  IslandWeights<double> i64;
  IslandWeights<float> i32;
  const float *W1l[kMaxLayers][3], *W1Tl[kMaxLayers][3], *W2l[kMaxLayers][3], *W2Tl[kMaxLayers][3];
  // BF16 copies of the mixing matrices (BF16 path)
  const __bf16 *Wemb16[3], *WembT16[3];
  const __bf16 *W1l16[kMaxLayers][3], *W1Tl16[kMaxLayers][3], *W2l16[kMaxLayers][3], *W2Tl16[kMaxLayers][3];
};

__device__ __forceinline__ const IslandWeights<double> &island(const MolWeights &w, double) { return w.i64; }
__device__ __forceinline__ const IslandWeights<float> &island(const MolWeights &w, float) { return w.i32; }

// The model's weight pointers for this path, uploaded once at model creation.
struct MolConst {
  MolWeights wt;
  PairFwdArgs pf;   // weight fields only; the workspace fields are filled per call
  PairBwdArgs pb;
  PairFwdArgsB pfb;
  PairBwdArgsB pbb;
};

// Per-call arguments (the setup kernel's argument).
struct MolCall {
  int64_t N = 0, S = 0, MP = 0, max_pairs = 0;
  int F = 0, K = 0, L = 0, max_z = 0, want_forces = 0;
  double rc2 = 0;
  const float *pos = nullptr;
  const int32_t *z = nullptr, *batch = nullptr;
  double *energy = nullptr;
  float *forces = nullptr;
  int64_t *n_pairs = nullptr;
  int32_t *status = nullptr;
  char *ws = nullptr;             // workspace: this call's MolArgs first, then the arrays
  const MolConst *c = nullptr;
};

// Everything the molecule kernel reads, built in the workspace by the setup kernel (too large
// for kernel arguments).
template <class TA>
struct MolArgs {
  int64_t N, S, MP, max_pairs;
  int F, K, L, max_z, want_forces;
  double rc2;
  const float *pos;
  const int32_t *z, *batch;
  double *energy;
  float *forces;
  int64_t *n_pairs;
  int32_t *status;
  MolWs<TA> w;
  MolWeights wt;
  PairFwdArgs pf;
  PairBwdArgs pb;
  PairFwdArgsB pfb;
  PairBwdArgsB pbb;
};

// Workspace plan: the argument block, then the arrays.
template <class TA>
__host__ __device__ inline MolArgs<TA> *plan_mol_call(WsPlan &p, int64_t F, int64_t L, int64_t N, int64_t MP,
                                                      bool fw, MolWs<TA> *w) {
  MolArgs<TA> *a = reinterpret_cast<MolArgs<TA> *>(p.take<char>(sizeof(MolArgs<TA>)));
  plan_mol(p, F, L, N, MP, fw, w);
  return a;
}

// The cutoff predicate of the neighbour search (FP64 on promoted positions, products rounded,
// no contraction), without a box.
__device__ inline bool mol_pair_within(const float *pos, int64_t i, int64_t j, double rc2) {
#pragma clang fp contract(off)
  const double dx = (double)pos[3 * j] - (double)pos[3 * i];
  const double dy = (double)pos[3 * j + 1] - (double)pos[3 * i + 1];
  const double dz = (double)pos[3 * j + 2] - (double)pos[3 * i + 2];
  const double xx = dx * dx;
  const double yy = dy * dy;
  const double zz = dz * dz;
  const double d2 = (xx + yy) + zz;
  return d2 < rc2;
}

// Shared memory of the molecule kernel's mixing and FP64 product stages (one buffer); the pair
// tiles bring their own LDS arrays.
template <int F>
struct MolLds {
  static constexpr size_t mixb = 16 * 5 * (F + 4) * 4;   // FP32 staging; the BF16 staging is smaller
  static_assert(16 * 5 * (F + kPadB) * 2 <= mixb, "BF16 mixing tile exceeds the buffer");
  static constexpr size_t gemmb = (32 + GBN) * (GBK + 1) * 8;
  static constexpr size_t bytes = mixb > gemmb ? mixb : gemmb;
};

// Carves a byte buffer into consecutive 16-byte aligned arrays.
struct Carve {
  char *p;
  template <class T> __device__ T *take(size_t count) {
    T *r = reinterpret_cast<T *>(p);
    p += (count * sizeof(T) + 15) / 16 * 16;
    return r;
  }
};

// Setup, one workgroup: the input checks (batch sorted and in range, z in range, finite
// positions), the pair counter cleared, and this call's MolArgs written to the workspace.
template <class TA>
__global__ void __launch_bounds__(kMolThreads) k_mol_setup(MolCall c) {
  const int tid = threadIdx.x;
  for (int64_t i = tid; i < c.N; i += kMolThreads) {
    const int32_t b = c.batch[i];
    if (i > 0 && b < c.batch[i - 1]) set_status(c.status, TN_STATUS_BATCH);
    if (b < 0 || b >= c.S) set_status(c.status, TN_STATUS_BATCH);
    if (c.z[i] < 0 || c.z[i] >= c.max_z) set_status(c.status, TN_STATUS_Z);
    if (!isfinite(c.pos[3 * i]) || !isfinite(c.pos[3 * i + 1]) || !isfinite(c.pos[3 * i + 2]))
      set_status(c.status, TN_STATUS_NONFINITE);
  }
  if (tid != 0) return;
  *c.n_pairs = 0;
  WsPlan plan(c.ws);
  MolWs<TA> w;
  MolArgs<TA> *a = plan_mol_call<TA>(plan, c.F, c.L, c.N, c.MP, c.want_forces != 0, &w);
  a->N = c.N;
  a->S = c.S;
  a->MP = c.MP;
  a->max_pairs = c.max_pairs;
  a->F = c.F;
  a->K = c.K;
  a->L = c.L;
  a->max_z = c.max_z;
  a->want_forces = c.want_forces;
  a->rc2 = c.rc2;
  a->pos = c.pos;
  a->z = c.z;
  a->batch = c.batch;
  a->energy = c.energy;
  a->forces = c.forces;
  a->n_pairs = c.n_pairs;
  a->status = c.status;
  a->w = w;
  a->wt = c.c->wt;
  a->pf = c.c->pf;
  a->pb = c.c->pb;
  a->pfb = c.c->pfb;
  a->pbb = c.c->pbb;
  // the workspace and input fields of the pair tiles' arguments
  auto common = [&](auto &p) {
    p.pairs = w.pairs;
    p.max_pairs = c.MP;
    p.n_pairs = c.n_pairs;
    p.pos = c.pos;
  };
  auto gather = [&](BwdGather &g) {
    g.z = c.z;
    g.dXr = w.dXr;
    for (int l = 0; l < c.L; ++l) {
      g.Y[l] = w.Y[l];
      g.dM[l] = w.dM[l];
    }
  };
  common(a->pf);
  common(a->pb);
  common(a->pfb);
  common(a->pbb);
  gather(a->pb.g);
  gather(a->pbb.g);
  for (int l = 0; l < c.L; ++l) {
    a->pbb.Y16[l] = w.Y16[l];
    a->pbb.dM16[l] = w.dM16[l];
  }
  a->pf.geo = a->pfb.geo = w.geo;
  a->pf.phi = a->pfb.phi = w.phi;
  a->pf.f0 = w.f0;
  a->pfb.f0 = reinterpret_cast<__bf16 *>(w.f0);
  a->pb.g.f0 = w.f0;
  a->pbb.g.f016 = reinterpret_cast<const __bf16 *>(w.f0);
  a->pb.gpair = a->pbb.gpair = w.gpair;
  for (int l = 0; l < c.L; ++l) {
    a->pf.z1[l] = w.z1[l];
    a->pf.z2[l] = w.z2[l];
    a->pf.z3[l] = w.z3[l];
    a->pf.h[l] = nullptr;   // not stored: the message gathers form h from z3 and phi
    a->pb.z1[l] = w.z1[l];
    a->pb.z2[l] = w.z2[l];
    a->pb.z3[l] = w.z3[l];
    a->pfb.z1[l] = reinterpret_cast<__bf16 *>(w.z1[l]);
    a->pfb.z2[l] = reinterpret_cast<__bf16 *>(w.z2[l]);
    a->pfb.z3[l] = reinterpret_cast<__bf16 *>(w.z3[l]);
    a->pfb.h[l] = nullptr;
    a->pbb.z1[l] = reinterpret_cast<const __bf16 *>(w.z1[l]);
    a->pbb.z2[l] = reinterpret_cast<const __bf16 *>(w.z2[l]);
    a->pbb.z3[l] = reinterpret_cast<const __bf16 *>(w.z3[l]);
  }
}

template <int F, int K, bool BF16>
__global__ void __launch_bounds__(kMolThreads, 1)
    k_molecules(const MolArgs<typename std::conditional<BF16, float, double>::type> *__restrict__ ap) {
  using TA = typename std::conditional<BF16, float, double>::type;
  const MolArgs<TA> &a = *ap;
  __shared__ __attribute__((aligned(16))) char smem[MolLds<F>::bytes];
  constexpr int TILE = 16 * kMolRB;
  constexpr int V = F / 128 > 0 ? F / 128 : 1, G = F / (64 * V);   // the wave gathers' channel split
  constexpr int NBMIX = F == 256 ? 2 : 1, NCB = F / (64 * NBMIX);
  constexpr int H = F / 2;
  using TH = typename std::conditional<BF16, __bf16, float>::type;   // the edge filters' type
  using TY = TH;   // the atom rows the gathers read (Y, dM)
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const MolWs<TA> &w = a.w;
  const MolWeights &wt = a.wt;
  const IslandWeights<TA> &iw = island(wt, TA(0));
  __shared__ int32_t s_i[kMolThreads];
  __shared__ double s_d[128];
  // the FP64 products' arguments in LDS (an argument struct in registers would be indexed
  // dynamically, which puts it in scratch memory)
  __shared__ __attribute__((aligned(16))) char s_gemm_raw[sizeof(GemmArgs<TA>)];
  GemmArgs<TA> &s_gemm = *reinterpret_cast<GemmArgs<TA> *>(s_gemm_raw);
  if (*a.status & TN_STATUS_BATCH) return;   // system ranges are undefined for an unsorted batch

  for (int64_t sys = blockIdx.x; sys < a.S; sys += gridDim.x) {
    const int64_t a0 = block_lower_bound(a.batch, a.N, (int32_t)sys);
    const int64_t a1 = block_lower_bound(a.batch, a.N, (int32_t)sys + 1);
    const int64_t n = a1 - a0;
    const int64_t pr0 = a.N > 0 ? (a.max_pairs * a0 / a.N + 15) / 16 * 16 : 0;
    const int64_t pr1 = a.N > 0 ? (a.max_pairs * a1 / a.N + 15) / 16 * 16 : 0;
    // ---- neighbour pairs: degree and upper degree of every atom (one wave per atom)
    for (int64_t s = a0 + wave; s < a1; s += 4) {
      int32_t full = 0, upper = 0;
      for (int64_t q0 = a0; q0 < a1; q0 += 64) {
        const int64_t j = q0 + lane;
        const bool pred = j < a1 && j != s && mol_pair_within(a.pos, s, j, a.rc2);
        full += __popcll(__ballot(pred));
        upper += __popcll(__ballot(pred && j > s));
      }
      if (lane == 0) {
        w.deg[s] = full;
        w.nup[s] = upper;
      }
    }
    __syncthreads();
    // ---- row offsets and pair bases: a workgroup scan in chunks of 256 atoms
    int32_t carry_e = 0, carry_p = 0;
    for (int64_t c0 = a0; c0 < a1; c0 += kMolThreads) {
      const int64_t s = c0 + tid;
      const int32_t dv = s < a1 ? w.deg[s] : 0, uv = s < a1 ? w.nup[s] : 0;
      // inclusive scans of (deg, nup) packed as one 64-bit value per thread
      s_i[tid] = dv;
      __syncthreads();
      for (int off = 1; off < kMolThreads; off <<= 1) {
        const int32_t t = tid >= off ? s_i[tid - off] : 0;
        __syncthreads();
        s_i[tid] += t;
        __syncthreads();
      }
      const int32_t incl_e = s_i[tid], tot_e = s_i[kMolThreads - 1];
      __syncthreads();
      s_i[tid] = uv;
      __syncthreads();
      for (int off = 1; off < kMolThreads; off <<= 1) {
        const int32_t t = tid >= off ? s_i[tid - off] : 0;
        __syncthreads();
        s_i[tid] += t;
        __syncthreads();
      }
      const int32_t incl_p = s_i[tid], tot_p = s_i[kMolThreads - 1];
      __syncthreads();
      if (s < a1) {
        w.rowbeg[s] = (int32_t)(2 * pr0) + carry_e + incl_e - dv;
        w.pbase[s] = (int32_t)pr0 + carry_p + incl_p - uv;
      }
      carry_e += tot_e;
      carry_p += tot_p;
    }
    const int64_t np = carry_p;   // pairs of this system
    if (tid == 0) {
      atomicAdd(reinterpret_cast<unsigned long long *>(a.n_pairs), (unsigned long long)np);
      if (np > pr1 - pr0) set_status(a.status, TN_STATUS_OVERFLOW);
    }
    if (np > pr1 - pr0) continue;   // outputs of this system stay undefined (flagged)
    __syncthreads();
    // ---- CSR rows sorted by neighbour, then the pair id of every directed edge
    for (int64_t s = a0 + wave; s < a1; s += 4) {
      const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
      int32_t e = w.rowbeg[s];
      for (int64_t q0 = a0; q0 < a1; q0 += 64) {
        const int64_t j = q0 + lane;
        const bool pred = j < a1 && j != s && mol_pair_within(a.pos, s, j, a.rc2);
        const uint64_t mk = __ballot(pred);
        if (pred) w.nbr[e + __popcll(mk & below)] = (int32_t)j;
        e += __popcll(mk);
      }
    }
    __syncthreads();
    for (int64_t s = a0 + wave; s < a1; s += 4) {
      const int32_t b0 = w.rowbeg[s], e1 = b0 + w.deg[s];
      const int32_t nlow = w.deg[s] - w.nup[s];
      for (int32_t k = b0 + lane; k < e1; k += 64) {
        const int32_t j = w.nbr[k];
        int32_t p;
        if (j > s) {
          p = w.pbase[s] + (k - b0 - nlow);
          w.pairs[p] = (int32_t)s;
          w.pairs[a.MP + p] = j;
        } else {
          const int32_t bj = w.rowbeg[j], ej = bj + w.deg[j];
          int32_t lo = bj, hi = ej;
          while (lo < hi) {
            const int32_t mm = (lo + hi) >> 1;
            if (w.nbr[mm] < (int32_t)s) lo = mm + 1; else hi = mm;
          }
          p = w.pbase[j] + (lo - bj - (w.deg[j] - w.nup[j]));
        }
        w.pid[k] = p;
      }
    }
    __syncthreads();
    const int64_t ntile = (np + TILE - 1) / TILE;
    // ---- pair tiles, forward
    for (int64_t t = 0; t < ntile; ++t) {
      const int64_t p0 = pr0 + t * TILE;
      const int nv = (int)(np - t * TILE < TILE ? np - t * TILE : TILE);
      if constexpr (BF16)
        pair_fwd_tile_bf16<F, K, kMolRB>(a.pfb, p0, nv);
      else
        pair_fwd_tile<F, K, kMolRB, 4>(a.pf, p0, nv);
      __syncthreads();
    }
    // ---- embedding gather (G waves per atom, 4 / G atoms at a time)
    auto atoms_waves = [&](auto &&fn) {
      for (int64_t i0 = a0; i0 < a1; i0 += 4 / G) {
        const int64_t i = i0 + wave / G;
        if (i < a1) fn((int32_t)i, ((wave % G) * 64 + lane) * V);
      }
    };
    atoms_waves([&](int32_t i, int f) {
      embed_gather_wave<V, G, TH>(i, f, w.rowbeg[i], w.rowbeg[i] + w.deg[i], w.nbr, w.pid, a.z, a.max_z, wt.U,
                                  wt.V, w.geo, w.phi, reinterpret_cast<const TH *>(w.f0), w.Xr);
    });
    __syncthreads();
    auto per_channel = [&](int64_t per_atom, auto &&fn) {
      for (int64_t t = a0 * per_atom + tid; t < a1 * per_atom; t += kMolThreads) fn(t);
    };
    auto per_row_wave = [&](auto &&fn) {
      for (int64_t r = a0 + wave; r < a1; r += 4) fn(r);
    };
    auto gemm_rows = [&](const GemmArgs<TA> &g0) {   // the product over this system's rows
      if (tid == 0) {
        GemmArgs<TA> g = g0;
        g.A += a0 * g.lda;
        g.C += a0 * g.ldc;
        if (g.Z) g.Z += a0 * g.ldz;
        if (g.gate) g.gate += a0 * g.ldg;
        g.M = n;
        s_gemm = g;
      }
      __syncthreads();
      const int64_t nb = (g0.N + GBN - 1) / GBN, mt = (n + 31) / 32;
      Carve c{smem};
      TA(*As)[GBK + 1] = reinterpret_cast<TA(*)[GBK + 1]>(c.take<TA>(32 * (GBK + 1)));
      TA(*Bs)[GBK + 1] = reinterpret_cast<TA(*)[GBK + 1]>(c.take<TA>(GBN * (GBK + 1)));
      for (int64_t blk = 0; blk < nb * mt; ++blk) gemm_tile<TA, 32>(s_gemm, blk, 0, As, Bs);
      __syncthreads();
    };
    // channel mixing of the system's rows: FP32 matrix cores, or BF16 operands in the BF16 path
    auto mix_rows = [&](const float *in, float *out, const float *const B[3], const __bf16 *const B16[3], int acc,
                        __bf16 *out16 = nullptr) {
      __bf16 *o16 = out16 ? out16 + a0 * 9 * F : nullptr;
      if constexpr (BF16) {
        constexpr int NB16 = MixBf16Shape<F>::NB, NCB16 = MixBf16Shape<F>::ncb;
        const int64_t nt = (n + 15) / 16 * NCB16 * 3;
        __bf16 *sA = reinterpret_cast<__bf16 *>(smem);
        for (int64_t t = 0; t < nt; ++t) {
          mix_tile_bf16<F, NB16>(in + a0 * 9 * F, out + a0 * 9 * F, n, B16[0], B16[1], B16[2], acc, NCB16, t, sA,
                                 o16);
          __syncthreads();
        }
      } else {
        const int64_t nt = (n + 15) / 16 * NCB * 3;
        float *sA = reinterpret_cast<float *>(smem);
        for (int64_t t = 0; t < nt; ++t) {
          mix_tile<F, NBMIX>(in + a0 * 9 * F, out + a0 * 9 * F, n, B[0], B[1], B[2], acc, NCB, t, sA, o16);
          __syncthreads();
        }
      }
    };
    // ---- embedding node stage (FP64)
    per_channel(F, [&](int64_t t) { node_norm_at<TA, float>(t, F, w.Xr, w.nrm0); });
    __syncthreads();
    per_row_wave([&](int64_t r) { layernorm_row_wave(r, F, w.nrm0, iw.ln_g, iw.ln_b, w.n0, w.xhat0, w.rstd0); });
    __syncthreads();
    gemm_rows(linear_fwd_args<TA>(w.n0, n, F, iw.W1, iw.b1, 2 * F, w.ea1, w.ez1, 1));
    gemm_rows(linear_fwd_args<TA>(w.ea1, n, 2 * F, iw.W2, iw.b2, 3 * F, w.g, w.ez2, 1));
    mix_rows(w.Xr, w.T0, wt.Wemb, wt.Wemb16, 0);
    if (a.L > 0)
      per_channel(F, [&](int64_t t) { gate_normalize_at<TA, float>(t, F, w.g, w.T0, w.X[0], w.nX[0], w.Xb[0]); });
    else
      per_channel(9 * F, [&](int64_t t) { gate_at<TA, float>(t, F, w.g, w.T0, w.X[0]); });
    __syncthreads();
    // ---- interaction layers
    for (int l = 0; l < a.L; ++l) {
      mix_rows(w.Xb[l], w.Y[l], wt.W1l[l], wt.W1l16[l], 0, BF16 ? w.Y16[l] : nullptr);
      const TY *yg = BF16 ? reinterpret_cast<const TY *>(w.Y16[l]) : reinterpret_cast<const TY *>(w.Y[l]);
      atoms_waves([&](int32_t i, int f) {
        message_product_wave<V, G, TH, TY, float, true>(i, f, w.rowbeg[i], w.rowbeg[i] + w.deg[i], w.nbr, w.pid,
                                                        reinterpret_cast<const TH *>(w.z3[l]), yg, w.Y[l], w.M[l],
                                                        w.P[l], w.nP[l], w.Pb[l], w.phi);
      });
      __syncthreads();
      mix_rows(w.Pb[l], w.D[l], wt.W2l[l], wt.W2l16[l], 0);
      if (l + 1 < a.L)
        per_channel(F, [&](int64_t t) {
          residual_normalize_at<float>(t, F, w.Xb[l], w.D[l], w.X[l + 1], w.nX[l + 1], w.Xb[l + 1]);
        });
      else
        per_channel(F, [&](int64_t t) { residual_at<float>(t, F, w.Xb[l], w.D[l], w.X[l + 1]); });
      __syncthreads();
    }
    // ---- output network (FP64) and the system's energy
    per_channel(F, [&](int64_t t) { out_norms_at<TA, float>(t, F, w.X[a.L], w.on); });
    __syncthreads();
    per_row_wave([&](int64_t r) {
      layernorm_row_wave(r, 3 * F, w.on, iw.oln_g, iw.oln_b, w.q, w.oxhat, w.orstd);
    });
    __syncthreads();
    gemm_rows(linear_fwd_args<TA>(w.q, n, 3 * F, iw.Wo, iw.bo, F, w.ox, w.oz, 1));
    gemm_rows(linear_fwd_args<TA>(w.ox, n, F, iw.Wh, iw.bh, H, w.hx, w.hz, 1));
    per_row_wave([&](int64_t r) { out_final_wave<TA>((int32_t)r, H, w.hx, iw.wout, iw.bout, w.eps); });
    __syncthreads();
    {  // E_s in FP64: 128 partial sums strided over the atoms, then a fixed tree
      double acc = 0.0;
      if (tid < 128)
        for (int64_t i = a0 + tid; i < a1; i += 128) acc += (double)w.eps[i];
      if (tid < 128) s_d[tid] = acc;
      __syncthreads();
      for (int st = 64; st > 0; st >>= 1) {
        if (tid < st) s_d[tid] += s_d[tid + st];
        __syncthreads();
      }
      if (tid == 0) {
        a.energy[sys] = s_d[0];
        if (!isfinite(s_d[0])) set_status(a.status, TN_STATUS_NONFINITE);
      }
      __syncthreads();
    }
    if (!a.want_forces) continue;
    // ================================================================ reverse sweep
    per_channel(H, [&](int64_t t) { out_final_bwd_at<TA>(t, H, w.hz, iw.wout, w.dhz); });
    __syncthreads();
    gemm_rows(linear_bwd_args<TA>(w.dhz, n, H, iw.Wh, F, w.dox, w.oz, 0));
    gemm_rows(linear_bwd_args<TA>(w.dox, n, F, iw.Wo, 3 * F, w.dq, nullptr, 0));
    per_row_wave([&](int64_t r) { layernorm_bwd_row_wave(r, 3 * F, w.dq, w.oxhat, w.orstd, iw.oln_g, w.don); });
    __syncthreads();
    per_channel(F, [&](int64_t t) { out_norms_bwd_at<TA, float>(t, F, w.X[a.L], w.don, w.dX); });
    __syncthreads();
    for (int l = a.L - 1; l >= 0; --l) {
      per_channel(F, [&](int64_t t) { residual_bwd_at<float>(t, F, w.D[l], w.dX, w.dD); });
      __syncthreads();
      mix_rows(w.dD, w.dPb, wt.W2Tl[l], wt.W2Tl16[l], 0);
      per_channel(F, [&](int64_t t) {
        product_bwd_at<float>(t, F, w.dPb, w.P[l], w.nP[l], w.Y[l], w.M[l], w.dY, w.dM[l],
                              BF16 ? w.dM16[l] : nullptr);
      });
      __syncthreads();
      const TY *dmg = BF16 ? reinterpret_cast<const TY *>(w.dM16[l]) : reinterpret_cast<const TY *>(w.dM[l]);
      atoms_waves([&](int32_t i, int f) {
        message_wave<V, G, TH, TY, float, true>(i, f, w.rowbeg[i], w.rowbeg[i] + w.deg[i], w.nbr, w.pid,
                                                reinterpret_cast<const TH *>(w.z3[l]), dmg, w.dY, 1, nullptr,
                                                w.phi);
      });
      __syncthreads();
      mix_rows(w.dY, w.dX, wt.W1Tl[l], wt.W1Tl16[l], 1);
      per_channel(F, [&](int64_t t) { normalize_bwd_at<float>(t, F, w.X[l], w.nX[l], w.dX); });
      __syncthreads();
    }
    per_channel(F, [&](int64_t t) { gate_bwd_at<TA, float>(t, F, w.dX, w.T0, w.g, w.dez2, w.dT0, w.ez2); });
    __syncthreads();
    mix_rows(w.dT0, w.dXr, wt.WembT, wt.WembT16, 0);
    gemm_rows(linear_bwd_args<TA>(w.dez2, n, 3 * F, iw.W2, 2 * F, w.dez1, w.ez1, 0));
    gemm_rows(linear_bwd_args<TA>(w.dez1, n, 2 * F, iw.W1, F, w.dn0, nullptr, 0));
    per_row_wave([&](int64_t r) { layernorm_bwd_row_wave(r, F, w.dn0, w.xhat0, w.rstd0, iw.ln_g, w.dnrm0); });
    __syncthreads();
    per_channel(F, [&](int64_t t) { norm_bwd_add_at<TA, float>(t, F, w.Xr, w.dnrm0, w.dXr); });
    __syncthreads();
    // ---- pair tiles, reverse
    for (int64_t t = 0; t < ntile; ++t) {
      const int64_t p0 = pr0 + t * TILE;
      const int nv = (int)(np - t * TILE < TILE ? np - t * TILE : TILE);
      if constexpr (BF16)
        pair_bwd_tile_bf16<F, K, kMolRB>(a.pbb, p0, nv);
      else
        pair_bwd_tile<F, K, kMolRB, 4, 2>(a.pb, p0, nv);
      __syncthreads();
    }
    // ---- forces: per-atom sums of the pair gradients in FP64
    per_row_wave([&](int64_t i) {
      force_gather_wave<float, float>((int32_t)i, i, true, w.rowbeg[i], w.rowbeg[i] + w.deg[i], w.nbr, w.pid,
                                      w.gpair, a.forces);
    });
    __syncthreads();
  }
}

template <int F, int K, bool BF16>
int launch_molecules(hipStream_t s, const MolArgs<typename std::conditional<BF16, float, double>::type> *a,
                     int grid) {
  hipLaunchKernelGGL((k_molecules<F, K, BF16>), dim3((unsigned)grid), dim3(kMolThreads), 0, s, a);
  TN_LAUNCH_CHECK();
  return TN_OK;
}

}  // namespace

bool molecule_kernels_support(int F, int K, bool bf16) {
  (void)bf16;
  return (F == 64 || F == 128) && K == 32;
}

size_t molecule_workspace_bytes(const tn_model *m, int64_t n, int64_t S, int64_t max_pairs, int prec,
                                int want_forces) {
  (void)S;
  if ((prec != TN_FP32 && prec != TN_BF16) || !molecule_kernels_support(m->F, m->K, prec == TN_BF16) ||
      m->L > kMaxLayers)
    return 0;
  WsPlan p(nullptr);
  if (prec == TN_BF16) {
    MolWs<float> w;
    plan_mol_call<float>(p, m->F, m->L, n, mol_pair_capacity(max_pairs), want_forces != 0, &w);
  } else {
    MolWs<double> w;
    plan_mol_call<double>(p, m->F, m->L, n, mol_pair_capacity(max_pairs), want_forces != 0, &w);
  }
  return p.off;
}

int molecule_run(const tn_model *m, hipStream_t s, const Problem &pb, int prec, void *ws, size_t ws_bytes) {
  const bool bf16 = prec == TN_BF16;
  if ((prec != TN_FP32 && prec != TN_BF16) || !molecule_kernels_support(m->F, m->K, bf16) || m->L > kMaxLayers ||
      pb.box.periodic)
    return TN_E_UNSUPPORTED;
  const int64_t N = pb.n, MP = mol_pair_capacity(pb.max_pairs), F = m->F, L = m->L;
  if (2 * MP >= (int64_t(1) << 31)) return TN_E_ARG;   // CSR offsets are int32
  if (!m->mol_const) return TN_E_UNSUPPORTED;
  auto go = [&](auto ta) -> int {
  using TA = decltype(ta);
  WsPlan plan(ws);
  MolWs<TA> w;
  MolArgs<TA> *args = plan_mol_call<TA>(plan, F, L, N, MP, pb.want_forces, &w);
  if (plan.off > ws_bytes) return TN_E_WORKSPACE;
  MolCall c;
  c.N = N;
  c.S = pb.S;
  c.MP = MP;
  c.max_pairs = pb.max_pairs;
  c.F = (int)F;
  c.K = m->K;
  c.L = (int)L;
  c.max_z = m->max_z;
  c.want_forces = pb.want_forces ? 1 : 0;
  c.rc2 = m->r_c * m->r_c;
  c.pos = static_cast<const float *>(pb.pos);
  c.z = pb.z;
  c.batch = pb.batch;
  c.energy = pb.energy;
  c.forces = static_cast<float *>(pb.forces);
  c.n_pairs = pb.n_pairs;
  c.status = pb.status;
  c.ws = static_cast<char *>(ws);
  c.c = static_cast<const MolConst *>(m->mol_const);
  hipLaunchKernelGGL(k_mol_setup<TA>, dim3(1), dim3(kMolThreads), 0, s, c);
  TN_LAUNCH_CHECK();
  if (pb.S <= 0) return TN_OK;
  int dev_cu = 256;
  (void)hipDeviceGetAttribute(&dev_cu, hipDeviceAttributeMultiprocessorCount, m->device);
  const int grid = (int)std::min<int64_t>(pb.S, (int64_t)(dev_cu > 0 ? dev_cu : 256));
  constexpr bool B = std::is_same<TA, float>::value;   // FP32 islands go with the BF16 pair tiles
  if (F == 64) return launch_molecules<64, 32, B>(s, args, grid);
  return launch_molecules<128, 32, B>(s, args, grid);
  };
  return bf16 ? go(float(0)) : go(double(0));
}

int molecule_setup(tn_model *m) {
  if (!molecule_kernels_support(m->F, m->K, false) || m->L > kMaxLayers) return TN_OK;
  auto W = [&](size_t off) { return wptr<float>(m, off); };
  auto WA = [&](size_t off) { return wptr<double>(m, off); };
  auto WB = [&](size_t off) { return static_cast<const __bf16 *>(m->w16 + off); };
  const WeightOff &o = m->off;
  const int64_t L = m->L;
  MolConst h{};
  MolWeights &wt = h.wt;
  wt.U = W(o.U);
  wt.V = W(o.V);
  for (int q = 0; q < 3; ++q) {
    wt.Wemb[q] = W(o.Wmixf[q]);
    wt.WembT[q] = W(o.WmixT[q]);
    wt.Wemb16[q] = WB(o.Wmixf[q]);
    wt.WembT16[q] = WB(o.WmixT[q]);
  }
  auto islands = [&](auto &iw, auto ptr) {
    iw.ln_g = ptr(o.ln_g);
    iw.ln_b = ptr(o.ln_b);
    iw.W1 = ptr(o.W1);
    iw.b1 = ptr(o.b1);
    iw.W2 = ptr(o.W2);
    iw.b2 = ptr(o.b2);
    iw.oln_g = ptr(o.oln_g);
    iw.oln_b = ptr(o.oln_b);
    iw.Wo = ptr(o.Wo);
    iw.bo = ptr(o.bo);
    iw.Wh = ptr(o.Wh);
    iw.bh = ptr(o.bh);
    iw.wout = ptr(o.wout);
    iw.bout = ptr(o.bout);
  };
  islands(wt.i64, WA);
  islands(wt.i32, W);
  for (int64_t l = 0; l < L; ++l)
    for (int q = 0; q < 3; ++q) {
      wt.W1l[l][q] = W(o.layer[l].W1f[q]);
      wt.W1Tl[l][q] = W(o.layer[l].W1T[q]);
      wt.W2l[l][q] = W(o.layer[l].W2f[q]);
      wt.W2Tl[l][q] = W(o.layer[l].W2T[q]);
      wt.W1l16[l][q] = WB(o.layer[l].W1f[q]);
      wt.W1Tl16[l][q] = WB(o.layer[l].W1T[q]);
      wt.W2l16[l][q] = WB(o.layer[l].W2f[q]);
      wt.W2Tl16[l][q] = WB(o.layer[l].W2T[q]);
    }
  auto model_fields = [&](auto &p) {
    p.lat = Lattice{};
    p.r_c = m->r_c;
    p.r_lo = m->r_lo;
    p.alpha = m->alpha;
    p.mu = WA(o.mu);
    p.beta = WA(o.beta);
    p.L = (int)L;
  };
  auto gather_fields = [&](BwdGather &g) {
    g.U = W(o.U);
    g.V = W(o.V);
    g.max_z = m->max_z;
  };
  model_fields(h.pf);
  model_fields(h.pb);
  model_fields(h.pfb);
  model_fields(h.pbb);
  gather_fields(h.pb.g);
  gather_fields(h.pbb.g);
  h.pf.W0 = W(o.W0f);
  h.pf.b0 = W(o.b0);
  h.pb.W0T = W(o.W0T);
  h.pfb.W0 = WB(o.W0f);
  h.pfb.b0 = W(o.b0);
  h.pbb.W0T = WB(o.W0T);
  for (int64_t l = 0; l < L; ++l) {
    const LayerOff &lo = o.layer[l];
    h.pf.Wa[l] = W(lo.Waf);
    h.pf.ba[l] = W(lo.ba);
    h.pf.Wb[l] = W(lo.Wbf);
    h.pf.bb[l] = W(lo.bb);
    h.pf.Wc[l] = W(lo.Wcf);
    h.pf.bc[l] = W(lo.bc);
    h.pb.WaT[l] = W(lo.WaT);
    h.pb.WbT[l] = W(lo.WbT);
    h.pb.WcT[l] = W(lo.WcT);
    h.pfb.Wa[l] = WB(lo.Waf);
    h.pfb.Wb[l] = WB(lo.Wbf);
    h.pfb.Wc[l] = WB(lo.Wcf);
    h.pfb.ba[l] = W(lo.ba);
    h.pfb.bb[l] = W(lo.bb);
    h.pfb.bc[l] = W(lo.bc);
    h.pbb.WaT[l] = WB(lo.WaT);
    h.pbb.WbT[l] = WB(lo.WbT);
    h.pbb.WcT[l] = WB(lo.WcT);
  }
  TN_HIP(hipMalloc(&m->mol_const, sizeof(MolConst)));
  TN_HIP(hipMemcpy(m->mol_const, &h, sizeof(MolConst), hipMemcpyHostToDevice));
  return TN_OK;
}

}  // namespace tn
