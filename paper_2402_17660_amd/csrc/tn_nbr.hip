// Neighbour search (Sec. 2.5.1 of the paper): unordered pairs of atoms of the
// same system closer than the cutoff, minimum image in a rectangular or triclinic cell.
//
// MI355X design.  The output is a receiver-major CSR graph that the model
// kernels consume directly, plus the public [2, max_pairs] pair list:
//   1. candidates: with the cell list (periodic boxes by default), atoms are
//      binned into cells of side >= cutoff (counting sort: atomic histogram,
//      device scan, scatter) and each atom sweeps its 27 stencil cells; with the
//      brute force (isolated systems by default, periodic boxes on request) each
//      atom binary-searches its system's atom range in the sorted batch vector
//      and sweeps all of it (no system count or offsets are ever needed on the
//      host).  A shared cell list with a batch test, as in the paper, lets one
//      launch serve any number of systems;
//   2. one wavefront per atom counts its neighbours (full and j > i), two device
//      scans turn the counts into CSR row offsets and pair offsets; the pair
//      budget is checked on the device (no host round trip);
//   3. the rows are written, sorted by neighbour index, and every directed edge
//      gets the id of its unordered pair (binary search in the partner's row).
// With the cell list the atoms are renumbered in cell order (counting sort, each
// cell's atoms by original index), so that spatial neighbours are close in
// index; the model kernels work in that order and map results back.  The
// wavefront of an atom sweeps its candidates as one flattened list; ballots
// place the neighbours, already sorted.  Pair writes use scanned offsets instead
// of one global atomic counter per pair.  The cutoff decision is an FP64
// predicate with contraction disabled.
#include "tn_internal.h"
#include "tn_device.h"

#include <cmath>

namespace tn {

// ------------------------------------------------------------------ fills
__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u8_zero(uint8_t *p, size_t n) {
  const size_t n4 = n / 4;
  uint32_t *q = reinterpret_cast<uint32_t *>(p);
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x) q[i] = 0u;
  if (blockIdx.x == 0 && threadIdx.x < (n & 3)) p[n4 * 4 + threadIdx.x] = 0;
}

static unsigned fill_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  return (unsigned)g;
}

int fill_i32(hipStream_t s, int32_t *p, int64_t n, int32_t v) {
  if (n <= 0) return TN_OK;
  hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
  TN_LAUNCH_CHECK();
  return TN_OK;
}

int fill_bytes_zero(hipStream_t s, void *p, size_t bytes) {
  if (bytes == 0) return TN_OK;
  hipLaunchKernelGGL(k_fill_u8_zero, dim3(fill_grid((int64_t)(bytes / 4 + 1))), dim3(256), 0, s,
                     static_cast<uint8_t *>(p), bytes);
  TN_LAUNCH_CHECK();
  return TN_OK;
}

// ------------------------------------------------------------------ exclusive scan (int32)
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

size_t scan_tmp_count(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 1; }

__device__ inline int32_t block_exclusive_scan(int32_t v, int32_t *lds, int32_t *total) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    int32_t add = (t >= off) ? lds[t - off] : 0;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  int32_t incl = lds[t];
  if (total) *total = lds[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tile(int32_t *data, int64_t n, int32_t *block_sums) {
  __shared__ int32_t lds[kScanThreads];
  __shared__ int32_t tot;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < n) ? data[base + k] : 0;
    sum += v[k];
  }
  int32_t run = block_exclusive_scan(sum, lds, &tot);
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) data[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// One block scans the block sums (any count, chunked with a carry), writes the
// grand total to data[n] and *total_out.
__global__ void __launch_bounds__(kScanThreads) k_scan_sums(int32_t *block_sums, int64_t nblk, int32_t *data,
                                                            int64_t n, int64_t *total_out) {
  __shared__ int32_t lds[kScanThreads];
  __shared__ int32_t tot;
  int32_t carry = 0;
  for (int64_t b0 = 0; b0 < nblk; b0 += kScanThreads) {
    const int64_t b = b0 + threadIdx.x;
    int32_t v = (b < nblk) ? block_sums[b] : 0;
    int32_t ex = block_exclusive_scan(v, lds, &tot);
    if (b < nblk) block_sums[b] = ex + carry;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    data[n] = carry;
    if (total_out) *total_out = (int64_t)carry;
  }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_add(int32_t *data, int64_t n, const int32_t *block_sums) {
  const int32_t add = block_sums[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * kScanItems;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) data[base + k] += add;
}

// Single-workgroup scans for short arrays (n <= kSmallScan): one launch instead of three.
constexpr int kSmallThreads = 1024, kSmallItems = 8, kSmallScan = kSmallThreads * kSmallItems;

__device__ int32_t small_scan_inplace(int32_t *data, int64_t n, int32_t *lds) {
  const int t = threadIdx.x;
  const int64_t base = (int64_t)t * kSmallItems;
  int32_t v[kSmallItems];
  int32_t sum = 0;
#pragma unroll
  for (int k = 0; k < kSmallItems; ++k) {
    v[k] = (base + k < n) ? data[base + k] : 0;
    sum += v[k];
  }
  lds[t] = sum;
  __syncthreads();
  for (int off = 1; off < kSmallThreads; off <<= 1) {
    const int32_t add = (t >= off) ? lds[t - off] : 0;
    __syncthreads();
    lds[t] += add;
    __syncthreads();
  }
  int32_t run = lds[t] - sum;
  const int32_t total = lds[kSmallThreads - 1];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kSmallItems; ++k) {
    if (base + k < n) data[base + k] = run;
    run += v[k];
  }
  if (t == 0) data[n] = total;
  return total;
}

__global__ void __launch_bounds__(kSmallThreads) k_scan_small(int32_t *data, int64_t n) {
  __shared__ int32_t lds[kSmallThreads];
  small_scan_inplace(data, n, lds);
}

// Both neighbour scans (full degree and upper pairs) and the pair total in one launch.
__global__ void __launch_bounds__(kSmallThreads) k_scan_nbr_small(int32_t *deg, int32_t *nup, int64_t n,
                                                                  int64_t *count64, int64_t max_pairs,
                                                                  int64_t *n_pairs, int32_t *status) {
  __shared__ int32_t lds[kSmallThreads];
  const int32_t full = small_scan_inplace(deg, n, lds);
  const int32_t up = small_scan_inplace(nup, n, lds);
  if (threadIdx.x == 0) {
    count64[0] = up;
    count64[1] = full;
    *n_pairs = up;
    if (up > max_pairs) set_status(status, TN_STATUS_OVERFLOW);
  }
}

// In-place exclusive scan of data[0..n); data[n] receives the total (data must hold n+1).
int exclusive_scan_i32(hipStream_t s, int32_t *data, int64_t n, int32_t *block_tmp, int64_t *total_out) {
  if (n <= kSmallScan && !total_out) {
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(kSmallThreads), 0, s, data, n);
    TN_LAUNCH_CHECK();
    return TN_OK;
  }
  const int64_t nblk = (n + kScanTile - 1) / kScanTile;
  if (nblk > 0) {
    hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)nblk), dim3(kScanThreads), 0, s, data, n, block_tmp);
    TN_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, block_tmp, nblk, data, n, total_out);
  TN_LAUNCH_CHECK();
  if (nblk > 0) {
    hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nblk), dim3(kScanThreads), 0, s, data, n, block_tmp);
    TN_LAUNCH_CHECK();
  }
  return TN_OK;
}

// ------------------------------------------------------------------ geometry of the box
int box_info(const double *box, double cutoff, BoxInfo *bi) {
  *bi = BoxInfo{};
  if (!(cutoff > 0.0) || !std::isfinite(cutoff)) return TN_E_ARG;
  if (!box) return TN_OK;
  for (int e = 0; e < 9; ++e)
    if (!std::isfinite(box[e])) return TN_E_ARG;
  // rows a, b, c, lower triangular (a along x, b in the xy plane)
  if (box[1] != 0.0 || box[2] != 0.0 || box[5] != 0.0) return TN_E_ARG;
  Lattice &L = bi->lat;
  L.periodic = 1;
  L.ax = box[0];
  L.bx = box[3];
  L.by = box[4];
  L.cx = box[6];
  L.cy = box[7];
  L.cz = box[8];
  if (!(L.ax > 0.0 && L.by > 0.0 && L.cz > 0.0)) return TN_E_ARG;
  // reduced form, which makes the sequential minimum image the nearest image
  if (std::fabs(L.bx) > 0.5 * L.ax || std::fabs(L.cx) > 0.5 * L.ax || std::fabs(L.cy) > 0.5 * L.by) return TN_E_ARG;
  bi->periodic = 1;
  bi->cells = 1;
  bi->tri = (L.bx != 0.0 || L.cx != 0.0 || L.cy != 0.0);
  bi->len[0] = L.ax;
  bi->len[1] = L.by;
  bi->len[2] = L.cz;
  // cell heights (distances between opposite faces) = 1 / |columns of H^-1|
  double h[3] = {L.ax, L.by, L.cz};
  if (bi->tri) {
    const double c0[3] = {1.0 / L.ax, -L.bx / (L.ax * L.by), (L.bx * L.cy - L.by * L.cx) / (L.ax * L.by * L.cz)};
    const double c1[2] = {1.0 / L.by, -L.cy / (L.by * L.cz)};
    h[0] = 1.0 / std::sqrt(c0[0] * c0[0] + c0[1] * c0[1] + c0[2] * c0[2]);
    h[1] = 1.0 / std::sqrt(c1[0] * c1[0] + c1[1] * c1[1]);
  }
  for (int a = 0; a < 3; ++a) {
    if (h[a] < 2.0 * cutoff) return TN_E_BOX;
    // cells at least as high as the cutoff with a relative margin: rounding in the binning
    // can then never put two atoms closer than the cutoff two cells apart (along each
    // fractional axis two such atoms differ by at most one cell)
    int nc = (int)std::floor(h[a] / (cutoff * (1.0 + 1e-6)));
    if (nc < 1) nc = 1;
    if (nc > 512) nc = 512;
    bi->nc[a] = nc;
    bi->side[a] = bi->len[a] / nc;
  }
  return TN_OK;
}

// Cells are numbered brick by brick: 4 x 4 x 4 cells per brick, bricks in row-major order
// (z fastest) and the cells of a brick likewise.  A run of consecutive atoms (cell order) is
// then a compact block of space, whose neighbours' rows, gathered by the kernels that follow,
// span fewer distinct atoms than a long pencil of cells would.  The index space is padded to
// whole bricks; the padding cells stay empty.
constexpr int kBrick = 4;
__host__ __device__ inline int64_t cell_space(const int nc[3]) {
  int64_t c = kBrick * kBrick * kBrick;
  for (int a = 0; a < 3; ++a) c *= (nc[a] + kBrick - 1) / kBrick;
  return c;
}
__host__ __device__ inline int cell_linear(int cx, int cy, int cz, const int nc[3]) {
  const int nby = (nc[1] + kBrick - 1) / kBrick, nbz = (nc[2] + kBrick - 1) / kBrick;
  const int brick = ((cx / kBrick) * nby + cy / kBrick) * nbz + cz / kBrick;
  return (brick * kBrick + cx % kBrick) * kBrick * kBrick + (cy % kBrick) * kBrick + cz % kBrick;
}
__host__ __device__ inline void cell_coords(int c, const int nc[3], int &cx, int &cy, int &cz) {
  const int nby = (nc[1] + kBrick - 1) / kBrick, nbz = (nc[2] + kBrick - 1) / kBrick;
  const int brick = c / (kBrick * kBrick * kBrick), local = c % (kBrick * kBrick * kBrick);
  const int bz = brick % nbz, by = (brick / nbz) % nby, bx = brick / (nbz * nby);
  cx = bx * kBrick + local / (kBrick * kBrick);
  cy = by * kBrick + (local / kBrick) % kBrick;
  cz = bz * kBrick + local % kBrick;
}

void plan_neighbors(WsPlan &p, int64_t n, int64_t max_pairs, const BoxInfo &bi, NbrWs *w) {
  const int64_t ncell = bi.cells ? cell_space(bi.nc) : 0;
  if (bi.cells) {
    w->cell_of = p.take<int32_t>(n);
    w->cell_count = p.take<int32_t>(ncell + 1);
    w->cell_fill = p.take<int32_t>(ncell);
    w->cell_atoms = p.take<int32_t>(n);
    w->cell_start = w->cell_count;   // scanned in place
  }
  if (bi.cells) {
    w->spos = p.take<double>(3 * n);
    w->sz = p.take<int32_t>(n);
    w->sbatch = p.take<int32_t>(n);
    w->scell = p.take<int32_t>(n);
  }
  w->ipairs = p.take<int32_t>(2 * max_pairs);
  w->deg = p.take<int32_t>(n + 1);
  w->nup = p.take<int32_t>(n + 1);
  w->nbr = p.take<int32_t>(2 * max_pairs);
  w->pid = p.take<int32_t>(2 * max_pairs);
  w->scan_tmp = p.take<int32_t>(scan_tmp_count(n > ncell ? n : ncell));
  w->count64 = p.take<int64_t>(4);
}

struct BoxDev {
  int periodic, cells, tri;
  Lattice lat;
  double len[3];
  double side[3];
  int nc[3];
};

static BoxDev to_dev(const BoxInfo &bi) {
  BoxDev b;
  b.periodic = bi.periodic;
  b.cells = bi.cells;
  b.tri = bi.tri;
  b.lat = bi.lat;
  for (int a = 0; a < 3; ++a) {
    b.len[a] = bi.len[a];
    b.side[a] = bi.side[a];
    b.nc[a] = bi.nc[a];
  }
  return b;
}

// The pinned FP64 cutoff predicate (no contraction into FMA).
__device__ inline bool pair_within(double xi, double yi, double zi, double xj, double yj, double zj,
                                         const BoxDev &b, double rc2) {
#pragma clang fp contract(off)
  double dx = xj - xi, dy = yj - yi, dz = zj - zi;
  min_image(b.lat, dx, dy, dz);
  double xx = dx * dx;
  double yy = dy * dy;
  double zz = dz * dz;
  double d2 = (xx + yy) + zz;
  return d2 < rc2;
}

template <class T>
__device__ inline void load_pos(const T *pos, int64_t i, double &x, double &y, double &z) {
  x = (double)pos[3 * i];
  y = (double)pos[3 * i + 1];
  z = (double)pos[3 * i + 2];
}

__device__ inline int cell_coord(double x, double L, double side, int nc) {
  double w = x - L * floor(x / L);
  int c = (int)floor(w / side);
  if (!(c >= 0)) c = 0;       // also catches NaN
  if (c > nc - 1) c = nc - 1;
  return c;
}

// The same from a fractional coordinate (triclinic cells).
__device__ inline int frac_cell(double s, int nc) {
  const double w = s - floor(s);
  int c = (int)floor(w * nc);
  if (!(c >= 0)) c = 0;
  if (c > nc - 1) c = nc - 1;
  return c;
}

template <class T>
__global__ void k_cell_assign(const T *pos, int64_t n, BoxDev b, int32_t *cell_of, int32_t *cell_count,
                              int32_t *status) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double x, y, z;
  load_pos(pos, i, x, y, z);
  if (!isfinite(x) || !isfinite(y) || !isfinite(z)) set_status(status, TN_STATUS_NONFINITE);
  int cx, cy, cz;
  if (b.tri) {
    double s0, s1, s2;
    fractional(b.lat, x, y, z, s0, s1, s2);
    cx = frac_cell(s0, b.nc[0]);
    cy = frac_cell(s1, b.nc[1]);
    cz = frac_cell(s2, b.nc[2]);
  } else {
    cx = cell_coord(x, b.len[0], b.side[0], b.nc[0]);
    cy = cell_coord(y, b.len[1], b.side[1], b.nc[1]);
    cz = cell_coord(z, b.len[2], b.side[2], b.nc[2]);
  }
  const int c = cell_linear(cx, cy, cz, b.nc);
  cell_of[i] = c;
  atomicAdd(&cell_count[c], 1);
}

__global__ void k_cell_scatter(int64_t n, const int32_t *cell_of, const int32_t *cell_start, int32_t *cell_fill,
                               int32_t *cell_atoms) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int c = cell_of[i];
  const int slot = atomicAdd(&cell_fill[c], 1);
  cell_atoms[cell_start[c] + slot] = (int32_t)i;
}

// Range of atoms sharing batch value bv (lower/upper bound in a sorted vector).
__device__ inline void system_range(const int32_t *batch, int64_t n, int32_t bv, int64_t &lo, int64_t &hi) {
  int64_t a = 0, e = n;
  while (a < e) {
    int64_t m = (a + e) >> 1;
    if (batch[m] < bv) a = m + 1; else e = m;
  }
  lo = a;
  e = n;
  while (a < e) {
    int64_t m = (a + e) >> 1;
    if (batch[m] <= bv) a = m + 1; else e = m;
  }
  hi = a;
}

// Input checks in one pass: batch sorted (systems contiguous) and in [0, n_systems) when
// n_systems > 0, z in [0, max_z) when z is given, finite positions when check_pos.  An
// unsorted batch sets TN_STATUS_BATCH, which the candidate sweep reads as "search all atoms".
template <class T>
__global__ void k_validate(const T *pos, const int32_t *z, const int32_t *batch, int64_t n, int64_t n_systems,
                           int max_z, int check_pos, int32_t *status, int32_t *zero_a, int64_t na, int32_t *zero_b,
                           int64_t nb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  // also clears the cell list's counters for the kernels that follow (saves two launches)
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = i; k < na; k += stride) zero_a[k] = 0;
  for (int64_t k = i; k < nb; k += stride) zero_b[k] = 0;
  if (i >= n) return;
  const int32_t b = batch[i];
  if (i > 0 && b < batch[i - 1]) set_status(status, TN_STATUS_BATCH);
  if (n_systems > 0 && (b < 0 || b >= n_systems)) set_status(status, TN_STATUS_BATCH);
  if (z && max_z > 0 && (z[i] < 0 || z[i] >= max_z)) set_status(status, TN_STATUS_Z);
  if (check_pos) {
    double x, y, zz;
    load_pos(pos, i, x, y, zz);
    if (!isfinite(x) || !isfinite(y) || !isfinite(zz)) set_status(status, TN_STATUS_NONFINITE);
  }
}

// Deterministic order inside each cell: the cell's atoms sorted by original index.  One
// wavefront per cell stages the (distinct) indices in LDS and gives every element its rank,
// the number of smaller indices in the cell; cells with more than kSortCap atoms (not met at
// physical densities) fall back to an insertion sort by one lane.
constexpr int kSortCap = 1024;

__global__ void __launch_bounds__(256) k_cell_sort(int64_t ncell, const int32_t *cell_start, int32_t *cell_atoms) {
  __shared__ int32_t buf[4][kSortCap];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * 4 + w;
  if (c >= ncell) return;
  const int32_t a = cell_start[c], e = cell_start[c + 1], n = e - a;
  if (n <= 1) return;
  if (n > kSortCap) {
    if (lane == 0) {
      for (int32_t k = a + 1; k < e; ++k) {
        const int32_t v = cell_atoms[k];
        int32_t q = k - 1;
        while (q >= a && cell_atoms[q] > v) {
          cell_atoms[q + 1] = cell_atoms[q];
          --q;
        }
        cell_atoms[q + 1] = v;
      }
    }
    return;
  }
  int32_t *b = buf[w];
  for (int k = lane; k < n; k += 64) b[k] = cell_atoms[a + k];
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  for (int k = lane; k < n; k += 64) {
    const int32_t v = b[k];
    int r = 0;
    for (int m = 0; m < n; ++m) r += b[m] < v;
    cell_atoms[a + r] = v;
  }
}

// Cell-ordered copies of the per-atom inputs (s = cell-ordered index, perm[s] = original index).
template <class T>
__global__ void k_permute(int64_t n, const int32_t *perm, const T *pos, const int32_t *z, const int32_t *batch,
                          const int32_t *cell_of, T *spos, int32_t *sz, int32_t *sbatch, int32_t *scell) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int64_t o = perm[s];
  spos[3 * s] = pos[3 * o];
  spos[3 * s + 1] = pos[3 * o + 1];
  spos[3 * s + 2] = pos[3 * o + 2];
  if (z) sz[s] = z[o];
  sbatch[s] = batch[o];
  scell[s] = cell_of[o];
}

// One wavefront per atom visits its candidates in ascending index order: the distinct
// stencil cells in ascending linear order (cell list) or the atom's system range (brute
// force), flattened into one list that the 64 lanes sweep together.
// f(pred, j) is called by every lane with its candidate; neighbours come out sorted.
constexpr int kNbrBlock = 256;

template <class T, class Fn>
__device__ inline void wave_candidates(int64_t s, const T *pos, const int32_t *batch, int64_t n, const BoxDev &b,
                                       double rc2, const int32_t *scell, const int32_t *cell_start,
                                       const int32_t *status, Fn &&f) {
  const int lane = threadIdx.x & 63;
  double xi, yi, zi;
  load_pos(pos, s, xi, yi, zi);
  const int32_t bs = batch[s];
  if (b.cells) {
    int cx, cy, cz;
    cell_coords(scell[s], b.nc, cx, cy, cz);
    // distinct wrapped coordinates per axis, ascending (1 cell -> 1 value, 2 -> 2, else 3)
    int xs[3], ys[3], zs[3], nx, ny, nz;
    auto axis = [](int cc, int nc, int out[3], int &cnt) {
      if (nc == 1) { out[0] = 0; cnt = 1; return; }
      if (nc == 2) { out[0] = 0; out[1] = 1; cnt = 2; return; }
      int v0 = (cc + nc - 1) % nc, v1 = cc, v2 = (cc + 1) % nc;
      // sort three values
      if (v0 > v1) { int t = v0; v0 = v1; v1 = t; }
      if (v1 > v2) { int t = v1; v1 = v2; v2 = t; }
      if (v0 > v1) { int t = v0; v0 = v1; v1 = t; }
      out[0] = v0; out[1] = v1; out[2] = v2; cnt = 3;
    };
    axis(cx, b.nc[0], xs, nx);
    axis(cy, b.nc[1], ys, ny);
    axis(cz, b.nc[2], zs, nz);
    const int ncells = nx * ny * nz;
    int cc = 0x7fffffff;
    if (lane < ncells) {
      const int ix = lane / (ny * nz), iy = (lane / nz) % ny, iz = lane % nz;
      cc = cell_linear(xs[ix], ys[iy], zs[iz], b.nc);
    }
    // the stencil cells (distinct) in ascending linear order: lane r takes the cell of rank r,
    // so the candidates, and with them the neighbour lists, come out sorted
    int rank = 0;
    for (int k = 0; k < 27; ++k) {
      const int ck = __shfl(cc, k, 64);
      if (k < ncells && ck < cc) ++rank;
    }
    int src = 0;
    for (int k = 0; k < 27; ++k) {
      const int rk = __shfl(rank, k, 64);
      if (k < ncells && rk == lane) src = k;
    }
    cc = __shfl(cc, src, 64);
    int cs = 0, cnt = 0;
    if (lane < ncells) {
      cs = cell_start[cc];
      cnt = cell_start[cc + 1] - cs;
    }
    int incl = cnt;
#pragma unroll
    for (int off = 1; off < 32; off <<= 1) {
      const int up = __shfl_up(incl, off, 64);
      if (lane >= off) incl += up;
    }
    const int excl = incl - cnt;
    const int total = __shfl(incl, ncells - 1, 64);
    for (int q0 = 0; q0 < total; q0 += 64) {
      const int q = q0 + lane;
      // slot k with excl[k] <= q (largest such k among the ncells slots)
      int lo = 0;
#pragma unroll
      for (int step = 16; step > 0; step >>= 1) {
        const int mid = lo + step;
        const int e_mid = __shfl(excl, mid < ncells ? mid : ncells - 1, 64);
        if (mid < ncells && e_mid <= q) lo = mid;
      }
      const int base = __shfl(cs, lo, 64), ex = __shfl(excl, lo, 64);
      bool pred = false;
      int32_t j = 0;
      if (q < total) {
        j = base + (q - ex);
        if (j != s && batch[j] == bs) {
          double xj, yj, zj;
          load_pos(pos, j, xj, yj, zj);
          pred = pair_within(xi, yi, zi, xj, yj, zj, b, rc2);
        }
      }
      f(pred, j);
    }
  } else {
    int64_t lo = 0, hi = n;
    if (!(*status & TN_STATUS_BATCH)) system_range(batch, n, bs, lo, hi);
    for (int64_t q0 = lo; q0 < hi; q0 += 64) {
      const int64_t j = q0 + lane;
      bool pred = false;
      if (j < hi && j != s && batch[j] == bs) {
        double xj, yj, zj;
        load_pos(pos, j, xj, yj, zj);
        pred = pair_within(xi, yi, zi, xj, yj, zj, b, rc2);
      }
      f(pred, (int32_t)j);
    }
  }
}

template <class T>
__global__ void __launch_bounds__(kNbrBlock) k_nbr_count(const T *pos, const int32_t *batch, int64_t n, BoxDev b,
                                                         double rc2, const int32_t *scell, const int32_t *cell_start,
                                                         const int32_t *status, int32_t *deg, int32_t *nup) {
  const int64_t s = (blockIdx.x * (int64_t)kNbrBlock + threadIdx.x) >> 6;
  if (s >= n) return;
  int32_t full = 0, upper = 0;
  wave_candidates(s, pos, batch, n, b, rc2, scell, cell_start, status, [&](bool pred, int32_t j) {
    const uint64_t m = __ballot(pred);
    const uint64_t mu = __ballot(pred && j > s);
    full += __popcll(m);
    upper += __popcll(mu);
  });
  if ((threadIdx.x & 63) == 0) {
    deg[s] = full;
    nup[s] = upper;
  }
}

template <class T>
__global__ void __launch_bounds__(kNbrBlock) k_nbr_write(const T *pos, const int32_t *batch, int64_t n, BoxDev b,
                                                         double rc2, const int32_t *scell, const int32_t *cell_start,
                                                         const int32_t *status, const int32_t *rowptr,
                                                         const int64_t *count64, int64_t max_pairs, int32_t *nbr) {
  const int64_t s = (blockIdx.x * (int64_t)kNbrBlock + threadIdx.x) >> 6;
  if (s >= n || count64[0] > max_pairs) return;
  const int lane = threadIdx.x & 63;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  int32_t e = rowptr[s];
  wave_candidates(s, pos, batch, n, b, rc2, scell, cell_start, status, [&](bool pred, int32_t j) {
    const uint64_t m = __ballot(pred);
    if (pred) nbr[e + __popcll(m & below)] = j;
    e += __popcll(m);
  });
}

__global__ void k_nbr_total(const int64_t *count64, int64_t max_pairs, int64_t *n_pairs, int32_t *status) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    const int64_t P = count64[0];
    *n_pairs = P;
    if (P > max_pairs) set_status(status, TN_STATUS_OVERFLOW);
  }
}

// Pair id of every directed edge (rows are sorted by neighbour); the internal pair list
// gets (s, t) for t > s, so it is ordered by (s, t).  One wavefront per atom, one lane per
// edge of its row; a lower edge finds its pair in the partner's row by binary search.
__global__ void __launch_bounds__(kNbrBlock) k_pair_ids(int64_t n, const int32_t *rowptr, const int32_t *pbase,
                                                        const int32_t *nbr, const int64_t *count64, int64_t max_pairs,
                                                        int32_t *pid, int32_t *pairs) {
  const int64_t i = (blockIdx.x * (int64_t)kNbrBlock + threadIdx.x) >> 6;
  if (i >= n || count64[0] > max_pairs) return;
  const int lane = threadIdx.x & 63;
  const int32_t a = rowptr[i], e = rowptr[i + 1];
  const int32_t nlow_i = (e - a) - (pbase[i + 1] - pbase[i]);
  const int32_t P = (int32_t)count64[0];
  for (int32_t k = a + lane; k < e; k += 64) {
    const int32_t j = nbr[k];
    int32_t p;
    if (j > i) {
      p = pbase[i] + (k - a - nlow_i);
      pairs[p] = (int32_t)i;
      pairs[max_pairs + p] = j;
    } else {
      const int32_t aj = rowptr[j], ej = rowptr[j + 1];
      int32_t lo = aj, hi = ej;
      while (lo < hi) {
        const int32_t m = (lo + hi) >> 1;
        if (nbr[m] < (int32_t)i) lo = m + 1; else hi = m;
      }
      const int32_t nlow_j = (ej - aj) - (pbase[j + 1] - pbase[j]);
      p = pbase[j] + (lo - aj - nlow_j);
      // the relation is symmetric, so i is always found; clamp defensively anyway
      if (p < 0) p = 0;
      if (p > P - 1) p = P - 1;
    }
    pid[k] = p;
  }
}

// Public pair list in original atom indices, (min, max) per pair; padding -1.
__global__ void k_pairs_public(const int64_t *count64, int64_t max_pairs, const int32_t *perm, const int32_t *ipairs,
                               int32_t *pairs) {
  const int64_t P = count64[0];
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < max_pairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    int32_t a = -1, c = -1;
    if (p < P && P <= max_pairs) {
      a = ipairs[p];
      c = ipairs[max_pairs + p];
      if (perm) {
        a = perm[a];
        c = perm[c];
      }
      if (a > c) {
        const int32_t t = a;
        a = c;
        c = t;
      }
    }
    pairs[p] = a;
    pairs[max_pairs + p] = c;
  }
}

template <class T>
int build_neighbors(hipStream_t s, int64_t n, const T *pos, const int32_t *z, const int32_t *batch,
                    const BoxInfo &bi, double cutoff, int64_t max_pairs, int32_t *public_pairs, int64_t *n_pairs,
                    int32_t *status, const NbrWs &w, NbrGraph<T> *graph, int64_t n_systems, int max_z) {
  const BoxDev b = to_dev(bi);
  const double rc2 = cutoff * cutoff;
  const int blk = 128;
  const unsigned g = grid_for(n > 0 ? n : 1, blk);
  const unsigned gw = grid_for(n > 0 ? n * 64 : 64, kNbrBlock);   // one wavefront per atom
  int rc;
  NbrGraph<T> out;
  out.pos = pos;
  out.z = z;
  out.batch = batch;
  out.perm = nullptr;
  const int64_t ncell = bi.cells ? cell_space(bi.nc) : 0;
  if (n > 0) {   // the cell binning checks the positions itself
    hipLaunchKernelGGL(k_validate<T>, dim3(g), dim3(blk), 0, s, pos, z, batch, n, n_systems, max_z,
                       bi.cells ? 0 : 1, status, w.cell_count, bi.cells ? ncell + 1 : 0, w.cell_fill, ncell);
    TN_LAUNCH_CHECK();
  } else if (bi.cells) {
    if ((rc = fill_i32(s, w.cell_count, ncell + 1, 0))) return rc;
    if ((rc = fill_i32(s, w.cell_fill, ncell, 0))) return rc;
  }
  if (bi.cells) {
    if (n > 0) {
      hipLaunchKernelGGL(k_cell_assign<T>, dim3(g), dim3(blk), 0, s, pos, n, b, w.cell_of, w.cell_count, status);
      TN_LAUNCH_CHECK();
    }
    if ((rc = exclusive_scan_i32(s, w.cell_count, ncell, w.scan_tmp, nullptr))) return rc;
    if (n > 0) {
      hipLaunchKernelGGL(k_cell_scatter, dim3(g), dim3(blk), 0, s, n, w.cell_of, w.cell_start, w.cell_fill,
                         w.cell_atoms);
      TN_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_cell_sort, dim3((unsigned)((ncell + 3) / 4)), dim3(256), 0, s, ncell, w.cell_start,
                         w.cell_atoms);
      TN_LAUNCH_CHECK();
      T *spos = static_cast<T *>(w.spos);
      hipLaunchKernelGGL(k_permute<T>, dim3(g), dim3(blk), 0, s, n, w.cell_atoms, pos, z, batch, w.cell_of, spos,
                         w.sz, w.sbatch, w.scell);
      TN_LAUNCH_CHECK();
      out.pos = spos;
      out.z = z ? w.sz : nullptr;
      out.batch = w.sbatch;
      out.perm = w.cell_atoms;
    }
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_nbr_count<T>, dim3(gw), dim3(kNbrBlock), 0, s, out.pos, out.batch, n, b, rc2, w.scell,
                       w.cell_start, status, w.deg, w.nup);
    TN_LAUNCH_CHECK();
  }
  if (n <= kSmallScan) {
    hipLaunchKernelGGL(k_scan_nbr_small, dim3(1), dim3(kSmallThreads), 0, s, w.deg, w.nup, n, w.count64, max_pairs,
                       n_pairs, status);
    TN_LAUNCH_CHECK();
  } else {
    if ((rc = exclusive_scan_i32(s, w.deg, n, w.scan_tmp, w.count64 + 1))) return rc;
    if ((rc = exclusive_scan_i32(s, w.nup, n, w.scan_tmp, w.count64 + 0))) return rc;
    hipLaunchKernelGGL(k_nbr_total, dim3(1), dim3(64), 0, s, w.count64, max_pairs, n_pairs, status);
    TN_LAUNCH_CHECK();
  }
  if (n > 0) {
    hipLaunchKernelGGL(k_nbr_write<T>, dim3(gw), dim3(kNbrBlock), 0, s, out.pos, out.batch, n, b, rc2, w.scell,
                       w.cell_start, status, w.deg, w.count64, max_pairs, w.nbr);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_pair_ids, dim3(gw), dim3(kNbrBlock), 0, s, n, w.deg, w.nup, w.nbr, w.count64, max_pairs,
                       w.pid, w.ipairs);
    TN_LAUNCH_CHECK();
  }
  if (public_pairs && max_pairs > 0) {
    hipLaunchKernelGGL(k_pairs_public, dim3(fill_grid(max_pairs)), dim3(256), 0, s, w.count64, max_pairs, out.perm,
                       w.ipairs, public_pairs);
    TN_LAUNCH_CHECK();
  }
  out.rowptr = w.deg;
  out.nbr = w.nbr;
  out.pid = w.pid;
  out.pairs = w.ipairs;
  if (graph) *graph = out;
  return TN_OK;
}

template int build_neighbors<float>(hipStream_t, int64_t, const float *, const int32_t *, const int32_t *,
                                    const BoxInfo &, double, int64_t, int32_t *, int64_t *, int32_t *, const NbrWs &,
                                    NbrGraph<float> *, int64_t, int);
template int build_neighbors<double>(hipStream_t, int64_t, const double *, const int32_t *, const int32_t *,
                                     const BoxInfo &, double, int64_t, int32_t *, int64_t *, int32_t *,
                                     const NbrWs &, NbrGraph<double> *, int64_t, int);

}  // namespace tn
