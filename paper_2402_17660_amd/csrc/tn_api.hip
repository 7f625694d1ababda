// C ABI entry points: weight-blob parsing, device weight upload, workspace
// queries and dispatch to the neighbour search and the model paths.
#include "tn_internal.h"
#include "tn_device.h"

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>

using namespace tn;

namespace {

constexpr size_t kHeaderBytes = 56;

struct TensorSpec {
  size_t *off;
  size_t count;
};

// The tensor order of the weight blob (generator order), with element counts.
std::vector<TensorSpec> blob_order(tn_model *m) {
  const size_t F = m->F, K = m->K, Z = m->max_z;
  WeightOff &o = m->off;
  std::vector<TensorSpec> t = {
      {&o.E, Z * F},      {&o.Wz, F * 2 * F}, {&o.bz, F},         {&o.W0, 3 * F * K}, {&o.b0, 3 * F},
      {&o.ln_g, F},       {&o.ln_b, F},       {&o.W1, 2 * F * F}, {&o.b1, 2 * F},     {&o.W2, 3 * F * 2 * F},
      {&o.b2, 3 * F},     {&o.Wmix[0], F * F}, {&o.Wmix[1], F * F}, {&o.Wmix[2], F * F}};
  o.layer.resize(m->L);
  for (int l = 0; l < m->L; ++l) {
    LayerOff &lo = o.layer[l];
    std::vector<TensorSpec> lt = {{&lo.Wa, F * K},         {&lo.ba, F},       {&lo.Wb, 2 * F * F},
                                  {&lo.bb, 2 * F},         {&lo.Wc, 3 * F * 2 * F}, {&lo.bc, 3 * F},
                                  {&lo.W1[0], F * F},      {&lo.W1[1], F * F}, {&lo.W1[2], F * F},
                                  {&lo.W2[0], F * F},      {&lo.W2[1], F * F}, {&lo.W2[2], F * F}};
    t.insert(t.end(), lt.begin(), lt.end());
  }
  std::vector<TensorSpec> ot = {{&o.oln_g, 3 * F}, {&o.oln_b, 3 * F}, {&o.Wo, F * 3 * F}, {&o.bo, F},
                                {&o.Wh, (F / 2) * F}, {&o.bh, F / 2}, {&o.wout, F / 2},  {&o.bout, 1}};
  t.insert(t.end(), ot.begin(), ot.end());
  return t;
}

uint32_t rd_u32(const unsigned char *p) {
  uint32_t v;
  std::memcpy(&v, p, 4);
  return v;
}
double rd_f64(const unsigned char *p) {
  double v;
  std::memcpy(&v, p, 8);
  return v;
}

int parse_blob(const void *blob, size_t bytes, tn_model *m, std::vector<double> &packed) {
  const unsigned char *b = static_cast<const unsigned char *>(blob);
  if (bytes < kHeaderBytes || std::memcmp(b, "TNETBLOB", 8) != 0) return TN_E_BLOB;
  const uint32_t version = rd_u32(b + 8);
  m->F = (int)rd_u32(b + 12);
  m->K = (int)rd_u32(b + 16);
  m->L = (int)rd_u32(b + 20);
  m->max_z = (int)rd_u32(b + 24);
  const uint32_t act = rd_u32(b + 28);
  m->r_lo = rd_f64(b + 40);
  m->r_c = rd_f64(b + 48);
  if (version != 1 || act != 1) return TN_E_BLOB;
  if (m->F < 2 || m->F % 2 || m->F > 1024 || m->K < 2 || m->K > kMaxK || m->L < 0 || m->L > 16 || m->max_z < 1 ||
      m->max_z > 1024)
    return TN_E_BLOB;
  if (!(m->r_c > m->r_lo) || !(m->r_lo >= 0.0) || !std::isfinite(m->r_c)) return TN_E_BLOB;
  std::vector<TensorSpec> order = blob_order(m);
  size_t total = 0;
  for (auto &t : order) total += t.count;
  if (bytes != kHeaderBytes + 8 * total) return TN_E_BLOB;
  const size_t F = m->F, K = m->K, Z = m->max_z;
  // room for the derived tables: species tables, basis constants, aligned and transposed
  // copies of the per-pair weights (each start aligned to 64 elements)
  const size_t extra = 2 * Z * F + 2 * K + 2 * (3 * F * K) + (size_t)m->L * 2 * (F * K + 2 * F * F + 6 * F * F) +
                       (size_t)(m->L + 1) * 12 * F * F + 64 * (14 + 18 * (size_t)m->L);
  packed.assign(total + extra, 0.0);
  size_t off = 0;
  const unsigned char *src = b + kHeaderBytes;
  for (auto &t : order) {
    *t.off = off;
    std::memcpy(packed.data() + off, src, 8 * t.count);
    src += 8 * t.count;
    off += t.count;
  }
  for (double v : packed)
    if (!std::isfinite(v)) return TN_E_BLOB;
  WeightOff &o = m->off;
  // species tables: Z_ij = W_z [E_zi ; E_zj] + b_z = U[z_i] + V[z_j]
  auto grab = [&](size_t count) {
    off = (off + 63) / 64 * 64;
    const size_t at = off;
    off += count;
    return at;
  };
  o.U = grab(Z * F);
  o.V = grab(Z * F);
  o.mu = grab(K);
  o.beta = grab(K);
  // copies for the fused kernels: W0 [3F][K] as is and transposed; per layer Wa [F][K],
  // Wb [2F][F], Wc [3F][2F] as is and transposed; every mixing matrix [F][F] transposed (adjoint
  // mixing) and as is (forward mixing; the blob's own copy need not be 16-byte aligned)
  auto copy = [&](size_t src, size_t rows, size_t cols, bool transpose) {
    const size_t at = grab(rows * cols);
    for (size_t r = 0; r < rows; ++r)
      for (size_t c = 0; c < cols; ++c)
        packed[at + (transpose ? c * rows + r : r * cols + c)] = packed[src + r * cols + c];
    return at;
  };
  o.W0f = copy(o.W0, 3 * F, K, false);
  o.W0T = copy(o.W0, 3 * F, K, true);
  for (int q = 0; q < 3; ++q) {
    o.WmixT[q] = copy(o.Wmix[q], F, F, true);
    o.Wmixf[q] = copy(o.Wmix[q], F, F, false);
  }
  for (int l = 0; l < m->L; ++l) {
    LayerOff &lo = o.layer[l];
    lo.Waf = copy(lo.Wa, F, K, false);
    lo.WaT = copy(lo.Wa, F, K, true);
    lo.Wbf = copy(lo.Wb, 2 * F, F, false);
    lo.WbT = copy(lo.Wb, 2 * F, F, true);
    lo.Wcf = copy(lo.Wc, 3 * F, 2 * F, false);
    lo.WcT = copy(lo.Wc, 3 * F, 2 * F, true);
    for (int q = 0; q < 3; ++q) {
      lo.W1T[q] = copy(lo.W1[q], F, F, true);
      lo.W2T[q] = copy(lo.W2[q], F, F, true);
      lo.W1f[q] = copy(lo.W1[q], F, F, false);
      lo.W2f[q] = copy(lo.W2[q], F, F, false);
    }
  }
  o.total = off;
  if (o.total > packed.size()) return TN_E_BLOB;
  packed.resize(o.total);
  const double *E = packed.data() + o.E, *Wz = packed.data() + o.Wz, *bz = packed.data() + o.bz;
  for (size_t s = 0; s < Z; ++s)
    for (size_t f = 0; f < F; ++f) {
      double u = bz[f], v = 0.0;
      for (size_t g = 0; g < F; ++g) {
        u += Wz[f * 2 * F + g] * E[s * F + g];
        v += Wz[f * 2 * F + F + g] * E[s * F + g];
      }
      packed[o.U + s * F + f] = u;
      packed[o.V + s * F + f] = v;
    }
  // exp-normal basis constants (Sec. 2.4, rbf_type expnorm, not trainable)
  const double span = m->r_c - m->r_lo;
  const double start = std::exp(-span);
  m->alpha = 5.0 / span;
  for (size_t k = 0; k < K; ++k) {
    packed[o.mu + k] = start + (1.0 - start) * (double)k / (double)(K - 1);
    const double w = 2.0 / (double)K * (1.0 - start);
    packed[o.beta + k] = 1.0 / (w * w);
  }
  return TN_OK;
}

// ------------------------------------------------------------------ static scratch
// The library's own device scratch for tn_energy_forces_static: one array per GPU (each device
// holds its own copy of a __device__ variable), never allocated or freed by a call.  In host
// code `scratch` is only a host-side stand-in for the symbol; its device address on each GPU
// is looked up once with hipGetSymbolAddress and kept in g_scratch_ptr.
static __device__ __align__(256) unsigned char scratch[TN_STATIC_WS_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The address of `scratch` on `device` (which must be current); looked up on the first call
// per device.  Returns TN_OK, TN_E_ARG (device index out of range) or TN_E_HIP.
int scratch_on_device(int device, void **out) {
  if (device < 0 || device >= kMaxDevices) return TN_E_ARG;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      std::fprintf(stderr, "tensornet: hipGetSymbolAddress(scratch) on device %d failed: %s\n", device,
                   hipGetErrorString(e));
      return TN_E_HIP;
    }
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return TN_OK;
}

// ------------------------------------------------------------------ timing registry
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  std::string name;
  bool used = false;
};
std::mutex g_timing_mu;
bool g_timing_on = false;
std::vector<EventPair> g_events;

}  // namespace

namespace tn {

TimedScope::TimedScope(const char *name, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  if (!g_timing_on) return;
  int k = -1;
  for (size_t q = 0; q < g_events.size(); ++q)
    if (!g_events[q].used) { k = (int)q; break; }
  if (k < 0) {
    EventPair e;
    if (hipEventCreate(&e.a) != hipSuccess || hipEventCreate(&e.b) != hipSuccess) return;
    g_events.push_back(e);
    k = (int)g_events.size() - 1;
  }
  g_events[k].used = true;
  g_events[k].name = name;
  if (hipEventRecord(g_events[k].a, s) != hipSuccess) return;
  slot = k;
  stream = s;
}

TimedScope::~TimedScope() {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  (void)hipEventRecord(g_events[slot].b, stream);
}

bool timing_swap(bool on) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  const bool was = g_timing_on;
  g_timing_on = on;
  return was;
}

}  // namespace tn

extern "C" {

int tn_timing_enable(int on) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  g_timing_on = on != 0;
  return TN_OK;
}

int tn_timing_reset(void) {
  std::lock_guard<std::mutex> lk(g_timing_mu);
  for (auto &e : g_events) e.used = false;
  return TN_OK;
}

int tn_timing_read(const char *name, double *total_ms, int64_t *launches) {
  if (!name || !total_ms || !launches) return TN_E_ARG;
  std::lock_guard<std::mutex> lk(g_timing_mu);
  double tot = 0.0;
  int64_t cnt = 0;
  for (auto &e : g_events) {
    if (!e.used || e.name != name) continue;
    if (hipEventSynchronize(e.b) != hipSuccess) return TN_E_HIP;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e.a, e.b) != hipSuccess) return TN_E_HIP;
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
  return TN_OK;
}


int tn_pair_variant_count(int precision) {
  if (precision == TN_FP32) return pair_variant_count(false);
  if (precision == TN_BF16) return pair_variant_count(true);
  return 0;
}

int tn_model_set_pair_variant(tn_model *m, int precision, int forward, int reverse) {
  if (!m || (precision != TN_FP32 && precision != TN_BF16)) return TN_E_ARG;
  const int n = tn_pair_variant_count(precision);
  if (forward < -1 || forward >= n || reverse < -1 || reverse >= n) return TN_E_ARG;
  const int p = precision == TN_BF16 ? 1 : 0;
  m->pair_force[p][0] = forward;
  m->pair_force[p][1] = reverse;
  return TN_OK;
}

int tn_autotune(tn_model *m, void *stream, int64_t n_atoms, int64_t n_systems, const void *pos, const int32_t *z,
                const int32_t *batch, const double *box, int64_t max_pairs, int precision, double *energy,
                void *forces, int64_t *n_pairs, int32_t *status, void *ws, size_t ws_bytes, int reps,
                int32_t *chosen) {
  if (!m || (precision != TN_FP32 && precision != TN_BF16) || reps < 1 || reps > 1000) return TN_E_ARG;
  const int p = precision == TN_BF16 ? 1 : 0;
  const int nv = tn_pair_variant_count(precision);
  const int saved[2] = {m->pair_force[p][0], m->pair_force[p][1]};
  const bool was_timing = timing_swap(true);
  std::vector<double> tf(nv, 1e30), tb(nv, 1e30);
  int rc = TN_OK;
  for (int v = 0; v < nv && rc == TN_OK; ++v) {
    m->pair_force[p][0] = m->pair_force[p][1] = v;
    rc = tn_energy_forces(m, stream, n_atoms, n_systems, pos, z, batch, box, max_pairs, precision, TN_FUSED,
                          energy, forces, n_pairs, status, ws, ws_bytes);   // warm-up
    if (rc) break;
    tn_timing_reset();
    for (int r = 0; r < reps && rc == TN_OK; ++r)
      rc = tn_energy_forces(m, stream, n_atoms, n_systems, pos, z, batch, box, max_pairs, precision, TN_FUSED,
                            energy, forces, n_pairs, status, ws, ws_bytes);
    if (rc) break;
    double tot = 0.0;
    int64_t cnt = 0;
    if ((rc = tn_timing_read("edge_fwd", &tot, &cnt))) break;
    if (cnt) tf[v] = tot / cnt;
    if ((rc = tn_timing_read("edge_bwd", &tot, &cnt))) break;
    if (cnt) tb[v] = tot / cnt;
  }
  tn_timing_reset();
  timing_swap(was_timing);
  m->pair_force[p][0] = saved[0];
  m->pair_force[p][1] = saved[1];
  if (rc) return rc;
  int bf = 0, bb = 0;
  for (int v = 1; v < nv; ++v) {
    if (tf[v] < tf[bf]) bf = v;
    if (tb[v] < tb[bb]) bb = v;
  }
  m->pair_tuned[p][pair_budget_class(max_pairs)] = {bf, bb};
  if (chosen) {
    chosen[0] = bf;
    chosen[1] = bb;
  }
  return TN_OK;
}

const char *tn_status_string(int status) {
  switch (status) {
    case TN_OK: return "ok";
    case TN_E_ARG: return "invalid argument";
    case TN_E_BLOB: return "invalid weight blob";
    case TN_E_HIP: return "HIP runtime error";
    case TN_E_BOX: return "box: a cell height is less than twice the cutoff";
    case TN_E_WORKSPACE: return "workspace too small";
    case TN_E_UNSUPPORTED: return "unsupported precision/path combination";
    default: return "unknown status";
  }
}

int tn_model_create(const void *blob, size_t blob_bytes, int device, tn_model **out) {
  if (!blob || !out) return TN_E_ARG;
  *out = nullptr;
  tn_model *m = new (std::nothrow) tn_model();
  if (!m) return TN_E_ARG;
  std::vector<double> packed;
  int rc = parse_blob(blob, blob_bytes, m, packed);
  if (rc) {
    delete m;
    return rc;
  }
  m->device = device;
  if (hipSetDevice(device) != hipSuccess) {
    delete m;
    return TN_E_HIP;
  }
  void *scratch_ptr = nullptr;   // set-up of tn_energy_forces_static's scratch on this device
  if (device < kMaxDevices && (rc = scratch_on_device(device, &scratch_ptr)) != TN_OK) {
    delete m;
    return rc;
  }
  const size_t n = packed.size();
  std::vector<float> f32(n);
  std::vector<__bf16> f16(n);
  for (size_t i = 0; i < n; ++i) {
    f32[i] = (float)packed[i];
    f16[i] = (__bf16)f32[i];
  }
  if (hipMalloc(&m->w64, n * sizeof(double)) != hipSuccess || hipMalloc(&m->w32, n * sizeof(float)) != hipSuccess ||
      hipMalloc(&m->w16, n * sizeof(__bf16)) != hipSuccess ||
      hipMemcpy(m->w64, packed.data(), n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->w32, f32.data(), n * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->w16, f16.data(), n * sizeof(__bf16), hipMemcpyHostToDevice) != hipSuccess) {
    tn_model_destroy(m);
    return TN_E_HIP;
  }
  if ((rc = molecule_setup(m)) != TN_OK) {
    tn_model_destroy(m);
    return rc;
  }
  *out = m;
  return TN_OK;
}

void tn_model_destroy(tn_model *m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  if (m->mol_const) (void)hipFree(m->mol_const);
  if (m->w64) (void)hipFree(m->w64);
  if (m->w32) (void)hipFree(m->w32);
  if (m->w16) (void)hipFree(m->w16);
  delete m;
}

int tn_model_info(const tn_model *m, int32_t *F, int32_t *K, int32_t *L, int32_t *max_z, double *r_lo, double *r_c) {
  if (!m) return TN_E_ARG;
  if (F) *F = m->F;
  if (K) *K = m->K;
  if (L) *L = m->L;
  if (max_z) *max_z = m->max_z;
  if (r_lo) *r_lo = m->r_lo;
  if (r_c) *r_c = m->r_c;
  return TN_OK;
}

size_t tn_neighbor_workspace_bytes(int64_t n_atoms, int64_t max_pairs, const double *box, double cutoff) {
  BoxInfo bi;
  if (n_atoms < 0 || max_pairs < 0 || box_info(box, cutoff, &bi) != TN_OK) return 0;
  WsPlan p(nullptr);
  NbrWs w;
  plan_neighbors(p, n_atoms, max_pairs, bi, &w);
  return p.off;
}

int tn_build_neighbors(void *stream, int64_t n_atoms, const void *pos, int pos_f64, const int32_t *batch,
                       const double *box, double cutoff, int64_t max_pairs, int32_t *pairs, int64_t *n_pairs,
                       int32_t *status, void *ws, size_t ws_bytes) {
  return tn_build_neighbors_method(stream, n_atoms, pos, pos_f64, batch, box, cutoff, max_pairs, pairs, n_pairs,
                                   status, ws, ws_bytes, TN_NBR_AUTO);
}

int tn_build_neighbors_method(void *stream, int64_t n_atoms, const void *pos, int pos_f64, const int32_t *batch,
                              const double *box, double cutoff, int64_t max_pairs, int32_t *pairs,
                              int64_t *n_pairs, int32_t *status, void *ws, size_t ws_bytes, int method) {
  if (n_atoms < 0 || max_pairs < 0 || max_pairs > (int64_t(1) << 30) || n_atoms >= (int64_t(1) << 31)) return TN_E_ARG;
  if (!n_pairs || !status || (n_atoms > 0 && (!pos || !batch)) || (max_pairs > 0 && !pairs)) return TN_E_ARG;
  if (method != TN_NBR_AUTO && method != TN_NBR_CELL && method != TN_NBR_BRUTE) return TN_E_ARG;
  BoxInfo bi;
  int rc = box_info(box, cutoff, &bi);
  if (rc) return rc;
  if (method == TN_NBR_CELL && !bi.periodic) return TN_E_UNSUPPORTED;
  if (method == TN_NBR_BRUTE) bi.cells = 0;
  WsPlan p(ws);
  NbrWs w;
  plan_neighbors(p, n_atoms, max_pairs, bi, &w);
  if (!ws || p.off > ws_bytes) return TN_E_WORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((rc = fill_i32(s, status, 1, 0))) return rc;
  if (pos_f64)
    return build_neighbors<double>(s, n_atoms, static_cast<const double *>(pos), nullptr, batch, bi, cutoff, max_pairs,
                                   pairs, n_pairs, status, w, nullptr);
  return build_neighbors<float>(s, n_atoms, static_cast<const float *>(pos), nullptr, batch, bi, cutoff, max_pairs,
                                pairs, n_pairs, status, w, nullptr);
}

size_t tn_workspace_bytes(const tn_model *m, int64_t n_atoms, int64_t n_systems, int64_t max_pairs,
                          const double *box, int precision, int path, int want_forces) {
  if (!m || n_atoms < 0 || max_pairs < 0 || n_systems < 0) return 0;
  BoxInfo bi;
  if (box_info(box, m->r_c, &bi) != TN_OK) return 0;
  if (path == TN_PLAIN) {
    if (precision != TN_FP32 && precision != TN_FP64) return 0;
    return plain_workspace_bytes(m, n_atoms, n_systems, max_pairs, bi, precision, want_forces);
  }
  if (path == TN_FUSED) {
    if (precision != TN_FP32 && precision != TN_BF16) return 0;
    return fused_workspace_bytes(m, n_atoms, n_systems, max_pairs, bi, precision, want_forces);
  }
  if (path == TN_MOLECULE) {
    if ((precision != TN_FP32 && precision != TN_BF16) || bi.periodic) return 0;
    return molecule_workspace_bytes(m, n_atoms, n_systems, max_pairs, precision, want_forces);
  }
  return 0;
}

static int run_model(const tn_model *m, void *stream, int64_t n_atoms, int64_t n_systems, const void *pos,
                     const int32_t *z, const int32_t *batch, const double *box, int64_t max_pairs, int precision,
                     int path, double *energy, void *forces, int64_t *n_pairs, int32_t *status, void *ws,
                     size_t ws_bytes) {
  if (!m || n_atoms < 0 || n_systems < 0 || max_pairs < 0 || max_pairs > (int64_t(1) << 30) ||
      n_atoms >= (int64_t(1) << 31))
    return TN_E_ARG;
  if (n_atoms > 0 && (!pos || !z || !batch || n_systems < 1)) return TN_E_ARG;
  if (!energy && n_systems > 0) return TN_E_ARG;
  if (!n_pairs || !status || !ws) return TN_E_ARG;
  if (precision != TN_FP32 && precision != TN_BF16 && precision != TN_FP64) return TN_E_ARG;
  if (path != TN_FUSED && path != TN_PLAIN && path != TN_MOLECULE) return TN_E_ARG;
  if (path == TN_PLAIN && precision == TN_BF16) return TN_E_UNSUPPORTED;
  if ((path == TN_FUSED || path == TN_MOLECULE) && precision == TN_FP64) return TN_E_UNSUPPORTED;
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
  pb.want_forces = forces != nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if ((rc = fill_i32(s, status, 1, 0))) return rc;
  if (path == TN_PLAIN) return plain_run(m, s, pb, precision, ws, ws_bytes);
  if (path == TN_MOLECULE) return molecule_run(m, s, pb, precision, ws, ws_bytes);
  return fused_run(m, s, pb, precision, ws, ws_bytes);
}

int tn_energy(const tn_model *m, void *stream, int64_t n_atoms, int64_t n_systems, const void *pos, const int32_t *z,
              const int32_t *batch, const double *box, int64_t max_pairs, int precision, int path, double *energy,
              int64_t *n_pairs, int32_t *status, void *ws, size_t ws_bytes) {
  return run_model(m, stream, n_atoms, n_systems, pos, z, batch, box, max_pairs, precision, path, energy, nullptr,
                   n_pairs, status, ws, ws_bytes);
}

int tn_energy_forces(const tn_model *m, void *stream, int64_t n_atoms, int64_t n_systems, const void *pos,
                     const int32_t *z, const int32_t *batch, const double *box, int64_t max_pairs, int precision,
                     int path, double *energy, void *forces, int64_t *n_pairs, int32_t *status, void *ws,
                     size_t ws_bytes) {
  if (!forces && n_atoms > 0) return TN_E_ARG;
  return run_model(m, stream, n_atoms, n_systems, pos, z, batch, box, max_pairs, precision, path, energy, forces,
                   n_pairs, status, ws, ws_bytes);
}

int tn_energy_forces_static(const tn_model *m, void *stream, int64_t n_atoms, int64_t n_systems, const void *pos,
                            const int32_t *z, const int32_t *batch, const double *box, int64_t max_pairs,
                            int precision, int path, double *energy, void *forces, int64_t *n_pairs,
                            int32_t *status) {
  if (!m || (!forces && n_atoms > 0)) return TN_E_ARG;
  const size_t need = tn_workspace_bytes(m, n_atoms, n_systems, max_pairs, box, precision, path, 1);
  if (need == 0) return TN_E_ARG;
  if (need > (size_t)TN_STATIC_WS_BYTES) {
    std::fprintf(stderr,
                 "tensornet: tn_energy_forces_static needs %zu bytes of scratch for %lld atoms and max_pairs %lld; "
                 "the static scratch holds %zu (use tn_energy_forces with a workspace)\n",
                 need, (long long)n_atoms, (long long)max_pairs, (size_t)TN_STATIC_WS_BYTES);
    return TN_E_WORKSPACE;
  }
  if (hipSetDevice(m->device) != hipSuccess) return TN_E_HIP;
  void *ws = nullptr;
  const int rc = scratch_on_device(m->device, &ws);
  if (rc) return rc;
  return run_model(m, stream, n_atoms, n_systems, pos, z, batch, box, max_pairs, precision, path, energy, forces,
                   n_pairs, status, ws, (size_t)TN_STATIC_WS_BYTES);
}

}  // extern "C"
