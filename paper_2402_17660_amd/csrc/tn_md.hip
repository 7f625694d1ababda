// HIP-graph capture of energy+forces evaluations and of velocity-Verlet MD steps.
//
// Sec. 2.5 of the paper captures the whole network into one CUDA graph to remove launch
// overhead, which static pair budgets make possible.  Every entry point of this library is
// already capture-safe (no allocation, no host synchronisation, no memset nodes), so a graph
// here is simply the recorded enqueue sequence: for MD, per step a half kick, a drift with
// wrapping into the box, the neighbour search and energy+forces, and a second half kick.
#include "tn_internal.h"

#include <new>

namespace tn {

constexpr double kAccel = 9.648533212e-3;   // (eV / angstrom) / amu in angstrom / fs^2

__global__ void k_md_kick(int64_t n, float *vel, const float *forces, const float *inv_mass, float half_dt_acc) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float s = half_dt_acc * inv_mass[i];
  vel[3 * i] += s * forces[3 * i];
  vel[3 * i + 1] += s * forces[3 * i + 1];
  vel[3 * i + 2] += s * forces[3 * i + 2];
}

// x += dt v, then wrap into the cell: [0, L) per axis for a rectangular box, fractional
// coordinates in [0, 1) for a triclinic cell.
__global__ void k_md_drift(int64_t n, float *pos, const float *vel, float dt, Lattice lat, int tri) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  float x[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) x[a] = pos[3 * i + a] + dt * vel[3 * i + a];
  if (lat.periodic && tri) {
    double s0, s1, s2;
    fractional(lat, x[0], x[1], x[2], s0, s1, s2);
    s0 -= floor(s0);
    s1 -= floor(s1);
    s2 -= floor(s2);
    x[0] = (float)(s0 * lat.ax + s1 * lat.bx + s2 * lat.cx);
    x[1] = (float)(s1 * lat.by + s2 * lat.cy);
    x[2] = (float)(s2 * lat.cz);
  } else if (lat.periodic) {
    const float L[3] = {(float)lat.ax, (float)lat.by, (float)lat.cz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      x[a] -= L[a] * floorf(x[a] / L[a]);
      if (x[a] >= L[a]) x[a] -= L[a];   // rounding can land exactly on L
      if (x[a] < 0.f) x[a] = 0.f;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) pos[3 * i + a] = x[a];
}

__global__ void k_status_or(const int32_t *step_status, int32_t *acc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *acc |= *step_status;
}

struct Graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

}  // namespace tn

using namespace tn;

extern "C" {

int tn_md_capture(const tn_model *m, void *stream, int64_t n_atoms, int64_t n_systems, void *pos, float *vel,
                  const float *inv_mass, const int32_t *z, const int32_t *batch, const double *box, double dt_fs,
                  int n_steps, int64_t max_pairs, int precision, int path, double *energy, void *forces,
                  int64_t *n_pairs, int32_t *status, void *ws, size_t ws_bytes, void **graph_out) {
  if (!m || !graph_out || n_steps < 0 || !status || !forces) return TN_E_ARG;
  if (n_steps > 0 && (!vel || !inv_mass || precision == TN_FP64 || !(dt_fs > 0.0))) return TN_E_ARG;
  *graph_out = nullptr;
  BoxInfo bi;
  int rc = box_info(box, m->r_c, &bi);
  if (rc) return rc;
  // a scratch status word for the steps (the caller's word accumulates them)
  const size_t need = tn_workspace_bytes(m, n_atoms, n_systems, max_pairs, box, precision, path, 1);
  if (need == 0) return TN_E_ARG;
  if (!ws || ws_bytes < need + 256) return TN_E_WORKSPACE;
  int32_t *step_status = reinterpret_cast<int32_t *>(static_cast<char *>(ws) + ((need + 255) / 256) * 256);
  if ((size_t)((char *)(step_status + 1) - (char *)ws) > ws_bytes) return TN_E_WORKSPACE;
  if (hipSetDevice(m->device) != hipSuccess) return TN_E_HIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Graph *g = new (std::nothrow) Graph();
  if (!g) return TN_E_ARG;
  const bool was_timing = timing_swap(false);   // no event records inside a graph
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    timing_swap(was_timing);
    delete g;
    return TN_E_HIP;
  }
  const unsigned blocks = grid_for(n_atoms > 0 ? n_atoms : 1, 256);
  const float half = (float)(0.5 * dt_fs * kAccel);
  rc = TN_OK;
  if (n_steps == 0) {
    rc = tn_energy_forces(m, stream, n_atoms, n_systems, pos, z, batch, box, max_pairs, precision, path, energy,
                          forces, n_pairs, status, ws, need);
  } else {
    rc = fill_i32(s, status, 1, 0);
    float *p32 = static_cast<float *>(pos);
    float *f32 = static_cast<float *>(forces);
    for (int st = 0; st < n_steps && rc == TN_OK; ++st) {
      if (n_atoms > 0) {
        hipLaunchKernelGGL(k_md_kick, dim3(blocks), dim3(256), 0, s, n_atoms, vel, f32, inv_mass, half);
        hipLaunchKernelGGL(k_md_drift, dim3(blocks), dim3(256), 0, s, n_atoms, p32, vel, (float)dt_fs, bi.lat,
                           bi.tri);
        if (hipGetLastError() != hipSuccess) { rc = TN_E_HIP; break; }
      }
      rc = tn_energy_forces(m, stream, n_atoms, n_systems, pos, z, batch, box, max_pairs, precision, path, energy,
                            forces, n_pairs, step_status, ws, need);
      if (rc) break;
      hipLaunchKernelGGL(k_status_or, dim3(1), dim3(64), 0, s, step_status, status);
      if (n_atoms > 0)
        hipLaunchKernelGGL(k_md_kick, dim3(blocks), dim3(256), 0, s, n_atoms, vel, f32, inv_mass, half);
      if (hipGetLastError() != hipSuccess) rc = TN_E_HIP;
    }
  }
  hipGraph_t graph = nullptr;
  const hipError_t e_end = hipStreamEndCapture(s, &graph);
  timing_swap(was_timing);
  if (rc != TN_OK || e_end != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    delete g;
    return rc != TN_OK ? rc : TN_E_HIP;
  }
  g->graph = graph;
  if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(graph);
    delete g;
    return TN_E_HIP;
  }
  *graph_out = g;
  return TN_OK;
}

int tn_graph_replay(void *graph, void *stream) {
  if (!graph) return TN_E_ARG;
  Graph *g = static_cast<Graph *>(graph);
  if (hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)) != hipSuccess) return TN_E_HIP;
  return TN_OK;
}

int tn_graph_destroy(void *graph) {
  if (!graph) return TN_OK;
  Graph *g = static_cast<Graph *>(graph);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return TN_OK;
}

}  // extern "C"
