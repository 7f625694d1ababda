/*
 * tensornet.h - C ABI of the MI355X TensorNet energy-and-forces library.
 *
 * One TensorNet evaluation (TorchMD-Net 2.0, arXiv 2402.17660): the neighbour
 * search of Sec. 2.5.1 (cell list with rectangular or triclinic periodic
 * boundaries, or a brute-force search inside each system), the TensorNet network of
 * Sec. 2.1.1 with the hyper-parameters of Sec. 2.4, and forces as the negative
 * position gradient of the per-system energy (Sec. 2, model composition); and
 * the training step on energies and forces (Sec. 2.5, Sec. 3): the loss and its
 * exact gradient with respect to every weight.
 *
 * Conventions shared by every entry point
 *   - Every array argument is a DEVICE pointer owned by the caller, except
 *     `box` and `blob`, which are host pointers.  The library allocates no
 *     memory per call: scratch space is the caller's `ws` buffer, sized by the
 *     matching *_workspace_bytes query.
 *   - `stream` is a hipStream_t passed as void*.  All work is enqueued on it
 *     and no call synchronises the host, so every call may be captured into a
 *     HIP graph (pointers and sizes stay fixed across replays).
 *   - Return value: TN_OK (0) or a negative tn_status for errors that the host
 *     can see without reading device memory (bad arguments, box too small,
 *     bad blob, HIP launch failure).  Data-dependent errors are OR-ed into the
 *     device word `*status` (TN_STATUS_* bits) which the call first clears;
 *     read it after your own synchronisation.  Outputs are undefined whenever
 *     the return value or *status is non-zero.
 *   - Positions are angstrom, energies eV, forces eV/angstrom.  `box` is a
 *     row-major 3x3 whose rows are the lattice vectors a, b, c of a periodic
 *     cell (Sec. 2.5.1: rectangular and triclinic).  It must be lower
 *     triangular (a = (a_x,0,0), b = (b_x,b_y,0), c = (c_x,c_y,c_z), positive
 *     diagonal) and reduced (|b_x|, |c_x| <= a_x/2, |c_y| <= b_y/2), else
 *     TN_E_ARG; every cell height (distance between opposite faces) must be
 *     at least twice the cutoff, else TN_E_BOX, so the minimum image is
 *     unique.  A rectangular box is the case of zero tilts.  box == NULL
 *     means isolated systems.
 *   - `batch[i]` is the system index of atom i.  It must be sorted ascending
 *     (systems contiguous) with values in [0, n_systems); violations set
 *     TN_STATUS_BATCH.  Systems never interact (Sec. 2.5.1).
 */
#ifndef TENSORNET_H
#define TENSORNET_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tn_model tn_model;

typedef enum {
  TN_OK = 0,
  TN_E_ARG = -1,        /* invalid argument (null pointer, size, enum, box not lower triangular/reduced) */
  TN_E_BLOB = -2,       /* weight blob: bad magic, version, size or hyper-parameters */
  TN_E_HIP = -3,        /* a HIP runtime call or kernel launch failed */
  TN_E_BOX = -4,        /* a cell height is less than twice the cutoff */
  TN_E_WORKSPACE = -5,  /* ws_bytes smaller than the workspace query returned */
  TN_E_UNSUPPORTED = -6 /* valid request this library does not implement (e.g. precision/path pair) */
} tn_status;

/* Bits of the device status word. */
#define TN_STATUS_OVERFLOW 1   /* more pairs than max_pairs; *n_pairs holds the true count */
#define TN_STATUS_BATCH 2      /* batch not sorted, or outside [0, n_systems) */
#define TN_STATUS_Z 4          /* atomic number outside [0, max_z) */
#define TN_STATUS_NONFINITE 8  /* non-finite position or energy */

typedef enum { TN_FP32 = 0, TN_BF16 = 1, TN_FP64 = 2 } tn_precision;
typedef enum { TN_FUSED = 0, TN_PLAIN = 1, TN_MOLECULE = 2 } tn_path;

/* Status code to a static English string. */
const char *tn_status_string(int status);

/* ---------------------------------------------------------------- model ---
 * tn_model_create: parse a weight blob (host bytes, copied) and upload the
 * weights to `device` in FP64, FP32 and BF16.  Blob layout: 8-byte magic
 * "TNETBLOB", u32 version (1), F, K, L, max_z, activation (1 = SiLU), two
 * reserved u32, f64 r_lo, f64 r_c, then the float64 tensors in the fixed order
 * of the generator (embedding, L interaction layers, output network).
 * Errors: TN_E_ARG (null pointers), TN_E_BLOB (format), TN_E_HIP (upload).
 * The model is owned by the caller and freed by tn_model_destroy. */
int tn_model_create(const void *blob, size_t blob_bytes, int device, tn_model **out);
void tn_model_destroy(tn_model *m);

/* Hyper-parameters of a created model (any pointer may be NULL). */
int tn_model_info(const tn_model *m, int32_t *F, int32_t *K, int32_t *L, int32_t *max_z,
                  double *r_lo, double *r_c);

/* ------------------------------------------------------ neighbour search ---
 * The unordered pair set {(i,j) : i<j, batch_i == batch_j, d_ij^2 < cutoff^2}
 * (Sec. 2.5.1), d by the minimum image when `box` is given.  The decision is
 * taken in FP64 on the positions promoted to FP64, D = r_j - r_i reduced
 * along c, then b, then a (box only):
 *   v = D - c rint(D_z / c_z);  v -= b rint(v_y / b_y);  v -= a rint(v_x / a_x)
 *   d^2 = (v_x*v_x + v_y*v_y) + v_z*v_z  (each product rounded, no FMA)
 * (for a rectangular box, v_a = D_a - L_a rint(D_a / L_a)).
 * box != NULL: one cell list over all systems (cells binned in fractional
 * coordinates, at least as high as the cutoff).
 * box == NULL: brute force over the atoms of each system.
 * Output: pairs[0][p] < pairs[1][p] (int32, layout [2, max_pairs]) for
 * p < *n_pairs, in a deterministic order (by (i, j) for isolated systems, by
 * cell order in a box); slots p >= *n_pairs hold -1.  *n_pairs
 * (device int64) is always the true count; if it exceeds max_pairs,
 * TN_STATUS_OVERFLOW is set and `pairs` is only padding.
 * pos: [n_atoms, 3] float32 (pos_f64 == 0) or float64 (pos_f64 != 0). */
size_t tn_neighbor_workspace_bytes(int64_t n_atoms, int64_t max_pairs, const double *box, double cutoff);
int tn_build_neighbors(void *stream, int64_t n_atoms, const void *pos, int pos_f64, const int32_t *batch,
                       const double *box, double cutoff, int64_t max_pairs, int32_t *pairs, int64_t *n_pairs,
                       int32_t *status, void *ws, size_t ws_bytes);

/* The same search with an explicit candidate strategy (Sec. 2.5.1 offers a
 * brute-force O(N^2) search for small inputs and a cell list for large ones):
 *   TN_NBR_AUTO   cell list in a periodic box, brute force for isolated systems
 *                 (what tn_build_neighbors and the model calls use)
 *   TN_NBR_CELL   cell list; needs a box (TN_E_UNSUPPORTED without one)
 *   TN_NBR_BRUTE  every atom of the same system is a candidate (system ranges
 *                 from the sorted batch vector); minimum image in a box
 * The pair set is the same for every strategy; the pair order is deterministic
 * per strategy (cell order with the cell list, by (i, j) with the brute force).
 * tn_neighbor_workspace_bytes covers every strategy.  Other arguments, outputs
 * and errors as for tn_build_neighbors; an unknown method is TN_E_ARG. */
#define TN_NBR_AUTO 0
#define TN_NBR_CELL 1
#define TN_NBR_BRUTE 2
int tn_build_neighbors_method(void *stream, int64_t n_atoms, const void *pos, int pos_f64, const int32_t *batch,
                              const double *box, double cutoff, int64_t max_pairs, int32_t *pairs,
                              int64_t *n_pairs, int32_t *status, void *ws, size_t ws_bytes, int method);

/* -------------------------------------------------------------- energies ---
 * tn_workspace_bytes returns the ws size needed by tn_energy (want_forces 0)
 * or tn_energy_forces (want_forces 1) for these sizes, box and cutoff, or 0
 * for an invalid request.
 * Per-system energies E_s = sum over atoms of system s of the per-atom output
 * of the network (Sec. 2: representation model -> scalar output model ->
 * sum aggregation), accumulated in FP64.  The neighbour search above runs
 * inside the call with the model's cutoff.
 *   pos     [n_atoms, 3]: float64 for TN_FP64, float32 otherwise
 *   z       [n_atoms] int32 atomic numbers (embedding rows), < max_z
 *   batch   [n_atoms] int32 sorted system index
 *   energy  [n_systems] float64 output
 * precision: TN_FP64 (plain path only), TN_FP32, TN_BF16 (GEMM operands in
 * BF16, FP32 accumulation; fused and molecule paths only).  path:
 *   TN_FUSED     every operation one launch over all atoms or pairs of the
 *                batch (the per-pair work of all layers in two MFMA kernels)
 *   TN_PLAIN     one kernel per operation, every intermediate through memory
 *   TN_MOLECULE  isolated systems only (box == NULL, else TN_E_UNSUPPORTED),
 *                TN_FP32 or TN_BF16, hidden size 64 or 128 with 32 radial
 *                functions (else TN_E_UNSUPPORTED): one launch over the batch
 *                in which a workgroup owns whole systems and runs every
 *                stage (neighbour search by brute force over the system,
 *                layers, output, reverse sweep) with workgroup barriers
 *                only, so a small molecule costs one launch instead of one
 *                per operation (Sec. 2.5: launch overhead bounds small
 *                systems).  The arithmetic is the fused path's.  The pair
 *                budget is split in proportion to the atoms: a system of n
 *                of the n_atoms atoms gets about n * max_pairs / n_atoms pair
 *                slots; a system with more pairs sets TN_STATUS_OVERFLOW
 *                (*n_pairs is still the true total).  Best for systems of up
 *                to a few hundred atoms. */
size_t tn_workspace_bytes(const tn_model *m, int64_t n_atoms, int64_t n_systems, int64_t max_pairs,
                          const double *box, int precision, int path, int want_forces);
int tn_energy(const tn_model *m, void *stream, int64_t n_atoms, int64_t n_systems, const void *pos,
              const int32_t *z, const int32_t *batch, const double *box, int64_t max_pairs, int precision,
              int path, double *energy, int64_t *n_pairs, int32_t *status, void *ws, size_t ws_bytes);

/* Energies and forces F = -dE/dpos (Sec. 2): a hand-written reverse sweep of
 * the network that recomputes the per-pair geometry, cutoff and radial basis,
 * with the per-pair position gradients summed per atom in FP64.
 *   forces [n_atoms, 3]: float64 for TN_FP64, float32 otherwise. */
int tn_energy_forces(const tn_model *m, void *stream, int64_t n_atoms, int64_t n_systems, const void *pos,
                     const int32_t *z, const int32_t *batch, const double *box, int64_t max_pairs,
                     int precision, int path, double *energy, void *forces, int64_t *n_pairs, int32_t *status,
                     void *ws, size_t ws_bytes);

/* ------------------------------------------- without a caller workspace ---
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).
 * tn_energy_forces_static is tn_energy_forces (same arguments, outputs,
 * status word and errors) with the scratch space taken from the library's
 * own static device array of TN_STATIC_WS_BYTES bytes instead of a `ws`
 * argument.  The call allocates and frees nothing: the array is part of the
 * library's code object, so every GPU the library runs on holds one copy of
 * it until the process ends; its device address is looked up once per device
 * (at tn_model_create, with that device current).
 *   - A request whose workspace (tn_workspace_bytes with want_forces 1)
 *     exceeds TN_STATIC_WS_BYTES is rejected with TN_E_WORKSPACE before any
 *     work is enqueued (and a message on stderr); use tn_energy_forces then.
 *     128 MiB covers, e.g., a molecule of a few hundred atoms with the pair
 *     budget of 32 pairs per atom at hidden size 128 on the fused path.
 *   - Every call on one GPU shares that GPU's array, which keeps the last
 *     call's contents (nothing in it needs to start at zero).  Calls whose
 *     work overlaps on one GPU (different streams, or host threads without
 *     ordering) RACE on it and give undefined results: order them on one
 *     stream or serialise them. */
#define TN_STATIC_WS_BYTES ((size_t)128 << 20)
int tn_energy_forces_static(const tn_model *m, void *stream, int64_t n_atoms, int64_t n_systems, const void *pos,
                            const int32_t *z, const int32_t *batch, const double *box, int64_t max_pairs,
                            int precision, int path, double *energy, void *forces, int64_t *n_pairs,
                            int32_t *status);

/* -------------------------------------------------------- training step ---
 * Force training (Sec. 2.5: training on forces differentiates through the
 * force computation a second time; Sec. 3 trains on energies and forces
 * together) with the loss
 *   loss = w_energy * mean_s (E_s - energy_ref_s)^2
 *        + w_force  * mean_{i,a} (F_ia - forces_ref_ia)^2,   F = -dE/dpos,
 * and its gradient with respect to every tensor of the weight blob.  Two
 * passes: energies and forces (as tn_energy_forces: the fused path in FP32
 * where its pair kernels cover the model's sizes, else the plain path), then
 * the reverse sweep to the
 * parameters on dual numbers whose positions carry the tangent d loss/dF, so
 * the force term's mixed second derivative comes out exactly (forward over
 * reverse), not by finite differences.
 *   tn_param_count: number of float64 values in the blob's tensors (the
 *     length of grad), or -1 for a null model.
 *   tn_train_workspace_bytes: ws size for tn_train_grad, 0 if invalid.
 *   precision: TN_FP64 or TN_FP32 (the second pass computes every step in that
 *     type; pos and forces typed as for tn_energy_forces).  Others:
 *     TN_E_UNSUPPORTED.
 *   energy_ref [n_systems], forces_ref [n_atoms, 3]: float64 targets (device).
 *   loss: one float64 (device); energy [n_systems] float64 and forces
 *     [n_atoms, 3] receive the model's predictions at pos.
 *   grad: [tn_param_count] float64 (device), overwritten, blob tensor order
 *     and shapes (the model's own weights are not changed).
 * Pair budget, size limits and status as for tn_energy_forces. */
int64_t tn_param_count(const tn_model *m);
size_t tn_train_workspace_bytes(const tn_model *m, int64_t n_atoms, int64_t n_systems, int64_t max_pairs,
                                const double *box, int precision);
int tn_train_grad(const tn_model *m, void *stream, int64_t n_atoms, int64_t n_systems, const void *pos,
                  const int32_t *z, const int32_t *batch, const double *box, int64_t max_pairs, int precision,
                  const double *energy_ref, const double *forces_ref, double w_energy, double w_force,
                  double *loss, double *energy, void *forces, double *grad, int64_t *n_pairs, int32_t *status,
                  void *ws, size_t ws_bytes);

/* ------------------------------------------------------ pair-tile tuning ---
 * The fused path evaluates every layer's edge filter once per unordered pair
 * in MFMA tiles (Sec. 2.5: per-pair work dominates; the paper picks kernel
 * variants by input size).  The tiles come in several shapes (pairs per tile,
 * workgroups per compute unit); each pair is computed with the same arithmetic
 * in the same order in every shape, so results are bitwise independent of it.
 *   tn_pair_variant_count(precision): number of shapes for TN_FP32 / TN_BF16
 *     (0 for other precisions).
 *   tn_model_set_pair_variant: forces a shape for the forward and the reverse
 *     pair kernel (-1 = the tuned choice, else shape 0).  TN_E_ARG for an
 *     out-of-range shape or precision.
 *   tn_autotune: runs tn_energy_forces (TN_FUSED) on the given inputs with
 *     every shape, `reps` timed calls each (1..1000), and records the fastest
 *     forward and reverse shapes in the model for calls whose max_pairs has the
 *     same bit length; `chosen` (host int32[2], may be NULL) receives them.
 *     It leaves energy/forces/n_pairs/status as one call would, resets the
 *     tn_timing_* registry and synchronises on its own timing events, so it must
 *     not be captured: call it before tn_md_capture.
 * Not thread-safe against other calls on the same model. */
int tn_pair_variant_count(int precision);
int tn_model_set_pair_variant(tn_model *m, int precision, int forward, int reverse);
int tn_autotune(tn_model *m, void *stream, int64_t n_atoms, int64_t n_systems, const void *pos, const int32_t *z,
                const int32_t *batch, const double *box, int64_t max_pairs, int precision, double *energy,
                void *forces, int64_t *n_pairs, int32_t *status, void *ws, size_t ws_bytes, int reps,
                int32_t *chosen);

/* ------------------------------------------------------- graphs and MD ---
 * tn_md_capture records work on `stream` into a HIP graph and instantiates
 * it; nothing runs until tn_graph_replay.  The arguments of tn_energy_forces
 * plus:
 *   vel       [n_atoms, 3] float32 velocities (angstrom/fs), updated in place
 *   inv_mass  [n_atoms] float32 inverse masses (1/amu)
 *   dt_fs     time step (fs)
 *   n_steps   0: the graph is one energy+forces evaluation (forces written to
 *             `forces`); >= 1: n_steps velocity-Verlet steps, each
 *               v += dt/2 * F/m;  x += dt * v;  x wrapped into the cell
 *               (fractional coordinates in [0, 1); box only);
 *               neighbour search + energy + forces;  v += dt/2 * F/m
 *             with F/m in eV/(angstrom amu) converted to angstrom/fs^2.  On entry
 *             `forces` must hold the forces of the current positions (call
 *             tn_energy_forces once before the first replay); pos is float32.
 *   status    device word; in MD graphs it accumulates (OR) the status bits of
 *             every step of a replay, cleared at the start of each replay.
 * Every buffer must stay allocated, at the same address, while the graph
 * exists.  Returns TN_OK or an error; *graph_out receives an opaque handle
 * freed by tn_graph_destroy.  Replays are ordered on the replay stream. */
int tn_md_capture(const tn_model *m, void *stream, int64_t n_atoms, int64_t n_systems, void *pos, float *vel,
                  const float *inv_mass, const int32_t *z, const int32_t *batch, const double *box, double dt_fs,
                  int n_steps, int64_t max_pairs, int precision, int path, double *energy, void *forces,
                  int64_t *n_pairs, int32_t *status, void *ws, size_t ws_bytes, void **graph_out);
int tn_graph_replay(void *graph, void *stream);
int tn_graph_destroy(void *graph);

/* ------------------------------------------------------------ diagnostics ---
 * Kernel timing for measurement tools.  While enabled, the library records a
 * HIP event pair on the launch stream around every launch of a timed kernel
 * (the dominant pair-tile kernels; names such as "edge_fwd").  tn_timing_read
 * waits for the recorded events and returns the summed duration (ms) and the
 * number of launches since the last reset.  Not for use under graph capture.
 * Returns TN_OK, TN_E_ARG (unknown name / null pointers) or TN_E_HIP. */
int tn_timing_enable(int on);
int tn_timing_reset(void);
int tn_timing_read(const char *name, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* TENSORNET_H */
