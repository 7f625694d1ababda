// Plain (unfused) TensorNet path: one kernel per operation, every intermediate
// kept in device memory, templated on the arithmetic type (float or double).
// It is the baseline the fused path is measured against, and in double it is
// the GPU-side correctness anchor.  Math follows TensorNet as described in
// Sec. 2.1.1 of the paper (I/A/S decomposition, channel mixing, messages,
// symmetric matrix products, normalisation) with the settings of Sec. 2.4
// (exp-normal basis, cosine cutoff, SiLU); energies are summed per system and
// forces are the negative position gradient (Sec. 2), here by a hand-written
// reverse sweep.
#include "tn_nodeops.h"

#include <cmath>

namespace tn {

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
  T *geo, *phi, *rbf, *f0, *Xr;
  TA *XrA, *T0, *nrm0, *xhat0, *rstd0, *n0, *ez1, *ea1, *ez2, *g, *X0A;
  std::vector<T *> X;              // L+1 layer inputs/outputs
  std::vector<T *> nX, Xb, Y, z1, a1, z2, a2, z3, h, M, P, nP, Pb, D;
  TA *XLA, *on, *oxhat, *orstd, *q, *oz, *ox, *hz, *hx, *eps, *eps_orig;
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
  w->eps_orig = p.take<TA>(N);
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

// ============================================================================ driver
template <class T>
static int run_plain(const tn_model *m, hipStream_t s, const Problem &pb, void *ws, size_t ws_bytes) {
  const int64_t N = pb.n, MP = pb.max_pairs, F = m->F, K = m->K, L = m->L;
  WsPlan plan(ws);
  PlainWs<T> w;
  plan_plain(plan, m, N, MP, pb.box, pb.want_forces, &w);
  if (plan.off > ws_bytes) return TN_E_WORKSPACE;
  const T *pos = nullptr;
  int rc;
  const unsigned bs = 256;
  auto W = [&](size_t off) { return wptr<T>(m, off); };
  auto WA = [&](size_t off) { return wptr<TA>(m, off); };
  const WeightOff &o = m->off;

  NbrGraph<T> gr;
  if ((rc = build_neighbors<T>(s, N, static_cast<const T *>(pb.pos), pb.z, pb.batch, pb.box, m->r_c, MP, nullptr,
                                 pb.n_pairs, pb.status, w.nb, &gr, pb.S, m->max_z)))
    return rc;
  const int64_t *np = pb.n_pairs;
  const int32_t *rowptr = gr.rowptr, *nbr = gr.nbr, *pid = gr.pid;
  const int32_t *zz = gr.z;
  pos = gr.pos;

  const Lattice bl = pb.box.lat;
  if (MP > 0) {
    hipLaunchKernelGGL(k_geom<T>, dim3(grid_for(MP, bs)), dim3(bs), 0, s, gr.pairs, MP, np, pos, bl, m->r_c, m->r_lo,
                       m->alpha, WA(o.mu), WA(o.beta), (int)K, w.geo, w.phi, w.rbf);
    TN_LAUNCH_CHECK();
  }
  // ---- embedding: pair part in T, node part in FP64
  if ((rc = linear_fwd<T>(s, w.rbf, MP, K, W(o.W0), W(o.b0), 3 * F, w.f0, nullptr, 0, nullptr, np))) return rc;
  const unsigned gNF = grid_for(N * F, bs);
  if (N > 0) {
    hipLaunchKernelGGL(k_embed_gather<T>, dim3(gNF), dim3(bs), 0, s, N, (int)F, rowptr, nbr, pid, np, MP, zz,
                       m->max_z, W(o.U), W(o.V), w.geo, w.phi, w.f0, w.Xr);
    TN_LAUNCH_CHECK();
  }
  if ((rc = convert<T, TA>(s, w.Xr, w.XrA, N * 9 * F))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_node_norm<TA>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.XrA, w.nrm0);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_layernorm<TA>, dim3(layernorm_grid(N)), dim3(256), 0, s, N, (int)F, w.nrm0, WA(o.ln_g),
                       WA(o.ln_b), w.n0, w.xhat0, w.rstd0);
    TN_LAUNCH_CHECK();
  }
  if ((rc = linear_fwd<TA>(s, w.n0, N, F, WA(o.W1), WA(o.b1), 2 * F, w.ea1, w.ez1, 1))) return rc;
  if ((rc = linear_fwd<TA>(s, w.ea1, N, 2 * F, WA(o.W2), WA(o.b2), 3 * F, w.g, w.ez2, 1))) return rc;
  const TA *Wemb[3] = {WA(o.Wmix[0]), WA(o.Wmix[1]), WA(o.Wmix[2])};
  if ((rc = mix<TA>(s, w.XrA, w.T0, N, F, Wemb, nullptr, 0, 0))) return rc;
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
    const T *W1T[3] = {W(lo.W1T[0]), W(lo.W1T[1]), W(lo.W1T[2])};
    if ((rc = mix<T>(s, w.Xb[l], w.Y[l], N, F, W1, W1T, 0, 0))) return rc;
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
    const T *W2T[3] = {W(lo.W2T[0]), W(lo.W2T[1]), W(lo.W2T[2])};
    if ((rc = mix<T>(s, w.Pb[l], w.D[l], N, F, W2, W2T, 0, 0))) return rc;
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
    hipLaunchKernelGGL(k_layernorm<TA>, dim3(layernorm_grid(N)), dim3(256), 0, s, N, (int)(3 * F), w.on, WA(o.oln_g),
                       WA(o.oln_b), w.q, w.oxhat, w.orstd);
    TN_LAUNCH_CHECK();
  }
  if ((rc = linear_fwd<TA>(s, w.q, N, 3 * F, WA(o.Wo), WA(o.bo), F, w.ox, w.oz, 1))) return rc;
  if ((rc = linear_fwd<TA>(s, w.ox, N, F, WA(o.Wh), WA(o.bh), H, w.hx, w.hz, 1))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_out_final_w<TA>, dim3(wave_atom_grid(N)), dim3(256), 0, s, N, (int)H, w.hx, WA(o.wout),
                       WA(o.bout), w.eps);
    TN_LAUNCH_CHECK();
  }
  const TA *eps_caller = w.eps;
  if (gr.perm && N > 0) {
    hipLaunchKernelGGL(k_unpermute<TA>, dim3(grid_for(N, bs)), dim3(bs), 0, s, N, gr.perm, w.eps, w.eps_orig);
    TN_LAUNCH_CHECK();
    eps_caller = w.eps_orig;
  }
  if (pb.S > 0) {
    hipLaunchKernelGGL(k_energy_reduce<TA>, dim3((unsigned)pb.S), dim3(128), 0, s, N, eps_caller, pb.batch,
                       pb.energy, pb.status);
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
    hipLaunchKernelGGL(k_layernorm_bwd<TA>, dim3(layernorm_grid(N)), dim3(256), 0, s, N, (int)(3 * F), w.dq, w.oxhat,
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
    const T *W1T[3] = {W(lo.W1T[0]), W(lo.W1T[1]), W(lo.W1T[2])};
    const T *W2[3] = {W(lo.W2[0]), W(lo.W2[1]), W(lo.W2[2])};
    const T *W2T[3] = {W(lo.W2T[0]), W(lo.W2T[1]), W(lo.W2T[2])};
    if (N > 0) {
      hipLaunchKernelGGL(k_residual_bwd<T>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.D[l], w.dX, w.dD);
      TN_LAUNCH_CHECK();
    }
    if ((rc = mix<T>(s, w.dD, w.dPb, N, F, W2, W2T, 1, 0))) return rc;
    if (N > 0) {
      hipLaunchKernelGGL(k_product_bwd<T>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.dPb, w.P[l], w.nP[l], w.Y[l],
                         w.M[l], w.dY, w.dM, nullptr);
      TN_LAUNCH_CHECK();
      hipLaunchKernelGGL(k_message<T>, dim3(gNF), dim3(bs), 0, s, N, (int)F, rowptr, nbr, pid, np, MP, w.h[l], w.dM,
                         w.dY, 1);
      TN_LAUNCH_CHECK();
    }
    if (MP > 0) {
      hipLaunchKernelGGL(k_message_bwd_pair<T>, dim3(grid_for(MP * F, bs)), dim3(bs), 0, s, gr.pairs, MP, np, (int)F,
                         w.Y[l], w.dM, w.dh);
      TN_LAUNCH_CHECK();
    }
    // dXb = dX (identity branch) + mix^T(W1, dY), accumulated in place
    if ((rc = mix<T>(s, w.dY, w.dX, N, F, W1, W1T, 1, 1))) return rc;
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
  if ((rc = mix<TA>(s, w.dT0, w.dXrA, N, F, Wemb, nullptr, 1, 0))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_mul_silu_grad<TA>, dim3(grid_for(N * 3 * F, bs)), dim3(bs), 0, s, N * 3 * F, w.dg, w.ez2,
                       w.dez2);
    TN_LAUNCH_CHECK();
  }
  if ((rc = linear_bwd<TA>(s, w.dez2, N, 3 * F, WA(o.W2), 2 * F, w.dez1, w.ez1, 0))) return rc;
  if ((rc = linear_bwd<TA>(s, w.dez1, N, 2 * F, WA(o.W1), F, w.dn0, nullptr, 0))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_layernorm_bwd<TA>, dim3(layernorm_grid(N)), dim3(256), 0, s, N, (int)F, w.dn0, w.xhat0, w.rstd0,
                       WA(o.ln_g), w.dnrm0);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_norm_bwd_add<TA>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.XrA, w.dnrm0, w.dXrA);
    TN_LAUNCH_CHECK();
  }
  if ((rc = convert<TA, T>(s, w.dXrA, w.dXr, N * 9 * F))) return rc;
  if (MP > 0) {
    hipLaunchKernelGGL(k_embed_bwd_pair<T>, dim3((unsigned)MP), dim3(128), 0, s, gr.pairs, MP, np, (int)F, zz,
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
                       w.gpair, gr.perm, static_cast<T *>(pb.forces));
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
