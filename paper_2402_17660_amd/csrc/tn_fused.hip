// Fused TensorNet path: the per-pair work (geometry, radial basis, the embedding's K->3F map
// and every layer's edge filter, forward and reverse) runs in two MFMA pair-tile kernels;
// the node-level steps use the shared node kernels.  Precision plan: FP32 arithmetic, with
// the geometry/basis, the embedding's node stage (norms, LayerNorm, MLP, gating; its channel
// mixing is linear and runs in FP32) and the output network in FP64 ("islands"), reading and
// writing the FP32 feature arrays directly; the per-system energy sum and the per-atom force
// sum in FP64.  The BF16 variant feeds the pair kernels' GEMMs and the channel mixing BF16
// operands (FP32 accumulation and FP32 feature arrays), stores the pre-activations and copies
// of Y and dE/dM in BF16 for the message gathers, and runs the islands in FP32 (its error
// budget is set by the BF16 operands).  In both precisions the edge filters h = phi silu(z3)
// are not stored: the message gathers form them from z3 and phi.
#include "tn_nodeops.h"

namespace tn {

int pair_budget_class(int64_t max_pairs) {
  int c = 0;
  while (max_pairs > 0) {
    ++c;
    max_pairs >>= 1;
  }
  return c;
}

int pair_variant(const tn_model *m, bool bf16, int64_t max_pairs, bool reverse) {
  const int prec = bf16 ? 1 : 0, dir = reverse ? 1 : 0;
  int v = m->pair_force[prec][dir];
  if (v < 0) {
    auto it = m->pair_tuned[prec].find(pair_budget_class(max_pairs));
    v = it != m->pair_tuned[prec].end() ? it->second[dir] : 0;
  }
  return (v >= 0 && v < pair_variant_count(bf16)) ? v : 0;
}

namespace {

template <class TA>
struct FusedWs {
  NbrWs nb;
  float *geo, *phi, *f0, *Xr, *T0;
  TA *nrm0, *xhat0, *rstd0, *n0, *ez1, *ea1, *ez2, *g;
  std::vector<float *> X, nX, Xb, Y, z1, z2, z3, h, M, P, nP, Pb, D, dM;
  std::vector<__bf16 *> Y16, dM16;   // BF16 copies of Y and dM for the gathers (BF16 path)
  TA *on, *oxhat, *orstd, *q, *oz, *ox, *hz, *hx, *eps, *eps_orig;
  float *dX = nullptr, *dD, *dPb, *dY, *dXr, *dT0;
  // BF16 path: Pb, dD, dY + its gathered sum, and dT0 are read only by the next channel mixing,
  // which rounds them to BF16, so their producers write them rounded, here (one at a time;
  // the FP32 buffers Pb, dD and dT0 are then not allocated)
  __bf16 *mix16 = nullptr;
  TA *dez2, *dez1, *dn0, *dnrm0, *dhz, *dox, *dq, *don;
  float *gpair;
};

template <class TA>
void plan_fused(WsPlan &p, const tn_model *m, int64_t N, int64_t MP, const BoxInfo &bi, bool fw, bool bf16,
                FusedWs<TA> *w) {
  const int64_t F = m->F, L = m->L;
  plan_neighbors(p, N, MP, bi, &w->nb);
  w->geo = p.take<float>(4 * MP);
  w->phi = p.take<float>(MP);
  w->f0 = p.take<float>(bf16 ? MP * 3 * F / 2 : MP * 3 * F);   // BF16 in the BF16 path
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
  w->X.resize(L + 1);
  for (int64_t l = 0; l <= L; ++l) w->X[l] = p.take<float>(N * 9 * F);
  auto per_layer = [&](std::vector<float *> &v, int64_t count) {
    v.resize(L);
    for (int64_t l = 0; l < L; ++l) v[l] = p.take<float>(count);
  };
  per_layer(w->nX, N * F);
  per_layer(w->Xb, N * 9 * F);
  per_layer(w->Y, N * 9 * F);
  // pre-activations per pair: row-major BF16 in the BF16 path; the FP32 kernels store z1 and z2
  // in whole 16-pair blocks
  const int64_t MP16 = (MP + 15) / 16 * 16;
  per_layer(w->z1, bf16 ? MP * F / 2 : MP16 * F);
  per_layer(w->z2, bf16 ? MP * F : MP16 * 2 * F);
  per_layer(w->z3, bf16 ? MP * 3 * F / 2 : MP * 3 * F);
  // no h per pair: the message gathers form it from z3 and phi
  w->h.assign(L, nullptr);
  per_layer(w->M, N * 9 * F);
  // P and ||P|| are formed again by the reverse pass (product_bwd_at), not stored
  w->P.assign(L, nullptr);
  w->nP.assign(L, nullptr);
  if (bf16) {   // Pb goes to mix16 in BF16
    w->Pb.assign(L, nullptr);
    w->mix16 = p.take<__bf16>(N * 9 * F);
  } else {
    per_layer(w->Pb, N * 9 * F);
  }
  per_layer(w->D, N * 9 * F);
  if (bf16) {
    w->Y16.resize(L);
    for (int64_t l = 0; l < L; ++l) w->Y16[l] = p.take<__bf16>(N * 9 * F);
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
  w->eps_orig = p.take<TA>(N);
  if (!fw) return;
  per_layer(w->dM, N * 9 * F);
  if (bf16) {
    w->dM16.resize(L);
    for (int64_t l = 0; l < L; ++l) w->dM16[l] = p.take<__bf16>(N * 9 * F);
  }
  w->dX = p.take<float>(N * 9 * F);
  w->dD = bf16 ? nullptr : p.take<float>(N * 9 * F);   // BF16: mix16
  w->dPb = p.take<float>(N * 9 * F);
  w->dY = p.take<float>(N * 9 * F);
  w->dXr = p.take<float>(N * 9 * F);
  w->dT0 = bf16 ? nullptr : p.take<float>(N * 9 * F);   // BF16: mix16
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

template <bool BF16>
int run_fused(const tn_model *m, hipStream_t s, const Problem &pb, void *ws, size_t ws_bytes) {
  using TA = typename std::conditional<BF16, float, double>::type;   // the islands' type
  using TH = typename std::conditional<BF16, __bf16, float>::type;   // the edge filters' type
  using TY = TH;   // the type of the atom rows the gathers read (Y, dM)
  const int64_t N = pb.n, MP = pb.max_pairs, F = m->F, K = m->K, L = m->L;
  WsPlan plan(ws);
  FusedWs<TA> w;
  plan_fused(plan, m, N, MP, pb.box, pb.want_forces, BF16, &w);
  if (plan.off > ws_bytes) return TN_E_WORKSPACE;
  const float *pos = nullptr;
  int rc;
  const unsigned bs = 256;
  auto W = [&](size_t off) { return wptr<float>(m, off); };
  auto WA = [&](size_t off) { return wptr<TA>(m, off); };
  auto WD = [&](size_t off) { return wptr<double>(m, off); };
  const WeightOff &o = m->off;

  NbrGraph<float> gr;
  if ((rc = build_neighbors<float>(s, N, static_cast<const float *>(pb.pos), pb.z, pb.batch, pb.box, m->r_c, MP, nullptr,
                                 pb.n_pairs, pb.status, w.nb, &gr, pb.S, m->max_z)))
    return rc;
  const int64_t *np = pb.n_pairs;
  const int32_t *rowptr = gr.rowptr, *nbr = gr.nbr, *pid = gr.pid;
  const int32_t *zz = gr.z;
  pos = gr.pos;

  // ---- all per-pair work of the forward pass in one MFMA kernel
  auto WB = [&](size_t off) { return static_cast<const __bf16 *>(m->w16 + off); };
  // Per-part channel mixing with one set of matrices (Wf: aligned copies, WT: their transposes):
  // FP32 matrix-core kernel, or BF16 operands with FP32 accumulation in the BF16 path.
  auto mixing = [&](const float *in, float *out, const size_t Wf[3], const size_t WT[3], int adjoint,
                    int accumulate, __bf16 *out16) -> int {
    if (BF16) {
      const size_t *off = adjoint ? WT : Wf;
      const __bf16 *Bt[3] = {WB(off[0]), WB(off[1]), WB(off[2])};
      return mix_bf16(s, in, out, N, F, Bt, accumulate, out16);
    }
    const float *Wm[3] = {W(Wf[0]), W(Wf[1]), W(Wf[2])};
    const float *WmT[3] = {W(WT[0]), W(WT[1]), W(WT[2])};
    return mix<float>(s, in, out, N, F, Wm, WmT, adjoint, accumulate, out16);
  };
  // the same mixing of an input already rounded to BF16 (BF16 path only)
  auto mixing16 = [&](const __bf16 *in, float *out, const size_t Wf[3], const size_t WT[3], int adjoint,
                      int accumulate) -> int {
    const size_t *off = adjoint ? WT : Wf;
    const __bf16 *Bt[3] = {WB(off[0]), WB(off[1]), WB(off[2])};
    return mix_bf16(s, in, out, N, F, Bt, accumulate);
  };
  auto fill_common = [&](auto &pf) {
    pf.pairs = gr.pairs;
    pf.max_pairs = MP;
    pf.n_pairs = np;
    pf.pos = pos;
    pf.lat = pb.box.lat;
    pf.r_c = m->r_c;
    pf.r_lo = m->r_lo;
    pf.alpha = m->alpha;
    pf.mu = WD(o.mu);
    pf.beta = WD(o.beta);
    pf.L = (int)L;
  };
  if (BF16) {
    PairFwdArgsB pf;
    fill_common(pf);
    pf.W0 = WB(o.W0f);
    pf.b0 = W(o.b0);
    for (int64_t l = 0; l < L; ++l) {
      const LayerOff &lo = o.layer[l];
      pf.Wa[l] = WB(lo.Waf);
      pf.Wb[l] = WB(lo.Wbf);
      pf.Wc[l] = WB(lo.Wcf);
      pf.ba[l] = W(lo.ba);
      pf.bb[l] = W(lo.bb);
      pf.bc[l] = W(lo.bc);
      pf.z1[l] = reinterpret_cast<__bf16 *>(w.z1[l]);
      pf.z2[l] = reinterpret_cast<__bf16 *>(w.z2[l]);
      pf.z3[l] = reinterpret_cast<__bf16 *>(w.z3[l]);
      pf.h[l] = nullptr;   // not stored: the message gathers form it from z3 and phi
    }
    pf.geo = w.geo;
    pf.phi = w.phi;
    pf.f0 = reinterpret_cast<__bf16 *>(w.f0);
    if ((rc = launch_pair_fwd_bf16(s, (int)F, (int)K, pf, pair_variant(m, true, MP, false)))) return rc;
  } else {
    PairFwdArgs pf;
    fill_common(pf);
    pf.W0 = W(o.W0f);
    pf.b0 = W(o.b0);
    for (int64_t l = 0; l < L; ++l) {
      const LayerOff &lo = o.layer[l];
      pf.Wa[l] = W(lo.Waf);
      pf.ba[l] = W(lo.ba);
      pf.Wb[l] = W(lo.Wbf);
      pf.bb[l] = W(lo.bb);
      pf.Wc[l] = W(lo.Wcf);
      pf.bc[l] = W(lo.bc);
      pf.z1[l] = w.z1[l];
      pf.z2[l] = w.z2[l];
      pf.z3[l] = w.z3[l];
      pf.h[l] = nullptr;   // not stored: the message gathers form it from z3 and phi
    }
    pf.geo = w.geo;
    pf.phi = w.phi;
    pf.f0 = w.f0;
    if ((rc = launch_pair_fwd(s, (int)F, (int)K, pf, pair_variant(m, false, MP, false)))) return rc;
  }

  // ---- embedding node stage (FP64)
  const unsigned gNF = grid_for(N * F, bs);
  if ((rc = embed_gather_w(s, F, N, rowptr, nbr, pid, np, MP, zz, m->max_z, W(o.U), W(o.V), w.geo, w.phi,
                           reinterpret_cast<const TH *>(w.f0), w.Xr)))
    return rc;
  if (N > 0) {
    hipLaunchKernelGGL((k_node_norm<TA, float>), dim3(gNF), dim3(bs), 0, s, N, (int)F, w.Xr, w.nrm0);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_layernorm<TA>, dim3(layernorm_grid(N)), dim3(256), 0, s, N, (int)F, w.nrm0, WA(o.ln_g),
                       WA(o.ln_b), w.n0, w.xhat0, w.rstd0);
    TN_LAUNCH_CHECK();
  }
  if ((rc = linear_fwd<TA>(s, w.n0, N, F, WA(o.W1), WA(o.b1), 2 * F, w.ea1, w.ez1, 1))) return rc;
  if ((rc = linear_fwd<TA>(s, w.ea1, N, 2 * F, WA(o.W2), WA(o.b2), 3 * F, w.g, w.ez2, 1))) return rc;
  // the embedding's channel mixing is linear in the FP32 features and runs in FP32 (BF16 operands
  // in the BF16 path); the gating product is formed in FP64 and rounded once
  if ((rc = mixing(w.Xr, w.T0, o.Wmixf, o.WmixT, 0, 0, nullptr))) return rc;
  // (with layers, the gating also normalises the first layer's input)
  if (N > 0 && L > 0) {
    hipLaunchKernelGGL((k_gate_normalize<TA, float>), dim3(gNF), dim3(bs), 0, s, N, (int)F, w.g, w.T0, w.X[0],
                       w.nX[0], w.Xb[0]);
    TN_LAUNCH_CHECK();
  } else if (N > 0) {
    hipLaunchKernelGGL((k_gate<TA, float>), dim3(grid_for(N * 9 * F, bs)), dim3(bs), 0, s, N, (int)F, w.g, w.T0,
                       w.X[0]);
    TN_LAUNCH_CHECK();
  }
  // ---- interaction layers: mix, message+product, mix, residual(+normalise)
  for (int64_t l = 0; l < L; ++l) {
    const LayerOff &lo = o.layer[l];
    __bf16 *y16 = BF16 ? w.Y16[l] : nullptr;
    if ((rc = mixing(w.Xb[l], w.Y[l], lo.W1f, lo.W1T, 0, 0, y16))) return rc;
    // the neighbours' rows from the BF16 copy in the BF16 path
    const TY *yg = BF16 ? reinterpret_cast<const TY *>(y16) : reinterpret_cast<const TY *>(w.Y[l]);
    // z3, from which the gathers form h = phi silu(z3)
    const TH *hl = reinterpret_cast<const TH *>(w.z3[l]);
    const float *hphi = w.phi;
    if (BF16) {
      if ((rc = message_product_w(s, F, N, rowptr, nbr, pid, np, MP, hl, hphi, yg, w.mix16, w.Y[l], w.M[l],
                                  w.P[l], w.nP[l])))
        return rc;
      if ((rc = mixing16(w.mix16, w.D[l], lo.W2f, lo.W2T, 0, 0))) return rc;
    } else {
      if ((rc = message_product_w(s, F, N, rowptr, nbr, pid, np, MP, hl, hphi, yg, w.Pb[l], w.Y[l], w.M[l],
                                  w.P[l], w.nP[l])))
        return rc;
      if ((rc = mixing(w.Pb[l], w.D[l], lo.W2f, lo.W2T, 0, 0, nullptr))) return rc;
    }
    if (N > 0) {
      if (l + 1 < L) {
        hipLaunchKernelGGL(k_residual_normalize<float>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.Xb[l], w.D[l],
                           w.X[l + 1], w.nX[l + 1], w.Xb[l + 1]);
      } else {
        hipLaunchKernelGGL(k_residual<float>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.Xb[l], w.D[l], w.X[l + 1]);
      }
      TN_LAUNCH_CHECK();
    }
  }
  // ---- output network (FP64) and energies
  const int64_t H = F / 2;
  if (N > 0) {
    hipLaunchKernelGGL((k_out_norms<TA, float>), dim3(gNF), dim3(bs), 0, s, N, (int)F, w.X[L], w.on);
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
    hipLaunchKernelGGL((k_out_norms_bwd<TA, float>), dim3(gNF), dim3(bs), 0, s, N, (int)F, w.X[L], w.don, w.dX);
    TN_LAUNCH_CHECK();
  }
  for (int64_t l = L - 1; l >= 0; --l) {
    const LayerOff &lo = o.layer[l];
    if (BF16) {
      if (N > 0) {
        hipLaunchKernelGGL((k_residual_bwd<float, __bf16>), dim3(gNF), dim3(bs), 0, s, N, (int)F, w.D[l], w.dX,
                           w.mix16);
        TN_LAUNCH_CHECK();
      }
      if ((rc = mixing16(w.mix16, w.dPb, lo.W2f, lo.W2T, 1, 0))) return rc;
    } else {
      if (N > 0) {
        hipLaunchKernelGGL(k_residual_bwd<float>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.D[l], w.dX, w.dD);
        TN_LAUNCH_CHECK();
      }
      if ((rc = mixing(w.dD, w.dPb, lo.W2f, lo.W2T, 1, 0, nullptr))) return rc;
    }
    if (N > 0) {
      hipLaunchKernelGGL(k_product_bwd<float>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.dPb, w.P[l], w.nP[l], w.Y[l],
                         w.M[l], w.dY, w.dM[l], BF16 ? w.dM16[l] : nullptr);
      TN_LAUNCH_CHECK();
    }
    const TY *dmg = BF16 ? reinterpret_cast<const TY *>(w.dM16[l]) : reinterpret_cast<const TY *>(w.dM[l]);
    const TH *hl = reinterpret_cast<const TH *>(w.z3[l]);
    const float *hphi = w.phi;
    if (BF16) {   // dY + the gathered sum, rounded to BF16 for the mixing
      if ((rc = message_w(s, F, N, rowptr, nbr, pid, np, MP, hl, hphi, dmg, w.mix16, 1, (const float *)w.dY)))
        return rc;
      if ((rc = mixing16(w.mix16, w.dX, lo.W1f, lo.W1T, 1, 1))) return rc;
    } else {
      if ((rc = message_w(s, F, N, rowptr, nbr, pid, np, MP, hl, hphi, dmg, w.dY, 1, (const float *)nullptr)))
        return rc;
      if ((rc = mixing(w.dY, w.dX, lo.W1f, lo.W1T, 1, 1, nullptr))) return rc;
    }
    if (N > 0) {
      hipLaunchKernelGGL(k_normalize_bwd<float>, dim3(gNF), dim3(bs), 0, s, N, (int)F, w.X[l], w.nX[l], w.dX);
      TN_LAUNCH_CHECK();
    }
  }
  // ---- embedding adjoint, node part in FP64
  if (BF16) {
    if (N > 0) {
      hipLaunchKernelGGL((k_gate_bwd<TA, float, __bf16>), dim3(gNF), dim3(bs), 0, s, N, (int)F, w.dX, w.T0, w.g,
                         w.dez2, w.mix16, w.ez2);
      TN_LAUNCH_CHECK();
    }
    if ((rc = mixing16(w.mix16, w.dXr, o.Wmixf, o.WmixT, 1, 0))) return rc;
  } else {
    if (N > 0) {
      hipLaunchKernelGGL((k_gate_bwd<TA, float>), dim3(gNF), dim3(bs), 0, s, N, (int)F, w.dX, w.T0, w.g, w.dez2,
                         w.dT0, w.ez2);
      TN_LAUNCH_CHECK();
    }
    if ((rc = mixing(w.dT0, w.dXr, o.Wmixf, o.WmixT, 1, 0, nullptr))) return rc;
  }
  if ((rc = linear_bwd<TA>(s, w.dez2, N, 3 * F, WA(o.W2), 2 * F, w.dez1, w.ez1, 0))) return rc;
  if ((rc = linear_bwd<TA>(s, w.dez1, N, 2 * F, WA(o.W1), F, w.dn0, nullptr, 0))) return rc;
  if (N > 0) {
    hipLaunchKernelGGL(k_layernorm_bwd<TA>, dim3(layernorm_grid(N)), dim3(256), 0, s, N, (int)F, w.dn0, w.xhat0, w.rstd0,
                       WA(o.ln_g), w.dnrm0);
    TN_LAUNCH_CHECK();
    hipLaunchKernelGGL((k_norm_bwd_add<TA, float>), dim3(gNF), dim3(bs), 0, s, N, (int)F, w.Xr, w.dnrm0, w.dXr);
    TN_LAUNCH_CHECK();
  }
  // ---- all per-pair work of the reverse sweep in one MFMA kernel
  if (BF16) {
    PairBwdArgsB pbw;
    fill_common(pbw);
    pbw.W0T = WB(o.W0T);
    pbw.g.z = zz;
    pbw.g.U = W(o.U);
    pbw.g.V = W(o.V);
    pbw.g.max_z = m->max_z;
    pbw.g.f016 = reinterpret_cast<const __bf16 *>(w.f0);
    pbw.g.dXr = w.dXr;
    for (int64_t l = 0; l < L; ++l) {
      const LayerOff &lo = o.layer[l];
      pbw.WaT[l] = WB(lo.WaT);
      pbw.WbT[l] = WB(lo.WbT);
      pbw.WcT[l] = WB(lo.WcT);
      pbw.z1[l] = reinterpret_cast<const __bf16 *>(w.z1[l]);
      pbw.z2[l] = reinterpret_cast<const __bf16 *>(w.z2[l]);
      pbw.z3[l] = reinterpret_cast<const __bf16 *>(w.z3[l]);
      pbw.g.Y[l] = w.Y[l];
      pbw.g.dM[l] = w.dM[l];
      pbw.Y16[l] = w.Y16[l];
      pbw.dM16[l] = w.dM16[l];
    }
    pbw.gpair = w.gpair;
    if ((rc = launch_pair_bwd_bf16(s, (int)F, (int)K, pbw, pair_variant(m, true, MP, true)))) return rc;
  } else {
    PairBwdArgs pbw;
    fill_common(pbw);
    pbw.W0T = W(o.W0T);
    pbw.g.z = zz;
    pbw.g.U = W(o.U);
    pbw.g.V = W(o.V);
    pbw.g.max_z = m->max_z;
    pbw.g.f0 = w.f0;
    pbw.g.dXr = w.dXr;
    for (int64_t l = 0; l < L; ++l) {
      const LayerOff &lo = o.layer[l];
      pbw.WaT[l] = W(lo.WaT);
      pbw.WbT[l] = W(lo.WbT);
      pbw.WcT[l] = W(lo.WcT);
      pbw.z1[l] = w.z1[l];
      pbw.z2[l] = w.z2[l];
      pbw.z3[l] = w.z3[l];
      pbw.g.Y[l] = w.Y[l];
      pbw.g.dM[l] = w.dM[l];
    }
    pbw.gpair = w.gpair;
    if ((rc = launch_pair_bwd(s, (int)F, (int)K, pbw, pair_variant(m, false, MP, true)))) return rc;
  }
  if (N > 0) {
    hipLaunchKernelGGL((k_force_gather_w<float, float>), dim3(wave_atom_grid(N)), dim3(256), 0, s, N, rowptr, nbr,
                       pid, np, MP, w.gpair, gr.perm, static_cast<float *>(pb.forces));
    TN_LAUNCH_CHECK();
  }
  return TN_OK;
}

}  // namespace

size_t fused_workspace_bytes(const tn_model *m, int64_t n, int64_t S, int64_t max_pairs, const BoxInfo &bi, int prec,
                             int want_forces) {
  (void)S;
  if ((prec != TN_FP32 && prec != TN_BF16) || !pair_kernels_support(m->F, m->K, m->L, prec == TN_BF16)) return 0;
  WsPlan p(nullptr);
  if (prec == TN_BF16) {
    FusedWs<float> w;
    plan_fused(p, m, n, max_pairs, bi, want_forces != 0, true, &w);
  } else {
    FusedWs<double> w;
    plan_fused(p, m, n, max_pairs, bi, want_forces != 0, false, &w);
  }
  return p.off;
}

int fused_run(const tn_model *m, hipStream_t s, const Problem &pb, int prec, void *ws, size_t ws_bytes) {
  if (!pair_kernels_support(m->F, m->K, m->L, prec == TN_BF16)) return TN_E_UNSUPPORTED;
  if (prec == TN_FP32) return run_fused<false>(m, s, pb, ws, ws_bytes);
  if (prec == TN_BF16) return run_fused<true>(m, s, pb, ws, ws_bytes);
  return TN_E_UNSUPPORTED;
}

}  // namespace tn
