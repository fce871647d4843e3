// Adjoint of the update of Alg. 2 (tt_update: the likelihood TT of Sec. 2.2
// built on the device, H = L o P_pred and c_k = sum(H) delta, eq.
// pmf_filtrace_b), for tt_update_adjoint.  Composes the library's own
// adjoints: the log c_k term as the log-mass adjoint of H
// (tt_normalize_adjoint), tt_hadamard_adjoint, tt_likelihood_adjoint onto
// the dense likelihood, and the analytic measurement-parameter derivative
// (lik_theta_kernel).  Included by api.hip after grad_run.h.
#pragma once

namespace ttg {

// dst[f].status |= src[f].status
__global__ void upd_adj_or_status_kernel(const DevTT* __restrict__ src, const DevTT* __restrict__ dst, int nf) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < nf) *dst[f].status |= *src[f].status;
}

struct UpdAdj {
  int B = 0, d = 0, nth = 0, lcap = 1;
  std::vector<tt_train> L, PD, HZ, CB, HB, LB, PDB;
  std::vector<FilterConst> fcs;
  FilterConst* dfc = nullptr;
  DevTT* tab = nullptr;
  std::vector<int32_t*> statuses;
  int32_t** stab = nullptr;
  void* sub = nullptr;
  size_t sub_bytes = 0;
};

static tt_status upd_adj_plan(int32_t batch, const tt_grid* grids, const tt_meas* meas, const tt_train* p_pred,
                              const tt_train* h, int32_t lik_rank_cap, Arena& ar, UpdAdj& u) {
  if (batch < 1 || !grids || !meas || !p_pred || !h || lik_rank_cap < 1) {
    set_error("tt_update_adjoint: null pointer or bad size");
    return TT_ERR_ARG;
  }
  const int d = p_pred[0].d;
  u.B = batch;
  u.d = d;
  const bool range = meas[0].kind == 1;
  u.nth = range ? d + 4 : d + 1;
  u.L.resize(batch);
  u.PD.resize(batch);
  u.HZ.resize(batch);
  u.CB.resize(batch);
  u.HB.resize(batch);
  u.LB.resize(batch);
  u.PDB.resize(batch);
  u.fcs.resize(batch);
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_grid(&grids[b]));
    TT_TRY(check_train(&p_pred[b], "p_pred", TT_F64));
    TT_TRY(check_train(&h[b], "h", TT_F64));
    if (p_pred[b].d != d || grids[b].d != d || h[b].d != d || (meas[b].kind == 1) != range || (range && d < 2)) {
      set_error("tt_update_adjoint: filter %d: d or the measurement kind differs (range needs d >= 2)", b);
      return TT_ERR_SHAPE;
    }
    int n[TT_MAXD], lc[TT_MAXD + 1], dc[TT_MAXD + 1];
    for (int k = 0; k < d; ++k) {
      n[k] = grids[b].n[k];
      if (p_pred[b].n[k] != n[k] || h[b].n[k] != n[k]) {
        set_error("tt_update_adjoint: filter %d: modes differ from the grid", b);
        return TT_ERR_SHAPE;
      }
    }
    for (int j = 0; j <= d; ++j) {
      lc[j] = (range && j == 1) ? std::min(lik_rank_cap, n[1]) : 1;
      dc[j] = (range && j == 1) ? n[1] : 1;
      if (h[b].cap[j] < lc[j] * p_pred[b].cap[j] && j > 0 && j < d) {
        set_error("tt_update_adjoint: filter %d: h cap[%d] below the product's", b, j);
        return TT_ERR_SHAPE;
      }
    }
    u.L[b] = gr_take(ar, d, n, lc);
    u.PD[b] = gr_take(ar, d, n, dc);
    u.HZ[b] = gr_take(ar, d, n, h[b].cap);
    u.CB[b] = gr_take(ar, d, n, h[b].cap);
    u.HB[b] = gr_take(ar, d, n, h[b].cap);
    u.LB[b] = gr_take(ar, d, n, lc);
    u.PDB[b] = gr_take(ar, d, n, dc);
    for (const tt_train* t : {&u.L[b], &u.PD[b], &u.HZ[b], &u.CB[b], &u.HB[b], &u.LB[b], &u.PDB[b]})
      u.statuses.push_back(t->status);
    u.fcs[b] = make_const(grids[b], &meas[b]);
  }
  u.dfc = ar.take<FilterConst>(batch);
  u.tab = ar.take<DevTT>((size_t)2 * batch);
  u.stab = ar.take<int32_t*>(u.statuses.size());
  size_t need = 0;
  auto upd = [&](size_t s) { need = std::max(need, s); };
  int rmax = 1;
  for (int b = 0; b < batch; ++b)
    for (int j = 0; j <= d; ++j) rmax = std::max({rmax, h[b].cap[j], (int)u.PD[b].cap[j]});
  upd(tt_update_workspace(batch, grids, meas, u.L.data(), u.L.data(), lik_rank_cap));
  upd(tt_update_workspace(batch, grids, meas, u.PD.data(), u.PD.data(), 1));
  upd(tt_adjoint_workspace(batch, d, rmax));
  upd(tt_likelihood_adjoint_workspace(batch, meas, u.PD.data(), u.L.data()));
  u.sub_bytes = need + 4096;
  u.sub = ar.take<char>(u.sub_bytes);
  return TT_OK;
}

}  // namespace ttg

extern "C" {

size_t tt_update_adjoint_workspace(int32_t batch, const tt_grid* grids, const tt_meas* meas, const tt_train* p_pred,
                                   const tt_train* h, int32_t lik_rank_cap) {
  using namespace ttg;
  Arena ar(nullptr, 0);
  UpdAdj u;
  if (upd_adj_plan(batch, grids, meas, p_pred, h, lik_rank_cap, ar, u) != TT_OK) return 0;
  return ar.used + 256;
}

tt_status tt_update_adjoint(int32_t batch, const tt_grid* grids, const tt_meas* meas, const double* z_dev,
                            int32_t z_stride, const tt_train* p_pred, const tt_train* h, const tt_train* h_bar,
                            const double* log_c_bar_dev, int32_t lik_rank_cap, const tt_train* p_pred_bar,
                            double* theta_bar_dev, void* ws, size_t ws_bytes, void* stream) {
  using namespace ttg;
  if (!z_dev || z_stride < 1 || !p_pred_bar || !theta_bar_dev || !ws) {
    set_error("tt_update_adjoint: null pointer or bad z stride");
    return TT_ERR_ARG;
  }
  Arena ar(ws, ws_bytes);
  UpdAdj u;
  TT_TRY(upd_adj_plan(batch, grids, meas, p_pred, h, lik_rank_cap, ar, u));
  if (!ar.fits()) {
    set_error("tt_update_adjoint: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  const int B = batch;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(u.stab, u.statuses, st));
  hipLaunchKernelGGL(zero_status_kernel, dim3(cdiv((int)u.statuses.size(), 256)), dim3(256), 0, st, u.stab,
                     (int)u.statuses.size());
  TTG_LAUNCH_CHECK("zero_status_kernel");
  TT_TRY(upload(u.dfc, u.fcs, st));
  // the forward's likelihood TT and its dense input, rebuilt
  TT_TRY(tt_likelihood(B, grids, meas, z_dev, z_stride, u.L.data(), lik_rank_cap, u.sub, u.sub_bytes, st));
  TT_TRY(tt_likelihood_dense(B, grids, meas, z_dev, z_stride, u.PD.data(), u.sub, u.sub_bytes, st));
  // H's adjoint: h_bar plus the log c_k term (the log-mass adjoint of H)
  {
    std::vector<DevTT> v(2 * B);
    for (int b = 0; b < B; ++b) {
      v[b] = make_dev(h[b]);
      v[B + b] = make_dev(u.HZ[b]);
    }
    TT_TRY(upload(u.tab, v, st));
    long long most = 1;
    for (int b = 0; b < B; ++b) most = std::max(most, (long long)elems_of(u.d, u.HZ[b].n, u.HZ[b].cap));
    hipLaunchKernelGGL(adj_zero_kernel, dim3(std::max(1, std::min(64, cdiv(most, 256 * 4))), B), dim3(256), 0, st,
                       u.tab, u.tab + B);
    TTG_LAUNCH_CHECK("adj_zero_kernel");
  }
  TT_TRY(tt_normalize_adjoint(B, h, u.HZ.data(), log_c_bar_dev, u.CB.data(), u.sub, u.sub_bytes, st));
  if (h_bar) {
    TT_TRY(tt_adjoint_axpy(B, 1.0, h_bar, u.CB.data(), u.sub, u.sub_bytes, st));
  }
  // H = L o P_pred, then L = build(dense likelihood) and the parameters
  TT_TRY(tt_hadamard_adjoint(B, u.L.data(), p_pred, u.CB.data(), u.LB.data(), p_pred_bar, u.sub, u.sub_bytes, st));
  TT_TRY(tt_likelihood_adjoint(B, meas, u.PD.data(), u.L.data(), u.LB.data(), u.PDB.data(), u.sub, u.sub_bytes, st));
  {
    std::vector<DevTT> v(2 * B);
    for (int b = 0; b < B; ++b) {
      v[b] = make_dev(u.PD[b]);
      v[B + b] = make_dev(u.PDB[b]);
    }
    TT_TRY(upload(u.tab, v, st));
    hipLaunchKernelGGL(lik_theta_kernel, dim3(B), dim3(256), 0, st, u.tab, u.tab + B, u.dfc, z_dev,
                       (long long)z_stride, u.nth, theta_bar_dev);
    TTG_LAUNCH_CHECK("lik_theta_kernel");
  }
  // the internal trains' statuses (a rank mismatch or capacity) reach p_pred_bar
  {
    std::vector<DevTT> v(B);
    for (int b = 0; b < B; ++b) v[b] = make_dev(p_pred_bar[b]);
    TT_TRY(upload(u.tab, v, st));
    for (const auto* tv : {&u.L, &u.CB, &u.LB, &u.PDB}) {
      std::vector<DevTT> w(B);
      for (int b = 0; b < B; ++b) w[b] = make_dev((*tv)[b]);
      TT_TRY(upload(u.tab + B, w, st));
      hipLaunchKernelGGL(upd_adj_or_status_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, u.tab + B, u.tab, B);
      TTG_LAUNCH_CHECK("upd_adj_or_status_kernel");
    }
  }
  return TT_OK;
}

}  // extern "C"
