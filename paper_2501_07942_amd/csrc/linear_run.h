// The point-mass filter for linear dynamics x_{k+1} = F x_k + w_k on
// re-designed grids (Alg. 3 with the grid re-design of Alg. 4), FP64:
// tt_interpolate_lattice (the second interpolation of Alg. 3, by TT-cross)
// and tt_filter_run_linear (the recursion).  Included by api.hip after
// cross.h.
#pragma once

namespace ttg {

// Gauss-Jordan inverse with partial pivoting of a general d x d matrix and
// its determinant; false when it is singular to working precision.
static bool invert_general(int d, const double* m, double* inv, double* det) {
  double a[TT_MAXD][2 * TT_MAXD];
  double amax = 0.0;
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < 2 * d; ++j) {
      a[i][j] = (j < d) ? m[i * d + j] : (j - d == i ? 1.0 : 0.0);
      if (j < d) amax = std::max(amax, std::fabs(a[i][j]));
    }
  double dt = 1.0;
  for (int c = 0; c < d; ++c) {
    int p = c;
    for (int i = c + 1; i < d; ++i)
      if (std::fabs(a[i][c]) > std::fabs(a[p][c])) p = i;
    if (!(std::fabs(a[p][c]) > 1e-14 * amax)) return false;
    if (p != c) {
      for (int j = 0; j < 2 * d; ++j) std::swap(a[p][j], a[c][j]);
      dt = -dt;
    }
    const double piv = a[c][c];
    dt *= piv;
    for (int j = 0; j < 2 * d; ++j) a[c][j] /= piv;
    for (int i = 0; i < d; ++i)
      if (i != c) {
        const double fct = a[i][c];
        for (int j = 0; j < 2 * d; ++j) a[i][j] -= fct * a[c][j];
      }
  }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) inv[i * d + j] = a[i][d + j];
  *det = dt;
  return true;
}

static tt_status lattice_args(int32_t batch, const double* f, const tt_grid* lattice, const tt_grid* to,
                              const tt_train* in, const tt_train* out, int* n) {
  if (batch < 1 || !f || !lattice || !to || !in || !out) {
    set_error("tt_interpolate_lattice: null argument");
    return TT_ERR_ARG;
  }
  const int d = to[0].d;
  if (d < 2 || d > 6) {
    set_error("tt_interpolate_lattice: d = %d out of range [2, 6]", d);
    return TT_ERR_SHAPE;
  }
  for (int k = 0; k < d; ++k) n[k] = to[0].n[k];
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_grid(&lattice[b]));
    TT_TRY(check_grid(&to[b]));
    TT_TRY(check_train(&in[b], "in", TT_F64));
    TT_TRY(check_train(&out[b], "out", out[0].dtype));
    if (lattice[b].d != d || to[b].d != d || in[b].d != d || out[b].d != d) {
      set_error("tt_interpolate_lattice: d differs");
      return TT_ERR_SHAPE;
    }
    for (int k = 0; k < d; ++k) {
      if (to[b].n[k] != n[k] || out[b].n[k] != n[k] || in[b].n[k] != lattice[b].n[k] || lattice[b].n[k] < 2) {
        set_error("tt_interpolate_lattice: filter %d: modes differ from the grids (or the target grids' sizes "
                  "differ within the batch)", b);
        return TT_ERR_SHAPE;
      }
    }
    for (int j = 0; j <= d; ++j)
      if (in[b].cap[j] > 32) {
        set_error("tt_interpolate_lattice: input rank capacity %d > 32", in[b].cap[j]);
        return TT_ERR_SHAPE;
      }
  }
  return TT_OK;
}

static tt_status lattice_fns(int32_t batch, const double* f, const tt_grid* lattice, const tt_grid* to,
                             const tt_train* in, std::vector<CrossInterpFn>& fns) {
  const int d = to[0].d;
  fns.resize(batch);
  for (int b = 0; b < batch; ++b) {
    CrossInterpFn& F = fns[b];
    memset(&F, 0, sizeof(F));
    F.d = d;
    double fd[TT_MAXD * TT_MAXD], det = 0.0;
    for (int l = 0; l < d; ++l) {
      const double dxl = (lattice[b].hi[l] - lattice[b].lo[l]) / (double)(lattice[b].n[l] - 1);
      for (int m = 0; m < d; ++m) fd[m * d + l] = f[m * d + l] * dxl;  // F diag(dx_lattice)
      F.lo[l] = to[b].lo[l];
      F.dx[l] = (to[b].hi[l] - to[b].lo[l]) / (double)(to[b].n[l] - 1);
    }
    if (!invert_general(d, fd, F.a, &det)) {
      set_error("tt_interpolate_lattice: F is singular");
      return TT_ERR_ARG;
    }
    for (int m = 0; m < d; ++m) {
      double s = 0.0;
      for (int l = 0; l < d; ++l) s += f[m * d + l] * lattice[b].lo[l];
      F.c[m] = s;
    }
    F.src = make_dev(in[b]);
  }
  return TT_OK;
}

}  // namespace ttg

extern "C" {

size_t tt_interpolate_lattice_workspace(int32_t batch, const tt_grid* to, const tt_train* out, int32_t max_rank) {
  using namespace ttg;
  if (batch < 1 || !to || !out || max_rank < 1) return 0;
  const int d = to[0].d;
  if (d < 2 || d > 6) return 0;
  Arena ar(nullptr, 0);
  CrossPlan p;
  if (cross_plan(batch, d, to[0].n, max_rank, sizeof(CrossInterpFn), out, ar, p) != TT_OK) return 0;
  return ar.used + 256;
}

tt_status tt_interpolate_lattice(int32_t batch, const double* f, const tt_grid* lattice, const tt_grid* to,
                                 const tt_train* in, double tol, int32_t max_rank, const tt_train* out, void* ws,
                                 size_t ws_bytes, void* stream) {
  using namespace ttg;
  int n[TT_MAXD];
  TT_TRY(lattice_args(batch, f, lattice, to, in, out, n));
  if (!ws || !(tol > 0.0) || max_rank < 1 || max_rank > CROSS_RMAX) {
    set_error("tt_interpolate_lattice: bad arguments (need tol > 0 and 1 <= max_rank <= %d)", CROSS_RMAX);
    return TT_ERR_ARG;
  }
  Arena ar(ws, ws_bytes);
  CrossPlan p;
  TT_TRY(cross_plan(batch, to[0].d, n, max_rank, sizeof(CrossInterpFn), out, ar, p));
  if (!ar.fits()) {
    set_error("tt_interpolate_lattice: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  std::vector<CrossInterpFn> fns;
  TT_TRY(lattice_fns(batch, f, lattice, to, in, fns));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(cross_run(p, fns, tol, max_rank, out, st));
  std::vector<DevTT> v(2 * batch);
  for (int b = 0; b < batch; ++b) {
    v[b] = make_dev(in[b]);
    v[batch + b] = make_dev(out[b]);
  }
  TT_TRY(upload(p.tab, v, st));
  hipLaunchKernelGGL(cross_add_log_scale_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, p.tab, p.tab + batch, batch);
  TTG_LAUNCH_CHECK("cross_add_log_scale_kernel");
  return TT_OK;
}

}  // extern "C"

namespace ttg {

// copy a [B][w] block into column block k of a [B][K][w] array
__global__ void scatter_step_kernel(const double* __restrict__ src, double* __restrict__ dst, int nf, int K, int k,
                                    int w) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nf * w) return;
  const int f = e / w, j = e % w;
  dst[((long long)f * K + k) * w + j] = src[e];
}

// kernel TT scale 1 / |det F| (the change of variables of the time update)
__global__ void add_log_kernel(const DevTT* __restrict__ t, int nf, double v) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < nf) *t[f].log_scale += v;
}

struct LinRun {
  int B = 0, d = 0, K = 0, N = 0, cap = 1, kcap = 1, lcap = 1, hmax = 0;
  double eps = 0.0;
  std::vector<tt_train> P, Ph, Kt, X, Pt, Pn, H;
  double *mean = nullptr, *cov = nullptr, *lm = nullptr, *lc = nullptr;
  void* sub = nullptr;
  size_t sub_bytes = 0;
  DevTT* tab = nullptr;
};

static tt_status lin_plan(int32_t batch, const tt_filter_spec* specs, int32_t K, Arena& ar, LinRun& g) {
  if (batch < 1 || !specs || K < 1) {
    set_error("tt_filter_run_linear: bad arguments");
    return TT_ERR_ARG;
  }
  const int d = specs[0].grid.d;
  if (d < 2 || d > 6) {
    set_error("tt_filter_run_linear: d = %d out of range [2, 6]", d);
    return TT_ERR_SHAPE;
  }
  g.B = batch;
  g.d = d;
  g.K = K;
  g.N = specs[0].grid.n[0];
  g.cap = specs[0].cap;
  g.kcap = specs[0].kernel_cap;
  g.eps = specs[0].eps;
  for (int b = 0; b < batch; ++b) {
    const tt_filter_spec& s = specs[b];
    TT_TRY(check_grid(&s.grid));
    bool same = s.grid.d == d && s.cap == g.cap && s.kernel_cap == g.kcap && s.eps == g.eps &&
                s.lik_rank_cap == specs[0].lik_rank_cap && s.meas.kind == specs[0].meas.kind;
    for (int k = 0; k < d; ++k) same = same && s.grid.n[k] == g.N;
    if (!same) {
      set_error("tt_filter_run_linear: filter %d: d, N (the same on every axis), cap, kernel_cap, eps, "
                "lik_rank_cap and the measurement kind must be shared by the batch", b);
      return TT_ERR_SHAPE;
    }
    if (s.cap < 1 || s.cap > 32 || s.kernel_cap < 1 || s.kernel_cap > 32 || !(s.eps >= 0.0)) {
      set_error("tt_filter_run_linear: cap and kernel_cap in [1, 32], eps >= 0 required");
      return TT_ERR_ARG;
    }
  }
  g.hmax = g.N - 1;
  g.lcap = specs[0].meas.kind == 1 ? std::min(specs[0].lik_rank_cap, g.N) : 1;
  int nn[TT_MAXD], kt[TT_MAXD], pc[TT_MAXD + 1], kc[TT_MAXD + 1], xc[TT_MAXD + 1], hc[TT_MAXD + 1],
      cc[TT_MAXD + 1];
  for (int k = 0; k < d; ++k) {
    nn[k] = g.N;
    kt[k] = 2 * g.hmax + 1;
  }
  for (int j = 0; j <= d; ++j) {
    const bool e = j == 0 || j == d;
    pc[j] = e ? 1 : g.cap;
    kc[j] = e ? 1 : g.kcap;
    xc[j] = pc[j] * kc[j];
    hc[j] = (j == 1 ? g.lcap : 1) * pc[j];
    cc[j] = e ? 1 : 64;
  }
  g.P.resize(batch);
  g.Ph.resize(batch);
  g.Kt.resize(batch);
  g.X.resize(batch);
  g.Pt.resize(batch);
  g.Pn.resize(batch);
  g.H.resize(batch);
  for (int b = 0; b < batch; ++b) {
    g.P[b] = cross_train(ar, d, nn, pc);
    g.Ph[b] = cross_train(ar, d, nn, pc);
    g.Kt[b] = cross_train(ar, d, kt, kc);
    g.X[b] = cross_train(ar, d, nn, xc);
    g.Pt[b] = cross_train(ar, d, nn, pc);
    g.Pn[b] = cross_train(ar, d, nn, cc);
    g.H[b] = cross_train(ar, d, nn, hc);
  }
  g.mean = ar.take<double>((size_t)batch * d);
  g.cov = ar.take<double>((size_t)batch * d * d);
  g.lm = ar.take<double>(batch);
  g.lc = ar.take<double>(batch);
  g.tab = ar.take<DevTT>((size_t)7 * batch);
  // the sub-calls' workspace
  std::vector<tt_grid> grids(batch);
  std::vector<tt_meas> meas(batch);
  for (int b = 0; b < batch; ++b) {
    grids[b] = specs[b].grid;
    meas[b] = specs[b].meas;
  }
  size_t need = 0;
  auto upd = [&](size_t s) { need = std::max(need, s); };
  upd(tt_normalize_moments_workspace(batch, g.P.data()));
  upd(tt_grid_redesign_workspace(batch, d));
  upd(tt_interpolate_workspace(batch));
  upd(tt_kernel_build_cross_workspace(batch, grids.data(), std::vector<int32_t>(d, g.hmax).data(), g.Kt.data()));
  upd(tt_predict_workspace(batch));
  upd(tt_round_workspace(batch, g.X.data(), g.Pt.data()));
  upd(tt_round_workspace(batch, g.Pn.data(), g.P.data()));
  upd(tt_round_workspace(batch, g.H.data(), g.P.data()));
  upd(tt_interpolate_lattice_workspace(batch, grids.data(), g.Pn.data(), 64));
  upd(tt_update_workspace(batch, grids.data(), meas.data(), g.P.data(), g.H.data(), specs[0].lik_rank_cap));
  upd((size_t)2 * batch * 4096 + 4096);  // tt_prior
  g.sub_bytes = need + 4096;
  g.sub = ar.take<char>(g.sub_bytes);
  return TT_OK;
}

}  // namespace ttg

extern "C" {

size_t tt_filter_run_linear_workspace(int32_t batch, const tt_filter_spec* specs, int32_t K) {
  using namespace ttg;
  Arena ar(nullptr, 0);
  LinRun g;
  if (lin_plan(batch, specs, K, ar, g) != TT_OK) return 0;
  return ar.used + 256;
}

tt_status tt_filter_run_linear(int32_t batch, const tt_filter_spec* specs, const double* f, const double* q,
                               double nsigma, double kernel_nsigma, double kernel_tol, const double* z_dev,
                               int32_t zdim, int32_t K, double* loglik_dev, double* log_c_dev, double* log_mpred_dev,
                               double* mean_dev, double* cov_dev, double* grids_out, int32_t* status_dev, void* ws,
                               size_t ws_bytes, void* stream) {
  using namespace ttg;
  if (!f || !q || !z_dev || zdim < 1 || !loglik_dev || !log_c_dev || !log_mpred_dev || !status_dev || !ws ||
      !(nsigma > 0.0) || !(kernel_nsigma > 0.0) || !(kernel_tol > 0.0)) {
    set_error("tt_filter_run_linear: null pointer or non-positive parameter");
    return TT_ERR_ARG;
  }
  Arena ar(ws, ws_bytes);
  LinRun g;
  TT_TRY(lin_plan(batch, specs, K, ar, g));
  if (!ar.fits()) {
    set_error("tt_filter_run_linear: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  const int B = batch, d = g.d;
  // the model: F^{-1}, |det F|, Q_e = F^{-1} Q F^{-T} (the kernel's covariance
  // in the coordinates of the grid re-designed before the time update)
  double finv[TT_MAXD * TT_MAXD], detf = 0.0;
  if (!invert_general(d, f, finv, &detf)) {
    set_error("tt_filter_run_linear: F is singular");
    return TT_ERR_ARG;
  }
  std::vector<double> qe((size_t)d * d, 0.0);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) {
      double s = 0.0;
      for (int a = 0; a < d; ++a)
        for (int c = 0; c < d; ++c) s += finv[i * d + a] * q[a * d + c] * finv[j * d + c];
      qe[(size_t)i * d + j] = s;
    }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::vector<tt_grid> grids(B), hat(B);
  std::vector<tt_meas> meas(B);
  std::vector<double> m0((size_t)B * d), p0((size_t)B * d);
  for (int b = 0; b < B; ++b) {
    grids[b] = specs[b].grid;
    meas[b] = specs[b].meas;
    for (int l = 0; l < d; ++l) {
      m0[(size_t)b * d + l] = specs[b].m0[l];
      p0[(size_t)b * d + l] = specs[b].p0_diag[l];
    }
  }
  HIP_TRY(hipMemsetAsync(status_dev, 0, B * sizeof(int32_t), st), "status");
  {  // the trains' status words start clear (the roundings OR bits in)
    std::vector<DevTT> v;
    for (const auto* tv : {&g.P, &g.Ph, &g.Kt, &g.X, &g.Pt, &g.Pn, &g.H})
      for (int b = 0; b < B; ++b) v.push_back(make_dev((*tv)[b]));
    TT_TRY(upload(g.tab, v, st));
    hipLaunchKernelGGL(cross_clear_status_kernel, dim3(cdiv((int)v.size(), 64)), dim3(64), 0, st, g.tab,
                       (int)v.size());
    TTG_LAUNCH_CHECK("cross_clear_status_kernel");
  }
  hipLaunchKernelGGL(fill_kernel, dim3(cdiv((long long)B * K, 256)), dim3(256), 0, st, log_mpred_dev,
                     (long long)B * K, 1LL, 0.0);
  TTG_LAUNCH_CHECK("fill_kernel");
  TT_TRY(tt_prior(B, grids.data(), m0.data(), p0.data(), g.P.data(), g.sub, g.sub_bytes, st));
  TT_TRY(tt_normalize_moments(B, grids.data(), g.P.data(), g.lm, nullptr, nullptr, g.sub, g.sub_bytes, st));
  const int zs = K * zdim;
  for (int k = 0; k < K; ++k) {
    if (k > 0) {
      // grid re-design before the time update (Alg. 4): moments, local
      // prediction, sigma box, corners through F^{-1}, bounding box
      TT_TRY(tt_normalize_moments(B, grids.data(), g.P.data(), g.lm, g.mean, g.cov, g.sub, g.sub_bytes, st));
      TT_TRY(tt_grid_redesign(B, d, f, q, nsigma, g.mean, g.cov, grids.data(), hat.data(), g.sub, g.sub_bytes, st));
      TT_TRY(tt_interpolate(B, grids.data(), hat.data(), g.P.data(), g.Ph.data(), g.sub, g.sub_bytes, st));
      // the time-update kernel on the re-designed grid: N(F (dx o m); 0, Q) dx^d
      // = N(dx o m; 0, Q_e) dx^d / |det F| on the box of kernel_nsigma sigma
      std::vector<int32_t> hw(d);
      for (int l = 0; l < d; ++l) {
        double dxmin = 1e300;
        for (int b = 0; b < B; ++b)
          dxmin = std::min(dxmin, (hat[b].hi[l] - hat[b].lo[l]) / (double)(hat[b].n[l] - 1));
        hw[l] = std::min(g.hmax, (int)std::floor(kernel_nsigma * std::sqrt(qe[(size_t)l * d + l]) / dxmin));
      }
      std::vector<tt_train> kt(B);
      for (int b = 0; b < B; ++b) {
        kt[b] = g.Kt[b];
        for (int l = 0; l < d; ++l) kt[b].n[l] = 2 * hw[l] + 1;
      }
      std::vector<double> qes((size_t)B * d * d);
      for (int b = 0; b < B; ++b)
        for (int e = 0; e < d * d; ++e) qes[(size_t)b * d * d + e] = qe[e];
      // (working rank 64; the kernel trains' capacities kernel_cap cap the result)
      TT_TRY(tt_kernel_build_cross(B, hat.data(), qes.data(), hw.data(), kernel_tol, 64, kt.data(), g.sub,
                                   g.sub_bytes, st));
      {
        std::vector<DevTT> v(B);
        for (int b = 0; b < B; ++b) v[b] = make_dev(kt[b]);
        TT_TRY(upload(g.tab, v, st));
        hipLaunchKernelGGL(add_log_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, g.tab, B, -std::log(std::fabs(detf)));
        TTG_LAUNCH_CHECK("add_log_kernel");
      }
      // time update on the lattice F xi(hat), then rounding
      TT_TRY(tt_predict(B, kt.data(), g.Ph.data(), g.X.data(), g.sub, g.sub_bytes, st));
      TT_TRY(tt_round(B, g.X.data(), g.Pt.data(), g.eps, g.cap, g.sub, g.sub_bytes, st));
      // grid re-design after it: the box of the lattice's corners, and the
      // interpolation onto that box (TT-cross), rounded and normalised
      for (int b = 0; b < B; ++b) {
        tt_grid& gn = grids[b];
        gn = hat[b];
        for (int l = 0; l < d; ++l) {
          double c = 0.0, h = 0.0;
          for (int m = 0; m < d; ++m) {
            c += f[l * d + m] * 0.5 * (hat[b].lo[m] + hat[b].hi[m]);
            h += std::fabs(f[l * d + m]) * 0.5 * (hat[b].hi[m] - hat[b].lo[m]);
          }
          gn.lo[l] = c - h;
          gn.hi[l] = c + h;
        }
      }
      TT_TRY(tt_interpolate_lattice(B, f, hat.data(), grids.data(), g.Pt.data(), kernel_tol, 64, g.Pn.data(), g.sub,
                                    g.sub_bytes, st));
      TT_TRY(tt_round(B, g.Pn.data(), g.P.data(), g.eps, g.cap, g.sub, g.sub_bytes, st));
      TT_TRY(tt_normalize_moments(B, grids.data(), g.P.data(), g.lm, nullptr, nullptr, g.sub, g.sub_bytes, st));
      hipLaunchKernelGGL(scatter_step_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, g.lm, log_mpred_dev, B, K, k, 1);
      TTG_LAUNCH_CHECK("scatter_step_kernel");
    }
    // the update of Alg. 2 on the current grid
    TT_TRY(tt_update(B, grids.data(), meas.data(), z_dev + (long long)k * zdim, zs, g.P.data(), g.H.data(),
                     specs[0].lik_rank_cap, g.lc, g.sub, g.sub_bytes, st));
    hipLaunchKernelGGL(scatter_step_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, g.lc, log_c_dev, B, K, k, 1);
    TTG_LAUNCH_CHECK("scatter_step_kernel");
    TT_TRY(tt_round(B, g.H.data(), g.P.data(), g.eps, g.cap, g.sub, g.sub_bytes, st));
    TT_TRY(tt_normalize_moments(B, grids.data(), g.P.data(), g.lm, g.mean, g.cov, g.sub, g.sub_bytes, st));
    if (mean_dev) {
      hipLaunchKernelGGL(scatter_step_kernel, dim3(cdiv(B * d, 64)), dim3(64), 0, st, g.mean, mean_dev, B, K, k, d);
      TTG_LAUNCH_CHECK("scatter_step_kernel");
    }
    if (cov_dev) {
      hipLaunchKernelGGL(scatter_step_kernel, dim3(cdiv(B * d * d, 64)), dim3(64), 0, st, g.cov, cov_dev, B, K, k,
                         d * d);
      TTG_LAUNCH_CHECK("scatter_step_kernel");
    }
    if (grids_out)
      for (int b = 0; b < B; ++b)
        for (int l = 0; l < d; ++l) {
          grids_out[((size_t)b * K + k) * 2 * d + l] = grids[b].lo[l];
          grids_out[((size_t)b * K + k) * 2 * d + d + l] = grids[b].hi[l];
        }
    std::vector<DevTT> v(B);
    for (int b = 0; b < B; ++b) v[b] = make_dev(g.P[b]);
    TT_TRY(upload(g.tab, v, st));
    hipLaunchKernelGGL(copy_status_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, g.tab, B, status_dev);
    TTG_LAUNCH_CHECK("copy_status_kernel");
  }
  hipLaunchKernelGGL(loglik_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, log_c_dev, K, K, B, loglik_dev);
  TTG_LAUNCH_CHECK("loglik_kernel");
  HIP_TRY(hipStreamSynchronize(st), "tt_filter_run_linear sync");
  return TT_OK;
}

}  // extern "C"
