// The differentiated recursion behind tt_filter_run_taped and
// tt_filter_run_adjoint: LL = sum_k log c_k (Sec. 2.2, eq. pmf_filtrace_b)
// and dLL/dtheta, composed from the library's forward and adjoint entry
// points in the loop order of Alg. 2 (materialised prediction of Sec. 4.2,
// rounding of Sec. 4.1 'round' at the forward's ranks).  Included by api.hip
// after the entry points it calls.
#pragma once

namespace ttg {

// ---------------------------------------------------------------------------
// device pieces of the parameter gradient
// ---------------------------------------------------------------------------

// Zero adjoint of src's layout: dst gets src's ranks, zero cores over its
// capacity, zero log-scale, status 0.
__global__ void adj_zero_kernel(const DevTT* __restrict__ src, const DevTT* __restrict__ dst) {
  const int f = blockIdx.y;
  const DevTT &S = src[f], &D = dst[f];
  long long tot = 0;
  for (int k = 0; k < D.d; ++k) tot += (long long)D.cap[k] * D.n[k] * D.cap[k + 1];
  double* c = reinterpret_cast<double*>(D.cores);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x)
    c[e] = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int j = 0; j <= D.d; ++j) D.ranks[j] = S.ranks[j];
    *D.log_scale = 0.0;
    *D.status = 0;
  }
}

// clears the status words of the run's trains (some builders only OR bits in)
__global__ void zero_status_kernel(int32_t* const* __restrict__ p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) *p[i] = 0;
}

// status[f] |= every train's status word (trains f, nf + f, 2 nf + f, ...)
__global__ void or_status_kernel(const DevTT* __restrict__ t, int nf, int ntr, int* __restrict__ status) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  int s = status[f];
  for (int j = 0; j < ntr; ++j) s |= *t[(long long)j * nf + f].status;
  status[f] = s;
}

// TT_STATUS_CAPACITY on status[f] when b's ranks differ from a's
__global__ void rank_match_kernel(const DevTT* __restrict__ a, const DevTT* __restrict__ b, int nf,
                                  int* __restrict__ status) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  bool same = true;
  for (int j = 0; j <= a[f].d; ++j) same = same && a[f].ranks[j] == b[f].ranks[j];
  if (!same) status[f] |= TT_STATUS_CAPACITY;
}

// loglik[f] = sum_k log_c[k * nf + f]
__global__ void grad_loglik_kernel(const double* __restrict__ log_c, int K, int nf, double* __restrict__ out) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  double s = 0.0;
  for (int k = 0; k < K; ++k) s += log_c[(long long)k * nf + f];
  out[f] = s;
}

// theta_bar[f * nth + j] = (v[(2j) nf + f] - v[(2j+1) nf + f]) / (2 h[j nf + f]), j < d
__global__ void kernel_theta_kernel(const double* __restrict__ v, const double* __restrict__ h, int d, int nf,
                                    int nth, double* __restrict__ theta_bar) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  for (int j = 0; j < d; ++j)
    theta_bar[(long long)f * nth + j] =
        (v[(long long)(2 * j) * nf + f] - v[(long long)(2 * j + 1) * nf + f]) / (2.0 * h[(long long)j * nf + f]);
}

// Measurement-parameter gradient of one step from the adjoint pbar of the
// dense likelihood train p (tt_likelihood_dense): the stored factor C_k of
// p is F_k / m_k with F_k the Gaussian factor (constants included) and
// m_k = F_k at its largest entry, and log_scale = sum_k log m_k, so
//   dL/dtheta = sum_k <Cbar_k, C_k (x) dlog F_k> - dlog F_k(argmax) (<Cbar_k, C_k> - lsbar)
// (the second term vanishes in exact arithmetic when L depends on the
// represented tensor only).  Range block: log F = -r^2/(2 sr^2) + const,
// r = z - rho, rho = ||xi - s||; linear factor: e = z - xi with sigma_lin.
// Accumulates into theta_bar[f * nth + d + ...] (sigma_r, sigma_lin, s1, s2
// for the range model; sigma_lin for the linear one).  One workgroup per
// filter, fixed summation order.
__global__ void __launch_bounds__(256) lik_theta_kernel(const DevTT* __restrict__ pd, const DevTT* __restrict__ pdb,
                                                        const FilterConst* __restrict__ fc,
                                                        const double* __restrict__ z, long long zstride, int nth,
                                                        double* __restrict__ theta_bar) {
  const int f = blockIdx.x;
  const DevTT &P = pd[f], &Pb = pdb[f];
  const FilterConst& C = fc[f];
  const double* zf = z + f * zstride;
  __shared__ double red[8];
  __shared__ double smax[256];
  __shared__ int sidx[256];
  const int tid = threadIdx.x;
  const double lsbar = *Pb.log_scale;
  double* tb = theta_bar + (long long)f * nth + C.d;
  const int first_lin = (C.meas_kind == 0) ? 0 : 2;
  const double sl = C.sigma_lin;
  double acc_lin = 0.0;
  for (int k = first_lin; k < C.d; ++k) {
    const double zk = zf[C.meas_kind == 0 ? k : k - 1];
    const int n = C.n[k];
    const double* c = core_ptr<double>(P, k);
    const double* cb = core_ptr<double>(Pb, k);
    double s_t = 0.0, s_d = 0.0, mx = -1.0;
    int im = 0;
    for (int i = tid; i < n; i += blockDim.x) {
      const double e = zk - (C.lo[k] + i * C.dx[k]);
      const double dl = e * e / (sl * sl * sl) - 1.0 / sl;
      s_t += cb[i] * c[i] * dl;
      s_d += cb[i] * c[i];
      if (c[i] > mx) {
        mx = c[i];
        im = i;
      }
    }
    smax[tid] = mx;
    sidx[tid] = im;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o && (smax[tid + o] > smax[tid] || (smax[tid + o] == smax[tid] && sidx[tid + o] < sidx[tid]))) {
        smax[tid] = smax[tid + o];
        sidx[tid] = sidx[tid + o];
      }
      __syncthreads();
    }
    const int ia = sidx[0];
    __syncthreads();
    s_t = block_sum(s_t, red);
    s_d = block_sum(s_d, red);
    const double ea = zk - (C.lo[k] + ia * C.dx[k]);
    acc_lin += s_t - (ea * ea / (sl * sl * sl) - 1.0 / sl) * (s_d - lsbar);
  }
  if (C.meas_kind == 0) {
    if (tid == 0) tb[0] += acc_lin;
    return;
  }
  // range block: core 0 of p is (1, n0, n1), entry (i, j) at i * n1 + j
  const int n0 = C.n[0], n1 = C.n[1];
  const double sr = C.sigma_r, zr = zf[0];
  const double* c = core_ptr<double>(P, 0);
  const double* cb = core_ptr<double>(Pb, 0);
  double t_sr = 0.0, t_s1 = 0.0, t_s2 = 0.0, s_d = 0.0, mx = -1.0;
  int im = 0;
  for (int e = tid; e < n0 * n1; e += blockDim.x) {
    const int i = e / n1, j = e % n1;
    const double x1 = C.lo[0] + i * C.dx[0] - C.sensor[0];
    const double x2 = C.lo[1] + j * C.dx[1] - C.sensor[1];
    const double rho = sqrt(x1 * x1 + x2 * x2);
    const double r = zr - rho;
    const double w = cb[e] * c[e];
    t_sr += w * (r * r / (sr * sr * sr) - 1.0 / sr);
    if (rho > 0.0) {
      t_s1 += w * (-(r / (sr * sr)) * x1 / rho);
      t_s2 += w * (-(r / (sr * sr)) * x2 / rho);
    }
    s_d += w;
    if (c[e] > mx) {
      mx = c[e];
      im = e;
    }
  }
  smax[tid] = mx;
  sidx[tid] = im;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o && (smax[tid + o] > smax[tid] || (smax[tid + o] == smax[tid] && sidx[tid + o] < sidx[tid]))) {
      smax[tid] = smax[tid + o];
      sidx[tid] = sidx[tid + o];
    }
    __syncthreads();
  }
  const int ea = sidx[0];
  __syncthreads();
  t_sr = block_sum(t_sr, red);
  t_s1 = block_sum(t_s1, red);
  t_s2 = block_sum(t_s2, red);
  s_d = block_sum(s_d, red);
  if (tid == 0) {
    const int i = ea / n1, j = ea % n1;
    const double x1 = C.lo[0] + i * C.dx[0] - C.sensor[0];
    const double x2 = C.lo[1] + j * C.dx[1] - C.sensor[1];
    const double rho = sqrt(x1 * x1 + x2 * x2);
    const double r = zr - rho;
    const double g = s_d - lsbar;
    tb[0] += t_sr - (r * r / (sr * sr * sr) - 1.0 / sr) * g;
    tb[1] += acc_lin;
    tb[2] += t_s1 - (rho > 0.0 ? -(r / (sr * sr)) * x1 / rho : 0.0) * g;
    tb[3] += t_s2 - (rho > 0.0 ? -(r / (sr * sr)) * x2 / rho : 0.0) * g;
  }
}

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------

using Batch = std::vector<tt_train>;

struct GradRun {
  // shape
  int B = 0, d = 0, K = 0, C = 1, nth = 0;
  bool taped = false, range = false;
  double eps = 0.0;
  int cap = 0, lik_cap = 0;
  std::vector<tt_grid> grids;
  std::vector<tt_meas> meas;
  std::vector<FilterConst> fcs;
  std::vector<double> qs, m0, p0;
  std::vector<int32_t> hw;
  double ktol = 0.0;
  bool cross = false;  // kernel TTs by TT-cross (the dense tensor is out of reach)
  int npert = 1;       // perturbed kernel builds per call (all 2d at once for TT-cross)
  int* kranks = nullptr;  // [npert * B][TT_MAXD + 1] the base kernels' ranks (device)
  int* kstate = nullptr;  // [B][CROSS_STATE_INTS] the base crosses' index sets (device)
  // persistent trains
  Batch kern, kbar, kp;
  double* logc = nullptr;   // [K][B]
  double* vals = nullptr;   // [2d][B] kernel-tangent inner products
  double* hstep = nullptr;  // [d][B] difference steps
  double* lmass = nullptr;  // [B]
  std::vector<Batch> pt, lik, h, hr, ckpt;  // [K] (taped) / ckpt at segment ends
  std::vector<std::vector<tt_round_tape>> xtape, htape;
  // one step's temporaries
  Batch X, xbar, hrbar, hbar, cbar, hzero, lbar, ppbar, ptbar, pbar, pbar2, kb, pd, pdbar;
  Batch s_pt, s_lik, s_h, s_hr;
  std::vector<Batch> seg;   // filtering densities inside a recomputed segment
  DevTT* tab = nullptr;     // device descriptor tables of this file's kernels
  FilterConst* dfc = nullptr;
  int tab_n = 0;
  void* sub = nullptr;      // workspace of the sub-calls
  size_t sub_bytes = 0;
  std::vector<int32_t*> statuses;  // every train's status word
  int32_t** stab = nullptr;        // the same on the device
};

// a train of the given capacities carved from the arena (pointers are
// placeholders when the arena only measures)
static tt_train gr_take(Arena& ar, int d, const int* n, const int* cap) {
  tt_train t;
  memset(&t, 0, sizeof(t));
  t.d = d;
  for (int k = 0; k < d; ++k) t.n[k] = n[k];
  for (int j = 0; j <= d; ++j) t.cap[j] = cap[j];
  t.dtype = TT_F64;
  char* fake = reinterpret_cast<char*>(4096);
  void* c = ar.take<double>(elems_of(d, n, cap));
  void* r = ar.take<int32_t>(TT_MAXD + 1);
  void* l = ar.take<double>(1);
  void* s = ar.take<int32_t>(1);
  t.cores = ar.base ? c : fake;
  t.ranks = reinterpret_cast<int32_t*>(ar.base ? r : fake);
  t.log_scale = reinterpret_cast<double*>(ar.base ? l : fake);
  t.status = reinterpret_cast<int32_t*>(ar.base ? s : fake);
  return t;
}

static Batch gr_batch(Arena& ar, GradRun& g, const std::vector<std::array<int, TT_MAXD + 1>>& caps,
                      const std::vector<std::array<int, TT_MAXD>>& ns) {
  Batch out(g.B);
  for (int b = 0; b < g.B; ++b) {
    out[b] = gr_take(ar, g.d, ns[b].data(), caps[b].data());
    g.statuses.push_back(out[b].status);
  }
  return out;
}

static tt_round_tape gr_tape(Arena& ar, const tt_train& in) {
  tt_round_tape tp;
  memset(&tp, 0, sizeof(tp));
  char* fake = reinterpret_cast<char*>(4096);
  for (int j = 1; j < in.d; ++j) {
    const int c = (j == 1) ? std::min(in.cap[1], in.n[0]) : in.cap[j];
    double* g = ar.take<double>((size_t)c * c);
    double* f = ar.take<double>((size_t)c * c);
    double* v = ar.take<double>((size_t)c * c);
    double* s = ar.take<double>(c);
    tp.g[j] = ar.base ? g : reinterpret_cast<double*>(fake);
    tp.f[j] = ar.base ? f : reinterpret_cast<double*>(fake);
    tp.v[j] = ar.base ? v : reinterpret_cast<double*>(fake);
    tp.s[j] = ar.base ? s : reinterpret_cast<double*>(fake);
  }
  int32_t* va = ar.take<int32_t>(TT_MAXD + 1);
  int32_t* rk = ar.take<int32_t>(TT_MAXD + 1);
  tp.valid = ar.base ? va : reinterpret_cast<int32_t*>(fake);
  tp.rank = ar.base ? rk : reinterpret_cast<int32_t*>(fake);
  return tp;
}

static std::vector<tt_round_tape> gr_tapes(Arena& ar, const Batch& in) {
  std::vector<tt_round_tape> t(in.size());
  for (size_t b = 0; b < in.size(); ++b) t[b] = gr_tape(ar, in[b]);
  return t;
}

// validation and the workspace layout; ar measures (base null) or carves
static tt_status grad_plan(int32_t batch, const tt_grad_spec* specs, int32_t K, int32_t ckpt_every, Arena& ar,
                           GradRun& g) {
  if (batch < 1 || !specs || K < 1 || ckpt_every < 1) {
    set_error("tt_filter_grad: need batch >= 1, specs, K >= 1 and ckpt_every >= 1");
    return TT_ERR_ARG;
  }
  const tt_filter_spec& f0 = specs[0].f;
  const int d = f0.grid.d;
  if (d < 2 || d > TT_MAXD) {
    set_error("tt_filter_grad: d = %d out of range [2, %d]", d, TT_MAXD);
    return TT_ERR_SHAPE;
  }
  g.B = batch;
  g.d = d;
  g.K = K;
  g.C = ckpt_every;
  g.taped = ckpt_every == 1;
  g.range = f0.meas.kind == 1;
  g.nth = g.range ? d + 4 : d + 1;
  g.eps = f0.eps;
  g.cap = f0.cap;
  g.lik_cap = f0.lik_rank_cap;
  g.ktol = specs[0].kernel_tol;
  g.grids.resize(batch);
  g.meas.resize(batch);
  g.fcs.resize(batch);
  g.qs.assign((size_t)batch * d * d, 0.0);
  g.m0.assign((size_t)batch * d, 0.0);
  g.p0.assign((size_t)batch * d, 0.0);
  g.hw.assign(specs[0].halfwidths, specs[0].halfwidths + d);
  {  // the dense kernel build up to d = 8 and 2^28 taps, TT-cross beyond
    double taps = 1.0;
    for (int l = 0; l < d; ++l) taps *= 2.0 * g.hw[l] + 1.0;
    g.cross = d > 8 || taps > 268435456.0;
    g.npert = g.cross ? 2 * d : 1;
  }
  for (int b = 0; b < batch; ++b) {
    const tt_grad_spec& s = specs[b];
    TT_TRY(check_grid(&s.f.grid));
    if (s.f.grid.d != d || s.f.meas.kind != f0.meas.kind || s.f.eps != f0.eps || s.f.cap != f0.cap ||
        s.f.kernel_cap != f0.kernel_cap || s.f.lik_rank_cap != f0.lik_rank_cap || s.kernel_tol != g.ktol) {
      set_error("tt_filter_grad: filter %d: d, measurement kind, eps, cap, kernel_cap, lik_rank_cap and "
                "kernel_tol must be shared by the batch", b);
      return TT_ERR_SHAPE;
    }
    for (int l = 0; l < d; ++l)
      if (s.halfwidths[l] != g.hw[l]) {
        set_error("tt_filter_grad: filter %d: the kernel box must be shared by the batch", b);
        return TT_ERR_SHAPE;
      }
    if (s.f.cap < 1 || s.f.kernel_cap < 1 || s.f.lik_rank_cap < 1 || !(s.f.eps >= 0.0) || !(s.kernel_tol > 0.0) ||
        (s.f.meas.kind != 0 && s.f.meas.kind != 1) || !(s.f.meas.sigma_lin > 0.0) ||
        (s.f.meas.kind == 1 && !(s.f.meas.sigma_r > 0.0))) {
      set_error("tt_filter_grad: filter %d: bad cap, tolerance or measurement parameters", b);
      return TT_ERR_ARG;
    }
    for (int l = 0; l < d; ++l) {
      if (!(s.q[l * d + l] > 0.0) || !(s.f.p0_diag[l] > 0.0) || s.halfwidths[l] < 0) {
        set_error("tt_filter_grad: filter %d: q's diagonal, the prior variances and the box must be positive", b);
        return TT_ERR_ARG;
      }
      g.m0[(size_t)b * d + l] = s.f.m0[l];
      g.p0[(size_t)b * d + l] = s.f.p0_diag[l];
    }
    for (int e = 0; e < d * d; ++e) g.qs[(size_t)b * d * d + e] = s.q[(e / d) * d + e % d];
    g.grids[b] = s.f.grid;
    g.meas[b] = s.f.meas;
    g.fcs[b] = make_const(s.f.grid, &s.f.meas);
  }
  // capacities per filter
  const int kcap = f0.kernel_cap;
  std::vector<std::array<int, TT_MAXD>> ngrid(batch), ntap(batch);
  std::vector<std::array<int, TT_MAXD + 1>> pc(batch), kc(batch), lc(batch), hc(batch), xc(batch), dc(batch);
  for (int b = 0; b < batch; ++b) {
    const tt_grid& gr = g.grids[b];
    ngrid[b].fill(0);
    ntap[b].fill(0);
    for (int k = 0; k < d; ++k) {
      ngrid[b][k] = gr.n[k];
      ntap[b][k] = 2 * g.hw[k] + 1;
    }
    for (int j = 0; j <= d; ++j) {
      const bool edge = j == 0 || j == d;
      pc[b][j] = edge ? 1 : g.cap;
      long long lp = 1, rp = 1;
      for (int k = 0; k < j; ++k) lp = std::min<long long>(lp * ntap[b][k], 1 << 20);
      for (int k = j; k < d; ++k) rp = std::min<long long>(rp * ntap[b][k], 1 << 20);
      kc[b][j] = edge ? 1
                      : (int)std::min<long long>(
                            std::min<long long>(kcap, std::min(1024 / ntap[b][j], 1024 / ntap[b][j - 1])),
                            std::min(lp, rp));
      const int lr = g.range ? std::min(g.lik_cap, gr.n[1]) : 1;
      lc[b][j] = (j == 1 && g.range) ? lr : 1;
      dc[b][j] = (j == 1 && g.range) ? gr.n[1] : 1;
      hc[b][j] = lc[b][j] * pc[b][j];
      xc[b][j] = kc[b][j] * pc[b][j];
    }
    for (int j = d + 1; j <= TT_MAXD; ++j) pc[b][j] = kc[b][j] = lc[b][j] = dc[b][j] = hc[b][j] = xc[b][j] = 0;
  }
  // persistent part
  g.kern = gr_batch(ar, g, kc, ntap);
  g.kbar = gr_batch(ar, g, kc, ntap);
  for (int pi = 0; pi < g.npert; ++pi) {
    const Batch kp = gr_batch(ar, g, kc, ntap);
    g.kp.insert(g.kp.end(), kp.begin(), kp.end());
  }
  g.logc = ar.take<double>((size_t)K * batch);
  g.kranks = ar.take<int>((size_t)g.npert * batch * (TT_MAXD + 1));
  if (g.cross) g.kstate = ar.take<int>((size_t)batch * CROSS_STATE_INTS);
  g.vals = ar.take<double>((size_t)2 * d * batch);
  g.hstep = ar.take<double>((size_t)d * batch);
  g.lmass = ar.take<double>(batch);
  g.pt.assign(K, Batch());
  g.lik.assign(K, Batch());
  g.h.assign(K, Batch());
  g.hr.assign(K, Batch());
  g.ckpt.assign(K, Batch());
  g.xtape.assign(K, {});
  g.htape.assign(K, {});
  for (int k = 0; k < K; ++k) {
    if (g.taped) {
      g.pt[k] = gr_batch(ar, g, pc, ngrid);
      g.lik[k] = gr_batch(ar, g, lc, ngrid);
      g.h[k] = gr_batch(ar, g, hc, ngrid);
      g.hr[k] = gr_batch(ar, g, pc, ngrid);
      g.htape[k] = gr_tapes(ar, g.h[k]);
      if (k > 0) {
        Batch xs(batch);  // the tape's shape only depends on the capacities
        for (int b = 0; b < batch; ++b) {
          memset(&xs[b], 0, sizeof(tt_train));
          xs[b].d = d;
          for (int q = 0; q < d; ++q) xs[b].n[q] = ngrid[b][q];
          for (int j = 0; j <= d; ++j) xs[b].cap[j] = xc[b][j];
        }
        g.xtape[k] = gr_tapes(ar, xs);
      }
    } else if ((k + 1) % g.C == 0 && k + 1 < K) {
      g.ckpt[k] = gr_batch(ar, g, pc, ngrid);
    }
  }
  // one step's temporaries
  g.X = gr_batch(ar, g, xc, ngrid);
  g.xbar = gr_batch(ar, g, xc, ngrid);
  g.hrbar = gr_batch(ar, g, pc, ngrid);
  g.hbar = gr_batch(ar, g, hc, ngrid);
  g.cbar = gr_batch(ar, g, hc, ngrid);
  g.hzero = gr_batch(ar, g, hc, ngrid);
  g.lbar = gr_batch(ar, g, lc, ngrid);
  g.ppbar = gr_batch(ar, g, pc, ngrid);
  g.ptbar = gr_batch(ar, g, pc, ngrid);
  g.pbar = gr_batch(ar, g, pc, ngrid);
  g.pbar2 = gr_batch(ar, g, pc, ngrid);
  g.kb = gr_batch(ar, g, kc, ntap);
  g.pd = gr_batch(ar, g, dc, ngrid);
  g.pdbar = gr_batch(ar, g, dc, ngrid);
  if (!g.taped) {
    g.s_pt = gr_batch(ar, g, pc, ngrid);
    g.s_lik = gr_batch(ar, g, lc, ngrid);
    g.s_h = gr_batch(ar, g, hc, ngrid);
    g.s_hr = gr_batch(ar, g, pc, ngrid);
    g.seg.assign(g.C, Batch());
    for (int c = 0; c < g.C; ++c) g.seg[c] = gr_batch(ar, g, pc, ngrid);
  }
  g.stab = ar.take<int32_t*>(g.statuses.size());
  g.tab_n = std::max(4, g.npert) * batch;
  g.tab = ar.take<DevTT>((size_t)g.tab_n);
  g.dfc = ar.take<FilterConst>(batch);
  // the sub-calls' workspace: the largest query
  size_t need = 0;
  auto upd = [&](size_t s) { need = std::max(need, s); };
  const tt_train* xs = g.X.data();
  {
    std::vector<int32_t> caps((size_t)batch * (d + 1));
    for (int b = 0; b < batch; ++b)
      for (int j = 0; j <= d; ++j) caps[(size_t)b * (d + 1) + j] = kc[b][j];
    std::vector<tt_grid> grep_;  // the grids once per perturbed build
    for (int pi = 0; pi < g.npert; ++pi) grep_.insert(grep_.end(), g.grids.begin(), g.grids.end());
    const size_t kw =
        g.cross ? std::max(tt_kernel_build_cross_workspace(batch, g.grids.data(), g.hw.data(), g.kern.data()),
                           tt_kernel_build_cross_workspace(g.npert * batch, grep_.data(), g.hw.data(), g.kp.data()))
                : tt_kernel_build_batch_workspace(batch, g.grids.data(), g.hw.data(), caps.data());
    if (kw == 0) {
      set_error("tt_filter_grad: the kernel box or capacities are not supported by the kernel build");
      return TT_ERR_SHAPE;
    }
    upd(kw);
  }
  upd(tt_predict_workspace(batch));
  upd(tt_round_workspace(batch, xs, g.pbar.data()));
  upd(tt_round_workspace(batch, g.hbar.data(), g.pbar.data()));
  upd(tt_normalize_moments_workspace(batch, g.pbar.data()));
  upd(tt_update_workspace(batch, g.grids.data(), g.meas.data(), g.pbar.data(), g.hbar.data(), g.lik_cap));
  upd(tt_update_workspace(batch, g.grids.data(), g.meas.data(), g.lbar.data(), g.lbar.data(), g.lik_cap));
  upd(tt_update_workspace(batch, g.grids.data(), g.meas.data(), g.pd.data(), g.pd.data(), 1));
  upd(tt_round_adjoint_workspace(batch, xs, g.pbar.data()));
  upd(tt_round_adjoint_workspace(batch, g.hbar.data(), g.pbar.data()));
  upd(tt_likelihood_adjoint_workspace(batch, g.meas.data(), g.pd.data(), g.lbar.data()));
  int rmax = 1;
  for (int b = 0; b < batch; ++b)
    for (int j = 0; j <= d; ++j) rmax = std::max({rmax, xc[b][j], hc[b][j], dc[b][j]});
  upd(tt_adjoint_workspace(batch, d, rmax));
  upd(tt_adjoint_workspace(g.npert * batch, d, rmax));
  upd((size_t)2 * batch * 4096 + 4096);  // tt_prior
  g.sub_bytes = need + 4096;
  g.sub = ar.take<char>(g.sub_bytes);
  return TT_OK;
}

// --- small launches of this file ---------------------------------------------
static tt_status gr_zero_like(GradRun& g, const Batch& src, const Batch& dst, hipStream_t st) {
  std::vector<DevTT> v(2 * g.B);
  for (int b = 0; b < g.B; ++b) {
    v[b] = make_dev(src[b]);
    v[g.B + b] = make_dev(dst[b]);
  }
  TT_TRY(upload(g.tab, v, st));
  long long most = 1;
  for (int b = 0; b < g.B; ++b) most = std::max(most, (long long)elems_of(g.d, dst[b].n, dst[b].cap));
  hipLaunchKernelGGL(adj_zero_kernel, dim3(std::max(1, std::min(64, cdiv(most, 256 * 4))), g.B), dim3(256), 0, st,
                     g.tab, g.tab + g.B);
  TTG_LAUNCH_CHECK("adj_zero_kernel");
  return TT_OK;
}

static tt_status gr_clear_status(GradRun& g, hipStream_t st) {
  TT_TRY(upload(g.stab, g.statuses, st));
  const int n = (int)g.statuses.size();
  hipLaunchKernelGGL(zero_status_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, g.stab, n);
  TTG_LAUNCH_CHECK("zero_status_kernel");
  return TT_OK;
}

static tt_status gr_or_status(GradRun& g, const std::vector<const Batch*>& trains, int32_t* status, hipStream_t st) {
  for (size_t i0 = 0; i0 < trains.size(); i0 += 4) {
    const int ntr = (int)std::min<size_t>(4, trains.size() - i0);
    std::vector<DevTT> v((size_t)ntr * g.B);
    for (int j = 0; j < ntr; ++j)
      for (int b = 0; b < g.B; ++b) v[(size_t)j * g.B + b] = make_dev((*trains[i0 + j])[b]);
    TT_TRY(upload(g.tab, v, st));
    hipLaunchKernelGGL(or_status_kernel, dim3(cdiv(g.B, 64)), dim3(64), 0, st, g.tab, g.B, ntr, status);
    TTG_LAUNCH_CHECK("or_status_kernel");
  }
  return TT_OK;
}

static tt_status gr_normalise(GradRun& g, const Batch& t, hipStream_t st) {
  return tt_normalize_moments(g.B, g.grids.data(), t.data(), g.lmass, nullptr, nullptr, g.sub, g.sub_bytes, st);
}

static tt_status gr_round(GradRun& g, const Batch& in, const Batch& out, const std::vector<tt_round_tape>* tape,
                          hipStream_t st) {
  if (tape)
    return tt_round_taped(g.B, in.data(), out.data(), g.eps, g.cap, tape->data(), g.sub, g.sub_bytes, st);
  return tt_round(g.B, in.data(), out.data(), g.eps, g.cap, g.sub, g.sub_bytes, st);
}

// Step k of the recursion from the filtering densities pprev (unused at
// k = 0) into (pt, lik, h, hr); records the roundings when tapes are given.
static tt_status gr_step(GradRun& g, int k, const Batch* pprev, const Batch& pt, const Batch& lik, const Batch& h,
                         const Batch& hr, const std::vector<tt_round_tape>* xtape,
                         const std::vector<tt_round_tape>* htape, const double* z, int zdim, hipStream_t st) {
  if (k == 0) {
    TT_TRY(tt_prior(g.B, g.grids.data(), g.m0.data(), g.p0.data(), pt.data(), g.sub, g.sub_bytes, st));
  } else {
    TT_TRY(tt_predict(g.B, g.kern.data(), pprev->data(), g.X.data(), g.sub, g.sub_bytes, st));
    TT_TRY(gr_round(g, g.X, pt, xtape, st));
  }
  TT_TRY(gr_normalise(g, pt, st));  // pt now holds the predictive (same cores)
  const double* zk = z + (long long)k * zdim;
  const int zs = g.K * zdim;
  TT_TRY(tt_likelihood(g.B, g.grids.data(), g.meas.data(), zk, zs, lik.data(), g.lik_cap, g.sub, g.sub_bytes, st));
  TT_TRY(tt_update(g.B, g.grids.data(), g.meas.data(), zk, zs, pt.data(), h.data(), g.lik_cap,
                   g.logc + (long long)k * g.B, g.sub, g.sub_bytes, st));
  TT_TRY(gr_round(g, h, hr, htape, st));
  return gr_normalise(g, hr, st);  // hr now holds the filtering density
}

// the kernel TTs at the specs' parameters
// (out.size() / B builds of the batch's kernels, q per build and filter).
// TT-cross: working rank 64 (the trains' capacities cap the result).  The
// base builds (forced null) save their index sets in kstate; a perturbed
// build i (forced: the base builds' ranks, stride TT_MAXD + 1) replays the
// index sets of filter i mod B and rounds to its ranks, so the perturbed
// kernels are the base's interpolant of the perturbed function, smooth in
// the parameters.
static tt_status gr_kernels(GradRun& g, const std::vector<double>& qs, const Batch& out, hipStream_t st,
                            const int* forced = nullptr) {
  const int n = (int)out.size();
  std::vector<tt_grid> grids;
  for (int i = 0; i < n / g.B; ++i) grids.insert(grids.end(), g.grids.begin(), g.grids.end());
  if (g.cross) {
    std::vector<int> ids(n);
    for (int i = 0; i < n; ++i) ids[i] = i % g.B;
    return kernel_cross_impl(n, grids.data(), qs.data(), g.hw.data(), g.ktol, 64, out.data(), g.sub, g.sub_bytes,
                             st, ids, forced, TT_MAXD + 1, forced ? nullptr : g.kstate, forced ? g.kstate : nullptr);
  }
  return tt_kernel_build_batch(n, grids.data(), qs.data(), g.hw.data(), g.ktol, out.data(), g.sub, g.sub_bytes, st);
}

}  // namespace ttg

extern "C" {

size_t tt_filter_grad_workspace(int32_t batch, const tt_grad_spec* specs, int32_t K, int32_t ckpt_every) {
  using namespace ttg;
  Arena ar(nullptr, 0);
  GradRun g;
  if (grad_plan(batch, specs, K, ckpt_every, ar, g) != TT_OK) return 0;
  return ar.used + 256;
}

tt_status tt_filter_run_taped(int32_t batch, const tt_grad_spec* specs, const double* z_dev, int32_t zdim,
                              int32_t K, int32_t ckpt_every, double* loglik_dev, int32_t* status_dev, void* ws,
                              size_t ws_bytes, void* stream) {
  using namespace ttg;
  if (!z_dev || !loglik_dev || !status_dev || !ws || zdim < 1) {
    set_error("tt_filter_run_taped: null pointer or zdim < 1");
    return TT_ERR_ARG;
  }
  Arena ar(ws, ws_bytes);
  GradRun g;
  TT_TRY(grad_plan(batch, specs, K, ckpt_every, ar, g));
  if (!ar.fits()) {
    set_error("tt_filter_run_taped: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(gr_clear_status(g, st));
  TT_TRY(gr_kernels(g, g.qs, g.kern, st));
  const Batch* prev = nullptr;
  for (int k = 0; k < K; ++k) {
    if (g.taped) {
      TT_TRY(gr_step(g, k, prev, g.pt[k], g.lik[k], g.h[k], g.hr[k], k > 0 ? &g.xtape[k] : nullptr, &g.htape[k],
                     z_dev, zdim, st));
      prev = &g.hr[k];
    } else {
      const Batch& dst = ((k + 1) % g.C == 0 && k + 1 < K) ? g.ckpt[k] : g.seg[k % g.C];
      TT_TRY(gr_step(g, k, prev, g.s_pt, g.s_lik, g.s_h, dst, nullptr, nullptr, z_dev, zdim, st));
      prev = &dst;
    }
    TT_TRY(gr_or_status(g, {&g.kern, prev}, status_dev, st));
  }
  hipLaunchKernelGGL(grad_loglik_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, g.logc, K, batch, loglik_dev);
  TTG_LAUNCH_CHECK("grad_loglik_kernel");
  HIP_TRY(hipStreamSynchronize(st), "tt_filter_run_taped sync");
  return TT_OK;
}

tt_status tt_filter_run_adjoint(int32_t batch, const tt_grad_spec* specs, const double* z_dev, int32_t zdim,
                                int32_t K, int32_t ckpt_every, const double* loglik_bar_dev, double* theta_bar_dev,
                                int32_t* status_dev, void* ws, size_t ws_bytes, void* stream) {
  using namespace ttg;
  if (!z_dev || !loglik_bar_dev || !theta_bar_dev || !status_dev || !ws || zdim < 1) {
    set_error("tt_filter_run_adjoint: null pointer or zdim < 1");
    return TT_ERR_ARG;
  }
  Arena ar(ws, ws_bytes);
  GradRun g;
  TT_TRY(grad_plan(batch, specs, K, ckpt_every, ar, g));
  if (!ar.fits()) {
    set_error("tt_filter_run_adjoint: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int B = batch, d = g.d;
  hipLaunchKernelGGL(fill_kernel, dim3(cdiv((long long)B * g.nth, 256)), dim3(256), 0, st, theta_bar_dev,
                     (long long)B * g.nth, 1LL, 0.0);
  TTG_LAUNCH_CHECK("fill_kernel");
  TT_TRY(upload(g.dfc, g.fcs, st));
  TT_TRY(gr_clear_status(g, st));
  TT_TRY(gr_zero_like(g, g.kern, g.kbar, st));
  const int zs = K * zdim;
  bool have_pbar = false;
  // segments of C steps from the last; with the tape every step is kept
  for (int s0 = ((K - 1) / g.C) * g.C; s0 >= 0; s0 -= g.C) {
    const int s1 = std::min(s0 + g.C, K);
    if (!g.taped) {  // recompute the segment's filtering densities
      const Batch* p = s0 > 0 ? &g.ckpt[s0 - 1] : nullptr;
      for (int k = s0; k < s1 - 1; ++k) {
        TT_TRY(gr_step(g, k, p, g.s_pt, g.s_lik, g.s_h, g.seg[k - s0], nullptr, nullptr, z_dev, zdim, st));
        p = &g.seg[k - s0];
      }
    }
    for (int k = s1 - 1; k >= s0; --k) {
      const Batch* prev = nullptr;
      if (k > 0) prev = g.taped ? &g.hr[k - 1] : (k - 1 >= s0 ? &g.seg[k - 1 - s0] : &g.ckpt[k - 1]);
      const Batch *pt, *lik, *h, *hr;
      const std::vector<tt_round_tape>*xt = nullptr, *ht = nullptr;
      if (g.taped) {
        pt = &g.pt[k];
        lik = &g.lik[k];
        h = &g.h[k];
        hr = &g.hr[k];
        xt = k > 0 ? &g.xtape[k] : nullptr;
        ht = &g.htape[k];
        if (k > 0) TT_TRY(tt_predict(B, g.kern.data(), prev->data(), g.X.data(), g.sub, g.sub_bytes, st));
      } else {
        TT_TRY(gr_step(g, k, prev, g.s_pt, g.s_lik, g.s_h, g.s_hr, nullptr, nullptr, z_dev, zdim, st));
        pt = &g.s_pt;
        lik = &g.s_lik;
        h = &g.s_h;
        hr = &g.s_hr;
      }
      if (!have_pbar) {
        TT_TRY(gr_zero_like(g, *hr, g.pbar, st));
        have_pbar = true;
      }
      // P_k = normalise(HR)
      TT_TRY(tt_normalize_adjoint(B, hr->data(), g.pbar.data(), nullptr, g.hrbar.data(), g.sub, g.sub_bytes, st));
      // HR = round(H)
      TT_TRY(tt_round_adjoint(B, h->data(), hr->data(), g.hrbar.data(), g.hbar.data(), ht ? ht->data() : nullptr,
                              g.sub, g.sub_bytes, st));
      // log c_k = log(sum(H) delta), seeded with loglik_bar
      TT_TRY(gr_zero_like(g, *h, g.hzero, st));
      TT_TRY(tt_normalize_adjoint(B, h->data(), g.hzero.data(), loglik_bar_dev, g.cbar.data(), g.sub, g.sub_bytes,
                                  st));
      TT_TRY(tt_adjoint_axpy(B, 1.0, g.cbar.data(), g.hbar.data(), g.sub, g.sub_bytes, st));
      // H = L o P_pred
      TT_TRY(tt_hadamard_adjoint(B, lik->data(), pt->data(), g.hbar.data(), g.lbar.data(), g.ppbar.data(), g.sub,
                                 g.sub_bytes, st));
      // L = build(dense likelihood): its adjoint, then the measurement parameters
      TT_TRY(tt_likelihood_dense(B, g.grids.data(), g.meas.data(), z_dev + (long long)k * zdim, zs, g.pd.data(),
                                 g.sub, g.sub_bytes, st));
      TT_TRY(tt_likelihood_adjoint(B, g.meas.data(), g.pd.data(), lik->data(), g.lbar.data(), g.pdbar.data(), g.sub,
                                   g.sub_bytes, st));
      {
        std::vector<DevTT> v(2 * B);
        for (int b = 0; b < B; ++b) {
          v[b] = make_dev(g.pd[b]);
          v[B + b] = make_dev(g.pdbar[b]);
        }
        TT_TRY(upload(g.tab, v, st));
        hipLaunchKernelGGL(lik_theta_kernel, dim3(B), dim3(256), 0, st, g.tab, g.tab + B, g.dfc,
                           z_dev + (long long)k * zdim, (long long)zs, g.nth, theta_bar_dev);
        TTG_LAUNCH_CHECK("lik_theta_kernel");
      }
      TT_TRY(gr_or_status(g, {&g.hrbar, &g.hbar, &g.lbar, &g.pdbar}, status_dev, st));
      if (k == 0) break;
      // P_pred = normalise(Pt), Pt = round(X), X = K (*) P_{k-1}
      TT_TRY(tt_normalize_adjoint(B, pt->data(), g.ppbar.data(), nullptr, g.ptbar.data(), g.sub, g.sub_bytes, st));
      TT_TRY(tt_round_adjoint(B, g.X.data(), pt->data(), g.ptbar.data(), g.xbar.data(), xt ? xt->data() : nullptr,
                              g.sub, g.sub_bytes, st));
      TT_TRY(tt_predict_adjoint(B, g.kern.data(), prev->data(), g.xbar.data(), g.pbar2.data(), g.kb.data(), g.sub,
                                g.sub_bytes, st));
      TT_TRY(tt_adjoint_axpy(B, 1.0, g.kb.data(), g.kbar.data(), g.sub, g.sub_bytes, st));
      TT_TRY(gr_or_status(g, {&g.ptbar, &g.xbar, &g.pbar2, &g.kbar}, status_dev, st));
      std::swap(g.pbar, g.pbar2);
    }
  }
  // sigma_w: central differences of the kernel builds, put into the base
  // build's bond bases, against the kernel adjoint; perturbation p = 2 j + s
  // (s = 0: +h, 1: -h), npert of them built per call
  std::vector<double> hs((size_t)d * B);
  const int P = 2 * d;
  for (int p0 = 0; p0 < P; p0 += g.npert) {
    const int pn = std::min(g.npert, P - p0);
    std::vector<double> qp((size_t)pn * B * d * d);
    Batch ref((size_t)pn * B), kbr((size_t)pn * B), kp(g.kp.begin(), g.kp.begin() + (size_t)pn * B);
    for (int pi = 0; pi < pn; ++pi) {
      const int j = (p0 + pi) / 2, sg = (p0 + pi) % 2;
      for (int b = 0; b < B; ++b) {
        const double* q = &g.qs[(size_t)b * d * d];
        std::vector<double> sw(d);
        for (int l = 0; l < d; ++l) sw[l] = sqrt(q[l * d + l]);
        const double hj = 1e-5 * std::max(1.0, sw[j]);
        hs[(size_t)j * B + b] = hj;
        std::vector<double> swp(sw);
        swp[j] += sg == 0 ? hj : -hj;
        double* o = &qp[((size_t)pi * B + b) * d * d];
        for (int l = 0; l < d; ++l)
          for (int m = 0; m < d; ++m) o[l * d + m] = q[l * d + m] / (sw[l] * sw[m]) * swp[l] * swp[m];
        ref[(size_t)pi * B + b] = g.kern[b];
        kbr[(size_t)pi * B + b] = g.kbar[b];
      }
    }
    const int* forced = nullptr;
    if (g.cross) {  // the base ranks, once per perturbed build
      std::vector<DevTT> v((size_t)pn * B);
      for (size_t i = 0; i < v.size(); ++i) v[i] = make_dev(ref[i]);
      TT_TRY(upload(g.tab, v, st));
      hipLaunchKernelGGL(record_ranks_kernel, dim3(cdiv(pn * B, 64)), dim3(64), 0, st, g.tab, pn * B, g.kranks,
                         (long long)(TT_MAXD + 1));
      TTG_LAUNCH_CHECK("record_ranks_kernel");
      forced = g.kranks;
    }
    TT_TRY(gr_kernels(g, qp, kp, st, forced));
    TT_TRY(tt_align_signs(pn * B, ref.data(), kp.data(), g.sub, g.sub_bytes, st));
    std::vector<Batch> parts(pn);
    std::vector<const Batch*> pp(pn);
    for (int pi = 0; pi < pn; ++pi) {
      parts[pi].assign(kp.begin() + (size_t)pi * B, kp.begin() + (size_t)(pi + 1) * B);
      pp[pi] = &parts[pi];
      std::vector<DevTT> v(2 * B);
      for (int b = 0; b < B; ++b) {
        v[b] = make_dev(g.kern[b]);
        v[B + b] = make_dev(parts[pi][b]);
      }
      TT_TRY(upload(g.tab, v, st));
      hipLaunchKernelGGL(rank_match_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, g.tab, g.tab + B, B, status_dev);
      TTG_LAUNCH_CHECK("rank_match_kernel");
    }
    TT_TRY(tt_adjoint_inner(pn * B, kbr.data(), kp.data(), g.vals + (size_t)p0 * B, g.sub, g.sub_bytes, st));
    TT_TRY(gr_or_status(g, pp, status_dev, st));
  }
  TT_TRY(upload(g.hstep, hs, st));
  hipLaunchKernelGGL(kernel_theta_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, g.vals, g.hstep, d, B, g.nth,
                     theta_bar_dev);
  TTG_LAUNCH_CHECK("kernel_theta_kernel");
  HIP_TRY(hipStreamSynchronize(st), "tt_filter_run_adjoint sync");
  return TT_OK;
}

}  // extern "C"
