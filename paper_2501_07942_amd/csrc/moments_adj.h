// Adjoint of the moments of tt_normalize_moments (the moments of Alg. 2:
// Sec. 4.1 'dot' and 'power'), for tt_normalize_moments_adjoint.  Included by
// api.hip after the normalisation adjoint it extends.
//
// With M_w = sum_i w(i) X(i) over the stored values (the cell volume and the
// log-scale cancel in the moments) and rank-one weights w, the outputs are
// mean_l = M_{x_l} / M_1 and cov_lj = M_{x_l x_j} / M_1 - mean_l mean_j.  Their
// adjoint is sum_w c_w dM_w / dX with
//   c_{x_l x_j} = (cbar_lj + cbar_jl) / M_1 (l < j),  c_{x_l^2} = cbar_ll / M_1,
//   mbar'_l = mbar_l - sum_{j != l} (cbar_lj + cbar_jl) mean_j - 2 cbar_ll mean_l,
//   c_{x_l} = mbar'_l / M_1,
//   c_1 = -sum_l mbar'_l mean_l / M_1 - sum_{l <= j} c_{x_l x_j} M_{x_l x_j} / M_1,
// and dM_w / dX_k(a, i, b) = L^w_k(a) w_k(i) R^w_{k+1}(b) (the weighted prefix
// and suffix chains).  Grouped by the power v of x_k(i) in w_k:
//   X_bar_k(a, i, b) += sum_v x_k(i)^v T^v_k(a, b),
//   T^v_k = sum_{w : w_k = x^v} c_w L^w_k (x) R^w_{k+1}.
#pragma once

namespace ttg {

// power of x on axis k in moment term t: t = 0 the ones; 1..d x_l; d+1..2d
// x_l^2; then x_l x_j for l < j in lexicographic order
__device__ inline int madj_pow(int t, int k, int d) {
  if (t == 0) return 0;
  if (t <= d) return (t - 1 == k) ? 1 : 0;
  if (t <= 2 * d) return (t - d - 1 == k) ? 2 : 0;
  int p = t - 2 * d - 1;
  for (int l = 0; l < d; ++l) {
    const int cnt = d - 1 - l;
    if (p < cnt) {
      const int j = l + 1 + p;
      return (k == l || k == j) ? 1 : 0;
    }
    p -= cnt;
  }
  return 0;
}

__host__ __device__ inline int madj_terms(int d) { return 1 + 2 * d + d * (d - 1) / 2; }

__host__ __device__ inline long long madj_scratch(int d, int rcap) {
  const long long mat = (long long)rcap * rcap, nt = madj_terms(d);
  return 6LL * d * mat + 2 * nt * (d + 1) * rcap + 2 * nt;
}

// one workgroup per filter; scratch per filter madj_scratch(d, rcap) doubles
template <typename T>
__global__ void __launch_bounds__(256) moments_adj_kernel(const DevTT* __restrict__ X, const DevTT* __restrict__ XB,
                                                          const FilterConst* __restrict__ fc,
                                                          const double* __restrict__ mean_bar,
                                                          const double* __restrict__ cov_bar,
                                                          double* __restrict__ scratch, int rcap) {
  const int f = blockIdx.x;
  const DevTT& A = X[f];
  const DevTT& G = XB[f];
  const FilterConst& C = fc[f];
  const int d = A.d, tid = threadIdx.x, nt = madj_terms(d);
  const long long mat = (long long)rcap * rcap;
  double* S = scratch + (long long)f * madj_scratch(d, rcap);  // [3][d][mat]
  double* Tm = S + 3LL * d * mat;                              // [3][d][mat]
  double* Lc = Tm + 3LL * d * mat;                             // [nt][d+1][rcap]
  double* Rc = Lc + (long long)nt * (d + 1) * rcap;            // [nt][d+1][rcap]
  double* Mv = Rc + (long long)nt * (d + 1) * rcap;            // [nt]
  double* cf = Mv + nt;                                        // [nt]
  // per-core sums with 1, x, x^2
  for (int k = 0; k < d; ++k) {
    const int r0 = A.ranks[k], r1 = A.ranks[k + 1], n = A.n[k];
    const T* c = core_ptr<T>(A, k);
    for (int q = tid; q < r0 * r1; q += blockDim.x) {
      const int a = q / r1, bq = q - (q / r1) * r1;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int i = 0; i < n; ++i) {
        const double x = C.lo[k] + i * C.dx[k];
        const double v = bulk_to_double(c[((long long)a * n + i) * r1 + bq]);
        s0 += v;
        s1 += x * v;
        s2 += x * x * v;
      }
      S[(0LL * d + k) * mat + a * r1 + bq] = s0;
      S[(1LL * d + k) * mat + a * r1 + bq] = s1;
      S[(2LL * d + k) * mat + a * r1 + bq] = s2;
    }
  }
  for (int t = tid; t < nt; t += blockDim.x) {
    Lc[(long long)t * (d + 1) * rcap] = 1.0;
    Rc[((long long)t * (d + 1) + d) * rcap] = 1.0;
  }
  __syncthreads();
  // weighted prefix chains L^t_{k+1} = L^t_k S^{pow}_k, suffix chains
  // R^t_k = S^{pow}_k R^t_{k+1}, every term at once
  for (int k = 0; k < d; ++k) {
    const int r0 = A.ranks[k], r1 = A.ranks[k + 1];
    for (int e = tid; e < nt * r1; e += blockDim.x) {
      const int t = e / r1, bq = e - (e / r1) * r1;
      const double* Sk = S + ((long long)madj_pow(t, k, d) * d + k) * mat;
      const double* l = Lc + ((long long)t * (d + 1) + k) * rcap;
      double s = 0.0;
      for (int a = 0; a < r0; ++a) s += l[a] * Sk[a * r1 + bq];
      Lc[((long long)t * (d + 1) + k + 1) * rcap + bq] = s;
    }
    const int kk = d - 1 - k;
    const int q0 = A.ranks[kk], q1 = A.ranks[kk + 1];
    for (int e = tid; e < nt * q0; e += blockDim.x) {
      const int t = e / q0, a = e - (e / q0) * q0;
      const double* Sk = S + ((long long)madj_pow(t, kk, d) * d + kk) * mat;
      const double* r = Rc + ((long long)t * (d + 1) + kk + 1) * rcap;
      double s = 0.0;
      for (int bq = 0; bq < q1; ++bq) s += Sk[a * q1 + bq] * r[bq];
      Rc[((long long)t * (d + 1) + kk) * rcap + a] = s;
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int t = 0; t < nt; ++t) Mv[t] = Lc[((long long)t * (d + 1) + d) * rcap];
    const double m0 = Mv[0];
    double mean[TT_MAXD], mb[TT_MAXD];
    for (int l = 0; l < d; ++l) {
      mean[l] = Mv[1 + l] / m0;
      mb[l] = mean_bar ? mean_bar[(long long)f * d + l] : 0.0;
    }
    double c0 = 0.0;
    int t = 2 * d + 1;
    for (int l = 0; l < d; ++l) {
      const double cb = cov_bar ? cov_bar[(long long)f * d * d + l * d + l] : 0.0;
      cf[d + 1 + l] = cb / m0;
      c0 -= cb * Mv[d + 1 + l] / (m0 * m0);
      mb[l] -= 2.0 * cb * mean[l];
    }
    for (int l = 0; l < d; ++l)
      for (int j = l + 1; j < d; ++j, ++t) {
        const double cb = cov_bar ? cov_bar[(long long)f * d * d + l * d + j] + cov_bar[(long long)f * d * d + j * d + l]
                                  : 0.0;
        cf[t] = cb / m0;
        c0 -= cb * Mv[t] / (m0 * m0);
        mb[l] -= cb * mean[j];
        mb[j] -= cb * mean[l];
      }
    for (int l = 0; l < d; ++l) {
      cf[1 + l] = mb[l] / m0;
      c0 -= mb[l] * mean[l] / m0;
    }
    cf[0] = c0;
  }
  __syncthreads();
  // T^v_k = sum over the terms whose axis-k weight is x^v
  for (int k = 0; k < d; ++k) {
    const int r0 = A.ranks[k], r1 = A.ranks[k + 1];
    for (int q = tid; q < r0 * r1; q += blockDim.x) {
      const int a = q / r1, bq = q - (q / r1) * r1;
      double acc[3] = {0.0, 0.0, 0.0};
      for (int t = 0; t < nt; ++t)
        acc[madj_pow(t, k, d)] += cf[t] * Lc[((long long)t * (d + 1) + k) * rcap + a] *
                                  Rc[((long long)t * (d + 1) + k + 1) * rcap + bq];
      for (int v = 0; v < 3; ++v) Tm[((long long)v * d + k) * mat + q] = acc[v];
    }
  }
  __syncthreads();
  for (int k = 0; k < d; ++k) {
    const int r0 = A.ranks[k], r1 = A.ranks[k + 1], n = A.n[k];
    T* gb = core_ptr<T>(G, k);
    for (long long e = tid; e < (long long)r0 * n * r1; e += blockDim.x) {
      const int a = (int)(e / ((long long)n * r1));
      const int rem = (int)(e - (long long)a * n * r1);
      const int i = rem / r1, bq = rem - (rem / r1) * r1;
      const double x = C.lo[k] + i * C.dx[k];
      const int q = a * r1 + bq;
      const double add = Tm[(0LL * d + k) * mat + q] + x * Tm[(1LL * d + k) * mat + q] +
                         x * x * Tm[(2LL * d + k) * mat + q];
      gb[e] = from_double<T>(bulk_to_double(gb[e]) + add);
    }
  }
}

}  // namespace ttg

extern "C" {

size_t tt_normalize_moments_adjoint_workspace(int32_t batch, const tt_train* x) {
  using namespace ttg;
  if (batch < 1 || !x) return 0;
  int rcap = 1, d = x[0].d;
  for (int b = 0; b < batch; ++b)
    for (int j = 0; j <= x[b].d && j <= TT_MAXD; ++j) rcap = std::max(rcap, x[b].cap[j]);
  if (d < 1 || d > TT_MAXD) return 0;
  const size_t w1 = tt_adjoint_workspace(batch, d, rcap);
  const size_t w2 = (size_t)batch * (2 * sizeof(DevTT) + sizeof(FilterConst)) +
                    (size_t)batch * madj_scratch(d, rcap) * sizeof(double);
  return w1 + w2 + 4096;
}

tt_status tt_normalize_moments_adjoint(int32_t batch, const tt_grid* grids, const tt_train* x,
                                       const tt_train* p_bar, const double* log_mass_bar_dev,
                                       const double* mean_bar_dev, const double* cov_bar_dev,
                                       const tt_train* x_bar, void* ws, size_t ws_bytes, void* stream) {
  using namespace ttg;
  if (batch < 1 || !grids || !x || !p_bar || !x_bar || !ws) {
    set_error("tt_normalize_moments_adjoint: null pointer or batch < 1");
    return TT_ERR_ARG;
  }
  const int d = x[0].d;
  int rcap = 1;
  std::vector<DevTT> vx(batch), vxb(batch);
  std::vector<FilterConst> vfc(batch);
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_grid(&grids[b]));
    if (grids[b].d != x[b].d || x[b].d != d) {
      set_error("tt_normalize_moments_adjoint: filter %d: grid and train dimensions differ", b);
      return TT_ERR_SHAPE;
    }
    for (int k = 0; k < d; ++k)
      if (grids[b].n[k] != x[b].n[k]) {
        set_error("tt_normalize_moments_adjoint: filter %d: grid and train modes differ", b);
        return TT_ERR_SHAPE;
      }
    for (int j = 0; j <= d; ++j) rcap = std::max(rcap, x[b].cap[j]);
    vx[b] = make_dev(x[b]);
    vxb[b] = make_dev(x_bar[b]);
    vfc[b] = make_const(grids[b], nullptr);
  }
  const size_t w1 = tt_adjoint_workspace(batch, d, rcap);
  if (ws_bytes < w1) {
    set_error("tt_normalize_moments_adjoint: workspace too small");
    return TT_ERR_WORKSPACE;
  }
  // the normalisation's adjoint (cores and log-scale), then the moments' terms
  TT_TRY(tt_normalize_adjoint(batch, x, p_bar, log_mass_bar_dev, x_bar, ws, w1, stream));
  if (!mean_bar_dev && !cov_bar_dev) return TT_OK;
  Arena ar(static_cast<char*>(ws) + w1, ws_bytes - w1);
  DevTT* dx = ar.take<DevTT>(batch);
  DevTT* dxb = ar.take<DevTT>(batch);
  FilterConst* dfc = ar.take<FilterConst>(batch);
  double* scr = ar.take<double>((size_t)batch * madj_scratch(d, rcap));
  if (!ar.fits()) {
    set_error("tt_normalize_moments_adjoint: workspace too small");
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(dx, vx, st));
  TT_TRY(upload(dxb, vxb, st));
  TT_TRY(upload(dfc, vfc, st));
  if (x[0].dtype == TT_F64)
    hipLaunchKernelGGL((moments_adj_kernel<double>), dim3(batch), dim3(256), 0, st, dx, dxb, dfc, mean_bar_dev,
                       cov_bar_dev, scr, rcap);
  else
    hipLaunchKernelGGL((moments_adj_kernel<float>), dim3(batch), dim3(256), 0, st, dx, dxb, dfc, mean_bar_dev,
                       cov_bar_dev, scr, rcap);
  TTG_LAUNCH_CHECK("moments_adj_kernel");
  return TT_OK;
}

}  // extern "C"
