// Grid re-design and interpolation onto the new grid (Alg. 3 and Alg. 4;
// Sec. 4.2, interpolation on the level of the cores).
//
// grid_box_kernel: per filter, the local Kalman prediction of the filtering
// moments (m' = F m, P' = F P F^T + Q), the predictive box m' +- nsigma
// sqrt(P'_ll), and the smallest axis-aligned box holding its 2^d corners
// mapped by F^{-1}: the image of a box c' +- h under a linear map A is
// A c' +- |A| h, so no corner is enumerated.
//
// interp_kernel: multilinear interpolation of a TT onto a new axis-aligned
// grid acts core by core: out_k(a, i', b) = (1 - t) in_k(a, j, b) +
// t in_k(a, j + 1, b) with x_j <= x'_{i'} <= x_{j+1} on axis k, and zero
// where x'_{i'} lies off the old grid.  Grid points are lo + (hi - lo) i /
// (n - 1) on both grids.  One pass over the output, two reads per output
// element (adjacent grid rows of the input, cache-resident).
#pragma once

#include "common.h"

namespace ttg {

struct GridBox {
  int d;
  double lo[TT_MAXD], hi[TT_MAXD];
};

// F, Finv, Q: d x d row-major (shared by the batch); mean[b*d + l],
// cov[b*d*d + l*d + j]; one thread per filter
__global__ void grid_box_kernel(int nf, int d, const double* __restrict__ fm, const double* __restrict__ finv,
                                const double* __restrict__ q, double nsigma, const double* __restrict__ mean,
                                const double* __restrict__ cov, GridBox* __restrict__ out) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const double* m = mean + (long long)f * d;
  const double* p = cov + (long long)f * d * d;
  double mp[TT_MAXD], h[TT_MAXD];
  for (int l = 0; l < d; ++l) {
    double s = 0.0, v = q[l * d + l];
    for (int a = 0; a < d; ++a) {
      s += fm[l * d + a] * m[a];
      double row = 0.0;  // (P F^T)(a, l)
      for (int b = 0; b < d; ++b) row += p[a * d + b] * fm[l * d + b];
      v += fm[l * d + a] * row;
    }
    mp[l] = s;
    h[l] = nsigma * sqrt(fmax(v, 0.0));
  }
  GridBox& o = out[f];
  o.d = d;
  for (int l = 0; l < d; ++l) {
    double c = 0.0, w = 0.0;
    for (int a = 0; a < d; ++a) {
      c += finv[l * d + a] * mp[a];
      w += fabs(finv[l * d + a]) * h[a];
    }
    o.lo[l] = c - w;
    o.hi[l] = c + w;
  }
}

#define IP_NMAX 2048  // new-grid points whose weights fit the LDS table

struct InterpArgs {
  int n_old[TT_MAXD], n_new[TT_MAXD];
  double lo_old[TT_MAXD], hi_old[TT_MAXD], lo_new[TT_MAXD], hi_new[TT_MAXD];
};

template <typename E>
__global__ void __launch_bounds__(256) interp_kernel(const DevTT* __restrict__ xin, const DevTT* __restrict__ xout,
                                                     const InterpArgs* __restrict__ ia) {
  const int f = blockIdx.z, k = blockIdx.y;
  const DevTT &X = xin[f], &O = xout[f];
  if (k >= X.d) return;
  const InterpArgs& g = ia[f];
  const int r0 = X.ranks[k], r1 = X.ranks[k + 1], no = g.n_old[k], nn = g.n_new[k];
  const double lo = g.lo_old[k], span = g.hi_old[k] - g.lo_old[k];
  const double lon = g.lo_new[k], spann = g.hi_new[k] - g.lo_new[k];
  const double x0 = lo + span * 0 / (no - 1), xl = lo + span * (no - 1) / (no - 1);
  const double step = (xl - x0) / (no - 1);
  const E* ic = core_ptr<E>(X, k);
  E* oc = core_ptr<E>(O, k);
  const long long tot = (long long)r0 * nn * r1;
  auto value = [&](long long row_in, int b, int i) -> double {  // row_in = a * no
    const double x = lon + spann * i / (nn - 1);
    if (!(x >= x0 && x <= xl)) return 0.0;
    const int j = min((int)floor((x - x0) / step), no - 2);
    const double xj = lo + span * j / (no - 1), xj1 = lo + span * (j + 1) / (no - 1);
    const double t = (x - xj) / (xj1 - xj);
    const E* col = ic + (row_in + j) * r1 + b;
    return (1.0 - t) * (double)col[0] + t * (double)col[r1];
  };
  if (tot < 0x7fffffffLL && nn <= IP_NMAX) {
    // the weights depend on the new grid point only: once per workgroup
    __shared__ int s_j[IP_NMAX];
    __shared__ double s_t[IP_NMAX];
    for (int i = threadIdx.x; i < nn; i += blockDim.x) {
      const double x = lon + spann * i / (nn - 1);
      int j = -1;
      double t = 0.0;
      if (x >= x0 && x <= xl) {
        j = min((int)floor((x - x0) / step), no - 2);
        const double xj = lo + span * j / (no - 1), xj1 = lo + span * (j + 1) / (no - 1);
        t = (x - xj) / (xj1 - xj);
      }
      s_j[i] = j;
      s_t[i] = t;
    }
    __syncthreads();
    const int itot = (int)tot;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < itot; e += gridDim.x * blockDim.x) {
      const int ai = e / r1, b = e - (e / r1) * r1;
      const int a = ai / nn, i = ai - (ai / nn) * nn;
      const int j = s_j[i];
      double v = 0.0;
      if (j >= 0) {
        const double t = s_t[i];
        const E* col = ic + ((long long)a * no + j) * r1 + b;
        v = (1.0 - t) * (double)col[0] + t * (double)col[r1];
      }
      oc[e] = (E)v;
    }
  } else {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
         e += (long long)gridDim.x * blockDim.x) {
      const long long ai = e / r1;
      const int b = (int)(e - ai * r1);
      const long long a = ai / nn;
      const int i = (int)(ai - a * nn);
      oc[e] = (E)value(a * no, b, i);
    }
  }
  if (k == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
    for (int j = 0; j <= X.d; ++j) O.ranks[j] = X.ranks[j];
    *O.log_scale = *X.log_scale;
    *O.status = *X.status;
  }
}

}  // namespace ttg
