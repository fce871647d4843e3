// Adjoints (reverse-mode derivatives) of the linear steps of one filter
// step: the core-wise convolution of the prediction (Sec. 4.2), the
// Hadamard product of the update (Sec. 4.1 'times') and the normalisation
// to unit mass (Sec. 2.2, the normaliser of eq. pmf_filtrace_b; Alg. 2
// step 4).
//
// A TT here is stored cores times exp(log_scale).  An adjoint train has the
// layout and ranks of its primal: its cores hold the derivative with
// respect to the primal's stored cores and its log_scale field holds the
// derivative with respect to the primal's log-scale.  Every sum runs in FP64
// in a fixed order, so results do not depend on the batch.
#pragma once

#include "common.h"

namespace ttg {

// Output adjoint trains take the ranks of their primals; the log-scale
// adjoint is copied from the incoming adjoint (the scale of a convolution or
// Hadamard product is the sum of its factors' scales).  A rank that does not
// fit the output capacity, or an incoming adjoint whose ranks are not the
// product ranks, sets TT_STATUS_CAPACITY.
__global__ void adj_init_kernel(const DevTT* __restrict__ prim, const DevTT* __restrict__ out,
                                const DevTT* __restrict__ incoming, const DevTT* __restrict__ fa,
                                const DevTT* __restrict__ fb, int nf) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const DevTT &p = prim[f], &o = out[f], &in = incoming[f];
  int bad = 0;
  for (int j = 0; j <= p.d; ++j) {
    int r = p.ranks[j];
    if (r > o.cap[j]) {
      bad = 1;
      r = o.cap[j];
    }
    o.ranks[j] = r;
    if (fa && fb && in.ranks[j] != fa[f].ranks[j] * fb[f].ranks[j]) bad = 1;
  }
  *o.log_scale = *in.log_scale;
  *o.status = bad ? TT_STATUS_CAPACITY : 0;
}

// ---------------------------------------------------------------------------
// prediction: C_k(a rp0 + c, i, b rp1 + e) = sum_m K_k(a, m + h, b) P_k(c, i - m, e)
// with P = 0 off the grid.
//   Pbar_k(c, j, e) = sum_{m, a, b} K_k(a, m + h, b) Cbar_k(a rp0 + c, j + m, b rp1 + e)
//   Kbar_k(a, m + h, b) = sum_{c, i, e} Cbar_k(a rp0 + c, i, b rp1 + e) P_k(c, i - m, e)
// ---------------------------------------------------------------------------
__device__ inline bool adj_shapes_ok(const DevTT& A, const DevTT& B, const DevTT& C, int k) {
  return C.ranks[k] == A.ranks[k] * B.ranks[k] && C.ranks[k + 1] == A.ranks[k + 1] * B.ranks[k + 1] &&
         A.ranks[k] <= A.cap[k] && B.ranks[k] <= B.cap[k] && C.ranks[k] <= C.cap[k] &&
         A.ranks[k + 1] <= A.cap[k + 1] && B.ranks[k + 1] <= B.cap[k + 1] && C.ranks[k + 1] <= C.cap[k + 1];
}

template <typename T>
__global__ void __launch_bounds__(256) pred_adj_p_kernel(const DevTT* __restrict__ kern,
                                                         const DevTT* __restrict__ pin,
                                                         const DevTT* __restrict__ cbar,
                                                         const DevTT* __restrict__ pbar) {
  const int f = blockIdx.z, k = blockIdx.y;
  const DevTT &K = kern[f], &P = pin[f], &C = cbar[f], &Q = pbar[f];
  if (k >= P.d || !adj_shapes_ok(K, P, C, k) || P.ranks[k] > Q.cap[k] || P.ranks[k + 1] > Q.cap[k + 1]) return;
  const int rk0 = K.ranks[k], rk1 = K.ranks[k + 1], rp0 = P.ranks[k], rp1 = P.ranks[k + 1];
  const int R1 = rk1 * rp1;
  const int n = P.n[k], taps = K.n[k], h = (taps - 1) / 2;
  const long long tot = (long long)rp0 * n * rp1;
  const T* kc = core_ptr<T>(K, k);
  const T* cc = core_ptr<T>(C, k);
  T* qc = core_ptr<T>(Q, k);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(e / ((long long)n * rp1));
    const int rem = (int)(e - (long long)c * n * rp1);
    const int j = rem / rp1, ee = rem - (rem / rp1) * rp1;
    double acc = 0.0;
    for (int m = -h; m <= h; ++m) {
      const int i = j + m;
      if (i < 0 || i >= n) continue;
      for (int a = 0; a < rk0; ++a) {
        const T* kr = kc + ((long long)a * taps + m + h) * rk1;
        const T* cr = cc + ((long long)(a * rp0 + c) * n + i) * R1 + ee;
        for (int b = 0; b < rk1; ++b) acc += bulk_to_double(kr[b]) * bulk_to_double(cr[(long long)b * rp1]);
      }
    }
    qc[e] = from_double<T>(acc);
  }
}

// one workgroup per kernel-core element, a block reduction over (c, i, e)
template <typename T>
__global__ void __launch_bounds__(256) pred_adj_k_kernel(const DevTT* __restrict__ kern,
                                                         const DevTT* __restrict__ pin,
                                                         const DevTT* __restrict__ cbar,
                                                         const DevTT* __restrict__ kbar) {
  const int f = blockIdx.z, k = blockIdx.y;
  const DevTT &K = kern[f], &P = pin[f], &C = cbar[f], &Q = kbar[f];
  if (k >= P.d || !adj_shapes_ok(K, P, C, k) || K.ranks[k] > Q.cap[k] || K.ranks[k + 1] > Q.cap[k + 1]) return;
  __shared__ double red[4];
  const int rk0 = K.ranks[k], rk1 = K.ranks[k + 1], rp0 = P.ranks[k], rp1 = P.ranks[k + 1];
  const int R1 = rk1 * rp1;
  const int n = P.n[k], taps = K.n[k], h = (taps - 1) / 2;
  const long long nel = (long long)rk0 * taps * rk1;
  const long long nt = (long long)rp0 * n * rp1;
  const T* cc = core_ptr<T>(C, k);
  const T* pc = core_ptr<T>(P, k);
  T* qc = core_ptr<T>(Q, k);
  for (long long el = blockIdx.x; el < nel; el += gridDim.x) {
    const int a = (int)(el / ((long long)taps * rk1));
    const int rem = (int)(el - (long long)a * taps * rk1);
    const int tm = rem / rk1, b = rem - (rem / rk1) * rk1;
    const int m = tm - h;
    double acc = 0.0;
    for (long long t = threadIdx.x; t < nt; t += blockDim.x) {
      const int c = (int)(t / ((long long)n * rp1));
      const int r2 = (int)(t - (long long)c * n * rp1);
      const int i = r2 / rp1, ee = r2 - (r2 / rp1) * rp1;
      const int ip = i - m;
      if (ip < 0 || ip >= n) continue;
      acc += bulk_to_double(cc[((long long)(a * rp0 + c) * n + i) * R1 + (long long)b * rp1 + ee]) *
             bulk_to_double(pc[((long long)c * n + ip) * rp1 + ee]);
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) qc[el] = from_double<T>(acc);
  }
}

// ---------------------------------------------------------------------------
// Hadamard: H_k(a rb0 + c, i, b rb1 + e) = A_k(a, i, b) B_k(c, i, e), A in
// FP64 (the likelihood), B and H in the bulk type.
//   Abar_k(a, i, b) = sum_{c, e} Hbar_k(a rb0 + c, i, b rb1 + e) B_k(c, i, e)
//   Bbar_k(c, i, e) = sum_{a, b} Hbar_k(a rb0 + c, i, b rb1 + e) A_k(a, i, b)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) hadamard_adj_kernel(const DevTT* __restrict__ ta,
                                                           const DevTT* __restrict__ tb,
                                                           const DevTT* __restrict__ hbar,
                                                           const DevTT* __restrict__ abar,
                                                           const DevTT* __restrict__ bbar) {
  const int f = blockIdx.z, k = blockIdx.y;
  const DevTT &A = ta[f], &Bt = tb[f], &H = hbar[f];
  if (k >= A.d || !adj_shapes_ok(A, Bt, H, k)) return;
  const int ra0 = A.ranks[k], ra1 = A.ranks[k + 1], rb0 = Bt.ranks[k], rb1 = Bt.ranks[k + 1];
  const int R1 = ra1 * rb1;
  const int n = A.n[k];
  const double* ac = core_ptr<double>(A, k);
  const T* bc = core_ptr<T>(Bt, k);
  const T* hc = core_ptr<T>(H, k);
  const long long na = (long long)ra0 * n * ra1, nb = (long long)rb0 * n * rb1;
  const bool do_a = abar && ra0 <= abar[f].cap[k] && ra1 <= abar[f].cap[k + 1];
  const bool do_b = bbar && rb0 <= bbar[f].cap[k] && rb1 <= bbar[f].cap[k + 1];
  const long long stride = (long long)gridDim.x * blockDim.x;
  if (do_b) {
    T* oc = core_ptr<T>(bbar[f], k);
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nb; e += stride) {
      const int c = (int)(e / ((long long)n * rb1));
      const int rem = (int)(e - (long long)c * n * rb1);
      const int i = rem / rb1, ee = rem - (rem / rb1) * rb1;
      double acc = 0.0;
      for (int a = 0; a < ra0; ++a) {
        const double* ar = ac + ((long long)a * n + i) * ra1;
        const T* hr = hc + ((long long)(a * rb0 + c) * n + i) * R1 + ee;
        for (int b = 0; b < ra1; ++b) acc += ar[b] * bulk_to_double(hr[(long long)b * rb1]);
      }
      oc[e] = from_double<T>(acc);
    }
  }
  if (do_a) {
    double* oc = core_ptr<double>(abar[f], k);
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < na; e += stride) {
      const int a = (int)(e / ((long long)n * ra1));
      const int rem = (int)(e - (long long)a * n * ra1);
      const int i = rem / ra1, b = rem - (rem / ra1) * ra1;
      double acc = 0.0;
      for (int c = 0; c < rb0; ++c) {
        const T* br = bc + ((long long)c * n + i) * rb1;
        const T* hr = hc + ((long long)(a * rb0 + c) * n + i) * R1 + (long long)b * rb1;
        for (int ee = 0; ee < rb1; ++ee) acc += bulk_to_double(br[ee]) * bulk_to_double(hr[ee]);
      }
      oc[e] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Normalisation to unit mass.  Forward: P keeps the cores of X and takes
// log_scale(P) = -log(S delta) with S = sum_i of the stored cores of X; the
// log-mass is log m = log_scale(X) + log(S delta).  Adjoint, with
// sbar = log_scale adjoint of P and mbar = adjoint of log m:
//   Xbar cores = Pbar cores + (mbar - sbar) / S * dS/dX,   Xbar log_scale = mbar
// where dS/dX_k(a, i, b) = left_k(a) right_k(b) (products of the summed
// cores on either side).  One workgroup per filter computes the
// environments and S; a second kernel writes the cores.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) sum_env_kernel(const DevTT* __restrict__ xt, double* __restrict__ env,
                                                      int rcap, double* __restrict__ ssum) {
  const int f = blockIdx.x;
  const DevTT& X = xt[f];
  const int d = X.d;
  double* left = env + (long long)f * 2 * (d + 1) * rcap;  // left[k][a], k = 0..d
  double* right = left + (long long)(d + 1) * rcap;        // right[k][b], k = 0..d (right of core k-1)
  if (threadIdx.x == 0) {
    left[0] = 1.0;
    right[(long long)d * rcap] = 1.0;
  }
  __syncthreads();
  for (int k = 0; k < d; ++k) {
    const int r0 = X.ranks[k], r1 = X.ranks[k + 1], n = X.n[k];
    const T* xc = core_ptr<T>(X, k);
    for (int b = threadIdx.x; b < r1; b += blockDim.x) {
      double acc = 0.0;
      for (int a = 0; a < r0; ++a) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += bulk_to_double(xc[((long long)a * n + i) * r1 + b]);
        acc += left[(long long)k * rcap + a] * s;
      }
      left[(long long)(k + 1) * rcap + b] = acc;
    }
    __syncthreads();
  }
  for (int k = d - 1; k >= 0; --k) {
    const int r0 = X.ranks[k], r1 = X.ranks[k + 1], n = X.n[k];
    const T* xc = core_ptr<T>(X, k);
    for (int a = threadIdx.x; a < r0; a += blockDim.x) {
      double acc = 0.0;
      for (int b = 0; b < r1; ++b) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += bulk_to_double(xc[((long long)a * n + i) * r1 + b]);
        acc += s * right[(long long)(k + 1) * rcap + b];
      }
      right[(long long)k * rcap + a] = acc;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) ssum[f] = left[(long long)d * rcap];
}

template <typename T>
__global__ void __launch_bounds__(256) normalize_adj_kernel(const DevTT* __restrict__ xt,
                                                            const DevTT* __restrict__ pbar,
                                                            const DevTT* __restrict__ xbar,
                                                            const double* __restrict__ log_mass_bar,
                                                            const double* __restrict__ env, int rcap,
                                                            const double* __restrict__ ssum) {
  const int f = blockIdx.z, k = blockIdx.y;
  const DevTT &X = xt[f], &Pb = pbar[f], &Xb = xbar[f];
  const int d = X.d;
  if (k >= d) return;
  const int r0 = X.ranks[k], r1 = X.ranks[k + 1], n = X.n[k];
  if (Pb.ranks[k] != r0 || Pb.ranks[k + 1] != r1 || r0 > Xb.cap[k] || r1 > Xb.cap[k + 1]) return;
  const double* left = env + (long long)f * 2 * (d + 1) * rcap + (long long)k * rcap;
  const double* right = env + (long long)f * 2 * (d + 1) * rcap + (long long)(d + 1) * rcap +
                        (long long)(k + 1) * rcap;
  const double mb = log_mass_bar ? log_mass_bar[f] : 0.0;
  const double coef = (mb - *Pb.log_scale) / ssum[f];
  const T* pc = core_ptr<T>(Pb, k);
  T* oc = core_ptr<T>(Xb, k);
  const long long tot = (long long)r0 * n * r1;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
       e += (long long)gridDim.x * blockDim.x) {
    const int a = (int)(e / ((long long)n * r1));
    const int b = (int)(e % r1);
    oc[e] = from_double<T>(bulk_to_double(pc[e]) + coef * left[a] * right[b]);
  }
}

__global__ void normalize_adj_init_kernel(const DevTT* __restrict__ xt, const DevTT* __restrict__ pbar,
                                          const DevTT* __restrict__ xbar, const double* __restrict__ log_mass_bar,
                                          int nf) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const DevTT &X = xt[f], &Pb = pbar[f], &Xb = xbar[f];
  int bad = 0;
  for (int j = 0; j <= X.d; ++j) {
    int r = X.ranks[j];
    if (r > Xb.cap[j] || Pb.ranks[j] != r) bad = 1;
    Xb.ranks[j] = min(r, Xb.cap[j]);
  }
  *Xb.log_scale = log_mass_bar ? log_mass_bar[f] : 0.0;
  *Xb.status = bad ? TT_STATUS_CAPACITY : 0;
}

}  // namespace ttg
