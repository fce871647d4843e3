// Adjoints (reverse-mode derivatives) of the linear steps of one filter
// step: the core-wise convolution of the prediction (Sec. 4.2), the
// Hadamard product of the update (Sec. 4.1 'times') and the normalisation
// to unit mass (Sec. 2.2, the normaliser of eq. pmf_filtrace_b; Alg. 2).
//
// A TT here is stored cores times exp(log_scale).  An adjoint train has the
// layout and ranks of its primal: its cores hold the derivative with
// respect to the primal's stored cores and its log_scale field holds the
// derivative with respect to the primal's log-scale.  Every sum runs in FP64
// in a fixed order, so results do not depend on the batch.
#pragma once

#include "common.h"
#include "linalg.h"

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

// Pbar with register windows: a work item is one density pair (c, e) and
// PADJ_JROWS consecutive grid points j; for every kernel pair (a, b) it loads
// the window of Cbar(a rp0 + c, i, b rp1 + e) over i = j + m that its rows
// and a chunk of PADJ_TAPS taps need, and multiplies it with the kernel
// values of that pair (staged once per workgroup in LDS).  Sums run over a,
// b, tap chunks and taps in a fixed order.  LDS: rk0 taps rk1 elements.
#define PADJ_JROWS 16
template <typename T>
__global__ void __launch_bounds__(256) pred_adj_p_reg_kernel(const DevTT* __restrict__ kern,
                                                             const DevTT* __restrict__ pin,
                                                             const DevTT* __restrict__ cbar,
                                                             const DevTT* __restrict__ pbar) {
  const int f = blockIdx.z, k = blockIdx.y;
  const DevTT &K = kern[f], &P = pin[f], &C = cbar[f], &Q = pbar[f];
  if (k >= P.d || !adj_shapes_ok(K, P, C, k) || P.ranks[k] > Q.cap[k] || P.ranks[k + 1] > Q.cap[k + 1]) return;
  const int rk0 = K.ranks[k], rk1 = K.ranks[k + 1], rp0 = P.ranks[k], rp1 = P.ranks[k + 1];
  const int R1 = rk1 * rp1;
  const int n = P.n[k], taps = K.n[k], h = (taps - 1) / 2;
  const int njb = (n + PADJ_JROWS - 1) / PADJ_JROWS;
  const long long items = (long long)rp0 * rp1 * njb;
  constexpr int TC = 32, W = PADJ_JROWS + TC - 1;
  extern __shared__ unsigned char padj_smem[];
  T* Ks = reinterpret_cast<T*>(padj_smem);  // K_k(a, tm, b) as stored
  const T* kc = core_ptr<T>(K, k);
  for (int e = threadIdx.x; e < rk0 * taps * rk1; e += blockDim.x) Ks[e] = kc[e];
  __syncthreads();
  const TTG_GLOBAL T* cc = gmem(core_ptr<T>(C, k));
  TTG_GLOBAL T* qc = gmem(core_ptr<T>(Q, k));
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < items;
       t += (long long)gridDim.x * blockDim.x) {
    const int e = (int)(t % rp1);
    const long long rest = t / rp1;
    const int c = (int)(rest % rp0), j0 = (int)(rest / rp0) * PADJ_JROWS;
    double acc[PADJ_JROWS];
#pragma unroll
    for (int r = 0; r < PADJ_JROWS; ++r) acc[r] = 0.0;
    for (int a = 0; a < rk0; ++a)
      for (int b = 0; b < rk1; ++b) {
        const TTG_GLOBAL T* crow = cc + ((long long)(a * rp0 + c) * n) * R1 + (long long)b * rp1 + e;
        const T* kr = Ks + (long long)a * taps * rk1 + b;
        for (int m0 = 0; m0 < taps; m0 += TC) {
          // output j = j0 + r and tap tm = m0 + u (offset m = tm - h) read
          // Cbar at i = j + m = base + r + u
          const int base = j0 + m0 - h;
          double w[W];
#pragma unroll
          for (int v = 0; v < W; ++v) {
            const int i = base + v;
            w[v] = (i >= 0 && i < n) ? bulk_to_double(crow[(long long)i * R1]) : 0.0;
          }
          const int mc = min(TC, taps - m0);
#pragma unroll
          for (int u = 0; u < TC; ++u) {
            if (u < mc) {
              const double kv = bulk_to_double(kr[(long long)(m0 + u) * rk1]);
#pragma unroll
              for (int r = 0; r < PADJ_JROWS; ++r) acc[r] += kv * w[r + u];
            }
          }
        }
      }
#pragma unroll
    for (int r = 0; r < PADJ_JROWS; ++r) {
      const int j = j0 + r;
      if (j < n) qc[((long long)c * n + j) * rp1 + e] = from_double<T>(acc[r]);
    }
  }
}

// One workgroup per kernel bond pair (a, b): one pass over its slice of
// Cbar per PADJ_TAPS taps accumulates every tap of that pair at once.  A
// work item is one density pair (c, e) and PADJ_ROWS consecutive grid points
// i: it holds their Cbar values and the window of density values
// P(c, i - m, e) those rows need for the chunk's taps in registers, so each
// load feeds several multiply-adds.  A fixed-order block reduction per tap
// follows.
#define PADJ_TAPS 32
#define PADJ_ROWS 8
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
  const int nib = (n + PADJ_ROWS - 1) / PADJ_ROWS;
  const long long items = (long long)rp0 * rp1 * nib;
  constexpr int W = PADJ_ROWS + PADJ_TAPS - 1;
  const T* cc = core_ptr<T>(C, k);
  const T* pc = core_ptr<T>(P, k);
  T* qc = core_ptr<T>(Q, k);
  for (int pair = blockIdx.x; pair < rk0 * rk1; pair += gridDim.x) {
    const int a = pair / rk1, b = pair - (pair / rk1) * rk1;
    for (int m0 = 0; m0 < taps; m0 += PADJ_TAPS) {
      const int mc = min(PADJ_TAPS, taps - m0);
      double acc[PADJ_TAPS];
#pragma unroll
      for (int u = 0; u < PADJ_TAPS; ++u) acc[u] = 0.0;
      for (long long t = threadIdx.x; t < items; t += blockDim.x) {
        const int e = (int)(t % rp1);
        const long long rest = t / rp1;
        const int c = (int)(rest % rp0), i0 = (int)(rest / rp0) * PADJ_ROWS;
        const T* crow = cc + ((long long)(a * rp0 + c) * n) * R1 + (long long)b * rp1 + e;
        const T* prow = pc + (long long)c * n * rp1 + e;
        double cv[PADJ_ROWS], w[W];
#pragma unroll
        for (int r = 0; r < PADJ_ROWS; ++r)
          cv[r] = (i0 + r < n) ? bulk_to_double(crow[(long long)(i0 + r) * R1]) : 0.0;
        // tap tm = m0 + u (offset m = tm - h) reads P(c, i0 + r - m, e) = w[PADJ_TAPS - 1 + r - u]
        const int base = i0 - m0 - (PADJ_TAPS - 1) + h;
#pragma unroll
        for (int v = 0; v < W; ++v) {
          const int ip = base + v;
          w[v] = (ip >= 0 && ip < n) ? bulk_to_double(prow[(long long)ip * rp1]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PADJ_TAPS; ++u)
#pragma unroll
          for (int r = 0; r < PADJ_ROWS; ++r) acc[u] += cv[r] * w[PADJ_TAPS - 1 + r - u];
      }
      for (int u = 0; u < mc; ++u) {
        const double sum = block_sum(acc[u], red);
        if (threadIdx.x == 0) qc[((long long)a * taps + m0 + u) * rk1 + b] = from_double<T>(sum);
      }
    }
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
  __shared__ double part[256];
  // left[k+1](b) = sum_a left[k](a) sum_i X_k(a, i, b): groups of nb threads
  // own the columns, the groups split the mode index i, an LDS pass sums the
  // groups (blockDim.x = 256); the mode sum of one row a is unrolled so that
  // several loads are in flight per thread
  for (int k = 0; k < d; ++k) {
    const int r0 = X.ranks[k], r1 = X.ranks[k + 1], n = X.n[k];
    const T* xc = core_ptr<T>(X, k);
    const double* lk = left + (long long)k * rcap;
    const int nb = min(r1, 256), G = 256 / nb;
    const int g = threadIdx.x / nb, tb = threadIdx.x - (threadIdx.x / nb) * nb;
    for (int b0 = 0; b0 < r1; b0 += nb) {
      const int b = b0 + tb;
      double acc = 0.0;
      if (g < G && b < r1) {
        const long long rs = (long long)G * r1;  // stride between this thread's i
        for (int a = 0; a < r0; ++a) {
          const T* xp = xc + ((long long)a * n + g) * r1 + b;
          double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
          int i = g;
          for (; i + 3 * G < n; i += 4 * G, xp += 4 * rs) {
            s0 += bulk_to_double(xp[0]);
            s1 += bulk_to_double(xp[rs]);
            s2 += bulk_to_double(xp[2 * rs]);
            s3 += bulk_to_double(xp[3 * rs]);
          }
          for (; i < n; i += G, xp += rs) s0 += bulk_to_double(xp[0]);
          acc += lk[a] * ((s0 + s1) + (s2 + s3));
        }
      }
      part[threadIdx.x] = acc;
      __syncthreads();
      if (threadIdx.x < nb && b < r1) {
        double t = 0.0;
        for (int q = 0; q < G; ++q) t += part[q * nb + tb];
        left[(long long)(k + 1) * rcap + b] = t;
      }
      __syncthreads();
    }
  }
  // right[k](a) = sum over (i, b) of X_k(a, i, b) right[k+1](b): one
  // wavefront per row a over the contiguous (i, b) block (the column of a
  // lane advances by 64 modulo r1), or the whole workgroup per row when the
  // core has fewer rows than wavefronts
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  for (int k = d - 1; k >= 0; --k) {
    const int r0 = X.ranks[k], r1 = X.ranks[k + 1], n = X.n[k];
    const T* xc = core_ptr<T>(X, k);
    const double* rk1 = right + (long long)(k + 1) * rcap;
    const int len = n * r1;
    if (r0 >= nw) {
      const int b0 = lane % r1, step = 64 % r1;
      for (int a = wv; a < r0; a += nw) {
        const T* row = xc + (long long)a * len;
        double s0 = 0.0, s1 = 0.0;
        int e = lane, b = b0;
        for (; e + 64 < len; e += 128) {
          const double x0 = bulk_to_double(row[e]), x1 = bulk_to_double(row[e + 64]);
          int b1 = b + step;
          if (b1 >= r1) b1 -= r1;
          s0 += x0 * rk1[b];
          s1 += x1 * rk1[b1];
          b = b1 + step;
          if (b >= r1) b -= r1;
        }
        if (e < len) s0 += bulk_to_double(row[e]) * rk1[b];
        double acc = s0 + s1;
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0) right[(long long)k * rcap + a] = acc;
      }
    } else {
      const int t = threadIdx.x, b0 = t % r1, step = 256 % r1;
      for (int a = 0; a < r0; ++a) {
        const T* row = xc + (long long)a * len;
        double s0 = 0.0, s1 = 0.0;
        int e = t, b = b0;
        for (; e + 256 < len; e += 512) {
          const double x0 = bulk_to_double(row[e]), x1 = bulk_to_double(row[e + 256]);
          int b1 = b + step;
          if (b1 >= r1) b1 -= r1;
          s0 += x0 * rk1[b];
          s1 += x1 * rk1[b1];
          b = b1 + step;
          if (b >= r1) b -= r1;
        }
        if (e < len) s0 += bulk_to_double(row[e]) * rk1[b];
        part[t] = s0 + s1;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
          if (t < h) part[t] += part[t + h];
          __syncthreads();
        }
        if (t == 0) right[(long long)k * rcap + a] = part[0];
        __syncthreads();
      }
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

// y += alpha x for adjoint trains of the same layout and ranks (cores and
// the log-scale adjoint)
__global__ void __launch_bounds__(256) adj_axpy_kernel(const DevTT* __restrict__ xs, const DevTT* __restrict__ ys,
                                                       double alpha) {
  const int f = blockIdx.z, k = blockIdx.y;
  const DevTT &X = xs[f], &Y = ys[f];
  if (k >= X.d) return;
  bool same = true;
  for (int j = 0; j <= X.d; ++j) same = same && X.ranks[j] == Y.ranks[j];
  if (!same) {
    if (blockIdx.x == 0 && threadIdx.x == 0 && k == 0) set_status(Y.status, TT_STATUS_CAPACITY);
    return;
  }
  const long long tot = (long long)X.ranks[k] * X.n[k] * X.ranks[k + 1];
  const double* xc = core_ptr<double>(X, k);
  double* yc = core_ptr<double>(Y, k);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x)
    yc[e] += alpha * xc[e];
  if (k == 0 && blockIdx.x == 0 && threadIdx.x == 0) *Y.log_scale += alpha * *X.log_scale;
}

// <Abar, B> = sum over cores of the stored entries + log-scale product, over
// the ranks the two trains share (index ranges beyond the smaller rank at a
// bond are skipped).  One workgroup per filter, fixed summation order.
__global__ void __launch_bounds__(256) adj_inner_kernel(const DevTT* __restrict__ as, const DevTT* __restrict__ bs,
                                                        double* __restrict__ out) {
  const int f = blockIdx.x;
  const DevTT &A = as[f], &Bt = bs[f];
  __shared__ double red[4];
  double acc = 0.0;
  for (int k = 0; k < A.d; ++k) {
    const int ra0 = A.ranks[k], ra1 = A.ranks[k + 1], rb0 = Bt.ranks[k], rb1 = Bt.ranks[k + 1], n = A.n[k];
    const int r0 = min(ra0, rb0), r1 = min(ra1, rb1);
    const double* ac = core_ptr<double>(A, k);
    const double* bc = core_ptr<double>(Bt, k);
    const long long tot = (long long)r0 * n * r1;
    for (long long e = threadIdx.x; e < tot; e += blockDim.x) {
      const int a = (int)(e / ((long long)n * r1));
      const int rem = (int)(e - (long long)a * n * r1);
      const int i = rem / r1, b = rem - (rem / r1) * r1;
      acc += ac[((long long)a * n + i) * ra1 + b] * bc[((long long)a * n + i) * rb1 + b];
    }
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) out[f] = acc + *A.log_scale * *Bt.log_scale;
}

// Alignment of a train T to a reference R of the same construction (a
// truncated-SVD build at nearby parameters), bond by bond from the left: the
// bond basis of T is rotated by the orthogonal polar factor O of the cosine
// matrix M(c, c') = <r_c, t_c'> / (|r_c| |t_c'|) between the columns of the
// left unfoldings of core k (T_k <- T_k O^T, T_{k+1} <- O T_{k+1}; the tensor
// is unchanged).  This removes sign flips and rotations among nearly equal
// singular values, which are choices of the build, not changes of the
// tensor.  The polar factor comes from a Jacobi SVD of the stacked matrix
// [M; I] (its lower block accumulates V): O = U V^T.  A bond whose cosine
// matrix has a singular value below 1e-6 (no counterpart) is left as is.
#define ALIGN_RMAX 64

// stacked [M; I] (2r x r, row-major) for bond k; r = the common bond rank
__global__ void __launch_bounds__(256) align_cos_kernel(const DevTT* __restrict__ refs, const DevTT* __restrict__ ts,
                                                        int k, double* __restrict__ buf, int* __restrict__ rbuf) {
  const int f = blockIdx.x;
  const DevTT &R = refs[f], &T = ts[f];
  double* X = buf + (long long)f * 2 * ALIGN_RMAX * ALIGN_RMAX;
  __shared__ double nr[ALIGN_RMAX], nt[ALIGN_RMAX];
  __shared__ double red[4];
  const int rr0 = R.ranks[k], rr1 = R.ranks[k + 1], rt0 = T.ranks[k], rt1 = T.ranks[k + 1], n = T.n[k];
  const int r = min(min(rr1, rt1), ALIGN_RMAX), r0 = min(rr0, rt0);
  const long long rows = (long long)r0 * n;
  const double* rc = core_ptr<double>(R, k);
  const double* tc = core_ptr<double>(T, k);
  for (int c = 0; c < r; ++c) {
    double a = 0.0, b = 0.0;
    for (long long e = threadIdx.x; e < rows; e += blockDim.x) {
      a += rc[e * rr1 + c] * rc[e * rr1 + c];
      b += tc[e * rt1 + c] * tc[e * rt1 + c];
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) {
      nr[c] = a > 0.0 ? 1.0 / sqrt(a) : 0.0;
      nt[c] = b > 0.0 ? 1.0 / sqrt(b) : 0.0;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
    const int c = e / r, c2 = e - (e / r) * r;
    double s = 0.0;
    for (long long w = 0; w < rows; ++w) s += rc[w * rr1 + c] * tc[w * rt1 + c2];
    X[(long long)c * r + c2] = s * nr[c] * nt[c2];
    X[(long long)(r + c) * r + c2] = c == c2 ? 1.0 : 0.0;
  }
  if (threadIdx.x == 0) rbuf[f] = r;
}

struct FAlignJacobi {
  double* buf;
  const int* rbuf;
  double* work;
  double* sigma;
  double* usv;
  __device__ bool operator()(int f, JacobiArgs& J) const {
    const int r = rbuf[f];
    J.rows = 2 * r;
    J.ncols = r;
    J.tol2 = 1e-30;
    J.x = buf + (long long)f * 2 * ALIGN_RMAX * ALIGN_RMAX;
    J.ldx = r;
    J.work = work + (long long)f * 2 * ALIGN_RMAX * ALIGN_RMAX;
    J.sigma = sigma + (long long)f * ALIGN_RMAX;
    J.usv = usv + (long long)f * 2 * ALIGN_RMAX * ALIGN_RMAX;
    J.ncols_out = nullptr;
    J.gcap = 2 * r;
    return r > 0;
  }
};

// O = U V^T from the Jacobi output (usv column c = [sigma_c u_c; v_c],
// column-major ld 2r); T_k <- T_k O^T, T_{k+1} <- O T_{k+1}
__global__ void __launch_bounds__(256) align_apply_kernel(const DevTT* __restrict__ ts, int k,
                                                          const double* __restrict__ sigma,
                                                          const double* __restrict__ usv,
                                                          const int* __restrict__ rbuf) {
  const int f = blockIdx.x;
  const DevTT& T = ts[f];
  const int r = rbuf[f];
  if (r <= 0) return;
  (void)sigma;
  const double* U = usv + (long long)f * 2 * ALIGN_RMAX * ALIGN_RMAX;
  __shared__ double O[ALIGN_RMAX * ALIGN_RMAX];
  __shared__ double tmp[256 / 64 * ALIGN_RMAX];
  __shared__ double sg[ALIGN_RMAX];
  // the upper block of column c is sigma_c u_c (sigma_c a singular value of M)
  for (int c = threadIdx.x; c < r; c += blockDim.x) {
    double s = 0.0;
    for (int a = 0; a < r; ++a) s += U[(long long)c * 2 * r + a] * U[(long long)c * 2 * r + a];
    sg[c] = sqrt(s);
  }
  __syncthreads();
  for (int c = 0; c < r; ++c)
    if (!(sg[c] > 1e-6)) return;  // same decision in every thread
  for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
    const int a = e / r, b = e - (e / r) * r;
    double s = 0.0;
    for (int c = 0; c < r; ++c) s += (U[(long long)c * 2 * r + a] / sg[c]) * U[(long long)c * 2 * r + r + b];
    O[e] = s;  // O(a, b) = sum_c u_c(a) v_c(b)
  }
  __syncthreads();
  const int rt0 = T.ranks[k], rt1 = T.ranks[k + 1], n = T.n[k];
  double* tc = core_ptr<double>(T, k);
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  double* tw = tmp + wid * ALIGN_RMAX;
  // columns of core k: each row (a, i) of the left unfolding, one wavefront per row
  for (long long row = wid; row < (long long)rt0 * n; row += nw) {
    double* tr = tc + row * rt1;
    if (lane < r) tw[lane] = tr[lane];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    double s = 0.0;
    if (lane < r)
      for (int c = 0; c < r; ++c) s += tw[c] * O[lane * r + c];  // (T O^T)(row, lane)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (lane < r) tr[lane] = s;
  }
  // rows of core k+1: each column (i, b) of its right unfolding
  const int n1 = T.n[k + 1], rt2 = T.ranks[k + 2];
  double* tn = core_ptr<double>(T, k + 1);
  const long long ncol = (long long)n1 * rt2;
  for (long long col = wid; col < ncol; col += nw) {
    if (lane < r) tw[lane] = tn[(long long)lane * ncol + col];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    double s = 0.0;
    if (lane < r)
      for (int c = 0; c < r; ++c) s += O[lane * r + c] * tw[c];  // (O T)(lane, col)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (lane < r) tn[(long long)lane * ncol + col] = s;
  }
}

}  // namespace ttg

namespace ttg {

// ---------------------------------------------------------------------------
// Adjoint of the likelihood build (Sec. 2.2 likelihood as a TT).  The
// (x_1, x_2) range block M (n0 x n1, max-shifted) is truncated by SVD into
// core 0 = M V_r and core 1 = V_r^T (V_r: leading right singular vectors).
// Rounding the two-core train A = (M^T, I_{n0}) to rank r yields exactly
// Y = (V_r, V_r^T M^T), the build's cores transposed and swapped, so the
// adjoint of the build is the rounding adjoint on A.  The dense train P
// holds the build's input: core 0 = M (bond 1 of full rank n1), core 1 =
// the identity, the linear-axis factors and the log-scale as in the build.
// ---------------------------------------------------------------------------
struct LikAdjJob {
  DevTT p, l, lbar, pbar;  // caller's trains
  DevTT a, y, ybar, abar;  // two-core trains in the workspace (range block only)
  int range;
};

// A, Y, Ybar of every range filter (one workgroup per filter)
__global__ void __launch_bounds__(256) lik_adj_pack_kernel(const LikAdjJob* __restrict__ jobs) {
  const LikAdjJob& J = jobs[blockIdx.x];
  if (!J.range) return;
  const int n0 = J.p.n[0], n1 = J.p.n[1], r = J.l.ranks[1];
  const double* m = core_ptr<double>(J.p, 0);
  double* a0 = core_ptr<double>(J.a, 0);
  double* a1 = core_ptr<double>(J.a, 1);
  for (int e = threadIdx.x; e < n0 * n1; e += blockDim.x) {
    const int i = e / n1, j = e - (e / n1) * n1;
    a0[(long long)j * n0 + i] = m[e];
  }
  for (int e = threadIdx.x; e < n0 * n0; e += blockDim.x) a1[e] = (e / n0 == e - (e / n0) * n0) ? 1.0 : 0.0;
  const double *l0 = core_ptr<double>(J.l, 0), *l1 = core_ptr<double>(J.l, 1);
  const double *b0 = core_ptr<double>(J.lbar, 0), *b1 = core_ptr<double>(J.lbar, 1);
  double *y0 = core_ptr<double>(J.y, 0), *y1 = core_ptr<double>(J.y, 1);
  double *yb0 = core_ptr<double>(J.ybar, 0), *yb1 = core_ptr<double>(J.ybar, 1);
  for (int e = threadIdx.x; e < n1 * r; e += blockDim.x) {  // Y_0(j, c) = L_1(c, j)
    const int j = e / r, c = e - (e / r) * r;
    y0[e] = l1[(long long)c * n1 + j];
    yb0[e] = b1[(long long)c * n1 + j];
  }
  for (int e = threadIdx.x; e < r * n0; e += blockDim.x) {  // Y_1(c, i) = L_0(i, c)
    const int c = e / n0, i = e - (e / n0) * n0;
    y1[e] = l0[(long long)i * r + c];
    yb1[e] = b0[(long long)i * r + c];
  }
  if (threadIdx.x == 0) {
    const int ra[3] = {1, n0, 1}, ry[3] = {1, r, 1};
    for (int j = 0; j < 3; ++j) {
      J.a.ranks[j] = ra[j];
      J.abar.ranks[j] = ra[j];
      J.y.ranks[j] = ry[j];
      J.ybar.ranks[j] = ry[j];
    }
    *J.a.log_scale = *J.y.log_scale = *J.ybar.log_scale = *J.abar.log_scale = 0.0;
    *J.a.status = *J.y.status = *J.ybar.status = *J.abar.status = 0;
  }
}

// Pbar: core 0 = Abar_0 transposed (range) or Lbar_0, core 1 zero (the build
// reads the identity core of P not at all) or Lbar_1, linear factors and the
// log-scale adjoint passed through (the build copies them).
__global__ void __launch_bounds__(256) lik_adj_unpack_kernel(const LikAdjJob* __restrict__ jobs) {
  const LikAdjJob& J = jobs[blockIdx.x];
  const int d = J.p.d;
  bool ok = true;
  for (int j = 0; j <= d; ++j) ok = ok && J.lbar.ranks[j] == J.l.ranks[j];
  for (int k = 0; k < d; ++k) {
    const int n = J.p.n[k];
    double* o = core_ptr<double>(J.pbar, k);
    if (J.range && k == 0) {
      const int n1 = J.p.n[1];
      const double* ab = core_ptr<double>(J.abar, 0);
      for (int e = threadIdx.x; e < n * n1; e += blockDim.x) {
        const int i = e / n1, j = e - (e / n1) * n1;
        o[e] = ab[(long long)j * n + i];
      }
    } else if (J.range && k == 1) {
      for (int e = threadIdx.x; e < n * n; e += blockDim.x) o[e] = 0.0;
    } else {
      const double* lb = core_ptr<double>(J.lbar, k);
      for (int e = threadIdx.x; e < n; e += blockDim.x) o[e] = lb[e];
    }
  }
  if (threadIdx.x == 0) {
    for (int j = 0; j <= d; ++j) J.pbar.ranks[j] = J.p.ranks[j];
    *J.pbar.log_scale = *J.lbar.log_scale;
    *J.pbar.status = ok ? 0 : TT_STATUS_CAPACITY;
  }
}

// the dense train P of every range filter: core 0 = the block, core 1 = I
__global__ void __launch_bounds__(256) lik_dense_pack_kernel(const DevTT* __restrict__ ps,
                                                             const FilterConst* __restrict__ fc,
                                                             const double* __restrict__ mbuf, long long mstride) {
  const int f = blockIdx.x;
  if (fc[f].meas_kind != 1) return;
  const DevTT& P = ps[f];
  const int n0 = P.n[0], n1 = P.n[1];
  const double* m = mbuf + f * mstride;
  double* c0 = core_ptr<double>(P, 0);
  double* c1 = core_ptr<double>(P, 1);
  for (int e = threadIdx.x; e < n0 * n1; e += blockDim.x) c0[e] = m[e];
  for (int e = threadIdx.x; e < n1 * n1; e += blockDim.x) c1[e] = (e / n1 == e - (e / n1) * n1) ? 1.0 : 0.0;
  if (threadIdx.x == 0) P.ranks[1] = n1;
}

}  // namespace ttg
