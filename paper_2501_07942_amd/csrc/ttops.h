// Kernels of the TT filter step that are not generic linear algebra:
// prediction by per-core convolution, Hadamard update, likelihood build,
// contractions for mass/normaliser/moments, prior and transition kernel.
#pragma once

#include "common.h"

// Per-filter constants of the grid and the measurement model.
struct FilterConst {
  int d;
  int n[TT_MAXD];
  double lo[TT_MAXD];
  double dx[TT_MAXD];
  double logdelta;
  int meas_kind;
  double sensor[2];
  double sigma_r, sigma_lin, lik_tol;
  int lik_max_rank;
  double m0[TT_MAXD], p0[TT_MAXD];
};

// ---------------------------------------------------------------------------
// Prediction: C_k(a*rp0+b, i, a2*rp1+b2) = sum_m K_k(a, m+h, a2) P_k(b, i-m, b2)
// (linear convolution cropped to the grid, P = 0 off the grid).
// grid.x = left pair (a, b), grid.y = core k, grid.z = filter.
// Each thread produces CONV_ROWS consecutive outputs along i of one column;
// the P fibre of row b (zero padded) and the kernel slice of row a sit in
// LDS, and taps are consumed in blocks of 8 from a register window.
// ---------------------------------------------------------------------------
#define CONV_ROWS 16
#define CONV_TB 8

template <typename T>
__global__ void __launch_bounds__(256) conv_kernel(const DevTT* __restrict__ kern,
                                                   const DevTT* __restrict__ pin,
                                                   const DevTT* __restrict__ xout, int all_cores) {
  const int f = blockIdx.z, k = blockIdx.y;
  const DevTT& K = kern[f];
  const DevTT& P = pin[f];
  const DevTT& X = xout[f];
  if (k >= P.d) return;
  // the fused prediction produces the interior cores inside the rounding;
  // only the first and last cores are materialised then
  if (!all_cores && k != 0 && k != P.d - 1) return;
  const int rk0 = K.ranks[k], rk1 = K.ranks[k + 1];
  const int rp0 = P.ranks[k], rp1 = P.ranks[k + 1];
  const int R0 = rk0 * rp0, R1 = rk1 * rp1;
  if ((int)blockIdx.x >= R0) return;
  if (R0 > X.cap[k] || R1 > X.cap[k + 1]) return;  // capacity flagged at init
  const int a = blockIdx.x / rp0, b = blockIdx.x % rp0;
  const int n = P.n[k];
  const int taps = K.n[k];
  const int h = (taps - 1) / 2;
  const int taps_pad = (taps + CONV_TB - 1) / CONV_TB * CONV_TB;
  const int front = CONV_TB;                       // extra zeros before P
  const int plen = front + n + 2 * h + CONV_ROWS;  // padded fibre length
  extern __shared__ unsigned char smem_raw[];
  T* Ks = reinterpret_cast<T*>(smem_raw);  // [taps_pad][rk1]
  T* Ps = Ks + taps_pad * rk1;             // [plen][rp1]
  const T* kc = core_ptr<T>(K, k) + (long long)a * taps * rk1;
  const T* pc = core_ptr<T>(P, k) + (long long)b * n * rp1;
  for (int e = threadIdx.x; e < taps_pad * rk1; e += blockDim.x)
    Ks[e] = (e < taps * rk1) ? kc[e] : (T)0;
  for (int e = threadIdx.x; e < plen * rp1; e += blockDim.x) {
    const int row = e / rp1 - front - h;  // grid index of this padded row
    Ps[e] = (row >= 0 && row < n) ? pc[(long long)row * rp1 + (e % rp1)] : (T)0;
  }
  __syncthreads();
  T* xc = core_ptr<T>(X, k) + (long long)blockIdx.x * n * R1;
  const int nblk = (n + CONV_ROWS - 1) / CONV_ROWS;
  const int tasks = R1 * nblk;
  for (int t = threadIdx.x; t < tasks; t += blockDim.x) {
    const int j = t % R1, blk = t / R1;
    const int a2 = j / rp1, b2 = j % rp1;
    const int i0 = blk * CONV_ROWS;
    T acc[CONV_ROWS];
#pragma unroll
    for (int r = 0; r < CONV_ROWS; ++r) acc[r] = (T)0;
    // output i uses Ppad[front + i + 2h - tm] for tap tm (offset m = tm - h);
    // whole blocks of CONV_TB taps, then the remaining taps one by one
    const int tfull = taps / CONV_TB * CONV_TB;
    for (int tm0 = 0; tm0 < tfull; tm0 += CONV_TB) {
      T kv[CONV_TB];
#pragma unroll
      for (int u = 0; u < CONV_TB; ++u) kv[u] = Ks[(tm0 + u) * rk1 + a2];
      // window w[v] = Ppad[base + v], base = front + i0 + 2h - tm0 - (TB-1)
      const int base = front + i0 + 2 * h - tm0 - (CONV_TB - 1);
      T w[CONV_ROWS + CONV_TB - 1];
#pragma unroll
      for (int v = 0; v < CONV_ROWS + CONV_TB - 1; ++v) w[v] = Ps[(base + v) * rp1 + b2];
#pragma unroll
      for (int u = 0; u < CONV_TB; ++u)
#pragma unroll
        for (int r = 0; r < CONV_ROWS; ++r) acc[r] += kv[u] * w[r - u + CONV_TB - 1];
    }
    for (int tm = tfull; tm < taps; ++tm) {
      const T kvt = Ks[tm * rk1 + a2];
      const int base = front + i0 + 2 * h - tm;
#pragma unroll
      for (int r = 0; r < CONV_ROWS; ++r) acc[r] += kvt * Ps[(base + r) * rp1 + b2];
    }
    // the product is far larger than the caches and is read back by the
    // rounding's own sweep: stream it past them
#pragma unroll
    for (int r = 0; r < CONV_ROWS; ++r) {
      const int i = i0 + r;
      if (i < n) __builtin_nontemporal_store(acc[r], &xc[(long long)i * R1 + j]);
    }
  }
}

// ranks/log-scale/status of a product TT (convolution or Hadamard):
// out.ranks = A.ranks * B.ranks, log_scale = sum; capacity overflow flagged.
__global__ void product_init_kernel(const DevTT* __restrict__ A, const DevTT* __restrict__ B,
                                    const DevTT* __restrict__ O, int nf) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const DevTT &a = A[f], &b = B[f], &o = O[f];
  int bad = 0;
  for (int j = 0; j <= o.d; ++j) {
    int r = a.ranks[j] * b.ranks[j];
    if (r > o.cap[j]) {
      bad = 1;
      r = o.cap[j];  // keep every later read inside the reserved storage
    }
    o.ranks[j] = r;
  }
  *o.log_scale = *a.log_scale + *b.log_scale;
  int st = *b.status;
  if (bad) st |= TT_STATUS_CAPACITY;
  *o.status = st;
}

// ---------------------------------------------------------------------------
// Hadamard: H_k(a*rp0+b, i, a2*rp1+b2) = L_k(a, i, a2) * P_k(b, i, b2)
// (Kronecker product of the core slices).  L is FP64, P and H bulk type.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) hadamard_kernel(const DevTT* __restrict__ lik,
                                                       const DevTT* __restrict__ pin,
                                                       const DevTT* __restrict__ hout) {
  // one filter per blockIdx.z; the workgroups of a filter walk all its cores
  // (few workgroups: the chip starts them at a bounded rate), each core as a
  // grid-stride loop over its output elements e = (row (a, b), i, column
  // (a', b')), every element written once, in order
  const int f = blockIdx.z;
  const DevTT &L = lik[f], &P = pin[f], &H = hout[f];
  const int stride = gridDim.x * blockDim.x;
  const int t0 = blockIdx.x * blockDim.x + threadIdx.x;
  for (int k = 0; k < P.d; ++k) {
    const int rl1 = L.ranks[k + 1];
    const int rp0 = P.ranks[k], rp1 = P.ranks[k + 1];
    const int R0 = L.ranks[k] * rp0, R1 = rl1 * rp1;
    if (R0 > H.cap[k] || R1 > H.cap[k + 1]) continue;
    const int n = P.n[k];
    if ((long long)R0 * n * R1 > 0x7fffffffLL) {  // 32-bit element indices below
      if (t0 == 0) set_status(H.status, TT_STATUS_CAPACITY);
      continue;
    }
    const double* lc = core_ptr<double>(L, k);
    const T* pc = core_ptr<T>(P, k);
    T* hc = core_ptr<T>(H, k);
    const int nR1 = n * R1;
    const int tot = R0 * nR1;
    const bool vec = sizeof(T) == 4 && (R1 & 3) == 0 && (rp1 & 3) == 0 &&
                     ((reinterpret_cast<uintptr_t>(hc) | reinterpret_cast<uintptr_t>(pc)) & 15) == 0;
    if (vec && stride % (R1 >> 2) == 0) {
      // a thread keeps one quad of columns (a', b'..b'+3) and steps over the
      // positions (row, i); one 16-byte load of P and one 16-byte store of H
      const int Q = R1 >> 2, qj = t0 % Q, pstep = stride / Q;
      const int j = qj << 2, a2 = j / rp1, b2 = j - a2 * rp1;
      const int npos = R0 * n;
      const int drow = pstep / n, di = pstep - drow * n;
      int p = t0 / Q;
      int row = p / n, i = p - row * n;
      for (; p < npos; p += pstep) {
        const int a = row / rp0, b = row - a * rp0;
        const double lv = lc[(a * n + i) * rl1 + a2];
        const float4 pv = *reinterpret_cast<const float4*>(pc + (b * n + i) * rp1 + b2);
        typedef float had_f4 __attribute__((ext_vector_type(4)));
        const had_f4 o = {from_double<float>(lv * (double)pv.x), from_double<float>(lv * (double)pv.y),
                          from_double<float>(lv * (double)pv.z), from_double<float>(lv * (double)pv.w)};
        __builtin_nontemporal_store(o, reinterpret_cast<had_f4*>(hc + (row * n + i) * R1 + j));
        row += drow;
        i += di;
        if (i >= n) {
          i -= n;
          ++row;
        }
      }
      continue;
    }
    if (vec) {
      // four consecutive columns share a' and read four consecutive b' of P:
      // one 16-byte load of P and one 16-byte store of H
      for (int q = t0; q < (tot >> 2); q += stride) {
        const int e = q << 2;
        const int row = e / nR1, rem = e - row * nR1;
        const int i = rem / R1, j = rem - i * R1;
        const int a = row / rp0, b = row - a * rp0;
        const int a2 = j / rp1, b2 = j - a2 * rp1;
        const double lv = lc[(a * n + i) * rl1 + a2];
        const float4 pv = *reinterpret_cast<const float4*>(pc + (b * n + i) * rp1 + b2);
        float4 o;
        o.x = from_double<float>(lv * (double)pv.x);
        o.y = from_double<float>(lv * (double)pv.y);
        o.z = from_double<float>(lv * (double)pv.z);
        o.w = from_double<float>(lv * (double)pv.w);
        *reinterpret_cast<float4*>(hc + e) = o;
      }
      continue;
    }
    for (int e = t0; e < tot; e += stride) {
      const int row = e / nR1, rem = e - row * nR1;
      const int i = rem / R1, j = rem - i * R1;
      const int a = row / rp0, b = row - a * rp0;
      const int a2 = j / rp1, b2 = j - a2 * rp1;
      hc[e] = from_double<T>(lc[(a * n + i) * rl1 + a2] * bulk_to_double(pc[(b * n + i) * rp1 + b2]));
    }
  }
}

// ---------------------------------------------------------------------------
// sum of all entries: v <- v * (sum_i A_k(:, i, :)) core by core, FP64.
// One workgroup per filter.  Writes log(sum) + logdelta + log_scale to
// out[f*stride] (NaN and a status bit when the sum is not positive/finite).
// Deterministic: fixed-order partial sums.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) sum_kernel(const DevTT* __restrict__ tt,
                                                  const FilterConst* __restrict__ fc,
                                                  double* __restrict__ out, long long stride,
                                                  double* __restrict__ vbuf, int vcap) {
  const int f = blockIdx.x;
  const DevTT& A = tt[f];
  double* v = vbuf + (long long)f * 2 * vcap;
  double* vn = v + vcap;
  __shared__ double part[256];
  const int tid = threadIdx.x;
  if (tid == 0) v[0] = 1.0;
  __syncthreads();
  for (int k = 0; k < A.d; ++k) {
    const int r0 = A.ranks[k], r1 = A.ranks[k + 1], n = A.n[k];
    const T* c = core_ptr<T>(A, k);
    for (int j0 = 0; j0 < r1; j0 += 256) {
      const int jc = min(256, r1 - j0);
      const int groups = max(1, 256 / jc);
      const int g = tid / jc, j = j0 + tid % jc;
      double s = 0.0;
      if (g < groups && tid < groups * jc) {
        for (long long q = g; q < (long long)r0 * n; q += groups) {
          const int aa = (int)(q / n);
          s += v[aa] * bulk_to_double(c[q * r1 + j]);
        }
      }
      part[tid] = s;
      __syncthreads();
      if (tid < jc) {
        double t = 0.0;
        for (int gg = 0; gg < groups; ++gg) t += part[gg * jc + tid];
        vn[j0 + tid] = t;
      }
      __syncthreads();
    }
    for (int j = tid; j < r1; j += 256) v[j] = vn[j];
    __syncthreads();
  }
  if (tid == 0) {
    const double s = v[0];
    double r;
    if (!(s == s) || fabs(s) > 1.7e308) {
      r = __longlong_as_double(0x7ff8000000000000LL);
      set_status(A.status, TT_STATUS_NONFINITE);
    } else if (!(s > 0.0)) {
      r = __longlong_as_double(0x7ff8000000000000LL);
      set_status(A.status, TT_STATUS_NONPOSITIVE);
    } else {
      r = log(s) + fc[f].logdelta + *A.log_scale;
    }
    if (*A.status & (TT_STATUS_NONFINITE | TT_STATUS_NONPOSITIVE))
      r = __longlong_as_double(0x7ff8000000000000LL);
    out[f * stride] = r;
  }
}

// ---------------------------------------------------------------------------
// normalisation and moments (one workgroup per filter).  Per core the
// contractions S^v_k = sum_i v(i) A_k(:, i, :) for v in {1, xi, xi^2} go to
// scratch; prefix/suffix chains then give mass, means and second moments.
// log_scale is decreased by log(mass) so the TT integrates to one.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) moments_kernel(const DevTT* __restrict__ tt,
                                                      const FilterConst* __restrict__ fc,
                                                      double* __restrict__ log_mass, long long lm_stride,
                                                      double* __restrict__ mean, long long mean_stride,
                                                      double* __restrict__ cov, long long cov_stride,
                                                      double* __restrict__ scratch, long long scr_per_filter,
                                                      int rcap) {
  const int f = blockIdx.x;
  const DevTT& A = tt[f];
  const FilterConst& C = fc[f];
  const int d = A.d, tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6, nwv = blockDim.x >> 6;
  const long long mat = (long long)rcap * rcap;
  double* S = scratch + f * scr_per_filter;      // [3][d][rcap*rcap]
  double* left = S + 3 * d * mat;                // [d+1][rcap]
  double* right = left + (d + 1) * rcap;         // [d+1][rcap]
  double* tmp = right + (d + 1) * rcap;          // [2][rcap] per wavefront (chains below)
  const bool want = (mean != nullptr);
  __shared__ double s_mean[TT_MAXD];
  __shared__ double s_total;
  __shared__ int s_ok;
  // per-core contractions with 1, xi and xi^2: one thread per (a, b) sums
  // over the grid index (consecutive threads read consecutive b)
  for (int k = 0; k < d; ++k) {
    const int r0 = A.ranks[k], r1 = A.ranks[k + 1], n = A.n[k];
    const T* c = core_ptr<T>(A, k);
    for (int q = tid; q < r0 * r1; q += blockDim.x) {
      const int a = q / r1, bq = q - (q / r1) * r1;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 8
      for (int i = 0; i < n; ++i) {
        const double x = C.lo[k] + i * C.dx[k];
        const double v = bulk_to_double(c[((long long)a * n + i) * r1 + bq]);
        s0 += v;
        if (want) {
          s1 += x * v;
          s2 += x * x * v;
        }
      }
      S[(0 * d + k) * mat + a * r1 + bq] = s0;
      if (want) {
        S[(1 * d + k) * mat + a * r1 + bq] = s1;
        S[(2 * d + k) * mat + a * r1 + bq] = s2;
      }
    }
  }
  __syncthreads();
  // prefix chains left[k] (1 x r_k) and suffix right[k] (r_k x 1) of S^1
  if (tid == 0) {
    left[0] = 1.0;
    right[d * rcap] = 1.0;
  }
  __syncthreads();
  for (int k = 0; k < d; ++k) {
    const int r0 = A.ranks[k], r1 = A.ranks[k + 1];
    for (int bq = tid; bq < r1; bq += blockDim.x) {
      double s = 0.0;
      for (int a = 0; a < r0; ++a) s += left[k * rcap + a] * S[(0 * d + k) * mat + a * r1 + bq];
      left[(k + 1) * rcap + bq] = s;
    }
    const int kk = d - 1 - k;  // the suffix chain advances at the same time
    const int q0 = A.ranks[kk], q1 = A.ranks[kk + 1];
    for (int a = tid; a < q0; a += blockDim.x) {
      double s = 0.0;
      for (int bq = 0; bq < q1; ++bq) s += S[(0 * d + kk) * mat + a * q1 + bq] * right[(kk + 1) * rcap + bq];
      right[kk * rcap + a] = s;
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double total = left[d * rcap];
    int st = *A.status;
    if (!(total == total) || fabs(total) > 1.7e308) st |= TT_STATUS_NONFINITE;
    else if (!(total > 0.0)) st |= TT_STATUS_NONPOSITIVE;
    const bool ok = (st & (TT_STATUS_NONFINITE | TT_STATUS_NONPOSITIVE)) == 0;
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    const double lm = ok ? log(total) + C.logdelta + *A.log_scale : nan;
    if (log_mass) log_mass[f * lm_stride] = lm;
    if (ok) *A.log_scale -= lm;
    if (st != *A.status) atomicOr(A.status, st);
    s_total = total;
    s_ok = ok ? 1 : 0;
  }
  __syncthreads();
  if (!want) return;
  const double total = s_total;
  const bool ok = s_ok != 0;
  const double nan = __longlong_as_double(0x7ff8000000000000LL);
  // means and E[x_l^2]: one wavefront per axis reduces left_l S_l right_{l+1}
  for (int l = wv; l < d; l += nwv) {
    const int r0 = A.ranks[l], r1 = A.ranks[l + 1];
    double m1 = 0.0, m2 = 0.0;
    for (int q = lane; q < r0 * r1; q += 64) {
      const int a = q / r1, bq = q - (q / r1) * r1;
      const double lr = left[l * rcap + a] * right[(l + 1) * rcap + bq];
      m1 += lr * S[(1 * d + l) * mat + q];
      m2 += lr * S[(2 * d + l) * mat + q];
    }
    m1 = wave_sum(m1) / total;
    m2 = wave_sum(m2) / total;
    if (lane == 0) {
      s_mean[l] = m1;
      mean[f * mean_stride + l] = ok ? m1 : nan;
      if (cov) cov[f * cov_stride + l * d + l] = ok ? m2 - m1 * m1 : nan;
    }
  }
  if (!cov) return;
  __syncthreads();
  // off-diagonal E[x_l x_j], l < j: one wavefront per chain l carries
  // w = left_l S^xi_l S^1_{l+1} ... and closes it with S^xi_j right_{j+1}
  for (int l = wv; l < d - 1; l += nwv) {
    double* w = tmp + (long long)wv * 2 * rcap;
    double* w2 = w + rcap;
    {
      const int r0 = A.ranks[l], r1 = A.ranks[l + 1];
      for (int bq = lane; bq < r1; bq += 64) {
        double s = 0.0;
        for (int a = 0; a < r0; ++a) s += left[l * rcap + a] * S[(1 * d + l) * mat + a * r1 + bq];
        w[bq] = s;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    for (int j = l + 1; j < d; ++j) {
      const int r0 = A.ranks[j], r1 = A.ranks[j + 1];
      double e = 0.0;
      for (int bq = lane; bq < r1; bq += 64) {
        double u = 0.0, nw = 0.0;
        for (int a = 0; a < r0; ++a) {
          const double wa = w[a];
          u += wa * S[(1 * d + j) * mat + a * r1 + bq];
          nw += wa * S[(0 * d + j) * mat + a * r1 + bq];
        }
        e += u * right[(j + 1) * rcap + bq];
        w2[bq] = nw;
      }
      e = wave_sum(e);
      if (lane == 0) {
        const double cv = e / total - s_mean[l] * s_mean[j];
        cov[f * cov_stride + l * d + j] = ok ? cv : nan;
        cov[f * cov_stride + j * d + l] = ok ? cv : nan;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      double* t = w;
      w = w2;
      w2 = t;
    }
  }
}

// ---------------------------------------------------------------------------
// Smallest value over every 1-D marginal of a TT: the sums of its point
// values over all axes but one, times exp(log_scale) (the negativity monitor:
// the paper reports negative PMD values, Sec. 5.1 and Sec. 6).  Per core the
// sums over the grid index S_k = sum_i A_k(:, i, :), prefix and suffix
// chains of them, then per axis l and grid point i
// left_l A_l(:, i, :) right_{l+1}.  One workgroup per filter;
// scratch per filter: d rcap^2 + 2 (d + 1) rcap doubles.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) marginal_min_kernel(const DevTT* __restrict__ tt, double* __restrict__ out,
                                                           long long stride, double* __restrict__ scratch,
                                                           long long spf, int rcap) {
  const int f = blockIdx.x;
  const DevTT& A = tt[f];
  const int d = A.d, tid = threadIdx.x;
  const long long mat = (long long)rcap * rcap;
  double* S = scratch + f * spf;          // [d][rcap * rcap]
  double* left = S + d * mat;             // [d + 1][rcap]
  double* right = left + (d + 1) * rcap;  // [d + 1][rcap]
  __shared__ double smin[256];
  for (int k = 0; k < d; ++k) {
    const int r0 = A.ranks[k], r1 = A.ranks[k + 1], n = A.n[k];
    const T* c = core_ptr<T>(A, k);
    for (int q = tid; q < r0 * r1; q += blockDim.x) {
      const int a = q / r1, bq = q - (q / r1) * r1;
      double s0 = 0.0;
      for (int i = 0; i < n; ++i) s0 += bulk_to_double(c[((long long)a * n + i) * r1 + bq]);
      S[k * mat + a * r1 + bq] = s0;
    }
  }
  if (tid == 0) {
    left[0] = 1.0;
    right[d * rcap] = 1.0;
  }
  __syncthreads();
  for (int k = 0; k < d; ++k) {
    const int r0 = A.ranks[k], r1 = A.ranks[k + 1];
    for (int bq = tid; bq < r1; bq += blockDim.x) {
      double s = 0.0;
      for (int a = 0; a < r0; ++a) s += left[k * rcap + a] * S[k * mat + a * r1 + bq];
      left[(k + 1) * rcap + bq] = s;
    }
    const int kk = d - 1 - k;
    const int q0 = A.ranks[kk], q1 = A.ranks[kk + 1];
    for (int a = tid; a < q0; a += blockDim.x) {
      double s = 0.0;
      for (int bq = 0; bq < q1; ++bq) s += S[kk * mat + a * q1 + bq] * right[(kk + 1) * rcap + bq];
      right[kk * rcap + a] = s;
    }
    __syncthreads();
  }
  double mn = 1.7e308;
  for (int l = 0; l < d; ++l) {
    const int r0 = A.ranks[l], r1 = A.ranks[l + 1], n = A.n[l];
    const T* c = core_ptr<T>(A, l);
    for (int i = tid; i < n; i += blockDim.x) {
      double v = 0.0;
      for (int a = 0; a < r0; ++a) {
        const T* row = c + ((long long)a * n + i) * r1;
        double w = 0.0;
        for (int bq = 0; bq < r1; ++bq) w += bulk_to_double(row[bq]) * right[(l + 1) * rcap + bq];
        v += left[l * rcap + a] * w;
      }
      mn = fmin(mn, v);
    }
  }
  smin[tid] = mn;
  __syncthreads();
  for (int o = blockDim.x / 2; o > 0; o >>= 1) {
    if (tid < o) smin[tid] = fmin(smin[tid], smin[tid + o]);
    __syncthreads();
  }
  if (tid == 0) out[f * stride] = smin[0] * exp(*A.log_scale);
}

// ---------------------------------------------------------------------------
// balance: scale the last core to unit Frobenius norm, log_scale += log(norm)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) balance_kernel(const DevTT* __restrict__ tt) {
  const int f = blockIdx.x;
  const DevTT& A = tt[f];
  const int k = A.d - 1;
  T* c = core_ptr<T>(A, k);
  const long long tot = (long long)A.ranks[k] * A.n[k] * A.ranks[k + 1];
  __shared__ double red[8];
  double s = 0.0;
  for (long long e = threadIdx.x; e < tot; e += blockDim.x) {
    const double x = bulk_to_double(c[e]);
    s += x * x;
  }
  s = block_sum(s, red);
  const double nrm = sqrt(s);
  if (!(nrm > 0.0) || !(nrm < 1.7e308)) {
    if (threadIdx.x == 0) set_status(A.status, nrm == 0.0 ? TT_STATUS_NONPOSITIVE : TT_STATUS_NONFINITE);
    return;
  }
  const double inv = 1.0 / nrm;
  for (long long e = threadIdx.x; e < tot; e += blockDim.x) c[e] = from_double<T>(bulk_to_double(c[e]) * inv);
  if (threadIdx.x == 0) *A.log_scale += log(nrm);
}

// ---------------------------------------------------------------------------
// Gaussian prior with diagonal covariance: rank-one cores, each scaled to a
// unit maximum, the shifts and normalising constants in log_scale.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) prior_kernel(const DevTT* __restrict__ tt,
                                                    const FilterConst* __restrict__ fc) {
  const int f = blockIdx.x;
  const DevTT& A = tt[f];
  const FilterConst& C = fc[f];
  __shared__ double red[8];
  double lsum = 0.0;
  for (int k = 0; k < A.d; ++k) {
    const int n = A.n[k];
    double mx = -1e308;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double x = C.lo[k] + i * C.dx[k] - C.m0[k];
      mx = fmax(mx, -0.5 * x * x / C.p0[k]);
    }
    // block max via negated sums is awkward; use shared reduction
    __shared__ double smx[256];
    smx[threadIdx.x] = mx;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
      if ((int)threadIdx.x < o) smx[threadIdx.x] = fmax(smx[threadIdx.x], smx[threadIdx.x + o]);
      __syncthreads();
    }
    mx = smx[0];
    __syncthreads();
    T* c = core_ptr<T>(A, k);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double x = C.lo[k] + i * C.dx[k] - C.m0[k];
      c[i] = from_double<T>(exp(-0.5 * x * x / C.p0[k] - mx));
    }
    lsum += mx - 0.5 * log(2.0 * M_PI * C.p0[k]);
  }
  (void)red;
  if (threadIdx.x == 0) {
    for (int j = 0; j <= A.d; ++j) A.ranks[j] = 1;
    *A.log_scale = lsum;
    *A.status = 0;
  }
}

// ---------------------------------------------------------------------------
// Likelihood, part 1 (one workgroup per filter): the linear axes become
// rank-one cores exp(log N(z_j; xi, sigma_lin^2) - max); for the range model
// the dense block M(i1, i2) = exp(log N(z_0; ||(xi_1, xi_2) - s||, sigma_r^2)
// - max) is written row-major to mbuf.  All shifts and constants go to
// log_scale.  Ranks are set to 1 everywhere (bond 1 is set by part 2).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) lik_dense_kernel(const DevTT* __restrict__ lik,
                                                        const FilterConst* __restrict__ fc,
                                                        const double* __restrict__ z, long long zstride,
                                                        double* __restrict__ mbuf, long long mstride) {
  const int f = blockIdx.x;
  const DevTT& L = lik[f];
  const FilterConst& C = fc[f];
  const double* zf = z + f * zstride;
  __shared__ double smx[256];
  const int tid = threadIdx.x;
  double lsum = 0.0;
  const int first_lin = (C.meas_kind == 0) ? 0 : 2;
  const double slin2 = C.sigma_lin * C.sigma_lin;
  for (int k = first_lin; k < C.d; ++k) {
    const double zk = zf[C.meas_kind == 0 ? k : k - 1];
    const int n = C.n[k];
    double mx = -1e308;
    for (int i = tid; i < n; i += blockDim.x) {
      const double e = zk - (C.lo[k] + i * C.dx[k]);
      mx = fmax(mx, -0.5 * e * e / slin2);
    }
    smx[tid] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) smx[tid] = fmax(smx[tid], smx[tid + o]);
      __syncthreads();
    }
    mx = smx[0];
    __syncthreads();
    double* c = core_ptr<double>(L, k);
    for (int i = tid; i < n; i += blockDim.x) {
      const double e = zk - (C.lo[k] + i * C.dx[k]);
      c[i] = exp(-0.5 * e * e / slin2 - mx);
    }
    lsum += mx - 0.5 * log(2.0 * M_PI * slin2);
  }
  if (C.meas_kind == 1) {
    const int n0 = C.n[0], n1 = C.n[1];
    const double sr2 = C.sigma_r * C.sigma_r;
    double mx = -1e308;
    for (int e = tid; e < n0 * n1; e += blockDim.x) {
      const int i = e / n1, j = e % n1;
      const double x1 = C.lo[0] + i * C.dx[0] - C.sensor[0];
      const double x2 = C.lo[1] + j * C.dx[1] - C.sensor[1];
      const double r = zf[0] - sqrt(x1 * x1 + x2 * x2);
      mx = fmax(mx, -0.5 * r * r / sr2);
    }
    smx[tid] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o) smx[tid] = fmax(smx[tid], smx[tid + o]);
      __syncthreads();
    }
    mx = smx[0];
    __syncthreads();
    double* m = mbuf + f * mstride;
    for (int e = tid; e < n0 * n1; e += blockDim.x) {
      const int i = e / n1, j = e % n1;
      const double x1 = C.lo[0] + i * C.dx[0] - C.sensor[0];
      const double x2 = C.lo[1] + j * C.dx[1] - C.sensor[1];
      const double r = zf[0] - sqrt(x1 * x1 + x2 * x2);
      m[e] = exp(-0.5 * r * r / sr2 - mx);
    }
    lsum += mx - 0.5 * log(2.0 * M_PI * sr2);
  }
  if (tid == 0) {
    for (int j = 0; j <= C.d; ++j) L.ranks[j] = 1;
    *L.log_scale = lsum;
    if (!(lsum == lsum)) atomicOr(L.status, TT_STATUS_NONFINITE);
  }
}

// ---------------------------------------------------------------------------
// dense transition kernel K(m) = c * exp(-0.5 y^T Q^{-1} y), y = Delta o m,
// over the offset box (row-major, axis 0 slowest); c includes the Gaussian
// constant and the cell volume.
// ---------------------------------------------------------------------------
struct KernelEvalArgs {
  int d;
  int taps[TT_MAXD];
  double dx[TT_MAXD];
  double qinv[64];
  double cnorm;
  long long total;
};

// one filter per blockIdx.y; filter f writes out + f * ostride
__global__ void __launch_bounds__(256) kernel_dense_kernel(const KernelEvalArgs* __restrict__ args,
                                                           double* __restrict__ outb, long long ostride) {
  const KernelEvalArgs& a = args[blockIdx.y];
  double* out = outb + blockIdx.y * ostride;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < a.total;
       e += (long long)gridDim.x * blockDim.x) {
    double y[8];
    long long rem = e;
    for (int l = a.d - 1; l >= 0; --l) {
      const int t = (int)(rem % a.taps[l]);
      rem /= a.taps[l];
      y[l] = (t - (a.taps[l] - 1) / 2) * a.dx[l];
    }
    double q = 0.0;
    for (int l = 0; l < a.d; ++l)
      for (int j = 0; j < a.d; ++j) q += y[l] * a.qinv[l * a.d + j] * y[j];
    out[e] = a.cnorm * exp(-0.5 * q);
  }
}

// copy cores of an FP64 TT into a TT of type T with the same ranks
template <typename T>
__global__ void __launch_bounds__(256) convert_tt_kernel(const DevTT* __restrict__ src,
                                                         const DevTT* __restrict__ dst) {
  const int f = blockIdx.y;
  const DevTT &S = src[f], &D = dst[f];
  for (int k = 0; k < S.d; ++k) {
    const long long tot = (long long)S.ranks[k] * S.n[k] * S.ranks[k + 1];
    const double* s = core_ptr<double>(S, k);
    T* o = core_ptr<T>(D, k);
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
         e += (long long)gridDim.x * blockDim.x)
      o[e] = from_double<T>(s[e]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int j = 0; j <= S.d; ++j) D.ranks[j] = S.ranks[j];
    *D.log_scale = *S.log_scale;
    *D.status = *S.status;
  }
}

// copy a TT into a TT of the same type and modes whose capacities may differ:
// ranks, log-scale and the stored cores, repacked at the destination's
// offsets.  A rank above the destination's capacity copies nothing and sets
// TT_STATUS_CAPACITY on the status word of the caller's side (the source when
// report_src, else the destination); otherwise the destination's status word,
// when it has one, is cleared.
template <typename T>
__global__ void __launch_bounds__(256) copy_tt_kernel(const DevTT* __restrict__ src, const DevTT* __restrict__ dst,
                                                      int report_src) {
  const int f = blockIdx.y;
  const DevTT &S = src[f], &D = dst[f];
  bool fits = S.d == D.d;
  for (int j = 0; fits && j <= S.d; ++j) fits = S.ranks[j] >= 1 && S.ranks[j] <= D.cap[j];
  for (int k = 0; fits && k < S.d; ++k) fits = S.n[k] == D.n[k];
  if (!fits) {
    if (blockIdx.x == 0 && threadIdx.x == 0) set_status(report_src ? S.status : D.status, TT_STATUS_CAPACITY);
    return;
  }
  for (int k = 0; k < S.d; ++k) {
    const long long tot = (long long)S.ranks[k] * S.n[k] * S.ranks[k + 1];
    const T* s = core_ptr<T>(S, k);
    T* o = core_ptr<T>(D, k);
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot;
         e += (long long)gridDim.x * blockDim.x)
      o[e] = s[e];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int j = 0; j <= S.d; ++j) D.ranks[j] = S.ranks[j];
    *D.log_scale = *S.log_scale;
    if (D.status) *D.status = 0;
  }
}

// ---------------------------------------------------------------------------
// Normaliser c_k = <L, P> * delta (Sec. 2.2 eq. pmf_filtrace_b; Sec. 4.1
// 'dot') computed from the two factors, never from their Hadamard product:
// per core, t(a', b, i) = sum_a v(a, b) L(a, i, a') and then
// v'(a', b') = sum_{b, i} t(a', b, i) P(b, i, b').  One workgroup per
// filter, one wavefront per output entry, fixed summation order.
// Writes log(c) + logdelta + log_scale(L) + log_scale(P) to out[f*stride].
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) dot_kernel(const DevTT* __restrict__ lik, const DevTT* __restrict__ pin,
                                                  const FilterConst* __restrict__ fc, double* __restrict__ out,
                                                  long long stride, double* __restrict__ vbuf, long long vstride,
                                                  long long tofs) {
  const int f = blockIdx.x;
  const DevTT &L = lik[f], &P = pin[f];
  double* v = vbuf + f * vstride;
  double* t = v + tofs;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid == 0) v[0] = 1.0;
  __syncthreads();
  for (int k = 0; k < P.d; ++k) {
    const int l0 = L.ranks[k], l1 = L.ranks[k + 1], p0 = P.ranks[k], p1 = P.ranks[k + 1], n = P.n[k];
    const double* lc = core_ptr<double>(L, k);
    const T* pc = core_ptr<T>(P, k);
    const int nt = l1 * p0 * n;  // 32-bit index arithmetic
    const int pn = p0 * n;
    for (int e = tid; e < nt; e += blockDim.x) {
      const int a2 = e / pn;
      const int rem = e - a2 * pn;
      const int b = rem / n, i = rem - (rem / n) * n;
      double s = 0.0;
      for (int a = 0; a < l0; ++a) s += v[a * p0 + b] * lc[((long long)a * n + i) * l1 + a2];
      t[e] = s;
    }
    __syncthreads();
    const int nout = l1 * p1;
    if (p0 * n <= 256 && nout >= 64) {
      // many short sums: one thread per output (consecutive threads take
      // consecutive b2, so the reads of P are coalesced)
      for (int o = tid; o < nout; o += blockDim.x) {
        const int a2 = o / p1, b2 = o % p1;
        double s = 0.0;
#pragma unroll 8
        for (int q = 0; q < p0 * n; ++q)
          s += t[(long long)a2 * p0 * n + q] * bulk_to_double(pc[(long long)q * p1 + b2]);
        v[o] = s;  // v is consumed only through t, already complete
      }
    } else {
      for (int o = wid; o < nout; o += 4) {
        const int a2 = o / p1, b2 = o % p1;
        double s = 0.0;
        for (int q = lane; q < p0 * n; q += 64) {
          const int b = q / n, i = q % n;
          s += t[((long long)a2 * p0 + b) * n + i] * bulk_to_double(pc[((long long)b * n + i) * p1 + b2]);
        }
        s = wave_sum(s);
        if (lane == 0) v[o] = s;  // v is consumed only through t, already complete
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double s = v[0];
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    double r;
    if (!(s == s) || fabs(s) > 1.7e308) {
      r = nan;
      set_status(P.status, TT_STATUS_NONFINITE);
    } else if (!(s > 0.0)) {
      r = nan;
      set_status(P.status, TT_STATUS_NONPOSITIVE);
    } else {
      r = log(s) + fc[f].logdelta + *L.log_scale + *P.log_scale;
    }
    if (*P.status & (TT_STATUS_NONFINITE | TT_STATUS_NONPOSITIVE)) r = nan;
    out[f * stride] = r;
  }
}
