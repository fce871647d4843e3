// Prediction by Einstein summation (Sec. 4.2, eqs. ttConvolutionP,
// ttConvolutionZ, ttConvolutionM and the backward recursion
// ttConvolutionZrecursion; Alg. 1): with the transition tensor held as a TT
// of 2d cores, T(i_1..i_d, j_1..j_d), the first d over the predicted grid
// and the last d over the current one, and the density P as a d-core TT,
//
//   P'(i) = sum_j T(i, j) P(j)
//
// keeps T's first d - 1 cores and replaces core d by T_d x_3 Z, where Z is
// built backwards over the second half of T from Z = 1:
//
//   Z'(a, c) = sum_{i, b, e} T_{d+k}(a, i, b) P_k(c, i, e) Z(b, e).
//
// The paper forms the four-way M_k = sum_i T_{d+k}(:, i, :) P_k(:, i, :)
// first; here each step is split into two passes that never form M_k:
//   Y(c, i, b)  = sum_e P_k(c, i, e) Z(b, e)            (einsum_y_kernel)
//   Z'(a, c)    = sum_{(i, b)} T_{d+k}(a, (i, b)) Y(c, (i, b))
//                                                     (einsum_z_kernel)
// which costs 2 r'_{k-1} N r'_k R_{d+k} + 2 R_{d+k-1} N R_{d+k} r'_{k-1}
// flops instead of the 2 R R r' r' N of M_k.  The second pass streams T's
// second half once, coalesced, against LDS-staged chunks of Y.  All sums
// are in FP64 whatever the storage type of the cores.  Ranks are read from
// the device (ragged batches); one batch dimension per filter.
#pragma once

#include "common.h"

namespace ttg {

// Y(c, i, b) = sum_e P_k(c, i, e) Z(b, e), with Z stored transposed
// (Zt[e][b], as the Z pass writes it); Z = 1 (1 x 1) for the last core.  One
// wavefront per row (c, i): the row of P is read by every lane, the lanes
// run over b, so Zt is read and Y written contiguously.
template <typename E>
__global__ void __launch_bounds__(256) einsum_y_kernel(const DevTT* __restrict__ tt, const DevTT* __restrict__ pp,
                                                       double* const* __restrict__ zin,
                                                       double* const* __restrict__ yout, int k) {
  const int f = blockIdx.z;
  const DevTT &T = tt[f], &P = pp[f];
  const int d = P.d;
  const int rp0 = P.ranks[k], n = P.n[k], rp1 = P.ranks[k + 1], R = T.ranks[d + k + 1];
  const E* pc = core_ptr<E>(P, k);
  const double* zt = zin ? zin[f] : nullptr;
  double* y = yout[f];
  const int rows = rp0 * n;
  const int lane = threadIdx.x & 63;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nwv = (gridDim.x * blockDim.x) >> 6;
  for (int ci = wid; ci < rows; ci += nwv) {
    const E* prow = pc + (long long)ci * rp1;
    double* yrow = y + (long long)ci * R;
    for (int b = lane; b < R; b += 64) {
      double acc;
      if (zt) {
        acc = 0.0;
        for (int q = 0; q < rp1; ++q) acc += (double)prow[q] * zt[(long long)q * R + b];
      } else {
        acc = (double)prow[0];
      }
      yrow[b] = acc;
    }
  }
}

// Z'(a, c) = sum over the contiguous (i, b) of T_{d+k}(a, i, b) Y(c, i, b),
// stored transposed (Zt[c][a]) for the next Y pass.  A workgroup of EZ_WAVES
// wavefronts owns EZ_ROWS rows a of T (four per wavefront) and EZ_CB
// entries c; chunks of EZ_TC columns (i, b) of those Y rows are staged in
// LDS and every lane multiplies its four T values per row against them, so
// T is streamed once, coalesced, and Y once per row block.  Each entry sums
// its lanes' partial sums by a shuffle tree (the order does not depend on
// the batch).
#define EZ_WAVES 8
#define EZ_ROWS (4 * EZ_WAVES)
#define EZ_CB 16
#define EZ_TC 256
template <typename E>
__global__ void __launch_bounds__(64 * EZ_WAVES) einsum_z_kernel(const DevTT* __restrict__ tt, const DevTT* __restrict__ pp,
                                                       double* const* __restrict__ yin,
                                                       double* const* __restrict__ zout, int k) {
  const int f = blockIdx.z;
  const DevTT &T = tt[f], &P = pp[f];
  const int d = P.d;
  const int R0 = T.ranks[d + k], n = T.n[d + k], R1 = T.ranks[d + k + 1], rp0 = P.ranks[k];
  const int a0 = blockIdx.x * EZ_ROWS, c0 = blockIdx.y * EZ_CB;
  if (a0 >= R0 || c0 >= rp0) return;  // uniform over the workgroup
  const int len = n * R1;
  const TTG_GLOBAL E* tc = gmem(core_ptr<E>(T, d + k));
  const TTG_GLOBAL double* y = gmem(static_cast<const double*>(yin[f]));
  TTG_GLOBAL double* z = gmem(zout[f]);
  __shared__ double Ys[EZ_CB][EZ_TC];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double acc[4][EZ_CB];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int c = 0; c < EZ_CB; ++c) acc[q][c] = 0.0;
  // the next chunk's T values and Y entries are loaded into registers while
  // the current chunk is multiplied (the LDS-only barriers leave them in flight)
  constexpr int YPT = EZ_CB * EZ_TC / (64 * EZ_WAVES);  // Y entries staged per thread
  double tv[4][4], yv[YPT];
  auto load = [&](int t0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int a = a0 + 4 * w + q;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int t = t0 + lane + 64 * u;
        tv[q][u] = (a < R0 && t < len) ? (double)tc[(long long)a * len + t] : 0.0;
      }
    }
#pragma unroll
    for (int x = 0; x < YPT; ++x) {
      const int e = threadIdx.x + x * 64 * EZ_WAVES;
      const int c = e / EZ_TC, j = e - (e / EZ_TC) * EZ_TC;
      const int cc = c0 + c, t = t0 + j;
      yv[x] = (cc < rp0 && t < len) ? y[(long long)cc * len + t] : 0.0;
    }
  };
  load(0);
  for (int t0 = 0; t0 < len; t0 += EZ_TC) {
#pragma unroll
    for (int x = 0; x < YPT; ++x) {
      const int e = threadIdx.x + x * 64 * EZ_WAVES;
      Ys[e / EZ_TC][e - (e / EZ_TC) * EZ_TC] = yv[x];
    }
    double tcur[4][4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) tcur[q][u] = tv[q][u];
    lds_barrier();
    if (t0 + EZ_TC < len) load(t0 + EZ_TC);
#pragma unroll
    for (int c = 0; c < EZ_CB; ++c)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double yvv = Ys[c][lane + 64 * u];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q][c] += tcur[q][u] * yvv;
      }
    lds_barrier();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int a = a0 + 4 * w + q;
#pragma unroll
    for (int c = 0; c < EZ_CB; ++c) {
      double v = acc[q][c];
      for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
      if (lane == 0 && a < R0 && c0 + c < rp0) z[(long long)(c0 + c) * R0 + a] = v;  // transposed
    }
  }
}

// P'_k = T_k for k < d - 1, P'_{d-1}(a, i) = sum_b T_{d-1}(a, i, b) Z(b);
// ranks of T's first half, log-scale of T plus that of P, status of P
template <typename E>
__global__ void __launch_bounds__(256) einsum_out_kernel(const DevTT* __restrict__ tt, const DevTT* __restrict__ pp,
                                                         const DevTT* __restrict__ oo,
                                                         double* const* __restrict__ zin) {
  const int f = blockIdx.z, k = blockIdx.y;
  const DevTT &T = tt[f], &P = pp[f], &O = oo[f];
  const int d = P.d;
  if (k >= d) return;
  const int r0 = T.ranks[k], n = T.n[k], r1 = T.ranks[k + 1];
  const E* tc = core_ptr<E>(T, k);
  E* oc = core_ptr<E>(O, k);
  if (k < d - 1) {
    const long long tot = (long long)r0 * n * r1;
    const long long gid = blockIdx.x * (long long)blockDim.x + threadIdx.x, gstride = (long long)gridDim.x * blockDim.x;
    long long done = 0;
    if (((reinterpret_cast<unsigned long long>(tc) | reinterpret_cast<unsigned long long>(oc)) & 15) == 0) {
      constexpr int U = 16 / (int)sizeof(E);  // elements per 16-byte unit
      const long long nv = tot / U;
      const uint4* s4 = reinterpret_cast<const uint4*>(tc);
      uint4* d4 = reinterpret_cast<uint4*>(oc);
      for (long long v = gid; v < nv; v += gstride) d4[v] = s4[v];
      done = nv * U;
    }
    for (long long e = done + gid; e < tot; e += gstride) oc[e] = tc[e];
  } else {
    // one wavefront per row (a, i), lanes over b, a shuffle tree per row
    const double* z = zin[f];
    const int rows = r0 * n, lane = threadIdx.x & 63;
    const int wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6, nwv = (gridDim.x * blockDim.x) >> 6;
    for (int e = wid; e < rows; e += nwv) {
      const E* trow = tc + (long long)e * r1;
      double acc = 0.0;
      for (int b = lane; b < r1; b += 64) acc += (double)trow[b] * z[b];
      for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m, 64);
      if (lane == 0) oc[e] = (E)acc;
    }
  }
  if (k == 0 && blockIdx.x == 0 && threadIdx.x == 0) {
    for (int j = 0; j < d; ++j) O.ranks[j] = T.ranks[j];
    O.ranks[d] = 1;
    *O.log_scale = *T.log_scale + *P.log_scale;
    *O.status = *P.status;
  }
}

}  // namespace ttg
