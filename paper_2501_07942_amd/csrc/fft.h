// Fused prediction + absorption through FFTs of the core fibres.
//
// For an interior core k of the predictive product X_k = conv(K_k, P_k)
// (Sec. 2.1 eq. tpmconvFFT; Sec. 4.2: the convolution of two TTs is the
// inverse FFT of the products of the core spectra) the right-to-left
// rounding sweep needs only Z_k = X_k x_3 L_{k+1}:
//   Y(b, i, a', j)  = sum_{b'} P_k(b, i, b') L(a' rp1 + b', j)
//   Yh(b, w, a', j) = FFT_L over i of Y (zero padded, L = 2^p >= n + h)
//   Zh(ab, w, j)    = sum_{a'} Kh_k(a, w, a') Yh(b, w, a', j)
//   Z(a rp0 + b, i, j) = IFFT_L(Zh)(h + i) / L,  i = 0..n-1
// where Kh_k(a, w, a') is the FFT of the kernel fibre K_k(a, 0..2h, a').  The
// circular convolution of length L >= n + h equals the cropped linear one.
// Z is written with columns ordered (j, i) (fibres contiguous); the Gram is
// indifferent to the column order and the triangular solve maps it back.
#pragma once

#include "common.h"

template <typename T>
struct Cpx;
template <>
struct Cpx<float> {
  using t = float2;
};
template <>
struct Cpx<double> {
  using t = double2;
};

template <typename C>
__device__ inline C cmul(C a, C b) {
  C r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
template <typename C>
__device__ inline C cadd(C a, C b) {
  C r;
  r.x = a.x + b.x;
  r.y = a.y + b.y;
  return r;
}
template <typename C>
__device__ inline C csub(C a, C b) {
  C r;
  r.x = a.x - b.x;
  r.y = a.y - b.y;
  return r;
}

// Per-filter description of the fused prediction.
struct FusedPred {
  int L, log2L, LHP, h;  // FFT length, spectrum row pitch (>= L/2+1), kernel half width
  void* khat;            // kernel spectra [core][w][a][a'] (complex bulk type), pitch kpitch per core
  long long kpitch;      // complex elements per core
  void* tw;              // twiddles W_L^t, t < L/2 (complex bulk type)
  int zt;                // 1: Z columns are ordered (j, i)
};

// twiddles W_L^t = exp(-2 pi i t / L), t < L/2, into LDS
template <typename C>
__device__ inline void make_twiddles(C* tw, int L) {
  for (int t = threadIdx.x; t < L / 2; t += blockDim.x) {
    double s, c;
    sincospi(-2.0 * (double)t / (double)L, &s, &c);
    tw[t].x = c;
    tw[t].y = s;
  }
}

// Radix-2 Stockham FFT of length L held by one wavefront in LDS (a -> b ->
// a ...).  Every thread of the block calls it (uniform trip counts) because
// stages are separated by __syncthreads.  Returns the buffer with the
// result.  inverse = true uses conjugate twiddles (no 1/L scaling).
template <typename C>
__device__ inline C* fft_stockham(C* a, C* b, int L, int log2L, const C* tw, bool inverse, int lane) {
  for (int s = 0, Ns = 1; s < log2L; ++s, Ns <<= 1) {
    for (int j = lane; j < L / 2; j += 64) {
      const int k = j & (Ns - 1);
      C w = tw[k * (L / (2 * Ns))];
      if (inverse) w.y = -w.y;
      const C v0 = a[j];
      const C v1 = cmul(a[j + L / 2], w);
      const int o = ((j - k) << 1) + k;  // (j / Ns) * 2 Ns + k
      b[o] = cadd(v0, v1);
      b[o + Ns] = csub(v0, v1);
    }
    __syncthreads();
    C* t = a;
    a = b;
    b = t;
  }
  return a;
}

// Kernel spectra of the interior cores of one kernel TT.  grid.x = fibres
// (a, a') in groups of 4 (one per wavefront), grid.y = core, block 256.
template <typename T>
__global__ void __launch_bounds__(256) kernel_spectra_kernel(const DevTT* __restrict__ kern, int L, int log2L,
                                                             int LHP, void* __restrict__ khat_v, long long kpitch) {
  using C = typename Cpx<T>::t;
  const DevTT& K = kern[0];
  const int k = blockIdx.y;
  if (k >= K.d) return;
  const int rk0 = K.ranks[k], rk1 = K.ranks[k + 1], taps = K.n[k];
  extern __shared__ unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);
  C* buf = tw + L / 2;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  C* a = buf + wid * 2 * L;
  C* b = a + L;
  make_twiddles(tw, L);
  const int f = blockIdx.x * 4 + wid;
  const bool live = f < rk0 * rk1;
  const int al = live ? f / rk1 : 0, al2 = live ? f % rk1 : 0;
  const T* kc = core_ptr<T>(K, k);
  for (int t = lane; t < L; t += 64) {
    C v;
    v.x = (live && t < taps) ? kc[((long long)al * taps + t) * rk1 + al2] : (T)0;
    v.y = (T)0;
    a[t] = v;
  }
  __syncthreads();
  C* r = fft_stockham(a, b, L, log2L, tw, false, lane);
  if (live) {
    C* kh = reinterpret_cast<C*>(khat_v) + (long long)k * kpitch;
    for (int w = lane; w <= L / 2; w += 64) kh[(long long)w * rk0 * rk1 + f] = r[w];
  }
}

// Twiddle table W_L^t = exp(-2 pi i t / L), t < L/2, computed once per L.
template <typename T>
__global__ void twiddle_kernel(void* tw_v, int L) {
  using C = typename Cpx<T>::t;
  C* tw = reinterpret_cast<C*>(tw_v);
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < L / 2; t += gridDim.x * blockDim.x) {
    double sn, cs;
    sincospi(-2.0 * (double)t / (double)L, &sn, &cs);
    tw[t].x = cs;
    tw[t].y = sn;
  }
}

// Radix-2 Stockham FFTs of nf fibres of length L (fibre f at a + f*L), all
// threads of the block cooperating; stages separated by __syncthreads.
// Returns the buffer holding the result.
template <typename C>
__device__ inline C* fft_multi(C* a, C* b, int L, int log2L, int nf, const C* tw, bool inverse) {
  const int half = L / 2;
  const int total = nf * half;
  for (int s = 0, Ns = 1; s < log2L; ++s, Ns <<= 1) {
    const int step = L / (2 * Ns);
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      const int fib = e / half, j = e - fib * half;
      const int k = j & (Ns - 1);
      C w = tw[k * step];
      if (inverse) w.y = -w.y;
      const C* src = a + fib * L;
      C* dst = b + fib * L;
      const C v0 = src[j];
      const C v1 = cmul(src[j + half], w);
      const int o = ((j - k) << 1) + k;
      dst[o] = cadd(v0, v1);
      dst[o + Ns] = csub(v0, v1);
    }
    __syncthreads();
    C* t = a;
    a = b;
    b = t;
  }
  return a;
}

// Fused prediction for NC output columns (b, j..j+NC-1) of core k per
// workgroup:
//   Y(a', i) = sum_{b'} P(b, i, b') L(a' rp1 + b', j),   a' < rk1
//   Yh = FFT(Y) (two real fibres per complex FFT), Zh(a) = sum_{a'} Kh(a, a') Yh(a')
//   Z(a rp0 + b, i, j) = IFFT(Zh(a))(h + i) / L       (two outputs per IFFT)
// Everything stays in LDS; the kernel spectra stream from L2 through LDS in
// frequency chunks shared by the NC columns.
// grid.x = column group, grid.z = filter.
#define FP_WCH 8  // frequencies per kernel-spectra chunk
template <typename T, int NC, typename F>
__global__ void __launch_bounds__(256) fused_pred_kernel(F fn) {
  using C = typename Cpx<T>::t;
  const int bz = blockIdx.z;
  typename F::Args g;
  if (!fn(bz, g)) return;
  const int N = g.N, rp0 = g.rp0, rp1 = g.rp1, rk0 = g.rk0, rk1 = g.rk1, n = g.n;
  const int L = g.fp.L, log2L = g.fp.log2L, h = g.hk;
  const int ncol = rp0 * N;
  const int col0 = blockIdx.x * NC;
  if (col0 >= ncol) return;
  const int nw = L / 2 + 1;
  const int pin = (rk1 + 1) / 2, pout = (rk0 + 1) / 2;
  const int pmax = max(pin, pout);
  const int rkm = max(rk0, rk1);
  // per column: two ping-pong buffers of bsz and a spectra buffer
  const int bsz = max(pmax * L, rkm * nw);
  extern __shared__ unsigned char smem_raw[];
  C* tw = reinterpret_cast<C*>(smem_raw);      // L/2
  C* kch = tw + L / 2;                         // FP_WCH * rk0 * rk1
  C* colbuf = kch + FP_WCH * rk0 * rk1;        // NC * (2 bsz + rkm nw)
  T* Ps = reinterpret_cast<T*>(colbuf + NC * (2 * bsz + rkm * nw));  // NC * n * rp1
  T* Lc = Ps + NC * n * rp1;                                         // NC * rk1 * rp1
  const int tid = threadIdx.x;
  const C* twg = reinterpret_cast<const C*>(g.fp.tw);
  for (int t = tid; t < L / 2; t += blockDim.x) tw[t] = twg[t];
  for (int c = 0; c < NC; ++c) {
    const int col = min(col0 + c, ncol - 1);  // a duplicate column is computed but not written
    const int be = col / N, j = col % N;
    const T* pc = g.p + (long long)be * n * rp1;
    for (int e = tid; e < n * rp1; e += blockDim.x) Ps[c * n * rp1 + e] = pc[e];
    for (int e = tid; e < rk1 * rp1; e += blockDim.x) Lc[c * rk1 * rp1 + e] = (T)g.lfac[(long long)e * g.gcap + j];
  }
  __syncthreads();
  C* bA[NC];
  C* bB[NC];
  C* sp[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    bA[c] = colbuf + c * (2 * bsz + rkm * nw);
    bB[c] = bA[c] + bsz;
    sp[c] = bB[c] + bsz;
  }
  // 1. input fibres, two per complex sequence (all columns at once)
  for (int e = tid; e < NC * pin * L; e += blockDim.x) {
    const int c = e / (pin * L), rem = e - c * pin * L;
    const int pq = rem / L, t = rem - pq * L;
    const int a0 = 2 * pq, a1 = 2 * pq + 1;
    T y0 = (T)0, y1 = (T)0;
    if (t < n) {
      const T* pr = Ps + c * n * rp1 + t * rp1;
      const T* lc = Lc + c * rk1 * rp1;
      for (int q = 0; q < rp1; ++q) {
        y0 += pr[q] * lc[a0 * rp1 + q];
        if (a1 < rk1) y1 += pr[q] * lc[a1 * rp1 + q];
      }
    }
    C v;
    v.x = y0;
    v.y = y1;
    bA[c][rem] = v;
  }
  __syncthreads();
  // forward FFTs: the NC columns' buffers are consecutive only per column, so
  // run them one column after another
  C* r[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) r[c] = fft_multi(bA[c], bB[c], L, log2L, pin, tw, false);
  // 2. unpack the two real spectra of every pair (w = 0..L/2)
  for (int e = tid; e < NC * pin * nw; e += blockDim.x) {
    const int c = e / (pin * nw), rem = e - c * pin * nw;
    const int pq = rem / nw, w = rem - pq * nw;
    const C* rr = r[0];
#pragma unroll
    for (int q = 1; q < NC; ++q)
      if (c == q) rr = r[q];
    C* spc = sp[0];
#pragma unroll
    for (int q = 1; q < NC; ++q)
      if (c == q) spc = sp[q];
    const C zw = rr[pq * L + w];
    C zc = rr[pq * L + ((L - w) & (L - 1))];
    zc.y = -zc.y;
    C x1, x2;
    x1.x = (zw.x + zc.x) * (T)0.5;
    x1.y = (zw.y + zc.y) * (T)0.5;
    const C dd_ = csub(zw, zc);  // (zw - conj z_{L-w}) / (2i) = -i d / 2
    x2.x = dd_.y * (T)0.5;
    x2.y = -dd_.x * (T)0.5;
    spc[(2 * pq) * nw + w] = x1;
    if (2 * pq + 1 < rk1) spc[(2 * pq + 1) * nw + w] = x2;
  }
  __syncthreads();
  // 3. frequency products, kernel spectra staged in chunks of FP_WCH
  //    frequencies; outputs go to the free ping-pong buffer of each column
  C* zsp[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) zsp[c] = (r[c] == bA[c]) ? bB[c] : bA[c];
  const C* kh = reinterpret_cast<const C*>(g.fp.khat) + (long long)g.k * g.fp.kpitch;
  const int kk = rk0 * rk1;
  for (int w0 = 0; w0 < nw; w0 += FP_WCH) {
    const int wc = min(FP_WCH, nw - w0);
    for (int e = tid; e < wc * kk; e += blockDim.x) kch[e] = kh[(long long)w0 * kk + e];
    __syncthreads();
    for (int e = tid; e < NC * rk0 * wc; e += blockDim.x) {
      const int c = e / (rk0 * wc), rem = e - c * rk0 * wc;
      const int al = rem / wc, wl = rem - al * wc;
      const int w = w0 + wl;
      const C* spc = sp[0];
      C* zc_ = zsp[0];
#pragma unroll
      for (int q = 1; q < NC; ++q)
        if (c == q) {
          spc = sp[q];
          zc_ = zsp[q];
        }
      const C* kr = kch + wl * kk + al * rk1;
      C acc;
      acc.x = (T)0;
      acc.y = (T)0;
      for (int q = 0; q < rk1; ++q) acc = cadd(acc, cmul(kr[q], spc[q * nw + w]));
      zc_[al * nw + w] = acc;
    }
    __syncthreads();
  }
  // 4. packed full spectra of the output pairs: Z = X1 + i X2 on w in [0, L);
  //    written into the spectra buffer region (free now), which holds
  //    rkm * nw >= pout * L?  not always, so use the other ping-pong buffer
  C* dst[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) dst[c] = (zsp[c] == bA[c]) ? bB[c] : bA[c];
  for (int e = tid; e < NC * pout * L; e += blockDim.x) {
    const int c = e / (pout * L), rem = e - c * pout * L;
    const int pq = rem / L, w = rem - pq * L;
    const C* zs = zsp[0];
    C* ds = dst[0];
#pragma unroll
    for (int q = 1; q < NC; ++q)
      if (c == q) {
        zs = zsp[q];
        ds = dst[q];
      }
    const int a0 = 2 * pq, a1 = 2 * pq + 1;
    C x1, x2;
    x2.x = (T)0;
    x2.y = (T)0;
    if (w < nw) {
      x1 = zs[a0 * nw + w];
      if (a1 < rk0) x2 = zs[a1 * nw + w];
    } else {  // Hermitian symmetry
      x1 = zs[a0 * nw + (L - w)];
      x1.y = -x1.y;
      if (a1 < rk0) {
        x2 = zs[a1 * nw + (L - w)];
        x2.y = -x2.y;
      }
    }
    C v;  // x1 + i x2
    v.x = x1.x - x2.y;
    v.y = x1.y + x2.x;
    ds[rem] = v;
  }
  __syncthreads();
  C* res[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) res[c] = fft_multi(dst[c], (dst[c] == bA[c]) ? bB[c] : bA[c], L, log2L, pout, tw, true);
  // 5. crop, scale and write both real outputs of every pair
  const T inv = (T)1 / (T)L;
  const long long rowpitch = (long long)n * N;
  for (int e = tid; e < NC * pout * n; e += blockDim.x) {
    const int c = e / (pout * n), rem = e - c * pout * n;
    if (col0 + c >= ncol) continue;
    const int col = col0 + c;
    const int be = col / N, j = col % N;
    const int pq = rem / n, i = rem - pq * n;
    const C* rs = res[0];
#pragma unroll
    for (int q = 1; q < NC; ++q)
      if (c == q) rs = res[q];
    const C v = rs[pq * L + h + i];
    const int a0 = 2 * pq, a1 = 2 * pq + 1;
    g.z[(long long)(a0 * rp0 + be) * rowpitch + (long long)j * n + i] = v.x * inv;
    if (a1 < rk0) g.z[(long long)(a1 * rp0 + be) * rowpitch + (long long)j * n + i] = v.y * inv;
  }
}

// ---------------------------------------------------------------------------
// Direct fused prediction (time domain), the default:
//   V(a, m, b', j) = sum_{a'} K_k(a, m, a') L(a' rp1 + b', j)
//   Z(a rp0 + b, i, j) = sum_m sum_{b'} P_k(b, i + h - m, b') V(a, m, b', j)
// (the same Z_k = X_k x_3 L_{k+1} as above, P = 0 off the grid).  A
// workgroup owns one output row block a, BB consecutive b and a chunk of JC
// columns j; V for that (a, j-chunk) and NB = 32 / JC zero-padded P fibres
// live in LDS.  JC (8, 16 or 32) follows the filter's own column count, so a
// narrow L_{k+1} does not leave threads computing padding.  Each thread
// produces 4 consecutive i x 4 consecutive j of one fibre; taps are consumed
// in blocks of DF_TB from a register window over the fibre.
// Z is written in the ordinary column order (i, j).
// ---------------------------------------------------------------------------
#define DF_TB 4
#define DF_JC 32

__host__ __device__ inline int direct_jc(int N) { return N <= 8 ? 8 : (N <= 16 ? 16 : DF_JC); }

template <typename T, typename F>
__global__ void __launch_bounds__(256) direct_pred_kernel(F fn, int BB) {
  const int bz = blockIdx.z;
  typename F::Args g;
  if (!fn(bz, g)) return;
  const int N = g.N, rp0 = g.rp0, rp1 = g.rp1, rk0 = g.rk0, rk1 = g.rk1, n = g.n;
  const int h = g.hk, taps = 2 * g.hk + 1;
  const int taps_pad = (taps + DF_TB - 1) / DF_TB * DF_TB;
  const int JC = direct_jc(N);
  const int NB = DF_JC / JC;  // fibres per pass
  // blocks are laid out for 32-column chunks; narrower chunks leave the
  // surplus chunk indices idle
  const int njc = (N + DF_JC - 1) / DF_JC;
  const int nbb = (rp0 + BB - 1) / BB;
  int blk = blockIdx.x;
  const int jc = blk % njc;
  blk /= njc;
  const int bb = blk % nbb;
  const int al = blk / nbb;
  if (al >= rk0) return;
  const int j0 = jc * JC;
  if (j0 >= N) return;
  // padded fibre rows: output i reads rows i + h - m + front, m in [0, taps_pad)
  const int front = DF_TB;
  const int plen = front + n + 2 * h + 4 + DF_TB;
  const int pp = rp1 + 1;  // odd pitch: the 8 rows a wavefront reads fall in distinct banks
  extern __shared__ unsigned char smem_raw[];
  T* Vs = reinterpret_cast<T*>(smem_raw);  // [taps_pad][rp1][JC]
  T* Ps = Vs + taps_pad * rp1 * JC;        // [NB][plen][pp]
  T* Ks = Ps + NB * plen * pp;             // [taps][rk1] of row a
  const int tid = threadIdx.x;
  const T* kc = g.kcore + (long long)al * taps * rk1;
  for (int e = tid; e < taps * rk1; e += blockDim.x) Ks[e] = kc[e];
  __syncthreads();
  // V for this (a, j-chunk); zero beyond taps and beyond N.  A thread owns
  // one (b', j) fibre: its rk1 (<= 32) values of L are loaded together, then
  // every tap is a short dot product with the kernel row held in LDS.
  for (int e = tid; e < rp1 * JC; e += blockDim.x) {
    const int q = e / JC, jj = e - q * JC;
    const int j = j0 + jj;
    T lv[32];
    const double* lc = g.lfac + (long long)q * g.gcap + j;  // row a' rp1 + q
#pragma unroll
    for (int a2 = 0; a2 < 32; ++a2)
      lv[a2] = (a2 < rk1 && j < N) ? (T)lc[(long long)a2 * rp1 * g.gcap] : (T)0;
    for (int m = 0; m < taps_pad; ++m) {
      T v = (T)0;
      if (m < taps) {
        const T* kr = Ks + m * rk1;
#pragma unroll
        for (int a2 = 0; a2 < 32; ++a2)
          if (a2 < rk1) v += kr[a2] * lv[a2];
      }
      Vs[(m * rp1 + q) * JC + jj] = v;
    }
  }
  const int tjn = JC / 4;
  const int ti = tid >> 3, r8 = tid & 7;  // 32 row groups x 8 (fibre, column group) slots
  const int fib = r8 / tjn, tj = r8 - fib * tjn;
  const int jj0 = tj * 4;
  const T* Pf = Ps + fib * plen * pp;
  for (int bo = 0; bo < BB; bo += NB) {
    const int bfirst = bb * BB + bo;
    if (bfirst >= rp0) break;
    __syncthreads();  // Vs ready / previous fibres consumed
    for (int e = tid; e < NB * plen * rp1; e += blockDim.x) {
      const int f = e / (plen * rp1), rem = e - f * plen * rp1;
      const int pr = rem / rp1, q = rem - pr * rp1;
      const int row = pr - front - h;
      const int bf = bfirst + f;
      T v = (T)0;
      if (bf < rp0 && bo + f < BB && row >= 0 && row < n) v = g.p[((long long)bf * n + row) * rp1 + q];
      Ps[(f * plen + pr) * pp + q] = v;
    }
    __syncthreads();
    const int be = bfirst + fib;
    if (be >= rp0 || bo + fib >= BB) continue;
    for (int i0 = ti * 4; i0 < n; i0 += 128) {
      T acc[4][4];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = (T)0;
      for (int q = 0; q < rp1; ++q) {
        for (int m0 = 0; m0 < taps_pad; m0 += DF_TB) {
          // row of P(i - (m - h)) in the padded fibre: front + 2h + i - m - ...
          const int base = front + 2 * h + i0 - m0 - (DF_TB - 1);
          T w[4 + DF_TB - 1];
#pragma unroll
          for (int v = 0; v < 4 + DF_TB - 1; ++v) w[v] = Pf[(base + v) * pp + q];
#pragma unroll
          for (int u = 0; u < DF_TB; ++u) {
            const T* vr = Vs + ((m0 + u) * rp1 + q) * JC + jj0;
            const T v0 = vr[0], v1 = vr[1], v2 = vr[2], v3 = vr[3];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const T pv = w[r - u + DF_TB - 1];
              acc[r][0] += pv * v0;
              acc[r][1] += pv * v1;
              acc[r][2] += pv * v2;
              acc[r][3] += pv * v3;
            }
          }
        }
      }
      const long long row = (long long)(al * rp0 + be) * n * N;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + r;
        if (i >= n) continue;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int j = j0 + jj0 + c;
          if (j < N) g.z[row + (long long)i * N + j] = acc[r][c];
        }
      }
    }
  }
}
