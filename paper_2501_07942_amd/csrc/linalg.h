// Batched small dense linear algebra used by TT rounding, TT-SVD and the
// likelihood SVD.  Every kernel takes a functor that, given the filter index
// b (blockIdx.z or blockIdx.x), reads that filter's current ranks from device
// memory and returns the operand shapes and pointers; grids are sized from
// capacities and surplus blocks exit at once.  This keeps every launch free
// of host synchronisation.
#pragma once

#include "common.h"

// ---------------------------------------------------------------------------
// Gram matrix  G(a, b) = sum_t X(a, t) X(b, t),  a, b < M,  t < T
// with X(a, t) = x[a*sa + t*st].  Split-K partials go to
// out + (b*splits + s)*gcap*gcap*words; gram_reduce sums them into split 0
// and mirrors the upper triangle.
// ---------------------------------------------------------------------------
struct GramArgs {
  int M, T;
  const void* x;
  long long sa, st;
  double* out;  // partials base for this filter
  int gcap, splits;  // splits = plane capacity on input
};

// split count used for a summation of length T with `planes` planes
__device__ inline int gram_split_count(int T, int planes) {
  const int s = (T + 511) / 512;
  return max(1, min(s, planes));
}

template <typename TB, typename Acc, int TS, typename F>
__global__ void __launch_bounds__(256) gram_partial_kernel(F f) {
  constexpr int RB = TS / 16;  // outputs per thread along each side
  constexpr int KC = 32;       // summation chunk
  const int b = blockIdx.z;
  GramArgs g;
  if (!f(b, g)) return;
  g.splits = gram_split_count(g.T, g.splits);
  // upper-triangular tile pair from blockIdx.x
  const int ntile = (g.M + TS - 1) / TS;
  int tp = blockIdx.x, ti = 0;
  while (ti < ntile && tp >= ntile - ti) {
    tp -= ntile - ti;
    ++ti;
  }
  if (ti >= ntile) return;
  const int tj = ti + tp;
  const int s = blockIdx.y;
  if (s >= g.splits) return;
  const int chunk = (g.T + g.splits - 1) / g.splits;
  const int t_begin = s * chunk, t_end = min(g.T, t_begin + chunk);

  __shared__ double As[TS][KC + 1];
  __shared__ double Bs[TS][KC + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  typename Acc::V acc[RB][RB];
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < RB; ++j) acc[i][j] = Acc::zero();
  const TB* x = reinterpret_cast<const TB*>(g.x);
  const bool t_fast = (g.st == 1);
  const int a0 = ti * TS, b0 = tj * TS;
  const bool diag_tile = (ti == tj);
  for (int t0 = t_begin; t0 < t_end; t0 += KC) {
    for (int e = threadIdx.x; e < TS * KC; e += blockDim.x) {
      int r, c;  // r = vector index within tile, c = summation index within chunk
      if (t_fast) {
        r = e / KC;
        c = e % KC;
      } else {
        c = e / TS;
        r = e % TS;
      }
      const int t = t0 + c;
      double va = 0.0, vb = 0.0;
      if (t < t_end) {
        if (a0 + r < g.M) va = bulk_to_double(x[(long long)(a0 + r) * g.sa + (long long)t * g.st]);
        if (!diag_tile && b0 + r < g.M) vb = bulk_to_double(x[(long long)(b0 + r) * g.sa + (long long)t * g.st]);
      }
      As[r][c] = va;
      Bs[r][c] = diag_tile ? va : vb;
    }
    __syncthreads();
    const int kmax = min(KC, t_end - t0);
    for (int c = 0; c < kmax; ++c) {
      double av[RB], bv[RB];
#pragma unroll
      for (int i = 0; i < RB; ++i) av[i] = As[ty * RB + i][c];
#pragma unroll
      for (int j = 0; j < RB; ++j) bv[j] = Bs[tx * RB + j][c];
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < RB; ++j) acc[i][j] = Acc::fma_(acc[i][j], av[i], bv[j]);
    }
    __syncthreads();
  }
  double* out = g.out + (long long)s * g.gcap * g.gcap * Acc::words;
#pragma unroll
  for (int i = 0; i < RB; ++i)
#pragma unroll
    for (int j = 0; j < RB; ++j) {
      const int a = a0 + ty * RB + i, bb = b0 + tx * RB + j;
      if (a < g.M && bb < g.M) Acc::store(out, (long long)a * g.gcap + bb, acc[i][j]);
    }
}

// ---------------------------------------------------------------------------
// The same Gram partials with FP64 accumulation on the matrix cores
// (v_mfma_f64_16x16x4f64): one 64 x 64 upper-triangular tile pair per
// workgroup, each wavefront a 32 x 32 quadrant (2 x 2 MFMA tiles).  Chunks
// of 32 summation indices of both row blocks are staged in LDS in the input
// type, double-buffered (one barrier per chunk: while a chunk is multiplied
// the chunk two ahead is fetched into registers and the next one is stored
// to the other buffer) and widened to FP64 as they are read; within a chunk the
// k-lane lk of an MFMA step s takes index lk * 8 + s, so a lane reads its
// eight operands as one contiguous run.  Products of FP32 inputs are exact
// in FP64.  A workgroup takes the splits blockIdx.y, blockIdx.y + gridDim.y,
// ... of its tile pair, so a launch sized for the largest split count does
// not leave most of its workgroups without work.  Lane layout of the MFMA:
// A(i, k) in lane i + 16 k, B(k, j) in lane j + 16 k, D(i, j) in lane
// j + 16 (i % 4), register i / 4.
// ---------------------------------------------------------------------------
typedef double md4 __attribute__((ext_vector_type(4)));
#define GM_KC 32
#define GM_YMIN 2  // split planes per launch row: at least this many,
#define GM_YMAX 4  // at most this many (workgroups loop over the rest)

template <typename TB>
struct GmLds {
  static constexpr int pitch = GM_KC + 16 / (int)sizeof(TB);  // 16-byte aligned rows
  // four consecutive elements widened to FP64
  __device__ static inline void read4(const TB* p, double* v) {
    if constexpr (sizeof(TB) == 4) {
      const float4 t = *reinterpret_cast<const float4*>(p);
      v[0] = t.x;
      v[1] = t.y;
      v[2] = t.z;
      v[3] = t.w;
    } else {
      const double2 t0 = *reinterpret_cast<const double2*>(p);
      const double2 t1 = *reinterpret_cast<const double2*>(p + 2);
      v[0] = t0.x;
      v[1] = t0.y;
      v[2] = t1.x;
      v[3] = t1.y;
    }
  }
  // element u of a thread's share of a chunk: row r of the block, index c
  __device__ static inline int2 rc(int tid, int u, bool t_fast) {
    const int e = tid + u * 256;
    return t_fast ? int2{e / GM_KC, e % GM_KC} : int2{e % 64, e / 64};
  }
};

template <typename TB, typename F>
__global__ void __launch_bounds__(256, 2) gram_mfma_kernel(F f) {
  const int b = blockIdx.z;
  GramArgs g;
  if (!f(b, g)) return;
  g.splits = gram_split_count(g.T, g.splits);
  const int ntile = (g.M + 63) / 64;
  int tp = blockIdx.x, ti = 0;
  while (ti < ntile && tp >= ntile - ti) {
    tp -= ntile - ti;
    ++ti;
  }
  if (ti >= ntile) return;
  const int tj = ti + tp;
  constexpr int PITCH = GmLds<TB>::pitch;
  constexpr int BUF = 64 * PITCH;  // one row block of one chunk
  __shared__ __align__(16) TB Ls[2 * 2 * BUF];  // [buffer][A or B][64][PITCH]
  const bool diag_tile = ti == tj;
  const TTG_GLOBAL TB* x = gmem(reinterpret_cast<const TB*>(g.x));
  const bool t_fast = g.st == 1;
  const int a0 = ti * 64, b0 = tj * 64;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int qa = wv >> 1, qb = wv & 1;
  const int lr = lane & 15, lk = lane >> 4;
  const int chunk = (g.T + g.splits - 1) / g.splits;
  constexpr int GM_PER = 64 * GM_KC / 256;
  for (int s = blockIdx.y; s < g.splits; s += gridDim.y) {
    const int t_begin = s * chunk, t_end = min(g.T, t_begin + chunk);
    md4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = md4{0.0, 0.0, 0.0, 0.0};
    // each thread stages GM_PER elements of both row blocks per chunk; two
    // register sets take chunks c and c + 1, so a chunk's loads are in
    // flight for two chunks of MFMAs before they are stored to LDS
    TB pa0[GM_PER], pb0[GM_PER], pa1[GM_PER], pb1[GM_PER];
    // element u sits at a wave-uniform base plus this lane's 32-bit offset
    // (loff), so the loads need no 64-bit address per element
    const unsigned loff = t_fast ? (unsigned)((tid >> 5) * g.sa + (tid & 31))
                                 : (unsigned)((tid & 63) * g.sa + (tid >> 6) * g.st);
    const long long ustep = t_fast ? 8 * g.sa : 4 * g.st;
    auto fetch = [&](TB (&pa_)[GM_PER], TB (&pb_)[GM_PER], int t0) {
      const TTG_GLOBAL TB* xa = x + (long long)a0 * g.sa + (long long)t0 * g.st;
      const TTG_GLOBAL TB* xb = x + (long long)b0 * g.sa + (long long)t0 * g.st;
#pragma unroll
      for (int u = 0; u < GM_PER; ++u) {
        const int2 q = GmLds<TB>::rc(tid, u, t_fast);
        const bool tv = t0 + q.y < t_end;
        pa_[u] = (tv && a0 + q.x < g.M) ? (xa + u * ustep)[loff] : (TB)0;
        pb_[u] = (!diag_tile && tv && b0 + q.x < g.M) ? (xb + u * ustep)[loff] : (TB)0;
      }
    };
    auto stage = [&](const TB (&pa_)[GM_PER], const TB (&pb_)[GM_PER], int buf) {
      TB* As = Ls + buf * 2 * BUF;
#pragma unroll
      for (int u = 0; u < GM_PER; ++u) {
        const int2 q = GmLds<TB>::rc(tid, u, t_fast);
        As[q.x * PITCH + q.y] = pa_[u];
        if (!diag_tile) As[BUF + q.x * PITCH + q.y] = pb_[u];
      }
    };
    // steps 0..3, then 4..7 of the chunk in LDS buffer buf
    auto multiply = [&](int buf) {
      const TB* As = Ls + buf * 2 * BUF;
      const TB* Bsrc = diag_tile ? As : As + BUF;
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
        double av[2][4], bv[2][4];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          GmLds<TB>::read4(As + (qa * 32 + i * 16 + lr) * PITCH + lk * 8 + 4 * hf, av[i]);
          GmLds<TB>::read4(Bsrc + (qb * 32 + i * 16 + lr) * PITCH + lk * 8 + 4 * hf, bv[i]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
              acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][u], bv[j][u], acc[i][j], 0, 0, 0);
      }
    };
    const int nch = t_begin < t_end ? (t_end - t_begin + GM_KC - 1) / GM_KC : 0;
    lds_barrier();  // the previous split's last chunk is consumed
    if (nch > 0) {
      fetch(pa0, pb0, t_begin);
      if (nch > 1) fetch(pa1, pb1, t_begin + GM_KC);
      stage(pa0, pb0, 0);
    }
    lds_barrier();
    // chunk c sits in LDS buffer c % 2; register set c % 2 takes chunk c + 2
    for (int c = 0; c < nch; c += 2) {
      if (c + 2 < nch) fetch(pa0, pb0, t_begin + (c + 2) * GM_KC);
      multiply(0);
      if (c + 1 < nch) stage(pa1, pb1, 1);
      lds_barrier();  // buffer 1 is stored; buffer 0 is consumed
      if (c + 1 >= nch) break;
      if (c + 3 < nch) fetch(pa1, pb1, t_begin + (c + 3) * GM_KC);
      multiply(1);
      if (c + 2 < nch) stage(pa0, pb0, 0);
      lds_barrier();  // buffer 0 is stored; buffer 1 is consumed
    }
    TTG_GLOBAL double* out = gmem(g.out) + (long long)s * g.gcap * g.gcap;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = a0 + qa * 32 + i * 16 + lk + 4 * v;
          const int c = b0 + qb * 32 + j * 16 + lr;
          if (a < g.M && c < g.M) out[(long long)a * g.gcap + c] = acc[i][j][v];
        }
  }
}

template <typename Acc, typename F>
__global__ void __launch_bounds__(256) gram_reduce_kernel(F f) {
  const int b = blockIdx.z;
  GramArgs g;
  if (!f(b, g)) return;
  g.splits = gram_split_count(g.T, g.splits);
  const int mm = g.M * g.M;  // 32-bit index arithmetic (M <= a few thousand)
  const long long plane = (long long)g.gcap * g.gcap;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < mm; e += gridDim.x * blockDim.x) {
    const int a = e / g.M, c = e - (e / g.M) * g.M;
    if (a > c) continue;
    const long long ix = (long long)a * g.gcap + c;
    typename Acc::V s = Acc::load(g.out, ix);
    // the planes' loads are issued four at a time (all in flight together);
    // the sum still runs over the planes in order
    int sp = 1;
    for (; sp + 4 <= g.splits; sp += 4) {
      const typename Acc::V v0 = Acc::load(g.out + (sp + 0) * plane * Acc::words, ix);
      const typename Acc::V v1 = Acc::load(g.out + (sp + 1) * plane * Acc::words, ix);
      const typename Acc::V v2 = Acc::load(g.out + (sp + 2) * plane * Acc::words, ix);
      const typename Acc::V v3 = Acc::load(g.out + (sp + 3) * plane * Acc::words, ix);
      s = Acc::add(s, v0);
      s = Acc::add(s, v1);
      s = Acc::add(s, v2);
      s = Acc::add(s, v3);
    }
    for (; sp < g.splits; ++sp) s = Acc::add(s, Acc::load(g.out + sp * plane * Acc::words, ix));
    Acc::store(g.out, (long long)a * g.gcap + c, s);
    Acc::store(g.out, (long long)c * g.gcap + a, s);
  }
}

// ---------------------------------------------------------------------------
// Pivoted Cholesky  G ~= P L L^T P^T  with diagonal pivoting, stopped when
// the largest remaining Schur diagonal is <= tau2 * trace(G) or when rmax
// columns exist.  One workgroup per filter.  The factor is kept in the
// accumulator precision (lwork, column-major gcap x rmax) and rounded to FP64
// into lfac (row-major, rows in the ORIGINAL order, so that rows piv[0..r)
// form a lower-triangular r x r block).  Writes *rank_out and the residual
// trace of the remaining Schur complement.
// ---------------------------------------------------------------------------
#define PC_LDS_COLS 48
struct PcholArgs {
  int M;                // dimension of G
  const double* g;      // G (accumulator type), ld gcap
  double* lwork;        // accumulator-type factor, column-major ld gcap
  double* lfac;         // FP64 factor, row-major ld gcap
  int* piv;             // pivots
  int* rank_out;        // where the rank is written
  double* resid_out;    // residual trace
  int* status;          // filter status (capacity overflow)
  int gcap;
  int rmax;             // rank capacity
  double tau2;          // relative threshold on the Schur diagonal
  double tau2_flag;     // a full-capacity stop flags TT_STATUS_CAPACITY only when the
                        // residual trace exceeds max(tau2, tau2_flag) x the trace
};

template <typename Acc, typename F>
__global__ void __launch_bounds__(256) pchol_kernel(F f, int ncl) {
  const int b = blockIdx.x;
  PcholArgs p;
  p.tau2_flag = 0.0;
  if (!f(b, p)) return;
  using V = typename Acc::V;
  extern __shared__ double smem[];
  // layout: diag (M V) | lp (rmax V) | flags (M int) | red
  const int jmax = min(p.M, p.rmax);
  V* diag = reinterpret_cast<V*>(smem);
  V* lp = diag + p.M;                           // jmax entries
  int* done = reinterpret_cast<int*>(lp + jmax);  // M entries
  // FP64 accumulation: the first ncl (<= PC_LDS_COLS, as many as the LDS
  // holds) factor columns are also kept in LDS (column-major, pitch M), so
  // each pivot step reads the thread's earlier entries from LDS instead of
  // global memory
  constexpr bool lds_cols = sizeof(V) == sizeof(double);
  V* lc = reinterpret_cast<V*>(smem + (((size_t)(p.M + jmax) * sizeof(V) + (size_t)p.M * sizeof(int) + 7) / 8));
  __shared__ double red_v[8];
  __shared__ int red_i[8];
  __shared__ int s_piv;
  __shared__ double s_trace;
  const int tid = threadIdx.x, nt = blockDim.x;
  double tr_part = 0.0;
  for (int i = tid; i < p.M; i += nt) {
    diag[i] = Acc::load(p.g, (long long)i * p.gcap + i);
    done[i] = 0;
    tr_part += Acc::hi(diag[i]);
  }
  __syncthreads();
  {
    double t = block_sum(tr_part, red_v);
    if (tid == 0) s_trace = t;
  }
  __syncthreads();
  const double thr = p.tau2 * s_trace;
  const bool bad = !(s_trace == s_trace) || s_trace > 1.7e308;
  int j = 0;
  for (; j < jmax; ++j) {
    // argmax of the remaining diagonal
    double bv = -1.0;
    int bi = -1;
    for (int i = tid; i < p.M; i += nt) {
      if (!done[i]) {
        const double v = Acc::hi(diag[i]);
        if (v > bv || (v == bv && bi >= 0 && i < bi)) {
          bv = v;
          bi = i;
        }
      }
    }
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(bi, o, 64);
      if (ov > bv || (ov == bv && oi >= 0 && (bi < 0 || oi < bi))) {
        bv = ov;
        bi = oi;
      }
    }
    if ((tid & 63) == 0) {
      red_v[tid >> 6] = bv;
      red_i[tid >> 6] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double v = red_v[0];
      int ii = red_i[0];
      for (int w = 1; w < (nt + 63) / 64; ++w)
        if (red_v[w] > v || (red_v[w] == v && red_i[w] >= 0 && (ii < 0 || red_i[w] < ii))) {
          v = red_v[w];
          ii = red_i[w];
        }
      // stop when nothing is left above the threshold; the first column is
      // always produced (a zero or non-finite matrix gets a unit pivot)
      if (j == 0)
        s_piv = (ii >= 0 && !bad && v > 0.0) ? ii : -2 - (ii < 0 ? 0 : ii);
      else
        s_piv = (ii < 0 || bad || !(v > thr)) ? -1 : ii;
    }
    __syncthreads();
    int pv = s_piv;
    if (pv == -1) break;
    const bool zero_col = pv <= -2;
    if (zero_col) pv = -2 - pv;
    const V lpp = zero_col ? Acc::from(1.0) : Acc::sqrt_(diag[pv]);
    // cache row pv of the factor
    for (int t = tid; t < j; t += nt)
      lp[t] = (lds_cols && t < ncl) ? lc[(long long)t * p.M + pv] : Acc::load(p.lwork, (long long)t * p.gcap + pv);
    __syncthreads();
    for (int i = tid; i < p.M; i += nt) {
      V l;
      if (i == pv) {
        l = lpp;
      } else if (done[i] || zero_col) {
        l = Acc::zero();
      } else {
        V s = Acc::load(p.g, (long long)i * p.gcap + pv);
        // unrolled so that several terms' loads are in flight (the sum still
        // runs over t in order)
        if constexpr (lds_cols) {
          const int tl = min(j, ncl);
#pragma unroll 4
          for (int t = 0; t < tl; ++t) s = Acc::sub(s, Acc::mul(lc[(long long)t * p.M + i], lp[t]));
#pragma unroll 4
          for (int t = tl; t < j; ++t)
            s = Acc::sub(s, Acc::mul(Acc::load(p.lwork, (long long)t * p.gcap + i), lp[t]));
        } else {
#pragma unroll 4
          for (int t = 0; t < j; ++t)
            s = Acc::sub(s, Acc::mul(Acc::load(p.lwork, (long long)t * p.gcap + i), lp[t]));
        }
        l = Acc::div(s, lpp);
        diag[i] = Acc::sub(diag[i], Acc::mul(l, l));
      }
      Acc::store(p.lwork, (long long)j * p.gcap + i, l);
      if (lds_cols && j < ncl) lc[(long long)j * p.M + i] = l;
    }
    __syncthreads();
    if (tid == 0) {
      p.piv[j] = pv;
      done[pv] = 1;
      diag[pv] = Acc::zero();
    }
    __syncthreads();
    if (zero_col) {
      ++j;
      break;
    }
  }
  const int rank = j;
  // residual: trace of the remaining Schur complement
  double rp = 0.0;
  for (int i = tid; i < p.M; i += nt)
    if (!done[i]) rp += fmax(Acc::hi(diag[i]), 0.0);
  const double resid = block_sum(rp, red_v);
  if (tid == 0) {
    *p.rank_out = rank;
    if (p.resid_out) *p.resid_out = resid;
    if (rank == jmax && jmax < p.M && resid > fmax(p.tau2, p.tau2_flag) * s_trace && p.status)
      atomicOr(p.status, TT_STATUS_CAPACITY);
    if (bad && p.status) atomicOr(p.status, TT_STATUS_NONFINITE);
  }
  // FP64 row-major copy, zero beyond the rank
  for (int e = tid; e < p.M * rank; e += nt) {  // 32-bit index arithmetic
    const int i = e / rank, t = e - (e / rank) * rank;
    p.lfac[(long long)i * p.gcap + t] = Acc::hi(Acc::load(p.lwork, (long long)t * p.gcap + i));
  }
}

// ---------------------------------------------------------------------------
// One-sided Jacobi (Hestenes) on the columns of an FP64 matrix X (rows x
// ncols, read row-major from x with leading dimension ldx).  Rotations are
// applied until every column pair is orthogonal to relative tolerance 1e-15;
// the pair order is a round-robin tournament so that the pairs of one round
// are disjoint and run in parallel, one per wavefront.  Outputs the column
// norms (singular values) in descending order and the correspondingly
// permuted columns sigma_j * u_j (column-major in usv, ld gcap).
// ---------------------------------------------------------------------------
struct JacobiArgs {
  int rows, ncols;
  double tol2;      // a pair is orthogonal when ga^2 <= tol2 * al * be
  const double* x;  // row-major input
  long long ldx;
  double* work;     // column-major scratch, ld gcap
  double* sigma;    // out, descending
  double* usv;      // out, column-major, ld gcap
  int* ncols_out;   // nullable: number of columns written
  int gcap;
};

// Rotation of one-sided Jacobi (Hestenes) for the column pair with squared
// norms al, be and inner product ga (Rutishauser's formulas):
//   zeta = (be - al) / (2 ga),  t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
//   c = 1 / sqrt(1 + t^2),  s = c t.
// Returns false when the pair is already orthogonal to the relative
// tolerance sqrt(tol2) (ga^2 <= tol2 al be).  Reciprocals and reciprocal square roots start
// from the hardware approximations and take two Newton steps each, which
// reaches FP64 accuracy with a much shorter dependency chain than IEEE
// division and square root.
__device__ inline double jac_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __fma_rn(-x, r, 1.0);
  r = __fma_rn(r, e, r);
  e = __fma_rn(-x, r, 1.0);
  return __fma_rn(r, e, r);
}
__device__ inline double jac_rsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x * y;
  double e = __fma_rn(-h, y, 0.5);
  y = __fma_rn(y, e, y);
  h = 0.5 * x * y;
  e = __fma_rn(-h, y, 0.5);
  return __fma_rn(y, e, y);
}
__device__ inline bool jac_rotation(double al, double be, double ga, double& cs, double& sn, double tol2) {
  if (!(ga != 0.0 && ga * ga > tol2 * (al * be))) return false;
  const double zeta = (be - al) * 0.5 * jac_rcp(ga);
  double t;
  if (fabs(zeta) > 1.3e154) {
    // zeta^2 would overflow (a column many orders below its partner, as
    // rank-deficient inputs produce): t = 1 / (2 zeta) to working precision
    t = 0.5 * jac_rcp(zeta);
  } else {
    const double s1 = __fma_rn(zeta, zeta, 1.0);
    const double root = s1 * jac_rsq(s1);
    t = (zeta >= 0.0 ? 1.0 : -1.0) * jac_rcp(fabs(zeta) + root);
  }
  cs = jac_rsq(__fma_rn(t, t, 1.0));
  sn = cs * t;
  return true;
}

// One-sided Jacobi for at most JW_NMAX columns and few rows per lane, run by
// a single wavefront:
// the n/2 column pairs of a round each get LP = 64 / (n/2) lanes (rounded
// down to a power of two), which split the rows and reduce the three dot
// products with log2(LP) lane exchanges.  Same round-robin pairing, rotation
// and stopping rule as the workgroup version below.  Writes sigma (descending)
// and the scaled left vectors like it.
#define JW_NMAX 64
__device__ inline double jw_group_sum(double v, int lp) {
  for (int o = lp >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ void jacobi_wave(double* W, long long ldw, int rows, int nc, double* s_sig,
                                            const JacobiArgs& J) {
  const int lane = threadIdx.x & 63;
  const int n = (nc + 1) & ~1;
  const int npair = n / 2;
  int lp = 64;
  while (lp > 1 && lp * npair > 64) lp >>= 1;
  const int grp = lane / lp, lip = lane - grp * lp;
  const int ngrp = 64 / lp;
  for (int sweep = 0; sweep < 60 && n >= 2; ++sweep) {
    int rot = 0;
    for (int r = 0; r < n - 1; ++r) {
      for (int i0 = 0; i0 < npair; i0 += ngrp) {
        const int i = i0 + grp;
        int pc = -1, qc = -1;
        if (i < npair) {
          if (i == 0) {
            pc = n - 1;
            qc = r;
          } else {
            pc = (r + i) % (n - 1);
            qc = (r - i + (n - 1)) % (n - 1);
          }
        }
        const bool live = i < npair && pc < nc && qc < nc;
        double* xp = W + (long long)(live ? pc : 0) * ldw;
        double* xq = W + (long long)(live ? qc : 0) * ldw;
        double al = 0.0, be = 0.0, ga = 0.0;
        if (live)
          for (int k = lip; k < rows; k += lp) {
            const double u = xp[k], v = xq[k];
            al = __fma_rn(u, u, al);
            be = __fma_rn(v, v, be);
            ga = __fma_rn(u, v, ga);
          }
        al = jw_group_sum(al, lp);
        be = jw_group_sum(be, lp);
        ga = jw_group_sum(ga, lp);
        double cs, sn;
        if (live && jac_rotation(al, be, ga, cs, sn, J.tol2)) {
          for (int k = lip; k < rows; k += lp) {
            const double u = xp[k], v = xq[k];
            xp[k] = cs * u - sn * v;
            xq[k] = sn * u + cs * v;
          }
          rot = 1;
        }
        // the next round reads columns other lanes just rotated
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      }
    }
    // any lane rotated in this sweep?
    const unsigned long long any = __ballot(rot);
    if (!any) break;
  }
  // column norms
  for (int c = lane; c < nc; c += 64) {
    const double* xc = W + (long long)c * ldw;
    double s = 0.0;
    for (int k = 0; k < rows; ++k) s = __fma_rn(xc[k], xc[k], s);
    s_sig[c] = sqrt(s);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  // rank of each column in descending order (ties by index)
  for (int c = 0; c < nc; ++c) {
    const double sc = s_sig[c];
    int rk = 0;
    for (int o = lane; o < nc; o += 64) {
      const double so = s_sig[o];
      rk += (so > sc || (so == sc && o < c)) ? 1 : 0;
    }
    for (int o = 32; o > 0; o >>= 1) rk += __shfl_xor(rk, o, 64);
    if (lane == 0) J.sigma[rk] = sc;
    const double* xc = W + (long long)c * ldw;
    double* dst = J.usv + (long long)rk * J.gcap;
    for (int k = lane; k < rows; k += 64) dst[k] = xc[k];
  }
  if (lane == 0 && J.ncols_out) *J.ncols_out = nc;
}

// The sweep body, instantiated separately for columns in LDS and in global
// memory so that the compiler knows the address space of every column
// access (a pointer chosen at run time between the two would turn them all
// into flat accesses with global-memory latency).
__device__ __forceinline__ void jacobi_body(double* W, long long ldw, const JacobiArgs& J, double* s_sig,
                                            int& s_rot) {
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  const int rows = J.rows, nc = J.ncols;
  for (int e = tid; e < rows * nc; e += blockDim.x) {  // 32-bit index arithmetic
    const int i = e / nc, c = e - (e / nc) * nc;
    W[(long long)c * ldw + i] = J.x[(long long)i * J.ldx + c];
  }
  __syncthreads();
  const int n = (nc + 1) & ~1;  // even number of players (one may be a dummy)
  int lpw = 1;  // lanes per pair the single-wavefront path would need for <= 8 rows per lane
  while (lpw < 64 && 8 * lpw < rows) lpw *= 2;
  if (n <= JW_NMAX && (n / 2) * lpw <= 64) {
    // small problem: wavefront 0 runs every sweep alone (no block barriers);
    // decided per filter, so a filter's result does not depend on its batch
    if (wid == 0) jacobi_wave(W, ldw, rows, nc, s_sig, J);
    return;
  }
  const int npair = n / 2;
  int lp = 1;
  while (lp < 64 && 4 * 2 * lp <= rows) lp *= 2;      // about four rows per lane
  while (lp > 1 && lp * npair > (int)blockDim.x) lp >>= 1;
  const int grp = tid / lp, lip = tid - (tid / lp) * lp;
  const int ngrp = blockDim.x / lp;
  for (int sweep = 0; sweep < 60 && n >= 2; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int r = 0; r < n - 1; ++r) {
      // every pair of the round at once: pair i gets lp lanes (a power of
      // two <= 64 sized to about four rows per lane), which split the rows
      // and reduce the three dot products among themselves
      for (int i0 = 0; i0 < npair; i0 += ngrp) {
        const int i = i0 + grp;
        int pc = -1, qc = -1;
        if (i < npair) {
          if (i == 0) {
            pc = n - 1;
            qc = r;
          } else {
            pc = (r + i) % (n - 1);
            qc = (r - i + (n - 1)) % (n - 1);
          }
        }
        const bool live = i < npair && pc < nc && qc < nc;
        double* xp = W + (long long)(live ? pc : 0) * ldw;
        double* xq = W + (long long)(live ? qc : 0) * ldw;
        double al = 0.0, be = 0.0, ga = 0.0;
        if (live)
          for (int k = lip; k < rows; k += lp) {
            const double u = xp[k], v = xq[k];
            al = __fma_rn(u, u, al);
            be = __fma_rn(v, v, be);
            ga = __fma_rn(u, v, ga);
          }
        al = jw_group_sum(al, lp);
        be = jw_group_sum(be, lp);
        ga = jw_group_sum(ga, lp);
        double cs, sn;
        if (live && jac_rotation(al, be, ga, cs, sn, J.tol2)) {
          for (int k = lip; k < rows; k += lp) {
            const double u = xp[k], v = xq[k];
            xp[k] = cs * u - sn * v;
            xq[k] = sn * u + cs * v;
          }
          if (lip == 0) s_rot = 1;
        }
      }
      __syncthreads();
    }
    const int any = s_rot;
    __syncthreads();
    if (!any) break;
  }
  // column norms
  for (int c = wid; c < nc; c += nw) {
    const double* xc = W + (long long)c * ldw;
    double s = 0.0;
    for (int k = lane; k < rows; k += 64) s = __fma_rn(xc[k], xc[k], s);
    s = wave_sum(s);
    if (lane == 0) s_sig[c] = sqrt(s);
  }
  __syncthreads();
  // rank of each column in descending order (ties by index)
  for (int c = wid; c < nc; c += nw) {
    const double sc = s_sig[c];
    int rk = 0;
    for (int o = lane; o < nc; o += 64) {
      const double so = s_sig[o];
      rk += (so > sc || (so == sc && o < c)) ? 1 : 0;
    }
    for (int o = 32; o > 0; o >>= 1) rk += __shfl_xor(rk, o, 64);
    if (lane == 0) J.sigma[rk] = sc;
    const double* xc = W + (long long)c * ldw;
    double* dst = J.usv + (long long)rk * J.gcap;
    for (int k = lane; k < rows; k += 64) dst[k] = xc[k];
  }
  if (tid == 0 && J.ncols_out) *J.ncols_out = nc;
}

template <typename F>
__global__ void __launch_bounds__(512) jacobi_kernel(F f, int lds_doubles) {
  const int b = blockIdx.x;
  JacobiArgs J;
  if (!f(b, J)) return;
  // columns live in LDS when they fit (leading dimension = rows), else in
  // the global scratch (leading dimension gcap)
  extern __shared__ double jsm[];
  __shared__ int s_rot;
  __shared__ double s_sig[1024];
  if ((long long)J.rows * J.ncols <= lds_doubles)
    jacobi_body(jsm, J.rows, J, s_sig, s_rot);
  else
    jacobi_body(J.work, J.gcap, J, s_sig, s_rot);
}

// ---------------------------------------------------------------------------
// Q(j, c) = [L11^{-1} Z(piv, :)](j, c) by forward substitution, one column c
// per lane, partial solutions kept in FP64 shared memory.  L11(j, t) =
// lfac[piv[j]*gcap + t].  Z rows are read with stride ldz, Q rows written with
// stride ldq.
// ---------------------------------------------------------------------------
struct TrsmArgs {
  int r, m;
  const double* lfac;
  const int* piv;
  int gcap;
  const void* z;
  long long ldz;
  void* q;
  long long ldq;
  int zt_n;  // 0: Z columns in output order; n: Z columns ordered (j, i), output c = i*(m/n) + j
  double* wbuf;  // gcap x gcap FP64 scratch for the explicit inverse (tri_* kernels)
};

template <typename TZ, typename TQ, typename F>
__global__ void __launch_bounds__(64) trsm_kernel(F f, int rcap, int l_in_lds) {
  const int b = blockIdx.z;
  TrsmArgs a;
  if (!f(b, a)) return;
  if (blockIdx.x * 64 >= a.m) return;
  extern __shared__ double qs[];  // rcap x 64 partial solutions, then r x r factor
  double* ls = qs + (long long)rcap * 64;
  const TZ* z = reinterpret_cast<const TZ*>(a.z);
  TQ* q = reinterpret_cast<TQ*>(a.q);
  const bool lds_l = l_in_lds && a.r <= rcap;
  if (lds_l) {
    for (int e = threadIdx.x; e < a.r * a.r; e += 64) {
      const int j = e / a.r, t = e % a.r;
      ls[e] = (t <= j) ? a.lfac[(long long)a.piv[j] * a.gcap + t] : 0.0;
    }
    __syncthreads();
  }
  // grid-stride over 64-column blocks (the grid is sized for the usual width)
  for (int cb = blockIdx.x; cb * 64 < a.m; cb += gridDim.x) {
  const int c = cb * 64 + threadIdx.x;
  const bool live = c < a.m;
  for (int j = 0; j < a.r; ++j) {
    const double* lrow = lds_l ? ls + (long long)j * a.r : a.lfac + (long long)a.piv[j] * a.gcap;
    long long zc = c;
    if (a.zt_n) {
      const int nn = a.m / a.zt_n;
      zc = (long long)(c % nn) * a.zt_n + c / nn;
    }
    double s = live ? bulk_to_double(z[(long long)a.piv[j] * a.ldz + zc]) : 0.0;
    for (int t = 0; t < j; ++t) s = __fma_rn(-lrow[t], qs[t * 64 + threadIdx.x], s);
    const double v = s / lrow[j];
    qs[j * 64 + threadIdx.x] = v;
    if (live) q[(long long)j * a.ldq + c] = from_double<TQ>(v);
  }
  }
}

// FP64 outputs: the same forward substitution with the partial solutions
// read back from the (exact, FP64) output rows instead of LDS, so a
// workgroup needs no capacity-sized LDS and many run per CU; the pivot
// block is staged in LDS when it is small.
#define TS_LDS_R 64
template <typename TZ, typename F>
__global__ void __launch_bounds__(256) trsm_f64_kernel(F f) {
  const int b = blockIdx.z;
  TrsmArgs a;
  if (!f(b, a)) return;
  if (blockIdx.x * 256 >= a.m) return;
  __shared__ double ls[TS_LDS_R * TS_LDS_R];
  const int r = a.r;
  const bool lds_l = r <= TS_LDS_R;
  if (lds_l) {
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
      const int j = e / r, t = e - (e / r) * r;
      ls[e] = (t <= j) ? a.lfac[(long long)a.piv[j] * a.gcap + t] : 0.0;
    }
    __syncthreads();
  }
  const TZ* z = reinterpret_cast<const TZ*>(a.z);
  double* q = reinterpret_cast<double*>(a.q);
  for (int cb = blockIdx.x; cb * 256 < a.m; cb += gridDim.x) {
    const int c = cb * 256 + threadIdx.x;
    if (c >= a.m) continue;
    long long zc = c;
    if (a.zt_n) {
      const int nn = a.m / a.zt_n;
      zc = (long long)(c % nn) * a.zt_n + c / nn;
    }
    for (int j = 0; j < r; ++j) {
      double s = bulk_to_double(z[(long long)a.piv[j] * a.ldz + zc]);
      if (lds_l) {
        const double* lrow = ls + (long long)j * r;
#pragma unroll 4
        for (int t = 0; t < j; ++t) s = __fma_rn(-lrow[t], q[(long long)t * a.ldq + c], s);
        q[(long long)j * a.ldq + c] = s / lrow[j];
      } else {
        const double* lrow = a.lfac + (long long)a.piv[j] * a.gcap;
#pragma unroll 4
        for (int t = 0; t < j; ++t) s = __fma_rn(-lrow[t], q[(long long)t * a.ldq + c], s);
        q[(long long)j * a.ldq + c] = s / lrow[j];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// The same Q = L_pp^{-1} Z_p through an explicit inverse (FP32 bulk path,
// where the factor's conditioning is bounded by the FP32 pre-truncation):
// tri_inverse_kernel forms W = L_pp^{-1} (one filter per workgroup; thread c
// solves L_pp w = e_c for its own column, so threads never wait for each
// other) and stores column c of W contiguously, wt[c * gcap + j] = W(j, c),
// zeros above the diagonal.  tri_apply_kernel gives each output column to
// one thread, which accumulates 32 rows at a time in FP64 registers while W
// is read with wave-uniform loads.
// ---------------------------------------------------------------------------
template <typename F, bool InLds>
__global__ void __launch_bounds__(256) tri_inverse_kernel(F f) {
  const int b = blockIdx.z;
  TrsmArgs a;
  if (!f(b, a)) return;
  // the pivot block L_pp (lower triangle, row j = lfac row piv[j]) in LDS
  // when it fits, else read in place (only t <= j is ever touched)
  extern __shared__ double lpp[];  // [r][r]
  const int r = a.r;
  if (InLds) {
    for (int e = threadIdx.x; e < r * r; e += blockDim.x) {
      const int j = e / r, t = e - (e / r) * r;
      lpp[e] = (t <= j) ? a.lfac[(long long)a.piv[j] * a.gcap + t] : 0.0;
    }
    __syncthreads();
  }
  double* wt = a.wbuf;
  for (int c = threadIdx.x; c < r; c += blockDim.x) {
    double* w = wt + (long long)c * a.gcap;
    for (int j = 0; j < c; ++j) w[j] = 0.0;
    for (int j = c; j < r; ++j) {
      const double* lrow = InLds ? lpp + (long long)j * r : a.lfac + (long long)a.piv[j] * a.gcap;
      double s = (j == c) ? 1.0 : 0.0;
#pragma unroll 4
      for (int t = c; t < j; ++t) s = __fma_rn(-lrow[t], w[t], s);
      w[j] = s / lrow[j];
    }
  }
}

#define TA_ROWS 32
#define TA_TMAX 128  // rows of W staged in LDS at a time
#define TA_ZB 8      // rows of Z loaded ahead per batch
template <typename TZ, typename TQ, typename F>
__global__ void __launch_bounds__(256) tri_apply_kernel(F f) {
  const int b = blockIdx.z;
  TrsmArgs a;
  if (!f(b, a)) return;
  if (blockIdx.x * 256 >= a.m) return;
  __shared__ double ws[TA_TMAX * TA_ROWS];  // W(j0 + u, t0 + t) at ws[t * 32 + u], zero past row r
  __shared__ int pvs[TA_TMAX];              // piv[t0 + t]
  const TTG_GLOBAL TZ* z = gmem(reinterpret_cast<const TZ*>(a.z));
  TTG_GLOBAL TQ* q = gmem(reinterpret_cast<TQ*>(a.q));
  const TTG_GLOBAL double* wt = gmem(static_cast<const double*>(a.wbuf));
  const TTG_GLOBAL int* piv = gmem(static_cast<const int*>(a.piv));
  const int r = a.r;
  for (int j0 = 0; j0 < r; j0 += TA_ROWS) {
    const int tend = min(r, j0 + TA_ROWS);  // W(j, t) = 0 for t > j
    const int jn = min(TA_ROWS, r - j0);
    // stage W(j0.., t0..t1) and the pivots of t0..t1 (workgroup-uniform calls)
    auto stage = [&](int t0, int t1) {
      lds_barrier();  // previous chunk consumed
      for (int e = threadIdx.x; e < (t1 - t0) * TA_ROWS; e += blockDim.x) {
        const int t = e / TA_ROWS, u = e - t * TA_ROWS;
        ws[e] = u < jn ? wt[(long long)(t0 + t) * a.gcap + j0 + u] : 0.0;
      }
      for (int t = threadIdx.x; t < t1 - t0; t += blockDim.x) pvs[t] = piv[t0 + t];
      lds_barrier();
    };
    const bool once = tend <= TA_TMAX;  // every t of this chunk fits at once
    if (once) stage(0, tend);
    // grid-stride over 256-column blocks: the grid is sized for the usual
    // width, not the capacity, so few workgroups start with nothing to do
    for (int cb = blockIdx.x; cb * 256 < a.m; cb += gridDim.x) {
      const int c = cb * 256 + threadIdx.x;
      const bool live = c < a.m;
      long long zc = live ? c : 0;
      if (a.zt_n) {
        const int nn = a.m / a.zt_n;
        zc = (long long)(zc % nn) * a.zt_n + zc / nn;
      }
      double acc[TA_ROWS];
#pragma unroll
      for (int u = 0; u < TA_ROWS; ++u) acc[u] = 0.0;
      for (int t0 = 0; t0 < tend; t0 += TA_TMAX) {
        const int t1 = min(tend, t0 + TA_TMAX);
        if (!once) stage(t0, t1);
        // TA_ZB rows of Z in flight at once; t ascends, as in the plain loop
        for (int tb = t0; tb < t1; tb += TA_ZB) {
          double zv[TA_ZB];
#pragma unroll
          for (int x = 0; x < TA_ZB; ++x) {
            const int t = min(tb + x, t1 - 1);
            zv[x] = bulk_to_double(z[(long long)pvs[t - t0] * a.ldz + zc]);
          }
#pragma unroll
          for (int x = 0; x < TA_ZB; ++x) {
            if (tb + x < t1) {
              const double* wrow = ws + (tb + x - t0) * TA_ROWS;
#pragma unroll
              for (int u = 0; u < TA_ROWS; ++u) acc[u] = __fma_rn(wrow[u], zv[x], acc[u]);
            }
          }
        }
      }
      if (live) {
#pragma unroll
        for (int u = 0; u < TA_ROWS; ++u)
          if (u < jn) q[(long long)(j0 + u) * a.ldq + c] = from_double<TQ>(acc[u]);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Generic batched GEMM  C(m, n) = sum_k A(m, k) B(k, n), strided operands,
// 64x64 output tiles, 16-wide k steps, 256 threads with 4x4 outputs each.
// ---------------------------------------------------------------------------
struct GemmArgs {
  int M, N, K;
  const void* a;
  long long sam, sak;
  const void* b;
  long long sbk, sbn;
  void* c;
  long long scm, scn;
};

template <typename TA, typename TB, typename TC, typename TAcc, typename F>
__global__ void __launch_bounds__(256) gemm_kernel(F f) {
  const int bz = blockIdx.z;
  GemmArgs g;
  if (!f(bz, g)) return;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  if (m0 >= g.M || n0 >= g.N) return;
  __shared__ TAcc As[16][64 + 1];
  __shared__ TAcc Bs[16][64 + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  TAcc acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = (TAcc)0;
  const TA* A = reinterpret_cast<const TA*>(g.a);
  const TB* B = reinterpret_cast<const TB*>(g.b);
  const bool a_kfast = (g.sak == 1);
  const bool b_nfast = (g.sbn == 1);
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      int mm, kk;
      if (a_kfast) {
        mm = e >> 4;
        kk = e & 15;
      } else {
        kk = e >> 6;
        mm = e & 63;
      }
      const int m = m0 + mm, k = k0 + kk;
      As[kk][mm] = (m < g.M && k < g.K) ? (TAcc)A[(long long)m * g.sam + (long long)k * g.sak] : (TAcc)0;
      int nn, kb;
      if (b_nfast) {
        kb = e >> 6;
        nn = e & 63;
      } else {
        nn = e >> 4;
        kb = e & 15;
      }
      const int n = n0 + nn, k2 = k0 + kb;
      Bs[kb][nn] = (n < g.N && k2 < g.K) ? (TAcc)B[(long long)k2 * g.sbk + (long long)n * g.sbn] : (TAcc)0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      TAcc av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] += av[i] * bv[j];
    }
    __syncthreads();
  }
  TC* C = reinterpret_cast<TC*>(g.c);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + ty * 4 + i, n = n0 + tx * 4 + j;
      if (m < g.M && n < g.N) C[(long long)m * g.scm + (long long)n * g.scn] = (TC)acc[i][j];
    }
}

// ---------------------------------------------------------------------------
// FP32 GEMM on the matrix cores, C(m, n) = sum_k A(m, k) B(k, n), FP32 output
// (A, B FP32 or FP64, rounded to FP32 as they are staged; FP32 accumulation
// with v_mfma_f32_16x16x4f32).  Output tiles of TM x TN (64 x 64, or
// 128 x 32 for tall-skinny products), a 32 x 32 quadrant per wavefront,
// chunks of 16 k staged in LDS with each lane's four operands of a chunk
// contiguous (k-lane lk takes k = 4 lk + s in step s).  The workgroups of a
// filter stride over its tiles.  Every element sums its k in the same order
// for any tile shape, so the result does not depend on the launch shape.
// ---------------------------------------------------------------------------
typedef float gf4 __attribute__((ext_vector_type(4)));
#define GF_KC 16
#define GF_PITCH (GF_KC + 4)
template <typename TA, typename TB, int TN, typename F>
__global__ void __launch_bounds__(256) gemm_mfma_kernel(F f) {
  constexpr int TM = 8192 / (TN * 2);  // 64 x 64 or 128 x 32
  constexpr int QN = TN / 32;          // quadrants across n
  const int bz = blockIdx.z;
  GemmArgs g;
  if (!f(bz, g)) return;
  __shared__ float As[TM * GF_PITCH];
  __shared__ float Bs[TN * GF_PITCH];
  const TTG_GLOBAL TA* A = gmem(reinterpret_cast<const TA*>(g.a));
  const TTG_GLOBAL TB* Bm = gmem(reinterpret_cast<const TB*>(g.b));
  TTG_GLOBAL float* C = gmem(reinterpret_cast<float*>(g.c));
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int qa = wv / QN, qb = wv - (wv / QN) * QN;
  const int lr = lane & 15, lk = lane >> 4;
  const int tnn = (g.N + TN - 1) / TN;
  const int ntiles = ((g.M + TM - 1) / TM) * tnn;
  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int m0 = (tile / tnn) * TM, n0 = (tile - (tile / tnn) * tnn) * TN;
    gf4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = gf4{0.f, 0.f, 0.f, 0.f};
    // each thread stages PA elements of A and PB of B per chunk; the next
    // chunk is loaded into registers while the current one is multiplied
    constexpr int PA = TM * GF_KC / 256, PB = TN * GF_KC / 256;
    float ra[PA], rb[PB];
    auto fetch = [&](int k0) {
#pragma unroll
      for (int u = 0; u < PA; ++u) {
        const int e = tid + u * 256;
        int m, kk;
        if (g.sak == 1) {
          m = e / GF_KC;
          kk = e - m * GF_KC;
        } else {
          kk = e / TM;
          m = e - kk * TM;
        }
        const int mg = m0 + m, k = k0 + kk;
        ra[u] = (mg < g.M && k < g.K) ? (float)A[(long long)mg * g.sam + (long long)k * g.sak] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < PB; ++u) {
        const int e = tid + u * 256;
        int n, kk;
        if (g.sbn == 1) {
          kk = e / TN;
          n = e - kk * TN;
        } else {
          n = e / GF_KC;
          kk = e - n * GF_KC;
        }
        const int ng = n0 + n, k = k0 + kk;
        rb[u] = (ng < g.N && k < g.K) ? (float)Bm[(long long)k * g.sbk + (long long)ng * g.sbn] : 0.f;
      }
    };
    fetch(0);
    for (int k0 = 0; k0 < g.K; k0 += GF_KC) {
      lds_barrier();  // previous chunk consumed
#pragma unroll
      for (int u = 0; u < PA; ++u) {
        const int e = tid + u * 256;
        int m, kk;
        if (g.sak == 1) {
          m = e / GF_KC;
          kk = e - m * GF_KC;
        } else {
          kk = e / TM;
          m = e - kk * TM;
        }
        As[m * GF_PITCH + kk] = ra[u];
      }
#pragma unroll
      for (int u = 0; u < PB; ++u) {
        const int e = tid + u * 256;
        int n, kk;
        if (g.sbn == 1) {
          kk = e / TN;
          n = e - kk * TN;
        } else {
          n = e / GF_KC;
          kk = e - n * GF_KC;
        }
        Bs[n * GF_PITCH + kk] = rb[u];
      }
      lds_barrier();
      if (k0 + GF_KC < g.K) fetch(k0 + GF_KC);
      constexpr int KS = GF_KC / 4;  // MFMA steps per chunk; lane lk takes k = KS lk + s
      float av[2][KS], bv[2][KS];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int u = 0; u < KS; u += 4) {
          const float4 ta = *reinterpret_cast<const float4*>(As + (qa * 32 + i * 16 + lr) * GF_PITCH + lk * KS + u);
          const float4 tb = *reinterpret_cast<const float4*>(Bs + (qb * 32 + i * 16 + lr) * GF_PITCH + lk * KS + u);
          av[i][u] = ta.x;
          av[i][u + 1] = ta.y;
          av[i][u + 2] = ta.z;
          av[i][u + 3] = ta.w;
          bv[i][u] = tb.x;
          bv[i][u + 1] = tb.y;
          bv[i][u + 2] = tb.z;
          bv[i][u + 3] = tb.w;
        }
#pragma unroll
      for (int u = 0; u < KS; ++u)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i][u], bv[j][u], acc[i][j], 0, 0, 0);
    }
    // D layout: lane (lr, lk), register v holds row 4 lk + v, column lr
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int m = m0 + qa * 32 + i * 16 + 4 * lk + v;
          const int n = n0 + qb * 32 + j * 16 + lr;
          if (m < g.M && n < g.N) C[(long long)m * g.scm + (long long)n * g.scn] = acc[i][j][v];
        }
  }
}

// ---------------------------------------------------------------------------
// Tall-skinny GEMM  C(m, n) = sum_k A(m, k) B(k, n)  for M >> K, N <= 128:
// A and C row-major (bulk type), B row-major FP64 (ld sbk).  Each thread owns
// one row and a group of 32 output columns (accumulators in registers); a
// workgroup stages 256/G rows x 32 k of A and the matching 32 x N slice of B
// in LDS (G = number of column groups), so A is read from HBM exactly once
// with coalesced 128-byte row segments.
// ---------------------------------------------------------------------------
#define TSK_KC 32
template <typename T, typename F>
__global__ void __launch_bounds__(256) tall_gemm_kernel(F f, int Gmax) {
  const int bz = blockIdx.z;
  GemmArgs g;
  if (!f(bz, g)) return;
  // column groups for this filter's actual N (a power of two <= Gmax); the
  // grid covers the smallest row block, surplus workgroups exit
  int G = 1;
  while (32 * G < g.N && G < Gmax) G *= 2;
  if (g.N > 32 * G) return;
  const int RW = 256 / G;  // rows per workgroup
  extern __shared__ unsigned char smem_raw[];
  T* Xs = reinterpret_cast<T*>(smem_raw);   // [RW][KC+1]
  T* Ls = Xs + RW * (TSK_KC + 1);           // [KC][32*G]
  const int tid = threadIdx.x;
  const int cg = tid / RW, row = tid % RW;
  const int NW = 32 * G;
  const T* A = reinterpret_cast<const T*>(g.a);
  const double* Bm = reinterpret_cast<const double*>(g.b);
  for (int m0 = blockIdx.x * RW; m0 < g.M; m0 += gridDim.x * RW) {
  T acc[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) acc[c] = (T)0;
  for (int k0 = 0; k0 < g.K; k0 += TSK_KC) {
    // stage A rows m0..m0+RW, columns k0..k0+KC
    for (int e = tid; e < RW * TSK_KC; e += 256) {
      const int r = e / TSK_KC, kk = e % TSK_KC;
      const int m = m0 + r, k = k0 + kk;
      Xs[r * (TSK_KC + 1) + kk] = (m < g.M && k < g.K) ? A[(long long)m * g.sam + k] : (T)0;
    }
    for (int e = tid; e < TSK_KC * NW; e += 256) {
      const int kk = e / NW, n = e % NW;
      const int k = k0 + kk;
      Ls[e] = (k < g.K && n < g.N) ? (T)Bm[(long long)k * g.sbk + n] : (T)0;
    }
    __syncthreads();
    const int kmax = min(TSK_KC, g.K - k0);
    for (int kk = 0; kk < kmax; ++kk) {
      const T x = Xs[row * (TSK_KC + 1) + kk];
      const T* lrow = Ls + kk * NW + cg * 32;
#pragma unroll
      for (int c = 0; c < 32; ++c) acc[c] += x * lrow[c];
    }
    __syncthreads();
  }
  const int m = m0 + row;
  if (m < g.M) {
    T* C = reinterpret_cast<T*>(g.c) + (long long)m * g.scm;
#pragma unroll
    for (int c = 0; c < 32; ++c) {
      const int n = cg * 32 + c;
      if (n < g.N) C[n] = acc[c];
    }
  }
  }
}
