// Deterministic TT-cross on the device (Sec. 3.3 cross approximation, with
// maxvol pivots in place of the paper's randomised greedy cross), used by
// tt_kernel_build_cross to build the transition kernel of eq. TPMmat from
// point values, for any d.  Included by api.hip.
//
// Per bond the fibre matrix is the core 0 of a two-core train (M, I); its
// rounding (the library's Gram / pivoted Cholesky / Jacobi SVD) gives an
// orthonormal basis U of M's numerical range, whose rank becomes the bond's
// cross rank; maxvol on U picks that many rows (the index sets of the next
// step) and, in a right-to-left sweep, B = U U_rows^{-1} is the core in
// interpolation form.
#pragma once

namespace ttg {

static const int CROSS_RMAX = 64;

// Everything the point-value functor of the kernel needs, per filter:
// K(m) = c exp(-1/2 y^T Lam y), y_l = dx_l (m_l - h_l), m_l in [0, 2 h_l].
struct CrossKernelFn {
  int d;
  int h[TT_MAXD];
  double dx[TT_MAXD];
  double lam[TT_MAXD * TT_MAXD];
  double c;
  __device__ double operator()(const int* idx) const {
    double y[TT_MAXD];
    for (int l = 0; l < d; ++l) y[l] = dx[l] * (double)(idx[l] - h[l]);
    double quad = 0.0;
    for (int l = 0; l < d; ++l) {
      double s = 0.0;
      for (int j = 0; j < d; ++j) s += lam[l * d + j] * y[j];
      quad += y[l] * s;
    }
    return c * exp(-0.5 * quad);
  }
};

// Value of a FP64 TT (ranks <= 32, log-scale left out) at a multi-index.
__device__ inline double cross_tt_value(const DevTT& t, const int* j) {
  double v[32], w[32];
  int r0 = 1;
  v[0] = 1.0;
  for (int k = 0; k < t.d; ++k) {
    const int r1 = t.ranks[k + 1], n = t.n[k];
    const double* c = core_ptr<double>(t, k);
    for (int b = 0; b < r1; ++b) {
      double s = 0.0;
      for (int a = 0; a < r0; ++a) s += v[a] * c[((long long)a * n + j[k]) * r1 + b];
      w[b] = s;
    }
    for (int b = 0; b < r1; ++b) v[b] = w[b];
    r0 = r1;
  }
  return v[0];
}

// Multilinear interpolation onto an axis-aligned grid of weights held on the
// lattice x(j) = F (lo_l + dx_l o j) (the temporary predictive of Alg. 3):
// at x = lo + dx o i, u = (F diag dx_l)^{-1} (x - F lo_l), weights over the
// 2^d lattice neighbours of u, zero for a neighbour off the lattice.
struct CrossInterpFn {
  int d;
  double lo[TT_MAXD], dx[TT_MAXD];  // the target grid
  double a[TT_MAXD * TT_MAXD];      // (F diag dx_l)^{-1}
  double c[TT_MAXD];                // F lo_l
  DevTT src;                        // weights on the lattice, FP64
  __device__ double operator()(const int* idx) const {
    double u[TT_MAXD], t[TT_MAXD];
    int j0[TT_MAXD];
    for (int l = 0; l < d; ++l) {
      double s = 0.0;
      for (int m = 0; m < d; ++m) s += a[l * d + m] * (lo[m] + dx[m] * idx[m] - c[m]);
      u[l] = s;
      const double fl = floor(s);
      j0[l] = (int)fl;
      t[l] = s - fl;
    }
    double acc = 0.0;
    for (int corner = 0; corner < (1 << d); ++corner) {
      int j[TT_MAXD];
      double w = 1.0;
      bool in = true;
      for (int l = 0; l < d; ++l) {
        const int bit = (corner >> l) & 1;
        j[l] = j0[l] + bit;
        w *= bit ? t[l] : 1.0 - t[l];
        in = in && j[l] >= 0 && j[l] < src.n[l];
      }
      if (in && w != 0.0) acc += w * cross_tt_value(src, j);
    }
    return acc;
  }
};

// Cross state per filter (device): index sets and their counts.
//   iset + (k * CROSS_RMAX + a) * TT_MAXD: tuple a of I_k (axes 0..k-1)
//   jset + (k * CROSS_RMAX + a) * TT_MAXD: tuple a of J_k (axes k..d-1)
//   cnt[0..d]: counts of I_k, cnt[TT_MAXD+1 + k]: counts of J_k
//   rowsk + k * CROSS_RMAX: the maxvol rows that made J_k and core k (the
//   last right-to-left pass), ruk[k] the rank of that fibre matrix's basis
//   and seedk + k * CROSS_RMAX the rows that completed it; tgt[0..d]: the
//   rank targets of the last level
// iset, jset, cnt, rowsk, ruk, seedk and tgt are one block of
// CROSS_STATE_INTS ints, so that a finished cross can be saved and replayed.
struct CrossState {
  int* iset;
  int* jset;
  int* cnt;
  int* rowsk;
  int* ruk;
  int* seedk;
  int* tgt;
  double* work;  // maxvol scratch: m x r working copy, B, r x 2r inverse
  int* rows;     // maxvol pivots
};
static const long long CROSS_SET_INTS = (long long)(TT_MAXD + 1) * CROSS_RMAX * TT_MAXD;
static const long long CROSS_STATE_INTS =
    2 * CROSS_SET_INTS + 2 * (TT_MAXD + 1) + 2LL * (TT_MAXD + 1) * CROSS_RMAX + 2 * (TT_MAXD + 1);

// Fibre matrix of core k as core 0 of the two-core train T (rows_cap rows,
// R columns), core 1 of T the R x R identity.
//   dir 0 (left to right): row a * n_k + i,  column b:  f(I_k[a], i, J_{k+1}[b])
//   dir 1 (right to left): row i * bcap + b, column a:  f(I_k[a], i, J_{k+1}[b])
// Entries outside the current counts are zero.  Grid (elements, filter).
template <typename Fn>
__global__ void cross_fibre_kernel(const Fn* __restrict__ fn, const CrossState* __restrict__ cs,
                                   const DevTT* __restrict__ T, int d, int k, int nk, int dir, int rows_cap, int R,
                                   int bcap) {
  const int f = blockIdx.y;
  const Fn& F = fn[f];
  const CrossState& S = cs[f];
  const DevTT& t = T[f];
  const int ci = S.cnt[k], cj = S.cnt[TT_MAXD + 1 + k + 1];
  double* core0 = core_ptr<double>(t, 0);
  double* core1 = core_ptr<double>(t, 1);
  const long long tot = (long long)rows_cap * R;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x) {
    const int row = (int)(e / R), col = (int)(e % R);
    int a, i, b;
    if (dir == 0) {
      a = row / nk;
      i = row % nk;
      b = col;
    } else {
      i = row / bcap;
      b = row % bcap;
      a = col;
    }
    double v = 0.0;
    if (a < ci && b < cj && i < nk) {
      int idx[TT_MAXD];
      const int* ti = S.iset + ((long long)k * CROSS_RMAX + a) * TT_MAXD;
      const int* tj = S.jset + ((long long)(k + 1) * CROSS_RMAX + b) * TT_MAXD;
      for (int l = 0; l < k; ++l) idx[l] = ti[l];
      idx[k] = i;
      for (int l = k + 1; l < d; ++l) idx[l] = tj[l - (k + 1)];
      v = F(idx);
    }
    core0[e] = v;
  }
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < (long long)R * R;
       e += (long long)gridDim.x * blockDim.x)
    core1[e] = (e / R == e % R) ? 1.0 : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    t.ranks[0] = 1;
    t.ranks[1] = R;
    t.ranks[2] = 1;
    *t.log_scale = 0.0;
    *t.status = 0;
  }
}

// Core 0 of the cross TT: (1, n_0, |J_1|), entries f(i, J_1[b]).
template <typename Fn>
__global__ void cross_first_core_kernel(const Fn* __restrict__ fn, const CrossState* __restrict__ cs,
                                        const DevTT* __restrict__ Y, int d, int n0) {
  const int f = blockIdx.y;
  const Fn& F = fn[f];
  const CrossState& S = cs[f];
  const DevTT& y = Y[f];
  const int cj = S.cnt[TT_MAXD + 1 + 1];
  double* c = core_ptr<double>(y, 0);
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n0 * cj; e += gridDim.x * blockDim.x) {
    const int i = e / cj, b = e % cj;
    int idx[TT_MAXD];
    idx[0] = i;
    const int* tj = S.jset + ((long long)1 * CROSS_RMAX + b) * TT_MAXD;
    for (int l = 1; l < d; ++l) idx[l] = tj[l - 1];
    c[e] = F(idx);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    y.ranks[0] = 1;
    y.ranks[1] = cj;
  }
}

// maxvol on the basis U = core 0 of the rounded two-core train (rows m,
// rank r0 = its ranks[1]), completed to `want` columns when r0 is smaller:
// initial rows by Gaussian elimination with partial pivoting,
// B = U U_rows^{-1}, then swaps while some |B_ij| > 1.05.  Then the
// index set of the next step and, right to left, core k of the cross TT.
//   dir 0: rows a * n_k + i -> I_{k+1}[j] = (I_k[a], i), cnt I_{k+1} = r
//   dir 1: rows i * bcap + b -> J_k[j] = (i, J_{k+1}[b]), cnt J_k = r, and
//          core k of Y (r, n_k, |J_{k+1}|) = B^T
// One workgroup per filter.
// frozen (dir 1 only): the rows are the saved rowsk of bond k and the rank
// the saved count of J_k (a cross replayed on the index sets of another).
__global__ void __launch_bounds__(256) cross_maxvol_kernel(const DevTT* __restrict__ U, const CrossState* __restrict__ cs,
                                                           const DevTT* __restrict__ Y, int k, int nk, int dir, int m,
                                                           int bcap, int want, int frozen = 0) {
  const int f = blockIdx.x;
  const DevTT& u = U[f];
  const CrossState& S = cs[f];
  const int ru = u.ranks[1];                                              // the rounding's basis of M's range
  const int r = frozen ? S.cnt[TT_MAXD + 1 + k] : max(ru, min(want, m));  // its width after completion
  const int r0 = min(ru, r);                                              // basis columns kept
  const double* u0 = core_ptr<double>(u, 0);
  double* Uc = S.work;                                  // m x r, the (completed) basis
  double* W = Uc + (long long)m * CROSS_RMAX;           // m x r, elimination copy
  double* Bm = W + (long long)m * CROSS_RMAX;           // m x r
  double* G = Bm + (long long)m * CROSS_RMAX;           // r x 2r
  int* rows = S.rows;
  __shared__ double sv[256];
  __shared__ int si[256];
  __shared__ int s_piv;
  __shared__ int s_used[CROSS_RMAX];
  __shared__ int s_seed[CROSS_RMAX];
  __shared__ double s_w[CROSS_RMAX];
  __shared__ double red[8];
  // rows already taken (a completion seed, or a pivot of the elimination),
  // flagged when the fibre matrix fits: a constant-time test per row
  constexpr int FLAG_MAX = 16384;
  __shared__ unsigned char s_flag[FLAG_MAX];
  const int tid = threadIdx.x;
  const bool use_flag = m <= FLAG_MAX;
  if (use_flag)
    for (int q = tid; q < m; q += blockDim.x) s_flag[q] = 0;
  // rows of existing index tuples (the others are zero padding)
  const int cvalid = dir == 0 ? S.cnt[k] : S.cnt[TT_MAXD + 1 + k + 1];
  // (32-bit index arithmetic: m r stays far below 2^31)
  for (int e = tid; e < m * r; e += blockDim.x) {
    const int i = e / r, c = e - (e / r) * r;
    Uc[e] = c < r0 ? u0[(long long)i * ru + c] : 0.0;
  }
  __syncthreads();
  // A rank-deficient fibre matrix leaves fewer basis vectors than rows to
  // pick: complete the basis with the unit vectors of the valid rows of
  // least leverage, orthogonalised twice (the pivots then still explore
  // the whole target rank).  Each row's leverage over the columns so far is
  // kept as a running sum (W is free until the elimination), added in the
  // columns' order.
  if (!frozen && r0 < r) {
    for (int q = tid; q < m; q += blockDim.x) {
      double lev = 0.0;
      for (int u2 = 0; u2 < r0; ++u2) lev += Uc[(long long)q * r + u2] * Uc[(long long)q * r + u2];
      W[q] = lev;
    }
    __syncthreads();
  }
  for (int c = r0; c < r; ++c) {
    int p;
    if (frozen) {
      p = S.seedk[k * CROSS_RMAX + (c - r0)];  // the completion of the replayed cross
    } else {
      double best = 1e300;
      int bi = m;
      for (int q = tid; q < m; q += blockDim.x) {
        const bool ok = dir == 0 ? (q / nk) < cvalid : (q % bcap) < cvalid;
        bool seeded = false;
        if (use_flag)
          seeded = s_flag[q] != 0;
        else
          for (int u2 = 0; u2 < c - r0; ++u2) seeded = seeded || s_seed[u2] == q;
        if (!ok || seeded) continue;
        const double lev = W[q];
        if (lev < best) {
          best = lev;
          bi = q;
        }
      }
      sv[tid] = best;
      si[tid] = bi;
      __syncthreads();
      for (int o = 128; o > 0; o >>= 1) {
        if (tid < o && (sv[tid + o] < sv[tid] || (sv[tid + o] == sv[tid] && si[tid + o] < si[tid]))) {
          sv[tid] = sv[tid + o];
          si[tid] = si[tid + o];
        }
        __syncthreads();
      }
      p = si[0];
      __syncthreads();
    }
    if (tid == 0) s_seed[c - r0] = p;
    if (p >= m) break;  // no valid row left (cannot happen when the target fits the valid rows)
    if (use_flag && tid == 0) s_flag[p] = 1;
    for (int i = tid; i < m; i += blockDim.x) {
      double v = (i == p) ? 1.0 : 0.0;
      for (int q = 0; q < c; ++q) v -= Uc[(long long)i * r + q] * Uc[(long long)p * r + q];
      Uc[(long long)i * r + c] = v;
    }
    __syncthreads();
    // the c projections at once: a wavefront per basis column q, each summed
    // over the rows by its own lanes (no workgroup reduction per column)
    {
      const int lane = tid & 63, nw = blockDim.x >> 6;
      for (int q = tid >> 6; q < c; q += nw) {
        double part = 0.0;
        for (int i = lane; i < m; i += 64) part += Uc[(long long)i * r + q] * Uc[(long long)i * r + c];
        part = wave_sum(part);
        if (lane == 0) s_w[q] = part;
      }
    }
    __syncthreads();
    double nn = 0.0;
    for (int i = tid; i < m; i += blockDim.x) {
      double v = Uc[(long long)i * r + c];
      for (int q = 0; q < c; ++q) v -= Uc[(long long)i * r + q] * s_w[q];
      Uc[(long long)i * r + c] = v;
      nn += v * v;
    }
    const double nrm = sqrt(block_sum(nn, red));
    for (int i = tid; i < m; i += blockDim.x) {
      Uc[(long long)i * r + c] /= nrm;
      if (!frozen) W[i] += Uc[(long long)i * r + c] * Uc[(long long)i * r + c];
    }
    __syncthreads();
  }
  const double* uc = Uc;
  for (int e = tid; e < m * r; e += blockDim.x) W[e] = uc[e];
  if (frozen)
    for (int j = tid; j < r; j += blockDim.x) s_used[j] = S.rowsk[k * CROSS_RMAX + j];
  if (use_flag)
    for (int q = tid; q < m; q += blockDim.x) s_flag[q] = 0;  // from now on: pivot rows
  __syncthreads();
  // Gaussian elimination with partial pivoting for the initial rows
  for (int j = 0; j < (frozen ? 0 : r); ++j) {
    double best = -1.0;
    int bi = 0;
    for (int i = tid; i < m; i += blockDim.x) {
      bool used = false;
      if (use_flag)
        used = s_flag[i] != 0;
      else
        for (int q = 0; q < j; ++q) used = used || (s_used[q] == i);
      const double v = used ? -1.0 : fabs(W[(long long)i * r + j]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o && (sv[tid + o] > sv[tid] || (sv[tid + o] == sv[tid] && si[tid + o] < si[tid]))) {
        sv[tid] = sv[tid + o];
        si[tid] = si[tid + o];
      }
      __syncthreads();
    }
    if (tid == 0) {
      s_piv = si[0];
      s_used[j] = si[0];
      if (use_flag) s_flag[si[0]] = 1;
    }
    __syncthreads();
    const int p = s_piv;
    const double pv = W[(long long)p * r + j];
    if (pv != 0.0 && use_flag) {
      // the rows' multipliers first (Bm is free until B is formed), then the
      // update with consecutive threads on consecutive columns of a row
      for (int i = tid; i < m; i += blockDim.x) Bm[i] = s_flag[i] ? 0.0 : W[(long long)i * r + j] / pv;
      __syncthreads();
      const int w = r - j;
      for (int e = tid; e < m * w; e += blockDim.x) {
        const int i = e / w, c = j + (e - (e / w) * w);
        if (s_flag[i]) continue;
        W[(long long)i * r + c] -= Bm[i] * W[(long long)p * r + c];
      }
    } else if (pv != 0.0) {
      for (int i = tid; i < m; i += blockDim.x) {
        bool used = false;
        for (int q = 0; q <= j; ++q) used = used || (s_used[q] == i);
        if (used) continue;
        const double fct = W[(long long)i * r + j] / pv;
        for (int c = j; c < r; ++c) W[(long long)i * r + c] -= fct * W[(long long)p * r + c];
      }
    }
    __syncthreads();
  }
  // G = [U_rows | I], Gauss-Jordan with partial pivoting -> U_rows^{-1}
  for (int e = tid; e < r * 2 * r; e += blockDim.x) {
    const int i = e / (2 * r), c = e % (2 * r);
    G[e] = c < r ? uc[(long long)s_used[i] * r + c] : (c - r == i ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int j = 0; j < r; ++j) {
    // partial pivot: the first row of largest |G(i, j)|, i >= j, found by
    // the first wavefront's lanes and a shuffle reduction
    if (tid < 64) {
      double bv = -1.0;
      int p = r;
      for (int i = j + tid; i < r; i += 64) {
        const double v = fabs(G[i * 2 * r + j]);
        if (v > bv) {
          bv = v;
          p = i;
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(bv, o, 64);
        const int oi = __shfl_xor(p, o, 64);
        if (ov > bv || (ov == bv && oi < p)) {
          bv = ov;
          p = oi;
        }
      }
      if (tid == 0) s_piv = p < r ? p : j;  // (no comparable entry: keep row j, as a serial scan would)
    }
    __syncthreads();
    const int p = s_piv;
    if (p != j)
      for (int c = tid; c < 2 * r; c += blockDim.x) {
        const double t = G[j * 2 * r + c];
        G[j * 2 * r + c] = G[p * 2 * r + c];
        G[p * 2 * r + c] = t;
      }
    __syncthreads();
    const double pv = G[j * 2 * r + j];
    __syncthreads();
    for (int c = tid; c < 2 * r; c += blockDim.x) G[j * 2 * r + c] /= pv;
    __syncthreads();
    for (int e = tid; e < r * 2 * r; e += blockDim.x) {
      const int i = e / (2 * r), c = e % (2 * r);
      if (i != j && c != j) G[e] -= G[i * 2 * r + j] * G[j * 2 * r + c];
    }
    __syncthreads();
    for (int i = tid; i < r; i += blockDim.x)
      if (i != j) G[i * 2 * r + j] = 0.0;
    __syncthreads();
  }
  // B = U inv(U_rows), the inverse staged in LDS
  {
    __shared__ double s_ginv[CROSS_RMAX * CROSS_RMAX];
    for (int e = tid; e < r * r; e += blockDim.x) {
      const int q = e / r, c = e - (e / r) * r;
      s_ginv[e] = G[q * 2 * r + r + c];
    }
    __syncthreads();
    for (int e = tid; e < m * r; e += blockDim.x) {
      const int i = e / r, c = e - (e / r) * r;
      double s = 0.0;
      for (int q = 0; q < r; ++q) s += uc[(long long)i * r + q] * s_ginv[q * r + c];
      Bm[e] = s;
    }
  }
  for (int j = tid; j < r; j += blockDim.x) rows[j] = s_used[j];
  __syncthreads();
  // swaps while some |B_ij| > 1.05 (each multiplies the volume by |B_ij|);
  // each update pass also finds the next candidate (same order of visits as
  // a separate search)
  double best = -1.0;
  int bi = 0;
  if (!frozen)
    for (int e = tid; e < m * r; e += blockDim.x) {
      const double v = fabs(Bm[e]);
      if (v > best) {
        best = v;
        bi = e;
      }
    }
  for (int it = 0; it < (frozen ? 0 : 8 * CROSS_RMAX); ++it) {
    sv[tid] = best;
    si[tid] = bi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (tid < o && (sv[tid + o] > sv[tid] || (sv[tid + o] == sv[tid] && si[tid + o] < si[tid]))) {
        sv[tid] = sv[tid + o];
        si[tid] = si[tid + o];
      }
      __syncthreads();
    }
    const double bv = sv[0];
    const int be = si[0];
    __syncthreads();
    if (bv <= 1.05) break;
    const int i = be / r, j = be % r;
    const double bij = Bm[be];
    // row i of B and column j of B before the update
    // (W is free after the pivots: r + m <= 2 m of its m x 64 entries)
    for (int c = tid; c < r; c += blockDim.x) W[c] = Bm[(long long)i * r + c] - (c == j ? 1.0 : 0.0);
    for (int q = tid; q < m; q += blockDim.x) W[r + q] = Bm[(long long)q * r + j];
    __syncthreads();
    best = -1.0;
    bi = 0;
    for (int e = tid; e < m * r; e += blockDim.x) {
      const int q = e / r, c = e - (e / r) * r;
      Bm[e] -= W[r + q] * W[c] / bij;
      const double v = fabs(Bm[e]);
      if (v > best) {
        best = v;
        bi = e;
      }
    }
    if (tid == 0) rows[j] = i;
    __syncthreads();
  }
  // the next index set
  if (dir == 0) {
    for (int j = tid; j < r; j += blockDim.x) {
      const int a = rows[j] / nk, i = rows[j] % nk;
      const int* src = S.iset + ((long long)k * CROSS_RMAX + a) * TT_MAXD;
      int* dst = S.iset + ((long long)(k + 1) * CROSS_RMAX + j) * TT_MAXD;
      for (int l = 0; l < k; ++l) dst[l] = src[l];
      dst[k] = i;
    }
    if (tid == 0) S.cnt[k + 1] = r;
  } else {
    // J_k tuples: written to a staging area first (J_{k+1} is read), then copied
    int* stage = reinterpret_cast<int*>(W);
    const int cj = S.cnt[TT_MAXD + 1 + k + 1];
    const int d = Y[f].d;
    for (int j = tid; j < r; j += blockDim.x) {
      const int i = rows[j] / bcap, b = rows[j] % bcap;
      const int* src = S.jset + ((long long)(k + 1) * CROSS_RMAX + b) * TT_MAXD;
      int* dst = stage + j * TT_MAXD;
      dst[0] = i;
      for (int l = 1; l < d - k; ++l) dst[l] = src[l - 1];
    }
    __syncthreads();
    for (int e = tid; e < r * TT_MAXD; e += blockDim.x)
      S.jset[((long long)k * CROSS_RMAX) * TT_MAXD + e] = stage[e];
    // core k of Y: (r, n_k, cj), entry (j, i, b) = B[(i * R + b), j]
    const DevTT& y = Y[f];
    double* yc = core_ptr<double>(y, k);
    const int nkcj = nk * cj;
    for (int e = tid; e < r * nkcj; e += blockDim.x) {
      const int j = e / nkcj;
      const int rem = e - j * nkcj;
      const int i = rem / cj, b = rem - (rem / cj) * cj;
      yc[e] = Bm[(long long)(i * bcap + b) * r + j];
    }
    for (int j = tid; j < r; j += blockDim.x) S.rowsk[k * CROSS_RMAX + j] = rows[j];
    for (int c = tid; c < r - r0; c += blockDim.x) S.seedk[k * CROSS_RMAX + c] = s_seed[c];
    if (tid == 0) S.ruk[k] = r0;
    if (tid == 0) {
      S.cnt[TT_MAXD + 1 + k] = r;
      y.ranks[k] = r;
      y.ranks[k + 1] = cj;
    }
  }
}

// J sets for a new target rank: J_k keeps its tuples and gets new, distinct
// ones up to the target (<= the bond's bound) from a counter-based generator
// (splitmix64 of the filter, bond, slot, attempt and axis); the first tuple
// of a fresh set is the middle point; when the target covers every tuple of
// the tail axes they are enumerated.  The count of I_0 and J_d is one.
__device__ inline unsigned long long cross_mix(unsigned long long x) {
  x += 0x9E3779B97F4A7C15ULL;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

__global__ void cross_extend_kernel(const CrossState* __restrict__ cs, const int* __restrict__ n, int d,
                                    const int* __restrict__ target, unsigned long long seed,
                                    const int* __restrict__ ids) {
  const int f = blockIdx.x;
  const CrossState& S = cs[f];
  const unsigned long long id = (unsigned long long)ids[f];  // the generator's stream of this function
  for (int k = threadIdx.x + 1; k < d; k += blockDim.x) {
    const int have = S.cnt[TT_MAXD + 1 + k];
    const int want = target[k];
    long long tail = 1;
    for (int l = k; l < d; ++l) tail = min(tail * n[l], (long long)1 << 20);
    if (want >= tail) {
      // every tuple of the tail axes (mixed radix, last axis fastest)
      for (int a = 0; a < want; ++a) {
        int* t = S.jset + ((long long)k * CROSS_RMAX + a) * TT_MAXD;
        int rem = a;
        for (int l = d - 1; l >= k; --l) {
          t[l - k] = rem % n[l];
          rem /= n[l];
        }
      }
    } else {
      for (int a = have; a < want; ++a) {
        int* t = S.jset + ((long long)k * CROSS_RMAX + a) * TT_MAXD;
        for (int attempt = 0; attempt < 64; ++attempt) {
          for (int l = k; l < d; ++l) {
            const unsigned long long h = cross_mix(
                seed ^ cross_mix((id << 44) ^ ((unsigned long long)k << 36) ^
                                 ((unsigned long long)a << 24) ^ ((unsigned long long)attempt << 8) ^
                                 (unsigned long long)l));
            t[l - k] = (a == 0 && attempt == 0) ? n[l] / 2 : (int)(h % (unsigned long long)n[l]);
          }
          bool dup = false;  // distinct tuples only (a repeated column adds no rank)
          for (int b = 0; b < a && !dup; ++b) {
            const int* u = S.jset + ((long long)k * CROSS_RMAX + b) * TT_MAXD;
            bool same = true;
            for (int l = 0; l < d - k && same; ++l) same = u[l] == t[l];
            dup = same;
          }
          if (!dup) break;
        }
      }
    }
    if (want > have) S.cnt[TT_MAXD + 1 + k] = want;
  }
  if (threadIdx.x == 0) {
    S.cnt[0] = 1;
    S.cnt[TT_MAXD + 1 + d] = 1;
  }
}

}  // namespace ttg

namespace ttg {

// ranks [1, ruk[k], 1] of the two-core fibre train of bond k (replay)
__global__ void cross_ru_kernel(const CrossState* __restrict__ cs, int nf, int k, int* __restrict__ out) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  out[f * 3] = 1;
  out[f * 3 + 1] = max(1, cs[f].ruk[k]);
  out[f * 3 + 2] = 1;
}

// the cross TT's log-scale and status before its rounding
__global__ void cross_y_init_kernel(const DevTT* __restrict__ Y, int nf) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  *Y[f].log_scale = 0.0;
  *Y[f].status = 0;
  Y[f].ranks[0] = 1;
  Y[f].ranks[Y[f].d] = 1;
}

// status words of the rounding's destination cleared (it ORs the source's in)
__global__ void cross_clear_status_kernel(const DevTT* __restrict__ t, int nf) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f < nf) *t[f].status = 0;
}

// out.log_scale += src.log_scale (the interpolant's values leave it out)
__global__ void cross_add_log_scale_kernel(const DevTT* __restrict__ src, const DevTT* __restrict__ out, int nf) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  *out[f].log_scale += *src[f].log_scale;
  *out[f].status |= *src[f].status;
}

struct CrossPlan {
  int B = 0, d = 0, mmax = 0, rmax = 1;
  int n[TT_MAXD] = {0};
  long long bound[TT_MAXD + 1] = {0};
  std::vector<CrossState> cs;
  void* dfn = nullptr;
  CrossState* dcs = nullptr;
  int* dn = nullptr;
  int* dtarget = nullptr;
  int* dranks = nullptr;  // batch x (d+1) ranks read back after a level
  int* dids = nullptr;    // generator stream per function
  int* dru = nullptr;     // batch x 3 forced ranks of a fibre matrix's rounding (replay)
  DevTT* tab = nullptr;   // 2 * batch descriptors
  std::vector<tt_train> T2, T2r, Y, Z;
  void* rws = nullptr;
  size_t rws_bytes = 0;
};

static tt_train cross_train(Arena& ar, int d, const int* n, const int* cap) {
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

// the two-core train of a fibre matrix with m rows and R columns
static tt_train cross_t2_view(const tt_train& t, int m, int R) {
  tt_train v = t;
  v.n[0] = m;
  v.n[1] = R;
  v.cap[0] = 1;
  v.cap[1] = R;
  v.cap[2] = 1;
  return v;
}

// layout of a cross over mode sizes n[d] with ranks up to max_rank (capped
// so that a fibre matrix has at most 4096 rows), for the outputs out
static tt_status cross_plan(int batch, int d, const int* n, int max_rank, size_t fn_bytes, const tt_train* out,
                            Arena& ar, CrossPlan& p) {
  p.B = batch;
  p.d = d;
  int nmax = 1;
  for (int k = 0; k < d; ++k) {
    if (n[k] < 1 || n[k] > 4096) {
      set_error("TT-cross: mode size %d out of range [1, 4096]", n[k]);
      return TT_ERR_SHAPE;
    }
    p.n[k] = n[k];
    nmax = std::max(nmax, n[k]);
  }
  p.rmax = std::max(1, std::min({max_rank, CROSS_RMAX, 4096 / nmax}));
  for (int j = 0; j <= d; ++j) {
    long long lp = 1, rp = 1;
    for (int k = 0; k < j; ++k) lp = std::min<long long>(lp * n[k], 1 << 20);
    for (int k = j; k < d; ++k) rp = std::min<long long>(rp * n[k], 1 << 20);
    p.bound[j] = std::min(lp, rp);
  }
  p.mmax = p.rmax * nmax;
  p.cs.resize(batch);
  p.dfn = ar.take<char>((size_t)batch * fn_bytes);
  p.dcs = ar.take<CrossState>(batch);
  p.dn = ar.take<int>(TT_MAXD);
  p.dtarget = ar.take<int>(TT_MAXD + 1);
  p.dranks = ar.take<int>((size_t)batch * (TT_MAXD + 1));
  p.dids = ar.take<int>(batch);
  p.dru = ar.take<int>((size_t)batch * 3);
  p.tab = ar.take<DevTT>((size_t)2 * batch);
  const int n2[2] = {p.mmax, p.rmax};
  const int c2[3] = {1, p.rmax, 1};
  int ycap[TT_MAXD + 1];
  for (int j = 0; j <= d; ++j) ycap[j] = (j == 0 || j == d) ? 1 : (int)std::min<long long>(p.rmax, p.bound[j]);
  p.T2.resize(batch);
  p.T2r.resize(batch);
  p.Y.resize(batch);
  p.Z.resize(batch);
  const bool f32 = out[0].dtype == TT_F32;
  for (int b = 0; b < batch; ++b) {
    CrossState& s = p.cs[b];
    int* blob = ar.take<int>((size_t)CROSS_STATE_INTS);
    s.iset = blob;
    s.jset = blob + CROSS_SET_INTS;
    s.cnt = blob + 2 * CROSS_SET_INTS;
    s.rowsk = s.cnt + 2 * (TT_MAXD + 1);
    s.ruk = s.rowsk + (TT_MAXD + 1) * CROSS_RMAX;
    s.seedk = s.ruk + (TT_MAXD + 1);
    s.tgt = s.seedk + (TT_MAXD + 1) * CROSS_RMAX;
    s.work = ar.take<double>((size_t)3 * p.mmax * CROSS_RMAX + 2 * CROSS_RMAX * CROSS_RMAX);
    s.rows = ar.take<int>(CROSS_RMAX);
    p.T2[b] = cross_train(ar, 2, n2, c2);
    p.T2r[b] = cross_train(ar, 2, n2, c2);
    p.Y[b] = cross_train(ar, d, n, ycap);
    if (f32) p.Z[b] = cross_train(ar, d, n, out[b].cap);
  }
  size_t need = tt_round_workspace(batch, p.T2.data(), p.T2r.data());
  need = std::max(need, tt_round_workspace(batch, p.Y.data(), f32 ? p.Z.data() : out));
  if (need == 0) {
    set_error("TT-cross: rounding workspace query failed");
    return TT_ERR_SHAPE;
  }
  p.rws_bytes = need + 256;
  p.rws = ar.take<char>(p.rws_bytes);
  return TT_OK;
}

static tt_status cross_upload_pair(CrossPlan& p, const std::vector<tt_train>& a, const std::vector<tt_train>& b,
                                   hipStream_t st) {
  std::vector<DevTT> v(2 * p.B);
  for (int f = 0; f < p.B; ++f) {
    v[f] = make_dev(a[f]);
    v[p.B + f] = make_dev(b[f]);
  }
  return upload(p.tab, v, st);
}

// The cross of the functions fns[b] (one per output), rounded at tol into
// out (capacities cap bound the ranks).  Synchronises after each rank level.
// ids (empty: 0, 1, ...) name each function's stream of random tuples;
// forced (device, nullable) replaces the final rounding's rank rule by the
// ranks forced[b * fstride + j] (rank replay).
// state_save (device, nullable): each function's final index sets, row
// choices and targets (CROSS_STATE_INTS ints per function) for cross_frozen.
template <typename Fn>
static tt_status cross_run(CrossPlan& p, const std::vector<Fn>& fns, double tol, int max_rank, const tt_train* out,
                           hipStream_t st, const std::vector<int>& ids = {}, const int* forced = nullptr,
                           long long fstride = 0, int* state_save = nullptr) {
  const int batch = p.B, d = p.d;
  Fn* dfn = reinterpret_cast<Fn*>(p.dfn);
  TT_TRY(upload(dfn, fns, st));
  TT_TRY(upload(p.dcs, p.cs, st));
  {
    std::vector<int> iv(batch);
    for (int b = 0; b < batch; ++b) iv[b] = ids.empty() ? b : ids[b];
    TT_TRY(upload(p.dids, iv, st));
  }
  {
    std::vector<int> nv(p.n, p.n + TT_MAXD);
    TT_TRY(upload(p.dn, nv, st));
  }
  for (int b = 0; b < batch; ++b) HIP_TRY(hipMemsetAsync(p.cs[b].cnt, 0, 2 * (TT_MAXD + 1) * sizeof(int), st), "cnt");
  int outcap = 1;
  for (int b = 0; b < batch; ++b)
    for (int j = 0; j <= d; ++j) outcap = std::max(outcap, out[b].cap[j]);
  const bool f32 = out[0].dtype == TT_F32;
  const double eps_rank = 1e-16;  // a basis of the fibre matrix's range (exact rank deficiency only)
  const int rtop = std::min(max_rank, p.rmax);
  int r = std::min(8, rtop);
  std::vector<int> prev_level, last_target;
  for (int level = 0;; ++level) {
    std::vector<int> target(TT_MAXD + 1, 1);
    for (int k = 1; k < d; ++k) target[k] = (int)std::min<long long>(r, p.bound[k]);
    last_target = target;
    TT_TRY(upload(p.dtarget, target, st));
    hipLaunchKernelGGL(cross_extend_kernel, dim3(batch), dim3(64), 0, st, p.dcs, p.dn, d, p.dtarget,
                       0x5eedULL + 977ULL * (unsigned long long)level, p.dids);
    TTG_LAUNCH_CHECK("cross_extend_kernel");
    std::vector<int> prev_got;
    bool slack = false;
    for (int sweep = 0; sweep < 6; ++sweep) {
      for (int k = 0; k + 1 < d; ++k) {  // left to right: the row sets I
        const int acap = k == 0 ? 1 : target[k], bcap = target[k + 1], m = acap * p.n[k];
        std::vector<tt_train> t2(batch), t2r(batch);
        for (int b = 0; b < batch; ++b) {
          t2[b] = cross_t2_view(p.T2[b], m, bcap);
          t2r[b] = cross_t2_view(p.T2r[b], m, bcap);
        }
        TT_TRY(cross_upload_pair(p, t2, t2r, st));
        hipLaunchKernelGGL((cross_fibre_kernel<Fn>), dim3(std::max(1, std::min(1024, cdiv((long long)m * bcap, 256))),
                                                          batch),
                           dim3(256), 0, st, dfn, p.dcs, p.tab, d, k, p.n[k], 0, m, bcap, bcap);
        TTG_LAUNCH_CHECK("cross_fibre_kernel");
        TT_TRY(tt_round(batch, t2.data(), t2r.data(), eps_rank, bcap, p.rws, p.rws_bytes, st));
        TT_TRY(cross_upload_pair(p, t2r, p.Y, st));
        hipLaunchKernelGGL(cross_maxvol_kernel, dim3(batch), dim3(256), 0, st, p.tab, p.dcs, p.tab + batch, k, p.n[k],
                           0, m, bcap, bcap);
        TTG_LAUNCH_CHECK("cross_maxvol_kernel");
      }
      for (int k = d - 1; k >= 1; --k) {  // right to left: the column sets J and the cores
        const int acap = target[k], bcap = k == d - 1 ? 1 : target[k + 1], m = p.n[k] * bcap;
        std::vector<tt_train> t2(batch), t2r(batch);
        for (int b = 0; b < batch; ++b) {
          t2[b] = cross_t2_view(p.T2[b], m, acap);
          t2r[b] = cross_t2_view(p.T2r[b], m, acap);
        }
        TT_TRY(cross_upload_pair(p, t2, t2r, st));
        hipLaunchKernelGGL((cross_fibre_kernel<Fn>), dim3(std::max(1, std::min(1024, cdiv((long long)m * acap, 256))),
                                                          batch),
                           dim3(256), 0, st, dfn, p.dcs, p.tab, d, k, p.n[k], 1, m, acap, bcap);
        TTG_LAUNCH_CHECK("cross_fibre_kernel");
        TT_TRY(tt_round(batch, t2.data(), t2r.data(), eps_rank, acap, p.rws, p.rws_bytes, st));
        TT_TRY(cross_upload_pair(p, t2r, p.Y, st));
        hipLaunchKernelGGL(cross_maxvol_kernel, dim3(batch), dim3(256), 0, st, p.tab, p.dcs, p.tab + batch, k, p.n[k],
                           1, m, bcap, acap);
        TTG_LAUNCH_CHECK("cross_maxvol_kernel");
      }
      TT_TRY(cross_upload_pair(p, p.Y, p.Y, st));
      hipLaunchKernelGGL((cross_first_core_kernel<Fn>), dim3(std::max(1, cdiv(p.n[0] * target[1], 256)), batch),
                         dim3(256), 0, st, dfn, p.dcs, p.tab, d, p.n[0]);
      TTG_LAUNCH_CHECK("cross_first_core_kernel");
      if (sweep == 0) continue;
      TT_TRY(cross_upload_pair(p, p.Y, p.Y, st));
      hipLaunchKernelGGL(cross_y_init_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, p.tab, batch);
      TTG_LAUNCH_CHECK("cross_y_init_kernel");
      const std::vector<tt_train> dst = f32 ? p.Z : std::vector<tt_train>(out, out + batch);
      TT_TRY(cross_upload_pair(p, dst, dst, st));
      hipLaunchKernelGGL(cross_clear_status_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, p.tab, batch);
      TTG_LAUNCH_CHECK("cross_clear_status_kernel");
      TT_TRY(tt_round(batch, p.Y.data(), dst.data(), tol, outcap, p.rws, p.rws_bytes, st));
      // ranks of the rounded result against the ranks the cross used
      {
        std::vector<DevTT> v(batch);
        for (int b = 0; b < batch; ++b) v[b] = make_dev(dst[b]);
        TT_TRY(upload(p.tab, v, st));
        hipLaunchKernelGGL(record_ranks_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, p.tab, batch, p.dranks,
                           (long long)(TT_MAXD + 1));
        TTG_LAUNCH_CHECK("record_ranks_kernel");
      }
      std::vector<int> got((size_t)batch * (TT_MAXD + 1));
      HIP_TRY(hipMemcpyAsync(got.data(), p.dranks, got.size() * sizeof(int), hipMemcpyDeviceToHost, st), "ranks");
      HIP_TRY(hipStreamSynchronize(st), "cross sync");
      slack = true;
      for (int b = 0; b < batch; ++b)
        for (int k = 1; k < d; ++k) {
          const int rr = got[(size_t)b * (TT_MAXD + 1) + k];
          if (!(rr + 2 <= target[k] || target[k] >= p.bound[k])) slack = false;
        }
      // more sweeps at this rank while the rounded ranks still move
      const bool stable = got == prev_got;
      prev_got = got;
      if (stable || !slack) break;
    }
    // done when the ranks have room at this level and did not move from the
    // previous level's (a doubled rank found nothing more)
    if ((slack && prev_got == prev_level) || r >= rtop) break;
    prev_level = prev_got;
    r = std::min(2 * r, rtop);
  }
  if (state_save)
    for (int b = 0; b < batch; ++b) {
      TT_TRY(upload(p.cs[b].tgt, last_target, st));
      HIP_TRY(hipMemcpyAsync(state_save + (long long)b * CROSS_STATE_INTS, p.cs[b].iset,
                             (size_t)CROSS_STATE_INTS * sizeof(int), hipMemcpyDeviceToDevice, st),
              "cross state save");
    }
  if (forced) {  // the last interpolant again, at the given ranks
    const std::vector<tt_train> dst = f32 ? p.Z : std::vector<tt_train>(out, out + batch);
    TT_TRY(cross_upload_pair(p, dst, dst, st));
    hipLaunchKernelGGL(cross_clear_status_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, p.tab, batch);
    TTG_LAUNCH_CHECK("cross_clear_status_kernel");
    TT_TRY(round_forced(batch, p.Y.data(), dst.data(), forced, fstride, p.rws, p.rws_bytes, st));
  }
  if (f32) {
    std::vector<DevTT> vz(batch), vo(batch);
    for (int b = 0; b < batch; ++b) {
      vz[b] = make_dev(p.Z[b]);
      vo[b] = make_dev(out[b]);
    }
    TT_TRY(upload(p.tab, vz, st));
    TT_TRY(upload(p.tab + batch, vo, st));
    hipLaunchKernelGGL((convert_tt_kernel<float>), dim3(64, batch), dim3(256), 0, st, p.tab, p.tab + batch);
    TTG_LAUNCH_CHECK("convert_tt_kernel");
  }
  return TT_OK;
}

// The cross of fns[b] replayed on the index sets and row choices of a
// finished cross (saved by cross_run at state_in + src[b] *
// CROSS_STATE_INTS): one right-to-left pass, each core in interpolation form
// B = U U_rows^{-1} with the saved rows, then the rounding into out (FP64) at
// the ranks forced (device, stride fstride) or, when null, at tol.  A small
// change of the function changes the interpolant smoothly: the index sets
// do not move.  Synchronous.
template <typename Fn>
static tt_status cross_frozen(CrossPlan& p, const std::vector<Fn>& fns, const int* state_in,
                              const std::vector<int>& src, double tol, const int* forced, long long fstride,
                              const tt_train* out, hipStream_t st) {
  const int batch = p.B, d = p.d;
  if (out[0].dtype != TT_F64) {
    set_error("TT-cross replay: FP64 output only");
    return TT_ERR_ARG;
  }
  Fn* dfn = reinterpret_cast<Fn*>(p.dfn);
  TT_TRY(upload(dfn, fns, st));
  TT_TRY(upload(p.dcs, p.cs, st));
  for (int b = 0; b < batch; ++b)
    HIP_TRY(hipMemcpyAsync(p.cs[b].iset, state_in + (long long)src[b] * CROSS_STATE_INTS,
                           (size_t)CROSS_STATE_INTS * sizeof(int), hipMemcpyDeviceToDevice, st),
            "cross state load");
  std::vector<int> target(TT_MAXD + 1);
  HIP_TRY(hipMemcpyAsync(target.data(), p.cs[0].tgt, (TT_MAXD + 1) * sizeof(int), hipMemcpyDeviceToHost, st),
          "cross targets");
  HIP_TRY(hipStreamSynchronize(st), "cross targets sync");
  for (int k = 1; k < d; ++k)
    if (target[k] < 1 || target[k] > p.rmax) {
      set_error("TT-cross replay: saved rank target %d out of range", target[k]);
      return TT_ERR_SHAPE;
    }
  for (int k = d - 1; k >= 1; --k) {
    const int acap = target[k], bcap = k == d - 1 ? 1 : target[k + 1], m = p.n[k] * bcap;
    std::vector<tt_train> t2(batch), t2r(batch);
    for (int b = 0; b < batch; ++b) {
      t2[b] = cross_t2_view(p.T2[b], m, acap);
      t2r[b] = cross_t2_view(p.T2r[b], m, acap);
    }
    TT_TRY(cross_upload_pair(p, t2, t2r, st));
    hipLaunchKernelGGL((cross_fibre_kernel<Fn>), dim3(std::max(1, std::min(1024, cdiv((long long)m * acap, 256))),
                                                      batch),
                       dim3(256), 0, st, dfn, p.dcs, p.tab, d, k, p.n[k], 1, m, acap, bcap);
    TTG_LAUNCH_CHECK("cross_fibre_kernel");
    // the basis at the replayed cross's rank (not at the rank rule, whose
    // decision at the round-off level may differ for a nearby function)
    hipLaunchKernelGGL(cross_ru_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, p.dcs, batch, k, p.dru);
    TTG_LAUNCH_CHECK("cross_ru_kernel");
    TT_TRY(round_forced(batch, t2.data(), t2r.data(), p.dru, 3, p.rws, p.rws_bytes, st));
    TT_TRY(cross_upload_pair(p, t2r, p.Y, st));
    hipLaunchKernelGGL(cross_maxvol_kernel, dim3(batch), dim3(256), 0, st, p.tab, p.dcs, p.tab + batch, k, p.n[k], 1,
                       m, bcap, acap, 1);
    TTG_LAUNCH_CHECK("cross_maxvol_kernel");
  }
  TT_TRY(cross_upload_pair(p, p.Y, p.Y, st));
  hipLaunchKernelGGL((cross_first_core_kernel<Fn>), dim3(std::max(1, cdiv(p.n[0] * target[1], 256)), batch),
                     dim3(256), 0, st, dfn, p.dcs, p.tab, d, p.n[0]);
  TTG_LAUNCH_CHECK("cross_first_core_kernel");
  hipLaunchKernelGGL(cross_y_init_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, p.tab, batch);
  TTG_LAUNCH_CHECK("cross_y_init_kernel");
  const std::vector<tt_train> dst(out, out + batch);
  TT_TRY(cross_upload_pair(p, dst, dst, st));
  hipLaunchKernelGGL(cross_clear_status_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, p.tab, batch);
  TTG_LAUNCH_CHECK("cross_clear_status_kernel");
  if (forced) {
    TT_TRY(round_forced(batch, p.Y.data(), dst.data(), forced, fstride, p.rws, p.rws_bytes, st));
  } else {
    int outcap = 1;
    for (int b = 0; b < batch; ++b)
      for (int j = 0; j <= d; ++j) outcap = std::max(outcap, out[b].cap[j]);
    TT_TRY(tt_round(batch, p.Y.data(), dst.data(), tol, outcap, p.rws, p.rws_bytes, st));
  }
  HIP_TRY(hipStreamSynchronize(st), "cross replay sync");
  return TT_OK;
}

static tt_status kernel_cross_args(int32_t batch, const tt_grid* grids, const int32_t* halfwidths,
                                   const tt_train* out, int* n) {
  if (batch < 1 || !grids || !halfwidths || !out) {
    set_error("tt_kernel_build_cross: null argument");
    return TT_ERR_ARG;
  }
  const int d = grids[0].d;
  if (d < 2 || d > TT_MAXD) {
    set_error("tt_kernel_build_cross: d = %d out of range [2, %d]", d, TT_MAXD);
    return TT_ERR_SHAPE;
  }
  for (int k = 0; k < d; ++k) {
    if (halfwidths[k] < 0 || 2 * halfwidths[k] + 1 > 4096) {
      set_error("tt_kernel_build_cross: halfwidths[%d] = %d out of range", k, halfwidths[k]);
      return TT_ERR_SHAPE;
    }
    n[k] = 2 * halfwidths[k] + 1;
  }
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_grid(&grids[b]));
    TT_TRY(check_train(&out[b], "out", out[0].dtype));
    if (grids[b].d != d || out[b].d != d) {
      set_error("tt_kernel_build_cross: d differs within the batch");
      return TT_ERR_SHAPE;
    }
    for (int k = 0; k < d; ++k)
      if (out[b].n[k] != n[k]) {
        set_error("tt_kernel_build_cross: out->n[%d] must be 2*h+1", k);
        return TT_ERR_SHAPE;
      }
  }
  return TT_OK;
}

}  // namespace ttg

namespace ttg {

// tt_kernel_build_cross, with the random-tuple streams ids, optional forced
// final ranks and the index sets saved (state_save) or replayed (state_load,
// function b on the saved state ids[b]; see cross_run and cross_frozen)
static tt_status kernel_cross_impl(int32_t batch, const tt_grid* grids, const double* q, const int32_t* halfwidths,
                                   double svd_tol, int32_t max_rank, const tt_train* out, void* ws, size_t ws_bytes,
                                   hipStream_t st, const std::vector<int>& ids = {},
                                   const int* forced = nullptr, long long fstride = 0, int* state_save = nullptr,
                                   const int* state_load = nullptr) {
  int n[TT_MAXD];
  TT_TRY(kernel_cross_args(batch, grids, halfwidths, out, n));
  if (!q || !ws || !(svd_tol > 0.0) || max_rank < 1 || max_rank > CROSS_RMAX) {
    set_error("tt_kernel_build_cross: bad arguments (need svd_tol > 0 and 1 <= max_rank <= %d)", CROSS_RMAX);
    return TT_ERR_ARG;
  }
  const int d = grids[0].d;
  Arena ar(ws, ws_bytes);
  CrossPlan p;
  TT_TRY(cross_plan(batch, d, n, CROSS_RMAX, sizeof(CrossKernelFn), out, ar, p));
  if (!ar.fits()) {
    set_error("tt_kernel_build_cross: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  std::vector<CrossKernelFn> fns(batch);
  for (int b = 0; b < batch; ++b) {
    CrossKernelFn& F = fns[b];
    memset(&F, 0, sizeof(F));
    F.d = d;
    double det = 0.0, logdelta = 0.0;
    if (!invert_spd(d, q + (size_t)b * d * d, F.lam, &det)) {
      set_error("tt_kernel_build_cross: Q is not positive definite (filter %d)", b);
      return TT_ERR_ARG;
    }
    for (int l = 0; l < d; ++l) {
      F.h[l] = halfwidths[l];
      F.dx[l] = (grids[b].hi[l] - grids[b].lo[l]) / (double)(grids[b].n[l] - 1);
      logdelta += std::log(F.dx[l]);
    }
    F.c = std::exp(-0.5 * d * std::log(2.0 * M_PI) - 0.5 * std::log(det) + logdelta);
  }
  if (state_load) {  // replay on saved index sets: function b on the state ids[b]
    std::vector<int> src(batch);
    for (int b = 0; b < batch; ++b) src[b] = ids.empty() ? b : ids[b];
    return cross_frozen(p, fns, state_load, src, svd_tol, forced, fstride, out, st);
  }
  return cross_run(p, fns, svd_tol, max_rank, out, st, ids, forced, fstride, state_save);
}

}  // namespace ttg

extern "C" {

size_t tt_kernel_build_cross_workspace(int32_t batch, const tt_grid* grids, const int32_t* halfwidths,
                                       const tt_train* out) {
  using namespace ttg;
  int n[TT_MAXD];
  if (kernel_cross_args(batch, grids, halfwidths, out, n) != TT_OK) return 0;
  Arena ar(nullptr, 0);
  CrossPlan p;
  if (cross_plan(batch, grids[0].d, n, CROSS_RMAX, sizeof(CrossKernelFn), out, ar, p) != TT_OK) return 0;
  return ar.used + 256;
}

tt_status tt_kernel_build_cross(int32_t batch, const tt_grid* grids, const double* q, const int32_t* halfwidths,
                                double svd_tol, int32_t max_rank, const tt_train* out, void* ws, size_t ws_bytes,
                                void* stream) {
  return ttg::kernel_cross_impl(batch, grids, q, halfwidths, svd_tol, max_rank, out, ws, ws_bytes,
                                reinterpret_cast<hipStream_t>(stream));
}

}  // extern "C"
