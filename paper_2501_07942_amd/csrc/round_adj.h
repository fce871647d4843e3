// Adjoint of the TT rounding of Sec. 4.1 'round' at fixed ranks (FP64).
//
// The rounding is written as a function of the input cores A_k alone (its
// value as a full tensor does not depend on the orthogonalisation used):
//
//   right-part Grams   G_{d-1} = 1,  G_{k-1} = sum_i A_k(:,i,:) G_k A_k(:,i,:)^T
//   left to right      N_k = W_k x_1 A_k  ((r_k n_k) x R_{k+1}),  W_0 = 1
//                      U_k = leading r_{k+1} eigenvectors of S_k = N_k G_k N_k^T
//                      W_{k+1} = U_k^T N_k
//   output             core k = U_k (k < d-1),  last core = W_{d-1} x_1 A_{d-1}
//
// The library's forward rounding returns these cores up to scalar factors
// moved into the log-scale and the signs of the bond indices.  The adjoint
// takes all eigen-data of S_k (kept and discarded vectors, eigenvalues) from
// its own SVD of M_k = N_k F_k, with F_k F_k^T = G_k a pivoted Cholesky
// factor of G_k accumulated in double-double (as the forward rounding does,
// so that small singular values are resolved); the SVD comes from a
// double-double Gram of M_k, its pivoted Cholesky factor and a one-sided
// Jacobi SVD of that factor, refined where tiny singular values were kept.
// The forward output and its adjoint are sign-matched to that basis bond by
// bond, so every quantity of the adjoint belongs to one decomposition.  For
// the leading eigenvectors,
// dU_j = sum_{i != j} u_i (u_i^T dS u_j) / (lam_j - lam_i); its adjoint is
// Sbar = X U^T with
//   X_j = (I - U_all U_all^T) Ubar_j / lam_j + sum_{i discarded} u_i (u_i^T Ubar_j) / (lam_j - lam_i)
//       = (I - U U^T) Ubar_j / lam_j + sum_{i discarded} u_i (u_i^T Ubar_j) lam_i / (lam_j (lam_j - lam_i))
// (couplings among kept vectors cancel because everything downstream
// depends on the rounded tensor only).  Kept directions below TAU of the
// largest singular value are left out: their terms carry rounding noise of
// order eps sigma_1^2 / sigma_j^2.  Then, per core from the right,
//   Nbar = U Wbar_{k+1} + X (W_{k+1} G_k) + U ((X^T N_k) G_k)
//   Gbar_k += (X^T N_k)^T W_{k+1}
//   Wbar_k = Nbar x A_k^T,  Abar_k += W_k^T Nbar
// and finally the Gram recursion from the left:
//   Abar_k(:,i,:) += (Gbar_{k-1} + Gbar_{k-1}^T) A_k(:,i,:) G_k
//   Gbar_k += sum_i A_k(:,i,:)^T Gbar_{k-1} A_k(:,i,:).
//
// Every step is a small dense product (one grouped GEMM launch per phase,
// described by a job table built on the host) or an elementwise pass.
#pragma once

#include "common.h"
#include "linalg.h"

namespace ttg {

#define RADJ_TAU 6e-6     // kept singular values below TAU * sigma_1 are left out
#define RADJ_DISC 1e-9    // discarded singular values below this (relative) count as null space
// pivoted-Cholesky stop of the adjoint's double-double Grams, relative to
// the trace (singular values down to about 1e-15 of the largest are kept: a
// rounding may keep directions that small, and each kept one needs its vector)
#define RADJ_PCHOL_TAU2 1e-30

// C = alpha * A B + beta * C (beta = 0 overwrites) for a table of FP64
// products with arbitrary strides, one 64 x 64 tile of one job per workgroup.
struct GJob {
  int M, N, K;
  const double* a;
  long long sam, sak;
  const double* b;
  long long sbk, sbn;
  double* c;
  long long scm, scn;
  double alpha, beta;
  int tile0;  // first global tile of this job
  int tn;     // tiles along N
  // split K: ks > 1 slices of kc (a multiple of 32) each write their partial
  // product to part[s][M][N]; gjob_reduce_kernel then sums the slices in
  // order and applies alpha and beta
  int ks, kc;
  double* part;
};

// The job table on the FP64 matrix cores: wavefront w of a tile owns rows
// 16 w .. 16 w + 15 and the four 16-column tiles, each
// 16 x 16 x 4 FP64 MFMA step reads A(i, k) in lane i + 16 k and B(k, j) in
// lane j + 16 k from the LDS stage; D(i, j) sits in lane j + 16 (i % 4),
// register i / 4.  Every element sums its k in MFMA chunks of four in
// increasing order, independent of the other jobs.
typedef double gj_d4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) gjob_mfma_kernel(const GJob* __restrict__ jobs, int njobs) {
  const int t = blockIdx.x;
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].tile0 <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  const GJob g = jobs[lo];
  const int tmn = ((g.M + 63) / 64) * g.tn;  // tiles of one K slice
  const int sl = (t - g.tile0) / tmn, lt = t - g.tile0 - sl * tmn;
  const int m0 = (lt / g.tn) * 64, n0 = (lt - (lt / g.tn) * g.tn) * 64;
  if (m0 >= g.M || n0 >= g.N) return;
  const int kbeg = g.ks > 1 ? sl * g.kc : 0;
  const int kend = g.ks > 1 ? min(g.K, kbeg + g.kc) : g.K;
  // K blocks of 32; the next block is fetched into registers while the
  // current one is multiplied out of the LDS
  constexpr int KB = 32;
  __shared__ double As[KB][64 + 1];
  __shared__ double Bs[KB][64 + 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const TTG_GLOBAL double* ga = gmem(g.a);
  const TTG_GLOBAL double* gb = gmem(g.b);
  gj_d4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = gj_d4{0.0, 0.0, 0.0, 0.0};
  double ra[8], rb[8];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + 256 * u;
      const int mm = e >> 5, kk = e & 31;  // A: 64 rows x 32 k
      const int m = m0 + mm, k = k0 + kk;
      ra[u] = (m < g.M && k < kend) ? ga[(long long)m * g.sam + (long long)k * g.sak] : 0.0;
      const int kb = e >> 6, nn = e & 63;  // B: 32 k x 64 columns
      const int n = n0 + nn, k2 = k0 + kb;
      rb[u] = (n < g.N && k2 < kend) ? gb[(long long)k2 * g.sbk + (long long)n * g.sbn] : 0.0;
    }
  };
  fetch(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += KB) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = threadIdx.x + 256 * u;
      As[e & 31][e >> 5] = ra[u];
      Bs[e >> 6][e & 63] = rb[u];
    }
    lds_barrier();
    if (k0 + KB < kend) fetch(k0 + KB);
#pragma unroll
    for (int kk = 0; kk < KB; kk += 4) {
      const double av = As[kk + lk][16 * w + li];
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, Bs[kk + lk][16 * j + li], acc[j], 0, 0, 0);
    }
    lds_barrier();
  }
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + 16 * w + 4 * v + lk, n = n0 + 16 * j + li;
      if (m < g.M && n < g.N) {
        if (g.ks > 1) {
          gmem(g.part)[((long long)sl * g.M + m) * g.N + n] = acc[j][v];
        } else {
          TTG_GLOBAL double* cp = gmem(g.c) + (long long)m * g.scm + (long long)n * g.scn;
          *cp = g.beta == 0.0 ? g.alpha * acc[j][v] : __fma_rn(g.alpha, acc[j][v], g.beta * *cp);
        }
      }
    }
}

// C = alpha * sum_s part[s] + beta * C for the split jobs of a table, the
// slices summed in increasing order; blockIdx.y selects the job
__global__ void __launch_bounds__(256) gjob_reduce_kernel(const GJob* __restrict__ jobs) {
  const GJob g = jobs[blockIdx.y];
  if (g.ks <= 1) return;
  const long long mn = (long long)g.M * g.N;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < mn; e += (long long)gridDim.x * blockDim.x) {
    double v = 0.0;
    for (int sl = 0; sl < g.ks; ++sl) v += g.part[sl * mn + e];
    const int m = (int)(e / g.N), n = (int)(e - (long long)m * g.N);
    double* cp = g.c + (long long)m * g.scm + (long long)n * g.scn;
    *cp = g.beta == 0.0 ? g.alpha * v : __fma_rn(g.alpha, v, g.beta * *cp);
  }
}

// ---------------------------------------------------------------------------
// elementwise passes; blockIdx.y selects the job
// ---------------------------------------------------------------------------
struct EJob {
  int op;
  long long cnt;
  const double* x;
  const double* y;
  double* out;
  double* out2;
  const double* s;  // device scalar
  int r, p, R;      // shapes for the eigen passes
  int ld;
};

enum {
  EJ_FILL = 0,      // out[e] = 0
  EJ_SCALE = 1,     // out[e] = s[0] * x[e]
  EJ_SYM = 2,       // out = x + x^T (r x r)
  EJ_ONE = 3,       // out[0] = 1
  EJ_DDHI = 4,      // out[e] = high word of the double-double x[e]
  EJ_COPY = 5,      // out[e] = x[e]
  EJ_ROWFLIP = 6,   // out[e] = x[e] * y[e / ld] (signs of the left bond index)
  EJ_COLDIV = 7,    // out[e] = x[e] / y[e / ld] where y > 0, else 0 (column-major columns)
};

__global__ void __launch_bounds__(256) ejob_kernel(const EJob* __restrict__ jobs) {
  const EJob j = jobs[blockIdx.y];
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < j.cnt; e += stride) {
    switch (j.op) {
      case EJ_FILL: j.out[e] = 0.0; break;
      case EJ_SCALE: j.out[e] = j.s[0] * j.x[e]; break;
      case EJ_SYM: {
        const int a = (int)(e / j.r), b = (int)(e - (long long)a * j.r);
        j.out[e] = j.x[e] + j.x[(long long)b * j.r + a];
        break;
      }
      case EJ_DDHI: j.out[e] = j.x[2 * e]; break;
      case EJ_COPY: j.out[e] = j.x[e]; break;
      case EJ_ROWFLIP: j.out[e] = j.x[e] * j.y[e / j.ld]; break;
      case EJ_COLDIV: {
        const double v = j.y[e / j.ld];
        j.out[e] = v > 0.0 ? j.x[e] / v : 0.0;
        break;
      }
      default: if (e == 0) j.out[0] = 1.0; break;
    }
  }
}

// Norm factor c of a core Y_k = c U_k with orthonormal columns (r of them):
// c = sqrt(||Y||^2 / r); writes c and U = Y / c.  One workgroup per job.
// With op = 1 instead: kappa = <x, y> / ||y||^2 (the last core Y = kappa L).
__global__ void __launch_bounds__(256) radj_scalar_kernel(const EJob* __restrict__ jobs) {
  const EJob j = jobs[blockIdx.x];
  __shared__ double red[4];
  double s = 0.0, t = 0.0;
  for (long long e = threadIdx.x; e < j.cnt; e += blockDim.x) {
    const double v = j.x[e];
    if (j.op == 0) {
      s = __fma_rn(v, v, s);
    } else {
      s = __fma_rn(v, j.y[e], s);
      t = __fma_rn(j.y[e], j.y[e], t);
    }
  }
  s = block_sum(s, red);
  t = block_sum(t, red);
  if (j.op == 0) {
    const double c = sqrt(s / (double)j.r);
    if (threadIdx.x == 0) j.out2[0] = c;
    const double ic = c > 0.0 ? 1.0 / c : 0.0;
    for (long long e = threadIdx.x; e < j.cnt; e += blockDim.x) j.out[e] = j.x[e] * ic;
  } else if (threadIdx.x == 0) {
    j.out2[0] = t > 0.0 ? s / t : 0.0;
  }
}

// From the Jacobi SVD of M (sigma descending, usv column c = sigma_c u_c,
// column-major ld p) and the kept count r: the discarded left vectors
// Ud (p x (R - r), row-major) = u_i for sigma_i > DISC sigma_1 (zero
// otherwise), the coupling corrections Fm ((R - r) x r) =
// 1 / (lam_j - lam_i) - 1 / lam_j for those i and live j, and linv (r) =
// 1 / lam_j for live j (sigma_j >= TAU sigma_1), zero for left-out j.  The
// eigenvector adjoint is then X = (I - U U^T) Ubar diag(linv) +
// Ud ((Ud^T Ubar) o Fm): the complement of the kept vectors U (taken from
// the forward's output) enters through U alone, and each discarded
// direction only through a correction weighted by its own lam_i, so
// rounding noise in small discarded directions stays small.  x = sigma, y = usv, out = Ud, out2 = Fm,
// s -> linv (written through out2 + (R - r) r).  One workgroup per job.
__global__ void __launch_bounds__(256) radj_eigprep_kernel(const EJob* __restrict__ jobs) {
  const EJob j = jobs[blockIdx.x];
  const int p = j.p, R = j.R, r = j.r, nd = R - r;
  const double* sig = j.x;
  const double s1 = sig[0];
  double* linv = j.out2 + (long long)nd * r;
  for (int c = threadIdx.x; c < r; c += blockDim.x) {
    const double sj = sig[c];
    linv[c] = (s1 > 0.0 && sj >= RADJ_TAU * s1) ? 1.0 / (sj * sj) : 0.0;
  }
  for (long long e = threadIdx.x; e < (long long)nd * r; e += blockDim.x) {
    const int i = (int)(e / r), c = (int)(e - (long long)i * r);
    const double si = sig[r + i], sj = sig[c];
    const bool ok = s1 > 0.0 && si > RADJ_DISC * s1 && sj >= RADJ_TAU * s1 && sj > si;
    // 1 / (lam_j - lam_i) - 1 / lam_j = lam_i / (lam_j (lam_j - lam_i))
    j.out2[e] = ok ? (si * si) / ((sj * sj) * ((sj - si) * (sj + si))) : 0.0;
  }
  for (long long e = threadIdx.x; e < (long long)p * nd; e += blockDim.x) {
    const int row = (int)(e / nd), i = (int)(e - (long long)row * nd);
    const double si = sig[r + i];
    j.out[e] = (s1 > 0.0 && si > RADJ_DISC * s1) ? j.y[(long long)(r + i) * j.ld + row] / si : 0.0;
  }
}

// X = Z diag(linv) in place (Z p x r) and P2 = P2 o Fm in place ((R - r) x r).
// x unused; out = Z, out2 = P2, y = Fm, s = linv.
__global__ void __launch_bounds__(256) radj_eigapply_kernel(const EJob* __restrict__ jobs) {
  const EJob j = jobs[blockIdx.y];
  const int r = j.r, nd = j.R - j.r;
  const long long nz = (long long)j.p * r, np = (long long)nd * r;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nz + np; e += stride) {
    if (e < nz) {
      j.out[e] *= j.s[e % r];
    } else {
      const long long f = e - nz;
      j.out2[f] *= j.y[f];
    }
  }
}

// The adjoint works in the basis of its own SVD of M_k (so that the kept
// vectors, their complement and the eigenvalues are mutually consistent to
// working precision); the forward's output core Y_k = c_k U_fwd differs from
// it by the signs of the bond indices.  Per job (filter, core k): with the
// previous bond's signs dprev (on the left index a of a row (a, i)), the
// sign of each kept column c is that of <dprev o U_fwd(:, c), u_c>; then
// U <- u_c (overwriting U_fwd) and ybt = c_k (dprev o Ybar_k) diag(dk),
// the output adjoint expressed in the adjoint's basis.  One workgroup per
// job.
struct AJob {
  const double* usv;
  const double* sig;
  double* U;
  double* ybt;
  const double* ybar;
  const double* c;
  const double* dprev;
  double* dk;
  int p, r, n, ldu;
};

__global__ void __launch_bounds__(256) radj_adopt_kernel(const AJob* __restrict__ jobs) {
  const AJob j = jobs[blockIdx.x];
  __shared__ double red[4];
  for (int c = 0; c < j.r; ++c) {
    double s = 0.0;
    for (int row = threadIdx.x; row < j.p; row += blockDim.x)
      s += j.dprev[row / j.n] * j.U[(long long)row * j.r + c] * j.usv[(long long)c * j.ldu + row];
    s = block_sum(s, red);
    if (threadIdx.x == 0) j.dk[c] = s >= 0.0 ? 1.0 : -1.0;
  }
  __syncthreads();
  const double c0 = j.c[0];
  for (long long e = threadIdx.x; e < (long long)j.p * j.r; e += blockDim.x) {
    const int row = (int)(e / j.r), c = (int)(e - (long long)row * j.r);
    const double sc = j.sig[c];
    j.U[e] = sc > 0.0 ? j.usv[(long long)c * j.ldu + row] / sc : 0.0;
    j.ybt[e] = c0 * j.dprev[row / j.n] * j.ybar[e] * j.dk[c];
  }
}

// pivoted Cholesky and Jacobi SVD over job tables
struct FAdjPchol {
  const PcholArgs* a;
  __device__ bool operator()(int b, PcholArgs& p) const {
    p = a[b];
    return p.M > 0;
  }
};

// Jacobi over a job table whose column count is capped by a device value
// (the rank a pivoted Cholesky factor reached)
struct RkJacobi {
  JacobiArgs ja;
  const int* ncols;
};
struct FAdjJacobiRk {
  const RkJacobi* a;
  __device__ bool operator()(int b, JacobiArgs& J) const {
    J = a[b].ja;
    if (J.rows <= 0) return false;
    J.ncols = min(J.ncols, *a[b].ncols);
    return J.ncols > 0;
  }
};

// The SVD of a tall M_k from its Gram gives sigma_c u_c = M_k v_c with v_c
// from the Jacobi SVD of the FP64 Cholesky factor; a singular vector u_c of
// a very small sigma_c then carries errors of order eps * sigma_1 / sigma_c.
// When a rounding kept a singular value below RADJ_REFINE * sigma_1 the SVD
// is refined: Mt = M_k V (the product summed in double-double, so each
// column is exact to its own size) has nearly orthogonal columns graded by
// sigma_c, and one-sided Jacobi on Mt removes what is left in a sweep or
// two, with accuracy relative to each column.  Flag per job.
#define RADJ_REFINE 1e-8
// The refinement keeps the columns that the adjoint resolves: the kept
// ones and the discarded ones above RADJ_DISC * sigma_1 (the rest count as
// null space anyway); flag[1] holds their number.
struct RefJob {
  double* sig;
  int r, R;
  int* flag;  // [0]: refine, [1]: columns kept for it
};
__global__ void radj_refine_flag_kernel(const RefJob* __restrict__ jobs, int njobs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= njobs) return;
  const RefJob j = jobs[i];
  if (!j.flag) return;
  const double s1 = j.sig[0], sr = j.r >= 1 ? j.sig[j.r - 1] : s1;
  j.flag[0] = (s1 > 0.0 && !(sr >= RADJ_REFINE * s1)) ? 1 : 0;
  int m = j.r;
  while (m < j.R && j.sig[m] > RADJ_DISC * s1) ++m;
  j.flag[1] = m;
}
struct CondJacobi {
  JacobiArgs ja;
  const int* flag;
};
struct FAdjJacobiIf {
  const CondJacobi* a;
  __device__ bool operator()(int b, JacobiArgs& J) const {
    J = a[b].ja;
    if (!a[b].flag || a[b].flag[0] == 0) return false;
    J.ncols = min(J.ncols, a[b].flag[1]);
    return J.rows > 0 && J.ncols > 0;
  }
};
// after the refinement: singular values beyond the refined columns are zero
__global__ void radj_refine_tail_kernel(const RefJob* __restrict__ jobs, int njobs) {
  const RefJob j = jobs[blockIdx.x];
  if (!j.flag || j.flag[0] == 0) return;
  for (int c = j.flag[1] + threadIdx.x; c < j.R; c += blockDim.x) j.sig[c] = 0.0;
}

// Mt(:, c) = M vs(:, c) / sigma_c summed in double-double, for flagged jobs
// (columns with sigma_c = 0 are zero).  M: p x R1 row-major; vs: column-major
// R1 x R1 (column c = sigma_c v_c); Mt: p x R1 row-major.  Grid: (blocks, jobs).
struct DJob {
  const double* vs;
  const double* M;
  const double* sig;
  double* usv;  // Mt
  const int* flag;
  int p, R1;
};
__global__ void __launch_bounds__(256) radj_ddprod_kernel(const DJob* __restrict__ jobs) {
  const DJob j = jobs[blockIdx.y];
  if (!j.flag || *j.flag == 0) return;
  const long long tot = (long long)j.p * j.R1;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += stride) {
    const int row = (int)(e / j.R1), c = (int)(e - (long long)row * j.R1);
    const double sc = j.sig[c];
    if (!(sc > 0.0) || c >= j.flag[1]) {
      j.usv[e] = 0.0;
      continue;
    }
    const double* vc = j.vs + (long long)c * j.R1;
    const double* mr = j.M + (long long)row * j.R1;
    dd acc = AccDD::zero();
    for (int q = 0; q < j.R1; ++q) acc = AccDD::fma_(acc, vc[q], mr[q]);
    j.usv[e] = dd_div(acc, AccDD::from(sc)).hi;
  }
}

}  // namespace ttg
