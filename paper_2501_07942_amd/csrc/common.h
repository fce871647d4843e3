// Internal definitions shared by the HIP sources of the TT grid-based filter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/ttgbf.h"

#define TTG_HOST_DEVICE __host__ __device__

// Global-memory view of a device pointer.  Pointers that a kernel reads out
// of a descriptor are generic, and loads and stores through them compile to
// flat instructions, which count against the LDS wait counter as well: every
// LDS wait in such a kernel then also waits for its HBM traffic in flight.
// Accesses through this view are global instructions instead.  The
// qualifier exists only in the device pass; host code never dereferences it.
#if defined(__HIP_DEVICE_COMPILE__)
#define TTG_GLOBAL __attribute__((address_space(1)))
#else
#define TTG_GLOBAL
#endif
template <typename T>
__device__ __forceinline__ TTG_GLOBAL T* gmem(T* p) {
  return (TTG_GLOBAL T*)p;
}

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also
// waits for every global store of the wavefront to complete; the kernels
// that use this never read back their own global writes, so their output
// stores stay in flight across the barrier.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ---------------------------------------------------------------------------
// device copy of a tt_train, with core offsets resolved
// ---------------------------------------------------------------------------
struct DevTT {
  int d;
  int n[TT_MAXD];
  int cap[TT_MAXD + 1];
  long long off[TT_MAXD];
  void* cores;
  int* ranks;
  double* log_scale;
  int* status;
};

template <typename T>
__device__ inline T* core_ptr(const DevTT& t, int k) {
  return reinterpret_cast<T*>(t.cores) + t.off[k];
}

// ---------------------------------------------------------------------------
// per-filter rounding scratch (all pointers are device memory)
// ---------------------------------------------------------------------------
struct RoundScratch {
  int rqcap[TT_MAXD + 1];   // capacities of the pre-truncated ranks
  long long qoff[TT_MAXD];  // element offsets of the orthogonal cores in qbuf
  int gcap;                 // leading dimension of every square scratch matrix
  int splits;               // split-K partial Gram matrices
  int max_rank;             // this filter's rank cap for the rank rule (0: the launch's)
  void* qbuf;               // orthogonal cores Q_k (bulk type)
  void* zbuf;               // Z_k = X_k x_3 T_{k+1} (bulk type)
  void* bbuf;               // B_k = W_k x_1 Q_k (bulk type)
  double* gram;             // Gram partials (accumulator type; dd = 2 doubles)
  double* lwork;            // pivoted Cholesky factor in accumulator type
  double* lfac;             // pivoted Cholesky factor rounded to FP64, row-major gcap x gcap
  double* jac;              // Jacobi workspace, column-major gcap x gcap
  double* sigma;            // singular values (descending), gcap
  double* usv;              // Jacobi columns sorted: column j = sigma_j * u_j, gcap x gcap
  double* vs;               // V_r Sigma_r^{-1}: rq x r row-major (ld gcap)
  double* w;                // Sigma_r V_r^T: r x rq row-major (ld gcap)
  int* piv;                 // pivot order, gcap
  int* rq;                  // pre-truncated ranks [d+1]
  int* ri;                  // ranks of the input TT at entry [d+1] (snapshot)
  int* misc;                // [0] = effective rank of the last pivoted Cholesky
  double* scal;             // [0] = ||A||, [1] = delta, [2] = pchol residual
};

// ---------------------------------------------------------------------------
// double-double arithmetic (error-free transformations; see Dekker 1971,
// Knuth TAOCP vol. 2, Ogita-Rump-Oishi 2005).  Used to accumulate the Gram
// matrices of FP64 TTs so that pivoted Cholesky resolves singular values far
// below sqrt(eps_64) of the largest one.
// ---------------------------------------------------------------------------
struct dd {
  double hi, lo;
};

// The transformations below are exact only if every product and sum is
// rounded on its own: forbid the compiler from fusing a*b + c into an FMA
// (HIP compiles with -ffp-contract=fast by default).
#define TTG_NO_CONTRACT _Pragma("clang fp contract(off)")

__device__ inline dd dd_two_sum(double a, double b) {
  TTG_NO_CONTRACT
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ inline dd dd_fast_two_sum(double a, double b) {
  TTG_NO_CONTRACT
  double s = a + b;
  double e = b - (s - a);
  return {s, e};
}
__device__ inline dd dd_two_prod(double a, double b) {
  TTG_NO_CONTRACT
  double p = a * b;
  double e = __fma_rn(a, b, -p);
  return {p, e};
}
__device__ inline dd dd_add(dd a, dd b) {
  TTG_NO_CONTRACT
  dd s = dd_two_sum(a.hi, b.hi);
  dd t = dd_two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = dd_fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return dd_fast_two_sum(s.hi, s.lo);
}
__device__ inline dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }
__device__ inline dd dd_mul(dd a, dd b) {
  TTG_NO_CONTRACT
  dd p = dd_two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return dd_fast_two_sum(p.hi, p.lo);
}
__device__ inline dd dd_mul_d(dd a, double b) {
  TTG_NO_CONTRACT
  dd p = dd_two_prod(a.hi, b);
  p.lo += a.lo * b;
  return dd_fast_two_sum(p.hi, p.lo);
}
__device__ inline dd dd_div(dd a, dd b) {
  TTG_NO_CONTRACT
  double q1 = a.hi / b.hi;
  dd r = dd_sub(a, dd_mul_d(b, q1));
  double q2 = r.hi / b.hi;
  r = dd_sub(r, dd_mul_d(b, q2));
  double q3 = r.hi / b.hi;
  dd q = dd_fast_two_sum(q1, q2);
  return dd_add(q, dd{q3, 0.0});
}
__device__ inline dd dd_sqrt(dd a) {
  TTG_NO_CONTRACT
  if (!(a.hi > 0.0)) return {0.0, 0.0};
  double x = sqrt(a.hi);
  dd x2 = dd_two_prod(x, x);
  double corr = ((a.hi - x2.hi) - x2.lo + a.lo) / (2.0 * x);
  return dd_fast_two_sum(x, corr);
}

// Accumulator policies: double (FP32 bulk path) and dd (FP64 path).
struct AccD {
  using V = double;
  static constexpr int words = 1;
  __device__ static V zero() { return 0.0; }
  __device__ static V from(double x) { return x; }
  __device__ static V add(V a, V b) { return a + b; }
  __device__ static V sub(V a, V b) { return a - b; }
  __device__ static V mul(V a, V b) { return a * b; }
  __device__ static V div(V a, V b) { return a / b; }
  __device__ static V sqrt_(V a) { return a > 0.0 ? sqrt(a) : 0.0; }
  __device__ static double hi(V a) { return a; }
  __device__ static V load(const double* p, long long i) { return p[i]; }
  __device__ static void store(double* p, long long i, V v) { p[i] = v; }
  // acc += a*b for FP64 inputs
  __device__ static V fma_(V acc, double a, double b) { return __fma_rn(a, b, acc); }
};

struct AccDD {
  using V = dd;
  static constexpr int words = 2;
  __device__ static V zero() { return {0.0, 0.0}; }
  __device__ static V from(double x) { return {x, 0.0}; }
  __device__ static V add(V a, V b) { return dd_add(a, b); }
  __device__ static V sub(V a, V b) { return dd_sub(a, b); }
  __device__ static V mul(V a, V b) { return dd_mul(a, b); }
  __device__ static V div(V a, V b) { return dd_div(a, b); }
  __device__ static V sqrt_(V a) { return dd_sqrt(a); }
  __device__ static double hi(V a) { return a.hi; }
  __device__ static V load(const double* p, long long i) { return {p[2 * i], p[2 * i + 1]}; }
  __device__ static void store(double* p, long long i, V v) {
    p[2 * i] = v.hi;
    p[2 * i + 1] = v.lo;
  }
  __device__ static V fma_(V acc, double a, double b) {
    TTG_NO_CONTRACT
    // Dot2-style compensated accumulation of an exact product
    dd p = dd_two_prod(a, b);
    dd s = dd_two_sum(acc.hi, p.hi);
    s.lo += acc.lo + p.lo;
    return dd_fast_two_sum(s.hi, s.lo);
  }
};

// ---------------------------------------------------------------------------
// wavefront / block reductions (64-lane wavefronts)
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline float wave_sumf(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the block; every thread gets the result.  `red` must hold
// blockDim.x/64 doubles of shared memory.
__device__ inline double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < nw; ++i) t += red[i];
  __syncthreads();
  return t;
}

__device__ inline double bulk_to_double(float x) { return (double)x; }
__device__ inline double bulk_to_double(double x) { return x; }

template <typename T>
__device__ inline T from_double(double x);
template <>
__device__ inline float from_double<float>(double x) {
  return (float)x;
}
template <>
__device__ inline double from_double<double>(double x) {
  return x;
}

__device__ inline void set_status(int* st, int bits) {
  if (st) atomicOr(st, bits);
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------
namespace ttg {
void set_error(const char* fmt, ...);
tt_status check_hip(hipError_t e, const char* what);
}  // namespace ttg

#define TTG_LAUNCH_CHECK(what)                                                   \
  do {                                                                           \
    hipError_t e_ = hipGetLastError();                                           \
    if (e_ != hipSuccess) return ttg::check_hip(e_, what);                       \
  } while (0)
