// Host side of the C ABI: argument checks, workspace planning, descriptor
// upload and the launch sequences of every entry point in ttgbf.h.
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "common.h"
#include "linalg.h"
#include "ttops.h"
#include "fft.h"
#include "adjoint.h"
#include "round_adj.h"
#include "einsum.h"
#include "interp.h"
#include "pred_mfma.h"

namespace ttg {

static thread_local char g_err[1024] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

tt_status check_hip(hipError_t e, const char* what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return TT_ERR_HIP;
}

// ---------------------------------------------------------------------------
// optional timing of kernel classes with HIP events on the launch stream
// ---------------------------------------------------------------------------
enum ProfClass {
  PC_CONV = 0, PC_HADAMARD, PC_GRAM, PC_PCHOL, PC_JACOBI, PC_TRSM, PC_GEMM, PC_LIK, PC_CONTRACT, PC_PRED, PC_EINSUM,
  PC_INTERP, PC_OTHER,
  PC_N
};
struct ProfRec {
  int cls;
  hipEvent_t a, b;
};
static std::vector<ProfRec> g_prof;
static std::vector<hipEvent_t> g_pool;
static int g_prof_mask = 0;
static size_t g_pool_next = 0;

// Algorithmic work of profiled launches: flops and HBM bytes per class,
// summed on the device by a one-workgroup kernel after each launch of a class
// that has a work model (so the counts follow the device-resident ranks).
static double* g_work = nullptr;  // [PC_N][2]: flops, bytes

static hipEvent_t prof_event() {
  if (g_pool_next == g_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    g_pool.push_back(e);
  }
  return g_pool[g_pool_next++];
}

struct ProfScope {
  int cls;
  hipStream_t st;
  hipEvent_t a = nullptr;
  ProfScope(int c, hipStream_t s) : cls(c), st(s) {
    if (g_prof_mask & (1 << c)) {
      a = prof_event();
      if (a) hipEventRecord(a, st);
    }
  }
  ~ProfScope() {
    if (a) {
      hipEvent_t b = prof_event();
      if (b) {
        hipEventRecord(b, st);
        g_prof.push_back({cls, a, b});
      }
    }
  }
};

#define HIP_TRY(expr, what)                              \
  do {                                                   \
    hipError_t e__ = (expr);                             \
    if (e__ != hipSuccess) return check_hip(e__, what);  \
  } while (0)

#define TT_TRY(expr)                 \
  do {                               \
    tt_status s__ = (expr);          \
    if (s__ != TT_OK) return s__;    \
  } while (0)

// ---------------------------------------------------------------------------
// bump allocator over the caller's workspace; with base == nullptr it only
// measures the bytes a plan needs (the *_workspace queries)
// ---------------------------------------------------------------------------
struct Arena {
  char* base;
  size_t cap;
  size_t used = 0;
  Arena(void* b, size_t c) : base(reinterpret_cast<char*>(b)), cap(c) {}
  template <typename T>
  T* take(size_t count) {
    size_t off = (used + 255) & ~size_t(255);
    used = off + count * sizeof(T);
    if (!base) return nullptr;
    return reinterpret_cast<T*>(base + off);
  }
  bool fits() const { return base != nullptr && used <= cap; }
};

static size_t elems_of(int d, const int* n, const int* cap) {
  size_t s = 0;
  for (int k = 0; k < d; ++k) s += (size_t)cap[k] * n[k] * cap[k + 1];
  return s;
}

static DevTT make_dev(const tt_train& t) {
  DevTT o;
  memset(&o, 0, sizeof(o));
  o.d = t.d;
  long long off = 0;
  for (int k = 0; k < t.d; ++k) {
    o.n[k] = t.n[k];
    o.off[k] = off;
    off += (long long)t.cap[k] * t.n[k] * t.cap[k + 1];
  }
  for (int k = 0; k <= t.d; ++k) o.cap[k] = t.cap[k];
  o.cores = t.cores;
  o.ranks = t.ranks;
  o.log_scale = t.log_scale;
  o.status = t.status;
  return o;
}

static tt_status check_train(const tt_train* t, const char* name, int want_dtype = -1) {
  if (!t) {
    set_error("%s is NULL", name);
    return TT_ERR_ARG;
  }
  if (t->d < 1 || t->d > TT_MAXD) {
    set_error("%s: d=%d out of range [1,%d]", name, t->d, TT_MAXD);
    return TT_ERR_SHAPE;
  }
  if (!t->cores || !t->ranks || !t->log_scale || !t->status) {
    set_error("%s: null device pointer", name);
    return TT_ERR_ARG;
  }
  if (t->dtype != TT_F64 && t->dtype != TT_F32) {
    set_error("%s: bad dtype %d", name, t->dtype);
    return TT_ERR_ARG;
  }
  if (want_dtype >= 0 && t->dtype != want_dtype) {
    set_error("%s: dtype %d, expected %d", name, t->dtype, want_dtype);
    return TT_ERR_ARG;
  }
  if (t->cap[0] != 1 || t->cap[t->d] != 1) {
    set_error("%s: cap[0] and cap[d] must be 1", name);
    return TT_ERR_SHAPE;
  }
  for (int k = 0; k < t->d; ++k)
    if (t->n[k] < 1 || t->n[k] > 4096) {
      set_error("%s: n[%d]=%d out of range", name, k, t->n[k]);
      return TT_ERR_SHAPE;
    }
  for (int k = 0; k <= t->d; ++k)
    if (t->cap[k] < 1 || t->cap[k] > 4096) {
      set_error("%s: cap[%d]=%d out of range", name, k, t->cap[k]);
      return TT_ERR_SHAPE;
    }
  return TT_OK;
}

// Descriptor uploads without a stream wait: the host data is copied into a
// page-locked ring (64 MB, allocated on first use) and uploaded from there
// with an event recorded behind the copy; a ring region is reused only after
// the event of every upload that occupied it has completed (the oldest
// uploads are waited for when the ring is full).  Regions are taken in
// order, so the in-flight uploads form one circular interval of the ring.
// An upload larger than the ring falls back to a copy and a stream wait.
// the upload with a stream wait and no library memory (the allocation-free
// entry point)
template <typename T>
static tt_status upload_wait(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return TT_OK;
  HIP_TRY(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s),
          "descriptor upload");
  HIP_TRY(hipStreamSynchronize(s), "descriptor upload sync");  // the host vectors die when the call returns
  return TT_OK;
}

struct UploadRing {
  struct Slot {
    hipEvent_t ev;
    size_t start, end;
  };
  std::mutex mu;
  char* buf = nullptr;
  size_t cap = 0;
  std::deque<Slot> inflight;
  std::vector<hipEvent_t> spare;
};
static UploadRing g_ring;

template <typename T>
static tt_status upload(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return TT_OK;
  const size_t bytes = src.size() * sizeof(T), need = (bytes + 255) & ~size_t(255);
  std::lock_guard<std::mutex> lk(g_ring.mu);
  if (!g_ring.buf) {
    const size_t c = size_t(64) << 20;
    HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&g_ring.buf), c, hipHostMallocPortable), "upload ring alloc");
    g_ring.cap = c;
  }
  if (need >= g_ring.cap / 2) {
    HIP_TRY(hipMemcpyAsync(dst, src.data(), bytes, hipMemcpyHostToDevice, s), "descriptor upload");
    HIP_TRY(hipStreamSynchronize(s), "descriptor upload sync");
    return TT_OK;
  }
  auto& q = g_ring.inflight;
  while (!q.empty() && hipEventQuery(q.front().ev) == hipSuccess) {  // completed uploads free their regions
    g_ring.spare.push_back(q.front().ev);
    q.pop_front();
  }
  size_t start = 0;
  for (;;) {
    if (q.empty()) {
      start = 0;
      break;
    }
    const size_t fs = q.front().start, be = q.back().end;
    if (be > fs) {  // occupied [fs, be): free [be, cap) and [0, fs)
      if (be + need <= g_ring.cap) {
        start = be;
        break;
      }
      if (need < fs) {
        start = 0;
        break;
      }
    } else if (be + need < fs) {  // wrapped, occupied [fs, cap) and [0, be): free [be, fs)
      start = be;
      break;
    }
    HIP_TRY(hipEventSynchronize(q.front().ev), "upload ring wait");
    g_ring.spare.push_back(q.front().ev);
    q.pop_front();
  }
  hipEvent_t ev;
  if (g_ring.spare.empty()) {
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming), "upload event");
  } else {
    ev = g_ring.spare.back();
    g_ring.spare.pop_back();
  }
  memcpy(g_ring.buf + start, src.data(), bytes);
  const hipError_t e1 = hipMemcpyAsync(dst, g_ring.buf + start, bytes, hipMemcpyHostToDevice, s);
  const hipError_t e2 = e1 == hipSuccess ? hipEventRecord(ev, s) : e1;
  if (e2 != hipSuccess) {
    // the region may still be read: drain the stream before it can be reused
    (void)hipStreamSynchronize(s);
    g_ring.spare.push_back(ev);
    return check_hip(e2, "descriptor upload");
  }
  q.push_back({ev, start, start + need});
  return TT_OK;
}

// Page-locked staging for the job tables of the calls that synchronise their
// stream before returning (the rounding adjoint): a table is copied into the
// staging area and uploaded without waiting; the area rewinds only after a
// synchronisation of the stream, so no pending copy reads rewritten memory.
// One call holds it at a time (the guard's lock).
struct PinnedStage {
  std::mutex mu;
  char* buf = nullptr;
  size_t cap = 0, off = 0;
};
static PinnedStage g_stage;

struct StageGuard {
  std::lock_guard<std::mutex> lock;
  hipStream_t st;
  explicit StageGuard(hipStream_t s) : lock(g_stage.mu), st(s) { g_stage.off = 0; }
  ~StageGuard() {
    if (g_stage.off) (void)hipStreamSynchronize(st);  // early error return: drain before the next holder
    g_stage.off = 0;
  }
};

template <typename T>
static tt_status stage_upload(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return TT_OK;
  const size_t bytes = src.size() * sizeof(T), need = (bytes + 255) & ~size_t(255);
  if (g_stage.off + need > g_stage.cap) {
    HIP_TRY(hipStreamSynchronize(s), "staging sync");
    g_stage.off = 0;
    if (need > g_stage.cap) {
      if (g_stage.buf) HIP_TRY(hipHostFree(g_stage.buf), "staging free");
      g_stage.buf = nullptr;
      g_stage.cap = 0;
      const size_t c = std::max(need, size_t(8) << 20);
      HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&g_stage.buf), c, hipHostMallocDefault), "staging alloc");
      g_stage.cap = c;
    }
  }
  char* p = g_stage.buf + g_stage.off;
  memcpy(p, src.data(), bytes);
  g_stage.off += need;
  HIP_TRY(hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, s), "descriptor upload");
  return TT_OK;
}

static int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

static FilterConst make_const(const tt_grid& g, const tt_meas* m) {
  FilterConst c;
  memset(&c, 0, sizeof(c));
  c.d = g.d;
  double ld = 0.0;
  for (int l = 0; l < g.d; ++l) {
    c.n[l] = g.n[l];
    c.lo[l] = g.lo[l];
    c.dx[l] = (g.hi[l] - g.lo[l]) / (double)(g.n[l] - 1);
    ld += std::log(c.dx[l]);
  }
  c.logdelta = ld;
  if (m) {
    c.meas_kind = m->kind;
    c.sensor[0] = m->sensor[0];
    c.sensor[1] = m->sensor[1];
    c.sigma_r = m->sigma_r;
    c.sigma_lin = m->sigma_lin;
    c.lik_tol = m->lik_tol;
    c.lik_max_rank = m->lik_max_rank;
  }
  return c;
}

static tt_status check_grid(const tt_grid* g) {
  if (!g || g->d < 1 || g->d > TT_MAXD) {
    set_error("bad grid");
    return TT_ERR_ARG;
  }
  for (int l = 0; l < g->d; ++l)
    if (g->n[l] < 2 || !(g->hi[l] > g->lo[l])) {
      set_error("grid axis %d: need n >= 2 and hi > lo", l);
      return TT_ERR_SHAPE;
    }
  return TT_OK;
}

// ===========================================================================
// rounding
// ===========================================================================
struct RoundShape {  // host-side maxima over the batch, for grid sizing
  int d = 0, B = 0;
  int rin[TT_MAXD + 1] = {0};   // input rank capacities
  int rq[TT_MAXD + 1] = {0};    // pre-truncated rank capacities
  int rout[TT_MAXD + 1] = {0};  // output rank capacities
  int n[TT_MAXD] = {0};
  int gcap = 0, splits = 1;
  bool f64 = true;
  bool merge = false;  // bond 1 wider than n_0: fold core 0 into the bond-1 step
};

static const int RQ_MAX_F64 = 256;
static const int RQ_MAX_F32 = 128;

// Capacity of the ranks kept by the pre-truncation of the right-to-left
// pass: 256 for FP64; for FP32 128, raised to 8x the output's largest rank
// capacity (at most 256) so that a wide cap is not starved by it.
static int rq_limit(bool f64, const int* out_cap, int d) {
  if (f64) return RQ_MAX_F64;
  int oc = 1;
  for (int j = 0; j <= d; ++j) oc = std::max(oc, out_cap[j]);
  return std::max(RQ_MAX_F32, std::min(2 * RQ_MAX_F32, 8 * oc));
}

struct RoundBufs {
  DevTT* din = nullptr;
  DevTT* dout = nullptr;
  RoundScratch* drs = nullptr;
};

// Per-filter scratch for one rounding (also used by the likelihood SVD and
// the kernel TT-SVD, which need the gram/pchol/jacobi parts only).
static void plan_round_scratch(Arena& ar, const DevTT& in, const DevTT& out, bool f64, int gcap,
                               int splits, RoundScratch& rs) {
  memset(&rs, 0, sizeof(rs));
  const int d = in.d;
  const int rqmax = rq_limit(f64, out.cap, out.d);
  rs.rqcap[0] = 1;
  rs.rqcap[d] = 1;
  for (int j = 1; j < d; ++j) rs.rqcap[j] = std::min(in.cap[j], rqmax);
  long long q = 0, zmax = 0, bmax = 0;
  for (int k = 0; k < d; ++k) {
    rs.qoff[k] = q;
    const int left = (k == 0) ? 1 : rs.rqcap[k];
    q += (long long)left * in.n[k] * rs.rqcap[k + 1];
    zmax = std::max(zmax, (long long)in.cap[k] * in.n[k] * rs.rqcap[k + 1]);
    bmax = std::max(bmax, (long long)out.cap[k] * in.n[k] * rs.rqcap[k + 1]);
  }
  if (d >= 2) bmax = std::max(bmax, (long long)in.n[0] * in.n[1] * rs.rqcap[2]);
  const size_t esz = f64 ? 8 : 4;
  const int words = 2;  // room for double-double (the likelihood SVD always uses it)
  rs.gcap = gcap;
  rs.splits = splits;
  rs.qbuf = ar.take<char>(q * esz);
  rs.zbuf = ar.take<char>(zmax * esz);
  rs.bbuf = ar.take<char>(bmax * esz);
  const long long g2 = (long long)gcap * gcap;
  rs.gram = ar.take<double>(g2 * words * splits);
  rs.lwork = ar.take<double>(g2 * words);
  rs.lfac = ar.take<double>(g2);
  rs.jac = ar.take<double>(g2);
  rs.sigma = ar.take<double>(gcap);
  rs.usv = ar.take<double>(g2);
  rs.vs = ar.take<double>(g2);
  rs.w = ar.take<double>(g2);
  rs.piv = ar.take<int>(gcap);
  rs.rq = ar.take<int>(TT_MAXD + 1);
  rs.ri = ar.take<int>(TT_MAXD + 1);
  rs.misc = ar.take<int>(8);
  rs.scal = ar.take<double>(8);
}

static int gram_tiles(int M) {
  const int t = (M + 31) / 32;
  return t * (t + 1) / 2;
}

// Split-K planes of every Gram scratch.  The split count a filter uses is
// a function of its own summation length only (gram_split_count), so a
// filter gives bitwise the same result alone or inside any batch.
static const int GRAM_PLANES = 8;
static int choose_splits(int pairs, int B, long long T, int smax) {
  (void)pairs;
  (void)B;
  (void)T;
  return std::min(smax, GRAM_PLANES);
}

// ---- functors (device side shape logic) ----------------------------------
struct RCtx {
  const DevTT* X;
  const DevTT* O;
  const RoundScratch* S;
  int k;
  int d;
  double tau2;
  int esz;    // bytes per bulk element
  int merge;  // fold core 0 into the bond-1 step (left rank bounded by n_0)
  const DevTT* Kn = nullptr;      // fused prediction: kernel TTs
  const DevTT* Pn = nullptr;      //                   PMD before prediction
  const FusedPred* FP = nullptr;  //                   FFT descriptors
  int fused = 0;                  // interior Z_k come from the fused path
  int zt = 0;                     // ... in (j, i) column order (FFT variant)
  double tau2_flag = 0.0;         // pre-truncation losses below this x ||X||^2 are not a capacity failure
};

template <typename T>
struct FArgs {
  int N, rp0, rp1, rk0, rk1, n, k, gcap;
  int hk;  // half width of this core's kernel fibre
  const T* p;
  const T* kcore;
  const double* lfac;
  FusedPred fp;
  T* z;
};

template <typename T>
struct FFused {
  using Args = FArgs<T>;
  RCtx c;
  __device__ bool operator()(int b, Args& g) const {
    const DevTT& K = c.Kn[b];
    const DevTT& P = c.Pn[b];
    const DevTT& X = c.X[b];
    const RoundScratch& s = c.S[b];
    const int k = c.k;
    g.rk0 = K.ranks[k];
    g.rk1 = K.ranks[k + 1];
    g.rp0 = P.ranks[k];
    g.rp1 = P.ranks[k + 1];
    // a capacity overflow was flagged when the product ranks were set
    if (g.rk0 * g.rp0 > X.cap[k] || g.rk1 * g.rp1 > X.cap[k + 1] || g.rk1 > 32) return false;
    g.N = s.rq[k + 1];
    g.n = P.n[k];
    g.k = k;
    g.gcap = s.gcap;
    g.p = core_ptr<T>(P, k);
    g.kcore = core_ptr<T>(K, k);
    g.hk = (K.n[k] - 1) / 2;
    g.lfac = s.lfac;
    g.fp = c.FP[b];
    g.z = reinterpret_cast<T*>(s.zbuf);
    return true;
  }
};

template <typename T>
__device__ inline T* qcore(const RoundScratch& s, int k) {
  return reinterpret_cast<T*>(s.qbuf) + s.qoff[k];
}

// Fold core 0 into the bond-1 step when bond 1 is wider than n_0 (its rank
// is bounded by n_0 from the left).  Decided per filter from its own ranks so
// that a filter gives the same result alone or in any batch.
__device__ inline bool merge_bond1(const DevTT& X, const RoundScratch& s) { return s.ri[1] > X.n[0]; }

template <typename T>
struct FRlAbsorb {  // Z_k = X_k x_3 L_{k+1}   (k = 0 writes the first core into qbuf)
  RCtx c;
  __device__ bool operator()(int b, GemmArgs& g) const {
    const DevTT& X = c.X[b];
    const RoundScratch& s = c.S[b];
    const int k = c.k;
    if (k == 0 && merge_bond1(X, s)) return false;  // first core comes from the bond-1 factor
    g.M = s.ri[k] * X.n[k];
    g.K = s.ri[k + 1];
    g.N = s.rq[k + 1];
    g.a = core_ptr<T>(X, k);
    g.sam = g.K;
    g.sak = 1;
    g.b = s.lfac;
    g.sbk = s.gcap;
    g.sbn = 1;
    g.c = (k == 0) ? (void*)qcore<T>(s, 0) : s.zbuf;
    g.scm = g.N;
    g.scn = 1;
    return true;
  }
};

template <typename T>
struct FRlMerge {  // Z'_1 = X_0 (n_0 x r_1) * Z_1 (r_1 x n_1 rq_2)  -> bbuf
  RCtx c;
  __device__ bool operator()(int b, GemmArgs& g) const {
    const DevTT& X = c.X[b];
    const RoundScratch& s = c.S[b];
    if (!merge_bond1(X, s)) return false;
    g.M = X.n[0];
    g.K = s.ri[1];
    g.N = X.n[1] * s.rq[2];
    g.a = core_ptr<T>(X, 0);
    g.sam = g.K;
    g.sak = 1;
    g.b = (c.d == 2) ? (const void*)core_ptr<T>(X, 1) : (const void*)s.zbuf;
    g.sbk = g.N;
    g.sbn = 1;
    g.c = s.bbuf;
    g.scm = g.N;
    g.scn = 1;
    return true;
  }
};

// merged case: the first core is the pivoted Cholesky factor L (n_0 x rq_1)
template <typename T>
__global__ void first_core_copy_kernel(const DevTT* __restrict__ X, const RoundScratch* __restrict__ S) {
  const int f = blockIdx.x;
  const RoundScratch& s = S[f];
  if (!merge_bond1(X[f], s)) return;
  const int n0 = X[f].n[0], r = s.rq[1];
  T* q = qcore<T>(s, 0);
  for (int e = threadIdx.x; e < n0 * r; e += blockDim.x) {
    const int i = e / r, j = e % r;
    q[e] = from_double<T>(s.lfac[(long long)i * s.gcap + j]);
  }
}

template <typename T>
struct FRlGram {
  RCtx c;
  __device__ bool operator()(int b, GramArgs& g) const {
    const DevTT& X = c.X[b];
    const RoundScratch& s = c.S[b];
    const int k = c.k;
    const bool mg = k == 1 && merge_bond1(X, s);
    g.M = mg ? X.n[0] : s.ri[k];
    g.T = X.n[k] * s.rq[k + 1];
    g.x = mg ? (const void*)s.bbuf
             : ((k == c.d - 1) ? (const void*)core_ptr<T>(X, k) : (const void*)s.zbuf);
    g.sa = g.T;
    g.st = 1;
    g.out = s.gram;
    g.gcap = s.gcap;
    g.splits = s.splits;
    return true;
  }
};

struct FRlPchol {
  RCtx c;
  __device__ bool operator()(int b, PcholArgs& p) const {
    const RoundScratch& s = c.S[b];
    const int k = c.k;
    p.M = (k == 1 && merge_bond1(c.X[b], s)) ? c.X[b].n[0] : s.ri[k];
    p.g = s.gram;
    p.lwork = s.lwork;
    p.lfac = s.lfac;
    p.piv = s.piv;
    p.rank_out = &s.rq[k];
    p.resid_out = nullptr;
    p.status = c.O[b].status;
    p.gcap = s.gcap;
    p.rmax = s.rqcap[k];
    p.tau2 = c.tau2;
    p.tau2_flag = c.tau2_flag;
    return true;
  }
};

template <typename T>
struct FRlTrsm {
  RCtx c;
  __device__ bool operator()(int b, TrsmArgs& a) const {
    const DevTT& X = c.X[b];
    const RoundScratch& s = c.S[b];
    const int k = c.k;
    a.r = s.rq[k];
    a.m = X.n[k] * s.rq[k + 1];
    a.lfac = s.lfac;
    a.piv = s.piv;
    a.gcap = s.gcap;
    const bool mg = k == 1 && merge_bond1(X, s);
    a.z = mg ? (const void*)s.bbuf
             : ((k == c.d - 1) ? (const void*)core_ptr<T>(X, k) : (const void*)s.zbuf);
    a.ldz = a.m;
    a.q = qcore<T>(s, k);
    a.ldq = a.m;
    a.zt_n = (c.zt && k >= 1 && k <= c.d - 2) ? X.n[k] : 0;
    a.wbuf = s.jac;  // free during the right-to-left sweep
    return true;
  }
};

template <typename T>
struct FLrB {  // B_k = W_k x_1 Q_k  (k >= 1)
  RCtx c;
  __device__ bool operator()(int b, GemmArgs& g) const {
    const DevTT& O = c.O[b];
    const RoundScratch& s = c.S[b];
    const int k = c.k;
    g.M = O.ranks[k];
    g.K = s.rq[k];
    g.N = O.n[k] * s.rq[k + 1];
    g.a = s.w;
    g.sam = s.gcap;
    g.sak = 1;
    g.b = qcore<T>(s, k);
    g.sbk = g.N;
    g.sbn = 1;
    g.c = (k == c.d - 1) ? (void*)core_ptr<T>(O, k) : s.bbuf;
    g.scm = g.N;
    g.scn = 1;
    return true;
  }
};

template <typename T>
struct FLrGram {
  RCtx c;
  __device__ bool operator()(int b, GramArgs& g) const {
    const DevTT& O = c.O[b];
    const RoundScratch& s = c.S[b];
    const int k = c.k;
    g.M = s.rq[k + 1];
    g.T = O.ranks[k] * O.n[k];
    g.x = (k == 0) ? (const void*)qcore<T>(s, 0) : (const void*)s.bbuf;
    g.sa = 1;
    g.st = g.M;
    g.out = s.gram;
    g.gcap = s.gcap;
    g.splits = s.splits;
    return true;
  }
};

struct FLrPchol {
  RCtx c;
  __device__ bool operator()(int b, PcholArgs& p) const {
    const RoundScratch& s = c.S[b];
    p.M = s.rq[c.k + 1];
    p.g = s.gram;
    p.lwork = s.lwork;
    p.lfac = s.lfac;
    p.piv = s.piv;
    p.rank_out = &s.misc[0];
    p.resid_out = &s.scal[2];
    p.status = c.O[b].status;
    p.gcap = s.gcap;
    p.rmax = s.gcap;
    p.tau2 = c.tau2;
    return true;
  }
};

struct FLrJacobi {
  RCtx c;
  __device__ bool operator()(int b, JacobiArgs& J) const {
    const RoundScratch& s = c.S[b];
    J.rows = s.rq[c.k + 1];
    J.ncols = s.misc[0];
    J.x = s.lfac;
    J.ldx = s.gcap;
    J.work = s.jac;
    J.sigma = s.sigma;
    J.usv = s.usv;
    J.ncols_out = nullptr;
    J.tol2 = c.esz == 4 ? 1e-16 : 1e-30;  // FP32 bulk: 1e-8 relative orthogonality
    J.gcap = s.gcap;
    return true;
  }
};

template <typename T>
struct FLrU {  // core k of the result = B_k V_r Sigma_r^{-1}
  RCtx c;
  __device__ bool operator()(int b, GemmArgs& g) const {
    const DevTT& O = c.O[b];
    const RoundScratch& s = c.S[b];
    const int k = c.k;
    g.M = O.ranks[k] * O.n[k];
    g.K = s.rq[k + 1];
    g.N = O.ranks[k + 1];
    g.a = (k == 0) ? (const void*)qcore<T>(s, 0) : (const void*)s.bbuf;
    g.sam = g.K;
    g.sak = 1;
    g.b = s.vs;
    g.sbk = s.gcap;
    g.sbn = 1;
    g.c = core_ptr<T>(O, k);
    g.scm = g.N;
    g.scn = 1;
    return true;
  }
};

// rank rule at bond k+1 of the output; prepares V_r Sigma_r^{-1} and Sigma_r V_r^T
// (forced != nullptr: rank replay, the rank at bond k+1 is
// forced[f * fstride + k + 1] instead of the rule, clamped like it)
__global__ void round_select_kernel(const DevTT* __restrict__ O, const RoundScratch* __restrict__ S,
                                    int k, int max_rank, const int* __restrict__ forced, long long fstride) {
  const int f = blockIdx.x;
  const DevTT& o = O[f];
  const RoundScratch& s = S[f];
  __shared__ int s_r;
  const int nc = s.misc[0];
  const int rq = s.rq[k + 1];
  if (threadIdx.x == 0 && forced) {
    int r = forced[f * fstride + k + 1];
    r = min(max(r, 1), max(nc, 1));
    if (r > o.cap[k + 1]) {
      r = o.cap[k + 1];
      atomicOr(o.status, TT_STATUS_CAPACITY);
    }
    o.ranks[k + 1] = r;
    s_r = r;
  } else if (threadIdx.x == 0) {
    const double delta = s.scal[1];
    double tail2 = fmax(s.scal[2], 0.0);
    // smallest r with sqrt(resid + sum_{j>=r} sigma_j^2) <= delta
    int r = nc;
    if (sqrt(tail2) <= delta) {
      r = nc;
      for (int j = nc - 1; j >= 0; --j) {
        const double t2 = tail2 + s.sigma[j] * s.sigma[j];
        if (sqrt(t2) <= delta) {
          tail2 = t2;
          r = j;
        } else {
          break;
        }
      }
    }
    r = max(r, 1);
    r = min(r, s.max_rank > 0 ? min(s.max_rank, max_rank) : max_rank);
    r = min(r, max(nc, 1));
    if (r > o.cap[k + 1]) {
      r = o.cap[k + 1];
      atomicOr(o.status, TT_STATUS_CAPACITY);
    }
    o.ranks[k + 1] = r;
    s_r = r;
  }
  if (threadIdx.x == 0) {  // the discarded part of this bond (the rounding's error bound, squared)
    double t2 = fmax(s.scal[2], 0.0);
    for (int j = s_r; j < nc; ++j) t2 += s.sigma[j] * s.sigma[j];
    s.scal[3] += t2;
  }
  __syncthreads();
  const int r = s_r;
  for (int e = threadIdx.x; e < r * rq; e += blockDim.x) {
    const int j = e / rq, t = e % rq;
    const double sg = (j < nc) ? s.sigma[j] : 0.0;
    const double x = (j < nc) ? s.usv[(long long)j * s.gcap + t] : 0.0;
    s.w[(long long)j * s.gcap + t] = x;
    s.vs[(long long)t * s.gcap + j] = (sg > 0.0) ? x / (sg * sg) : 0.0;
  }
}

// snapshot input ranks, fix boundary ranks, carry log-scale and status
__global__ void round_init_kernel(const DevTT* __restrict__ X, const DevTT* __restrict__ O,
                                  const RoundScratch* __restrict__ S, int nf) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const DevTT &x = X[f], &o = O[f];
  const RoundScratch& s = S[f];
  int over = 0;
  for (int j = 0; j <= x.d; ++j) {
    int r = x.ranks[j];
    if (r > x.cap[j] || r < 1) {  // never read outside the reserved storage
      over = 1;
      r = max(1, min(r, x.cap[j]));
    }
    s.ri[j] = r;
  }
  if (over) atomicOr(o.status, TT_STATUS_CAPACITY);
  s.rq[0] = 1;
  s.rq[x.d] = 1;
  const double ls = *x.log_scale;
  const int st = *x.status;
  o.ranks[0] = 1;
  o.ranks[x.d] = 1;
  *o.log_scale = ls;
  if (o.status != x.status) atomicOr(o.status, st);
}

// ||first core|| -> scal[0]; delta = eps * ||A|| / sqrt(d-1) -> scal[1]
template <typename T>
__global__ void round_norm_kernel(const DevTT* __restrict__ X, const RoundScratch* __restrict__ S,
                                  double eps) {
  const int f = blockIdx.x;
  const RoundScratch& s = S[f];
  const DevTT& x = X[f];
  const T* c = qcore<T>(s, 0);
  const long long tot = (long long)x.n[0] * s.rq[1];
  __shared__ double red[8];
  double a = 0.0;
  for (long long e = threadIdx.x; e < tot; e += blockDim.x) {
    const double v = bulk_to_double(c[e]);
    a += v * v;
  }
  a = block_sum(a, red);
  if (threadIdx.x == 0) {
    s.scal[0] = sqrt(a);
    s.scal[1] = eps * sqrt(a) / sqrt((double)max(x.d - 1, 1));
    s.scal[3] = 0.0;  // discarded tail^2, summed over the bonds by round_select_kernel
  }
}

// tails[f * stride] = sqrt(sum of the bonds' discarded tail^2) / ||A|| of the
// last rounding (its relative error bound)
__global__ void tail_record_kernel(const RoundScratch* __restrict__ S, int nf, double* __restrict__ tails,
                                   long long stride) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const RoundScratch& s = S[f];
  tails[f * stride] = s.scal[0] > 0.0 ? sqrt(fmax(s.scal[3], 0.0)) / s.scal[0] : 0.0;
}

// Workgroups per filter for a grid-stride kernel: enough to fill the chip
// for this batch (about 4096 workgroups in all), never more than the
// capacity needs.  Idle workgroups are not free: sizing by capacity alone
// can cost more than the work.
static int stride_grid(long long cap_blocks, int B, int target = 4096) {
  const long long want = std::max<long long>(4, target / std::max(1, B));
  return (int)std::max<long long>(1, std::min(cap_blocks, want));
}

template <typename F>
static tt_status launch_pchol_any(bool f64, F f, int B, int gcap, hipStream_t st);

template <typename Acc, typename F>
static tt_status launch_pchol(F f, int B, int gcap, hipStream_t st) {
  ProfScope ps_(PC_PCHOL, st);
  using V = typename Acc::V;
  const size_t base = (size_t)(2 * gcap) * sizeof(V) + (size_t)gcap * sizeof(int) + 64;
  int ncl = 0;  // factor columns mirrored in LDS (FP64 accumulation only)
  if (sizeof(V) == sizeof(double) && base < 150 * 1024)
    ncl = (int)std::min<size_t>(PC_LDS_COLS, (150 * 1024 - base) / ((size_t)gcap * sizeof(V)));
  const size_t smem = base + (size_t)ncl * gcap * sizeof(V);
  if (smem > 48 * 1024)
    HIP_TRY(hipFuncSetAttribute((const void*)pchol_kernel<Acc, F>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem),
            "pchol smem attribute");
  hipLaunchKernelGGL((pchol_kernel<Acc, F>), dim3(B), dim3(256), smem, st, f, ncl);
  TTG_LAUNCH_CHECK("pchol_kernel");
  return TT_OK;
}

// compute units of the current device, read once per device
static tt_status device_cus(int* out) {
  static std::mutex mu;
  static int cached[64] = {0};
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lk(mu);
  if (dev < 0 || dev >= 64) {
    set_error("device_cus: device index %d out of range", dev);
    return TT_ERR_ARG;
  }
  if (!cached[dev]) {
    int n = 0;
    HIP_TRY(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev), "compute unit count");
    cached[dev] = std::max(1, n);
  }
  *out = cached[dev];
  return TT_OK;
}

template <typename T, typename Acc, typename F>
static tt_status launch_gram(F f, int B, int Mcap, long long Tcap, int smax, hipStream_t st) {
  ProfScope ps_(PC_GRAM, st);
  (void)Tcap;
  // the split count a filter uses is derived on the device from its own T
  // (at most smax planes).  FP64 accumulation runs on the matrix cores for
  // every size, so that each element's summation order depends on the
  // filter alone; double-double accumulation uses the vector ALUs with
  // 32 x 32 or 64 x 64 tiles (both sum every element in the same order).
  const int t = (Mcap + 63) / 64;
  if constexpr (std::is_same<Acc, AccD>::value) {
    // split planes per launch row: about one full wave of workgroups (two
    // fit per CU at this kernel's register use) counting one tile pair per
    // filter (the tile pairs are sized for the rank capacity, and those
    // beyond a filter's own rank exit at once), within [GM_YMIN, GM_YMAX];
    // every result bit is the same whatever the row holds
    int cus = 0;
    TT_TRY(device_cus(&cus));
    const int rows = std::min(GM_YMAX, std::max(GM_YMIN, (2 * cus + B - 1) / B));
    hipLaunchKernelGGL((gram_mfma_kernel<T, F>), dim3(t * (t + 1) / 2, std::min(smax, rows), B), dim3(256), 0, st, f);
  } else {
    if (Mcap > 32)
      hipLaunchKernelGGL((gram_partial_kernel<T, Acc, 64, F>), dim3(t * (t + 1) / 2, smax, B), dim3(256), 0, st, f);
    else
      hipLaunchKernelGGL((gram_partial_kernel<T, Acc, 32, F>), dim3(1, smax, B), dim3(256), 0, st, f);
  }
  TTG_LAUNCH_CHECK("gram_partial_kernel");
  const long long mm = (long long)Mcap * Mcap;
  hipLaunchKernelGGL((gram_reduce_kernel<Acc, F>), dim3(stride_grid(cdiv(mm, 256), B), 1, B), dim3(256), 0, st, f);
  TTG_LAUNCH_CHECK("gram_reduce_kernel");
  return TT_OK;
}

// FP32 products run on the matrix cores (for every shape, so a filter's
// result does not depend on its batch); 128 x 32 tiles when no filter has
// more than 32 columns
template <typename TA, typename TB, typename F>
static tt_status launch_gemm_mfma(F f, int B, long long Mcap, long long Ncap, hipStream_t st) {
  if (Ncap <= 32) {
    const long long tiles = std::max(1, cdiv(Mcap, 128));
    hipLaunchKernelGGL((gemm_mfma_kernel<TA, TB, 32, F>), dim3(stride_grid(tiles, B, 16384), 1, B), dim3(256), 0, st,
                       f);
  } else {
    const long long tiles = (long long)std::max(1, cdiv(Mcap, 64)) * std::max(1, cdiv(Ncap, 64));
    hipLaunchKernelGGL((gemm_mfma_kernel<TA, TB, 64, F>), dim3(stride_grid(tiles, B, 16384), 1, B), dim3(256), 0, st,
                       f);
  }
  TTG_LAUNCH_CHECK("gemm_mfma_kernel");
  return TT_OK;
}

template <typename TA, typename TB, typename TC, typename TAcc, typename F>
static tt_status launch_gemm(F f, int B, long long Mcap, long long Ncap, hipStream_t st) {
  ProfScope ps_(PC_GEMM, st);
  if constexpr (std::is_same<TC, float>::value) return launch_gemm_mfma<TA, TB>(f, B, Mcap, Ncap, st);
  const int tm = std::max(1, cdiv(Mcap, 64)), tn = std::max(1, cdiv(Ncap, 64));
  hipLaunchKernelGGL((gemm_kernel<TA, TB, TC, TAcc, F>), dim3(tn, tm, B), dim3(256), 0, st, f);
  TTG_LAUNCH_CHECK("gemm_kernel");
  return TT_OK;
}

// A (bulk) x B (FP64, N <= 128) for very tall A
template <typename T, typename F>
static tt_status launch_tall(F f, int B, long long Mcap, int Ncap, hipStream_t st) {
  ProfScope ps_(PC_GEMM, st);
  if constexpr (std::is_same<T, float>::value) return launch_gemm_mfma<float, double>(f, B, Mcap, Ncap, st);
  if (Ncap > 256) {
    set_error("tall GEMM: N capacity %d > 256", Ncap);
    return TT_ERR_SHAPE;
  }
  int G = 1;  // column groups of 32, a power of two so that 256 / G is exact
  while (32 * G < Ncap) G *= 2;
  const int RW = 256 / G;  // smallest row block any filter can use
  // LDS for the largest row block (G = 1) or the widest B slice (G = Gmax)
  const size_t smem = std::max((size_t)256 * (TSK_KC + 1) + (size_t)TSK_KC * 32,
                               (size_t)RW * (TSK_KC + 1) + (size_t)TSK_KC * 32 * G) * sizeof(T);
  if (smem > 48 * 1024)
    HIP_TRY(hipFuncSetAttribute((const void*)tall_gemm_kernel<T, F>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)smem),
            "tall gemm smem attribute");
  hipLaunchKernelGGL((tall_gemm_kernel<T, F>), dim3(stride_grid(cdiv(Mcap, RW), B), 1, B), dim3(256), smem, st, f,
                     G);
  TTG_LAUNCH_CHECK("tall_gemm_kernel");
  return TT_OK;
}

// the fused FFT prediction of interior core k (see fft.h)
// prediction inside the filter step: 0 direct fused (default), 1 FFT fused,
// 2 materialised product + tall GEMM
static int g_predict_mode = 0;

// Fibres per workgroup of the MFMA prediction (BB), picked by
// tt_autotune_prediction per launch shape; BB only regroups work, every
// output element sums the same terms in the same order whatever BB is.
struct TuneKey {
  int f64, B, hmax, nmax, pcap, kcap;
  bool operator==(const TuneKey& o) const {
    return f64 == o.f64 && B == o.B && hmax == o.hmax && nmax == o.nmax && pcap == o.pcap && kcap == o.kcap;
  }
};
static std::vector<std::pair<TuneKey, int>> g_tuned_bb;
static int g_force_bb = 0;       // candidate under test (0: none)
static TuneKey g_last_key{};     // shape of the last MFMA prediction launch
static bool g_have_key = false;

static int pred_bb(const TuneKey& key, int B) {
  g_last_key = key;
  g_have_key = true;
  if (g_force_bb) return g_force_bb;
  for (const auto& e : g_tuned_bb)
    if (e.first == key) return e.second;
  return B >= 64 ? 16 : 2;
}

template <typename T>
static size_t direct_smem(int hmax, int nmax, int pcap, int kcap) {
  const int taps = 2 * hmax + 1;
  const int taps_pad = (taps + DF_TB - 1) / DF_TB * DF_TB;
  const int plen = DF_TB + nmax + 2 * hmax + 4 + DF_TB;
  size_t most = 0;
  for (int jc = 8; jc <= DF_JC; jc *= 2)  // every column chunk the kernel may pick
    most = std::max(most, (size_t)taps_pad * pcap * jc + (size_t)(DF_JC / jc) * plen * (pcap + 1));
  return (most + (size_t)taps * kcap) * sizeof(T);
}

// Work model of the direct fused prediction for one filter and core: the
// contraction over taps and the next bond (2 flops per multiply-add) and the
// V = K x L product, each counted once; bytes = read P_k, K_k and L (FP64),
// write Z_k once.
template <typename T>
__global__ void __launch_bounds__(256) pred_work_kernel(FFused<T> fn, int B, double* work) {
  __shared__ double red[4];
  double fl = 0.0, by = 0.0;
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    FArgs<T> g;
    if (!fn(b, g)) continue;
    const double taps = 2.0 * g.hk + 1.0;
    const double out = (double)g.rk0 * g.rp0 * g.n * g.N;
    fl += 2.0 * out * taps * g.rp1 + 2.0 * g.rk0 * taps * g.rp1 * g.N * g.rk1;
    by += sizeof(T) * (out + (double)g.rp0 * g.n * g.rp1 + (double)g.rk0 * taps * g.rk1) +
          8.0 * g.rk1 * g.rp1 * g.N;
  }
  fl = block_sum(fl, red);
  by = block_sum(by, red);
  if (threadIdx.x == 0) {
    work[2 * PC_PRED] += fl;
    work[2 * PC_PRED + 1] += by;
  }
}

// the direct prediction runs on the matrix cores unless mode 3 asks for the
// vector-ALU kernel or the MFMA kernel's LDS would not fit.  The choice
// depends on the launch's capacities only, never on the batch size.
template <typename T>
static int use_mfma_pred(int hmax, int nmax, int pcap, int kcap) {
  return g_predict_mode != 3 ? mfma_pred_variant<T>(hmax, nmax, pcap, kcap) : 0;
}

template <typename T>
static tt_status launch_direct(const RCtx& c, int B, int hmax, int kcap, int nmax, int pcap, int ncap,
                               hipStream_t st) {
  ProfScope ps_(PC_PRED, st);
  FFused<T> f{c};
  if (const int var = use_mfma_pred<T>(hmax, nmax, pcap, kcap)) {
    const bool big = var == 2;
    const size_t ms = mfma_pred_smem<T>(hmax, nmax, pcap, kcap, big);
    const void* kfn = big ? (const void*)mfma_pred_kernel<T, FFused<T>, true>
                          : (const void*)mfma_pred_kernel<T, FFused<T>, false>;
    if (ms > 48 * 1024)
      HIP_TRY(hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)ms),
              "mfma prediction smem");
    const int BB = pred_bb(TuneKey{sizeof(T) == 8 ? 1 : 0, B, hmax, nmax, pcap, kcap}, B);
    const int grid = kcap * ((pcap + BB - 1) / BB);
    if (big)
      hipLaunchKernelGGL((mfma_pred_kernel<T, FFused<T>, true>), dim3(std::max(1, grid), 1, B), dim3(MP_NT_BIG), ms,
                         st, f, BB);
    else
      hipLaunchKernelGGL((mfma_pred_kernel<T, FFused<T>, false>), dim3(std::max(1, grid), 1, B), dim3(256), ms, st,
                         f, BB);
    TTG_LAUNCH_CHECK("mfma_pred_kernel");
    if (g_work && (g_prof_mask & (1 << PC_PRED))) {
      hipLaunchKernelGGL((pred_work_kernel<T>), dim3(1), dim3(256), 0, st, f, B, g_work);
      TTG_LAUNCH_CHECK("pred_work_kernel");
    }
    return TT_OK;
  }
  const size_t smem = direct_smem<T>(hmax, nmax, pcap, kcap);
  if (smem > 160 * 1024) {
    set_error("direct prediction: %zu bytes of LDS needed", smem);
    return TT_ERR_SHAPE;
  }
  if (smem > 48 * 1024)
    HIP_TRY(hipFuncSetAttribute((const void*)direct_pred_kernel<T, FFused<T>>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem),
            "direct smem");
  const int BB = B >= 64 ? 4 : 1;
  const int grid = kcap * ((pcap + BB - 1) / BB) * ((ncap + DF_JC - 1) / DF_JC);
  hipLaunchKernelGGL((direct_pred_kernel<T, FFused<T>>), dim3(std::max(1, grid), 1, B), dim3(256), smem, st, f, BB);
  TTG_LAUNCH_CHECK("direct_pred_kernel");
  if (g_work && (g_prof_mask & (1 << PC_PRED))) {
    hipLaunchKernelGGL((pred_work_kernel<T>), dim3(1), dim3(256), 0, st, f, B, g_work);
    TTG_LAUNCH_CHECK("pred_work_kernel");
  }
  return TT_OK;
}

template <typename T>
constexpr int fused_cols() {
  return sizeof(T) == 4 ? 2 : 1;  // output columns per workgroup
}

template <typename T>
static size_t fused_smem(int L, int kcap, int nmax, int pcap) {
  using C = typename Cpx<T>::t;
  const int NC = fused_cols<T>();
  const int pm = (kcap + 1) / 2;
  const size_t nw = (size_t)L / 2 + 1;
  const size_t bsz = std::max((size_t)pm * L, (size_t)kcap * nw);
  return ((size_t)L / 2 + (size_t)FP_WCH * kcap * kcap + NC * (2 * bsz + (size_t)kcap * nw)) * sizeof(C) +
         (size_t)NC * ((size_t)nmax * pcap + (size_t)kcap * pcap) * sizeof(T);
}

template <typename T>
static tt_status launch_fused(const RCtx& c, int B, int Lmax, int kcap, int nmax, int pcap, int ncolcap,
                              hipStream_t st) {
  ProfScope ps_(PC_PRED, st);
  constexpr int NC = fused_cols<T>();
  FFused<T> f{c};
  const size_t smem = fused_smem<T>(Lmax, kcap, nmax, pcap);
  if (smem > 160 * 1024) {
    set_error("fused prediction: %zu bytes of LDS needed", smem);
    return TT_ERR_SHAPE;
  }
  if (smem > 48 * 1024)
    HIP_TRY(hipFuncSetAttribute((const void*)fused_pred_kernel<T, NC, FFused<T>>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem),
            "fused smem");
  hipLaunchKernelGGL((fused_pred_kernel<T, NC, FFused<T>>), dim3(std::max(1, cdiv(ncolcap, NC)), 1, B), dim3(256),
                     smem, st, f);
  TTG_LAUNCH_CHECK("fused_pred_kernel");
  return TT_OK;
}

// Jacobi columns in LDS up to rows*cols <= 16384 doubles (128 KB)
static const int JAC_LDS_DOUBLES = 16384;

template <typename F>
static tt_status launch_jacobi(F f, int B, hipStream_t st, int lds_doubles = JAC_LDS_DOUBLES) {
  ProfScope ps_(PC_JACOBI, st);
  const size_t smem = (size_t)lds_doubles * sizeof(double);
  HIP_TRY(hipFuncSetAttribute((const void*)jacobi_kernel<F>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem),
          "jacobi smem attribute");
  hipLaunchKernelGGL((jacobi_kernel<F>), dim3(B), dim3(512), smem, st, f, lds_doubles);
  TTG_LAUNCH_CHECK("jacobi_kernel");
  return TT_OK;
}

template <typename TZ, typename TQ, typename F>
static tt_status launch_trsm(F f, int B, long long mcap, int rcap, hipStream_t st) {
  ProfScope ps_(PC_TRSM, st);
  if constexpr (sizeof(TQ) == 4) {
    // FP32 bulk: explicit inverse of the pivot block (in LDS when it fits),
    // then one thread per column
    const size_t lb = (size_t)rcap * rcap * sizeof(double);
    if (lb > 160 * 1024) {
      hipLaunchKernelGGL((tri_inverse_kernel<F, false>), dim3(1, 1, B), dim3(256), 0, st, f);
    } else {
      if (lb > 48 * 1024)
        HIP_TRY(hipFuncSetAttribute((const void*)tri_inverse_kernel<F, true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lb),
                "tri inverse smem");
      hipLaunchKernelGGL((tri_inverse_kernel<F, true>), dim3(1, 1, B), dim3(256), lb, st, f);
    }
    TTG_LAUNCH_CHECK("tri_inverse_kernel");
    hipLaunchKernelGGL((tri_apply_kernel<TZ, TQ, F>), dim3(stride_grid(cdiv(mcap, 256), B), 1, B), dim3(256), 0,
                       st, f);
    TTG_LAUNCH_CHECK("tri_apply_kernel");
    return TT_OK;
  }
  if constexpr (sizeof(TQ) == 8) {
    hipLaunchKernelGGL((trsm_f64_kernel<TZ, F>), dim3(stride_grid(cdiv(mcap, 256), B), 1, B), dim3(256), 0, st, f);
    TTG_LAUNCH_CHECK("trsm_f64_kernel");
    return TT_OK;
  }
  const size_t qbytes = (size_t)rcap * 64 * sizeof(double);
  const size_t lbytes = (size_t)rcap * rcap * sizeof(double);
  const int l_in_lds = (qbytes + lbytes <= 150 * 1024) ? 1 : 0;
  const size_t smem = qbytes + (l_in_lds ? lbytes : 0);
  if (smem > 48 * 1024)
    HIP_TRY(hipFuncSetAttribute((const void*)trsm_kernel<TZ, TQ, F>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem),
            "trsm smem attribute");
  hipLaunchKernelGGL((trsm_kernel<TZ, TQ, F>), dim3(stride_grid(cdiv(mcap, 64), B), 1, B), dim3(64), smem, st,
                     f, rcap, l_in_lds);
  TTG_LAUNCH_CHECK("trsm_kernel");
  return TT_OK;
}

// The launch sequence of one batched rounding.  Shapes come from device
// ranks; `sh` only bounds the grids.
struct FusedLaunch {
  const DevTT* Kn = nullptr;
  const DevTT* Pn = nullptr;
  const FusedPred* FP = nullptr;
  int Lmax = 0, kcap = 1, pcap = 1, nmax = 1, hmax = 0;
  int mode = 0;  // 0 direct, 1 FFT
};

// Record of the right-to-left sweep for the rounding adjoint, written after
// the pivoted Cholesky of bond k: the Gram (FP64 high words) and the FP64
// factor, rows in the original order, compacted to leading dimension r_k
// (n_0 for a bond 1 folded with core 0: the Gram of the folded unfolding),
// the factor's columns beyond its rank zeroed.  The folded bond is recorded
// only when its pivoted Cholesky could reach full rank (n_0 <= rqcap[1]), as
// the adjoint's own does.  One workgroup per filter.
__global__ void __launch_bounds__(256) round_tape_kernel(const DevTT* __restrict__ din,
                                                         const RoundScratch* __restrict__ drs, int k,
                                                         const tt_round_tape* __restrict__ tapes) {
  const int f = blockIdx.x;
  const DevTT& X = din[f];
  const RoundScratch& s = drs[f];
  const tt_round_tape& t = tapes[f];
  const bool mg = k == 1 && merge_bond1(X, s);
  if (mg && X.n[0] > s.rqcap[1]) {
    if (threadIdx.x == 0) t.valid[1] = 0;
    return;
  }
  const int R = mg ? X.n[0] : s.ri[k], rank = s.rq[k], gc = s.gcap;
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    const int i = e / R, j = e - (e / R) * R;
    t.g[k][e] = s.gram[2LL * ((long long)i * gc + j)];
    t.f[k][e] = j < rank ? s.lfac[(long long)i * gc + j] : 0.0;
  }
  if (threadIdx.x == 0) {
    t.valid[k] = mg ? 2 : 1;
    t.rank[k] = rank;
  }
}

// Record of the left-to-right step k: the Jacobi singular vectors (column c
// = vector c, rq[k+1] components in the coordinates of the bond-(k+1)
// factor) and values of B_k, compacted to r_{k+1} x r_{k+1} column-major,
// zeros beyond the pivoted-Cholesky rank; not for a first core folded into
// bond 1.  One workgroup per filter.
__global__ void __launch_bounds__(256) round_tape_svd_kernel(const DevTT* __restrict__ din,
                                                             const RoundScratch* __restrict__ drs, int k,
                                                             const tt_round_tape* __restrict__ tapes) {
  const int f = blockIdx.x;
  const RoundScratch& s = drs[f];
  const tt_round_tape& t = tapes[f];
  if (k == 0 && merge_bond1(din[f], s)) return;  // the folded first core: its adjoint works from S_0
  const int R = s.ri[k + 1], rq = s.rq[k + 1], nc = s.misc[0], gc = s.gcap;
  double* v = t.v[k + 1];
  double* sg = t.s[k + 1];
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    const int c = e / R, j = e - (e / R) * R;
    v[e] = (c < nc && j < rq) ? s.usv[(long long)c * gc + j] : 0.0;
  }
  for (int c = threadIdx.x; c < R; c += blockDim.x) sg[c] = c < nc ? s.sigma[c] : 0.0;
  if (threadIdx.x == 0) t.valid[k + 1] |= 4;
}

template <typename T, typename Acc>
static tt_status round_launch(const RoundShape& sh, const RoundBufs& rb, double eps, int max_rank,
                              hipStream_t st, const FusedLaunch* fl = nullptr, const int* forced = nullptr,
                              long long fstride = 0, const tt_round_tape* dtape = nullptr) {
  const int B = sh.B, d = sh.d;
  const bool f64 = sizeof(T) == 8;
  const double tau2_rl = f64 ? 1e-30 : 1e-14;
  const double tau2_lr = f64 ? 1e-31 : 1e-16;
  RCtx c{rb.din, rb.dout, rb.drs, 0, d, 0.0, (int)sizeof(T), sh.merge ? 1 : 0};
  if (fl) {
    c.Kn = fl->Kn;
    c.Pn = fl->Pn;
    c.FP = fl->FP;
    c.fused = 1;
    c.zt = fl->mode == 1 ? 1 : 0;
  }
  hipLaunchKernelGGL(round_init_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, rb.din, rb.dout, rb.drs, B);
  TTG_LAUNCH_CHECK("round_init_kernel");
  if (d == 1) {
    // a single core: nothing to truncate; copy when not in place is handled by
    // the caller (d == 1 is rejected there)
    return TT_OK;
  }
  // ---- right-to-left orthogonalisation with pre-truncation -------------
  for (int k = d - 1; k >= 1; --k) {
    c.k = k;
    if (k < d - 1) {
      if (fl && fl->mode == 1) {
        TT_TRY(launch_fused<T>(c, B, fl->Lmax, fl->kcap, fl->nmax, fl->pcap, fl->pcap * sh.rq[k + 1], st));
      } else if (fl) {
        TT_TRY(launch_direct<T>(c, B, fl->hmax, fl->kcap, fl->nmax, fl->pcap, sh.rq[k + 1], st));
      } else {
        TT_TRY((launch_tall<T>(FRlAbsorb<T>{c}, B, (long long)sh.rin[k] * sh.n[k], sh.rq[k + 1], st)));
      }
    }
    const bool mg = sh.merge && k == 1;  // some filter may fold core 0 into this step
    if (mg) TT_TRY((launch_gemm<T, T, T, T>(FRlMerge<T>{c}, B, sh.n[0], (long long)sh.n[1] * sh.rq[2], st)));
    c.tau2 = tau2_rl;
    // the pre-truncation to rqcap ranks fails only when it drops more than
    // (1% of the rounding's tolerance)^2 of ||X||^2 (the result then still
    // meets eps); at eps = 0 any drop above the precision's level fails
    c.tau2_flag = (0.01 * eps) * (0.01 * eps);
    const int mcap = (k == 1) ? std::min(sh.rin[1], std::max(sh.n[0], 1)) : sh.rin[k];
    TT_TRY((launch_gram<T, Acc>(FRlGram<T>{c}, B, mcap, (long long)sh.n[k] * sh.rq[k + 1], sh.splits, st)));
    TT_TRY((launch_pchol<Acc>(FRlPchol{c}, B, sh.gcap, st)));
    if (dtape) {
      hipLaunchKernelGGL(round_tape_kernel, dim3(B), dim3(256), 0, st, rb.din, rb.drs, k, dtape);
      TTG_LAUNCH_CHECK("round_tape_kernel");
    }
    TT_TRY((launch_trsm<T, T>(FRlTrsm<T>{c}, B, (long long)sh.n[k] * sh.rq[k + 1], sh.rq[k], st)));
  }
  c.k = 0;
  if (sh.merge) {
    hipLaunchKernelGGL((first_core_copy_kernel<T>), dim3(B), dim3(256), 0, st, rb.din, rb.drs);
    TTG_LAUNCH_CHECK("first_core_copy_kernel");
  }
  TT_TRY((launch_tall<T>(FRlAbsorb<T>{c}, B, (long long)sh.n[0], sh.rq[1], st)));
  hipLaunchKernelGGL((round_norm_kernel<T>), dim3(B), dim3(256), 0, st, rb.din, rb.drs, eps);
  TTG_LAUNCH_CHECK("round_norm_kernel");
  // ---- left-to-right truncation ------------------------------------------
  for (int k = 0; k <= d - 2; ++k) {
    c.k = k;
    if (k >= 1) {
      TT_TRY((launch_gemm<double, T, T, T>(FLrB<T>{c}, B, sh.rout[k], (long long)sh.n[k] * sh.rq[k + 1], st)));
    }
    c.tau2 = tau2_lr;
    TT_TRY((launch_gram<T, Acc>(FLrGram<T>{c}, B, sh.rq[k + 1], (long long)sh.rout[k] * sh.n[k], sh.splits, st)));
    TT_TRY((launch_pchol<Acc>(FLrPchol{c}, B, sh.gcap, st)));
    TT_TRY((launch_jacobi(FLrJacobi{c}, B, st)));
    if (dtape) {
      hipLaunchKernelGGL(round_tape_svd_kernel, dim3(B), dim3(256), 0, st, rb.din, rb.drs, k, dtape);
      TTG_LAUNCH_CHECK("round_tape_svd_kernel");
    }
    hipLaunchKernelGGL(round_select_kernel, dim3(B), dim3(256), 0, st, rb.dout, rb.drs, k, max_rank, forced, fstride);
    TTG_LAUNCH_CHECK("round_select_kernel");
    TT_TRY((launch_tall<T>(FLrU<T>{c}, B, (long long)sh.rout[k] * sh.n[k], sh.rout[k + 1], st)));
  }
  c.k = d - 1;
  TT_TRY((launch_gemm<double, T, T, T>(FLrB<T>{c}, B, sh.rout[d - 1], (long long)sh.n[d - 1], st)));
  hipLaunchKernelGGL((balance_kernel<T>), dim3(B), dim3(256), 0, st, rb.dout);
  TTG_LAUNCH_CHECK("balance_kernel");
  return TT_OK;
}

// host-side shape maxima and scratch planning for a batch of roundings
static void round_shape(int B, const std::vector<DevTT>& in, const std::vector<DevTT>& out, bool f64,
                        RoundShape& sh) {
  sh.B = B;
  sh.d = in[0].d;
  sh.f64 = f64;
  int gcap = 1;
  for (int b = 0; b < B; ++b) {
    const int rqmax = rq_limit(f64, out[b].cap, out[b].d);
    for (int j = 0; j <= sh.d; ++j) {
      sh.rin[j] = std::max(sh.rin[j], in[b].cap[j]);
      sh.rout[j] = std::max(sh.rout[j], out[b].cap[j]);
      const int rq = (j == 0 || j == sh.d) ? 1 : std::min(in[b].cap[j], rqmax);
      sh.rq[j] = std::max(sh.rq[j], rq);
    }
    for (int k = 0; k < sh.d; ++k) sh.n[k] = std::max(sh.n[k], in[b].n[k]);
    if (in[b].cap[1] > in[b].n[0]) sh.merge = true;
  }
  for (int j = 1; j < sh.d; ++j) {
    gcap = std::max(gcap, j == 1 ? std::min(sh.rin[1], sh.n[0]) : sh.rin[j]);
    gcap = std::max(gcap, sh.rq[j]);
  }
  sh.gcap = gcap;
  // split-K planes: enough workgroups for small batches
  int pairs = gram_tiles(gcap);
  long long Tmax = 0;
  for (int k = 0; k < sh.d; ++k)
    Tmax = std::max(Tmax, (long long)sh.n[k] * std::max(sh.rq[k + 1], sh.rout[k]));
  (void)pairs;
  (void)Tmax;
  sh.splits = GRAM_PLANES;
}

}  // namespace ttg

using namespace ttg;

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

size_t tt_train_elems(int32_t d, const int32_t* n, const int32_t* cap) {
  if (d < 1 || d > TT_MAXD || !n || !cap) return 0;
  return elems_of(d, n, cap);
}

const char* tt_last_error(void) { return g_err; }

const char* tt_version(void) { return "ttgbf 0.1 gfx950"; }

// ---------------------------------------------------------------------------
// tt_round
// ---------------------------------------------------------------------------
static tt_status round_plan(int32_t batch, const tt_train* t_in, const tt_train* t_out, Arena& ar,
                            RoundShape& sh, RoundBufs& rb, std::vector<DevTT>& vin,
                            std::vector<DevTT>& vout, std::vector<RoundScratch>& vrs) {
  if (batch < 1) {
    set_error("batch must be >= 1");
    return TT_ERR_ARG;
  }
  const int dtype = t_in[0].dtype;
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_train(&t_in[b], "t_in", dtype));
    TT_TRY(check_train(&t_out[b], "t_out", dtype));
    if (t_in[b].d != t_in[0].d || t_out[b].d != t_in[0].d) {
      set_error("all TTs of a batch must share d");
      return TT_ERR_SHAPE;
    }
    if (t_in[0].d < 2) {
      set_error("rounding needs d >= 2");
      return TT_ERR_SHAPE;
    }
    for (int k = 0; k < t_in[b].d; ++k)
      if (t_in[b].n[k] != t_out[b].n[k]) {
        set_error("t_in and t_out mode sizes differ");
        return TT_ERR_SHAPE;
      }
  }
  const bool f64 = dtype == TT_F64;
  vin.resize(batch);
  vout.resize(batch);
  vrs.resize(batch);
  for (int b = 0; b < batch; ++b) {
    vin[b] = make_dev(t_in[b]);
    vout[b] = make_dev(t_out[b]);
  }
  round_shape(batch, vin, vout, f64, sh);
  if (sh.gcap > 1024) {
    set_error("tt_round: rank capacity %d exceeds 1024", sh.gcap);
    return TT_ERR_SHAPE;
  }
  rb.din = ar.take<DevTT>(batch);
  rb.dout = ar.take<DevTT>(batch);
  rb.drs = ar.take<RoundScratch>(batch);
  for (int b = 0; b < batch; ++b) plan_round_scratch(ar, vin[b], vout[b], f64, sh.gcap, sh.splits, vrs[b]);
  return TT_OK;
}

size_t tt_round_workspace(int32_t batch, const tt_train* t_in, const tt_train* t_out) {
  if (batch < 1 || !t_in || !t_out) return 0;
  Arena ar(nullptr, 0);
  RoundShape sh;
  RoundBufs rb;
  std::vector<DevTT> a, b;
  std::vector<RoundScratch> r;
  if (round_plan(batch, t_in, t_out, ar, sh, rb, a, b, r) != TT_OK) return 0;
  ar.take<tt_round_tape>(batch);  // the record table of tt_round_taped
  return ar.used + 256;
}

tt_status tt_round_taped(int32_t batch, const tt_train* t_in, const tt_train* t_out, double eps, int32_t max_rank,
                         const tt_round_tape* tape, void* ws, size_t ws_bytes, void* stream) {
  if (!t_in || !t_out || !ws || !tape) {
    set_error("tt_round_taped: null argument");
    return TT_ERR_ARG;
  }
  if (!(eps >= 0.0) || max_rank < 1) {
    set_error("tt_round_taped: need eps >= 0 and max_rank >= 1");
    return TT_ERR_ARG;
  }
  for (int b = 0; b < batch; ++b) {
    if (t_in[b].dtype != TT_F64 || t_out[b].dtype != TT_F64) {
      set_error("tt_round_taped: FP64 trains only");
      return TT_ERR_ARG;
    }
    if (!tape[b].valid || !tape[b].rank) {
      set_error("tt_round_taped: null valid or rank array (filter %d)", b);
      return TT_ERR_ARG;
    }
    for (int j = 1; j < t_in[b].d; ++j)
      if (!tape[b].g[j] || !tape[b].f[j] || !tape[b].v[j] || !tape[b].s[j]) {
        set_error("tt_round_taped: null record buffer (filter %d, bond %d)", b, j);
        return TT_ERR_ARG;
      }
  }
  Arena ar(ws, ws_bytes);
  RoundShape sh;
  RoundBufs rb;
  std::vector<DevTT> vin, vout;
  std::vector<RoundScratch> vrs;
  TT_TRY(round_plan(batch, t_in, t_out, ar, sh, rb, vin, vout, vrs));
  tt_round_tape* dtape = ar.take<tt_round_tape>(batch);
  if (!ar.fits()) {
    set_error("tt_round_taped: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(rb.din, vin, st));
  TT_TRY(upload(rb.dout, vout, st));
  TT_TRY(upload(rb.drs, vrs, st));
  std::vector<tt_round_tape> vt(tape, tape + batch);
  TT_TRY(upload(dtape, vt, st));
  return round_launch<double, AccDD>(sh, rb, eps, max_rank, st, nullptr, nullptr, 0, dtape);
}

tt_status tt_round(int32_t batch, const tt_train* t_in, const tt_train* t_out, double eps, int32_t max_rank,
                   void* ws, size_t ws_bytes, void* stream) {
  if (!t_in || !t_out || !ws) {
    set_error("tt_round: null argument");
    return TT_ERR_ARG;
  }
  if (!(eps >= 0.0) || max_rank < 1) {
    set_error("tt_round: need eps >= 0 and max_rank >= 1");
    return TT_ERR_ARG;
  }
  Arena ar(ws, ws_bytes);
  RoundShape sh;
  RoundBufs rb;
  std::vector<DevTT> vin, vout;
  std::vector<RoundScratch> vrs;
  TT_TRY(round_plan(batch, t_in, t_out, ar, sh, rb, vin, vout, vrs));
  if (!ar.fits()) {
    set_error("tt_round: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(rb.din, vin, st));
  TT_TRY(upload(rb.dout, vout, st));
  TT_TRY(upload(rb.drs, vrs, st));
  if (sh.f64) return round_launch<double, AccDD>(sh, rb, eps, max_rank, st);
  return round_launch<float, AccD>(sh, rb, eps, max_rank, st);
}

}  // extern "C"

namespace ttg {

// tt_round with the rank of every bond j forced to forced[b * fstride + j]
// (device; rank replay, clamped to the numerical rank and the capacity like
// the rule)
static tt_status round_forced(int32_t batch, const tt_train* t_in, const tt_train* t_out, const int* forced,
                              long long fstride, void* ws, size_t ws_bytes, hipStream_t st) {
  Arena ar(ws, ws_bytes);
  RoundShape sh;
  RoundBufs rb;
  std::vector<DevTT> vin, vout;
  std::vector<RoundScratch> vrs;
  TT_TRY(round_plan(batch, t_in, t_out, ar, sh, rb, vin, vout, vrs));
  if (!ar.fits()) {
    set_error("tt_round (forced ranks): workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  TT_TRY(upload(rb.din, vin, st));
  TT_TRY(upload(rb.dout, vout, st));
  TT_TRY(upload(rb.drs, vrs, st));
  if (sh.f64) return round_launch<double, AccDD>(sh, rb, 0.0, 1 << 30, st, nullptr, forced, fstride);
  return round_launch<float, AccD>(sh, rb, 0.0, 1 << 30, st, nullptr, forced, fstride);
}

}  // namespace ttg

// ===========================================================================
// adjoint of the rounding (FP64): host orchestration of the phases described
// in round_adj.h; every shape is known on the host after one read of the
// ranks, so every product is a job of a grouped GEMM launch
// ===========================================================================
namespace ttg {

#define RADJ_PLANES 4
struct RadjCore {  // per filter and core k (0-based)
  double *G, *T, *W, *U, *c, *N, *lfac, *lwork, *gdd, *M, *jw, *sig, *usv, *Ud, *Fm, *Gbar, *D, *YBt, *vs, *js;
  double* fac;  // F_k used in the products: lfac, or the forward's recorded factor
  int* flag;
  int* piv;
  int* prank;
};

struct RadjFilter {
  int d, n[TT_MAXD], Ra[TT_MAXD + 1], ry[TT_MAXD + 1];
  RadjCore c[TT_MAXD];
  double *L, *kappa, *Lbar, *Wb0, *Wb1, *Nbar, *Ubar, *P1, *P2, *WG, *XtN, *XtNG, *Gs, *T2, *Tg, *one;
  // first core wider than its rows (Ra[1] > n[0], d >= 2): the SVD of M_0
  // from S_0 = M'_0 M'_0^T, M'_0 = A_0 x_3 Z_1 (n[0] x n[1] Ra[2])
  bool wide0;
  double *Mw, *sdd, *slw, *slf;
  double* Yw;  // V A_1 and (V A_1) x_3 G_1 for V = W_1, X^T N (four blocks of r_1 n_1 R_2)
  int *spiv, *srank;
};

// lays out the buffers of every filter in the arena (sizes from ranks Ra, ry)
static void radj_layout(Arena& ar, RadjFilter& F) {
  const int d = F.d;
  long long tmax = 1, pmax = 1, rmax = 1, Rmax = 1, prmax = 1, pRmax = 1, rRmax = 1;
  for (int k = 0; k < d; ++k) {
    const long long Rk = F.Ra[k], Rk1 = F.Ra[k + 1], rk = F.ry[k], rk1 = F.ry[k + 1], n = F.n[k];
    RadjCore& C = F.c[k];
    C.G = ar.take<double>(Rk1 * Rk1);
    C.Gbar = ar.take<double>(Rk1 * Rk1);
    C.lfac = ar.take<double>(Rk1 * Rk1);
    C.fac = C.lfac;
    C.lwork = ar.take<double>(2 * Rk1 * Rk1);
    C.piv = ar.take<int>(Rk1);
    C.prank = ar.take<int>(1);
    C.gdd = ar.take<double>(2 * RADJ_PLANES * Rk * Rk);  // double-double Gram planes of G_{k-1}
    C.W = ar.take<double>(std::max(1LL, rk * Rk));
    tmax = std::max(tmax, Rk * n * Rk1);
    rmax = std::max(rmax, std::max(rk, rk1));
    Rmax = std::max(Rmax, std::max(Rk, Rk1));
    if (k < d - 1) {
      const long long p = rk * n;
      pmax = std::max(pmax, p);
      prmax = std::max(prmax, p * rk1);
      pRmax = std::max(pRmax, p * Rk1);
      rRmax = std::max(rRmax, std::max(rk * Rk, rk1 * Rk1));
      const long long nd = std::max(0LL, Rk1 - rk1);
      C.U = ar.take<double>(p * rk1);
      C.c = ar.take<double>(1);
      C.N = ar.take<double>(p * Rk1);
      C.M = ar.take<double>(p * Rk1);
      C.D = ar.take<double>(rk1);
      C.YBt = ar.take<double>(p * rk1);
      C.jw = ar.take<double>(p * Rk1);
      C.sig = ar.take<double>(Rk1);
      C.usv = ar.take<double>(p * Rk1);
      C.Ud = ar.take<double>(std::max(1LL, p * nd));
      C.Fm = ar.take<double>(nd * rk1 + rk1);
      C.vs = ar.take<double>(Rk1 * Rk1);
      C.js = ar.take<double>(Rk1 * Rk1);
      C.flag = ar.take<int>(2);
    }
  }
  F.wide0 = d >= 2 && F.Ra[1] > F.n[0];
  if (F.wide0) {
    const long long n0 = F.n[0];
    F.Mw = ar.take<double>(n0 * F.n[1] * F.Ra[2]);
    F.sdd = ar.take<double>(2 * RADJ_PLANES * n0 * n0);
    F.slw = ar.take<double>(2 * n0 * n0);
    F.slf = ar.take<double>(n0 * n0);
    F.spiv = ar.take<int>(n0);
    F.srank = ar.take<int>(1);
    F.Yw = ar.take<double>(4LL * F.ry[1] * F.n[1] * F.Ra[2]);
  }
  const int rl = F.ry[d - 1], nl = F.n[d - 1];
  F.L = ar.take<double>((long long)rl * nl);
  F.Lbar = ar.take<double>((long long)rl * nl);
  F.kappa = ar.take<double>(1);
  F.Wb0 = ar.take<double>(rRmax);
  F.Wb1 = ar.take<double>(rRmax);
  F.Nbar = ar.take<double>(pRmax);
  F.Ubar = ar.take<double>(prmax);
  F.P1 = ar.take<double>(rmax * rmax);
  F.P2 = ar.take<double>(Rmax * rmax);
  F.WG = ar.take<double>(rmax * Rmax);
  F.XtN = ar.take<double>(rmax * Rmax);
  F.XtNG = ar.take<double>(rmax * Rmax);
  F.Gs = ar.take<double>(Rmax * Rmax);
  F.T2 = ar.take<double>(tmax);
  F.Tg = ar.take<double>(tmax);
  F.one = ar.take<double>(1);
}

struct RadjRun {
  hipStream_t st;
  GJob* dg;
  EJob* de;
  PcholArgs* dp;
  GramArgs* dga;
  AJob* daj;
  RkJacobi* drj;
  DJob* ddj;
  CondJacobi* dcj;
  RefJob* drf;
  int jcap;
  double* part = nullptr;  // partial products of split-K jobs
  long long part_cap = 0;
  std::vector<GJob> g;
  std::vector<EJob> e;
  template <typename T>
  tt_status up(T* dst, const std::vector<T>& v) const {
    return stage_upload(dst, v, st);
  }
  // device regions a job may touch (workspace, the trains' core buffers):
  // every job's extent is checked on the host before anything is launched
  std::vector<std::pair<const double*, long long>> regions;
  bool inside(const void* p, long long last) const {
    if (last < 0) return true;
    const double* q = reinterpret_cast<const double*>(p);
    for (const auto& r : regions)
      if (q >= r.first && q + last < r.first + r.second) return true;
    return false;
  }
  tt_status check(bool ok, const char* what) const {
    if (ok) return TT_OK;
    set_error("tt_round_adjoint: internal extent check failed (%s)", what);
    return TT_ERR_ARG;
  }
  tt_status gemm() {  // launch the queued products
    if (g.empty()) return TT_OK;
    if ((int)g.size() > jcap) {
      set_error("tt_round_adjoint: job table overflow");
      return TT_ERR_ARG;
    }
    for (const auto& j : g) {
      TT_TRY(check(j.K == 0 || inside(j.a, (long long)(j.M - 1) * j.sam + (long long)(j.K - 1) * j.sak), "gemm a"));
      TT_TRY(check(j.K == 0 || inside(j.b, (long long)(j.K - 1) * j.sbk + (long long)(j.N - 1) * j.sbn), "gemm b"));
      TT_TRY(check(inside(j.c, (long long)(j.M - 1) * j.scm + (long long)(j.N - 1) * j.scn), "gemm c"));
    }
    // long products with few output tiles split K over the partial-product
    // area (at most 32 slices of >= 1024, while the area lasts)
    long long avail = part_cap;
    double* pp = part;
    bool split = false;
    int tiles = 0, mx = 1;
    for (auto& j : g) {
      j.tn = std::max(1, (j.N + 63) / 64);
      j.ks = 1;
      j.kc = j.K;
      j.part = nullptr;
      const int tm = std::max(1, (j.M + 63) / 64);
      const long long mn = (long long)j.M * j.N;
      if (j.K >= 4096 && tm * j.tn <= 16 && mn > 0) {
        int ks = (int)std::min<long long>(std::min(32, j.K / 1024), avail / mn);
        if (ks >= 2) {
          const int kc = ((j.K + ks - 1) / ks + 31) / 32 * 32;
          ks = (j.K + kc - 1) / kc;
          j.ks = ks;
          j.kc = kc;
          j.part = pp;
          pp += ks * mn;
          avail -= ks * mn;
          split = true;
          mx = std::max(mx, cdiv(mn, 256));
        }
      }
      j.tile0 = tiles;
      tiles += tm * j.tn * j.ks;
    }
    for (const auto& j : g)
      if (j.ks > 1) TT_TRY(check(inside(j.part, (long long)j.ks * j.M * j.N - 1), "gemm partials"));
    static const bool trace = getenv("TTGBF_TRACE_GEMM") != nullptr;
    if (trace) {  // one line per launch: its distinct job shapes (M N K slices) and counts
      std::vector<std::pair<std::array<int, 4>, int>> shapes;
      for (const auto& j : g) {
        const std::array<int, 4> key{j.M, j.N, j.K, j.ks};
        bool found = false;
        for (auto& sh : shapes)
          if (sh.first == key) {
            ++sh.second;
            found = true;
          }
        if (!found) shapes.push_back({key, 1});
      }
      fprintf(stderr, "gjob tiles=%d", tiles);
      for (const auto& sh : shapes)
        fprintf(stderr, " [%dx%dx%d/%d]x%d", sh.first[0], sh.first[1], sh.first[2], sh.first[3], sh.second);
      fprintf(stderr, "\n");
    }
    TT_TRY(up(dg, g));
    hipLaunchKernelGGL(gjob_mfma_kernel, dim3(tiles), dim3(256), 0, st, dg, (int)g.size());
    TTG_LAUNCH_CHECK("gjob_mfma_kernel");
    if (split) {
      hipLaunchKernelGGL(gjob_reduce_kernel, dim3(std::min(mx, 1024), (int)g.size()), dim3(256), 0, st, dg);
      TTG_LAUNCH_CHECK("gjob_reduce_kernel");
    }
    g.clear();
    return TT_OK;
  }
  tt_status elem() {
    if (e.empty()) return TT_OK;
    if ((int)e.size() > jcap) {
      set_error("tt_round_adjoint: job table overflow");
      return TT_ERR_ARG;
    }
    for (const auto& j : e) {
      const long long n = j.op == EJ_SYM ? (long long)j.r * j.r : j.cnt;
      TT_TRY(check(inside(j.out, n - 1), "elementwise out"));
      if (j.op == EJ_SCALE || j.op == EJ_SYM) TT_TRY(check(inside(j.x, n - 1), "elementwise x"));
      if (j.op == EJ_DDHI) TT_TRY(check(inside(j.x, 2 * n - 1), "elementwise x"));
      if (j.op == EJ_COPY || j.op == EJ_ROWFLIP || j.op == EJ_COLDIV) TT_TRY(check(inside(j.x, n - 1), "elementwise x"));
      if (j.op == EJ_ROWFLIP || j.op == EJ_COLDIV)
        TT_TRY(check(j.ld > 0 && inside(j.y, (n - 1) / j.ld), "elementwise y"));
      if (j.op == EJ_SCALE) TT_TRY(check(inside(j.s, 0), "elementwise s"));
    }
    long long mx = 1;
    for (auto& j : e) mx = std::max(mx, j.cnt);
    TT_TRY(up(de, e));
    hipLaunchKernelGGL(ejob_kernel, dim3(std::min(cdiv(mx, 256), 1024), (int)e.size()), dim3(256), 0, st, de);
    TTG_LAUNCH_CHECK("ejob_kernel");
    e.clear();
    return TT_OK;
  }
  void mm(int M, int N, int K, const double* a, long long sam, long long sak, const double* b, long long sbk,
          long long sbn, double* c, long long scm, double alpha, double beta) {
    if (M <= 0 || N <= 0) return;
    GJob j;
    memset(&j, 0, sizeof(j));
    j.M = M;
    j.N = N;
    j.K = K;
    j.a = a;
    j.sam = sam;
    j.sak = sak;
    j.b = b;
    j.sbk = sbk;
    j.sbn = sbn;
    j.c = c;
    j.scm = scm;
    j.scn = 1;
    j.alpha = alpha;
    j.beta = beta;
    g.push_back(j);
  }
  void ej(int op, long long cnt, const double* x, const double* y, double* out, double* out2, const double* sc,
          int r = 0, int p = 0, int R = 0, int ld = 0) {
    EJob j;
    memset(&j, 0, sizeof(j));
    j.op = op;
    j.cnt = cnt;
    j.x = x;
    j.y = y;
    j.out = out;
    j.out2 = out2;
    j.s = sc;
    j.r = r;
    j.p = p;
    j.R = R;
    j.ld = ld;
    e.push_back(j);
  }
};

struct FAdjGram {
  const GramArgs* a;
  __device__ bool operator()(int b, GramArgs& g) const {
    g = a[b];
    return g.M > 0;
  }
};

static long long radj_bytes(const RadjFilter& proto) {
  RadjFilter F = proto;
  Arena ar(nullptr, 0);
  radj_layout(ar, F);
  return (long long)ar.used;
}

}  // namespace ttg

extern "C" {

// partial-product area of the split-K products, per filter (from the capacities)
static long long radj_part_elems(const tt_train& a) {
  long long rm = 1;
  for (int k = 0; k <= a.d; ++k) rm = std::max<long long>(rm, a.cap[k]);
  return std::min(8 * rm * rm, 1LL << 20);
}

size_t tt_round_adjoint_workspace(int32_t batch, const tt_train* a, const tt_train* y) {
  if (batch < 1 || !a || !y) return 0;
  const int dd = a[0].d;
  size_t total = (size_t)batch * (3 * dd + 8) *
                     (sizeof(GJob) + sizeof(EJob) + sizeof(PcholArgs) + sizeof(GramArgs) +
                      sizeof(AJob) + sizeof(RkJacobi) + sizeof(DJob) + sizeof(CondJacobi) + sizeof(RefJob)) +
                 8192;
  for (int b = 0; b < batch; ++b) {
    RadjFilter F;
    memset(&F, 0, sizeof(F));
    F.d = a[b].d;
    for (int k = 0; k < F.d; ++k) F.n[k] = a[b].n[k];
    for (int k = 0; k <= F.d; ++k) {
      F.Ra[k] = a[b].cap[k];
      F.ry[k] = y[b].cap[k];
    }
    total += (size_t)radj_bytes(F) + 256 * 64 + sizeof(double) * (size_t)radj_part_elems(a[b]);
  }
  return total;
}

tt_status tt_round_adjoint(int32_t batch, const tt_train* a, const tt_train* y, const tt_train* y_bar,
                           const tt_train* a_bar, const tt_round_tape* tape, void* ws, size_t ws_bytes,
                           void* stream) {
  if (batch < 1 || !a || !y || !y_bar || !a_bar || !ws) {
    set_error("tt_round_adjoint: bad arguments");
    return TT_ERR_ARG;
  }
  const int d = a[0].d;
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_train(&a[b], "a", TT_F64));
    TT_TRY(check_train(&y[b], "y", TT_F64));
    TT_TRY(check_train(&y_bar[b], "y_bar", TT_F64));
    TT_TRY(check_train(&a_bar[b], "a_bar", TT_F64));
    if (a[b].d != d || y[b].d != d || y_bar[b].d != d || a_bar[b].d != d) {
      set_error("tt_round_adjoint: d differs");
      return TT_ERR_SHAPE;
    }
    for (int k = 0; k < d; ++k)
      if (y[b].n[k] != a[b].n[k] || y_bar[b].n[k] != a[b].n[k] || a_bar[b].n[k] != a[b].n[k]) {
        set_error("tt_round_adjoint: mode sizes differ");
        return TT_ERR_SHAPE;
      }
    for (int k = 0; k <= d; ++k)
      if (y_bar[b].cap[k] != y[b].cap[k] || a_bar[b].cap[k] != a[b].cap[k]) {
        set_error("tt_round_adjoint: adjoint capacities differ from their primals");
        return TT_ERR_SHAPE;
      }
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  StageGuard stage(st);  // job tables go through page-locked staging (the call ends synchronised)
  // the ranks, once, to the host
  std::vector<int> hr((size_t)batch * 3 * (d + 1));
  for (int b = 0; b < batch; ++b) {
    HIP_TRY(hipMemcpyAsync(&hr[(size_t)(3 * b) * (d + 1)], a[b].ranks, sizeof(int) * (d + 1), hipMemcpyDeviceToHost,
                           st), "ranks");
    HIP_TRY(hipMemcpyAsync(&hr[(size_t)(3 * b + 1) * (d + 1)], y[b].ranks, sizeof(int) * (d + 1),
                           hipMemcpyDeviceToHost, st), "ranks");
    HIP_TRY(hipMemcpyAsync(&hr[(size_t)(3 * b + 2) * (d + 1)], y_bar[b].ranks, sizeof(int) * (d + 1),
                           hipMemcpyDeviceToHost, st), "ranks");
  }
  // bonds recorded by the forward (tt_round_taped)
  std::vector<int> hv(tape ? (size_t)batch * (d + 1) : 0, 0);
  if (tape)
    for (int b = 0; b < batch; ++b) {
      if (!tape[b].valid || !tape[b].rank) {
        set_error("tt_round_adjoint: tape without a valid or rank array (filter %d)", b);
        return TT_ERR_ARG;
      }
      HIP_TRY(hipMemcpyAsync(&hv[(size_t)b * (d + 1)], tape[b].valid, sizeof(int) * (d + 1), hipMemcpyDeviceToHost,
                             st), "tape flags");
    }
  HIP_TRY(hipStreamSynchronize(st), "ranks sync");
  auto taped = [&](int b, int j) { return tape && j >= 1 && j < d && (hv[(size_t)b * (d + 1) + j] & 1); };
  std::vector<RadjFilter> F(batch);
  Arena ar(ws, ws_bytes);
  RadjRun R;
  R.st = st;
  R.jcap = batch * (3 * d + 8);
  R.dg = ar.take<GJob>(R.jcap);
  R.de = ar.take<EJob>(R.jcap);
  R.dp = ar.take<PcholArgs>((size_t)batch * d);
  R.dga = ar.take<GramArgs>((size_t)batch);
  R.daj = ar.take<AJob>((size_t)batch);
  R.drj = ar.take<RkJacobi>((size_t)batch);
  R.ddj = ar.take<DJob>((size_t)batch);
  R.dcj = ar.take<CondJacobi>((size_t)batch);
  R.drf = ar.take<RefJob>((size_t)batch);
  int Rmax = 1;
  for (int b = 0; b < batch; ++b) {
    RadjFilter& f = F[b];
    memset(&f, 0, sizeof(f));
    f.d = d;
    for (int k = 0; k < d; ++k) f.n[k] = a[b].n[k];
    const int* ra = &hr[(size_t)(3 * b) * (d + 1)];
    const int* ry = &hr[(size_t)(3 * b + 1) * (d + 1)];
    const int* rb = &hr[(size_t)(3 * b + 2) * (d + 1)];
    for (int k = 0; k <= d; ++k) {
      if (ra[k] < 1 || ra[k] > a[b].cap[k] || ry[k] < 1 || ry[k] > y[b].cap[k] || rb[k] != ry[k]) {
        set_error("tt_round_adjoint: ranks out of range or y_bar ranks differ from y (filter %d)", b);
        return TT_ERR_SHAPE;
      }
      if (k > 0 && k < d && ry[k] > ra[k]) {
        set_error("tt_round_adjoint: output rank above the input rank (filter %d)", b);
        return TT_ERR_SHAPE;
      }
      f.Ra[k] = ra[k];
      f.ry[k] = ry[k];
      Rmax = std::max(Rmax, ra[k]);
    }
    radj_layout(ar, f);
  }
  for (int b = 0; b < batch; ++b) R.part_cap += radj_part_elems(a[b]);
  R.part = ar.take<double>(R.part_cap);
  if (!ar.fits()) {
    set_error("tt_round_adjoint: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  R.regions.push_back({reinterpret_cast<const double*>(ws), (long long)(ar.used / sizeof(double))});
  for (int b = 0; b < batch; ++b)
    for (const tt_train* t : {&a[b], &y[b], &y_bar[b], &a_bar[b]})
      R.regions.push_back({reinterpret_cast<const double*>(t->cores), (long long)elems_of(t->d, t->n, t->cap)});
  // the folded first bond: the Gram of n0 x (n1 r2) unfolding A_0 Z_1 and its factor
  auto taped_s0 = [&](int b) { return tape && F[b].wide0 && (hv[(size_t)b * (d + 1) + 1] & 2); };
  // the SVD of a tall unfolding M_k = N_k F_k, recorded by the forward in the
  // coordinates of F_k (so only where F_k itself is the recorded factor)
  auto taped_svd = [&](int b, int k) {
    return k + 1 < d && !(k == 0 && F[b].wide0) && taped(b, k + 1) && (hv[(size_t)b * (d + 1) + k + 1] & 4);
  };
  for (int b = 0; b < batch; ++b)
    if (taped_s0(b)) {
      if (!tape[b].g[1] || !tape[b].f[1]) {
        set_error("tt_round_adjoint: null record buffer (filter %d, bond 1)", b);
        return TT_ERR_ARG;
      }
      const long long c1 = std::min(a[b].cap[1], a[b].n[0]);
      R.regions.push_back({tape[b].f[1], c1 * c1});
    }
  for (int b = 0; b < batch; ++b)
    for (int j = 1; j < d; ++j)
      if (taped(b, j)) {
        if (!tape[b].g[j] || !tape[b].f[j]) {
          set_error("tt_round_adjoint: null record buffer (filter %d, bond %d)", b, j);
          return TT_ERR_ARG;
        }
        const long long cj = j == 1 ? std::min(a[b].cap[1], a[b].n[0]) : a[b].cap[j];
        const long long c2 = cj * cj;
        R.regions.push_back({tape[b].g[j], c2});
        R.regions.push_back({tape[b].f[j], c2});
        if (taped_svd(b, j - 1)) {
          if (!tape[b].v[j] || !tape[b].s[j]) {
            set_error("tt_round_adjoint: null singular-vector record (filter %d, bond %d)", b, j);
            return TT_ERR_ARG;
          }
          R.regions.push_back({tape[b].v[j], c2});
          R.regions.push_back({tape[b].s[j], cj});
        }
        F[b].c[j - 1].G = tape[b].g[j];    // G of bond j, leading dimension r_j
        F[b].c[j - 1].fac = tape[b].f[j];  // its factor
      }
  auto check_scalar_jobs = [&](int kind) -> tt_status {
    for (const auto& j : R.e) {
      if (kind == 0) {  // radj_scalar_kernel
        TT_TRY(R.check(R.inside(j.x, j.cnt - 1) && R.inside(j.out2, 0), "scalar x"));
        TT_TRY(R.check(j.op == 0 ? R.inside(j.out, j.cnt - 1) : R.inside(j.y, j.cnt - 1), "scalar out"));
      } else if (kind == 1) {  // eigprep
        const long long nd = j.R - j.r;
        TT_TRY(R.check(j.R >= j.r && R.inside(j.x, j.R - 1) && R.inside(j.y, (long long)j.R * j.ld - 1) &&
                           j.ld >= j.p && R.inside(j.out, (long long)j.p * nd - 1) &&
                           R.inside(j.out2, nd * j.r + j.r - 1),
                       "eigprep"));
      } else {  // eigapply
        const long long nd = j.R - j.r;
        TT_TRY(R.check(R.inside(j.out, (long long)j.p * j.r - 1) && R.inside(j.out2, nd * j.r - 1) &&
                           R.inside(j.y, nd * j.r - 1) && R.inside(j.s, j.r - 1),
                       "eigapply"));
      }
    }
    return TT_OK;
  };
  auto acore = [&](int b, int k) { return reinterpret_cast<const double*>(a[b].cores) + make_dev(a[b]).off[k]; };
  auto ycore = [&](int b, int k) { return reinterpret_cast<const double*>(y[b].cores) + make_dev(y[b]).off[k]; };
  auto ybcore = [&](int b, int k) {
    return reinterpret_cast<const double*>(y_bar[b].cores) + make_dev(y_bar[b]).off[k];
  };
  auto abcore = [&](int b, int k) { return reinterpret_cast<double*>(a_bar[b].cores) + make_dev(a_bar[b]).off[k]; };
  auto ywblk = [&](const RadjFilter& f, int v) { return f.Yw + (long long)v * f.ry[1] * f.n[1] * f.Ra[2]; };
  // zero accumulators and factors; G_{d-1} = 1, W_0 = 1
  for (int b = 0; b < batch; ++b) {
    RadjFilter& f = F[b];
    for (int k = 0; k < d; ++k) {
      const long long asz = (long long)f.Ra[k] * f.n[k] * f.Ra[k + 1];
      R.ej(EJ_FILL, asz, nullptr, nullptr, abcore(b, k), nullptr, nullptr);
      R.ej(EJ_FILL, (long long)f.Ra[k + 1] * f.Ra[k + 1], nullptr, nullptr, f.c[k].Gbar, nullptr, nullptr);
      R.ej(EJ_FILL, (long long)f.Ra[k + 1] * f.Ra[k + 1], nullptr, nullptr, f.c[k].lfac, nullptr, nullptr);
    }
    R.ej(EJ_ONE, 1, nullptr, nullptr, f.c[d - 1].G, nullptr, nullptr);
    R.ej(EJ_ONE, 1, nullptr, nullptr, f.c[0].W, nullptr, nullptr);
    R.ej(EJ_ONE, 1, nullptr, nullptr, f.one, nullptr, nullptr);
    TT_TRY(R.elem());
  }
  // phase 1: right-part Grams and their factors, from the right: with
  // G_k = F_k F_k^T, Z_k = A_k x_3 F_k and G_{k-1} = Z_k Z_k^T accumulated in
  // double-double (the forward rounding's accuracy), F_{k-1} by pivoted
  // Cholesky of G_{k-1}; G_{k-1} in FP64 for the products below
  for (int b = 0; b < batch; ++b) {
    RadjFilter& f = F[b];
    R.ej(EJ_ONE, 1, nullptr, nullptr, f.c[d - 1].lfac, nullptr, nullptr);
  }
  TT_TRY(R.elem());
  for (int k = d - 1; k >= 1; --k) {
    int mcap = 1;
    long long tcap = 1;
    std::vector<GramArgs> gj;
    std::vector<PcholArgs> pj;
    for (int b = 0; b < batch; ++b) {
      RadjFilter& f = F[b];
      const int R0 = f.Ra[k], R1 = f.Ra[k + 1], n = f.n[k];
      const bool rec = taped(b, k);  // G_{k-1} and F_{k-1} recorded by the forward
      // a folded first bond needs neither G_0 nor F_0 (phase 4 applies G_0
      // through A_1 and G_1); Z_1 only feeds S_0 when that was not recorded
      const bool w1 = k == 1 && f.wide0;
      if (!rec && !(w1 && taped_s0(b))) R.mm(R0 * n, R1, R1, acore(b, k), R1, 1, f.c[k].fac, R1, 1, f.Tg, R1, 1.0, 0.0);
      GramArgs ga;
      memset(&ga, 0, sizeof(ga));
      ga.M = R0;
      ga.T = n * R1;
      ga.x = f.Tg;
      ga.sa = (long long)n * R1;
      ga.st = 1;
      ga.out = f.c[k].gdd;
      ga.gcap = R0;
      ga.splits = RADJ_PLANES;
      if (rec || w1) ga.M = 0;
      gj.push_back(ga);
      TT_TRY(R.check(R.inside(f.c[k].gdd, 2LL * RADJ_PLANES * R0 * R0 - 1) &&
                         R.inside(f.Tg, (long long)R0 * n * R1 - 1),
                     "gram"));
      PcholArgs pa;
      memset(&pa, 0, sizeof(pa));
      pa.M = R0;
      pa.g = f.c[k].gdd;
      pa.lwork = f.c[k - 1].lwork;
      pa.lfac = f.c[k - 1].lfac;
      pa.piv = f.c[k - 1].piv;
      pa.rank_out = f.c[k - 1].prank;
      pa.gcap = R0;
      pa.rmax = R0;
      pa.tau2 = RADJ_PCHOL_TAU2;
      if (k == 1 && f.wide0) pa.M = 0;  // F_0 is not needed: M_0's SVD comes from S_0
      if (rec) pa.M = 0;
      pj.push_back(pa);
      if (!w1) mcap = std::max(mcap, R0);  // (a folded first bond has no Gram here)
      tcap = std::max(tcap, (long long)n * R1);
    }
    TT_TRY(R.gemm());
    TT_TRY(R.up(R.dga, gj));
    TT_TRY((launch_gram<double, AccDD>(FAdjGram{R.dga}, batch, mcap, tcap, RADJ_PLANES, st)));
    TT_TRY(R.up(R.dp, pj));
    TT_TRY((launch_pchol<AccDD, FAdjPchol>(FAdjPchol{R.dp}, batch, mcap, st)));
    for (int b = 0; b < batch; ++b) {
      RadjFilter& f = F[b];
      const int R0 = f.Ra[k];
      if (!taped(b, k) && !(k == 1 && f.wide0))
        R.ej(EJ_DDHI, (long long)R0 * R0, f.c[k].gdd, nullptr, f.c[k - 1].G, nullptr, nullptr);
    }
    TT_TRY(R.elem());
  }
  // the forward's scaled kept vectors U_fwd = Y_k / c_k (compared with the
  // adjoint's own below)
  for (int b = 0; b < batch; ++b) {
    RadjFilter& f = F[b];
    for (int k = 0; k < d - 1; ++k)
      R.ej(0, (long long)f.ry[k] * f.n[k] * f.ry[k + 1], ycore(b, k), nullptr, f.c[k].U, f.c[k].c, nullptr,
           f.ry[k + 1]);
  }
  if (!R.e.empty()) {
    TT_TRY(check_scalar_jobs(0));
    TT_TRY(R.up(R.de, R.e));
    hipLaunchKernelGGL(radj_scalar_kernel, dim3((int)R.e.size()), dim3(256), 0, st, R.de);
    TTG_LAUNCH_CHECK("radj_scalar_kernel");
    R.e.clear();
  }
  // phase 2/3, core by core: N_k = W_k x_1 A_k, M_k = N_k F_k and its
  // Jacobi SVD; the kept vectors of that SVD (signs matched to the forward's
  // output) become U_k, and W_{k+1} = U_k^T N_k
  int gmax = 1;  // the largest Gram of these phases (n[0] for a folded first bond)
  for (int b = 0; b < batch; ++b)
    for (int k = 0; k < d; ++k) gmax = std::max(gmax, (k == 0 && F[b].wide0) ? F[b].n[0] : F[b].Ra[k + 1]);
  if (gmax > 1024) {
    set_error("tt_round_adjoint: rank above 1024");
    return TT_ERR_SHAPE;
  }
  for (int k = 0; k < d - 1; ++k) {
    for (int b = 0; b < batch; ++b) {
      RadjFilter& f = F[b];
      const int R0 = f.Ra[k], R1 = f.Ra[k + 1], n = f.n[k], r0 = f.ry[k];
      R.mm(r0, n * R1, R0, f.c[k].W, R0, 1, acore(b, k), (long long)n * R1, 1, f.c[k].N, (long long)n * R1, 1.0, 0.0);
    }
    TT_TRY(R.gemm());
    for (int b = 0; b < batch; ++b) {
      RadjFilter& f = F[b];
      const int R1 = f.Ra[k + 1], p = f.ry[k] * f.n[k];
      if (k == 0 && f.wide0) {
        // M'_0 = A_0 Z_1 (Z_1 = A_1 x_3 F_1 is left in Tg by the right sweep)
        const long long T = (long long)f.n[1] * f.Ra[2];
        if (!taped_s0(b)) R.mm(f.n[0], (int)T, f.Ra[1], acore(b, 0), f.Ra[1], 1, f.Tg, T, 1, f.Mw, T, 1.0, 0.0);
        continue;
      }
      R.mm(p, R1, R1, f.c[k].N, R1, 1, f.c[k].fac, R1, 1, f.c[k].M, R1, 1.0, 0.0);
    }
    TT_TRY(R.gemm());
    // The SVD of M_k from a double-double Gram, its pivoted Cholesky factor C
    // (pre-truncated far below the singular values the adjoint resolves) and
    // the one-sided Jacobi SVD of C.  Tall M_k (p >= R1): Gram M_k^T M_k, the
    // Jacobi vectors are the right singular vectors v_c and the columns
    // sigma_c u_c = M_k v_c follow by one product.  Wide first core: Gram
    // S_0 = M'_0 M'_0^T, the Jacobi vectors are the left singular vectors.
    {
      int mcap = 1;
      long long tcap = 1;
      std::vector<GramArgs> gj(batch);
      std::vector<PcholArgs> pj(batch);
      std::vector<RkJacobi> rj(batch);
      for (int b = 0; b < batch; ++b) {
        RadjFilter& f = F[b];
        memset(&gj[b], 0, sizeof(GramArgs));
        memset(&pj[b], 0, sizeof(PcholArgs));
        memset(&rj[b], 0, sizeof(RkJacobi));
        const int R1 = f.Ra[k + 1], p = f.ry[k] * f.n[k];
        const bool wide = k == 0 && f.wide0;
        const int gm = wide ? f.n[0] : R1;                       // Gram dimension
        const long long T = wide ? (long long)f.n[1] * f.Ra[2] : p;  // summation length
        double* gout = wide ? f.sdd : f.c[k + 1].gdd;
        double* lw = wide ? f.slw : f.c[k].lwork;
        double* lf = wide ? f.slf : f.c[k].lfac;
        int* pv = wide ? f.spiv : f.c[k].piv;
        int* rk = wide ? f.srank : f.c[k].prank;
        double* jv = wide ? f.c[0].usv : f.c[k].vs;
        double* jwk = wide ? f.c[0].jw : f.c[k].js;
        const bool rsvd = taped_svd(b, k);
        if (rsvd) {  // V and sigma from the forward's record; no Gram, factor or Jacobi here
          R.ej(EJ_COPY, R1, tape[b].s[k + 1], nullptr, f.c[k].sig, nullptr, nullptr);
          R.ej(EJ_COPY, (long long)gm * gm, tape[b].v[k + 1], nullptr, jv, nullptr, nullptr);
        } else {
          R.ej(EJ_FILL, R1, nullptr, nullptr, f.c[k].sig, nullptr, nullptr);
          R.ej(EJ_FILL, (long long)gm * gm, nullptr, nullptr, jv, nullptr, nullptr);
        }
        GramArgs& ga = gj[b];
        ga.M = gm;
        ga.T = (int)T;
        ga.x = wide ? f.Mw : f.c[k].M;
        ga.sa = wide ? T : 1;
        ga.st = wide ? 1 : R1;
        ga.out = gout;
        ga.gcap = gm;
        ga.splits = RADJ_PLANES;
        PcholArgs& pa = pj[b];
        pa.M = gm;
        pa.g = gout;
        pa.lwork = lw;
        pa.lfac = lf;
        pa.piv = pv;
        pa.rank_out = rk;
        pa.gcap = gm;
        pa.rmax = gm;
        pa.tau2 = RADJ_PCHOL_TAU2;
        JacobiArgs& ja = rj[b].ja;
        ja.rows = gm;
        ja.ncols = gm;
        ja.tol2 = 1e-30;
        ja.x = lf;
        ja.ldx = gm;
        ja.work = jwk;
        ja.sigma = f.c[k].sig;
        ja.usv = jv;
        ja.gcap = gm;
        rj[b].ncols = rk;
        if (rsvd) {
          ga.M = 0;
          pa.M = 0;
          rj[b].ja.rows = 0;
        }
        if (wide && taped_s0(b)) {  // S_0's factor and rank from the forward's record
          ga.M = 0;
          pa.M = 0;
          R.ej(EJ_COPY, (long long)gm * gm, tape[b].f[1], nullptr, lf, nullptr, nullptr);
          rj[b].ncols = tape[b].rank + 1;
        }
        TT_TRY(R.check((wide ? (f.ry[0] == 1 && R1 > f.n[0]) : p >= 1) &&
                           R.inside(ga.x, wide ? (long long)gm * T - 1 : (long long)p * R1 - 1) &&
                           R.inside(gout, 2LL * RADJ_PLANES * gm * gm - 1) && R.inside(lw, 2LL * gm * gm - 1) &&
                           R.inside(lf, (long long)gm * gm - 1) && R.inside(jwk, (long long)gm * gm - 1) &&
                           R.inside(jv, (long long)gm * gm - 1) && R.inside(f.c[k].sig, R1 - 1) && gm <= R1,
                       "svd of M_k"));
        mcap = std::max(mcap, gm);
        tcap = std::max(tcap, T);
      }
      TT_TRY(R.elem());
      TT_TRY(R.up(R.dga, gj));
      TT_TRY((launch_gram<double, AccDD>(FAdjGram{R.dga}, batch, mcap, tcap, RADJ_PLANES, st)));
      TT_TRY(R.up(R.dp, pj));
      TT_TRY((launch_pchol<AccDD, FAdjPchol>(FAdjPchol{R.dp}, batch, mcap, st)));
      TT_TRY(R.up(R.drj, rj));
      TT_TRY(launch_jacobi(FAdjJacobiRk{R.drj}, batch, st));
      for (int b = 0; b < batch; ++b) {  // sigma_c u_c = M_k v_c (tall cores)
        RadjFilter& f = F[b];
        if (k == 0 && f.wide0) continue;
        const int R1 = f.Ra[k + 1], p = f.ry[k] * f.n[k];
        R.mm(R1, p, R1, f.c[k].vs, R1, 1, f.c[k].M, 1, R1, f.c[k].usv, p, 1.0, 0.0);
      }
      TT_TRY(R.gemm());
      for (int b = 0; b < batch; ++b) {
        RadjFilter& f = F[b];
        if (k == 0 && f.wide0) continue;
        const int R1 = f.Ra[k + 1], p = f.ry[k] * f.n[k];
        R.ej(EJ_COLDIV, (long long)p * R1, f.c[k].usv, f.c[k].sig, f.c[k].usv, nullptr, nullptr, 0, 0, 0, p);
      }
      TT_TRY(R.elem());
      // tall cores that kept a very small singular value: Mt = M_k V in
      // double-double (into jw), then one-sided Jacobi on Mt (M_k's buffer as
      // its scratch)
      std::vector<RefJob> rf(batch);
      std::vector<DJob> dj(batch);
      std::vector<CondJacobi> cj(batch);
      long long dmax = 1;
      for (int b = 0; b < batch; ++b) {
        RadjFilter& f = F[b];
        memset(&rf[b], 0, sizeof(RefJob));
        memset(&dj[b], 0, sizeof(DJob));
        memset(&cj[b], 0, sizeof(CondJacobi));
        if (k == 0 && f.wide0) continue;
        const int R1 = f.Ra[k + 1], p = f.ry[k] * f.n[k];
        rf[b].sig = f.c[k].sig;
        rf[b].r = f.ry[k + 1];
        rf[b].R = R1;
        rf[b].flag = f.c[k].flag;
        DJob& q = dj[b];
        q.vs = f.c[k].vs;
        q.M = f.c[k].M;
        q.sig = f.c[k].sig;
        q.usv = f.c[k].jw;
        q.flag = f.c[k].flag;
        q.p = p;
        q.R1 = R1;
        JacobiArgs& ja = cj[b].ja;
        ja.rows = p;
        ja.ncols = R1;
        ja.tol2 = 1e-30;
        ja.x = f.c[k].jw;
        ja.ldx = R1;
        ja.work = f.c[k].M;
        ja.sigma = f.c[k].sig;
        ja.usv = f.c[k].usv;
        ja.gcap = p;
        cj[b].flag = f.c[k].flag;
        TT_TRY(R.check(f.ry[k + 1] <= R1 && R.inside(q.M, (long long)p * R1 - 1) &&
                           R.inside(q.vs, (long long)R1 * R1 - 1) && R.inside(q.usv, (long long)R1 * p - 1) &&
                           R.inside(q.sig, R1 - 1) && R.inside(ja.work, (long long)R1 * p - 1) &&
                           R.inside(ja.usv, (long long)R1 * p - 1),
                       "refinement"));
        dmax = std::max(dmax, (long long)p * R1);
      }
      TT_TRY(R.up(R.drf, rf));
      hipLaunchKernelGGL(radj_refine_flag_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, R.drf, batch);
      TTG_LAUNCH_CHECK("radj_refine_flag_kernel");
      TT_TRY(R.up(R.ddj, dj));
      hipLaunchKernelGGL(radj_ddprod_kernel, dim3((int)std::min<long long>(cdiv(dmax, 256), 4096), batch), dim3(256),
                         0, st, R.ddj);
      TTG_LAUNCH_CHECK("radj_ddprod_kernel");
      TT_TRY(R.up(R.dcj, cj));
      TT_TRY(launch_jacobi(FAdjJacobiIf{R.dcj}, batch, st));
      hipLaunchKernelGGL(radj_refine_tail_kernel, dim3(batch), dim3(64), 0, st, R.drf, batch);
      TTG_LAUNCH_CHECK("radj_refine_tail_kernel");
    }
    std::vector<AJob> aj;
    for (int b = 0; b < batch; ++b) {
      RadjFilter& f = F[b];
      const int R1 = f.Ra[k + 1], r1 = f.ry[k + 1], p = f.ry[k] * f.n[k];
      AJob a1;
      memset(&a1, 0, sizeof(a1));
      a1.usv = f.c[k].usv;
      a1.sig = f.c[k].sig;
      a1.U = f.c[k].U;
      a1.ybt = f.c[k].YBt;
      a1.ybar = ybcore(b, k);
      a1.c = f.c[k].c;
      a1.dprev = k == 0 ? f.one : f.c[k - 1].D;
      a1.dk = f.c[k].D;
      a1.p = p;
      a1.r = r1;
      a1.n = f.n[k];
      a1.ldu = p;
      TT_TRY(R.check(r1 <= R1 && R.inside(a1.U, (long long)p * r1 - 1) && R.inside(a1.ybt, (long long)p * r1 - 1) &&
                         R.inside(a1.ybar, (long long)p * r1 - 1) && R.inside(a1.dk, r1 - 1) &&
                         R.inside(a1.dprev, f.ry[k] - 1),
                     "adopt"));
      aj.push_back(a1);
    }
    TT_TRY(R.up(R.daj, aj));
    hipLaunchKernelGGL(radj_adopt_kernel, dim3(batch), dim3(256), 0, st, R.daj);
    TTG_LAUNCH_CHECK("radj_adopt_kernel");
    for (int b = 0; b < batch; ++b) {
      RadjFilter& f = F[b];
      const int R1 = f.Ra[k + 1], r1 = f.ry[k + 1], p = f.ry[k] * f.n[k];
      R.mm(r1, R1, p, f.c[k].U, 1, r1, f.c[k].N, R1, 1, f.c[k + 1].W, R1, 1.0, 0.0);
    }
    TT_TRY(R.gemm());
  }
  // last core: L = W_{d-1} x_1 A_{d-1}; Y_{d-1} (left signs matched) = kappa L
  for (int b = 0; b < batch; ++b) {
    RadjFilter& f = F[b];
    const int R0 = f.Ra[d - 1], n = f.n[d - 1], r0 = f.ry[d - 1];
    R.mm(r0, n, R0, f.c[d - 1].W, R0, 1, acore(b, d - 1), n, 1, f.L, n, 1.0, 0.0);
  }
  TT_TRY(R.gemm());
  for (int b = 0; b < batch; ++b) {
    RadjFilter& f = F[b];
    const int n = f.n[d - 1], r0 = f.ry[d - 1];
    R.ej(EJ_ROWFLIP, (long long)r0 * n, ycore(b, d - 1), d > 1 ? f.c[d - 2].D : f.one, f.Lbar, nullptr, nullptr,
         0, 0, 0, n);
  }
  TT_TRY(R.elem());
  for (int b = 0; b < batch; ++b) {
    RadjFilter& f = F[b];
    R.ej(1, (long long)f.ry[d - 1] * f.n[d - 1], f.Lbar, f.L, nullptr, f.kappa, nullptr);
  }
  TT_TRY(check_scalar_jobs(0));
  TT_TRY(R.up(R.de, R.e));
  hipLaunchKernelGGL(radj_scalar_kernel, dim3((int)R.e.size()), dim3(256), 0, st, R.de);
  TTG_LAUNCH_CHECK("radj_scalar_kernel");
  R.e.clear();
  for (int b = 0; b < batch; ++b) {
    RadjFilter& f = F[b];
    const int n = f.n[d - 1], r0 = f.ry[d - 1];
    R.ej(EJ_ROWFLIP, (long long)r0 * n, ybcore(b, d - 1), d > 1 ? f.c[d - 2].D : f.one, f.Lbar, nullptr, nullptr,
         0, 0, 0, n);
  }
  TT_TRY(R.elem());
  for (int b = 0; b < batch; ++b) {
    RadjFilter& f = F[b];
    R.ej(EJ_SCALE, (long long)f.ry[d - 1] * f.n[d - 1], f.Lbar, nullptr, f.Lbar, nullptr, f.kappa);
  }
  TT_TRY(R.elem());
  // eigen data of every core for the backward sweep
  if (d > 1) {
    for (int b = 0; b < batch; ++b) {
      RadjFilter& f = F[b];
      for (int k = 0; k < d - 1; ++k) {
        const int R1 = f.Ra[k + 1], r1 = f.ry[k + 1], p = f.ry[k] * f.n[k];
        R.ej(0, 0, f.c[k].sig, f.c[k].usv, f.c[k].Ud, f.c[k].Fm, nullptr, r1, p, R1, p);
      }
    }
    TT_TRY(check_scalar_jobs(1));
    TT_TRY(R.up(R.de, R.e));
    hipLaunchKernelGGL(radj_eigprep_kernel, dim3((int)R.e.size()), dim3(256), 0, st, R.de);
    TTG_LAUNCH_CHECK("radj_eigprep_kernel");
    R.e.clear();
  }
  // phase 4: the left-to-right sweep backwards
  for (int b = 0; b < batch; ++b) {
    RadjFilter& f = F[b];
    const int R0 = f.Ra[d - 1], n = f.n[d - 1], r0 = f.ry[d - 1];
    // Wbar_{d-1} = Lbar A_{d-1}^T, Abar_{d-1} += W_{d-1}^T Lbar
    R.mm(r0, R0, n, f.Lbar, n, 1, acore(b, d - 1), 1, n, f.Wb0, R0, 1.0, 0.0);
    R.mm(R0, n, r0, f.c[d - 1].W, 1, R0, f.Lbar, n, 1, abcore(b, d - 1), n, 1.0, 1.0);
  }
  TT_TRY(R.gemm());
  bool cur0 = true;  // Wbar_{k+1} lives in Wb0 when true
  for (int k = d - 2; k >= 0; --k) {
    auto wb_in = [&](RadjFilter& f) { return cur0 ? f.Wb0 : f.Wb1; };
    auto wb_out = [&](RadjFilter& f) { return cur0 ? f.Wb1 : f.Wb0; };
    for (int b = 0; b < batch; ++b) {
      RadjFilter& f = F[b];
      const int R1 = f.Ra[k + 1], r1 = f.ry[k + 1], p = f.ry[k] * f.n[k];
      R.mm(p, R1, r1, f.c[k].U, r1, 1, wb_in(f), R1, 1, f.Nbar, R1, 1.0, 0.0);
      R.ej(EJ_COPY, (long long)p * r1, f.c[k].YBt, nullptr, f.Ubar, nullptr, nullptr);
    }
    TT_TRY(R.gemm());
    TT_TRY(R.elem());
    for (int b = 0; b < batch; ++b) {  // Ubar += N W_bar^T
      RadjFilter& f = F[b];
      const int R1 = f.Ra[k + 1], r1 = f.ry[k + 1], p = f.ry[k] * f.n[k];
      R.mm(p, r1, R1, f.c[k].N, R1, 1, wb_in(f), 1, R1, f.Ubar, r1, 1.0, 1.0);
    }
    TT_TRY(R.gemm());
    for (int b = 0; b < batch; ++b) {  // P1 = U^T Ubar, P2 = Ud^T Ubar
      RadjFilter& f = F[b];
      const int R1 = f.Ra[k + 1], r1 = f.ry[k + 1], p = f.ry[k] * f.n[k], nd = R1 - r1;
      R.mm(r1, r1, p, f.c[k].U, 1, r1, f.Ubar, r1, 1, f.P1, r1, 1.0, 0.0);
      R.mm(nd, r1, p, f.c[k].Ud, 1, nd, f.Ubar, r1, 1, f.P2, r1, 1.0, 0.0);
    }
    TT_TRY(R.gemm());
    for (int b = 0; b < batch; ++b) {  // Ubar -= U P1
      RadjFilter& f = F[b];
      const int r1 = f.ry[k + 1], p = f.ry[k] * f.n[k];
      R.mm(p, r1, r1, f.c[k].U, r1, 1, f.P1, r1, 1, f.Ubar, r1, -1.0, 1.0);
    }
    TT_TRY(R.gemm());
    for (int b = 0; b < batch; ++b) {  // X = Ubar diag(linv), P2 = P2 o Fm
      RadjFilter& f = F[b];
      const int R1 = f.Ra[k + 1], r1 = f.ry[k + 1], p = f.ry[k] * f.n[k], nd = R1 - r1;
      R.ej(0, 0, nullptr, f.c[k].Fm, f.Ubar, f.P2, f.c[k].Fm + (long long)nd * r1, r1, p, R1, 0);
    }
    {
      long long mx = 1;
      for (auto& j : R.e) mx = std::max(mx, (long long)j.p * j.r + (long long)(j.R - j.r) * j.r);
      TT_TRY(check_scalar_jobs(2));
      TT_TRY(R.up(R.de, R.e));
      hipLaunchKernelGGL(radj_eigapply_kernel, dim3(std::min(cdiv(mx, 256), 1024), (int)R.e.size()), dim3(256), 0, st,
                         R.de);
      TTG_LAUNCH_CHECK("radj_eigapply_kernel");
      R.e.clear();
    }
    for (int b = 0; b < batch; ++b) {  // X += Ud P2
      RadjFilter& f = F[b];
      const int R1 = f.Ra[k + 1], r1 = f.ry[k + 1], p = f.ry[k] * f.n[k], nd = R1 - r1;
      R.mm(p, r1, nd, f.c[k].Ud, nd, 1, f.P2, r1, 1, f.Ubar, r1, 1.0, 1.0);
    }
    TT_TRY(R.gemm());
    for (int b = 0; b < batch; ++b) {  // WG = W_{k+1} G_k, XtN = X^T N
      RadjFilter& f = F[b];
      const int R1 = f.Ra[k + 1], r1 = f.ry[k + 1], p = f.ry[k] * f.n[k];
      if (!(k == 0 && f.wide0)) R.mm(r1, R1, R1, f.c[k + 1].W, R1, 1, f.c[k].G, R1, 1, f.WG, R1, 1.0, 0.0);
      R.mm(r1, R1, p, f.Ubar, 1, r1, f.c[k].N, R1, 1, f.XtN, R1, 1.0, 0.0);
    }
    TT_TRY(R.gemm());
    if (k == 0) {
      // folded first bond: V G_0 = sum_i (V A_1(:,i,:)) G_1 A_1(:,i,:)^T for
      // V = W_1 and X^T N (G_0 itself is never formed); Y_V = V A_1 and
      // Y'_V = Y_V x_3 G_1 stay in Yw for the Gram recursion below
      for (int b = 0; b < batch; ++b) {
        RadjFilter& f = F[b];
        if (!f.wide0) continue;
        const int R1 = f.Ra[1], r1 = f.ry[1], T = f.n[1] * f.Ra[2];
        for (int v = 0; v < 2; ++v)
          R.mm(r1, T, R1, v == 0 ? f.c[1].W : f.XtN, R1, 1, acore(b, 1), T, 1, ywblk(f, v), T, 1.0, 0.0);
      }
      TT_TRY(R.gemm());
      for (int b = 0; b < batch; ++b) {
        RadjFilter& f = F[b];
        if (!f.wide0) continue;
        const int r1 = f.ry[1], R2 = f.Ra[2];
        for (int v = 0; v < 2; ++v)
          R.mm(r1 * f.n[1], R2, R2, ywblk(f, v), R2, 1, f.c[1].G, R2, 1, ywblk(f, 2 + v), R2, 1.0, 0.0);
      }
      TT_TRY(R.gemm());
      for (int b = 0; b < batch; ++b) {
        RadjFilter& f = F[b];
        if (!f.wide0) continue;
        const int R1 = f.Ra[1], r1 = f.ry[1], T = f.n[1] * f.Ra[2];
        for (int v = 0; v < 2; ++v)
          R.mm(r1, R1, T, ywblk(f, 2 + v), T, 1, acore(b, 1), 1, T, v == 0 ? f.WG : f.XtNG, R1, 1.0, 0.0);
      }
      TT_TRY(R.gemm());
    }
    for (int b = 0; b < batch; ++b) {  // XtNG = XtN G, Nbar += X WG, Gbar_k += XtN^T W_{k+1}
      RadjFilter& f = F[b];
      const int R1 = f.Ra[k + 1], r1 = f.ry[k + 1], p = f.ry[k] * f.n[k];
      if (!(k == 0 && f.wide0)) R.mm(r1, R1, R1, f.XtN, R1, 1, f.c[k].G, R1, 1, f.XtNG, R1, 1.0, 0.0);
      R.mm(p, R1, r1, f.Ubar, r1, 1, f.WG, R1, 1, f.Nbar, R1, 1.0, 1.0);
      R.mm(R1, R1, r1, f.XtN, 1, R1, f.c[k + 1].W, R1, 1, f.c[k].Gbar, R1, 1.0, 1.0);
    }
    TT_TRY(R.gemm());
    for (int b = 0; b < batch; ++b) {  // Nbar += U XtNG
      RadjFilter& f = F[b];
      const int R1 = f.Ra[k + 1], r1 = f.ry[k + 1], p = f.ry[k] * f.n[k];
      R.mm(p, R1, r1, f.c[k].U, r1, 1, f.XtNG, R1, 1, f.Nbar, R1, 1.0, 1.0);
    }
    TT_TRY(R.gemm());
    for (int b = 0; b < batch; ++b) {  // Wbar_k = Nbar A_k^T, Abar_k += W_k^T Nbar
      RadjFilter& f = F[b];
      const int R0 = f.Ra[k], R1 = f.Ra[k + 1], n = f.n[k], r0 = f.ry[k];
      R.mm(r0, R0, n * R1, f.Nbar, (long long)n * R1, 1, acore(b, k), 1, (long long)n * R1, wb_out(f), R0, 1.0, 0.0);
      R.mm(R0, n * R1, r0, f.c[k].W, 1, R0, f.Nbar, (long long)n * R1, 1, abcore(b, k), (long long)n * R1, 1.0, 1.0);
    }
    TT_TRY(R.gemm());
    cur0 = !cur0;
  }
  // phase 5: the Gram recursion backwards, from the left.  Every Gram is
  // symmetric, so only the symmetric part of its adjoint reaches the input
  // (the next step reads Gbar_k through Gbar_k + Gbar_k^T, and sum_i
  // A_i^T S A_i is antisymmetric for antisymmetric S): Gbar_k takes
  // (1/2) A_k^T (Gbar_{k-1} + Gbar_{k-1}^T) A_k, which reuses the product
  // of the A_k adjoint instead of forming Gbar_{k-1} A_k
  for (int k = 1; k < d; ++k) {
    for (int b = 0; b < batch; ++b) {
      RadjFilter& f = F[b];
      const int R0 = f.Ra[k];
      R.ej(EJ_SYM, (long long)R0 * R0, f.c[k - 1].Gbar, nullptr, f.Gs, nullptr, nullptr, R0);
    }
    TT_TRY(R.elem());
    for (int b = 0; b < batch; ++b) {
      RadjFilter& f = F[b];
      if (k == 1 && f.wide0) continue;
      const int R0 = f.Ra[k], R1 = f.Ra[k + 1], n = f.n[k];
      R.mm(R0, n * R1, R0, f.Gs, R0, 1, acore(b, k), (long long)n * R1, 1, f.Tg, (long long)n * R1, 1.0, 0.0);
    }
    TT_TRY(R.gemm());
    for (int b = 0; b < batch; ++b) {
      RadjFilter& f = F[b];
      if (k == 1 && f.wide0) continue;
      const int R0 = f.Ra[k], R1 = f.Ra[k + 1], n = f.n[k];
      R.mm(R0 * n, R1, R1, f.Tg, R1, 1, f.c[k].G, R1, 1, abcore(b, k), R1, 1.0, 1.0);
      if (k < d - 1) R.mm(R1, R1, R0 * n, acore(b, k), 1, R1, f.Tg, R1, 1, f.c[k].Gbar, R1, 0.5, 1.0);
    }
    TT_TRY(R.gemm());
    if (k == 1) {
      // folded first bond: Gbar_0 = (X^T N)^T W_1 comes from the backward
      // sweep alone, so Gs A_1 = (X^T N)^T Y_W + W_1^T Y_X has rank 2 r_1:
      //   Abar_1 += (X^T N)^T Y'_W + W_1^T Y'_X,
      //   Gbar_1 += (Y_X^T Y_W + Y_W^T Y_X) / 2  (summed over the mode index)
      for (int v = 0; v < 2; ++v) {
        for (int b = 0; b < batch; ++b) {
          RadjFilter& f = F[b];
          if (!f.wide0) continue;
          const int R1 = f.Ra[1], r1 = f.ry[1], R2 = f.Ra[2], T = f.n[1] * R2;
          R.mm(R1, T, r1, v == 0 ? f.XtN : f.c[1].W, 1, R1, ywblk(f, 2 + v), T, 1, abcore(b, 1), T, 1.0, 1.0);
          if (d > 2)
            R.mm(R2, R2, r1 * f.n[1], ywblk(f, 1 - v), 1, R2, ywblk(f, v), R2, 1, f.c[1].Gbar, R2, 0.5, 1.0);
        }
        TT_TRY(R.gemm());
      }
    }
  }
  // the adjoint train: ranks of a, log-scale adjoint of y_bar, status 0
  for (int b = 0; b < batch; ++b) {
    HIP_TRY(hipMemcpyAsync(a_bar[b].ranks, &hr[(size_t)(3 * b) * (d + 1)], sizeof(int) * (d + 1),
                           hipMemcpyHostToDevice, st), "a_bar ranks");
    HIP_TRY(hipMemcpyAsync(a_bar[b].log_scale, y_bar[b].log_scale, sizeof(double), hipMemcpyDeviceToDevice, st),
            "a_bar log_scale");
    HIP_TRY(hipMemsetAsync(a_bar[b].status, 0, sizeof(int), st), "a_bar status");
  }
  HIP_TRY(hipStreamSynchronize(st), "tt_round_adjoint");
  return TT_OK;
}

}  // extern "C"

// ===========================================================================
// likelihood SVD, kernel TT-SVD helpers
// ===========================================================================
namespace ttg {

// Likelihood rank rule: smallest r with sqrt(resid + sum_{j>=r} s_j^2) <=
// lik_tol * ||M||_F; writes core 1 = V_r^T and vs = V_r (for core 0 = M V_r).
__global__ void lik_select_kernel(const DevTT* __restrict__ L, const RoundScratch* __restrict__ S,
                                  const FilterConst* __restrict__ fc) {
  const int f = blockIdx.x;
  const FilterConst& C = fc[f];
  if (C.meas_kind != 1) return;
  const DevTT& l = L[f];
  const RoundScratch& s = S[f];
  __shared__ int s_r;
  const int nc = s.misc[0];
  const int n1 = C.n[1];
  if (threadIdx.x == 0) {
    double tot = fmax(s.scal[2], 0.0);
    for (int j = 0; j < nc; ++j) tot += s.sigma[j] * s.sigma[j];
    const double delta = C.lik_tol * sqrt(tot);
    double tail2 = fmax(s.scal[2], 0.0);
    int r = nc;
    if (sqrt(tail2) <= delta) {
      for (int j = nc - 1; j >= 0; --j) {
        const double t2 = tail2 + s.sigma[j] * s.sigma[j];
        if (sqrt(t2) <= delta) {
          tail2 = t2;
          r = j;
        } else {
          break;
        }
      }
    }
    r = max(r, 1);
    r = min(r, max(nc, 1));
    if (C.lik_max_rank > 0) r = min(r, C.lik_max_rank);
    if (r > l.cap[1]) {
      r = l.cap[1];
      atomicOr(l.status, TT_STATUS_CAPACITY);
    }
    l.ranks[1] = r;
    s_r = r;
  }
  __syncthreads();
  const int r = s_r;
  double* core1 = core_ptr<double>(l, 1);
  for (int e = threadIdx.x; e < r * n1; e += blockDim.x) {
    const int j = e / n1, i = e % n1;
    const double sg = (j < nc) ? s.sigma[j] : 0.0;
    const double v = (j < nc && sg > 0.0) ? s.usv[(long long)j * s.gcap + i] / sg : 0.0;
    core1[(long long)j * n1 + i] = v;
    s.vs[(long long)i * s.gcap + j] = v;
  }
}

struct LikCtx {
  const DevTT* L;
  const RoundScratch* S;
  const FilterConst* C;
  const double* mbuf;
  long long mstride;
  double tau2;  // relative pre-truncation of the pivoted Cholesky
  double jtol2;  // Jacobi stop: squared relative orthogonality (1e-8 for FP32 bulk)
};

struct FLikGram {  // Gram of the columns of M (n0 x n1)
  LikCtx c;
  __device__ bool operator()(int b, GramArgs& g) const {
    if (c.C[b].meas_kind != 1) return false;
    const RoundScratch& s = c.S[b];
    g.M = c.C[b].n[1];
    g.T = c.C[b].n[0];
    g.x = c.mbuf + b * c.mstride;
    g.sa = 1;
    g.st = g.M;
    g.out = s.gram;
    g.gcap = s.gcap;
    g.splits = s.splits;
    return true;
  }
};
struct FLikPchol {
  LikCtx c;
  __device__ bool operator()(int b, PcholArgs& p) const {
    if (c.C[b].meas_kind != 1) return false;
    const RoundScratch& s = c.S[b];
    p.M = c.C[b].n[1];
    p.g = s.gram;
    p.lwork = s.lwork;
    p.lfac = s.lfac;
    p.piv = s.piv;
    p.rank_out = &s.misc[0];
    p.resid_out = &s.scal[2];
    p.status = c.L[b].status;
    p.gcap = s.gcap;
    p.rmax = s.gcap;
    p.tau2 = c.tau2;
    return true;
  }
};
struct FLikJacobi {
  LikCtx c;
  __device__ bool operator()(int b, JacobiArgs& J) const {
    if (c.C[b].meas_kind != 1) return false;
    const RoundScratch& s = c.S[b];
    J.rows = c.C[b].n[1];
    J.ncols = s.misc[0];
    J.x = s.lfac;
    J.ldx = s.gcap;
    J.work = s.jac;
    J.sigma = s.sigma;
    J.usv = s.usv;
    J.ncols_out = nullptr;
    J.tol2 = c.jtol2;
    J.gcap = s.gcap;
    return true;
  }
};
struct FLikCore0 {  // core 0 = M V_r  (n0 x r)
  LikCtx c;
  __device__ bool operator()(int b, GemmArgs& g) const {
    if (c.C[b].meas_kind != 1) return false;
    const DevTT& l = c.L[b];
    const RoundScratch& s = c.S[b];
    g.M = c.C[b].n[0];
    g.K = c.C[b].n[1];
    g.N = l.ranks[1];
    g.a = c.mbuf + b * c.mstride;
    g.sam = g.K;
    g.sak = 1;
    g.b = s.vs;
    g.sbk = s.gcap;
    g.sbn = 1;
    g.c = core_ptr<double>(l, 0);
    g.scm = g.N;
    g.scn = 1;
    return true;
  }
};

// Likelihood TT for a batch (FP64): dense factors, range-block SVD.
// The range block's SVD: FP64 path with double-double Gram and pivoted
// Cholesky (singular values resolved far below 1e-12 of the largest); the
// FP32 bulk path with an FP64 Gram and a pre-truncation at the FP32 noise
// level (the likelihood cores are FP32 there, so components below ~1e-7 of
// the block's norm cannot be represented anyway).
static tt_status lik_launch(int B, const DevTT* dL, const RoundScratch* drs, const FilterConst* dfc,
                            const double* z, long long zstride, double* mbuf, long long mstride,
                            bool any_range, int n0max, int n1max, int gcap, int splits, hipStream_t st,
                            bool f32 = false) {
  ProfScope ps_(PC_LIK, st);
  hipLaunchKernelGGL(lik_dense_kernel, dim3(B), dim3(256), 0, st, dL, dfc, z, zstride, mbuf, mstride);
  TTG_LAUNCH_CHECK("lik_dense_kernel");
  if (!any_range) return TT_OK;
  LikCtx c{dL, drs, dfc, mbuf, mstride, f32 ? 1e-14 : 1e-31, f32 ? 1e-16 : 1e-30};
  if (f32) {
    TT_TRY((launch_gram<double, AccD>(FLikGram{c}, B, n1max, n0max, splits, st)));
    TT_TRY((launch_pchol<AccD>(FLikPchol{c}, B, gcap, st)));
  } else {
    TT_TRY((launch_gram<double, AccDD>(FLikGram{c}, B, n1max, n0max, splits, st)));
    TT_TRY((launch_pchol<AccDD>(FLikPchol{c}, B, gcap, st)));
  }
  TT_TRY((launch_jacobi(FLikJacobi{c}, B, st)));
  hipLaunchKernelGGL(lik_select_kernel, dim3(B), dim3(256), 0, st, dL, drs, dfc);
  TTG_LAUNCH_CHECK("lik_select_kernel");
  TT_TRY((launch_gemm<double, double, double, double>(FLikCore0{c}, B, n0max, n1max, st)));
  return TT_OK;
}

// ---- kernel TT-SVD --------------------------------------------------------
struct KsvdCtx {
  const DevTT* K;  // FP64 result
  const RoundScratch* S;
  const double* a;   // current unfolding (row-major rows x cols), filter b at a + b * bstride
  double* next;      // next unfolding
  long long cols;    // columns of the current unfolding
  int k;
  int d;
  long long bstride;  // elements between the unfoldings of consecutive filters
};
struct FKsvdGram {
  KsvdCtx c;
  __device__ bool operator()(int b, GramArgs& g) const {
    const DevTT& K = c.K[b];
    const RoundScratch& s = c.S[b];
    g.M = K.ranks[c.k] * K.n[c.k];
    g.T = (int)c.cols;
    g.x = c.a + b * c.bstride;
    g.sa = c.cols;
    g.st = 1;
    g.out = s.gram;
    g.gcap = s.gcap;
    g.splits = s.splits;
    return true;
  }
};
struct FKsvdPchol {
  KsvdCtx c;
  __device__ bool operator()(int b, PcholArgs& p) const {
    const DevTT& K = c.K[b];
    const RoundScratch& s = c.S[b];
    p.M = K.ranks[c.k] * K.n[c.k];
    p.g = s.gram;
    p.lwork = s.lwork;
    p.lfac = s.lfac;
    p.piv = s.piv;
    p.rank_out = &s.misc[0];
    p.resid_out = &s.scal[2];
    p.status = K.status;
    p.gcap = s.gcap;
    p.rmax = s.gcap;
    p.tau2 = 1e-30;
    return true;
  }
};
struct FKsvdJacobi {
  KsvdCtx c;
  __device__ bool operator()(int b, JacobiArgs& J) const {
    const DevTT& K = c.K[b];
    const RoundScratch& s = c.S[b];
    J.rows = K.ranks[c.k] * K.n[c.k];
    J.ncols = s.misc[0];
    J.x = s.lfac;
    J.ldx = s.gcap;
    J.work = s.jac;
    J.sigma = s.sigma;
    J.usv = s.usv;
    J.ncols_out = nullptr;
    J.tol2 = 1e-30;
    J.gcap = s.gcap;
    return true;
  }
};
struct FKsvdNext {  // next = U_r^T A
  KsvdCtx c;
  __device__ bool operator()(int b, GemmArgs& g) const {
    const DevTT& K = c.K[b];
    const int r = K.ranks[c.k + 1];
    g.M = r;
    g.K = K.ranks[c.k] * K.n[c.k];
    g.N = (int)c.cols;
    g.a = core_ptr<double>(K, c.k);
    g.sam = 1;
    g.sak = r;
    g.b = c.a + b * c.bstride;
    g.sbk = c.cols;
    g.sbn = 1;
    g.c = c.next + b * c.bstride;
    g.scm = c.cols;
    g.scn = 1;
    return true;
  }
};

__global__ void ksvd_select_kernel(const DevTT* __restrict__ Kt, const RoundScratch* __restrict__ S, int k,
                                   double tol) {
  const DevTT& K = Kt[blockIdx.x];
  const RoundScratch& s = S[blockIdx.x];
  __shared__ int s_r;
  const int nc = s.misc[0];
  const int rows = K.ranks[k] * K.n[k];
  if (threadIdx.x == 0) {
    if (k == 0) {
      double tot = fmax(s.scal[2], 0.0);
      for (int j = 0; j < nc; ++j) tot += s.sigma[j] * s.sigma[j];
      s.scal[0] = sqrt(tot);
      s.scal[1] = tol * sqrt(tot) / sqrt((double)max(K.d - 1, 1));
    }
    const double delta = s.scal[1];
    double tail2 = fmax(s.scal[2], 0.0);
    int r = nc;
    if (sqrt(tail2) <= delta) {
      for (int j = nc - 1; j >= 0; --j) {
        const double t2 = tail2 + s.sigma[j] * s.sigma[j];
        if (sqrt(t2) <= delta) {
          tail2 = t2;
          r = j;
        } else {
          break;
        }
      }
    }
    r = max(r, 1);
    r = min(r, max(nc, 1));
    if (r > K.cap[k + 1]) {
      r = K.cap[k + 1];
      atomicOr(K.status, TT_STATUS_CAPACITY);
    }
    K.ranks[k + 1] = r;
    s_r = r;
  }
  __syncthreads();
  const int r = s_r;
  double* core = core_ptr<double>(K, k);
  for (int e = threadIdx.x; e < rows * r; e += blockDim.x) {
    const int row = e / r, j = e % r;
    const double sg = (j < nc) ? s.sigma[j] : 0.0;
    core[e] = (j < nc && sg > 0.0) ? s.usv[(long long)j * s.gcap + row] / sg : 0.0;
  }
}

__global__ void ksvd_init_kernel(const DevTT* __restrict__ Kt) {
  const DevTT& K = Kt[blockIdx.x];
  for (int j = 0; j <= K.d; ++j) K.ranks[j] = 1;
  *K.log_scale = 0.0;
  *K.status = 0;
}

__global__ void ksvd_last_kernel(const DevTT* __restrict__ Kt, const double* __restrict__ ab, long long bstride) {
  const DevTT& K = Kt[blockIdx.y];
  const double* a = ab + blockIdx.y * bstride;
  const int k = K.d - 1;
  const long long tot = (long long)K.ranks[k] * K.n[k];
  double* core = core_ptr<double>(K, k);
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < tot; e += (long long)gridDim.x * blockDim.x)
    core[e] = a[e];
}

__global__ void fill_kernel(double* p, long long n, long long stride, double v) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    p[e * stride] = v;
}

__global__ void record_ranks_kernel(const DevTT* __restrict__ P, int nf, int* out, long long stride) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  for (int j = 0; j <= P[f].d; ++j) out[f * stride + j] = P[f].ranks[j];
}

__global__ void loglik_kernel(const double* log_c, int K, int kdone, int nf, double* out) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  double s = 0.0;
  for (int k = 0; k < kdone; ++k) s += log_c[(long long)f * K + k];
  out[f] = s;
}

__global__ void copy_status_kernel(const DevTT* __restrict__ P, int nf, int* out) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  if (P[f].status != out + f) out[f] = *P[f].status;
}

static size_t moments_scratch_per_filter(int d, int rcap) {
  return (size_t)3 * d * rcap * rcap + 2 * (size_t)(d + 1) * rcap + 8 * (size_t)rcap + 8;  // chains: 2 rcap per wavefront
}

template <typename T>
static tt_status launch_moments(int B, const DevTT* dt, const FilterConst* dfc, double* log_mass, long long lms,
                                double* mean, long long ms, double* cov, long long cs, double* scratch,
                                long long spf, int rcap, hipStream_t st) {
  ProfScope ps_(PC_CONTRACT, st);
  hipLaunchKernelGGL((moments_kernel<T>), dim3(B), dim3(256), 0, st, dt, dfc, log_mass, lms, mean, ms, cov, cs,
                     scratch, spf, rcap);
  TTG_LAUNCH_CHECK("moments_kernel");
  return TT_OK;
}

template <typename T>
static tt_status launch_conv(int B, int d, int r0cap, size_t smem, const DevTT* dk, const DevTT* dp,
                             const DevTT* dx, hipStream_t st, int all_cores = 1) {
  hipLaunchKernelGGL(product_init_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, dk, dp, dx, B);
  TTG_LAUNCH_CHECK("product_init_kernel");
  if (smem > 48 * 1024)
    HIP_TRY(hipFuncSetAttribute((const void*)conv_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem),
            "conv smem attribute");
  ProfScope ps_(PC_CONV, st);
  hipLaunchKernelGGL((conv_kernel<T>), dim3(r0cap, d, B), dim3(256), smem, st, dk, dp, dx, all_cores);
  TTG_LAUNCH_CHECK("conv_kernel");
  return TT_OK;
}

template <typename T>
static tt_status launch_dot(int B, const DevTT* dl, const DevTT* dp, const FilterConst* dfc, double* out,
                            long long stride, double* vbuf, long long vstride, long long tofs, hipStream_t st) {
  ProfScope ps_(PC_CONTRACT, st);
  hipLaunchKernelGGL((dot_kernel<T>), dim3(B), dim3(256), 0, st, dl, dp, dfc, out, stride, vbuf, vstride, tofs);
  TTG_LAUNCH_CHECK("dot_kernel");
  return TT_OK;
}

// Work model of the Hadamard product: no flops counted (one multiply per
// output element), bytes = write H once, read the likelihood (FP64) and the
// density cores once, with the device ranks of the launch.
template <typename T>
__global__ void __launch_bounds__(256) hadamard_work_kernel(const DevTT* __restrict__ dl,
                                                            const DevTT* __restrict__ dp, int B, double* work) {
  __shared__ double red[4];
  double by = 0.0;
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    const DevTT &L = dl[b], &P = dp[b];
    for (int k = 0; k < P.d; ++k) {
      const double n = P.n[k];
      const double rl = (double)L.ranks[k] * L.ranks[k + 1], rp = (double)P.ranks[k] * P.ranks[k + 1];
      by += sizeof(T) * rl * rp * n + 8.0 * rl * n + sizeof(T) * rp * n;
    }
  }
  by = block_sum(by, red);
  if (threadIdx.x == 0) work[2 * PC_HADAMARD + 1] += by;
}

template <typename T>
static tt_status launch_hadamard(int B, int d, int r0cap, const DevTT* dl, const DevTT* dp, const DevTT* dh,
                                 hipStream_t st) {
  hipLaunchKernelGGL(product_init_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, dl, dp, dh, B);
  TTG_LAUNCH_CHECK("product_init_kernel");
  {
    ProfScope ps_(PC_HADAMARD, st);
    hipLaunchKernelGGL((hadamard_kernel<T>), dim3(stride_grid(r0cap, B, 8192), 1, B), dim3(256), 0, st, dl, dp, dh);
    TTG_LAUNCH_CHECK("hadamard_kernel");
  }
  if (g_work && (g_prof_mask & (1 << PC_HADAMARD))) {
    hipLaunchKernelGGL((hadamard_work_kernel<T>), dim3(1), dim3(256), 0, st, dl, dp, B, g_work);
    TTG_LAUNCH_CHECK("hadamard_work_kernel");
  }
  return TT_OK;
}

template <typename T>
static size_t conv_smem(const DevTT& K, const DevTT& P) {
  size_t m = 0;
  for (int k = 0; k < P.d; ++k) {
    const int taps = K.n[k], h = (taps - 1) / 2;
    const int taps_pad = (taps + CONV_TB - 1) / CONV_TB * CONV_TB;
    const size_t s = ((size_t)taps_pad * K.cap[k + 1] + (size_t)(CONV_TB + P.n[k] + 2 * h + CONV_ROWS) * P.cap[k + 1]) * sizeof(T);
    m = std::max(m, s);
  }
  return m;
}

}  // namespace ttg

extern "C" {

// ---------------------------------------------------------------------------
// tt_predict
// ---------------------------------------------------------------------------
size_t tt_predict_workspace(int32_t batch) {
  if (batch < 1) return 0;
  return (size_t)3 * batch * sizeof(DevTT) + 1024;
}

tt_status tt_predict(int32_t batch, const tt_train* kernels, const tt_train* p_in, const tt_train* p_out, void* ws,
                     size_t ws_bytes, void* stream) {
  if (batch < 1 || !kernels || !p_in || !p_out || !ws) {
    set_error("tt_predict: bad arguments");
    return TT_ERR_ARG;
  }
  const int dtype = p_in[0].dtype;
  std::vector<DevTT> vk(batch), vp(batch), vx(batch);
  int r0cap = 1;
  size_t smem = 0;
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_train(&kernels[b], "kernel", dtype));
    TT_TRY(check_train(&p_in[b], "p_in", dtype));
    TT_TRY(check_train(&p_out[b], "p_out", dtype));
    if (kernels[b].d != p_in[0].d || p_in[b].d != p_in[0].d || p_out[b].d != p_in[0].d) {
      set_error("tt_predict: d differs");
      return TT_ERR_SHAPE;
    }
    for (int k = 0; k < p_in[b].d; ++k) {
      if (p_out[b].n[k] != p_in[b].n[k] || (kernels[b].n[k] % 2) != 1) {
        set_error("tt_predict: n mismatch or even kernel length");
        return TT_ERR_SHAPE;
      }
      r0cap = std::max(r0cap, kernels[b].cap[k] * p_in[b].cap[k]);
    }
    vk[b] = make_dev(kernels[b]);
    vp[b] = make_dev(p_in[b]);
    vx[b] = make_dev(p_out[b]);
    smem = std::max(smem, dtype == TT_F64 ? conv_smem<double>(vk[b], vp[b]) : conv_smem<float>(vk[b], vp[b]));
  }
  if (smem > 160 * 1024) {
    set_error("tt_predict: kernel/fibre too long for LDS (%zu bytes)", smem);
    return TT_ERR_SHAPE;
  }
  Arena ar(ws, ws_bytes);
  DevTT* dk = ar.take<DevTT>(batch);
  DevTT* dp = ar.take<DevTT>(batch);
  DevTT* dx = ar.take<DevTT>(batch);
  if (!ar.fits()) {
    set_error("tt_predict: workspace too small");
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(dk, vk, st));
  TT_TRY(upload(dp, vp, st));
  TT_TRY(upload(dx, vx, st));
  if (dtype == TT_F64) return launch_conv<double>(batch, p_in[0].d, r0cap, smem, dk, dp, dx, st);
  return launch_conv<float>(batch, p_in[0].d, r0cap, smem, dk, dp, dx, st);
}

// ---------------------------------------------------------------------------
// prediction by Einstein summation with a 2d-core transition TT
// ---------------------------------------------------------------------------
static tt_status einsum_check(int32_t batch, const tt_train* tpm, const tt_train* p_in, const tt_train* p_out) {
  if (batch < 1 || !tpm || !p_in) {
    set_error("tt_predict_einsum: bad arguments");
    return TT_ERR_ARG;
  }
  const int dtype = p_in[0].dtype, d = p_in[0].d;
  if (2 * d > TT_MAXD) {
    set_error("tt_predict_einsum: 2d = %d cores exceed %d", 2 * d, TT_MAXD);
    return TT_ERR_SHAPE;
  }
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_train(&tpm[b], "tpm", dtype));
    TT_TRY(check_train(&p_in[b], "p_in", dtype));
    if (p_out) TT_TRY(check_train(&p_out[b], "p_out", dtype));
    if (p_in[b].d != d || tpm[b].d != 2 * d || (p_out && p_out[b].d != d)) {
      set_error("tt_predict_einsum: need d-core densities and 2d-core transition trains of one d");
      return TT_ERR_SHAPE;
    }
    for (int k = 0; k < d; ++k) {
      if (tpm[b].n[k] != p_in[b].n[k] || tpm[b].n[d + k] != p_in[b].n[k] || (p_out && p_out[b].n[k] != p_in[b].n[k])) {
        set_error("tt_predict_einsum: mode sizes differ (filter %d, axis %d)", b, k);
        return TT_ERR_SHAPE;
      }
      if (p_out && p_out[b].cap[k] < tpm[b].cap[k]) {
        set_error("tt_predict_einsum: p_out cap[%d] = %d below the transition train's %d", k, p_out[b].cap[k],
                  tpm[b].cap[k]);
        return TT_ERR_SHAPE;
      }
    }
  }
  return TT_OK;
}

// scratch of one filter, in doubles: Y, then two Z buffers
static void einsum_sizes(const tt_train& t, const tt_train& p, long long& ysz, long long& zsz) {
  const int d = p.d;
  ysz = 1;
  zsz = 1;
  for (int k = 0; k < d; ++k) {
    ysz = std::max(ysz, (long long)p.cap[k] * p.n[k] * t.cap[d + k + 1]);
    zsz = std::max(zsz, (long long)t.cap[d + k] * p.cap[k]);
  }
}

size_t tt_predict_einsum_workspace(int32_t batch, const tt_train* tpm, const tt_train* p_in) {
  if (einsum_check(batch, tpm, p_in, nullptr) != TT_OK) return 0;
  size_t total = (size_t)batch * (3 * sizeof(DevTT) + 3 * sizeof(double*)) + 4096;
  for (int b = 0; b < batch; ++b) {
    long long ysz, zsz;
    einsum_sizes(tpm[b], p_in[b], ysz, zsz);
    total += (size_t)(ysz + 2 * zsz) * sizeof(double) + 3 * 256;
  }
  return total;
}

tt_status tt_predict_einsum(int32_t batch, const tt_train* tpm, const tt_train* p_in, const tt_train* p_out,
                            void* ws, size_t ws_bytes, void* stream) {
  if (!p_out || !ws) {
    set_error("tt_predict_einsum: bad arguments");
    return TT_ERR_ARG;
  }
  TT_TRY(einsum_check(batch, tpm, p_in, p_out));
  const int d = p_in[0].d;
  const bool f64 = p_in[0].dtype == TT_F64;
  Arena ar(ws, ws_bytes);
  DevTT* dt = ar.take<DevTT>(batch);
  DevTT* dp = ar.take<DevTT>(batch);
  DevTT* dout = ar.take<DevTT>(batch);
  double** dy = ar.take<double*>(batch);
  double** dz0 = ar.take<double*>(batch);
  double** dz1 = ar.take<double*>(batch);
  std::vector<DevTT> vt(batch), vp(batch), vo(batch);
  std::vector<double*> vy(batch), vz0(batch), vz1(batch);
  long long ymax = 1, zmax = 1, omax = 1;
  int rtmax = 1, rpmax = 1;  // row blocks of the Z pass
  for (int b = 0; b < batch; ++b) {
    vt[b] = make_dev(tpm[b]);
    vp[b] = make_dev(p_in[b]);
    vo[b] = make_dev(p_out[b]);
    long long ysz, zsz;
    einsum_sizes(tpm[b], p_in[b], ysz, zsz);
    vy[b] = ar.take<double>(ysz);
    vz0[b] = ar.take<double>(zsz);
    vz1[b] = ar.take<double>(zsz);
    ymax = std::max(ymax, ysz);
    zmax = std::max(zmax, zsz);
    for (int k = 0; k < d; ++k) {
      omax = std::max(omax, (long long)tpm[b].cap[k] * tpm[b].n[k] * tpm[b].cap[k + 1]);
      rtmax = std::max(rtmax, tpm[b].cap[d + k]);
      rpmax = std::max(rpmax, p_in[b].cap[k]);
    }
  }
  if (!ar.fits()) {
    set_error("tt_predict_einsum: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  {
    // the descriptors and scratch pointers sit contiguously at the start of
    // the arena: one upload
    const char* base = reinterpret_cast<const char*>(dt);
    const size_t span = reinterpret_cast<const char*>(dz1 + batch) - base;
    std::vector<char> h(span, 0);
    auto put = [&](const void* dst, const void* src, size_t bytes) {
      memcpy(h.data() + (reinterpret_cast<const char*>(dst) - base), src, bytes);
    };
    put(dt, vt.data(), batch * sizeof(DevTT));
    put(dp, vp.data(), batch * sizeof(DevTT));
    put(dout, vo.data(), batch * sizeof(DevTT));
    put(dy, vy.data(), batch * sizeof(double*));
    put(dz0, vz0.data(), batch * sizeof(double*));
    put(dz1, vz1.data(), batch * sizeof(double*));
    TT_TRY(upload(const_cast<char*>(base), h, st));
  }
  const dim3 gy(stride_grid(cdiv(ymax, 256), batch), 1, batch), gz(cdiv(rtmax, EZ_ROWS), cdiv(rpmax, EZ_CB), batch);
  ProfScope ps_(PC_EINSUM, st);
  double** zc = nullptr;  // Z of the cores already summed (none: Z = 1)
  for (int k = d - 1; k >= 0; --k) {
    double** zn = (zc == dz0) ? dz1 : dz0;
    if (f64) {
      hipLaunchKernelGGL((einsum_y_kernel<double>), gy, dim3(256), 0, st, dt, dp, zc, dy, k);
      hipLaunchKernelGGL((einsum_z_kernel<double>), gz, dim3(64 * EZ_WAVES), 0, st, dt, dp, dy, zn, k);
    } else {
      hipLaunchKernelGGL((einsum_y_kernel<float>), gy, dim3(256), 0, st, dt, dp, zc, dy, k);
      hipLaunchKernelGGL((einsum_z_kernel<float>), gz, dim3(64 * EZ_WAVES), 0, st, dt, dp, dy, zn, k);
    }
    TTG_LAUNCH_CHECK("einsum_y_kernel / einsum_z_kernel");
    zc = zn;
  }
  const dim3 go(stride_grid(cdiv(omax, 256), batch * d), d, batch);
  if (f64)
    hipLaunchKernelGGL((einsum_out_kernel<double>), go, dim3(256), 0, st, dt, dp, dout, zc);
  else
    hipLaunchKernelGGL((einsum_out_kernel<float>), go, dim3(256), 0, st, dt, dp, dout, zc);
  TTG_LAUNCH_CHECK("einsum_out_kernel");
  return TT_OK;
}

// ---------------------------------------------------------------------------
// grid re-design and interpolation onto the new grid
// ---------------------------------------------------------------------------
size_t tt_grid_redesign_workspace(int32_t batch, int32_t d) {
  if (batch < 1 || d < 1 || d > TT_MAXD) return 0;
  return (size_t)batch * sizeof(GridBox) + 3 * (size_t)d * d * sizeof(double) + 4 * 256;
}

tt_status tt_grid_redesign(int32_t batch, int32_t d, const double* f, const double* q, double nsigma,
                           const double* mean_dev, const double* cov_dev, const tt_grid* old_grids,
                           tt_grid* new_grids, void* ws, size_t ws_bytes, void* stream) {
  if (batch < 1 || d < 1 || d > TT_MAXD || !f || !q || !mean_dev || !cov_dev || !old_grids || !new_grids || !ws ||
      !(nsigma > 0.0)) {
    set_error("tt_grid_redesign: bad arguments");
    return TT_ERR_ARG;
  }
  for (int b = 0; b < batch; ++b)
    if (old_grids[b].d != d) {
      set_error("tt_grid_redesign: grid %d has d = %d, not %d", b, old_grids[b].d, d);
      return TT_ERR_SHAPE;
    }
  // F^{-1} of the model matrix (d x d, once per call): Gauss-Jordan with
  // partial pivoting on the host
  std::vector<double> a(f, f + (size_t)d * d), inv((size_t)d * d, 0.0);
  for (int i = 0; i < d; ++i) inv[(size_t)i * d + i] = 1.0;
  double fmaxabs = 0.0;
  for (int i = 0; i < d * d; ++i) fmaxabs = std::max(fmaxabs, std::fabs(a[i]));
  for (int c = 0; c < d; ++c) {
    int piv = c;
    for (int r = c + 1; r < d; ++r)
      if (std::fabs(a[(size_t)r * d + c]) > std::fabs(a[(size_t)piv * d + c])) piv = r;
    if (!(std::fabs(a[(size_t)piv * d + c]) > 1e-14 * fmaxabs)) {
      set_error("tt_grid_redesign: F is singular");
      return TT_ERR_ARG;
    }
    for (int j = 0; j < d; ++j) {
      std::swap(a[(size_t)c * d + j], a[(size_t)piv * d + j]);
      std::swap(inv[(size_t)c * d + j], inv[(size_t)piv * d + j]);
    }
    const double dinv = 1.0 / a[(size_t)c * d + c];
    for (int j = 0; j < d; ++j) {
      a[(size_t)c * d + j] *= dinv;
      inv[(size_t)c * d + j] *= dinv;
    }
    for (int r = 0; r < d; ++r) {
      if (r == c) continue;
      const double m = a[(size_t)r * d + c];
      if (m == 0.0) continue;
      for (int j = 0; j < d; ++j) {
        a[(size_t)r * d + j] -= m * a[(size_t)c * d + j];
        inv[(size_t)r * d + j] -= m * inv[(size_t)c * d + j];
      }
    }
  }
  Arena ar(ws, ws_bytes);
  GridBox* dbox = ar.take<GridBox>(batch);
  double* dmat = ar.take<double>(3 * (size_t)d * d);
  if (!ar.fits()) {
    set_error("tt_grid_redesign: workspace too small");
    return TT_ERR_WORKSPACE;
  }
  std::vector<double> mats(3 * (size_t)d * d);
  std::copy(f, f + (size_t)d * d, mats.begin());
  std::copy(inv.begin(), inv.end(), mats.begin() + (size_t)d * d);
  std::copy(q, q + (size_t)d * d, mats.begin() + 2 * (size_t)d * d);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(dmat, mats, st));
  hipLaunchKernelGGL(grid_box_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, (int)batch, (int)d, dmat,
                     dmat + (size_t)d * d, dmat + 2 * (size_t)d * d, nsigma, mean_dev, cov_dev, dbox);
  TTG_LAUNCH_CHECK("grid_box_kernel");
  std::vector<GridBox> hb(batch);
  HIP_TRY(hipMemcpyAsync(hb.data(), dbox, batch * sizeof(GridBox), hipMemcpyDeviceToHost, st), "box download");
  HIP_TRY(hipStreamSynchronize(st), "tt_grid_redesign");
  for (int b = 0; b < batch; ++b) {
    tt_grid g = old_grids[b];
    for (int l = 0; l < d; ++l) {
      if (!(hb[b].hi[l] > hb[b].lo[l]) || !std::isfinite(hb[b].lo[l]) || !std::isfinite(hb[b].hi[l])) {
        set_error("tt_grid_redesign: degenerate box for filter %d, axis %d", b, l);
        return TT_ERR_ARG;
      }
      g.lo[l] = hb[b].lo[l];
      g.hi[l] = hb[b].hi[l];
    }
    new_grids[b] = g;
  }
  return TT_OK;
}

size_t tt_interpolate_workspace(int32_t batch) {
  if (batch < 1) return 0;
  return (size_t)batch * (2 * sizeof(DevTT) + sizeof(InterpArgs)) + 3 * 256;
}

tt_status tt_interpolate(int32_t batch, const tt_grid* from, const tt_grid* to, const tt_train* in,
                         const tt_train* out, void* ws, size_t ws_bytes, void* stream) {
  if (batch < 1 || !from || !to || !in || !out || !ws) {
    set_error("tt_interpolate: bad arguments");
    return TT_ERR_ARG;
  }
  const int dtype = in[0].dtype;
  std::vector<DevTT> vi(batch), vo(batch);
  std::vector<InterpArgs> va(batch);
  long long omax = 1;
  int dmax = 1;
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_train(&in[b], "in", dtype));
    TT_TRY(check_train(&out[b], "out", dtype));
    const int d = in[b].d;
    if (out[b].d != d || from[b].d != d || to[b].d != d) {
      set_error("tt_interpolate: d differs (filter %d)", b);
      return TT_ERR_SHAPE;
    }
    InterpArgs& g = va[b];
    memset(&g, 0, sizeof(g));
    for (int k = 0; k < d; ++k) {
      if (from[b].n[k] != in[b].n[k] || to[b].n[k] != out[b].n[k] || in[b].n[k] < 2 || out[b].n[k] < 2 ||
          !(from[b].hi[k] > from[b].lo[k]) || !(to[b].hi[k] > to[b].lo[k])) {
        set_error("tt_interpolate: grids and trains disagree, or an axis has < 2 points (filter %d, axis %d)", b,
                  k);
        return TT_ERR_SHAPE;
      }
      if (out[b].cap[k + 1] < in[b].cap[k + 1]) {
        set_error("tt_interpolate: out cap[%d] below in's", k + 1);
        return TT_ERR_SHAPE;
      }
      g.n_old[k] = in[b].n[k];
      g.n_new[k] = out[b].n[k];
      g.lo_old[k] = from[b].lo[k];
      g.hi_old[k] = from[b].hi[k];
      g.lo_new[k] = to[b].lo[k];
      g.hi_new[k] = to[b].hi[k];
      omax = std::max(omax, (long long)in[b].cap[k] * out[b].n[k] * in[b].cap[k + 1]);
    }
    dmax = std::max(dmax, d);
    vi[b] = make_dev(in[b]);
    vo[b] = make_dev(out[b]);
  }
  Arena ar(ws, ws_bytes);
  DevTT* di = ar.take<DevTT>(batch);
  DevTT* dout = ar.take<DevTT>(batch);
  InterpArgs* da = ar.take<InterpArgs>(batch);
  if (!ar.fits()) {
    set_error("tt_interpolate: workspace too small");
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(di, vi, st));
  TT_TRY(upload(dout, vo, st));
  TT_TRY(upload(da, va, st));
  const dim3 grid(stride_grid(cdiv(omax, 256), batch * dmax), dmax, batch);
  ProfScope ps_(PC_INTERP, st);
  if (dtype == TT_F64)
    hipLaunchKernelGGL((interp_kernel<double>), grid, dim3(256), 0, st, di, dout, da);
  else
    hipLaunchKernelGGL((interp_kernel<float>), grid, dim3(256), 0, st, di, dout, da);
  TTG_LAUNCH_CHECK("interp_kernel");
  return TT_OK;
}

// ---------------------------------------------------------------------------
// adjoints of the linear steps
// ---------------------------------------------------------------------------
static tt_status check_like(const tt_train& a, const tt_train& b, const char* what) {
  if (a.d != b.d) {
    set_error("%s: d differs", what);
    return TT_ERR_SHAPE;
  }
  for (int k = 0; k < a.d; ++k)
    if (a.n[k] != b.n[k]) {
      set_error("%s: mode sizes differ", what);
      return TT_ERR_SHAPE;
    }
  return TT_OK;
}

size_t tt_adjoint_workspace(int32_t batch, int32_t d, int32_t rcap) {
  if (batch < 1 || d < 1 || rcap < 1) return 0;
  const size_t align = (size_t)batch * (3 * 2 * ALIGN_RMAX * ALIGN_RMAX + ALIGN_RMAX + 1) * sizeof(double);
  return (size_t)5 * batch * sizeof(DevTT) +
         std::max((size_t)batch * (2 * (d + 1) * rcap + 1) * sizeof(double), align) + 4096;
}

tt_status tt_predict_adjoint(int32_t batch, const tt_train* kernels, const tt_train* p_in, const tt_train* c_bar,
                             const tt_train* p_bar, const tt_train* k_bar, void* ws, size_t ws_bytes,
                             void* stream) {
  if (batch < 1 || !kernels || !p_in || !c_bar || !p_bar || !k_bar || !ws) {
    set_error("tt_predict_adjoint: bad arguments");
    return TT_ERR_ARG;
  }
  const int dtype = p_in[0].dtype, d = p_in[0].d;
  std::vector<DevTT> vk(batch), vp(batch), vc(batch), vpb(batch), vkb(batch);
  int r0cap = 1, rkcap = 1, tapmax = 1;
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_train(&kernels[b], "kernel", dtype));
    TT_TRY(check_train(&p_in[b], "p_in", dtype));
    TT_TRY(check_train(&c_bar[b], "c_bar", dtype));
    TT_TRY(check_train(&p_bar[b], "p_bar", dtype));
    TT_TRY(check_train(&k_bar[b], "k_bar", dtype));
    if (p_in[b].d != d || kernels[b].d != d) {
      set_error("tt_predict_adjoint: d differs");
      return TT_ERR_SHAPE;
    }
    TT_TRY(check_like(p_in[b], c_bar[b], "tt_predict_adjoint c_bar"));
    TT_TRY(check_like(p_in[b], p_bar[b], "tt_predict_adjoint p_bar"));
    TT_TRY(check_like(kernels[b], k_bar[b], "tt_predict_adjoint k_bar"));
    for (int k = 0; k < d; ++k) {
      if ((kernels[b].n[k] % 2) != 1) {
        set_error("tt_predict_adjoint: even kernel length");
        return TT_ERR_SHAPE;
      }
      r0cap = std::max(r0cap, p_in[b].cap[k]);
      rkcap = std::max(rkcap, kernels[b].cap[k] * kernels[b].cap[k + 1]);  // kernel bond pairs
      tapmax = std::max(tapmax, kernels[b].n[k]);
    }
    vk[b] = make_dev(kernels[b]);
    vp[b] = make_dev(p_in[b]);
    vc[b] = make_dev(c_bar[b]);
    vpb[b] = make_dev(p_bar[b]);
    vkb[b] = make_dev(k_bar[b]);
  }
  Arena ar(ws, ws_bytes);
  DevTT* dk = ar.take<DevTT>(batch);
  DevTT* dp = ar.take<DevTT>(batch);
  DevTT* dc = ar.take<DevTT>(batch);
  DevTT* dpb = ar.take<DevTT>(batch);
  DevTT* dkb = ar.take<DevTT>(batch);
  if (!ar.fits()) {
    set_error("tt_predict_adjoint: workspace too small");
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(dk, vk, st));
  TT_TRY(upload(dp, vp, st));
  TT_TRY(upload(dc, vc, st));
  TT_TRY(upload(dpb, vpb, st));
  TT_TRY(upload(dkb, vkb, st));
  hipLaunchKernelGGL(adj_init_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, dp, dpb, dc, dk, dp, batch);
  TTG_LAUNCH_CHECK("adj_init_kernel");
  hipLaunchKernelGGL(adj_init_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, dk, dkb, dc, dk, dp, batch);
  TTG_LAUNCH_CHECK("adj_init_kernel");
  int pel = 1;
  for (int b = 0; b < batch; ++b)
    for (int k = 0; k < d; ++k) pel = std::max(pel, p_in[b].cap[k] * p_in[b].n[k] * p_in[b].cap[k + 1]);
  // the register-window Pbar kernel when the kernel core fits the LDS
  // (decided from capacities only)
  int kelcap = 1, rp0cap = 1, rp1cap = 1, nmax = 1;
  for (int b = 0; b < batch; ++b)
    for (int k = 0; k < d; ++k) {
      kelcap = std::max(kelcap, kernels[b].cap[k] * kernels[b].n[k] * kernels[b].cap[k + 1]);
      rp0cap = std::max(rp0cap, p_in[b].cap[k]);
      rp1cap = std::max(rp1cap, p_in[b].cap[k + 1]);
      nmax = std::max(nmax, p_in[b].n[k]);
    }
  const size_t padj_lds = (size_t)kelcap * (dtype == TT_F64 ? 8 : 4);
  const bool staged = padj_lds <= 64 * 1024;
  const long long padj_items = (long long)rp0cap * rp1cap * cdiv(nmax, PADJ_JROWS);
  const int padj_grid = stride_grid(cdiv(padj_items, 256), batch * d);
  if (staged && padj_lds > 48 * 1024) {
    const void* fn = dtype == TT_F64 ? (const void*)pred_adj_p_reg_kernel<double>
                                     : (const void*)pred_adj_p_reg_kernel<float>;
    HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)padj_lds), "padj smem");
  }
  if (dtype == TT_F64) {
    if (staged)
      hipLaunchKernelGGL((pred_adj_p_reg_kernel<double>), dim3(padj_grid, d, batch), dim3(256), padj_lds, st, dk, dp,
                         dc, dpb);
    else
      hipLaunchKernelGGL((pred_adj_p_kernel<double>), dim3(stride_grid(cdiv(pel, 256), batch), d, batch), dim3(256),
                         0, st, dk, dp, dc, dpb);
    TTG_LAUNCH_CHECK("pred_adj_p_kernel");
    hipLaunchKernelGGL((pred_adj_k_kernel<double>), dim3(std::min(rkcap, 65535), d, batch), dim3(256), 0, st, dk, dp,
                       dc, dkb);
    TTG_LAUNCH_CHECK("pred_adj_k_kernel");
  } else {
    if (staged)
      hipLaunchKernelGGL((pred_adj_p_reg_kernel<float>), dim3(padj_grid, d, batch), dim3(256), padj_lds, st, dk, dp,
                         dc, dpb);
    else
      hipLaunchKernelGGL((pred_adj_p_kernel<float>), dim3(stride_grid(cdiv(pel, 256), batch), d, batch), dim3(256),
                         0, st, dk, dp, dc, dpb);
    TTG_LAUNCH_CHECK("pred_adj_p_kernel");
    hipLaunchKernelGGL((pred_adj_k_kernel<float>), dim3(std::min(rkcap, 65535), d, batch), dim3(256), 0, st, dk, dp,
                       dc, dkb);
    TTG_LAUNCH_CHECK("pred_adj_k_kernel");
  }
  (void)r0cap;
  (void)tapmax;
  return TT_OK;
}

tt_status tt_hadamard_adjoint(int32_t batch, const tt_train* a, const tt_train* b, const tt_train* h_bar,
                              const tt_train* a_bar, const tt_train* b_bar, void* ws, size_t ws_bytes,
                              void* stream) {
  if (batch < 1 || !a || !b || !h_bar || (!a_bar && !b_bar) || !ws) {
    set_error("tt_hadamard_adjoint: bad arguments");
    return TT_ERR_ARG;
  }
  const int dtype = b[0].dtype, d = b[0].d;
  std::vector<DevTT> va(batch), vb(batch), vh(batch), vab(batch), vbb(batch);
  int pel = 1;
  for (int f = 0; f < batch; ++f) {
    TT_TRY(check_train(&a[f], "a", TT_F64));
    TT_TRY(check_train(&b[f], "b", dtype));
    TT_TRY(check_train(&h_bar[f], "h_bar", dtype));
    if (a_bar) TT_TRY(check_train(&a_bar[f], "a_bar", TT_F64));
    if (b_bar) TT_TRY(check_train(&b_bar[f], "b_bar", dtype));
    if (b[f].d != d) {
      set_error("tt_hadamard_adjoint: d differs");
      return TT_ERR_SHAPE;
    }
    TT_TRY(check_like(b[f], a[f], "tt_hadamard_adjoint a"));
    TT_TRY(check_like(b[f], h_bar[f], "tt_hadamard_adjoint h_bar"));
    if (a_bar) TT_TRY(check_like(b[f], a_bar[f], "tt_hadamard_adjoint a_bar"));
    if (b_bar) TT_TRY(check_like(b[f], b_bar[f], "tt_hadamard_adjoint b_bar"));
    for (int k = 0; k < d; ++k)
      pel = std::max(pel, std::max(a[f].cap[k] * a[f].n[k] * a[f].cap[k + 1], b[f].cap[k] * b[f].n[k] * b[f].cap[k + 1]));
    va[f] = make_dev(a[f]);
    vb[f] = make_dev(b[f]);
    vh[f] = make_dev(h_bar[f]);
    if (a_bar) vab[f] = make_dev(a_bar[f]);
    if (b_bar) vbb[f] = make_dev(b_bar[f]);
  }
  Arena ar(ws, ws_bytes);
  DevTT* da = ar.take<DevTT>(batch);
  DevTT* db = ar.take<DevTT>(batch);
  DevTT* dh = ar.take<DevTT>(batch);
  DevTT* dab = ar.take<DevTT>(batch);
  DevTT* dbb = ar.take<DevTT>(batch);
  if (!ar.fits()) {
    set_error("tt_hadamard_adjoint: workspace too small");
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(da, va, st));
  TT_TRY(upload(db, vb, st));
  TT_TRY(upload(dh, vh, st));
  if (a_bar) {
    TT_TRY(upload(dab, vab, st));
    hipLaunchKernelGGL(adj_init_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, da, dab, dh, da, db, batch);
    TTG_LAUNCH_CHECK("adj_init_kernel");
  }
  if (b_bar) {
    TT_TRY(upload(dbb, vbb, st));
    hipLaunchKernelGGL(adj_init_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, db, dbb, dh, da, db, batch);
    TTG_LAUNCH_CHECK("adj_init_kernel");
  }
  const dim3 grid(stride_grid(cdiv(pel, 256), batch), d, batch);
  if (dtype == TT_F64)
    hipLaunchKernelGGL((hadamard_adj_kernel<double>), grid, dim3(256), 0, st, da, db, dh, a_bar ? dab : nullptr,
                       b_bar ? dbb : nullptr);
  else
    hipLaunchKernelGGL((hadamard_adj_kernel<float>), grid, dim3(256), 0, st, da, db, dh, a_bar ? dab : nullptr,
                       b_bar ? dbb : nullptr);
  TTG_LAUNCH_CHECK("hadamard_adj_kernel");
  return TT_OK;
}

tt_status tt_normalize_adjoint(int32_t batch, const tt_train* x, const tt_train* p_bar,
                               const double* log_mass_bar_dev, const tt_train* x_bar, void* ws, size_t ws_bytes,
                               void* stream) {
  if (batch < 1 || !x || !p_bar || !x_bar || !ws) {
    set_error("tt_normalize_adjoint: bad arguments");
    return TT_ERR_ARG;
  }
  const int dtype = x[0].dtype, d = x[0].d;
  std::vector<DevTT> vx(batch), vpb(batch), vxb(batch);
  int rcap = 1, pel = 1;
  for (int f = 0; f < batch; ++f) {
    TT_TRY(check_train(&x[f], "x", dtype));
    TT_TRY(check_train(&p_bar[f], "p_bar", dtype));
    TT_TRY(check_train(&x_bar[f], "x_bar", dtype));
    if (x[f].d != d) {
      set_error("tt_normalize_adjoint: d differs");
      return TT_ERR_SHAPE;
    }
    TT_TRY(check_like(x[f], p_bar[f], "tt_normalize_adjoint p_bar"));
    TT_TRY(check_like(x[f], x_bar[f], "tt_normalize_adjoint x_bar"));
    for (int k = 0; k <= d; ++k) rcap = std::max(rcap, x[f].cap[k]);
    for (int k = 0; k < d; ++k) pel = std::max(pel, x[f].cap[k] * x[f].n[k] * x[f].cap[k + 1]);
    vx[f] = make_dev(x[f]);
    vpb[f] = make_dev(p_bar[f]);
    vxb[f] = make_dev(x_bar[f]);
  }
  Arena ar(ws, ws_bytes);
  DevTT* dx = ar.take<DevTT>(batch);
  DevTT* dpb = ar.take<DevTT>(batch);
  DevTT* dxb = ar.take<DevTT>(batch);
  double* env = ar.take<double>((size_t)batch * 2 * (d + 1) * rcap);
  double* ssum = ar.take<double>(batch);
  if (!ar.fits()) {
    set_error("tt_normalize_adjoint: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(dx, vx, st));
  TT_TRY(upload(dpb, vpb, st));
  TT_TRY(upload(dxb, vxb, st));
  hipLaunchKernelGGL(normalize_adj_init_kernel, dim3(cdiv(batch, 64)), dim3(64), 0, st, dx, dpb, dxb,
                     log_mass_bar_dev, batch);
  TTG_LAUNCH_CHECK("normalize_adj_init_kernel");
  const dim3 grid(stride_grid(cdiv(pel, 256), batch), d, batch);
  if (dtype == TT_F64) {
    hipLaunchKernelGGL((sum_env_kernel<double>), dim3(batch), dim3(256), 0, st, dx, env, rcap, ssum);
    TTG_LAUNCH_CHECK("sum_env_kernel");
    hipLaunchKernelGGL((normalize_adj_kernel<double>), grid, dim3(256), 0, st, dx, dpb, dxb, log_mass_bar_dev, env,
                       rcap, ssum);
  } else {
    hipLaunchKernelGGL((sum_env_kernel<float>), dim3(batch), dim3(256), 0, st, dx, env, rcap, ssum);
    TTG_LAUNCH_CHECK("sum_env_kernel");
    hipLaunchKernelGGL((normalize_adj_kernel<float>), grid, dim3(256), 0, st, dx, dpb, dxb, log_mass_bar_dev, env,
                       rcap, ssum);
  }
  TTG_LAUNCH_CHECK("normalize_adj_kernel");
  return TT_OK;
}

// ---------------------------------------------------------------------------
// tt_update
// ---------------------------------------------------------------------------
struct UpdatePlan {
  std::vector<DevTT> vl, vp, vh;
  std::vector<RoundScratch> vrs;
  std::vector<FilterConst> vfc;
  DevTT *dl, *dp, *dh;
  RoundScratch* drs;
  FilterConst* dfc;
  double* mbuf;
  long long mstride;
  double* vbuf;
  int vcap;
  long long vstride, tofs;
  bool any_range;
  int n0max, n1max, gcap, splits, r0cap;
};

static tt_status update_plan(int32_t batch, const tt_grid* grids, const tt_meas* meas, const tt_train* p_pred,
                             const tt_train* h_out, int32_t lik_rank_cap, Arena& ar, UpdatePlan& u) {
  if (batch < 1 || !grids || !meas || !p_pred || !h_out || lik_rank_cap < 1) {
    set_error("tt_update: bad arguments");
    return TT_ERR_ARG;
  }
  const int dtype = p_pred[0].dtype;
  u.vl.resize(batch);
  u.vp.resize(batch);
  u.vh.resize(batch);
  u.vrs.resize(batch);
  u.vfc.resize(batch);
  u.any_range = false;
  u.n0max = u.n1max = 1;
  u.r0cap = 1;
  u.vcap = 1;
  const int d = p_pred[0].d;
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_grid(&grids[b]));
    TT_TRY(check_train(&p_pred[b], "p_pred", dtype));
    TT_TRY(check_train(&h_out[b], "h_out", dtype));
    if (grids[b].d != d || p_pred[b].d != d || h_out[b].d != d) {
      set_error("tt_update: d differs");
      return TT_ERR_SHAPE;
    }
    if (meas[b].kind != 0 && meas[b].kind != 1) {
      set_error("tt_update: meas kind must be 0 or 1");
      return TT_ERR_ARG;
    }
    if (meas[b].kind == 1 && d < 2) {
      set_error("tt_update: range model needs d >= 2");
      return TT_ERR_SHAPE;
    }
    for (int k = 0; k < d; ++k)
      if (grids[b].n[k] != p_pred[b].n[k] || h_out[b].n[k] != p_pred[b].n[k]) {
        set_error("tt_update: grid / TT mode sizes differ");
        return TT_ERR_SHAPE;
      }
    u.vfc[b] = make_const(grids[b], &meas[b]);
    u.vp[b] = make_dev(p_pred[b]);
    u.vh[b] = make_dev(h_out[b]);
    u.any_range = u.any_range || meas[b].kind == 1;
    u.n0max = std::max(u.n0max, grids[b].n[0]);
    if (d > 1) u.n1max = std::max(u.n1max, grids[b].n[1]);
    for (int j = 0; j <= d; ++j) u.vcap = std::max(u.vcap, h_out[b].cap[j]);
  }
  u.gcap = u.n1max;
  if (u.gcap > 1024) {
    set_error("tt_update: n[1] = %d exceeds 1024", u.gcap);
    return TT_ERR_SHAPE;
  }
  u.splits = GRAM_PLANES;
  u.dl = ar.take<DevTT>(batch);
  u.dp = ar.take<DevTT>(batch);
  u.dh = ar.take<DevTT>(batch);
  u.drs = ar.take<RoundScratch>(batch);
  u.dfc = ar.take<FilterConst>(batch);
  u.mstride = (long long)u.n0max * u.n1max;
  u.mbuf = u.any_range ? ar.take<double>((size_t)batch * u.mstride) : nullptr;
  {
    long long tmax = 1;
    for (int b = 0; b < batch; ++b)
      for (int k = 0; k < d; ++k) {
        const int lc1 = (meas[b].kind == 1 && k == 0) ? std::min(lik_rank_cap, p_pred[b].n[1]) : 1;
        tmax = std::max(tmax, (long long)lc1 * p_pred[b].cap[k] * p_pred[b].n[k]);
      }
    u.tofs = u.vcap;
    u.vstride = u.vcap + tmax;
  }
  u.vbuf = ar.take<double>((size_t)batch * u.vstride);
  for (int b = 0; b < batch; ++b) {
    tt_train lt;
    memset(&lt, 0, sizeof(lt));
    lt.d = d;
    lt.dtype = TT_F64;
    for (int k = 0; k < d; ++k) lt.n[k] = p_pred[b].n[k];
    for (int j = 0; j <= d; ++j) lt.cap[j] = 1;
    if (meas[b].kind == 1) lt.cap[1] = std::min(lik_rank_cap, p_pred[b].n[1]);
    lt.cores = ar.take<double>(elems_of(d, lt.n, lt.cap));
    lt.ranks = ar.take<int>(TT_MAXD + 1);
    lt.log_scale = ar.take<double>(1);
    lt.status = h_out[b].status;  // shares the output's status word
    u.vl[b] = make_dev(lt);
    for (int k = 0; k < d; ++k) u.r0cap = std::max(u.r0cap, lt.cap[k] * p_pred[b].cap[k]);
    // SVD scratch (gram/pchol/jacobi parts of a round scratch)
    RoundScratch& rs = u.vrs[b];
    memset(&rs, 0, sizeof(rs));
    rs.gcap = u.gcap;
    rs.splits = u.splits;
    const long long g2 = (long long)u.gcap * u.gcap;
    rs.gram = ar.take<double>(g2 * 2 * u.splits);
    rs.lwork = ar.take<double>(g2 * 2);
    rs.lfac = ar.take<double>(g2);
    rs.jac = ar.take<double>(g2);
    rs.sigma = ar.take<double>(u.gcap);
    rs.usv = ar.take<double>(g2);
    rs.vs = ar.take<double>(g2);
    rs.piv = ar.take<int>(u.gcap);
    rs.misc = ar.take<int>(8);
    rs.scal = ar.take<double>(8);
  }
  return TT_OK;
}

static size_t update_ws_bytes(int32_t batch, const tt_grid* grids, const tt_meas* meas, const tt_train* p_pred,
                              const tt_train* h_out, int32_t lik_rank_cap) {
  Arena ar(nullptr, 0);
  UpdatePlan u;
  if (update_plan(batch, grids, meas, p_pred, h_out, lik_rank_cap, ar, u) != TT_OK) return 0;
  return ar.used + 256;
}

tt_status tt_likelihood(int32_t batch, const tt_grid* grids, const tt_meas* meas, const double* z_dev,
                        int32_t z_stride, const tt_train* l_out, int32_t lik_rank_cap, void* ws, size_t ws_bytes,
                        void* stream) {
  if (!z_dev || !ws || !l_out || batch < 1) {
    set_error("tt_likelihood: bad arguments");
    return TT_ERR_ARG;
  }
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_train(&l_out[b], "l_out", TT_F64));
    for (int j = 0; j <= l_out[b].d; ++j) {
      const int want = (meas[b].kind == 1 && j == 1) ? std::min(lik_rank_cap, l_out[b].n[1]) : 1;
      if (l_out[b].cap[j] != want) {
        set_error("tt_likelihood: l_out capacities must be 1 except cap[1] = min(lik_rank_cap, n[1]) (range)");
        return TT_ERR_SHAPE;
      }
    }
  }
  Arena ar(ws, ws_bytes);
  UpdatePlan u;
  TT_TRY(update_plan(batch, grids, meas, l_out, l_out, lik_rank_cap, ar, u));
  if (!ar.fits()) {
    set_error("tt_likelihood: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  for (int b = 0; b < batch; ++b) u.vl[b] = make_dev(l_out[b]);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(u.dl, u.vl, st));
  TT_TRY(upload(u.drs, u.vrs, st));
  TT_TRY(upload(u.dfc, u.vfc, st));
  return lik_launch(batch, u.dl, u.drs, u.dfc, z_dev, z_stride, u.mbuf, u.mstride, u.any_range, u.n0max, u.n1max,
                    u.gcap, u.splits, st);
}

tt_status tt_likelihood_dense(int32_t batch, const tt_grid* grids, const tt_meas* meas, const double* z_dev,
                              int32_t z_stride, const tt_train* p_out, void* ws, size_t ws_bytes, void* stream) {
  if (!z_dev || !ws || !p_out || !meas || batch < 1) {
    set_error("tt_likelihood_dense: bad arguments");
    return TT_ERR_ARG;
  }
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_train(&p_out[b], "p_out", TT_F64));
    for (int j = 0; j <= p_out[b].d; ++j) {
      const int want = (meas[b].kind == 1 && j == 1) ? p_out[b].n[1] : 1;
      if (p_out[b].cap[j] != want) {
        set_error("tt_likelihood_dense: p_out capacities must be 1 except cap[1] = n[1] (range)");
        return TT_ERR_SHAPE;
      }
    }
  }
  Arena ar(ws, ws_bytes);
  UpdatePlan u;
  TT_TRY(update_plan(batch, grids, meas, p_out, p_out, 1, ar, u));
  if (!ar.fits()) {
    set_error("tt_likelihood_dense: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  for (int b = 0; b < batch; ++b) u.vl[b] = make_dev(p_out[b]);
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(u.dl, u.vl, st));
  TT_TRY(upload(u.dfc, u.vfc, st));
  hipLaunchKernelGGL(lik_dense_kernel, dim3(batch), dim3(256), 0, st, u.dl, u.dfc, z_dev, (long long)z_stride, u.mbuf,
                     u.mstride);
  TTG_LAUNCH_CHECK("lik_dense_kernel");
  if (u.any_range) {
    hipLaunchKernelGGL(lik_dense_pack_kernel, dim3(batch), dim3(256), 0, st, u.dl, u.dfc, u.mbuf, u.mstride);
    TTG_LAUNCH_CHECK("lik_dense_pack_kernel");
  }
  return TT_OK;
}

}  // extern "C"

namespace ttg {

// host descriptors of the two-core trains of the likelihood-build adjoint
struct LikAdjPlan {
  std::vector<tt_train> a, y, ybar, abar;
  std::vector<int> idx;  // range filters
};

static tt_status lik_adj_plan(int32_t batch, const tt_meas* meas, const tt_train* p, const tt_train* l,
                              const tt_train* l_bar, const tt_train* p_bar, Arena* ar, LikAdjPlan& pl) {
  for (int b = 0; b < batch; ++b) {
    for (const tt_train* t : {&p[b], &l[b]}) TT_TRY(check_train(t, "tt_likelihood_adjoint", TT_F64));
    if (l_bar) TT_TRY(check_train(&l_bar[b], "l_bar", TT_F64));
    if (p_bar) TT_TRY(check_train(&p_bar[b], "p_bar", TT_F64));
    const int d = p[b].d;
    const bool range = meas[b].kind == 1;
    if (meas[b].kind != 0 && meas[b].kind != 1) {
      set_error("tt_likelihood_adjoint: meas kind must be 0 or 1");
      return TT_ERR_ARG;
    }
    if (l[b].d != d || (range && d < 2)) {
      set_error("tt_likelihood_adjoint: d differs or range model with d < 2");
      return TT_ERR_SHAPE;
    }
    for (int k = 0; k < d; ++k)
      if (l[b].n[k] != p[b].n[k]) {
        set_error("tt_likelihood_adjoint: mode sizes differ");
        return TT_ERR_SHAPE;
      }
    for (int j = 0; j <= d; ++j) {
      const int pw = (range && j == 1) ? p[b].n[1] : 1;
      if (p[b].cap[j] != pw || (j != 1 || !range ? l[b].cap[j] != 1 : l[b].cap[1] > p[b].n[1])) {
        set_error("tt_likelihood_adjoint: capacities of p or l do not match the likelihood layout");
        return TT_ERR_SHAPE;
      }
      if ((l_bar && l_bar[b].cap[j] != l[b].cap[j]) || (p_bar && p_bar[b].cap[j] != p[b].cap[j])) {
        set_error("tt_likelihood_adjoint: adjoint capacities differ from their primals");
        return TT_ERR_SHAPE;
      }
    }
    if (l_bar && p_bar)
      for (int k = 0; k < d; ++k)
        if (l_bar[b].n[k] != p[b].n[k] || p_bar[b].n[k] != p[b].n[k]) {
          set_error("tt_likelihood_adjoint: mode sizes differ");
          return TT_ERR_SHAPE;
        }
    if (!range) continue;
    pl.idx.push_back(b);
    // the build's rank is at most min(n0, n1), below the capacity
    const int n0 = p[b].n[0], n1 = p[b].n[1], rc = std::min(l[b].cap[1], n0);
    auto mk = [&](int cap1) {
      tt_train t;
      memset(&t, 0, sizeof(t));
      t.d = 2;
      t.n[0] = n1;
      t.n[1] = n0;
      t.cap[0] = t.cap[2] = 1;
      t.cap[1] = cap1;
      t.dtype = TT_F64;
      if (ar) {
        t.cores = ar->take<double>(elems_of(2, t.n, t.cap));
        t.ranks = ar->take<int>(TT_MAXD + 1);
        t.log_scale = ar->take<double>(1);
        t.status = ar->take<int>(1);
      }
      return t;
    };
    pl.a.push_back(mk(n0));
    pl.y.push_back(mk(rc));
    pl.ybar.push_back(mk(rc));
    pl.abar.push_back(mk(n0));
  }
  return TT_OK;
}

}  // namespace ttg

extern "C" {

size_t tt_likelihood_adjoint_workspace(int32_t batch, const tt_meas* meas, const tt_train* p, const tt_train* l) {
  if (batch < 1 || !meas || !p || !l) return 0;
  Arena ar(nullptr, 0);
  LikAdjPlan pl;
  ar.take<LikAdjJob>(batch);
  if (lik_adj_plan(batch, meas, p, l, nullptr, nullptr, &ar, pl) != TT_OK) return 0;
  size_t total = ar.used + 1024;
  if (!pl.idx.empty())
    total += tt_round_adjoint_workspace((int32_t)pl.idx.size(), pl.a.data(), pl.y.data()) + 256;
  return total;
}

tt_status tt_likelihood_adjoint(int32_t batch, const tt_meas* meas, const tt_train* p, const tt_train* l,
                                const tt_train* l_bar, const tt_train* p_bar, void* ws, size_t ws_bytes,
                                void* stream) {
  if (batch < 1 || !meas || !p || !l || !l_bar || !p_bar || !ws) {
    set_error("tt_likelihood_adjoint: bad arguments");
    return TT_ERR_ARG;
  }
  Arena ar(ws, ws_bytes);
  LikAdjPlan pl;
  LikAdjJob* dj = ar.take<LikAdjJob>(batch);
  TT_TRY(lik_adj_plan(batch, meas, p, l, l_bar, p_bar, &ar, pl));
  const int nr = (int)pl.idx.size();
  size_t rbytes = 0;
  void* rws = nullptr;
  if (nr > 0) {
    rbytes = tt_round_adjoint_workspace(nr, pl.a.data(), pl.y.data());
    rws = ar.take<char>(rbytes);
  }
  if (!ar.fits()) {
    set_error("tt_likelihood_adjoint: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  std::vector<LikAdjJob> jobs(batch);
  for (int b = 0, q = 0; b < batch; ++b) {
    LikAdjJob& J = jobs[b];
    memset(&J, 0, sizeof(J));
    J.p = make_dev(p[b]);
    J.l = make_dev(l[b]);
    J.lbar = make_dev(l_bar[b]);
    J.pbar = make_dev(p_bar[b]);
    J.range = meas[b].kind == 1;
    if (J.range) {
      J.a = make_dev(pl.a[q]);
      J.y = make_dev(pl.y[q]);
      J.ybar = make_dev(pl.ybar[q]);
      J.abar = make_dev(pl.abar[q]);
      ++q;
    }
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(dj, jobs, st));
  if (nr > 0) {
    hipLaunchKernelGGL(lik_adj_pack_kernel, dim3(batch), dim3(256), 0, st, dj);
    TTG_LAUNCH_CHECK("lik_adj_pack_kernel");
    TT_TRY(tt_round_adjoint(nr, pl.a.data(), pl.y.data(), pl.ybar.data(), pl.abar.data(), nullptr, rws, rbytes,
                            stream));
  }
  hipLaunchKernelGGL(lik_adj_unpack_kernel, dim3(batch), dim3(256), 0, st, dj);
  TTG_LAUNCH_CHECK("lik_adj_unpack_kernel");
  return TT_OK;
}

tt_status tt_prior(int32_t batch, const tt_grid* grids, const double* m0, const double* p0_diag, const tt_train* out,
                   void* ws, size_t ws_bytes, void* stream) {
  if (batch < 1 || !grids || !m0 || !p0_diag || !out || !ws) {
    set_error("tt_prior: bad arguments");
    return TT_ERR_ARG;
  }
  const int dtype = out[0].dtype, d = out[0].d;
  std::vector<DevTT> vt(batch);
  std::vector<FilterConst> vfc(batch);
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_grid(&grids[b]));
    TT_TRY(check_train(&out[b], "out", dtype));
    if (grids[b].d != d || out[b].d != d) {
      set_error("tt_prior: d differs");
      return TT_ERR_SHAPE;
    }
    for (int k = 0; k < d; ++k) {
      if (grids[b].n[k] != out[b].n[k]) {
        set_error("tt_prior: grid and train mode sizes differ");
        return TT_ERR_SHAPE;
      }
      if (!(p0_diag[b * d + k] > 0.0)) {
        set_error("tt_prior: prior variances must be positive");
        return TT_ERR_ARG;
      }
    }
    vt[b] = make_dev(out[b]);
    vfc[b] = make_const(grids[b], nullptr);
    for (int k = 0; k < d; ++k) {
      vfc[b].m0[k] = m0[b * d + k];
      vfc[b].p0[k] = p0_diag[b * d + k];
    }
  }
  Arena ar(ws, ws_bytes);
  DevTT* dt = ar.take<DevTT>(batch);
  FilterConst* dfc = ar.take<FilterConst>(batch);
  if (!ar.fits()) {
    set_error("tt_prior: workspace too small");
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(dt, vt, st));
  TT_TRY(upload(dfc, vfc, st));
  if (dtype == TT_F64)
    hipLaunchKernelGGL((prior_kernel<double>), dim3(batch), dim3(256), 0, st, dt, dfc);
  else
    hipLaunchKernelGGL((prior_kernel<float>), dim3(batch), dim3(256), 0, st, dt, dfc);
  TTG_LAUNCH_CHECK("prior_kernel");
  return TT_OK;
}

static tt_status adj_pair(int32_t batch, const tt_train* x, const tt_train* y, const char* what, DevTT** dx,
                          DevTT** dy, void* ws, size_t ws_bytes, hipStream_t st) {
  std::vector<DevTT> vx(batch), vy(batch);
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_train(&x[b], what, TT_F64));
    TT_TRY(check_train(&y[b], what, TT_F64));
    TT_TRY(check_like(x[b], y[b], what));
    vx[b] = make_dev(x[b]);
    vy[b] = make_dev(y[b]);
  }
  Arena ar(ws, ws_bytes);
  *dx = ar.take<DevTT>(batch);
  *dy = ar.take<DevTT>(batch);
  if (!ar.fits()) {
    set_error("%s: workspace too small", what);
    return TT_ERR_WORKSPACE;
  }
  TT_TRY(upload(*dx, vx, st));
  TT_TRY(upload(*dy, vy, st));
  return TT_OK;
}

tt_status tt_adjoint_axpy(int32_t batch, double alpha, const tt_train* x, const tt_train* y, void* ws,
                          size_t ws_bytes, void* stream) {
  if (batch < 1 || !x || !y || !ws) {
    set_error("tt_adjoint_axpy: bad arguments");
    return TT_ERR_ARG;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  DevTT *dx, *dy;
  TT_TRY(adj_pair(batch, x, y, "tt_adjoint_axpy", &dx, &dy, ws, ws_bytes, st));
  int pel = 1;
  for (int b = 0; b < batch; ++b)
    for (int k = 0; k < x[b].d; ++k) pel = std::max(pel, x[b].cap[k] * x[b].n[k] * x[b].cap[k + 1]);
  hipLaunchKernelGGL(adj_axpy_kernel, dim3(stride_grid(cdiv(pel, 256), batch), x[0].d, batch), dim3(256), 0, st, dx,
                     dy, alpha);
  TTG_LAUNCH_CHECK("adj_axpy_kernel");
  return TT_OK;
}

tt_status tt_adjoint_inner(int32_t batch, const tt_train* a_bar, const tt_train* b, double* out_dev, void* ws,
                           size_t ws_bytes, void* stream) {
  if (batch < 1 || !a_bar || !b || !out_dev || !ws) {
    set_error("tt_adjoint_inner: bad arguments");
    return TT_ERR_ARG;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  DevTT *da, *db;
  TT_TRY(adj_pair(batch, a_bar, b, "tt_adjoint_inner", &da, &db, ws, ws_bytes, st));
  hipLaunchKernelGGL(adj_inner_kernel, dim3(batch), dim3(256), 0, st, da, db, out_dev);
  TTG_LAUNCH_CHECK("adj_inner_kernel");
  return TT_OK;
}

tt_status tt_align_signs(int32_t batch, const tt_train* ref, const tt_train* t, void* ws, size_t ws_bytes,
                         void* stream) {
  if (batch < 1 || !ref || !t || !ws) {
    set_error("tt_align_signs: bad arguments");
    return TT_ERR_ARG;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  std::vector<DevTT> vr(batch), vt(batch);
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_train(&ref[b], "tt_align_signs", TT_F64));
    TT_TRY(check_train(&t[b], "tt_align_signs", TT_F64));
    TT_TRY(check_like(ref[b], t[b], "tt_align_signs"));
    if (t[b].d != t[0].d) {
      set_error("tt_align_signs: d differs");
      return TT_ERR_SHAPE;
    }
    vr[b] = make_dev(ref[b]);
    vt[b] = make_dev(t[b]);
  }
  const size_t m2 = (size_t)2 * ALIGN_RMAX * ALIGN_RMAX;
  Arena ar(ws, ws_bytes);
  DevTT* dr = ar.take<DevTT>(batch);
  DevTT* dt = ar.take<DevTT>(batch);
  double* buf = ar.take<double>(batch * m2);
  double* work = ar.take<double>(batch * m2);
  double* usv = ar.take<double>(batch * m2);
  double* sigma = ar.take<double>((size_t)batch * ALIGN_RMAX);
  int* rbuf = ar.take<int>(batch);
  if (!ar.fits()) {
    set_error("tt_align_signs: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  TT_TRY(upload(dr, vr, st));
  TT_TRY(upload(dt, vt, st));
  for (int k = 0; k + 1 < t[0].d; ++k) {
    hipLaunchKernelGGL(align_cos_kernel, dim3(batch), dim3(256), 0, st, dr, dt, k, buf, rbuf);
    TTG_LAUNCH_CHECK("align_cos_kernel");
    TT_TRY(launch_jacobi(FAlignJacobi{buf, rbuf, work, sigma, usv}, batch, st));
    hipLaunchKernelGGL(align_apply_kernel, dim3(batch), dim3(256), 0, st, dt, k, sigma, usv, rbuf);
    TTG_LAUNCH_CHECK("align_apply_kernel");
  }
  return TT_OK;
}

size_t tt_update_workspace(int32_t batch, const tt_grid* grids, const tt_meas* meas, const tt_train* p_pred,
                           const tt_train* h_out, int32_t lik_rank_cap) {
  return update_ws_bytes(batch, grids, meas, p_pred, h_out, lik_rank_cap);
}

tt_status tt_update(int32_t batch, const tt_grid* grids, const tt_meas* meas, const double* z_dev, int32_t z_stride,
                    const tt_train* p_pred, const tt_train* h_out, int32_t lik_rank_cap, double* log_c_dev, void* ws,
                    size_t ws_bytes, void* stream) {
  if (!z_dev || !log_c_dev || !ws) {
    set_error("tt_update: null pointer");
    return TT_ERR_ARG;
  }
  Arena ar(ws, ws_bytes);
  UpdatePlan u;
  TT_TRY(update_plan(batch, grids, meas, p_pred, h_out, lik_rank_cap, ar, u));
  if (!ar.fits()) {
    set_error("tt_update: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(u.dl, u.vl, st));
  TT_TRY(upload(u.dp, u.vp, st));
  TT_TRY(upload(u.dh, u.vh, st));
  TT_TRY(upload(u.drs, u.vrs, st));
  TT_TRY(upload(u.dfc, u.vfc, st));
  TT_TRY(lik_launch(batch, u.dl, u.drs, u.dfc, z_dev, z_stride, u.mbuf, u.mstride, u.any_range, u.n0max, u.n1max,
                    u.gcap, u.splits, st));
  const int d = p_pred[0].d;
  if (p_pred[0].dtype == TT_F64) {
    TT_TRY(launch_dot<double>(batch, u.dl, u.dp, u.dfc, log_c_dev, 1LL, u.vbuf, u.vstride, u.tofs, st));
    TT_TRY(launch_hadamard<double>(batch, d, u.r0cap, u.dl, u.dp, u.dh, st));
  } else {
    TT_TRY(launch_dot<float>(batch, u.dl, u.dp, u.dfc, log_c_dev, 1LL, u.vbuf, u.vstride, u.tofs, st));
    TT_TRY(launch_hadamard<float>(batch, d, u.r0cap, u.dl, u.dp, u.dh, st));
  }
  return TT_OK;
}

// ---------------------------------------------------------------------------
// tt_normalize_moments
// ---------------------------------------------------------------------------
size_t tt_normalize_moments_workspace(int32_t batch, const tt_train* t) {
  if (batch < 1 || !t) return 0;
  int rcap = 1;
  for (int b = 0; b < batch; ++b)
    for (int j = 0; j <= t[b].d && j <= TT_MAXD; ++j) rcap = std::max(rcap, t[b].cap[j]);
  Arena ar(nullptr, 0);
  ar.take<DevTT>(batch);
  ar.take<FilterConst>(batch);
  ar.take<double>((size_t)batch * moments_scratch_per_filter(t[0].d, rcap));
  return ar.used + 256;
}

}  // extern "C"

namespace ttg {

// tt_normalize_moments on an explicit scratch area (the caller's workspace,
// or the library's static array for tt_normalize_moments_noalloc).
static tt_status normalize_moments_impl(const char* who, int32_t batch, const tt_grid* grids, const tt_train* t,
                                        double* log_mass_dev, double* mean_dev, double* cov_dev, void* ws,
                                        size_t ws_bytes, void* stream, bool no_ring = false) {
  if (batch < 1 || !grids || !t || !ws) {
    set_error("%s: bad arguments", who);
    return TT_ERR_ARG;
  }
  if (cov_dev && !mean_dev) {
    set_error("%s: cov needs mean", who);
    return TT_ERR_ARG;
  }
  const int dtype = t[0].dtype, d = t[0].d;
  std::vector<DevTT> vt(batch);
  std::vector<FilterConst> vfc(batch);
  int rcap = 1;
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_grid(&grids[b]));
    TT_TRY(check_train(&t[b], "t", dtype));
    if (t[b].d != d || grids[b].d != d) {
      set_error("%s: d differs", who);
      return TT_ERR_SHAPE;
    }
    for (int j = 0; j <= d; ++j) rcap = std::max(rcap, t[b].cap[j]);
    vt[b] = make_dev(t[b]);
    vfc[b] = make_const(grids[b], nullptr);
  }
  if (rcap > 64) {
    set_error("%s: rank capacity %d > 64", who, rcap);
    return TT_ERR_SHAPE;
  }
  Arena ar(ws, ws_bytes);
  DevTT* dt = ar.take<DevTT>(batch);
  FilterConst* dfc = ar.take<FilterConst>(batch);
  const long long spf = (long long)moments_scratch_per_filter(d, rcap);
  double* scratch = ar.take<double>((size_t)batch * spf);
  if (!ar.fits()) {
    set_error("%s: %zu bytes of scratch needed, %zu available", who, ar.used, ws_bytes);
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (no_ring) {
    TT_TRY(upload_wait(dt, vt, st));
    TT_TRY(upload_wait(dfc, vfc, st));
  } else {
    TT_TRY(upload(dt, vt, st));
    TT_TRY(upload(dfc, vfc, st));
  }
  if (dtype == TT_F64)
    return launch_moments<double>(batch, dt, dfc, log_mass_dev, 1, mean_dev, d, cov_dev, (long long)d * d, scratch,
                                  spf, rcap, st);
  return launch_moments<float>(batch, dt, dfc, log_mass_dev, 1, mean_dev, d, cov_dev, (long long)d * d, scratch, spf,
                               rcap, st);
}

// Scratch of tt_normalize_moments_noalloc: one static array per device (the
// descriptor tables and the per-filter contraction chains), reached from the
// host only through the device address hipGetSymbolAddress returns for the
// current device, looked up once per device on the first call there.
namespace noalloc {
static __device__ __align__(256) char scratch[TT_NOALLOC_SCRATCH_BYTES];
}

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];

static tt_status scratch_address(void** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) {
    set_error("tt_normalize_moments_noalloc: device %d out of range", dev);
    return TT_ERR_ARG;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(noalloc::scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) {
      set_error("tt_normalize_moments_noalloc: no device address for the scratch array");
      return TT_ERR_HIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return TT_OK;
}

}  // namespace ttg

extern "C" {

tt_status tt_normalize_moments(int32_t batch, const tt_grid* grids, const tt_train* t, double* log_mass_dev,
                               double* mean_dev, double* cov_dev, void* ws, size_t ws_bytes, void* stream) {
  return ttg::normalize_moments_impl("tt_normalize_moments", batch, grids, t, log_mass_dev, mean_dev, cov_dev, ws,
                                     ws_bytes, stream);
}

tt_status tt_normalize_moments_noalloc(int32_t batch, const tt_grid* grids, const tt_train* t, double* log_mass_dev,
                                       double* mean_dev, double* cov_dev, void* stream) {
  using namespace ttg;
  if (batch < 1 || !grids || !t) {
    set_error("tt_normalize_moments_noalloc: bad arguments");
    return TT_ERR_ARG;
  }
  void* ptr = nullptr;
  TT_TRY(scratch_address(&ptr));
  return normalize_moments_impl("tt_normalize_moments_noalloc", batch, grids, t, log_mass_dev, mean_dev, cov_dev, ptr,
                                TT_NOALLOC_SCRATCH_BYTES, stream, true);
}

// ---------------------------------------------------------------------------
// tt_kernel_build
// ---------------------------------------------------------------------------
static bool invert_spd(int d, const double* q, double* inv, double* det) {
  // Gauss-Jordan with partial pivoting on a copy
  double a[TT_MAXD][2 * TT_MAXD];
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < 2 * d; ++j) a[i][j] = (j < d) ? q[i * d + j] : (j - d == i ? 1.0 : 0.0);
  double dt = 1.0;
  for (int c = 0; c < d; ++c) {
    int p = c;
    for (int i = c + 1; i < d; ++i)
      if (std::fabs(a[i][c]) > std::fabs(a[p][c])) p = i;
    if (!(std::fabs(a[p][c]) > 0.0)) return false;
    if (p != c) {
      for (int j = 0; j < 2 * d; ++j) std::swap(a[p][j], a[c][j]);
      dt = -dt;
    }
    const double piv = a[c][c];
    dt *= piv;
    for (int j = 0; j < 2 * d; ++j) a[c][j] /= piv;
    for (int i = 0; i < d; ++i)
      if (i != c) {
        const double f = a[i][c];
        for (int j = 0; j < 2 * d; ++j) a[i][j] -= f * a[c][j];
      }
  }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) inv[i * d + j] = a[i][d + j];
  *det = dt;
  return dt > 0.0;
}

struct KernelPlan {
  long long total;
  int taps[TT_MAXD];
  double* dense;  // batch x total
  double* buf2;   // batch x total
  DevTT* dK64;
  DevTT* dKout;
  RoundScratch* drs;
  KernelEvalArgs* dka;
  std::vector<DevTT> k64;  // FP64 result per filter (the output itself when it is FP64)
  std::vector<RoundScratch> rs;
  int gcap, splits;
};

// Buffers of a batched kernel build: every filter shares d and the offset
// box (taps); grids, Q and rank capacities may differ.  outs == nullptr
// sizes the FP64 staging TTs for FP32 outputs of the given capacities.
static tt_status kernel_plan(int batch, const tt_grid* grids, const int32_t* halfwidths, const int32_t* caps,
                             const int* out_dtypes, Arena& ar, KernelPlan& kp) {
  const int d = grids[0].d;
  if (d > 8) {
    set_error("tt_kernel_build: dense build supports d <= 8");
    return TT_ERR_SHAPE;
  }
  long long total = 1;
  for (int l = 0; l < d; ++l) {
    if (halfwidths[l] < 0 || 2 * halfwidths[l] + 1 > 4095) {
      set_error("tt_kernel_build: bad halfwidth");
      return TT_ERR_SHAPE;
    }
    kp.taps[l] = 2 * halfwidths[l] + 1;
    total *= kp.taps[l];
    if (total > (1LL << 28)) {
      set_error("tt_kernel_build: dense kernel larger than 2^28 taps");
      return TT_ERR_SHAPE;
    }
  }
  kp.total = total;
  int gcap = 1;
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_grid(&grids[b]));
    if (grids[b].d != d) {
      set_error("tt_kernel_build: d differs within the batch");
      return TT_ERR_SHAPE;
    }
    const int32_t* cap = caps + (long long)b * (d + 1);
    if (cap[0] != 1 || cap[d] != 1) {
      set_error("tt_kernel_build: cap[0] and cap[d] must be 1");
      return TT_ERR_SHAPE;
    }
    for (int k = 0; k < d; ++k) gcap = std::max(gcap, cap[k] * kp.taps[k]);
  }
  if (gcap > 1024) {
    set_error("tt_kernel_build: cap*taps = %d exceeds 1024", gcap);
    return TT_ERR_SHAPE;
  }
  if ((double)batch * (double)total > 4.0e9) {
    set_error("tt_kernel_build: batch x dense kernel too large");
    return TT_ERR_SHAPE;
  }
  kp.gcap = gcap;
  kp.splits = GRAM_PLANES;
  kp.dense = ar.take<double>((size_t)batch * total);
  kp.buf2 = ar.take<double>((size_t)batch * total);
  kp.k64.assign(batch, DevTT{});
  kp.rs.assign(batch, RoundScratch{});
  for (int b = 0; b < batch; ++b) {
    const int32_t* cap = caps + (long long)b * (d + 1);
    if (!out_dtypes || out_dtypes[b] != TT_F64) {  // FP64 staging for an FP32 output
      tt_train t64;
      memset(&t64, 0, sizeof(t64));
      t64.d = d;
      t64.dtype = TT_F64;
      for (int k = 0; k < d; ++k) t64.n[k] = kp.taps[k];
      for (int j = 0; j <= d; ++j) t64.cap[j] = cap[j];
      t64.cores = ar.take<double>(elems_of(d, t64.n, t64.cap));
      t64.ranks = ar.take<int>(TT_MAXD + 1);
      t64.log_scale = ar.take<double>(1);
      t64.status = ar.take<int>(1);
      kp.k64[b] = make_dev(t64);
    }
    RoundScratch& rs = kp.rs[b];
    memset(&rs, 0, sizeof(rs));
    rs.gcap = gcap;
    rs.splits = kp.splits;
    const long long g2 = (long long)gcap * gcap;
    rs.gram = ar.take<double>(g2 * 2 * kp.splits);
    rs.lwork = ar.take<double>(g2 * 2);
    rs.lfac = ar.take<double>(g2);
    rs.jac = ar.take<double>(g2);
    rs.sigma = ar.take<double>(gcap);
    rs.usv = ar.take<double>(g2);
    rs.piv = ar.take<int>(gcap);
    rs.misc = ar.take<int>(8);
    rs.scal = ar.take<double>(8);
  }
  kp.dK64 = ar.take<DevTT>(batch);
  kp.dKout = ar.take<DevTT>(batch);
  kp.drs = ar.take<RoundScratch>(batch);
  kp.dka = ar.take<KernelEvalArgs>(batch);
  return TT_OK;
}

static tt_status kernel_build_run(int batch, const tt_grid* grids, const double* q, const int32_t* halfwidths,
                                  double svd_tol, const tt_train* out, void* ws, size_t ws_bytes, void* stream) {
  if (batch < 1 || !grids || !q || !halfwidths || !out || !ws || !(svd_tol >= 0.0)) {
    set_error("tt_kernel_build: bad arguments");
    return TT_ERR_ARG;
  }
  const int d = grids[0].d;
  std::vector<int32_t> caps((size_t)batch * (d + 1));
  std::vector<int> dtypes(batch);
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_train(&out[b], "out"));
    if (out[b].d != d) {
      set_error("tt_kernel_build: out->d != grid->d");
      return TT_ERR_SHAPE;
    }
    for (int k = 0; k < d; ++k)
      if (out[b].n[k] != 2 * halfwidths[k] + 1) {
        set_error("tt_kernel_build: out->n[%d] must be 2*h+1", k);
        return TT_ERR_SHAPE;
      }
    for (int j = 0; j <= d; ++j) caps[(size_t)b * (d + 1) + j] = out[b].cap[j];
    dtypes[b] = out[b].dtype;
    if (dtypes[b] != dtypes[0]) {
      set_error("tt_kernel_build: output dtypes differ within the batch");
      return TT_ERR_ARG;
    }
  }
  Arena ar(ws, ws_bytes);
  KernelPlan kp;
  TT_TRY(kernel_plan(batch, grids, halfwidths, caps.data(), dtypes.data(), ar, kp));
  if (!ar.fits()) {
    set_error("tt_kernel_build: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  std::vector<KernelEvalArgs> vka(batch);
  std::vector<DevTT> vout(batch);
  bool any_f32 = false;
  for (int b = 0; b < batch; ++b) {
    KernelEvalArgs& ka = vka[b];
    memset(&ka, 0, sizeof(ka));
    ka.d = d;
    double det = 0.0, logdelta = 0.0;
    if (!invert_spd(d, q + (size_t)b * d * d, ka.qinv, &det)) {
      set_error("tt_kernel_build: Q is not positive definite (filter %d)", b);
      return TT_ERR_ARG;
    }
    for (int l = 0; l < d; ++l) {
      ka.taps[l] = kp.taps[l];
      ka.dx[l] = (grids[b].hi[l] - grids[b].lo[l]) / (double)(grids[b].n[l] - 1);
      logdelta += std::log(ka.dx[l]);
    }
    ka.cnorm = std::exp(-0.5 * d * std::log(2.0 * M_PI) - 0.5 * std::log(det) + logdelta);
    ka.total = kp.total;
    vout[b] = make_dev(out[b]);
    if (out[b].dtype == TT_F64)
      kp.k64[b] = vout[b];
    else
      any_f32 = true;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(kp.dK64, kp.k64, st));
  TT_TRY(upload(kp.dKout, vout, st));
  TT_TRY(upload(kp.drs, kp.rs, st));
  TT_TRY(upload(kp.dka, vka, st));
  hipLaunchKernelGGL(ksvd_init_kernel, dim3(batch), dim3(1), 0, st, kp.dK64);
  TTG_LAUNCH_CHECK("ksvd_init_kernel");
  hipLaunchKernelGGL(kernel_dense_kernel, dim3(std::min(cdiv(kp.total, 256), 8192), batch), dim3(256), 0, st, kp.dka,
                     kp.dense, kp.total);
  TTG_LAUNCH_CHECK("kernel_dense_kernel");
  double* cur = kp.dense;
  double* nxt = kp.buf2;
  long long cols = kp.total / kp.taps[0];
  int capmax[TT_MAXD + 1] = {0};
  for (int b = 0; b < batch; ++b)
    for (int j = 0; j <= d; ++j) capmax[j] = std::max(capmax[j], out[b].cap[j]);
  for (int k = 0; k < d - 1; ++k) {
    KsvdCtx c{kp.dK64, kp.drs, cur, nxt, cols, k, d, kp.total};
    const int rows_cap = capmax[k] * kp.taps[k];
    TT_TRY((launch_gram<double, AccDD>(FKsvdGram{c}, batch, rows_cap, cols, kp.splits, st)));
    TT_TRY((launch_pchol<AccDD>(FKsvdPchol{c}, batch, kp.gcap, st)));
    TT_TRY((launch_jacobi(FKsvdJacobi{c}, batch, st)));
    hipLaunchKernelGGL(ksvd_select_kernel, dim3(batch), dim3(256), 0, st, kp.dK64, kp.drs, k, svd_tol);
    TTG_LAUNCH_CHECK("ksvd_select_kernel");
    TT_TRY((launch_gemm<double, double, double, double>(FKsvdNext{c}, batch, capmax[k + 1], cols, st)));
    std::swap(cur, nxt);
    cols /= kp.taps[k + 1];
  }
  hipLaunchKernelGGL(ksvd_last_kernel, dim3(64, batch), dim3(256), 0, st, kp.dK64, cur, kp.total);
  TTG_LAUNCH_CHECK("ksvd_last_kernel");
  if (any_f32) {  // every output is FP32 (one dtype per batch)
    hipLaunchKernelGGL((convert_tt_kernel<float>), dim3(64, batch), dim3(256), 0, st, kp.dK64, kp.dKout);
    TTG_LAUNCH_CHECK("convert_tt_kernel");
  }
  return TT_OK;
}

}  // namespace ttg

extern "C" {

size_t tt_kernel_build_workspace(const tt_grid* grid, const int32_t* halfwidths, const int32_t* cap) {
  if (!grid || !halfwidths || !cap) return 0;
  Arena ar(nullptr, 0);
  KernelPlan kp;
  if (kernel_plan(1, grid, halfwidths, cap, nullptr, ar, kp) != TT_OK) return 0;
  return ar.used + 256;
}

size_t tt_kernel_build_batch_workspace(int32_t batch, const tt_grid* grids, const int32_t* halfwidths,
                                       const int32_t* caps) {
  if (batch < 1 || !grids || !halfwidths || !caps) return 0;
  Arena ar(nullptr, 0);
  KernelPlan kp;
  if (kernel_plan(batch, grids, halfwidths, caps, nullptr, ar, kp) != TT_OK) return 0;
  return ar.used + 256;
}

tt_status tt_kernel_build(const tt_grid* grid, const double* q, const int32_t* halfwidths, double svd_tol,
                          const tt_train* out, void* ws, size_t ws_bytes, void* stream) {
  return kernel_build_run(1, grid, q, halfwidths, svd_tol, out, ws, ws_bytes, stream);
}

tt_status tt_kernel_build_batch(int32_t batch, const tt_grid* grids, const double* q, const int32_t* halfwidths,
                                double svd_tol, const tt_train* out, void* ws, size_t ws_bytes, void* stream) {
  return kernel_build_run(batch, grids, q, halfwidths, svd_tol, out, ws, ws_bytes, stream);
}

}  // extern "C"

// ===========================================================================
// tt_filter_run
// ===========================================================================
namespace ttg {

struct RunPlan {
  std::vector<DevTT> vP, vX, vL, vH, vK;
  std::vector<RoundScratch> vrs;
  std::vector<FilterConst> vfc;
  DevTT *dP = nullptr, *dX = nullptr, *dL = nullptr, *dH = nullptr, *dK = nullptr;
  RoundScratch* drs = nullptr;
  FilterConst* dfc = nullptr;
  double* mbuf = nullptr;
  long long mstride = 0;
  double* vbuf = nullptr;
  int vcap = 1;
  long long vstride = 0, tofs = 0;
  double* mscr = nullptr;
  long long mspf = 0;
  int mrcap = 1;
  double* lmass = nullptr;
  RoundShape shX, shH;
  int r0capX = 1, r0capH = 1;
  size_t csmem = 0;
  // fused FFT prediction
  bool fused = false;
  std::vector<FusedPred> vfp;
  FusedPred* dfp = nullptr;
  std::vector<int> kL, klog2;        // FFT length per kernel
  std::vector<void*> khat;           // spectra per kernel
  std::vector<void*> ktw;            // twiddles per kernel
  std::vector<long long> kpitch;
  DevTT* dKk = nullptr;              // one descriptor per kernel (for the spectra launch)
  std::vector<DevTT> vKk;
  int Lmax = 0, kcap = 1, pcap = 1, hmax = 0;
  bool any_range = false;
  int n0max = 1, n1max = 1, gcap = 1, splits = 1;
  int d = 0;
  DevTT* dS = nullptr;               // source and destination tables of tt_filter_state
};

static tt_status run_plan(int32_t batch, const tt_filter_spec* specs, const tt_train* kernels, int32_t n_kernels,
                          int32_t precision, int32_t* status_dev, Arena& ar, RunPlan& p) {
  if (batch < 1 || !specs) {
    set_error("tt_filter_run: bad arguments");
    return TT_ERR_ARG;
  }
  if (precision != TT_F64 && precision != TT_F32) {
    set_error("tt_filter_run: precision must be TT_F64 or TT_F32");
    return TT_ERR_ARG;
  }
  const bool f64 = precision == TT_F64;
  const int d = specs[0].grid.d;
  p.d = d;
  if (d < 2) {
    set_error("tt_filter_run: d must be >= 2");
    return TT_ERR_SHAPE;
  }
  p.vP.resize(batch);
  p.vX.resize(batch);
  p.vL.resize(batch);
  p.vH.resize(batch);
  p.vK.resize(batch);
  p.vrs.resize(batch);
  p.vfc.resize(batch);
  std::vector<DevTT> vU(batch);
  const size_t esz = f64 ? 8 : 4;
  p.dP = ar.take<DevTT>(batch);
  p.dX = ar.take<DevTT>(batch);
  p.dL = ar.take<DevTT>(batch);
  p.dH = ar.take<DevTT>(batch);
  p.dK = ar.take<DevTT>(batch);
  p.drs = ar.take<RoundScratch>(batch);
  p.dfc = ar.take<FilterConst>(batch);
  int* ints = ar.take<int>((size_t)batch * 4 * (TT_MAXD + 1));
  double* dbl = ar.take<double>((size_t)batch * 4);
  for (int b = 0; b < batch; ++b) {
    const tt_filter_spec& s = specs[b];
    TT_TRY(check_grid(&s.grid));
    if (s.grid.d != d) {
      set_error("tt_filter_run: all filters must share d");
      return TT_ERR_SHAPE;
    }
    if (s.cap < 1 || s.kernel_cap < 1 || s.lik_rank_cap < 1 || !(s.eps >= 0.0)) {
      set_error("tt_filter_run: filter %d: cap, kernel_cap, lik_rank_cap >= 1 and eps >= 0 required", b);
      return TT_ERR_ARG;
    }
    if (s.eps != specs[0].eps) {
      set_error("tt_filter_run: filter %d: every filter of a batch must share the rounding tolerance eps", b);
      return TT_ERR_ARG;
    }
    if (s.meas.kind != 0 && s.meas.kind != 1) {
      set_error("tt_filter_run: meas kind must be 0 or 1");
      return TT_ERR_ARG;
    }
    for (int l = 0; l < d; ++l)
      if (!(s.p0_diag[l] > 0.0)) {
        set_error("tt_filter_run: prior variances must be positive");
        return TT_ERR_ARG;
      }
    if (kernels) {
      if (s.kernel_index < 0 || s.kernel_index >= n_kernels) {
        set_error("tt_filter_run: filter %d: kernel_index out of range", b);
        return TT_ERR_ARG;
      }
      const tt_train& kt = kernels[s.kernel_index];
      TT_TRY(check_train(&kt, "kernel", precision));
      if (kt.d != d) {
        set_error("tt_filter_run: kernel d differs");
        return TT_ERR_SHAPE;
      }
      for (int k = 0; k < d; ++k) {
        if (kt.n[k] % 2 != 1) {
          set_error("tt_filter_run: kernel length must be odd");
          return TT_ERR_SHAPE;
        }
        if (kt.cap[k + 1] > s.kernel_cap && k + 1 < d) {
          set_error("tt_filter_run: kernel cap exceeds spec.kernel_cap");
          return TT_ERR_SHAPE;
        }
      }
      p.vK[b] = make_dev(kt);
    }
    p.vfc[b] = make_const(s.grid, &s.meas);
    for (int l = 0; l < d; ++l) {
      p.vfc[b].m0[l] = s.m0[l];
      p.vfc[b].p0[l] = s.p0_diag[l];
    }
    p.any_range = p.any_range || s.meas.kind == 1;
    p.n0max = std::max(p.n0max, s.grid.n[0]);
    p.n1max = std::max(p.n1max, s.grid.n[1]);
    tt_train tP, tX, tL, tH;
    memset(&tP, 0, sizeof(tP));
    tP.d = d;
    tP.dtype = precision;
    for (int k = 0; k < d; ++k) tP.n[k] = s.grid.n[k];
    tX = tH = tL = tP;
    tL.dtype = TT_F64;
    const int lc = (s.meas.kind == 1) ? std::min(s.lik_rank_cap, s.grid.n[1]) : 1;
    for (int j = 0; j <= d; ++j) {
      const bool edge = (j == 0 || j == d);
      tP.cap[j] = edge ? 1 : s.cap;
      tX.cap[j] = edge ? 1 : s.cap * s.kernel_cap;
      tL.cap[j] = (j == 1 && d > 1) ? lc : 1;
      tH.cap[j] = tL.cap[j] * tP.cap[j];
    }
    int* rk = ints + (size_t)b * 4 * (TT_MAXD + 1);
    double* ls = dbl + (size_t)b * 4;
    int* stw = status_dev ? status_dev + b : nullptr;
    tP.cores = ar.take<char>(elems_of(d, tP.n, tP.cap) * esz);
    tX.cores = ar.take<char>(elems_of(d, tX.n, tX.cap) * esz);
    tL.cores = ar.take<double>(elems_of(d, tL.n, tL.cap));
    tH.cores = ar.take<char>(elems_of(d, tH.n, tH.cap) * esz);
    tP.ranks = rk;
    tX.ranks = rk ? rk + (TT_MAXD + 1) : nullptr;
    tL.ranks = rk ? rk + 2 * (TT_MAXD + 1) : nullptr;
    tH.ranks = rk ? rk + 3 * (TT_MAXD + 1) : nullptr;
    tP.log_scale = ls;
    tX.log_scale = ls ? ls + 1 : nullptr;
    tL.log_scale = ls ? ls + 2 : nullptr;
    tH.log_scale = ls ? ls + 3 : nullptr;
    tP.status = tX.status = tL.status = tH.status = stw;
    p.vP[b] = make_dev(tP);
    p.vX[b] = make_dev(tX);
    p.vL[b] = make_dev(tL);
    p.vH[b] = make_dev(tH);
    tt_train tU = tX;
    for (int j = 0; j <= d; ++j) tU.cap[j] = std::max(tX.cap[j], tH.cap[j]);
    vU[b] = make_dev(tU);
    for (int j = 0; j <= d; ++j) p.vcap = std::max(p.vcap, tH.cap[j]);
    for (int k = 0; k < d; ++k) {
      p.r0capX = std::max(p.r0capX, tX.cap[k]);
      p.r0capH = std::max(p.r0capH, tH.cap[k]);
    }
    p.mrcap = std::max(p.mrcap, s.cap);
    if (kernels) p.csmem = std::max(p.csmem, f64 ? conv_smem<double>(p.vK[b], p.vP[b]) : conv_smem<float>(p.vK[b], p.vP[b]));
  }
  if (p.csmem > 160 * 1024) {
    set_error("tt_filter_run: kernel/fibre too long for LDS");
    return TT_ERR_SHAPE;
  }
  if (p.mrcap > 64) {
    set_error("tt_filter_run: rank cap > 64 not supported");
    return TT_ERR_SHAPE;
  }
  // rounding scratch sized for both roundings (X -> P and H -> P)
  RoundShape shU;
  round_shape(batch, vU, p.vP, f64, shU);
  p.gcap = std::max(shU.gcap, p.n1max);
  if (p.gcap > 1024) {
    set_error("tt_filter_run: rank capacity or n[1] exceeds 1024 (%d)", p.gcap);
    return TT_ERR_SHAPE;
  }
  p.splits = shU.splits;
  for (int b = 0; b < batch; ++b) {
    plan_round_scratch(ar, vU[b], p.vP[b], f64, p.gcap, p.splits, p.vrs[b]);
    p.vrs[b].max_rank = specs[b].cap;  // ragged batches: each filter's own cap
  }
  round_shape(batch, p.vX, p.vP, f64, p.shX);
  round_shape(batch, p.vH, p.vP, f64, p.shH);
  // fused FFT prediction (interior cores exist for d >= 3)
  p.fused = (d >= 3) && kernels != nullptr && g_predict_mode != 2;
  if (d >= 3) {
    const size_t csz = f64 ? sizeof(double2) : sizeof(float2);
    const int nk = kernels ? n_kernels : 1;
    p.kL.assign(nk, 0);
    p.klog2.assign(nk, 0);
    p.khat.assign(nk, nullptr);
    p.ktw.assign(nk, nullptr);
    p.kpitch.assign(nk, 0);
    p.vKk.resize(nk);
    // FFT length per kernel: the smallest power of two >= n + h over the
    // grids that use it (a kernel belongs to one grid)
    for (int b = 0; b < batch; ++b) {
      const int ki = kernels ? specs[b].kernel_index : 0;
      int hmax = 0;
      if (kernels)
        for (int k = 0; k < d; ++k) hmax = std::max(hmax, (kernels[ki].n[k] - 1) / 2);
      int need = 0;
      for (int k = 0; k < d; ++k) need = std::max(need, specs[b].grid.n[k] + hmax);
      int L = 2, lg = 1;
      while (L < need) {
        L *= 2;
        ++lg;
      }
      p.kL[ki] = std::max(p.kL[ki], L);
      p.klog2[ki] = std::max(p.klog2[ki], lg);
      p.Lmax = std::max(p.Lmax, L);
      p.kcap = std::max(p.kcap, specs[b].kernel_cap);
      p.pcap = std::max(p.pcap, specs[b].cap);
    }
    if (p.kcap > 32) {
      set_error("tt_filter_run: kernel rank capacity %d > 32", p.kcap);
      return TT_ERR_SHAPE;
    }
    {
      int nmax = 1;
      for (int b = 0; b < batch; ++b)
        for (int k = 0; k < d; ++k) nmax = std::max(nmax, specs[b].grid.n[k]);
      int hmax = 0;
      if (kernels)
        for (int ki = 0; ki < n_kernels; ++ki)
          for (int k = 0; k < d; ++k) hmax = std::max(hmax, (kernels[ki].n[k] - 1) / 2);
      p.hmax = hmax;
      const size_t need = g_predict_mode == 1
                              ? (f64 ? fused_smem<double>(p.Lmax, p.kcap, nmax, p.pcap)
                                     : fused_smem<float>(p.Lmax, p.kcap, nmax, p.pcap))
                              : (f64 ? (use_mfma_pred<double>(hmax, nmax, p.pcap, p.kcap)
                                            ? mfma_pred_smem<double>(hmax, nmax, p.pcap, p.kcap,
                                                                     use_mfma_pred<double>(hmax, nmax, p.pcap, p.kcap) == 2)
                                            : direct_smem<double>(hmax, nmax, p.pcap, p.kcap))
                                     : (use_mfma_pred<float>(hmax, nmax, p.pcap, p.kcap)
                                            ? mfma_pred_smem<float>(hmax, nmax, p.pcap, p.kcap,
                                                                    use_mfma_pred<float>(hmax, nmax, p.pcap, p.kcap) == 2)
                                            : direct_smem<float>(hmax, nmax, p.pcap, p.kcap)));
      // a fused prediction that does not fit the LDS of a CU gives way to
      // the materialised convolution and the plain rounding (mode 2)
      if (need > 160 * 1024) p.fused = false;
    }
    for (int ki = 0; ki < nk; ++ki) {
      if (p.kL[ki] == 0) continue;
      const long long lhp = (p.kL[ki] / 2 + 1 + 7) / 8 * 8;
      p.kpitch[ki] = lhp * p.kcap * p.kcap;
      p.khat[ki] = ar.take<char>((size_t)d * p.kpitch[ki] * csz);
      p.ktw[ki] = ar.take<char>((size_t)(p.kL[ki] / 2) * csz);
      if (kernels) p.vKk[ki] = make_dev(kernels[ki]);
    }
    p.dKk = ar.take<DevTT>(nk);
    p.vfp.resize(batch);
    for (int b = 0; b < batch; ++b) {
      const int ki = kernels ? specs[b].kernel_index : 0;
      FusedPred& fp = p.vfp[b];
      memset(&fp, 0, sizeof(fp));
      fp.L = p.kL[ki];
      fp.log2L = p.klog2[ki];
      fp.LHP = (fp.L / 2 + 1 + 7) / 8 * 8;
      fp.h = 0;
      if (kernels)
        for (int k = 0; k < d; ++k) fp.h = std::max(fp.h, (kernels[ki].n[k] - 1) / 2);
      fp.khat = p.khat[ki];
      fp.kpitch = p.kpitch[ki];
      fp.tw = p.ktw[ki];
      fp.zt = 1;
    }
    p.dfp = ar.take<FusedPred>(batch);
  }
  p.shX.gcap = p.shH.gcap = p.gcap;
  p.shX.splits = p.shH.splits = p.splits;
  p.mstride = (long long)p.n0max * p.n1max;
  p.mbuf = p.any_range ? ar.take<double>((size_t)batch * p.mstride) : nullptr;
  {
    long long tmax = 1;
    for (int b = 0; b < batch; ++b)
      for (int k = 0; k < d; ++k)
        tmax = std::max(tmax, (long long)p.vL[b].cap[k + 1] * p.vP[b].cap[k] * p.vP[b].n[k]);
    p.tofs = p.vcap;
    p.vstride = p.vcap + tmax;
  }
  p.vbuf = ar.take<double>((size_t)batch * p.vstride);
  p.mspf = (long long)moments_scratch_per_filter(d, p.mrcap);
  p.mscr = ar.take<double>((size_t)batch * p.mspf);
  p.lmass = ar.take<double>((size_t)batch);
  p.dS = ar.take<DevTT>((size_t)2 * batch);
  return TT_OK;
}

template <typename T, typename Acc>
static tt_status run_steps(RunPlan& p, int B, const double* z, int zdim, int K, int k_begin, int k_count,
                           double* loglik, double* log_c, double* log_mpred, double* mean, double* cov,
                           int* ranks_out, int* ranks_pred_out, const int* replay_pred, const int* replay_filt,
                           const tt_filter_spec* specs, hipStream_t st, const tt_monitor* mon) {
  const int d = p.d;
  double* tails = mon ? mon->tail_dev : nullptr;
  double* mmin = mon ? mon->marg_min_dev : nullptr;
  // all filters of a batch share eps (checked by run_plan); the rank rule
  // takes each filter's own cap from its rounding scratch, bounded by maxcap
  const double eps = specs[0].eps;
  int maxcap = 1;
  for (int b = 0; b < B; ++b) maxcap = std::max(maxcap, specs[b].cap);
  if (k_begin == 0) {
    hipLaunchKernelGGL((prior_kernel<T>), dim3(B), dim3(256), 0, st, p.dP, p.dfc);
    TTG_LAUNCH_CHECK("prior_kernel");
    TT_TRY(launch_moments<T>(B, p.dP, p.dfc, p.lmass, 1, nullptr, 0, nullptr, 0, p.mscr, p.mspf, p.mrcap, st));
    hipLaunchKernelGGL(fill_kernel, dim3(cdiv(B, 256)), dim3(256), 0, st, log_mpred, (long long)B, (long long)K,
                       0.0);
    TTG_LAUNCH_CHECK("fill_kernel");
  }
  RoundBufs rx{p.dX, p.dP, p.drs}, rh{p.dH, p.dP, p.drs};
  FusedLaunch fl;
  if (p.fused && g_predict_mode == 1) {
    // kernel spectra (the FFT of every kernel fibre), once per kernel TT
    using C = typename Cpx<T>::t;
    for (size_t ki = 0; ki < p.khat.size(); ++ki) {
      if (!p.khat[ki]) continue;
      const int L = p.kL[ki];
      const size_t smem = ((size_t)L / 2 + (size_t)8 * L) * sizeof(C);
      if (smem > 48 * 1024)
        HIP_TRY(hipFuncSetAttribute((const void*)kernel_spectra_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)smem), "spectra smem");
      hipLaunchKernelGGL((kernel_spectra_kernel<T>), dim3(cdiv((long long)p.kcap * p.kcap, 4), d), dim3(256), smem, st,
                         p.dKk + ki, L, p.klog2[ki], (int)((L / 2 + 1 + 7) / 8 * 8), p.khat[ki], p.kpitch[ki]);
      TTG_LAUNCH_CHECK("kernel_spectra_kernel");
      hipLaunchKernelGGL((twiddle_kernel<T>), dim3(1), dim3(256), 0, st, p.ktw[ki], L);
      TTG_LAUNCH_CHECK("twiddle_kernel");
    }
  }
  if (p.fused) {
    fl.mode = g_predict_mode == 1 ? 1 : 0;
    fl.hmax = p.hmax;
    fl.Kn = p.dK;
    fl.Pn = p.dP;
    fl.FP = p.dfp;
    fl.Lmax = p.Lmax;
    fl.kcap = p.kcap;
    fl.pcap = p.pcap;
    fl.nmax = p.shX.n[0];
    for (int kk = 0; kk < d; ++kk) fl.nmax = std::max(fl.nmax, p.shX.n[kk]);
  }
  const long long rstride = (long long)K * (d + 1);  // per filter, in the rank arrays
  for (int k = k_begin; k < k_begin + k_count; ++k) {
    if (k > 0) {
      TT_TRY(launch_conv<T>(B, d, p.r0capX, p.csmem, p.dK, p.dP, p.dX, st, p.fused ? 0 : 1));
      TT_TRY((round_launch<T, Acc>(p.shX, rx, eps, maxcap, st, p.fused ? &fl : nullptr,
                                   replay_pred ? replay_pred + (long long)k * (d + 1) : nullptr, rstride)));
      if (tails) {
        hipLaunchKernelGGL(tail_record_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, p.drs, B, tails + (long long)k * 2,
                           (long long)K * 2);
        TTG_LAUNCH_CHECK("tail_record_kernel");
      }
      TT_TRY(launch_moments<T>(B, p.dP, p.dfc, log_mpred + k, K, nullptr, 0, nullptr, 0, p.mscr, p.mspf, p.mrcap, st));
    } else if (tails) {  // no prediction at step 0
      hipLaunchKernelGGL(fill_kernel, dim3(cdiv(B, 256)), dim3(256), 0, st, tails, (long long)B, (long long)K * 2, 0.0);
      TTG_LAUNCH_CHECK("fill_kernel");
    }
    if (ranks_pred_out) {  // ranks of the predictive (the prior's at k = 0)
      hipLaunchKernelGGL(record_ranks_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, p.dP, B,
                         ranks_pred_out + (long long)k * (d + 1), rstride);
      TTG_LAUNCH_CHECK("record_ranks_kernel");
    }
    TT_TRY(lik_launch(B, p.dL, p.drs, p.dfc, z + (long long)k * zdim, (long long)K * zdim, p.mbuf, p.mstride,
                      p.any_range, p.n0max, p.n1max, p.gcap, p.splits, st, sizeof(T) == 4));
    TT_TRY(launch_dot<T>(B, p.dL, p.dP, p.dfc, log_c + k, (long long)K, p.vbuf, p.vstride, p.tofs, st));
    TT_TRY(launch_hadamard<T>(B, d, p.r0capH, p.dL, p.dP, p.dH, st));
    TT_TRY((round_launch<T, Acc>(p.shH, rh, eps, maxcap, st, nullptr,
                                 replay_filt ? replay_filt + (long long)k * (d + 1) : nullptr, rstride)));
    if (tails) {
      hipLaunchKernelGGL(tail_record_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, p.drs, B,
                         tails + (long long)k * 2 + 1, (long long)K * 2);
      TTG_LAUNCH_CHECK("tail_record_kernel");
    }
    TT_TRY(launch_moments<T>(B, p.dP, p.dfc, p.lmass, 1, mean ? mean + (long long)k * d : nullptr, (long long)K * d,
                             cov ? cov + (long long)k * d * d : nullptr, (long long)K * d * d, p.mscr, p.mspf,
                             p.mrcap, st));
    if (mmin) {  // after the moments: the scratch is free again
      hipLaunchKernelGGL((marginal_min_kernel<T>), dim3(B), dim3(256), 0, st, p.dP, mmin + k, (long long)K, p.mscr,
                         p.mspf, p.mrcap);
      TTG_LAUNCH_CHECK("marginal_min_kernel");
    }
    if (ranks_out) {
      hipLaunchKernelGGL(record_ranks_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, p.dP, B,
                         ranks_out + (long long)k * (d + 1), rstride);
      TTG_LAUNCH_CHECK("record_ranks_kernel");
    }
  }
  hipLaunchKernelGGL(loglik_kernel, dim3(cdiv(B, 64)), dim3(64), 0, st, log_c, K, k_begin + k_count, B, loglik);
  TTG_LAUNCH_CHECK("loglik_kernel");
  return TT_OK;
}

}  // namespace ttg

extern "C" {

size_t tt_filter_run_workspace(int32_t batch, const tt_filter_spec* specs, const tt_train* kernels,
                               int32_t n_kernels, int32_t precision) {
  if (!kernels || n_kernels < 1) return 0;
  Arena ar(nullptr, 0);
  RunPlan p;
  if (run_plan(batch, specs, kernels, n_kernels, precision, nullptr, ar, p) != TT_OK) return 0;
  return ar.used + 256;
}

}  // extern "C"

namespace ttg {

// Validation, planning and the descriptor upload of tt_filter_run; then the
// steps, launched on st, or recorded into *graph when graph is non-null.
static tt_status filter_run_impl(int32_t batch, const tt_filter_spec* specs, const tt_train* kernels,
                                 int32_t n_kernels, const double* z_dev, int32_t zdim, int32_t K, int32_t k_begin,
                                 int32_t k_count, int32_t precision, double* loglik_dev, double* log_c_dev,
                                 double* log_mpred_dev, double* mean_dev, double* cov_dev, int32_t* ranks_dev,
                                 int32_t* status_dev, int32_t* ranks_pred_dev, const int32_t* replay_pred_dev,
                                 const int32_t* replay_filt_dev, void* ws, size_t ws_bytes, hipStream_t st,
                                 hipGraph_t* graph, const tt_monitor* mon = nullptr) {
  if (!kernels || n_kernels < 1 || !z_dev || K < 1 || zdim < 1 || !loglik_dev || !log_c_dev || !log_mpred_dev ||
      !status_dev || !ws) {
    set_error("tt_filter_run: null pointer or bad size");
    return TT_ERR_ARG;
  }
  if (k_begin < 0 || k_count < 1 || k_begin + k_count > K) {
    set_error("tt_filter_run: need 0 <= k_begin, k_count >= 1, k_begin + k_count <= K");
    return TT_ERR_ARG;
  }
  if (cov_dev && !mean_dev) {
    set_error("tt_filter_run: cov needs mean");
    return TT_ERR_ARG;
  }
  for (int b = 0; b < batch; ++b) {
    const int need = specs[b].meas.kind == 0 ? specs[b].grid.d : specs[b].grid.d - 1;
    if (need > zdim) {
      set_error("tt_filter_run: zdim %d smaller than the measurement size %d", zdim, need);
      return TT_ERR_SHAPE;
    }
    if (specs[b].eps != specs[0].eps) {
      set_error("tt_filter_run: all filters of a batch must share eps");
      return TT_ERR_ARG;
    }
  }
  Arena ar(ws, ws_bytes);
  RunPlan p;
  TT_TRY(run_plan(batch, specs, kernels, n_kernels, precision, status_dev, ar, p));
  if (!ar.fits()) {
    set_error("tt_filter_run: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  TT_TRY(upload(p.dP, p.vP, st));
  TT_TRY(upload(p.dX, p.vX, st));
  TT_TRY(upload(p.dL, p.vL, st));
  TT_TRY(upload(p.dH, p.vH, st));
  TT_TRY(upload(p.dK, p.vK, st));
  TT_TRY(upload(p.drs, p.vrs, st));
  TT_TRY(upload(p.dfc, p.vfc, st));
  if (p.fused) {
    TT_TRY(upload(p.dfp, p.vfp, st));
    TT_TRY(upload(p.dKk, p.vKk, st));
  }
  hipStream_t run_st = st;
  if (graph) {
    // capture on a stream of our own (the caller's may be the null stream);
    // the descriptors are on the device once the uploads on st are done (the
    // replays may run on any stream), so nothing in the recorded steps reads
    // host memory
    HIP_TRY(hipStreamSynchronize(st), "descriptor uploads before capture");
    HIP_TRY(hipStreamCreateWithFlags(&run_st, hipStreamNonBlocking), "capture stream");
    const hipError_t e = hipStreamBeginCapture(run_st, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) {
      hipStreamDestroy(run_st);
      return check_hip(e, "hipStreamBeginCapture");
    }
  }
  tt_status rs = precision == TT_F64
                     ? run_steps<double, AccDD>(p, batch, z_dev, zdim, K, k_begin, k_count, loglik_dev, log_c_dev,
                                                log_mpred_dev, mean_dev, cov_dev, ranks_dev, ranks_pred_dev,
                                                replay_pred_dev, replay_filt_dev, specs, run_st, mon)
                     : run_steps<float, AccD>(p, batch, z_dev, zdim, K, k_begin, k_count, loglik_dev, log_c_dev,
                                              log_mpred_dev, mean_dev, cov_dev, ranks_dev, ranks_pred_dev,
                                              replay_pred_dev, replay_filt_dev, specs, run_st, mon);
  if (graph) {
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(run_st, &g);
    hipStreamDestroy(run_st);
    if (rs != TT_OK) {
      if (g) hipGraphDestroy(g);
      return rs;
    }
    if (e != hipSuccess) {
      if (g) hipGraphDestroy(g);
      return check_hip(e, "hipStreamEndCapture");
    }
    *graph = g;
  }
  return rs;
}

}  // namespace ttg

struct tt_graph_s {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

extern "C" {

tt_status tt_filter_run(int32_t batch, const tt_filter_spec* specs, const tt_train* kernels, int32_t n_kernels,
                        const double* z_dev, int32_t zdim, int32_t K, int32_t k_begin, int32_t k_count,
                        int32_t precision, double* loglik_dev,
                        double* log_c_dev, double* log_mpred_dev, double* mean_dev, double* cov_dev,
                        int32_t* ranks_dev, int32_t* status_dev, int32_t* ranks_pred_dev,
                        const int32_t* replay_pred_dev, const int32_t* replay_filt_dev, void* ws,
                        size_t ws_bytes, void* stream) {
  return filter_run_impl(batch, specs, kernels, n_kernels, z_dev, zdim, K, k_begin, k_count, precision, loglik_dev,
                         log_c_dev, log_mpred_dev, mean_dev, cov_dev, ranks_dev, status_dev, ranks_pred_dev,
                         replay_pred_dev, replay_filt_dev, ws, ws_bytes, reinterpret_cast<hipStream_t>(stream),
                         nullptr);
}

tt_status tt_filter_run_monitored(int32_t batch, const tt_filter_spec* specs, const tt_train* kernels,
                                  int32_t n_kernels, const double* z_dev, int32_t zdim, int32_t K, int32_t k_begin,
                                  int32_t k_count, int32_t precision, double* loglik_dev, double* log_c_dev,
                                  double* log_mpred_dev, double* mean_dev, double* cov_dev, int32_t* ranks_dev,
                                  int32_t* status_dev, int32_t* ranks_pred_dev, const int32_t* replay_pred_dev,
                                  const int32_t* replay_filt_dev, const tt_monitor* monitor, void* ws,
                                  size_t ws_bytes, void* stream) {
  return filter_run_impl(batch, specs, kernels, n_kernels, z_dev, zdim, K, k_begin, k_count, precision, loglik_dev,
                         log_c_dev, log_mpred_dev, mean_dev, cov_dev, ranks_dev, status_dev, ranks_pred_dev,
                         replay_pred_dev, replay_filt_dev, ws, ws_bytes, reinterpret_cast<hipStream_t>(stream),
                         nullptr, monitor);
}

size_t tt_marginal_min_workspace(int32_t batch, const tt_train* tts) {
  if (batch < 1 || !tts) return 0;
  int rcap = 1, dmax = 1;
  for (int b = 0; b < batch; ++b) {
    dmax = std::max(dmax, tts[b].d);
    for (int j = 0; j <= tts[b].d && j <= TT_MAXD; ++j) rcap = std::max(rcap, tts[b].cap[j]);
  }
  const size_t spf = (size_t)dmax * rcap * rcap + 2 * (size_t)(dmax + 1) * rcap;
  return (size_t)batch * (spf * sizeof(double) + sizeof(DevTT)) + 4096;
}

tt_status tt_marginal_min(int32_t batch, const tt_train* tts, double* out_dev, void* ws, size_t ws_bytes,
                          void* stream) {
  if (batch < 1 || !tts || !out_dev || !ws) {
    set_error("tt_marginal_min: null pointer or batch < 1");
    return TT_ERR_ARG;
  }
  const int dtype = tts[0].dtype;
  int rcap = 1, dmax = 1;
  std::vector<DevTT> v(batch);
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_train(&tts[b], "tt_marginal_min", dtype));
    dmax = std::max(dmax, tts[b].d);
    for (int j = 0; j <= tts[b].d; ++j) rcap = std::max(rcap, tts[b].cap[j]);
    v[b] = make_dev(tts[b]);
  }
  const long long spf = (long long)dmax * rcap * rcap + 2LL * (dmax + 1) * rcap;
  Arena ar(ws, ws_bytes);
  DevTT* dt = ar.take<DevTT>(batch);
  double* scr = ar.take<double>((size_t)batch * spf);
  if (!ar.fits()) {
    set_error("tt_marginal_min: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(dt, v, st));
  if (dtype == TT_F64)
    hipLaunchKernelGGL((marginal_min_kernel<double>), dim3(batch), dim3(256), 0, st, dt, out_dev, 1LL, scr, spf, rcap);
  else
    hipLaunchKernelGGL((marginal_min_kernel<float>), dim3(batch), dim3(256), 0, st, dt, out_dev, 1LL, scr, spf, rcap);
  TTG_LAUNCH_CHECK("marginal_min_kernel");
  return TT_OK;
}

tt_status tt_filter_graph_create(int32_t batch, const tt_filter_spec* specs, const tt_train* kernels,
                                 int32_t n_kernels, const double* z_dev, int32_t zdim, int32_t K, int32_t k_begin,
                                 int32_t k_count, int32_t precision, double* loglik_dev, double* log_c_dev,
                                 double* log_mpred_dev, double* mean_dev, double* cov_dev, int32_t* ranks_dev,
                                 int32_t* status_dev, int32_t* ranks_pred_dev, const int32_t* replay_pred_dev,
                                 const int32_t* replay_filt_dev, void* ws, size_t ws_bytes, void* stream,
                                 tt_graph** out) {
  if (!out) {
    set_error("tt_filter_graph_create: null output handle");
    return TT_ERR_ARG;
  }
  *out = nullptr;
  if (k_begin < 1) {
    set_error("tt_filter_graph_create: k_begin must be >= 1 (step 0 starts from the prior: run it eagerly)");
    return TT_ERR_ARG;
  }
  if (g_prof_mask) {
    set_error("tt_filter_graph_create: profiling is active");
    return TT_ERR_ARG;
  }
  hipGraph_t g = nullptr;
  TT_TRY(filter_run_impl(batch, specs, kernels, n_kernels, z_dev, zdim, K, k_begin, k_count, precision, loglik_dev,
                         log_c_dev, log_mpred_dev, mean_dev, cov_dev, ranks_dev, status_dev, ranks_pred_dev,
                         replay_pred_dev, replay_filt_dev, ws, ws_bytes, reinterpret_cast<hipStream_t>(stream),
                         &g));
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return check_hip(e, "hipGraphInstantiate");
  }
  tt_graph* h = new (std::nothrow) tt_graph_s{g, ex};
  if (!h) {
    hipGraphExecDestroy(ex);
    hipGraphDestroy(g);
    set_error("tt_filter_graph_create: out of host memory");
    return TT_ERR_ARG;
  }
  *out = h;
  return TT_OK;
}

tt_status tt_filter_graph_launch(tt_graph* g, void* stream) {
  if (!g) {
    set_error("tt_filter_graph_launch: null handle");
    return TT_ERR_ARG;
  }
  HIP_TRY(hipGraphLaunch(g->exec, reinterpret_cast<hipStream_t>(stream)), "hipGraphLaunch");
  return TT_OK;
}

void tt_filter_graph_destroy(tt_graph* g) {
  if (!g) return;
  hipGraphExecDestroy(g->exec);
  hipGraphDestroy(g->graph);
  delete g;
}


tt_status tt_filter_state(int32_t batch, const tt_filter_spec* specs, const tt_train* kernels, int32_t n_kernels,
                          int32_t precision, int32_t direction, const tt_train* trains, void* ws, size_t ws_bytes,
                          void* stream) {
  using namespace ttg;
  if (!kernels || n_kernels < 1 || !trains || !ws || (direction != TT_STATE_SAVE && direction != TT_STATE_LOAD)) {
    set_error("tt_filter_state: null pointer or bad direction");
    return TT_ERR_ARG;
  }
  Arena ar(ws, ws_bytes);
  RunPlan p;
  TT_TRY(run_plan(batch, specs, kernels, n_kernels, precision, nullptr, ar, p));
  if (!ar.fits()) {
    set_error("tt_filter_state: workspace too small (%zu < %zu)", ws_bytes, ar.used);
    return TT_ERR_WORKSPACE;
  }
  std::vector<DevTT> tab(2 * (size_t)batch);
  for (int b = 0; b < batch; ++b) {
    TT_TRY(check_train(&trains[b], "tt_filter_state train", precision));
    const tt_train& t = trains[b];
    if (t.d != p.d) {
      set_error("tt_filter_state: train %d has d=%d, the run d=%d", b, t.d, p.d);
      return TT_ERR_SHAPE;
    }
    for (int k = 0; k < t.d; ++k)
      if (t.n[k] != specs[b].grid.n[k]) {
        set_error("tt_filter_state: train %d mode %d is %d, the grid's %d", b, k, t.n[k], specs[b].grid.n[k]);
        return TT_ERR_SHAPE;
      }
    const DevTT w = p.vP[b], c = make_dev(t);
    tab[b] = direction == TT_STATE_SAVE ? w : c;
    tab[batch + b] = direction == TT_STATE_SAVE ? c : w;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  TT_TRY(upload(p.dS, tab, st));
  long long most = 1;
  for (int b = 0; b < batch; ++b) most = std::max(most, (long long)elems_of(p.d, p.vP[b].n, p.vP[b].cap));
  const dim3 grid(std::max(1, std::min(64, cdiv(most, 256 * 8))), batch);
  if (precision == TT_F64)
    hipLaunchKernelGGL((copy_tt_kernel<double>), grid, dim3(256), 0, st, p.dS, p.dS + batch,
                       direction == TT_STATE_LOAD ? 1 : 0);
  else
    hipLaunchKernelGGL((copy_tt_kernel<float>), grid, dim3(256), 0, st, p.dS, p.dS + batch,
                       direction == TT_STATE_LOAD ? 1 : 0);
  TTG_LAUNCH_CHECK("copy_tt_kernel");
  return TT_OK;
}

}  // extern "C"

namespace ttg {

static tt_status device_arch(char* out, size_t len) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
  size_t i = 0;
  for (; i + 1 < len && prop.gcnArchName[i] && prop.gcnArchName[i] != ':'; ++i) out[i] = prop.gcnArchName[i];
  out[i] = 0;
  return TT_OK;
}

// value of "key": <int> or "key": "<word>" inside one JSON object's text
static bool json_int(const char* obj, const char* key, int* v) {
  char pat[64];
  snprintf(pat, sizeof(pat), "\"%s\"", key);
  const char* p = strstr(obj, pat);
  if (!p) return false;
  p = strchr(p + strlen(pat), ':');
  return p && sscanf(p + 1, " %d", v) == 1;
}

static bool json_word(const char* obj, const char* key, char* out, size_t len) {
  char pat[64];
  snprintf(pat, sizeof(pat), "\"%s\"", key);
  const char* p = strstr(obj, pat);
  if (!p) return false;
  p = strchr(p + strlen(pat), ':');
  if (!p) return false;
  p = strchr(p, '"');
  if (!p) return false;
  const char* e = strchr(p + 1, '"');
  if (!e || (size_t)(e - p - 1) >= len) return false;
  memcpy(out, p + 1, e - p - 1);
  out[e - p - 1] = 0;
  return true;
}

}  // namespace ttg

extern "C" {

tt_status tt_autotune_save(const char* path) {
  using namespace ttg;
  if (!path) {
    set_error("tt_autotune_save: null path");
    return TT_ERR_ARG;
  }
  char arch[64];
  TT_TRY(device_arch(arch, sizeof(arch)));
  FILE* f = fopen(path, "w");
  if (!f) {
    set_error("tt_autotune_save: cannot write %s", path);
    return TT_ERR_ARG;
  }
  fprintf(f, "[\n");
  for (size_t i = 0; i < g_tuned_bb.size(); ++i) {
    const TuneKey& k = g_tuned_bb[i].first;
    fprintf(f,
            "  {\"arch\": \"%s\", \"knob\": \"prediction_fibres_per_workgroup\", \"dtype\": \"%s\", "
            "\"batch\": %d, \"halfwidth\": %d, \"n\": %d, \"rank_cap\": %d, \"kernel_rank_cap\": %d, "
            "\"value\": %d}%s\n",
            arch, k.f64 ? "f64" : "f32", k.B, k.hmax, k.nmax, k.pcap, k.kcap, g_tuned_bb[i].second,
            i + 1 < g_tuned_bb.size() ? "," : "");
  }
  fprintf(f, "]\n");
  const bool ok = fclose(f) == 0;
  if (!ok) {
    set_error("tt_autotune_save: writing %s failed", path);
    return TT_ERR_ARG;
  }
  return TT_OK;
}

tt_status tt_autotune_load(const char* path, int32_t* n_loaded) {
  using namespace ttg;
  if (!path) {
    set_error("tt_autotune_load: null path");
    return TT_ERR_ARG;
  }
  char arch[64];
  TT_TRY(device_arch(arch, sizeof(arch)));
  FILE* f = fopen(path, "r");
  if (!f) {
    set_error("tt_autotune_load: cannot read %s", path);
    return TT_ERR_ARG;
  }
  std::vector<char> text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), f)) > 0) text.insert(text.end(), buf, buf + got);
  fclose(f);
  text.push_back(0);
  std::vector<std::pair<TuneKey, int>> found;
  const char* p = text.data();
  while ((p = strchr(p, '{')) != nullptr) {
    const char* e = strchr(p, '}');
    if (!e) {
      set_error("tt_autotune_load: unterminated entry in %s", path);
      return TT_ERR_ARG;
    }
    std::string obj(p, e - p + 1);
    char a[64], knob[64], dt[16];
    TuneKey k{};
    int v = 0;
    if (!json_word(obj.c_str(), "arch", a, sizeof(a)) || !json_word(obj.c_str(), "knob", knob, sizeof(knob)) ||
        !json_word(obj.c_str(), "dtype", dt, sizeof(dt)) || !json_int(obj.c_str(), "batch", &k.B) ||
        !json_int(obj.c_str(), "halfwidth", &k.hmax) || !json_int(obj.c_str(), "n", &k.nmax) ||
        !json_int(obj.c_str(), "rank_cap", &k.pcap) || !json_int(obj.c_str(), "kernel_rank_cap", &k.kcap) ||
        !json_int(obj.c_str(), "value", &v) || strcmp(knob, "prediction_fibres_per_workgroup") != 0 ||
        (strcmp(dt, "f32") != 0 && strcmp(dt, "f64") != 0) || (v != 2 && v != 4 && v != 8 && v != 16)) {
      set_error("tt_autotune_load: entry does not parse: %.200s", obj.c_str());
      return TT_ERR_ARG;
    }
    k.f64 = strcmp(dt, "f64") == 0;
    if (strcmp(a, arch) == 0) found.push_back({k, v});
    p = e + 1;
  }
  for (const auto& fe : found) {
    bool rep = false;
    for (auto& e : g_tuned_bb)
      if (e.first == fe.first) {
        e.second = fe.second;
        rep = true;
      }
    if (!rep) g_tuned_bb.push_back(fe);
  }
  if (n_loaded) *n_loaded = (int32_t)found.size();
  return TT_OK;
}

const char* tt_status_string(int32_t code) {
  switch (code) {
    case TT_OK:
      return "TT_OK: success";
    case TT_ERR_ARG:
      return "TT_ERR_ARG: null pointer, non-positive size or bad enumeration value";
    case TT_ERR_SHAPE:
      return "TT_ERR_SHAPE: inconsistent dimension, modes, ranks or capacities";
    case TT_ERR_WORKSPACE:
      return "TT_ERR_WORKSPACE: workspace smaller than its query returns";
    case TT_ERR_HIP:
      return "TT_ERR_HIP: a HIP call failed (tt_last_error holds the message)";
    default:
      return "unknown tt_status code";
  }
}

const char* tt_device_status_string(int32_t bits) {
  switch (bits) {
    case 0:
      return "ok";
    case TT_STATUS_NONPOSITIVE:
      return "TT_STATUS_NONPOSITIVE: a mass or normaliser c_k was not positive";
    case TT_STATUS_NONFINITE:
      return "TT_STATUS_NONFINITE: a NaN or infinity was met";
    case TT_STATUS_CAPACITY:
      return "TT_STATUS_CAPACITY: a rank needed more room than its capacity";
    case TT_STATUS_NONPOSITIVE | TT_STATUS_NONFINITE:
      return "TT_STATUS_NONPOSITIVE | TT_STATUS_NONFINITE";
    case TT_STATUS_NONPOSITIVE | TT_STATUS_CAPACITY:
      return "TT_STATUS_NONPOSITIVE | TT_STATUS_CAPACITY";
    case TT_STATUS_NONFINITE | TT_STATUS_CAPACITY:
      return "TT_STATUS_NONFINITE | TT_STATUS_CAPACITY";
    case TT_STATUS_NONPOSITIVE | TT_STATUS_NONFINITE | TT_STATUS_CAPACITY:
      return "TT_STATUS_NONPOSITIVE | TT_STATUS_NONFINITE | TT_STATUS_CAPACITY";
    default:
      return "unknown device status bits";
  }
}

}  // extern "C"

extern "C" {

void tt_profile_begin(int32_t class_mask) {
  g_prof.clear();
  g_pool_next = 0;
  g_prof_mask = class_mask;
  if (!g_work && hipMalloc((void**)&g_work, sizeof(double) * 2 * PC_N) != hipSuccess) g_work = nullptr;
  if (g_work && hipMemset(g_work, 0, sizeof(double) * 2 * PC_N) != hipSuccess) g_work = nullptr;
}

int32_t tt_profile_end(double* ms, int32_t* launches, double* flops, double* bytes, int32_t nclass) {
  for (int c = 0; c < nclass; ++c) {
    if (ms) ms[c] = 0.0;
    if (launches) launches[c] = 0;
    if (flops) flops[c] = 0.0;
    if (bytes) bytes[c] = 0.0;
  }
  for (const ProfRec& r : g_prof) {
    if (hipEventSynchronize(r.b) != hipSuccess) {
      set_error("tt_profile_end: event synchronisation failed");
      g_prof_mask = 0;
      return -1;
    }
    float t = 0.f;
    if (hipEventElapsedTime(&t, r.a, r.b) != hipSuccess) continue;
    if (r.cls < nclass) {
      if (ms) ms[r.cls] += t;
      if (launches) launches[r.cls] += 1;
    }
  }
  g_prof.clear();
  g_prof_mask = 0;
  if (g_work && (flops || bytes)) {
    double w[2 * PC_N];
    if (hipMemcpy(w, g_work, sizeof(w), hipMemcpyDeviceToHost) != hipSuccess) {
      set_error("tt_profile_end: reading the work counters failed");
      return -1;
    }
    for (int c = 0; c < nclass && c < PC_N; ++c) {
      if (flops) flops[c] = w[2 * c];
      if (bytes) bytes[c] = w[2 * c + 1];
    }
  }
  return PC_N;
}

}  // extern "C"

extern "C" {

tt_status tt_set_predict_mode(int32_t mode) {
  if (mode < 0 || mode > 3) {
    set_error("tt_set_predict_mode: mode must be 0, 1, 2 or 3");
    return TT_ERR_ARG;
  }
  g_predict_mode = mode;
  return TT_OK;
}

int32_t tt_get_predict_mode(void) { return g_predict_mode; }

tt_status tt_autotune_prediction(int32_t batch, const tt_filter_spec* specs, const tt_train* kernels,
                                 int32_t n_kernels, const double* z_dev, int32_t zdim, int32_t K,
                                 int32_t precision, double* loglik_dev, double* log_c_dev, double* log_mpred_dev,
                                 int32_t* status_dev, void* ws, size_t ws_bytes, void* stream,
                                 int32_t warmup_steps, int32_t rounds, int32_t* best_bb, float* ms_per_candidate) {
  static const int cand[TT_TUNE_CANDIDATES] = {2, 4, 8, 16};
  if (!best_bb || !ms_per_candidate || warmup_steps < 0 || rounds < 1 ||
      K < 1 + warmup_steps + TT_TUNE_CANDIDATES * rounds) {
    set_error("tt_autotune_prediction: need outputs, rounds >= 1 and K >= 1 + warmup_steps + %d * rounds",
              TT_TUNE_CANDIDATES);
    return TT_ERR_ARG;
  }
  if (g_prof_mask) {
    set_error("tt_autotune_prediction: profiling is active");
    return TT_ERR_ARG;
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  auto run = [&](int kb, int kc) {
    return filter_run_impl(batch, specs, kernels, n_kernels, z_dev, zdim, K, kb, kc, precision, loglik_dev,
                           log_c_dev, log_mpred_dev, nullptr, nullptr, nullptr, status_dev, nullptr, nullptr,
                           nullptr, ws, ws_bytes, st, nullptr);
  };
  // step 0 and the warm-up steps bring the ranks to their working size
  TT_TRY(run(0, 1 + warmup_steps));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0), "tune event");
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    set_error("tt_autotune_prediction: event creation failed");
    return TT_ERR_HIP;
  }
  for (int c = 0; c < TT_TUNE_CANDIDATES; ++c) ms_per_candidate[c] = 3.4e38f;
  g_have_key = false;
  tt_status rs = TT_OK;
  int k = 1 + warmup_steps;
  // one step per candidate per round, candidates in turn, so that a slow
  // drift of the ranks affects all of them alike; each keeps its fastest step
  for (int r = 0; r < rounds && rs == TT_OK; ++r)
    for (int c = 0; c < TT_TUNE_CANDIDATES && rs == TT_OK; ++c, ++k) {
      g_force_bb = cand[c];
      hipEventRecord(e0, st);
      rs = run(k, 1);
      hipEventRecord(e1, st);
      if (rs != TT_OK) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        set_error("tt_autotune_prediction: event synchronisation failed");
        rs = TT_ERR_HIP;
        break;
      }
      float ms = 0.f;
      hipEventElapsedTime(&ms, e0, e1);
      ms_per_candidate[c] = std::min(ms_per_candidate[c], ms);
    }
  g_force_bb = 0;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rs != TT_OK) return rs;
  int best = 0;
  for (int c = 1; c < TT_TUNE_CANDIDATES; ++c)
    if (ms_per_candidate[c] < ms_per_candidate[best]) best = c;
  *best_bb = g_have_key ? cand[best] : 0;  // 0: the matrix-core prediction was not used by this batch
  if (g_have_key) {
    bool found = false;
    for (auto& e : g_tuned_bb)
      if (e.first == g_last_key) {
        e.second = cand[best];
        found = true;
      }
    if (!found) g_tuned_bb.push_back({g_last_key, cand[best]});
  }
  return TT_OK;
}

}  // extern "C"

#include "cross.h"
#include "grad_run.h"
#include "linear_run.h"
#include "moments_adj.h"
#include "update_adj.h"
