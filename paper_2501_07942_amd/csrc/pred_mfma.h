// Direct fused prediction on the matrix cores (FP32 and FP64).
//
// The product core X_k(a rp0 + b, i, a' rp1 + b') is the linear convolution
// of the kernel fibres with the density fibres along grid axis k (the
// translation-invariant transition kernel of Sec. 2.1, applied core by core
// as in Sec. 3.1).  The rounding's right-to-left sweep needs only
// Z_k = X_k x_3 L_{k+1}; for every output row block (a, b) this is one dense
// contraction over t = (m, b'):
//
//   Z_ab(i, j) = sum_t A_b(i, t) V_a(t, j)
//   A_b(i, (m, b')) = P_k(b, i + h - m, b')         (a Hankel gather of P_k)
//   V_a((m, b'), j) = sum_{a'} K_k(a, m, a') L(a' rp1 + b', j)
//
// with P = 0 off the grid.  A workgroup owns one row block a, a group of BB
// fibres b and all columns j (in passes of JC = 32 for FP32, 16 for FP64);
// V_a for the pass and a double-buffered zero-padded fibre of P sit in LDS,
// and the four wavefronts issue 16 x 16 x 4 MFMAs (v_mfma_f32_16x16x4f32 or
// v_mfma_f64_16x16x4f64) over 16 x 16 output tiles, two i-tiles x one or
// two j-tiles per wavefront.
//
// The bond b' is padded with zeros to qp = 4 S (S in {1, 2, 4, 8}).  Within
// one tap m the four k-lanes of an MFMA step s take b' = lk S + s, so a lane
// reads its S operands of A and of B for the whole tap as one contiguous
// vector; the S-element units of a V row are XOR-swizzled by column against
// LDS bank conflicts.  Every output element sums its terms in the same order
// whatever the batch, so a filter's result does not depend on the filters it
// is batched with.
//
// Lane layout of both MFMAs: A(i, k) in lane i + 16 k, B(k, j) in lane
// j + 16 k; D(i, j) in lane j + 16 (i / 4), register i % 4 for FP32 and in
// lane j + 16 (i % 4), register i / 4 for FP64.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4p __attribute__((ext_vector_type(4)));

#define MP_JT 16  // columns of one MFMA tile
#define MP_PF 6   // 16-byte prefetch registers per thread (fibres of up to 24 KB)
#define MP_PF_BIG 5   // the same for the single-buffer variant, 512 threads (fibres of up to 40 KB)
#define MP_NT_BIG 512 // threads of the single-buffer variant's workgroup

template <typename E>
struct MpT;
template <>
struct MpT<float> {
  using acc = mf4;
  static constexpr int JC = 32;  // columns per pass (two tiles)
  __device__ static inline acc mfma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int drow(int lk, int v) { return 4 * lk + v; }
};
template <>
struct MpT<double> {
  using acc = md4p;
  static constexpr int JC = 16;  // one tile per pass (FP64 V fills the LDS)
  __device__ static inline acc mfma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int drow(int lk, int v) { return lk + 4 * v; }
};

__host__ __device__ inline int mp_s(int rp1) { return rp1 <= 4 ? 1 : (rp1 <= 8 ? 2 : (rp1 <= 16 ? 4 : 8)); }
__host__ __device__ inline int mp_nit2(int n) { return ((n + 15) / 16 + 1) / 2 * 2; }  // even tile count
__host__ __device__ inline int mp_plen(int n, int h) { return mp_nit2(n) * 16 + 2 * h; }

// S consecutive elements at an address aligned to S elements (8- or
// 16-byte vector loads where possible)
template <typename E, int S>
struct MpVec {
  E v[S];
  __device__ inline void load(const E* p) {
    constexpr int U = 16 / (int)sizeof(E);  // elements per 16 bytes
    if constexpr (S == 1) {
      v[0] = p[0];
    } else if constexpr (sizeof(E) == 4 && S == 2) {
      const float2 t = *reinterpret_cast<const float2*>(p);
      v[0] = t.x;
      v[1] = t.y;
    } else if constexpr (sizeof(E) == 4) {
#pragma unroll
      for (int c = 0; c < S; c += 4) {
        const float4 t = *reinterpret_cast<const float4*>(p + c);
        v[c] = t.x;
        v[c + 1] = t.y;
        v[c + 2] = t.z;
        v[c + 3] = t.w;
      }
    } else {
#pragma unroll
      for (int c = 0; c < S; c += 2) {
        const double2 t = *reinterpret_cast<const double2*>(p + c);
        v[c] = t.x;
        v[c + 1] = t.y;
      }
    }
  }
};

// Position of bond b' of column jl in a V row block: the four S-element
// units of a column are XOR-swizzled by the column index so that the 16
// columns an MFMA operand read touches spread over distinct LDS banks.
template <int S>
__device__ inline int mp_vswz(int jl, int q) {
  constexpr int QP = 4 * S;
  constexpr int per = 16 / S;  // columns whose rows would share banks
  const int u = (q / S) ^ ((jl / per) & 3);
  return jl * QP + u * S + (q % S);
}

// Operands of one tap for one pair of 16-row tiles and NJ 16-column tiles.
template <typename E, int S, int NJ>
struct MpTap {
  MpVec<E, S> a0, a1, b0, b1;
  __device__ inline void load(const E* pa, const E* vb, int m, int pp, int vstride) {
    const E* p = pa - m * pp;
    const E* v = vb + m * 16 * (4 * S);
    a0.load(p);
    a1.load(p + 16 * pp);  // second i-tile
    b0.load(v);
    if constexpr (NJ == 2) b1.load(v + vstride);
  }
  __device__ inline void mma(typename MpT<E>::acc* acc) const {
#pragma unroll
    for (int s = 0; s < S; ++s) {
      acc[0] = MpT<E>::mfma(a0.v[s], b0.v[s], acc[0]);
      acc[1] = MpT<E>::mfma(a1.v[s], b0.v[s], acc[1]);
      if constexpr (NJ == 2) {
        acc[2] = MpT<E>::mfma(a0.v[s], b1.v[s], acc[2]);
        acc[3] = MpT<E>::mfma(a1.v[s], b1.v[s], acc[3]);
      }
    }
  }
};

// One pair of 16-row tiles times NJ 16-column tiles over all taps.  Two
// operand sets alternate (taps m and m + 1): the LDS reads of one tap are
// issued before the MFMAs of the other, and scheduling barriers keep the
// compiler from sinking them below those MFMAs, so each wait covers only
// reads that have had a whole tap of matrix work to land.
template <typename E, int S, int NJ>
__device__ inline void mp_tiles(const E* pa, const E* vb, int taps, int pp, int vstride,
                                typename MpT<E>::acc* acc) {
  MpTap<E, S, NJ> x, y;
  x.load(pa, vb, 0, pp, vstride);
  int m = 0;
  for (; m + 1 < taps; m += 2) {
    y.load(pa, vb, m + 1, pp, vstride);
    __builtin_amdgcn_sched_barrier(0);
    x.mma(acc);
    __builtin_amdgcn_sched_barrier(0);
    x.load(pa, vb, min(m + 2, taps - 1), pp, vstride);  // a valid tap; unused past the end
    __builtin_amdgcn_sched_barrier(0);
    y.mma(acc);
    __builtin_amdgcn_sched_barrier(0);
  }
  if (m < taps) x.mma(acc);
}

// Big: the variant for long fibres and many taps (one 16-column tile per
// pass and one fibre buffer, the next fibre held in registers across two
// barriers), at one workgroup of eight wavefronts per CU (two per SIMD).
template <typename E, int S, bool Big, typename F>
__device__ inline void mp_body(const typename F::Args& g, int al, int bb, int BB, E* smem) {
  using Acc = typename MpT<E>::acc;
  constexpr int QP = 4 * S;
  constexpr int JC = Big ? MP_JT : MpT<E>::JC;
  constexpr int NB = Big ? 1 : 2;  // fibre buffers
  constexpr int PF = Big ? MP_PF_BIG : MP_PF;
  constexpr int NT = Big ? MP_NT_BIG : 256;  // threads of the workgroup
  constexpr int NW = NT / 64;                // its wavefronts
  constexpr int U = 16 / (int)sizeof(E);  // elements per 16-byte unit
  const int N = g.N, rp0 = g.rp0, rp1 = g.rp1, rk1 = g.rk1, n = g.n;
  const int h = g.hk, taps = 2 * g.hk + 1;
  const int nit = (n + 15) >> 4;
  const int plen = mp_plen(n, h);
  const int pp = QP + 4;           // fibre row pitch (keeps 16-byte alignment)
  const int vstride = taps * 16 * QP;
  E* Vs = smem;                    // [JC/16][taps][16][QP]: j-tile, tap, column, bond
  E* Ps = Vs + (JC / 16) * vstride;  // [NB][plen][pp]: fibre buffers
  E* Ks = Ps + NB * plen * pp;     // [taps][32] of row a, zero beyond rk1
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lr = lane & 15, lk = lane >> 4;
  const TTG_GLOBAL E* gp = gmem(g.p);
  TTG_GLOBAL E* gz = gmem(g.z);
  const TTG_GLOBAL E* kc = gmem(g.kcore) + (long long)al * taps * rk1;
  for (int e = tid; e < taps * 32; e += blockDim.x) {
    const int m = e >> 5, a2 = e & 31;
    Ks[e] = a2 < rk1 ? kc[m * rk1 + a2] : (E)0;
  }
  const int bfirst = bb * BB;
  const int nfib = min(BB, rp0 - bfirst);
  const int pelu = plen * QP / U;  // 16-byte units of one padded fibre
  const bool vec = rp1 == QP;      // P rows are whole 16-byte units
  for (int jc0 = 0; jc0 < N; jc0 += JC) {
    const int njt = (N - jc0 > MP_JT && JC > MP_JT) ? 2 : 1;
    lds_barrier();  // Ks ready; the previous pass's V and P are consumed
    // V for this pass: a thread owns one (b', j) fibre.  Its 32 values of L
    // are loaded from clamped (always valid) addresses; rows past rk1 meet
    // the zero padding of Ks, and fibres outside the bond or the columns
    // are written as zeros.
    for (int e = tid; e < QP * JC; e += blockDim.x) {
      const int q = e / JC, jj = e - q * JC;
      const int j = jc0 + jj;
      const bool live = q < rp1 && j < N;
      const TTG_GLOBAL double* lc = gmem(g.lfac) + (long long)min(q, rp1 - 1) * g.gcap + min(j, N - 1);
      E lv[32];
#pragma unroll
      for (int a2 = 0; a2 < 32; ++a2) lv[a2] = (E)lc[(long long)min(a2, rk1 - 1) * rp1 * g.gcap];
      E* vcol = Vs + (jj >> 4) * vstride + mp_vswz<S>(jj & 15, q);
      for (int m = 0; m < taps; ++m) {
        const E* kr = Ks + m * 32;
        E v = (E)0;
#pragma unroll
        for (int a2 = 0; a2 < 32; ++a2) v += kr[a2] * lv[a2];
        vcol[m * 16 * QP] = live ? v : (E)0;
      }
    }
    // first fibre staged directly
    for (int e = tid; e < plen * QP; e += blockDim.x) {
      const int pr = e / QP, q = e - pr * QP;
      const int row = pr - h;
      Ps[pr * pp + q] = (q < rp1 && row >= 0 && row < n) ? gp[((long long)bfirst * n + row) * rp1 + q] : (E)0;
    }
    lds_barrier();
    for (int bo = 0; bo < nfib; ++bo) {
      const int be = bfirst + bo;
      E* Pc = Ps + (NB == 2 ? (bo & 1) : 0) * plen * pp;
      E* Pn = Ps + (NB == 2 ? ((bo + 1) & 1) : 0) * plen * pp;
      const bool next = bo + 1 < nfib;
      // the next fibre goes to registers while this one is multiplied
      float4 pf[PF];
      if (next) {
        const TTG_GLOBAL E* pc = gp + (long long)(be + 1) * n * rp1;
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          const int eu = tid + u * NT;
          const int pr = eu / (QP / U), cu = eu - pr * (QP / U);
          const int row = pr - h;
          float4 t = {0.f, 0.f, 0.f, 0.f};
          if (eu < pelu && row >= 0 && row < n) {
            if (vec) {
              t = *reinterpret_cast<const TTG_GLOBAL float4*>(pc + (long long)row * QP + U * cu);
            } else {
              E tmp[U];
              const TTG_GLOBAL E* src = pc + (long long)row * rp1;
#pragma unroll
              for (int x = 0; x < U; ++x) tmp[x] = (U * cu + x < rp1) ? src[U * cu + x] : (E)0;
              __builtin_memcpy(&t, tmp, 16);
            }
          }
          pf[u] = t;
        }
      }
      const long long zrow = (long long)(al * rp0 + be) * n * N;
      for (int it0 = 2 * wv; it0 < nit; it0 += 2 * NW) {
        Acc acc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = Acc{0, 0, 0, 0};
        // lane (lr, lk): A rows it*16 + lr + 2h - m, bond lk S .. lk S + S - 1;
        // B: column lr of the tile, the same bond unit (swizzled position)
        const E* pa = Pc + (it0 * 16 + lr + 2 * h) * pp + lk * S;
        const E* vb = Vs + mp_vswz<S>(lr, lk * S);
        if (njt == 2)
          mp_tiles<E, S, 2>(pa, vb, taps, pp, vstride, acc);
        else
          mp_tiles<E, S, 1>(pa, vb, taps, pp, vstride, acc);
        // D: lane (lr, lk), register v holds row drow(lk, v), column lr
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i0 = it0 * 16 + MpT<E>::drow(lk, v), i1 = i0 + 16;
          const int j0 = jc0 + lr, j1 = j0 + MP_JT;
          if (i0 < n) {
            if (j0 < N) gz[zrow + (long long)i0 * N + j0] = acc[0][v];
            if (njt == 2 && j1 < N) gz[zrow + (long long)i0 * N + j1] = acc[2][v];
          }
          if (i1 < n) {
            if (j0 < N) gz[zrow + (long long)i1 * N + j0] = acc[1][v];
            if (njt == 2 && j1 < N) gz[zrow + (long long)i1 * N + j1] = acc[3][v];
          }
        }
      }
      if constexpr (Big) lds_barrier();  // the one fibre buffer is consumed
      if (next) {
#pragma unroll
        for (int u = 0; u < PF; ++u) {
          const int eu = tid + u * NT;
          if (eu < pelu) {
            const int pr = eu / (QP / U), cu = eu - pr * (QP / U);
            *reinterpret_cast<float4*>(Pn + pr * pp + U * cu) = pf[u];
          }
        }
      }
      lds_barrier();  // next fibre stored; current one consumed
    }
  }
}

template <typename E, typename F, bool Big>
__global__ void __launch_bounds__(Big ? MP_NT_BIG : 256, (sizeof(E) == 4 && !Big) ? 2 : 1) mfma_pred_kernel(F fn, int BB) {
  typename F::Args g;
  if (!fn(blockIdx.z, g)) return;
  const int nbb = (g.rp0 + BB - 1) / BB;
  const int al = blockIdx.x / nbb, bb = blockIdx.x - al * nbb;
  if (al >= g.rk0) return;
  extern __shared__ unsigned char msm_raw[];
  E* msm = reinterpret_cast<E*>(msm_raw);
  switch (mp_s(g.rp1)) {
    case 1: mp_body<E, 1, Big, F>(g, al, bb, BB, msm); break;
    case 2: mp_body<E, 2, Big, F>(g, al, bb, BB, msm); break;
    case 4: mp_body<E, 4, Big, F>(g, al, bb, BB, msm); break;
    default: mp_body<E, 8, Big, F>(g, al, bb, BB, msm); break;
  }
}

// LDS bytes of mfma_pred_kernel<E, F, big> for the largest shapes of a launch
template <typename E>
inline size_t mfma_pred_smem(int hmax, int nmax, int pcap, int kcap, bool big = false) {
  (void)kcap;
  const int taps = 2 * hmax + 1;
  const int qp = 4 * mp_s(pcap);
  const int jc = big ? 16 : (sizeof(E) == 4 ? 32 : 16);
  const int nb = big ? 1 : 2;
  return ((size_t)(jc / 16) * taps * 16 * qp + (size_t)nb * mp_plen(nmax, hmax) * (qp + 4) + (size_t)taps * 32) *
         sizeof(E);
}

// Which variant of mfma_pred_kernel<E> a launch takes: 1 (two fibre
// buffers, two workgroups per CU), 2 (the single-buffer variant for long
// fibres or many taps) or 0 (neither fits: bond or kernel rank above 32,
// the next fibre beyond the prefetch registers, or the LDS).
template <typename E>
inline int mfma_pred_variant(int hmax, int nmax, int pcap, int kcap) {
  if (pcap > 32 || kcap > 32) return 0;
  const long long bytes = (long long)mp_plen(nmax, hmax) * 4 * mp_s(pcap) * sizeof(E);
  if (bytes <= 256LL * MP_PF * 16 && mfma_pred_smem<E>(hmax, nmax, pcap, kcap) <= 160 * 1024) return 1;
  // (FP32 only: the FP64 variant would not fit its registers)
  if (sizeof(E) == 4 && bytes <= (long long)MP_NT_BIG * MP_PF_BIG * 16 &&
      mfma_pred_smem<E>(hmax, nmax, pcap, kcap, true) <= 160 * 1024)
    return 2;
  return 0;
}
