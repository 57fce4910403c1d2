// ntt.hip -- batched negacyclic NTT over 64-bit RNS limbs for gfx950.
//
// One workgroup transforms one limb of N = 2^LOGN words entirely in LDS.
// Each thread holds 16 words; the LOGN butterfly stages are split into
// ceil(LOGN/4) register passes of radix 2^3 or 2^4, separated by LDS
// exchanges (padded by one word every 16 to spread banks).
//
// Forward: Cooley-Tukey with twiddles psi^brv(k), output in bit-reversed
// order: slot i holds a(psi^(2 brv(i) + 1)).  Inverse: Gentleman-Sande with
// psi^-brv(k), then N^-1.
//
// Two butterfly arithmetics, chosen per workgroup by the limb's prime:
//  - integer (any prime below 2^61): Harvey's lazy butterflies with Shoup
//    twiddles; forward values stay in [0, 4q), inverse values in [0, 2q);
//  - FP64 (primes below 2^50): residues are integer-valued doubles.  y w mod
//    q is the exact two-product h + l (one FMA) less qt q, qt the floor of
//    y (w/q), which is within one of the true quotient while |y w / q| <
//    2^52; the result lies in (-q, 2q).  Sums are folded back to [-1, 2q+1]
//    by x - 2q floor(x / 2q).  Every intermediate is an integer below 2^53
//    in magnitude, so the arithmetic is exact, and a butterfly is eleven
//    full-rate FP64 operations against about twice that many 32-bit integer
//    operations for the Shoup one.
//
// The prologue can lift a digit while loading (centred representative of a
// residue mod another prime: key-switch ModUp) or form r = [x + h]_p (the
// divide-and-round of ModDown and rescale, less h); the epilogue then finishes
// the division: dst = (u - NTT(r - h)) * p^-1 mod q (+ an addend).
#include <algorithm>

#include "butterfly.h"
#include "device.h"
#include "inner.h"

namespace {

__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// element index of word c of group gi in a pass over bits [lo, lo + r)
__device__ __forceinline__ int gidx(int gi, int c, int lo, int r) {
  return ((gi >> lo) << (lo + r)) | (c << lo) | (gi & ((1 << lo) - 1));
}

__device__ __forceinline__ void decode_job(const NttJob& J, int w, int& a, int& b) {
  if (J.skip_diag) {
    const int nb1 = J.nb - 1;
    a = w / nb1;
    b = w - a * nb1;
    const int j = J.amod > 0 ? a % J.amod : a;
    b += (b >= j) ? 1 : 0;
  } else {
    a = w / J.nb;
    b = w - a * J.nb;
  }
}

// the butterfly arithmetics (IntAr, FpAr) live in butterfly.h

// ---------------- pass schedules ----------------
// A workgroup holds a local array of 2^LOGM words, 16 per thread, and runs
// the butterfly stages of local bits [BLO, BHI) in register passes of at
// most 4 bits with LDS exchanges between them.  A forward pass goes from the
// top bit down, an inverse pass from the bottom bit up.  The twiddle of the
// stage on local bit lb at local element l is psi^brv at index
// 2^(LOGS - 1 - lb) + ((toff + l) >> (lb + 1)), where LOGS and toff place
// the local array in the limb (LOGS = LOGN, toff = the workgroup's first
// element, for contiguous blocks; LOGS = LOGM, toff = 0, for columns).
// LOGR caps the bits of one pass (the radix): with LOGR < LOGE a thread
// runs E / 2^R butterfly groups per pass.
template <int LOGM, int BLO, int BHI, int LOGE = 4, int LOGR = LOGE>
struct Sched {
  static_assert(LOGR <= LOGE, "a pass cannot span more words than a thread holds");
  static constexpr int M = 1 << LOGM;
  static constexpr int E = 1 << LOGE;  // words per thread
  static constexpr int T = M / E;
  static constexpr int NB = BHI - BLO;
  static constexpr int NP = (NB + LOGR - 1) / LOGR;
  static constexpr int bits(int p) { return NB / NP + (p < NB % NP ? 1 : 0); }
  static constexpr int consumed(int p) {
    int s = 0;
    for (int i = 0; i < p; i++) s += bits(i);
    return s;
  }
  static constexpr int flo(int p) { return BHI - consumed(p + 1); }  // forward pass p: bits [flo, flo + bits)
  static constexpr int ilo(int p) { return BLO + consumed(p); }      // inverse pass p
  static constexpr int lds_words() { return M + (M >> 4); }
};

// One workgroup per limb: the whole limb in LDS, E = 2^HE_SINGLE_LOGE words
// per thread, passes over all LOGN bits.
#ifndef HE_SINGLE_LOGE
#define HE_SINGLE_LOGE 3
#endif
// words per thread of the one-workgroup-per-limb kernels: at most 1024
// threads per workgroup
constexpr int single_loge(int logn) { return logn - 10 > HE_SINGLE_LOGE ? logn - 10 : HE_SINGLE_LOGE; }
template <int LOGN>
struct Cfg : Sched<LOGN, 0, LOGN, single_loge(LOGN)> {
  static constexpr int N = 1 << LOGN;
  // waves per SIMD for two workgroups per compute unit (LDS allows two up
  // to N = 8192)
  static constexpr int WAVES2 = (LOGN <= 13 ? 2 : 1) * (Sched<LOGN, 0, LOGN, single_loge(LOGN)>::T / 256);
};

template <class S, int LO, int R, int LO2, int R2, class Ar>
__device__ __forceinline__ void exchange(typename Ar::T (&x)[S::E], u64* lds, int tid) {
  constexpr int G = S::E >> R, G2 = S::E >> R2;
#pragma unroll
  for (int u = 0; u < G; u++)
#pragma unroll
    for (int c = 0; c < (1 << R); c++) lds[pad(gidx(tid + S::T * u, c, LO, R))] = Ar::bits(x[u * (1 << R) + c]);
  __syncthreads();
#pragma unroll
  for (int u = 0; u < G2; u++)
#pragma unroll
    for (int c = 0; c < (1 << R2); c++)
      x[u * (1 << R2) + c] = Ar::unbits(lds[pad(gidx(tid + S::T * u, c, LO2, R2))]);
}

// Twiddle index of a pass whose group bits start at LO: for LO >= 6 the
// index (gi >> LO) is the same for the 64 lanes of a wave (gi = tid + T*u
// with T a multiple of 64), so it is made wave-uniform and the twiddle comes
// through the scalar cache instead of 64 vector lanes.
template <class S, int LO>
__device__ __forceinline__ int tw_index(int ti) {
  if constexpr (LO >= 6 && S::T % 64 == 0)
    return __builtin_amdgcn_readfirstlane(ti);
  else
    return ti;
}

// ---------------- forward passes ----------------
// Twiddles of one pass for one thread, loaded ahead of the butterflies.
// Stage pb of a pass of R bits uses 2^(R-1-pb) twiddles per group, kept
// at heap positions 2^(R-1-pb) - 1 + j.
template <class S, int LOGS, int P, bool FWD, class Ar>
struct PassTw {
  static constexpr int R = S::bits(P);
  static constexpr int G = S::E >> R;
  static constexpr int PER = (1 << R) - 1;
  static constexpr int LO = FWD ? S::flo(P) : S::ilo(P);
  typename Ar::TW t[G * PER];
  __device__ __forceinline__ void load(const typename Ar::TW* __restrict__ W, int tid, int toff) {
#pragma unroll
    for (int pb = 0; pb < R; pb++) {
      const int lb = LO + pb;
      const int base = (1 << (LOGS - 1 - lb)) + (toff >> (lb + 1));
#pragma unroll
      for (int u = 0; u < G; u++) {
        const int gi = tid + S::T * u;
#pragma unroll
        for (int j = 0; j < (1 << (R - 1 - pb)); j++)
          t[u * PER + (1 << (R - 1 - pb)) - 1 + j] = W[tw_index<S, LO>(base + (((gi >> LO) << (R - 1 - pb)) | j))];
      }
    }
  }
};

// Butterflies of pass P.  With PRE, the twiddles come from `tw` and the next
// pass's are loaded before this pass's butterflies, so their latency
// overlaps arithmetic and the exchange (one-wave workgroups have no other
// waves to hide it); otherwise each stage loads its own.
// With PRE false and toff 0, the twiddles of the stages lb >= TWLB (indices
// below 2^(LOGS - TWLB)) come from the LDS copy Wl, the others' from W.
template <class S, int LOGS, int P, class Ar, bool PRE, int TWLB = 99>
__device__ __forceinline__ void fwd_passes(typename Ar::T (&x)[S::E], u64* lds, const typename Ar::TW* __restrict__ W,
                                           const Ar& ar, int tid, int toff,
                                           const PassTw<S, LOGS, P, true, Ar>* tw = nullptr,
                                           const typename Ar::TW* Wl = nullptr) {
  constexpr int R = S::bits(P);
  constexpr int LO = S::flo(P);
  constexpr int G = S::E >> R;
  constexpr int PER = (1 << R) - 1;
  constexpr bool MORE = P + 1 < S::NP;
  PassTw<S, LOGS, (MORE ? P + 1 : P), true, Ar> nxt;
  if (PRE && MORE) nxt.load(W, tid, toff);
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int pb = R - 1 - r;
    const int lb = LO + pb;
    const int base = (1 << (LOGS - 1 - lb)) + (toff >> (lb + 1));
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) {
        if (c & (1 << pb)) continue;
        const int i0 = u * (1 << R) + c, i1 = i0 + (1 << pb);
        if constexpr (PRE) {
          ar.fwd(x[i0], x[i1], tw->t[u * PER + (1 << (R - 1 - pb)) - 1 + (c >> (pb + 1))]);
        } else {
          const int ti = base + (((gi >> LO) << (R - 1 - pb)) | (c >> (pb + 1)));
          if (lb >= TWLB)
            ar.fwd(x[i0], x[i1], Wl[tw_index<S, LO>(ti)]);
          else
            ar.fwd(x[i0], x[i1], W[tw_index<S, LO>(ti)]);
        }
      }
    }
  }
  if constexpr (MORE) {
    if (P > 0) __syncthreads();
    exchange<S, LO, R, S::flo(P + 1), S::bits(P + 1), Ar>(x, lds, tid);
    fwd_passes<S, LOGS, P + 1, Ar, PRE, TWLB>(x, lds, W, ar, tid, toff, &nxt, Wl);
  }
}

// ---------------- inverse passes ----------------
template <class S, int LOGS, int P, class Ar, bool PRE>
__device__ __forceinline__ void inv_passes(typename Ar::T (&x)[S::E], u64* lds, const typename Ar::TW* __restrict__ W,
                                           const Ar& ar, int tid, int toff,
                                           const PassTw<S, LOGS, P, false, Ar>* tw = nullptr) {
  constexpr int R = S::bits(P);
  constexpr int LO = S::ilo(P);
  constexpr int G = S::E >> R;
  constexpr int PER = (1 << R) - 1;
  constexpr bool MORE = P + 1 < S::NP;
  PassTw<S, LOGS, (MORE ? P + 1 : P), false, Ar> nxt;
  if (PRE && MORE) nxt.load(W, tid, toff);
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int pb = r;
    const int lb = LO + pb;
    const int base = (1 << (LOGS - 1 - lb)) + (toff >> (lb + 1));
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) {
        if (c & (1 << pb)) continue;
        const int i0 = u * (1 << R) + c, i1 = i0 + (1 << pb);
        if constexpr (PRE) {
          ar.inv(x[i0], x[i1], tw->t[u * PER + (1 << (R - 1 - pb)) - 1 + (c >> (pb + 1))]);
        } else {
          const int ti = base + (((gi >> LO) << (R - 1 - pb)) | (c >> (pb + 1)));
          ar.inv(x[i0], x[i1], W[tw_index<S, LO>(ti)]);
        }
      }
    }
  }
  if constexpr (MORE) {
    if (P > 0) __syncthreads();
    exchange<S, LO, R, S::ilo(P + 1), S::bits(P + 1), Ar>(x, lds, tid);
    inv_passes<S, LOGS, P + 1, Ar, PRE>(x, lds, W, ar, tid, toff, &nxt);
  }
}

// ---------------- forward kernel ----------------
// C: the thread layout (a Sched over all LOGN bits); the kernels below use
// Cfg<LOGN>, the work-queue kernels a fixed 1024-thread layout
// tid: the thread's index (the work-queue kernel passes one the compiler
// cannot hoist out of its task loop, so that the per-thread exchange
// addresses are recomputed per task instead of held across tasks)
template <int LOGN, int PRO, int EPI, class Ar, class C = Cfg<LOGN>>
__device__ __forceinline__ void fwd_body(const NttJob& J, const PrimeDev* __restrict__ primes,
                                         const typename Ar::TW* __restrict__ W, const PrimeDev& P, int a, int b,
                                         u64* lds, const int tid = threadIdx.x) {
  const Ar ar(P);
  const u64 q = P.q;
  const u64* __restrict__ src = J.src + a * J.sa + b * J.sb;
  typename Ar::T x[C::E];
  {
    constexpr int R = C::bits(0), LO = LOGN - R, G = C::E >> R;
    u64 sq = 0, sh = 0;
    const u64 hq_b = (PRO == PRO_ROUNDDIV_LIFT) ? J.hq[b] : 0;
    if (PRO != PRO_PLAIN) {
      const int sp = J.src_prime >= 0 ? J.src_prime : (J.amod > 0 ? a % J.amod : a);
      sq = primes[sp].q;
      sh = (sq - 1) >> 1;
    }
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + C::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) {
        u64 v = src[(c << LO) | gi];
        if (PRO == PRO_CENTRED_LIFT) {
          if (v > sh) {
            const u64 r = red64(sq - v, P);
            v = r ? q - r : 0;
          } else {
            v = red64(v, P);
          }
        } else if (PRO == PRO_ROUNDDIV_LIFT) {
          // r = [x + h]_p lifted to q, minus h: the epilogue then forms
          // (x + h - r) / p coefficient-wise as (u - NTT(r - h)) * p^-1
          v += sh;
          v = v >= sq ? v - sq : v;
          v = submod(red64(v, P), hq_b, q);
        }
        x[u * (1 << R) + c] = ar.from_res(v);
      }
    }
  }
  fwd_passes<C, LOGN, 0, Ar, false>(x, lds, W, ar, tid, 0);
  {
    constexpr int R = C::bits(C::NP - 1), G = C::E >> R;
    u64* __restrict__ dst = J.dst + a * J.da + b * J.db;
    const u64* __restrict__ uu = nullptr;
    const u64* __restrict__ ad = nullptr;
    const u64* __restrict__ ad2 = nullptr;
    u64 ag = 1;
    u64 inv = 0, inv_sh = 0;
    if (EPI == EPI_ROUNDDIV) {
      uu = J.u + a * J.ua + b * J.ub;
      ad = (J.add && !(J.add_even_only && (a & 1))) ? J.add + a * J.aa + b * J.ab : nullptr;
      ad2 = J.add2 ? J.add2 + a * J.a2a + b * J.ab : nullptr;
      ag = J.add_gather ? J.gal[a >> 1] : 1;
      inv = J.inv[b];
      inv_sh = J.inv_sh[b];
    }
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + C::T * u;
      if constexpr (EPI == EPI_STORE && R >= 1) {
        // each thread's run of 2^R consecutive words leaves as 16-byte stores
#pragma unroll
        for (int c = 0; c < (1 << R); c += 2) {
          ulonglong2 v2;
          v2.x = ar.fwd_res(x[u * (1 << R) + c]);
          v2.y = ar.fwd_res(x[u * (1 << R) + c + 1]);
          *reinterpret_cast<ulonglong2*>(dst + ((gi << R) | c)) = v2;
        }
      } else {
#pragma unroll
        for (int c = 0; c < (1 << R); c++) {
          u64 v = ar.fwd_res(x[u * (1 << R) + c]);
          const int idx = (gi << R) | c;
          if (EPI == EPI_ROUNDDIV) {
            v = shoup(submod(uu[idx], v, q), inv, inv_sh, q);
            if (ad) v = addmod(v, ad[ag != 1 ? gal_src(idx, LOGN, ag) : idx], q);
            if (ad2) v = addmod(v, ad2[idx], q);
          }
          dst[idx] = v;
        }
      }
    }
  }
}

template <int LOGN, int PRO, int EPI>
__global__ void __launch_bounds__(Cfg<LOGN>::T, Cfg<LOGN>::WAVES2)
k_ntt_fwd(const NttJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  constexpr int N = Cfg<LOGN>::N;
  extern __shared__ u64 lds[];
  int a, b;
  decode_job(J, blockIdx.x, a, b);
  const int dp = J.dst_prime[b];
  const PrimeDev P = primes[dp];
  if (P.use_fp)
    fwd_body<LOGN, PRO, EPI, FpAr>(J, primes, reinterpret_cast<const double2*>(tabs.fwd_fp) + (size_t)dp * N, P, a,
                                   b, lds);
  else
    fwd_body<LOGN, PRO, EPI, IntAr>(J, primes, reinterpret_cast<const ulonglong2*>(tabs.fwd) + (size_t)dp * N, P, a,
                                    b, lds);
}

// ---------------- inverse kernel ----------------
template <int LOGN, bool GATHER, class Ar, class C = Cfg<LOGN>>
__device__ __forceinline__ void inv_body(const NttJob& J, const typename Ar::TW* __restrict__ W, const PrimeDev& P,
                                         int a, int b, u64* lds, const int tid = threadIdx.x) {
  const Ar ar(P);
  const u64* __restrict__ src = J.src + a * J.sa + b * J.sb;
  typename Ar::T x[C::E];
  {
    constexpr int R = C::bits(0), G = C::E >> R;  // bits [0, R): contiguous runs
    const u64 g = GATHER ? J.gal[a / J.gal_div] : 1;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + C::T * u;
      if constexpr (!GATHER && R >= 1) {
        // each thread's run of 2^R consecutive words arrives as 16-byte loads
#pragma unroll
        for (int c = 0; c < (1 << R); c += 2) {
          const ulonglong2 v2 = *reinterpret_cast<const ulonglong2*>(src + ((gi << R) | c));
          x[u * (1 << R) + c] = ar.from_res(v2.x);
          x[u * (1 << R) + c + 1] = ar.from_res(v2.y);
        }
      } else {
#pragma unroll
        for (int c = 0; c < (1 << R); c++) {
          const int idx = (gi << R) | c;
          x[u * (1 << R) + c] = ar.from_res(src[GATHER ? gal_src(idx, LOGN, g) : idx]);
        }
      }
    }
  }
  inv_passes<C, LOGN, 0, Ar, false>(x, lds, W, ar, tid, 0);
  {
    constexpr int R = C::bits(C::NP - 1), LO = LOGN - R, G = C::E >> R;
    u64* __restrict__ dst = J.dst + a * J.da + b * J.db;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + C::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) dst[(c << LO) | gi] = ar.inv_res(x[u * (1 << R) + c], P);
    }
  }
}

template <int LOGN, bool GATHER>
__global__ void __launch_bounds__(Cfg<LOGN>::T, Cfg<LOGN>::WAVES2)
k_ntt_inv(const NttJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  constexpr int N = Cfg<LOGN>::N;
  extern __shared__ u64 lds[];
  int a, b;
  decode_job(J, blockIdx.x, a, b);
  const int dp = J.dst_prime[b];
  const PrimeDev P = primes[dp];
  if (P.use_fp)
    inv_body<LOGN, GATHER, FpAr>(J, reinterpret_cast<const double2*>(tabs.inv_fp) + (size_t)dp * N, P, a, b, lds);
  else
    inv_body<LOGN, GATHER, IntAr>(J, reinterpret_cast<const ulonglong2*>(tabs.inv) + (size_t)dp * N, P, a, b, lds);
}

// ---------------- alternative thread layouts (tuned) ----------------
// The plain transforms (no prologue or epilogue) in other layouts: E = 2^LOGE
// words per thread, passes of at most 2^LOGR.  Same butterflies in the same
// order per element, so the results are identical.
template <int LOGN, int LOGE, int LOGR>
using Shape = Sched<LOGN, 0, LOGN, LOGE, LOGR>;

template <int LOGN, bool FWD, int LOGE, int LOGR>
__global__ void __launch_bounds__((Shape<LOGN, LOGE, LOGR>::T))
k_ntt_shape(const NttJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  using S = Shape<LOGN, LOGE, LOGR>;
  constexpr int N = 1 << LOGN;
  extern __shared__ u64 lds[];
  int a, b;
  decode_job(J, blockIdx.x, a, b);
  const int dp = J.dst_prime[b];
  const PrimeDev P = primes[dp];
  if constexpr (FWD) {
    if (P.use_fp)
      fwd_body<LOGN, PRO_PLAIN, EPI_STORE, FpAr, S>(J, primes,
                                                   reinterpret_cast<const double2*>(tabs.fwd_fp) + (size_t)dp * N, P,
                                                   a, b, lds);
    else
      fwd_body<LOGN, PRO_PLAIN, EPI_STORE, IntAr, S>(
          J, primes, reinterpret_cast<const ulonglong2*>(tabs.fwd) + (size_t)dp * N, P, a, b, lds);
  } else {
    if (P.use_fp)
      inv_body<LOGN, false, FpAr, S>(J, reinterpret_cast<const double2*>(tabs.inv_fp) + (size_t)dp * N, P, a, b, lds);
    else
      inv_body<LOGN, false, IntAr, S>(J, reinterpret_cast<const ulonglong2*>(tabs.inv) + (size_t)dp * N, P, a, b,
                                      lds);
  }
}

// the alternative layouts per ring degree (index 1.. of ntt_shapes)
template <int LOGN>
struct ShapeList;
template <>
struct ShapeList<12> {
  static constexpr int n = 4;
  static constexpr int e[n] = {2, 3, 4, 4}, r[n] = {2, 2, 4, 3};
};
template <>
struct ShapeList<13> {
  static constexpr int n = 3;
  static constexpr int e[n] = {4, 4, 3}, r[n] = {4, 3, 2};
};
template <>
struct ShapeList<14> {
  static constexpr int n = 3;
  static constexpr int e[n] = {4, 5, 5}, r[n] = {3, 5, 4};
};

template <int LOGN, bool FWD, int I>
hipError_t shape_launch_i(const NttJob& J, const PrimeDev* primes, const NttTables& tabs, hipStream_t st,
                          int jobs) {
  constexpr int LOGE = ShapeList<LOGN>::e[I], LOGR = ShapeList<LOGN>::r[I];
  using S = Shape<LOGN, LOGE, LOGR>;
  const size_t shm = sizeof(u64) * S::lds_words();
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_ntt_shape<LOGN, FWD, LOGE, LOGR>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL((k_ntt_shape<LOGN, FWD, LOGE, LOGR>), dim3(jobs), dim3(S::T), shm, st, J, primes, tabs);
  return hipGetLastError();
}

template <int LOGN, bool FWD>
hipError_t shape_launch(int id, const NttJob& J, const PrimeDev* primes, const NttTables& tabs, hipStream_t st,
                        int jobs) {
  switch (id) {
    case 1: return shape_launch_i<LOGN, FWD, 0>(J, primes, tabs, st, jobs);
    case 2: return shape_launch_i<LOGN, FWD, 1>(J, primes, tabs, st, jobs);
    case 3: return shape_launch_i<LOGN, FWD, 2>(J, primes, tabs, st, jobs);
    case 4:
      if constexpr (ShapeList<LOGN>::n > 3) return shape_launch_i<LOGN, FWD, 3>(J, primes, tabs, st, jobs);
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
}

// the tuned layout of a plain launch of `jobs` limbs (0: the default)
int tuned_shape(const NttTables& tabs, int jobs) {
  if (tabs.layout > 0) return tabs.layout;
  if (!tabs.tuned) return 0;
  int b = 0;
  while (b + 1 < tabs.n_buckets && jobs > (16 << b)) b++;
  return tabs.shape[b];
}

// ---------------- two-phase transforms for small batches ----------------
// The limb is viewed as 2^A rows of 2^K columns (K = ceil(LOGN / 2)): the
// first A forward stages only mix elements of one column (stride 2^K), the
// last K stages only elements of one contiguous block of 2^K; the inverse
// runs the same split in the other order.  Each phase spreads a limb over
// several workgroups of one or two waves, so that a launch of a few limbs
// still occupies many compute units; the intermediate values (lazy, in the
// limb's own arithmetic) pass through a scratch buffer of N words per job.
#ifndef HE_SPLIT_LOGE
#define HE_SPLIT_LOGE 2
#endif
template <int LOGN>
struct Split {
  static constexpr int K = (LOGN + 1) / 2;                     // block bits
  static constexpr int A = LOGN - K;                           // row bits
  static constexpr int LOGMA = (A + 4 < LOGN) ? A + 4 : LOGN;  // 16 columns per workgroup
  static constexpr int LOGC = LOGMA - A;
  static constexpr int LOGMB = (10 < LOGN) ? 10 : LOGN;
  using SA = Sched<LOGMA, LOGC, LOGMA, HE_SPLIT_LOGE>;  // column phase over the row bits
  using SB = Sched<LOGMB, 0, K, HE_SPLIT_LOGE>;          // block phase over the low bits
  static constexpr int WA = 1 << (LOGN - LOGMA);  // workgroups per limb
  static constexpr int WB = 1 << (LOGN - LOGMB);
};

// limb index of local element l of column workgroup sub
template <int LOGN>
__device__ __forceinline__ int col_g(int l, int sub) {
  using Sp = Split<LOGN>;
  return ((l >> Sp::LOGC) << Sp::K) | (sub << Sp::LOGC) | (l & ((1 << Sp::LOGC) - 1));
}

template <int LOGN, int PRO, class Ar>
__device__ __forceinline__ void fwd_a_body(const NttJob& J, const PrimeDev* __restrict__ primes,
                                           const typename Ar::TW* __restrict__ W, const PrimeDev& P, int w, int a,
                                           int b, int sub, u64* __restrict__ tmp, u64* lds) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SA;
  const Ar ar(P);
  const int tid = threadIdx.x;
  const u64 q = P.q;
  const u64* __restrict__ src = J.src + a * J.sa + b * J.sb;
  typename Ar::T x[S::E];
  PassTw<S, Sp::LOGMA, 0, true, Ar> tw0;
  tw0.load(W, tid, 0);
  {
    constexpr int R = S::bits(0), LO = S::flo(0), G = S::E >> R;
    u64 sq = 0, sh = 0;
    const u64 hq_b = (PRO == PRO_ROUNDDIV_LIFT) ? J.hq[b] : 0;
    if (PRO != PRO_PLAIN) {
      const int sp = J.src_prime >= 0 ? J.src_prime : (J.amod > 0 ? a % J.amod : a);
      sq = primes[sp].q;
      sh = (sq - 1) >> 1;
    }
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) {
        u64 v = src[col_g<LOGN>(gidx(gi, c, LO, R), sub)];
        if (PRO == PRO_CENTRED_LIFT) {
          if (v > sh) {
            const u64 r = red64(sq - v, P);
            v = r ? q - r : 0;
          } else {
            v = red64(v, P);
          }
        } else if (PRO == PRO_ROUNDDIV_LIFT) {
          v += sh;
          v = v >= sq ? v - sq : v;
          v = submod(red64(v, P), hq_b, q);
        }
        x[u * (1 << R) + c] = ar.from_res(v);
      }
    }
  }
  fwd_passes<S, Sp::LOGMA, 0, Ar, true>(x, lds, W, ar, tid, 0, &tw0);
  {
    constexpr int R = S::bits(S::NP - 1), LO = S::flo(S::NP - 1), G = S::E >> R;
    u64* __restrict__ t = tmp + (size_t)w * (1 << LOGN);
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) t[col_g<LOGN>(gidx(gi, c, LO, R), sub)] = Ar::bits(x[u * (1 << R) + c]);
    }
  }
}

template <int LOGN, int EPI, class Ar>
__device__ __forceinline__ void fwd_b_body(const NttJob& J, const typename Ar::TW* __restrict__ W, const PrimeDev& P,
                                           int w, int a, int b, int sub, const u64* __restrict__ tmp, u64* lds) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SB;
  const Ar ar(P);
  const int tid = threadIdx.x;
  const u64 q = P.q;
  const int toff = sub << Sp::LOGMB;
  const u64* __restrict__ t = tmp + (size_t)w * (1 << LOGN) + toff;
  typename Ar::T x[S::E];
  PassTw<S, LOGN, 0, true, Ar> tw0;
  tw0.load(W, tid, toff);
  {
    constexpr int R = S::bits(0), LO = S::flo(0), G = S::E >> R;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) x[u * (1 << R) + c] = Ar::unbits(t[gidx(gi, c, LO, R)]);
    }
  }
  fwd_passes<S, LOGN, 0, Ar, true>(x, lds, W, ar, tid, toff, &tw0);
  {
    constexpr int R = S::bits(S::NP - 1), G = S::E >> R;
    u64* __restrict__ dst = J.dst + a * J.da + b * J.db;
    const u64* __restrict__ uu = nullptr;
    const u64* __restrict__ ad = nullptr;
    const u64* __restrict__ ad2 = nullptr;
    u64 ag = 1;
    u64 inv = 0, inv_sh = 0;
    if (EPI == EPI_ROUNDDIV) {
      uu = J.u + a * J.ua + b * J.ub;
      ad = (J.add && !(J.add_even_only && (a & 1))) ? J.add + a * J.aa + b * J.ab : nullptr;
      ad2 = J.add2 ? J.add2 + a * J.a2a + b * J.ab : nullptr;
      ag = J.add_gather ? J.gal[a >> 1] : 1;
      inv = J.inv[b];
      inv_sh = J.inv_sh[b];
    }
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) {
        u64 v = ar.fwd_res(x[u * (1 << R) + c]);
        const int idx = toff + ((gi << R) | c);
        if (EPI == EPI_ROUNDDIV) {
          v = shoup(submod(uu[idx], v, q), inv, inv_sh, q);
          if (ad) v = addmod(v, ad[ag != 1 ? gal_src(idx, LOGN, ag) : idx], q);
          if (ad2) v = addmod(v, ad2[idx], q);
        }
        dst[idx] = v;
      }
    }
  }
}

template <int LOGN, bool GATHER, class Ar>
__device__ __forceinline__ void inv_1_body(const NttJob& J, const typename Ar::TW* __restrict__ W, const PrimeDev& P,
                                           int w, int a, int b, int sub, u64* __restrict__ tmp, u64* lds) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SB;
  const Ar ar(P);
  const int tid = threadIdx.x;
  const int toff = sub << Sp::LOGMB;
  const u64* __restrict__ src = J.src + a * J.sa + b * J.sb;
  typename Ar::T x[S::E];
  PassTw<S, LOGN, 0, false, Ar> tw0;
  tw0.load(W, tid, toff);
  {
    constexpr int R = S::bits(0), G = S::E >> R;
    const u64 g = GATHER ? J.gal[a / J.gal_div] : 1;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) {
        const int idx = toff + ((gi << R) | c);
        x[u * (1 << R) + c] = ar.from_res(src[GATHER ? gal_src(idx, LOGN, g) : idx]);
      }
    }
  }
  inv_passes<S, LOGN, 0, Ar, true>(x, lds, W, ar, tid, toff, &tw0);
  {
    constexpr int R = S::bits(S::NP - 1), LO = S::ilo(S::NP - 1), G = S::E >> R;
    u64* __restrict__ t = tmp + (size_t)w * (1 << LOGN) + toff;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) t[gidx(gi, c, LO, R)] = Ar::bits(x[u * (1 << R) + c]);
    }
  }
}

template <int LOGN, class Ar>
__device__ __forceinline__ void inv_2_body(const NttJob& J, const typename Ar::TW* __restrict__ W, const PrimeDev& P,
                                           int w, int a, int b, int sub, const u64* __restrict__ tmp, u64* lds) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SA;
  const Ar ar(P);
  const int tid = threadIdx.x;
  const u64* __restrict__ t = tmp + (size_t)w * (1 << LOGN);
  typename Ar::T x[S::E];
  PassTw<S, Sp::LOGMA, 0, false, Ar> tw0;
  tw0.load(W, tid, 0);
  {
    constexpr int R = S::bits(0), LO = S::ilo(0), G = S::E >> R;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) x[u * (1 << R) + c] = Ar::unbits(t[col_g<LOGN>(gidx(gi, c, LO, R), sub)]);
    }
  }
  inv_passes<S, Sp::LOGMA, 0, Ar, true>(x, lds, W, ar, tid, 0, &tw0);
  {
    constexpr int R = S::bits(S::NP - 1), LO = S::ilo(S::NP - 1), G = S::E >> R;
    u64* __restrict__ dst = J.dst + a * J.da + b * J.db;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++)
        dst[col_g<LOGN>(gidx(gi, c, LO, R), sub)] = ar.inv_res(x[u * (1 << R) + c], P);
    }
  }
}

#define HE_PHASE_PRELUDE(WPL)                          \
  constexpr int N = 1 << LOGN;                         \
  const int w = blockIdx.x / (WPL);                    \
  const int sub = blockIdx.x - w * (WPL);              \
  int a, b;                                            \
  decode_job(J, w, a, b);                              \
  const int dp = J.dst_prime[b];                       \
  const PrimeDev P = primes[dp];                       \
  const double2* Wf = reinterpret_cast<const double2*>(tabs_fp) + (size_t)dp * N;                 \
  const ulonglong2* Wi = reinterpret_cast<const ulonglong2*>(tabs_int) + (size_t)dp * N;

template <int LOGN, int PRO>
__global__ void __launch_bounds__(Split<LOGN>::SA::T)
k_ntt_fwd_a(const NttJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  __shared__ u64 lds[Split<LOGN>::SA::lds_words()];
  const u64* tabs_fp = tabs.fwd_fp;
  const u64* tabs_int = tabs.fwd;
  HE_PHASE_PRELUDE(Split<LOGN>::WA)
  if (P.use_fp)
    fwd_a_body<LOGN, PRO, FpAr>(J, primes, Wf, P, w, a, b, sub, J.mid ? J.mid : tabs.tmp, lds);
  else
    fwd_a_body<LOGN, PRO, IntAr>(J, primes, Wi, P, w, a, b, sub, J.mid ? J.mid : tabs.tmp, lds);
}

// FAM names the launch family (the block phase has no prologue): the PRO_*
// value of the launch, or FAM_RESCALE for the last kernel of a fused rescale
template <int LOGN, int FAM, int EPI>
__global__ void __launch_bounds__(Split<LOGN>::SB::T)
k_ntt_fwd_b(const NttJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  __shared__ u64 lds[Split<LOGN>::SB::lds_words()];
  const u64* tabs_fp = tabs.fwd_fp;
  const u64* tabs_int = tabs.fwd;
  HE_PHASE_PRELUDE(Split<LOGN>::WB)
  if (P.use_fp)
    fwd_b_body<LOGN, EPI, FpAr>(J, Wf, P, w, a, b, sub, J.mid ? J.mid : tabs.tmp, lds);
  else
    fwd_b_body<LOGN, EPI, IntAr>(J, Wi, P, w, a, b, sub, J.mid ? J.mid : tabs.tmp, lds);
}

// TAG names the launch family: 0 plain inverse, 1 the first kernel of a
// fused key-switch ModUp, 2 that of a fused rescale
template <int LOGN, bool GATHER, int TAG>
__global__ void __launch_bounds__(Split<LOGN>::SB::T)
k_ntt_inv_1(const NttJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  __shared__ u64 lds[Split<LOGN>::SB::lds_words()];
  const u64* tabs_fp = tabs.inv_fp;
  const u64* tabs_int = tabs.inv;
  HE_PHASE_PRELUDE(Split<LOGN>::WB)
  if (P.use_fp)
    inv_1_body<LOGN, GATHER, FpAr>(J, Wf, P, w, a, b, sub, J.mid ? J.mid : tabs.tmp, lds);
  else
    inv_1_body<LOGN, GATHER, IntAr>(J, Wi, P, w, a, b, sub, J.mid ? J.mid : tabs.tmp, lds);
}

template <int LOGN>
__global__ void __launch_bounds__(Split<LOGN>::SA::T)
k_ntt_inv_2(const NttJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  __shared__ u64 lds[Split<LOGN>::SA::lds_words()];
  const u64* tabs_fp = tabs.inv_fp;
  const u64* tabs_int = tabs.inv;
  HE_PHASE_PRELUDE(Split<LOGN>::WA)
  if (P.use_fp)
    inv_2_body<LOGN, FpAr>(J, Wf, P, w, a, b, sub, J.mid ? J.mid : tabs.tmp, lds);
  else
    inv_2_body<LOGN, IntAr>(J, Wi, P, w, a, b, sub, J.mid ? J.mid : tabs.tmp, lds);
}
#undef HE_PHASE_PRELUDE

// ---------------- fused key switch (small batches) ----------------
// Column phases of two transforms in one workgroup: the inverse column phase
// of a limb under prime s finishes its coefficients, which are lifted to
// prime t (centred digit for ModUp, r - h of the divide-and-round for
// ModDown) and run through the forward column phase under prime t.
template <int LOGN, int PRO, class ArS, class ArT>
__device__ __forceinline__ void cols_fused_body(const u64* __restrict__ tin, u64* __restrict__ tout,
                                                const PrimeDev& Ps, const PrimeDev& Pt,
                                                const typename ArS::TW* __restrict__ Wi,
                                                const typename ArT::TW* __restrict__ Wf, u64 hs, u64 hq_t, int sub,
                                                u64* lds) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SA;
  constexpr int E = S::E;
  const ArS ars(Ps);
  const ArT art(Pt);
  const int tid = threadIdx.x;
  PassTw<S, Sp::LOGMA, 0, false, ArS> twi;
  PassTw<S, Sp::LOGMA, 0, true, ArT> twf;
  twi.load(Wi, tid, 0);
  twf.load(Wf, tid, 0);
  typename ArS::T x[E];
  {
    constexpr int R = S::bits(0), LO = S::ilo(0), G = E >> R;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) x[u * (1 << R) + c] = ArS::unbits(tin[col_g<LOGN>(gidx(gi, c, LO, R), sub)]);
    }
  }
  inv_passes<S, Sp::LOGMA, 0, ArS, true>(x, lds, Wi, ars, tid, 0, &twi);
  // coefficients mod q_s, lifted to q_t
  const u64 qs = Ps.q, qt = Pt.q;
  u64 v[E];
#pragma unroll
  for (int i = 0; i < E; i++) {
    u64 r = ars.inv_res(x[i], Ps);
    if (PRO == PRO_CENTRED_LIFT) {
      if (r > hs) {
        const u64 m = red64(qs - r, Pt);
        r = m ? qt - m : 0;
      } else {
        r = red64(r, Pt);
      }
    } else {
      r += hs;
      r = r >= qs ? r - qs : r;
      r = submod(red64(r, Pt), hq_t, qt);
    }
    v[i] = r;
  }
  constexpr int RI = S::bits(S::NP - 1), LOI = S::ilo(S::NP - 1);
  constexpr int RF = S::bits(0), LOF = S::flo(0);
  __syncthreads();  // the inverse passes' last reads of LDS are done
  if constexpr (RI != RF || LOI != LOF) {
    exchange<S, LOI, RI, LOF, RF, IntAr>(v, lds, tid);
    __syncthreads();
  }
  typename ArT::T y[E];
#pragma unroll
  for (int i = 0; i < E; i++) y[i] = art.from_res(v[i]);
  fwd_passes<S, Sp::LOGMA, 0, ArT, true>(y, lds, Wf, art, tid, 0, &twf);
  {
    constexpr int R = S::bits(S::NP - 1), LO = S::flo(S::NP - 1), G = E >> R;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) tout[col_g<LOGN>(gidx(gi, c, LO, R), sub)] = ArT::bits(y[u * (1 << R) + c]);
    }
  }
}

template <int LOGN, int PRO>
__device__ __forceinline__ void cols_fused_dispatch(const u64* tin, u64* tout, const PrimeDev* __restrict__ primes,
                                                    int ps, int pt, const NttTables& tabs, u64 hs, u64 hq_t,
                                                    int sub, u64* lds) {
  constexpr int N = 1 << LOGN;
  const PrimeDev Ps = primes[ps], Pt = primes[pt];
  const ulonglong2* Ii = reinterpret_cast<const ulonglong2*>(tabs.inv) + (size_t)ps * N;
  const double2* If = reinterpret_cast<const double2*>(tabs.inv_fp) + (size_t)ps * N;
  const ulonglong2* Fi = reinterpret_cast<const ulonglong2*>(tabs.fwd) + (size_t)pt * N;
  const double2* Ff = reinterpret_cast<const double2*>(tabs.fwd_fp) + (size_t)pt * N;
  if (Ps.use_fp) {
    if (Pt.use_fp)
      cols_fused_body<LOGN, PRO, FpAr, FpAr>(tin, tout, Ps, Pt, If, Ff, hs, hq_t, sub, lds);
    else
      cols_fused_body<LOGN, PRO, FpAr, IntAr>(tin, tout, Ps, Pt, If, Fi, hs, hq_t, sub, lds);
  } else {
    if (Pt.use_fp)
      cols_fused_body<LOGN, PRO, IntAr, FpAr>(tin, tout, Ps, Pt, Ii, Ff, hs, hq_t, sub, lds);
    else
      cols_fused_body<LOGN, PRO, IntAr, IntAr>(tin, tout, Ps, Pt, Ii, Fi, hs, hq_t, sub, lds);
  }
}

// ModUp: job w = (b*Lp + j)*Lp + tt lifts digit j of item b to modulus
// t = tt (tt < j) or tt + 1 (t = Lp is the special prime)
template <int LOGN>
__global__ void __launch_bounds__(Split<LOGN>::SA::T)
k_ks_modup_cols(const KsJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[Split<LOGN>::SA::lds_words()];
  const int w = blockIdx.x / Split<LOGN>::WA;
  const int sub = blockIdx.x - w * Split<LOGN>::WA;
  const int a = w / J.Lp, tt = w - a * J.Lp;
  const int j = a % J.Lp;
  const int t = tt < j ? tt : tt + 1;
  const int pt = t < J.Lp ? t : J.special;
  const u64 hs = (primes[j].q - 1) >> 1;
  cols_fused_dispatch<LOGN, PRO_CENTRED_LIFT>(J.t1 + (size_t)a * N, J.t2 + (size_t)w * N, primes, j, pt, tabs, hs, 0,
                                              sub, lds);
}

// ModDown columns: job w = a*Lp + t, a = 2b + k (TAG names the launch
// family: 0 key-switch ModDown, 1 rescale)
template <int LOGN, int TAG>
__global__ void __launch_bounds__(Split<LOGN>::SA::T)
k_ks_moddown_cols(const KsJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[Split<LOGN>::SA::lds_words()];
  const int w = blockIdx.x / Split<LOGN>::WA;
  const int sub = blockIdx.x - w * Split<LOGN>::WA;
  const int a = w / J.Lp, t = w - a * J.Lp;
  cols_fused_dispatch<LOGN, PRO_ROUNDDIV_LIFT>(J.t3 + (size_t)a * N, J.t4 + (size_t)w * N, primes, J.special, t,
                                               tabs, J.h_src, J.hq[t], sub, lds);
}

// Column phase of a ModDown fused with a rescale: one limb's inverse
// column stages under P (canonical residues, in the last inverse pass's
// layout), and values in that layout through the forward column stages
// under P into tout.
template <int LOGN, class Ar>
__device__ __forceinline__ void inv_cols_to(const u64* __restrict__ tin, const PrimeDev& P,
                                            const typename Ar::TW* __restrict__ W, int sub, u64* lds,
                                            u64 (&out)[Split<LOGN>::SA::E]) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SA;
  const Ar ar(P);
  const int tid = threadIdx.x;
  PassTw<S, Sp::LOGMA, 0, false, Ar> tw;
  tw.load(W, tid, 0);
  typename Ar::T x[S::E];
  {
    constexpr int R = S::bits(0), LO = S::ilo(0), G = S::E >> R;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) x[u * (1 << R) + c] = Ar::unbits(tin[col_g<LOGN>(gidx(gi, c, LO, R), sub)]);
    }
  }
  inv_passes<S, Sp::LOGMA, 0, Ar, true>(x, lds, W, ar, tid, 0, &tw);
#pragma unroll
  for (int i = 0; i < S::E; i++) out[i] = ar.inv_res(x[i], P);
}

template <int LOGN, class Ar>
__device__ __forceinline__ void fwd_cols_from(u64 (&v)[Split<LOGN>::SA::E], const PrimeDev& P,
                                              const typename Ar::TW* __restrict__ W, int sub, u64* lds,
                                              u64* __restrict__ tout) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SA;
  constexpr int E = S::E;
  constexpr int RI = S::bits(S::NP - 1), LOI = S::ilo(S::NP - 1);
  constexpr int RF = S::bits(0), LOF = S::flo(0);
  const Ar ar(P);
  const int tid = threadIdx.x;
  PassTw<S, Sp::LOGMA, 0, true, Ar> tw;
  tw.load(W, tid, 0);
  __syncthreads();  // the inverse passes' last reads of LDS are done
  if constexpr (RI != RF || LOI != LOF) {
    exchange<S, LOI, RI, LOF, RF, IntAr>(v, lds, tid);
    __syncthreads();
  }
  typename Ar::T y[E];
#pragma unroll
  for (int i = 0; i < E; i++) y[i] = ar.from_res(v[i]);
  fwd_passes<S, Sp::LOGMA, 0, Ar, true>(y, lds, W, ar, tid, 0, &tw);
  {
    constexpr int R = S::bits(S::NP - 1), LO = S::flo(S::NP - 1), G = E >> R;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) tout[col_g<LOGN>(gidx(gi, c, LO, R), sub)] = Ar::bits(y[u * (1 << R) + c]);
    }
  }
}

// job w = a * l + t (t < l = Lp - 1): the special limb's and v_l's inverse
// column stages, out_l = (v_l - lift_l(u_p)) p^-1 in coefficient form, and
// lift_t(u_p) p^-1 + lift_t(out_l) through the forward column stages (both
// lifts round: x + h, reduced, minus h)
template <int LOGN>
__global__ void __launch_bounds__(Split<LOGN>::SA::T)
k_ks_moddown_resc_cols(const KsJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  constexpr int N = 1 << LOGN;
  using Sp = Split<LOGN>;
  constexpr int E = Sp::SA::E;
  __shared__ u64 lds[Sp::SA::lds_words()];
  const int l = J.Lp - 1;
  const int w = blockIdx.x / Sp::WA;
  const int sub = blockIdx.x - w * Sp::WA;
  const int a = w / l, t = w - a * l;
  const int sp = J.special;
  const PrimeDev Ps = primes[sp], Pl = primes[l], Pt = primes[t];
  u64 cs[E], cv[E], v[E];
  if (Ps.use_fp)
    inv_cols_to<LOGN, FpAr>(J.t3 + (size_t)a * N, Ps, reinterpret_cast<const double2*>(tabs.inv_fp) + (size_t)sp * N,
                            sub, lds, cs);
  else
    inv_cols_to<LOGN, IntAr>(J.t3 + (size_t)a * N, Ps,
                             reinterpret_cast<const ulonglong2*>(tabs.inv) + (size_t)sp * N, sub, lds, cs);
  __syncthreads();  // the first transform's last LDS reads are done
  if (Pl.use_fp)
    inv_cols_to<LOGN, FpAr>(J.t3b + (size_t)a * N, Pl, reinterpret_cast<const double2*>(tabs.inv_fp) + (size_t)l * N,
                            sub, lds, cv);
  else
    inv_cols_to<LOGN, IntAr>(J.t3b + (size_t)a * N, Pl,
                             reinterpret_cast<const ulonglong2*>(tabs.inv) + (size_t)l * N, sub, lds, cv);
  const u64 qs = Ps.q, ql = Pl.q, qt = Pt.q;
#pragma unroll
  for (int i = 0; i < E; i++) {
    u64 r = cs[i] + J.h_src;
    r = r >= qs ? r - qs : r;
    const u64 sl = submod(red64(r, Pl), J.hq[l], ql);
    const u64 st = submod(red64(r, Pt), J.hq[t], qt);
    u64 o = shoup(submod(cv[i], sl, ql), J.inv[l], J.inv_sh[l], ql);
    o += J.h_l;
    o = o >= ql ? o - ql : o;
    const u64 rt = submod(red64(o, Pt), J.hq2[t], qt);
    v[i] = addmod(shoup(st, J.inv[t], J.inv_sh[t], qt), rt, qt);
  }
  u64* __restrict__ tout = J.t4 + (size_t)w * N;
  if (Pt.use_fp)
    fwd_cols_from<LOGN, FpAr>(v, Pt, reinterpret_cast<const double2*>(tabs.fwd_fp) + (size_t)t * N, sub, lds, tout);
  else
    fwd_cols_from<LOGN, IntAr>(v, Pt, reinterpret_cast<const ulonglong2*>(tabs.fwd) + (size_t)t * N, sub, lds, tout);
}

// digits of the key-switch inner product whose loads are in flight together
#ifndef HE_KS_UNROLL
#define HE_KS_UNROLL 2
#endif
constexpr int kKsUnroll = HE_KS_UNROLL;
// inner products of item b's digits with its key at modulus t for poly k, at
// the E limb indices idx[] (Montgomery form keys: a lazy 128-bit sum of at
// most 8 products, one reduction per group).  The E elements advance
// together so that each digit issues 2E independent loads.
template <int E>
__device__ __forceinline__ void ks_inner(const KsJob& J, const PrimeDev& P, int log_n, int b, int k, int t, int kt,
                                         const int (&idx)[E], bool diag, u64 (&r)[E]) {
  const size_t n = (size_t)1 << log_n;
  const int km = J.km[b];
  const u64* __restrict__ ext = J.ext + ((size_t)b * J.Lp * J.nm + t) * n;
  const u64* __restrict__ kp = J.key[b] + ((size_t)k * km + kt) * n;
  const size_t ks_j = 2 * (size_t)km * n, es_j = (size_t)J.nm * n;
  const u64 g = J.gal[b];
  u64 dv[E];
#pragma unroll
  for (int e = 0; e < E; e++) {
    dv[e] = diag ? J.d[b * J.ds + (size_t)t * n + (g != 1 ? gal_src(idx[e], log_n, g) : idx[e])] : 0;
    r[e] = 0;
  }
  for (int j0 = 0; j0 < J.Lp; j0 += 8) {
    U128 acc[E];
#pragma unroll
    for (int e = 0; e < E; e++) acc[e] = U128{0, 0};
    const int j1 = min(J.Lp, j0 + 8);
    // unrolled so that the key loads of several digits are in flight at once
#pragma unroll kKsUnroll
    for (int j = j0; j < j1; j++) {
      u64 dj[E], kj[E];
#pragma unroll
      for (int e = 0; e < E; e++) {
        dj[e] = (diag && j == t) ? dv[e] : ext[j * es_j + idx[e]];
        kj[e] = kp[j * ks_j + idx[e]];
      }
#pragma unroll
      for (int e = 0; e < E; e++) acc[e] = add128(acc[e], mul_wide(dj[e], kj[e]));
    }
#pragma unroll
    for (int e = 0; e < E; e++) r[e] = addmod(r[e], mont_reduce(acc[e], P), P.q);
  }
}

// ModDown, special modulus: inner product and inverse block phase -> t3
template <int LOGN, class Ar>
__device__ __forceinline__ void special_blocks_body(const KsJob& J, const typename Ar::TW* __restrict__ W,
                                                    const PrimeDev& P, int a, int sub, u64* lds) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SB;
  constexpr int E = S::E;
  const Ar ar(P);
  const int tid = threadIdx.x;
  const int toff = sub << Sp::LOGMB;
  const int b = a >> 1, k = a & 1;
  PassTw<S, LOGN, 0, false, Ar> tw0;
  tw0.load(W, tid, toff);
  typename Ar::T x[E];
  {
    constexpr int R = S::bits(0), G = E >> R;
    int idx[E];
    u64 v[E];
#pragma unroll
    for (int u = 0; u < G; u++)
#pragma unroll
      for (int c = 0; c < (1 << R); c++) idx[u * (1 << R) + c] = toff + (((tid + S::T * u) << R) | c);
    ks_inner<E>(J, P, LOGN, b, k, J.Lp, J.km[b] - 1, idx, false, v);
#pragma unroll
    for (int i = 0; i < E; i++) x[i] = ar.from_res(v[i]);
  }
  inv_passes<S, LOGN, 0, Ar, true>(x, lds, W, ar, tid, toff, &tw0);
  {
    constexpr int R = S::bits(S::NP - 1), LO = S::ilo(S::NP - 1), G = E >> R;
    u64* __restrict__ t = J.t3 + ((size_t)a << LOGN) + toff;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) t[gidx(gi, c, LO, R)] = Ar::bits(x[u * (1 << R) + c]);
    }
  }
}

// ModDown fused with a rescale: the dropped limb l of poly a = 2b + k,
// v_l = u_l + p * (addends), and its inverse block phase -> t3b
template <int LOGN, class Ar>
__device__ __forceinline__ void resc_top_body(const KsJob& J, const typename Ar::TW* __restrict__ W,
                                              const PrimeDev& P, int a, int t, int sub, u64* lds) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SB;
  constexpr int E = S::E;
  constexpr size_t N = (size_t)1 << LOGN;
  const Ar ar(P);
  const int tid = threadIdx.x;
  const int toff = sub << Sp::LOGMB;
  const int b = a >> 1;
  const u64 q = P.q;
  PassTw<S, LOGN, 0, false, Ar> tw0;
  tw0.load(W, tid, toff);
  typename Ar::T x[E];
  {
    constexpr int R = S::bits(0), G = E >> R;
    int idx[E];
    u64 v[E];
#pragma unroll
    for (int u = 0; u < G; u++)
#pragma unroll
      for (int c = 0; c < (1 << R); c++) idx[u * (1 << R) + c] = toff + (((tid + S::T * u) << R) | c);
    ks_inner<E>(J, P, LOGN, b, a & 1, t, t, idx, true, v);
    const u64* __restrict__ ad =
        (J.add && !(J.add_even_only && (a & 1))) ? J.add + a * J.aa + (size_t)t * N : nullptr;
    const u64* __restrict__ ad2 = J.add2 ? J.add2 + a * J.a2a + (size_t)t * N : nullptr;
    const u64 ag = J.add_gather ? J.gal[b] : 1;
#pragma unroll
    for (int e = 0; e < E; e++) {
      u64 sum = ad ? ad[ag != 1 ? gal_src(idx[e], LOGN, ag) : idx[e]] : 0;
      if (ad2) sum = addmod(sum, ad2[idx[e]], q);
      x[e] = ar.from_res(addmod(v[e], shoup(sum, J.pl, J.pl_sh, q), q));
    }
  }
  inv_passes<S, LOGN, 0, Ar, true>(x, lds, W, ar, tid, toff, &tw0);
  {
    constexpr int R = S::bits(S::NP - 1), LO = S::ilo(S::NP - 1), G = E >> R;
    u64* __restrict__ tt = J.t3b + ((size_t)a << LOGN) + toff;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) tt[gidx(gi, c, LO, R)] = Ar::bits(x[u * (1 << R) + c]);
    }
  }
}

template <int LOGN>
__global__ void __launch_bounds__(Split<LOGN>::SB::T)
k_ks_special_blocks(const KsJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  constexpr int N = 1 << LOGN;
  using Sp = Split<LOGN>;
  using S = typename Sp::SB;
  __shared__ u64 lds[S::lds_words()];
  const int n_special = 2 * J.B * Sp::WB;
  if ((int)blockIdx.x >= n_special) {
    // the data-limb inner products of poly a = 2b + k, limb t, on one
    // block of 2^LOGMB words: no transform, so they run beside the special
    // limb's workgroups instead of in the ModDown blocks kernel
    const int w = (blockIdx.x - n_special) / Sp::WB;
    const int sub = blockIdx.x - n_special - w * Sp::WB;
    const int a = w / J.Lp, t = w - a * J.Lp;
    if (J.resc && t == J.Lp - 1) {
      const PrimeDev P = primes[t];
      if (P.use_fp)
        resc_top_body<LOGN, FpAr>(J, reinterpret_cast<const double2*>(tabs.inv_fp) + (size_t)t * N, P, a, t, sub,
                                  lds);
      else
        resc_top_body<LOGN, IntAr>(J, reinterpret_cast<const ulonglong2*>(tabs.inv) + (size_t)t * N, P, a, t, sub,
                                   lds);
      return;
    }
    const int toff = sub << Sp::LOGMB;
    int idx[S::E];
    u64 v[S::E];
#pragma unroll
    for (int e = 0; e < S::E; e++) idx[e] = toff + threadIdx.x + S::T * e;
    ks_inner<S::E>(J, primes[t], LOGN, a >> 1, a & 1, t, t, idx, true, v);
    u64* __restrict__ dst = J.t5 + ((size_t)w << LOGN);
#pragma unroll
    for (int e = 0; e < S::E; e++) dst[idx[e]] = v[e];
    return;
  }
  const int a = blockIdx.x / Sp::WB;
  const int sub = blockIdx.x - a * Sp::WB;
  const PrimeDev P = primes[J.special];
  if (P.use_fp)
    special_blocks_body<LOGN, FpAr>(J, reinterpret_cast<const double2*>(tabs.inv_fp) + (size_t)J.special * N, P, a,
                                    sub, lds);
  else
    special_blocks_body<LOGN, IntAr>(J, reinterpret_cast<const ulonglong2*>(tabs.inv) + (size_t)J.special * N, P,
                                     a, sub, lds);
}

// ModDown, data limb t of poly a = 2b + k: forward block phase of the lifted
// divisor, then (inner product - NTT(r - h)) * p^-1 + addends -> out
template <int LOGN, class Ar, bool RESC>
__device__ __forceinline__ void moddown_blocks_body(const KsJob& J, const typename Ar::TW* __restrict__ W,
                                                    const PrimeDev& P, int w, int a, int t, int sub, u64* lds) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SB;
  constexpr int E = S::E;
  const Ar ar(P);
  const int tid = threadIdx.x;
  const int toff = sub << Sp::LOGMB;
  const int b = a >> 1;
  const u64 q = P.q;
  PassTw<S, LOGN, 0, true, Ar> tw0;
  tw0.load(W, tid, toff);
  const u64* __restrict__ tin = J.t4 + ((size_t)w << LOGN) + toff;
  typename Ar::T x[E];
  {
    constexpr int R = S::bits(0), LO = S::flo(0), G = E >> R;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) x[u * (1 << R) + c] = Ar::unbits(tin[gidx(gi, c, LO, R)]);
    }
  }
  // the data-limb inner products at this thread's output indices (computed
  // by the special-limb launch), loaded before the transform
  constexpr int RL = S::bits(S::NP - 1), GL = E >> RL;
  u64 uu[E];
  const u64* __restrict__ tu = J.t5 + ((size_t)(RESC ? a * J.Lp + t : w) << LOGN);
#pragma unroll
  for (int u = 0; u < GL; u++)
#pragma unroll
    for (int c = 0; c < (1 << RL); c++) uu[u * (1 << RL) + c] = tu[toff + (((tid + S::T * u) << RL) | c)];
  fwd_passes<S, LOGN, 0, Ar, true>(x, lds, W, ar, tid, toff, &tw0);
  {
    constexpr int R = S::bits(S::NP - 1), G = E >> R;
    u64* __restrict__ dst = J.out + a * J.oa + ((size_t)t << LOGN);
    const u64* __restrict__ ad =
        (J.add && !(J.add_even_only && (a & 1))) ? J.add + a * J.aa + ((size_t)t << LOGN) : nullptr;
    const u64* __restrict__ ad2 = J.add2 ? J.add2 + a * J.a2a + ((size_t)t << LOGN) : nullptr;
    const u64 ag = J.add_gather ? J.gal[b] : 1;
    const u64 inv = J.inv[t], inv_sh = J.inv_sh[t];
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) {
        const int idx = toff + ((gi << R) | c);
        const int e = u * (1 << R) + c;
        u64 v;
        if constexpr (RESC) {
          // ((u_t p^-1 + addends) - NTT(lift_t(u_p) p^-1 + lift_t(out_l))) q_l^-1
          v = shoup(uu[e], inv, inv_sh, q);
          if (ad) v = addmod(v, ad[ag != 1 ? gal_src(idx, LOGN, ag) : idx], q);
          if (ad2) v = addmod(v, ad2[idx], q);
          v = shoup(submod(v, ar.fwd_res(x[e]), q), J.inv2[t], J.inv2_sh[t], q);
        } else {
          v = shoup(submod(uu[e], ar.fwd_res(x[e]), q), inv, inv_sh, q);
          if (ad) v = addmod(v, ad[ag != 1 ? gal_src(idx, LOGN, ag) : idx], q);
          if (ad2) v = addmod(v, ad2[idx], q);
        }
        dst[idx] = v;
      }
    }
  }
}

// RESC: the ModDown fused with a rescale (l = Lp - 1 limbs out per poly,
// job w = a * l + t)
template <int LOGN, bool RESC>
__global__ void __launch_bounds__(Split<LOGN>::SB::T)
k_ks_moddown_blocks(const KsJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[Split<LOGN>::SB::lds_words()];
  const int w = blockIdx.x / Split<LOGN>::WB;
  const int sub = blockIdx.x - w * Split<LOGN>::WB;
  const int lo = RESC ? J.Lp - 1 : J.Lp;
  const int a = w / lo, t = w - a * lo;
  const PrimeDev P = primes[t];
  if (P.use_fp)
    moddown_blocks_body<LOGN, FpAr, RESC>(J, reinterpret_cast<const double2*>(tabs.fwd_fp) + (size_t)t * N, P, w, a,
                                          t, sub, lds);
  else
    moddown_blocks_body<LOGN, IntAr, RESC>(J, reinterpret_cast<const ulonglong2*>(tabs.fwd) + (size_t)t * N, P, w,
                                           a, t, sub, lds);
}

// ---------------- rotations of coefficient-form ciphertexts ----------------
// A rotate-and-sum chain keeps its ciphertext in coefficient form between
// steps: the automorphism X -> X^g is then a signed permutation of
// coefficients, the digits need no inverse transform, and the ModDown's
// inverse transforms leave the result in coefficient form.  Four launches
// per step instead of six; the residues are those of the transform-domain
// path (every map is exact), so results are bit-identical.

// coefficient m of a(X^g): +-a[i], i = m g^-1 mod 2N (negated when i >= N)
__device__ __forceinline__ int cauto_src(int m, int log_n, u64 ginv, bool& neg) {
  const u32 i = ((u32)m * (u32)ginv) & ((2u << log_n) - 1u);
  neg = (i >> log_n) != 0;
  return (int)(i & ((1u << log_n) - 1u));
}

// ModUp, job w = (b Lp + j) nm + t: digit j (poly 1, limb j, read at the
// automorphism's source) lifted (centred) to modulus t (t = Lp: the special
// prime; t = j: the digit itself) through the forward column stages -> t2
template <int LOGN, class Ar>
__device__ __forceinline__ void cks_modup_body(const KsJob& J, const typename Ar::TW* __restrict__ W,
                                               const PrimeDev& P, const PrimeDev& Pj, int w, int b, int j, int sub,
                                               u64* lds) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SA;
  constexpr size_t N = (size_t)1 << LOGN;
  const Ar ar(P);
  const int tid = threadIdx.x;
  const u64 q = P.q, qj = Pj.q, hj = (qj - 1) >> 1;
  const u64 ginv = J.ginv[b];
  const u64* __restrict__ src = J.cin + ((size_t)(2 * b + 1) * J.Lp + j) * N;
  typename Ar::T x[S::E];
  PassTw<S, Sp::LOGMA, 0, true, Ar> tw0;
  tw0.load(W, tid, 0);
  {
    constexpr int R = S::bits(0), LO = S::flo(0), G = S::E >> R;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) {
        const int m = col_g<LOGN>(gidx(gi, c, LO, R), sub);
        bool neg = false;
        const int si = ginv != 1 ? cauto_src(m, LOGN, ginv, neg) : m;
        u64 v = src[si];
        if (neg) v = v ? qj - v : 0;
        if (v > hj) {
          const u64 r = red64(qj - v, P);
          v = r ? q - r : 0;
        } else {
          v = red64(v, P);
        }
        x[u * (1 << R) + c] = ar.from_res(v);
      }
    }
  }
  fwd_passes<S, Sp::LOGMA, 0, Ar, true>(x, lds, W, ar, tid, 0, &tw0);
  {
    constexpr int R = S::bits(S::NP - 1), LO = S::flo(S::NP - 1), G = S::E >> R;
    u64* __restrict__ t = J.t2 + (size_t)w * N;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) t[col_g<LOGN>(gidx(gi, c, LO, R), sub)] = Ar::bits(x[u * (1 << R) + c]);
    }
  }
}

template <int LOGN>
__global__ void __launch_bounds__(Split<LOGN>::SA::T)
k_cks_modup_cols(const KsJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[Split<LOGN>::SA::lds_words()];
  const int w = blockIdx.x / Split<LOGN>::WA;
  const int sub = blockIdx.x - w * Split<LOGN>::WA;
  const int a = w / J.nm, t = w - a * J.nm;
  const int b = a / J.Lp, j = a - b * J.Lp;
  const int pt = t < J.Lp ? t : J.special;
  const PrimeDev P = primes[pt], Pj = primes[j];
  if (P.use_fp)
    cks_modup_body<LOGN, FpAr>(J, reinterpret_cast<const double2*>(tabs.fwd_fp) + (size_t)pt * N, P, Pj, w, b, j,
                               sub, lds);
  else
    cks_modup_body<LOGN, IntAr>(J, reinterpret_cast<const ulonglong2*>(tabs.fwd) + (size_t)pt * N, P, Pj, w, b, j,
                                sub, lds);
}

// inner product of poly a = 2b + k at modulus t (every modulus, the special
// one at t = Lp) on block sub, and its inverse block stages -> t3[a nm + t]
template <int LOGN, class Ar>
__device__ __forceinline__ void cks_inner_body(const KsJob& J, const typename Ar::TW* __restrict__ W,
                                               const PrimeDev& P, int a, int t, int kt, int sub, u64* lds) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SB;
  constexpr int E = S::E;
  const Ar ar(P);
  const int tid = threadIdx.x;
  const int toff = sub << Sp::LOGMB;
  PassTw<S, LOGN, 0, false, Ar> tw0;
  tw0.load(W, tid, toff);
  typename Ar::T x[E];
  {
    constexpr int R = S::bits(0), G = E >> R;
    int idx[E];
    u64 v[E];
#pragma unroll
    for (int u = 0; u < G; u++)
#pragma unroll
      for (int c = 0; c < (1 << R); c++) idx[u * (1 << R) + c] = toff + (((tid + S::T * u) << R) | c);
    ks_inner<E>(J, P, LOGN, a >> 1, a & 1, t, kt, idx, false, v);
#pragma unroll
    for (int i = 0; i < E; i++) x[i] = ar.from_res(v[i]);
  }
  inv_passes<S, LOGN, 0, Ar, true>(x, lds, W, ar, tid, toff, &tw0);
  {
    constexpr int R = S::bits(S::NP - 1), LO = S::ilo(S::NP - 1), G = E >> R;
    u64* __restrict__ tt = J.t3 + ((size_t)(a * J.nm + t) << LOGN) + toff;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) tt[gidx(gi, c, LO, R)] = Ar::bits(x[u * (1 << R) + c]);
    }
  }
}

template <int LOGN>
__global__ void __launch_bounds__(Split<LOGN>::SB::T)
k_cks_inner_blocks(const KsJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[Split<LOGN>::SB::lds_words()];
  const int w = blockIdx.x / Split<LOGN>::WB;
  const int sub = blockIdx.x - w * Split<LOGN>::WB;
  const int a = w / J.nm, t = w - a * J.nm;
  const bool sp = t >= J.Lp;
  const int pt = sp ? J.special : t;
  const int kt = sp ? J.km[a >> 1] - 1 : t;
  const PrimeDev P = primes[pt];
  if (P.use_fp)
    cks_inner_body<LOGN, FpAr>(J, reinterpret_cast<const double2*>(tabs.inv_fp) + (size_t)pt * N, P, a, t, kt, sub,
                               lds);
  else
    cks_inner_body<LOGN, IntAr>(J, reinterpret_cast<const ulonglong2*>(tabs.inv) + (size_t)pt * N, P, a, t, kt,
                                sub, lds);
}

// ModDown, job w = a Lp + t: the inverse column stages of the special limb
// and of limb t, (u_t - lift_t(u_p)) p^-1 plus the addends (poly 0 of the
// input at the automorphism's source; the input itself with add2) -> out.
// TAG names the launch family: 0 a rotation, 1 a rescale into coefficient
// form (the dropped limb in the special limb's place, no addends)
template <int LOGN, int TAG>
__global__ void __launch_bounds__(Split<LOGN>::SA::T)
k_cks_moddown_cols(const KsJob J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  constexpr int N = 1 << LOGN;
  using Sp = Split<LOGN>;
  using S = typename Sp::SA;
  constexpr int E = S::E;
  __shared__ u64 lds[S::lds_words()];
  const int w = blockIdx.x / Sp::WA;
  const int sub = blockIdx.x - w * Sp::WA;
  const int a = w / J.Lp, t = w - a * J.Lp;
  const int b = a >> 1;
  const int sp = J.special;
  const PrimeDev Ps = primes[sp], Pt = primes[t];
  u64 cs[E], ct[E];
  if (Ps.use_fp)
    inv_cols_to<LOGN, FpAr>(J.t3 + (size_t)(a * J.nm + J.Lp) * N, Ps,
                            reinterpret_cast<const double2*>(tabs.inv_fp) + (size_t)sp * N, sub, lds, cs);
  else
    inv_cols_to<LOGN, IntAr>(J.t3 + (size_t)(a * J.nm + J.Lp) * N, Ps,
                             reinterpret_cast<const ulonglong2*>(tabs.inv) + (size_t)sp * N, sub, lds, cs);
  __syncthreads();  // the first transform's last LDS reads are done
  if (Pt.use_fp)
    inv_cols_to<LOGN, FpAr>(J.t3 + (size_t)(a * J.nm + t) * N, Pt,
                            reinterpret_cast<const double2*>(tabs.inv_fp) + (size_t)t * N, sub, lds, ct);
  else
    inv_cols_to<LOGN, IntAr>(J.t3 + (size_t)(a * J.nm + t) * N, Pt,
                             reinterpret_cast<const ulonglong2*>(tabs.inv) + (size_t)t * N, sub, lds, ct);
  const u64 qs = Ps.q, qt = Pt.q;
  const u64* __restrict__ ad =
      (J.add && !(J.add_even_only && (a & 1))) ? J.add + a * J.aa + (size_t)t * N : nullptr;
  const u64* __restrict__ ad2 = J.add2 ? J.add2 + a * J.a2a + (size_t)t * N : nullptr;
  const u64 ginv = J.add_gather ? J.ginv[b] : 1;
  u64* __restrict__ dst = J.out + a * J.oa + (size_t)t * N;
  constexpr int R = S::bits(S::NP - 1), LO = S::ilo(S::NP - 1), G = E >> R;
#pragma unroll
  for (int u = 0; u < G; u++) {
    const int gi = threadIdx.x + S::T * u;
#pragma unroll
    for (int c = 0; c < (1 << R); c++) {
      const int e = u * (1 << R) + c;
      const int m = col_g<LOGN>(gidx(gi, c, LO, R), sub);
      u64 r = cs[e] + J.h_src;
      r = r >= qs ? r - qs : r;
      const u64 st = submod(red64(r, Pt), J.hq[t], qt);
      u64 o = shoup(submod(ct[e], st, qt), J.inv[t], J.inv_sh[t], qt);
      if (ad) {
        bool neg = false;
        const int si = ginv != 1 ? cauto_src(m, LOGN, ginv, neg) : m;
        u64 v = ad[si];
        if (neg) v = v ? qt - v : 0;
        o = addmod(o, v, qt);
      }
      if (ad2) o = addmod(o, ad2[m], qt);
      dst[m] = o;
    }
  }
}

// ---------------- hoisted rotations: ModDown + multiply-accumulate ----------------
// ModDown of each item (an NTT of its special-prime limb, lifted) with the
// plaintext multiply-accumulate of the vector-matrix product in the
// epilogue.  Workgroup (chunk, k, t) loops over its items; each thread
// keeps the running sums of its E output words in registers and writes
// them to its workgroup's slice of `partial` once at the end.
// words per thread of the multiply-accumulate kernel's NTT
#ifndef HE_HOIST_LOGE
#define HE_HOIST_LOGE 0
#endif
constexpr int hoist_loge(int logn) { return HE_HOIST_LOGE > 0 ? HE_HOIST_LOGE : single_loge(logn); }
template <int LOGN>
struct HCfg : Sched<LOGN, 0, LOGN, hoist_loge(LOGN)> {
  static constexpr int N = 1 << LOGN;
};
// LDS of the multiply-accumulate kernel (160 KiB per workgroup at most):
// the NTT exchange buffer, then a copy of the prime's first TWN twiddles
// (16 bytes each), TWN the largest power of two up to N/2 that fits: the
// stages lb >= TWLB read their twiddles there.
template <int LOGN>
struct HoistLds {
  static constexpr int BUDGET = 160 * 1024 / 8;
  static constexpr int EXW = HCfg<LOGN>::lds_words();
  static constexpr int twn() {
    int n = 1 << (LOGN - 1);
    while (n > 1 && EXW + 2 * n > BUDGET) n >>= 1;
    return EXW + 2 * n <= BUDGET ? n : 0;
  }
  static constexpr int TWN = twn();
  static constexpr int log2i(int v) { return v <= 1 ? 0 : 1 + log2i(v >> 1); }
  static constexpr int TWLB = TWN >= 2 ? LOGN - log2i(TWN) : 99;
  static constexpr int WORDS = EXW + 2 * TWN;
};
template <int LOGN>
constexpr int hoist_lds_words() {
  return HoistLds<LOGN>::WORDS;
}

template <int LOGN, bool DIAG, class Ar>
__device__ __forceinline__ void hoist_body(const HoistMac& J, const PrimeDev* __restrict__ primes,
                                           const typename Ar::TW* __restrict__ W, const PrimeDev& P, int chunk,
                                           int k, int t, u64* lds) {
  using C = HCfg<LOGN>;
  constexpr int N = C::N;
  constexpr int R0 = C::bits(0), LO0 = LOGN - R0, G0 = C::E >> R0;
  constexpr int RF = C::bits(C::NP - 1), GF = C::E >> RF;
  const Ar ar(P);
  const int tid = threadIdx.x;
  const u64 q = P.q;
  const u64 sq = primes[J.special_prime].q, sh = J.h_src;
  const u64 hq = J.hq[t], inv = J.inv[t], inv_sh = J.inv_sh[t];
  u64* __restrict__ out = J.partial + (((size_t)chunk * 2 + k) * J.n_dig + t) * N;
  const int rb = chunk * J.chunk, re = min(J.R, rb + J.chunk);
  u64 acc[C::E];
#pragma unroll
  for (int e = 0; e < C::E; e++) acc[e] = 0;
  // this workgroup's prime is fixed: its first TWN twiddles are copied to
  // LDS once and read from there for all items
  using Lay = HoistLds<LOGN>;
  typename Ar::TW* Wl = reinterpret_cast<typename Ar::TW*>(lds + Lay::EXW);
  if constexpr (Lay::TWN > 0) {
    for (int i = tid; i < Lay::TWN; i += C::T) Wl[i] = W[i];
    __syncthreads();
  }
  for (int r = rb; r < re; r++) {
    const HoistItem it = J.items[r];
    const u64* __restrict__ src = J.ucoef + ((size_t)r * 2 + k) * N;
    typename Ar::T x[C::E];
#pragma unroll
    for (int u = 0; u < G0; u++) {
      const int gi = tid + C::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R0); c++) {
        u64 v = src[(c << LO0) | gi] + sh;
        v = v >= sq ? v - sq : v;
        x[u * (1 << R0) + c] = ar.from_res(submod(red64(v, P), hq, q));
      }
    }
    // keep the twiddle loads inside the loop (hoisting them out would hold
    // every stage's twiddles in registers across items)
    const typename Ar::TW* Wr = W;
    asm volatile("" : "+v"(Wr));
    fwd_passes<C, LOGN, 0, Ar, false, Lay::TWLB>(x, lds, Wr, ar, tid, 0, nullptr, Wl);
    // final values through LDS so the epilogue runs in natural order:
    // coalesced accesses and a bounded number of loads in flight
    __syncthreads();
#pragma unroll
    for (int u = 0; u < GF; u++) {
      const int gi = tid + C::T * u;
#pragma unroll
      for (int c = 0; c < (1 << RF); c++) lds[pad((gi << RF) | c)] = ar.fwd_res(x[u * (1 << RF) + c]);
    }
    __syncthreads();
    const u64* __restrict__ uw = J.u + (((size_t)r * 2 + k) * J.nm + t) * N;
    if constexpr (DIAG) {
      // Barrett product with the diagonal: no precomputed companion, so
      // one diagonal word per output word is read
      const u64* __restrict__ dg = J.diags + ((size_t)it.diag * J.n_dig + t) * N;
#pragma unroll
      for (int e = 0; e < C::E; e++) {
        const int idx = tid + C::T * e;
        const u64 v = lds[pad(idx)];
        const u64 ks = shoup(submod(uw[idx], v, q), inv, inv_sh, q);
        acc[e] = addmod(acc[e], mulmod(ks, dg[idx], P), q);
      }
    } else {
      // a replication: the rotations are only summed
#pragma unroll
      for (int e = 0; e < C::E; e++) {
        const int idx = tid + C::T * e;
        const u64 v = lds[pad(idx)];
        acc[e] = addmod(acc[e], shoup(submod(uw[idx], v, q), inv, inv_sh, q), q);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int e = 0; e < C::E; e++) out[tid + C::T * e] = acc[e];
}

// one workgroup per compute unit: the registers hold the running sums
// (two workgroups would spill them)
template <int LOGN, bool DIAG>
__global__ void __launch_bounds__(HCfg<LOGN>::T, HCfg<LOGN>::T / 256)
k_hoist_mac(const HoistMac J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  constexpr int N = HCfg<LOGN>::N;
  extern __shared__ u64 lds[];
  // block b runs on XCD b % 8: blocks b and b + 8 (same XCD, consecutive
  // there) are the two polys of one (chunk, t) unit
  const int b = blockIdx.x;
  const int slot = b >> 3;
  const int k = slot & 1;
  const int unit = ((slot >> 1) << 3) | (b & 7);
  if (unit >= J.n_units) return;
  const int chunk = unit / J.n_dig, t = unit - chunk * J.n_dig;
  const PrimeDev P = primes[t];
  if (P.use_fp)
    hoist_body<LOGN, DIAG, FpAr>(J, primes, reinterpret_cast<const double2*>(tabs.fwd_fp) + (size_t)t * N, P,
                                 chunk, k, t, lds);
  else
    hoist_body<LOGN, DIAG, IntAr>(J, primes, reinterpret_cast<const ulonglong2*>(tabs.fwd) + (size_t)t * N, P,
                                  chunk, k, t, lds);
}

// ---------------- hoisted multiply-accumulate, two-phase form ----------------
// u[r][k][t] at the words idx[] (the hoisted inner product, computed where
// it is consumed): sum_j D_{j,t}[src_r(i)] * key_r[j][k][t][i], with D_{j,t}
// the shared ModUp digit (the input's c1 itself for j = t), plus
// p * c0[t][src_r(i)] for poly 0 of a data limb.  t = n_dig is the special
// prime's slot.  Key words pass once (non-temporal); the digits stay in L2.
template <int LOGN, int E, int UNROLL = 1>
__device__ __forceinline__ void hoist_inner_at(const HoistMac& J, const HoistItem& it, const PrimeDev& P, int k,
                                               int t, const int (&idx)[E], u64 (&r)[E]) {
  constexpr size_t N = (size_t)1 << LOGN;
  const bool special = t >= J.n_dig;
  const int kt = special ? it.km - 1 : t;
  const u64* __restrict__ kp = it.key + ((size_t)k * it.km + kt) * N;
  const size_t ks_j = 2 * (size_t)it.km * N;
  int src[E];
#pragma unroll
  for (int e = 0; e < E; e++) {
    src[e] = gal_src(idx[e], LOGN, it.g);
    r[e] = 0;
  }
  for (int j0 = 0; j0 < J.n_dig; j0 += 8) {
    U128 acc[E];
#pragma unroll
    for (int e = 0; e < E; e++) acc[e] = U128{0, 0};
    const int j1 = min(J.n_dig, j0 + 8);
#pragma unroll UNROLL
    for (int j = j0; j < j1; j++) {
      const u64* __restrict__ dj = (j == t) ? J.c1 + (size_t)t * N : J.ext + ((size_t)j * J.nm + t) * N;
      u64 d[E], kv[E];
#pragma unroll
      for (int e = 0; e < E; e++) {
        d[e] = dj[src[e]];
        kv[e] = __builtin_nontemporal_load(kp + j * ks_j + idx[e]);
      }
#pragma unroll
      for (int e = 0; e < E; e++) acc[e] = add128(acc[e], mul_wide(d[e], kv[e]));
    }
#pragma unroll
    for (int e = 0; e < E; e++) r[e] = addmod(r[e], mont_reduce(acc[e], P), P.q);
  }
  if (!special && k == 0) {
    const u64* __restrict__ c0 = J.c0 + (size_t)t * N;
#pragma unroll
    for (int e = 0; e < E; e++) r[e] = addmod(r[e], shoup(c0[src[e]], J.pq[t], J.pq_sh[t], P.q), P.q);
  }
}

// Special-prime limb of item a / 2, poly a % 2: its inner product on block
// sub and the inverse transform's block stages, into ucoef (the column
// phase below finishes the transform).
template <int LOGN, class Ar>
__device__ __forceinline__ void hoist_special_body(const HoistMac& J, const typename Ar::TW* __restrict__ W,
                                                   const PrimeDev& P, int a, int sub, u64* lds) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SB;
  constexpr int E = S::E;
  const Ar ar(P);
  const int tid = threadIdx.x;
  const int toff = sub << Sp::LOGMB;
  PassTw<S, LOGN, 0, false, Ar> tw0;
  tw0.load(W, tid, toff);
  typename Ar::T x[E];
  {
    constexpr int R = S::bits(0), G = E >> R;
    int idx[E];
    u64 v[E];
#pragma unroll
    for (int u = 0; u < G; u++)
#pragma unroll
      for (int c = 0; c < (1 << R); c++) idx[u * (1 << R) + c] = toff + (((tid + S::T * u) << R) | c);
    hoist_inner_at<LOGN, E, 2>(J, J.items[a >> 1], P, a & 1, J.n_dig, idx, v);
#pragma unroll
    for (int i = 0; i < E; i++) x[i] = ar.from_res(v[i]);
  }
  inv_passes<S, LOGN, 0, Ar, true>(x, lds, W, ar, tid, toff, &tw0);
  {
    constexpr int R = S::bits(S::NP - 1), LO = S::ilo(S::NP - 1), G = E >> R;
    u64* __restrict__ t = const_cast<u64*>(J.ucoef) + ((size_t)a << LOGN) + toff;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) t[gidx(gi, c, LO, R)] = Ar::bits(x[u * (1 << R) + c]);
    }
  }
}

template <int LOGN>
__global__ void __launch_bounds__(Split<LOGN>::SB::T)
k_hoist_special(const HoistMac J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  constexpr int N = 1 << LOGN;
  using Sp = Split<LOGN>;
  __shared__ u64 lds[Sp::SB::lds_words()];
  const int a = blockIdx.x / Sp::WB;
  const int sub = blockIdx.x - a * Sp::WB;
  const int sp = J.special_prime;
  const PrimeDev P = primes[sp];
  if (P.use_fp)
    hoist_special_body<LOGN, FpAr>(J, reinterpret_cast<const double2*>(tabs.inv_fp) + (size_t)sp * N, P, a, sub,
                                   lds);
  else
    hoist_special_body<LOGN, IntAr>(J, reinterpret_cast<const ulonglong2*>(tabs.inv) + (size_t)sp * N, P, a, sub,
                                    lds);
}

// Column phase, workgroup (a, sub) for item a / 2, poly a % 2 and the 16
// columns of group sub: the inverse transform's column stages finish the
// special-prime limb's coefficients in these columns (its block stages ran
// before, into ucoef), kept in LDS; then for every modulus t the lift and
// the forward transform's column stages, into mid (job a * n_dig + t).
template <int LOGN, class Ar>
__device__ __forceinline__ void hoist_cols_inv(const HoistMac& J, const typename Ar::TW* __restrict__ W,
                                               const PrimeDev& P, int a, int sub, u64* coef, u64* lds) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SA;
  const Ar ar(P);
  const int tid = threadIdx.x;
  const u64* __restrict__ t = J.ucoef + ((size_t)a << LOGN);
  typename Ar::T x[S::E];
  PassTw<S, Sp::LOGMA, 0, false, Ar> tw0;
  tw0.load(W, tid, 0);
  {
    constexpr int R = S::bits(0), LO = S::ilo(0), G = S::E >> R;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) x[u * (1 << R) + c] = Ar::unbits(t[col_g<LOGN>(gidx(gi, c, LO, R), sub)]);
    }
  }
  inv_passes<S, Sp::LOGMA, 0, Ar, true>(x, lds, W, ar, tid, 0, &tw0);
  {
    constexpr int R = S::bits(S::NP - 1), LO = S::ilo(S::NP - 1), G = S::E >> R;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) coef[gidx(gi, c, LO, R)] = ar.inv_res(x[u * (1 << R) + c], P);
    }
  }
}

template <int LOGN, class Ar>
__device__ __forceinline__ void hoist_cols_fwd(const HoistMac& J, const typename Ar::TW* __restrict__ W,
                                               const PrimeDev& P, int a, int t, int sub, u64 sq, const u64* coef,
                                               u64* lds) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SA;
  const Ar ar(P);
  const int tid = threadIdx.x;
  const u64 q = P.q, sh = J.h_src, hq = J.hq[t];
  typename Ar::T x[S::E];
  PassTw<S, Sp::LOGMA, 0, true, Ar> tw0;
  tw0.load(W, tid, 0);
  {
    constexpr int R = S::bits(0), LO = S::flo(0), G = S::E >> R;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) {
        u64 v = coef[gidx(gi, c, LO, R)] + sh;
        v = v >= sq ? v - sq : v;
        x[u * (1 << R) + c] = ar.from_res(submod(red64(v, P), hq, q));
      }
    }
  }
  fwd_passes<S, Sp::LOGMA, 0, Ar, true>(x, lds, W, ar, tid, 0, &tw0);
  {
    constexpr int R = S::bits(S::NP - 1), LO = S::flo(S::NP - 1), G = S::E >> R;
    u64* __restrict__ out = J.mid + ((size_t)(a * J.n_dig + t) << LOGN);
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) out[col_g<LOGN>(gidx(gi, c, LO, R), sub)] = Ar::bits(x[u * (1 << R) + c]);
    }
  }
}

template <int LOGN>
__global__ void __launch_bounds__(Split<LOGN>::SA::T)
k_hoist_cols(const HoistMac J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  using Sp = Split<LOGN>;
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[Sp::SA::lds_words()];
  __shared__ u64 coef[Sp::SA::M];
  const int a = blockIdx.x / Sp::WA;
  const int sub = blockIdx.x - a * Sp::WA;
  const int sp = J.special_prime;
  const PrimeDev Ps = primes[sp];
  if (Ps.use_fp)
    hoist_cols_inv<LOGN, FpAr>(J, reinterpret_cast<const double2*>(tabs.inv_fp) + (size_t)sp * N, Ps, a, sub, coef,
                               lds);
  else
    hoist_cols_inv<LOGN, IntAr>(J, reinterpret_cast<const ulonglong2*>(tabs.inv) + (size_t)sp * N, Ps, a, sub, coef,
                                lds);
  for (int t = 0; t < J.n_dig; t++) {
    // the coefficients are complete, and the exchange buffer is free again
    __syncthreads();
    const PrimeDev P = primes[t];
    if (P.use_fp)
      hoist_cols_fwd<LOGN, FpAr>(J, reinterpret_cast<const double2*>(tabs.fwd_fp) + (size_t)t * N, P, a, t, sub,
                                 Ps.q, coef, lds);
    else
      hoist_cols_fwd<LOGN, IntAr>(J, reinterpret_cast<const ulonglong2*>(tabs.fwd) + (size_t)t * N, P, a, t, sub,
                                  Ps.q, coef, lds);
  }
}

// waves per SIMD of the block kernel (four: at most 128 VGPRs), and the
// digits of one item's inner product whose loads are in flight together
#ifndef HE_HOIST_B_WAVES
#define HE_HOIST_B_WAVES 4
#endif
#ifndef HE_HOIST_B_UNROLL
#define HE_HOIST_B_UNROLL 1
#endif
// Block phase: workgroup (chunk, k, t, sub) finishes block sub of every
// item's transform in modulus t, poly k, and keeps the running sums of its
// E words in registers.
template <int LOGN, bool DIAG, class Ar>
__device__ __forceinline__ void hoist_b_body(const HoistMac& J, const typename Ar::TW* __restrict__ W,
                                             const PrimeDev& P, int chunk, int k, int t, int sub, u64* lds) {
  using Sp = Split<LOGN>;
  using S = typename Sp::SB;
  constexpr int N = 1 << LOGN;
  constexpr int R0 = S::bits(0), LO0 = S::flo(0), G0 = S::E >> R0;
  constexpr int RF = S::bits(S::NP - 1), GF = S::E >> RF;
  const Ar ar(P);
  const int tid = threadIdx.x;
  const u64 q = P.q;
  const u64 inv = J.inv[t], inv_sh = J.inv_sh[t];
  const int toff = sub << Sp::LOGMB;
  const int rb = chunk * J.chunk, re = min(J.R, rb + J.chunk);
  u64 acc[S::E];
#pragma unroll
  for (int e = 0; e < S::E; e++) acc[e] = 0;
  // the first pass's twiddles depend on the block only: loaded once
  PassTw<S, LOGN, 0, true, Ar> tw0;
  tw0.load(W, tid, toff);
  // the column-phase output of the next rotation is loaded while the
  // current one is transformed
  u64 nx[S::E];
  if (rb < re) {
    const u64* __restrict__ src = J.mid + (((size_t)rb * 2 + k) * J.n_dig + t) * N + toff;
#pragma unroll
    for (int u = 0; u < G0; u++) {
      const int gi = tid + S::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R0); c++) nx[u * (1 << R0) + c] = src[gidx(gi, c, LO0, R0)];
    }
  }
  for (int r = rb; r < re; r++) {
    const HoistItem it = J.items[r];
    // the thread index, opaque to the compiler inside each iteration: the
    // per-thread addresses are recomputed per item instead of being held
    // in registers across the loop (which spills)
    int tr = tid;
    asm volatile("" : "+v"(tr));
    typename Ar::T x[S::E];
#pragma unroll
    for (int e = 0; e < S::E; e++) x[e] = Ar::unbits(nx[e]);
    // the epilogue's operands: the diagonal words, and this item's inner
    // product at the thread's output words
    const u64* __restrict__ dg = DIAG ? J.diags + ((size_t)it.diag * J.n_dig + t) * N : nullptr;
    int oidx[S::E];
    u64 uv[S::E], dv[S::E];
#pragma unroll
    for (int u = 0; u < GF; u++) {
#pragma unroll
      for (int c = 0; c < (1 << RF); c++) {
        const int e = u * (1 << RF) + c;
        oidx[e] = toff + (((tr + S::T * u) << RF) | c);
        dv[e] = DIAG ? dg[oidx[e]] : 0;
      }
    }
    hoist_inner_at<LOGN, S::E, HE_HOIST_B_UNROLL>(J, it, P, k, t, oidx, uv);
    // the next item's column-phase output, in flight during the transform
    asm volatile("" : "+v"(tr));
    if (r + 1 < re) {
      const u64* __restrict__ src = J.mid + (((size_t)(r + 1) * 2 + k) * J.n_dig + t) * N + toff;
#pragma unroll
      for (int u = 0; u < G0; u++) {
        const int gi = tr + S::T * u;
#pragma unroll
        for (int c = 0; c < (1 << R0); c++) nx[u * (1 << R0) + c] = src[gidx(gi, c, LO0, R0)];
      }
    }
    fwd_passes<S, LOGN, 0, Ar, true>(x, lds, W, ar, tr, toff, &tw0);
#pragma unroll
    for (int e = 0; e < S::E; e++) {
      u64 ks = shoup(submod(uv[e], ar.fwd_res(x[e]), q), inv, inv_sh, q);
      if constexpr (DIAG) ks = mulmod(ks, dv[e], P);
      acc[e] = addmod(acc[e], ks, q);
    }
    // the next item's first exchange reuses the LDS buffer
    __syncthreads();
  }
  u64* __restrict__ out = J.partial + (((size_t)chunk * 2 + k) * J.n_dig + t) * N;
#pragma unroll
  for (int u = 0; u < GF; u++) {
    const int gi = tid + S::T * u;
#pragma unroll
    for (int c = 0; c < (1 << RF); c++) out[toff + ((gi << RF) | c)] = acc[u * (1 << RF) + c];
  }
}

// unit = (chunk * n_dig + t) * WB + sub; block b runs on XCD b % 8, and
// blocks b and b + 8 are the two polys of one unit (the diagonal block is
// read twice from that XCD's L2).
template <int LOGN, bool DIAG>
__global__ void __launch_bounds__(Split<LOGN>::SB::T, HE_HOIST_B_WAVES)
k_hoist_mac_b(const HoistMac J, const PrimeDev* __restrict__ primes, const NttTables tabs) {
  using Sp = Split<LOGN>;
  constexpr int N = 1 << LOGN;
  __shared__ u64 lds[Sp::SB::lds_words()];
  const int b = blockIdx.x;
  const int slot = b >> 3;
  const int k = slot & 1;
  const int unit = ((slot >> 1) << 3) | (b & 7);
  if (unit >= J.n_units) return;
  const int ct = unit / Sp::WB, sub = unit - ct * Sp::WB;
  const int chunk = ct / J.n_dig, t = ct - chunk * J.n_dig;
  const PrimeDev P = primes[t];
  if (P.use_fp)
    hoist_b_body<LOGN, DIAG, FpAr>(J, reinterpret_cast<const double2*>(tabs.fwd_fp) + (size_t)t * N, P, chunk, k,
                                   t, sub, lds);
  else
    hoist_b_body<LOGN, DIAG, IntAr>(J, reinterpret_cast<const ulonglong2*>(tabs.fwd) + (size_t)t * N, P, chunk, k,
                                    t, sub, lds);
}

// ---------------- launchers ----------------
int n_jobs(const NttJob& J) { return J.na * (J.skip_diag ? J.nb - 1 : J.nb); }

template <class K>
hipError_t set_lds(K kernel, size_t shm, bool& done) {
  if (done) return hipSuccess;
  hipError_t e = hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
  if (e == hipSuccess) done = true;
  return e;
}

// two phases when the batch is small (or the tuned table says so for its
// size) and the scratch buffer holds it
bool use_split(const NttJob& J, const NttTables& tabs, int log_n) {
  const int jobs = n_jobs(J);
  if (!tabs.tmp || (long long)jobs << log_n > tabs.tmp_words) return false;
  if (!tabs.tuned) return jobs <= tabs.split_jobs;
  int b = 0;
  while (b + 1 < tabs.n_buckets && jobs > (16 << b)) b++;
  return (tabs.split_mask >> b) & 1;
}

template <int LOGN, int PRO, int EPI>
hipError_t fwd_launch(const NttJob& J, const PrimeDev* primes, const NttTables& tabs, hipStream_t st) {
  using C = Cfg<LOGN>;
  using Sp = Split<LOGN>;
  const int jobs = n_jobs(J);
  if (jobs <= 0) return hipSuccess;
  if (use_split(J, tabs, LOGN)) {
    hipLaunchKernelGGL((k_ntt_fwd_a<LOGN, PRO>), dim3(jobs * Sp::WA), dim3(Sp::SA::T), 0, st, J, primes, tabs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_ntt_fwd_b<LOGN, PRO, EPI>), dim3(jobs * Sp::WB), dim3(Sp::SB::T), 0, st, J, primes, tabs);
    return hipGetLastError();
  }
  if constexpr (PRO == PRO_PLAIN && EPI == EPI_STORE && LOGN >= 12) {
    const int id = tuned_shape(tabs, jobs);
    if (id > 0) return shape_launch<LOGN, true>(id, J, primes, tabs, st, jobs);
  }
  const size_t shm = sizeof(u64) * C::lds_words();
  static bool attr = false;
  hipError_t e = set_lds(k_ntt_fwd<LOGN, PRO, EPI>, shm, attr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_ntt_fwd<LOGN, PRO, EPI>), dim3(jobs), dim3(C::T), shm, st, J, primes, tabs);
  return hipGetLastError();
}

template <int LOGN, bool GATHER>
hipError_t inv_launch(const NttJob& J, const PrimeDev* primes, const NttTables& tabs, hipStream_t st) {
  using C = Cfg<LOGN>;
  using Sp = Split<LOGN>;
  const int jobs = n_jobs(J);
  if (jobs <= 0) return hipSuccess;
  if (use_split(J, tabs, LOGN)) {
    hipLaunchKernelGGL((k_ntt_inv_1<LOGN, GATHER, 0>), dim3(jobs * Sp::WB), dim3(Sp::SB::T), 0, st, J, primes, tabs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_ntt_inv_2<LOGN>), dim3(jobs * Sp::WA), dim3(Sp::SA::T), 0, st, J, primes, tabs);
    return hipGetLastError();
  }
  if constexpr (!GATHER && LOGN >= 12) {
    const int id = tuned_shape(tabs, jobs);
    if (id > 0) return shape_launch<LOGN, false>(id, J, primes, tabs, st, jobs);
  }
  const size_t shm = sizeof(u64) * C::lds_words();
  static bool attr = false;
  hipError_t e = set_lds(k_ntt_inv<LOGN, GATHER>, shm, attr);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_ntt_inv<LOGN, GATHER>), dim3(jobs), dim3(C::T), shm, st, J, primes, tabs);
  return hipGetLastError();
}

template <int LOGN, bool DIAG>
hipError_t hoist_launch_as(const HoistMac& J, const PrimeDev* primes, const NttTables& tabs, hipStream_t st) {
  using C = HCfg<LOGN>;
  const size_t shm = sizeof(u64) * hoist_lds_words<LOGN>();
  static bool attr = false;
  hipError_t e = set_lds(k_hoist_mac<LOGN, DIAG>, shm, attr);
  if (e != hipSuccess) return e;
  const int n_chunks = (J.R + J.chunk - 1) / J.chunk;
  if (n_chunks <= 0 || J.n_units != n_chunks * J.n_dig) return hipErrorInvalidValue;
  // two blocks per unit, units padded to a multiple of 8 (the padding
  // blocks exit at once)
  const int blocks = ((J.n_units + 7) / 8) * 16;
  hipLaunchKernelGGL((k_hoist_mac<LOGN, DIAG>), dim3(blocks), dim3(C::T), shm, st, J, primes, tabs);
  return hipGetLastError();
}

// column phase: the inverse transform's block stages of every (item, poly)
// special-prime limb of u into ucoef, then k_hoist_cols
template <int LOGN>
hipError_t hoist_cols_launch(const HoistMac& J, const PrimeDev* primes, const NttTables& tabs, hipStream_t st) {
  using Sp = Split<LOGN>;
  if (J.R <= 0 || J.n_dig <= 0 || J.n_dig > HE_MAXM || J.nm != J.n_dig + 1 || !J.mid || !J.ucoef || !J.ext ||
      !J.c1 || !J.c0 || !J.items)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_hoist_special<LOGN>), dim3(2 * J.R * Sp::WB), dim3(Sp::SB::T), 0, st, J, primes, tabs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_hoist_cols<LOGN>), dim3(2 * J.R * Sp::WA), dim3(Sp::SA::T), 0, st, J, primes, tabs);
  return hipGetLastError();
}

// block phase with the multiply-accumulate (after the column phase)
template <int LOGN, bool DIAG>
hipError_t hoist_split_launch_as(const HoistMac& J, const PrimeDev* primes, const NttTables& tabs, hipStream_t st) {
  using Sp = Split<LOGN>;
  const int n_chunks = J.chunk > 0 ? (J.R + J.chunk - 1) / J.chunk : 0;
  if (n_chunks <= 0 || J.n_dig <= 0 || J.n_dig > HE_MAXM || !J.mid || !J.ext || !J.c1 || !J.c0 || !J.items)
    return hipErrorInvalidValue;
  HoistMac B = J;
  B.n_units = n_chunks * J.n_dig * Sp::WB;
  const int blocks = ((B.n_units + 7) / 8) * 16;
  hipLaunchKernelGGL((k_hoist_mac_b<LOGN, DIAG>), dim3(blocks), dim3(Sp::SB::T), 0, st, B, primes, tabs);
  return hipGetLastError();
}

// the diagonal product and the plain sum (a replication) are separate
// instantiations: no branch on the diagonal pointer inside the kernel
template <int LOGN>
hipError_t hoist_launch(const HoistMac& J, const PrimeDev* primes, const NttTables& tabs, hipStream_t st) {
  if (J.mid)
    return J.diags ? hoist_split_launch_as<LOGN, true>(J, primes, tabs, st)
                   : hoist_split_launch_as<LOGN, false>(J, primes, tabs, st);
  return J.diags ? hoist_launch_as<LOGN, true>(J, primes, tabs, st)
                 : hoist_launch_as<LOGN, false>(J, primes, tabs, st);
}

template <int LOGN>
hipError_t fwd_dispatch(int pro, int epi, const NttJob& J, const PrimeDev* primes, const NttTables& tabs,
                        hipStream_t st) {
  if (pro == PRO_PLAIN && epi == EPI_STORE) return fwd_launch<LOGN, PRO_PLAIN, EPI_STORE>(J, primes, tabs, st);
  if (pro == PRO_CENTRED_LIFT && epi == EPI_STORE)
    return fwd_launch<LOGN, PRO_CENTRED_LIFT, EPI_STORE>(J, primes, tabs, st);
  if (pro == PRO_ROUNDDIV_LIFT && epi == EPI_ROUNDDIV)
    return fwd_launch<LOGN, PRO_ROUNDDIV_LIFT, EPI_ROUNDDIV>(J, primes, tabs, st);
  return hipErrorInvalidValue;
}

template <int LOGN>
hipError_t inv_dispatch(const NttJob& J, const PrimeDev* primes, const NttTables& tabs, hipStream_t st) {
  return J.gather_src ? inv_launch<LOGN, true>(J, primes, tabs, st) : inv_launch<LOGN, false>(J, primes, tabs, st);
}

template <int LOGN>
hipError_t inv_blocks_launch(const NttJob& J, const PrimeDev* primes, const NttTables& tabs, int tag,
                             hipStream_t st) {
  using Sp = Split<LOGN>;
  const int jobs = n_jobs(J);
  if (jobs <= 0) return hipSuccess;
  const dim3 grid(jobs * Sp::WB), blk(Sp::SB::T);
  if (tag == 2)
    hipLaunchKernelGGL((k_ntt_inv_1<LOGN, false, 2>), grid, blk, 0, st, J, primes, tabs);
  else if (J.gather_src)
    hipLaunchKernelGGL((k_ntt_inv_1<LOGN, true, 1>), grid, blk, 0, st, J, primes, tabs);
  else
    hipLaunchKernelGGL((k_ntt_inv_1<LOGN, false, 1>), grid, blk, 0, st, J, primes, tabs);
  return hipGetLastError();
}

template <int LOGN>
hipError_t fwd_blocks_launch(int pro, int epi, const NttJob& J, const PrimeDev* primes, const NttTables& tabs,
                             hipStream_t st) {
  using Sp = Split<LOGN>;
  const int jobs = n_jobs(J);
  if (jobs <= 0) return hipSuccess;
  const dim3 grid(jobs * Sp::WB), blk(Sp::SB::T);
  if (pro == PRO_PLAIN && epi == EPI_STORE)
    hipLaunchKernelGGL((k_ntt_fwd_b<LOGN, PRO_PLAIN, EPI_STORE>), grid, blk, 0, st, J, primes, tabs);
  else if (pro == PRO_CENTRED_LIFT && epi == EPI_STORE)
    hipLaunchKernelGGL((k_ntt_fwd_b<LOGN, PRO_CENTRED_LIFT, EPI_STORE>), grid, blk, 0, st, J, primes, tabs);
  else if (pro == PRO_ROUNDDIV_LIFT && epi == EPI_ROUNDDIV)
    hipLaunchKernelGGL((k_ntt_fwd_b<LOGN, PRO_ROUNDDIV_LIFT, EPI_ROUNDDIV>), grid, blk, 0, st, J, primes, tabs);
  else if (pro == FAM_RESCALE && epi == EPI_ROUNDDIV)
    hipLaunchKernelGGL((k_ntt_fwd_b<LOGN, FAM_RESCALE, EPI_ROUNDDIV>), grid, blk, 0, st, J, primes, tabs);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <int LOGN>
hipError_t ks_launch(int which, const KsJob& J, const PrimeDev* primes, const NttTables& tabs, hipStream_t st) {
  using Sp = Split<LOGN>;
  const int B = J.B, Lp = J.Lp;
  if (B <= 0 || Lp <= 0) return hipSuccess;
  switch (which) {
    case 0:
      hipLaunchKernelGGL((k_ks_modup_cols<LOGN>), dim3(B * Lp * Lp * Sp::WA), dim3(Sp::SA::T), 0, st, J, primes,
                         tabs);
      break;
    case 1:
      // the special limb's blocks, then the data limbs' inner products
      hipLaunchKernelGGL((k_ks_special_blocks<LOGN>), dim3(2 * B * (1 + Lp) * Sp::WB), dim3(Sp::SB::T), 0, st, J,
                         primes, tabs);
      break;
    case 2:
      hipLaunchKernelGGL((k_ks_moddown_cols<LOGN, 0>), dim3(2 * B * Lp * Sp::WA), dim3(Sp::SA::T), 0, st, J, primes,
                         tabs);
      break;
    case 4:
      hipLaunchKernelGGL((k_ks_moddown_cols<LOGN, 1>), dim3(2 * B * Lp * Sp::WA), dim3(Sp::SA::T), 0, st, J, primes,
                         tabs);
      break;
    case 5:
      if (Lp < 2) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_ks_moddown_resc_cols<LOGN>), dim3(2 * B * (Lp - 1) * Sp::WA), dim3(Sp::SA::T), 0, st, J,
                         primes, tabs);
      break;
    case 6:
      if (Lp < 2) return hipErrorInvalidValue;
      hipLaunchKernelGGL((k_ks_moddown_blocks<LOGN, true>), dim3(2 * B * (Lp - 1) * Sp::WB), dim3(Sp::SB::T), 0, st,
                         J, primes, tabs);
      break;
    case 7:
      hipLaunchKernelGGL((k_cks_modup_cols<LOGN>), dim3(B * Lp * (Lp + 1) * Sp::WA), dim3(Sp::SA::T), 0, st, J,
                         primes, tabs);
      break;
    case 8:
      hipLaunchKernelGGL((k_cks_inner_blocks<LOGN>), dim3(2 * B * (Lp + 1) * Sp::WB), dim3(Sp::SB::T), 0, st, J,
                         primes, tabs);
      break;
    case 9:
    case 10:
      if (which == 9)
        hipLaunchKernelGGL((k_cks_moddown_cols<LOGN, 0>), dim3(2 * B * Lp * Sp::WA), dim3(Sp::SA::T), 0, st, J,
                           primes, tabs);
      else
        hipLaunchKernelGGL((k_cks_moddown_cols<LOGN, 1>), dim3(2 * B * Lp * Sp::WA), dim3(Sp::SA::T), 0, st, J,
                           primes, tabs);
      break;
    default:
      hipLaunchKernelGGL((k_ks_moddown_blocks<LOGN, false>), dim3(2 * B * Lp * Sp::WB), dim3(Sp::SB::T), 0, st, J,
                         primes, tabs);
  }
  return hipGetLastError();
}

// ---------------- work queue over heterogeneous transforms ----------------
// 1024 threads at every ring degree of the queue (2^12..2^14): 4, 8 or 16
// words per thread.
template <int LOGN>
using QCfg = Sched<LOGN, 0, LOGN, LOGN - 10>;
constexpr int QT = 1024;

template <int KIND, int LOGN>
__device__ __forceinline__ void q_transform(const NttJob& J, const QTables& T, int w, u64* lds, int tid) {
  constexpr int N = 1 << LOGN;
  int a, b;
  decode_job(J, w, a, b);
  const int dp = J.dst_prime[b];
  const PrimeDev P = T.primes[dp];
  if constexpr (KIND == QK_INV) {
    const double2* wf = reinterpret_cast<const double2*>(T.inv_fp) + (size_t)dp * N;
    const ulonglong2* wi = reinterpret_cast<const ulonglong2*>(T.inv) + (size_t)dp * N;
    if (J.gather_src) {
      if (P.use_fp)
        inv_body<LOGN, true, FpAr, QCfg<LOGN>>(J, wf, P, a, b, lds, tid);
      else
        inv_body<LOGN, true, IntAr, QCfg<LOGN>>(J, wi, P, a, b, lds, tid);
    } else {
      if (P.use_fp)
        inv_body<LOGN, false, FpAr, QCfg<LOGN>>(J, wf, P, a, b, lds, tid);
      else
        inv_body<LOGN, false, IntAr, QCfg<LOGN>>(J, wi, P, a, b, lds, tid);
    }
  } else {
    constexpr int PRO = KIND == QK_FWD_RD ? PRO_ROUNDDIV_LIFT : PRO_CENTRED_LIFT;
    constexpr int EPI = KIND == QK_FWD_RD ? EPI_ROUNDDIV : EPI_STORE;
    if (P.use_fp)
      fwd_body<LOGN, PRO, EPI, FpAr, QCfg<LOGN>>(J, T.primes, reinterpret_cast<const double2*>(T.fwd_fp) + (size_t)dp * N,
                                                 P, a, b, lds, tid);
    else
      fwd_body<LOGN, PRO, EPI, IntAr, QCfg<LOGN>>(
          J, T.primes, reinterpret_cast<const ulonglong2*>(T.fwd) + (size_t)dp * N, P, a, b, lds, tid);
  }
}

template <int KIND>
__global__ void __launch_bounds__(QT) k_queue(const QTask* __restrict__ tasks, int n, const void* __restrict__ jobs,
                                             const QTables* __restrict__ tabs, unsigned* head) {
  extern __shared__ u64 lds[];
  __shared__ int s_next;
  for (;;) {
    if (threadIdx.x == 0) s_next = (int)atomicAdd(head, 1u);
    __syncthreads();
    // wave-uniform (scalar registers): the task and job records then come
    // through scalar loads
    const int k = __builtin_amdgcn_readfirstlane(s_next);
    if (k >= n) return;  // the same value in every thread: the workgroup leaves together
    const QTask t = tasks[k];
    const QTables T = tabs[t.tab];
    if constexpr (KIND == QK_TENSOR) {
      const QTensor& J = static_cast<const QTensor*>(jobs)[t.job];
      const int nn = 1 << t.log_n, limb = t.w;
      const PrimeDev P = T.primes[limb];
      const long long per = (long long)J.Lp * nn;
      for (int i = threadIdx.x; i < nn; i += QT) {
        const long long e = (long long)limb * nn + i;
        const u64 a0 = J.a[e], a1 = J.a[per + e], b0 = J.b[e], b1 = J.b[per + e];
        J.out01[e] = mulmod(a0, b0, P);
        J.out01[per + e] = addmod(mulmod(a0, b1, P), mulmod(a1, b0, P), P.q);
        J.out2[e] = mulmod(a1, b1, P);
      }
    } else if constexpr (KIND == QK_INNER) {
      // modulus t, coefficients [1024 s, 1024 s + 1024) of every item of
      // the job (items that share one key): each thread reads its key
      // words once and applies them to every item
      const InnerJob& J = static_cast<const InnerJob*>(jobs)[t.job];
      const int nn = 1 << t.log_n, nm = J.n_dig + 1;
      const int slices = nn / QT, tt = t.w / slices, i = (t.w - tt * slices) * QT + (int)threadIdx.x;
      const PrimeDev P = T.primes[tt < J.n_dig ? tt : J.special_prime];
      inner_shared_key(J, P, t.log_n, tt, i);
    } else {
      const NttJob& J = static_cast<const NttJob*>(jobs)[t.job];
      int tid = threadIdx.x;
      asm volatile("" : "+v"(tid));  // opaque per task: no hoisting across tasks
      if (t.log_n == 12)
        q_transform<KIND, 12>(J, T, t.w, lds, tid);
      else if (t.log_n == 13)
        q_transform<KIND, 13>(J, T, t.w, lds, tid);
      else
        q_transform<KIND, 14>(J, T, t.w, lds, tid);
    }
    __syncthreads();  // LDS and s_next are free for the next task
  }
}

__global__ void k_fill_u32(unsigned* p, int n, unsigned v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

hipError_t launch_ntt_inv_blocks(int log_n, const NttJob& job, const PrimeDev* primes, const NttTables& tabs,
                                 int tag, hipStream_t st) {
  if (tag == 2 && job.gather_src) return hipErrorInvalidValue;
#define C_(L) inv_blocks_launch<L>(job, primes, tabs, tag, st)
  switch (log_n) {
    case 10: return C_(10);
    case 11: return C_(11);
    case 12: return C_(12);
    case 13: return C_(13);
    case 14: return C_(14);
    default: return hipErrorInvalidValue;
  }
#undef C_
}

hipError_t launch_ntt_fwd_blocks(int log_n, int pro, int epi, const NttJob& job, const PrimeDev* primes,
                                 const NttTables& tabs, hipStream_t st) {
#define C_(L) fwd_blocks_launch<L>(pro, epi, job, primes, tabs, st)
  switch (log_n) {
    case 10: return C_(10);
    case 11: return C_(11);
    case 12: return C_(12);
    case 13: return C_(13);
    case 14: return C_(14);
    default: return hipErrorInvalidValue;
  }
#undef C_
}

static hipError_t ks_any(int which, int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                         hipStream_t st) {
  switch (log_n) {
    case 10: return ks_launch<10>(which, job, primes, tabs, st);
    case 11: return ks_launch<11>(which, job, primes, tabs, st);
    case 12: return ks_launch<12>(which, job, primes, tabs, st);
    case 13: return ks_launch<13>(which, job, primes, tabs, st);
    case 14: return ks_launch<14>(which, job, primes, tabs, st);
    default: return hipErrorInvalidValue;
  }
}
hipError_t launch_ks_modup_cols(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                hipStream_t st) {
  return ks_any(0, log_n, job, primes, tabs, st);
}
hipError_t launch_ks_special_blocks(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                    hipStream_t st) {
  return ks_any(1, log_n, job, primes, tabs, st);
}
hipError_t launch_ks_moddown_cols(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                  hipStream_t st) {
  return ks_any(2, log_n, job, primes, tabs, st);
}
hipError_t launch_ks_moddown_blocks(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                    hipStream_t st) {
  return ks_any(3, log_n, job, primes, tabs, st);
}
hipError_t launch_rescale_cols(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                               hipStream_t st) {
  return ks_any(4, log_n, job, primes, tabs, st);
}
hipError_t launch_cks_modup_cols(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                 hipStream_t st) {
  return ks_any(7, log_n, job, primes, tabs, st);
}
hipError_t launch_cks_inner_blocks(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                   hipStream_t st) {
  return ks_any(8, log_n, job, primes, tabs, st);
}
hipError_t launch_cks_moddown_cols(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                   hipStream_t st) {
  return ks_any(9, log_n, job, primes, tabs, st);
}
hipError_t launch_cks_rescale_cols(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                   hipStream_t st) {
  return ks_any(10, log_n, job, primes, tabs, st);
}
hipError_t launch_ks_moddown_resc_cols(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                       hipStream_t st) {
  return ks_any(5, log_n, job, primes, tabs, st);
}
hipError_t launch_ks_moddown_resc_blocks(int log_n, const KsJob& job, const PrimeDev* primes,
                                         const NttTables& tabs, hipStream_t st) {
  return ks_any(6, log_n, job, primes, tabs, st);
}

hipError_t launch_ntt_fwd(int log_n, int pro, int epi, const NttJob& job, const PrimeDev* primes,
                          const NttTables& tabs, hipStream_t st) {
  switch (log_n) {
    case 10: return fwd_dispatch<10>(pro, epi, job, primes, tabs, st);
    case 11: return fwd_dispatch<11>(pro, epi, job, primes, tabs, st);
    case 12: return fwd_dispatch<12>(pro, epi, job, primes, tabs, st);
    case 13: return fwd_dispatch<13>(pro, epi, job, primes, tabs, st);
    case 14: return fwd_dispatch<14>(pro, epi, job, primes, tabs, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ntt_inv(int log_n, const NttJob& job, const PrimeDev* primes, const NttTables& tabs,
                          hipStream_t st) {
  switch (log_n) {
    case 10: return inv_dispatch<10>(job, primes, tabs, st);
    case 11: return inv_dispatch<11>(job, primes, tabs, st);
    case 12: return inv_dispatch<12>(job, primes, tabs, st);
    case 13: return inv_dispatch<13>(job, primes, tabs, st);
    case 14: return inv_dispatch<14>(job, primes, tabs, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_hoisted_cols(int log_n, const HoistMac& job, const PrimeDev* primes, const NttTables& tabs,
                               hipStream_t st) {
  switch (log_n) {
    case 10: return hoist_cols_launch<10>(job, primes, tabs, st);
    case 11: return hoist_cols_launch<11>(job, primes, tabs, st);
    case 12: return hoist_cols_launch<12>(job, primes, tabs, st);
    case 13: return hoist_cols_launch<13>(job, primes, tabs, st);
    case 14: return hoist_cols_launch<14>(job, primes, tabs, st);
    default: return hipErrorInvalidValue;
  }
}

int hoist_split_blocks(int log_n) {
  switch (log_n) {
    case 10: return Split<10>::WB;
    case 11: return Split<11>::WB;
    case 12: return Split<12>::WB;
    case 13: return Split<13>::WB;
    case 14: return Split<14>::WB;
    default: return 0;
  }
}

hipError_t launch_hoisted_moddown_mac(int log_n, const HoistMac& job, const PrimeDev* primes, const NttTables& tabs,
                                      hipStream_t st) {
  switch (log_n) {
    case 10: return hoist_launch<10>(job, primes, tabs, st);
    case 11: return hoist_launch<11>(job, primes, tabs, st);
    case 12: return hoist_launch<12>(job, primes, tabs, st);
    case 13: return hoist_launch<13>(job, primes, tabs, st);
    case 14: return hoist_launch<14>(job, primes, tabs, st);
    default: return hipErrorInvalidValue;
  }
}

// ---------------- work-queue launches ----------------
size_t queue_lds_bytes(int kind, int log_n) {
  if (kind == QK_TENSOR || kind == QK_INNER) return 0;
  switch (log_n) {
    case 12: return sizeof(u64) * QCfg<12>::lds_words();
    case 13: return sizeof(u64) * QCfg<13>::lds_words();
    case 14: return sizeof(u64) * QCfg<14>::lds_words();
    default: return 0;
  }
}

int queue_grid(int device, size_t lds_bytes) {
  int cus = 0, lds_cu = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
    cus = 256;
  if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device) != hipSuccess ||
      lds_cu <= 0)
    lds_cu = 160 * 1024;
  // at most two 1024-thread workgroups per compute unit (32 waves)
  int per = 2;
  if (lds_bytes > 0) per = std::max(1, std::min(2, (int)((size_t)lds_cu / (lds_bytes + 1024))));
  return cus * per;
}

template <int KIND>
static hipError_t queue_launch_as(const QTask* tasks, int n, const void* jobs, const QTables* tabs, unsigned* head,
                                  int grid, size_t lds, hipStream_t st) {
  // the attribute allows the largest task's LDS (ring degree 2^14) once
  static bool attr = false;
  if (lds > 0) {
    if (lds > queue_lds_bytes(KIND, 14)) return hipErrorInvalidValue;
    hipError_t e = set_lds(k_queue<KIND>, queue_lds_bytes(KIND, 14), attr);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_queue<KIND>), dim3(grid), dim3(QT), lds, st, tasks, n, jobs, tabs, head);
  return hipGetLastError();
}

hipError_t launch_queue(int kind, const QTask* tasks, int n, const void* jobs, const QTables* tabs, unsigned* head,
                        int grid, size_t lds_bytes, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (grid <= 0 || !tasks || !jobs || !tabs || !head) return hipErrorInvalidValue;
  switch (kind) {
    case QK_TENSOR: return queue_launch_as<QK_TENSOR>(tasks, n, jobs, tabs, head, grid, lds_bytes, st);
    case QK_INV: return queue_launch_as<QK_INV>(tasks, n, jobs, tabs, head, grid, lds_bytes, st);
    case QK_FWD_LIFT: return queue_launch_as<QK_FWD_LIFT>(tasks, n, jobs, tabs, head, grid, lds_bytes, st);
    case QK_INNER: return queue_launch_as<QK_INNER>(tasks, n, jobs, tabs, head, grid, lds_bytes, st);
    case QK_FWD_RD: return queue_launch_as<QK_FWD_RD>(tasks, n, jobs, tabs, head, grid, lds_bytes, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

int ntt_shapes(int log_n, NttShape* out, int cap) {
  auto fill = [&](auto list, int loge0) {
    using Lst = decltype(list);
    int k = 0;
    if (k < cap) out[k] = NttShape{loge0, loge0, 1 << (log_n - loge0)};
    k++;
    for (int i = 0; i < Lst::n; i++, k++)
      if (k < cap) out[k] = NttShape{Lst::e[i], Lst::r[i], 1 << (log_n - Lst::e[i])};
    return k;
  };
  switch (log_n) {
    case 12: return fill(ShapeList<12>{}, single_loge(12));
    case 13: return fill(ShapeList<13>{}, single_loge(13));
    case 14: return fill(ShapeList<14>{}, single_loge(14));
    default:
      if (cap > 0) out[0] = NttShape{single_loge(log_n), single_loge(log_n), 1 << (log_n - single_loge(log_n))};
      return 1;
  }
}
