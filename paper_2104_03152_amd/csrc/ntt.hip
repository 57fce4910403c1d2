// ntt.hip -- batched negacyclic NTT over 64-bit RNS limbs for gfx950.
//
// One workgroup transforms one limb of N = 2^LOGN words entirely in LDS.
// Each thread holds 16 words; the LOGN butterfly stages are split into
// ceil(LOGN/4) register passes of radix 2^3 or 2^4, separated by LDS
// exchanges (padded by one word every 16 to spread banks).  Butterflies are
// Harvey's lazy ones with Shoup twiddles: forward values stay in [0, 4q),
// inverse values in [0, 2q), one reduction at the end.
//
// Forward: Cooley-Tukey with twiddles psi^brv(k), output in bit-reversed
// order: slot i holds a(psi^(2 brv(i) + 1)).  Inverse: Gentleman-Sande with
// psi^-brv(k), then N^-1.
//
// The prologue can lift a digit while loading (centred representative of a
// residue mod another prime: key-switch ModUp) or form r = [x + h]_p (the
// divide-and-round of ModDown and rescale, less h); the epilogue then finishes
// the division: dst = (u - NTT(r - h)) * p^-1 mod q (+ an addend).
#include "device.h"

namespace {

template <int LOGN>
struct Cfg {
  static constexpr int N = 1 << LOGN;
  static constexpr int E = 16;  // words per thread
  static constexpr int T = N / E;
  static constexpr int NP = (LOGN + 3) / 4;
  static constexpr int bits(int p) { return LOGN / NP + (p < LOGN % NP ? 1 : 0); }
  static constexpr int consumed(int p) {
    int s = 0;
    for (int i = 0; i < p; i++) s += bits(i);
    return s;
  }
  static constexpr int lds_words() { return N + (N >> 4); }
};

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

// ---------------- forward passes ----------------
template <int LOGN, int P>
__device__ __forceinline__ void fwd_passes(u64 (&x)[16], u64* lds, const ulonglong2* __restrict__ W,
                                           u64 q, int tid) {
  using C = Cfg<LOGN>;
  constexpr int R = C::bits(P);
  constexpr int LO = LOGN - C::consumed(P + 1);
  constexpr int G = 16 >> R;
  const u64 q2 = q << 1;
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int pb = R - 1 - r;
    const int s = LOGN - 1 - (LO + pb);
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + C::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) {
        if (c & (1 << pb)) continue;
        const int i0 = u * (1 << R) + c, i1 = i0 + (1 << pb);
        const int ti = (1 << s) + (((gi >> LO) << (R - 1 - pb)) | (c >> (pb + 1)));
        const ulonglong2 w = W[ti];
        u64 X = x[i0];
        X = X >= q2 ? X - q2 : X;
        const u64 V = shoup_lazy(x[i1], w.x, w.y, q);
        x[i0] = X + V;
        x[i1] = X - V + q2;
      }
    }
  }
  if constexpr (P + 1 < C::NP) {
    constexpr int R2 = C::bits(P + 1);
    constexpr int LO2 = LOGN - C::consumed(P + 2);
    constexpr int G2 = 16 >> R2;
    if (P > 0) __syncthreads();
#pragma unroll
    for (int u = 0; u < G; u++)
#pragma unroll
      for (int c = 0; c < (1 << R); c++) lds[pad(gidx(tid + C::T * u, c, LO, R))] = x[u * (1 << R) + c];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < G2; u++)
#pragma unroll
      for (int c = 0; c < (1 << R2); c++) x[u * (1 << R2) + c] = lds[pad(gidx(tid + C::T * u, c, LO2, R2))];
    fwd_passes<LOGN, P + 1>(x, lds, W, q, tid);
  }
}

template <int LOGN, int PRO, int EPI>
__global__ void __launch_bounds__(Cfg<LOGN>::T)
k_ntt_fwd(const NttJob J, const PrimeDev* __restrict__ primes, const u64* __restrict__ tw) {
  using C = Cfg<LOGN>;
  constexpr int N = C::N;
  extern __shared__ u64 lds[];
  const int tid = threadIdx.x;
  int a, b;
  decode_job(J, blockIdx.x, a, b);
  const int dp = J.dst_prime[b];
  const PrimeDev P = primes[dp];
  const u64 q = P.q;
  const ulonglong2* W = reinterpret_cast<const ulonglong2*>(tw) + (size_t)dp * N;
  const u64* __restrict__ src = J.src + a * J.sa + b * J.sb;
  u64 x[16];
  {
    constexpr int R = C::bits(0), LO = LOGN - R, G = 16 >> R;
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
        x[u * (1 << R) + c] = v;
      }
    }
  }
  fwd_passes<LOGN, 0>(x, lds, W, q, tid);
  {
    constexpr int R = C::bits(C::NP - 1), G = 16 >> R;
    u64* __restrict__ dst = J.dst + a * J.da + b * J.db;
    const u64 q2 = q << 1;
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
#pragma unroll
      for (int c = 0; c < (1 << R); c++) {
        u64 v = x[u * (1 << R) + c];
        v = v >= q2 ? v - q2 : v;
        v = v >= q ? v - q : v;
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

// ---------------- inverse passes ----------------
template <int LOGN, int P>
__device__ __forceinline__ void inv_passes(u64 (&x)[16], u64* lds, const ulonglong2* __restrict__ W,
                                           u64 q, int tid) {
  using C = Cfg<LOGN>;
  constexpr int R = C::bits(P);
  constexpr int LO = C::consumed(P);
  constexpr int G = 16 >> R;
  const u64 q2 = q << 1;
#pragma unroll
  for (int r = 0; r < R; r++) {
    const int pb = r;
    const int m_log = LOGN - 1 - (LO + pb);
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + C::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) {
        if (c & (1 << pb)) continue;
        const int i0 = u * (1 << R) + c, i1 = i0 + (1 << pb);
        const int ti = (1 << m_log) + (((gi >> LO) << (R - 1 - pb)) | (c >> (pb + 1)));
        const ulonglong2 w = W[ti];
        const u64 X = x[i0], Y = x[i1];
        u64 S = X + Y;
        S = S >= q2 ? S - q2 : S;
        x[i0] = S;
        x[i1] = shoup_lazy(X - Y + q2, w.x, w.y, q);
      }
    }
  }
  if constexpr (P + 1 < C::NP) {
    constexpr int R2 = C::bits(P + 1);
    constexpr int LO2 = C::consumed(P + 1);
    constexpr int G2 = 16 >> R2;
    if (P > 0) __syncthreads();
#pragma unroll
    for (int u = 0; u < G; u++)
#pragma unroll
      for (int c = 0; c < (1 << R); c++) lds[pad(gidx(tid + C::T * u, c, LO, R))] = x[u * (1 << R) + c];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < G2; u++)
#pragma unroll
      for (int c = 0; c < (1 << R2); c++) x[u * (1 << R2) + c] = lds[pad(gidx(tid + C::T * u, c, LO2, R2))];
    inv_passes<LOGN, P + 1>(x, lds, W, q, tid);
  }
}

template <int LOGN, bool GATHER>
__global__ void __launch_bounds__(Cfg<LOGN>::T)
k_ntt_inv(const NttJob J, const PrimeDev* __restrict__ primes, const u64* __restrict__ tw) {
  using C = Cfg<LOGN>;
  constexpr int N = C::N;
  extern __shared__ u64 lds[];
  const int tid = threadIdx.x;
  int a, b;
  decode_job(J, blockIdx.x, a, b);
  const int dp = J.dst_prime[b];
  const PrimeDev P = primes[dp];
  const u64 q = P.q;
  const ulonglong2* W = reinterpret_cast<const ulonglong2*>(tw) + (size_t)dp * N;
  const u64* __restrict__ src = J.src + a * J.sa + b * J.sb;
  u64 x[16];
  {
    constexpr int R = C::bits(0), G = 16 >> R;  // bits [0, R): contiguous runs
    const u64 g = GATHER ? J.gal[a / J.gal_div] : 1;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + C::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) {
        const int idx = (gi << R) | c;
        x[u * (1 << R) + c] = src[GATHER ? gal_src(idx, LOGN, g) : idx];
      }
    }
  }
  inv_passes<LOGN, 0>(x, lds, W, q, tid);
  {
    constexpr int R = C::bits(C::NP - 1), LO = LOGN - R, G = 16 >> R;
    u64* __restrict__ dst = J.dst + a * J.da + b * J.db;
#pragma unroll
    for (int u = 0; u < G; u++) {
      const int gi = tid + C::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R); c++) dst[(c << LO) | gi] = shoup(x[u * (1 << R) + c], P.ninv, P.ninv_sh, q);
    }
  }
}

// Hoisted rotations: ModDown of each item (an NTT of its special-prime limb,
// lifted) with the plaintext multiply-accumulate of the vector-matrix
// product in the epilogue.  Workgroup (chunk, k, t) loops over its items;
// the running sums live in its own slice of `partial` (each thread re-reads
// exactly the words it wrote, so no barrier is needed for them).
template <int LOGN>
__global__ void __launch_bounds__(Cfg<LOGN>::T, (LOGN <= 13 ? 4 : 1))
k_hoist_mac(const HoistMac J, const PrimeDev* __restrict__ primes, const u64* __restrict__ tw) {
  using C = Cfg<LOGN>;
  constexpr int N = C::N;
  constexpr int R0 = C::bits(0), LO0 = LOGN - R0, G0 = 16 >> R0;
  constexpr int RF = C::bits(C::NP - 1), GF = 16 >> RF;
  extern __shared__ u64 lds[];
  const int tid = threadIdx.x;
  const int pairs = 2 * J.n_dig;
  const int chunk = blockIdx.x / pairs;
  const int kt = blockIdx.x - chunk * pairs;
  const int k = kt / J.n_dig, t = kt - k * J.n_dig;
  const PrimeDev P = primes[t];
  const u64 q = P.q, q2 = q << 1;
  const ulonglong2* W = reinterpret_cast<const ulonglong2*>(tw) + (size_t)t * N;
  const u64 sq = primes[J.special_prime].q, sh = J.h_src;
  const u64 hq = J.hq[t], inv = J.inv[t], inv_sh = J.inv_sh[t];
  u64* __restrict__ out = J.partial + (((size_t)chunk * 2 + k) * J.n_dig + t) * N;
  const int rb = chunk * J.chunk, re = min(J.R, rb + J.chunk);
  for (int r = rb; r < re; r++) {
    const HoistItem it = J.items[r];
    const u64* __restrict__ src = J.ucoef + ((size_t)r * 2 + k) * N;
    u64 x[16];
#pragma unroll
    for (int u = 0; u < G0; u++) {
      const int gi = tid + C::T * u;
#pragma unroll
      for (int c = 0; c < (1 << R0); c++) {
        u64 v = src[(c << LO0) | gi] + sh;
        v = v >= sq ? v - sq : v;
        x[u * (1 << R0) + c] = submod(red64(v, P), hq, q);
      }
    }
    // keep the twiddle loads inside the loop (hoisting them out would hold
    // every stage's twiddles in registers across items)
    const ulonglong2* Wr = W;
    asm volatile("" : "+v"(Wr));
    fwd_passes<LOGN, 0>(x, lds, Wr, q, tid);
    // final values through LDS so the epilogue runs in natural order:
    // coalesced accesses and a bounded number of loads in flight
    __syncthreads();
#pragma unroll
    for (int u = 0; u < GF; u++) {
      const int gi = tid + C::T * u;
#pragma unroll
      for (int c = 0; c < (1 << RF); c++) {
        u64 v = x[u * (1 << RF) + c];
        v = v >= q2 ? v - q2 : v;
        lds[pad((gi << RF) | c)] = v >= q ? v - q : v;
      }
    }
    __syncthreads();
    const u64* __restrict__ uu = J.u + (((size_t)r * 2 + k) * J.nm + t) * N;
    const u64* __restrict__ dg = J.diags + ((size_t)it.diag * J.n_dig + t) * N;
    const u64* __restrict__ dgs = J.diags_sh + ((size_t)it.diag * J.n_dig + t) * N;
    const u64* __restrict__ c0 = J.c0 + (size_t)t * N;
    const bool first = (r == rb);
#pragma unroll 4
    for (int e = 0; e < 16; e++) {
      const int idx = tid + C::T * e;
      const u64 v = lds[pad(idx)];
      u64 ks = shoup(submod(uu[idx], v, q), inv, inv_sh, q);
      if (k == 0) ks = addmod(ks, c0[gal_src(idx, LOGN, it.g)], q);
      const u64 prod = shoup(ks, dg[idx], dgs[idx], q);
      out[idx] = first ? prod : addmod(out[idx], prod, q);
    }
    __syncthreads();
  }
}

template <int LOGN>
hipError_t hoist_launch(const HoistMac& J, const PrimeDev* primes, const u64* tw, hipStream_t st) {
  using C = Cfg<LOGN>;
  const size_t shm = sizeof(u64) * C::lds_words();
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_hoist_mac<LOGN>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int n_chunks = (J.R + J.chunk - 1) / J.chunk;
  const int blocks = n_chunks * 2 * J.n_dig;
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_hoist_mac<LOGN>), dim3(blocks), dim3(C::T), shm, st, J, primes, tw);
  return hipGetLastError();
}

int n_jobs(const NttJob& J) { return J.na * (J.skip_diag ? J.nb - 1 : J.nb); }

template <int LOGN, int PRO, int EPI>
hipError_t fwd_launch(const NttJob& J, const PrimeDev* primes, const u64* tw, hipStream_t st) {
  using C = Cfg<LOGN>;
  const size_t shm = sizeof(u64) * C::lds_words();
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_ntt_fwd<LOGN, PRO, EPI>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int jobs = n_jobs(J);
  if (jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_ntt_fwd<LOGN, PRO, EPI>), dim3(jobs), dim3(C::T), shm, st, J, primes, tw);
  return hipGetLastError();
}

template <int LOGN, bool GATHER>
hipError_t inv_launch(const NttJob& J, const PrimeDev* primes, const u64* tw, hipStream_t st) {
  using C = Cfg<LOGN>;
  const size_t shm = sizeof(u64) * C::lds_words();
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute((const void*)k_ntt_inv<LOGN, GATHER>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int jobs = n_jobs(J);
  if (jobs <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_ntt_inv<LOGN, GATHER>), dim3(jobs), dim3(C::T), shm, st, J, primes, tw);
  return hipGetLastError();
}

template <int LOGN>
hipError_t inv_dispatch(const NttJob& J, const PrimeDev* primes, const u64* tw, hipStream_t st) {
  return J.gather_src ? inv_launch<LOGN, true>(J, primes, tw, st) : inv_launch<LOGN, false>(J, primes, tw, st);
}

template <int LOGN>
hipError_t fwd_dispatch(int pro, int epi, const NttJob& J, const PrimeDev* primes, const u64* tw,
                        hipStream_t st) {
  if (pro == PRO_PLAIN && epi == EPI_STORE) return fwd_launch<LOGN, PRO_PLAIN, EPI_STORE>(J, primes, tw, st);
  if (pro == PRO_CENTRED_LIFT && epi == EPI_STORE)
    return fwd_launch<LOGN, PRO_CENTRED_LIFT, EPI_STORE>(J, primes, tw, st);
  if (pro == PRO_ROUNDDIV_LIFT && epi == EPI_ROUNDDIV)
    return fwd_launch<LOGN, PRO_ROUNDDIV_LIFT, EPI_ROUNDDIV>(J, primes, tw, st);
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_ntt_fwd(int log_n, int pro, int epi, const NttJob& job, const PrimeDev* primes,
                          const u64* fwd_tw, hipStream_t st) {
  switch (log_n) {
    case 10: return fwd_dispatch<10>(pro, epi, job, primes, fwd_tw, st);
    case 11: return fwd_dispatch<11>(pro, epi, job, primes, fwd_tw, st);
    case 12: return fwd_dispatch<12>(pro, epi, job, primes, fwd_tw, st);
    case 13: return fwd_dispatch<13>(pro, epi, job, primes, fwd_tw, st);
    case 14: return fwd_dispatch<14>(pro, epi, job, primes, fwd_tw, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_ntt_inv(int log_n, const NttJob& job, const PrimeDev* primes, const u64* inv_tw,
                          hipStream_t st) {
  switch (log_n) {
    case 10: return inv_dispatch<10>(job, primes, inv_tw, st);
    case 11: return inv_dispatch<11>(job, primes, inv_tw, st);
    case 12: return inv_dispatch<12>(job, primes, inv_tw, st);
    case 13: return inv_dispatch<13>(job, primes, inv_tw, st);
    case 14: return inv_dispatch<14>(job, primes, inv_tw, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_hoisted_moddown_mac(int log_n, const HoistMac& job, const PrimeDev* primes, const u64* fwd_tw,
                                      hipStream_t st) {
  switch (log_n) {
    case 10: return hoist_launch<10>(job, primes, fwd_tw, st);
    case 11: return hoist_launch<11>(job, primes, fwd_tw, st);
    case 12: return hoist_launch<12>(job, primes, fwd_tw, st);
    case 13: return hoist_launch<13>(job, primes, fwd_tw, st);
    case 14: return hoist_launch<14>(job, primes, fwd_tw, st);
    default: return hipErrorInvalidValue;
  }
}
