// kernels.hip -- samplers, pointwise NTT-domain arithmetic, the Galois
// automorphism and the key-switch inner product for gfx950.
//
// All polynomials are limb-major [poly][limb][N] u64 rows; a thread owns one
// coefficient of one row, so every access is a coalesced 8-byte word.
#include <mutex>

#include "../../include/ckks_hip.h"
#include "device.h"
#include "inner.h"

// The no-allocation entry point's scratch: every intermediate of one call
// lives here.  Each device holds its own copy for the life of the process;
// host code reaches it only through the address hipGetSymbolAddress gives
// for that device (the array's name is a host-side stand-in).
static __device__ __align__(256) u64 scratch[HE_NOALLOC_SCRATCH_BYTES / sizeof(u64)];

hipError_t noalloc_scratch(int device, u64** ptr, size_t* bytes) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static u64* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = static_cast<u64*>(p);
  }
  *ptr = addr[device];
  *bytes = HE_NOALLOC_SCRATCH_BYTES;
  return hipSuccess;
}

namespace {

constexpr int BLK = 256;

// ---------------- ChaCha20 (RFC 8439 block function) ----------------
__device__ __forceinline__ u32 rotl32(u32 v, int c) { return (v << c) | (v >> (32 - c)); }
#define QR(a, b, c, d)   \
  a += b;                \
  d ^= a;                \
  d = rotl32(d, 16);     \
  c += d;                \
  b ^= c;                \
  b = rotl32(b, 12);     \
  a += b;                \
  d ^= a;                \
  d = rotl32(d, 8);      \
  c += d;                \
  b ^= c;                \
  b = rotl32(b, 7);

// key = seed (LE) || 24 zero bytes, nonce = (tag, a, b), counter = block
__device__ void chacha_block(uint64_t seed, u32 counter, u32 n0, u32 n1, u32 n2, u32 out[16]) {
  const u32 s[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u, (u32)seed, (u32)(seed >> 32),
                     0u,          0u,          0u,          0u,          0u,         0u,
                     counter,     n0,          n1,          n2};
  u32 x[16];
#pragma unroll
  for (int i = 0; i < 16; i++) x[i] = s[i];
#pragma unroll
  for (int i = 0; i < 10; i++) {
    QR(x[0], x[4], x[8], x[12]);
    QR(x[1], x[5], x[9], x[13]);
    QR(x[2], x[6], x[10], x[14]);
    QR(x[3], x[7], x[11], x[15]);
    QR(x[0], x[5], x[10], x[15]);
    QR(x[1], x[6], x[11], x[12]);
    QR(x[2], x[7], x[8], x[13]);
    QR(x[3], x[4], x[9], x[14]);
  }
#pragma unroll
  for (int i = 0; i < 16; i++) out[i] = x[i] + s[i];
}

// P(|x| <= k) * 2^63 for the discrete Gaussian of sigma 3.2 cut at 19
__constant__ u64 kCdt[20] = {
    0x0ff52b40a5917f1dull, 0x2e5a25d4bf0e400eull, 0x489ae26955b04bd6ull, 0x5d2bc20f621bf185ull,
    0x6bc8694c3cc80ff4ull, 0x7532d89ac6ba7dceull, 0x7ab396cb74436798ull, 0x7d9e4e916643eb07ull,
    0x7f05495819eb2051ull, 0x7fa1ce9c0039a957ull, 0x7fdfb3f212e8c4e8ull, 0x7ff5e6f9d2314fccull,
    0x7ffd1f97bc4406a2ull, 0x7fff40fa0088d11dull, 0x7fffd2e835e1c57dull, 0x7ffff6524386ff1eull,
    0x7ffffe1db4769da5ull, 0x7fffffac0a1dcb08ull, 0x7ffffff428673853ull, 0x8000000000000000ull};

// one thread per ChaCha block = 8 coefficients
__global__ void k_sample_small(int n, int kind, uint64_t seed, u32 tag, u32 a, ModList mods, u64* out,
                               const PrimeDev* __restrict__ primes) {
  const int blk = blockIdx.x * blockDim.x + threadIdx.x;
  if (blk * 8 >= n) return;
  u32 w[16];
  chacha_block(seed, (u32)blk, tag, a, 0u, w);
#pragma unroll
  for (int r = 0; r < 8; r++) {
    const u64 word = (u64)w[2 * r] | ((u64)w[2 * r + 1] << 32);
    i64 v;
    if (kind == 0) {
      v = (i64)(word % 3) - 1;
    } else {
      const u64 uu = word >> 1;
      int k = 0;
      while (!(uu < kCdt[k])) k++;
      v = (word & 1) ? -(i64)k : (i64)k;
    }
    const int i = blk * 8 + r;
    for (int m = 0; m < mods.n; m++) out[(size_t)m * n + i] = red_signed(v, primes[mods.p[m]]);
  }
}

// one thread per ChaCha block = 4 coefficients (2 words each)
__global__ void k_sample_uniform(int n, uint64_t seed, u32 tag, u32 a_base, int n_rows, ModList mods,
                                 ModList pidx, u64* out, const PrimeDev* __restrict__ primes) {
  const int per = n / 4;
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= (long long)per * n_rows * mods.n) return;
  const int blk = (int)(g % per);
  const int rm = (int)(g / per);
  const int m = rm % mods.n, row = rm / mods.n;
  const PrimeDev P = primes[mods.p[m]];
  u32 w[16];
  chacha_block(seed, (u32)blk, tag, a_base + (u32)row, (u32)pidx.p[m], w);
  const u64 t64 = addmod(red64(~0ull, P), 1, P.q);  // 2^64 mod q
  u64* o = out + (size_t)rm * n + (size_t)blk * 4;
#pragma unroll
  for (int r = 0; r < 4; r++) {
    const u64 lo = (u64)w[4 * r] | ((u64)w[4 * r + 1] << 32);
    const u64 hi = (u64)w[4 * r + 2] | ((u64)w[4 * r + 3] << 32);
    o[r] = addmod(mulmod(red64(hi, P), t64, P), red64(lo, P), P.q);
  }
}

// ---------------- pointwise ----------------
__global__ void k_addsub(int n, int op, const u64* __restrict__ a, const u64* __restrict__ b,
                         u64* __restrict__ out, long long total, int n_limbs, ModList mods,
                         const PrimeDev* __restrict__ primes) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int limb = (int)((e / n) % n_limbs);
  const u64 q = primes[mods.p[limb]].q;
  const u64 x = a[e];
  u64 r;
  if (op == 0)
    r = addmod(x, b[e], q);
  else if (op == 1)
    r = submod(x, b[e], q);
  else
    r = x ? q - x : 0;
  out[e] = r;
}

__global__ void k_mul_plain(int n, const u64* __restrict__ a, const u64* __restrict__ p, u64* __restrict__ out,
                            long long total, int n_limbs, ModList mods, const PrimeDev* __restrict__ primes) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const long long row = e / n;
  const int limb = (int)(row % n_limbs);
  const PrimeDev P = primes[mods.p[limb]];
  out[e] = mulmod(a[e], p[(long long)limb * n + (e - row * n)], P);
}

__global__ void k_add_plain(int n, const u64* __restrict__ a, const u64* __restrict__ p, u64* __restrict__ out,
                            long long total, int n_limbs, ModList mods, const PrimeDev* __restrict__ primes,
                            int neg) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const long long row = e / n;
  const int limb = (int)(row % n_limbs);
  const u64 q = primes[mods.p[limb]].q;
  const long long per_poly = (long long)n_limbs * n;
  out[e] = (e < per_poly) ? (neg ? submod(a[e], p[e], q) : addmod(a[e], p[e], q)) : a[e];
}

__global__ void k_tensor(int n, const u64* __restrict__ a, const u64* __restrict__ b, u64* __restrict__ out01,
                         u64* __restrict__ out2, int n_limbs, ModList mods, const PrimeDev* __restrict__ primes) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)n_limbs * n;
  if (e >= per) return;
  const int limb = (int)(e / n);
  const PrimeDev P = primes[mods.p[limb]];
  const u64 a0 = a[e], a1 = a[per + e], b0 = b[e], b1 = b[per + e];
  out01[e] = mulmod(a0, b0, P);
  out01[per + e] = addmod(mulmod(a0, b1, P), mulmod(a1, b0, P), P.q);
  out2[e] = mulmod(a1, b1, P);
}

__global__ void k_tensor_many(int log_n, CtList A, CtList Bl, u64* __restrict__ out01, u64* __restrict__ out2,
                              int n_limbs, long long total, const PrimeDev* __restrict__ primes) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const long long per = (long long)n_limbs << log_n;
  const int item = (int)(e / per);
  const long long r = e - item * per;
  const PrimeDev P = primes[r >> log_n];
  const u64* a = A.p[item];
  const u64* b = Bl.p[item];
  const u64 a0 = a[r], a1 = a[per + r], b0 = b[r], b1 = b[per + r];
  u64* o = out01 + (size_t)item * 2 * per;
  o[r] = mulmod(a0, b0, P);
  o[per + r] = addmod(mulmod(a0, b1, P), mulmod(a1, b0, P), P.q);
  out2[(size_t)item * per + r] = mulmod(a1, b1, P);
}

__global__ void k_gather_cts(CtList A, u64* __restrict__ out, long long per_ct, long long total) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int item = (int)(e / per_ct);
  out[e] = A.p[item][e - item * per_ct];
}

__global__ void k_mul_plain_many(int log_n, CtList in, CtList pl, int n_limbs, u64* __restrict__ out,
                                 long long total, const PrimeDev* __restrict__ primes) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const long long per_poly = (long long)n_limbs << log_n, per = 2 * per_poly;
  const int b = (int)(e / per);
  const long long r = e - b * per;
  const long long rl = r >= per_poly ? r - per_poly : r;  // index within the poly
  const PrimeDev P = primes[rl >> log_n];
  out[e] = mulmod(in.p[b][r], pl.p[b][rl], P);
}

__global__ void k_add_plain_many(int log_n, CtList in, CtList pl, OutList outl, int n_limbs, long long total,
                                 const PrimeDev* __restrict__ primes) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const long long per_poly = (long long)n_limbs << log_n, per = 2 * per_poly;
  const int b = (int)(e / per);
  const long long r = e - b * per;
  const u64 v = in.p[b][r];
  outl.p[b][r] = r < per_poly ? addmod(v, pl.p[b][r], primes[r >> log_n].q) : v;
}

__global__ void k_sum_cts(int log_n, CtList in, int B, int n_limbs, u64* __restrict__ out, long long total,
                          const PrimeDev* __restrict__ primes) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const long long per_poly = (long long)n_limbs << log_n;
  const u64 q = primes[(e >= per_poly ? e - per_poly : e) >> log_n].q;
  u64 v = in.p[0][e];
  for (int b = 1; b < B; b++) v = addmod(v, in.p[b][e], q);
  out[e] = v;
}

__global__ void k_copy(const u64* __restrict__ src, u64* __restrict__ dst, long long words) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < words) dst[e] = src[e];
}

__global__ void k_decrypt(int n, const u64* __restrict__ ct, const u64* __restrict__ s, u64* __restrict__ m,
                          int n_limbs, const PrimeDev* __restrict__ primes) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)n_limbs * n;
  if (e >= per) return;
  const int limb = (int)(e / n);
  const PrimeDev P = primes[limb];
  m[e] = addmod(ct[e], mulmod(ct[per + e], s[e], P), P.q);
}

__global__ void k_automorphism(int log_n, const u64* __restrict__ in, u64* __restrict__ out, long long total,
                               AutJob J) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int n = 1 << log_n;
  const long long row = e >> log_n;
  const int i = (int)(e & (n - 1));
  const int b = (int)(row / J.rows_per_item);
  out[e] = in[row * n + gal_src(i, log_n, J.g[b])];
}

// key-switch inner product with lazy 128-bit accumulation (8 terms at most
// per Montgomery reduction: 8 q^2 < q 2^64 for q < 2^60)
__global__ void k_inner(int log_n, InnerJob J, const PrimeDev* __restrict__ primes) {
  const int n = 1 << log_n;
  const int nm = J.n_dig + 1;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)J.B * nm * n) return;
  const int i = (int)(e & (n - 1));
  const long long bt = e >> log_n;
  const int t = (int)(bt % nm), b = (int)(bt / nm);
  const PrimeDev P = primes[t < J.n_dig ? t : J.special_prime];
  u64 r0, r1;
  inner_point(J, P, log_n, b, t, i, r0, r1);
  u64* u = J.u + (size_t)b * 2 * nm * n;
  u[(size_t)t * n + i] = r0;
  u[((size_t)nm + t) * n + i] = r1;
}

__global__ void k_keygen_combine(int n, const u64* __restrict__ a, const u64* __restrict__ ee,
                                 const u64* __restrict__ s, const u64* __restrict__ sp, u64* __restrict__ key,
                                 int nd, int nm, ModList pidx, int special, const PrimeDev* __restrict__ primes) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)nd * nm * n) return;
  const int i = (int)(e % n);
  const int jt = (int)(e / n);
  const int t = jt % nm, j = jt / nm;
  const int pi = pidx.p[t];
  const PrimeDev P = primes[pi];
  const u64 av = a[e], ev = ee[e];
  u64 k0 = submod(ev, mulmod(av, s[(size_t)pi * n + i], P), P.q);
  if (t == j) k0 = addmod(k0, mulmod(red64(primes[special].q, P), sp[(size_t)pi * n + i], P), P.q);
  u64* out = key + ((size_t)j * 2 * nm) * n;
  out[(size_t)t * n + i] = mont_reduce(mul_wide(k0, P.r2), P);
  out[((size_t)nm + t) * n + i] = mont_reduce(mul_wide(av, P.r2), P);
}

__global__ void k_pk_combine(int n, const u64* __restrict__ a, const u64* __restrict__ ee,
                             const u64* __restrict__ s, u64* __restrict__ out, int limbs,
                             const PrimeDev* __restrict__ primes) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)limbs * n) return;
  const PrimeDev P = primes[e / n];
  out[e] = submod(ee[e], mulmod(a[e], s[e], P), P.q);
}

__global__ void k_encrypt_combine(int n, const u64* __restrict__ v, const u64* __restrict__ pk0,
                                  const u64* __restrict__ pk1, const u64* __restrict__ e0,
                                  const u64* __restrict__ e1, const u64* __restrict__ s,
                                  const u64* __restrict__ m, u64* __restrict__ ct, int limbs, int pk_limbs,
                                  const PrimeDev* __restrict__ primes) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long per = (long long)limbs * n;
  if (e >= per) return;
  const int limb = (int)(e / n);
  const PrimeDev P = primes[limb];
  const u64 vv = v[e];
  if (pk0) {
    const long long pe = e;  // pk rows share the limb layout for limb < pk_limbs
    ct[e] = addmod(addmod(mulmod(vv, pk0[pe], P), e0[e], P.q), m[e], P.q);
    ct[per + e] = addmod(mulmod(vv, pk1[pe], P), e1[e], P.q);
  } else {
    ct[e] = addmod(submod(e0[e], mulmod(vv, s[e], P), P.q), m[e], P.q);
    ct[per + e] = vv;
  }
  (void)pk_limbs;
}

__global__ void k_mont(int n, u64* data, long long total, int to, ModList mods,
                       const PrimeDev* __restrict__ primes) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int row = (int)(e / n);
  const PrimeDev P = primes[mods.p[row % mods.n]];
  const u64 v = data[e];
  data[e] = to ? mont_reduce(mul_wide(v, P.r2), P) : mont_reduce(U128{v, 0}, P);
}

// batched inner product of hoisted rotations: every item reads the shared
// ModUp digits (and, for poly 0, the input's c0) at its own Galois source
// index.  Keys and outputs pass once: non-temporal loads and stores, so
// that L2 keeps the gathered digits.  Each thread computes two
// neighbouring words (16-byte key loads and output stores); the digits are
// gathered word by word (they stay in L2, shared by all items).
__global__ void k_inner_hoisted(int log_n, HoistInner J, const PrimeDev* __restrict__ primes) {
  const int n = 1 << log_n;
  const int nt = J.t_end - J.t_begin;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)J.R * nt * (n >> 1)) return;
  const int i = (int)(e & ((n >> 1) - 1)) << 1;
  const long long rt = e >> (log_n - 1);
  const int t = J.t_begin + (int)(rt % nt);
  const int r = (int)(rt / nt);
  const HoistItem it = J.items[r];
  const int src0 = gal_src(i, log_n, it.g), src1 = gal_src(i + 1, log_n, it.g);
  const int kt = t < J.n_dig ? t : it.km - 1;
  const PrimeDev P = primes[t < J.n_dig ? t : J.special_prime];
  const size_t ks_k = (size_t)it.km * n, ks_j = 2 * ks_k;
  const u64* kp = it.key + (size_t)kt * n + i;
  u64 r00 = 0, r01 = 0, r10 = 0, r11 = 0;  // [poly][word]
  for (int j0 = 0; j0 < J.n_dig; j0 += 8) {
    U128 a00 = {0, 0}, a01 = {0, 0}, a10 = {0, 0}, a11 = {0, 0};
    const int j1 = min(J.n_dig, j0 + 8);
    for (int j = j0; j < j1; j++) {
      const u64* dj = (j == t) ? J.c1 + (size_t)t * n : J.ext + ((size_t)j * J.nm + t) * n;
      const u64 d0 = dj[src0], d1 = dj[src1];
      const u64* kq = kp + j * ks_j;  // poly 0; poly 1 at kq + ks_k
      a00 = add128(a00, mul_wide(d0, __builtin_nontemporal_load(kq)));
      a01 = add128(a01, mul_wide(d1, __builtin_nontemporal_load(kq + 1)));
      a10 = add128(a10, mul_wide(d0, __builtin_nontemporal_load(kq + ks_k)));
      a11 = add128(a11, mul_wide(d1, __builtin_nontemporal_load(kq + ks_k + 1)));
    }
    r00 = addmod(r00, mont_reduce(a00, P), P.q);
    r01 = addmod(r01, mont_reduce(a01, P), P.q);
    r10 = addmod(r10, mont_reduce(a10, P), P.q);
    r11 = addmod(r11, mont_reduce(a11, P), P.q);
  }
  if (t < J.n_dig) {
    const u64* c0 = J.c0 + (size_t)t * n;
    r00 = addmod(r00, shoup(c0[src0], J.pq[t], J.pq_sh[t], P.q), P.q);
    r01 = addmod(r01, shoup(c0[src1], J.pq[t], J.pq_sh[t], P.q), P.q);
  }
  u64* u0 = J.u + (((size_t)r * 2 + 0) * J.nm + t) * n + i;
  u64* u1 = J.u + (((size_t)r * 2 + 1) * J.nm + t) * n + i;
  __builtin_nontemporal_store(r00, u0);
  __builtin_nontemporal_store(r01, u0 + 1);
  __builtin_nontemporal_store(r10, u1);
  __builtin_nontemporal_store(r11, u1 + 1);
}

// s + sum_c p[c * stride] mod q, eight loads in flight at a time
__device__ __forceinline__ u64 add_partials(u64 s, const u64* __restrict__ p, long long stride, int n, u64 q) {
  int c = 0;
  for (; c + 8 <= n; c += 8) {
    u64 v[8];
#pragma unroll
    for (int m = 0; m < 8; m++) v[m] = p[(size_t)(c + m) * stride];
#pragma unroll
    for (int m = 0; m < 8; m++) s = addmod(s, v[m], q);
  }
  for (; c < n; c++) s = addmod(s, p[(size_t)c * stride], q);
  return s;
}

__global__ void k_mac_finish(int log_n, const u64* __restrict__ partial, int n_chunks, const u64* __restrict__ x,
                             const u64* __restrict__ diag0, u64* __restrict__ out, int n_dig,
                             const PrimeDev* __restrict__ primes) {
  const int n = 1 << log_n;
  const long long per = 2LL * n_dig * n;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= per) return;
  const int t = (int)((e >> log_n) % n_dig);
  const int i = (int)(e & (n - 1));
  const PrimeDev P = primes[t];
  u64 s = mulmod(x[e], diag0[(size_t)t * n + i], P);
  out[e] = add_partials(s, partial + e, per, n_chunks, P.q);
}

// out[k][t] = x[k][t] + sum_c partial[c][k][t] (the replication: no diagonal)
__global__ void k_rep_finish(int log_n, const u64* __restrict__ partial, int n_chunks, const u64* __restrict__ x,
                             u64* __restrict__ out, int n_dig, const PrimeDev* __restrict__ primes) {
  const int n = 1 << log_n;
  const long long per = 2LL * n_dig * n;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= per) return;
  const int t = (int)((e >> log_n) % n_dig);
  const u64 q = primes[t].q;
  out[e] = add_partials(x[e], partial + e, per, n_chunks, q);
}

inline dim3 grid_for(long long total) { return dim3((unsigned)((total + BLK - 1) / BLK)); }

}  // namespace

hipError_t launch_sample_small(int log_n, int kind, uint64_t seed, uint32_t tag, uint32_t a,
                               const ModList& mods, u64* out, const PrimeDev* primes, hipStream_t st) {
  const int n = 1 << log_n;
  hipLaunchKernelGGL(k_sample_small, grid_for(n / 8), dim3(BLK), 0, st, n, kind, seed, tag, a, mods, out,
                     primes);
  return hipGetLastError();
}

hipError_t launch_sample_uniform(int log_n, uint64_t seed, uint32_t tag, uint32_t a_base, int n_rows,
                                 const ModList& mods, const ModList& pidx, u64* out, const PrimeDev* primes,
                                 hipStream_t st) {
  const int n = 1 << log_n;
  const long long total = (long long)(n / 4) * n_rows * mods.n;
  hipLaunchKernelGGL(k_sample_uniform, grid_for(total), dim3(BLK), 0, st, n, seed, tag, a_base, n_rows, mods,
                     pidx, out, primes);
  return hipGetLastError();
}

hipError_t launch_addsub(int log_n, int op, const u64* a, const u64* b, u64* out, int n_poly,
                         const ModList& mods, const PrimeDev* primes, hipStream_t st) {
  const int n = 1 << log_n;
  const long long total = (long long)n_poly * mods.n * n;
  hipLaunchKernelGGL(k_addsub, grid_for(total), dim3(BLK), 0, st, n, op, a, b, out, total, mods.n, mods,
                     primes);
  return hipGetLastError();
}

hipError_t launch_mul_plain(int log_n, const u64* a, const u64* p, u64* out, int n_poly, const ModList& mods,
                            const PrimeDev* primes, hipStream_t st) {
  const int n = 1 << log_n;
  const long long total = (long long)n_poly * mods.n * n;
  hipLaunchKernelGGL(k_mul_plain, grid_for(total), dim3(BLK), 0, st, n, a, p, out, total, mods.n, mods,
                     primes);
  return hipGetLastError();
}

hipError_t launch_add_plain(int log_n, const u64* a, const u64* p, u64* out, int n_poly, const ModList& mods,
                            const PrimeDev* primes, hipStream_t st, int neg) {
  const int n = 1 << log_n;
  const long long total = (long long)n_poly * mods.n * n;
  hipLaunchKernelGGL(k_add_plain, grid_for(total), dim3(BLK), 0, st, n, a, p, out, total, mods.n, mods,
                     primes, neg);
  return hipGetLastError();
}

hipError_t launch_tensor(int log_n, const u64* a, const u64* b, u64* out01, u64* out2, const ModList& mods,
                         const PrimeDev* primes, hipStream_t st) {
  const int n = 1 << log_n;
  hipLaunchKernelGGL(k_tensor, grid_for((long long)mods.n * n), dim3(BLK), 0, st, n, a, b, out01, out2, mods.n,
                     mods, primes);
  return hipGetLastError();
}

hipError_t launch_tensor_many(int log_n, const CtList& a, const CtList& b, int B, u64* out01, u64* out2,
                              int n_limbs, const PrimeDev* primes, hipStream_t st) {
  const long long total = ((long long)B * n_limbs) << log_n;
  hipLaunchKernelGGL(k_tensor_many, grid_for(total), dim3(BLK), 0, st, log_n, a, b, out01, out2, n_limbs, total,
                     primes);
  return hipGetLastError();
}

hipError_t launch_gather_cts(int log_n, const CtList& a, int B, int n_limbs, u64* out, hipStream_t st) {
  const long long per = (2LL * n_limbs) << log_n;
  hipLaunchKernelGGL(k_gather_cts, grid_for(per * B), dim3(BLK), 0, st, a, out, per, per * B);
  return hipGetLastError();
}

hipError_t launch_mul_plain_many(int log_n, const CtList& in, const CtList& p, int B, int n_limbs, u64* out,
                                 const PrimeDev* primes, hipStream_t st) {
  const long long total = ((2LL * n_limbs) << log_n) * B;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mul_plain_many, grid_for(total), dim3(BLK), 0, st, log_n, in, p, n_limbs, out, total, primes);
  return hipGetLastError();
}

hipError_t launch_add_plain_many(int log_n, const CtList& in, const CtList& p, const OutList& out, int B,
                                 int n_limbs, const PrimeDev* primes, hipStream_t st) {
  const long long total = ((2LL * n_limbs) << log_n) * B;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_add_plain_many, grid_for(total), dim3(BLK), 0, st, log_n, in, p, out, n_limbs, total, primes);
  return hipGetLastError();
}

hipError_t launch_sum_cts(int log_n, const CtList& in, int B, int n_limbs, u64* out, const PrimeDev* primes,
                          hipStream_t st) {
  const long long total = (2LL * n_limbs) << log_n;
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sum_cts, grid_for(total), dim3(BLK), 0, st, log_n, in, B, n_limbs, out, total, primes);
  return hipGetLastError();
}

hipError_t launch_copy(const u64* src, u64* dst, long long words, hipStream_t st) {
  if (words <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy, grid_for(words), dim3(BLK), 0, st, src, dst, words);
  return hipGetLastError();
}

hipError_t launch_decrypt(int log_n, const u64* ct, const u64* s, u64* m, int n_limbs, const PrimeDev* primes,
                          hipStream_t st) {
  const int n = 1 << log_n;
  hipLaunchKernelGGL(k_decrypt, grid_for((long long)n_limbs * n), dim3(BLK), 0, st, n, ct, s, m, n_limbs,
                     primes);
  return hipGetLastError();
}

hipError_t launch_automorphism(int log_n, const u64* in, u64* out, const AutJob& job, hipStream_t st) {
  const long long total = ((long long)job.B * job.rows_per_item) << log_n;
  hipLaunchKernelGGL(k_automorphism, grid_for(total), dim3(BLK), 0, st, log_n, in, out, total, job);
  return hipGetLastError();
}

hipError_t launch_inner(int log_n, const InnerJob& job, const PrimeDev* primes, hipStream_t st) {
  const long long total = ((long long)job.B * (job.n_dig + 1)) << log_n;
  hipLaunchKernelGGL(k_inner, grid_for(total), dim3(BLK), 0, st, log_n, job, primes);
  return hipGetLastError();
}

hipError_t launch_keygen_combine(int log_n, const u64* a, const u64* e, const u64* s, const u64* sp, u64* key,
                                 int nd, int nm, const ModList& pidx, int special_prime, const PrimeDev* primes,
                                 hipStream_t st) {
  const int n = 1 << log_n;
  hipLaunchKernelGGL(k_keygen_combine, grid_for((long long)nd * nm * n), dim3(BLK), 0, st, n, a, e, s, sp, key,
                     nd, nm, pidx, special_prime, primes);
  return hipGetLastError();
}

hipError_t launch_pk_combine(int log_n, const u64* a, const u64* e, const u64* s, u64* out, int limbs,
                             const PrimeDev* primes, hipStream_t st) {
  const int n = 1 << log_n;
  hipLaunchKernelGGL(k_pk_combine, grid_for((long long)limbs * n), dim3(BLK), 0, st, n, a, e, s, out, limbs,
                     primes);
  return hipGetLastError();
}

hipError_t launch_encrypt_combine(int log_n, const u64* v, const u64* pk0, const u64* pk1, const u64* e0,
                                  const u64* e1, const u64* s, const u64* m, u64* ct, int n_limbs, int pk_limbs,
                                  const PrimeDev* primes, hipStream_t st) {
  const int n = 1 << log_n;
  hipLaunchKernelGGL(k_encrypt_combine, grid_for((long long)n_limbs * n), dim3(BLK), 0, st, n, v, pk0, pk1, e0,
                     e1, s, m, ct, n_limbs, pk_limbs, primes);
  return hipGetLastError();
}

hipError_t launch_from_mont(int log_n, u64* data, int n_rows, const ModList& mods, const PrimeDev* primes,
                            hipStream_t st) {
  const long long total = (long long)n_rows << log_n;
  hipLaunchKernelGGL(k_mont, grid_for(total), dim3(BLK), 0, st, 1 << log_n, data, total, 0, mods, primes);
  return hipGetLastError();
}

// ---- exact encoding of the coefficients the FP64 FFT's bound cannot round:
// 2 scale / N * sum_j z_j cos(pi t_jk / N), t_jk = 5^j k mod 2N, in
// double-double (error-free sums and FMA products), rounded half away from
// zero.  One workgroup per coefficient.
struct DD {
  double hi, lo;
};
__device__ __forceinline__ DD dd_two_sum(double a, double b) {
  const double s = a + b, bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__device__ __forceinline__ DD dd_fast_sum(double a, double b) {
  const double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ DD dd_plus(DD a, DD b) {
  DD s = dd_two_sum(a.hi, b.hi);
  const DD t = dd_two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = dd_fast_sum(s.hi, s.lo);
  s.lo += t.lo;
  return dd_fast_sum(s.hi, s.lo);
}
// nearest integer of a non-negative double-double, halves up
__device__ __forceinline__ long long dd_round(DD a) {
  if (a.hi >= 4503599627370496.0) {  // 2^52: hi is an integer
    const double fl = floor(a.lo);
    return (long long)a.hi + (long long)fl + (a.lo - fl >= 0.5 ? 1 : 0);
  }
  const double fi = floor(a.hi);
  const DD s = dd_two_sum(a.hi - fi, a.lo);  // the exact fraction
  double F = floor(s.hi);
  if (s.hi == F && s.lo < 0) F -= 1.0;
  const double d = (s.hi - F) - 0.5;
  const bool up = d > 0 || (d == 0 && s.lo >= 0);
  return (long long)fi + (long long)F + (up ? 1 : 0);
}

constexpr int kEncT = 256;
__global__ void __launch_bounds__(kEncT) k_encode_exact(int log_n, const double* __restrict__ z, int nz,
                                                        const uint32_t* __restrict__ rot5,
                                                        const double* __restrict__ chi,
                                                        const double* __restrict__ clo, const int* __restrict__ amb,
                                                        double twice, int64_t* __restrict__ co) {
  __shared__ double sh[kEncT], sl[kEncT];
  const int k = amb[blockIdx.x];
  const uint32_t mask = (2u << log_n) - 1u;
  DD acc = {0.0, 0.0};
  for (int j = threadIdx.x; j < nz; j += kEncT) {
    const double zj = z[j];
    if (zj == 0.0) continue;
    const uint32_t t = (uint32_t)(((uint64_t)rot5[j] * (uint64_t)k) & mask);
    const double ph = zj * chi[t];
    double pl = fma(zj, chi[t], -ph);
    pl += zj * clo[t];
    acc = dd_plus(acc, dd_fast_sum(ph, pl));
  }
  sh[threadIdx.x] = acc.hi;
  sl[threadIdx.x] = acc.lo;
  __syncthreads();
  for (int w = kEncT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const DD r = dd_plus(DD{sh[threadIdx.x], sl[threadIdx.x]}, DD{sh[threadIdx.x + w], sl[threadIdx.x + w]});
      sh[threadIdx.x] = r.hi;
      sl[threadIdx.x] = r.lo;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // times 2 scale / N (a power of two times scale: one more product)
    const double ph = sh[0] * twice;
    double pl = fma(sh[0], twice, -ph);
    pl += sl[0] * twice;
    DD a = dd_fast_sum(ph, pl);
    const bool neg = a.hi < 0 || (a.hi == 0 && a.lo < 0);
    if (neg) a = DD{-a.hi, -a.lo};
    const long long mag = dd_round(a);
    co[k] = neg ? -mag : mag;
  }
}

hipError_t launch_encode_exact(int log_n, const double* z, int nz, const uint32_t* rot5, const double* chi,
                               const double* clo, const int* amb, int n_amb, double twice, int64_t* co,
                               hipStream_t st) {
  if (n_amb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_encode_exact, dim3(n_amb), dim3(kEncT), 0, st, log_n, z, nz, rot5, chi, clo, amb, twice, co);
  return hipGetLastError();
}

// signed coefficients (|v| < 2^62) into the residues of limbs 0..n_limbs-1
__global__ void k_coeffs_to_limbs(int log_n, const int64_t* __restrict__ co, u64* __restrict__ out, long long total,
                                  const PrimeDev* __restrict__ primes) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  out[e] = red_signed(co[e & ((1LL << log_n) - 1)], primes[e >> log_n]);
}

hipError_t launch_coeffs_to_limbs(int log_n, const int64_t* co, u64* out, int n_limbs, const PrimeDev* primes,
                                  hipStream_t st) {
  const long long total = (long long)n_limbs << log_n;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coeffs_to_limbs, grid_for(total), dim3(BLK), 0, st, log_n, co, out, total, primes);
  return hipGetLastError();
}

hipError_t launch_to_mont(int log_n, u64* data, int n_rows, const ModList& mods, const PrimeDev* primes,
                          hipStream_t st) {
  const long long total = (long long)n_rows << log_n;
  hipLaunchKernelGGL(k_mont, grid_for(total), dim3(BLK), 0, st, 1 << log_n, data, total, 1, mods, primes);
  return hipGetLastError();
}

hipError_t launch_inner_hoisted(int log_n, const HoistInner& job, const PrimeDev* primes, hipStream_t st) {
  // two words per thread
  const long long total = ((long long)job.R * (job.t_end - job.t_begin)) << (log_n - 1);
  if (total == 0) return hipSuccess;
  hipLaunchKernelGGL(k_inner_hoisted, grid_for(total), dim3(BLK), 0, st, log_n, job, primes);
  return hipGetLastError();
}

hipError_t launch_mac_finish(int log_n, const u64* partial, int n_chunks, const u64* x, const u64* diag0, u64* out,
                             int n_dig, const PrimeDev* primes, hipStream_t st) {
  const long long total = (2LL * n_dig) << log_n;
  if (diag0)
    hipLaunchKernelGGL(k_mac_finish, grid_for(total), dim3(BLK), 0, st, log_n, partial, n_chunks, x, diag0, out,
                       n_dig, primes);
  else
    hipLaunchKernelGGL(k_rep_finish, grid_for(total), dim3(BLK), 0, st, log_n, partial, n_chunks, x, out, n_dig,
                       primes);
  return hipGetLastError();
}
