// modarith.h -- 64-bit modular arithmetic for gfx950 built from 32x32->64
// multiplies (CDNA4 has no 64x64->128 integer multiply).  Primes are below
// 2^61, so lazy values up to 4q fit in a word.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef int64_t i64;

// Per-prime constants, resident in device memory.
struct PrimeDev {
  u64 q;
  u64 mu;        // floor(2^(2k) / q), k = bit length of q (HAC 14.42 Barrett)
  u64 mu64;      // floor((2^64 - 1) / q): one-word reduction
  u64 qinv_neg;  // -q^-1 mod 2^64 (Montgomery)
  u64 r2;        // 2^128 mod q (into Montgomery form)
  u64 ninv, ninv_sh;  // N^-1 mod q and its Shoup companion
  u32 k;         // bit length of q
  u32 use_fp;    // q < 2^50: the NTT runs in exact FP64 arithmetic
  double qd, inv2qd;  // q and 1/(2q) as doubles
  double ninv_d, ninv_qd;  // N^-1 mod q and N^-1 / q as doubles
};

struct U128 {
  u64 lo, hi;
};

// full 64x64 -> 128 product as a chain of 32x32+64 multiply-adds
__device__ __forceinline__ U128 mul_wide(u64 a, u64 b) {
  const u32 a0 = (u32)a, a1 = (u32)(a >> 32), b0 = (u32)b, b1 = (u32)(b >> 32);
  const u64 t = (u64)a0 * b0;
  const u64 x = (u64)a1 * b0 + (t >> 32);
  const u64 y = (u64)a0 * b1 + (u32)x;
  U128 r;
  r.lo = (y << 32) | (u32)t;
  r.hi = (u64)a1 * b1 + (x >> 32) + (y >> 32);
  return r;
}

// high word of a 64x64 product as a chain of 32x32+64 multiply-adds
// (v_mad_u64_u32): the partial carries ride in the 64-bit addend.
__host__ __device__ __forceinline__ u64 mulhi64(u64 a, u64 b) {
  const u32 a0 = (u32)a, a1 = (u32)(a >> 32), b0 = (u32)b, b1 = (u32)(b >> 32);
  const u64 t = (u64)a0 * b0;
  const u64 x = (u64)a1 * b0 + (t >> 32);
  const u64 y = (u64)a0 * b1 + (u32)x;
  return (u64)a1 * b1 + (x >> 32) + (y >> 32);
}

__device__ __forceinline__ U128 add128(U128 a, U128 b) {
  U128 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo ? 1 : 0);
  return r;
}

// x < q^2 (x < 2^(2k)) -> x mod q.  q1 = x >> (k-1), q3 = (q1 mu) >> (k+1),
// r = x - q3 q in [0, 3q).
__device__ __forceinline__ u64 barrett_reduce(U128 x, const PrimeDev& P) {
  const u32 k = P.k;
  u64 q1 = (x.hi << (65 - k)) | (x.lo >> (k - 1));
  U128 t = mul_wide(q1, P.mu);
  u64 q3 = (t.hi << (63 - k)) | (t.lo >> (k + 1));
  u64 r = x.lo - q3 * P.q;
  r = r >= P.q ? r - P.q : r;
  r = r >= P.q ? r - P.q : r;
  return r;
}

__device__ __forceinline__ u64 mulmod(u64 a, u64 b, const PrimeDev& P) {
  return barrett_reduce(mul_wide(a, b), P);
}

// any 64-bit x -> x mod q (qhat = floor(x mu64 / 2^64) is within 1 of x / q)
__device__ __forceinline__ u64 red64(u64 x, const PrimeDev& P) {
  u64 qh = mulhi64(x, P.mu64);
  u64 r = x - qh * P.q;
  return r >= P.q ? r - P.q : r;
}

// Shoup: w < q, ws = floor(w 2^64 / q); a < 2^64 -> a w mod q in [0, 2q)
__host__ __device__ __forceinline__ u64 shoup_lazy(u64 a, u64 w, u64 ws, u64 q) {
  u64 qh = mulhi64(a, ws);
  return a * w - qh * q;
}
__host__ __device__ __forceinline__ u64 shoup(u64 a, u64 w, u64 ws, u64 q) {
  u64 r = shoup_lazy(a, w, ws, q);
  return r >= q ? r - q : r;
}

// Montgomery: x < q 2^64 -> x 2^-64 mod q
__device__ __forceinline__ u64 mont_reduce(U128 x, const PrimeDev& P) {
  u64 m = x.lo * P.qinv_neg;
  U128 mq = mul_wide(m, P.q);
  // x + m q is divisible by 2^64; its high word is the result (< 2q)
  u64 carry = (x.lo + mq.lo) < x.lo ? 1 : 0;
  u64 r = x.hi + mq.hi + carry;
  return r >= P.q ? r - P.q : r;
}

__device__ __forceinline__ u64 addmod(u64 a, u64 b, u64 q) {
  u64 s = a + b;
  return s >= q ? s - q : s;
}
__device__ __forceinline__ u64 submod(u64 a, u64 b, u64 q) {
  return a >= b ? a - b : a + q - b;
}

// a signed small integer (|v| < 2^62) into [0, q)
__device__ __forceinline__ u64 red_signed(i64 v, const PrimeDev& P) {
  if (v >= 0) return red64((u64)v, P);
  u64 r = red64((u64)(-v), P);
  return r ? P.q - r : 0;
}

__device__ __forceinline__ u32 bitrev(u32 x, int bits) {
  return __builtin_bitreverse32(x) >> (32 - bits);
}

// NTT slot i holds a(psi^(2 brv(i) + 1)) (bit-reversed evaluation order), so
// X -> X^g reads slot brv(((2 brv(i) + 1) g mod 2N - 1) / 2).  For 64
// consecutive aligned slots the sources are a permutation of one aligned
// 64-slot block (the map is affine in the reversed index), so the gather
// stays coalesced.
__device__ __forceinline__ int gal_src(int i, int log_n, u64 g) {
  const u32 n2mask = (2u << log_n) - 1u;
  const u32 e = ((2u * bitrev((u32)i, log_n) + 1u) * (u32)g) & n2mask;
  return (int)bitrev((e - 1u) >> 1, log_n);
}
