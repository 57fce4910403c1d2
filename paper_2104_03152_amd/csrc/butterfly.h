// butterfly.h -- the two NTT butterfly arithmetics, host- and device-callable
// (the host build serves the range tests of the arithmetic on the CPU).
//
// IntAr: 64-bit words, Harvey's lazy butterflies with Shoup twiddles
// (forward values in [0, 4q), inverse in [0, 2q)), for primes of 50 bits and
// more.  FpAr: residues held as integer-valued doubles for primes below
// 2^50; every operation is exact (all intermediates are integers below
// 2^53), so its results equal the integer path's bit for bit after the
// final reduction.
#pragma once
#include "modarith.h"

// ---------------- butterfly arithmetics ----------------
struct IntAr {
  typedef u64 T;
  typedef ulonglong2 TW;  // (w, floor(w 2^64 / q))
  u64 q, q2;
  __host__ __device__ explicit IntAr(const PrimeDev& P) : q(P.q), q2(P.q << 1) {}
  // inputs in [0, 4q): X reduced to [0, 2q), outputs in [0, 4q)
  __host__ __device__ __forceinline__ void fwd(T& X, T& Y, const TW w) const {
    const u64 x = X >= q2 ? X - q2 : X;
    const u64 v = shoup_lazy(Y, w.x, w.y, q);
    X = x + v;
    Y = x - v + q2;
  }
  // inputs and outputs in [0, 2q)
  __host__ __device__ __forceinline__ void inv(T& X, T& Y, const TW w) const {
    const u64 s = X + Y;
    const u64 d = X - Y + q2;
    X = s >= q2 ? s - q2 : s;
    Y = shoup_lazy(d, w.x, w.y, q);
  }
  __host__ __device__ __forceinline__ T from_res(u64 v) const { return v; }
  __host__ __device__ __forceinline__ u64 fwd_res(T v) const {
    v = v >= q2 ? v - q2 : v;
    return v >= q ? v - q : v;
  }
  __host__ __device__ __forceinline__ u64 inv_res(T v, const PrimeDev& P) const { return shoup(v, P.ninv, P.ninv_sh, q); }
  static __host__ __device__ __forceinline__ u64 bits(T v) { return v; }
  static __host__ __device__ __forceinline__ T unbits(u64 b) { return b; }
};

struct FpAr {
  typedef double T;
  typedef double2 TW;  // (w, w / q)
  double q, q2, inv2q;
  long long qi;
  __host__ __device__ explicit FpAr(const PrimeDev& P) : q(P.qd), q2(2.0 * P.qd), inv2q(P.inv2qd), qi((long long)P.q) {}
  // y w mod q in (-q, 2q) for |y w / q| < 2^52, 0 <= w < q < 2^50
  __host__ __device__ __forceinline__ double mul(double y, double w, double wq) const {
#pragma clang fp contract(off)
    const double h = y * w;
    const double l = __builtin_fma(y, w, -h);
    const double qt = __builtin_floor(y * wq);
    return __builtin_fma(-qt, q, h) + l;
  }
  // x - 2q floor(x / 2q), in [-1, 2q + 1] for |x| < 2^52
  __host__ __device__ __forceinline__ double fold(double x) const {
#pragma clang fp contract(off)
    return __builtin_fma(-__builtin_floor(x * inv2q), q2, x);
  }
  // inputs in (-2q - 1, 4q + 1); X folded first, outputs in the same range
  __host__ __device__ __forceinline__ void fwd(T& X, T& Y, const TW w) const {
#pragma clang fp contract(off)
    const double x = fold(X);
    const double v = mul(Y, w.x, w.y);
    X = x + v;
    Y = x - v;
  }
  // inputs in (-q, 2q + 1]; outputs: X in [-1, 2q + 1], Y in (-q, 2q)
  __host__ __device__ __forceinline__ void inv(T& X, T& Y, const TW w) const {
#pragma clang fp contract(off)
    const double a = X + Y, b = X - Y;
    X = fold(a);
    Y = mul(b, w.x, w.y);
  }
  __host__ __device__ __forceinline__ T from_res(u64 v) const { return (double)(long long)v; }
  // an integer-valued double in [-q, 3q) -> [0, q)
  __host__ __device__ __forceinline__ u64 to_res(double v) const {
    long long t = (long long)v;
    t += t < 0 ? qi : 0;
    t -= t >= qi ? qi : 0;
    t -= t >= qi ? qi : 0;
    return (u64)t;
  }
  __host__ __device__ __forceinline__ u64 fwd_res(T v) const { return to_res(fold(v)); }
  __host__ __device__ __forceinline__ u64 inv_res(T v, const PrimeDev& P) const { return to_res(mul(v, P.ninv_d, P.ninv_qd)); }
  static __host__ __device__ __forceinline__ u64 bits(T v) { return __builtin_bit_cast(u64, v); }
  static __host__ __device__ __forceinline__ T unbits(u64 b) { return __builtin_bit_cast(double, b); }
};

