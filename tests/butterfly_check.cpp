// Range and congruence checks of the library's NTT butterfly arithmetics
// (paper_2104_03152_amd/csrc/butterfly.h), run on the host against exact
// 128-bit integer arithmetic.  Usage: butterfly_check q1 q2 ...  Prints one
// line per prime and "ok" or the first failures; exits non-zero on failure.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "../paper_2104_03152_amd/csrc/butterfly.h"

typedef __int128 i128;
typedef unsigned __int128 u128;

static long long failures = 0;
static void bad(const char* what, u64 q, double a, double b, double w) {
  if (++failures <= 20) std::printf("FAIL %s q=%llu a=%.0f b=%.0f w=%.0f\n", what, (unsigned long long)q, a, b, w);
}
static i128 mod(i128 a, i128 q) {
  i128 r = a % q;
  return r < 0 ? r + q : r;
}
static bool is_int(double v) { return v == (double)(long long)v; }

static PrimeDev prime_dev(u64 q) {
  PrimeDev d{};
  d.q = q;
  d.qd = (double)q;
  d.inv2qd = 1.0 / (2.0 * (double)q);
  return d;
}

// floor(y w / q) exactly
static long long true_quot(long long y, u64 w, u64 q) {
  i128 p = (i128)y * (i128)w;
  i128 qq = (i128)q;
  i128 f = p / qq;
  if (p % qq != 0 && p < 0) f -= 1;
  return (long long)f;
}

static long long off_by_one = 0;

static void check_fp(u64 q, std::mt19937_64& rng) {
  const PrimeDev P = prime_dev(q);
  const FpAr ar(P);
  const long long Q = (long long)q;
  // multiplicands at the extremes of every input range the butterflies see
  std::vector<long long> ys = {-2 * Q, -2 * Q + 1, -Q - 1, -Q, -Q + 1, -2, -1, 0, 1, 2, Q - 1, Q, Q + 1,
                               2 * Q - 1, 2 * Q, 2 * Q + 1, 3 * Q, 4 * Q - 1, 4 * Q};
  std::vector<u64> ws = {0, 1, 2, q - 1, q - 2, q / 2, q / 3 + 1};
  for (int i = 0; i < 24; i++) ws.push_back(rng() % q);
  // adversarial multiplicands: y w mod q in {0, 1, q - 1}, so y w / q sits
  // next to an integer and the floating quotient estimate can miss by one
  std::vector<long long> yadv;
  for (u64 w : ws) {
    if (w == 0) continue;
    const u64 winv = [&] {  // w^-1 mod q (q prime)
      u64 r = 1, b = w, e = q - 2;
      while (e) {
        if (e & 1) r = (u64)((u128)r * b % q);
        b = (u64)((u128)b * b % q);
        e >>= 1;
      }
      return r;
    }();
    for (u64 t : {(u64)0, (u64)1, q - 1, (u64)2, q - 2}) {
      const long long y0 = (long long)((u128)t * winv % q);
      for (long long m = -2; m <= 3; m++) yadv.push_back(y0 + m * Q);
    }
  }
  for (u64 w : ws) {
    const double wd = (double)w, wq = (double)w / (double)q;
    auto run = [&](long long y) {
      if (y <= -2 * Q - 1 || y >= 4 * Q + 1) return;
      const double r = ar.mul((double)y, wd, wq);
      if (!is_int(r) || !(r > -(double)Q && r < 2.0 * (double)Q) ||
          mod((i128)(long long)r - (i128)y * (i128)w, Q) != 0)
        bad("FpAr.mul", q, (double)y, 0, wd);
      if ((long long)__builtin_floor((double)y * wq) != true_quot(y, w, q)) off_by_one++;
    };
    for (long long y : ys) run(y);
    for (long long y : yadv) run(y);
    for (int i = 0; i < 64; i++) run((long long)(rng() % (u64)(6 * Q + 1)) - 2 * Q);
  }
  // fold over the whole |x| < 2^52 range, next to multiples of 2q
  const long long LIM = (1LL << 52) - 1;
  std::vector<long long> xs = {-LIM, LIM, 0, -1, 1};
  for (long long k : {-(LIM / (2 * Q)), -3LL, -1LL, 0LL, 1LL, 2LL, LIM / (2 * Q)})
    for (long long d = -2; d <= 2; d++) xs.push_back(k * 2 * Q + d);
  for (int i = 0; i < 256; i++) xs.push_back((long long)(rng() % (u64)(2 * LIM + 1)) - LIM);
  for (long long x : xs) {
    if (x < -LIM || x > LIM) continue;
    const double f = ar.fold((double)x);
    if (!is_int(f) || f < -1.0 || f > 2.0 * (double)Q + 1.0 || mod((i128)(long long)f - x, 2 * (i128)Q) != 0)
      bad("FpAr.fold", q, (double)x, 0, 0);
  }
  // forward butterfly: inputs in (-2q - 1, 4q + 1) stay there
  std::vector<long long> in_f = {-2 * Q, -2 * Q + 1, -Q, -1, 0, 1, Q - 1, 2 * Q, 2 * Q + 1, 3 * Q, 4 * Q - 1, 4 * Q};
  std::vector<long long> in_i = {-Q + 1, -1, 0, 1, Q - 1, Q, 2 * Q - 1, 2 * Q, 2 * Q + 1};
  for (u64 w : ws) {
    const double2 tw = make_double2((double)w, (double)w / (double)q);
    for (long long X : in_f)
      for (long long Y : in_f) {
        double a = (double)X, b = (double)Y;
        ar.fwd(a, b, tw);
        const bool rng_ok = a > -2.0 * (double)Q - 1 && a < 4.0 * (double)Q + 1 && b > -2.0 * (double)Q - 1 &&
                            b < 4.0 * (double)Q + 1;
        if (!is_int(a) || !is_int(b) || !rng_ok || mod((i128)(long long)a - X - (i128)Y * w, Q) != 0 ||
            mod((i128)(long long)b - X + (i128)Y * w, Q) != 0)
          bad("FpAr.fwd", q, (double)X, (double)Y, (double)w);
      }
    // inverse butterfly: inputs in (-q, 2q + 1]; X' in [-1, 2q + 1], Y' in (-q, 2q)
    for (long long X : in_i)
      for (long long Y : in_i) {
        double a = (double)X, b = (double)Y;
        ar.inv(a, b, tw);
        const bool rng_ok = a >= -1.0 && a <= 2.0 * (double)Q + 1 && b > -(double)Q && b < 2.0 * (double)Q;
        if (!is_int(a) || !is_int(b) || !rng_ok || mod((i128)(long long)a - X - Y, Q) != 0 ||
            mod((i128)(long long)b - (i128)(X - Y) * w, Q) != 0)
          bad("FpAr.inv", q, (double)X, (double)Y, (double)w);
      }
  }
  // final conversion: integer-valued doubles in [-q, 3q) to [0, q)
  for (long long v : {-Q, -Q + 1, -1LL, 0LL, 1LL, Q - 1, Q, 2 * Q, 3 * Q - 1}) {
    const u64 r = ar.to_res((double)v);
    if (r >= q || (i128)r != mod(v, Q)) bad("FpAr.to_res", q, (double)v, 0, 0);
  }
}

static void check_int(u64 q, std::mt19937_64& rng) {
  const PrimeDev P = prime_dev(q);
  const IntAr ar(P);
  std::vector<u64> ws = {0, 1, 2, q - 1, q - 2, q / 2};
  for (int i = 0; i < 24; i++) ws.push_back(rng() % q);
  std::vector<u64> in_f = {0, 1, q - 1, q, 2 * q - 1, 2 * q, 3 * q, 4 * q - 1};
  std::vector<u64> in_i = {0, 1, q - 1, q, 2 * q - 1};
  for (int i = 0; i < 8; i++) in_f.push_back(rng() % (4 * q));
  for (int i = 0; i < 8; i++) in_i.push_back(rng() % (2 * q));
  for (u64 w : ws) {
    const u64 wsh = (u64)(((u128)w << 64) / q);
    const ulonglong2 tw = make_ulonglong2(w, wsh);
    for (u64 X : in_f)
      for (u64 Y : in_f) {
        u64 a = X, b = Y;
        ar.fwd(a, b, tw);
        if (a >= 4 * q || b >= 4 * q || (u128)a % q != ((u128)X + (u128)Y * w) % q ||
            (u128)b % q != (u128)mod((i128)X - (i128)Y * w, q))
          bad("IntAr.fwd", q, (double)X, (double)Y, (double)w);
      }
    for (u64 X : in_i)
      for (u64 Y : in_i) {
        u64 a = X, b = Y;
        ar.inv(a, b, tw);
        if (a >= 2 * q || b >= 2 * q || (u128)a % q != ((u128)X + Y) % q ||
            (u128)b % q != (u128)mod(((i128)X - (i128)Y) * (i128)w, q))
          bad("IntAr.inv", q, (double)X, (double)Y, (double)w);
      }
  }
  for (u64 v : in_f) {
    const u64 r = ar.fwd_res(v);
    if (r >= q || r != v % q) bad("IntAr.fwd_res", q, (double)v, 0, 0);
  }
}

int main(int argc, char** argv) {
  std::mt19937_64 rng(20210407);
  for (int i = 1; i < argc; i++) {
    const u64 q = std::strtoull(argv[i], nullptr, 10);
    const long long before = failures;
    if (q < (1ull << 50)) check_fp(q, rng);
    check_int(q, rng);
    std::printf("%llu %s %s\n", (unsigned long long)q, q < (1ull << 50) ? "fp+int" : "int",
                failures == before ? "ok" : "FAILED");
  }
  std::printf("quotient estimates off by one: %lld\n", off_by_one);
  std::printf("%s\n", failures ? "FAILED" : "ALL OK");
  return failures ? 1 : 0;
}
