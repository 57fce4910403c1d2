// encode.cpp -- host-side CKKS encoding and decoding (canonical embedding).
//
// Slot j of a CKKSVector (N/2 reals) is the value of the plaintext polynomial
// at zeta^(5^j), zeta = exp(i pi / N).  Encoding inverts the embedding with
// one complex FFT of size N:
//   m_k = (1/N) zeta^-k sum_r G_r exp(-2 pi i r k / N),
// where G_r is the slot value sitting at the odd exponent 2r + 1 (z_j at
// 5^j, its conjugate at -5^j).  Coefficients are round(scale * m_k), ties
// away from zero.  The FFT result carries a proven error bound; any
// coefficient the bound cannot place on one side of a rounding boundary is
// recomputed as an exact-enough double-double sum
//   m_k = (2/N) sum_j z_j cos(pi (5^j k mod 2N) / N),
// so the integer coefficients are the correctly rounded ones.
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <atomic>
#include <thread>
#include <vector>

#include "encode.h"

namespace {

// ---- double-double arithmetic ----
struct dd {
  double hi, lo;
};
inline dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
inline dd quick_two_sum(double a, double b) {
  double s = a + b;
  return {s, b - (s - a)};
}
inline dd two_prod(double a, double b) {
  double p = a * b;
  return {p, std::fma(a, b, -p)};
}
inline dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}
inline dd dd_mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return quick_two_sum(p.hi, p.lo);
}
inline dd dd_mul_d(dd a, double b) {
  dd p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return quick_two_sum(p.hi, p.lo);
}
inline dd dd_div_d(dd a, double b) {
  double q1 = a.hi / b;
  dd p = two_prod(q1, b);
  double r = ((a.hi - p.hi) - p.lo + a.lo) / b;
  return quick_two_sum(q1, r);
}

const dd kPi = {3.141592653589793116e+00, 1.224646799147353207e-16};

// cos and sin of x in [0, pi/4] by their Taylor series in double-double
void dd_cos_sin(dd x, dd* c, dd* s) {
  dd x2 = dd_mul(x, x);
  dd term = {1.0, 0.0}, cs = {1.0, 0.0};
  for (int k = 1; k <= 20; k++) {
    term = dd_div_d(dd_mul(term, x2), (double)((2 * k - 1) * (2 * k)));
    dd t = {-term.hi, -term.lo};
    cs = dd_add(cs, (k & 1) ? t : term);
  }
  term = x;
  dd sn = x;
  for (int k = 1; k <= 20; k++) {
    term = dd_div_d(dd_mul(term, x2), (double)((2 * k) * (2 * k + 1)));
    dd t = {-term.hi, -term.lo};
    sn = dd_add(sn, (k & 1) ? t : term);
  }
  *c = cs;
  *s = sn;
}

// sign of (fractional part of a) - 1/2 decided exactly for a = hi + lo >= 0
// given as a normalised double-double; returns round-half-up of a.
int64_t round_dd_nonneg(dd a) {
  if (a.hi >= 4503599627370496.0) {  // 2^52: hi is an integer
    double fl = std::floor(a.lo);
    double fr = a.lo - fl;
    return (int64_t)a.hi + (int64_t)fl + (fr >= 0.5 ? 1 : 0);
  }
  double fi = std::floor(a.hi);
  dd s = two_sum(a.hi - fi, a.lo);  // exact fraction, s.hi in [-1/2, 3/2)
  double F = std::floor(s.hi);
  if (s.hi == F && s.lo < 0) F -= 1.0;
  double d = (s.hi - F) - 0.5;
  bool up = d > 0 || (d == 0 && s.lo >= 0);
  return (int64_t)fi + (int64_t)F + (up ? 1 : 0);
}

void fft(std::vector<std::complex<double>>& a, const EncodeTables& T, bool inverse_sign) {
  const int n = T.n;
  for (int i = 0; i < n; i++) {
    int j = (int)T.brv[i];
    if (j > i) std::swap(a[i], a[j]);
  }
  for (int len = 2; len <= n; len <<= 1) {
    const int half = len >> 1, step = n / len;
    for (int i = 0; i < n; i += len)
      for (int j = 0; j < half; j++) {
        std::complex<double> w = T.w[(size_t)j * step];
        if (inverse_sign) w = std::conj(w);
        std::complex<double> u = a[i + j], v = a[i + j + half] * w;
        a[i + j] = u + v;
        a[i + j + half] = u - v;
      }
  }
}

}  // namespace

void encode_tables_init(EncodeTables& T, int log_n) {
  const int n = 1 << log_n;
  T.log_n = log_n;
  T.n = n;
  T.chi.assign(2 * (size_t)n, 0.0);
  T.clo.assign(2 * (size_t)n, 0.0);
  // cos(pi u / N) for u in [0, N/2] from x <= pi/4 by symmetry
  std::vector<dd> quarter((size_t)n / 2 + 1);
  for (int u = 0; u <= n / 2; u++) {
    dd c, s;
    if (u <= n / 4) {
      dd x = dd_div_d(dd_mul_d(kPi, (double)u), (double)n);
      dd_cos_sin(x, &c, &s);
      quarter[u] = c;
    } else {
      dd x = dd_div_d(dd_mul_d(kPi, (double)(n / 2 - u)), (double)n);
      dd_cos_sin(x, &c, &s);
      quarter[u] = s;
    }
  }
  for (int t = 0; t < 2 * n; t++) {
    int u = t;
    if (u > n) u = 2 * n - u;  // cos(pi (2N - u)/N) = cos(pi u / N), u in [0, N]
    dd v;
    if (u <= n / 2) {
      v = quarter[u];
    } else {
      dd w = quarter[n - u];  // cos(pi u/N) = -cos(pi (N - u)/N)
      v = {-w.hi, -w.lo};
    }
    T.chi[t] = v.hi;
    T.clo[t] = v.lo;
  }
  T.rot5.resize((size_t)n / 2);
  uint32_t p = 1;
  for (int j = 0; j < n / 2; j++) {
    T.rot5[j] = p;
    p = (uint32_t)((uint64_t)p * 5 % (2 * (uint64_t)n));
  }
  T.brv.resize(n);
  for (int i = 0; i < n; i++) {
    uint32_t r = 0;
    for (int b = 0; b < log_n; b++) r |= ((uint32_t)(i >> b) & 1u) << (log_n - 1 - b);
    T.brv[i] = r;
  }
  // w_k = exp(-2 pi i k / N) = cos(pi 2k / N) - i sin(pi 2k / N)
  T.w.resize((size_t)n / 2);
  for (int k = 0; k < n / 2; k++) {
    double c = T.chi[(2 * (size_t)k) % (2 * n)];
    // sin(pi 2k/N) = cos(pi (N/2 - 2k)/N)
    long long u = (long long)n / 2 - 2LL * k;
    u %= 2LL * n;
    if (u < 0) u += 2LL * n;
    double s = T.chi[(size_t)u];
    T.w[k] = std::complex<double>(c, -s);
  }
  // zeta^k = exp(i pi k / N), k < N
  T.zeta.resize(n);
  for (int k = 0; k < n; k++) {
    long long u = (long long)n / 2 - k;
    u %= 2LL * n;
    if (u < 0) u += 2LL * n;
    T.zeta[k] = std::complex<double>(T.chi[k], T.chi[(size_t)u]);
  }
}

int encode_coeffs(const EncodeTables& T, const double* z, size_t nz, double scale, int64_t* out,
                  std::vector<int>* amb_out) {
  const int n = T.n;
  if (nz > (size_t)n / 2) return -2;
  double sumabs = 0;
  for (size_t j = 0; j < nz; j++) {
    if (!std::isfinite(z[j])) return -2;
    sumabs += std::fabs(z[j]);
  }
  std::vector<std::complex<double>> G((size_t)n, 0.0);
  const uint64_t two_n = 2 * (uint64_t)n;
  for (size_t j = 0; j < nz; j++) {
    const uint64_t e = T.rot5[j];
    G[(e - 1) / 2] += z[j];
    G[(two_n - e - 1) / 2] += z[j];
  }
  fft(G, T, false);
  const double fac = scale / (double)n;
  // error bound: log2(N) radix-2 levels of complex rounding (< 8 ulp each,
  // twiddles included) on partial sums bounded by ||G||_1 = 2 sum|z|, plus
  // the twist and scaling; doubled
  const double eps = std::ldexp(1.0, -53);
  const double fft_bound = 2.0 * fac * (2.0 * sumabs) * (8.0 * (T.log_n + 2)) * eps;
  const double twice = 2.0 * scale / (double)n;
  std::vector<int> amb;  // coefficients the bound cannot round
  for (int k = 0; k < n; k++) {
    std::complex<double> zk = std::conj(T.zeta[k]);
    double v = (G[k] * zk).real() * fac;
    double av = std::fabs(v);
    double bound = fft_bound + 8.0 * eps * av;
    if (av + bound >= 4611686018427387904.0) return -2;  // 2^62
    double fl = std::floor(av);
    double fr = av - fl;
    if (std::fabs(fr - 0.5) > bound && bound < 0.25) {
      int64_t mag = (int64_t)fl + (fr > 0.5 ? 1 : 0);
      out[k] = v < 0 ? -mag : mag;
      continue;
    }
    amb.push_back(k);
    out[k] = 0;
  }
  if (amb_out) {
    // the range check above covers them too: |exact - v| stays within the bound
    amb_out->swap(amb);
    return 0;
  }
  // double-double recomputation of the ambiguous coefficients, split over
  // host threads when there are many (a full vector at scale 2^40 leaves a
  // few percent of them, each an O(n) sum)
  std::atomic<int> bad{0};
  auto exact = [&](size_t i0, size_t i1) {
    for (size_t i = i0; i < i1; i++) {
      const int k = amb[i];
      dd acc = {0.0, 0.0};
      for (size_t j = 0; j < nz; j++) {
        if (z[j] == 0.0) continue;
        const size_t t = (size_t)(((uint64_t)T.rot5[j] * (uint64_t)k) % two_n);
        dd p = two_prod(z[j], T.chi[t]);
        p.lo += z[j] * T.clo[t];
        acc = dd_add(acc, quick_two_sum(p.hi, p.lo));
      }
      acc = dd_mul_d(acc, twice);
      bool neg = acc.hi < 0 || (acc.hi == 0 && acc.lo < 0);
      dd a = neg ? dd{-acc.hi, -acc.lo} : acc;
      if (a.hi >= 4611686018427387904.0) {
        bad = 1;
        return;
      }
      int64_t mag = round_dd_nonneg(a);
      out[k] = neg ? -mag : mag;
    }
  };
  const size_t work = amb.size() * nz;
  unsigned nth = std::min<unsigned>(16, std::max(1u, std::thread::hardware_concurrency()));
  if (work < (1u << 18) || nth < 2) {
    exact(0, amb.size());
  } else {
    nth = (unsigned)std::min<size_t>(nth, amb.size());
    std::vector<std::thread> th;
    const size_t per = (amb.size() + nth - 1) / nth;
    for (unsigned t = 0; t < nth; t++) {
      const size_t i0 = t * per, i1 = std::min(amb.size(), i0 + per);
      if (i0 < i1) th.emplace_back(exact, i0, i1);
    }
    for (auto& x : th) x.join();
  }
  return bad ? -2 : 0;
}

void decode_values(const EncodeTables& T, const double* m, double scale, double* out, size_t nz) {
  const int n = T.n;
  std::vector<std::complex<double>> H((size_t)n);
  for (int k = 0; k < n; k++) H[k] = m[k] * T.zeta[k];
  fft(H, T, true);
  for (size_t j = 0; j < nz; j++) out[j] = H[(T.rot5[j] - 1) / 2].real() / scale;
}
