// encode.h -- host-side canonical-embedding encoder/decoder tables and calls.
#pragma once
#include <complex>
#include <cstdint>
#include <vector>

struct EncodeTables {
  int log_n = 0, n = 0;
  std::vector<double> chi, clo;                // cos(pi t / N) as double-double, t < 2N
  std::vector<uint32_t> rot5;                  // 5^j mod 2N, j < N/2
  std::vector<uint32_t> brv;                   // bit reversal over log_n bits
  std::vector<std::complex<double>> w;         // exp(-2 pi i k / N), k < N/2
  std::vector<std::complex<double>> zeta;      // exp(i pi k / N), k < N
};

void encode_tables_init(EncodeTables& T, int log_n);
// integer coefficients round(scale * m_k); 0 or -2 (range) on failure.
// amb (nullable): the indices whose FP64 value the error bound cannot round
// are listed there and left 0 in out, for the caller to compute exactly
// (otherwise they are recomputed here in double-double)
int encode_coeffs(const EncodeTables& T, const double* z, size_t nz, double scale, int64_t* out,
                  std::vector<int>* amb = nullptr);
// slot values from centred coefficients given as doubles
void decode_values(const EncodeTables& T, const double* m, double scale, double* out, size_t nz);
