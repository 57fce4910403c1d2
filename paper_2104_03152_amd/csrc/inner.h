// inner.h -- the key-switch inner product at one coefficient, shared by the
// batched inner-product kernel and the work-queue kernel.
#pragma once
#include "device.h"

// Item b, modulus t (t < n_dig: data prime t; t == n_dig: the special
// prime), coefficient i: r_k = sum_j D_{j,t}[i] * key_b[j][k][kt][i] for both
// polys k, with D_{j,t} = ext[b][j][t] for j != t and the item's own input
// limb t (read at the Galois source of gal[b]) for j == t.  Keys are in
// Montgomery form: up to eight products are summed exactly in 128 bits and
// reduced once (8 q^2 < q 2^64).
__device__ __forceinline__ void inner_point(const InnerJob& J, const PrimeDev& P, int log_n, int b, int t, int i,
                                            u64& r0, u64& r1) {
  const int n = 1 << log_n;
  const int nm = J.n_dig + 1;
  const int km = J.km[b];
  const int kt = t < J.n_dig ? t : km - 1;
  const size_t ks_k = (size_t)km * n, ks_j = 2 * ks_k;
  const u64* kp = J.key[b] + (size_t)kt * n + i;
  const u64* diag = J.diag_p[b] ? J.diag_p[b] : J.diag + b * J.diag_stride;
  const u64* ext = J.ext + (size_t)b * J.n_dig * nm * n;
  const int di = J.gal[b] != 1 ? gal_src(i, log_n, J.gal[b]) : i;
  r0 = 0;
  r1 = 0;
  for (int j0 = 0; j0 < J.n_dig; j0 += 8) {
    U128 acc0 = {0, 0}, acc1 = {0, 0};
    const int j1 = min(J.n_dig, j0 + 8);
    for (int j = j0; j < j1; j++) {
      const u64 d = (j == t) ? diag[(size_t)t * n + di] : ext[((size_t)j * nm + t) * n + i];
      acc0 = add128(acc0, mul_wide(d, kp[j * ks_j]));
      acc1 = add128(acc1, mul_wide(d, kp[j * ks_j + ks_k]));
    }
    r0 = addmod(r0, mont_reduce(acc0, P), P.q);
    r1 = addmod(r1, mont_reduce(acc1, P), P.q);
  }
}

// Modulus t, coefficient i of all J.B items, which share one key (key[0]):
// the key words are read once and applied to every item; results into
// u[b][k][t][i].  Same arithmetic as inner_point.
__device__ __forceinline__ void inner_shared_key(const InnerJob& J, const PrimeDev& P, int log_n, int t, int i) {
  const int n = 1 << log_n;
  const int nm = J.n_dig + 1;
  const int km = J.km[0];
  const int kt = t < J.n_dig ? t : km - 1;
  const size_t ks_k = (size_t)km * n, ks_j = 2 * ks_k;
  const u64* kp = J.key[0] + (size_t)kt * n + i;
  for (int j0 = 0; j0 < J.n_dig; j0 += 8) {
    const int j1 = min(J.n_dig, j0 + 8);
    u64 k0[8], k1[8];
#pragma unroll
    for (int q = 0; q < 8; q++) {
      k0[q] = j0 + q < j1 ? kp[(j0 + q) * ks_j] : 0;
      k1[q] = j0 + q < j1 ? kp[(j0 + q) * ks_j + ks_k] : 0;
    }
    for (int b = 0; b < J.B; b++) {
      const u64* diag = J.diag_p[b] ? J.diag_p[b] : J.diag + b * J.diag_stride;
      const u64* ext = J.ext + (size_t)b * J.n_dig * nm * n;
      const int di = J.gal[b] != 1 ? gal_src(i, log_n, J.gal[b]) : i;
      U128 acc0 = {0, 0}, acc1 = {0, 0};
#pragma unroll
      for (int q = 0; q < 8; q++) {
        const int j = j0 + q;
        if (j < j1) {
          const u64 d = (j == t) ? diag[(size_t)t * n + di] : ext[((size_t)j * nm + t) * n + i];
          acc0 = add128(acc0, mul_wide(d, k0[q]));
          acc1 = add128(acc1, mul_wide(d, k1[q]));
        }
      }
      u64* u = J.u + (size_t)b * 2 * nm * n;
      u64* p0 = u + (size_t)t * n + i;
      u64* p1 = u + ((size_t)nm + t) * n + i;
      const u64 r0 = mont_reduce(acc0, P), r1 = mont_reduce(acc1, P);
      // digits beyond the first eight add to the partial results
      *p0 = j0 == 0 ? r0 : addmod(*p0, r0, P.q);
      *p1 = j0 == 0 ? r1 : addmod(*p1, r1, P.q);
    }
  }
}
