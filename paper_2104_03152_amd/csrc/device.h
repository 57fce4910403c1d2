// device.h -- declarations shared by the host library and the kernel
// translation units: job descriptors and kernel launchers.  All launchers
// enqueue on `st` and return the launch status.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "modarith.h"

#define HE_MAXM 33  // data primes + special prime

// One batched NTT launch: job w = a * nb + b, or, with skip_diag, over
// nb - 1 targets per a skipping b == (a mod amod).  Source a*sa + b*sb,
// destination a*da + b*db (u64 element offsets); destination prime
// dst_prime[b]; source prime src_prime, or (a mod amod) when src_prime < 0.
struct NttJob {
  const u64* src;
  u64* dst;
  long long sa, sb, da, db;
  int na, nb;
  int skip_diag;
  int src_prime;
  int amod;
  unsigned char dst_prime[HE_MAXM];
  // divide-and-round: prologue r - h_b, epilogue dst = (u - NTT(r - h_b)) * inv_b
  // plus the addend add[a*aa + b*ab] (for every a, or even a only)
  const u64* u;
  long long ua, ub;
  const u64* add;
  long long aa, ab;
  int add_even_only;
  int add_gather;      // the addend is read at the Galois source of item a / 2
  const u64* add2;     // second addend add2[a*a2a + b*ab] (every a), nullable
  long long a2a;
  u64 h_src;
  u64 hq[HE_MAXM], inv[HE_MAXM], inv_sh[HE_MAXM];
  // inverse transforms: read the source at the Galois source index of item
  // a / gal_div (gather_src set), i.e. transform tau_g(src) directly
  int gather_src, gal_div;
  u64 gal[32];
  // two-phase transforms: intermediate of job w at mid + w*N (NULL: the
  // context's scratch)
  u64* mid;
};

#define HE_MAX_BATCH 32
enum { PRO_PLAIN = 0, PRO_CENTRED_LIFT = 1, PRO_ROUNDDIV_LIFT = 2 };
// launch_ntt_fwd_blocks: the last kernel of a fused rescale (a divide-and-
// round epilogue, named apart from the key-switch ModDown)
enum { FAM_RESCALE = 3 };
enum { EPI_STORE = 0, EPI_ROUNDDIV = 1 };

// forward (lazy Cooley-Tukey, bit-reversed output) and inverse (Gentleman-
// Sande, bit-reversed input, times N^-1) batched negacyclic NTT
// Twiddle tables, N entries per prime: (w, floor(w 2^64 / q)) pairs for the
// integer butterflies and (w, w / q) double pairs for the FP64 ones.  A
// launch of at most split_jobs transforms runs in two phases (each limb
// spread over several workgroups) through tmp, tmp_words words of device
// scratch owned by the context; all launches are ordered on one stream.
// After tuning, split_mask bit i chooses the two-phase form for launches of
// up to 16 * 2^i jobs (the last bit for anything larger); split_jobs then
// only caps the scratch.
struct NttTables {
  const u64* fwd;
  const u64* inv;
  const u64* fwd_fp;
  const u64* inv_fp;
  u64* tmp;
  long long tmp_words;
  int split_jobs;
  int tuned;
  unsigned split_mask;
  int n_buckets;
  // plain one-workgroup-per-limb transforms: thread layout (words per
  // thread, radix) chosen per bucket of launch size by the tuner, 0 the
  // default layout; ntt_shapes() lists the layouts of a ring degree
  unsigned char shape[16];
  int layout;  // > 0: every plain one-workgroup launch uses this layout (not tuned)
};
// one-workgroup-per-limb thread layouts of ring degree 2^log_n: words per
// thread (log2) and pass radix (log2) of layout i; layout 0 is the default
struct NttShape {
  int loge, logr, threads;
};
int ntt_shapes(int log_n, NttShape* out, int cap);
hipError_t launch_ntt_fwd(int log_n, int pro, int epi, const NttJob& job,
                          const PrimeDev* primes, const NttTables& tabs, hipStream_t st);
hipError_t launch_ntt_inv(int log_n, const NttJob& job, const PrimeDev* primes,
                          const NttTables& tabs, hipStream_t st);

// single phases of the two-phase transforms (intermediate at job.mid): the
// inverse block phase (tag 1: first kernel of a key-switch ModUp, 2: of a
// rescale, gather not allowed), and the forward block phase with its epilogue
hipError_t launch_ntt_inv_blocks(int log_n, const NttJob& job, const PrimeDev* primes, const NttTables& tabs,
                                 int tag, hipStream_t st);
hipError_t launch_ntt_fwd_blocks(int log_n, int pro, int epi, const NttJob& job, const PrimeDev* primes,
                                 const NttTables& tabs, hipStream_t st);

// Fused key switch of B items at Lp data limbs for small batches.  ModUp:
// inverse block phase of the (gathered) input -> t1; inverse column phase,
// centred lift to every other modulus and forward column phase -> t2;
// forward block phase -> ext.  ModDown: inner product on the special
// modulus and inverse block phase -> t3; inverse column phase, rounding lift
// to each data prime and forward column phase -> t4; forward block phase
// with the data-limb inner product, the division by p and the addends in its
// epilogue -> out.
struct KsJob {
  int B, Lp, nm, special;         // items, digits (= data limbs), Lp + 1 moduli, special prime index
  const u64* d;                   // item b's input at d + b*ds: [Lp][N], NTT domain
  long long ds;
  u64 gal[HE_MAX_BATCH];          // Galois element of item b (1: none)
  const u64* key[HE_MAX_BATCH];   // item b's key [digit][2][km][N], Montgomery form
  int km[HE_MAX_BATCH];           // moduli stored per digit in that key
  u64* t1;                        // [B*Lp][N]
  u64* t2;                        // [B*Lp*Lp][N]: job (b*Lp + j)*Lp + tt, target tt (< j) or tt + 1
  u64* ext;                       // [B][Lp][nm][N]; slots [b][j][j] unused
  u64* t3;                        // [2B][N]
  u64* t4;                        // [2B*Lp][N]
  u64* t5;                        // [2B*Lp][N]: data-limb inner products (ModDown)
  u64* out;                       // poly a = 2b + k at out + a*oa: [Lp][N]
  long long oa;
  const u64* add;                 // addend poly a at add + a*aa (every a, or even a only)
  long long aa;
  int add_even_only, add_gather;  // gather: read at the Galois source of gal[b]
  const u64* add2;                // second addend at add2 + a*a2a (nullable)
  long long a2a;
  u64 h_src;                      // (p - 1) / 2
  u64 hq[HE_MAXM], inv[HE_MAXM], inv_sh[HE_MAXM];  // per data prime t: h mod q_t, p^-1 mod q_t
  // ModDown fused with the rescale that follows it (resc = 1): the top data
  // limb l = Lp - 1 is dropped.  The special-limb launch also forms
  // v_l = u_l + p * addends (NTT domain) and its inverse block phase
  // (-> t3b); the column kernel (job a * l + t, t < l) finishes both inverse
  // transforms, forms out_l's coefficients (v_l - lift_l(u_p)) p^-1, and
  // transforms lift_t(u_p) p^-1 + lift_t(out_l) (-> t4); the block kernel
  // writes ((u_t p^-1 + addends) - NTT(that)) q_l^-1, l limbs per poly.
  int resc;
  u64* t3b;                       // [2B][N]
  // rotations of coefficient-form ciphertexts (k_cks_*): input [B][2][Lp][N]
  // in coefficient form, the automorphism applied by the inverse Galois
  // element; out is in coefficient form too
  const u64* cin;
  u64 ginv[HE_MAX_BATCH];
  u64 pl, pl_sh;                  // p mod q_l and its Shoup companion
  u64 h_l;                        // (q_l - 1) / 2
  u64 hq2[HE_MAXM], inv2[HE_MAXM], inv2_sh[HE_MAXM];  // per t < l: h_l mod q_t, q_l^-1 mod q_t (+ Shoup)
};
// ModUp columns (t1 -> t2), ModDown inner + blocks (ext -> t3, and the
// data-limb inner products ext -> t5 by extra workgroups of the same
// launch), ModDown columns (t3 -> t4), ModDown blocks + epilogue (t4, t5 ->
// out).  The column
// kernels also serve a rescale: `special` is then the dropped limb's prime,
// t3 its inverse block phase, and the block phase runs as a plain NTT job.
hipError_t launch_ks_modup_cols(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                hipStream_t st);
hipError_t launch_ks_special_blocks(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                    hipStream_t st);
hipError_t launch_ks_moddown_cols(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                  hipStream_t st);
hipError_t launch_ks_moddown_blocks(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                    hipStream_t st);
// the ModDown column kernel run for a rescale
// ModDown fused with a rescale (resc = 1): the column and block kernels
// (the special-limb launch is launch_ks_special_blocks)
hipError_t launch_ks_moddown_resc_cols(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                       hipStream_t st);
hipError_t launch_ks_moddown_resc_blocks(int log_n, const KsJob& job, const PrimeDev* primes,
                                         const NttTables& tabs, hipStream_t st);
// rotation of coefficient-form ciphertexts: ModUp (lift + forward column
// stages from the automorphism's source coefficients -> t2; the forward
// block stages run as a plain two-phase block launch into ext), inner
// products + inverse block stages for every modulus (-> t3 [2B][nm][N]),
// inverse column stages + division + addends (-> out, coefficient form)
hipError_t launch_cks_modup_cols(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                 hipStream_t st);
hipError_t launch_cks_inner_blocks(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                   hipStream_t st);
hipError_t launch_cks_moddown_cols(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                   hipStream_t st);
// the same column kernel as the last launch of a rescale into coefficient
// form (t3: the inverse block stages of every limb; special: the dropped limb)
hipError_t launch_cks_rescale_cols(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                                   hipStream_t st);
hipError_t launch_rescale_cols(int log_n, const KsJob& job, const PrimeDev* primes, const NttTables& tabs,
                               hipStream_t st);

// ---- samplers (ChaCha20 streams) ----
// signed small polynomial (ternary: kind 0, Gaussian CDT: kind 1) reduced into
// n_mod moduli: out[m][N], prime of m = primes_of[m]
struct ModList {
  int n;
  unsigned char p[HE_MAXM];
};
hipError_t launch_sample_small(int log_n, int kind, uint64_t seed, uint32_t tag,
                               uint32_t a, const ModList& mods, u64* out,
                               const PrimeDev* primes, hipStream_t st);
// uniform residues: for each (row r < n_rows, modulus m): stream
// (tag, a_base + r, prime index pidx[m]) -> out[(r * mods.n + m) * N]
hipError_t launch_sample_uniform(int log_n, uint64_t seed, uint32_t tag,
                                 uint32_t a_base, int n_rows, const ModList& mods,
                                 const ModList& pidx, u64* out,
                                 const PrimeDev* primes, hipStream_t st);

// ---- pointwise (NTT domain); limb i of every poly under prime mods.p[i] ----
// op: 0 add, 1 sub, 2 negate (b unused); n_poly polys of mods.n limbs
hipError_t launch_addsub(int log_n, int op, const u64* a, const u64* b, u64* out,
                         int n_poly, const ModList& mods, const PrimeDev* primes,
                         hipStream_t st);
// out[k][i] = a[k][i] * p[i]  (k < n_poly)
hipError_t launch_mul_plain(int log_n, const u64* a, const u64* p, u64* out,
                            int n_poly, const ModList& mods, const PrimeDev* primes,
                            hipStream_t st);
// add p to poly 0 only, or subtract it (neg) (a and out: [n_poly][n][N])
hipError_t launch_add_plain(int log_n, const u64* a, const u64* p, u64* out,
                            int n_poly, const ModList& mods, const PrimeDev* primes,
                            hipStream_t st, int neg = 0);
// tensor: (d0, d1) -> out01 [2][n][N], d2 -> out2 [n][N]
hipError_t launch_tensor(int log_n, const u64* a, const u64* b, u64* out01,
                         u64* out2, const ModList& mods, const PrimeDev* primes,
                         hipStream_t st);
// B ciphertexts at one level, each at its own address ([2][n_limbs][N])
struct CtList {
  const u64* p[HE_MAX_BATCH];
};
// B ciphertexts or plaintexts written at their own addresses
struct OutList {
  u64* p[HE_MAX_BATCH];
};
// out[b] = in[b] (x) p[b] for B ciphertexts [2][n_limbs][N] (plaintexts
// [>= n_limbs][N]); out contiguous [B][2][n_limbs][N]
hipError_t launch_mul_plain_many(int log_n, const CtList& in, const CtList& p, int B, int n_limbs, u64* out,
                                 const PrimeDev* primes, hipStream_t st);
// out[b] = in[b] + p[b] on poly 0 (poly 1 copied)
hipError_t launch_add_plain_many(int log_n, const CtList& in, const CtList& p, const OutList& out, int B,
                                 int n_limbs, const PrimeDev* primes, hipStream_t st);
// out = sum of B ciphertexts [2][n_limbs][N]
hipError_t launch_sum_cts(int log_n, const CtList& in, int B, int n_limbs, u64* out, const PrimeDev* primes,
                          hipStream_t st);
// tensor of B pairs: out01 [B][2][n_limbs][N], out2 [B][n_limbs][N]
hipError_t launch_tensor_many(int log_n, const CtList& a, const CtList& b, int B, u64* out01, u64* out2,
                              int n_limbs, const PrimeDev* primes, hipStream_t st);
// device copy of `words` words (a kernel, so that graph capture records a
// kernel node)
hipError_t launch_copy(const u64* src, u64* dst, long long words, hipStream_t st);
// copy of B ciphertexts into one contiguous [B][2][n_limbs][N] buffer
hipError_t launch_gather_cts(int log_n, const CtList& a, int B, int n_limbs, u64* out, hipStream_t st);
// decrypt: m[i] = c0[i] + c1[i] * s[i]   (s: [L+1][N], limb i under prime i)
hipError_t launch_decrypt(int log_n, const u64* ct, const u64* s, u64* m,
                          int n_limbs, const PrimeDev* primes, hipStream_t st);
// Galois automorphism in the NTT domain: item b has rows_per_item rows,
// out[b][r][n] = in[b][r][src_{g_b}(n)]
struct AutJob {
  int B, rows_per_item;
  u64 g[HE_MAX_BATCH];
};
hipError_t launch_automorphism(int log_n, const u64* in, u64* out, const AutJob& job, hipStream_t st);
// key-switch inner product of B items (keys in Montgomery form):
// u[b][k][t][n] = sum_j D_{b,j,t}[n] * key_b[j][k][kt][n],
// D_{b,j,t} = (j == t) ? diag[b][t] : ext[b][j][t]; t < n_dig are data moduli
// (prime t), t == n_dig is the special prime.
struct InnerJob {
  const u64* ext;    // [B][n_dig][n_dig + 1][N]
  const u64* diag;   // item b at diag + b * diag_stride: [n_dig][N] NTT domain,
  long long diag_stride;  // read at the Galois source of gal[b] (1: none)
  u64 gal[HE_MAX_BATCH];
  u64* u;            // [B][2][n_dig + 1][N]
  int B, n_dig, special_prime;
  const u64* key[HE_MAX_BATCH];
  int km[HE_MAX_BATCH];  // moduli stored in each key
  // item b's input limbs at diag_p[b] when set (items not laid out with
  // one stride), else at diag + b * diag_stride
  const u64* diag_p[HE_MAX_BATCH];
};
hipError_t launch_inner(int log_n, const InnerJob& job, const PrimeDev* primes,
                        hipStream_t st);
// keygen combine: K0 = -a*s + e + [t == j] pmod_j * s', K1 = a, both turned
// into Montgomery form. a, e: [nd][nm][N] NTT domain; s, sp: [L+1][N] NTT.
hipError_t launch_keygen_combine(int log_n, const u64* a, const u64* e,
                                 const u64* s, const u64* sp, u64* key, int nd,
                                 int nm, const ModList& pidx, int special_prime,
                                 const PrimeDev* primes, hipStream_t st);
// public-key pieces: out[i] = -a[i]*s[i] + e[i]   (i < n)
hipError_t launch_pk_combine(int log_n, const u64* a, const u64* e, const u64* s,
                             u64* out, int n, const PrimeDev* primes, hipStream_t st);
// encryption: c0 = v*pk0 + e0 + m, c1 = v*pk1 + e1 (pk path) or
// c0 = -a*s + e0 + m, c1 = a (sk path: pk0 = NULL, v = a)
hipError_t launch_encrypt_combine(int log_n, const u64* v, const u64* pk0,
                                  const u64* pk1, const u64* e0, const u64* e1,
                                  const u64* s, const u64* m, u64* ct, int n_limbs,
                                  int pk_limbs, const PrimeDev* primes, hipStream_t st);
// key export: Montgomery -> normal form, in place over n words of prime rows
hipError_t launch_from_mont(int log_n, u64* data, int n_rows, const ModList& mods,
                            const PrimeDev* primes, hipStream_t st);
// ---- hoisted rotations of one ciphertext (vector-matrix product) ----
// item r: left rotation with Galois element gal[r] and key keys[r] (km[r]
// moduli stored), multiplied by diagonal diag_idx[r].
struct HoistItem {
  const u64* key;
  u64 g;
  int km;
  int diag;
};
// u[r][k][t][n] = sum_j D_{j,t}[src_r(n)] * key_r[j][k][kt][n]  (t < nm),
// plus p c0[t][src_r(n)] for k = 0 and t < n_dig: the ModDown then yields
// (u - v) p^-1 + c0[t][src_r(n)], the rotation's poly 0, exactly
struct HoistInner {
  const u64* ext;   // [n_dig][nm][N] ModUp digits (diagonal slots unused)
  const u64* c1;    // [n_dig][N] poly 1 of the input (NTT domain)
  const u64* c0;    // [n_dig][N] poly 0 of the input (NTT domain)
  const HoistItem* items;
  u64* u;           // [R][2][nm][N]
  int R, n_dig, nm, t_begin, t_end, special_prime;
  u64 pq[HE_MAXM], pq_sh[HE_MAXM];  // p mod q_t and its Shoup companion
};
hipError_t launch_inner_hoisted(int log_n, const HoistInner& job, const PrimeDev* primes,
                                hipStream_t st);
// ModDown of every item fused with the diagonal multiply-accumulate: WG
// (chunk c, poly k, modulus t) sums over its items r:
//   (u[r][k][t] - NTT(r_r - h)) p^-1 * diag[r][t]
// (u[r][0] carries the rotated c0, see HoistInner)
// into partial[c][k][t] (without the diagonal factor when diags is NULL).
// The two workgroups (k = 0, 1) of one (chunk, t) run on the same XCD, one
// after the other in dispatch order, so the second reads the diagonals
// from that XCD's L2.  The two-phase form splits each transform as the
// two-phase NTTs do: the column phase (the special limb's inverse transform,
// then for every modulus the lift and the forward column stages, into mid),
// then a block kernel whose workgroups (chunk, poly, modulus, block) finish
// their block's stages item after item and accumulate.  The two-phase form
// computes u itself where it is used (the special limb in the kernel before
// the column phase, the data limbs in the block kernel), from the shared
// digits and the keys: u is never stored.
struct HoistMac {
  // [R][2][N] special-prime limb of u: coefficient form (one-kernel form);
  // the two-phase form's column phase writes there the inverse transform's
  // block-phase output
  const u64* ucoef;
  const u64* u;      // [R][2][nm][N] (one-kernel form)
  // two-phase form: the ModUp digits [n_dig][nm][N] shared by the items,
  // the input's polys [n_dig][N] (NTT domain) and p mod q_t (+ Shoup)
  const u64* ext;
  const u64* c1;
  const u64* c0;
  u64 pq[HE_MAXM], pq_sh[HE_MAXM];
  const u64* diags;  // [n_diag][n_dig][N] plaintext diagonals (NTT domain)
  const HoistItem* items;
  u64* partial;      // [n_chunks][2][n_dig][N]
  // two-phase form when non-NULL: [R][2][n_dig][N] column-phase output of
  // every (item, poly, modulus) forward transform
  u64* mid;
  int R, n_dig, nm, chunk, special_prime;
  int n_units;       // n_chunks * n_dig (one-kernel form); set by the launcher in the two-phase form
  u64 h_src;
  u64 hq[HE_MAXM], inv[HE_MAXM], inv_sh[HE_MAXM];
};
hipError_t launch_hoisted_moddown_mac(int log_n, const HoistMac& job, const PrimeDev* primes,
                                      const NttTables& tabs, hipStream_t st);
// the two-phase form: launch_hoisted_cols runs the column phase, then
// launch_hoisted_moddown_mac the block phase with the multiply-accumulate
hipError_t launch_hoisted_cols(int log_n, const HoistMac& job, const PrimeDev* primes,
                               const NttTables& tabs, hipStream_t st);
// workgroups per (chunk, poly, modulus) of the two-phase form's block phase
int hoist_split_blocks(int log_n);
// out[k][t] = x[k][t] * diag0[t] + sum_c partial[c][k][t] (x[k][t] itself
// when diag0 is NULL)
hipError_t launch_mac_finish(int log_n, const u64* partial, int n_chunks, const u64* x,
                             const u64* diag0, u64* out, int n_dig, const PrimeDev* primes,
                             hipStream_t st);
// Montgomery form of plaintext rows
// encoding: the coefficients amb[0..n_amb) recomputed exactly (double-double
// sums of z_j cos(pi t / N), chi + clo the cosine table as double-double,
// rot5[j] = 5^j mod 2N) and rounded into co[k]; twice = 2 scale / N
hipError_t launch_encode_exact(int log_n, const double* z, int nz, const uint32_t* rot5, const double* chi,
                               const double* clo, const int* amb, int n_amb, double twice, int64_t* co,
                               hipStream_t st);
// signed coefficients co[N] (|v| < 2^62) reduced into limbs 0..n_limbs-1: out[i][k] = co[k] mod q_i
hipError_t launch_coeffs_to_limbs(int log_n, const int64_t* co, u64* out, int n_limbs, const PrimeDev* primes,
                                  hipStream_t st);
hipError_t launch_to_mont(int log_n, u64* data, int n_rows, const ModList& mods,
                          const PrimeDev* primes, hipStream_t st);

// ---- work-queue launches over heterogeneous work ----
// One task is one limb-sized piece of one job: the job's record (an NttJob,
// an InnerJob or a QTensor, by the launch's kind), the job-local index w
// (decoded as a launch decodes its block index; for INNER the modulus, for
// TENSOR the limb), the task's ring degree and the tables of its context.
struct QTask {
  int log_n;
  int job;
  int w;
  int tab;
};
struct QTables {
  const PrimeDev* primes;
  const u64* fwd;
  const u64* inv;
  const u64* fwd_fp;
  const u64* inv_fp;
};
// the tensor of one product: (d0, d1) = (a0 b0, a0 b1 + a1 b0), d2 = a1 b1
struct QTensor {
  const u64* a;  // [2][Lp][N]
  const u64* b;  // [2][Lp][N]
  u64* out01;    // [2][Lp][N]
  u64* out2;     // [Lp][N]
  int Lp;
};
enum { QK_TENSOR = 0, QK_INV = 1, QK_FWD_LIFT = 2, QK_INNER = 3, QK_FWD_RD = 4 };
// Drains tasks[0..n) of one kind: `grid` resident workgroups of 1024
// threads each take the next task from *head (an atomic counter that must
// be zero) until none is left; tasks may mix ring degrees 2^12..2^14 and
// contexts.  INV runs inv_body (gathering when the job asks), FWD_LIFT the
// forward transform with the centred lift, FWD_RD with the divide-and-round
// prologue and epilogue.
hipError_t launch_queue(int kind, const QTask* tasks, int n, const void* jobs, const QTables* tabs,
                        unsigned* head, int grid, size_t lds_bytes, hipStream_t st);
// dynamic LDS of a queue task of this kind at ring degree 2^log_n
size_t queue_lds_bytes(int kind, int log_n);
// workgroups of a queue launch that fit on the device at once
int queue_grid(int device, size_t lds_bytes);
// p[0..n) = v (a kernel, so that graph capture records a kernel node)
hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t st);

// Fixed device scratch of the no-allocation entry point: the device address
// of this device's copy of the array (looked up once per device, with that
// device current) and its size in bytes.
hipError_t noalloc_scratch(int device, u64** ptr, size_t* bytes);

// Job descriptors travel by value in the kernarg segment, which holds at
// most 4 KiB per launch together with the other arguments (a table pointer,
// the NttTables block and a few scalars).
constexpr size_t kKernargBudget = 4096 - sizeof(NttTables) - 64;
static_assert(sizeof(NttJob) <= kKernargBudget, "NttJob exceeds the kernel-argument budget");
static_assert(sizeof(KsJob) <= kKernargBudget, "KsJob exceeds the kernel-argument budget");
static_assert(sizeof(HoistMac) <= kKernargBudget, "HoistMac exceeds the kernel-argument budget");
static_assert(sizeof(HoistInner) <= kKernargBudget, "HoistInner exceeds the kernel-argument budget");
static_assert(sizeof(InnerJob) <= kKernargBudget, "InnerJob exceeds the kernel-argument budget");
