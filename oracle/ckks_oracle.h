/*
 * ckks_oracle.h -- plain, slow CPU reference implementation of RNS-CKKS.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link or
 * call this code: only tests/, __graft_entry__.smoke() and bench.py's
 * cpu_baseline leg use it.  It shares no source with the GPU library.
 *
 * Everything is kept in the coefficient domain; ring products go through a
 * textbook twisted-cyclic NTT that is pinned against schoolbook negacyclic
 * multiplication.  Paper references: TenSEAL (arXiv 2104.03152) section 2.1
 * (context, keys, automatic relinearisation/rescaling), section 3 (CKKSVector
 * holding N/2 reals; element-wise ops), section 3.1 (replicated-input
 * vector-matrix product with left rotations only), section 3.2 and appendix
 * A.4 (im2col convolution in one ciphertext), section 5 (the MNIST CNN).
 * The CKKS scheme itself is the one the paper builds on (Cheon et al. 2017).
 *
 * Parity unpinned: none of the functions below is unpinned; the pins live in
 * tests/test_oracle_*.py.
 */
#ifndef CKKS_ORACLE_H
#define CKKS_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_ctx orc_ctx;

/* A ciphertext: two polynomials, limbs 0..level, coefficient form,
 * data laid out [2][level+1][N], residues in [0, q_i). */
typedef struct {
  int level;
  double scale;
  uint64_t* data;
} orc_ct;

/* A plaintext: one polynomial, limbs 0..level, layout [level+1][N]. */
typedef struct {
  int level;
  double scale;
  uint64_t* data;
} orc_pt;

enum {
  ORC_OK = 0,
  ORC_EINVAL = -1,
  ORC_ERANGE = -2,
  ORC_ELEVEL = -3,
  ORC_ESCALE = -4,
  ORC_ENOKEY = -5,
  ORC_ENOMEM = -6
};

/* last error code of the calling thread (set when a call returns NULL) */
int orc_last_error(void);

/* ---- primitives exposed for pinning ---- */
void orc_chacha20_block(const uint32_t key[8], uint32_t counter,
                        const uint32_t nonce[3], uint32_t out[16]);
/* words[w] of the stream (seed, tag, a, b), w in [0, nwords) */
void orc_stream_words(uint64_t seed, uint32_t tag, uint32_t a, uint32_t b,
                      size_t nwords, uint64_t* out);
int orc_is_prime(uint64_t n);
/* primes for a chain: bits[0..count-1], ring degree 2^log_n */
int orc_gen_primes(int log_n, const int* bits, int count, uint64_t* out);
const uint64_t* orc_cdt_table(void); /* 20 entries */
/* sample one small / uniform polynomial of the stream (for moment tests) */
void orc_sample_ternary(uint64_t seed, uint32_t tag, uint32_t a, int n, int64_t* out);
void orc_sample_gaussian(uint64_t seed, uint32_t tag, uint32_t a, int n, int64_t* out);
void orc_sample_uniform(uint64_t seed, uint32_t tag, uint32_t a, uint32_t b,
                        uint64_t q, int n, uint64_t* out);
/* negacyclic product c = a*b mod (X^n + 1, q), through the NTT */
int orc_negacyclic_mul(const uint64_t* a, const uint64_t* b, uint64_t* c,
                       int log_n, uint64_t q);

/* ---- context ---- */
/* bits: data primes then the special prime (last). */
orc_ctx* orc_create(int log_n, const int* bits, int n_bits, double scale,
                    uint64_t seed);
void orc_free(orc_ctx*);
int orc_n(const orc_ctx*);
int orc_num_data_primes(const orc_ctx*);
void orc_primes(const orc_ctx*, uint64_t* out); /* L data primes + special */
double orc_scale(const orc_ctx*);

/* secret key, public key and relinearisation key */
int orc_keygen(orc_ctx*);
/* Galois key for a left rotation by step (0 < step < N/2), valid up to
 * max_level (restriction of the top-level key).  max_level < 0: top level. */
int orc_galois_keygen(orc_ctx*, int step, int max_level);
int orc_export_secret(const orc_ctx*, int64_t* s);
int orc_export_pk(const orc_ctx*, uint64_t* out); /* [2][L][N] */
/* key layout [digit j][poly k][modulus t][N]; t = 0..max_level then p. */
int orc_key_max_level(const orc_ctx*, int kind, int step);
int orc_export_key(const orc_ctx*, int kind, int step, uint64_t* out);

/* ---- encoding ---- */
/* integer coefficients round(scale * m_k), ties away from zero */
int orc_encode_coeffs(const orc_ctx*, const double* z, size_t n, double scale,
                      int64_t* coeffs);
orc_pt* orc_encode(const orc_ctx*, const double* z, size_t n, double scale,
                   int level);
orc_pt* orc_pt_from_coeffs(const orc_ctx*, const int64_t* coeffs,
                           double scale, int level);
/* slot values of a plaintext (CRT-centred, then evaluated) */
int orc_decode(const orc_ctx*, const orc_pt*, double* z, size_t n);
/* centred integer coefficients as long double divided by nothing */
int orc_pt_centered(const orc_ctx*, const orc_pt*, long double* out);

/* ---- objects ---- */
orc_ct* orc_ct_new(const orc_ctx*, int level, double scale);
orc_pt* orc_pt_new(const orc_ctx*, int level, double scale);
void orc_ct_free(orc_ct*);
void orc_pt_free(orc_pt*);

/* ---- encryption ---- */
orc_ct* orc_encrypt(const orc_ctx*, const orc_pt*, uint32_t enc_index,
                    int use_secret_key);
orc_pt* orc_decrypt(const orc_ctx*, const orc_ct*);

/* ---- homomorphic operations (no automatic rescale) ---- */
orc_ct* orc_add(const orc_ctx*, const orc_ct*, const orc_ct*);
orc_ct* orc_sub(const orc_ctx*, const orc_ct*, const orc_ct*);
orc_ct* orc_negate(const orc_ctx*, const orc_ct*);
orc_ct* orc_add_plain(const orc_ctx*, const orc_ct*, const orc_pt*);
orc_ct* orc_sub_plain(const orc_ctx*, const orc_ct*, const orc_pt*);
orc_ct* orc_mul_plain(const orc_ctx*, const orc_ct*, const orc_pt*);
/* (d0, d1, d2) tensor followed by relinearisation */
orc_ct* orc_mul_relin(const orc_ctx*, const orc_ct*, const orc_ct*);
orc_ct* orc_rescale(const orc_ctx*, const orc_ct*);
orc_ct* orc_drop_to(const orc_ctx*, const orc_ct*, int level);
orc_ct* orc_rotate(const orc_ctx*, const orc_ct*, int step);
/* key switch of one polynomial d at level l (for pinning): out [2][l+1][N] */
int orc_key_switch(const orc_ctx*, int kind, int step, const uint64_t* d,
                   int level, uint64_t* out);
/* Galois automorphism X -> X^g of one limb (coefficient form) */
void orc_automorphism(const uint64_t* a, uint64_t* out, int log_n, uint64_t g,
                      uint64_t q);

/* ---- composites ---- */
orc_ct* orc_sum_slots(const orc_ctx*, const orc_ct*, uint32_t n);
orc_ct* orc_conv_im2col(const orc_ctx*, const orc_ct*, const double* kernel,
                        uint32_t kk, uint32_t windows, double bias);
orc_ct* orc_matmul(const orc_ctx*, const orc_ct*, const double* w,
                   uint32_t n_in, uint32_t n_out, const double* bias);
orc_ct* orc_pack(const orc_ctx*, orc_ct* const* parts, uint32_t n_parts,
                 uint32_t width);
orc_ct* orc_square(const orc_ctx*, const orc_ct*); /* mul_relin + rescale */

/* plain im2col, vertical scan: out[k*windows + w] */
void orc_im2col(const double* img, uint32_t h, uint32_t w, uint32_t k,
                uint32_t stride, double* out);

/* The encrypted MNIST-shaped CNN (conv 4x7x7 stride 3, square, FC 256->64,
 * square, FC 64->10), returning the output ciphertext. */
orc_ct* orc_cnn(const orc_ctx*, const orc_ct* x, const double* conv_k,
                const double* conv_b, const double* w1, const double* b1,
                const double* w2, const double* b2);

#ifdef __cplusplus
}
#endif
#endif
