/*
 * ckks_oracle.c -- plain, slow CPU reference implementation of RNS-CKKS.
 *
 * TEST INFRASTRUCTURE ONLY (see ckks_oracle.h): the product library never
 * includes, links or calls this file, and this file includes nothing of the
 * product library.
 *
 * Style: every residue is kept in [0, q); products are (unsigned __int128) a*b
 * % q; every polynomial lives in the coefficient domain; a ring product is a
 * textbook twisted cyclic radix-2 NTT.  No lazy reduction, no Shoup/Barrett,
 * no fusion.  Where the paper is silent the reading taken is stated at the
 * function (prime chain, sampler streams, key layout, digit representative,
 * rounding of rescale/ModDown, slot order, replication and im2col layouts).
 */
#include "ckks_oracle.h"

#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>

typedef uint64_t u64;
typedef int64_t i64;
typedef uint32_t u32;
typedef unsigned __int128 u128;

#define MAXP 40 /* data primes + special */

static _Thread_local int g_err;
int orc_last_error(void) { return g_err; }
#define FAIL(code)     \
  do {                 \
    g_err = (code);    \
    return NULL;       \
  } while (0)

/* ------------------------------------------------------------------ */
/* Modular arithmetic, the plain way.                                   */
/* ------------------------------------------------------------------ */
static u64 addm(u64 a, u64 b, u64 q) {
  u64 s = a + b;
  return s >= q ? s - q : s;
}
static u64 subm(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }
static u64 mulm(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }
static u64 powm(u64 a, u64 e, u64 q) {
  u64 r = 1 % q;
  a %= q;
  while (e) {
    if (e & 1) r = mulm(r, a, q);
    a = mulm(a, a, q);
    e >>= 1;
  }
  return r;
}
static u64 invm(u64 a, u64 q) { return powm(a, q - 2, q); } /* q prime */
/* a signed integer reduced into [0, q) */
static u64 red_i64(i64 v, u64 q) {
  if (v >= 0) return (u64)v % q;
  u64 mag = (u64)(-(v + 1)) + 1u;
  u64 r = mag % q;
  return r ? q - r : 0;
}

/* ------------------------------------------------------------------ */
/* Primes (reading of the paper's "coefficient modulus" bit sizes):     */
/* for each requested bit size in order, the largest prime below 2^b    */
/* with q = 1 mod 2N that is not already in the chain.                  */
/* ------------------------------------------------------------------ */
int orc_is_prime(u64 n) {
  static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  if (n < 2) return 0;
  for (int i = 0; i < 12; i++)
    if (n % bases[i] == 0) return n == bases[i];
  u64 d = n - 1;
  int r = 0;
  while (!(d & 1)) {
    d >>= 1;
    r++;
  }
  for (int i = 0; i < 12; i++) {
    u64 x = powm(bases[i], d, n);
    if (x == 1 || x == n - 1) continue;
    int witness = 1;
    for (int k = 1; k < r; k++) {
      x = mulm(x, x, n);
      if (x == n - 1) {
        witness = 0;
        break;
      }
    }
    if (witness) return 0;
  }
  return 1;
}

int orc_gen_primes(int log_n, const int* bits, int count, u64* out) {
  u64 m = 2ull << log_n;
  for (int i = 0; i < count; i++) {
    int b = bits[i];
    if (b < log_n + 2 || b > 61) return ORC_EINVAL;
    u64 c = (((1ull << b) - 2) / m) * m + 1;
    u64 lo = 1ull << (b - 1);
    int found = 0;
    while (c > lo) {
      int used = 0;
      for (int k = 0; k < i; k++) used |= (out[k] == c);
      if (!used && orc_is_prime(c)) {
        found = 1;
        break;
      }
      c -= m;
    }
    if (!found) return ORC_EINVAL;
    out[i] = c;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* ChaCha20 block function (RFC 8439, section 2.3) and the sampler      */
/* streams: key = seed (8 bytes LE) || 24 zero bytes, nonce = (tag, a,  */
/* b) as little-endian u32, counter = block index; each 64-byte block   */
/* gives eight little-endian u64 words.                                 */
/* ------------------------------------------------------------------ */
#define ROTL32(v, c) (((v) << (c)) | ((v) >> (32 - (c))))
#define QROUND(a, b, c, d) \
  a += b;                  \
  d ^= a;                  \
  d = ROTL32(d, 16);       \
  c += d;                  \
  b ^= c;                  \
  b = ROTL32(b, 12);       \
  a += b;                  \
  d ^= a;                  \
  d = ROTL32(d, 8);        \
  c += d;                  \
  b ^= c;                  \
  b = ROTL32(b, 7);

void orc_chacha20_block(const u32 key[8], u32 counter, const u32 nonce[3],
                        u32 out[16]) {
  u32 s[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u,
               key[0],      key[1],      key[2],      key[3],
               key[4],      key[5],      key[6],      key[7],
               counter,     nonce[0],    nonce[1],    nonce[2]};
  u32 x[16];
  memcpy(x, s, sizeof x);
  for (int i = 0; i < 10; i++) {
    QROUND(x[0], x[4], x[8], x[12]);
    QROUND(x[1], x[5], x[9], x[13]);
    QROUND(x[2], x[6], x[10], x[14]);
    QROUND(x[3], x[7], x[11], x[15]);
    QROUND(x[0], x[5], x[10], x[15]);
    QROUND(x[1], x[6], x[11], x[12]);
    QROUND(x[2], x[7], x[8], x[13]);
    QROUND(x[3], x[4], x[9], x[14]);
  }
  for (int i = 0; i < 16; i++) out[i] = x[i] + s[i];
}

void orc_stream_words(u64 seed, u32 tag, u32 a, u32 b, size_t nwords,
                      u64* out) {
  u32 key[8] = {(u32)seed, (u32)(seed >> 32), 0, 0, 0, 0, 0, 0};
  u32 nonce[3] = {tag, a, b};
  u32 blk[16];
  for (size_t w = 0; w < nwords; w++) {
    if (w % 8 == 0) orc_chacha20_block(key, (u32)(w / 8), nonce, blk);
    size_t r = w % 8;
    out[w] = (u64)blk[2 * r] | ((u64)blk[2 * r + 1] << 32);
  }
}

/* Discrete Gaussian, sigma = 3.2, cut at |x| <= 19: T[k] = floor(2^63 *
 * P(|x| <= k)).  Pinned against a 60-digit recomputation in the tests. */
static const u64 CDT[20] = {
    0x0ff52b40a5917f1dull, 0x2e5a25d4bf0e400eull, 0x489ae26955b04bd6ull,
    0x5d2bc20f621bf185ull, 0x6bc8694c3cc80ff4ull, 0x7532d89ac6ba7dceull,
    0x7ab396cb74436798ull, 0x7d9e4e916643eb07ull, 0x7f05495819eb2051ull,
    0x7fa1ce9c0039a957ull, 0x7fdfb3f212e8c4e8ull, 0x7ff5e6f9d2314fccull,
    0x7ffd1f97bc4406a2ull, 0x7fff40fa0088d11dull, 0x7fffd2e835e1c57dull,
    0x7ffff6524386ff1eull, 0x7ffffe1db4769da5ull, 0x7fffffac0a1dcb08ull,
    0x7ffffff428673853ull, 0x8000000000000000ull};
const u64* orc_cdt_table(void) { return CDT; }

/* coefficient i of a ternary polynomial: (w[i] mod 3) - 1 */
void orc_sample_ternary(u64 seed, u32 tag, u32 a, int n, i64* out) {
  u64* w = malloc(sizeof(u64) * (size_t)n);
  orc_stream_words(seed, tag, a, 0, (size_t)n, w);
  for (int i = 0; i < n; i++) out[i] = (i64)(w[i] % 3) - 1;
  free(w);
}
/* coefficient i: u = w[i] >> 1, |x| = min{k : u < T[k]}, sign = w[i] & 1 */
void orc_sample_gaussian(u64 seed, u32 tag, u32 a, int n, i64* out) {
  u64* w = malloc(sizeof(u64) * (size_t)n);
  orc_stream_words(seed, tag, a, 0, (size_t)n, w);
  for (int i = 0; i < n; i++) {
    u64 u = w[i] >> 1;
    i64 k = 0;
    while (!(u < CDT[k])) k++;
    out[i] = (w[i] & 1) ? -k : k;
  }
  free(w);
}
/* coefficient i: (w[2i+1] * 2^64 + w[2i]) mod q */
void orc_sample_uniform(u64 seed, u32 tag, u32 a, u32 b, u64 q, int n,
                        u64* out) {
  u64* w = malloc(sizeof(u64) * 2 * (size_t)n);
  orc_stream_words(seed, tag, a, b, 2 * (size_t)n, w);
  for (int i = 0; i < n; i++)
    out[i] = (u64)((((u128)w[2 * i + 1] << 64) | w[2 * i]) % q);
  free(w);
}

/* ------------------------------------------------------------------ */
/* Negacyclic ring product via the textbook twisted cyclic NTT:         */
/* A_k = sum_j a_j psi^j omega^(jk) with omega = psi^2, psi a primitive */
/* 2N-th root of unity, so a*b mod (X^N+1) = untwist(iDFT(A . B)).      */
/* ------------------------------------------------------------------ */
typedef struct {
  int log_n, n;
  u64 q, psi, n_inv;
  u64* psi_pow;  /* psi^j, j < N        */
  u64* ipsi_pow; /* psi^-j, j < N       */
  u64* w_pow;    /* omega^k, k < N/2    */
  u64* iw_pow;   /* omega^-k, k < N/2   */
} ntt_tab;

static u64 find_psi(u64 q, int log_n) {
  u64 two_n = 2ull << log_n;
  for (u64 g = 2;; g++) {
    u64 x = powm(g, (q - 1) / two_n, q);
    if (powm(x, two_n / 2, q) == q - 1) return x;
  }
}

static int ntt_tab_init(ntt_tab* t, int log_n, u64 q) {
  int n = 1 << log_n;
  t->log_n = log_n;
  t->n = n;
  t->q = q;
  t->psi = find_psi(q, log_n);
  t->n_inv = invm((u64)n % q, q);
  t->psi_pow = malloc(sizeof(u64) * (size_t)n);
  t->ipsi_pow = malloc(sizeof(u64) * (size_t)n);
  t->w_pow = malloc(sizeof(u64) * (size_t)(n / 2 + 1));
  t->iw_pow = malloc(sizeof(u64) * (size_t)(n / 2 + 1));
  if (!t->psi_pow || !t->ipsi_pow || !t->w_pow || !t->iw_pow) return ORC_ENOMEM;
  u64 ipsi = invm(t->psi, q);
  u64 w = mulm(t->psi, t->psi, q), iw = mulm(ipsi, ipsi, q);
  t->psi_pow[0] = t->ipsi_pow[0] = 1;
  for (int j = 1; j < n; j++) {
    t->psi_pow[j] = mulm(t->psi_pow[j - 1], t->psi, q);
    t->ipsi_pow[j] = mulm(t->ipsi_pow[j - 1], ipsi, q);
  }
  t->w_pow[0] = t->iw_pow[0] = 1;
  for (int k = 1; k <= n / 2; k++) {
    t->w_pow[k] = mulm(t->w_pow[k - 1], w, q);
    t->iw_pow[k] = mulm(t->iw_pow[k - 1], iw, q);
  }
  return ORC_OK;
}
static void ntt_tab_free(ntt_tab* t) {
  free(t->psi_pow);
  free(t->ipsi_pow);
  free(t->w_pow);
  free(t->iw_pow);
}

static unsigned bitrev(unsigned x, int bits) {
  unsigned r = 0;
  for (int i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

/* in-place cyclic DFT, radix-2 decimation in time after a bit-reversal */
static void dft(u64* a, int log_n, const u64* wpow, u64 q) {
  int n = 1 << log_n;
  for (int i = 0; i < n; i++) {
    int j = (int)bitrev((unsigned)i, log_n);
    if (j > i) {
      u64 t = a[i];
      a[i] = a[j];
      a[j] = t;
    }
  }
  for (int len = 2; len <= n; len <<= 1) {
    int half = len / 2, step = n / len;
    for (int i = 0; i < n; i += len)
      for (int j = 0; j < half; j++) {
        u64 u = a[i + j];
        u64 v = mulm(a[i + j + half], wpow[j * step], q);
        a[i + j] = addm(u, v, q);
        a[i + j + half] = subm(u, v, q);
      }
  }
}

static void to_eval(const ntt_tab* t, const u64* a, u64* out) {
  for (int j = 0; j < t->n; j++) out[j] = mulm(a[j], t->psi_pow[j], t->q);
  dft(out, t->log_n, t->w_pow, t->q);
}
static void from_eval(const ntt_tab* t, const u64* a, u64* out) {
  if (out != a) memcpy(out, a, sizeof(u64) * (size_t)t->n);
  dft(out, t->log_n, t->iw_pow, t->q);
  for (int j = 0; j < t->n; j++)
    out[j] = mulm(mulm(out[j], t->n_inv, t->q), t->ipsi_pow[j], t->q);
}

int orc_negacyclic_mul(const u64* a, const u64* b, u64* c, int log_n, u64 q) {
  ntt_tab t;
  if (ntt_tab_init(&t, log_n, q)) return ORC_ENOMEM;
  int n = 1 << log_n;
  u64* A = malloc(sizeof(u64) * (size_t)n);
  u64* B = malloc(sizeof(u64) * (size_t)n);
  to_eval(&t, a, A);
  to_eval(&t, b, B);
  for (int i = 0; i < n; i++) A[i] = mulm(A[i], B[i], q);
  from_eval(&t, A, c);
  free(A);
  free(B);
  ntt_tab_free(&t);
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Context                                                              */
/* ------------------------------------------------------------------ */
typedef struct {
  int max_level; /* key valid for levels 0..max_level */
  u64* data;     /* [max_level+1 digits][2][max_level+2 moduli][N] */
  u64* eval;     /* same, transformed (kept only to avoid re-transforming) */
} orc_key;

struct orc_ctx {
  int log_n, n, L; /* L data primes, q[L] = special prime p */
  u64 q[MAXP];
  ntt_tab tab[MAXP];
  double scale;
  u64 seed;
  int have_keys;
  i64* s;           /* secret, ternary, coefficient form */
  u64* s_eval;      /* [L+1][N] */
  u64* pk;          /* [2][L][N] coefficient form */
  orc_key relin;
  orc_key** gal;    /* indexed by step, N/2 entries */
  u64* rot5;        /* 5^j mod 2N, j < N/2 */
  long double* cos_ld; /* cos(pi t / N), t < 2N */
  __float128* cos_q;
};

int orc_n(const orc_ctx* c) { return c->n; }
int orc_num_data_primes(const orc_ctx* c) { return c->L; }
void orc_primes(const orc_ctx* c, u64* out) {
  memcpy(out, c->q, sizeof(u64) * (size_t)(c->L + 1));
}
double orc_scale(const orc_ctx* c) { return c->scale; }

orc_ctx* orc_create(int log_n, const int* bits, int n_bits, double scale,
                    u64 seed) {
  if (log_n < 2 || log_n > 17 || n_bits < 2 || n_bits > MAXP) FAIL(ORC_EINVAL);
  orc_ctx* c = calloc(1, sizeof *c);
  if (!c) FAIL(ORC_ENOMEM);
  c->log_n = log_n;
  c->n = 1 << log_n;
  c->L = n_bits - 1;
  c->scale = scale;
  c->seed = seed;
  if (orc_gen_primes(log_n, bits, n_bits, c->q)) {
    free(c);
    FAIL(ORC_EINVAL);
  }
  for (int i = 0; i <= c->L; i++) ntt_tab_init(&c->tab[i], log_n, c->q[i]);
  int n = c->n;
  c->rot5 = malloc(sizeof(u64) * (size_t)(n / 2));
  u64 two_n = 2ull * (u64)n, p5 = 1;
  for (int j = 0; j < n / 2; j++) {
    c->rot5[j] = p5;
    p5 = p5 * 5 % two_n;
  }
  c->cos_ld = malloc(sizeof(long double) * 2 * (size_t)n);
  c->cos_q = malloc(sizeof(__float128) * 2 * (size_t)n);
  for (int t = 0; t < 2 * n; t++) {
    c->cos_q[t] = cosq(M_PIq * (__float128)t / (__float128)n);
    c->cos_ld[t] = (long double)c->cos_q[t];
  }
  c->gal = calloc((size_t)(n / 2), sizeof(orc_key*));
  return c;
}

static void key_free(orc_key* k) {
  if (!k) return;
  free(k->data);
  free(k->eval);
}

void orc_free(orc_ctx* c) {
  if (!c) return;
  for (int i = 0; i <= c->L; i++) ntt_tab_free(&c->tab[i]);
  free(c->rot5);
  free(c->cos_ld);
  free(c->cos_q);
  free(c->s);
  free(c->s_eval);
  free(c->pk);
  key_free(&c->relin);
  if (c->gal) {
    for (int i = 0; i < c->n / 2; i++)
      if (c->gal[i]) {
        key_free(c->gal[i]);
        free(c->gal[i]);
      }
    free(c->gal);
  }
  free(c);
}

/* ------------------------------------------------------------------ */
/* Objects                                                              */
/* ------------------------------------------------------------------ */
orc_ct* orc_ct_new(const orc_ctx* c, int level, double scale) {
  if (level < 0 || level >= c->L) FAIL(ORC_ELEVEL);
  orc_ct* ct = malloc(sizeof *ct);
  if (!ct) FAIL(ORC_ENOMEM);
  ct->level = level;
  ct->scale = scale;
  ct->data = calloc(2 * (size_t)(level + 1) * (size_t)c->n, sizeof(u64));
  if (!ct->data) {
    free(ct);
    FAIL(ORC_ENOMEM);
  }
  return ct;
}
orc_pt* orc_pt_new(const orc_ctx* c, int level, double scale) {
  if (level < 0 || level >= c->L) FAIL(ORC_ELEVEL);
  orc_pt* pt = malloc(sizeof *pt);
  if (!pt) FAIL(ORC_ENOMEM);
  pt->level = level;
  pt->scale = scale;
  pt->data = calloc((size_t)(level + 1) * (size_t)c->n, sizeof(u64));
  if (!pt->data) {
    free(pt);
    FAIL(ORC_ENOMEM);
  }
  return pt;
}
void orc_ct_free(orc_ct* ct) {
  if (!ct) return;
  free(ct->data);
  free(ct);
}
void orc_pt_free(orc_pt* pt) {
  if (!pt) return;
  free(pt->data);
  free(pt);
}
/* limb i of polynomial k of a ciphertext at level l */
static u64* ct_limb(const orc_ctx* c, const orc_ct* ct, int k, int i) {
  return ct->data + ((size_t)k * (size_t)(ct->level + 1) + (size_t)i) * (size_t)c->n;
}

/* ------------------------------------------------------------------ */
/* Keys.  Streams: s = ternary(tag 1); pk: a = uniform(tag 2, 0, i),     */
/* e = gaussian(tag 3); relin digit j: a = uniform(tag 4, j, i), e =     */
/* gaussian(tag 5, j); Galois step k digit j: a = uniform(tag 6,         */
/* 256k + j, i), e = gaussian(tag 7, 256k + j).  Prime index i of the    */
/* special prime is L whatever level the key is cut at.                  */
/*                                                                       */
/* Switching key from s' to s, one digit per data prime (dnum = L):      */
/*   evk_j mod q_t = -a_{j,t} s + e_j + [t = j] (p mod q_j) s'           */
/*   evk_j mod p   = -a_{j,p} s + e_j,      evk_j poly 1 = a_{j,t}.      */
/* A key cut at level l is the restriction to digits and moduli 0..l     */
/* plus p, which is exact.                                                */
/* ------------------------------------------------------------------ */
static int keymod_prime_index(const orc_ctx* c, int max_level, int t) {
  return t <= max_level ? t : c->L;
}

static int make_switch_key(orc_ctx* c, orc_key* key, int max_level,
                           const u64* s_prime /* [L+1][N] coefficient */,
                           u32 tag_a, u32 tag_e, u32 idx_base) {
  int n = c->n, nm = max_level + 2, nd = max_level + 1;
  size_t sz = (size_t)nd * 2 * (size_t)nm * (size_t)n;
  key->max_level = max_level;
  key->data = malloc(sizeof(u64) * sz);
  key->eval = malloc(sizeof(u64) * sz);
  i64* e = malloc(sizeof(i64) * (size_t)n);
  u64* a = malloc(sizeof(u64) * (size_t)n);
  u64* tmp = malloc(sizeof(u64) * (size_t)n);
  if (!key->data || !key->eval || !e || !a || !tmp) return ORC_ENOMEM;
  for (int j = 0; j < nd; j++) {
    orc_sample_gaussian(c->seed, tag_e, idx_base + (u32)j, n, e);
    for (int t = 0; t < nm; t++) {
      int pi = keymod_prime_index(c, max_level, t);
      u64 q = c->q[pi];
      const ntt_tab* tb = &c->tab[pi];
      orc_sample_uniform(c->seed, tag_a, idx_base + (u32)j, (u32)pi, q, n, a);
      /* a*s */
      to_eval(tb, a, tmp);
      for (int i = 0; i < n; i++)
        tmp[i] = mulm(tmp[i], c->s_eval[(size_t)pi * n + i], q);
      from_eval(tb, tmp, tmp);
      u64* k0 = key->data + (((size_t)j * 2 + 0) * nm + t) * n;
      u64* k1 = key->data + (((size_t)j * 2 + 1) * nm + t) * n;
      u64 pmod = c->q[c->L] % q;
      for (int i = 0; i < n; i++) {
        u64 v = subm(red_i64(e[i], q), tmp[i], q);
        if (t == j) v = addm(v, mulm(pmod, s_prime[(size_t)pi * n + i], q), q);
        k0[i] = v;
        k1[i] = a[i];
      }
      to_eval(tb, k0, key->eval + (((size_t)j * 2 + 0) * nm + t) * n);
      to_eval(tb, k1, key->eval + (((size_t)j * 2 + 1) * nm + t) * n);
    }
  }
  free(e);
  free(a);
  free(tmp);
  return ORC_OK;
}

int orc_keygen(orc_ctx* c) {
  int n = c->n, L = c->L;
  c->s = malloc(sizeof(i64) * (size_t)n);
  c->s_eval = malloc(sizeof(u64) * (size_t)(L + 1) * n);
  c->pk = malloc(sizeof(u64) * 2 * (size_t)L * n);
  if (!c->s || !c->s_eval || !c->pk) return ORC_ENOMEM;
  orc_sample_ternary(c->seed, 1, 0, n, c->s);
  u64* tmp = malloc(sizeof(u64) * (size_t)n);
  for (int i = 0; i <= L; i++) {
    for (int k = 0; k < n; k++) tmp[k] = red_i64(c->s[k], c->q[i]);
    to_eval(&c->tab[i], tmp, c->s_eval + (size_t)i * n);
  }
  /* public key over the data primes */
  i64* e = malloc(sizeof(i64) * (size_t)n);
  orc_sample_gaussian(c->seed, 3, 0, n, e);
  for (int i = 0; i < L; i++) {
    u64 q = c->q[i];
    u64* a = c->pk + ((size_t)L + i) * n;
    u64* b = c->pk + (size_t)i * n;
    orc_sample_uniform(c->seed, 2, 0, (u32)i, q, n, a);
    to_eval(&c->tab[i], a, tmp);
    for (int k = 0; k < n; k++)
      tmp[k] = mulm(tmp[k], c->s_eval[(size_t)i * n + k], q);
    from_eval(&c->tab[i], tmp, tmp);
    for (int k = 0; k < n; k++) b[k] = subm(red_i64(e[k], q), tmp[k], q);
  }
  free(e);
  /* relinearisation key: s' = s^2 */
  u64* s2 = malloc(sizeof(u64) * (size_t)(L + 1) * n);
  for (int i = 0; i <= L; i++) {
    u64 q = c->q[i];
    for (int k = 0; k < n; k++)
      tmp[k] = mulm(c->s_eval[(size_t)i * n + k], c->s_eval[(size_t)i * n + k], q);
    from_eval(&c->tab[i], tmp, s2 + (size_t)i * n);
  }
  int rc = make_switch_key(c, &c->relin, L - 1, s2, 4, 5, 0);
  free(s2);
  free(tmp);
  c->have_keys = 1;
  return rc;
}

/* X -> X^g on one limb in coefficient form: X^i maps to +-X^(ig mod N) */
void orc_automorphism(const u64* a, u64* out, int log_n, u64 g, u64 q) {
  u64 n = 1ull << log_n, two_n = 2 * n;
  for (u64 i = 0; i < n; i++) {
    u64 e = (i * g) % two_n;
    if (e < n)
      out[e] = a[i];
    else
      out[e - n] = a[i] ? q - a[i] : 0;
  }
}

static u64 galois_elt(const orc_ctx* c, int step) {
  return c->rot5[step];
}

int orc_galois_keygen(orc_ctx* c, int step, int max_level) {
  if (!c->have_keys) return ORC_ENOKEY;
  int half = c->n / 2;
  step %= half;
  if (step < 0) step += half;
  if (step == 0) return ORC_EINVAL;
  if (max_level < 0 || max_level >= c->L) max_level = c->L - 1;
  if (c->gal[step]) {
    if (c->gal[step]->max_level >= max_level) return ORC_OK;
    key_free(c->gal[step]);
    free(c->gal[step]);
    c->gal[step] = NULL;
  }
  int n = c->n, L = c->L;
  u64 g = galois_elt(c, step);
  u64* sp = malloc(sizeof(u64) * (size_t)(L + 1) * n);
  u64* tmp = malloc(sizeof(u64) * (size_t)n);
  for (int i = 0; i <= L; i++) {
    for (int k = 0; k < n; k++) tmp[k] = red_i64(c->s[k], c->q[i]);
    orc_automorphism(tmp, sp + (size_t)i * n, c->log_n, g, c->q[i]);
  }
  orc_key* k = calloc(1, sizeof *k);
  int rc = make_switch_key(c, k, max_level, sp, 6, 7, (u32)step * 256u);
  free(sp);
  free(tmp);
  if (rc) {
    key_free(k);
    free(k);
    return rc;
  }
  c->gal[step] = k;
  return ORC_OK;
}

int orc_export_secret(const orc_ctx* c, i64* s) {
  if (!c->have_keys) return ORC_ENOKEY;
  memcpy(s, c->s, sizeof(i64) * (size_t)c->n);
  return ORC_OK;
}
int orc_export_pk(const orc_ctx* c, u64* out) {
  if (!c->have_keys) return ORC_ENOKEY;
  memcpy(out, c->pk, sizeof(u64) * 2 * (size_t)c->L * c->n);
  return ORC_OK;
}
static const orc_key* find_key(const orc_ctx* c, int kind, int step) {
  if (!c->have_keys) return NULL;
  if (kind == 0) return &c->relin;
  int half = c->n / 2;
  step %= half;
  if (step < 0) step += half;
  return c->gal[step];
}
int orc_key_max_level(const orc_ctx* c, int kind, int step) {
  const orc_key* k = find_key(c, kind, step);
  return k ? k->max_level : ORC_ENOKEY;
}
int orc_export_key(const orc_ctx* c, int kind, int step, u64* out) {
  const orc_key* k = find_key(c, kind, step);
  if (!k) return ORC_ENOKEY;
  size_t sz = (size_t)(k->max_level + 1) * 2 * (size_t)(k->max_level + 2) * c->n;
  memcpy(out, k->data, sizeof(u64) * sz);
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Encoding (reading of "a CKKSVector holds N/2 real values"):          */
/* slot j <-> zeta^(5^j mod 2N), zeta = exp(i pi / N).  For real z the  */
/* inverse canonical embedding is m_k = (2/N) sum_j z_j cos(pi 5^j k/N) */
/* and coefficient k is round(scale * m_k), ties away from zero.  The   */
/* sum is taken in long double with a rigorous error bound; a value     */
/* that the bound cannot separate from a rounding boundary is redone in */
/* __float128.                                                          */
/* ------------------------------------------------------------------ */
int orc_encode_coeffs(const orc_ctx* c, const double* z, size_t nz,
                      double scale, i64* coeffs) {
  int n = c->n;
  if (nz > (size_t)(n / 2)) return ORC_ERANGE;
  u64 two_n = 2ull * (u64)n;
  long double sumabs = 0;
  size_t nnz = 0;
  for (size_t j = 0; j < nz; j++) {
    if (!isfinite(z[j])) return ORC_ERANGE;
    if (z[j] != 0) nnz++;
    sumabs += fabsl((long double)z[j]);
  }
  const long double u = ldexpl(1.0L, -63); /* long double unit, doubled */
  long double fac = (long double)scale * 2.0L / (long double)n;
  long double bound = 2.0L * fac * ((long double)nnz + 4.0L) * u * sumabs;
  for (int k = 0; k < n; k++) {
    long double acc = 0;
    for (size_t j = 0; j < nz; j++) {
      if (z[j] == 0) continue;
      u64 t = (c->rot5[j] * (u64)k) % two_n;
      acc += (long double)z[j] * c->cos_ld[t];
    }
    long double v = acc * fac;
    long double av = fabsl(v);
    long double fl = floorl(av);
    long double fr = av - fl;
    i64 mag;
    if (fabsl(fr - 0.5L) <= bound + 2.0L * u * av) {
      __float128 accq = 0;
      for (size_t j = 0; j < nz; j++) {
        if (z[j] == 0) continue;
        u64 t = (c->rot5[j] * (u64)k) % two_n;
        accq += (__float128)z[j] * c->cos_q[t];
      }
      __float128 vq = accq * (__float128)scale * 2 / (__float128)n;
      __float128 aq = fabsq(vq);
      if (aq >= 4611686018427387904.0Q) return ORC_ERANGE; /* 2^62 */
      mag = (i64)floorq(aq + 0.5Q);
      v = (long double)vq;
    } else {
      if (av >= 4611686018427387904.0L) return ORC_ERANGE;
      mag = (i64)fl + (fr >= 0.5L ? 1 : 0);
    }
    coeffs[k] = v < 0 ? -mag : mag;
  }
  return ORC_OK;
}

orc_pt* orc_pt_from_coeffs(const orc_ctx* c, const i64* coeffs, double scale,
                           int level) {
  orc_pt* pt = orc_pt_new(c, level, scale);
  if (!pt) return NULL;
  for (int i = 0; i <= level; i++)
    for (int k = 0; k < c->n; k++)
      pt->data[(size_t)i * c->n + k] = red_i64(coeffs[k], c->q[i]);
  return pt;
}

orc_pt* orc_encode(const orc_ctx* c, const double* z, size_t n, double scale,
                   int level) {
  if (level < 0 || level >= c->L) FAIL(ORC_ELEVEL);
  i64* co = malloc(sizeof(i64) * (size_t)c->n);
  if (!co) FAIL(ORC_ENOMEM);
  int rc = orc_encode_coeffs(c, z, n, scale, co);
  if (rc) {
    free(co);
    FAIL(rc);
  }
  orc_pt* pt = orc_pt_from_coeffs(c, co, scale, level);
  free(co);
  return pt;
}

/* ---- CRT: centred integer value of each coefficient (little bignums) ---- */
#define BW (MAXP + 2)
typedef struct {
  u64 w[BW];
} big;
static void big_zero(big* a) { memset(a, 0, sizeof *a); }
static void big_mul_u64(big* a, u64 m) { /* a *= m */
  u64 carry = 0;
  for (int i = 0; i < BW; i++) {
    u128 t = (u128)a->w[i] * m + carry;
    a->w[i] = (u64)t;
    carry = (u64)(t >> 64);
  }
}
static void big_addmul(big* acc, const big* a, u64 m) { /* acc += a*m */
  u64 carry = 0;
  for (int i = 0; i < BW; i++) {
    u128 t = (u128)a->w[i] * m + acc->w[i] + carry;
    acc->w[i] = (u64)t;
    carry = (u64)(t >> 64);
  }
}
static int big_cmp(const big* a, const big* b) {
  for (int i = BW - 1; i >= 0; i--) {
    if (a->w[i] != b->w[i]) return a->w[i] < b->w[i] ? -1 : 1;
  }
  return 0;
}
static void big_sub(big* a, const big* b) { /* a -= b, a >= b */
  u64 borrow = 0;
  for (int i = 0; i < BW; i++) {
    u64 bi = b->w[i];
    u64 d = a->w[i] - bi - borrow;
    borrow = (a->w[i] < bi || (a->w[i] == bi && borrow)) ? 1 : 0;
    a->w[i] = d;
  }
}
static long double big_to_ld(const big* a) {
  long double r = 0;
  for (int i = BW - 1; i >= 0; i--) r = r * 18446744073709551616.0L + (long double)a->w[i];
  return r;
}

int orc_pt_centered(const orc_ctx* c, const orc_pt* pt, long double* out) {
  int l = pt->level, n = c->n;
  big Q, half, qhat[MAXP];
  u64 inv[MAXP];
  big_zero(&Q);
  Q.w[0] = 1;
  for (int i = 0; i <= l; i++) big_mul_u64(&Q, c->q[i]);
  for (int i = 0; i <= l; i++) {
    big_zero(&qhat[i]);
    qhat[i].w[0] = 1;
    u64 r = 1;
    for (int j = 0; j <= l; j++)
      if (j != i) {
        big_mul_u64(&qhat[i], c->q[j]);
        r = mulm(r, c->q[j] % c->q[i], c->q[i]);
      }
    inv[i] = invm(r, c->q[i]);
  }
  /* half = floor(Q / 2) */
  half = Q;
  for (int i = 0; i < BW; i++) {
    half.w[i] >>= 1;
    if (i + 1 < BW) half.w[i] |= Q.w[i + 1] << 63;
  }
  for (int k = 0; k < n; k++) {
    big x;
    big_zero(&x);
    for (int i = 0; i <= l; i++)
      big_addmul(&x, &qhat[i], mulm(pt->data[(size_t)i * n + k], inv[i], c->q[i]));
    while (big_cmp(&x, &Q) >= 0) big_sub(&x, &Q);
    if (big_cmp(&x, &half) > 0) {
      big y = Q;
      big_sub(&y, &x);
      out[k] = -big_to_ld(&y);
    } else {
      out[k] = big_to_ld(&x);
    }
  }
  return ORC_OK;
}

/* z_j = Re m(zeta^(5^j)) / scale = sum_k m_k cos(pi 5^j k / N) / scale */
int orc_decode(const orc_ctx* c, const orc_pt* pt, double* z, size_t nz) {
  int n = c->n;
  if (nz > (size_t)(n / 2)) return ORC_ERANGE;
  long double* m = malloc(sizeof(long double) * (size_t)n);
  if (!m) return ORC_ENOMEM;
  orc_pt_centered(c, pt, m);
  u64 two_n = 2ull * (u64)n;
  for (size_t j = 0; j < nz; j++) {
    long double acc = 0;
    for (int k = 0; k < n; k++) {
      if (m[k] == 0) continue;
      acc += m[k] * c->cos_ld[(c->rot5[j] * (u64)k) % two_n];
    }
    z[j] = (double)(acc / (long double)pt->scale);
  }
  free(m);
  return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Encryption.  Public key: (v*pk0 + e0 + m, v*pk1 + e1), v ternary    */
/* (tag 8), e0, e1 Gaussian (tags 9, 10), stream index = enc_index.    */
/* Secret key: (-a*s + e + m, a), a uniform (tag 11, enc_index, i),     */
/* e Gaussian (tag 12).                                                 */
/* ------------------------------------------------------------------ */
orc_ct* orc_encrypt(const orc_ctx* c, const orc_pt* pt, u32 idx, int use_sk) {
  if (!c->have_keys) FAIL(ORC_ENOKEY);
  int n = c->n, l = pt->level;
  orc_ct* ct = orc_ct_new(c, l, pt->scale);
  if (!ct) return NULL;
  u64* A = malloc(sizeof(u64) * (size_t)n);
  u64* B = malloc(sizeof(u64) * (size_t)n);
  i64* e0 = malloc(sizeof(i64) * (size_t)n);
  i64* e1 = malloc(sizeof(i64) * (size_t)n);
  i64* v = malloc(sizeof(i64) * (size_t)n);
  if (use_sk) {
    orc_sample_gaussian(c->seed, 12, idx, n, e0);
    for (int i = 0; i <= l; i++) {
      u64 q = c->q[i];
      u64* c0 = ct_limb(c, ct, 0, i);
      u64* c1 = ct_limb(c, ct, 1, i);
      orc_sample_uniform(c->seed, 11, idx, (u32)i, q, n, c1);
      to_eval(&c->tab[i], c1, A);
      for (int k = 0; k < n; k++) A[k] = mulm(A[k], c->s_eval[(size_t)i * n + k], q);
      from_eval(&c->tab[i], A, A);
      for (int k = 0; k < n; k++)
        c0[k] = addm(subm(red_i64(e0[k], q), A[k], q), pt->data[(size_t)i * n + k], q);
    }
  } else {
    orc_sample_ternary(c->seed, 8, idx, n, v);
    orc_sample_gaussian(c->seed, 9, idx, n, e0);
    orc_sample_gaussian(c->seed, 10, idx, n, e1);
    for (int i = 0; i <= l; i++) {
      u64 q = c->q[i];
      const ntt_tab* tb = &c->tab[i];
      u64* c0 = ct_limb(c, ct, 0, i);
      u64* c1 = ct_limb(c, ct, 1, i);
      for (int k = 0; k < n; k++) B[k] = red_i64(v[k], q);
      to_eval(tb, B, B);
      to_eval(tb, c->pk + (size_t)i * n, A);
      for (int k = 0; k < n; k++) A[k] = mulm(A[k], B[k], q);
      from_eval(tb, A, A);
      for (int k = 0; k < n; k++)
        c0[k] = addm(addm(A[k], red_i64(e0[k], q), q), pt->data[(size_t)i * n + k], q);
      to_eval(tb, c->pk + ((size_t)c->L + i) * n, A);
      for (int k = 0; k < n; k++) A[k] = mulm(A[k], B[k], q);
      from_eval(tb, A, A);
      for (int k = 0; k < n; k++) c1[k] = addm(A[k], red_i64(e1[k], q), q);
    }
  }
  free(A);
  free(B);
  free(e0);
  free(e1);
  free(v);
  return ct;
}

orc_pt* orc_decrypt(const orc_ctx* c, const orc_ct* ct) {
  if (!c->have_keys) FAIL(ORC_ENOKEY);
  int n = c->n, l = ct->level;
  orc_pt* pt = orc_pt_new(c, l, ct->scale);
  if (!pt) return NULL;
  u64* A = malloc(sizeof(u64) * (size_t)n);
  for (int i = 0; i <= l; i++) {
    u64 q = c->q[i];
    to_eval(&c->tab[i], ct_limb(c, ct, 1, i), A);
    for (int k = 0; k < n; k++) A[k] = mulm(A[k], c->s_eval[(size_t)i * n + k], q);
    from_eval(&c->tab[i], A, A);
    const u64* c0 = ct_limb(c, ct, 0, i);
    for (int k = 0; k < n; k++) pt->data[(size_t)i * n + k] = addm(c0[k], A[k], q);
  }
  free(A);
  return pt;
}

/* ------------------------------------------------------------------ */
/* Level alignment (drop limbs, exact) and scale check (relative 2^-20) */
/* ------------------------------------------------------------------ */
orc_ct* orc_drop_to(const orc_ctx* c, const orc_ct* a, int level) {
  if (level > a->level || level < 0) FAIL(ORC_ELEVEL);
  orc_ct* r = orc_ct_new(c, level, a->scale);
  if (!r) return NULL;
  for (int k = 0; k < 2; k++)
    for (int i = 0; i <= level; i++)
      memcpy(ct_limb(c, r, k, i), ct_limb(c, a, k, i), sizeof(u64) * (size_t)c->n);
  return r;
}
static int scales_match(double a, double b) {
  double m = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
  return fabs(a - b) <= ldexp(m, -20);
}

static orc_ct* addsub(const orc_ctx* c, const orc_ct* a, const orc_ct* b, int sub) {
  if (!scales_match(a->scale, b->scale)) FAIL(ORC_ESCALE);
  int l = a->level < b->level ? a->level : b->level;
  orc_ct* r = orc_ct_new(c, l, a->scale);
  if (!r) return NULL;
  for (int k = 0; k < 2; k++)
    for (int i = 0; i <= l; i++) {
      u64 q = c->q[i];
      const u64* x = ct_limb(c, a, k, i);
      const u64* y = ct_limb(c, b, k, i);
      u64* z = ct_limb(c, r, k, i);
      for (int t = 0; t < c->n; t++) z[t] = sub ? subm(x[t], y[t], q) : addm(x[t], y[t], q);
    }
  return r;
}
orc_ct* orc_add(const orc_ctx* c, const orc_ct* a, const orc_ct* b) { return addsub(c, a, b, 0); }
orc_ct* orc_sub(const orc_ctx* c, const orc_ct* a, const orc_ct* b) { return addsub(c, a, b, 1); }

orc_ct* orc_negate(const orc_ctx* c, const orc_ct* a) {
  orc_ct* r = orc_ct_new(c, a->level, a->scale);
  if (!r) return NULL;
  for (int k = 0; k < 2; k++)
    for (int i = 0; i <= a->level; i++) {
      u64 q = c->q[i];
      const u64* x = ct_limb(c, a, k, i);
      u64* z = ct_limb(c, r, k, i);
      for (int t = 0; t < c->n; t++) z[t] = x[t] ? q - x[t] : 0;
    }
  return r;
}

orc_ct* orc_add_plain(const orc_ctx* c, const orc_ct* a, const orc_pt* p) {
  if (!scales_match(a->scale, p->scale)) FAIL(ORC_ESCALE);
  if (p->level < a->level) FAIL(ORC_ELEVEL);
  orc_ct* r = orc_ct_new(c, a->level, a->scale);
  if (!r) return NULL;
  memcpy(r->data, a->data, sizeof(u64) * 2 * (size_t)(a->level + 1) * c->n);
  for (int i = 0; i <= a->level; i++) {
    u64 q = c->q[i];
    u64* z = ct_limb(c, r, 0, i);
    const u64* y = p->data + (size_t)i * c->n;
    for (int t = 0; t < c->n; t++) z[t] = addm(z[t], y[t], q);
  }
  return r;
}

/* c0 - p: the plaintext subtracted from the first polynomial (section 3,  */
/* element-wise operations with plain vectors)                            */
orc_ct* orc_sub_plain(const orc_ctx* c, const orc_ct* a, const orc_pt* p) {
  if (!scales_match(a->scale, p->scale)) FAIL(ORC_ESCALE);
  if (p->level < a->level) FAIL(ORC_ELEVEL);
  orc_ct* r = orc_ct_new(c, a->level, a->scale);
  if (!r) return NULL;
  memcpy(r->data, a->data, sizeof(u64) * 2 * (size_t)(a->level + 1) * c->n);
  for (int i = 0; i <= a->level; i++) {
    u64 q = c->q[i];
    u64* z = ct_limb(c, r, 0, i);
    const u64* y = p->data + (size_t)i * c->n;
    for (int t = 0; t < c->n; t++) z[t] = subm(z[t], y[t], q);
  }
  return r;
}

orc_ct* orc_mul_plain(const orc_ctx* c, const orc_ct* a, const orc_pt* p) {
  if (p->level < a->level) FAIL(ORC_ELEVEL);
  int n = c->n;
  orc_ct* r = orc_ct_new(c, a->level, a->scale * p->scale);
  if (!r) return NULL;
  u64* P = malloc(sizeof(u64) * (size_t)n);
  u64* A = malloc(sizeof(u64) * (size_t)n);
  for (int i = 0; i <= a->level; i++) {
    u64 q = c->q[i];
    to_eval(&c->tab[i], p->data + (size_t)i * n, P);
    for (int k = 0; k < 2; k++) {
      to_eval(&c->tab[i], ct_limb(c, a, k, i), A);
      for (int t = 0; t < n; t++) A[t] = mulm(A[t], P[t], q);
      from_eval(&c->tab[i], A, ct_limb(c, r, k, i));
    }
  }
  free(P);
  free(A);
  return r;
}

/* ------------------------------------------------------------------ */
/* Key switching of one polynomial d at level l.                        */
/*  ModUp: digit j = [d]_{q_j} taken CENTRED in (-q_j/2, q_j/2), lifted  */
/*         to every modulus q_0..q_l and p.                               */
/*  Inner product: u_k = sum_j digit_j * evk_j[k].                       */
/*  ModDown: out = round(u / p): with h = (p-1)/2 and r = [u + h]_p,     */
/*         out_i = (u_i + h - r) * p^-1 mod q_i.                         */
/* ------------------------------------------------------------------ */
static int key_switch_poly(const orc_ctx* c, const orc_key* key, const u64* d,
                           int l, u64* out) {
  int n = c->n, nm = key->max_level + 2;
  if (key->max_level < l) return ORC_ENOKEY;
  u64* u = malloc(sizeof(u64) * 2 * (size_t)(l + 2) * n); /* [2][l+2][N] */
  u64* D = malloc(sizeof(u64) * (size_t)n);
  u64* acc0 = malloc(sizeof(u64) * (size_t)n);
  u64* acc1 = malloc(sizeof(u64) * (size_t)n);
  if (!u || !D || !acc0 || !acc1) return ORC_ENOMEM;
  for (int m = 0; m <= l + 1; m++) {
    int pi = (m <= l) ? m : c->L;   /* prime of this modulus */
    int kt = (m <= l) ? m : nm - 1; /* its index inside the key */
    u64 qt = c->q[pi];
    const ntt_tab* tb = &c->tab[pi];
    memset(acc0, 0, sizeof(u64) * (size_t)n);
    memset(acc1, 0, sizeof(u64) * (size_t)n);
    for (int j = 0; j <= l; j++) {
      u64 qj = c->q[j];
      const u64* dj = d + (size_t)j * n;
      for (int t = 0; t < n; t++) {
        i64 v = dj[t] > (qj - 1) / 2 ? (i64)dj[t] - (i64)qj : (i64)dj[t];
        D[t] = red_i64(v, qt);
      }
      to_eval(tb, D, D);
      const u64* e0 = key->eval + (((size_t)j * 2 + 0) * nm + kt) * n;
      const u64* e1 = key->eval + (((size_t)j * 2 + 1) * nm + kt) * n;
      for (int t = 0; t < n; t++) {
        acc0[t] = addm(acc0[t], mulm(D[t], e0[t], qt), qt);
        acc1[t] = addm(acc1[t], mulm(D[t], e1[t], qt), qt);
      }
    }
    from_eval(tb, acc0, u + ((size_t)0 * (l + 2) + m) * n);
    from_eval(tb, acc1, u + ((size_t)1 * (l + 2) + m) * n);
  }
  u64 p = c->q[c->L], h = (p - 1) / 2;
  for (int k = 0; k < 2; k++) {
    const u64* up = u + ((size_t)k * (l + 2) + l + 1) * n;
    for (int i = 0; i <= l; i++) {
      u64 q = c->q[i];
      u64 pinv = invm(p % q, q);
      u64 hq = h % q;
      const u64* ui = u + ((size_t)k * (l + 2) + i) * n;
      u64* o = out + ((size_t)k * (l + 1) + i) * n;
      for (int t = 0; t < n; t++) {
        u64 r = addm(up[t], h, p);
        o[t] = mulm(subm(addm(ui[t], hq, q), r % q, q), pinv, q);
      }
    }
  }
  free(u);
  free(D);
  free(acc0);
  free(acc1);
  return ORC_OK;
}

int orc_key_switch(const orc_ctx* c, int kind, int step, const u64* d, int level,
                   u64* out) {
  const orc_key* k = find_key(c, kind, step);
  if (!k) return ORC_ENOKEY;
  return key_switch_poly(c, k, d, level, out);
}

orc_ct* orc_mul_relin(const orc_ctx* c, const orc_ct* a, const orc_ct* b) {
  if (!c->have_keys) FAIL(ORC_ENOKEY);
  int l = a->level < b->level ? a->level : b->level, n = c->n;
  orc_ct* r = orc_ct_new(c, l, a->scale * b->scale);
  if (!r) return NULL;
  u64* d2 = malloc(sizeof(u64) * (size_t)(l + 1) * n);
  u64* A0 = malloc(sizeof(u64) * (size_t)n);
  u64* A1 = malloc(sizeof(u64) * (size_t)n);
  u64* B0 = malloc(sizeof(u64) * (size_t)n);
  u64* B1 = malloc(sizeof(u64) * (size_t)n);
  u64* T = malloc(sizeof(u64) * (size_t)n);
  for (int i = 0; i <= l; i++) {
    u64 q = c->q[i];
    const ntt_tab* tb = &c->tab[i];
    to_eval(tb, ct_limb(c, a, 0, i), A0);
    to_eval(tb, ct_limb(c, a, 1, i), A1);
    to_eval(tb, ct_limb(c, b, 0, i), B0);
    to_eval(tb, ct_limb(c, b, 1, i), B1);
    for (int t = 0; t < n; t++) T[t] = mulm(A0[t], B0[t], q);
    from_eval(tb, T, ct_limb(c, r, 0, i)); /* d0 */
    for (int t = 0; t < n; t++) T[t] = addm(mulm(A0[t], B1[t], q), mulm(A1[t], B0[t], q), q);
    from_eval(tb, T, ct_limb(c, r, 1, i)); /* d1 */
    for (int t = 0; t < n; t++) T[t] = mulm(A1[t], B1[t], q);
    from_eval(tb, T, d2 + (size_t)i * n); /* d2 */
  }
  u64* ks = malloc(sizeof(u64) * 2 * (size_t)(l + 1) * n);
  int rc = key_switch_poly(c, &c->relin, d2, l, ks);
  if (rc == ORC_OK) {
    for (int k = 0; k < 2; k++)
      for (int i = 0; i <= l; i++) {
        u64 q = c->q[i];
        u64* z = ct_limb(c, r, k, i);
        const u64* y = ks + ((size_t)k * (l + 1) + i) * n;
        for (int t = 0; t < n; t++) z[t] = addm(z[t], y[t], q);
      }
  }
  free(d2);
  free(A0);
  free(A1);
  free(B0);
  free(B1);
  free(T);
  free(ks);
  if (rc) {
    orc_ct_free(r);
    FAIL(rc);
  }
  return r;
}

/* Rescale: round(c / q_l) mod Q_{l-1}; the new scale is scale / q_l.     */
/* With h = (q_l-1)/2, r = [c_l + h]_{q_l}: c_i <- (c_i + h - r) q_l^-1.  */
orc_ct* orc_rescale(const orc_ctx* c, const orc_ct* a) {
  int l = a->level, n = c->n;
  if (l < 1) FAIL(ORC_ELEVEL);
  u64 ql = c->q[l], h = (ql - 1) / 2;
  orc_ct* r = orc_ct_new(c, l - 1, a->scale / (double)ql);
  if (!r) return NULL;
  for (int k = 0; k < 2; k++) {
    const u64* xl = ct_limb(c, a, k, l);
    for (int i = 0; i < l; i++) {
      u64 q = c->q[i];
      u64 inv = invm(ql % q, q), hq = h % q;
      const u64* xi = ct_limb(c, a, k, i);
      u64* o = ct_limb(c, r, k, i);
      for (int t = 0; t < n; t++) {
        u64 rr = addm(xl[t], h, ql);
        o[t] = mulm(subm(addm(xi[t], hq, q), rr % q, q), inv, q);
      }
    }
  }
  return r;
}

/* Left rotation by step: tau_g with g = 5^step mod 2N on both polys, then */
/* key switch of tau_g(c1) from tau_g(s) back to s.                        */
orc_ct* orc_rotate(const orc_ctx* c, const orc_ct* a, int step) {
  int half = c->n / 2, n = c->n, l = a->level;
  step %= half;
  if (step < 0) step += half;
  orc_ct* r = orc_ct_new(c, l, a->scale);
  if (!r) return NULL;
  if (step == 0) {
    memcpy(r->data, a->data, sizeof(u64) * 2 * (size_t)(l + 1) * n);
    return r;
  }
  const orc_key* key = c->gal[step];
  if (!key || key->max_level < l) {
    orc_ct_free(r);
    FAIL(ORC_ENOKEY);
  }
  u64 g = galois_elt(c, step);
  u64* t1 = malloc(sizeof(u64) * (size_t)(l + 1) * n);
  for (int i = 0; i <= l; i++) {
    orc_automorphism(ct_limb(c, a, 0, i), ct_limb(c, r, 0, i), c->log_n, g, c->q[i]);
    orc_automorphism(ct_limb(c, a, 1, i), t1 + (size_t)i * n, c->log_n, g, c->q[i]);
  }
  u64* ks = malloc(sizeof(u64) * 2 * (size_t)(l + 1) * n);
  int rc = key_switch_poly(c, key, t1, l, ks);
  if (rc == ORC_OK) {
    for (int i = 0; i <= l; i++) {
      u64 q = c->q[i];
      u64* z0 = ct_limb(c, r, 0, i);
      u64* z1 = ct_limb(c, r, 1, i);
      const u64* y0 = ks + (size_t)i * n;
      const u64* y1 = ks + ((size_t)(l + 1) + i) * n;
      for (int t = 0; t < n; t++) {
        z0[t] = addm(z0[t], y0[t], q);
        z1[t] = y1[t];
      }
    }
  }
  free(t1);
  free(ks);
  if (rc) {
    orc_ct_free(r);
    FAIL(rc);
  }
  return r;
}

/* ------------------------------------------------------------------ */
/* Composites                                                           */
/* ------------------------------------------------------------------ */
static int ceil_log2(uint32_t n) {
  int k = 0;
  while ((1u << k) < n) k++;
  return k;
}
/* x <- x + rot(x, stride * 2^j), j = 0 .. ceil(log2 count) - 1 */
static orc_ct* rotate_and_sum(const orc_ctx* c, orc_ct* x, uint32_t count,
                              uint32_t stride) {
  int steps = ceil_log2(count);
  for (int j = 0; j < steps; j++) {
    orc_ct* r = orc_rotate(c, x, (int)(stride << j));
    if (!r) {
      orc_ct_free(x);
      return NULL;
    }
    orc_ct* y = orc_add(c, x, r);
    orc_ct_free(r);
    orc_ct_free(x);
    if (!y) return NULL;
    x = y;
  }
  return x;
}

/* dot-product style slot sum: slot 0 gets the sum of slots 0..n-1 */
orc_ct* orc_sum_slots(const orc_ctx* c, const orc_ct* a, uint32_t n) {
  if (n == 0 || n > (uint32_t)c->n / 2) FAIL(ORC_ERANGE);
  orc_ct* x = orc_drop_to(c, a, a->level);
  if (!x) return NULL;
  return rotate_and_sum(c, x, n, 1);
}

/* add a vector held in slots 0..len-1, encoded at the ciphertext's scale */
static orc_ct* add_slot_vector(const orc_ctx* c, orc_ct* x, const double* v,
                               uint32_t len) {
  orc_pt* p = orc_encode(c, v, len, x->scale, x->level);
  if (!p) {
    orc_ct_free(x);
    return NULL;
  }
  orc_ct* y = orc_add_plain(c, x, p);
  orc_pt_free(p);
  orc_ct_free(x);
  return y;
}

/* im2col convolution on one ciphertext (section 3.2, appendix A.4).  The  */
/* input slot k*windows + w holds pixel k of window w (vertical scan of the */
/* windows-by-kk im2col matrix).  Multiply by the kernel replicated over    */
/* windows, rescale, sum the kk blocks with ceil(log2 kk) left rotations by */
/* windows * 2^j, and add the bias to slots 0..windows-1.                   */
orc_ct* orc_conv_im2col(const orc_ctx* c, const orc_ct* x, const double* kernel,
                        uint32_t kk, uint32_t windows, double bias) {
  uint32_t half = (uint32_t)c->n / 2;
  if (kk == 0 || windows == 0 || (uint64_t)kk * windows > half) FAIL(ORC_ERANGE);
  double* v = calloc(half, sizeof(double));
  for (uint32_t k = 0; k < kk; k++)
    for (uint32_t w = 0; w < windows; w++) v[k * windows + w] = kernel[k];
  orc_pt* p = orc_encode(c, v, (size_t)kk * windows, c->scale, x->level);
  free(v);
  if (!p) return NULL;
  orc_ct* m = orc_mul_plain(c, x, p);
  orc_pt_free(p);
  if (!m) return NULL;
  orc_ct* y = orc_rescale(c, m);
  orc_ct_free(m);
  if (!y) return NULL;
  y = rotate_and_sum(c, y, kk, windows);
  if (!y) return NULL;
  double* b = malloc(sizeof(double) * windows);
  for (uint32_t w = 0; w < windows; w++) b[w] = bias;
  y = add_slot_vector(c, y, b, windows);
  free(b);
  return y;
}

/* Vector-matrix product (section 3.1): replicate x (zero beyond n_in) R    */
/* times, R the largest power of two with n_in * R <= N/2, as x plus its    */
/* right rotations by n_in * m, m = 1..R-1; then                            */
/* y = sum_i rot_left(x_rep, i) * diag_i with                               */
/* diag_i[j] = W[(i + j) mod n_in][j] for j < n_out (0 elsewhere); one      */
/* rescale after the sum; bias added to slots 0..n_out-1.                   */
orc_ct* orc_matmul(const orc_ctx* c, const orc_ct* x, const double* w,
                   uint32_t n_in, uint32_t n_out, const double* bias) {
  uint32_t half = (uint32_t)c->n / 2;
  if (n_in == 0 || n_out == 0 || n_in > half || n_out > half) FAIL(ORC_ERANGE);
  /* replication: R copies (the largest power of two that fits), the input  */
  /* plus its right rotations by n_in * m, m = 1..R-1, each rotation of the  */
  /* input itself                                                            */
  uint32_t reps = 1;
  while ((uint64_t)n_in * reps * 2 <= half) reps *= 2;
  orc_ct* xr = orc_drop_to(c, x, x->level);
  if (!xr) return NULL;
  for (uint32_t m = 1; m < reps; m++) {
    orc_ct* r = orc_rotate(c, x, (int)((half - n_in * m) % half));
    if (!r) {
      orc_ct_free(xr);
      return NULL;
    }
    orc_ct* y = orc_add(c, xr, r);
    orc_ct_free(r);
    orc_ct_free(xr);
    if (!y) return NULL;
    xr = y;
  }
  if ((uint64_t)n_in + n_out - 1 > (uint64_t)n_in * reps) {
    orc_ct_free(xr);
    FAIL(ORC_ERANGE);
  }
  double* d = calloc(n_out, sizeof(double));
  orc_ct* acc = NULL;
  int ok = 1;
  for (uint32_t i = 0; i < n_in && ok; i++) {
    orc_ct* r = orc_rotate(c, xr, (int)i);
    if (!r) {
      ok = 0;
      break;
    }
    for (uint32_t j = 0; j < n_out; j++) d[j] = w[(size_t)((i + j) % n_in) * n_out + j];
    orc_pt* p = orc_encode(c, d, n_out, c->scale, r->level);
    orc_ct* t = p ? orc_mul_plain(c, r, p) : NULL;
    orc_pt_free(p);
    orc_ct_free(r);
    if (!t) {
      ok = 0;
      break;
    }
    if (acc) {
      orc_ct* s = orc_add(c, acc, t);
      orc_ct_free(acc);
      orc_ct_free(t);
      acc = s;
      ok = acc != NULL;
    } else {
      acc = t;
    }
  }
  free(d);
  orc_ct_free(xr);
  if (!ok) {
    orc_ct_free(acc);
    return NULL;
  }
  orc_ct* y = orc_rescale(c, acc);
  orc_ct_free(acc);
  if (!y) return NULL;
  double* b = calloc(n_out, sizeof(double));
  if (bias)
    for (uint32_t j = 0; j < n_out; j++) b[j] = bias[j];
  y = add_slot_vector(c, y, b, n_out);
  free(b);
  return y;
}

/* Channel packing: mask part c to slots 0..width-1 (ones at the context  */
/* scale), rescale, rotate right by width*c, and add the parts.           */
orc_ct* orc_pack(const orc_ctx* c, orc_ct* const* parts, uint32_t n_parts,
                 uint32_t width) {
  uint32_t half = (uint32_t)c->n / 2;
  if (n_parts == 0 || width == 0 || (uint64_t)width * n_parts > half) FAIL(ORC_ERANGE);
  int l = parts[0]->level;
  for (uint32_t k = 1; k < n_parts; k++)
    if (parts[k]->level < l) l = parts[k]->level;
  double* ones = malloc(sizeof(double) * width);
  for (uint32_t w = 0; w < width; w++) ones[w] = 1.0;
  orc_pt* mask = orc_encode(c, ones, width, c->scale, l);
  free(ones);
  if (!mask) return NULL;
  orc_ct* acc = NULL;
  for (uint32_t k = 0; k < n_parts; k++) {
    orc_ct* a = orc_drop_to(c, parts[k], l);
    orc_ct* m = a ? orc_mul_plain(c, a, mask) : NULL;
    orc_ct_free(a);
    orc_ct* r = m ? orc_rescale(c, m) : NULL;
    orc_ct_free(m);
    if (r && k > 0) {
      orc_ct* t = orc_rotate(c, r, (int)(half - width * k));
      orc_ct_free(r);
      r = t;
    }
    if (!r) {
      orc_ct_free(acc);
      orc_pt_free(mask);
      return NULL;
    }
    if (acc) {
      orc_ct* s = orc_add(c, acc, r);
      orc_ct_free(acc);
      orc_ct_free(r);
      acc = s;
      if (!acc) break;
    } else {
      acc = r;
    }
  }
  orc_pt_free(mask);
  return acc;
}

orc_ct* orc_square(const orc_ctx* c, const orc_ct* a) {
  orc_ct* m = orc_mul_relin(c, a, a);
  if (!m) return NULL;
  orc_ct* r = orc_rescale(c, m);
  orc_ct_free(m);
  return r;
}

void orc_im2col(const double* img, uint32_t h, uint32_t w, uint32_t k,
                uint32_t stride, double* out) {
  uint32_t oh = (h - k) / stride + 1, ow = (w - k) / stride + 1;
  uint32_t windows = oh * ow;
  for (uint32_t ky = 0; ky < k; ky++)
    for (uint32_t kx = 0; kx < k; kx++)
      for (uint32_t oy = 0; oy < oh; oy++)
        for (uint32_t ox = 0; ox < ow; ox++)
          out[(size_t)(ky * k + kx) * windows + oy * ow + ox] =
              img[(size_t)(oy * stride + ky) * w + ox * stride + kx];
}

/* Section 5 network: conv (4 kernels 7x7, stride 3) -> pack -> square ->  */
/* FC 256->64 -> square -> FC 64->10.  Dimensions follow the arguments:     */
/* conv_k is [4][49], conv_b [4], w1 [256][64], b1 [64], w2 [64][10], b2.   */
orc_ct* orc_cnn(const orc_ctx* c, const orc_ct* x, const double* conv_k,
                const double* conv_b, const double* w1, const double* b1,
                const double* w2, const double* b2) {
  enum { CH = 4, KK = 49, WIN = 64, HID = 64, OUT = 10 };
  orc_ct* parts[CH] = {0};
  for (int ch = 0; ch < CH; ch++) {
    parts[ch] = orc_conv_im2col(c, x, conv_k + ch * KK, KK, WIN, conv_b[ch]);
    if (!parts[ch]) {
      for (int k = 0; k < ch; k++) orc_ct_free(parts[k]);
      return NULL;
    }
  }
  orc_ct* p = orc_pack(c, parts, CH, WIN);
  for (int k = 0; k < CH; k++) orc_ct_free(parts[k]);
  if (!p) return NULL;
  orc_ct* s1 = orc_square(c, p);
  orc_ct_free(p);
  if (!s1) return NULL;
  orc_ct* h = orc_matmul(c, s1, w1, CH * WIN, HID, b1);
  orc_ct_free(s1);
  if (!h) return NULL;
  orc_ct* s2 = orc_square(c, h);
  orc_ct_free(h);
  if (!s2) return NULL;
  orc_ct* o = orc_matmul(c, s2, w2, HID, OUT, b2);
  orc_ct_free(s2);
  return o;
}
