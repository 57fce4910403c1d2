// ckks.cpp -- host side of the MI355X RNS-CKKS library: context, prime chain
// and tables, caching device allocator, keys, encryption and every operation
// of include/ckks_hip.h, sequenced as kernel launches on the context stream.
//
// Ciphertext and plaintext polynomials live on the device in the NTT domain,
// limb-major [poly][limb][N] u64 with residues in [0, q_i).  Keys are kept in
// the NTT domain and in Montgomery form, layout [digit][poly][modulus][N].
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <functional>
#include <map>
#include <tuple>
#include <memory>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ckks_hip.h"
#include "device.h"
#include "encode.h"

typedef unsigned __int128 u128;

// ---------------------------------------------------------------- errors
static thread_local char g_msg[512];

static he_status fail(he_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_msg, sizeof g_msg, fmt, ap);
  va_end(ap);
  return code;
}

#define HIPC(x)                                                                      \
  do {                                                                               \
    hipError_t e_ = (x);                                                             \
    if (e_ != hipSuccess) return fail(HE_EHIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)
#define TRY(x)                 \
  do {                         \
    he_status s_ = (x);        \
    if (s_ != HE_OK) return s_; \
  } while (0)

// ---------------------------------------------------------------- host modular arithmetic
static u64 h_mulm(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }
static u64 h_powm(u64 a, u64 e, u64 q) {
  u64 r = 1;
  a %= q;
  for (; e; e >>= 1) {
    if (e & 1) r = h_mulm(r, a, q);
    a = h_mulm(a, a, q);
  }
  return r;
}
static u64 h_inv(u64 a, u64 q) { return h_powm(a % q, q - 2, q); }
static bool h_is_prime(u64 n) {
  if (n < 2) return false;
  const u64 small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
  for (u64 p : small)
    if (n % p == 0) return n == p;
  u64 d = n - 1;
  int s = 0;
  while ((d & 1) == 0) d >>= 1, s++;
  for (u64 a : small) {
    u64 x = h_powm(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int r = 1; r < s && comp; r++) {
      x = h_mulm(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}
static u64 h_shoup(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }
static uint32_t h_brv(uint32_t x, int bits) {
  uint32_t r = 0;
  for (int i = 0; i < bits; i++) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

// ---------------------------------------------------------------- allocator
struct Pool {
  he_alloc_fn alloc = nullptr;
  he_free_fn release = nullptr;
  void* user = nullptr;
  // the context's stream: every use of a block is ordered on it, so a block
  // goes back to the allocator only once the stream has drained
  hipStream_t st = nullptr;
  std::unordered_map<size_t, std::vector<void*>> cache;
  std::unordered_map<void*, size_t> live;
  size_t bytes_live = 0;

  void* raw_alloc(size_t b) {
    if (alloc) return alloc(b, user);
    void* p = nullptr;
    return hipMalloc(&p, b) == hipSuccess ? p : nullptr;
  }
  void raw_free(void* p, size_t b) {
    if (release)
      release(p, b, user);
    else
      (void)hipFree(p);
  }
  void trim() {
    if (cache.empty()) return;
    if (st) (void)hipStreamSynchronize(st);
    for (auto& kv : cache)
      for (void* p : kv.second) raw_free(p, kv.first);
    cache.clear();
  }
  void* get(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    if (bytes == 0) bytes = 256;
    auto it = cache.find(bytes);
    void* p = nullptr;
    if (it != cache.end() && !it->second.empty()) {
      p = it->second.back();
      it->second.pop_back();
    } else {
      p = raw_alloc(bytes);
      if (!p && !retain) {  // no stream synchronisation inside a graph capture
        trim();
        p = raw_alloc(bytes);
      }
      if (!p) return nullptr;
    }
    live[p] = bytes;
    bytes_live += bytes;
    return p;
  }
  // while a graph is captured, freed buffers stay with the graph (its
  // replays write them) instead of going back to the cache
  bool retain = false;
  std::vector<void*> retained;
  void put(void* p) {
    if (!p) return;
    auto it = live.find(p);
    if (it == live.end()) return;
    if (retain) {
      retained.push_back(p);
      return;
    }
    cache[it->second].push_back(p);
    bytes_live -= it->second;
    live.erase(it);
  }
  void destroy() {
    trim();
    for (auto& kv : live) raw_free(kv.first, kv.second);
    live.clear();
  }
};

// ---------------------------------------------------------------- objects
struct Key {
  int ml = -1;  // valid for levels 0..ml
  u64* d = nullptr;
  size_t bytes = 0;
};

struct ProfRec {
  std::string fam;
  hipEvent_t a, b;
  double units, bytes;  // limb-NTTs (NTT families) and algorithmic HBM bytes
};

struct he_ctx {
  int log_n = 0, n = 0, L = 0;
  std::vector<u64> q;  // L data primes then the special prime
  double scale = 0;
  int auto_rescale = 0;
  u64 seed = 0;
  hipStream_t st = nullptr;
  bool own_stream = false;
  int device = 0;
  Pool pool;
  PrimeDev* d_primes = nullptr;
  u64* d_fwd = nullptr;
  u64* d_inv = nullptr;
  u64* d_fwd_fp = nullptr;
  u64* d_inv_fp = nullptr;
  NttTables tabs{};
  bool capturing = false;  // a graph capture of st is open
  int fuse_max = 256;      // fused key switch when B*Lp^2 <= this, fused rescale when 2*n_ct*l <= this
  // rotate-and-sum chains in coefficient form (HE_COEF_ROT=0: in the
  // transform domain)
  int coef_rot = 1;
  int hoist_split_wgs = 4096;  // two-phase hoisted multiply-accumulate, about this many workgroups (0: one kernel)
  bool have_keys = false;
  u64* d_s = nullptr;   // [L+1][N]
  u64* d_pk = nullptr;  // [2][L][N]
  Key relin;
  std::map<int, Key> gal;
  EncodeTables enc;
  // the encoder's cosine table (double-double) and 5^j mod 2N on the device,
  // for the exact recomputation of the coefficients the FFT cannot round
  double* d_chi = nullptr;
  double* d_clo = nullptr;
  uint32_t* d_rot5 = nullptr;
  std::map<std::pair<int, int>, he_pt*> masks;
  bool prof = false;
  hipEvent_t ev_cross = nullptr;  // orders this stream against another context's (batches across contexts)
  std::vector<ProfRec> prof_recs;
  uint64_t key_epoch = 0;  // bumped whenever a key is (re)generated
  // divide-and-round constants for divisor prime s and target prime t:
  // (q_s mod q_t)^-1, its Shoup companion, and (q_s - 1)/2 mod q_t
  std::vector<u64> rd_inv, rd_inv_sh, rd_hq;
  // this device's fixed no-allocation scratch, and while a no-allocation
  // call runs, the bump arena carved from it (every intermediate of the
  // call comes from there instead of the pool)
  u64* scratch = nullptr;
  size_t scratch_words = 0;
  struct Arena {
    u64* base;
    size_t cap, used;  // words
  };
  Arena* arena = nullptr;
};

struct he_ct {
  he_ctx* ctx;
  int level;
  double scale;
  u64* d;
  std::shared_ptr<void> blk;  // set when d lies in a block shared by a batch
};
struct he_pt {
  he_ctx* ctx;
  int level;
  double scale;
  u64* d;
};

enum PlanKind { PLAN_CONV = 1, PLAN_MATMUL = 2 };
struct he_plan {
  he_ctx* ctx;
  int kind;
  int level;      // input level
  double scale;   // input scale
  uint32_t kk = 0, windows = 0;  // conv
  uint32_t n_in = 0, n_out = 0;  // matmul
  he_pt* kernel = nullptr;       // conv plaintext
  he_pt* bias = nullptr;         // at the post-rescale scale and level
  u64* diags = nullptr;          // matmul diagonals [n_in][level+1][N], NTT domain
  HoistItem* items = nullptr;    // device table of the hoisted rotations
  uint64_t items_epoch = ~0ull;
  HoistItem* rep_items = nullptr;  // device table of the replication rotations
  uint64_t rep_epoch = ~0ull;
};

// Every handle passed to a call must belong to that call's context.  A
// context's stream is the only thing that orders the kernels writing a
// handle's memory before the kernels reading it; a handle of another context
// would be read on this stream while its own stream may still be writing it
// (a race that shows only when the two streams overlap), and its buffers
// would return to the wrong pool.
template <class H>
static he_status own(const he_ctx* c, const H* h) {
  if (c && h && h->ctx != c) return fail(HE_EINVAL, "handle of another context");
  return HE_OK;
}
template <class H>
static he_status own_all(const he_ctx* c, const H* const* hs, size_t n) {
  if (hs)
    for (size_t i = 0; i < n; i++) TRY(own(c, hs[i]));
  return HE_OK;
}

namespace {

// ---------------------------------------------------------------- profiling
struct Prof {
  he_ctx* c;
  const char* fam;
  hipEvent_t a{}, b{};
  bool on;
  double units, bytes;
  hipStream_t st;  // the stream the timed launches go on (default: the context's)
  Prof(he_ctx* c_, const char* f, double units_ = 0, double bytes_ = 0, hipStream_t st_ = nullptr)
      : c(c_), fam(f), on(c_->prof && !c_->capturing && !c_->arena), units(units_), bytes(bytes_),
        st(st_ ? st_ : c_->st) {
    if (on) {
      (void)hipEventCreate(&a);
      (void)hipEventCreate(&b);
      (void)hipEventRecord(a, st);
    }
  }
  ~Prof() {
    if (on) {
      (void)hipEventRecord(b, st);
      c->prof_recs.push_back({fam, a, b, units, bytes});
    }
  }
};

// ---------------------------------------------------------------- buffers
struct DBuf {
  he_ctx* c = nullptr;
  u64* p = nullptr;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() {
    if (p) c->pool.put(p);
  }
};

// Device memory for one intermediate: from the pool, or (inside a
// no-allocation call) the next 256-byte-aligned slice of the scratch arena.
// Arena slices are never in the pool's table, so handing one to pool.put
// (DBuf, he_ct_free) does nothing.
static u64* ctx_alloc(he_ctx* c, size_t words) {
  if (c->arena) {
    he_ctx::Arena& a = *c->arena;
    const size_t w = (words + 31) & ~(size_t)31;
    if (w > a.cap - a.used) return nullptr;
    u64* p = a.base + a.used;
    a.used += w;
    return p;
  }
  return (u64*)c->pool.get(words * sizeof(u64));
}
static he_status alloc_failed(he_ctx* c, const char* what, size_t words) {
  if (c->arena)
    return fail(HE_ERANGE, "%s of %zu bytes exceeds the %u-byte no-allocation scratch", what,
                words * sizeof(u64), HE_NOALLOC_SCRATCH_BYTES);
  return fail(HE_EOOM, "%s of %zu bytes failed", what, words * sizeof(u64));
}

he_status dalloc(he_ctx* c, DBuf& b, size_t words) {
  b.c = c;
  b.p = ctx_alloc(c, words);
  if (!b.p) return alloc_failed(c, "device allocation", words);
  return HE_OK;
}

size_t ct_words(const he_ctx* c, int level) { return 2 * (size_t)(level + 1) * c->n; }
size_t pt_words(const he_ctx* c, int level) { return (size_t)(level + 1) * c->n; }

he_status new_ct(he_ctx* c, int level, double scale, he_ct** out) {
  u64* d = ctx_alloc(c, ct_words(c, level));
  if (!d) return alloc_failed(c, "ciphertext allocation", ct_words(c, level));
  *out = new he_ct{c, level, scale, d};
  return HE_OK;
}
he_status new_pt(he_ctx* c, int level, double scale, he_pt** out) {
  u64* d = ctx_alloc(c, pt_words(c, level));
  if (!d) return alloc_failed(c, "plaintext allocation", pt_words(c, level));
  *out = new he_pt{c, level, scale, d};
  return HE_OK;
}
struct CtGuard {  // frees an intermediate ciphertext on scope exit
  he_ct* p = nullptr;
  ~CtGuard() { he_ct_free(p); }
};
struct PtGuard {
  he_pt* p = nullptr;
  ~PtGuard() { he_pt_free(p); }
};

ModList mods_range(int n) {
  ModList m{};
  m.n = n;
  for (int i = 0; i < n; i++) m.p[i] = (unsigned char)i;
  return m;
}

bool scales_match(double a, double b) {
  double m = std::fmax(std::fabs(a), std::fabs(b));
  return std::fabs(a - b) <= std::ldexp(m, -20);
}

// ---------------------------------------------------------------- NTT helpers
// in-place or out-of-place batched transform of n_poly polys x n_limbs limbs
he_status ntt_rows(he_ctx* c, bool fwd, const u64* src, u64* dst, int n_poly, int n_limbs,
                   long long poly_stride_src, long long poly_stride_dst) {
  NttJob J{};
  J.src = src;
  J.dst = dst;
  J.na = n_poly;
  J.nb = n_limbs;
  J.sa = poly_stride_src;
  J.sb = c->n;
  J.da = poly_stride_dst;
  J.db = c->n;
  J.src_prime = 0;
  for (int i = 0; i < n_limbs; i++) J.dst_prime[i] = (unsigned char)i;
  Prof pr(c, fwd ? "ntt_fwd" : "ntt_inv", (double)n_poly * n_limbs, 16.0 * c->n * n_poly * n_limbs);
  hipError_t e = fwd ? launch_ntt_fwd(c->log_n, PRO_PLAIN, EPI_STORE, J, c->d_primes, c->tabs, c->st)
                     : launch_ntt_inv(c->log_n, J, c->d_primes, c->tabs, c->st);
  if (e != hipSuccess) return fail(HE_EHIP, "ntt launch: %s", hipGetErrorString(e));
  return HE_OK;
}

// rows with an explicit prime per limb (keys: the last modulus is special)
he_status ntt_rows_mods(he_ctx* c, bool fwd, const u64* src, u64* dst, int n_poly, const ModList& mods) {
  NttJob J{};
  J.src = src;
  J.dst = dst;
  J.na = n_poly;
  J.nb = mods.n;
  J.sa = (long long)mods.n * c->n;
  J.sb = c->n;
  J.da = J.sa;
  J.db = c->n;
  J.src_prime = 0;
  for (int i = 0; i < mods.n; i++) J.dst_prime[i] = mods.p[i];
  Prof pr(c, fwd ? "ntt_fwd" : "ntt_inv", (double)n_poly * mods.n, 16.0 * c->n * n_poly * mods.n);
  hipError_t e = fwd ? launch_ntt_fwd(c->log_n, PRO_PLAIN, EPI_STORE, J, c->d_primes, c->tabs, c->st)
                     : launch_ntt_inv(c->log_n, J, c->d_primes, c->tabs, c->st);
  if (e != hipSuccess) return fail(HE_EHIP, "ntt launch: %s", hipGetErrorString(e));
  return HE_OK;
}

u64 galois_elt(const he_ctx* c, int step) {
  return h_powm(5, (u64)step, 2 * (u64)c->n);
}

int norm_step(const he_ctx* c, long long step) {
  long long half = c->n / 2;
  step %= half;
  if (step < 0) step += half;
  return (int)step;
}

// dst = round(u / q_src) over targets 0..n_t-1 for n_poly polynomials:
// src_coef [n_poly][N] holds the coefficient form of each divisor limb; u is
// the NTT-domain dividend, poly a at u + a*ua; result poly a at dst + a*da;
// optional addend at add + a*aa + t*N (every poly, or even polys only).
struct Addend {
  const u64* p = nullptr;
  long long aa = 0;
  int even_only = 0;
  const u64* gals = nullptr;   // read p at the Galois source of item a / 2
  const u64* p2 = nullptr;     // second addend (every poly)
  long long a2a = 0;
};
// the divide-and-round transform job: dst[a][t] = (u[a][t] - NTT_t(r - h)) * q_s^-1
// (+ addends), r the rounding lift of src_coef[a] (coefficients mod q_s)
static NttJob round_div_job(const he_ctx* c, int n_poly, const u64* src_coef, int src_prime, const u64* u,
                            long long ua, u64* dst, long long da, int n_t, const Addend& add) {
  NttJob J{};
  J.src = src_coef;
  J.sa = c->n;
  J.sb = 0;
  J.dst = dst;
  J.da = da;
  J.db = c->n;
  J.na = n_poly;
  J.nb = n_t;
  J.src_prime = src_prime;
  J.u = u;
  J.ua = ua;
  J.ub = c->n;
  J.add = add.p;
  J.aa = add.aa;
  J.ab = c->n;
  J.add_even_only = add.even_only;
  J.add2 = add.p2;
  J.a2a = add.a2a;
  if (add.gals) {
    J.add_gather = 1;
    for (int a = 0; a < (n_poly + 1) / 2 && a < HE_MAX_BATCH; a++) J.gal[a] = add.gals[a];
  }
  J.h_src = (c->q[src_prime] - 1) / 2;
  const size_t np = c->q.size();
  for (int t = 0; t < n_t; t++) {
    J.dst_prime[t] = (unsigned char)t;
    J.hq[t] = c->rd_hq[src_prime * np + t];
    J.inv[t] = c->rd_inv[src_prime * np + t];
    J.inv_sh[t] = c->rd_inv_sh[src_prime * np + t];
  }
  return J;
}

he_status round_div(he_ctx* c, int n_poly, const u64* src_coef, int src_prime, const u64* u, long long ua,
                    u64* dst, long long da, int n_t, Addend add, const char* fam) {
  const NttJob J = round_div_job(c, n_poly, src_coef, src_prime, u, ua, dst, da, n_t, add);
  // per job: divisor limb, dividend limb, optional addend read; result written
  const double jobs = (double)n_poly * n_t;
  Prof pr(c, fam, jobs, 8.0 * c->n * jobs * (add.p ? 4.0 : 3.0));
  hipError_t e = launch_ntt_fwd(c->log_n, PRO_ROUNDDIV_LIFT, EPI_ROUNDDIV, J, c->d_primes, c->tabs, c->st);
  if (e != hipSuccess) return fail(HE_EHIP, "round_div launch: %s", hipGetErrorString(e));
  return HE_OK;
}

// ModUp of B items: centred digit j of item b (coefficient form, [B][Lp][N])
// lifted to every other modulus (data 0..Lp-1, then the special prime) and
// transformed into ext [B][Lp][nm][N]; the diagonal slots ext[b][j][j] are
// left out (they are the input limbs themselves).
he_status modup(he_ctx* c, const u64* coef, int B, int Lp, u64* ext) {
  const int n = c->n, nm = Lp + 1;
  NttJob J{};
  J.src = coef;
  J.sa = n;
  J.sb = 0;
  J.dst = ext;
  J.da = (long long)nm * n;
  J.db = n;
  J.na = B * Lp;
  J.nb = nm;
  J.skip_diag = 1;
  J.src_prime = -1;
  J.amod = Lp;
  for (int t = 0; t < nm; t++) J.dst_prime[t] = (unsigned char)(t < Lp ? t : c->L);
  Prof pr(c, "modup", (double)B * Lp * Lp, 16.0 * n * B * Lp * Lp);
  hipError_t e = launch_ntt_fwd(c->log_n, PRO_CENTRED_LIFT, EPI_STORE, J, c->d_primes, c->tabs, c->st);
  if (e != hipSuccess) return fail(HE_EHIP, "modup: %s", hipGetErrorString(e));
  return HE_OK;
}

// ---------------------------------------------------------------- key switching
// calls that synchronise or copy from host memory are refused while a graph
// capture is open (a captured host copy would replay from freed memory)
#define NO_CAPTURE(c)                                                                  \
  do {                                                                                 \
    if ((c) && (c)->capturing)                                                         \
      return fail(HE_EINVAL, "%s: not allowed during a graph capture", __func__);       \
  } while (0)

// ---------------------------------------------------------------- fused key switch
// Small batches: ModUp in three launches (inverse block phase; inverse
// column phase + centred lift + forward column phase; forward block phase),
// ModDown in three (inner product on p + inverse block phase; inverse
// column phase + rounding lift + forward column phase; forward block phase
// with the data-limb inner product, the division and the addends).
static bool ks_fusable(const he_ctx* c, int B, int Lp) {
  return (long long)B * Lp * Lp <= c->fuse_max;
}

struct KsBufs {
  DBuf t1, t2, ext, t3, t4, t5;
};

// fills K for B items at level l; allocates the intermediates
static he_status ks_prepare(he_ctx* c, int B, const u64* d, long long ds, int l, const Key* const* keys,
                            const u64* gals, KsJob& K, KsBufs& bufs, bool moddown) {
  const int n = c->n, Lp = l + 1, nm = Lp + 1;
  TRY(dalloc(c, bufs.t1, (size_t)B * Lp * n));
  TRY(dalloc(c, bufs.t2, (size_t)B * Lp * Lp * n));
  TRY(dalloc(c, bufs.ext, (size_t)B * Lp * nm * n));
  if (moddown) {
    TRY(dalloc(c, bufs.t3, (size_t)2 * B * n));
    TRY(dalloc(c, bufs.t4, (size_t)2 * B * Lp * n));
    TRY(dalloc(c, bufs.t5, (size_t)2 * B * Lp * n));
  }
  K = KsJob{};
  K.B = B;
  K.Lp = Lp;
  K.nm = nm;
  K.special = c->L;
  K.d = d;
  K.ds = ds;
  for (int b = 0; b < B; b++) {
    K.gal[b] = gals ? gals[b] : 1;
    K.key[b] = keys ? keys[b]->d : nullptr;
    K.km[b] = keys ? keys[b]->ml + 2 : 0;
  }
  K.t1 = bufs.t1.p;
  K.t2 = bufs.t2.p;
  K.ext = bufs.ext.p;
  K.t3 = bufs.t3.p;
  K.t4 = bufs.t4.p;
  K.t5 = bufs.t5.p;
  const size_t np = c->q.size();
  K.h_src = (c->q[c->L] - 1) / 2;
  for (int t = 0; t < Lp; t++) {
    K.hq[t] = c->rd_hq[c->L * np + t];
    K.inv[t] = c->rd_inv[c->L * np + t];
    K.inv_sh[t] = c->rd_inv_sh[c->L * np + t];
  }
  return HE_OK;
}

// ext [B][Lp][nm][N] = ModUp of the (gathered) inputs
static he_status modup_fused(he_ctx* c, const KsJob& K, bool gather) {
  const int n = c->n, B = K.B, Lp = K.Lp, nm = K.nm;
  Prof pr(c, "modup", (double)B * Lp * (1 + Lp), 8.0 * n * B * Lp * (1 + Lp));
  NttJob J{};
  J.src = K.d;
  J.sa = K.ds;
  J.sb = n;
  J.na = B;
  J.nb = Lp;
  for (int i = 0; i < Lp; i++) J.dst_prime[i] = (unsigned char)i;
  if (gather) {
    J.gather_src = 1;
    J.gal_div = 1;
    for (int b = 0; b < B; b++) J.gal[b] = K.gal[b];
  }
  J.mid = K.t1;
  hipError_t e = launch_ntt_inv_blocks(c->log_n, J, c->d_primes, c->tabs, 1, c->st);
  if (e == hipSuccess) e = launch_ks_modup_cols(c->log_n, K, c->d_primes, c->tabs, c->st);
  if (e == hipSuccess) {
    NttJob F{};
    F.dst = K.ext;
    F.da = (long long)nm * n;
    F.db = n;
    F.na = B * Lp;
    F.nb = nm;
    F.skip_diag = 1;
    F.src_prime = -1;
    F.amod = Lp;
    for (int t = 0; t < nm; t++) F.dst_prime[t] = (unsigned char)(t < Lp ? t : c->L);
    F.mid = K.t2;
    e = launch_ntt_fwd_blocks(c->log_n, PRO_CENTRED_LIFT, EPI_STORE, F, c->d_primes, c->tabs, c->st);
  }
  if (e != hipSuccess) return fail(HE_EHIP, "fused modup: %s", hipGetErrorString(e));
  return HE_OK;
}

// out = ModDown(inner products) + addends
static he_status moddown_fused(he_ctx* c, KsJob& K, const Addend& add, u64* out) {
  const int n = c->n, B = K.B, Lp = K.Lp, nm = K.nm;
  K.out = out;
  K.oa = (long long)Lp * n;
  K.add = add.p;
  K.aa = add.aa;
  K.add_even_only = add.even_only;
  K.add_gather = add.gals ? 1 : 0;
  K.add2 = add.p2;
  K.a2a = add.a2a;
  // algorithmic bytes: each distinct key 2*Lp*nm limbs (read once however
  // many items share it); per item the digits Lp*nm limbs, addends read and
  // 2*Lp limbs written
  const double adds = (add.p ? (add.even_only ? 1.0 : 2.0) : 0.0) + (add.p2 ? 2.0 : 0.0);
  int distinct = 0;
  for (int b = 0; b < B; b++) {
    bool seen = false;
    for (int a = 0; a < b; a++) seen |= K.key[a] == K.key[b];
    distinct += seen ? 0 : 1;
  }
  Prof pr(c, "moddown", 2.0 * B * (1 + Lp),
          8.0 * n * (2.0 * distinct * Lp * nm + B * (Lp * nm + 2.0 * Lp + adds * Lp)));
  hipError_t e = launch_ks_special_blocks(c->log_n, K, c->d_primes, c->tabs, c->st);
  if (e == hipSuccess) e = launch_ks_moddown_cols(c->log_n, K, c->d_primes, c->tabs, c->st);
  if (e == hipSuccess) e = launch_ks_moddown_blocks(c->log_n, K, c->d_primes, c->tabs, c->st);
  if (e != hipSuccess) return fail(HE_EHIP, "fused moddown: %s", hipGetErrorString(e));
  return HE_OK;
}

// ModDown fused with the rescale that follows it: out [B][2][l][N] =
// Rescale(ModDown(inner products) + addends), l = Lp - 1 (the division by p
// and by q_l with both roundings of the two separate steps, in three
// launches instead of six)
static he_status moddown_rescale_fused(he_ctx* c, KsJob& K, const Addend& add, u64* out) {
  const int n = c->n, B = K.B, Lp = K.Lp, nm = K.nm, l = Lp - 1;
  K.out = out;
  K.oa = (long long)l * n;
  K.add = add.p;
  K.aa = add.aa;
  K.add_even_only = add.even_only;
  K.add_gather = add.gals ? 1 : 0;
  K.add2 = add.p2;
  K.a2a = add.a2a;
  K.resc = 1;
  const size_t np = c->q.size();
  K.pl = c->q[c->L] % c->q[l];
  K.pl_sh = h_shoup(K.pl, c->q[l]);
  K.h_l = (c->q[l] - 1) / 2;
  for (int t = 0; t < l; t++) {
    K.hq2[t] = c->rd_hq[l * np + t];
    K.inv2[t] = c->rd_inv[l * np + t];
    K.inv2_sh[t] = c->rd_inv_sh[l * np + t];
  }
  const double adds = (add.p ? (add.even_only ? 1.0 : 2.0) : 0.0) + (add.p2 ? 2.0 : 0.0);
  int distinct = 0;
  for (int b = 0; b < B; b++) {
    bool seen = false;
    for (int a = 0; a < b; a++) seen |= K.key[a] == K.key[b];
    distinct += seen ? 0 : 1;
  }
  // as the ModDown (keys, digits, addends) with l limbs written per poly
  Prof pr(c, "moddown", 2.0 * B * (1 + Lp),
          8.0 * n * (2.0 * distinct * Lp * nm + B * (Lp * nm + 2.0 * l + adds * Lp)));
  hipError_t e = launch_ks_special_blocks(c->log_n, K, c->d_primes, c->tabs, c->st);
  if (e == hipSuccess) e = launch_ks_moddown_resc_cols(c->log_n, K, c->d_primes, c->tabs, c->st);
  if (e == hipSuccess) e = launch_ks_moddown_resc_blocks(c->log_n, K, c->d_primes, c->tabs, c->st);
  if (e != hipSuccess) return fail(HE_EHIP, "fused moddown + rescale: %s", hipGetErrorString(e));
  return HE_OK;
}

// Key switch of B polynomials at level l: item b's input d + b*ds (NTT domain
// [l+1][N]), read at the Galois source of gals[b] when gals is given (the
// rotated poly without materialising it), with keys[b];
// out [B][2][l+1][N] = KeySwitch(d_b) + addends, or with resc (only where
// ks_fusable(c, B, l + 1) and l >= 1) out [B][2][l][N] = that rescaled.
he_status key_switch(he_ctx* c, int B, const u64* d, long long ds, int l, const Key* const* keys,
                     const u64* gals, Addend add, u64* out, bool resc = false) {
  const int n = c->n, Lp = l + 1, nm = Lp + 1;
  if (B < 1 || B > HE_MAX_BATCH) return fail(HE_EINVAL, "key-switch batch of %d", B);
  for (int b = 0; b < B; b++)
    if (keys[b]->ml < l)
      return fail(HE_ENOKEY, "key valid up to level %d, ciphertext at level %d", keys[b]->ml, l);
  if (resc && (l < 1 || !ks_fusable(c, B, Lp))) return fail(HE_EINVAL, "fused rescale outside the fused form");
  if (ks_fusable(c, B, Lp)) {
    KsJob K;
    KsBufs bufs;
    TRY(ks_prepare(c, B, d, ds, l, keys, gals, K, bufs, true));
    DBuf t3b;
    if (resc) {
      TRY(dalloc(c, t3b, (size_t)2 * B * n));
      K.t3b = t3b.p;
    }
    TRY(modup_fused(c, K, gals != nullptr));
    return resc ? moddown_rescale_fused(c, K, add, out) : moddown_fused(c, K, add, out);
  }
  DBuf coef, ext, u, ucoef;
  TRY(dalloc(c, coef, (size_t)B * Lp * n));
  TRY(dalloc(c, ext, (size_t)B * Lp * nm * n));
  TRY(dalloc(c, u, (size_t)B * 2 * nm * n));
  TRY(dalloc(c, ucoef, (size_t)B * 2 * n));
  {  // coefficient form of (the rotation of) each input
    NttJob J{};
    J.src = d;
    J.dst = coef.p;
    J.na = B;
    J.nb = Lp;
    J.sa = ds;
    J.sb = n;
    J.da = (long long)Lp * n;
    J.db = n;
    for (int i = 0; i < Lp; i++) J.dst_prime[i] = (unsigned char)i;
    if (gals) {
      J.gather_src = 1;
      J.gal_div = 1;
      for (int b = 0; b < B; b++) J.gal[b] = gals[b];
    }
    Prof pr(c, "ntt_inv", (double)B * Lp, 16.0 * n * B * Lp);
    hipError_t e = launch_ntt_inv(c->log_n, J, c->d_primes, c->tabs, c->st);
    if (e != hipSuccess) return fail(HE_EHIP, "intt: %s", hipGetErrorString(e));
  }
  TRY(modup(c, coef.p, B, Lp, ext.p));
  {
    InnerJob I{};
    I.ext = ext.p;
    I.diag = d;
    I.diag_stride = ds;
    I.u = u.p;
    I.B = B;
    I.n_dig = Lp;
    I.special_prime = c->L;
    for (int b = 0; b < B; b++) {
      I.key[b] = keys[b]->d;
      I.km[b] = keys[b]->ml + 2;
      I.gal[b] = gals ? gals[b] : 1;
    }
    // per item: key 2 Lp nm limbs + digits Lp nm limbs read, 2 nm written
    Prof pr(c, "keyswitch_inner", (double)B, 8.0 * n * B * (3.0 * Lp * nm + 2.0 * nm));
    hipError_t e = launch_inner(c->log_n, I, c->d_primes, c->st);
    if (e != hipSuccess) return fail(HE_EHIP, "inner: %s", hipGetErrorString(e));
  }
  {  // special-prime limbs back to coefficients
    NttJob J{};
    J.src = u.p + (size_t)Lp * n;
    J.sa = (long long)nm * n;
    J.dst = ucoef.p;
    J.da = n;
    J.na = 2 * B;
    J.nb = 1;
    J.dst_prime[0] = (unsigned char)c->L;
    Prof pr(c, "ntt_inv", 2.0 * B, 16.0 * n * 2 * B);
    hipError_t e = launch_ntt_inv(c->log_n, J, c->d_primes, c->tabs, c->st);
    if (e != hipSuccess) return fail(HE_EHIP, "intt special: %s", hipGetErrorString(e));
  }
  return round_div(c, 2 * B, ucoef.p, c->L, u.p, (long long)nm * n, out, (long long)Lp * n, Lp, add, "moddown");
}

// Left rotations of B ciphertexts stored contiguously ([B][2][l+1][N] at in)
// by steps[b]: the key switch reads tau_g(c1) by gather and adds tau_g(c0)
// (gathered) in its last kernel; with add_in, also adds the input itself
// (x + rot(x), the rotate-and-sum step).  out: [B][2][l+1][N].
// key_ctx (nullable): item b's Galois key comes from key_ctx[b] instead of c
he_status rotate_multi(he_ctx* c, const u64* in, int B, int l, const int* steps, u64* out, bool add_in = false,
                       he_ctx* const* key_ctx = nullptr) {
  const int n = c->n, Lp = l + 1;
  const Key* keys[HE_MAX_BATCH];
  u64 gals[HE_MAX_BATCH];
  for (int b = 0; b < B; b++) {
    const auto& gal = key_ctx ? key_ctx[b]->gal : c->gal;
    auto it = gal.find(steps[b]);
    if (it == gal.end()) return fail(HE_ENOKEY, "no Galois key for step %d", steps[b]);
    if (it->second.ml < l)
      return fail(HE_ENOKEY, "Galois key for step %d cut at level %d, ciphertext at %d", steps[b], it->second.ml, l);
    keys[b] = &it->second;
    gals[b] = galois_elt(c, steps[b]);
  }
  Addend add;
  add.p = in;
  add.aa = (long long)Lp * n;
  add.even_only = 1;
  add.gals = gals;
  if (add_in) {
    add.p2 = in;
    add.a2a = (long long)Lp * n;
  }
  return key_switch(c, B, in + (size_t)Lp * n, 2LL * Lp * n, l, keys, gals, add, out);
}

// Left rotations of B coefficient-form ciphertexts ([B][2][l+1][N] at in) by
// steps[b] into coefficient form at out; with add_in, out = in + rot(in).
// Only in the fused form (ks_fusable): four launches per rotation (ModUp
// from the automorphism's source coefficients, its block stages, inner
// products + inverse block stages, inverse column stages + division +
// addends), the residues those of rotate_multi on the transformed input.
static bool coef_rotations(const he_ctx* c, int B, int Lp) { return c->coef_rot && ks_fusable(c, B, Lp); }

he_status rotate_multi_coef(he_ctx* c, const u64* in, int B, int l, const int* steps, u64* out, bool add_in) {
  const int n = c->n, Lp = l + 1, nm = Lp + 1;
  if (B < 1 || B > HE_MAX_BATCH) return fail(HE_EINVAL, "rotation batch of %d", B);
  if (!coef_rotations(c, B, Lp)) return fail(HE_EINVAL, "coefficient-form rotations outside the fused form");
  KsJob K{};
  K.B = B;
  K.Lp = Lp;
  K.nm = nm;
  K.special = c->L;
  for (int b = 0; b < B; b++) {
    auto it = c->gal.find(steps[b]);
    if (it == c->gal.end()) return fail(HE_ENOKEY, "no Galois key for step %d", steps[b]);
    if (it->second.ml < l)
      return fail(HE_ENOKEY, "Galois key for step %d cut at level %d, ciphertext at %d", steps[b], it->second.ml, l);
    K.key[b] = it->second.d;
    K.km[b] = it->second.ml + 2;
    const u64 g = galois_elt(c, steps[b]);
    K.gal[b] = g;
    K.ginv[b] = h_powm(g, (u64)n - 1, 2 * (u64)n);  // the group of odd residues mod 2N has order N
  }
  DBuf t2, ext, t3;
  TRY(dalloc(c, t2, (size_t)B * Lp * nm * n));
  TRY(dalloc(c, ext, (size_t)B * Lp * nm * n));
  TRY(dalloc(c, t3, (size_t)2 * B * nm * n));
  K.cin = in;
  K.t2 = t2.p;
  K.ext = ext.p;
  K.t3 = t3.p;
  K.out = out;
  K.oa = (long long)Lp * n;
  K.add = in;
  K.aa = (long long)Lp * n;
  K.add_even_only = 1;
  K.add_gather = 1;
  if (add_in) {
    K.add2 = in;
    K.a2a = (long long)Lp * n;
  }
  const size_t np = c->q.size();
  K.h_src = (c->q[c->L] - 1) / 2;
  for (int t = 0; t < Lp; t++) {
    K.hq[t] = c->rd_hq[c->L * np + t];
    K.inv[t] = c->rd_inv[c->L * np + t];
    K.inv_sh[t] = c->rd_inv_sh[c->L * np + t];
  }
  NttJob F{};
  F.dst = ext.p;
  F.da = (long long)nm * n;
  F.db = n;
  F.na = B * Lp;
  F.nb = nm;
  F.mid = t2.p;
  for (int t = 0; t < nm; t++) F.dst_prime[t] = (unsigned char)(t < Lp ? t : c->L);
  int distinct = 0;
  for (int b = 0; b < B; b++) {
    bool seen = false;
    for (int a = 0; a < b; a++) seen |= K.key[a] == K.key[b];
    distinct += seen ? 0 : 1;
  }
  hipError_t e;
  {
    // the digits read, every (item, digit, modulus) written
    Prof pr(c, "modup", (double)B * Lp * nm, 8.0 * n * B * Lp * (1 + nm));
    e = launch_cks_modup_cols(c->log_n, K, c->d_primes, c->tabs, c->st);
    if (e == hipSuccess)
      e = launch_ntt_fwd_blocks(c->log_n, PRO_CENTRED_LIFT, EPI_STORE, F, c->d_primes, c->tabs, c->st);
  }
  if (e == hipSuccess) {
    // as the ModDown: keys (each distinct one once), digits, addends, output
    const double adds = 1.0 + (add_in ? 2.0 : 0.0);
    Prof pr(c, "moddown", 2.0 * B * (1 + Lp),
            8.0 * n * (2.0 * distinct * Lp * nm + B * (Lp * nm + 2.0 * Lp + adds * Lp)));
    e = launch_cks_inner_blocks(c->log_n, K, c->d_primes, c->tabs, c->st);
    if (e == hipSuccess) e = launch_cks_moddown_cols(c->log_n, K, c->d_primes, c->tabs, c->st);
  }
  if (e != hipSuccess) return fail(HE_EHIP, "coefficient-form rotation: %s", hipGetErrorString(e));
  return HE_OK;
}

// rescale of n_ct ciphertexts [n_ct][2][l+1][N] (transform domain) into
// coefficient form [n_ct][2][l][N]: the inverse block stages of every limb,
// then per kept limb t the inverse column stages of limb t and of the
// dropped limb l and (x_t - lift_t(x_l)) q_l^-1 -- the column kernel of the
// coefficient-form rotations with the dropped limb in the special prime's
// place and no addends (two launches; the residues are those of the
// rescale followed by an inverse transform)
he_status rescale_to_coef(he_ctx* c, const u64* in, int n_ct, int l, u64* out) {
  const int n = c->n, nm = l + 1;
  if (l < 1) return fail(HE_ELEVEL, "no level left to rescale");
  if (n_ct < 1 || n_ct > HE_MAX_BATCH) return fail(HE_EINVAL, "rescale of %d ciphertexts", n_ct);
  DBuf t3;
  TRY(dalloc(c, t3, (size_t)2 * n_ct * nm * n));
  NttJob J{};
  J.src = in;
  J.sa = (long long)nm * n;
  J.sb = n;
  J.na = 2 * n_ct;
  J.nb = nm;
  for (int t = 0; t < nm; t++) J.dst_prime[t] = (unsigned char)t;
  J.mid = t3.p;
  KsJob K{};
  K.B = n_ct;
  K.Lp = l;
  K.nm = nm;
  K.special = l;
  K.t3 = t3.p;
  K.out = out;
  K.oa = (long long)l * n;
  const size_t np = c->q.size();
  K.h_src = (c->q[l] - 1) / 2;
  for (int t = 0; t < l; t++) {
    K.hq[t] = c->rd_hq[l * np + t];
    K.inv[t] = c->rd_inv[l * np + t];
    K.inv_sh[t] = c->rd_inv_sh[l * np + t];
  }
  // every limb read once, the kept limbs written
  Prof pr(c, "rescale", 2.0 * n_ct * nm, 8.0 * n * 2 * n_ct * (2.0 * l + 1));
  hipError_t e = launch_ntt_inv_blocks(c->log_n, J, c->d_primes, c->tabs, 2, c->st);
  if (e == hipSuccess) e = launch_cks_rescale_cols(c->log_n, K, c->d_primes, c->tabs, c->st);
  if (e != hipSuccess) return fail(HE_EHIP, "rescale into coefficient form: %s", hipGetErrorString(e));
  return HE_OK;
}

// rescale of n_ct contiguous ciphertexts [n_ct][2][l+1][N] -> [n_ct][2][l][N]
// add0 (nullable, n_ct = 1): a plaintext added to poly 0 of the result
he_status rescale_multi(he_ctx* c, const u64* in, int n_ct, int l, u64* out, const u64* add0 = nullptr) {
  const int n = c->n;
  if (l < 1) return fail(HE_ELEVEL, "no level left to rescale");
  if (add0 && n_ct != 1) return fail(HE_EINVAL, "rescale addend for one ciphertext only");
  if (2LL * n_ct * l <= c->fuse_max) {
    // three launches: inverse block phase of limb l; its inverse column
    // phase, rounding lift and forward column phase for each t < l; forward
    // block phase with the division epilogue
    DBuf t3, t4;
    TRY(dalloc(c, t3, (size_t)2 * n_ct * n));
    TRY(dalloc(c, t4, (size_t)2 * n_ct * l * n));
    const size_t np = c->q.size();
    KsJob K{};
    K.B = n_ct;
    K.Lp = l;
    K.nm = l + 1;
    K.special = l;
    K.t3 = t3.p;
    K.t4 = t4.p;
    K.h_src = (c->q[l] - 1) / 2;
    NttJob J{};
    J.src = in + (size_t)l * n;
    J.sa = (long long)(l + 1) * n;
    J.na = 2 * n_ct;
    J.nb = 1;
    J.dst_prime[0] = (unsigned char)l;
    J.mid = t3.p;
    NttJob F{};
    F.dst = out;
    F.da = (long long)l * n;
    F.db = n;
    F.na = 2 * n_ct;
    F.nb = l;
    F.u = in;
    F.ua = (long long)(l + 1) * n;
    F.ub = n;
    F.mid = t4.p;
    if (add0) {
      F.add = add0;
      F.aa = 0;
      F.ab = n;
      F.add_even_only = 1;
    }
    for (int t = 0; t < l; t++) {
      K.hq[t] = c->rd_hq[l * np + t];
      F.dst_prime[t] = (unsigned char)t;
      F.inv[t] = c->rd_inv[l * np + t];
      F.inv_sh[t] = c->rd_inv_sh[l * np + t];
    }
    // per poly: the dropped limb and the l kept limbs read, l limbs written
    Prof pr(c, "rescale", 2.0 * n_ct * (1 + l), 8.0 * n * 2 * n_ct * (2.0 * l + 1));
    hipError_t e = launch_ntt_inv_blocks(c->log_n, J, c->d_primes, c->tabs, 2, c->st);
    if (e == hipSuccess) e = launch_rescale_cols(c->log_n, K, c->d_primes, c->tabs, c->st);
    if (e == hipSuccess) e = launch_ntt_fwd_blocks(c->log_n, FAM_RESCALE, EPI_ROUNDDIV, F, c->d_primes, c->tabs, c->st);
    if (e != hipSuccess) return fail(HE_EHIP, "fused rescale: %s", hipGetErrorString(e));
    return HE_OK;
  }
  DBuf coef;
  TRY(dalloc(c, coef, 2 * (size_t)n_ct * n));
  {
    NttJob J{};
    J.src = in + (size_t)l * n;
    J.sa = (long long)(l + 1) * n;
    J.dst = coef.p;
    J.da = n;
    J.na = 2 * n_ct;
    J.nb = 1;
    J.dst_prime[0] = (unsigned char)l;
    Prof pr(c, "ntt_inv", 2.0 * n_ct, 16.0 * n * 2 * n_ct);
    hipError_t e = launch_ntt_inv(c->log_n, J, c->d_primes, c->tabs, c->st);
    if (e != hipSuccess) return fail(HE_EHIP, "rescale intt: %s", hipGetErrorString(e));
  }
  Addend add;
  if (add0) {
    add.p = add0;
    add.aa = 0;
    add.even_only = 1;
  }
  return round_div(c, 2 * n_ct, coef.p, l, in, (long long)(l + 1) * n, out, (long long)l * n, l, add,
                   "rescale");
}

// copy a ciphertext's limbs 0..level into a fresh buffer layout
he_status drop_copy(he_ctx* c, const he_ct* a, int level, he_ct** out) {
  TRY(new_ct(c, level, a->scale, out));
  const size_t row = (size_t)(level + 1) * c->n * sizeof(u64);
  for (int k = 0; k < 2; k++)
    HIPC(launch_copy(a->d + (size_t)k * (a->level + 1) * c->n, (*out)->d + (size_t)k * (level + 1) * c->n,
                     (long long)(row / sizeof(u64)), c->st));
  return HE_OK;
}

// bring two ciphertexts to a common level; the returned guards own copies
he_status align2(he_ctx* c, const he_ct* a, const he_ct* b, const he_ct** ra, const he_ct** rb, CtGuard& ga,
                 CtGuard& gb) {
  *ra = a;
  *rb = b;
  if (a->level > b->level) {
    TRY(drop_copy(c, a, b->level, &ga.p));
    *ra = ga.p;
  } else if (b->level > a->level) {
    TRY(drop_copy(c, b, a->level, &gb.p));
    *rb = gb.p;
  }
  return HE_OK;
}


// ---------------------------------------------------------------- key generation
// switching key from s' (NTT domain [L+1][N]) to s, valid up to level ml
he_status make_key(he_ctx* c, Key& key, int ml, const u64* sp, uint32_t tag_a, uint32_t tag_e, uint32_t base) {
  const int n = c->n, nd = ml + 1, nm = ml + 2;
  ModList pidx{};
  pidx.n = nm;
  for (int t = 0; t < nm; t++) pidx.p[t] = (unsigned char)(t <= ml ? t : c->L);
  DBuf A, E;
  TRY(dalloc(c, A, (size_t)nd * nm * n));
  TRY(dalloc(c, E, (size_t)nd * nm * n));
  {
    Prof pr(c, "sample");
    hipError_t e = launch_sample_uniform(c->log_n, c->seed, tag_a, base, nd, pidx, pidx, A.p, c->d_primes, c->st);
    if (e != hipSuccess) return fail(HE_EHIP, "sample uniform: %s", hipGetErrorString(e));
    for (int j = 0; j < nd; j++) {
      e = launch_sample_small(c->log_n, 1, c->seed, tag_e, base + (uint32_t)j, pidx, E.p + (size_t)j * nm * n,
                              c->d_primes, c->st);
      if (e != hipSuccess) return fail(HE_EHIP, "sample gaussian: %s", hipGetErrorString(e));
    }
  }
  TRY(ntt_rows_mods(c, true, A.p, A.p, nd, pidx));
  TRY(ntt_rows_mods(c, true, E.p, E.p, nd, pidx));
  const size_t words = (size_t)nd * 2 * nm * n;
  u64* kd = (u64*)c->pool.get(words * sizeof(u64));
  if (!kd) return fail(HE_EOOM, "key allocation failed");
  hipError_t e = launch_keygen_combine(c->log_n, A.p, E.p, c->d_s, sp, kd, nd, nm, pidx, c->L, c->d_primes, c->st);
  if (e != hipSuccess) {
    c->pool.put(kd);
    return fail(HE_EHIP, "keygen combine: %s", hipGetErrorString(e));
  }
  if (key.d) c->pool.put(key.d);
  key.d = kd;
  key.ml = ml;
  key.bytes = words * sizeof(u64);
  c->key_epoch++;
  return HE_OK;
}

he_status galois_key(he_ctx* c, int step, int ml) {
  if (!c->have_keys) return fail(HE_ENOKEY, "he_keygen must run first");
  step = norm_step(c, step);
  if (step == 0) return HE_OK;
  if (ml < 0 || ml >= c->L) ml = c->L - 1;
  auto it = c->gal.find(step);
  if (it != c->gal.end() && it->second.ml >= ml) return HE_OK;
  DBuf sp;
  TRY(dalloc(c, sp, (size_t)(c->L + 1) * c->n));
  AutJob A{};
  A.B = 1;
  A.rows_per_item = c->L + 1;
  A.g[0] = galois_elt(c, step);
  hipError_t e = launch_automorphism(c->log_n, c->d_s, sp.p, A, c->st);
  if (e != hipSuccess) return fail(HE_EHIP, "automorphism: %s", hipGetErrorString(e));
  Key& k = c->gal[step];
  return make_key(c, k, ml, sp.p, 6, 7, (uint32_t)step * 256u);
}

// ---------------------------------------------------------------- encode helpers
// z, nz, amb (nullable): the encoded values and the indices of the
// coefficients left for the exact recomputation on the device
he_status upload_coeffs(he_ctx* c, const int64_t* co, int level, double scale, he_pt** out,
                        const double* z = nullptr, size_t nz = 0, const std::vector<int>* amb = nullptr) {
  const int n = c->n, Lp = level + 1;
  const size_t na = amb ? amb->size() : 0;
  // the N signed coefficients go up once (with the values and indices the
  // exact recomputation needs); the device finishes, reduces them into every
  // limb and transforms
  he_pt* pt = nullptr;
  TRY(new_pt(c, level, scale, &pt));
  DBuf raw;
  he_status s = dalloc(c, raw, (size_t)n + (na ? nz + (na + 1) / 2 : 0));
  hipError_t e = hipSuccess;
  if (s == HE_OK) {
    double* dz = (double*)(raw.p + n);
    int* damb = (int*)(raw.p + n + nz);
    e = hipMemcpyAsync(raw.p, co, (size_t)n * sizeof(int64_t), hipMemcpyHostToDevice, c->st);
    if (e == hipSuccess && na) e = hipMemcpyAsync(dz, z, nz * sizeof(double), hipMemcpyHostToDevice, c->st);
    if (e == hipSuccess && na) e = hipMemcpyAsync(damb, amb->data(), na * sizeof(int), hipMemcpyHostToDevice, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);  // the sources are the caller's (pageable) memory
    if (e == hipSuccess && na)
      e = launch_encode_exact(c->log_n, dz, (int)nz, c->d_rot5, c->d_chi, c->d_clo, damb, (int)na,
                              2.0 * scale / (double)n, (int64_t*)raw.p, c->st);
    if (e == hipSuccess) e = launch_coeffs_to_limbs(c->log_n, (const int64_t*)raw.p, pt->d, Lp, c->d_primes, c->st);
    if (e != hipSuccess) s = fail(HE_EHIP, "plaintext upload: %s", hipGetErrorString(e));
  }
  if (s == HE_OK) s = ntt_rows(c, true, pt->d, pt->d, 1, Lp, 0, 0);
  if (s != HE_OK) {
    he_pt_free(pt);
    return s;
  }
  *out = pt;
  return HE_OK;
}

he_status encode_impl(he_ctx* c, const double* v, size_t n, double scale, int level, he_pt** out) {
  if (level < 0 || level >= c->L) return fail(HE_ELEVEL, "level %d outside 0..%d", level, c->L - 1);
  if (n > (size_t)c->n / 2) return fail(HE_ERANGE, "%zu values exceed N/2 = %d slots", n, c->n / 2);
  if (!(scale > 0) || !std::isfinite(scale)) return fail(HE_EINVAL, "bad scale");
  std::vector<int64_t> co(c->n);
  std::vector<int> amb;
  if (encode_coeffs(c->enc, v, n, scale, co.data(), &amb) != 0)
    return fail(HE_ERANGE, "encoded coefficient reaches 2^62 (or a value is not finite)");
  return upload_coeffs(c, co.data(), level, scale, out, v, n, &amb);
}

// coefficient form of rows (INTT on a copy) copied to the host
he_status download_coeff(he_ctx* c, const u64* d, int n_poly, int Lp, std::vector<u64>& h) {
  const size_t words = (size_t)n_poly * Lp * c->n;
  DBuf tmp;
  TRY(dalloc(c, tmp, words));
  TRY(ntt_rows(c, false, d, tmp.p, n_poly, Lp, (long long)Lp * c->n, (long long)Lp * c->n));
  h.resize(words);
  HIPC(hipMemcpyAsync(h.data(), tmp.p, words * sizeof(u64), hipMemcpyDeviceToHost, c->st));
  HIPC(hipStreamSynchronize(c->st));
  return HE_OK;
}

// centred value of each coefficient as a double (approximate CRT: the
// quotient sum_i y_i / q_i is rounded in FP64, the value itself is formed
// exactly mod 2^128, which holds any value a valid decryption produces)
void crt_centered(const he_ctx* c, const u64* res, int Lp, double* out) {
  const int n = c->n;
  std::vector<u64> inv(Lp);
  std::vector<u128> qhat(Lp);
  u128 Q = 1;
  for (int i = 0; i < Lp; i++) Q *= (u128)c->q[i];
  for (int i = 0; i < Lp; i++) {
    u64 r = 1;
    u128 h = 1;
    for (int j = 0; j < Lp; j++)
      if (j != i) {
        r = h_mulm(r, c->q[j] % c->q[i], c->q[i]);
        h *= (u128)c->q[j];
      }
    inv[i] = h_inv(r, c->q[i]);
    qhat[i] = h;
  }
  for (int k = 0; k < n; k++) {
    double frac = 0;
    u128 acc = 0;
    for (int i = 0; i < Lp; i++) {
      const u64 y = h_mulm(res[(size_t)i * n + k], inv[i], c->q[i]);
      frac += (double)y / (double)c->q[i];
      acc += (u128)y * qhat[i];
    }
    const u128 v = (u128)(unsigned long long)std::floor(frac + 0.5);
    acc -= v * Q;
    __int128 s = (__int128)acc;
    out[k] = (double)s;
  }
}

}  // namespace

// =================================================================== ABI
extern "C" {

const char* he_last_error(void) { return g_msg; }

he_status he_ctx_create(const he_params* P, he_alloc_fn alloc, he_free_fn free_fn, void* alloc_user,
                        void* hip_stream, he_ctx** out) {
  if (!P || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  if (P->log_n < 10 || P->log_n > 14) return fail(HE_EINVAL, "log_n %d outside 10..14", P->log_n);
  if (P->n_primes < 2 || P->n_primes > HE_MAX_PRIMES) return fail(HE_EINVAL, "n_primes %d", P->n_primes);
  if ((alloc == nullptr) != (free_fn == nullptr)) return fail(HE_EINVAL, "allocator needs both callbacks");
  const int n = 1 << P->log_n;
  // prime chain
  std::vector<u64> q;
  const u64 m = 2 * (u64)n;
  for (int i = 0; i < P->n_primes; i++) {
    const int b = P->prime_bits[i];
    if (b < P->log_n + 2 || b > 60) return fail(HE_EINVAL, "prime bit size %d outside %d..60", b, P->log_n + 2);
    u64 cand = (((1ull << b) - 2) / m) * m + 1;
    bool found = false;
    for (; cand > (1ull << (b - 1)); cand -= m) {
      bool used = false;
      for (u64 x : q) used |= (x == cand);
      if (!used && h_is_prime(cand)) {
        found = true;
        break;
      }
    }
    if (!found) return fail(HE_EINVAL, "no %d-bit prime = 1 mod 2N left", b);
    q.push_back(cand);
  }
  he_ctx* c = new he_ctx();
  c->log_n = P->log_n;
  c->n = n;
  c->L = P->n_primes - 1;
  c->q = q;
  c->scale = P->scale;
  c->auto_rescale = P->auto_rescale;
  c->seed = P->seed;
  c->pool.alloc = alloc;
  c->pool.release = free_fn;
  c->pool.user = alloc_user;
  if (hipGetDevice(&c->device) != hipSuccess) {
    delete c;
    return fail(HE_EHIP, "no HIP device");
  }
  if (hip_stream) {
    c->st = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(HE_EHIP, "stream creation failed");
    }
    c->own_stream = true;
  }
  c->pool.st = c->st;
  if (hipEventCreateWithFlags(&c->ev_cross, hipEventDisableTiming) != hipSuccess) {
    if (c->own_stream) (void)hipStreamDestroy(c->st);
    delete c;
    return fail(HE_EHIP, "event creation failed");
  }
  // this device's no-allocation scratch (a fixed array; looked up once per
  // device, with the device current)
  if (noalloc_scratch(c->device, &c->scratch, &c->scratch_words) != hipSuccess) {
    c->scratch = nullptr;
    c->scratch_words = 0;
  }
  c->scratch_words /= sizeof(u64);
  // per-prime constants and twiddles
  const int np = (int)q.size();
  std::vector<PrimeDev> hp(np);
  std::vector<u64> fwd((size_t)np * n * 2), inv((size_t)np * n * 2);
  std::vector<double> fwd_fp((size_t)np * n * 2), inv_fp((size_t)np * n * 2);
  for (int i = 0; i < np; i++) {
    const u64 qi = q[i];
    PrimeDev& d = hp[i];
    d.q = qi;
    d.k = 64 - __builtin_clzll(qi);
    d.mu = (u64)(((u128)1 << (2 * d.k)) / qi);
    d.mu64 = ~0ull / qi;
    u64 inv64 = 1;  // Newton: inverse of q mod 2^64
    for (int it = 0; it < 7; it++) inv64 *= 2 - qi * inv64;
    d.qinv_neg = (u64)0 - inv64;
    u64 r64 = (u64)((((u128)1) << 64) % qi);
    d.r2 = h_mulm(r64, r64, qi);
    d.ninv = h_inv((u64)n % qi, qi);
    d.ninv_sh = h_shoup(d.ninv, qi);
    // exact FP64 butterflies need every intermediate below 2^53: q < 2^50
    d.use_fp = qi < (1ull << 50) ? 1 : 0;
    d.qd = (double)qi;
    d.inv2qd = 1.0 / (2.0 * (double)qi);
    d.ninv_d = (double)d.ninv;
    d.ninv_qd = (double)d.ninv / (double)qi;
    // primitive 2N-th root of unity
    u64 psi = 0;
    for (u64 g = 2;; g++) {
      u64 x = h_powm(g, (qi - 1) / m, qi);
      if (h_powm(x, (u64)n, qi) == qi - 1) {
        psi = x;
        break;
      }
    }
    const u64 ipsi = h_inv(psi, qi);
    std::vector<u64> pw(n), ipw(n);
    pw[0] = ipw[0] = 1;
    for (int k = 1; k < n; k++) {
      pw[k] = h_mulm(pw[k - 1], psi, qi);
      ipw[k] = h_mulm(ipw[k - 1], ipsi, qi);
    }
    for (int k = 0; k < n; k++) {
      const uint32_t r = h_brv((uint32_t)k, P->log_n);
      const size_t o = ((size_t)i * n + k) * 2;
      fwd[o] = pw[r];
      fwd[o + 1] = h_shoup(pw[r], qi);
      inv[o] = ipw[r];
      inv[o + 1] = h_shoup(ipw[r], qi);
      fwd_fp[o] = (double)pw[r];
      fwd_fp[o + 1] = (double)pw[r] / (double)qi;
      inv_fp[o] = (double)ipw[r];
      inv_fp[o + 1] = (double)ipw[r] / (double)qi;
    }
  }
  c->d_primes = (PrimeDev*)c->pool.get(sizeof(PrimeDev) * np);
  c->d_fwd = (u64*)c->pool.get(fwd.size() * sizeof(u64));
  c->d_inv = (u64*)c->pool.get(inv.size() * sizeof(u64));
  c->d_fwd_fp = (u64*)c->pool.get(fwd_fp.size() * sizeof(double));
  c->d_inv_fp = (u64*)c->pool.get(inv_fp.size() * sizeof(double));
  if (!c->d_primes || !c->d_fwd || !c->d_inv || !c->d_fwd_fp || !c->d_inv_fp) {
    he_ctx_destroy(c);
    return fail(HE_EOOM, "table allocation failed");
  }
  // uploads on the context's stream: a block from the caller's allocator may
  // still be in use by earlier work on that stream
  if (hipMemcpyAsync(c->d_primes, hp.data(), sizeof(PrimeDev) * np, hipMemcpyHostToDevice, c->st) != hipSuccess ||
      hipMemcpyAsync(c->d_fwd, fwd.data(), fwd.size() * sizeof(u64), hipMemcpyHostToDevice, c->st) != hipSuccess ||
      hipMemcpyAsync(c->d_inv, inv.data(), inv.size() * sizeof(u64), hipMemcpyHostToDevice, c->st) != hipSuccess ||
      hipMemcpyAsync(c->d_fwd_fp, fwd_fp.data(), fwd_fp.size() * sizeof(double), hipMemcpyHostToDevice, c->st) !=
          hipSuccess ||
      hipMemcpyAsync(c->d_inv_fp, inv_fp.data(), inv_fp.size() * sizeof(double), hipMemcpyHostToDevice, c->st) !=
          hipSuccess ||
      hipStreamSynchronize(c->st) != hipSuccess) {
    he_ctx_destroy(c);
    return fail(HE_EHIP, "table upload failed");
  }
  // two-phase transforms for launches of up to split_jobs limbs (a few
  // ciphertexts), scratch for exactly that many
  int split_jobs = 256;
  if (const char* env = getenv("HE_NTT_SPLIT_JOBS")) split_jobs = atoi(env);
  if (const char* env = getenv("HE_FUSE_MAX")) c->fuse_max = atoi(env);
  if (const char* env = getenv("HE_HOIST_SPLIT_WGS")) c->hoist_split_wgs = atoi(env);
  if (const char* env = getenv("HE_COEF_ROT")) c->coef_rot = atoi(env);
  int forced_shape = -1;
  if (const char* env = getenv("HE_NTT_LAYOUT")) forced_shape = atoi(env);
  u64* tmp = nullptr;
  if (split_jobs > 0) {
    tmp = (u64*)c->pool.get((size_t)split_jobs * n * sizeof(u64));
    if (!tmp) {
      he_ctx_destroy(c);
      return fail(HE_EOOM, "scratch allocation failed");
    }
  }
  c->tabs = NttTables{c->d_fwd, c->d_inv, c->d_fwd_fp, c->d_inv_fp, tmp, (long long)split_jobs * n, split_jobs,
                      0, 0u, 0, {0}, 0};
  if (forced_shape > 0) {
    NttShape shapes[8];
    if (forced_shape < std::min(8, ntt_shapes(c->log_n, shapes, 8))) c->tabs.layout = forced_shape;
  }
  c->rd_inv.assign((size_t)np * np, 0);
  c->rd_inv_sh.assign((size_t)np * np, 0);
  c->rd_hq.assign((size_t)np * np, 0);
  for (int a = 0; a < np; a++)
    for (int t = 0; t < np; t++) {
      if (a == t) continue;
      const size_t i = (size_t)a * np + t;
      c->rd_inv[i] = h_inv(q[a] % q[t], q[t]);
      c->rd_inv_sh[i] = h_shoup(c->rd_inv[i], q[t]);
      c->rd_hq[i] = ((q[a] - 1) / 2) % q[t];
    }
  encode_tables_init(c->enc, c->log_n);
  c->d_chi = (double*)c->pool.get(c->enc.chi.size() * sizeof(double));
  c->d_clo = (double*)c->pool.get(c->enc.clo.size() * sizeof(double));
  c->d_rot5 = (uint32_t*)c->pool.get(c->enc.rot5.size() * sizeof(uint32_t));
  if (!c->d_chi || !c->d_clo || !c->d_rot5) {
    he_ctx_destroy(c);
    return fail(HE_EOOM, "encoder table allocation failed");
  }
  if (hipMemcpyAsync(c->d_chi, c->enc.chi.data(), c->enc.chi.size() * sizeof(double), hipMemcpyHostToDevice,
                     c->st) != hipSuccess ||
      hipMemcpyAsync(c->d_clo, c->enc.clo.data(), c->enc.clo.size() * sizeof(double), hipMemcpyHostToDevice,
                     c->st) != hipSuccess ||
      hipMemcpyAsync(c->d_rot5, c->enc.rot5.data(), c->enc.rot5.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                     c->st) != hipSuccess ||
      hipStreamSynchronize(c->st) != hipSuccess) {
    he_ctx_destroy(c);
    return fail(HE_EHIP, "encoder table upload failed");
  }
  *out = c;
  return HE_OK;
}

void he_ctx_destroy(he_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->st);
  for (auto& kv : c->masks) he_pt_free(kv.second);
  c->masks.clear();
  for (auto& r : c->prof_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  c->pool.destroy();
  if (c->ev_cross) (void)hipEventDestroy(c->ev_cross);
  if (c->own_stream) (void)hipStreamDestroy(c->st);
  delete c;
}

he_status he_ctx_info(const he_ctx* c, int32_t* log_n, int32_t* n_data, uint64_t* primes) {
  if (!c) return fail(HE_EINVAL, "NULL context");
  if (log_n) *log_n = c->log_n;
  if (n_data) *n_data = c->L;
  if (primes)
    for (size_t i = 0; i < c->q.size(); i++) primes[i] = c->q[i];
  return HE_OK;
}

he_status he_keygen(he_ctx* c, const int32_t* steps, size_t n_steps) {
  NO_CAPTURE(c);
  if (!c) return fail(HE_EINVAL, "NULL context");
  const int n = c->n, L = c->L;
  if (!c->have_keys) {
    u64* s = (u64*)c->pool.get((size_t)(L + 1) * n * sizeof(u64));
    u64* pk = s ? (u64*)c->pool.get(2 * (size_t)L * n * sizeof(u64)) : nullptr;
    if (!s || !pk) {
      c->pool.put(s);
      return fail(HE_EOOM, "key allocation failed");
    }
    c->d_s = s;
    c->d_pk = pk;
    ModList all = mods_range(L + 1), data = mods_range(L);
    {
      Prof pr(c, "sample");
      hipError_t e = launch_sample_small(c->log_n, 0, c->seed, 1, 0, all, s, c->d_primes, c->st);
      if (e != hipSuccess) return fail(HE_EHIP, "sample s: %s", hipGetErrorString(e));
    }
    TRY(ntt_rows(c, true, s, s, 1, L + 1, 0, 0));
    DBuf A, E;
    TRY(dalloc(c, A, (size_t)L * n));
    TRY(dalloc(c, E, (size_t)L * n));
    {
      Prof pr(c, "sample");
      hipError_t e = launch_sample_uniform(c->log_n, c->seed, 2, 0, 1, data, data, A.p, c->d_primes, c->st);
      if (e == hipSuccess) e = launch_sample_small(c->log_n, 1, c->seed, 3, 0, data, E.p, c->d_primes, c->st);
      if (e != hipSuccess) return fail(HE_EHIP, "sample pk: %s", hipGetErrorString(e));
    }
    TRY(ntt_rows(c, true, A.p, A.p, 1, L, 0, 0));
    TRY(ntt_rows(c, true, E.p, E.p, 1, L, 0, 0));
    hipError_t e = launch_pk_combine(c->log_n, A.p, E.p, s, pk, L, c->d_primes, c->st);
    if (e != hipSuccess) return fail(HE_EHIP, "pk: %s", hipGetErrorString(e));
    HIPC(hipMemcpyAsync(pk + (size_t)L * n, A.p, (size_t)L * n * sizeof(u64), hipMemcpyDeviceToDevice, c->st));
    // relinearisation key for s^2
    DBuf s2;
    TRY(dalloc(c, s2, (size_t)(L + 1) * n));
    e = launch_mul_plain(c->log_n, s, s, s2.p, 1, all, c->d_primes, c->st);
    if (e != hipSuccess) return fail(HE_EHIP, "s^2: %s", hipGetErrorString(e));
    TRY(make_key(c, c->relin, L - 1, s2.p, 4, 5, 0));
    c->have_keys = true;
  }
  for (size_t i = 0; i < n_steps; i++) TRY(galois_key(c, steps[i], -1));
  HIPC(hipStreamSynchronize(c->st));
  return HE_OK;
}

he_status he_keygen_galois(he_ctx* c, int32_t step, int32_t max_level) {
  NO_CAPTURE(c);
  if (!c) return fail(HE_EINVAL, "NULL context");
  return galois_key(c, step, max_level);
}

he_status he_encode(he_ctx* c, const double* v, size_t n, double scale, int32_t level, he_pt** out) {
  NO_CAPTURE(c);
  if (!c || !out || (!v && n)) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  return encode_impl(c, v, n, scale, level, out);
}

he_status he_pt_import(he_ctx* c, const int64_t* coeffs, double scale, int32_t level, he_pt** out) {
  NO_CAPTURE(c);
  if (!c || !coeffs || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  if (level < 0 || level >= c->L) return fail(HE_ELEVEL, "level %d outside 0..%d", level, c->L - 1);
  return upload_coeffs(c, coeffs, level, scale, out);
}

he_status he_pt_export(he_ctx* c, const he_pt* pt, uint64_t* h, size_t cap, int32_t* level, double* scale) {
  TRY(own(c, pt));
  NO_CAPTURE(c);
  if (!c || !pt || !h) return fail(HE_EINVAL, "NULL argument");
  const size_t words = pt_words(c, pt->level);
  if (cap < words) return fail(HE_EINVAL, "capacity %zu < %zu words", cap, words);
  std::vector<u64> v;
  TRY(download_coeff(c, pt->d, 1, pt->level + 1, v));
  std::memcpy(h, v.data(), words * sizeof(u64));
  if (level) *level = pt->level;
  if (scale) *scale = pt->scale;
  return HE_OK;
}

he_status he_decode(he_ctx* c, const he_pt* pt, double* out, size_t nv) {
  TRY(own(c, pt));
  NO_CAPTURE(c);
  if (!c || !pt || (!out && nv)) return fail(HE_EINVAL, "NULL argument");
  if (nv > (size_t)c->n / 2) return fail(HE_ERANGE, "%zu values exceed N/2", nv);
  std::vector<u64> v;
  TRY(download_coeff(c, pt->d, 1, pt->level + 1, v));
  std::vector<double> m(c->n);
  crt_centered(c, v.data(), pt->level + 1, m.data());
  decode_values(c->enc, m.data(), pt->scale, out, nv);
  return HE_OK;
}

he_status he_encrypt(he_ctx* c, const he_pt* pt, uint32_t idx, int32_t use_sk, he_ct** out) {
  TRY(own(c, pt));
  if (!c || !pt || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  if (!c->have_keys) return fail(HE_ENOKEY, "he_keygen must run first");
  const int n = c->n, Lp = pt->level + 1;
  ModList mods = mods_range(Lp);
  DBuf buf;  // [3][Lp][N]: v (or a), e0, e1
  TRY(dalloc(c, buf, 3 * (size_t)Lp * n));
  u64* v = buf.p;
  u64* e0 = buf.p + (size_t)Lp * n;
  u64* e1 = buf.p + 2 * (size_t)Lp * n;
  {
    Prof pr(c, "sample");
    hipError_t e;
    if (use_sk) {
      e = launch_sample_uniform(c->log_n, c->seed, 11, idx, 1, mods, mods, v, c->d_primes, c->st);
      if (e == hipSuccess) e = launch_sample_small(c->log_n, 1, c->seed, 12, idx, mods, e0, c->d_primes, c->st);
    } else {
      e = launch_sample_small(c->log_n, 0, c->seed, 8, idx, mods, v, c->d_primes, c->st);
      if (e == hipSuccess) e = launch_sample_small(c->log_n, 1, c->seed, 9, idx, mods, e0, c->d_primes, c->st);
      if (e == hipSuccess) e = launch_sample_small(c->log_n, 1, c->seed, 10, idx, mods, e1, c->d_primes, c->st);
    }
    if (e != hipSuccess) return fail(HE_EHIP, "encryption sampling: %s", hipGetErrorString(e));
  }
  TRY(ntt_rows(c, true, buf.p, buf.p, use_sk ? 2 : 3, Lp, (long long)Lp * n, (long long)Lp * n));
  he_ct* ct = nullptr;
  TRY(new_ct(c, pt->level, pt->scale, &ct));
  hipError_t e = launch_encrypt_combine(c->log_n, v, use_sk ? nullptr : c->d_pk,
                                        use_sk ? nullptr : c->d_pk + (size_t)c->L * n, e0, e1, c->d_s, pt->d,
                                        ct->d, Lp, c->L, c->d_primes, c->st);
  if (e != hipSuccess) {
    he_ct_free(ct);
    return fail(HE_EHIP, "encrypt: %s", hipGetErrorString(e));
  }
  *out = ct;
  return HE_OK;
}

he_status he_decrypt(he_ctx* c, const he_ct* ct, he_pt** out) {
  TRY(own(c, ct));
  if (!c || !ct || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  if (!c->have_keys) return fail(HE_ENOKEY, "no secret key");
  he_pt* pt = nullptr;
  TRY(new_pt(c, ct->level, ct->scale, &pt));
  hipError_t e = launch_decrypt(c->log_n, ct->d, c->d_s, pt->d, ct->level + 1, c->d_primes, c->st);
  if (e != hipSuccess) {
    he_pt_free(pt);
    return fail(HE_EHIP, "decrypt: %s", hipGetErrorString(e));
  }
  *out = pt;
  return HE_OK;
}

he_status he_ct_export(he_ctx* c, const he_ct* ct, uint64_t* h, size_t cap, int32_t* level, double* scale) {
  TRY(own(c, ct));
  NO_CAPTURE(c);
  if (!c || !ct || !h) return fail(HE_EINVAL, "NULL argument");
  const size_t words = ct_words(c, ct->level);
  if (cap < words) return fail(HE_EINVAL, "capacity %zu < %zu words", cap, words);
  std::vector<u64> v;
  TRY(download_coeff(c, ct->d, 2, ct->level + 1, v));
  std::memcpy(h, v.data(), words * sizeof(u64));
  if (level) *level = ct->level;
  if (scale) *scale = ct->scale;
  return HE_OK;
}

he_status he_ct_import(he_ctx* c, const uint64_t* h, int32_t level, double scale, he_ct** out) {
  NO_CAPTURE(c);
  if (!c || !h || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  if (level < 0 || level >= c->L) return fail(HE_ELEVEL, "level %d outside 0..%d", level, c->L - 1);
  const int Lp = level + 1;
  for (int k = 0; k < 2; k++)
    for (int i = 0; i < Lp; i++)
      for (int t = 0; t < c->n; t++)
        if (h[((size_t)k * Lp + i) * c->n + t] >= c->q[i]) return fail(HE_ERANGE, "residue not below its prime");
  he_ct* ct = nullptr;
  TRY(new_ct(c, level, scale, &ct));
  hipError_t e = hipMemcpyAsync(ct->d, h, ct_words(c, level) * sizeof(u64), hipMemcpyHostToDevice, c->st);
  if (e == hipSuccess) e = hipStreamSynchronize(c->st);
  if (e != hipSuccess) {
    he_ct_free(ct);
    return fail(HE_EHIP, "ciphertext upload: %s", hipGetErrorString(e));
  }
  he_status s = ntt_rows(c, true, ct->d, ct->d, 2, Lp, (long long)Lp * c->n, (long long)Lp * c->n);
  if (s != HE_OK) {
    he_ct_free(ct);
    return s;
  }
  *out = ct;
  return HE_OK;
}

he_status he_ct_info(const he_ct* ct, int32_t* level, double* scale) {
  if (!ct) return fail(HE_EINVAL, "NULL ciphertext");
  if (level) *level = ct->level;
  if (scale) *scale = ct->scale;
  return HE_OK;
}

static he_status addsub(he_ctx* c, const he_ct* a, const he_ct* b, int op, he_ct** out) {
  TRY(own(c, a));
  TRY(own(c, b));
  if (!c || !a || !b || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  if (!scales_match(a->scale, b->scale)) return fail(HE_ESCALE, "scales %g and %g differ", a->scale, b->scale);
  const he_ct *x, *y;
  CtGuard gx, gy;
  TRY(align2(c, a, b, &x, &y, gx, gy));
  he_ct* r = nullptr;
  TRY(new_ct(c, x->level, a->scale, &r));
  Prof pr(c, "pointwise", 0, 24.0 * 2 * (x->level + 1) * c->n);
  hipError_t e = launch_addsub(c->log_n, op, x->d, y->d, r->d, 2, mods_range(x->level + 1), c->d_primes, c->st);
  if (e != hipSuccess) {
    he_ct_free(r);
    return fail(HE_EHIP, "add/sub: %s", hipGetErrorString(e));
  }
  *out = r;
  return HE_OK;
}

he_status he_add(he_ctx* c, const he_ct* a, const he_ct* b, he_ct** out) { return addsub(c, a, b, 0, out); }
he_status he_sub(he_ctx* c, const he_ct* a, const he_ct* b, he_ct** out) { return addsub(c, a, b, 1, out); }

he_status he_negate(he_ctx* c, const he_ct* a, he_ct** out) {
  TRY(own(c, a));
  if (!c || !a || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  he_ct* r = nullptr;
  TRY(new_ct(c, a->level, a->scale, &r));
  hipError_t e = launch_addsub(c->log_n, 2, a->d, a->d, r->d, 2, mods_range(a->level + 1), c->d_primes, c->st);
  if (e != hipSuccess) {
    he_ct_free(r);
    return fail(HE_EHIP, "negate: %s", hipGetErrorString(e));
  }
  *out = r;
  return HE_OK;
}

static he_status add_plain_impl(he_ctx* c, const he_ct* a, const he_pt* p, int neg, he_ct** out) {
  TRY(own(c, a));
  TRY(own(c, p));
  if (!c || !a || !p || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  if (!scales_match(a->scale, p->scale)) return fail(HE_ESCALE, "scales %g and %g differ", a->scale, p->scale);
  if (p->level < a->level) return fail(HE_ELEVEL, "plaintext level %d below ciphertext level %d", p->level, a->level);
  he_ct* r = nullptr;
  TRY(new_ct(c, a->level, a->scale, &r));
  Prof pr(c, "pointwise");
  hipError_t e =
      launch_add_plain(c->log_n, a->d, p->d, r->d, 2, mods_range(a->level + 1), c->d_primes, c->st, neg);
  if (e != hipSuccess) {
    he_ct_free(r);
    return fail(HE_EHIP, "add_plain: %s", hipGetErrorString(e));
  }
  *out = r;
  return HE_OK;
}

he_status he_add_plain(he_ctx* c, const he_ct* a, const he_pt* p, he_ct** out) {
  return add_plain_impl(c, a, p, 0, out);
}
he_status he_sub_plain(he_ctx* c, const he_ct* a, const he_pt* p, he_ct** out) {
  return add_plain_impl(c, a, p, 1, out);
}

static he_status mul_plain_raw(he_ctx* c, const he_ct* a, const he_pt* p, he_ct** out) {
  if (p->level < a->level) return fail(HE_ELEVEL, "plaintext level %d below ciphertext level %d", p->level, a->level);
  he_ct* r = nullptr;
  TRY(new_ct(c, a->level, a->scale * p->scale, &r));
  Prof pr(c, "pointwise");
  hipError_t e = launch_mul_plain(c->log_n, a->d, p->d, r->d, 2, mods_range(a->level + 1), c->d_primes, c->st);
  if (e != hipSuccess) {
    he_ct_free(r);
    return fail(HE_EHIP, "mul_plain: %s", hipGetErrorString(e));
  }
  *out = r;
  return HE_OK;
}

static he_status rescale_raw(he_ctx* c, const he_ct* a, he_ct** out) {
  const int l = a->level;
  if (l < 1) return fail(HE_ELEVEL, "no level left to rescale");
  he_ct* r = nullptr;
  TRY(new_ct(c, l - 1, a->scale / (double)c->q[l], &r));
  he_status s = rescale_multi(c, a->d, 1, l, r->d);
  if (s != HE_OK) {
    he_ct_free(r);
    return s;
  }
  *out = r;
  return HE_OK;
}

he_status he_rescale(he_ctx* c, const he_ct* a, he_ct** out) {
  TRY(own(c, a));
  if (!c || !a || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  return rescale_raw(c, a, out);
}

static he_status maybe_rescale(he_ctx* c, he_ct* r, he_ct** out) {
  if (!c->auto_rescale) {
    *out = r;
    return HE_OK;
  }
  he_status s = rescale_raw(c, r, out);
  he_ct_free(r);
  return s;
}

he_status he_mul_plain(he_ctx* c, const he_ct* a, const he_pt* p, he_ct** out) {
  TRY(own(c, a));
  TRY(own(c, p));
  if (!c || !a || !p || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  he_ct* r = nullptr;
  TRY(mul_plain_raw(c, a, p, &r));
  return maybe_rescale(c, r, out);
}

// the product, relinearised; with resc where the fused key switch applies,
// also rescaled (*rescaled says whether it was)
static he_status mul_relin_raw(he_ctx* c, const he_ct* a, const he_ct* b, he_ct** out, bool resc = false,
                               bool* rescaled = nullptr) {
  if (!c->have_keys) return fail(HE_ENOKEY, "no relinearisation key");
  const he_ct *x, *y;
  CtGuard gx, gy;
  TRY(align2(c, a, b, &x, &y, gx, gy));
  const int l = x->level, Lp = l + 1, n = c->n;
  const bool fuse = resc && l >= 1 && ks_fusable(c, 1, Lp);
  if (rescaled) *rescaled = fuse;
  he_ct* r = nullptr;
  TRY(new_ct(c, l, a->scale * b->scale, &r));
  DBuf d2;
  he_status s = dalloc(c, d2, (size_t)Lp * n);
  if (s == HE_OK) {
    Prof pr(c, "pointwise");
    hipError_t e = launch_tensor(c->log_n, x->d, y->d, r->d, d2.p, mods_range(Lp), c->d_primes, c->st);
    if (e != hipSuccess) s = fail(HE_EHIP, "tensor: %s", hipGetErrorString(e));
  }
  he_ct* f = nullptr;
  if (s == HE_OK && fuse) s = new_ct(c, l - 1, a->scale * b->scale / (double)c->q[l], &f);
  if (s == HE_OK) {
    const Key* kp = &c->relin;
    Addend add;
    add.p = r->d;
    add.aa = (long long)Lp * n;
    s = key_switch(c, 1, d2.p, 0, l, &kp, nullptr, add, fuse ? f->d : r->d, fuse);
  }
  if (s != HE_OK) {
    he_ct_free(f);
    he_ct_free(r);
    return s;
  }
  if (fuse) {
    he_ct_free(r);
    *out = f;
  } else {
    *out = r;
  }
  return HE_OK;
}

he_status he_mul_relin(he_ctx* c, const he_ct* a, const he_ct* b, he_ct** out) {
  TRY(own(c, a));
  TRY(own(c, b));
  if (!c || !a || !b || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  he_ct* r = nullptr;
  bool rescaled = false;
  TRY(mul_relin_raw(c, a, b, &r, c->auto_rescale, &rescaled));
  if (rescaled) {
    *out = r;
    return HE_OK;
  }
  return maybe_rescale(c, r, out);
}

he_status he_square(he_ctx* c, const he_ct* a, he_ct** out) { return he_mul_relin(c, a, a, out); }

// Scratch words he_mul_relin needs at operand levels la, lb: every
// intermediate of the path (level alignment copy, tensor, key switch in
// either form, rescale) allocated once, none reused.
static size_t noalloc_mul_relin_words(const he_ctx* c, int la, int lb) {
  const size_t n = c->n, Lp = (size_t)std::min(la, lb) + 1, nm = Lp + 1;
  size_t w = 0;
  if (la != lb) w += 2 * Lp;                                   // aligned copy
  w += 2 * Lp + Lp;                                            // d0, d1 and d2
  const size_t fused = Lp + Lp * Lp + Lp * nm + 2 + 4 * Lp;    // t1 t2 ext t3 t4 t5
  const size_t plain = Lp + Lp * nm + 2 * nm + 2;              // coef ext u ucoef
  w += std::max(fused, plain);
  if (c->auto_rescale) w += 2 * (Lp - 1) + std::max<size_t>(2 + 2 * (Lp - 1), 2);
  return w * n;
}

he_status he_mul_relin_noalloc(he_ctx* c, const he_ct* a, const he_ct* b, he_ct* out) {
  TRY(own(c, a));
  TRY(own(c, b));
  TRY(own(c, out));
  if (!c || !a || !b || !out) return fail(HE_EINVAL, "NULL argument");
  if (c->arena) return fail(HE_EINVAL, "a no-allocation call is already running on this context");
  if (!c->scratch) return fail(HE_EHIP, "no-allocation scratch unavailable on device %d", c->device);
  if (!c->have_keys) return fail(HE_ENOKEY, "no relinearisation key");
  const int l = std::min(a->level, b->level);
  if (c->auto_rescale && l < 1) return fail(HE_ELEVEL, "no level left to rescale");
  const int lo = c->auto_rescale ? l - 1 : l;
  if (out->level != lo) return fail(HE_ELEVEL, "output ciphertext at level %d, the result is at level %d", out->level, lo);
  const size_t need = noalloc_mul_relin_words(c, a->level, b->level);
  if (need > c->scratch_words)
    return fail(HE_ERANGE, "the product at level %d needs %zu bytes of scratch, more than the %u-byte maximum", l,
                need * sizeof(u64), HE_NOALLOC_SCRATCH_BYTES);
  he_ctx::Arena arena{c->scratch, c->scratch_words, 0};
  c->arena = &arena;
  he_ct* r = nullptr;
  he_ct* f = nullptr;
  he_status s = mul_relin_raw(c, a, b, &r);
  if (s == HE_OK) s = maybe_rescale(c, r, &f);  // frees r when it rescales
  if (s == HE_OK) {
    hipError_t e = launch_copy(f->d, out->d, (long long)ct_words(c, lo), c->st);
    if (e != hipSuccess) s = fail(HE_EHIP, "copy: %s", hipGetErrorString(e));
    else out->scale = f->scale;
  }
  he_ct_free(f);  // host handle only: arena memory is not pooled
  c->arena = nullptr;
  return s;
}

he_status he_drop_to(he_ctx* c, const he_ct* a, int32_t level, he_ct** out) {
  TRY(own(c, a));
  if (!c || !a || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  if (level < 0 || level > a->level) return fail(HE_ELEVEL, "cannot drop from level %d to %d", a->level, level);
  return drop_copy(c, a, level, out);
}

static he_status rotate_raw(he_ctx* c, const he_ct* a, int step, he_ct** out) {
  const int l = a->level;
  step = norm_step(c, step);
  if (step == 0) return drop_copy(c, a, l, out);
  he_ct* r = nullptr;
  TRY(new_ct(c, l, a->scale, &r));
  he_status s = rotate_multi(c, a->d, 1, l, &step, r->d);
  if (s != HE_OK) {
    he_ct_free(r);
    return s;
  }
  *out = r;
  return HE_OK;
}

he_status he_rotate(he_ctx* c, const he_ct* a, int32_t step, he_ct** out) {
  TRY(own(c, a));
  if (!c || !a || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  return rotate_raw(c, a, step, out);
}

// ---------------------------------------------------------------- power, polyval
// a*b (levels aligned by dropping), relinearised and rescaled
static he_status mul_rescale(he_ctx* c, const he_ct* a, const he_ct* b, he_ct** out) {
  he_ct* r = nullptr;
  TRY(mul_relin_raw(c, a, b, &r));
  he_status s = rescale_raw(c, r, out);
  he_ct_free(r);
  return s;
}

// cache of the squares a^(2^i); entry 0 is the input (not owned)
struct Squares {
  std::vector<he_ct*> v;
  ~Squares() {
    for (size_t i = 1; i < v.size(); i++) he_ct_free(v[i]);
  }
};

// a^k at multiplicative depth ceil(log2 k): the squares of the set bits of
// k, then the two factors of least (depth, exponent) multiplied until one is
// left.  *owned tells whether *out is a new ciphertext or a cached square.
static he_status power_impl(he_ctx* c, const he_ct* a, long long k, Squares& sq, he_ct** out, bool* owned) {
  *out = nullptr;
  if (k < 1) return fail(HE_EINVAL, "power: exponent %lld < 1", k);
  if (sq.v.empty()) sq.v.push_back(const_cast<he_ct*>(a));
  int top = 0;
  while ((k >> (top + 1)) > 0) top++;
  while ((int)sq.v.size() <= top) {
    he_ct* r = nullptr;
    TRY(mul_rescale(c, sq.v.back(), sq.v.back(), &r));
    sq.v.push_back(r);
  }
  struct Fac {
    int depth;
    long long e;
    he_ct* ct;
    bool own;
  };
  std::vector<Fac> fac;
  for (int i = 0; i <= top; i++)
    if ((k >> i) & 1) fac.push_back(Fac{i, 1LL << i, sq.v[i], false});
  he_status s = HE_OK;
  while (fac.size() > 1 && s == HE_OK) {
    std::stable_sort(fac.begin(), fac.end(), [](const Fac& x, const Fac& y) {
      return x.depth != y.depth ? x.depth < y.depth : x.e < y.e;
    });
    const Fac fa = fac[0], fb = fac[1];
    he_ct* r = nullptr;
    s = mul_rescale(c, fa.ct, fb.ct, &r);
    if (fa.own) he_ct_free(fa.ct);
    if (fb.own) he_ct_free(fb.ct);
    fac.erase(fac.begin(), fac.begin() + 2);
    if (s == HE_OK) fac.push_back(Fac{std::max(fa.depth, fb.depth) + 1, fa.e + fb.e, r, true});
  }
  if (s != HE_OK) {
    for (auto& f : fac)
      if (f.own) he_ct_free(f.ct);
    return s;
  }
  *out = fac[0].ct;
  *owned = fac[0].own;
  return HE_OK;
}

he_status he_power(he_ctx* c, const he_ct* a, uint32_t k, he_ct** out) {
  TRY(own(c, a));
  if (!c || !a || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  Squares sq;
  he_ct* r = nullptr;
  bool owned = false;
  TRY(power_impl(c, a, k, sq, &r, &owned));
  if (owned) {
    *out = r;
    return HE_OK;
  }
  return drop_copy(c, r, r->level, out);  // k a power of two: a cached square
}

// sum_i coeffs[i] a^i: each a^i (i >= 1, coeffs[i] != 0) from the power
// circuit times the constant coeffs[i] encoded at scale Delta * q_l /
// scale(a^i) at a^i's level l and rescaled (every term at scale Delta), cut
// to the lowest level and summed in increasing i; coeffs[0] added last.
he_status he_polyval(he_ctx* c, const he_ct* a, const double* coeffs, size_t n_coeffs, he_ct** out) {
  TRY(own(c, a));
  if (!c || !a || !out || (n_coeffs && !coeffs)) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  std::vector<size_t> idx;
  for (size_t i = 1; i < n_coeffs; i++)
    if (coeffs[i] != 0.0) idx.push_back(i);
  if (idx.empty()) return fail(HE_EINVAL, "polyval: no non-constant term");
  const size_t half = (size_t)c->n / 2;
  Squares sq;
  std::vector<he_ct*> terms;
  auto free_terms = [&]() {
    for (he_ct* t : terms) he_ct_free(t);
    terms.clear();
  };
  for (size_t i : idx) {
    he_ct* x = nullptr;
    bool owned = false;
    he_status s = power_impl(c, a, (long long)i, sq, &x, &owned);
    he_pt* p = nullptr;
    if (s == HE_OK) {
      const double ps = c->scale * (double)c->q[x->level] / x->scale;
      std::vector<double> v(half, coeffs[i]);
      s = encode_impl(c, v.data(), half, ps, x->level, &p);
    }
    he_ct* m = nullptr;
    if (s == HE_OK) s = mul_plain_raw(c, x, p, &m);
    he_pt_free(p);
    if (owned) he_ct_free(x);
    he_ct* t = nullptr;
    if (s == HE_OK) s = rescale_raw(c, m, &t);
    he_ct_free(m);
    if (s != HE_OK) {
      free_terms();
      return s;
    }
    terms.push_back(t);
  }
  int low = terms[0]->level;
  for (he_ct* t : terms) low = std::min(low, t->level);
  he_ct* acc = nullptr;
  he_status s = HE_OK;
  for (size_t j = 0; j < terms.size() && s == HE_OK; j++) {
    he_ct* t = terms[j];
    he_ct* td = nullptr;
    if (t->level != low) {
      s = drop_copy(c, t, low, &td);
      if (s != HE_OK) break;
      t = td;
    }
    if (!acc) {
      s = drop_copy(c, t, low, &acc);
    } else {
      he_ct* r = nullptr;
      s = he_add(c, acc, t, &r);
      he_ct_free(acc);
      acc = r;
    }
    he_ct_free(td);
  }
  free_terms();
  if (s == HE_OK && coeffs[0] != 0.0) {
    std::vector<double> v(half, coeffs[0]);
    he_pt* p = nullptr;
    s = encode_impl(c, v.data(), half, acc->scale, acc->level, &p);
    he_ct* r = nullptr;
    if (s == HE_OK) s = he_add_plain(c, acc, p, &r);
    he_pt_free(p);
    he_ct_free(acc);
    acc = r;
  }
  if (s != HE_OK) {
    he_ct_free(acc);
    return s;
  }
  *out = acc;
  return HE_OK;
}

// ---------------------------------------------------------------- batches
// B ciphertexts that share one pooled block [B][2][level+1][N]; the block
// returns to the pool with the last of them
static void split_block(he_ctx* c, u64* blk, int B, int level, const double* scales, he_ct** out) {
  std::shared_ptr<void> owner(blk, [c](void* p) { c->pool.put(p); });
  const size_t per = ct_words(c, level);
  for (int b = 0; b < B; b++) out[b] = new he_ct{c, level, scales[b], blk + b * per, owner};
}

static he_status batch_level(const he_ct* const* a, const he_ct* const* b, size_t n, int* level) {
  *level = -1;
  for (size_t i = 0; i < n; i++) {
    if (!a[i] || (b && !b[i])) return fail(HE_EINVAL, "NULL ciphertext at %zu", i);
    const int la = a[i]->level;
    if (*level < 0) *level = la;
    if (la != *level || (b && b[i]->level != *level))
      return fail(HE_ELEVEL, "batched operands must share one level (%d vs %d at %zu)", *level,
                  b && b[i]->level != *level ? b[i]->level : la, i);
  }
  return HE_OK;
}

// n products at one level run on c (its stream, pool and tables); item i
// relinearises with the key of a[i]'s context (c itself unless the batch
// spans contexts); the results are c's, in shared blocks
static he_status mul_relin_many_impl(he_ctx* c, const he_ct* const* a, const he_ct* const* b, size_t n,
                                     he_ct** out) {
  for (size_t i = 0; i < n; i++) out[i] = nullptr;
  if (n == 0) return HE_OK;
  for (size_t i = 0; i < n; i++)
    if (!a[i] || !a[i]->ctx->have_keys) return fail(HE_ENOKEY, "no relinearisation key");
  int l = 0;
  TRY(batch_level(a, b, n, &l));
  if (c->auto_rescale && l < 1) return fail(HE_ELEVEL, "no level left to rescale");
  const int Lp = l + 1, nn = c->n;
  for (size_t i0 = 0; i0 < n; i0 += HE_MAX_BATCH) {
    const int B = (int)std::min<size_t>(HE_MAX_BATCH, n - i0);
    CtList A{}, Bl{};
    const Key* keys[HE_MAX_BATCH];
    for (int k = 0; k < B; k++) {
      A.p[k] = a[i0 + k]->d;
      Bl.p[k] = b[i0 + k]->d;
      keys[k] = &a[i0 + k]->ctx->relin;
    }
    // with automatic rescaling, the fused key switch rescales in its last
    // kernels where it applies
    const bool fuse = c->auto_rescale && ks_fusable(c, B, Lp);
    u64* R = (u64*)c->pool.get((size_t)B * ct_words(c, l) * sizeof(u64));
    if (!R) return fail(HE_EOOM, "batch allocation failed");
    u64* F = fuse ? (u64*)c->pool.get((size_t)B * ct_words(c, l - 1) * sizeof(u64)) : nullptr;
    if (fuse && !F) {
      c->pool.put(R);
      return fail(HE_EOOM, "batch allocation failed");
    }
    DBuf d2;
    he_status s = dalloc(c, d2, (size_t)B * Lp * nn);
    if (s == HE_OK) {
      Prof pr(c, "pointwise");
      hipError_t e = launch_tensor_many(c->log_n, A, Bl, B, R, d2.p, Lp, c->d_primes, c->st);
      if (e != hipSuccess) s = fail(HE_EHIP, "tensor: %s", hipGetErrorString(e));
    }
    if (s == HE_OK) {
      Addend add;
      add.p = R;
      add.aa = (long long)Lp * nn;
      s = key_switch(c, B, d2.p, (long long)Lp * nn, l, keys, nullptr, add, fuse ? F : R, fuse);
    }
    u64* O = R;
    int lo = l;
    if (fuse) {
      c->pool.put(R);
      O = F;
      lo = l - 1;
      if (s != HE_OK) c->pool.put(F);
    } else if (s == HE_OK && c->auto_rescale) {
      O = (u64*)c->pool.get((size_t)B * ct_words(c, l - 1) * sizeof(u64));
      s = O ? rescale_multi(c, R, B, l, O) : fail(HE_EOOM, "batch allocation failed");
      c->pool.put(R);
      lo = l - 1;
      if (s != HE_OK && O) c->pool.put(O);
    } else if (s != HE_OK) {
      c->pool.put(R);
    }
    if (s != HE_OK) {
      for (size_t i = 0; i < i0; i++) {
        he_ct_free(out[i]);
        out[i] = nullptr;
      }
      return s;
    }
    double sc[HE_MAX_BATCH];
    for (int k = 0; k < B; k++) {
      sc[k] = a[i0 + k]->scale * b[i0 + k]->scale;
      if (lo < l) sc[k] /= (double)c->q[l];
    }
    split_block(c, O, B, lo, sc, out + i0);
  }
  return HE_OK;
}

he_status he_mul_relin_many(he_ctx* c, const he_ct* const* a, const he_ct* const* b, size_t n, he_ct** out) {
  TRY(own_all(c, a, n));
  TRY(own_all(c, b, n));
  if (!c || !out || (n && (!a || !b))) return fail(HE_EINVAL, "NULL argument");
  return mul_relin_many_impl(c, a, b, n, out);
}

static he_status rotate_many_impl(he_ctx* c, const he_ct* const* a, const int32_t* steps, size_t n,
                                  he_ct** out);
he_status he_rotate_many(he_ctx* c, const he_ct* const* a, const int32_t* steps, size_t n, he_ct** out) {
  TRY(own_all(c, a, n));
  if (!c || !out || (n && (!a || !steps))) return fail(HE_EINVAL, "NULL argument");
  return rotate_many_impl(c, a, steps, n, out);
}

// n rotations at one level run on c; item i uses the Galois key of a[i]'s
// context; the results are c's, in shared blocks
static he_status rotate_many_impl(he_ctx* c, const he_ct* const* a, const int32_t* steps, size_t n,
                                  he_ct** out) {
  for (size_t i = 0; i < n; i++) out[i] = nullptr;
  if (n == 0) return HE_OK;
  int l = 0;
  TRY(batch_level(a, nullptr, n, &l));
  const size_t per = ct_words(c, l);
  for (size_t i0 = 0; i0 < n; i0 += HE_MAX_BATCH) {
    const int B = (int)std::min<size_t>(HE_MAX_BATCH, n - i0);
    CtList A{};
    int st[HE_MAX_BATCH];
    he_ctx* kc[HE_MAX_BATCH];
    for (int k = 0; k < B; k++) {
      A.p[k] = a[i0 + k]->d;
      st[k] = norm_step(c, steps[i0 + k]);
      kc[k] = a[i0 + k]->ctx;
    }
    DBuf in;
    he_status s = dalloc(c, in, (size_t)B * per);
    u64* O = s == HE_OK ? (u64*)c->pool.get((size_t)B * per * sizeof(u64)) : nullptr;
    if (s == HE_OK && !O) s = fail(HE_EOOM, "batch allocation failed");
    if (s == HE_OK) {
      Prof pr(c, "pointwise");
      hipError_t e = launch_gather_cts(c->log_n, A, B, l + 1, in.p, c->st);
      if (e != hipSuccess) s = fail(HE_EHIP, "gather: %s", hipGetErrorString(e));
    }
    // step 0 items are copies; the rest rotate together
    if (s == HE_OK) {
      int idx[HE_MAX_BATCH], nr = 0;
      for (int k = 0; k < B; k++) {
        if (st[k] == 0) {
          if (launch_copy(in.p + k * per, O + k * per, (long long)per, c->st) != hipSuccess)
            s = fail(HE_EHIP, "copy failed");
        } else {
          idx[nr++] = k;
        }
      }
      if (s == HE_OK && nr == B) {
        s = rotate_multi(c, in.p, B, l, st, O, false, kc);
      } else if (s == HE_OK && nr > 0) {
        // pack the rotating items, rotate, scatter back
        DBuf pin, pout;
        s = dalloc(c, pin, (size_t)nr * per);
        if (s == HE_OK) s = dalloc(c, pout, (size_t)nr * per);
        int pst[HE_MAX_BATCH];
        he_ctx* pkc[HE_MAX_BATCH];
        for (int r = 0; r < nr && s == HE_OK; r++) {
          pst[r] = st[idx[r]];
          pkc[r] = kc[idx[r]];
          if (launch_copy(in.p + idx[r] * per, pin.p + r * per, (long long)per, c->st) != hipSuccess)
            s = fail(HE_EHIP, "copy failed");
        }
        if (s == HE_OK) s = rotate_multi(c, pin.p, nr, l, pst, pout.p, false, pkc);
        for (int r = 0; r < nr && s == HE_OK; r++)
          if (launch_copy(pout.p + r * per, O + idx[r] * per, (long long)per, c->st) != hipSuccess)
            s = fail(HE_EHIP, "copy failed");
      }
    }
    if (s != HE_OK) {
      if (O) c->pool.put(O);
      for (size_t i = 0; i < i0; i++) {
        he_ct_free(out[i]);
        out[i] = nullptr;
      }
      return s;
    }
    double sc[HE_MAX_BATCH];
    for (int k = 0; k < B; k++) sc[k] = a[i0 + k]->scale;
    split_block(c, O, B, l, sc, out + i0);
  }
  return HE_OK;
}

// ---------------------------------------------------------------- batches across contexts
// Contexts whose ciphertexts can share one batched key switch: same ring,
// primes, rescaling rule and device (each item keeps its own keys).
static bool same_params(const he_ctx* a, const he_ctx* b) {
  return a->n == b->n && a->q == b->q && a->auto_rescale == b->auto_rescale && a->device == b->device;
}

// The batch runs on run's stream after the work already queued on every
// other involved context's stream (their inputs, and the previous users of
// the blocks their results take), and each of those streams then waits for
// the batch before its later work (which may read the results or reuse the
// inputs' blocks).
static he_status across_contexts(he_ctx* run, const he_ct* const* a, const he_ct* const* b, size_t n,
                                 he_ct** out, const std::function<he_status()>& batch) {
  if (!run || !out || (n && !a)) return fail(HE_EINVAL, "NULL argument");
  for (size_t i = 0; i < n; i++) out[i] = nullptr;
  if (run->capturing) return fail(HE_EINVAL, "a batch across contexts cannot be captured");
  std::vector<he_ctx*> others;
  for (size_t i = 0; i < n; i++) {
    if (!a[i] || (b && !b[i])) return fail(HE_EINVAL, "NULL ciphertext at %zu", i);
    he_ctx* x = a[i]->ctx;
    if (b && b[i]->ctx != x) return fail(HE_EINVAL, "operands %zu belong to different contexts", i);
    if (!same_params(run, x)) return fail(HE_EINVAL, "item %zu: its context has other parameters", i);
    if (x->capturing) return fail(HE_EINVAL, "item %zu: its context is capturing a graph", i);
    if (x != run && std::find(others.begin(), others.end(), x) == others.end()) others.push_back(x);
  }
  for (he_ctx* o : others) {
    HIPC(hipEventRecord(o->ev_cross, o->st));
    HIPC(hipStreamWaitEvent(run->st, o->ev_cross, 0));
  }
  he_status s = batch();
  // results of other contexts' items move into their own context's memory
  for (size_t i = 0; i < n && s == HE_OK; i++) {
    he_ctx* x = a[i]->ctx;
    if (x == run) continue;
    he_ct* r = nullptr;
    s = new_ct(x, out[i]->level, out[i]->scale, &r);
    if (s == HE_OK && launch_copy(out[i]->d, r->d, (long long)ct_words(run, r->level), run->st) != hipSuccess) {
      he_ct_free(r);
      r = nullptr;
      s = fail(HE_EHIP, "result copy failed");
    }
    if (s == HE_OK) {
      he_ct_free(out[i]);
      out[i] = r;
    }
  }
  const hipError_t e = hipEventRecord(run->ev_cross, run->st);
  for (he_ctx* o : others)
    if (e == hipSuccess) (void)hipStreamWaitEvent(o->st, run->ev_cross, 0);
  if (s == HE_OK && e != hipSuccess) s = fail(HE_EHIP, "event record: %s", hipGetErrorString(e));
  if (s != HE_OK)
    for (size_t i = 0; i < n; i++) {
      he_ct_free(out[i]);
      out[i] = nullptr;
    }
  return s;
}

// ---------------------------------------------------------------- work queue
// Key switches (multiply + relinearise (+ rescale), rotate) of any mix of
// contexts, ring degrees and levels as eight launches in all, each draining
// one stage's task list with a resident grid: tensor; inverse transform of
// the digits; ModUp (lift + forward transform); inner products; inverse
// transform of the special limbs; ModDown; and for rescaled products the
// inverse transform of the top limb and the division.  A task is one limb
// of one operation; each stage's tasks are ordered largest ring first.
namespace {
struct QueueBuild {
  std::vector<NttJob> ntt;
  std::vector<InnerJob> inner;
  std::vector<QTensor> tensor;
  std::vector<QTables> tabs;
  std::vector<const he_ctx*> tab_ctx;
  std::vector<QTask> stage[8];
  size_t lds[8] = {0};
  int tab_of(const he_ctx* c) {
    for (size_t i = 0; i < tab_ctx.size(); i++)
      if (tab_ctx[i] == c) return (int)i;
    tab_ctx.push_back(c);
    tabs.push_back(QTables{c->d_primes, c->tabs.fwd, c->tabs.inv, c->tabs.fwd_fp, c->tabs.inv_fp});
    return (int)tabs.size() - 1;
  }
  void add(int st, int kind, int log_n, int job, int n_w, int tab) {
    for (int w = 0; w < n_w; w++) stage[st].push_back(QTask{log_n, job, w, tab});
    lds[st] = std::max(lds[st], queue_lds_bytes(kind, log_n));
  }
};
const int kQueueKind[8] = {QK_TENSOR, QK_INV, QK_FWD_LIFT, QK_INNER, QK_INV, QK_FWD_RD, QK_INV, QK_FWD_RD};
}  // namespace

he_status he_queue_run(he_ctx* run, const he_qop* ops, size_t n, he_ct** out) {
  if (!run || !out || (n && !ops)) return fail(HE_EINVAL, "NULL argument");
  for (size_t i = 0; i < n; i++) out[i] = nullptr;
  if (n == 0) return HE_OK;
  NO_CAPTURE(run);
  // validation and the operations' own contexts
  std::vector<he_ctx*> others;
  std::vector<const Key*> keys(n);
  std::vector<int> levels(n), steps(n, 0);
  size_t scratch_words = 0;
  for (size_t i = 0; i < n; i++) {
    const he_qop& o = ops[i];
    he_ctx* c = o.ctx;
    if (!c || !o.a) return fail(HE_EINVAL, "operation %zu: NULL context or operand", i);
    if (o.a->ctx != c || (o.b && o.b->ctx != c)) return fail(HE_EINVAL, "operation %zu: handle of another context", i);
    if (c->device != run->device) return fail(HE_EINVAL, "operation %zu: context on another device", i);
    if (c->log_n < 12 || c->log_n > 14) return fail(HE_EINVAL, "operation %zu: ring degree 2^%d outside 2^12..2^14", i, c->log_n);
    if (c->capturing) return fail(HE_EINVAL, "operation %zu: its context is capturing a graph", i);
    const int l = o.a->level, Lp = l + 1, nm = Lp + 1;
    const size_t N = (size_t)c->n;
    levels[i] = l;
    if (o.kind == HE_QOP_MUL_RELIN) {
      if (!o.b) return fail(HE_EINVAL, "operation %zu: NULL second factor", i);
      if (o.b->level != l) return fail(HE_ELEVEL, "operation %zu: factors at levels %d and %d", i, l, o.b->level);
      if (!c->have_keys) return fail(HE_ENOKEY, "operation %zu: no relinearisation key", i);
      if (c->relin.ml < l) return fail(HE_ENOKEY, "operation %zu: relinearisation key below level %d", i, l);
      if (c->auto_rescale && l < 1) return fail(HE_ELEVEL, "operation %zu: no level left to rescale", i);
      keys[i] = &c->relin;
      scratch_words += N * (3 * Lp + Lp + Lp * nm + 2 * nm + 2 + (c->auto_rescale ? 2 * Lp + 2 : 0));
    } else if (o.kind == HE_QOP_ROTATE) {
      const int st = norm_step(c, o.step);
      if (st == 0) return fail(HE_EINVAL, "operation %zu: rotation by 0 slots", i);
      auto it = c->gal.find(st);
      if (it == c->gal.end()) return fail(HE_ENOKEY, "operation %zu: no Galois key for step %d", i, st);
      if (it->second.ml < l) return fail(HE_ENOKEY, "operation %zu: Galois key for step %d below level %d", i, st, l);
      keys[i] = &it->second;
      steps[i] = st;
      scratch_words += N * (Lp + Lp * nm + 2 * nm + 2);
    } else {
      return fail(HE_EINVAL, "operation %zu: unknown kind %d", i, o.kind);
    }
    if (c != run && std::find(others.begin(), others.end(), c) == others.end()) others.push_back(c);
  }
  // results, in each operation's own context
  for (size_t i = 0; i < n; i++) {
    const he_qop& o = ops[i];
    const int l = levels[i];
    const bool resc = o.kind == HE_QOP_MUL_RELIN && o.ctx->auto_rescale;
    double sc = o.kind == HE_QOP_MUL_RELIN ? o.a->scale * o.b->scale : o.a->scale;
    if (resc) sc /= (double)o.ctx->q[l];
    he_status s = new_ct(o.ctx, resc ? l - 1 : l, sc, &out[i]);
    if (s != HE_OK) {
      for (size_t k = 0; k < i; k++) {
        he_ct_free(out[k]);
        out[k] = nullptr;
      }
      return s;
    }
  }
  auto release = [&](he_status s) {
    for (size_t i = 0; i < n; i++) {
      he_ct_free(out[i]);
      out[i] = nullptr;
    }
    return s;
  };
  DBuf scratch;
  if (dalloc(run, scratch, scratch_words) != HE_OK) return release(fail(HE_EOOM, "queue intermediates"));
  // jobs and tasks
  QueueBuild Q;
  u64* mem = scratch.p;
  auto take = [&](size_t words) {
    u64* p = mem;
    mem += words;
    return p;
  };
  // operations sharing a key (same context, key and level) form groups of up
  // to HE_MAX_BATCH whose inner products run as one task per modulus, so
  // the key words are read once for the group
  std::vector<size_t> order(n);
  for (size_t i = 0; i < n; i++) order[i] = i;
  auto gkey = [&](size_t i) { return std::make_tuple((const void*)ops[i].ctx, (const void*)keys[i]->d, levels[i]); };
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return gkey(x) < gkey(y); });
  for (size_t g0 = 0; g0 < n;) {
    size_t g1 = g0 + 1;
    while (g1 < n && g1 - g0 < HE_MAX_BATCH && gkey(order[g1]) == gkey(order[g0])) g1++;
    const int B = (int)(g1 - g0);
    he_ctx* c = ops[order[g0]].ctx;
    const int l = levels[order[g0]], Lp = l + 1, nm = Lp + 1, N = c->n, L = c->L, ln = c->log_n;
    const int tab = Q.tab_of(c);
    u64* ext_g = take((size_t)B * Lp * nm * N);
    u64* u_g = take((size_t)B * 2 * nm * N);
    InnerJob I{};
    I.ext = ext_g;
    I.u = u_g;
    I.B = B;
    I.n_dig = Lp;
    I.special_prime = L;
    for (int b = 0; b < B; b++) {
      const size_t i = order[g0 + b];
      const he_qop& o = ops[i];
      const bool mul = o.kind == HE_QOP_MUL_RELIN, resc = mul && c->auto_rescale;
      const u64* d;
      u64 g = 1;
      Addend add;
      if (mul) {
        u64* d01 = take((size_t)2 * Lp * N);
        u64* d2 = take((size_t)Lp * N);
        Q.tensor.push_back(QTensor{o.a->d, o.b->d, d01, d2, Lp});
        Q.add(0, QK_TENSOR, ln, (int)Q.tensor.size() - 1, Lp, tab);
        d = d2;
        add.p = d01;
        add.aa = (long long)Lp * N;
      } else {
        g = galois_elt(c, steps[i]);
        d = o.a->d + (size_t)Lp * N;  // tau_g(c1) is read by gather
        add.p = o.a->d;                // tau_g(c0) joins poly 0
        add.aa = (long long)Lp * N;
        add.even_only = 1;
      }
      u64 gals[1] = {g};
      if (!mul) add.gals = gals;
      u64* coef = take((size_t)Lp * N);
      u64* ext = ext_g + (size_t)b * Lp * nm * N;
      u64* u = u_g + (size_t)b * 2 * nm * N;
      u64* ucoef = take((size_t)2 * N);
      {  // digits to coefficients (tau_g applied by the gather)
        NttJob J{};
        J.src = d;
        J.dst = coef;
        J.na = 1;
        J.nb = Lp;
        J.sb = N;
        J.da = (long long)Lp * N;
        J.db = N;
        for (int t = 0; t < Lp; t++) J.dst_prime[t] = (unsigned char)t;
        if (!mul) {
          J.gather_src = 1;
          J.gal_div = 1;
          J.gal[0] = g;
        }
        Q.ntt.push_back(J);
        Q.add(1, QK_INV, ln, (int)Q.ntt.size() - 1, Lp, tab);
      }
      {  // ModUp: centred digit j lifted to every other modulus
        NttJob J{};
        J.src = coef;
        J.sa = N;
        J.dst = ext;
        J.da = (long long)nm * N;
        J.db = N;
        J.na = Lp;
        J.nb = nm;
        J.skip_diag = 1;
        J.src_prime = -1;
        J.amod = Lp;
        for (int t = 0; t < nm; t++) J.dst_prime[t] = (unsigned char)(t < Lp ? t : L);
        Q.ntt.push_back(J);
        Q.add(2, QK_FWD_LIFT, ln, (int)Q.ntt.size() - 1, Lp * (nm - 1), tab);
      }
      I.key[b] = keys[i]->d;  // the group's key
      I.km[b] = keys[i]->ml + 2;
      I.gal[b] = g;
      I.diag_p[b] = d;
      {  // the special limbs to coefficients
        NttJob J{};
        J.src = u + (size_t)Lp * N;
        J.sa = (long long)nm * N;
        J.dst = ucoef;
        J.da = N;
        J.na = 2;
        J.nb = 1;
        J.dst_prime[0] = (unsigned char)L;
        Q.ntt.push_back(J);
        Q.add(4, QK_INV, ln, (int)Q.ntt.size() - 1, 2, tab);
      }
      u64* ks_out = resc ? take((size_t)2 * Lp * N) : out[i]->d;
      Q.ntt.push_back(round_div_job(c, 2, ucoef, L, u, (long long)nm * N, ks_out, (long long)Lp * N, Lp, add));
      Q.add(5, QK_FWD_RD, ln, (int)Q.ntt.size() - 1, 2 * Lp, tab);
      if (resc) {  // rescale: the top limb to coefficients, then the division
        u64* rcoef = take((size_t)2 * N);
        NttJob J{};
        J.src = ks_out + (size_t)l * N;
        J.sa = (long long)Lp * N;
        J.dst = rcoef;
        J.da = N;
        J.na = 2;
        J.nb = 1;
        J.dst_prime[0] = (unsigned char)l;
        Q.ntt.push_back(J);
        Q.add(6, QK_INV, ln, (int)Q.ntt.size() - 1, 2, tab);
        Q.ntt.push_back(round_div_job(c, 2, rcoef, l, ks_out, (long long)Lp * N, out[i]->d, (long long)l * N, l,
                                      Addend{}));
        Q.add(7, QK_FWD_RD, ln, (int)Q.ntt.size() - 1, 2 * l, tab);
      }
    }
    Q.inner.push_back(I);
    Q.add(3, QK_INNER, ln, (int)Q.inner.size() - 1, nm * (N / 1024), tab);
    g0 = g1;
  }
  if ((size_t)(mem - scratch.p) != scratch_words) return release(fail(HE_EINVAL, "queue layout mismatch"));
  // one device image: stage counters, tables, tasks, job records
  for (auto& st : Q.stage)
    std::stable_sort(st.begin(), st.end(), [](const QTask& x, const QTask& y) { return x.log_n > y.log_n; });
  auto align = [](size_t b) { return (b + 255) & ~(size_t)255; };
  size_t off = align(8 * sizeof(unsigned));
  const size_t o_tabs = off;
  off = align(off + Q.tabs.size() * sizeof(QTables));
  size_t o_task[8];
  for (int k = 0; k < 8; k++) {
    o_task[k] = off;
    off = align(off + Q.stage[k].size() * sizeof(QTask));
  }
  const size_t o_ntt = off;
  off = align(off + Q.ntt.size() * sizeof(NttJob));
  const size_t o_inner = off;
  off = align(off + Q.inner.size() * sizeof(InnerJob));
  const size_t o_tensor = off;
  off = align(off + Q.tensor.size() * sizeof(QTensor));
  std::vector<unsigned char> img(off, 0);
  std::memcpy(img.data() + o_tabs, Q.tabs.data(), Q.tabs.size() * sizeof(QTables));
  for (int k = 0; k < 8; k++)
    if (!Q.stage[k].empty()) std::memcpy(img.data() + o_task[k], Q.stage[k].data(), Q.stage[k].size() * sizeof(QTask));
  std::memcpy(img.data() + o_ntt, Q.ntt.data(), Q.ntt.size() * sizeof(NttJob));
  std::memcpy(img.data() + o_inner, Q.inner.data(), Q.inner.size() * sizeof(InnerJob));
  if (!Q.tensor.empty()) std::memcpy(img.data() + o_tensor, Q.tensor.data(), Q.tensor.size() * sizeof(QTensor));
  DBuf dimg;
  if (dalloc(run, dimg, (off + 7) / 8) != HE_OK) return release(fail(HE_EOOM, "queue descriptors"));
  unsigned char* base = reinterpret_cast<unsigned char*>(dimg.p);
  // order: run's stream after the other contexts' queued work
  for (he_ctx* o : others) {
    if (hipEventRecord(o->ev_cross, o->st) != hipSuccess || hipStreamWaitEvent(run->st, o->ev_cross, 0) != hipSuccess)
      return release(fail(HE_EHIP, "stream ordering failed"));
  }
  he_status s = HE_OK;
  hipError_t e = hipMemcpyAsync(base, img.data(), off, hipMemcpyHostToDevice, run->st);
  if (e == hipSuccess) e = launch_fill_u32(reinterpret_cast<unsigned*>(base), 8, 0u, run->st);
  {
    size_t units = 0;
    for (auto& st : Q.stage) units += st.size();
    Prof pr(run, "queue", (double)units, 0.0);
    for (int k = 0; k < 8 && e == hipSuccess; k++) {
      const int cnt = (int)Q.stage[k].size();
      if (cnt == 0) continue;
      const int kind = kQueueKind[k];
      const void* jobs = kind == QK_INNER    ? (const void*)(base + o_inner)
                         : kind == QK_TENSOR ? (const void*)(base + o_tensor)
                                             : (const void*)(base + o_ntt);
      const int grid = std::min(cnt, queue_grid(run->device, Q.lds[k]));
      e = launch_queue(kind, reinterpret_cast<const QTask*>(base + o_task[k]), cnt, jobs,
                       reinterpret_cast<const QTables*>(base + o_tabs), reinterpret_cast<unsigned*>(base) + k, grid,
                       Q.lds[k], run->st);
    }
  }
  if (e != hipSuccess) s = fail(HE_EHIP, "queue launch: %s", hipGetErrorString(e));
  // the host image must outlive the copy; later work of the other contexts
  // waits for the queue
  const hipError_t e2 = hipStreamSynchronize(run->st);
  if (s == HE_OK && e2 != hipSuccess) s = fail(HE_EHIP, "queue: %s", hipGetErrorString(e2));
  if (s != HE_OK) return release(s);
  return HE_OK;
}

he_status he_mul_relin_across(he_ctx* run, const he_ct* const* a, const he_ct* const* b, size_t n, he_ct** out) {
  if (n && !b) return fail(HE_EINVAL, "NULL argument");
  return across_contexts(run, a, b, n, out, [&]() { return mul_relin_many_impl(run, a, b, n, out); });
}

he_status he_rotate_across(he_ctx* run, const he_ct* const* a, const int32_t* steps, size_t n, he_ct** out) {
  if (n && !steps) return fail(HE_EINVAL, "NULL argument");
  return across_contexts(run, a, nullptr, n, out, [&]() { return rotate_many_impl(run, a, steps, n, out); });
}

// x <- x + rot(x, stride 2^j), j < ceil(log2 count); each step is one fused
// rotate-and-add
static he_status rotate_and_sum(he_ctx* c, he_ct* x, uint32_t count, uint32_t stride, he_ct** out) {
  int steps = 0;
  while ((1u << steps) < count) steps++;
  // three or more steps in coefficient form (where the fused key switch
  // applies and no step is a rotation by a multiple of N/2): one inverse
  // and one forward transform around the chain
  const int l = x->level, n = c->n;
  bool coef = steps >= 3 && coef_rotations(c, 1, l + 1);
  for (int j = 0; j < steps && coef; j++) coef = norm_step(c, (long long)stride << j) != 0;
  if (coef) {
    he_ct* y = nullptr;
    he_status s = new_ct(c, l, x->scale, &y);
    DBuf A, B;
    const size_t w = 2 * (size_t)(l + 1) * n;
    if (s == HE_OK) s = dalloc(c, A, w);
    if (s == HE_OK) s = dalloc(c, B, w);
    if (s == HE_OK) s = ntt_rows(c, false, x->d, A.p, 2, l + 1, (long long)(l + 1) * n, (long long)(l + 1) * n);
    for (int j = 0; j < steps && s == HE_OK; j++) {
      const int st = norm_step(c, (long long)stride << j);
      s = rotate_multi_coef(c, A.p, 1, l, &st, B.p, true);
      std::swap(A.p, B.p);
    }
    if (s == HE_OK) s = ntt_rows(c, true, A.p, y->d, 2, l + 1, (long long)(l + 1) * n, (long long)(l + 1) * n);
    he_ct_free(x);
    if (s != HE_OK) {
      he_ct_free(y);
      return s;
    }
    *out = y;
    return HE_OK;
  }
  for (int j = 0; j < steps; j++) {
    he_ct* y = nullptr;
    const int st = norm_step(c, (long long)stride << j);
    he_status s = HE_OK;
    if (st == 0) {
      s = he_add(c, x, x, &y);
    } else {
      s = new_ct(c, x->level, x->scale, &y);
      if (s == HE_OK) s = rotate_multi(c, x->d, 1, x->level, &st, y->d, true);
    }
    he_ct_free(x);
    if (s != HE_OK) {
      he_ct_free(y);
      return s;
    }
    x = y;
  }
  *out = x;
  return HE_OK;
}

he_status he_sum_slots(he_ctx* c, const he_ct* a, uint32_t nv, he_ct** out) {
  TRY(own(c, a));
  if (!c || !a || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  if (nv == 0 || nv > (uint32_t)c->n / 2) return fail(HE_ERANGE, "slot count %u outside 1..N/2", nv);
  he_ct* x = nullptr;
  TRY(drop_copy(c, a, a->level, &x));
  return rotate_and_sum(c, x, nv, 1, out);
}

// ---------------------------------------------------------------- composites
static he_status encode_slots(he_ctx* c, const std::vector<double>& v, double scale, int level, he_pt** out) {
  return encode_impl(c, v.data(), v.size(), scale, level, out);
}

he_status he_conv_plan(he_ctx* c, const he_ct* like, const double* kernel, uint32_t kk, uint32_t windows,
                       double bias, he_plan** out) {
  TRY(own(c, like));
  NO_CAPTURE(c);
  if (!c || !like || !kernel || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  const uint32_t half = (uint32_t)c->n / 2;
  if (kk == 0 || windows == 0 || (uint64_t)kk * windows > half) return fail(HE_ERANGE, "kk * windows > N/2");
  if (like->level < 1) return fail(HE_ELEVEL, "convolution needs one level");
  he_plan* p = new he_plan();
  p->ctx = c;
  p->kind = PLAN_CONV;
  p->level = like->level;
  p->scale = like->scale;
  p->kk = kk;
  p->windows = windows;
  std::vector<double> v((size_t)kk * windows);
  for (uint32_t k = 0; k < kk; k++)
    for (uint32_t w = 0; w < windows; w++) v[(size_t)k * windows + w] = kernel[k];
  he_status s = encode_slots(c, v, c->scale, like->level, &p->kernel);
  if (s == HE_OK) {
    const double post = like->scale * p->kernel->scale / (double)c->q[like->level];
    std::vector<double> b(windows, bias);
    s = encode_slots(c, b, post, like->level - 1, &p->bias);
  }
  if (s != HE_OK) {
    he_plan_free(p);
    return s;
  }
  *out = p;
  return HE_OK;
}

he_status he_matmul_plan(he_ctx* c, const he_ct* like, const double* W, uint32_t n_in, uint32_t n_out,
                         const double* bias, he_plan** out) {
  TRY(own(c, like));
  NO_CAPTURE(c);
  if (!c || !like || !W || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  const uint32_t half = (uint32_t)c->n / 2;
  if (n_in == 0 || n_out == 0 || n_in > half || n_out > half) return fail(HE_ERANGE, "matrix shape");
  uint32_t reps = 1;
  while ((uint64_t)n_in * reps * 2 <= half) reps *= 2;
  if ((uint64_t)n_in + n_out - 1 > (uint64_t)n_in * reps) return fail(HE_ERANGE, "n_in + n_out - 1 > copies");
  if (like->level < 1) return fail(HE_ELEVEL, "matmul needs one level");
  const int n = c->n, Lp = like->level + 1;
  he_plan* p = new he_plan();
  p->ctx = c;
  p->kind = PLAN_MATMUL;
  p->level = like->level;
  p->scale = like->scale;
  p->n_in = n_in;
  p->n_out = n_out;
  // diagonals: diag_i[j] = W[(i + j) mod n_in][j], encoded at Delta, all in
  // one device buffer [n_in][Lp][N] (coefficients uploaded, one batched NTT)
  const size_t words = (size_t)n_in * Lp * n;
  std::vector<u64> h(words);
  std::vector<double> d(n_out);
  std::vector<int64_t> co(n);
  for (uint32_t i = 0; i < n_in; i++) {
    for (uint32_t j = 0; j < n_out; j++) d[j] = W[(size_t)((i + j) % n_in) * n_out + j];
    if (encode_coeffs(c->enc, d.data(), n_out, c->scale, co.data()) != 0) {
      he_plan_free(p);
      return fail(HE_ERANGE, "diagonal %u does not encode", i);
    }
    for (int t = 0; t < Lp; t++) {
      const u64 q = c->q[t];
      u64* row = h.data() + ((size_t)i * Lp + t) * n;
      for (int k = 0; k < n; k++) {
        const int64_t v = co[k];
        u64 r = v >= 0 ? (u64)v % q : ((u64)(-(v + 1)) + 1u) % q;
        row[k] = (v < 0 && r) ? q - r : r;
      }
    }
  }
  // device buffer: [n_in][Lp][N] diagonals (NTT domain)
  p->diags = (u64*)c->pool.get(words * sizeof(u64));
  he_status s = p->diags ? HE_OK : fail(HE_EOOM, "diagonal allocation failed");
  if (s == HE_OK) {
    hipError_t e = hipMemcpyAsync(p->diags, h.data(), words * sizeof(u64), hipMemcpyHostToDevice, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    if (e != hipSuccess) s = fail(HE_EHIP, "diagonal upload: %s", hipGetErrorString(e));
  }
  if (s == HE_OK) s = ntt_rows(c, true, p->diags, p->diags, (int)n_in, Lp, (long long)Lp * n, (long long)Lp * n);
  if (s == HE_OK) {
    const double post = like->scale * c->scale / (double)c->q[like->level];
    std::vector<double> b(n_out, 0.0);
    if (bias)
      for (uint32_t j = 0; j < n_out; j++) b[j] = bias[j];
    s = encode_slots(c, b, post, like->level - 1, &p->bias);
  }
  if (s != HE_OK) {
    he_plan_free(p);
    return s;
  }
  *out = p;
  return HE_OK;
}

// n convolution plans on the same input in lock step: the n channel
// ciphertexts live side by side ([n][2][l+1][N]) so every rotation step is one
// batched key switch.  Same operations, same results as n single applies.
static he_status conv_apply_many(he_ctx* c, const he_plan* const* plans, int nb, const he_ct* x, he_ct** outs) {
  const int n = c->n, l = x->level, Lp = l + 1;
  const size_t ct_w = 2 * (size_t)Lp * n, ct_w1 = 2 * (size_t)l * n;
  DBuf M, Y, R;
  TRY(dalloc(c, M, nb * ct_w));
  TRY(dalloc(c, Y, nb * ct_w1));
  TRY(dalloc(c, R, nb * ct_w1));
  {
    CtList in{}, kp{};
    for (int b = 0; b < nb; b++) {
      in.p[b] = x->d;
      kp.p[b] = plans[b]->kernel->d;
    }
    Prof pr(c, "pointwise");
    hipError_t e = launch_mul_plain_many(c->log_n, in, kp, nb, Lp, M.p, c->d_primes, c->st);
    if (e != hipSuccess) return fail(HE_EHIP, "mul_plain: %s", hipGetErrorString(e));
  }
  const double scale = x->scale * plans[0]->kernel->scale / (double)c->q[l];
  int steps = 0;
  while ((1u << steps) < plans[0]->kk) steps++;
  std::vector<int> st(nb);
  // the chain in coefficient form where the fused key switch applies: the
  // rescale leaves its result in coefficient form, one forward transform
  // follows the chain
  const bool coef = steps > 0 && coef_rotations(c, nb, l);
  if (coef)
    TRY(rescale_to_coef(c, M.p, nb, l, Y.p));
  else
    TRY(rescale_multi(c, M.p, nb, l, Y.p));
  for (int j = 0; j < steps; j++) {
    for (int b = 0; b < nb; b++) st[b] = norm_step(c, (long long)plans[0]->windows << j);
    if (st[0] == 0) {  // rotation by a multiple of N/2: x + x (in either form)
      Prof pr(c, "pointwise");
      hipError_t e = launch_addsub(c->log_n, 0, Y.p, Y.p, Y.p, 2 * nb, mods_range(l), c->d_primes, c->st);
      if (e != hipSuccess) return fail(HE_EHIP, "add: %s", hipGetErrorString(e));
      continue;
    }
    if (coef)
      TRY(rotate_multi_coef(c, Y.p, nb, l - 1, st.data(), R.p, true));
    else
      TRY(rotate_multi(c, Y.p, nb, l - 1, st.data(), R.p, true));
    std::swap(Y.p, R.p);
  }
  if (coef) TRY(ntt_rows(c, true, Y.p, Y.p, 2 * nb, l, (long long)l * n, (long long)l * n));
  CtList in{}, bp{};
  OutList ol{};
  for (int b = 0; b < nb; b++) {
    if (!scales_match(scale, plans[b]->bias->scale)) {
      for (int k = 0; k < b; k++) {
        he_ct_free(outs[k]);
        outs[k] = nullptr;
      }
      return fail(HE_ESCALE, "bias scale");
    }
    he_status s = new_ct(c, l - 1, scale, &outs[b]);
    if (s != HE_OK) {
      for (int k = 0; k < b; k++) {
        he_ct_free(outs[k]);
        outs[k] = nullptr;
      }
      return s;
    }
    in.p[b] = Y.p + b * ct_w1;
    bp.p[b] = plans[b]->bias->d;
    ol.p[b] = outs[b]->d;
  }
  Prof pr(c, "pointwise");
  hipError_t e = launch_add_plain_many(c->log_n, in, bp, ol, nb, l, c->d_primes, c->st);
  if (e != hipSuccess) {
    for (int b = 0; b < nb; b++) {
      he_ct_free(outs[b]);
      outs[b] = nullptr;
    }
    return fail(HE_EHIP, "add_plain: %s", hipGetErrorString(e));
  }
  return HE_OK;
}

static he_status conv_apply(he_ctx* c, const he_plan* p, const he_ct* x, he_ct** out) {
  return conv_apply_many(c, &p, 1, x, out);
}

// device table of hoisted rotations by steps[r] (diagonal index diags[r],
// -1 for none), keys checked at `level`; rebuilt when keys change
static he_status build_items(he_ctx* c, const std::vector<int>& steps, const std::vector<int>& diags, int level,
                             HoistItem** dev, uint64_t* epoch) {
  const int R = (int)steps.size();
  if (R <= 0) return HE_OK;
  if (*dev && *epoch == c->key_epoch) return HE_OK;
  if (c->capturing) return fail(HE_EINVAL, "apply the plan once before capturing it");
  std::vector<HoistItem> h(R);
  for (int r = 0; r < R; r++) {
    const int step = norm_step(c, steps[r]);
    auto it = c->gal.find(step);
    if (it == c->gal.end()) return fail(HE_ENOKEY, "no Galois key for step %d", step);
    if (it->second.ml < level) return fail(HE_ENOKEY, "Galois key for step %d cut below level %d", step, level);
    h[r].key = it->second.d;
    h[r].g = galois_elt(c, step);
    h[r].km = it->second.ml + 2;
    h[r].diag = diags[r];
  }
  if (!*dev) {
    *dev = (HoistItem*)c->pool.get(sizeof(HoistItem) * R);
    if (!*dev) return fail(HE_EOOM, "item table allocation failed");
  }
  HIPC(hipMemcpyAsync(*dev, h.data(), sizeof(HoistItem) * R, hipMemcpyHostToDevice, c->st));
  HIPC(hipStreamSynchronize(c->st));
  *epoch = c->key_epoch;
  return HE_OK;
}

// the rotations 1..n_in-1 of the vector-matrix product, item r multiplied
// by diagonal r
static he_status hoist_items(he_ctx* c, he_plan* p, int level) {
  const int R = (int)p->n_in - 1;
  std::vector<int> steps(std::max(R, 0)), diags(std::max(R, 0));
  for (int r = 0; r < R; r++) {
    steps[r] = r + 1;
    diags[r] = r + 1;
  }
  return build_items(c, steps, diags, level, &p->items, &p->items_epoch);
}

// replication copies: R the largest power of two with n_in * R <= N/2, the
// right rotations by n_in * m, m = 1..R-1 (no diagonal)
static int replication_count(const he_ctx* c, uint32_t n_in) {
  const uint32_t half = (uint32_t)c->n / 2;
  int reps = 1;
  while ((uint64_t)n_in * reps * 2 <= half) reps *= 2;
  return reps;
}
static he_status rep_items(he_ctx* c, he_plan* p, int level) {
  const int R = replication_count(c, p->n_in) - 1;
  std::vector<int> steps(std::max(R, 0)), diags(std::max(R, 0), -1);
  for (int m = 1; m <= R; m++) steps[m - 1] = (int)((long long)c->n / 2 - (long long)p->n_in * m);
  return build_items(c, steps, diags, level, &p->rep_items, &p->rep_epoch);
}

// acc = sum_i rot_left(x, i) * diag_i, the n_in - 1 rotations hoisted: one
// ModUp of x's poly 1, one batched inner product, one batched ModDown NTT
// fused with the multiply-accumulate (partial sums per chunk of rotations)
// R hoisted rotations of x by the items' steps; with diagonals (rows of
// diags) each rotation is multiplied by its diagonal and the i = 0 term is
// x * diags[0]; without, the rotations and x are summed.  out_scale: the
// result's scale.
static he_status hoisted_core(he_ctx* c, const HoistItem* items, int R, const u64* diags, const he_ct* x,
                              double out_scale, he_ct** out) {
  const int l = x->level, Lp = l + 1, nm = Lp + 1, n = c->n;
  he_ct* acc = nullptr;
  TRY(new_ct(c, l, out_scale, &acc));
  CtGuard gacc{acc};
  int n_chunks = 0;
  DBuf partial;
  if (R > 0) {
    DBuf coef, ext, u, ucoef;
    KsJob K;
    KsBufs bufs;
    const bool split = c->hoist_split_wgs > 0;
    // the two-phase form computes the inner products where it uses them
    if (!split) TRY(dalloc(c, u, (size_t)R * 2 * nm * n));
    TRY(dalloc(c, ucoef, (size_t)R * 2 * n));
    const u64* c1 = x->d + (size_t)Lp * n;
    const u64* extp = nullptr;
    if (ks_fusable(c, 1, Lp)) {  // one ModUp shared by every rotation
      TRY(ks_prepare(c, 1, c1, 0, l, nullptr, nullptr, K, bufs, false));
      TRY(modup_fused(c, K, false));
      extp = bufs.ext.p;
    } else {
      TRY(dalloc(c, coef, (size_t)Lp * n));
      TRY(dalloc(c, ext, (size_t)Lp * nm * n));
      TRY(ntt_rows(c, false, c1, coef.p, 1, Lp, 0, 0));
      TRY(modup(c, coef.p, 1, Lp, ext.p));
      extp = ext.p;
    }
    HoistInner I{};
    I.ext = extp;
    I.c1 = c1;
    I.c0 = x->d;
    for (int t = 0; t < Lp; t++) {
      I.pq[t] = c->q[c->L] % c->q[t];
      I.pq_sh[t] = h_shoup(I.pq[t], c->q[t]);
    }
    I.n_dig = Lp;
    I.nm = nm;
    I.t_begin = 0;
    I.t_end = nm;
    I.special_prime = c->L;
    // chunks of rotations so that the multiply-accumulate's workgroups fill
    // the chip: chunks x 2 x Lp of the one-kernel form (one per compute
    // unit), chunks x 2 x Lp x blocks of the two-phase form (several per
    // compute unit)
    const int per_chunk = 2 * Lp * (split ? hoist_split_blocks(c->log_n) : 1);
    const int target = split ? c->hoist_split_wgs : 512;
    n_chunks = std::max(1, std::min(R, (target + per_chunk - 1) / per_chunk));
    // at least two rotations per chunk in the two-phase form: a chunk of one
    // leaves the block phase a single item to overlap and the finish one
    // partial sum per rotation
    const int chunk = std::max(split ? 2 : 1, (R + n_chunks - 1) / n_chunks);
    n_chunks = (R + chunk - 1) / chunk;
    TRY(dalloc(c, partial, (size_t)n_chunks * 2 * Lp * n));
    DBuf mid;
    if (split) TRY(dalloc(c, mid, (size_t)R * 2 * Lp * n));
    HoistMac M{};
    M.ucoef = ucoef.p;
    M.u = u.p;
    M.diags = diags;
    M.items = items;
    M.partial = partial.p;
    M.mid = mid.p;
    M.R = R;
    M.n_dig = Lp;
    M.nm = nm;
    M.chunk = chunk;
    M.n_units = n_chunks * Lp;
    M.special_prime = c->L;
    M.ext = extp;
    M.c1 = c1;
    M.c0 = x->d;
    for (int t = 0; t < Lp; t++) {
      M.pq[t] = I.pq[t];
      M.pq_sh[t] = I.pq_sh[t];
    }
    M.h_src = (c->q[c->L] - 1) / 2;
    const size_t np = c->q.size();
    for (int t = 0; t < Lp; t++) {
      M.hq[t] = c->rd_hq[c->L * np + t];
      M.inv[t] = c->rd_inv[c->L * np + t];
      M.inv_sh[t] = c->rd_inv_sh[c->L * np + t];
    }
    if (!split) {
      I.items = items;
      I.u = u.p;
      I.R = R;
      // algorithmic bytes: the keys of the R items and the shared digits
      // once (the u written for the ModDown is an intermediate of this
      // design, not of the key switch)
      Prof pr(c, "hoisted_inner", (double)R, 8.0 * n * (2.0 * R * Lp * nm + Lp * nm));
      hipError_t e = launch_inner_hoisted(c->log_n, I, c->d_primes, c->st);
      if (e != hipSuccess) return fail(HE_EHIP, "hoisted inner: %s", hipGetErrorString(e));
    }
    if (!split) {
      // the special-prime limbs to coefficient form (the two-phase form's
      // column phase runs this transform itself)
      NttJob J{};
      J.src = u.p + (size_t)Lp * n;
      J.sa = (long long)nm * n;
      J.dst = ucoef.p;
      J.da = n;
      J.na = 2 * R;
      J.nb = 1;
      J.dst_prime[0] = (unsigned char)c->L;
      Prof pr(c, "ntt_inv", 2.0 * R, 16.0 * n * 2 * R);
      hipError_t e = launch_ntt_inv(c->log_n, J, c->d_primes, c->tabs, c->st);
      if (e != hipSuccess) return fail(HE_EHIP, "hoisted intt: %s", hipGetErrorString(e));
    }
    // work units: limb-NTT equivalents of butterflies (the two-phase form's
    // column phase runs the first log N - K stages, its block phase the
    // last K = ceil(log N / 2))
    const double nt = 2.0 * R * Lp;
    const int kb = (c->log_n + 1) / 2;
    if (split) {
      // the inner product and inverse transform of every (item, poly)
      // special limb, the column stages of every (item, poly, limb).
      // Algorithmic bytes: the keys' special-prime rows (R x 2 x Lp limbs)
      // and the shared digits' special limbs (the column-phase output is an
      // intermediate of this design)
      Prof pa(c, "hoisted_cols", 2.0 * R + nt * (c->log_n - kb) / c->log_n, 8.0 * n * (2.0 * R * Lp + Lp));
      hipError_t e = launch_hoisted_cols(c->log_n, M, c->d_primes, c->tabs, c->st);
      if (e != hipSuccess) return fail(HE_EHIP, "hoisted columns: %s", hipGetErrorString(e));
    }
    // algorithmic bytes per (item, poly, limb): the two-phase form reads the
    // key's Lp words of the inner product and the diagonal (the column-phase
    // output and the partial sums are intermediates of this design, and the
    // shared digits are read once: Lp x Lp limbs); the one-kernel form reads
    // the u limb, the special limb's coefficients and the diagonal, and
    // writes the partial sums
    Prof pr(c, diags ? "hoisted_moddown" : "hoisted_replication", split ? nt * kb / c->log_n : nt,
            split ? 8.0 * n * (Lp * nt + (diags ? nt : 0.0) + (double)Lp * Lp)
                  : 8.0 * n * (2.0 * nt + (diags ? nt : 0.0) + 2.0 * n_chunks * Lp));
    hipError_t e = launch_hoisted_moddown_mac(c->log_n, M, c->d_primes, c->tabs, c->st);
    if (e != hipSuccess) return fail(HE_EHIP, "hoisted moddown: %s", hipGetErrorString(e));
  }
  {
    Prof pr(c, "pointwise");
    hipError_t e = launch_mac_finish(c->log_n, partial.p, n_chunks, x->d, diags, acc->d, Lp, c->d_primes, c->st);
    if (e != hipSuccess) return fail(HE_EHIP, "mac finish: %s", hipGetErrorString(e));
  }
  *out = acc;
  gacc.p = nullptr;
  return HE_OK;
}

static he_status hoisted_mac(he_ctx* c, he_plan* p, const he_ct* x, he_ct** out) {
  TRY(hoist_items(c, p, x->level));
  return hoisted_core(c, p->items, (int)p->n_in - 1, p->diags, x, x->scale * c->scale, out);
}

// x replicated: x plus its hoisted right rotations by n_in * m
static he_status hoisted_rep(he_ctx* c, he_plan* p, const he_ct* x, he_ct** out) {
  TRY(rep_items(c, p, x->level));
  return hoisted_core(c, p->rep_items, replication_count(c, p->n_in) - 1, nullptr, x, x->scale, out);
}

static he_status matmul_apply(he_ctx* c, he_plan* p, const he_ct* x, he_ct** out) {
  CtGuard gxr;
  if (replication_count(c, p->n_in) > 1)
    TRY(hoisted_rep(c, p, x, &gxr.p));
  else
    TRY(drop_copy(c, x, x->level, &gxr.p));
  CtGuard acc;
  TRY(hoisted_mac(c, p, gxr.p, &acc.p));
  // rescale with the bias added to poly 0 in the same kernel
  const int la = acc.p->level;
  if (la < 1) return fail(HE_ELEVEL, "no level left to rescale");
  const double sc = acc.p->scale / (double)c->q[la];
  if (!scales_match(sc, p->bias->scale)) return fail(HE_ESCALE, "scales %g and %g differ", sc, p->bias->scale);
  if (p->bias->level < la - 1) return fail(HE_ELEVEL, "bias level %d below %d", p->bias->level, la - 1);
  he_ct* y = nullptr;
  TRY(new_ct(c, la - 1, sc, &y));
  he_status s = rescale_multi(c, acc.p->d, 1, la, y->d, p->bias->d);
  if (s != HE_OK) {
    he_ct_free(y);
    return s;
  }
  *out = y;
  return HE_OK;
}

he_status he_plan_apply(he_ctx* c, const he_plan* p, const he_ct* x, he_ct** out) {
  TRY(own(c, p));
  TRY(own(c, x));
  if (!c || !p || !x || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  if (x->level != p->level) return fail(HE_ELEVEL, "plan made for level %d, input at %d", p->level, x->level);
  if (!scales_match(x->scale, p->scale)) return fail(HE_ESCALE, "plan made for scale %g, input at %g", p->scale, x->scale);
  if (p->kind == PLAN_CONV) return conv_apply(c, p, x, out);
  return matmul_apply(c, const_cast<he_plan*>(p), x, out);
}

he_status he_plan_apply_many(he_ctx* c, const he_plan* const* plans, uint32_t nb, const he_ct* x,
                             he_ct** outs) {
  TRY(own_all(c, plans, nb));
  TRY(own(c, x));
  if (!c || !plans || !x || !outs) return fail(HE_EINVAL, "NULL argument");
  for (uint32_t b = 0; b < nb; b++) outs[b] = nullptr;
  if (nb == 0) return HE_OK;
  bool lockstep = nb <= HE_MAX_BATCH;
  for (uint32_t b = 0; b < nb; b++) {
    if (!plans[b]) return fail(HE_EINVAL, "NULL plan");
    if (x->level != plans[b]->level) return fail(HE_ELEVEL, "plan made for level %d, input at %d", plans[b]->level, x->level);
    if (!scales_match(x->scale, plans[b]->scale)) return fail(HE_ESCALE, "plan scale differs from the input's");
    lockstep = lockstep && plans[b]->kind == PLAN_CONV && plans[b]->kk == plans[0]->kk &&
               plans[b]->windows == plans[0]->windows && plans[b]->kernel->scale == plans[0]->kernel->scale;
  }
  he_status s = HE_OK;
  if (lockstep) {
    s = conv_apply_many(c, plans, (int)nb, x, outs);
  } else {
    for (uint32_t b = 0; b < nb && s == HE_OK; b++) s = he_plan_apply(c, plans[b], x, &outs[b]);
  }
  if (s != HE_OK)
    for (uint32_t b = 0; b < nb; b++) {
      he_ct_free(outs[b]);
      outs[b] = nullptr;
    }
  return s;
}

he_status he_enc_conv_im2col(he_ctx* c, const he_ct* x, const double* kernel, uint32_t kk, uint32_t windows,
                             double bias, he_ct** out) {
  NO_CAPTURE(c);
  he_plan* p = nullptr;
  TRY(he_conv_plan(c, x, kernel, kk, windows, bias, &p));
  he_status s = he_plan_apply(c, p, x, out);
  he_plan_free(p);
  return s;
}

he_status he_enc_matmul(he_ctx* c, const he_ct* x, const double* W, uint32_t n_in, uint32_t n_out,
                        const double* bias, he_ct** out) {
  NO_CAPTURE(c);
  he_plan* p = nullptr;
  TRY(he_matmul_plan(c, x, W, n_in, n_out, bias, &p));
  he_status s = he_plan_apply(c, p, x, out);
  he_plan_free(p);
  return s;
}

he_status he_pack(he_ctx* c, he_ct* const* parts, uint32_t n_parts, uint32_t width, he_ct** out) {
  TRY(own_all(c, (const he_ct* const*)parts, n_parts));
  if (!c || !parts || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  const uint32_t half = (uint32_t)c->n / 2;
  if (n_parts == 0 || width == 0 || (uint64_t)width * n_parts > half) return fail(HE_ERANGE, "width * parts > N/2");
  if (n_parts > HE_MAX_BATCH + 1) return fail(HE_ERANGE, "more than %d parts", HE_MAX_BATCH + 1);
  int l = parts[0] ? parts[0]->level : 0;
  for (uint32_t k = 0; k < n_parts; k++) {
    if (!parts[k]) return fail(HE_EINVAL, "NULL part");
    l = std::min(l, parts[k]->level);
  }
  if (l < 1) return fail(HE_ELEVEL, "packing needs one level");
  he_pt* mask = nullptr;
  auto key = std::make_pair((int)width, l);
  auto it = c->masks.find(key);
  if (it != c->masks.end()) {
    mask = it->second;
  } else {
    std::vector<double> ones(width, 1.0);
    TRY(encode_slots(c, ones, c->scale, l, &mask));
    c->masks[key] = mask;
  }
  const int n = c->n, Lp = l + 1, np = (int)n_parts;
  const size_t ct_w = 2 * (size_t)Lp * n, ct_w1 = 2 * (size_t)l * n;
  DBuf M, Y;
  TRY(dalloc(c, M, np * ct_w));
  TRY(dalloc(c, Y, np * ct_w1));
  {
    std::vector<CtGuard> dropped(np);
    CtList in{}, mp{};
    for (int k = 0; k < np; k++) {
      const he_ct* src = parts[k];
      if (src->level != l) {
        TRY(drop_copy(c, src, l, &dropped[k].p));
        src = dropped[k].p;
      }
      in.p[k] = src->d;
      mp.p[k] = mask->d;
    }
    Prof pr(c, "pointwise");
    hipError_t e = launch_mul_plain_many(c->log_n, in, mp, np, Lp, M.p, c->d_primes, c->st);
    if (e != hipSuccess) return fail(HE_EHIP, "mul_plain: %s", hipGetErrorString(e));
  }
  TRY(rescale_multi(c, M.p, np, l, Y.p));
  const double scale0 = parts[0]->scale * mask->scale / (double)c->q[l];
  for (int k = 1; k < np; k++)
    if (!scales_match(parts[k]->scale * mask->scale / (double)c->q[l], scale0))
      return fail(HE_ESCALE, "part scales differ");
  DBuf R;
  if (np > 1) {
    TRY(dalloc(c, R, (np - 1) * ct_w1));
    std::vector<int> st(np - 1);
    for (int k = 1; k < np; k++) st[k - 1] = norm_step(c, (long long)half - (long long)width * k);
    TRY(rotate_multi(c, Y.p + ct_w1, np - 1, l - 1, st.data(), R.p));
  }
  he_ct* r = nullptr;
  TRY(new_ct(c, l - 1, scale0, &r));
  CtGuard gr{r};
  {
    CtList in{};
    in.p[0] = Y.p;
    for (int k = 1; k < np; k++) in.p[k] = R.p + (k - 1) * ct_w1;
    Prof pr(c, "pointwise");
    HIPC(launch_sum_cts(c->log_n, in, np, l, r->d, c->d_primes, c->st));
  }
  *out = r;
  gr.p = nullptr;
  return HE_OK;
}

// ---------------------------------------------------------------- raw transforms
he_status he_ntt_forward(he_ctx* c, uint64_t* data, size_t n_polys, int32_t n_limbs) {
  if (!c || !data) return fail(HE_EINVAL, "NULL argument");
  if ((uintptr_t)data % 16) return fail(HE_EINVAL, "data must be 16-byte aligned");
  if (n_limbs < 1 || n_limbs > c->L) return fail(HE_EINVAL, "n_limbs %d outside 1..%d", n_limbs, c->L);
  return ntt_rows(c, true, data, data, (int)n_polys, n_limbs, (long long)n_limbs * c->n, (long long)n_limbs * c->n);
}
he_status he_ntt_inverse(he_ctx* c, uint64_t* data, size_t n_polys, int32_t n_limbs) {
  if (!c || !data) return fail(HE_EINVAL, "NULL argument");
  if ((uintptr_t)data % 16) return fail(HE_EINVAL, "data must be 16-byte aligned");
  if (n_limbs < 1 || n_limbs > c->L) return fail(HE_EINVAL, "n_limbs %d outside 1..%d", n_limbs, c->L);
  return ntt_rows(c, false, data, data, (int)n_polys, n_limbs, (long long)n_limbs * c->n, (long long)n_limbs * c->n);
}

// ---------------------------------------------------------------- key export
he_status he_export_secret(he_ctx* c, int64_t* s) {
  NO_CAPTURE(c);
  if (!c || !s) return fail(HE_EINVAL, "NULL argument");
  if (!c->have_keys) return fail(HE_ENOKEY, "no secret key");
  std::vector<u64> v;
  TRY(download_coeff(c, c->d_s, 1, 1, v));
  const u64 q = c->q[0];
  for (int k = 0; k < c->n; k++) s[k] = v[k] > q / 2 ? (int64_t)v[k] - (int64_t)q : (int64_t)v[k];
  return HE_OK;
}

he_status he_export_key(he_ctx* c, int32_t kind, int32_t step, uint64_t* out, size_t cap, int32_t* max_level) {
  NO_CAPTURE(c);
  if (!c || !out) return fail(HE_EINVAL, "NULL argument");
  const Key* k = nullptr;
  if (kind == 0) {
    if (c->have_keys) k = &c->relin;
  } else {
    auto it = c->gal.find(norm_step(c, step));
    if (it != c->gal.end()) k = &it->second;
  }
  if (!k || !k->d) return fail(HE_ENOKEY, "no such key");
  const int nd = k->ml + 1, nm = k->ml + 2, n = c->n;
  const size_t words = (size_t)nd * 2 * nm * n;
  if (cap < words) return fail(HE_EINVAL, "capacity %zu < %zu words", cap, words);
  ModList pidx{};
  pidx.n = nm;
  for (int t = 0; t < nm; t++) pidx.p[t] = (unsigned char)(t <= k->ml ? t : c->L);
  DBuf tmp;
  TRY(dalloc(c, tmp, words));
  HIPC(hipMemcpyAsync(tmp.p, k->d, words * sizeof(u64), hipMemcpyDeviceToDevice, c->st));
  hipError_t e = launch_from_mont(c->log_n, tmp.p, nd * 2 * nm, pidx, c->d_primes, c->st);
  if (e != hipSuccess) return fail(HE_EHIP, "from_mont: %s", hipGetErrorString(e));
  TRY(ntt_rows_mods(c, false, tmp.p, tmp.p, nd * 2, pidx));
  HIPC(hipMemcpyAsync(out, tmp.p, words * sizeof(u64), hipMemcpyDeviceToHost, c->st));
  HIPC(hipStreamSynchronize(c->st));
  if (max_level) *max_level = k->ml;
  return HE_OK;
}

// ---------------------------------------------------------------- housekeeping
// ---------------------------------------------------------------- NTT autotuner
// Times batched forward + inverse transforms of J limbs (the context's data
// primes in turn) with one workgroup per limb and with the two-phase
// kernels, for J = 16, 32, ... up to max_jobs, and keeps the faster form for
// each size (launches are bucketed by the next candidate J).
he_status he_tune_ntt(he_ctx* c, int32_t max_jobs, int32_t* split_jobs, double* table, size_t table_cap) {
  if (!c) return fail(HE_EINVAL, "NULL context");
  NO_CAPTURE(c);
  if (max_jobs < 16) return fail(HE_EINVAL, "max_jobs %d < 16", max_jobs);
  const int n = c->n, L = c->L;
  std::vector<int> cand;
  for (int j = 16; j <= max_jobs && cand.size() < 16; j *= 2) cand.push_back(j);
  const int jmax = cand.back();
  NttShape shapes[8];
  const int n_shapes = std::min(8, ntt_shapes(c->log_n, shapes, 8));
  DBuf buf;
  TRY(dalloc(c, buf, (size_t)jmax * n));
  {
    // uniform residues (a stream of the tuner's own): the timing of
    // all-zero data is not that of real data (the part draws less power on
    // it and runs at a higher clock)
    const int nbf = std::min(L, jmax);
    ModList mods;
    mods.n = nbf;
    for (int i = 0; i < nbf; i++) mods.p[i] = (unsigned char)i;
    HIPC(launch_sample_uniform(c->log_n, c->seed, 0x7e, 0, jmax / nbf, mods, mods, buf.p, c->d_primes, c->st));
  }
  u64* tmp = (u64*)c->pool.get((size_t)jmax * n * sizeof(u64));
  if (!tmp) return fail(HE_EOOM, "tuning scratch");
  const NttTables saved = c->tabs;
  hipEvent_t ea, eb;
  HIPC(hipEventCreate(&ea));
  HIPC(hipEventCreate(&eb));
  he_status s = HE_OK;
  unsigned mask = 0;
  unsigned char best_shape[16] = {0};
  int largest = 0;  // largest J that chose the two-phase form
  size_t row = 0;
  for (size_t ci = 0; ci < cand.size() && s == HE_OK; ci++) {
    const int J = cand[ci];
    const int nb = std::min(L, J), na = J / nb;
    // candidate 0: the two-phase form; 1 + k: one workgroup per limb in layout k
    std::vector<float> ms(1 + n_shapes, 0.f);
    for (int cnd = 0; cnd < 1 + n_shapes && s == HE_OK; cnd++) {
      c->tabs = saved;
      c->tabs.tmp = tmp;
      c->tabs.tmp_words = (long long)jmax * n;
      if (cnd == 0) {
        c->tabs.tuned = 0;
        c->tabs.split_jobs = jmax;
      } else {
        c->tabs.tuned = 1;
        c->tabs.split_mask = 0;
        c->tabs.n_buckets = 1;
        c->tabs.shape[0] = (unsigned char)(cnd - 1);
      }
      for (int rep = 0; rep < 6 && s == HE_OK; rep++) {  // the first repetition warms up
        if (rep == 1) (void)hipEventRecord(ea, c->st);
        s = ntt_rows(c, true, buf.p, buf.p, na, nb, (long long)nb * n, (long long)nb * n);
        if (s == HE_OK) s = ntt_rows(c, false, buf.p, buf.p, na, nb, (long long)nb * n, (long long)nb * n);
      }
      (void)hipEventRecord(eb, c->st);
      (void)hipEventSynchronize(eb);
      (void)hipEventElapsedTime(&ms[cnd], ea, eb);
    }
    if (s != HE_OK) break;
    int win = 0;
    for (int cnd = 1; cnd < 1 + n_shapes; cnd++)
      if (ms[cnd] < ms[win]) win = cnd;
    if (table && row + 2 + n_shapes <= table_cap) {
      table[row++] = J;
      for (int cnd = 0; cnd < 1 + n_shapes; cnd++) table[row++] = ms[cnd] / 5 * 1e3;  // us per forward + inverse
    }
    if (win == 0) {
      mask |= 1u << ci;
      largest = J;
    } else {
      best_shape[ci] = (unsigned char)(win - 1);
    }
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  c->tabs = saved;
  if (s != HE_OK) {
    c->pool.put(tmp);
    return s;
  }
  // scratch for the largest two-phase batch (launches beyond it run one
  // workgroup per limb)
  if (c->tabs.tmp) c->pool.put(c->tabs.tmp);
  c->pool.put(tmp);
  c->tabs.tmp = nullptr;
  c->tabs.tmp_words = 0;
  c->tabs.split_jobs = largest;
  c->tabs.tuned = 1;
  c->tabs.split_mask = mask;
  c->tabs.n_buckets = (int)cand.size();
  for (size_t ci = 0; ci < 16; ci++) c->tabs.shape[ci] = best_shape[ci];
  if (largest > 0) {
    c->tabs.tmp = (u64*)c->pool.get((size_t)largest * n * sizeof(u64));
    if (!c->tabs.tmp) {
      c->tabs.tuned = 0;
      c->tabs.split_jobs = 0;
      return fail(HE_EOOM, "scratch allocation failed");
    }
    c->tabs.tmp_words = (long long)largest * n;
  }
  if (split_jobs) *split_jobs = largest;
  return HE_OK;
}

he_status he_ntt_layouts(he_ctx* c, int32_t* loge, int32_t* logr, size_t cap, size_t* count) {
  if (!c || !count) return fail(HE_EINVAL, "NULL argument");
  NttShape shapes[8];
  const int k = std::min(8, ntt_shapes(c->log_n, shapes, 8));
  *count = (size_t)k;
  for (int i = 0; i < k && (size_t)i < cap; i++) {
    if (loge) loge[i] = shapes[i].loge;
    if (logr) logr[i] = shapes[i].logr;
  }
  return HE_OK;
}


// ---------------------------------------------------------------- graphs
struct he_graph {
  he_ctx* ctx;
  hipGraph_t graph;
  hipGraphExec_t exec;
  std::vector<void*> retained;  // intermediates the replays write
};

he_status he_graph_begin(he_ctx* c) {
  if (!c) return fail(HE_EINVAL, "NULL context");
  if (c->capturing) return fail(HE_EINVAL, "a capture is already open");
  hipError_t e = hipStreamBeginCapture(c->st, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return fail(HE_EHIP, "capture begin: %s", hipGetErrorString(e));
  c->capturing = true;
  c->pool.retain = true;
  return HE_OK;
}

he_status he_graph_end(he_ctx* c, he_graph** out) {
  if (!c || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  if (!c->capturing) return fail(HE_EINVAL, "no capture open");
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->st, &g);
  c->capturing = false;
  c->pool.retain = false;
  std::vector<void*> kept;
  kept.swap(c->pool.retained);
  hipGraphExec_t x = nullptr;
  if (e == hipSuccess && g) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess || !g || !x) {
    if (g) (void)hipGraphDestroy(g);
    for (void* p : kept) c->pool.put(p);
    return fail(HE_EHIP, "graph capture failed: %s", hipGetErrorString(e));
  }
  *out = new he_graph{c, g, x, std::move(kept)};
  return HE_OK;
}

he_status he_graph_launch(he_ctx* c, const he_graph* g) {
  if (!c || !g) return fail(HE_EINVAL, "NULL argument");
  if (g->ctx != c) return fail(HE_EINVAL, "graph of another context");
  if (c->capturing) return fail(HE_EINVAL, "capture open on this context");
  HIPC(hipGraphLaunch(g->exec, c->st));
  return HE_OK;
}

void he_graph_free(he_graph* g) {
  if (!g) return;
  (void)hipStreamSynchronize(g->ctx->st);
  (void)hipGraphExecDestroy(g->exec);
  (void)hipGraphDestroy(g->graph);
  for (void* p : g->retained) g->ctx->pool.put(p);
  delete g;
}

he_status he_ct_copy(he_ctx* c, he_ct* dst, const he_ct* src) {
  TRY(own(c, dst));
  TRY(own(c, src));
  if (!c || !dst || !src) return fail(HE_EINVAL, "NULL argument");
  if (dst->level != src->level) return fail(HE_ELEVEL, "levels %d and %d differ", dst->level, src->level);
  HIPC(launch_copy(src->d, dst->d, (long long)ct_words(c, src->level), c->st));
  dst->scale = src->scale;
  return HE_OK;
}

void he_ct_free(he_ct* ct) {
  if (!ct) return;
  if (!ct->blk) ct->ctx->pool.put(ct->d);
  delete ct;  // a shared block goes back to the pool with its last view
}
void he_pt_free(he_pt* pt) {
  if (!pt) return;
  pt->ctx->pool.put(pt->d);
  delete pt;
}
void he_plan_free(he_plan* p) {
  if (!p) return;
  he_pt_free(p->kernel);
  he_pt_free(p->bias);
  if (p->diags) p->ctx->pool.put(p->diags);
  if (p->items) p->ctx->pool.put(p->items);
  if (p->rep_items) p->ctx->pool.put(p->rep_items);
  delete p;
}

he_status he_sync(he_ctx* c) {
  if (!c) return fail(HE_EINVAL, "NULL context");
  NO_CAPTURE(c);
  HIPC(hipStreamSynchronize(c->st));
  return HE_OK;
}

size_t he_ct_bytes(const he_ct* ct) { return ct ? ct_words(ct->ctx, ct->level) * sizeof(u64) : 0; }

size_t he_key_bytes(const he_ctx* c) {
  if (!c) return 0;
  size_t b = c->relin.bytes;
  for (auto& kv : c->gal) b += kv.second.bytes;
  if (c->have_keys) b += (size_t)(c->L + 1) * c->n * 8 + 2 * (size_t)c->L * c->n * 8;
  return b;
}

void he_im2col(const double* img, uint32_t h, uint32_t w, uint32_t k, uint32_t stride, double* out) {
  if (!img || !out || k == 0 || stride == 0 || k > h || k > w) return;
  const uint32_t oh = (h - k) / stride + 1, ow = (w - k) / stride + 1, windows = oh * ow;
  for (uint32_t oy = 0; oy < oh; oy++)
    for (uint32_t ox = 0; ox < ow; ox++) {
      const uint32_t win = oy * ow + ox;
      for (uint32_t ky = 0; ky < k; ky++)
        for (uint32_t kx = 0; kx < k; kx++)
          out[(size_t)(ky * k + kx) * windows + win] = img[(size_t)(oy * stride + ky) * w + ox * stride + kx];
    }
}

he_status he_profile_enable(he_ctx* c, int32_t enable) {
  if (!c) return fail(HE_EINVAL, "NULL context");
  HIPC(hipStreamSynchronize(c->st));
  for (auto& r : c->prof_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  c->prof_recs.clear();
  c->prof = enable != 0;
  return HE_OK;
}

he_status he_profile_read(he_ctx* c, const char* fam, uint64_t* launches, double* total_ms, double* units,
                          double* bytes) {
  if (!c || !fam) return fail(HE_EINVAL, "NULL argument");
  HIPC(hipStreamSynchronize(c->st));
  uint64_t cnt = 0;
  double ms = 0, un = 0, by = 0;
  for (auto& r : c->prof_recs) {
    if (r.fam != fam) continue;
    float t = 0;
    HIPC(hipEventElapsedTime(&t, r.a, r.b));
    ms += t;
    un += r.units;
    by += r.bytes;
    cnt++;
  }
  if (launches) *launches = cnt;
  if (total_ms) *total_ms = ms;
  if (units) *units = un;
  if (bytes) *bytes = by;
  return HE_OK;
}


// ---------------------------------------------------------------- tensors
// CKKSTensor with a batched axis (section 2, the tensor flavours): the last
// axis of a shape d_0 x ... x d_{r-1} lies in the slots, in chunks of N/2;
// the other axes index ciphertexts.  Ciphertext (row, chunk) holds elements
// row * d_{r-1} + chunk * N/2 + j, j < N/2, of the row-major value array.
struct he_tensor {
  he_ctx* ctx = nullptr;
  std::vector<int64_t> shape;
  size_t rows = 0, chunks = 0;
  int64_t last = 0;
  std::vector<he_ct*> cts;  // [rows][chunks], owned
};

static void tensor_release(he_tensor* t) {
  for (he_ct* x : t->cts) he_ct_free(x);
  delete t;
}

static he_status tensor_alloc(he_ctx* c, const std::vector<int64_t>& shape, he_tensor** out) {
  if (shape.empty() || shape.size() > HE_TENSOR_MAX_DIMS) return fail(HE_EINVAL, "tensor rank %zu", shape.size());
  size_t rows = 1;
  for (size_t i = 0; i + 1 < shape.size(); i++) {
    if (shape[i] <= 0) return fail(HE_EINVAL, "tensor axis %zu has size %lld", i, (long long)shape[i]);
    rows *= (size_t)shape[i];
  }
  const int64_t last = shape.back();
  if (last <= 0) return fail(HE_EINVAL, "tensor last axis has size %lld", (long long)last);
  const int64_t half = c->n / 2;
  he_tensor* t = new he_tensor();
  t->ctx = c;
  t->shape = shape;
  t->rows = rows;
  t->last = last;
  t->chunks = (size_t)((last + half - 1) / half);
  t->cts.assign(rows * t->chunks, nullptr);
  *out = t;
  return HE_OK;
}

// values of chunk (row, j): offset into the row-major array and count
static void chunk_span(const he_tensor* t, size_t row, size_t j, size_t* off, size_t* cnt) {
  const int64_t half = t->ctx->n / 2;
  *off = row * (size_t)t->last + j * (size_t)half;
  *cnt = (size_t)std::min<int64_t>(half, t->last - (int64_t)j * half);
}

static he_status tensor_check(he_ctx* c, const he_tensor* a) {
  if (!c || !a) return fail(HE_EINVAL, "NULL argument");
  if (a->ctx != c) return fail(HE_EINVAL, "tensor of another context");
  return HE_OK;
}

static he_status tensor_same_shape(const he_tensor* a, const he_tensor* b) {
  if (a->shape != b->shape) return fail(HE_EINVAL, "tensor shapes differ");
  return HE_OK;
}

he_status he_tensor_encrypt(he_ctx* c, const double* values, const int64_t* shape, int32_t ndim, double scale,
                            int32_t level, uint32_t enc_index0, int32_t use_secret_key, he_tensor** out) {
  if (!c || !values || !shape || !out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  if (ndim < 1) return fail(HE_EINVAL, "tensor rank %d", ndim);
  he_tensor* t = nullptr;
  TRY(tensor_alloc(c, std::vector<int64_t>(shape, shape + ndim), &t));
  for (size_t r = 0; r < t->rows; r++)
    for (size_t j = 0; j < t->chunks; j++) {
      size_t off, cnt;
      chunk_span(t, r, j, &off, &cnt);
      he_pt* pt = nullptr;
      he_status s = he_encode(c, values + off, cnt, scale, level, &pt);
      const size_t i = r * t->chunks + j;
      if (s == HE_OK) s = he_encrypt(c, pt, enc_index0 + (uint32_t)i, use_secret_key, &t->cts[i]);
      he_pt_free(pt);
      if (s != HE_OK) {
        tensor_release(t);
        return s;
      }
    }
  *out = t;
  return HE_OK;
}

he_status he_tensor_decrypt(he_ctx* c, const he_tensor* t, double* out, size_t n) {
  TRY(tensor_check(c, t));
  if (!out) return fail(HE_EINVAL, "NULL argument");
  if (n < t->rows * (size_t)t->last) return fail(HE_EINVAL, "output holds %zu of %zu values", n,
                                                 t->rows * (size_t)t->last);
  for (size_t r = 0; r < t->rows; r++)
    for (size_t j = 0; j < t->chunks; j++) {
      size_t off, cnt;
      chunk_span(t, r, j, &off, &cnt);
      he_pt* pt = nullptr;
      TRY(he_decrypt(c, t->cts[r * t->chunks + j], &pt));
      he_status s = he_decode(c, pt, out + off, cnt);
      he_pt_free(pt);
      if (s != HE_OK) return s;
    }
  return HE_OK;
}

he_status he_tensor_shape(const he_tensor* t, int64_t* shape, int32_t* ndim, size_t* n_ct) {
  if (!t) return fail(HE_EINVAL, "NULL argument");
  if (ndim) *ndim = (int32_t)t->shape.size();
  if (shape)
    for (size_t i = 0; i < t->shape.size(); i++) shape[i] = t->shape[i];
  if (n_ct) *n_ct = t->cts.size();
  return HE_OK;
}

he_status he_tensor_ct(const he_tensor* t, size_t i, const he_ct** out) {
  if (!t || !out) return fail(HE_EINVAL, "NULL argument");
  if (i >= t->cts.size()) return fail(HE_EINVAL, "ciphertext %zu of %zu", i, t->cts.size());
  *out = t->cts[i];
  return HE_OK;
}

void he_tensor_free(he_tensor* t) {
  if (t) tensor_release(t);
}

// result tensor of a's shape, ciphertext i = f(i)
extern "C++" {
template <class F>
static he_status tensor_map(he_ctx* c, const he_tensor* a, he_tensor** out, F f) {
  *out = nullptr;
  he_tensor* t = nullptr;
  TRY(tensor_alloc(c, a->shape, &t));
  for (size_t i = 0; i < t->cts.size(); i++) {
    he_status s = f(i, &t->cts[i]);
    if (s != HE_OK) {
      tensor_release(t);
      return s;
    }
  }
  *out = t;
  return HE_OK;
}
}  // extern "C++"

he_status he_tensor_add(he_ctx* c, const he_tensor* a, const he_tensor* b, he_tensor** out) {
  TRY(tensor_check(c, a));
  TRY(tensor_check(c, b));
  TRY(tensor_same_shape(a, b));
  if (!out) return fail(HE_EINVAL, "NULL argument");
  return tensor_map(c, a, out, [&](size_t i, he_ct** o) { return he_add(c, a->cts[i], b->cts[i], o); });
}

he_status he_tensor_sub(he_ctx* c, const he_tensor* a, const he_tensor* b, he_tensor** out) {
  TRY(tensor_check(c, a));
  TRY(tensor_check(c, b));
  TRY(tensor_same_shape(a, b));
  if (!out) return fail(HE_EINVAL, "NULL argument");
  return tensor_map(c, a, out, [&](size_t i, he_ct** o) { return he_sub(c, a->cts[i], b->cts[i], o); });
}

he_status he_tensor_negate(he_ctx* c, const he_tensor* a, he_tensor** out) {
  TRY(tensor_check(c, a));
  if (!out) return fail(HE_EINVAL, "NULL argument");
  return tensor_map(c, a, out, [&](size_t i, he_ct** o) { return he_negate(c, a->cts[i], o); });
}

// products of all ciphertext pairs as batches (shared key reads)
static he_status tensor_products(he_ctx* c, const he_tensor* a, const he_tensor* b, he_tensor** out) {
  *out = nullptr;
  he_tensor* t = nullptr;
  TRY(tensor_alloc(c, a->shape, &t));
  he_status s = he_mul_relin_many(c, a->cts.data(), b->cts.data(), a->cts.size(), t->cts.data());
  if (s != HE_OK) {
    tensor_release(t);
    return s;
  }
  *out = t;
  return HE_OK;
}

he_status he_tensor_mul(he_ctx* c, const he_tensor* a, const he_tensor* b, he_tensor** out) {
  TRY(tensor_check(c, a));
  TRY(tensor_check(c, b));
  TRY(tensor_same_shape(a, b));
  if (!out) return fail(HE_EINVAL, "NULL argument");
  return tensor_products(c, a, b, out);
}

he_status he_tensor_square(he_ctx* c, const he_tensor* a, he_tensor** out) {
  TRY(tensor_check(c, a));
  if (!out) return fail(HE_EINVAL, "NULL argument");
  return tensor_products(c, a, a, out);
}

// plain operand of a's shape, chunk i encoded at ciphertext i's level, at
// the ciphertext's scale (sums) or at the context's (products)
enum PlainOp { PLAIN_ADD, PLAIN_SUB, PLAIN_MUL };
static he_status tensor_plain(he_ctx* c, const he_tensor* a, const double* v, PlainOp op, he_tensor** out) {
  TRY(tensor_check(c, a));
  if (!v || !out) return fail(HE_EINVAL, "NULL argument");
  return tensor_map(c, a, out, [&](size_t i, he_ct** o) {
    size_t off, cnt;
    chunk_span(a, i / a->chunks, i % a->chunks, &off, &cnt);
    const he_ct* x = a->cts[i];
    he_pt* pt = nullptr;
    TRY(he_encode(c, v + off, cnt, op == PLAIN_MUL ? c->scale : x->scale, x->level, &pt));
    he_status s = op == PLAIN_ADD ? he_add_plain(c, x, pt, o)
                  : op == PLAIN_SUB ? he_sub_plain(c, x, pt, o)
                                    : he_mul_plain(c, x, pt, o);
    he_pt_free(pt);
    return s;
  });
}

he_status he_tensor_add_plain(he_ctx* c, const he_tensor* a, const double* v, he_tensor** out) {
  return tensor_plain(c, a, v, PLAIN_ADD, out);
}
he_status he_tensor_sub_plain(he_ctx* c, const he_tensor* a, const double* v, he_tensor** out) {
  return tensor_plain(c, a, v, PLAIN_SUB, out);
}
he_status he_tensor_mul_plain(he_ctx* c, const he_tensor* a, const double* v, he_tensor** out) {
  return tensor_plain(c, a, v, PLAIN_MUL, out);
}

he_status he_tensor_power(he_ctx* c, const he_tensor* a, uint32_t k, he_tensor** out) {
  TRY(tensor_check(c, a));
  if (!out) return fail(HE_EINVAL, "NULL argument");
  return tensor_map(c, a, out, [&](size_t i, he_ct** o) { return he_power(c, a->cts[i], k, o); });
}

he_status he_tensor_polyval(he_ctx* c, const he_tensor* a, const double* coeffs, size_t n_coeffs,
                            he_tensor** out) {
  TRY(tensor_check(c, a));
  if (!out) return fail(HE_EINVAL, "NULL argument");
  return tensor_map(c, a, out,
                    [&](size_t i, he_ct** o) { return he_polyval(c, a->cts[i], coeffs, n_coeffs, o); });
}

// sum over the batched (last) axis: each row's chunks added in order, then
// the rotate-and-sum of its slots; the result has last axis 1 (slot 0)
he_status he_tensor_sum(he_ctx* c, const he_tensor* a, he_tensor** out) {
  TRY(tensor_check(c, a));
  if (!out) return fail(HE_EINVAL, "NULL argument");
  *out = nullptr;
  std::vector<int64_t> shape = a->shape;
  shape.back() = 1;
  he_tensor* t = nullptr;
  TRY(tensor_alloc(c, shape, &t));
  const uint32_t width = (uint32_t)std::min<int64_t>(a->last, c->n / 2);
  for (size_t r = 0; r < a->rows; r++) {
    CtGuard acc;
    he_status s = HE_OK;
    const he_ct* cur = a->cts[r * a->chunks];
    for (size_t j = 1; j < a->chunks && s == HE_OK; j++) {
      he_ct* nxt = nullptr;
      s = he_add(c, cur, a->cts[r * a->chunks + j], &nxt);
      if (s == HE_OK) {
        he_ct_free(acc.p);
        acc.p = nxt;
        cur = nxt;
      }
    }
    if (s == HE_OK) s = he_sum_slots(c, cur, width, &t->cts[r]);
    if (s != HE_OK) {
      tensor_release(t);
      return s;
    }
  }
  *out = t;
  return HE_OK;
}

he_status he_tensor_dot(he_ctx* c, const he_tensor* a, const he_tensor* b, he_tensor** out) {
  if (!out) return fail(HE_EINVAL, "NULL argument");
  he_tensor* p = nullptr;
  TRY(he_tensor_mul(c, a, b, &p));
  he_status s = he_tensor_sum(c, p, out);
  tensor_release(p);
  return s;
}

he_status he_tensor_dot_plain(he_ctx* c, const he_tensor* a, const double* w, he_tensor** out) {
  if (!out) return fail(HE_EINVAL, "NULL argument");
  he_tensor* p = nullptr;
  TRY(he_tensor_mul_plain(c, a, w, &p));
  he_status s = he_tensor_sum(c, p, out);
  tensor_release(p);
  return s;
}

}  // extern "C"
