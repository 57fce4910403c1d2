/*
 * ckks_hip.h -- C ABI of the MI355X (gfx950) RNS-CKKS library.
 *
 * The library evaluates the ciphertext arithmetic under TenSEAL's encrypted
 * tensor operations (arXiv 2104.03152): the context and its keys (section
 * 2.1), CKKSVector element-wise operations (section 3, table of supported
 * operations in appendix A.2), the replicated-input dot/vector-matrix product
 * (section 3.1, appendix A.3), the im2col convolution on one ciphertext
 * (section 3.2, appendix A.4) and the MNIST-shaped network of section 5.
 * The scheme is CKKS (Cheon et al. 2017) over Z_Q[X]/(X^N + 1) in RNS form.
 *
 * Conventions
 *  - Handles are opaque.  Every `out` handle is new and owned by the caller,
 *    who frees it with the matching he_*_free.  Inputs are never consumed or
 *    modified.
 *  - Handles belong to the context that made them; a call given a handle of
 *    another context fails with HE_EINVAL before anything is enqueued (the
 *    context's stream is what orders the work on a handle's memory).
 *  - Device memory comes from the allocator callbacks given to he_ctx_create
 *    (NULL: the library's own caching pool over hipMalloc).  Freed blocks are
 *    cached by the context and reused in stream order; they go back to the
 *    allocator only after the context's stream has drained (when a failed
 *    allocation trims the cache, and at he_ctx_destroy).  An allocator that
 *    returns NULL makes the call fail with HE_EOOM after the cache has been
 *    trimmed and the allocation retried; the call's partial results are
 *    released and the context stays usable.
 *  - Every operation is enqueued on the context's HIP stream and returns
 *    before the GPU finishes, except the calls that return host data
 *    (export, decode, decrypt+decode paths), which synchronise the stream.
 *    One context per host thread.
 *  - Levels: a ciphertext at level l holds limbs 0..l of the data-prime chain
 *    (level L-1 is fresh).  Binary operations on different levels drop limbs
 *    of the higher operand (exact).  Scales must agree to 2^-20 relative.
 *  - Rotations are LEFT rotations of the N/2 slots (section 3.1 uses left
 *    rotations only); a right rotation by r is the left rotation N/2 - r.
 *  - Status codes: HE_OK = 0 or one of the negative codes below; on error
 *    `*out` is left NULL and he_last_error() describes the failure.
 */
#ifndef CKKS_HIP_H
#define CKKS_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t he_status;
enum {
  HE_OK = 0,
  HE_EINVAL = -1, /* bad argument (NULL handle, bad size, bad parameters)  */
  HE_ERANGE = -2, /* more than N/2 values, or an encoded coefficient >= 2^62 */
  HE_ELEVEL = -3, /* no level left (the leveled limit of section 6)          */
  HE_ESCALE = -4, /* operand scales differ by more than 2^-20 relative       */
  HE_ENOKEY = -5, /* missing key (rotation step, or key cut below the level) */
  HE_EOOM = -6,   /* the allocator returned NULL                             */
  HE_EHIP = -7    /* a HIP runtime error                                     */
};

typedef struct he_ctx he_ctx;
typedef struct he_ct he_ct;     /* ciphertext: 2 polys x (level+1) limbs      */
typedef struct he_pt he_pt;     /* plaintext: 1 poly x (level+1) limbs        */
typedef struct he_plan he_plan; /* a composite with its plaintexts prepared   */

/* Device allocator: return `bytes` of device memory (256-byte aligned) or
 * NULL.  `user` is the alloc_user pointer given to he_ctx_create. */
typedef void* (*he_alloc_fn)(size_t bytes, void* user);
typedef void (*he_free_fn)(void* ptr, size_t bytes, void* user);

#define HE_MAX_PRIMES 32

typedef struct {
  int32_t log_n;     /* ring degree N = 2^log_n, 10 <= log_n <= 14           */
  int32_t n_primes;  /* data primes + 1 special prime, 2..HE_MAX_PRIMES       */
  int32_t prime_bits[HE_MAX_PRIMES]; /* bit sizes, data first, special last;
                        each in [log_n + 2, 61].  For each size in order the
                        prime is the largest q < 2^b with q = 1 mod 2N that is
                        not already in the chain.                           */
  double scale;      /* encoding scale Delta for plaintext operands          */
  int32_t auto_rescale; /* he_mul_plain / he_mul_relin rescale their result */
  uint64_t seed;     /* seed of every sampler stream (ChaCha20 key)          */
} he_params;

/* ---- context and keys (section 2.1) ---- */

/* Create a context: prime chain, NTT tables.  hip_stream: a hipStream_t to
 * enqueue on (NULL: the library creates a stream of default priority).
 * Kernel-shape settings read from the environment here (results do not
 * depend on them): HE_NTT_SPLIT_JOBS (two-phase transforms for launches of
 * up to this many limbs, default 256), HE_FUSE_MAX (fused key switch while
 * items x digits^2 stays within it, default 256), HE_HOIST_SPLIT_WGS (about
 * this many workgroups for the hoisted multiply-accumulate's block phase,
 * at least two rotations each, default 4096; 0 selects the one-kernel form), HE_COEF_ROT (rotate-and-sum
 * chains -- the convolution's, slot sums of three or more steps -- with the
 * ciphertext in coefficient form between steps, default 1; 0: in the
 * transform domain).
 * Errors: HE_EINVAL for bad parameters, HE_EHIP, HE_EOOM. */
he_status he_ctx_create(const he_params* params, he_alloc_fn alloc,
                        he_free_fn free_fn, void* alloc_user, void* hip_stream,
                        he_ctx** out);
/* Waits for the context's stream and releases all its device memory.  Free
 * every ciphertext, plaintext, plan and graph of the context before: their
 * handles are invalid afterwards (freeing one then is undefined). */
void he_ctx_destroy(he_ctx* ctx);
/* primes: n_data_primes + 1 entries (special prime last). */
he_status he_ctx_info(const he_ctx* ctx, int32_t* log_n, int32_t* n_data_primes,
                      uint64_t* primes);

/* Secret key (ternary), public key, relinearisation key (for s^2) and one
 * Galois key per left-rotation step in rot_steps (steps mod N/2, 0 skipped),
 * all on the device.  Sampling: ChaCha20 streams keyed by params.seed. */
he_status he_keygen(he_ctx* ctx, const int32_t* rot_steps, size_t n_steps);
/* One Galois key valid for levels 0..max_level (max_level < 0: top level).
 * A key cut at a lower level is the exact restriction of the top-level key,
 * so results are identical; it takes (max_level+1)(max_level+2)/(L(L+1))
 * of the memory.  Requires he_keygen first (HE_ENOKEY). */
he_status he_keygen_galois(he_ctx* ctx, int32_t step, int32_t max_level);

/* ---- encoding (section 3: a CKKSVector holds N/2 reals) ---- */

/* Encode n <= N/2 reals into slots 0..n-1 (the rest 0) at `scale`, level
 * `level`.  Slot j is the evaluation at zeta^(5^j), zeta = exp(i pi/N);
 * coefficients are round(scale * m_k), ties away from zero, correctly
 * rounded.  HE_ERANGE: n > N/2 or a coefficient >= 2^62. */
he_status he_encode(he_ctx* ctx, const double* v, size_t n, double scale,
                    int32_t level, he_pt** out);
/* Decode slots 0..n-1 of a plaintext (synchronises). */
he_status he_decode(he_ctx* ctx, const he_pt* pt, double* out, size_t n);
/* Plaintext from N signed integer coefficients (reduced into every limb). */
he_status he_pt_import(he_ctx* ctx, const int64_t* coeffs, double scale,
                       int32_t level, he_pt** out);
/* Plaintext residues in coefficient form, [level+1][N]; cap in words. */
he_status he_pt_export(he_ctx* ctx, const he_pt* pt, uint64_t* coeff_form,
                       size_t cap, int32_t* level, double* scale);

/* ---- encryption (section 2.1: the context's public key encrypts, its secret
 * key decrypts; section 2.3's encrypted tensors hold these ciphertexts) ---- */

/* Public-key encryption (use_secret_key = 0): (v*pk0 + e0 + m, v*pk1 + e1);
 * secret-key: (-a*s + e + m, a).  enc_index selects the sampler streams, so
 * equal indices give equal ciphertexts. */
he_status he_encrypt(he_ctx* ctx, const he_pt* pt, uint32_t enc_index,
                     int32_t use_secret_key, he_ct** out);
/* m = c0 + c1*s at the ciphertext's level and scale. */
he_status he_decrypt(he_ctx* ctx, const he_ct* ct, he_pt** out);

/* Ciphertext residues in coefficient form, [2][level+1][N]; cap in words. */
he_status he_ct_export(he_ctx* ctx, const he_ct* ct, uint64_t* coeff_form,
                       size_t cap, int32_t* level, double* scale);
he_status he_ct_import(he_ctx* ctx, const uint64_t* coeff_form, int32_t level,
                       double scale, he_ct** out);
he_status he_ct_info(const he_ct* ct, int32_t* level, double* scale);

/* ---- element-wise operations (section 3; appendix A.2) ---- */
he_status he_add(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct** out);
he_status he_sub(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct** out);
he_status he_negate(he_ctx* ctx, const he_ct* a, he_ct** out);
/* plaintext at the ciphertext's scale, level >= the ciphertext's */
he_status he_add_plain(he_ctx* ctx, const he_ct* a, const he_pt* p, he_ct** out);
/* c0 - p (poly 0 only), the plaintext subtracted */
he_status he_sub_plain(he_ctx* ctx, const he_ct* a, const he_pt* p, he_ct** out);
/* ciphertext x plaintext; scale multiplies; rescales if auto_rescale */
he_status he_mul_plain(he_ctx* ctx, const he_ct* a, const he_pt* p, he_ct** out);
/* tensor product, relinearisation with the s^2 key; rescales if auto_rescale */
he_status he_mul_relin(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct** out);
/* he_mul_relin(a, a) */
he_status he_square(he_ctx* ctx, const he_ct* a, he_ct** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): he_mul_relin
 * writing into the caller's ciphertext `out`, which must belong to ctx and
 * already be at the result's level (min(level a, level b), minus one with
 * auto_rescale).  Every intermediate lives in a fixed device array of
 * HE_NOALLOC_SCRATCH_BYTES per GPU (held until the process ends), not in the
 * context's allocator; the call makes no device allocation.  Its result is
 * bit-identical to he_mul_relin's.  The array is shared by every call on
 * that GPU and keeps the last call's contents (nothing in it needs to start
 * at zero): calls on one GPU whose streams overlap race, so serialise them
 * (one stream, or synchronise between them).  HE_ERANGE when the call would
 * need more scratch than the maximum (at N = 16384: more than 10 limbs);
 * HE_ELEVEL when `out` is not at the result's level; HE_EINVAL for handles
 * of another context. */
#define HE_NOALLOC_SCRATCH_BYTES (48u * 1024u * 1024u)
he_status he_mul_relin_noalloc(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct* out);
/* round(c / q_l) onto limbs 0..l-1; scale / q_l.  HE_ELEVEL at level 0. */
he_status he_rescale(he_ctx* ctx, const he_ct* a, he_ct** out);
/* drop limbs down to `level` (exact) */
he_status he_drop_to(he_ctx* ctx, const he_ct* a, int32_t level, he_ct** out);
/* left rotation of the slots by step: X -> X^(5^step mod 2N) and a key
 * switch with the Galois key of that step (HE_ENOKEY if none). */
he_status he_rotate(he_ctx* ctx, const he_ct* a, int32_t step, he_ct** out);

/* ---- power and polynomial evaluation (section 3: minimum-depth circuits;
 * appendix, table of encrypted operations) ----
 * Every product is relinearised and rescaled (whatever auto_rescale says);
 * operands at different levels are aligned by dropping limbs (exact). */
/* a^k, k >= 1, at multiplicative depth ceil(log2 k): the squares a^(2^i) of
 * the set bits of k, then the two factors of least depth (ties: smaller
 * exponent) multiplied until one is left.  HE_EINVAL for k = 0, HE_ELEVEL
 * when the chain is too short. */
he_status he_power(he_ctx* ctx, const he_ct* a, uint32_t k, he_ct** out);
/* sum_i coeffs[i] a^i (n_coeffs = degree + 1).  Each a^i with i >= 1 and
 * coeffs[i] != 0 comes from the power circuit (squares shared), is
 * multiplied by the constant coeffs[i] encoded at scale Delta*q_l/scale(a^i)
 * at its level l and rescaled, so every term lands at scale Delta; terms are
 * cut to the lowest level, summed in increasing i, and coeffs[0] is added.
 * Depth ceil(log2 d) + 1.  HE_EINVAL when no term has i >= 1. */
he_status he_polyval(he_ctx* ctx, const he_ct* a, const double* coeffs, size_t n_coeffs,
                     he_ct** out);

/* ---- NTT autotuner (the ring products under every section 3 operation;
 * section 2.1's thread pool sizes its work to the machine, this picks the
 * launch form per size) ----
 * Times batched forward + inverse NTTs of J limb-transforms (J = 16, 32, ...
 * up to max_jobs; J limbs are the data limbs of J / L' ciphertext polys at
 * L' limbs) in every candidate form: the two-phase kernels (a limb spread
 * over several workgroups) and one workgroup per limb in each thread
 * layout of he_ntt_layouts (words per thread and pass radix).  From then on
 * each launch of plain transforms runs in the form that won for its size
 * (rounded up to the next J; larger launches follow the largest J), and
 * the fused key-switch transforms use the two-phase form where it won.
 * *split_jobs: the largest J won by the two-phase form (0: none).  The
 * choice changes timing only, never results.
 * table (nullable) receives rows (J, us two-phase, us layout 0, us layout
 * 1, ...) of 2 + layouts doubles each, at most table_cap doubles.
 * Synchronises; not allowed during a capture.  HE_NTT_LAYOUT=k in the
 * environment at context creation forces layout k for every plain
 * one-workgroup launch of that context (a test and tuning aid). */
/* The one-workgroup-per-limb thread layouts of the context's ring degree:
 * log2 words per thread and log2 pass radix of layout i (layout 0 is the
 * default), up to cap of them; *count: how many there are. */
he_status he_ntt_layouts(he_ctx* ctx, int32_t* loge, int32_t* logr, size_t cap, size_t* count);
he_status he_tune_ntt(he_ctx* ctx, int32_t max_jobs, int32_t* split_jobs, double* table,
                      size_t table_cap);

/* ---- captured graphs (a fixed op sequence replayed with one launch: the
 * batch-1 inference of section 5, table 2) ----
 * Everything the library enqueues on the context's stream between
 * he_graph_begin and he_graph_end is captured (HIP stream capture, relaxed
 * mode) into a graph; he_graph_launch replays it.  Ciphertexts created
 * during the capture are the graph's outputs: every replay rewrites them, so
 * free them only after he_graph_free.  Inputs are read at their addresses
 * at replay time: feed new data with he_ct_copy into the captured inputs
 * (same level and scale).  Intermediates freed during the capture stay
 * reserved for the graph until he_graph_free.  Only asynchronous calls may
 * be captured (no decrypt, decode, export, encode, key or plan creation —
 * they synchronise, and the capture then fails at he_graph_end); a plan
 * applied in a capture must have been applied once before.  Profiling is
 * off inside a capture. */
typedef struct he_graph he_graph;
he_status he_graph_begin(he_ctx* ctx);
he_status he_graph_end(he_ctx* ctx, he_graph** out);
he_status he_graph_launch(he_ctx* ctx, const he_graph* g);
void he_graph_free(he_graph* g);
/* dst <- src (device copy; levels must match, dst takes src's scale) */
he_status he_ct_copy(he_ctx* ctx, he_ct* dst, const he_ct* src);

/* ---- batches (the key switch of section 3 applied to many ciphertexts) ----
 * n operations on operands that all sit at one level (HE_ELEVEL otherwise).
 * Up to 32 key switches run in one set of launches, sharing the key reads;
 * every result is bit-identical to the one-at-a-time call.  out[i] is a new
 * ciphertext owned by the caller (he_ct_free); results of one batch share
 * device storage that is released with the last of them.  On error every
 * out[i] is NULL. */
/* out[i] = he_mul_relin(a[i], b[i]) */
he_status he_mul_relin_many(he_ctx* ctx, const he_ct* const* a, const he_ct* const* b,
                            size_t n, he_ct** out);
/* out[i] = he_rotate(a[i], steps[i]) */
he_status he_rotate_many(he_ctx* ctx, const he_ct* const* a, const int32_t* steps,
                         size_t n, he_ct** out);

/* The same batches across contexts: a server holding one context (and key
 * set, section 2.1) per client runs the key switches of several clients'
 * ciphertexts in one set of launches, each item with the keys of its own
 * context.  a[i] (and b[i], of the same context) may belong to any context
 * with the same ring degree, primes and auto_rescale as `run`, on the same
 * device; out[i] belongs to a[i]'s context and equals, bit for bit, what
 * that context's own he_mul_relin / he_rotate gives.  The batch runs on
 * run's stream after the work already queued on every involved context's
 * stream, and each of those streams waits for the batch before its later
 * work (HIP events), so no synchronisation is needed around the call.
 * HE_EINVAL for mismatched contexts, NULL items, or an open graph capture on
 * any involved context. */
he_status he_mul_relin_across(he_ctx* run, const he_ct* const* a, const he_ct* const* b,
                              size_t n, he_ct** out);
he_status he_rotate_across(he_ctx* run, const he_ct* const* a, const int32_t* steps,
                           size_t n, he_ct** out);

/* ---- one work queue over uneven operations (section 2.1's thread pool of
 * independent operations, as device work queues) ---- */
#define HE_QOP_MUL_RELIN 0 /* he_mul_relin(a, b), rescaled if ctx auto_rescale */
#define HE_QOP_ROTATE 1    /* he_rotate(a, step), step != 0 mod N/2          */
typedef struct {
  he_ctx* ctx;     /* the operation's context: its keys, tables and results */
  int32_t kind;    /* HE_QOP_MUL_RELIN or HE_QOP_ROTATE                     */
  const he_ct* a;  /* operand (belongs to ctx)                              */
  const he_ct* b;  /* second factor of a product (same level as a)          */
  int32_t step;    /* left rotation                                         */
} he_qop;
/* Runs n operations of any mix of contexts (ring degrees 2^12..2^14, any
 * levels) on one device as eight launches in all, one per stage of the key
 * switch (tensor; inverse transform of the digits; ModUp; inner products;
 * inverse transform of the special limbs; ModDown; for rescaled products
 * the top limb's inverse transform and the division).  Each launch is a
 * resident grid of 1024-thread workgroups that take limb-sized tasks of all
 * operations from a device queue (an atomic counter) until it is empty,
 * larger rings first.  out[i] is a new ciphertext of ops[i].ctx, bit-
 * identical to that context's own he_mul_relin / he_rotate.  The work runs
 * on run's stream after the work queued on every involved context's stream;
 * the call returns when it is done (it synchronises run's stream).
 * HE_EINVAL for NULL or foreign handles, unsupported ring degrees, a zero
 * rotation, another device or an open capture; HE_ENOKEY, HE_ELEVEL as the
 * single calls; HE_EOOM. */
he_status he_queue_run(he_ctx* run, const he_qop* ops, size_t n, he_ct** out);

/* ---- composites (sections 3.1, 3.2; appendix A.3, A.4) ---- */

/* x <- x + rot(x, 2^j), j < ceil(log2 n): slot 0 gets the sum of slots
 * 0..n-1 (the rotate-and-sum of the dot product). */
he_status he_sum_slots(he_ctx* ctx, const he_ct* a, uint32_t n, he_ct** out);
/* im2col convolution: slot k*windows + w of x holds pixel k of window w
 * (vertical scan).  Multiply by the kernel replicated over the windows
 * (scale Delta), rescale, add ceil(log2 kk) left rotations by windows*2^j,
 * and add `bias` to slots 0..windows-1.  Result in slots 0..windows-1. */
he_status he_enc_conv_im2col(he_ctx* ctx, const he_ct* x, const double* kernel,
                             uint32_t kk, uint32_t windows, double bias,
                             he_ct** out);
/* vector-matrix product y = x W + bias, W row-major n_in x n_out: replicate
 * x (zero beyond n_in) R times, R the largest power of two with
 * n_in * R <= N/2, as x plus its right rotations by n_in * m (m = 1..R-1),
 * then y = sum_i rot_left(x_rep, i) * diag_i with
 * diag_i[j] = W[(i+j) mod n_in][j] (j < n_out), one rescale, bias added.
 * Both sets of rotations (R - 1 of x, n_in - 1 of x_rep) share one digit
 * decomposition each (hoisted); results are identical to rotating one by
 * one.  Needs Galois keys for the steps N/2 - n_in*m and 1..n_in-1. */
he_status he_enc_matmul(he_ctx* ctx, const he_ct* x, const double* W,
                        uint32_t n_in, uint32_t n_out, const double* bias,
                        he_ct** out);
/* mask part c to slots 0..width-1 (ones at Delta), rescale, rotate right by
 * width*c, add: n_parts vectors of `width` packed side by side. */
he_status he_pack(he_ctx* ctx, he_ct* const* parts, uint32_t n_parts,
                  uint32_t width, he_ct** out);

/* Prepared composites: the plaintext operands (replicated kernel, matrix
 * diagonals, biases) are encoded once for inputs at `like`'s level and
 * scale and kept on the device; he_plan_apply then runs the composite with
 * bit-identical results to the one-shot calls above. */
he_status he_conv_plan(he_ctx* ctx, const he_ct* like, const double* kernel,
                       uint32_t kk, uint32_t windows, double bias,
                       he_plan** out);
he_status he_matmul_plan(he_ctx* ctx, const he_ct* like, const double* W,
                         uint32_t n_in, uint32_t n_out, const double* bias,
                         he_plan** out);
/* HE_ELEVEL / HE_ESCALE if x does not match the plan's level and scale. */
he_status he_plan_apply(he_ctx* ctx, const he_plan* plan, const he_ct* x,
                        he_ct** out);
/* n plans on the same input, outs[0..n-1].  Convolution plans that share
 * (kk, windows) run in lock step: their channels' rotations go out as one
 * batched key switch per step (the section 5 network's 4 channels).  Results
 * are identical to n calls of he_plan_apply; on error every outs[i] is NULL. */
he_status he_plan_apply_many(he_ctx* ctx, const he_plan* const* plans,
                             uint32_t n, const he_ct* x, he_ct** outs);

/* ---- raw transforms (batched negacyclic NTT on caller device buffers: the
 * ring arithmetic of the CKKS scheme that section 2 builds on) ---- */
/* data: device pointer to n_polys polynomials of n_limbs limbs, layout
 * [n_polys][n_limbs][N] u64, limb i under data prime i, residues in [0, q_i),
 * 16-byte aligned (HE_EINVAL otherwise).  In place, enqueued on the context
 * stream. */
he_status he_ntt_forward(he_ctx* ctx, uint64_t* data, size_t n_polys,
                         int32_t n_limbs);
he_status he_ntt_inverse(he_ctx* ctx, uint64_t* data, size_t n_polys,
                         int32_t n_limbs);

/* ---- keys for parity checks (section 2.1's secret, relinearisation and
 * Galois keys) ---- */
he_status he_export_secret(he_ctx* ctx, int64_t* s); /* N ternary coeffs */
/* kind 0: relinearisation key, kind 1: Galois key of `step`.  Coefficient
 * form, layout [digit j][poly k][modulus t][N], t = 0..max_level then the
 * special prime; cap in words. */
he_status he_export_key(he_ctx* ctx, int32_t kind, int32_t step,
                        uint64_t* out, size_t cap, int32_t* max_level);

/* ---- tensors of several ciphertexts (section 2: the CKKSTensor flavour,
 * which batches one axis into the slots; the appendix operation tables at
 * vector sizes above N/2) ----
 * A tensor of shape d_0 x ... x d_{r-1} (1 <= r <= HE_TENSOR_MAX_DIMS) keeps
 * its last axis in the slots, in chunks of N/2, and indexes ciphertexts by
 * the other axes: ciphertext i = row * chunks + chunk holds the values
 * row * d_{r-1} + chunk * N/2 + j, j < N/2, of the row-major value array.
 * The tensor owns its ciphertexts; every operation returns a new tensor
 * (he_tensor_free) and applies the one-ciphertext operation above to each
 * ciphertext (products as batches), so each result ciphertext is
 * bit-identical to the one-ciphertext call.  Shapes of the operands must
 * match (HE_EINVAL); level and scale rules are those of the operations. */
typedef struct he_tensor he_tensor;
#define HE_TENSOR_MAX_DIMS 8
/* encode + encrypt values[prod(shape)] (host, row-major) at scale / level;
 * ciphertext i uses enc_index0 + i */
he_status he_tensor_encrypt(he_ctx* ctx, const double* values, const int64_t* shape,
                            int32_t ndim, double scale, int32_t level,
                            uint32_t enc_index0, int32_t use_secret_key, he_tensor** out);
/* decrypt + decode into out[prod(shape)] (host, row-major; n = capacity) */
he_status he_tensor_decrypt(he_ctx* ctx, const he_tensor* t, double* out, size_t n);
/* shape (HE_TENSOR_MAX_DIMS entries of room), rank and ciphertext count */
he_status he_tensor_shape(const he_tensor* t, int64_t* shape, int32_t* ndim, size_t* n_ct);
/* ciphertext i, still owned by the tensor */
he_status he_tensor_ct(const he_tensor* t, size_t i, const he_ct** out);
he_status he_tensor_add(he_ctx* ctx, const he_tensor* a, const he_tensor* b, he_tensor** out);
he_status he_tensor_sub(he_ctx* ctx, const he_tensor* a, const he_tensor* b, he_tensor** out);
he_status he_tensor_negate(he_ctx* ctx, const he_tensor* a, he_tensor** out);
/* element-wise product / square: he_mul_relin_many over all ciphertexts */
he_status he_tensor_mul(he_ctx* ctx, const he_tensor* a, const he_tensor* b, he_tensor** out);
he_status he_tensor_square(he_ctx* ctx, const he_tensor* a, he_tensor** out);
/* plain operand v[prod(shape)] (host), each chunk encoded at its
 * ciphertext's level: at the ciphertext's scale for add/sub, at the
 * context's scale Delta for mul */
he_status he_tensor_add_plain(he_ctx* ctx, const he_tensor* a, const double* v, he_tensor** out);
he_status he_tensor_sub_plain(he_ctx* ctx, const he_tensor* a, const double* v, he_tensor** out);
he_status he_tensor_mul_plain(he_ctx* ctx, const he_tensor* a, const double* v, he_tensor** out);
he_status he_tensor_power(he_ctx* ctx, const he_tensor* a, uint32_t k, he_tensor** out);
he_status he_tensor_polyval(he_ctx* ctx, const he_tensor* a, const double* coeffs,
                            size_t n_coeffs, he_tensor** out);
/* sum over the last axis: each row's chunks added in chunk order, then
 * he_sum_slots over min(d_{r-1}, N/2) slots; result shape [..., 1] */
he_status he_tensor_sum(he_ctx* ctx, const he_tensor* a, he_tensor** out);
/* he_tensor_sum(he_tensor_mul(a, b)) and he_tensor_sum(he_tensor_mul_plain(a, w)) */
he_status he_tensor_dot(he_ctx* ctx, const he_tensor* a, const he_tensor* b, he_tensor** out);
he_status he_tensor_dot_plain(he_ctx* ctx, const he_tensor* a, const double* w, he_tensor** out);
void he_tensor_free(he_tensor* t);

/* ---- housekeeping (section 2.1: the context owns keys and device memory;
 * section 3.2's client-side im2col) ---- */
void he_ct_free(he_ct* ct);
void he_pt_free(he_pt* pt);
void he_plan_free(he_plan* plan);
he_status he_sync(he_ctx* ctx);
/* message of the calling thread's last failure ("" if none) */
const char* he_last_error(void);
size_t he_ct_bytes(const he_ct* ct);    /* device bytes held by a ciphertext */
size_t he_key_bytes(const he_ctx* ctx); /* device bytes held by all keys    */
/* plain im2col (client side, section 3.2): out[(ky*k + kx)*windows + w] =
 * img[(oy*stride + ky)*w_img + ox*stride + kx], w = oy*ow + ox. */
void he_im2col(const double* img, uint32_t h, uint32_t w, uint32_t k,
               uint32_t stride, double* out);

/* ---- kernel timing: HIP events around each launch of a named kernel
 * family while enabled (adds no work to the kernels themselves; the
 * per-stage times of section 5, table 2). ---- */
he_status he_profile_enable(he_ctx* ctx, int32_t enable);
/* launches, summed milliseconds, summed work units (limb-NTTs for the NTT
 * families, items for the inner products) and summed algorithmic HBM bytes
 * of a kernel family since enabling (synchronises).  Families: "ntt_fwd",
 * "ntt_inv", "modup", "moddown", "rescale", "keyswitch_inner",
 * "hoisted_inner", "hoisted_cols", "hoisted_moddown", "hoisted_replication",
 * "pointwise", "sample". */
he_status he_profile_read(he_ctx* ctx, const char* family, uint64_t* launches,
                          double* total_ms, double* units, double* bytes);

#ifdef __cplusplus
}
#endif
#endif
