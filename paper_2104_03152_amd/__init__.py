"""Python binding of libckks_hip.so (include/ckks_hip.h): the same names as
the C ABI, argument marshalling only.  Every step of every operation runs in
the HIP library; there is no fallback: if the library is not built, loading
raises.  Build it with `python -m paper_2104_03152_amd.build`.

PyTorch is used for plumbing only: device memory comes from torch's caching
allocator (through the he_alloc_fn / he_free_fn callbacks, on the context's
stream), the context enqueues on a torch stream, and raw device buffers for
he_ntt_* may be torch tensors."""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libckks_hip.so")

HE_OK, HE_EINVAL, HE_ERANGE, HE_ELEVEL, HE_ESCALE, HE_ENOKEY, HE_EOOM, HE_EHIP = (
    0, -1, -2, -3, -4, -5, -6, -7)
HE_MAX_PRIMES = 32
HE_TENSOR_MAX_DIMS = 8


class HeError(RuntimeError):
    def __init__(self, code, where):
        msg = lib().he_last_error().decode(errors="replace")
        super().__init__("%s: code %d: %s" % (where, code, msg))
        self.code = code


class he_params(C.Structure):
    _fields_ = [("log_n", C.c_int32), ("n_primes", C.c_int32),
                ("prime_bits", C.c_int32 * HE_MAX_PRIMES), ("scale", C.c_double),
                ("auto_rescale", C.c_int32), ("seed", C.c_uint64)]


_P = C.POINTER
_vp = C.c_void_p
_pvp = _P(C.c_void_p)
_u64p = _P(C.c_uint64)
_i64p = _P(C.c_int64)
_dp = _P(C.c_double)
_i32p = _P(C.c_int32)

_SIGS = {
    "he_ctx_create": (C.c_int32, [_P(he_params), _vp, _vp, _vp, _vp, _pvp]),
    "he_ctx_destroy": (None, [_vp]),
    "he_ctx_info": (C.c_int32, [_vp, _i32p, _i32p, _u64p]),
    "he_keygen": (C.c_int32, [_vp, _i32p, C.c_size_t]),
    "he_keygen_galois": (C.c_int32, [_vp, C.c_int32, C.c_int32]),
    "he_encode": (C.c_int32, [_vp, _dp, C.c_size_t, C.c_double, C.c_int32, _pvp]),
    "he_decode": (C.c_int32, [_vp, _vp, _dp, C.c_size_t]),
    "he_pt_import": (C.c_int32, [_vp, _i64p, C.c_double, C.c_int32, _pvp]),
    "he_pt_export": (C.c_int32, [_vp, _vp, _u64p, C.c_size_t, _i32p, _dp]),
    "he_encrypt": (C.c_int32, [_vp, _vp, C.c_uint32, C.c_int32, _pvp]),
    "he_decrypt": (C.c_int32, [_vp, _vp, _pvp]),
    "he_ct_export": (C.c_int32, [_vp, _vp, _u64p, C.c_size_t, _i32p, _dp]),
    "he_ct_import": (C.c_int32, [_vp, _u64p, C.c_int32, C.c_double, _pvp]),
    "he_ct_info": (C.c_int32, [_vp, _i32p, _dp]),
    "he_add": (C.c_int32, [_vp, _vp, _vp, _pvp]),
    "he_sub": (C.c_int32, [_vp, _vp, _vp, _pvp]),
    "he_negate": (C.c_int32, [_vp, _vp, _pvp]),
    "he_add_plain": (C.c_int32, [_vp, _vp, _vp, _pvp]),
    "he_mul_plain": (C.c_int32, [_vp, _vp, _vp, _pvp]),
    "he_sub_plain": (C.c_int32, [_vp, _vp, _vp, _pvp]),
    "he_power": (C.c_int32, [_vp, _vp, C.c_uint32, _pvp]),
    "he_polyval": (C.c_int32, [_vp, _vp, _dp, C.c_size_t, _pvp]),
    "he_mul_relin": (C.c_int32, [_vp, _vp, _vp, _pvp]),
    "he_square": (C.c_int32, [_vp, _vp, _pvp]),
    "he_mul_relin_noalloc": (C.c_int32, [_vp, _vp, _vp, _vp]),
    "he_rescale": (C.c_int32, [_vp, _vp, _pvp]),
    "he_drop_to": (C.c_int32, [_vp, _vp, C.c_int32, _pvp]),
    "he_rotate": (C.c_int32, [_vp, _vp, C.c_int32, _pvp]),
    "he_mul_relin_many": (C.c_int32, [_vp, _pvp, _pvp, C.c_size_t, _pvp]),
    "he_tune_ntt": (C.c_int32, [_vp, C.c_int32, _i32p, _dp, C.c_size_t]),
    "he_graph_begin": (C.c_int32, [_vp]),
    "he_graph_end": (C.c_int32, [_vp, _pvp]),
    "he_graph_launch": (C.c_int32, [_vp, _vp]),
    "he_graph_free": (None, [_vp]),
    "he_ct_copy": (C.c_int32, [_vp, _vp, _vp]),
    "he_rotate_many": (C.c_int32, [_vp, _pvp, _i32p, C.c_size_t, _pvp]),
    "he_queue_run": (C.c_int32, [_vp, _vp, C.c_size_t, _pvp]),
    "he_ntt_layouts": (C.c_int32, [_vp, _i32p, _i32p, C.c_size_t, C.POINTER(C.c_size_t)]),
    "he_mul_relin_across": (C.c_int32, [_vp, _pvp, _pvp, C.c_size_t, _pvp]),
    "he_rotate_across": (C.c_int32, [_vp, _pvp, _i32p, C.c_size_t, _pvp]),
    "he_sum_slots": (C.c_int32, [_vp, _vp, C.c_uint32, _pvp]),
    "he_enc_conv_im2col": (C.c_int32, [_vp, _vp, _dp, C.c_uint32, C.c_uint32, C.c_double, _pvp]),
    "he_enc_matmul": (C.c_int32, [_vp, _vp, _dp, C.c_uint32, C.c_uint32, _dp, _pvp]),
    "he_pack": (C.c_int32, [_vp, _pvp, C.c_uint32, C.c_uint32, _pvp]),
    "he_conv_plan": (C.c_int32, [_vp, _vp, _dp, C.c_uint32, C.c_uint32, C.c_double, _pvp]),
    "he_matmul_plan": (C.c_int32, [_vp, _vp, _dp, C.c_uint32, C.c_uint32, _dp, _pvp]),
    "he_plan_apply": (C.c_int32, [_vp, _vp, _vp, _pvp]),
    "he_plan_apply_many": (C.c_int32, [_vp, _pvp, C.c_uint32, _vp, _pvp]),
    "he_ntt_forward": (C.c_int32, [_vp, _vp, C.c_size_t, C.c_int32]),
    "he_ntt_inverse": (C.c_int32, [_vp, _vp, C.c_size_t, C.c_int32]),
    "he_export_secret": (C.c_int32, [_vp, _i64p]),
    "he_export_key": (C.c_int32, [_vp, C.c_int32, C.c_int32, _u64p, C.c_size_t, _i32p]),
    "he_ct_free": (None, [_vp]),
    "he_pt_free": (None, [_vp]),
    "he_plan_free": (None, [_vp]),
    "he_tensor_encrypt": (C.c_int32, [_vp, _dp, _i64p, C.c_int32, C.c_double, C.c_int32, C.c_uint32,
                                      C.c_int32, _pvp]),
    "he_tensor_decrypt": (C.c_int32, [_vp, _vp, _dp, C.c_size_t]),
    "he_tensor_shape": (C.c_int32, [_vp, _i64p, _i32p, _P(C.c_size_t)]),
    "he_tensor_ct": (C.c_int32, [_vp, C.c_size_t, _pvp]),
    "he_tensor_add": (C.c_int32, [_vp, _vp, _vp, _pvp]),
    "he_tensor_sub": (C.c_int32, [_vp, _vp, _vp, _pvp]),
    "he_tensor_mul": (C.c_int32, [_vp, _vp, _vp, _pvp]),
    "he_tensor_dot": (C.c_int32, [_vp, _vp, _vp, _pvp]),
    "he_tensor_negate": (C.c_int32, [_vp, _vp, _pvp]),
    "he_tensor_square": (C.c_int32, [_vp, _vp, _pvp]),
    "he_tensor_sum": (C.c_int32, [_vp, _vp, _pvp]),
    "he_tensor_add_plain": (C.c_int32, [_vp, _vp, _dp, _pvp]),
    "he_tensor_sub_plain": (C.c_int32, [_vp, _vp, _dp, _pvp]),
    "he_tensor_mul_plain": (C.c_int32, [_vp, _vp, _dp, _pvp]),
    "he_tensor_dot_plain": (C.c_int32, [_vp, _vp, _dp, _pvp]),
    "he_tensor_power": (C.c_int32, [_vp, _vp, C.c_uint32, _pvp]),
    "he_tensor_polyval": (C.c_int32, [_vp, _vp, _dp, C.c_size_t, _pvp]),
    "he_tensor_free": (None, [_vp]),
    "he_sync": (C.c_int32, [_vp]),
    "he_last_error": (C.c_char_p, []),
    "he_ct_bytes": (C.c_size_t, [_vp]),
    "he_key_bytes": (C.c_size_t, [_vp]),
    "he_im2col": (None, [_dp, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, _dp]),
    "he_profile_enable": (C.c_int32, [_vp, C.c_int32]),
    "he_profile_read": (C.c_int32, [_vp, C.c_char_p, _u64p, _dp, _dp, _dp]),
}

_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError("libckks_hip.so is not built (python -m paper_2104_03152_amd.build); "
                               "there is no non-HIP implementation")
        L = C.CDLL(LIBPATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _chk(rc, where):
    if rc != HE_OK:
        raise HeError(rc, where)


def _ptr(a, ct):
    return a.ctypes.data_as(_P(ct))


class _Handle:
    _free = None

    def __init__(self, ctx, ptr):
        self.ctx, self.ptr = ctx, ptr

    def free(self):
        if self.ptr:
            # a handle that outlives its context is only dropped: the
            # context's destruction released its device memory
            if self.ctx is None or getattr(self.ctx, "ptr", None):
                getattr(lib(), self._free)(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Ct(_Handle):
    _free = "he_ct_free"

    def info(self):
        lv, sc = C.c_int32(), C.c_double()
        _chk(lib().he_ct_info(self.ptr, C.byref(lv), C.byref(sc)), "he_ct_info")
        return lv.value, sc.value

    @property
    def level(self):
        return self.info()[0]

    @property
    def scale(self):
        return self.info()[1]


class Pt(_Handle):
    _free = "he_pt_free"


class Plan(_Handle):
    _free = "he_plan_free"


class _BorrowedCt(Ct):
    """A ciphertext owned by a tensor (kept alive through `owner`)."""

    def __init__(self, ctx, ptr, owner):
        super().__init__(ctx, ptr)
        self.owner = owner

    def free(self):
        self.ptr = None


class Tensor(_Handle):
    """Tensor of several ciphertexts, last axis in the slots (he_tensor_*)."""
    _free = "he_tensor_free"

    def _info(self):
        shape = (C.c_int64 * HE_TENSOR_MAX_DIMS)()
        nd, nct = C.c_int32(), C.c_size_t()
        _chk(lib().he_tensor_shape(self.ptr, shape, C.byref(nd), C.byref(nct)), "he_tensor_shape")
        return tuple(int(shape[i]) for i in range(nd.value)), nct.value

    @property
    def shape(self):
        return self._info()[0]

    @property
    def n_ct(self):
        return self._info()[1]

    def ct(self, i):
        out = C.c_void_p()
        _chk(lib().he_tensor_ct(self.ptr, int(i), C.byref(out)), "he_tensor_ct")
        return _BorrowedCt(self.ctx, out.value, self)


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_size_t, C.c_void_p)


class Allocator:
    """Device-memory callbacks for he_ctx_create.  alloc(nbytes) returns a
    device address (int) or None; free(ptr, nbytes) releases it.  A failing
    alloc makes the library return HE_EOOM."""

    def __init__(self, alloc, free):
        self._alloc, self._free = alloc, free

        def a(nbytes, user):
            try:
                return self._alloc(int(nbytes))
            except Exception:  # out of memory: the library reports HE_EOOM
                return None

        def f(ptr, nbytes, user):
            try:
                self._free(ptr, int(nbytes))
            except Exception:
                pass

        self.c_alloc, self.c_free = _ALLOC_FN(a), _FREE_FN(f)


def torch_allocator(stream_handle, device=None):
    """torch's caching allocator, blocks associated with the given stream (the
    context's): torch reuses a freed block only for work on that stream."""
    import torch
    dev = torch.cuda.current_device() if device is None else device
    return Allocator(lambda n: torch.cuda.caching_allocator_alloc(n, dev, stream_handle),
                     lambda ptr, n: torch.cuda.caching_allocator_delete(ptr))


class Ctx:
    def __init__(self, ptr, keep=()):
        self.ptr = ptr
        self._keep = keep  # callbacks and the stream object outlive the context
        lg, L = C.c_int32(), C.c_int32()
        primes = (C.c_uint64 * (HE_MAX_PRIMES + 1))()
        _chk(lib().he_ctx_info(ptr, C.byref(lg), C.byref(L), primes), "he_ctx_info")
        self.log_n, self.L = lg.value, L.value
        self.n = 1 << self.log_n
        self.primes = [int(primes[i]) for i in range(self.L + 1)]

    def close(self):
        if self.ptr:
            lib().he_ctx_destroy(self.ptr)
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def he_ctx_create(log_n, prime_bits, scale, seed, auto_rescale=True, stream="torch", allocator="torch"):
    """stream: "torch" (torch's current stream, or a new torch stream when
    that is the null stream), None (a new torch stream when the allocator is
    torch's, else one the library creates) or a raw hipStream_t.
    allocator: "torch" (torch's caching allocator on the context's stream),
    None (the library's pool over hipMalloc) or an Allocator."""
    p = he_params()
    p.log_n = log_n
    p.n_primes = len(prime_bits)
    for i, b in enumerate(prime_bits):
        p.prime_bits[i] = b
    p.scale = float(scale)
    p.auto_rescale = 1 if auto_rescale else 0
    p.seed = seed
    keep = []
    st = stream
    if stream == "torch" or (stream is None and allocator == "torch"):
        import torch
        ts = torch.cuda.current_stream() if stream == "torch" else None
        if ts is None or ts.cuda_stream == 0:
            ts = torch.cuda.Stream()  # default priority
        keep.append(ts)
        st = ts.cuda_stream
    if isinstance(st, C.c_void_p):
        st = st.value
    if allocator == "torch":
        allocator = torch_allocator(st or 0)
    if allocator is not None:
        keep.append(allocator)
        fa, ff = allocator.c_alloc, allocator.c_free
    else:
        fa = ff = None
    out = C.c_void_p()
    _chk(lib().he_ctx_create(C.byref(p), fa, ff, None, C.c_void_p(st) if st else None, C.byref(out)),
         "he_ctx_create")
    return Ctx(out.value, tuple(keep))


def he_ctx_destroy(ctx):
    ctx.close()


def he_keygen(ctx, steps=()):
    arr = (C.c_int32 * max(1, len(steps)))(*[int(s) for s in steps])
    _chk(lib().he_keygen(ctx.ptr, arr, len(steps)), "he_keygen")


def he_keygen_galois(ctx, step, max_level=-1):
    _chk(lib().he_keygen_galois(ctx.ptr, int(step), int(max_level)), "he_keygen_galois")


def _new(cls, ctx, fn, where, *args):
    out = C.c_void_p()
    _chk(fn(*args, C.byref(out)), where)
    return cls(ctx, out.value)


def he_encode(ctx, v, scale, level):
    v = np.ascontiguousarray(v, dtype=np.float64)
    return _new(Pt, ctx, lib().he_encode, "he_encode", ctx.ptr, _ptr(v, C.c_double), v.size,
                float(scale), int(level))


def he_decode(ctx, pt, n):
    out = np.zeros(n, dtype=np.float64)
    _chk(lib().he_decode(ctx.ptr, pt.ptr, _ptr(out, C.c_double), n), "he_decode")
    return out


def he_pt_import(ctx, coeffs, scale, level):
    c = np.ascontiguousarray(coeffs, dtype=np.int64)
    return _new(Pt, ctx, lib().he_pt_import, "he_pt_import", ctx.ptr, _ptr(c, C.c_int64),
                float(scale), int(level))


def he_pt_export(ctx, pt, level_hint=None):
    cap = (ctx.L) * ctx.n
    buf = np.zeros(cap, dtype=np.uint64)
    lv, sc = C.c_int32(), C.c_double()
    _chk(lib().he_pt_export(ctx.ptr, pt.ptr, _ptr(buf, C.c_uint64), cap, C.byref(lv), C.byref(sc)),
         "he_pt_export")
    return buf[:(lv.value + 1) * ctx.n].reshape(lv.value + 1, ctx.n), lv.value, sc.value


def he_encrypt(ctx, pt, enc_index=0, use_secret_key=False):
    return _new(Ct, ctx, lib().he_encrypt, "he_encrypt", ctx.ptr, pt.ptr, int(enc_index),
                1 if use_secret_key else 0)


def he_decrypt(ctx, ct):
    return _new(Pt, ctx, lib().he_decrypt, "he_decrypt", ctx.ptr, ct.ptr)


def he_ct_export(ctx, ct):
    cap = 2 * ctx.L * ctx.n
    buf = np.zeros(cap, dtype=np.uint64)
    lv, sc = C.c_int32(), C.c_double()
    _chk(lib().he_ct_export(ctx.ptr, ct.ptr, _ptr(buf, C.c_uint64), cap, C.byref(lv), C.byref(sc)),
         "he_ct_export")
    return buf[:2 * (lv.value + 1) * ctx.n].reshape(2, lv.value + 1, ctx.n)


def he_ct_import(ctx, data, level, scale):
    d = np.ascontiguousarray(data, dtype=np.uint64).reshape(-1)
    return _new(Ct, ctx, lib().he_ct_import, "he_ct_import", ctx.ptr, _ptr(d, C.c_uint64),
                int(level), float(scale))


def _binary(name):
    def f(ctx, a, b):
        return _new(Ct, ctx, getattr(lib(), name), name, ctx.ptr, a.ptr, b.ptr)
    f.__name__ = name
    return f


def _unary(name):
    def f(ctx, a):
        return _new(Ct, ctx, getattr(lib(), name), name, ctx.ptr, a.ptr)
    f.__name__ = name
    return f


he_add = _binary("he_add")
he_sub = _binary("he_sub")
he_add_plain = _binary("he_add_plain")
he_mul_plain = _binary("he_mul_plain")
he_sub_plain = _binary("he_sub_plain")
he_mul_relin = _binary("he_mul_relin")
he_negate = _unary("he_negate")
he_square = _unary("he_square")
he_rescale = _unary("he_rescale")


def he_drop_to(ctx, a, level):
    return _new(Ct, ctx, lib().he_drop_to, "he_drop_to", ctx.ptr, a.ptr, int(level))


def he_rotate(ctx, a, step):
    return _new(Ct, ctx, lib().he_rotate, "he_rotate", ctx.ptr, a.ptr, int(step))


def he_power(ctx, a, k):
    return _new(Ct, ctx, lib().he_power, "he_power", ctx.ptr, a.ptr, int(k))


def he_polyval(ctx, a, coeffs):
    cs = np.ascontiguousarray(coeffs, dtype=np.float64)
    return _new(Ct, ctx, lib().he_polyval, "he_polyval", ctx.ptr, a.ptr, _ptr(cs, C.c_double), cs.size)


def he_ntt_layouts(ctx):
    """[(log2 words per thread, log2 pass radix)] of the one-workgroup layouts."""
    e, r = (C.c_int32 * 8)(), (C.c_int32 * 8)()
    cnt = C.c_size_t()
    _chk(lib().he_ntt_layouts(ctx.ptr, e, r, 8, C.byref(cnt)), "he_ntt_layouts")
    return [(e[i], r[i]) for i in range(min(8, cnt.value))]


def he_tune_ntt(ctx, max_jobs=1024):
    """Returns (split_jobs chosen, rows of (J, us two-phase, us layout 0,
    us layout 1, ...)) for forward + inverse pairs."""
    chosen = C.c_int32()
    width = 2 + len(he_ntt_layouts(ctx))
    cap = width * 16
    table = np.zeros(cap, dtype=np.float64)
    _chk(lib().he_tune_ntt(ctx.ptr, int(max_jobs), C.byref(chosen), _ptr(table, C.c_double), cap),
         "he_tune_ntt")
    rows = [tuple(table[i:i + width]) for i in range(0, cap, width) if table[i] > 0]
    return chosen.value, rows


class Graph(_Handle):
    _free = "he_graph_free"


def he_graph_begin(ctx):
    _chk(lib().he_graph_begin(ctx.ptr), "he_graph_begin")


def he_graph_end(ctx):
    return _new(Graph, ctx, lib().he_graph_end, "he_graph_end", ctx.ptr)


def he_graph_launch(ctx, g):
    _chk(lib().he_graph_launch(ctx.ptr, g.ptr), "he_graph_launch")


def he_ct_copy(ctx, dst, src):
    _chk(lib().he_ct_copy(ctx.ptr, dst.ptr, src.ptr), "he_ct_copy")


def he_mul_relin_noalloc(ctx, a, b, out):
    """he_mul_relin into the existing ciphertext `out` (at the result's level),
    every intermediate in the library's fixed device scratch."""
    _chk(lib().he_mul_relin_noalloc(ctx.ptr, a.ptr, b.ptr, out.ptr), "he_mul_relin_noalloc")


def he_mul_relin_many(ctx, a, b):
    """[he_mul_relin(x, y) for x, y in zip(a, b)] as one batch."""
    n = len(a)
    if len(b) != n:
        raise ValueError("operand lists differ in length")
    pa = (C.c_void_p * n)(*[x.ptr for x in a])
    pb = (C.c_void_p * n)(*[x.ptr for x in b])
    outs = (C.c_void_p * n)()
    _chk(lib().he_mul_relin_many(ctx.ptr, pa, pb, n, outs), "he_mul_relin_many")
    return [Ct(ctx, outs[i]) for i in range(n)]


def he_rotate_many(ctx, a, steps):
    """[he_rotate(x, s) for x, s in zip(a, steps)] as one batch."""
    n = len(a)
    st = np.ascontiguousarray(steps, dtype=np.int32)
    if st.size != n:
        raise ValueError("one step per ciphertext")
    pa = (C.c_void_p * n)(*[x.ptr for x in a])
    outs = (C.c_void_p * n)()
    _chk(lib().he_rotate_many(ctx.ptr, pa, _ptr(st, C.c_int32), n, outs), "he_rotate_many")
    return [Ct(ctx, outs[i]) for i in range(n)]


def he_mul_relin_across(run, a, b):
    """he_mul_relin_many over ciphertexts of several compatible contexts, run
    on `run`'s stream; each result belongs to its input's context."""
    n = len(a)
    if len(b) != n:
        raise ValueError("operand lists differ in length")
    pa = (C.c_void_p * n)(*[x.ptr for x in a])
    pb = (C.c_void_p * n)(*[x.ptr for x in b])
    outs = (C.c_void_p * n)()
    _chk(lib().he_mul_relin_across(run.ptr, pa, pb, n, outs), "he_mul_relin_across")
    return [Ct(a[i].ctx, outs[i]) for i in range(n)]


def he_rotate_across(run, a, steps):
    """he_rotate_many over ciphertexts of several compatible contexts."""
    n = len(a)
    st = np.ascontiguousarray(steps, dtype=np.int32)
    if st.size != n:
        raise ValueError("one step per ciphertext")
    pa = (C.c_void_p * n)(*[x.ptr for x in a])
    outs = (C.c_void_p * n)()
    _chk(lib().he_rotate_across(run.ptr, pa, _ptr(st, C.c_int32), n, outs), "he_rotate_across")
    return [Ct(a[i].ctx, outs[i]) for i in range(n)]


HE_QOP_MUL_RELIN, HE_QOP_ROTATE = 0, 1


class he_qop(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("kind", C.c_int32), ("a", C.c_void_p), ("b", C.c_void_p),
                ("step", C.c_int32)]


def he_queue_run(run, ops):
    """ops: (ctx, "mul", a, b) or (ctx, "rotate", a, step) tuples, any mix of
    contexts, ring degrees and levels, run as one set of work-queue launches
    on `run`'s stream; returns one new ciphertext per operation, in its
    context."""
    n = len(ops)
    arr = (he_qop * max(1, n))()
    for i, op in enumerate(ops):
        ctx, kind, a, x = op
        arr[i].ctx, arr[i].a = ctx.ptr, a.ptr
        if kind == "mul":
            arr[i].kind, arr[i].b, arr[i].step = HE_QOP_MUL_RELIN, x.ptr, 0
        elif kind == "rotate":
            arr[i].kind, arr[i].b, arr[i].step = HE_QOP_ROTATE, None, int(x)
        else:
            raise ValueError("unknown operation kind %r" % (kind,))
    outs = (C.c_void_p * max(1, n))()
    _chk(lib().he_queue_run(run.ptr, arr, n, outs), "he_queue_run")
    return [Ct(ops[i][0], outs[i]) for i in range(n)]


def he_sum_slots(ctx, a, n):
    return _new(Ct, ctx, lib().he_sum_slots, "he_sum_slots", ctx.ptr, a.ptr, int(n))


def he_enc_conv_im2col(ctx, x, kernel, windows, bias):
    k = np.ascontiguousarray(kernel, dtype=np.float64)
    return _new(Ct, ctx, lib().he_enc_conv_im2col, "he_enc_conv_im2col", ctx.ptr, x.ptr,
                _ptr(k, C.c_double), k.size, int(windows), float(bias))


def he_enc_matmul(ctx, x, W, bias=None):
    W = np.ascontiguousarray(W, dtype=np.float64)
    b = None if bias is None else np.ascontiguousarray(bias, dtype=np.float64)
    return _new(Ct, ctx, lib().he_enc_matmul, "he_enc_matmul", ctx.ptr, x.ptr, _ptr(W, C.c_double),
                W.shape[0], W.shape[1], None if b is None else _ptr(b, C.c_double))


def he_pack(ctx, parts, width):
    arr = (C.c_void_p * len(parts))(*[p.ptr for p in parts])
    return _new(Ct, ctx, lib().he_pack, "he_pack", ctx.ptr, arr, len(parts), int(width))


def he_conv_plan(ctx, like, kernel, windows, bias):
    k = np.ascontiguousarray(kernel, dtype=np.float64)
    return _new(Plan, ctx, lib().he_conv_plan, "he_conv_plan", ctx.ptr, like.ptr,
                _ptr(k, C.c_double), k.size, int(windows), float(bias))


def he_matmul_plan(ctx, like, W, bias=None):
    W = np.ascontiguousarray(W, dtype=np.float64)
    b = None if bias is None else np.ascontiguousarray(bias, dtype=np.float64)
    return _new(Plan, ctx, lib().he_matmul_plan, "he_matmul_plan", ctx.ptr, like.ptr,
                _ptr(W, C.c_double), W.shape[0], W.shape[1],
                None if b is None else _ptr(b, C.c_double))


def he_plan_apply(ctx, plan, x):
    return _new(Ct, ctx, lib().he_plan_apply, "he_plan_apply", ctx.ptr, plan.ptr, x.ptr)


def he_plan_apply_many(ctx, plans, x):
    n = len(plans)
    arr = (C.c_void_p * n)(*[p.ptr for p in plans])
    outs = (C.c_void_p * n)()
    _chk(lib().he_plan_apply_many(ctx.ptr, arr, n, x.ptr, outs), "he_plan_apply_many")
    return [Ct(ctx, outs[i]) for i in range(n)]


def he_ntt_forward(ctx, dev_ptr, n_polys, n_limbs):
    _chk(lib().he_ntt_forward(ctx.ptr, C.c_void_p(int(dev_ptr)), n_polys, n_limbs), "he_ntt_forward")


def he_ntt_inverse(ctx, dev_ptr, n_polys, n_limbs):
    _chk(lib().he_ntt_inverse(ctx.ptr, C.c_void_p(int(dev_ptr)), n_polys, n_limbs), "he_ntt_inverse")


def he_export_secret(ctx):
    s = np.zeros(ctx.n, dtype=np.int64)
    _chk(lib().he_export_secret(ctx.ptr, _ptr(s, C.c_int64)), "he_export_secret")
    return s


def he_export_key(ctx, kind, step=0):
    L = ctx.L
    cap = L * 2 * (L + 1) * ctx.n
    buf = np.zeros(cap, dtype=np.uint64)
    ml = C.c_int32()
    _chk(lib().he_export_key(ctx.ptr, int(kind), int(step), _ptr(buf, C.c_uint64), cap, C.byref(ml)),
         "he_export_key")
    m = ml.value
    return buf[:(m + 1) * 2 * (m + 2) * ctx.n].reshape(m + 1, 2, m + 2, ctx.n)


def he_sync(ctx):
    _chk(lib().he_sync(ctx.ptr), "he_sync")


def he_last_error():
    return lib().he_last_error().decode(errors="replace")


def he_ct_bytes(ct):
    return lib().he_ct_bytes(ct.ptr)


def he_key_bytes(ctx):
    return lib().he_key_bytes(ctx.ptr)


def he_im2col(img, k, stride):
    img = np.ascontiguousarray(img, dtype=np.float64)
    h, w = img.shape
    oh, ow = (h - k) // stride + 1, (w - k) // stride + 1
    out = np.zeros(k * k * oh * ow, dtype=np.float64)
    lib().he_im2col(_ptr(img, C.c_double), h, w, k, stride, _ptr(out, C.c_double))
    return out


def he_profile_enable(ctx, enable=True):
    _chk(lib().he_profile_enable(ctx.ptr, 1 if enable else 0), "he_profile_enable")


def he_profile_read(ctx, family):
    """(launches, total ms, work units, algorithmic HBM bytes) of a family"""
    n, ms, units, by = C.c_uint64(), C.c_double(), C.c_double(), C.c_double()
    _chk(lib().he_profile_read(ctx.ptr, family.encode(), C.byref(n), C.byref(ms), C.byref(units),
                               C.byref(by)), "he_profile_read")
    return n.value, ms.value, units.value, by.value


# ---- tensors of several ciphertexts (he_tensor_*) ----

def he_tensor_encrypt(ctx, values, scale, level, enc_index0=0, use_sk=False):
    v = np.ascontiguousarray(values, dtype=np.float64)
    if v.ndim == 0:
        v = v.reshape(1)
    shape = np.asarray(v.shape, dtype=np.int64)
    return _new(Tensor, ctx, lib().he_tensor_encrypt, "he_tensor_encrypt", ctx.ptr, _ptr(v, C.c_double),
                _ptr(shape, C.c_int64), v.ndim, float(scale), int(level), int(enc_index0),
                1 if use_sk else 0)


def he_tensor_decrypt(ctx, t):
    shape = t.shape
    out = np.empty(int(np.prod(shape)), dtype=np.float64)
    _chk(lib().he_tensor_decrypt(ctx.ptr, t.ptr, _ptr(out, C.c_double), out.size), "he_tensor_decrypt")
    return out.reshape(shape)


def _tensor_binary(name):
    def f(ctx, a, b):
        return _new(Tensor, ctx, getattr(lib(), name), name, ctx.ptr, a.ptr, b.ptr)
    f.__name__ = name
    return f


def _tensor_unary(name):
    def f(ctx, a):
        return _new(Tensor, ctx, getattr(lib(), name), name, ctx.ptr, a.ptr)
    f.__name__ = name
    return f


def _tensor_plain(name):
    def f(ctx, a, values):
        v = np.ascontiguousarray(values, dtype=np.float64).reshape(-1)
        if v.size != int(np.prod(a.shape)):
            raise ValueError("plain operand has %d values, tensor %d" % (v.size, int(np.prod(a.shape))))
        return _new(Tensor, ctx, getattr(lib(), name), name, ctx.ptr, a.ptr, _ptr(v, C.c_double))
    f.__name__ = name
    return f


he_tensor_add = _tensor_binary("he_tensor_add")
he_tensor_sub = _tensor_binary("he_tensor_sub")
he_tensor_mul = _tensor_binary("he_tensor_mul")
he_tensor_dot = _tensor_binary("he_tensor_dot")
he_tensor_negate = _tensor_unary("he_tensor_negate")
he_tensor_square = _tensor_unary("he_tensor_square")
he_tensor_sum = _tensor_unary("he_tensor_sum")
he_tensor_add_plain = _tensor_plain("he_tensor_add_plain")
he_tensor_sub_plain = _tensor_plain("he_tensor_sub_plain")
he_tensor_mul_plain = _tensor_plain("he_tensor_mul_plain")
he_tensor_dot_plain = _tensor_plain("he_tensor_dot_plain")


def he_tensor_power(ctx, a, k):
    return _new(Tensor, ctx, lib().he_tensor_power, "he_tensor_power", ctx.ptr, a.ptr, int(k))


def he_tensor_polyval(ctx, a, coeffs):
    cf = np.ascontiguousarray(coeffs, dtype=np.float64)
    return _new(Tensor, ctx, lib().he_tensor_polyval, "he_tensor_polyval", ctx.ptr, a.ptr,
                _ptr(cf, C.c_double), cf.size)
