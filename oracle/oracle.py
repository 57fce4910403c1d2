"""ctypes wrapper over the plain C CKKS oracle (oracle/ckks_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py.  The product library never imports this module.
"""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ckks_oracle.c")
LIB = os.path.join(HERE, "libckks_oracle.so")

ORC_OK, ORC_EINVAL, ORC_ERANGE, ORC_ELEVEL, ORC_ESCALE, ORC_ENOKEY, ORC_ENOMEM = (
    0, -1, -2, -3, -4, -5, -6)


def build(force=False):
    """Compile the oracle with gcc (plain -O2, single thread)."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "ckks_oracle.h"))):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-fPIC", "-shared",
                           "-o", tmp, SRC, "-lquadmath", "-lm"])
    os.replace(tmp, LIB)
    return LIB


class _Ct(C.Structure):
    _fields_ = [("level", C.c_int), ("scale", C.c_double), ("data", C.POINTER(C.c_uint64))]


_P = C.POINTER
_u64p = _P(C.c_uint64)
_i64p = _P(C.c_int64)
_dp = _P(C.c_double)
_ctp = _P(_Ct)

_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    L = C.CDLL(build())
    sig = {
        "orc_last_error": (C.c_int, []),
        "orc_chacha20_block": (None, [_P(C.c_uint32), C.c_uint32, _P(C.c_uint32), _P(C.c_uint32)]),
        "orc_stream_words": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_size_t, _u64p]),
        "orc_is_prime": (C.c_int, [C.c_uint64]),
        "orc_gen_primes": (C.c_int, [C.c_int, _P(C.c_int), C.c_int, _u64p]),
        "orc_cdt_table": (_u64p, []),
        "orc_sample_ternary": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_int, _i64p]),
        "orc_sample_gaussian": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_int, _i64p]),
        "orc_sample_uniform": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64,
                                      C.c_int, _u64p]),
        "orc_negacyclic_mul": (C.c_int, [_u64p, _u64p, _u64p, C.c_int, C.c_uint64]),
        "orc_create": (C.c_void_p, [C.c_int, _P(C.c_int), C.c_int, C.c_double, C.c_uint64]),
        "orc_free": (None, [C.c_void_p]),
        "orc_n": (C.c_int, [C.c_void_p]),
        "orc_num_data_primes": (C.c_int, [C.c_void_p]),
        "orc_primes": (None, [C.c_void_p, _u64p]),
        "orc_scale": (C.c_double, [C.c_void_p]),
        "orc_keygen": (C.c_int, [C.c_void_p]),
        "orc_galois_keygen": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
        "orc_export_secret": (C.c_int, [C.c_void_p, _i64p]),
        "orc_export_pk": (C.c_int, [C.c_void_p, _u64p]),
        "orc_key_max_level": (C.c_int, [C.c_void_p, C.c_int, C.c_int]),
        "orc_export_key": (C.c_int, [C.c_void_p, C.c_int, C.c_int, _u64p]),
        "orc_encode_coeffs": (C.c_int, [C.c_void_p, _dp, C.c_size_t, C.c_double, _i64p]),
        "orc_encode": (_ctp, [C.c_void_p, _dp, C.c_size_t, C.c_double, C.c_int]),
        "orc_pt_from_coeffs": (_ctp, [C.c_void_p, _i64p, C.c_double, C.c_int]),
        "orc_decode": (C.c_int, [C.c_void_p, _ctp, _dp, C.c_size_t]),
        "orc_pt_centered": (C.c_int, [C.c_void_p, _ctp, _P(C.c_longdouble)]),
        "orc_ct_new": (_ctp, [C.c_void_p, C.c_int, C.c_double]),
        "orc_pt_new": (_ctp, [C.c_void_p, C.c_int, C.c_double]),
        "orc_ct_free": (None, [_ctp]),
        "orc_pt_free": (None, [_ctp]),
        "orc_encrypt": (_ctp, [C.c_void_p, _ctp, C.c_uint32, C.c_int]),
        "orc_decrypt": (_ctp, [C.c_void_p, _ctp]),
        "orc_add": (_ctp, [C.c_void_p, _ctp, _ctp]),
        "orc_sub": (_ctp, [C.c_void_p, _ctp, _ctp]),
        "orc_negate": (_ctp, [C.c_void_p, _ctp]),
        "orc_add_plain": (_ctp, [C.c_void_p, _ctp, _ctp]),
        "orc_sub_plain": (_ctp, [C.c_void_p, _ctp, _ctp]),
        "orc_mul_plain": (_ctp, [C.c_void_p, _ctp, _ctp]),
        "orc_mul_relin": (_ctp, [C.c_void_p, _ctp, _ctp]),
        "orc_rescale": (_ctp, [C.c_void_p, _ctp]),
        "orc_drop_to": (_ctp, [C.c_void_p, _ctp, C.c_int]),
        "orc_rotate": (_ctp, [C.c_void_p, _ctp, C.c_int]),
        "orc_key_switch": (C.c_int, [C.c_void_p, C.c_int, C.c_int, _u64p, C.c_int, _u64p]),
        "orc_automorphism": (None, [_u64p, _u64p, C.c_int, C.c_uint64, C.c_uint64]),
        "orc_sum_slots": (_ctp, [C.c_void_p, _ctp, C.c_uint32]),
        "orc_conv_im2col": (_ctp, [C.c_void_p, _ctp, _dp, C.c_uint32, C.c_uint32, C.c_double]),
        "orc_matmul": (_ctp, [C.c_void_p, _ctp, _dp, C.c_uint32, C.c_uint32, _dp]),
        "orc_pack": (_ctp, [C.c_void_p, _P(_ctp), C.c_uint32, C.c_uint32]),
        "orc_square": (_ctp, [C.c_void_p, _ctp]),
        "orc_im2col": (None, [_dp, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, _dp]),
        "orc_cnn": (_ctp, [C.c_void_p, _ctp, _dp, _dp, _dp, _dp, _dp, _dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _ptr(a, ct):
    return a.ctypes.data_as(_P(ct))


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__("%s failed with oracle code %d" % (what, code))
        self.code = code


class _Obj:
    """Owned oracle ciphertext (two polys) or plaintext (one poly)."""

    def __init__(self, ctx, ptr, npoly):
        self.ctx, self.ptr, self.npoly = ctx, ptr, npoly

    @property
    def level(self):
        return self.ptr.contents.level

    @property
    def scale(self):
        return self.ptr.contents.scale

    def data(self):
        """copy of the residues, shape [npoly][level+1][N] (ct) or [level+1][N] (pt)"""
        n = self.ctx.n
        cnt = self.npoly * (self.level + 1) * n
        a = np.ctypeslib.as_array(self.ptr.contents.data, shape=(cnt,)).copy()
        if self.npoly == 2:
            return a.reshape(2, self.level + 1, n)
        return a.reshape(self.level + 1, n)

    def __del__(self):
        try:
            if self.ptr:
                (lib().orc_ct_free if self.npoly == 2 else lib().orc_pt_free)(self.ptr)
                self.ptr = None
        except Exception:
            pass


class Oracle:
    """One oracle context: parameters, prime chain, keys."""

    def __init__(self, log_n, bits, scale, seed):
        L = lib()
        b = (C.c_int * len(bits))(*bits)
        self.h = L.orc_create(log_n, b, len(bits), float(scale), seed)
        if not self.h:
            raise OracleError(L.orc_last_error(), "orc_create")
        self.log_n = log_n
        self.n = L.orc_n(self.h)
        self.L = L.orc_num_data_primes(self.h)
        p = np.zeros(self.L + 1, dtype=np.uint64)
        L.orc_primes(self.h, _ptr(p, C.c_uint64))
        self.primes = [int(x) for x in p]
        self.scale = float(scale)

    def __del__(self):
        try:
            if self.h:
                lib().orc_free(self.h)
                self.h = None
        except Exception:
            pass

    def _chk(self, rc, what):
        if rc != ORC_OK:
            raise OracleError(rc, what)

    def _wrap(self, ptr, npoly, what):
        if not ptr:
            raise OracleError(lib().orc_last_error(), what)
        return _Obj(self, ptr, npoly)

    # keys
    def keygen(self):
        self._chk(lib().orc_keygen(self.h), "keygen")

    def galois_keygen(self, step, max_level=-1):
        self._chk(lib().orc_galois_keygen(self.h, int(step), int(max_level)), "galois_keygen")

    def secret(self):
        s = np.zeros(self.n, dtype=np.int64)
        self._chk(lib().orc_export_secret(self.h, _ptr(s, C.c_int64)), "export_secret")
        return s

    def public_key(self):
        a = np.zeros((2, self.L, self.n), dtype=np.uint64)
        self._chk(lib().orc_export_pk(self.h, _ptr(a, C.c_uint64)), "export_pk")
        return a

    def key(self, kind, step=0):
        """kind 0 = relinearisation, 1 = Galois(step); [digit][2][modulus][N]"""
        ml = lib().orc_key_max_level(self.h, kind, step)
        if ml < 0:
            raise OracleError(ml, "key")
        a = np.zeros((ml + 1, 2, ml + 2, self.n), dtype=np.uint64)
        self._chk(lib().orc_export_key(self.h, kind, step, _ptr(a, C.c_uint64)), "export_key")
        return a

    # encoding
    def encode_coeffs(self, z, scale):
        z = np.ascontiguousarray(z, dtype=np.float64)
        out = np.zeros(self.n, dtype=np.int64)
        self._chk(lib().orc_encode_coeffs(self.h, _ptr(z, C.c_double), z.size, float(scale),
                                          _ptr(out, C.c_int64)), "encode_coeffs")
        return out

    def encode(self, z, scale, level):
        z = np.ascontiguousarray(z, dtype=np.float64)
        return self._wrap(lib().orc_encode(self.h, _ptr(z, C.c_double), z.size, float(scale), level),
                          1, "encode")

    def pt_from_coeffs(self, coeffs, scale, level):
        c = np.ascontiguousarray(coeffs, dtype=np.int64)
        return self._wrap(lib().orc_pt_from_coeffs(self.h, _ptr(c, C.c_int64), float(scale), level),
                          1, "pt_from_coeffs")

    def decode(self, pt, n):
        z = np.zeros(n, dtype=np.float64)
        self._chk(lib().orc_decode(self.h, pt.ptr, _ptr(z, C.c_double), n), "decode")
        return z

    def centered(self, pt):
        out = np.zeros(self.n, dtype=np.longdouble)
        self._chk(lib().orc_pt_centered(self.h, pt.ptr, _ptr(out, C.c_longdouble)), "centered")
        return out

    def ct_from_data(self, data, level, scale):
        obj = self._wrap(lib().orc_ct_new(self.h, level, float(scale)), 2, "ct_new")
        d = np.ascontiguousarray(data, dtype=np.uint64).reshape(-1)
        assert d.size == 2 * (level + 1) * self.n
        C.memmove(obj.ptr.contents.data, d.ctypes.data, d.nbytes)
        return obj

    def pt_from_data(self, data, level, scale):
        obj = self._wrap(lib().orc_pt_new(self.h, level, float(scale)), 1, "pt_new")
        d = np.ascontiguousarray(data, dtype=np.uint64).reshape(-1)
        assert d.size == (level + 1) * self.n
        C.memmove(obj.ptr.contents.data, d.ctypes.data, d.nbytes)
        return obj

    # encryption
    def encrypt(self, pt, enc_index=0, use_sk=False):
        return self._wrap(lib().orc_encrypt(self.h, pt.ptr, enc_index, 1 if use_sk else 0), 2,
                          "encrypt")

    def decrypt(self, ct):
        return self._wrap(lib().orc_decrypt(self.h, ct.ptr), 1, "decrypt")

    # ops
    def add(self, a, b):
        return self._wrap(lib().orc_add(self.h, a.ptr, b.ptr), 2, "add")

    def sub(self, a, b):
        return self._wrap(lib().orc_sub(self.h, a.ptr, b.ptr), 2, "sub")

    def negate(self, a):
        return self._wrap(lib().orc_negate(self.h, a.ptr), 2, "negate")

    def add_plain(self, a, p):
        return self._wrap(lib().orc_add_plain(self.h, a.ptr, p.ptr), 2, "add_plain")

    def sub_plain(self, a, p):
        return self._wrap(lib().orc_sub_plain(self.h, a.ptr, p.ptr), 2, "sub_plain")

    def mul_plain(self, a, p):
        return self._wrap(lib().orc_mul_plain(self.h, a.ptr, p.ptr), 2, "mul_plain")

    def mul_relin(self, a, b):
        return self._wrap(lib().orc_mul_relin(self.h, a.ptr, b.ptr), 2, "mul_relin")

    def rescale(self, a):
        return self._wrap(lib().orc_rescale(self.h, a.ptr), 2, "rescale")

    def drop_to(self, a, level):
        return self._wrap(lib().orc_drop_to(self.h, a.ptr, level), 2, "drop_to")

    def rotate(self, a, step):
        return self._wrap(lib().orc_rotate(self.h, a.ptr, int(step)), 2, "rotate")

    def key_switch(self, kind, step, d, level):
        d = np.ascontiguousarray(d, dtype=np.uint64)
        out = np.zeros((2, level + 1, self.n), dtype=np.uint64)
        self._chk(lib().orc_key_switch(self.h, kind, step, _ptr(d, C.c_uint64), level,
                                       _ptr(out, C.c_uint64)), "key_switch")
        return out

    # -- power and polynomial evaluation (section 3: minimum-depth circuits;
    # the circuits are the readings stated in power_plan / polyval) --
    def _mul_rescale(self, a, b):
        la, lb = a.level, b.level
        if la > lb:
            a = self.drop_to(a, lb)
        elif lb > la:
            b = self.drop_to(b, la)
        return self.rescale(self.mul_relin(a, b))

    def power(self, a, k, squares=None):
        """a^k with multiplicative depth ceil(log2 k): the squares a^(2^i) of
        the set bits of k, then the two factors of least depth (ties: the
        smaller exponent) multiplied until one is left; every product is
        relinearised and rescaled.  `squares` caches a^(2^i) across calls."""
        k = int(k)
        if k < 1:
            raise OracleError(ORC_EINVAL, "power: exponent %d < 1" % k)
        sq = squares if squares is not None else {}
        sq.setdefault(0, a)
        top = k.bit_length() - 1
        for i in range(1, top + 1):
            if i not in sq:
                sq[i] = self._mul_rescale(sq[i - 1], sq[i - 1])
        # (depth, exponent, ciphertext)
        fac = [(i, 1 << i, sq[i]) for i in range(top + 1) if (k >> i) & 1]
        while len(fac) > 1:
            fac.sort(key=lambda f: (f[0], f[1]))
            (da, ea, ca), (db, eb, cb) = fac[0], fac[1]
            fac = fac[2:] + [(max(da, db) + 1, ea + eb, self._mul_rescale(ca, cb))]
        return fac[0][2]

    def polyval(self, a, coeffs):
        """sum_i coeffs[i] a^i: each a^i (i >= 1, coeffs[i] != 0) from the
        power circuit, times the constant coeffs[i] encoded at scale
        Delta * q_l / scale(a^i) at the level l of a^i and rescaled, so that
        every term lands at scale Delta; the terms are cut to the lowest
        level and summed in increasing i, then coeffs[0] is added at that
        scale.  Depth ceil(log2 d) + 1."""
        cs = [float(x) for x in coeffs]
        idx = [i for i in range(1, len(cs)) if cs[i] != 0.0]
        if not idx:
            raise OracleError(ORC_EINVAL, "polyval: no non-constant term")
        half = self.n // 2
        sq = {}
        terms = []
        for i in idx:
            x = self.power(a, i, sq)
            ps = self.scale * self.primes[x.level] / x.scale
            p = self.encode(np.full(half, cs[i]), ps, x.level)
            terms.append(self.rescale(self.mul_plain(x, p)))
        low = min(t.level for t in terms)
        terms = [t if t.level == low else self.drop_to(t, low) for t in terms]
        acc = terms[0]
        for t in terms[1:]:
            acc = self.add(acc, t)
        if cs[0] != 0.0:
            acc = self.add_plain(acc, self.encode(np.full(half, cs[0]), acc.scale, acc.level))
        return acc

    def sum_slots(self, a, n):
        return self._wrap(lib().orc_sum_slots(self.h, a.ptr, n), 2, "sum_slots")

    def conv_im2col(self, a, kernel, windows, bias):
        k = np.ascontiguousarray(kernel, dtype=np.float64)
        return self._wrap(lib().orc_conv_im2col(self.h, a.ptr, _ptr(k, C.c_double), k.size,
                                                windows, float(bias)), 2, "conv_im2col")

    def matmul(self, a, w, bias=None):
        w = np.ascontiguousarray(w, dtype=np.float64)
        n_in, n_out = w.shape
        bp = None
        if bias is not None:
            bias = np.ascontiguousarray(bias, dtype=np.float64)
            bp = _ptr(bias, C.c_double)
        return self._wrap(lib().orc_matmul(self.h, a.ptr, _ptr(w, C.c_double), n_in, n_out, bp),
                          2, "matmul")

    def pack(self, parts, width):
        arr = (_ctp * len(parts))(*[p.ptr for p in parts])
        return self._wrap(lib().orc_pack(self.h, arr, len(parts), width), 2, "pack")

    def square(self, a):
        return self._wrap(lib().orc_square(self.h, a.ptr), 2, "square")

    def cnn(self, x, conv_k, conv_b, w1, b1, w2, b2):
        arrs = [np.ascontiguousarray(v, dtype=np.float64) for v in (conv_k, conv_b, w1, b1, w2, b2)]
        ptrs = [_ptr(v, C.c_double) for v in arrs]
        return self._wrap(lib().orc_cnn(self.h, x.ptr, *ptrs), 2, "cnn")


def im2col(img, k, stride):
    img = np.ascontiguousarray(img, dtype=np.float64)
    h, w = img.shape
    oh, ow = (h - k) // stride + 1, (w - k) // stride + 1
    out = np.zeros(k * k * oh * ow, dtype=np.float64)
    lib().orc_im2col(_ptr(img, C.c_double), h, w, k, stride, _ptr(out, C.c_double))
    return out


def chacha20_block(key_words, counter, nonce_words):
    k = (C.c_uint32 * 8)(*key_words)
    n = (C.c_uint32 * 3)(*nonce_words)
    out = (C.c_uint32 * 16)()
    lib().orc_chacha20_block(k, counter, n, out)
    return list(out)


def stream_words(seed, tag, a, b, nwords):
    out = np.zeros(nwords, dtype=np.uint64)
    lib().orc_stream_words(seed, tag, a, b, nwords, _ptr(out, C.c_uint64))
    return out


def is_prime(n):
    return bool(lib().orc_is_prime(n))


def gen_primes(log_n, bits):
    b = (C.c_int * len(bits))(*bits)
    out = np.zeros(len(bits), dtype=np.uint64)
    rc = lib().orc_gen_primes(log_n, b, len(bits), _ptr(out, C.c_uint64))
    if rc:
        raise OracleError(rc, "gen_primes")
    return [int(x) for x in out]


def cdt_table():
    p = lib().orc_cdt_table()
    return [int(p[i]) for i in range(20)]


def sample_ternary(seed, tag, a, n):
    out = np.zeros(n, dtype=np.int64)
    lib().orc_sample_ternary(seed, tag, a, n, _ptr(out, C.c_int64))
    return out


def sample_gaussian(seed, tag, a, n):
    out = np.zeros(n, dtype=np.int64)
    lib().orc_sample_gaussian(seed, tag, a, n, _ptr(out, C.c_int64))
    return out


def sample_uniform(seed, tag, a, b, q, n):
    out = np.zeros(n, dtype=np.uint64)
    lib().orc_sample_uniform(seed, tag, a, b, q, n, _ptr(out, C.c_uint64))
    return out


def negacyclic_mul(a, b, log_n, q):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    c = np.zeros_like(a)
    rc = lib().orc_negacyclic_mul(_ptr(a, C.c_uint64), _ptr(b, C.c_uint64), _ptr(c, C.c_uint64),
                                  log_n, q)
    if rc:
        raise OracleError(rc, "negacyclic_mul")
    return c


def automorphism(a, log_n, g, q):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.zeros_like(a)
    lib().orc_automorphism(_ptr(a, C.c_uint64), _ptr(out, C.c_uint64), log_n, g, q)
    return out
