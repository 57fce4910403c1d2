"""Pins of the oracle's scheme operations against exact identities and big-
integer recomputations (section 2.1: keys, automatic relinearisation and
rescaling; section 3: element-wise ops, rotations; sections 3.1, 3.2, 5:
dot product, vector-matrix product, im2col convolution, the CNN).

Exact pins: each key satisfies evk0 + evk1*s = e + [t=j] p s' with the sampled
e; each encryption decrypts to m plus exactly the sampled noise terms;
ModDown and rescale equal round(x / p) on CRT-reconstructed integers; a key
switch equals the big-integer digit decomposition, inner product and
rounding.  Approximate pins: decrypted results against FP64 arithmetic."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_03152_amd import inputs as I
from tests.bigint_ref import centered, crt, negacyclic_int, residues
from tests.plain_ref import cnn_fp64


@pytest.fixture(scope="module")
def small():
    p = I.SMALL
    o = O.Oracle(p["log_n"], p["bits"], p["scale"], p["seed"])
    o.keygen()
    for t in range(11):
        o.galois_keygen(1 << t)
    o.galois_keygen(3)
    return o


def _mul(a, b, o, q):
    return O.negacyclic_mul(a, b, o.log_n, q)


def _red(v, q):
    return np.array([int(x) % q for x in v], dtype=np.uint64)


def test_public_key_identity(small):
    o = small
    s = o.secret()
    pk = o.public_key()
    e = O.sample_gaussian(o_seed(o), 3, 0, o.n)
    for i in range(o.L):
        q = o.primes[i]
        lhs = (pk[0, i].astype(object) + _mul(pk[1, i], _red(s, q), o, q).astype(object)) % q
        assert np.array_equal(lhs.astype(np.uint64), _red(e, q))
        assert np.array_equal(pk[1, i], O.sample_uniform(o_seed(o), 2, 0, i, q, o.n))


def o_seed(o):
    return I.SMALL["seed"] if o.n == 4096 else None


def _check_switch_key(o, key, sprime_res, tag_a, tag_e, idx_base, seed):
    s = o.secret()
    ml = key.shape[0] - 1
    mods = list(range(ml + 1)) + [o.L]
    p = o.primes[o.L]
    for j in range(ml + 1):
        e = O.sample_gaussian(seed, tag_e, idx_base + j, o.n)
        for t, pi in enumerate(mods):
            q = o.primes[pi]
            a = key[j, 1, t]
            assert np.array_equal(a, O.sample_uniform(seed, tag_a, idx_base + j, pi, q, o.n))
            lhs = (key[j, 0, t].astype(object) + _mul(a, _red(s, q), o, q).astype(object)) % q
            want = _red(e, q).astype(object)
            if t == j:
                want = (want + (p % q) * sprime_res[pi].astype(object)) % q
            assert np.array_equal(lhs.astype(np.uint64), want.astype(np.uint64))


def test_relin_key_identity(small):
    o = small
    s = o.secret()
    s2 = {pi: _mul(_red(s, o.primes[pi]), _red(s, o.primes[pi]), o, o.primes[pi])
          for pi in range(o.L + 1)}
    _check_switch_key(o, o.key(0), s2, 4, 5, 0, I.SMALL["seed"])


def test_galois_key_identity(small):
    o = small
    s = o.secret()
    for step in (1, 3, 1024):
        g = pow(5, step, 2 * o.n)
        ts = {pi: O.automorphism(_red(s, o.primes[pi]), o.log_n, g, o.primes[pi])
              for pi in range(o.L + 1)}
        _check_switch_key(o, o.key(1, step), ts, 6, 7, 256 * step, I.SMALL["seed"])


def test_key_level_restriction_is_exact():
    # a key cut at a lower level equals the restriction of the top-level key
    p = I.SMALL
    a = O.Oracle(12, [40, 40, 40, 40], 2.0 ** 30, 5)
    b = O.Oracle(12, [40, 40, 40, 40], 2.0 ** 30, 5)
    a.keygen()
    b.keygen()
    a.galois_keygen(5)
    b.galois_keygen(5, 1)
    ka, kb = a.key(1, 5), b.key(1, 5)
    assert kb.shape[0] == 2
    assert np.array_equal(kb[:, :, :2], ka[:2, :, :2])
    assert np.array_equal(kb[:, :, 2], ka[:2, :, 3])  # special prime last
    del p


def test_secret_key_encryption_identity(small):
    o = small
    x, _, _ = I.small_vectors()
    pt = o.encode(x, o.scale, 1)
    ct = o.encrypt(pt, 5, use_sk=True)
    s = o.secret()
    e = O.sample_gaussian(I.SMALL["seed"], 12, 5, o.n)
    c = ct.data()
    m = pt.data()
    for i in range(2):
        q = o.primes[i]
        assert np.array_equal(c[1, i], O.sample_uniform(I.SMALL["seed"], 11, 5, i, q, o.n))
        dec = (c[0, i].astype(object) + _mul(c[1, i], _red(s, q), o, q).astype(object)) % q
        want = (_red(e, q).astype(object) + m[i].astype(object)) % q
        assert np.array_equal(dec.astype(np.uint64), want.astype(np.uint64))


def test_public_key_encryption_identity(small):
    o = small
    x, _, _ = I.small_vectors()
    pt = o.encode(x, o.scale, 1)
    ct = o.encrypt(pt, 9, use_sk=False)
    seed = I.SMALL["seed"]
    s = o.secret()
    v = O.sample_ternary(seed, 8, 9, o.n)
    e0 = O.sample_gaussian(seed, 9, 9, o.n)
    e1 = O.sample_gaussian(seed, 10, 9, o.n)
    epk = O.sample_gaussian(seed, 3, 0, o.n)
    c, m = ct.data(), pt.data()
    for i in range(2):
        q = o.primes[i]
        dec = (c[0, i].astype(object) + _mul(c[1, i], _red(s, q), o, q).astype(object)) % q
        noise = (_mul(_red(v, q), _red(epk, q), o, q).astype(object) + _red(e0, q).astype(object)
                 + _mul(_red(e1, q), _red(s, q), o, q).astype(object)) % q
        assert np.array_equal(dec.astype(np.uint64),
                              ((noise + m[i].astype(object)) % q).astype(np.uint64))


def test_key_switch_big_integer_tiny():
    # N = 16, three data primes and p: recompute digit decomposition (centred),
    # inner product over Z mod Q_l * p, and round(u / p) mod Q_l with Python ints
    o = O.Oracle(4, [30, 28, 29, 31], 2.0 ** 20, 3)
    o.keygen()
    o.galois_keygen(3)
    rng = np.random.default_rng(0)
    for kind, step in ((0, 0), (1, 3)):
        key = o.key(kind, step)
        ml = key.shape[0] - 1
        for level in (ml, 1, 0):
            qs = o.primes[:level + 1]
            p = o.primes[o.L]
            d = np.stack([rng.integers(0, q, o.n, dtype=np.uint64) for q in qs])
            got = o.key_switch(kind, step, d, level)
            mods = qs + [p]
            P = 1
            for q in mods:
                P *= q
            kmods = list(range(level + 1)) + [ml + 1]
            u = [[0] * o.n, [0] * o.n]
            for j in range(level + 1):
                qj = qs[j]
                dj = [int(v) - qj if int(v) > (qj - 1) // 2 else int(v) for v in d[j]]
                for k in range(2):
                    kv, _ = crt([key[j, k, t] for t in kmods], mods)
                    prod = negacyclic_int(dj, kv)
                    u[k] = [a + b for a, b in zip(u[k], prod)]
            Q = P // p
            for k in range(2):
                uu = [v % P for v in u[k]]
                y = [((v + (p - 1) // 2) // p) % Q for v in uu]
                assert np.array_equal(got[k], residues(y, qs))


def test_rescale_is_rounded_division_full_size():
    o = O.Oracle(12, [60, 40, 40, 40, 60], 2.0 ** 40, 4)
    rng = np.random.default_rng(4)
    for level in (3, 1):
        qs = o.primes[:level + 1]
        data = np.stack([np.stack([rng.integers(0, q, o.n, dtype=np.uint64) for q in qs])
                         for _ in range(2)])
        ct = o.ct_from_data(data, level, 2.0 ** 80)
        r = o.rescale(ct)
        assert r.level == level - 1 and r.scale == 2.0 ** 80 / qs[-1]
        ql = qs[-1]
        Qn = 1
        for q in qs[:-1]:
            Qn *= q
        for k in range(2):
            x, _ = crt(data[k], qs)
            y = [((v + (ql - 1) // 2) // ql) % Qn for v in x]
            assert np.array_equal(r.data()[k], residues(y, qs[:-1]))


def _dec(o, ct, n):
    return o.decode(o.decrypt(ct), n)


def test_exact_homomorphisms(small):
    o = small
    x, y, pv = I.small_vectors()
    cx = o.encrypt(o.encode(x, o.scale, 1), 0, True)
    cy = o.encrypt(o.encode(y, o.scale, 1), 1, True)
    pp = o.encode(pv, o.scale, 1)
    dx, dy = o.decrypt(cx).data(), o.decrypt(cy).data()
    for i in range(2):
        q = o.primes[i]
        assert np.array_equal(o.decrypt(o.add(cx, cy)).data()[i], (dx[i] + dy[i]) % q)
        assert np.array_equal(o.decrypt(o.sub(cx, cy)).data()[i],
                              ((dx[i].astype(object) - dy[i].astype(object)) % q).astype(np.uint64))
        assert np.array_equal(o.decrypt(o.negate(cx)).data()[i], (q - dx[i]) % q)
        assert np.array_equal(o.decrypt(o.mul_plain(cx, pp)).data()[i],
                              _mul(dx[i], pp.data()[i], o, q))
        assert np.array_equal(o.decrypt(o.add_plain(cx, pp)).data()[i], (dx[i] + pp.data()[i]) % q)


def test_relin_and_rotation_noise_is_small(small):
    # decrypt(mul_relin(a, b)) - decrypt(a) * decrypt(b) and
    # decrypt(rot(a)) - tau(decrypt(a)) are key-switch noise only
    o = small
    x, y, _ = I.small_vectors()
    cx = o.encrypt(o.encode(x, o.scale, 1), 0, True)
    cy = o.encrypt(o.encode(y, o.scale, 1), 1, True)
    dx, dy = o.decrypt(cx).data(), o.decrypt(cy).data()
    m = o.decrypt(o.mul_relin(cx, cy)).data()
    prod = np.stack([_mul(dx[i], dy[i], o, o.primes[i]) for i in range(2)])
    diff = np.stack([((m[i].astype(object) - prod[i].astype(object)) % o.primes[i])
                     for i in range(2)]).astype(np.uint64)
    v, Q = crt(diff, o.primes[:2])
    assert max(abs(t) for t in centered(v, Q)) < 2 ** 16
    r = o.decrypt(o.rotate(cx, 3)).data()
    g = pow(5, 3, 2 * o.n)
    tr = np.stack([O.automorphism(dx[i], o.log_n, g, o.primes[i]) for i in range(2)])
    diff = np.stack([((r[i].astype(object) - tr[i].astype(object)) % o.primes[i])
                     for i in range(2)]).astype(np.uint64)
    v, Q = crt(diff, o.primes[:2])
    assert max(abs(t) for t in centered(v, Q)) < 2 ** 16


def test_small_op_set_tolerances(small):
    # the N=4096 op set: decrypted results against FP64 (tolerances from the
    # noise at scale 2^20 with secret-key encryption)
    o = small
    x, y, pv = I.small_vectors()
    cx = o.encrypt(o.encode(x, o.scale, 1), 0, True)
    cy = o.encrypt(o.encode(y, o.scale, 1), 1, True)
    pp = o.encode(pv, o.scale, 1)
    n = 2048
    assert np.abs(_dec(o, cx, n) - x).max() < 1e-2
    assert np.abs(_dec(o, o.add(cx, cy), n) - (x + y)).max() < 1e-2
    assert np.abs(_dec(o, o.rescale(o.mul_plain(cx, pp)), n) - x * pv).max() < 1e-2
    assert np.abs(_dec(o, o.rescale(o.mul_relin(cx, cy)), n) - x * y).max() < 1e-2
    assert np.abs(_dec(o, o.rotate(cx, 1), n) - np.roll(x, -1)).max() < 2e-2
    s = _dec(o, o.sum_slots(cx, n), 1)[0]
    assert abs(s - x.sum()) < 1.0
    cpk = o.encrypt(o.encode(x, o.scale, 1), 3, False)
    assert np.abs(_dec(o, cpk, n) - x).max() < 0.1


def test_error_codes(small):
    o = small
    x, y, _ = I.small_vectors()
    cx = o.encrypt(o.encode(x, o.scale, 1), 0, True)
    low = o.rescale(o.mul_relin(cx, cx))
    with pytest.raises(O.OracleError) as e:
        o.rescale(low)
    assert e.value.code == O.ORC_ELEVEL
    with pytest.raises(O.OracleError) as e:
        o.add(low, cx)
    assert e.value.code == O.ORC_ESCALE
    with pytest.raises(O.OracleError) as e:
        o.rotate(cx, 5)
    assert e.value.code == O.ORC_ENOKEY
    with pytest.raises(O.OracleError) as e:
        o.sum_slots(cx, 4096)
    assert e.value.code == O.ORC_ERANGE
    # operands at different levels align by dropping limbs (exact)
    c2 = o.rescale(o.mul_plain(cx, o.encode(np.ones(2048), 1.0, 1)))
    assert c2.level == 0
    r = o.add(o.drop_to(cx, 0), o.encrypt(o.encode(y, cx.scale, 0), 4, True))
    r2 = o.add(cx, o.encrypt(o.encode(y, cx.scale, 0), 4, True))
    assert np.array_equal(r.data(), r2.data())


@pytest.fixture(scope="module")
def deep():
    # N=4096 with room for several rescales at scale 2^40 (test-only chain)
    o = O.Oracle(12, [60, 40, 40, 40, 60], 2.0 ** 40, 6)
    o.keygen()
    return o


def test_composites_vs_fp64(deep):
    o = deep
    half = o.n // 2
    rng = np.random.default_rng(8)
    # im2col convolution: 14x14 image, 4x4 kernel, stride 2 -> 36 windows, 16 offsets
    img = rng.uniform(0, 1, (14, 14))
    K = rng.normal(0, 0.1, 16)
    v = O.im2col(img, 4, 2)
    win = v.reshape(16, 36)
    for j in range(4):
        o.galois_keygen(36 << j)
    ct = o.encrypt(o.encode(v, o.scale, 3), 1)
    conv = o.conv_im2col(ct, K, 36, 0.05)
    want = K @ win + 0.05
    assert conv.level == 2
    assert np.abs(_dec(o, conv, 36) - want).max() < 1e-6
    # im2col layout: slot k*windows + w = pixel k of window w
    assert win[5, 7] == img[(7 // 6) * 2 + 5 // 4, (7 % 6) * 2 + 5 % 4]
    # vector-matrix product with replication (n_in = 48 is not a power of two)
    n_in, n_out = 48, 20
    W = rng.normal(0, 0.1, (n_in, n_out))
    b = rng.normal(0, 0.1, n_out)
    xv = rng.uniform(-1, 1, n_in)
    for st in I.replication_steps(n_in, half):
        o.galois_keygen(st)
    for i in range(1, n_in):
        o.galois_keygen(i)
    cx = o.encrypt(o.encode(xv, o.scale, 3), 2)
    y = o.matmul(cx, W, b)
    dec = _dec(o, y, half)
    assert np.abs(dec[:n_out] - (xv @ W + b)).max() < 1e-6
    assert np.abs(dec[n_out:]).max() < 1e-6  # slots beyond n_out are zero
    # channel packing of 3 parts of width 10
    parts_v = [rng.uniform(-1, 1, 40) for _ in range(3)]
    for c in (1, 2):
        o.galois_keygen(half - 10 * c)
    parts = [o.encrypt(o.encode(pv, o.scale, 3), 10 + k) for k, pv in enumerate(parts_v)]
    pk = o.pack(parts, 10)
    dec = _dec(o, pk, half)
    want = np.zeros(half)
    for c in range(3):
        want[10 * c:10 * c + 10] = parts_v[c][:10]
    assert np.abs(dec - want).max() < 1e-6
    # slot sum of a non-power-of-two count
    for t in range(6):
        o.galois_keygen(1 << t)
    s = o.sum_slots(o.encrypt(o.encode(xv, o.scale, 3), 3), 48)
    assert abs(_dec(o, s, 1)[0] - xv.sum()) < 1e-6


def test_cnn_vs_fp64_full_size():
    # section 5 network at N = 8192, 8 primes, scale 2^40: logits within 1e-3
    p = I.CNN
    o = O.Oracle(p["log_n"], p["bits"], p["scale"], p["seed"])
    o.keygen()
    steps = I.cnn_rotation_steps()
    # conv 6, packing 3, FC1 15 + 255, FC2 63 + 63 steps; their union
    assert len(steps) == 315
    for st, lv in sorted(steps.items()):
        o.galois_keygen(st, lv)
    d = I.cnn_inputs()
    ct = o.encrypt(o.encode(O.im2col(d["img"], 7, 3), o.scale, o.L - 1), 0)
    out = o.cnn(ct, d["conv_k"], d["conv_b"], d["w1"], d["b1"], d["w2"], d["b2"])
    assert out.level == 0
    logits = _dec(o, out, 10)
    assert np.abs(logits - cnn_fp64(d)).max() < 1e-3
