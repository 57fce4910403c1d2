"""GPU parity of the multi-ciphertext tensors (the CKKSTensor flavour of
section 2, batched along the last axis; the appendix tables' vector sizes
above N/2): every ciphertext of every result equals the oracle's
one-ciphertext operation on the same chunk, bit for bit, and the decrypted
values match plaintext arithmetic."""
import numpy as np
import pytest

from tests.gpu_common import Pair, say

pytestmark = pytest.mark.gpu

SCALE = 2.0 ** 40


@pytest.fixture(scope="module")
def pair():
    # N = 8192, the 200-bit chain of the appendix tables, slot-sum steps
    return Pair(13, [60, 40, 40, 60], SCALE, 21, steps=[1 << t for t in range(12)], auto_rescale=True)


def _chunks(v, half):
    rows = v.reshape(-1, v.shape[-1])
    return [r[j:j + half] for r in rows for j in range(0, v.shape[-1], half)]


def _otensor(P, v, level, idx0):
    o = P.o
    return [o.encrypt(o.encode(c, SCALE, level), idx0 + i, False) for i, c in enumerate(_chunks(v, P.n // 2))]


def _equal(P, gt, octs, what):
    assert gt.n_ct == len(octs), what
    for i, oc in enumerate(octs):
        P.ct_equal(gt.ct(i), oc, "%s ct %d" % (what, i))


def test_tensor_ops_bit_exact(pair):
    P, H, o = pair, pair.H, pair.o
    half = P.n // 2
    top = P.g.L - 1
    rng = np.random.default_rng(8)
    x = rng.uniform(-1, 1, (2, 10000))  # 3 chunks per row, the last ragged
    y = rng.uniform(-1, 1, (2, 10000))
    w = rng.uniform(-1, 1, (2, 10000))
    say("tensor encrypt", x.shape)
    gx = H.he_tensor_encrypt(P.g, x, SCALE, top, 0)
    gy = H.he_tensor_encrypt(P.g, y, SCALE, top, 100)
    assert gx.shape == (2, 10000) and gx.n_ct == 6
    ox, oy = _otensor(P, x, top, 0), _otensor(P, y, top, 100)
    _equal(P, gx, ox, "encrypt")
    assert np.abs(H.he_tensor_decrypt(P.g, gx) - x).max() < 1e-6

    say("tensor add, sub, negate")
    _equal(P, H.he_tensor_add(P.g, gx, gy), [o.add(a, b) for a, b in zip(ox, oy)], "add")
    _equal(P, H.he_tensor_sub(P.g, gx, gy), [o.sub(a, b) for a, b in zip(ox, oy)], "sub")
    _equal(P, H.he_tensor_negate(P.g, gx), [o.negate(a) for a in ox], "negate")
    assert np.abs(H.he_tensor_decrypt(P.g, H.he_tensor_sub(P.g, gx, gy)) - (x - y)).max() < 1e-6

    say("tensor products")
    gm = H.he_tensor_mul(P.g, gx, gy)
    om = [o.rescale(o.mul_relin(a, b)) for a, b in zip(ox, oy)]
    _equal(P, gm, om, "mul")
    assert np.abs(H.he_tensor_decrypt(P.g, gm) - x * y).max() < 1e-6
    _equal(P, H.he_tensor_square(P.g, gx), [o.rescale(o.mul_relin(a, a)) for a in ox], "square")

    say("tensor plain operands")
    wc = _chunks(w, half)
    gp = H.he_tensor_mul_plain(P.g, gx, w)
    op_ = [o.rescale(o.mul_plain(a, o.encode(c, SCALE, a.level))) for a, c in zip(ox, wc)]
    _equal(P, gp, op_, "mul_plain")
    assert np.abs(H.he_tensor_decrypt(P.g, gp) - x * w).max() < 1e-6
    _equal(P, H.he_tensor_add_plain(P.g, gx, w),
           [o.add_plain(a, o.encode(c, a.scale, a.level)) for a, c in zip(ox, wc)], "add_plain")
    _equal(P, H.he_tensor_sub_plain(P.g, gx, w),
           [o.sub_plain(a, o.encode(c, a.scale, a.level)) for a, c in zip(ox, wc)], "sub_plain")

    say("tensor sum and dot")

    def osum(cts):
        out = []
        for r in range(2):
            acc = cts[3 * r]
            for j in (1, 2):
                acc = o.add(acc, cts[3 * r + j])
            out.append(o.sum_slots(acc, half))
        return out

    gs = H.he_tensor_sum(P.g, gm)
    assert gs.shape == (2, 1)
    _equal(P, gs, osum(om), "sum")
    assert np.abs(H.he_tensor_decrypt(P.g, gs)[:, 0] - (x * y).sum(axis=1)).max() < 1e-4
    gd = H.he_tensor_dot_plain(P.g, gx, w)
    _equal(P, gd, osum(op_), "dot_plain")
    _equal(P, H.he_tensor_dot(P.g, gx, gy), osum(om), "dot")


def test_tensor_power_polyval_and_shapes(pair):
    P, H, o = pair, pair.H, pair.o
    top = P.g.L - 1
    rng = np.random.default_rng(9)
    x = rng.uniform(-1, 1, 5000)  # rank 1, two chunks
    gx = H.he_tensor_encrypt(P.g, x, SCALE, top, 7)
    ox = _otensor(P, x, top, 7)
    _equal(P, H.he_tensor_power(P.g, gx, 2), [o.power(a, 2) for a in ox], "power")
    _equal(P, H.he_tensor_polyval(P.g, gx, [0.5, 1.0, 2.0]), [o.polyval(a, [0.5, 1.0, 2.0]) for a in ox],
           "polyval")
    got = H.he_tensor_decrypt(P.g, H.he_tensor_polyval(P.g, gx, [0.5, 1.0, 2.0]))
    assert np.abs(got - (0.5 + x + 2 * x * x)).max() < 1e-5
    # a rank-3 tensor: rows are the leading indices in row-major order
    z = rng.uniform(-1, 1, (2, 3, 7))
    gz = H.he_tensor_encrypt(P.g, z, SCALE, top, 50)
    assert gz.shape == (2, 3, 7) and gz.n_ct == 6
    assert np.abs(H.he_tensor_decrypt(P.g, gz) - z).max() < 1e-6
    gzs = H.he_tensor_sum(P.g, gz)
    assert gzs.shape == (2, 3, 1)
    assert np.abs(H.he_tensor_decrypt(P.g, gzs)[..., 0] - z.sum(axis=2)).max() < 1e-5
    # shape mismatch and a wrong plain operand size are errors
    with pytest.raises(H.HeError):
        H.he_tensor_add(P.g, gx, gz)
    with pytest.raises(ValueError):
        H.he_tensor_mul_plain(P.g, gz, np.ones(5))
