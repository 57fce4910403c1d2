"""GPU parity of the batched entry points (he_mul_relin_many,
he_rotate_many) against the oracle's one-at-a-time results, bit for bit,
across more than one batch of 32 key switches."""
import numpy as np
import pytest

from paper_2104_03152_amd import inputs as I
from tests.gpu_common import Pair, say

pytestmark = pytest.mark.gpu

STEPS = [1, 2, 5, 100, 2047]


@pytest.fixture(scope="module")
def deep():
    return Pair(12, [60, 40, 40, 40, 60], 2.0 ** 40, 7, steps=STEPS)


def _encs(P, n, level, seed):
    rng = np.random.default_rng(seed)
    H = P.H
    g, o = [], []
    for i in range(n):
        v = rng.uniform(-1, 1, 2048)
        g.append(H.he_encrypt(P.g, H.he_encode(P.g, v, P.scale, level), 100 + i, False))
        o.append(P.o.encrypt(P.o.encode(v, P.scale, level), 100 + i, False))
    return g, o


@pytest.mark.parametrize("n", [1, 37])
def test_mul_relin_many_bit_exact(deep, n):
    P = deep
    ga, oa = _encs(P, n, 3, n)
    gb, ob = _encs(P, n, 3, n + 1)
    say("mul_relin_many", n)
    outs = P.H.he_mul_relin_many(P.g, ga, gb)
    assert len(outs) == n
    for i in range(n):
        P.ct_equal(outs[i], P.o.mul_relin(oa[i], ob[i]), "pair %d" % i)
    # freeing some views of a batch leaves the others intact
    for i in range(0, n, 2):
        outs[i].free()
    for i in range(1, n, 2):
        P.ct_equal(outs[i], P.o.mul_relin(oa[i], ob[i]), "pair %d after frees" % i)


def test_mul_relin_many_auto_rescale_bit_exact():
    P = Pair(12, [60, 40, 40, 40, 60], 2.0 ** 40, 8, auto_rescale=True)
    ga, oa = _encs(P, 33, 2, 5)
    say("mul_relin_many rescaled")
    outs = P.H.he_mul_relin_many(P.g, ga, ga[::-1])
    for i in range(33):
        P.ct_equal(outs[i], P.o.rescale(P.o.mul_relin(oa[i], oa[32 - i])), "pair %d" % i)


def test_rotate_many_bit_exact(deep):
    P = deep
    n = 35
    g, o = _encs(P, n, 2, 9)
    steps = [STEPS[i % len(STEPS)] if i % 7 else 0 for i in range(n)]
    say("rotate_many")
    outs = P.H.he_rotate_many(P.g, g, steps)
    for i in range(n):
        P.ct_equal(outs[i], P.o.rotate(o[i], steps[i]), "item %d step %d" % (i, steps[i]))


def test_batches_reject_mixed_levels(deep):
    P = deep
    g3, _ = _encs(P, 1, 3, 1)
    g2, _ = _encs(P, 1, 2, 2)
    with pytest.raises(P.H.HeError):
        P.H.he_mul_relin_many(P.g, [g3[0], g2[0]], [g3[0], g2[0]])
    with pytest.raises(P.H.HeError):
        P.H.he_rotate_many(P.g, [g3[0], g2[0]], [1, 1])
    with pytest.raises(P.H.HeError):
        P.H.he_rotate_many(P.g, [g3[0]], [3])  # no key for step 3


def test_n16384_batched_keyswitch_sampled():
    # the launch configuration of the N=16384 key-switch bench: 34 products
    # of uniform-residue ciphertexts at the top level in batches of 32
    # (one workgroup per limb, the unfused key switch), auto-rescaled;
    # sampled items against the oracle bit for bit
    p = I.RAW
    P = Pair(p["log_n"], p["bits"], p["scale"], p["seed"], auto_rescale=True)
    L = P.o.L
    data = I.raw_residues(P.g.primes, 34, L, P.n, seed=31)
    g = [P.H.he_ct_import(P.g, data[i], L - 1, p["scale"]) for i in range(34)]
    say("n16384 mul_relin_many")
    outs = P.H.he_mul_relin_many(P.g, g, g[1:] + g[:1])
    for i in (0, 31, 33):
        a = P.o.ct_from_data(data[i], L - 1, p["scale"])
        b = P.o.ct_from_data(data[(i + 1) % 34], L - 1, p["scale"])
        P.ct_equal(outs[i], P.o.rescale(P.o.mul_relin(a, b)), "item %d" % i)
