"""GPU parity of the composites (slot sum, im2col convolution, replicated
vector-matrix product, channel packing) and of the MNIST-shaped CNN of
section 5 against the oracle, bit for bit, plus the decrypted logits against
FP64 within 1e-3."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_03152_amd import inputs as I
from tests.gpu_common import Pair, say
from tests.plain_ref import cnn_fp64

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def deep():
    return Pair(12, [60, 40, 40, 40, 60], 2.0 ** 40, 6)


def _keys(P, steps):
    for st in steps:
        P.o.galois_keygen(st)
        P.H.he_keygen_galois(P.g, st, -1)


def _enc(P, v, idx, level):
    H = P.H
    return (H.he_encrypt(P.g, H.he_encode(P.g, v, P.scale, level), idx, False),
            P.o.encrypt(P.o.encode(v, P.scale, level), idx, False))


@pytest.mark.parametrize("img,k,stride", [(14, 4, 2), (12, 3, 3), (9, 1, 2)])
def test_conv_im2col_bit_exact(deep, img, k, stride):
    P = deep
    rng = np.random.default_rng(img * 10 + k)
    image = rng.uniform(0, 1, (img, img))
    K = rng.normal(0, 0.1, k * k)
    v = P.H.he_im2col(image, k, stride)
    assert np.array_equal(v, O.im2col(image, k, stride))
    windows = ((img - k) // stride + 1) ** 2
    _keys(P, [windows << j for j in range(max(1, (k * k - 1).bit_length()))])
    g, o = _enc(P, v, 1, 3)
    say("conv", img, k, stride)
    gc, oc = P.H.he_enc_conv_im2col(P.g, g, K, windows, 0.05), P.o.conv_im2col(o, K, windows, 0.05)
    P.ct_equal(gc, oc, "conv")
    plan = P.H.he_conv_plan(P.g, g, K, windows, 0.05)
    P.ct_equal(P.H.he_plan_apply(P.g, plan, g), oc, "conv plan")
    want = K @ v.reshape(k * k, windows) + 0.05
    assert np.abs(P.H.he_decode(P.g, P.H.he_decrypt(P.g, gc), windows) - want).max() < 1e-6


@pytest.mark.parametrize("n_in,n_out", [(48, 20), (64, 10), (5, 3), (1, 1), (100, 100)])
def test_matmul_bit_exact(deep, n_in, n_out):
    P = deep
    half = P.n // 2
    rng = np.random.default_rng(n_in * 1000 + n_out)
    W = rng.normal(0, 0.1, (n_in, n_out))
    b = rng.normal(0, 0.1, n_out)
    x = rng.uniform(-1, 1, n_in)
    _keys(P, I.replication_steps(n_in, half) + list(range(1, n_in)))
    g, o = _enc(P, x, 2, 3)
    say("matmul", n_in, n_out)
    gy, oy = P.H.he_enc_matmul(P.g, g, W, b), P.o.matmul(o, W, b)
    P.ct_equal(gy, oy, "matmul")
    dec = P.H.he_decode(P.g, P.H.he_decrypt(P.g, gy), half)
    assert np.abs(dec[:n_out] - (x @ W + b)).max() < 1e-6
    assert np.abs(dec[n_out:]).max() < 1e-6


def test_conv_plans_in_lock_step(deep):
    # four convolution plans applied together (batched rotations) give the
    # oracle's per-channel ciphertexts bit for bit
    P = deep
    rng = np.random.default_rng(21)
    image = rng.uniform(0, 1, (14, 14))
    v = P.H.he_im2col(image, 4, 2)
    _keys(P, [36 << j for j in range(4)])
    g, o = _enc(P, v, 5, 3)
    Ks = rng.normal(0, 0.1, (4, 16))
    bs = rng.normal(0, 0.1, 4)
    plans = [P.H.he_conv_plan(P.g, g, Ks[c], 36, bs[c]) for c in range(4)]
    outs = P.H.he_plan_apply_many(P.g, plans, g)
    for c in range(4):
        P.ct_equal(outs[c], P.o.conv_im2col(o, Ks[c], 36, bs[c]), "channel %d" % c)


def test_pack_and_sum_bit_exact(deep):
    P = deep
    half = P.n // 2
    rng = np.random.default_rng(3)
    _keys(P, [half - 10 * c for c in (1, 2)] + [1 << t for t in range(6)])
    vals = [rng.uniform(-1, 1, 40) for _ in range(3)]
    pairs = [_enc(P, v, 10 + i, 3) for i, v in enumerate(vals)]
    say("pack")
    gp = P.H.he_pack(P.g, [p[0] for p in pairs], 10)
    op = P.o.pack([p[1] for p in pairs], 10)
    P.ct_equal(gp, op, "pack")
    say("sum")
    P.ct_equal(P.H.he_sum_slots(P.g, pairs[0][0], 48), P.o.sum_slots(pairs[0][1], 48), "sum48")


def cnn_plans(H, g, x, d):
    """The section 5 network's plaintext operands, prepared (and each plan
    applied once) on the input x."""
    s = I.CNN_SHAPE
    conv = [H.he_conv_plan(g, x, d["conv_k"][c], s["windows"], d["conv_b"][c]) for c in range(s["channels"])]
    s1 = H.he_square(g, H.he_pack(g, H.he_plan_apply_many(g, conv, x), s["windows"]))
    fc1 = H.he_matmul_plan(g, s1, d["w1"], d["b1"])
    s2 = H.he_square(g, H.he_plan_apply(g, fc1, s1))
    fc2 = H.he_matmul_plan(g, s2, d["w2"], d["b2"])
    H.he_plan_apply(g, fc2, s2)
    return conv, fc1, fc2


def cnn_step(H, g, plans, x):
    conv, fc1, fc2 = plans
    p = H.he_pack(g, H.he_plan_apply_many(g, conv, x), I.CNN_SHAPE["windows"])
    h = H.he_plan_apply(g, fc1, H.he_square(g, p))
    return H.he_plan_apply(g, fc2, H.he_square(g, h))


def run_cnn_gpu(H, g, x, d):
    """The section 5 network through the C ABI (one-shot calls, plans built
    from x inside them)."""
    s = I.CNN_SHAPE
    plans = [H.he_conv_plan(g, x, d["conv_k"][c], s["windows"], d["conv_b"][c])
             for c in range(s["channels"])]
    parts = H.he_plan_apply_many(g, plans, x)
    p = H.he_pack(g, parts, s["windows"])
    s1 = H.he_square(g, p)
    h = H.he_enc_matmul(g, s1, d["w1"], d["b1"])
    s2 = H.he_square(g, h)
    return H.he_enc_matmul(g, s2, d["w2"], d["b2"])


def test_cnn_bit_exact_and_logits():
    p = I.CNN
    P = Pair(p["log_n"], p["bits"], p["scale"], p["seed"], step_levels=I.cnn_rotation_steps(),
             auto_rescale=True)
    d = I.cnn_inputs()
    v = O.im2col(d["img"], 7, 3)
    gx = P.H.he_encrypt(P.g, P.H.he_encode(P.g, v, P.scale, P.o.L - 1), 0, False)
    ox = P.o.encrypt(P.o.encode(v, P.scale, P.o.L - 1), 0)
    P.ct_equal(gx, ox, "input")
    say("cnn oracle")
    oy = P.o.cnn(ox, d["conv_k"], d["conv_b"], d["w1"], d["b1"], d["w2"], d["b2"])
    say("cnn gpu")
    gy = run_cnn_gpu(P.H, P.g, gx, d)
    P.ct_equal(gy, oy, "cnn output")
    logits = P.H.he_decode(P.g, P.H.he_decrypt(P.g, gy), 10)
    assert np.abs(logits - cnn_fp64(d)).max() < 1e-3
    # the same step with prepared plans, eager and replayed from a captured
    # graph (input: a copy of x), every result against the oracle
    H, g = P.H, P.g
    plans = cnn_plans(H, g, gx, d)
    P.ct_equal(cnn_step(H, g, plans, gx), oy, "cnn step with plans")
    xin = H.he_drop_to(g, gx, P.o.L - 1)
    say("cnn graph capture")
    H.he_graph_begin(g)
    out = cnn_step(H, g, plans, xin)
    graph = H.he_graph_end(g)
    for rep in range(3):
        H.he_graph_launch(g, graph)
        H.he_sync(g)
        P.ct_equal(out, oy, "graph replay %d" % rep)
        # eager work between the replays
        P.ct_equal(cnn_step(H, g, plans, gx), oy, "eager step after replay %d" % rep)
    graph.free()


def test_matmul_n16384_bit_exact():
    # the hoisted replication and product at N = 16384, whose kernels use a
    # different workgroup shape and LDS plan than at N = 8192, against the
    # oracle bit for bit, and the decrypted result against plaintext
    n_in, n_out = 256, 8
    half = 8192
    steps = sorted(set(I.replication_steps(n_in, half)) | set(range(1, n_in)))
    P = Pair(14, [60, 40, 40, 60], 2.0 ** 40, 17, steps=steps, auto_rescale=True)
    rng = np.random.default_rng(16384)
    W = rng.normal(0, 0.1, (n_in, n_out))
    b = rng.normal(0, 0.1, n_out)
    x = rng.uniform(-1, 1, n_in)
    gx, ox = _enc(P, x, 3, 2)
    say("matmul n16384")
    gy, oy = P.H.he_enc_matmul(P.g, gx, W, b), P.o.matmul(ox, W, b)
    P.ct_equal(gy, oy, "matmul n16384")
    dec = P.H.he_decode(P.g, P.H.he_decrypt(P.g, gy), half)
    assert np.abs(dec[:n_out] - (x @ W + b)).max() < 1e-6
    assert np.abs(dec[n_out:]).max() < 1e-6
