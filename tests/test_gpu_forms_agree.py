"""The library's alternative kernel forms of one operation give the same
ciphertext bit for bit (each is also checked against the oracle by the
composite and operation tests):

- the conv's rotate-and-sum and a 48-slot sum with the ciphertext kept in
  coefficient form between steps (the automorphism as a signed coefficient
  permutation) and in the transform domain;
- a product with automatic rescaling through the fused small-batch kernels
  (the ModDown fused with the rescale) and through the one-workgroup-per-
  limb kernels with a separate rescale."""
import os

import numpy as np
import pytest

from paper_2104_03152_amd import inputs as I
from tests.gpu_common import hip, say

pytestmark = pytest.mark.gpu

BITS = [60, 40, 40, 40, 40, 40, 40, 60]


def _ctx(H, env, steps):
    # the forms are context settings, read from the environment at creation
    old = {k: os.environ.get(k) for k in env}
    os.environ.update(env)
    try:
        g = H.he_ctx_create(13, BITS, 2.0 ** 40, 31, auto_rescale=True, stream=None)
    finally:
        for k, v in old.items():
            if v is None:
                del os.environ[k]
            else:
                os.environ[k] = v
    H.he_keygen(g, [])
    for st in steps:
        H.he_keygen_galois(g, st, -1)
    return g


def _conv_and_sum(H, g, d):
    s = I.CNN_SHAPE
    v = H.he_im2col(d["img"], s["k"], s["stride"])
    x = H.he_encrypt(g, H.he_encode(g, v, 2.0 ** 40, g.L - 1), 3, False)
    plans = [H.he_conv_plan(g, x, d["conv_k"][c], s["windows"], d["conv_b"][c]) for c in range(s["channels"])]
    outs = [H.he_ct_export(g, y) for y in H.he_plan_apply_many(g, plans, x)]
    outs.append(H.he_ct_export(g, H.he_sum_slots(g, x, 48)))
    return outs


def test_coefficient_form_rotations_equal_transform_domain():
    H = hip()
    d = I.cnn_inputs()
    s = I.CNN_SHAPE
    steps = [s["windows"] << j for j in range(6)] + [1 << t for t in range(6)]
    res = []
    for env in ({"HE_COEF_ROT": "1"}, {"HE_COEF_ROT": "0"}):
        say("conv + slot sum", env)
        g = _ctx(H, env, steps)
        res.append(_conv_and_sum(H, g, d))
        g.close()
    for i, (a, b) in enumerate(zip(*res)):
        assert np.array_equal(a, b), "output %d" % i


def test_fused_product_rescale_equals_separate_steps():
    H = hip()
    res = []
    # HE_FUSE_MAX=0 and HE_NTT_SPLIT_JOBS=0: one workgroup per limb and the
    # separate rescale
    for env in ({}, {"HE_FUSE_MAX": "0", "HE_NTT_SPLIT_JOBS": "0"}):
        say("square + product", env)
        g = _ctx(H, env, [])
        r = np.random.default_rng(7)
        a = H.he_encrypt(g, H.he_encode(g, r.uniform(-1, 1, 4096), 2.0 ** 40, g.L - 1), 1, False)
        b = H.he_encrypt(g, H.he_encode(g, r.uniform(-1, 1, 4096), 2.0 ** 40, g.L - 2), 2, False)
        sq = H.he_square(g, a)
        res.append([H.he_ct_export(g, sq), H.he_ct_export(g, H.he_mul_relin(g, sq, b)),
                    H.he_ct_export(g, H.he_square(g, H.he_square(g, sq)))])
        del a, b, sq
        g.close()
    for i, (x, y) in enumerate(zip(*res)):
        assert np.array_equal(x, y), "output %d" % i
