"""The hoisted vector-matrix product (rotations of section 2's CKKSVector
product, hoisted) in its two kernel forms: the two-phase form (column phase
over every rotation's transforms, then block-phase workgroups that
accumulate; several chunk sizes) and the one-kernel form give the same
ciphertext bit for bit.  Each form's parity with the oracle is covered by
the composite tests, which run the default (two-phase) form."""
import os

import numpy as np
import pytest

from paper_2104_03152_amd import inputs as I
from tests.gpu_common import hip, say

pytestmark = pytest.mark.gpu

BITS = [60, 40, 40, 40, 60]


def _product(H, wgs, log_n, n_in, n_out):
    # the form is a context setting, read from the environment at creation
    os.environ["HE_HOIST_SPLIT_WGS"] = str(wgs)
    try:
        g = H.he_ctx_create(log_n, BITS, 2.0 ** 40, 77, auto_rescale=True, stream=None)
    finally:
        del os.environ["HE_HOIST_SPLIT_WGS"]
    H.he_keygen(g, [])
    half = g.n // 2
    steps = set(range(1, n_in)) | set(I.replication_steps(n_in, half))
    for st in sorted(steps):
        H.he_keygen_galois(g, st, -1)
    rng = np.random.default_rng(n_in + n_out)
    W = rng.normal(0, 0.1, (n_in, n_out))
    b = rng.normal(0, 0.1, n_out)
    x = rng.uniform(-1, 1, n_in)
    gx = H.he_encrypt(g, H.he_encode(g, x, 2.0 ** 40, g.L - 1), 5, False)
    gy = H.he_enc_matmul(g, gx, W, b)
    out = H.he_ct_export(g, gy)
    dec = H.he_decode(g, H.he_decrypt(g, gy), half)
    assert np.abs(dec[:n_out] - (x @ W + b)).max() < 1e-6
    del gx, gy
    g.close()
    return out


@pytest.mark.parametrize("log_n,n_in,n_out", [(12, 256, 64), (13, 300, 1), (13, 64, 10), (14, 256, 8)])
def test_forms_equal(log_n, n_in, n_out):
    H = hip()
    say("hoist forms", log_n, n_in, n_out)
    ref = _product(H, 0, log_n, n_in, n_out)
    for wgs in (2048, 100, 1 << 20):
        say("  two-phase, about %d workgroups" % wgs)
        assert np.array_equal(_product(H, wgs, log_n, n_in, n_out), ref), wgs
