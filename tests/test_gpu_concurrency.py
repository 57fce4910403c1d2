"""Two contexts, each on its own stream, running vector-matrix products at
the same time: every result is the same ciphertext as when the context runs
alone.  Both the replicated product (hoisted replication, then the
diagonal multiply-accumulate) and the product without replication (the
multiply-accumulate alone, the case where two contexts' long
multiply-accumulate launches overlap) are covered."""
import numpy as np
import pytest

from paper_2104_03152_amd import inputs as I
from tests.gpu_common import hip, say

pytestmark = pytest.mark.gpu

BITS = [60, 40, 40, 40, 60]


def _context(H, cid, n_in, n_out, log_n=12):
    half = (1 << log_n) // 2
    g = H.he_ctx_create(log_n, BITS, 2.0 ** 40, 500 + cid, auto_rescale=True, stream=None)
    H.he_keygen(g, [])
    steps = set(range(1, n_in))
    if n_out > 1:
        steps |= set(I.replication_steps(n_in, half))
    for st in sorted(steps):
        H.he_keygen_galois(g, st, -1)
    rng = np.random.default_rng(cid)
    W = rng.normal(0, 0.1, (n_in, n_out))
    b = rng.normal(0, 0.1, n_out)
    x = H.he_encrypt(g, H.he_encode(g, rng.uniform(-1, 1, n_in), 2.0 ** 40, g.L - 1), 7 + cid, False)
    p = H.he_matmul_plan(g, x, W, b)
    ref = H.he_ct_export(g, H.he_plan_apply(g, p, x))
    H.he_sync(g)
    return g, p, x, ref


@pytest.mark.parametrize("n_in,n_out", [(256, 64), (1100, 1)])
def test_concurrent_products_equal_solo(n_in, n_out):
    H = hip()
    say("contexts", n_in, n_out)
    ctxs = [_context(H, cid, n_in, n_out) for cid in range(2)]
    for it in range(8):
        ys = [H.he_plan_apply(g, p, x) for g, p, x, _ in ctxs]
        for g, _, _, _ in ctxs:
            H.he_sync(g)
        for k, ((g, _, _, ref), y) in enumerate(zip(ctxs, ys)):
            assert np.array_equal(H.he_ct_export(g, y), ref), "iteration %d context %d" % (it, k)
    gs = [c[0] for c in ctxs]
    del ctxs, ys  # every handle before its context
    for g in gs:
        g.close()
