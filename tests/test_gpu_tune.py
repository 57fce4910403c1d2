"""The NTT autotuner: it reports a timing table and a threshold, and the
results after tuning stay bit-exact with the oracle (both NTT shapes are
exact)."""
import numpy as np
import pytest

from tests.gpu_common import Pair, say

pytestmark = pytest.mark.gpu


def test_tune_then_parity():
    P = Pair(13, [60, 40, 40, 40, 60], 2.0 ** 40, 9, steps=[3])
    H, g = P.H, P.g
    say("tune")
    chosen, rows = H.he_tune_ntt(g, 512)
    assert [r[0] for r in rows] == [16, 32, 64, 128, 256, 512]
    assert all(r[1] > 0 and r[2] > 0 for r in rows)
    assert chosen in (0,) + tuple(int(r[0]) for r in rows)
    rng = np.random.default_rng(9)
    x, y = rng.uniform(-1, 1, 4096), rng.uniform(-1, 1, 4096)
    gx = H.he_encrypt(g, H.he_encode(g, x, P.scale, 3), 0, False)
    gy = H.he_encrypt(g, H.he_encode(g, y, P.scale, 3), 1, False)
    ox = P.o.encrypt(P.o.encode(x, P.scale, 3), 0, False)
    oy = P.o.encrypt(P.o.encode(y, P.scale, 3), 1, False)
    P.ct_equal(H.he_mul_relin(g, gx, gy), P.o.mul_relin(ox, oy), "mul_relin after tuning")
    P.ct_equal(H.he_rotate(g, gx, 3), P.o.rotate(ox, 3), "rotate after tuning")
    many = H.he_rotate_many(g, [gx] * 40, [3] * 40)  # 40 x 4 x 4 ModUp jobs: large-batch shapes
    want = P.o.rotate(ox, 3)
    for i in (0, 17, 39):
        P.ct_equal(many[i], want, "batched rotate %d after tuning" % i)
