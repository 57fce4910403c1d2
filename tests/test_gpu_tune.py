"""The NTT autotuner: it reports a timing table (two-phase form and every
one-workgroup thread layout per launch size) and a threshold, and the
results after tuning stay bit-exact with the oracle; every thread layout
gives the default layout's transform bit for bit."""
import os

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
    width = 2 + len(H.he_ntt_layouts(g))
    assert all(len(r) == width and all(v > 0 for v in r[1:]) for r in rows)
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


@pytest.mark.parametrize("log_n", [12, 13, 14])
def test_every_layout_equals_default(log_n):
    from tests.gpu_common import hip
    from paper_2104_03152_amd import inputs as I
    import torch
    H = hip()
    bits = [50] * 5
    n_polys = 80  # 80 x 4 = 320 limb transforms: one workgroup per limb
    ref_f = None
    g0 = H.he_ctx_create(log_n, bits, 2.0 ** 40, 1)
    layouts = H.he_ntt_layouts(g0)
    g0.close()
    assert len(layouts) >= 3 and layouts[0][0] >= layouts[0][1]
    data = I.residues(g0.primes[:4], (n_polys,), 1 << log_n, log_n)
    for k in range(len(layouts)):
        os.environ["HE_NTT_LAYOUT"] = str(k)
        try:
            g = H.he_ctx_create(log_n, bits, 2.0 ** 40, 1)
        finally:
            del os.environ["HE_NTT_LAYOUT"]
        say("layout %d of 2^%d: %s" % (k, log_n, layouts[k]))
        t = torch.from_numpy(data.view(np.int64).copy()).cuda()
        torch.cuda.synchronize()  # the copy is done before the context's stream reads t
        H.he_ntt_forward(g, t.data_ptr(), n_polys, 4)
        H.he_sync(g)
        f = t.cpu().numpy().view(np.uint64).copy()
        if ref_f is None:
            ref_f = f
        assert np.array_equal(f, ref_f), "forward, layout %d" % k
        H.he_ntt_inverse(g, t.data_ptr(), n_polys, 4)
        H.he_sync(g)
        assert np.array_equal(t.cpu().numpy().view(np.uint64), data), "inverse, layout %d" % k
        del t
        g.close()
