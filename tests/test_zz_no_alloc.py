"""he_mul_relin_noalloc, the entry point for callers that cannot allocate
device memory: its result equals he_mul_relin's bit for bit (and the
oracle's), on two calls in a row, the second with a smaller input; it makes
no allocator call; it refuses an output at the wrong level and a product
that needs more than its fixed scratch."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_03152_amd import inputs as I
from tests.gpu_common import hip, say

pytestmark = pytest.mark.gpu


class CountingTorchAlloc:
    def __init__(self, H, stream):
        import torch
        self.torch, self.stream, self.calls = torch, stream, 0
        self.dev = torch.cuda.current_device()
        self.a = H.Allocator(self.alloc, self.free)

    def alloc(self, n):
        self.calls += 1
        return self.torch.cuda.caching_allocator_alloc(n, self.dev, self.stream)

    def free(self, p, n):
        self.torch.cuda.caching_allocator_delete(p)


def test_noalloc_equals_mul_relin_twice_smaller_second():
    H = hip()
    import torch
    p = I.CNN
    ts = torch.cuda.Stream()
    al = CountingTorchAlloc(H, ts.cuda_stream)
    g = H.he_ctx_create(p["log_n"], p["bits"], p["scale"], p["seed"], auto_rescale=True,
                        stream=ts.cuda_stream, allocator=al.a)
    H.he_keygen(g, [])
    o = O.Oracle(p["log_n"], p["bits"], p["scale"], p["seed"])
    o.keygen()
    rng = np.random.default_rng(55)
    top = g.L - 1
    cases = [(top, top, 40), (2, 3, 41)]  # the second: smaller operands, levels differ
    for k, (la, lb, idx) in enumerate(cases):
        xa, xb = rng.uniform(-1, 1, 4096), rng.uniform(-1, 1, 4096)
        ga = H.he_encrypt(g, H.he_encode(g, xa, p["scale"], la), idx, False)
        gb = H.he_encrypt(g, H.he_encode(g, xb, p["scale"], lb), idx + 100, False)
        ref = H.he_mul_relin(g, ga, gb)
        lo = min(la, lb) - 1
        out = H.he_drop_to(g, ga, lo)  # the caller's output buffer, allocated beforehand
        H.he_sync(g)
        before = al.calls
        say("noalloc call %d: levels %d, %d" % (k, la, lb))
        H.he_mul_relin_noalloc(g, ga, gb, out)
        H.he_sync(g)
        assert al.calls == before, "the call allocated"
        assert out.info() == ref.info()
        want = H.he_ct_export(g, ref)
        assert np.array_equal(H.he_ct_export(g, out), want), "call %d" % k
        oa = o.encrypt(o.encode(xa, p["scale"], la), idx)
        ob = o.encrypt(o.encode(xb, p["scale"], lb), idx + 100)
        assert np.array_equal(o.rescale(o.mul_relin(oa, ob)).data(), want), "oracle, call %d" % k
        dec = H.he_decode(g, H.he_decrypt(g, out), 4096)
        assert np.abs(dec - xa * xb).max() < 1e-3
        del ga, gb, ref, out
    g.close()


def test_noalloc_refusals():
    H = hip()
    p = I.SMALL
    g = H.he_ctx_create(p["log_n"], p["bits"], p["scale"], p["seed"], auto_rescale=True)
    H.he_keygen(g, [])
    x = H.he_encrypt(g, H.he_encode(g, np.ones(8), p["scale"], 1), 0, True)
    wrong = H.he_drop_to(g, x, 1)  # the result would be at level 0
    with pytest.raises(H.HeError) as ei:
        H.he_mul_relin_noalloc(g, x, x, wrong)
    assert ei.value.code == H.HE_ELEVEL
    del x, wrong
    g.close()
    # N = 16384 with 12 data limbs needs more than the fixed scratch
    big = H.he_ctx_create(14, [60] + [40] * 11 + [60], 2.0 ** 40, 3, auto_rescale=True)
    H.he_keygen(big, [])
    y = H.he_encrypt(big, H.he_encode(big, np.ones(8), 2.0 ** 40, big.L - 1), 0, True)
    out = H.he_drop_to(big, y, big.L - 2)
    with pytest.raises(H.HeError) as ei:
        H.he_mul_relin_noalloc(big, y, y, out)
    assert ei.value.code == H.HE_ERANGE
    assert "scratch" in str(ei.value)
    # a smaller level of the same context fits and is exact
    y3 = H.he_drop_to(big, y, 3)
    out3 = H.he_drop_to(big, y, 2)
    H.he_mul_relin_noalloc(big, y3, y3, out3)
    assert np.array_equal(H.he_ct_export(big, out3), H.he_ct_export(big, H.he_mul_relin(big, y3, y3)))
    del y, out, y3, out3
    big.close()
