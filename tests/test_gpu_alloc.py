"""The device-memory contract of the C ABI: memory comes from the caller's
allocator callbacks (torch's caching allocator by default in the binding),
an allocator that returns NULL makes the call fail with HE_EOOM at every
allocation point and leaves the context usable (the next result is still
bit-exact against the oracle), and a handle passed to a context it does not
belong to is refused before anything is enqueued."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_03152_amd import inputs as I
from tests.gpu_common import hip, say

pytestmark = pytest.mark.gpu

P = I.SMALL


class CountingAlloc:
    """torch's caching allocator on one stream, counting calls; from call
    number fail_from on (while armed) it returns NULL."""

    def __init__(self, H, stream):
        import torch
        self.torch, self.stream = torch, stream
        self.dev = torch.cuda.current_device()
        self.calls, self.fail_from, self.live = 0, None, {}
        self.a = H.Allocator(self.alloc, self.free)

    def alloc(self, n):
        self.calls += 1
        if self.fail_from is not None and self.calls >= self.fail_from:
            return None
        p = self.torch.cuda.caching_allocator_alloc(n, self.dev, self.stream)
        self.live[p] = n
        return p

    def free(self, p, n):
        assert self.live.pop(p) == n, "freed with another size"
        self.torch.cuda.caching_allocator_delete(p)


def _ctx(H, alloc, stream, seed=P["seed"], auto_rescale=True):
    return H.he_ctx_create(P["log_n"], P["bits"], P["scale"], seed, auto_rescale=auto_rescale,
                           stream=stream, allocator=alloc.a)


def test_default_allocator_is_torch():
    H = hip()
    import torch
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    g = H.he_ctx_create(P["log_n"], P["bits"], P["scale"], P["seed"])
    grown = torch.cuda.memory_allocated() - before
    # the NTT tables alone: 4 tables of N words per prime
    assert grown >= 4 * 8 * g.n * len(g.primes), grown
    g.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before


def test_eoom_in_context_creation_releases_everything():
    H = hip()
    import torch
    ts = torch.cuda.Stream()
    k = 1
    while True:
        al = CountingAlloc(H, ts.cuda_stream)
        al.fail_from = k
        try:
            g = _ctx(H, al, ts.cuda_stream)
        except H.HeError as e:
            assert e.code == H.HE_EOOM, e
            assert not al.live, "%d blocks not returned after a failed creation" % len(al.live)
            k += 1
            continue
        g.close()
        assert not al.live
        break
    say("context creation allocates %d blocks" % (k - 1))
    assert k > 2


def _oom_sweep(H, build, op, what):
    """For k = 1, 2, ...: a fresh context whose allocator fails from the
    k-th call made by `op` on: op must raise HE_EOOM, until k passes the
    number of calls op makes.  Returns the number of failure points."""
    import torch
    ts = torch.cuda.Stream()
    k = 1
    while True:
        al = CountingAlloc(H, ts.cuda_stream)
        st = build(al, ts.cuda_stream)
        al.fail_from = al.calls + k
        try:
            res = op(st)
        except H.HeError as e:
            assert e.code == H.HE_EOOM, "%s, failure at call %d: %s" % (what, k, e)
            # the context stays usable: the same operation now succeeds
            al.fail_from = None
            res = op(st)
            st["check"](res)
            del res, st
            k += 1
            continue
        st["check"](res)
        del res, st
        break
    say("%s: %d allocation failure points" % (what, k - 1))
    return k - 1


def test_eoom_mul_relin_then_bit_exact():
    H = hip()
    o = O.Oracle(P["log_n"], P["bits"], P["scale"], P["seed"])
    o.keygen()
    x, y, _ = I.small_vectors()
    ox = o.encrypt(o.encode(x, P["scale"], 1), 0, True)
    oy = o.encrypt(o.encode(y, P["scale"], 1), 1, True)
    want = o.rescale(o.mul_relin(ox, oy)).data()

    def build(al, stream):
        g = _ctx(H, al, stream)
        H.he_keygen(g, [])
        gx = H.he_encrypt(g, H.he_encode(g, x, P["scale"], 1), 0, True)
        gy = H.he_encrypt(g, H.he_encode(g, y, P["scale"], 1), 1, True)
        return {"g": g, "x": gx, "y": gy,
                "check": lambda r: np.testing.assert_array_equal(H.he_ct_export(g, r), want)}

    n = _oom_sweep(H, build, lambda s: H.he_mul_relin(s["g"], s["x"], s["y"]), "mul_relin")
    assert n >= 3


def test_eoom_matmul_then_bit_exact():
    H = hip()
    n_in, n_out = 16, 4
    bits = [60, 40, 40, 60]
    half = 2048
    rng = np.random.default_rng(33)
    W = rng.normal(0, 0.1, (n_in, n_out))
    b = rng.normal(0, 0.1, n_out)
    xv = rng.uniform(-1, 1, n_in)
    steps = sorted(set(I.replication_steps(n_in, half)) | set(range(1, n_in)))
    o = O.Oracle(12, bits, 2.0 ** 40, 9)
    o.keygen()
    for st in steps:
        o.galois_keygen(st)
    want = o.matmul(o.encrypt(o.encode(xv, 2.0 ** 40, 2), 4), W, b).data()

    def build(al, stream):
        g = H.he_ctx_create(12, bits, 2.0 ** 40, 9, auto_rescale=True, stream=stream, allocator=al.a)
        H.he_keygen(g, [])
        for st in steps:
            H.he_keygen_galois(g, st, -1)
        gx = H.he_encrypt(g, H.he_encode(g, xv, 2.0 ** 40, 2), 4, False)
        return {"g": g, "x": gx,
                "check": lambda r: np.testing.assert_array_equal(H.he_ct_export(g, r), want)}

    n = _oom_sweep(H, build, lambda s: H.he_enc_matmul(s["g"], s["x"], W, b), "enc_matmul")
    assert n >= 5


def test_foreign_handles_are_refused():
    H = hip()
    ga = H.he_ctx_create(P["log_n"], P["bits"], P["scale"], 41, auto_rescale=True)
    gb = H.he_ctx_create(P["log_n"], P["bits"], P["scale"], 42, auto_rescale=True)
    for g in (ga, gb):
        H.he_keygen(g, [1])
    x, y, p = I.small_vectors()
    ca = H.he_encrypt(ga, H.he_encode(ga, x, P["scale"], 1), 0, True)
    cb = H.he_encrypt(gb, H.he_encode(gb, y, P["scale"], 1), 0, True)
    pa = H.he_encode(ga, p, P["scale"], 1)
    calls = [
        ("add", lambda: H.he_add(gb, cb, ca)),
        ("mul_plain", lambda: H.he_mul_plain(gb, cb, pa)),
        ("mul_relin", lambda: H.he_mul_relin(gb, ca, cb)),
        ("rotate", lambda: H.he_rotate(gb, ca, 1)),
        ("rescale", lambda: H.he_rescale(gb, ca)),
        ("mul_relin_many", lambda: H.he_mul_relin_many(gb, [cb, ca], [cb, cb])),
        ("export", lambda: H.he_ct_export(gb, ca)),
        ("decrypt", lambda: H.he_decrypt(gb, ca)),
    ]
    for what, call in calls:
        with pytest.raises(H.HeError) as ei:
            call()
        assert ei.value.code == H.HE_EINVAL, what
        assert "another context" in str(ei.value), what
    # both contexts are untouched and keep working
    got = H.he_decode(gb, H.he_decrypt(gb, H.he_mul_relin(gb, cb, cb)), 2048)
    assert np.abs(got - y * y).max() < 1e-2
    got = H.he_decode(ga, H.he_decrypt(ga, H.he_add(ga, ca, ca)), 2048)
    assert np.abs(got - 2 * x).max() < 1e-2
    del ca, cb, pa
    ga.close()
    gb.close()
