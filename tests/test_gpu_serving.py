"""The continuous-batching request loop: every request's result is the same
ciphertext alone and in a mix of CNN and logistic-regression requests from
two clients, the decrypted results match plaintext arithmetic, and one CNN
and one logistic-regression request of the mix equal, bit for bit, the
oracle run with that client's seed, keys and encryption indices."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_03152_amd import inputs as I
from tests.gpu_common import hip, say
from tests.plain_ref import cnn_fp64

pytestmark = pytest.mark.gpu


def test_alone_equals_mix():
    H = hip()
    from paper_2104_03152_amd import serve as S
    d = I.cnn_inputs()
    say("clients")
    clients = [S.Client(H, c, d) for c in range(2)]
    reqs = S.make_requests(H, clients, 8, 0, seed=5, per_client=4)
    kinds = [r.kind for r in reqs]
    assert "cnn" in kinds and "lr" in kinds
    say("mix")
    lat = S.serve(H, reqs, 4 << 30, batched=True)
    assert len(lat) == 8
    mix = {r.rid: H.he_ct_export(r.client.g, r.out) for r in reqs}
    for r in reqs:
        g = r.client.g
        if r.kind == "cnn":
            got = H.he_decode(g, H.he_decrypt(g, r.out), 10)
            assert np.abs(got - cnn_fp64(d, r.extra["img"])).max() < 1e-3
        else:
            got = H.he_decode(g, H.he_decrypt(g, r.out), 1)[0]
            assert abs(got - (r.extra["w"] @ r.extra["x"] + r.extra["b"])) < 1e-3
    say("oracle for one client")
    check_against_oracle(H, S, clients, reqs, mix)
    say("alone")
    for r in reqs:
        S.reset([r])
        S.serve(H, [r], 4 << 30, batched=True)
        assert np.array_equal(H.he_ct_export(r.client.g, r.out), mix[r.rid]), "request %d" % r.rid
    say("one at a time")
    S.reset(reqs)
    S.serve(H, reqs, 4 << 30, batched=False)
    for r in reqs:
        assert np.array_equal(H.he_ct_export(r.client.g, r.out), mix[r.rid]), "request %d" % r.rid
    del reqs, lat  # every handle before its context
    for c in clients:
        c.close()


def check_against_oracle(H, S, clients, reqs, mix):
    # a client with both kinds of request (else the first CNN request's)
    by_client = {}
    for r in reqs:
        by_client.setdefault(r.client.cid, {}).setdefault(r.kind, r)
    cid = next((c for c, k in by_client.items() if len(k) == 2), None)
    assert cid is not None, "no client with both request kinds"
    client = next(c for c in clients if c.cid == cid)
    g = client.g
    o = O.Oracle(13, S.CNN_BITS, S.SCALE, 1000 + cid)
    o.keygen()
    levels = dict(I.cnn_rotation_steps())
    for st in S.lr_steps(1024):
        levels[st] = max(levels.get(st, -1), o.L - 2)
    for st, lv in sorted(levels.items()):
        o.galois_keygen(st, lv)
    assert o.primes == g.primes
    d = I.cnn_inputs()
    cnn = by_client[cid]["cnn"]
    v = H.he_im2col(cnn.extra["img"], 7, 3)
    ox = o.encrypt(o.encode(v, S.SCALE, o.L - 1), 10_000 + cnn.rid)
    assert np.array_equal(H.he_ct_export(g, cnn.ct), ox.data()), "cnn input"
    say("oracle cnn (request %d)" % cnn.rid)
    oy = o.cnn(ox, d["conv_k"], d["conv_b"], d["w1"], d["b1"], d["w2"], d["b2"])
    assert np.array_equal(mix[cnn.rid], oy.data()), "cnn request %d" % cnn.rid
    lr = by_client[cid]["lr"]
    e = lr.extra
    ox = o.encrypt(o.encode(e["x"], S.SCALE, o.L - 1), 10_000 + lr.rid)
    assert np.array_equal(H.he_ct_export(g, lr.ct), ox.data()), "lr input"
    say("oracle lr (request %d, d=%d)" % (lr.rid, e["d"]))
    y = o.rescale(o.mul_plain(ox, o.encode(e["w"], S.SCALE, o.L - 1)))
    for st in S.lr_steps(e["d"]):
        y = o.add(y, o.rotate(y, st))
    bvec = np.zeros(o.n // 2)
    bvec[0] = e["b"]
    y = o.add_plain(y, o.encode(bvec, S.SCALE * S.SCALE / g.primes[o.L - 1], o.L - 2))
    assert np.array_equal(mix[lr.rid], y.data()), "lr request %d" % lr.rid
