"""The continuous-batching request loop: every request's result is the same
ciphertext alone and in a mix of CNN and logistic-regression requests from
two clients, and the decrypted results match plaintext arithmetic."""
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
