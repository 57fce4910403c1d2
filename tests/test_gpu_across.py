"""Key switches batched across contexts (a server holding one context and
key set per client): every result equals, bit for bit, what the item's own
context gives one operation at a time (and, for one context, the oracle),
belongs to that context, and can be used there at once without
synchronisation; mismatched contexts are refused."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.gpu_common import hip, say

pytestmark = pytest.mark.gpu

LOG_N, BITS, SCALE = 12, [60, 40, 40, 60], 2.0 ** 40
STEPS = [1, 3, 5, 7]


def _client(H, seed):
    g = H.he_ctx_create(LOG_N, BITS, SCALE, seed, auto_rescale=True)
    H.he_keygen(g, STEPS)
    return g


def test_across_contexts_equal_own_context():
    H = hip()
    gs = [_client(H, 300 + c) for c in range(3)]
    rng = np.random.default_rng(9)
    cts = []  # (context index, ciphertext, plaintext)
    for i in range(10):
        c = i % 3
        v = rng.uniform(-1, 1, 2048)
        cts.append((c, H.he_encrypt(gs[c], H.he_encode(gs[c], v, SCALE, 2), 50 + i, False), v))
    a = [x for _, x, _ in cts]
    b = a[1:] + a[:1]
    # b[i] must share a[i]'s context: pair each with the next of the same context
    b = [next(y for (cj, y, _) in cts[i + 1:] + cts[:i + 1] if cj == ci) for i, (ci, _, _) in enumerate(cts)]
    say("mul_relin across 3 contexts")
    outs = H.he_mul_relin_across(gs[0], a, b)
    for (c, x, _), y, o in zip(cts, b, outs):
        assert o.ctx is gs[c]
        assert np.array_equal(H.he_ct_export(gs[c], o), H.he_ct_export(gs[c], H.he_mul_relin(gs[c], x, y)))
    say("rotate across 3 contexts")
    steps = [STEPS[i % 4] if i % 5 else 0 for i in range(len(a))]
    rots = H.he_rotate_across(gs[1], a, steps)
    for (c, x, v), st, o in zip(cts, steps, rots):
        assert np.array_equal(H.he_ct_export(gs[c], o), H.he_ct_export(gs[c], H.he_rotate(gs[c], x, st)))
    # results used at once on their own stream, no synchronisation between
    sums = [H.he_add(gs[c], o, o) for (c, _, _), o in zip(cts, rots)]
    for (c, _, v), st, sm in zip(cts, steps, sums):
        got = H.he_decode(gs[c], H.he_decrypt(gs[c], sm), 2048)
        assert np.abs(got - 2 * np.roll(v, -st)).max() < 1e-5
    # one context against the oracle
    c = 2
    o = O.Oracle(LOG_N, BITS, SCALE, 300 + c)
    o.keygen()
    for st in STEPS:
        o.galois_keygen(st)
    i = next(k for k, (ck, _, _) in enumerate(cts) if ck == c)
    ox = o.encrypt(o.encode(cts[i][2], SCALE, 2), 50 + i)
    assert np.array_equal(H.he_ct_export(gs[c], cts[i][1]), ox.data())
    assert np.array_equal(H.he_ct_export(gs[c], rots[i]), o.rotate(ox, steps[i]).data())
    oy = o.encrypt(o.encode(next(v for (ck, y, v) in cts if y is b[i]), SCALE, 2),
                   50 + next(k for k, (ck, y, _) in enumerate(cts) if y is b[i]))
    assert np.array_equal(H.he_ct_export(gs[c], outs[i]), o.rescale(o.mul_relin(ox, oy)).data())
    del a, b, outs, rots, sums, cts
    for g in gs:
        g.close()


def test_across_refuses_mismatched_contexts():
    H = hip()
    g1 = _client(H, 1)
    g2 = H.he_ctx_create(LOG_N, [60, 40, 60], SCALE, 2, auto_rescale=True)  # other primes
    H.he_keygen(g2, [1])
    x1 = H.he_encrypt(g1, H.he_encode(g1, np.ones(4), SCALE, 1), 0, True)
    x2 = H.he_encrypt(g2, H.he_encode(g2, np.ones(4), SCALE, 1), 0, True)
    with pytest.raises(H.HeError) as ei:
        H.he_mul_relin_across(g1, [x1, x2], [x1, x2])
    assert ei.value.code == H.HE_EINVAL
    with pytest.raises(H.HeError) as ei:  # operands of one item from two contexts
        H.he_mul_relin_across(g1, [x1], [x2])
    assert ei.value.code == H.HE_EINVAL
    # g1 unaffected: slots (1, 1, 1, 1, 0, ...) rotated left by one
    got = H.he_decode(g1, H.he_decrypt(g1, H.he_rotate_across(g1, [x1], [1])[0]), 4)
    assert np.abs(got - np.array([1, 1, 1, 0])).max() < 1e-3
    del x1, x2
    g1.close()
    g2.close()
