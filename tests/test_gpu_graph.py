"""Captured graphs: a fixed sequence of library calls (fused key switches,
rotate-and-sum, the hoisted vector-matrix product, rescales, device copies)
captured once and replayed.  Every replay must equal the eager result bit
for bit — with eager work and synchronisations between replays, and after
new input data is copied into the captured input."""
import numpy as np
import pytest

from paper_2104_03152_amd import inputs as I
from tests.gpu_common import Pair, say

pytestmark = pytest.mark.gpu


def pipeline(H, g, x, plan, gp):
    y = H.he_mul_relin(g, x, x)                 # relinearise + rescale
    y = H.he_add(g, y, H.he_rotate(g, y, 1))   # fused key switch
    y = H.he_sum_slots(g, y, 8)                 # rotate-and-sum chain
    y = H.he_mul_plain(g, y, gp)                # rescale
    return H.he_plan_apply(g, plan, y)          # hoisted rotations


def test_graph_replays_match_eager():
    P = Pair(12, [60, 40, 40, 40, 40, 60], 2.0 ** 40, 12, auto_rescale=True)
    H, g = P.H, P.g
    rng = np.random.default_rng(12)
    # rotations: 1, 2, 4 (sum of 8 slots), 1..15 (the hoisted product of a
    # 16-input matrix) and its replication steps
    steps = sorted(set([1, 2, 4] + list(range(1, 16)) + I.replication_steps(16, 2048)))
    for st in steps:
        H.he_keygen_galois(g, st, -1)
    W = rng.normal(0, 0.1, (16, 6))
    x1, x2 = rng.uniform(-1, 1, 2048), rng.uniform(-1, 1, 2048)
    top = 4
    c1 = H.he_encrypt(g, H.he_encode(g, x1, P.scale, top), 1, False)
    c2 = H.he_encrypt(g, H.he_encode(g, x2, P.scale, top), 2, False)
    # the product is at level 3 after its rescale; the plaintext product
    # rescales to level 2, where the plan applies
    gp = H.he_encode(g, rng.uniform(-1, 1, 2048), P.scale, 3)
    probe = H.he_mul_plain(g, H.he_sum_slots(g, H.he_mul_relin(g, c1, c1), 8), gp)
    plan = H.he_matmul_plan(g, probe, W)
    say("eager")
    ref1 = H.he_ct_export(g, pipeline(H, g, c1, plan, gp))
    ref2 = H.he_ct_export(g, pipeline(H, g, c2, plan, gp))
    xin = H.he_drop_to(g, c1, top)  # the graph's input
    say("capture")
    H.he_graph_begin(g)
    out = pipeline(H, g, xin, plan, gp)
    graph = H.he_graph_end(g)
    for rep in range(4):
        H.he_graph_launch(g, graph)
        H.he_sync(g)
        assert np.array_equal(H.he_ct_export(g, out), ref1), "replay %d" % rep
        # eager work between replays, on the same stream
        assert np.array_equal(H.he_ct_export(g, pipeline(H, g, c2, plan, gp)), ref2)
    H.he_ct_copy(g, xin, c2)
    for rep in range(3):
        H.he_graph_launch(g, graph)
        H.he_sync(g)
        assert np.array_equal(H.he_ct_export(g, out), ref2), "replay %d on new input" % rep
    graph.free()
    # the graph's intermediates are back in the pool; eager results still hold
    assert np.array_equal(H.he_ct_export(g, pipeline(H, g, c1, plan, gp)), ref1)


def test_graph_capture_refuses_synchronising_calls():
    P = Pair(12, [40, 20, 40], 2.0 ** 20, 1)
    H, g = P.H, P.g
    # secret-key encryption at scale 2^20: slot noise about 1e-4
    x = H.he_encrypt(P.g, H.he_encode(g, np.ones(8), P.scale, 1), 0, True)
    H.he_graph_begin(g)
    with pytest.raises(P.H.HeError):
        H.he_graph_begin(g)  # nested
    with pytest.raises(P.H.HeError):
        H.he_ct_export(g, x)  # would synchronise: refused before any HIP call
    with pytest.raises(P.H.HeError):
        H.he_sync(g)
    y = H.he_add(g, x, x)
    graph = H.he_graph_end(g)
    H.he_graph_launch(g, graph)
    H.he_sync(g)
    assert np.abs(H.he_decode(g, H.he_decrypt(g, y), 8) - 2).max() < 1e-2
    graph.free()
