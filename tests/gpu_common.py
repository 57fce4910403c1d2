"""Helpers shared by the GPU parity tests: matching oracle and HIP contexts
built from the same parameters and seed."""
import sys

import numpy as np
import pytest

from oracle import oracle as O


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def hip():
    """The HIP binding; skips (never falls back) when no GPU is visible."""
    import paper_2104_03152_amd as H
    try:
        import torch
        if not torch.cuda.is_available():
            pytest.skip("no GPU visible")
    except ImportError:
        pytest.skip("torch missing")
    H.lib()  # raises if the library is not built
    return H


class Pair:
    """An oracle context and a HIP context with identical parameters/keys."""

    def __init__(self, log_n, bits, scale, seed, steps=(), step_levels=None, auto_rescale=False):
        self.H = hip()
        say("pair: log_n=%d bits=%s seed=%d" % (log_n, bits, seed))
        self.o = O.Oracle(log_n, bits, scale, seed)
        self.o.keygen()
        self.g = self.H.he_ctx_create(log_n, bits, scale, seed, auto_rescale=auto_rescale, stream=None)
        self.H.he_keygen(self.g, [])
        for st in steps:
            self.o.galois_keygen(st)
            self.H.he_keygen_galois(self.g, st, -1)
        for st, lv in (step_levels or {}).items():
            self.o.galois_keygen(st, lv)
            self.H.he_keygen_galois(self.g, st, lv)
        assert self.g.primes == self.o.primes
        self.n = self.o.n
        self.scale = scale

    def ct_equal(self, gct, oct_, what):
        got = self.H.he_ct_export(self.g, gct)
        want = oct_.data()
        lv, sc = gct.info()
        assert lv == oct_.level, "%s: level %d vs %d" % (what, lv, oct_.level)
        assert sc == oct_.scale, "%s: scale %r vs %r" % (what, sc, oct_.scale)
        if not np.array_equal(got, want):
            bad = np.argwhere(got != want)
            raise AssertionError("%s: %d of %d residues differ, first at %s: %d vs %d" % (
                what, len(bad), got.size, tuple(bad[0]), got[tuple(bad[0])], want[tuple(bad[0])]))

    def pt_equal(self, gpt, opt, what):
        got, lv, sc = self.H.he_pt_export(self.g, gpt)
        want = opt.data()
        assert lv == opt.level and sc == opt.scale, what
        if not np.array_equal(got, want):
            bad = np.argwhere(got != want)
            raise AssertionError("%s: %d residues differ, first at %s" % (what, len(bad), tuple(bad[0])))
