"""Seeded synthetic workloads shared by the tests, the oracle runs and bench.py.

This module holds parameter sets and random draws only: no encoding, no
modular arithmetic, nothing of the method.  The MNIST images and trained
weights of the paper's evaluation (section 5) are not available; the shapes
here stand in for them: a 28x28 image with pixels uniform in [0, 1], and
weights and biases drawn N(0, 0.1^2).
"""
import numpy as np

# Parameter sets: ring degree 2^log_n, prime bit sizes (data primes, then the
# key-switching special prime), encoding scale, sampler seed.
SMALL = dict(name="ckks-n4096-3primes", log_n=12, bits=[40, 20, 40], scale=2.0 ** 20, seed=1)
CNN = dict(name="ckks-n8192-8primes", log_n=13, bits=[60] + [40] * 6 + [60], scale=2.0 ** 40,
           seed=2)
RAW = dict(name="ckks-n16384-9x50bit", log_n=14, bits=[50] * 9, scale=2.0 ** 40, seed=3)

# MNIST-shaped network of section 5: conv 4 kernels 7x7 stride 3 on 28x28,
# square, FC 256 -> 64, square, FC 64 -> 10.
CNN_SHAPE = dict(img=28, k=7, stride=3, channels=4, windows=64, hidden=64, out=10)


def small_vectors(n=2048, seed=1):
    """x, y, p ~ U[-1, 1]^n drawn in that order."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, n)
    y = rng.uniform(-1.0, 1.0, n)
    p = rng.uniform(-1.0, 1.0, n)
    return x, y, p


def cnn_inputs(seed=2):
    """image, conv kernels [4][49], conv bias [4], W1 [256][64], b1 [64],
    W2 [64][10], b2 [10]; drawn in that order."""
    s = CNN_SHAPE
    rng = np.random.default_rng(seed)
    img = rng.uniform(0.0, 1.0, (s["img"], s["img"]))
    conv_k = rng.normal(0.0, 0.1, (s["channels"], s["k"] * s["k"]))
    conv_b = rng.normal(0.0, 0.1, s["channels"])
    w1 = rng.normal(0.0, 0.1, (s["channels"] * s["windows"], s["hidden"]))
    b1 = rng.normal(0.0, 0.1, s["hidden"])
    w2 = rng.normal(0.0, 0.1, (s["hidden"], s["out"]))
    b2 = rng.normal(0.0, 0.1, s["out"])
    return dict(img=img, conv_k=conv_k, conv_b=conv_b, w1=w1, b1=b1, w2=w2, b2=b2)


def replication_steps(n_in, n_slots):
    """Left-rotation steps that replicate an n_in-vector R times (R the
    largest power of two with n_in * R <= n_slots): right rotations by
    n_in * m, m = 1..R-1."""
    reps = 1
    while n_in * reps * 2 <= n_slots:
        reps *= 2
    return [n_slots - n_in * m for m in range(1, reps)]


def cnn_rotation_steps(n_slots=4096):
    """Left-rotation steps the MNIST-shaped network uses, each with the
    highest level it is used at (levels counted as in a 7-data-prime chain:
    the input is at level 6).  Conv sums at level 5, packing at level 4,
    FC1 (replication + 255 diagonals) at level 3, FC2 at level 1."""
    s = CNN_SHAPE
    levels = {}

    def use(step, level):
        step %= n_slots
        if step:
            levels[step] = max(levels.get(step, -1), level)

    win = s["windows"]
    for j in range(6):                      # conv: 49 blocks of 64 windows
        use(win << j, 5)
    for c in range(1, s["channels"]):       # channel packing: right by 64c
        use(n_slots - win * c, 4)
    n_in = s["channels"] * win
    for st in replication_steps(n_in, n_slots):   # FC1 replication
        use(st, 3)
    for i in range(1, n_in):                # FC1 diagonals
        use(i, 3)
    n_in = s["hidden"]
    for st in replication_steps(n_in, n_slots):   # FC2 replication
        use(st, 1)
    for i in range(1, n_in):                # FC2 diagonals
        use(i, 1)
    return levels


def raw_residues(primes, n_ct, n_limbs, n, seed=3):
    """n_ct ciphertexts [n_ct][2][n_limbs][n] of residues uniform in [0, q_i)."""
    rng = np.random.default_rng(seed)
    out = np.empty((n_ct, 2, n_limbs, n), dtype=np.uint64)
    for i in range(n_limbs):
        out[:, :, i, :] = rng.integers(0, primes[i], size=(n_ct, 2, n), dtype=np.uint64)
    return out


def residues(primes, shape_prefix, n, seed):
    """array [*shape_prefix][len(primes)][n] uniform below each prime."""
    rng = np.random.default_rng(seed)
    out = np.empty(tuple(shape_prefix) + (len(primes), n), dtype=np.uint64)
    for i, q in enumerate(primes):
        out[..., i, :] = rng.integers(0, q, size=tuple(shape_prefix) + (n,), dtype=np.uint64)
    return out
