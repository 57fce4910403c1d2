"""Python big-integer helpers for the pins (test side only): CRT
reconstruction, centring and schoolbook negacyclic products over Z."""
import numpy as np


def crt(limbs, primes):
    """limbs [L][N] residues -> list of N ints in [0, prod(primes))."""
    Q = 1
    for q in primes:
        Q *= q
    out = [0] * len(limbs[0])
    for i, q in enumerate(primes):
        qh = Q // q
        f = qh * pow(qh % q, -1, q)
        col = limbs[i]
        for k in range(len(out)):
            out[k] += int(col[k]) * f
    return [x % Q for x in out], Q


def centered(x, Q):
    return [v - Q if v > Q // 2 else v for v in x]


def residues(x, primes):
    return np.array([[v % q for v in x] for q in primes], dtype=np.uint64)


def negacyclic_int(a, b):
    """schoolbook product of integer polynomials mod X^N + 1 over Z"""
    n = len(a)
    c = [0] * n
    for i in range(n):
        ai = a[i]
        if not ai:
            continue
        for j in range(n):
            k = i + j
            if k < n:
                c[k] += ai * b[j]
            else:
                c[k - n] -= ai * b[j]
    return c
