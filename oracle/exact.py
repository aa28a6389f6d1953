"""Brute force over exact rationals for tiny N -- a checker.

Test infrastructure: never imported by the product path.

For phi = identity or x - 1/2 every entry of Y is rational, so X = Y A can be
formed exactly with ``fractions.Fraction`` (A's binary floats are exact
rationals).  Lattice coordinates are {n g_j / N} (Section 2.1); GF(2)
coordinates are the first m digits of the Laurent expansion of
n(x) q_j(x) / p(x) (Remark 1), found here with plain Python integers by
repeated doubling of n(x) (n(x) q(x) = sum over set bits i of q of x^i n(x));
the union of Korobov rules has {n b^e_j / K} in row (b-1)(K-1) + (n-1)
(Section 2.2), with Python's built-in modular power.
"""
from __future__ import annotations

from fractions import Fraction
from typing import List

import numpy as np

from .points import PHI_CENTERED, PHI_IDENTITY, RULE_KOROBOV_UNION, RULE_LATTICE


def _gf2_point(m: int, p: int, n: int, q: int) -> Fraction:
    # r = n(x) q(x) mod p(x): add x^i n(x) (reduced) for each set bit i of q
    r, term = 0, n
    for i in range(m):
        if (q >> i) & 1:
            r ^= term
        term <<= 1
        if (term >> m) & 1:
            term ^= p
    val, rem = Fraction(0), r
    for l in range(1, m + 1):
        rem <<= 1
        if (rem >> m) & 1:
            rem ^= p
            val += Fraction(1, 1 << l)
    return val


def point_matrix(inst) -> List[List[Fraction]]:
    assert inst.phi in (PHI_IDENTITY, PHI_CENTERED)
    num, den = inst.shift
    shift = Fraction(int(num), int(den))
    off = Fraction(1, 2) if inst.phi == PHI_CENTERED else Fraction(0)
    g = [int(v) for v in np.asarray(inst.gen)]
    rows = []
    for n in range(inst.N):
        row = []
        for gj in g:
            if inst.rule == RULE_LATTICE:
                x = Fraction((n * gj) % inst.N, inst.N)
            elif inst.rule == RULE_KOROBOV_UNION:
                K = int(inst.modulus)
                b, k = n // (K - 1) + 1, n % (K - 1) + 1
                x = Fraction(k * pow(b, gj, K) % K, K)
            else:
                x = _gf2_point(inst.N.bit_length() - 1, inst.modulus, n, gj)
            x = x + shift
            x = x - int(x)
            row.append(x - off)
        rows.append(row)
    return rows


def product(inst, A=None) -> List[List[Fraction]]:
    A = np.asarray(inst.A if A is None else A, dtype=np.float64)
    Af = [[Fraction(float(v)) for v in row] for row in A]
    Y = point_matrix(inst)
    t = A.shape[1]
    return [[sum((Y[n][j] * Af[j][c] for j in range(len(Af))), Fraction(0))
             for c in range(t)] for n in range(inst.N)]
