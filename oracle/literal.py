"""The paper's own construction, evaluated literally -- a checker.

Test infrastructure: never imported by the product path.

Section 2.1 (and Remark 1 for polynomial lattice rules): take a primitive
element beta of the cyclic group (Z_N^* for prime N; the nonzero residues of
GF(2)[x]/p(x) for primitive p), write each generator component as
g_j = beta^(c_j - 1) with 1 <= c_j <= N-1, order the points as
x_0 = 0 and x_n = ({beta^(c_j - n) / N})_j for n = 1..N-1 (substituting the
conventional index by beta^-(n-1)), build the circulant Z with generator
z_k = phi({beta^k / N}) (Z[r][c] = z_{(c-r) mod (N-1)}) and the selection
matrix P (p_{k,j} = 1 iff k = c_j), so that Y' = Z P (eq. (ZPa)).  Y a is then
y_0 a = phi(x_0) sum_j a_j plus Z (P a) for the other rows.

Everything here is brute force: the primitive element is the smallest one
whose powers run through the whole group, c_j is found by scanning the list of
powers, and Z (P a) is a dense O(N^2) product.  The rows come out in the
paper's order and are mapped back to conventional order through the
substitution n -> beta^-(n-1).
"""
from __future__ import annotations

from fractions import Fraction
from typing import List

import numpy as np

from .points import RULE_LATTICE, RULE_POLY_GF2, phi_apply


class _Lattice:
    def __init__(self, N: int):
        self.N = N
        self.order = N - 1

    def mul(self, a: int, b: int) -> int:
        return a * b % self.N

    def coord(self, r: int, shift) -> float:
        num, den = shift
        return float(Fraction(r, self.N) + Fraction(num, den) - int(Fraction(r, self.N) + Fraction(num, den)))


class _GF2:
    def __init__(self, N: int, p: int):
        self.N = N
        self.m = N.bit_length() - 1
        self.p = p
        self.order = N - 1

    def mul(self, a: int, b: int) -> int:
        # schoolbook carry-less product, then reduction by p (pure Python ints)
        prod = 0
        for i in range(self.m):
            if (b >> i) & 1:
                prod ^= a << i
        for k in range(2 * self.m - 2, self.m - 1, -1):
            if (prod >> k) & 1:
                prod ^= self.p << (k - self.m)
        return prod

    def coord(self, r: int, shift) -> float:
        # digits of the Laurent expansion r(x)/p(x) = sum u_l x^-l, l = 1..m
        val = Fraction(0)
        rem = r
        for l in range(1, self.m + 1):
            rem <<= 1
            if (rem >> self.m) & 1:
                rem ^= self.p
                val += Fraction(1, 1 << l)
        num, den = shift
        v = val + Fraction(num, den)
        return float(v - int(v))


def _group(rule: int, N: int, modulus: int):
    return _Lattice(N) if rule == RULE_LATTICE else _GF2(N, modulus)


def powers(grp, beta: int) -> List[int]:
    out, x = [], 1
    for _ in range(grp.order):
        out.append(x)
        x = grp.mul(x, beta)
    return out


def primitive_element(grp) -> int:
    """Smallest element whose powers beta^0..beta^(order-1) are all distinct."""
    for beta in range(1, grp.N):
        pw = powers(grp, beta)
        if len(set(pw)) == grp.order:
            return beta
    raise ValueError("no primitive element (N not prime / p not primitive?)")


class Construction:
    """Beta, c_j, z, Z, P and the row maps of Section 2.1 for one instance."""

    def __init__(self, inst, beta: int = None):
        self.inst = inst
        grp = _group(inst.rule, inst.N, inst.modulus)
        self.grp = grp
        self.beta = primitive_element(grp) if beta is None else beta
        pw = powers(grp, self.beta)
        assert len(set(pw)) == grp.order, "beta is not primitive"
        self.pow = pw
        index = {v: k for k, v in enumerate(pw)}
        g = [int(v) for v in np.asarray(inst.gen)]
        # g_j = beta^(c_j - 1), 1 <= c_j <= N-1
        self.c = [index[gj] + 1 for gj in g]
        L = grp.order
        self.L = L
        coords = [grp.coord(pw[k], inst.shift) for k in range(L)]
        self.z = phi_apply(inst.phi, np.array(coords))
        r = np.arange(L)[:, None]
        cc = np.arange(L)[None, :]
        self.Z = self.z[(cc - r) % L]
        self.P = np.zeros((L, len(g)))
        for j, cj in enumerate(self.c):
            self.P[cj - 1, j] = 1.0
        self.y0 = float(phi_apply(inst.phi, np.array([grp.coord(0, inst.shift)]))[0])
        # paper row n (1..N-1) is the conventional point with index beta^-(n-1)
        beta_inv = pw[(L - 1) % L] if L > 1 else 1
        inv_pw = powers(grp, beta_inv)
        self.conv_index = [0] + [inv_pw[n - 1] for n in range(1, L + 1)]

    def Yprime(self) -> np.ndarray:
        """Y' = Z P, rows in the paper's order (points x_1..x_{N-1})."""
        return self.Z @ self.P

    def product(self, A=None) -> np.ndarray:
        """X = Y A in conventional row order, via y_0 a and Z (P a)."""
        A = np.asarray(self.inst.A if A is None else A, dtype=np.float64)
        X = np.empty((self.inst.N, A.shape[1]))
        X[0] = self.y0 * A.sum(axis=0)
        Pa = self.P @ A
        ZPa = self.Z @ Pa
        for n in range(1, self.L + 1):
            X[self.conv_index[n]] = ZPa[n - 1]
        return X
