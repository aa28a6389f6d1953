"""Point sets in conventional order, written from their definitions.

Test infrastructure (see the package docstring): never imported by the
product path.

* Rank-1 lattice rule with prime N and generator g in (Z_N^*)^s
  (Section 2.1): x_{n,j} = { n g_j / N } for n = 0..N-1.  With an equal shift
  Delta = num/den in every coordinate (Remark 2) the coordinate is
  { n g_j / N + Delta }.  Computed from exact integers:
  x = ((n g_j mod N) den + num N) mod (N den) / (N den), one rounding.
* Polynomial lattice rule over GF(2) with N = 2^m (Remark 1; the paper gives
  no formulas, so the standard construction of Niederreiter is used): the
  index n is the polynomial n(x) = sum_i n_i x^i (bit i of n is the
  coefficient of x^i), r(x) = n(x) q_j(x) mod p(x), and the coordinate is
  nu_m(r/p) = sum_{l=1}^m u_l 2^-l where r(x)/p(x) = sum_{l>=1} u_l x^-l.
  Equivalently u_1..u_m are the bits (most significant first) of the
  quotient floor(r(x) x^m / p(x)).  The product path of the oracle
  (``coords_rational``, ``explicit_Y``) takes the digital-net form of the
  same points: digit l of x_{n,j} is sum_i n_i u_{i+l} (mod 2) with u_k the
  Laurent digits of q_j(x)/p(x) (the Hankel generating matrix), which is
  GF(2)-linear in n; ``gf2_coords`` keeps the direct route (product mod p,
  then the quotient) and the tests check that both agree bit for bit.
  An equal shift is applied as for lattices.
* Union of all Korobov lattice point sets with a prime K (Section 2.2, the
  point set of Hua and Wang): for b, n = 1..K-1 the point
  x_{b,n} = ({n b^0 / K}, {n b^1 / K}, ..., {n b^{s-1} / K}); conventional
  order is b-major, row (b-1)(K-1) + (n-1), N = (K-1)^2.  The coordinate of
  column j is taken for the exponent e_j given in ``gen`` (e_j = j for the
  point set itself; a subset of exponents selects columns).  The equal shift
  is applied as for lattices.
* phi (Section 2.1): identity, the tent transform 1 - |2x - 1|, the inverse
  normal CDF; and x - 1/2 (Experiment 2).
"""
from __future__ import annotations

import numpy as np
from scipy.special import ndtri

PHI_IDENTITY = 0
PHI_CENTERED = 1
PHI_INVNORM = 2
PHI_TENT = 3

RULE_LATTICE = 0
RULE_POLY_GF2 = 1
RULE_KOROBOV_UNION = 2


def phi_apply(kind: int, x: np.ndarray) -> np.ndarray:
    """The univariate map phi applied to floating coordinates x in [0, 1)."""
    x = np.asarray(x, dtype=np.float64)
    if kind == PHI_IDENTITY:
        return x.copy()
    if kind == PHI_CENTERED:
        return x - 0.5
    if kind == PHI_INVNORM:
        return ndtri(x)
    if kind == PHI_TENT:
        return 1.0 - np.abs(2.0 * x - 1.0)
    raise ValueError(f"unknown phi kind {kind}")


def phi_rational(kind: int, K: np.ndarray, D: int) -> np.ndarray:
    """phi of the exact coordinate K/D (integers, 0 <= K < D), rounded once:
    identity K/D, centered (2K-D)/(2D), tent (D-|2K-D|)/D; the inverse normal
    CDF is evaluated on the nearer tail, -Phi^-1((D-K)/D) when K/D > 1/2, so
    the complement is exact."""
    K = np.asarray(K, dtype=np.int64)
    fD = float(D)
    if kind == PHI_IDENTITY:
        return K.astype(np.float64) / fD
    if kind == PHI_CENTERED:
        return (2 * K - D).astype(np.float64) / (2.0 * fD)
    if kind == PHI_TENT:
        return (D - np.abs(2 * K - D)).astype(np.float64) / fD
    if kind == PHI_INVNORM:
        upper = 2 * K > D
        lo = np.where(upper, D - K, K).astype(np.float64) / fD
        y = ndtri(lo)
        return np.where(upper, -y, y)
    raise ValueError(f"unknown phi kind {kind}")


def _shifted_numer(numer: np.ndarray, N: int, shift):
    """{ numer/N + num/den } as the exact fraction K/D with D = N den."""
    num, den = int(shift[0]), int(shift[1])
    D = N * den
    assert D < (1 << 62), "shifted coordinate denominator too large"
    K = (np.asarray(numer, dtype=np.int64) * den + num * N) % D
    return K, D


def _shifted_fraction(numer: np.ndarray, N: int, shift) -> np.ndarray:
    K, D = _shifted_numer(numer, N, shift)
    return K.astype(np.float64) / float(D)


def lattice_coords(N: int, gen, shift=(0, 1), rows=None) -> np.ndarray:
    """Coordinates {n g_j / N + Delta} for the given rows n (default 0..N-1)."""
    g = np.asarray(gen, dtype=np.int64)
    n = np.arange(N, dtype=np.int64) if rows is None else np.asarray(rows, dtype=np.int64)
    resid = (n[:, None] * g[None, :]) % N
    return _shifted_fraction(resid, N, shift)


# ---- GF(2) polynomial arithmetic, vectorised over numpy uint64 arrays ------

def _clmul(a: np.ndarray, b: np.ndarray, nbits: int) -> np.ndarray:
    """Carry-less (GF(2)[x]) product of a and b, where b has < nbits bits."""
    a = a.astype(np.uint64)
    b = b.astype(np.uint64)
    r = np.zeros(np.broadcast(a, b).shape, dtype=np.uint64)
    for i in range(nbits):
        bit = (b >> np.uint64(i)) & np.uint64(1)
        r ^= np.where(bit == 1, a << np.uint64(i), np.uint64(0))
    return r


def _poly_divmod(a: np.ndarray, p: int, abits: int):
    """Quotient and remainder of a(x) by p(x) over GF(2); a has < abits bits."""
    m = int(p).bit_length() - 1
    a = a.astype(np.uint64).copy()
    q = np.zeros_like(a)
    pp = np.uint64(p)
    for k in range(abits - 1 - m, -1, -1):
        top = (a >> np.uint64(m + k)) & np.uint64(1)
        a ^= np.where(top == 1, pp << np.uint64(k), np.uint64(0))
        q |= np.where(top == 1, np.uint64(1) << np.uint64(k), np.uint64(0))
    return q, a


def gf2_residues(m: int, p: int, gen, rows=None) -> np.ndarray:
    """r = n(x) q_j(x) mod p(x) for the given rows n (default 0..2^m-1)."""
    N = 1 << m
    q = np.asarray(gen, dtype=np.uint64)
    n = np.arange(N, dtype=np.uint64) if rows is None else np.asarray(rows, dtype=np.uint64)
    prod = _clmul(n[:, None], q[None, :], m)
    _, r = _poly_divmod(prod, p, 2 * m)
    return r


def gf2_value_of_residue(m: int, p: int, r: np.ndarray) -> np.ndarray:
    """Integer Q with Q/2^m = nu_m(r/p): the quotient floor(r(x) x^m / p(x))."""
    q, _ = _poly_divmod(np.asarray(r, dtype=np.uint64) << np.uint64(m), p, 2 * m)
    return q


def gf2_laurent_digits(p: int, q, count: int) -> np.ndarray:
    """The first ``count`` digits u_1..u_count of the Laurent expansion
    q(x)/p(x) = sum_{l>=1} u_l x^-l over GF(2), deg q < deg p, by long
    division (u_l = 1 when x times the remainder reaches degree m).  Row l-1
    of the result holds u_l for every q."""
    m = int(p).bit_length() - 1
    rem = np.asarray(q, dtype=np.uint64).copy()
    out = np.zeros((count,) + rem.shape, dtype=np.uint64)
    pp = np.uint64(p)
    for l in range(count):
        rem = rem << np.uint64(1)
        u = (rem >> np.uint64(m)) & np.uint64(1)
        rem ^= np.where(u == 1, pp, np.uint64(0))
        out[l] = u
    return out


def gf2_numerators_digital(m: int, p: int, gen, rows=None) -> np.ndarray:
    """Integer Q with Q/2^m = nu_m(n(x) q_j(x) / p(x)) for the requested rows,
    from the digital-net form of the polynomial lattice rule: with n_i the
    bit i of n and u_k the Laurent digits of q_j/p, the coefficient of
    x^-l in n(x) q_j(x)/p(x) is sum_i n_i u_{i+l} (mod 2).  Reducing
    n(x) q_j(x) modulo p(x) first only removes a polynomial part, which has no
    negative powers, so these are the digits of the point; digit l = 1 is the
    most significant.  So Q is the XOR over the set bits i of n of the m-bit
    word (u_{i+1} .. u_{i+m}) (the columns of the Hankel generating matrix)."""
    q = np.asarray(gen, dtype=np.uint64)
    N = 1 << m
    n = np.arange(N, dtype=np.uint64) if rows is None else np.asarray(rows, dtype=np.uint64)
    u = gf2_laurent_digits(p, q, 2 * m - 1)          # u[k-1] = u_k, shape (2m-1, s)
    basis = np.zeros((m,) + q.shape, dtype=np.uint64)  # basis[i] = word of n = x^i
    for i in range(m):
        for l in range(1, m + 1):
            basis[i] |= u[i + l - 1] << np.uint64(m - l)
    Q = np.zeros((len(n),) + q.shape, dtype=np.uint64)
    for i in range(m):
        bit = ((n >> np.uint64(i)) & np.uint64(1)) == 1
        Q ^= np.where(bit[:, None], basis[i][None, :], np.uint64(0))
    return Q


def gf2_coords(m: int, p: int, gen, shift=(0, 1), rows=None) -> np.ndarray:
    """Coordinates nu_m(n(x) q_j(x) / p(x)) (+ Delta, mod 1)."""
    r = gf2_residues(m, p, gen, rows)
    Q = gf2_value_of_residue(m, p, r).astype(np.int64)
    return _shifted_fraction(Q, 1 << m, shift)


def gf2_digits_coords(m: int, p: int, gen, rows=None) -> np.ndarray:
    """Second route to the GF(2) coordinates (no shift): the digits u_l of the
    Laurent expansion r/p are read off one at a time by long division of the
    remainder (u_l = 1 when x * remainder reaches degree m)."""
    r = gf2_residues(m, p, gen, rows)
    rem = r.copy()
    val = np.zeros(r.shape, dtype=np.float64)
    scale = 0.5
    pp = np.uint64(p)
    for _ in range(m):
        rem = rem << np.uint64(1)
        u = (rem >> np.uint64(m)) & np.uint64(1)
        rem ^= np.where(u == 1, pp, np.uint64(0))
        val += u.astype(np.float64) * scale
        scale *= 0.5
    return val


def _powmod(base: np.ndarray, exp: np.ndarray, K: int) -> np.ndarray:
    """base^exp mod K elementwise (square and multiply; K < 2^31)."""
    base = np.asarray(base, dtype=np.int64) % K
    exp = np.asarray(exp, dtype=np.int64).copy()
    base, exp = np.broadcast_arrays(base, exp)
    base, exp = base.copy(), exp.copy()
    out = np.ones(base.shape, dtype=np.int64)
    while np.any(exp > 0):
        odd = (exp & 1) == 1
        out = np.where(odd, out * base % K, out)
        base = base * base % K
        exp >>= 1
    return out


def korobov_union_numerators(K: int, exps, rows=None) -> np.ndarray:
    """(n b^{e_j}) mod K for the requested rows (b, n) of the union."""
    N = (K - 1) ** 2
    rho = np.arange(N, dtype=np.int64) if rows is None else np.asarray(rows, dtype=np.int64)
    b = rho // (K - 1) + 1
    n = rho % (K - 1) + 1
    e = np.asarray(exps, dtype=np.int64)
    return n[:, None] * _powmod(b[:, None], e[None, :], K) % K


def unshifted_numerators(rule: int, N: int, gen, modulus: int = 0, rows=None):
    """(numerators, base) of the unshifted coordinates numer/base of the
    requested rows: n g_j mod N (lattice), the digit value Q of
    nu_m(n q_j / p) (GF(2), digital-net form), n b^{e_j} mod K (union of
    Korobov rules, base K).  Every numerator lies in [0, base)."""
    if rule == RULE_LATTICE:
        g = np.asarray(gen, dtype=np.int64)
        n = np.arange(N, dtype=np.int64) if rows is None else np.asarray(rows, dtype=np.int64)
        return (n[:, None] * g[None, :]) % N, N
    if rule == RULE_POLY_GF2:
        m = int(N).bit_length() - 1
        assert 1 << m == N, "polynomial lattice rules need N = 2^m"
        return gf2_numerators_digital(m, modulus, gen, rows).astype(np.int64), N
    if rule == RULE_KOROBOV_UNION:
        K = int(modulus)
        assert N == (K - 1) ** 2, "the union of Korobov rules has (K-1)^2 points"
        return korobov_union_numerators(K, gen, rows), K
    raise ValueError(f"unknown rule {rule}")


def coords_rational(rule: int, N: int, gen, modulus: int = 0, shift=(0, 1), rows=None):
    """Exact coordinates K/D of the requested rows (conventional order)."""
    numer, base = unshifted_numerators(rule, N, gen, modulus, rows)
    return _shifted_numer(numer, base, shift)


def coords(rule: int, N: int, gen, modulus: int = 0, shift=(0, 1), rows=None) -> np.ndarray:
    if rule == RULE_LATTICE:
        return lattice_coords(N, gen, shift, rows)
    if rule == RULE_POLY_GF2:
        m = int(N).bit_length() - 1
        assert 1 << m == N, "polynomial lattice rules need N = 2^m"
        return gf2_coords(m, modulus, gen, shift, rows)
    if rule == RULE_KOROBOV_UNION:
        K, D = coords_rational(rule, N, gen, modulus, shift, rows)
        return K.astype(np.float64) / float(D)
    raise ValueError(f"unknown rule {rule}")


def explicit_Y(rule: int, N: int, gen, phi: int, modulus: int = 0, shift=(0, 1),
               rows=None) -> np.ndarray:
    """Y[n, j] = phi(x_{n,j}) in conventional row order, FP64 (phi of the
    exact rational coordinate, rounded once).  The shifted coordinate, and so
    its phi value, depends only on the unshifted numerator in [0, base): when
    there are more entries than numerators, phi is evaluated once per
    numerator (the same exact rational, the same rounding) and looked up."""
    numer, base = unshifted_numerators(rule, N, gen, modulus, rows)
    if numer.size <= base:
        K, D = _shifted_numer(numer, base, shift)
        return phi_rational(phi, K, D)
    K, D = _shifted_numer(np.arange(base, dtype=np.int64), base, shift)
    return phi_rational(phi, K, D)[numer]


def phi_residue_values(rule: int, N: int, phi: int, modulus: int = 0,
                       shift=(0, 1)) -> np.ndarray:
    """The value of phi for every one-dimensional point: entry r is phi of the
    coordinate of residue r (lattice: {r/N + Delta}; GF(2): nu_m(r/p) + Delta).
    Obtained as the column of Y for the generator component 1."""
    return explicit_Y(rule, N, np.array([1], dtype=np.uint64), phi, modulus, shift)[:, 0]
