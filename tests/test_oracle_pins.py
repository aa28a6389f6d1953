"""Pins of the CPU oracle against what the paper and the mathematics fix.

No GPU.  Each check is chosen so that a plausible slip in the oracle (a
dropped shift, a wrong index, a transposed operand, a wrong digit order)
fails at least one of them; ``test_planted_mistakes_are_caught`` plants such
slips in copies of the oracle and checks that the pins notice.
"""
import dataclasses
import json
import math
import os
import statistics
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import literal, exact
import qmc_inputs as qi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _inst(rule, N, gen, phi, A=None, modulus=0, shift=(0, 1), t=2, seed=0):
    gen = np.asarray(gen, dtype=np.uint64)
    if A is None:
        A = np.random.default_rng(seed).standard_normal((len(gen), t))
    return qi.Instance("pin", rule, N, len(gen), A.shape[1], gen, modulus, phi,
                       shift, "f64", np.asarray(A, dtype=np.float64))


# ---------------------------------------------------------------------------
# Example 1 (Section 2.1): printed values
# ---------------------------------------------------------------------------

def _example():
    with open(os.path.join(GOLDEN, "example_n7.json")) as f:
        return json.load(f)


def test_example1_conventional_points():
    ex = _example()
    x = oracle.lattice_coords(ex["N"], ex["gen"])
    assert np.array_equal(np.rint(x * ex["N"]).astype(int), np.array(ex["conventional_numerators_over_N"]))
    # the coordinates are exactly k/7 rounded once
    assert np.array_equal(x, np.array(ex["conventional_numerators_over_N"]) / 7.0)


def test_example1_paper_construction():
    ex = _example()
    inst = _inst(qi.RULE_LATTICE, ex["N"], ex["gen"], qi.PHI_IDENTITY)
    con = literal.Construction(inst)
    assert con.beta == ex["beta"]
    assert con.c == ex["c"]
    assert con.pow[(con.L - 1) % con.L] == ex["beta_inverse"]
    assert np.array_equal(np.rint(con.Z * 7).astype(int), np.array(ex["Z_numerators_over_N"]))
    assert np.array_equal(con.P.astype(int), np.array(ex["P"]))
    # Y' = Z P reproduces the paper's reordered points x_1..x_6
    yp = np.rint(con.Yprime() * 7).astype(int)
    assert np.array_equal(yp, np.array(ex["paper_order_numerators_over_N"])[1:])
    # and the row map sends paper row n to the conventional point beta^-(n-1)
    conv = np.array(ex["conventional_numerators_over_N"])
    for n in range(1, 7):
        assert list(conv[con.conv_index[n]]) == ex["paper_order_numerators_over_N"][n]


def test_example1_product_matches_dense():
    ex = _example()
    A = np.random.default_rng(3).standard_normal((3, 4))
    for phi in (qi.PHI_IDENTITY, qi.PHI_CENTERED, qi.PHI_TENT):
        inst = _inst(qi.RULE_LATTICE, 7, ex["gen"], phi, A)
        np.testing.assert_allclose(literal.Construction(inst).product(), oracle.matmul(inst),
                                   rtol=0, atol=1e-14)


# ---------------------------------------------------------------------------
# brute force over exact rationals (tiny N)
# ---------------------------------------------------------------------------

SMALL_PRIMES = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31]


@pytest.mark.parametrize("N", SMALL_PRIMES)
@pytest.mark.parametrize("phi", [qi.PHI_IDENTITY, qi.PHI_CENTERED])
def test_lattice_exact_bruteforce(N, phi):
    rg = np.random.default_rng(N * 10 + phi)
    for s in (1, 2, 3, 6):
        gen = rg.integers(1, N, size=s) if N > 2 else np.ones(s, dtype=np.int64)
        A = rg.standard_normal((s, 3))
        inst = _inst(qi.RULE_LATTICE, N, gen, phi, A)
        ex = exact.product(inst)
        X = oracle.matmul(inst)
        for n in range(N):
            for c in range(3):
                assert abs(X[n, c] - float(ex[n][c])) <= 4e-16 * (1 + sum(abs(A[:, c])))


def test_lattice_identity_integer_A_is_exact():
    """phi = identity and integer A: N X is an integer combination of A."""
    N, s = 31, 6
    rg = np.random.default_rng(5)
    gen = rg.integers(1, N, size=s)
    A = rg.integers(-50, 50, size=(s, 4)).astype(np.float64)
    inst = _inst(qi.RULE_LATTICE, N, gen, qi.PHI_IDENTITY, A)
    X = oracle.matmul(inst)
    NX = np.rint(X * N)
    assert np.max(np.abs(X * N - NX)) < 1e-9
    # exact integer reference: sum_j ((n g_j) mod N) A_jc
    n = np.arange(N)[:, None]
    ref = ((n * gen[None, :]) % N) @ A.astype(np.int64)
    assert np.array_equal(NX.astype(np.int64), ref)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5])
def test_gf2_exact_bruteforce(m):
    rg = np.random.default_rng(100 + m)
    p = qi.draw_primitive_poly(m, rg)
    N = 1 << m
    for s in (1, 3):
        q = rg.integers(1, N, size=s)
        A = rg.standard_normal((s, 2))
        inst = _inst(qi.RULE_POLY_GF2, N, q, qi.PHI_CENTERED, A, modulus=p)
        ex = exact.product(inst)
        X = oracle.matmul(inst)
        for n in range(N):
            for c in range(2):
                assert abs(X[n, c] - float(ex[n][c])) <= 4e-16 * (1 + sum(abs(A[:, c])))


def test_gf2_known_small_field():
    """GF(4) = GF(2)[x]/(x^2+x+1), q = x: n(x) x mod p and its digit value.

    n = 1 -> r = x      -> x/(x^2+x+1) = x^-1 + x^-2 + ...   -> 0.11b = 3/4
    n = 2 -> r = x^2 = x+1 -> (x+1)/(x^2+x+1) = x^-1 + 0 x^-2 ... -> 0.10b = 1/2
    n = 3 -> r = x^2+x = 1 -> 1/(x^2+x+1) = 0 x^-1 + x^-2 ...  -> 0.01b = 1/4
    """
    x = oracle.gf2_coords(2, 0b111, [0b10])
    assert list(x[:, 0]) == [0.0, 0.75, 0.5, 0.25]
    K, D = oracle.coords_rational(qi.RULE_POLY_GF2, 4, [0b10], modulus=0b111)
    assert list(K[:, 0] / D) == [0.0, 0.75, 0.5, 0.25]
    assert list(oracle.gf2_digits_coords(2, 0b111, [0b10])[:, 0]) == [0.0, 0.75, 0.5, 0.25]


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8, 12, 16])
def test_gf2_digital_net_form_equals_direct_definition(m):
    """The digital-net numerators (Hankel generating matrix of the Laurent
    digits of q/p) equal the direct route r = n q mod p, Q = floor(r x^m / p)
    bit for bit, on every row for small m and on sampled rows otherwise."""
    rg = np.random.default_rng(300 + m)
    p = qi.draw_primitive_poly(m, rg)
    N = 1 << m
    q = rg.integers(1, N, size=7)
    rows = np.arange(N) if m <= 8 else rg.choice(N, size=2000, replace=False)
    direct = oracle.points.gf2_value_of_residue(m, p, oracle.points.gf2_residues(m, p, q, rows))
    digital = oracle.points.gf2_numerators_digital(m, p, q, rows)
    np.testing.assert_array_equal(direct, digital)


@pytest.mark.parametrize("rule", [qi.RULE_LATTICE, qi.RULE_POLY_GF2, qi.RULE_KOROBOV_UNION])
@pytest.mark.parametrize("phi,shift", [(qi.PHI_IDENTITY, (0, 1)), (qi.PHI_CENTERED, (0, 1)),
                                       (qi.PHI_TENT, (1, 3)), (qi.PHI_INVNORM, "half")])
def test_phi_table_lookup_is_elementwise_phi(rule, phi, shift):
    """explicit_Y evaluates phi once per numerator and looks it up when the
    rows hold more entries than there are numerators: the same bits as phi of
    every entry's exact coordinate."""
    if rule == qi.RULE_LATTICE:
        N, gen, mod, base = 101, np.array([1, 5, 17, 44, 99]), 0, 101
    elif rule == qi.RULE_POLY_GF2:
        N, mod = 128, qi.draw_primitive_poly(7, np.random.default_rng(1))
        gen, base = np.array([1, 3, 77, 127, 64]), 128
    else:
        N, gen, mod, base = 100, np.arange(6), 11, 11
    if shift == "half":
        shift = (1, 2 * base)
    Y = oracle.explicit_Y(rule, N, gen, phi, mod, shift)
    K, D = oracle.coords_rational(rule, N, gen, mod, shift)
    np.testing.assert_array_equal(Y, oracle.phi_rational(phi, K, D))
    rows = np.array([0, 1, N - 1, N // 2])  # fewer entries than numerators: no table
    np.testing.assert_array_equal(oracle.explicit_Y(rule, N, gen, phi, mod, shift, rows), Y[rows])


def test_planted_gf2_hankel_index_is_caught():
    """A digital-net form that reads the Hankel matrix one digit off (u_{i+l-1}
    or u_{i+l+1}) breaks the GF(4) hand pin and the direct route."""
    def shifted(off):
        def numer(m, p, q, rows=None):
            qq = np.asarray(q, dtype=np.uint64)
            n = np.arange(1 << m, dtype=np.uint64) if rows is None else np.asarray(rows, np.uint64)
            u = oracle.points.gf2_laurent_digits(p, qq, 2 * m + 1)
            out = np.zeros((len(n), len(qq)), dtype=np.uint64)
            for i in range(m):
                word = np.zeros(len(qq), dtype=np.uint64)
                for l in range(1, m + 1):
                    k = i + l + off  # the right index is u_{i+l}, row i + l - 1
                    word |= (u[k - 1] if k >= 1 else 0) << np.uint64(m - l)
                bit = ((n >> np.uint64(i)) & np.uint64(1)) == 1
                out ^= np.where(bit[:, None], word[None, :], np.uint64(0))
            return out
        return numer
    assert np.array_equal(oracle.points.gf2_numerators_digital(2, 0b111, [0b10])[:, 0], [0, 3, 2, 1])
    for off in (-1, 1):
        assert not np.array_equal(shifted(off)(2, 0b111, [0b10])[:, 0], [0, 3, 2, 1])


@pytest.mark.parametrize("m", [6, 8, 10])
def test_gf2_columns_are_permutations(m):
    """For q_j != 0, n -> n q_j mod p is a bijection and so is the digit map:
    every column of the (unshifted, identity) point matrix is {k / 2^m}."""
    rg = np.random.default_rng(m)
    p = qi.draw_primitive_poly(m, rg)
    q = rg.integers(1, 1 << m, size=5)
    x = oracle.gf2_coords(m, p, q)
    for j in range(5):
        assert np.array_equal(np.sort(np.rint(x[:, j] * (1 << m)).astype(int)), np.arange(1 << m))
    np.testing.assert_array_equal(x, oracle.gf2_digits_coords(m, p, q))


# ---------------------------------------------------------------------------
# closed forms: column sums
# ---------------------------------------------------------------------------

def test_column_sum_identity_lattice():
    """sum_n {n g / N} = (N-1)/2 for g coprime to N, so 1^T X = (N-1)/2 1^T A."""
    inst = qi.small_lattice(1009, 37, 3)
    X = oracle.matmul(inst)
    np.testing.assert_allclose(X.sum(axis=0), (1009 - 1) / 2 * inst.A.sum(axis=0), rtol=1e-12)


def test_column_sum_invnorm_shifted_is_zero():
    """Phi^-1((2r+1)/(2N)) is odd about the middle residue: columns sum to 0."""
    N = 2003
    inst = qi.small_lattice(N, 64, 2, phi=qi.PHI_INVNORM, shift=(1, 2 * N))
    Y = oracle.Y_rows(inst)
    assert np.max(np.abs(Y.sum(axis=0))) < 1e-10
    # and every column is a permutation of the one-dimensional value table
    T = oracle.phi_residue_values(qi.RULE_LATTICE, N, qi.PHI_INVNORM, shift=(1, 2 * N))
    for j in range(4):
        np.testing.assert_array_equal(np.sort(Y[:, j]), np.sort(T))


def test_column_sum_gf2_centered():
    """sum over the 2^m points of (k/2^m - 1/2) = -1/2 in every column."""
    inst = qi.small_gf2(10, 40, 2, phi=qi.PHI_CENTERED)
    Y = oracle.Y_rows(inst)
    np.testing.assert_allclose(Y.sum(axis=0), -0.5, atol=1e-12)


def _tent_pins_pass(tent_fn) -> bool:
    """Closed forms of the tent map 1 - |2x - 1| (Section 2.1) that a
    candidate phi_rational-like routine tent_fn(K, D) must meet on the columns
    of the oracle's point sets:

    * lattice, odd N, g coprime to N: a column runs through every k/N once and
      sum_{k<N} tent(k/N) = 2 sum_{k<=(N-1)/2} 2k/N = (N^2 - 1)/(2N);
    * GF(2), N = 2^m: a column runs through every k/2^m once and
      sum_k tent(k/N) = N/2 (the terms 2k/N for k <= N/2 add up to
      (N/2 + 1)/2, the terms 2 - 2k/N for k > N/2 to (N/2 - 1)/2);
    * reflection: tent(1 - x) = tent(x), and for a lattice {(N - n) g / N} =
      1 - {n g / N} when n g != 0 mod N, so rows n and N - n are equal;
    * tent(1/2) = 1 and tent(0) = 0 (row 0 of the unshifted lattice)."""
    for N in (101, 1009):
        gen = np.random.default_rng(N).integers(1, N, size=9)
        K, D = oracle.coords_rational(qi.RULE_LATTICE, N, gen)
        Y = tent_fn(K, D)
        if not np.allclose(Y.sum(axis=0), (N * N - 1) / (2 * N), rtol=1e-13, atol=0):
            return False
        if not np.array_equal(Y[1:], Y[:0:-1]) or np.any(Y[0] != 0.0):
            return False
    for m in (6, 9):
        rg = np.random.default_rng(40 + m)
        p = qi.draw_primitive_poly(m, rg)
        q = rg.integers(1, 1 << m, size=5)
        K, D = oracle.coords_rational(qi.RULE_POLY_GF2, 1 << m, q, modulus=p)
        if not np.allclose(tent_fn(K, D).sum(axis=0), (1 << m) / 2, rtol=1e-13, atol=0):
            return False
    return bool(tent_fn(np.array([1]), 2)[0] == 1.0)


def test_tent_closed_forms():
    """The oracle's tent branch meets the closed forms, through the same
    product path the GPU parity tests use (explicit Y, dense multiply)."""
    assert _tent_pins_pass(lambda K, D: oracle.phi_rational(qi.PHI_TENT, K, D))
    N = 1009
    inst = qi.small_lattice(N, 33, 3, phi=qi.PHI_TENT)
    X = oracle.matmul(inst)
    np.testing.assert_allclose(X.sum(axis=0), (N * N - 1) / (2 * N) * inst.A.sum(axis=0),
                               rtol=1e-11)
    np.testing.assert_allclose(X[1:], X[:0:-1], rtol=0, atol=1e-13)


def test_tent_planted_mistakes_are_caught():
    """Plausible slips in the tent branch fail the pins: the complement
    |2x - 1|, a dropped factor 2 (1 - |x - 1/2|), the ramp 1 - |x - 1| = x,
    and the half-height tent."""
    for bad in (lambda K, D: np.abs(2 * K - D) / float(D),
                lambda K, D: 1.0 - np.abs(K / float(D) - 0.5),
                lambda K, D: K / float(D),
                lambda K, D: (D - np.abs(2 * K - D)) / (2.0 * D)):
        assert not _tent_pins_pass(bad)


def test_row_zero_is_phi_of_shift():
    inst = qi.small_lattice(101, 9, 2, phi=qi.PHI_INVNORM, shift=(1, 202))
    Y = oracle.Y_rows(inst)
    assert np.all(Y[0] == Y[0, 0])
    assert abs(Y[0, 0] - statistics.NormalDist().inv_cdf(1 / 202)) < 1e-14


# ---------------------------------------------------------------------------
# the paper's literal construction against the dense product (medium N)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("N,s,t", [(101, 20, 3), (257, 300, 2), (1009, 64, 2)])
@pytest.mark.parametrize("phi,shift", [(qi.PHI_IDENTITY, None), (qi.PHI_CENTERED, None),
                                       (qi.PHI_INVNORM, "half"), (qi.PHI_TENT, None)])
def test_literal_construction_matches_dense(N, s, t, phi, shift):
    sh = (1, 2 * N) if shift == "half" else (0, 1)
    inst = qi.small_lattice(N, s, t, phi=phi, shift=sh)
    con = literal.Construction(inst)
    Xl = con.product()
    Xd = oracle.matmul(inst)
    scale = np.max(np.abs(oracle.Y_rows(inst))) * np.abs(inst.A).sum(axis=0)
    assert np.max(np.abs(Xl - Xd) / scale) < 1e-13


@pytest.mark.parametrize("m,s", [(6, 10), (8, 300)])
def test_literal_construction_matches_dense_gf2(m, s):
    inst = qi.small_gf2(m, s, 2, phi=qi.PHI_CENTERED)
    con = literal.Construction(inst)
    assert con.beta == 2  # x generates the group when p is primitive
    np.testing.assert_allclose(con.product(), oracle.matmul(inst), rtol=0, atol=1e-12)


def test_output_independent_of_primitive_root():
    """Conventional-order output does not depend on which beta is used."""
    N = 101
    inst = qi.small_lattice(N, 30, 2, phi=qi.PHI_INVNORM, shift=(1, 2 * N))
    grp = literal._Lattice(N)
    roots = [b for b in range(2, N) if len(set(literal.powers(grp, b))) == N - 1][:4]
    outs = [literal.Construction(inst, beta=b).product() for b in roots]
    for o in outs[1:]:
        np.testing.assert_allclose(o, outs[0], rtol=0, atol=1e-12)


def test_identity_A_regenerates_points():
    """A = I_s gives X = Y (the point set itself, Section 2.1 remark)."""
    inst = qi.small_lattice(211, 15, 15)
    I = np.eye(15)
    np.testing.assert_allclose(literal.Construction(inst).product(I), oracle.Y_rows(inst), atol=1e-15)


# ---------------------------------------------------------------------------
# inverse normal CDF and the adjoint
# ---------------------------------------------------------------------------

def test_invnorm_against_stdlib_and_erfc():
    nd = statistics.NormalDist()
    ps = np.concatenate([np.linspace(1e-12, 1 - 1e-12, 2001), [1e-300, 1e-100, 1e-20, 0.5, 0.975, 0.999999]])
    ys = oracle.phi_apply(qi.PHI_INVNORM, ps)
    for p, y in zip(ps, ys):
        ref = nd.inv_cdf(float(p))
        assert abs(y - ref) <= 8e-16 * max(1.0, abs(ref)), (p, y, ref)
        if 1e-300 < p < 1:
            back = 0.5 * math.erfc(-y / math.sqrt(2.0))
            # one ulp of y moves Phi(y) by about |y| ulp(y) relative: allow that
            assert abs(back - p) <= 4e-15 * max(1.0, y * y) * p + 1e-300, (p, back)


def test_adjoint_is_transpose():
    inst = qi.small_lattice(257, 40, 3, phi=qi.PHI_INVNORM, shift=(1, 514))
    G = np.random.default_rng(1).standard_normal((257, 3))
    dA = oracle.adjoint(inst, G)
    X = oracle.matmul(inst)
    # <Y A, G> = <A, Y^T G>
    assert abs(np.sum(X * G) - np.sum(inst.A * dA)) < 1e-10 * np.sum(np.abs(X * G))
    # entry-sampled adjoint agrees with the full one
    ent = [(0, 0), (5, 2), (39, 1), (17, 0)]
    got = oracle.adjoint_entries(dataclasses.replace(inst, G=G), ent, chunk=50)
    np.testing.assert_allclose(got, [dA[j, k] for j, k in ent], rtol=1e-12, atol=1e-12)


def test_row_sampled_matmul_agrees():
    inst = qi.small_gf2(9, 50, 3)
    X = oracle.matmul(inst)
    rows = np.array([0, 1, 7, 511, 300])
    np.testing.assert_allclose(oracle.matmul_rows(inst, rows, chunk=2), X[rows], rtol=0, atol=1e-13)


def test_cholesky_closed_form():
    """The C2 matrix A is the upper Cholesky factor of exp(-|i-j|/410)."""
    s = 300
    A = qi.cholesky_exp_upper(s)
    i = np.arange(s)
    Sigma = np.exp(-np.abs(i[:, None] - i[None, :]) / 410.0)
    np.testing.assert_allclose(A.T @ A, Sigma, atol=1e-13)
    np.testing.assert_allclose(A, np.linalg.cholesky(Sigma).T, atol=1e-12)


# ---------------------------------------------------------------------------
# planted mistakes: mutated copies of oracle routines must fail the pins
# ---------------------------------------------------------------------------

def _pins_pass(coord_fn) -> bool:
    """Run the coordinate-level pins against a candidate coordinate routine."""
    ex = _example()
    x = coord_fn(7, np.array(ex["gen"]), (0, 1))
    if not np.array_equal(np.rint(x * 7).astype(int), np.array(ex["conventional_numerators_over_N"])):
        return False
    N = 101
    x = coord_fn(N, np.arange(1, 6), (1, 2 * N))
    ref = [[float((Fraction(n * g % N, N) + Fraction(1, 2 * N)) % 1) for g in range(1, 6)] for n in range(N)]
    return bool(np.array_equal(x, np.array(ref)))


def test_planted_mistakes_are_caught():
    good = lambda N, g, sh: oracle.lattice_coords(N, g, sh)
    assert _pins_pass(good)
    dropped_shift = lambda N, g, sh: oracle.lattice_coords(N, g, (0, 1))
    off_by_one_row = lambda N, g, sh: oracle.lattice_coords(N, g, sh, rows=np.arange(1, N + 1))
    swapped = lambda N, g, sh: oracle.lattice_coords(N, (np.asarray(g) * 2) % N, sh)
    for bad in (dropped_shift, off_by_one_row, swapped):
        assert not _pins_pass(bad)


def test_planted_gf2_digit_order_is_caught():
    """Reading the quotient bits least-significant-first breaks the GF(4) pin."""
    def reversed_digits(m, p, q):
        x = oracle.gf2_coords(m, p, q)
        k = np.rint(x * (1 << m)).astype(int)
        rev = np.array([[int(format(v, f"0{m}b")[::-1], 2) for v in row] for row in k])
        return rev / float(1 << m)
    assert list(reversed_digits(2, 0b111, [0b10])[:, 0]) != [0.0, 0.75, 0.5, 0.25]


# ---------------------------------------------------------------------------
# union of all Korobov lattice point sets (Section 2.2)
# ---------------------------------------------------------------------------

def _kor(K, s, phi, shift=(0, 1), t=3, seed=0):
    return qi.small_korobov(K, s, t, phi=phi, shift=shift, dtype="f64", seed=seed)


@pytest.mark.parametrize("K", [3, 5, 7, 11, 13])
@pytest.mark.parametrize("phi,shift", [(qi.PHI_IDENTITY, (0, 1)), (qi.PHI_CENTERED, (0, 1)),
                                       (qi.PHI_IDENTITY, (1, 3))])
def test_korobov_exact_bruteforce(K, phi, shift):
    for s in (1, 2, 5):
        inst = _kor(K, s, phi, shift, seed=K + s)
        ex = exact.product(inst)
        X = oracle.matmul(inst)
        assert X.shape == ((K - 1) ** 2, 3)
        for r in range(inst.N):
            for c in range(3):
                assert abs(X[r, c] - float(ex[r][c])) <= 4e-16 * (1 + sum(abs(inst.A[:, c])))


def test_korobov_blocks_are_korobov_lattice_rules():
    """Block b is the lattice rule with generating vector (b^j mod K)_j
    without its point n = 0 (Section 2.2, Y' stacks the Y'_g)."""
    K, s = 31, 6
    Y = oracle.Y_rows(_kor(K, s, qi.PHI_IDENTITY))
    for b in range(1, K):
        gen = [pow(b, j, K) for j in range(s)]
        lat = oracle.explicit_Y(qi.RULE_LATTICE, K, np.array(gen), qi.PHI_IDENTITY)
        np.testing.assert_array_equal(Y[(b - 1) * (K - 1):b * (K - 1)], lat[1:])


@pytest.mark.parametrize("K", [7, 13, 31])
def test_korobov_paper_ordering(K):
    """The paper's ordering of Section 2.2: with a primitive root beta, its
    point (n, g) is ({beta^(c_{g,j} - n) / K})_j with c_{g,j} read as
    ((j-1)(g-1) mod (K-1)) + 1 in [1, K-1]; it is the conventional point of
    block b = beta^(g-1) and row n' = beta^-(n-1).  The printed
    (j-1)(g-1)+1 mod (K-1) agrees with that reading modulo K-1."""
    s = 5
    beta = literal.primitive_element(literal._group(qi.RULE_LATTICE, K, 0))
    Y = oracle.Y_rows(_kor(K, s, qi.PHI_IDENTITY))
    for g in range(1, K):
        for n in range(1, K):
            c = [((j - 1) * (g - 1)) % (K - 1) + 1 for j in range(1, s + 1)]
            assert all(1 <= v <= K - 1 for v in c)
            assert all((v - ((j - 1) * (g - 1) + 1)) % (K - 1) == 0 for j, v in zip(range(1, s + 1), c))
            paper = [pow(beta, (v - n) % (K - 1), K) / K for v in c]
            b = pow(beta, g - 1, K)
            n_conv = pow(beta, (-(n - 1)) % (K - 1), K)
            row = (b - 1) * (K - 1) + (n_conv - 1)
            np.testing.assert_array_equal(Y[row], np.array(paper))


@pytest.mark.parametrize("K", [5, 11, 101])
def test_korobov_column_sums(K):
    """Every block column is a permutation of the residues 1..K-1 (b^j is a
    unit), so each column of Y sums to (K-1) times the sum of phi over the
    nonzero residues: (K-1)^2/2 for the identity, 0 for x - 1/2, and
    -(K-1) Phi^-1(1/(2K)) for the inverse normal CDF with shift 1/(2K)."""
    s = 7
    Yi = oracle.Y_rows(_kor(K, s, qi.PHI_IDENTITY))
    num = np.rint(Yi * K).astype(np.int64)
    for b in range(1, K):
        blk = num[(b - 1) * (K - 1):b * (K - 1)]
        for j in range(s):
            assert sorted(blk[:, j]) == list(range(1, K))
    np.testing.assert_array_equal(num.sum(axis=0), np.full(s, (K - 1) ** 2 * K // 2))
    Yc = oracle.Y_rows(_kor(K, s, qi.PHI_CENTERED))
    np.testing.assert_allclose(Yc.sum(axis=0), 0.0, atol=1e-12 * K * K)
    Yn = oracle.Y_rows(_kor(K, s, qi.PHI_INVNORM, (1, 2 * K)))
    expect = -(K - 1) * statistics.NormalDist().inv_cdf(1 / (2 * K))
    np.testing.assert_allclose(Yn.sum(axis=0), expect, rtol=1e-12, atol=1e-10 * K)


def _korobov_pins_pass(numer_fn) -> bool:
    """The union's coordinate pins (exact values, block permutations, the
    paper's ordering) run against a candidate numerator routine
    numer_fn(K, exponents) -> (K-1)^2 x s array of (n b^e) mod K."""
    K, s = 7, 4
    num = numer_fn(K, np.arange(s))
    # exact values of the definition (Fractions, Python's pow)
    ex = exact.point_matrix(_kor(K, s, qi.PHI_IDENTITY))
    if not all(Fraction(int(num[r, j]), K) == ex[r][j] for r in range((K - 1) ** 2) for j in range(s)):
        return False
    for b in range(1, K):  # every block column permutes 1..K-1
        blk = num[(b - 1) * (K - 1):b * (K - 1)]
        if any(sorted(blk[:, j]) != list(range(1, K)) for j in range(s)):
            return False
    beta = literal.primitive_element(literal._group(qi.RULE_LATTICE, K, 0))
    for g in range(1, K):  # the paper's ordering
        for n in range(1, K):
            c = [((j - 1) * (g - 1)) % (K - 1) + 1 for j in range(1, s + 1)]
            row = (pow(beta, g - 1, K) - 1) * (K - 1) + pow(beta, (-(n - 1)) % (K - 1), K) - 1
            if [int(v) for v in num[row]] != [pow(beta, (v - n) % (K - 1), K) for v in c]:
                return False
    return True


def test_korobov_planted_mistakes_are_caught():
    """Mutated copies of the union's coordinate routine fail the pins: n
    counted from 0, the exponent shifted by one, n-major block order."""
    good = oracle.points.korobov_union_numerators
    assert _korobov_pins_pass(good)

    def mutate(f):
        def numer(K, exps):
            N = (K - 1) ** 2
            return np.array([[f(K, r, int(e)) for e in exps] for r in range(N)])
        return numer

    bad_n0 = mutate(lambda K, r, e: (r % (K - 1)) * pow(r // (K - 1) + 1, e, K) % K)
    bad_exp = mutate(lambda K, r, e: (r % (K - 1) + 1) * pow(r // (K - 1) + 1, e + 1, K) % K)
    bad_major = mutate(lambda K, r, e: (r // (K - 1) + 1) * pow(r % (K - 1) + 1, e, K) % K)
    for bad in (bad_n0, bad_exp, bad_major):
        assert not _korobov_pins_pass(bad)


# ---------------------------------------------------------------------------
# epilogues of the PDE applications (Sections 3.2 and 3.3)
# ---------------------------------------------------------------------------

def _fe_1d(n_el):
    """Piecewise linear hat functions on the uniform mesh of (0, 1): the
    stiffness pairs (k, l) with a common element, k, l = 1..n_el-1."""
    h = 1.0 / n_el
    pairs = [(k, k) for k in range(1, n_el)] + [(k, k + 1) for k in range(1, n_el - 1)]
    return h, pairs


def _psi(j, x):
    return (1.0 + x) if j == 0 else np.sin(j * np.pi * x) / (j * j)


def _psi_elem_integral(j, a, b):
    """Closed form of the integral of psi_j over [a, b]."""
    if j == 0:
        return (b - a) + (b * b - a * a) / 2
    return (np.cos(j * np.pi * a) - np.cos(j * np.pi * b)) / (j * np.pi) / (j * j)


def test_uniform_pde_stiffness_entries():
    """b_{n,k,l} = a_{0,k,l} + y_n . a_{k,l} (eq. (Ya)) with the closed-form
    a_{j,k,l} equals the stiffness integral of a(x, y_n) grad phi_k grad phi_l
    computed by Gauss-Legendre quadrature on every element."""
    n_el, s = 9, 6
    h, pairs = _fe_1d(n_el)
    nodes = np.linspace(0.0, 1.0, n_el + 1)

    def a_entry(j, k, l):  # integral of psi_j phi_k' phi_l'
        if k == l:
            return (_psi_elem_integral(j, nodes[k - 1], nodes[k]) +
                    _psi_elem_integral(j, nodes[k], nodes[k + 1])) / h ** 2
        return -_psi_elem_integral(j, nodes[k], nodes[k + 1]) / h ** 2

    A = np.array([[a_entry(j, k, l) for (k, l) in pairs] for j in range(1, s + 1)])
    bias = np.array([a_entry(0, k, l) for (k, l) in pairs])
    inst = qi.small_lattice(31, s, len(pairs), phi=qi.PHI_CENTERED, dtype="f64", seed=3)
    inst = dataclasses.replace(inst, A=A, t=len(pairs))
    b = oracle.epilogue(oracle.matmul(inst), oracle.EPI_AFFINE, bias)
    Y = oracle.Y_rows(inst)  # y_n in [-1/2, 1/2]^s (Section 3.2)
    gx, gw = np.polynomial.legendre.leggauss(20)
    for n in range(inst.N):
        for c, (k, l) in enumerate(pairs):
            elems = [k - 1, k] if k == l else [k]
            sign = 1.0 if k == l else -1.0
            total = 0.0
            for e in elems:
                x = nodes[e] + (gx + 1) * h / 2
                a = _psi(0, x) + sum(Y[n, j - 1] * _psi(j, x) for j in range(1, s + 1))
                total += sign * np.sum(gw * a) * h / 2 / h ** 2
            assert abs(b[n, c] - total) <= 1e-10 * (1 + abs(total))


def test_lognormal_coefficient_and_weighted_entries():
    """exp(Psi^ + Y Psi) (eqs. (fastB), (eq_as)) at quadrature points x_i,
    scaled by the quadrature weight times grad phi_k grad phi_l, is the
    coefficient exp(psi_0(x_i) + sum_j y_j psi_j(x_i)) point by point, and
    its sum over the points of an element is the quadrature (def:b nkl) of
    the element's stiffness entry, close to the integral by a finer rule."""
    n_el, s, I = 5, 4, 6
    h = 1.0 / n_el
    gx, gw = np.polynomial.legendre.leggauss(I)
    e = 2  # the element [x_2, x_3]; entry (k, l) = (2, 3): grad product -1/h^2
    xq = 2 * h + (gx + 1) * h / 2
    wq = gw * h / 2 * (-1.0 / h ** 2)
    Psi = np.array([[_psi(j, x) for x in xq] for j in range(1, s + 1)])
    inst = qi.small_lattice(37, s, I, phi=qi.PHI_INVNORM, shift=(1, 74), dtype="f64", seed=4)
    inst = dataclasses.replace(inst, A=Psi, t=I)
    th = oracle.epilogue(oracle.matmul(inst), oracle.EPI_EXP, _psi(0, xq), wq)
    Y = oracle.Y_rows(inst)
    for n in range(inst.N):
        direct = [wq[i] * math.exp(_psi(0, xq[i]) + sum(Y[n, j] * Psi[j, i] for j in range(s)))
                  for i in range(I)]
        np.testing.assert_allclose(th[n], direct, rtol=1e-13)
        fx, fw = np.polynomial.legendre.leggauss(40)
        xf = 2 * h + (fx + 1) * h / 2
        fine = np.sum(fw * h / 2 * (-1.0 / h ** 2) * np.exp(
            _psi(0, xf) + sum(Y[n, j] * _psi(j + 1, xf) for j in range(s))))
        assert abs(th[n].sum() - fine) <= 1e-6 * abs(fine)


def test_epilogue_definitions():
    X = np.array([[0.5, -1.0], [2.0, 0.25]])
    b, w = np.array([1.0, -2.0]), np.array([3.0, 0.5])
    np.testing.assert_array_equal(oracle.epilogue(X, oracle.EPI_NONE), X)
    np.testing.assert_array_equal(oracle.epilogue(X, oracle.EPI_AFFINE, b), X + b)
    np.testing.assert_array_equal(oracle.epilogue(X, oracle.EPI_AFFINE, None, w), X * w)
    np.testing.assert_allclose(oracle.epilogue(X, oracle.EPI_EXP, b, w), w * np.exp(X + b))
