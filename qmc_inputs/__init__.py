"""Seeded synthetic inputs for the fast QMC matrix product.

This module is shared by the CPU oracle (through the tests) and by the GPU
path (through the tests and the benchmark).  It only draws numbers: point-set
parameters (the number of points, generating vectors, a primitive modulus for
polynomial lattice rules) and the matrices A and G.  It does not evaluate
points, build tables or multiply anything.

Workloads follow the shapes and value distributions of the paper's
applications (Section 3 and the three experiments of Section 4):

* ``c1``  plain lattice rule, N = 2003, s = 500, one column, phi = identity,
          FP64 (a parity-sized case);
* ``c2``  Gaussian sampling with a general covariance (Section 3.1,
          Experiment 1): N = 65537, s = t = 4096, phi = inverse normal CDF with
          the equal shift 1/(2N), A = upper Cholesky factor of
          exp(-|i-j|/410);
* ``c3``  affine-parametric PDE input field (Section 3.2, Experiment 2) on a
          polynomial lattice rule over GF(2) with N = 2^16, s = 16384,
          t = 4096, phi(y) = y - 1/2, A_jk = j^-2 sin(j pi x_k);
* ``c4``  256 heterogeneous lattice instances for one batched launch;
* ``c5``  a large lattice rule (N = 1048573, s = 65536, t = 256) with the
          adjoint product;
* ``korobov``  the union of all Korobov lattice point sets (Section 2.2) for
          K = 1021 (N = 1020^2 = 1040400 points), s = 512, t = 256,
          phi = inverse normal CDF with the equal shift 1/(2K), A i.i.d.
          N(0,1)/sqrt(s) (Gaussian-sampling shapes as in ``c2``; the paper
          runs no experiment on this point set).

Every draw uses ``numpy.random.default_rng(150106286 + 1000*config + stream)``
with streams 0 = generating vector, 1 = A, 2 = G, 3 = finite-difference
entries, 4 = polynomial modulus.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

SEED_BASE = 150106286

# phi kinds (same numbering as the C interface)
PHI_IDENTITY = 0
PHI_CENTERED = 1
PHI_INVNORM = 2
PHI_TENT = 3

RULE_LATTICE = 0
RULE_POLY_GF2 = 1
RULE_KOROBOV_UNION = 2   # union of Korobov rules: N = (K-1)^2, modulus = K, gen = exponents j


def rng(config: int, stream: int) -> np.random.Generator:
    """The seeded generator of (config, stream)."""
    return np.random.default_rng(SEED_BASE + 1000 * config + stream)


# ---------------------------------------------------------------------------
# primes and primitive polynomials (input selection only)
# ---------------------------------------------------------------------------

def is_prime(n: int) -> bool:
    if n < 2:
        return False
    if n % 2 == 0:
        return n == 2
    f = 3
    while f * f <= n:
        if n % f == 0:
            return False
        f += 2
    return True


def primes_in_range(lo: int, hi: int) -> np.ndarray:
    """All primes p with lo <= p <= hi (sieve of Eratosthenes)."""
    sieve = np.ones(hi + 1, dtype=bool)
    sieve[:2] = False
    for f in range(2, int(math.isqrt(hi)) + 1):
        if sieve[f]:
            sieve[f * f::f] = False
    idx = np.nonzero(sieve)[0]
    return idx[idx >= lo]


def _prime_factors(n: int) -> List[int]:
    out, f = [], 2
    while f * f <= n:
        if n % f == 0:
            out.append(f)
            while n % f == 0:
                n //= f
        f += 1
    if n > 1:
        out.append(n)
    return out


def _gf2_mulmod(a: int, b: int, p: int, m: int) -> int:
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if a >> m & 1:
            a ^= p
    return r


def _gf2_xpow(e: int, p: int, m: int) -> int:
    """x^e mod p over GF(2) by square and multiply."""
    result, base = 1, 2 % p if m > 1 else 1
    if m == 1:
        return 1
    while e:
        if e & 1:
            result = _gf2_mulmod(result, base, p, m)
        base = _gf2_mulmod(base, base, p, m)
        e >>= 1
    return result


def draw_primitive_poly(m: int, gen: np.random.Generator) -> int:
    """Draw odd (m+1)-bit words with bit m set until one is primitive over
    GF(2): x^(2^m-1) = 1 and x^((2^m-1)/q) != 1 for every prime q | 2^m-1."""
    order = (1 << m) - 1
    qs = _prime_factors(order)
    while True:
        low = int(gen.integers(0, 1 << (m - 1))) if m > 1 else 0
        p = (1 << m) | (low << 1) | 1
        if _gf2_xpow(order, p, m) != 1:
            continue
        if all(_gf2_xpow(order // q, p, m) != 1 for q in qs):
            return p


# ---------------------------------------------------------------------------
# matrices A
# ---------------------------------------------------------------------------

def cholesky_exp_upper(s: int, ell: float = 410.0) -> np.ndarray:
    """Upper Cholesky factor A (A^T A = Sigma) of Sigma_ij = exp(-|i-j|/ell),
    written in closed form: with rho = exp(-1/ell), A[i,k] = rho^(k-i) for
    k >= i, times sqrt(1-rho^2) when i > 0."""
    rho = math.exp(-1.0 / ell)
    i = np.arange(s)[:, None]
    k = np.arange(s)[None, :]
    d = (k - i).astype(np.float64)
    a = np.where(k >= i, rho ** np.maximum(d, 0.0), 0.0)
    a[1:, :] *= math.sqrt(1.0 - rho * rho)
    return a


def pde_field_matrix(s: int, t: int) -> np.ndarray:
    """A_jk = j^-2 sin(j pi x_k) with 1-based j and x_k = k/(t+1), k = 1..t."""
    j = np.arange(1, s + 1, dtype=np.float64)[:, None]
    x = np.arange(1, t + 1, dtype=np.float64)[None, :] / (t + 1)
    return np.sin(j * math.pi * x) / (j * j)


# ---------------------------------------------------------------------------
# workload descriptions
# ---------------------------------------------------------------------------

@dataclass
class Instance:
    """One product X = Y A (and optionally dA = Y^T G)."""
    name: str
    rule: int
    N: int
    s: int
    t: int
    gen: np.ndarray              # uint64, g_j (lattice), q_j bitmask (GF(2)) or the
                                 # exponent j of coordinate j (Korobov union)
    modulus: int                 # GF(2) primitive polynomial, K (Korobov union), 0 for lattice
    phi: int
    shift: Tuple[int, int]       # equal shift Delta = num/den
    dtype: str                   # "f32" or "f64"
    A: np.ndarray = field(repr=False, default=None)   # float64, already rounded to dtype
    G: Optional[np.ndarray] = field(repr=False, default=None)


def _round_to(a: np.ndarray, dtype: str) -> np.ndarray:
    if dtype == "f32":
        return a.astype(np.float32).astype(np.float64)
    return np.ascontiguousarray(a, dtype=np.float64)


def lattice_gen(N: int, s: int, gen: np.random.Generator) -> np.ndarray:
    return gen.integers(1, N, size=s, dtype=np.int64).astype(np.uint64)


def make_c1() -> Instance:
    N, s, t = 2003, 500, 1
    g = lattice_gen(N, s, rng(1, 0))
    A = rng(1, 1).standard_normal((s, t))
    return Instance("c1_lattice_n2003_s500_t1", RULE_LATTICE, N, s, t, g, 0,
                    PHI_IDENTITY, (0, 1), "f64", _round_to(A, "f64"))


def make_c2(dtype: str = "f32", s: int = 4096, t: Optional[int] = None,
            N: int = 65537) -> Instance:
    t = s if t is None else t
    g = lattice_gen(N, s, rng(2, 0))
    A = cholesky_exp_upper(s)[:, :t]
    return Instance(f"c2_gauss_n{N}_s{s}_t{t}", RULE_LATTICE, N, s, t, g, 0,
                    PHI_INVNORM, (1, 2 * N), dtype, _round_to(A, dtype))


def make_c2_nonprime(dtype: str = "f32", s: int = 4096, t: Optional[int] = None,
                     N: int = 65536) -> Instance:
    """The Gaussian-sampling shapes on a lattice rule whose number of points
    is not prime (N = 2^16 by default): unit generator components, the same
    A and phi as make_c2."""
    t = s if t is None else t
    g = unit_gen(N, s, rng(6, 0))
    A = cholesky_exp_upper(s)[:, :t]
    return Instance(f"c2n_gauss_n{N}_s{s}_t{t}", RULE_LATTICE, N, s, t, g, 0,
                    PHI_INVNORM, (1, 2 * N), dtype, _round_to(A, dtype))


def make_c3(dtype: str = "f32", m: int = 16, s: int = 16384, t: int = 4096) -> Instance:
    p = draw_primitive_poly(m, rng(3, 4))
    N = 1 << m
    q = rng(3, 0).integers(1, N, size=s, dtype=np.int64).astype(np.uint64)
    A = pde_field_matrix(s, t)
    return Instance(f"c3_pde_gf2_m{m}_s{s}_t{t}", RULE_POLY_GF2, N, s, t, q, p,
                    PHI_CENTERED, (0, 1), dtype, _round_to(A, dtype))


def make_c4(count: int = 256, n_lo: int = 1000, n_hi: int = 200000,
            s_lo: int = 256, s_hi: int = 8192, t_lo: int = 1, t_hi: int = 64,
            dtype: str = "f32", with_A: bool = True) -> List[Instance]:
    primes = primes_in_range(n_lo, n_hi)
    g0 = rng(4, 0)
    Ns = primes[g0.integers(0, len(primes), size=count)]
    ss = g0.integers(s_lo, s_hi + 1, size=count)
    ts = g0.integers(t_lo, t_hi + 1, size=count)
    out = []
    for i in range(count):
        N, s, t = int(Ns[i]), int(ss[i]), int(ts[i])
        gi = np.random.default_rng([SEED_BASE + 4000, i, 0])
        ga = np.random.default_rng([SEED_BASE + 4000, i, 1])
        g = lattice_gen(N, s, gi)
        A = ga.standard_normal((s, t)) / math.sqrt(s) if with_A else None
        out.append(Instance(f"c4_inst{i}_n{N}_s{s}_t{t}", RULE_LATTICE, N, s, t, g, 0,
                            PHI_INVNORM, (1, 2 * N), dtype,
                            _round_to(A, dtype) if with_A else None))
    return out


def make_c5(dtype: str = "f32", N: int = 1048573, s: int = 65536, t: int = 256,
            with_G: bool = True) -> Instance:
    g = lattice_gen(N, s, rng(5, 0))
    A = rng(5, 1).standard_normal((s, t))
    G = rng(5, 2).standard_normal((N, t)) if with_G else None
    return Instance(f"c5_large_n{N}_s{s}_t{t}", RULE_LATTICE, N, s, t, g, 0,
                    PHI_INVNORM, (1, 2 * N), dtype, _round_to(A, dtype),
                    _round_to(G, dtype) if with_G else None)


def fd_entries(s: int, t: int, count: int = 32) -> List[Tuple[int, int]]:
    """Seeded (j, k) entries of A for the finite-difference gradient check."""
    g = rng(5, 3)
    js = g.integers(0, s, size=count)
    ks = g.integers(0, t, size=count)
    return [(int(a), int(b)) for a, b in zip(js, ks)]


def small_lattice(N: int, s: int, t: int, phi: int = PHI_IDENTITY,
                  shift: Tuple[int, int] = (0, 1), dtype: str = "f64",
                  seed: int = 0) -> Instance:
    """A small seeded lattice instance for parity tests."""
    gen = np.random.default_rng([SEED_BASE, 7, N, s, t, seed])
    g = lattice_gen(N, s, gen)
    A = gen.standard_normal((s, t))
    return Instance(f"small_lat_n{N}_s{s}_t{t}", RULE_LATTICE, N, s, t, g, 0,
                    phi, shift, dtype, _round_to(A, dtype))


def unit_gen(N: int, s: int, gen: np.random.Generator) -> np.ndarray:
    """s generator components drawn uniformly from the units modulo N (the
    residues in [1, N-1] coprime to N), for lattice rules with any N."""
    out = np.empty(0, dtype=np.int64)
    while len(out) < s:
        g = gen.integers(1, N, size=2 * (s - len(out)) + 8, dtype=np.int64)
        keep = np.array([math.gcd(int(v), N) == 1 for v in g], dtype=bool)
        out = np.concatenate([out, g[keep]])
    return out[:s].astype(np.uint64)


def unit_lattice(N: int, s: int, t: int, phi: int = PHI_IDENTITY,
                 shift: Tuple[int, int] = (0, 1), dtype: str = "f64",
                 seed: int = 0) -> Instance:
    """A seeded lattice instance for any N (prime or not) whose generator
    components are units modulo N."""
    gen = np.random.default_rng([SEED_BASE, 10, N, s, t, seed])
    g = unit_gen(N, s, gen)
    A = gen.standard_normal((s, t))
    return Instance(f"unit_lat_n{N}_s{s}_t{t}", RULE_LATTICE, N, s, t, g, 0,
                    phi, shift, dtype, _round_to(A, dtype))


def small_gf2(m: int, s: int, t: int, phi: int = PHI_CENTERED,
              shift: Tuple[int, int] = (0, 1), dtype: str = "f64",
              seed: int = 0) -> Instance:
    """A small seeded polynomial-lattice instance for parity tests."""
    gen = np.random.default_rng([SEED_BASE, 8, m, s, t, seed])
    p = draw_primitive_poly(m, gen)
    N = 1 << m
    q = gen.integers(1, N, size=s, dtype=np.int64).astype(np.uint64)
    A = gen.standard_normal((s, t))
    return Instance(f"small_gf2_m{m}_s{s}_t{t}", RULE_POLY_GF2, N, s, t, q, p,
                    phi, shift, dtype, _round_to(A, dtype))


def randn(shape, seed, dtype="f64") -> np.ndarray:
    g = np.random.default_rng([SEED_BASE, 9] + list(np.atleast_1d(seed)))
    return _round_to(g.standard_normal(shape), dtype)


def make_korobov(dtype: str = "f32", K: int = 1021, s: int = 512, t: int = 256) -> Instance:
    """Union of all Korobov lattice point sets, Gaussian sampling shapes."""
    A = rng(6, 1).standard_normal((s, t)) / math.sqrt(s)
    return Instance(f"korobov_k{K}_s{s}_t{t}", RULE_KOROBOV_UNION, (K - 1) ** 2, s, t,
                    np.arange(s, dtype=np.uint64), K, PHI_INVNORM, (1, 2 * K), dtype,
                    _round_to(A, dtype))


def small_korobov(K: int, s: int, t: int, phi: int = PHI_IDENTITY,
                  shift: Tuple[int, int] = (0, 1), dtype: str = "f64",
                  seed: int = 0) -> Instance:
    """A small seeded union-of-Korobov instance for parity tests."""
    gen = np.random.default_rng([SEED_BASE, 9, K, s, t, seed])
    A = gen.standard_normal((s, t))
    return Instance(f"small_kor_k{K}_s{s}_t{t}", RULE_KOROBOV_UNION, (K - 1) ** 2, s, t,
                    np.arange(s, dtype=np.uint64), K, phi, shift, dtype, _round_to(A, dtype))
