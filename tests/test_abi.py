"""The C-ABI library builds, loads and exports every symbol include/qmc.h
declares; host-side argument checks reject bad input before any GPU work.
No GPU needed (only calls that fail validation are made)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1501_06286_amd as q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "qmc.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qmc_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("qmc_plan_create", "qmc_matmul", "qmc_matmul_adjoint", "qmc_matmul_batched",
              "qmc_plan_destroy", "qmc_workspace_size", "qmc_strerror"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = q.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(q.EXPORTED)


def test_header_constants_match_the_binding():
    with open(os.path.join(ROOT, "include", "qmc.h")) as f:
        text = f.read()
    m = re.search(r"#define QMC_BATCH_CHUNK_DEFAULT \(\(int64_t\)(\d+) << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == q.BATCH_CHUNK_DEFAULT
    m = re.search(r"#define QMC_PROF_SLOTS (\d+)", text)
    assert m and int(m.group(1)) == q.PROF_SLOTS


def test_strerror_strings():
    L = q.lib()
    for code in range(0, -10, -1):
        assert L.qmc_strerror(code)
    assert b"unit" in L.qmc_strerror(-4)
    assert b"prime" in L.qmc_strerror(-2)


def _create(rule=0, N=7, gen=(1, 5, 3), modulus=0, phi=0, snum=0, sden=1, dtype=0, s=None):
    L = q.lib()
    g = np.asarray(gen, dtype=np.uint64)
    h = ctypes.c_void_p()
    return L.qmc_plan_create(ctypes.byref(h), rule, N, len(g) if s is None else s,
                             g.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), modulus, phi,
                             snum, sden, dtype, None), h


@pytest.mark.parametrize("kw,code", [
    (dict(N=9), -4),                 # non-prime N: 3 is not a unit mod 9
    (dict(N=12, gen=(1, 5, 6)), -4), # 6 shares the factor 2 with 12
    (dict(N=1 << 26, gen=(1, 3)), -9),  # non-prime N above 2^25: refused before device work
    (dict(N=1), -1),                 # too small
    (dict(gen=(1, 7, 3)), -4),       # g = 0 mod 7
    (dict(dtype=5), -1),
    (dict(phi=9), -1),
    (dict(phi=2), -1),               # inverse normal CDF without a shift hits x = 0
    # a shift D with N D an integer puts the coordinate of residue -N D mod N
    # at 0, where the inverse normal CDF is -inf
    (dict(phi=2, snum=1, sden=7), -1),
    (dict(phi=2, snum=3, sden=7), -1),
    (dict(phi=2, snum=2, sden=14), -1),
    (dict(rule=1, N=16, gen=(1, 2), modulus=0b10011, phi=2), -1),
    (dict(rule=1, N=16, gen=(1, 2), modulus=0b10011, phi=2, snum=1, sden=4), -1),
    (dict(rule=1, N=16, gen=(1, 2), modulus=0b10011, phi=2, snum=3, sden=16), -1),
    (dict(snum=3, sden=2), -1),      # shift outside [0, 1)
    (dict(s=0), -1),
    (dict(rule=1, N=12, modulus=0b10011), -1),        # N not a power of two
    (dict(rule=1, N=16, gen=(1, 2), modulus=0b10101), -3),  # x^4+x^2+1 = (x^2+x+1)^2: not primitive
    (dict(rule=1, N=16, gen=(1, 2), modulus=0b11111), -3),  # order of x is 5, not 15
    (dict(rule=1, N=16, gen=(0, 2), modulus=0b10011), -4),  # q = 0
    (dict(rule=1, N=16, gen=(16, 2), modulus=0b10011), -4), # q outside the field
    (dict(rule=2), -1),
    # the first lengths past the longest outer split (M = 4096 x 64 x 64):
    # refused before any device work
    (dict(N=8388617, gen=(1, 5)), -9),
    (dict(N=8388617, gen=(1, 5), dtype=1), -9),
    (dict(rule=1, N=1 << 25, gen=(1, 2), modulus=(1 << 25) | 0b1001), -9),  # x^25+x^3+1
])
def test_plan_create_rejects_bad_input(kw, code):
    rc, h = _create(**kw)
    assert rc == code
    assert not h.value


def test_null_arguments_rejected():
    L = q.lib()
    assert L.qmc_matmul(None, None, 1, 1, None, 1, None, 0, None) == -1
    assert L.qmc_matmul_adjoint(None, None, 1, 1, None, 1, None, 0, None) == -1
    assert L.qmc_workspace_size(None, 1, None) == -1
    assert L.qmc_plan_info(None, None) == -1
    L.qmc_plan_destroy(None)


@pytest.mark.parametrize("K,s,phi,snum,sden,dtype,code", [
    (9, 3, 0, 0, 1, 0, -2),      # K not prime
    (2, 3, 0, 0, 1, 0, -1),      # K < 3
    (7, 0, 0, 0, 1, 0, -1),      # s < 1
    (7, 3, 9, 0, 1, 0, -1),      # unknown phi
    (7, 3, 0, 3, 2, 0, -1),      # shift outside [0, 1)
    (7, 3, 0, 0, 1, 5, -1),      # unknown dtype
    (7, 3, 2, 1, 7, 0, -1),      # inverse normal CDF, shift 1/K: a coordinate is 0
    (11, 3, 2, 4, 11, 1, -1),    # shift 4/K likewise
])
def test_korobov_create_rejects_before_gpu_work(K, s, phi, snum, sden, dtype, code):
    L = q.lib()
    h = ctypes.c_void_p()
    assert L.qmc_korobov_create(ctypes.byref(h), K, s, phi, snum, sden, dtype, None) == code
    assert not h.value
    assert L.qmc_korobov_plan(None) is None
