"""The register DFTs of the kernels (csrc/cx.hpp: Stockham stages of radix
4 and 2, and one radix-3 or radix-5 stage for the lengths 3 x 2^k and
5 x 2^k of the outer transform) built for the host with g++ and compared
with numpy's FFT on a fixed input: forward exp(-2 pi i jk/N) and the
unscaled inverse, every length the kernels instantiate (2^k <= 64,
3 x 2^k <= 96, 5 x 2^k <= 80)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
LENGTHS = [1, 2, 4, 8, 16, 32, 64, 3, 6, 12, 24, 48, 96, 5, 10, 20, 40, 80]


@pytest.fixture(scope="module")
def dfts(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("regdft") / "regdft")
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", os.path.join(HERE, "host_shim"), "-o", exe,
                    os.path.join(HERE, "host_regdft.cpp")], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    res, i = {}, 0
    while i < len(out) and out[i]:
        _, n, d = out[i].split()
        n, d = int(n), int(d)
        vals = np.array([[float(x) for x in out[i + 1 + k].split()] for k in range(n)])
        res[(n, d)] = vals[:, 0] + 1j * vals[:, 1]
        i += 1 + n
    return res


@pytest.mark.parametrize("n", LENGTHS)
def test_register_dft_matches_numpy(dfts, n):
    i = np.arange(n)
    x = np.sin(1.3 * i + 0.2) + 1j * np.cos(0.7 * i * i + 1.0)
    fwd, inv = dfts[(n, -1)], dfts[(n, +1)]
    scale = np.abs(x).sum()
    assert np.max(np.abs(fwd - np.fft.fft(x))) <= 1e-15 * scale * max(1, np.log2(n))
    assert np.max(np.abs(inv - n * np.fft.ifft(x))) <= 1e-15 * scale * max(1, np.log2(n))
