"""The register FFTs of the pair kernels (fft_reg.hpp), built for the host from
the same source and compared with a direct DFT (the discrete sums of Eq. (15)).

Covers every transform length of the supported grids and a few longer mixed
lengths, both signs, with and without twiddle folding, in FP64 and FP32. A wrong
twiddle, index map or sign gives errors of order one; the bounds sit about ten
times above the rounding the transforms show."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1507_05156_amd", "csrc")
LENGTHS = {2, 3, 4, 5, 6, 8, 10, 12, 16, 20, 24, 32, 40, 48}


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("fft") / "fft_host_check")
    subprocess.run([gxx, "-O1", "-std=c++17", "-DFOCKMI_FFT_HOST_CHECK", "-I", CSRC,
                    os.path.join(HERE, "host", "fft_host_check.cpp"), "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    rows = {}
    for line in out.split("\n"):
        if line.strip():
            n, sign, fold, typ, err = line.split()
            rows[(int(n), int(sign), int(fold), typ)] = float(err)
    return rows


def test_every_case_ran(results):
    assert {k[0] for k in results} == LENGTHS
    assert len(results) == len(LENGTHS) * 2 * 2 * 2


def test_fp64_transforms_match_the_dft(results):
    # largest output error over the input's 2-norm; rounding gives < 1e-15
    bad = {k: e for k, e in results.items() if k[3] == "f64" and not e < 1e-14}
    assert not bad, bad


def test_fp32_transforms_match_the_dft(results):
    # relative 2-norm error; FP32 rounding gives 5e-8 to 8e-8 at these lengths
    bad = {k: e for k, e in results.items() if k[3] == "f32" and not e < 4e-7}
    assert not bad, bad
