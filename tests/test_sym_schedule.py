"""The push order of the split 32^3 kernel's pair-symmetric form (W of source b on
target a is the conjugate of W of a on b, so each pair of k-points is transformed
once and its conjugate term pushed to the other target), checked on the host
against the library's own table builder: every ordered (target, source) pair
covered exactly once, each mirror copy's ranks in the key order that keeps the
kernel's waits free of deadlock, and the push counts. Configurations: the 32^3 /
216 k / 16-band workload, even and odd k counts, fewer targets than CU pairs, more
bands than 16, other workgroup counts, and four band orders."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
LIBDIR = os.path.join(os.path.dirname(HERE), "paper_1507_05156_amd")


def test_symmetric_schedule(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    if not os.path.exists(os.path.join(LIBDIR, "libfockmi.so")):
        pytest.skip("library not built")
    exe = str(tmp_path / "sym_schedule_check")
    subprocess.run([gxx, "-O2", "-std=c++17", os.path.join(HERE, "host", "sym_schedule_check.cpp"),
                    "-L", LIBDIR, "-lfockmi", f"-Wl,-rpath,{LIBDIR}", "-o", exe], check=True)
    run = subprocess.run([exe], capture_output=True, text=True)
    lines = [l.split() for l in run.stdout.strip().split("\n")]
    assert len(lines) == 9 * 4, run.stdout
    for nwg, nk, nb, shift, pairs, pushes, faults in lines:
        assert int(faults) == 0, (nwg, nk, nb, shift)
        nk, nb = int(nk), int(nb)
        # own pairs + pushes = every ordered pair of the application
        assert int(pairs) + int(pushes) == (nk * nb) ** 2
    assert run.returncode == 0
    big = [l for l in lines if l[1] == "216" and l[3] == "1"][0]
    assert int(big[4]) == 6027264 and int(big[5]) == 5916672
