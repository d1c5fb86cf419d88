"""The split 32^3 kernel reads data that another CU stored during the same launch:
the other half's exchange mailbox and, in the pair-symmetric form, the mirror
copies' partial and FP64 sums. On gfx950 an ordinary load may return a line of
this CU's L1 that the other CU's stores have made stale, and an L1 invalidate at
workgroup scope does not remove such lines. These reads must therefore be
device-coherent loads (cache policy SC1). This test compiles the kernel for
gfx950 on the host and checks its buffer loads: per thread and pair, 32 mailbox
loads in both forms, plus 32 partial-sum loads and 6 fold loads (two partial,
two FP64 sum, two compensation) in the symmetric form; no other load is SC1,
and no cache invalidate is left."""

import os
import re
import subprocess

import pytest

from paper_1507_05156_amd import build as B

SRC = os.path.join(B.CSRC, "split32.hip")
KERNELS = {
    True: "_ZN6fockmi12_GLOBAL__N_114split32_kernelILb1EEEvNS_9SplitArgsE",
    False: "_ZN6fockmi12_GLOBAL__N_114split32_kernelILb0EEEvNS_9SplitArgsE",
}


@pytest.fixture(scope="module")
def device_asm(tmp_path_factory):
    try:
        hipcc = B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not found")
    out = str(tmp_path_factory.mktemp("split32") / "split32.s")
    cmd = [hipcc, *B.FLAGS, "--cuda-device-only", "-S", SRC, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return open(out).read()


def _body(asm: str, sym: str) -> str:
    start = asm.index(sym + ":")
    return asm[start:asm.index(".Lfunc_end", start)]


@pytest.mark.parametrize("sym,coherent", [(True, 32 + 32 + 6), (False, 32)])
def test_cross_cu_reads_are_device_coherent(device_asm, sym, coherent):
    body = _body(device_asm, KERNELS[sym])
    loads = [l.strip() for l in body.split("\n") if l.strip().startswith("buffer_load")]
    sc1 = [l for l in loads if re.search(r"\bsc1\b", l)]
    assert len(sc1) == coherent, "\n".join(sc1)
    assert "buffer_inv" not in body
