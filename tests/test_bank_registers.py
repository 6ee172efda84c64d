"""The register-bank scan kernels (plain scores, and the quality split's
reads with one score pair) keep their state in v64..v255 between asm
statements, so the compiler's own code in them must stay in v0..v63.  This
compiles the scan source to gfx950 assembly (no GPU needed) and checks the
compiler-generated instructions of each kernel, outside the asm statements,
against that range, and that the kernels spill no VGPRs."""
import os
import re
import subprocess
import tempfile

import pytest

from paper_1403_2136_amd import build as b

KERNELS = ["_ZN5maxss16scan_kernel_bankENS_8ScanArgsE",
           "_ZN5maxss21scan_kernel_bank_qualENS_8ScanArgsE"]


def _vgprs(line):
    regs = [int(x) for x in re.findall(r"\bv(\d+)\b", line)]
    for lo, hi in re.findall(r"\bv\[(\d+):(\d+)\]", line):
        regs += list(range(int(lo), int(hi) + 1))
    return regs


@pytest.fixture(scope="module")
def scan_asm():
    if not os.path.exists(b.HIPCC):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "scan.s")
        cmd = [b.HIPCC] + b.FLAGS + ["-S", "--cuda-device-only",
                                     os.path.join(b.CSRC, "scan.hip"), "-o", out]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return open(out).read()


@pytest.fixture(params=KERNELS, ids=["plain", "quality"])
def kernel_asm(scan_asm, request):
    text, kernel = scan_asm, request.param
    start = text.index(kernel + ":")
    end = text.index(".Lfunc_end", start)
    name = text.index(".name:           " + kernel)
    meta = text[text.rindex("- .agpr_count", 0, name):name + 600]
    return text[start:end], meta


def test_compiler_code_stays_below_v64(kernel_asm):
    body, _ = kernel_asm
    inside, bad, seen = False, [], 0
    for line in body.split("\n"):
        s = line.strip()
        if s.startswith(";;#ASMSTART"):
            inside = True
            continue
        if s.startswith(";;#ASMEND"):
            inside = False
            continue
        if inside or not s or s.startswith((";", ".")) or s.endswith(":"):
            continue
        seen += 1
        if any(v >= 64 for v in _vgprs(s.split(";")[0])):
            bad.append(s)
    assert seen > 100
    assert not bad, "compiler code touches v64+: %s" % bad[:5]


def test_no_vgpr_spills_and_all_registers_allocated(kernel_asm):
    _, meta = kernel_asm
    assert re.search(r"\.vgpr_spill_count:\s+0\b", meta), meta
    assert re.search(r"\.vgpr_count:\s+256\b", meta), meta
    assert re.search(r"\.agpr_count:\s+0\b", meta), meta
