"""The library's host-only entry points (SAM formatting, MAPQ argument
checks, index parameter validation) under the host address and
undefined-behaviour sanitizers: tests/host_checks.cpp is linked with the
index and report sources, instrumented on the host side only, and run on
the CPU (no GPU needed)."""
import os
import shutil
import subprocess
import tempfile

import pytest

from paper_1403_2136_amd import build as b

HERE = os.path.dirname(os.path.abspath(__file__))
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-fno-omit-frame-pointer"]


def test_host_entry_points_clean_under_sanitizers():
    if not os.path.exists(b.HIPCC):
        pytest.skip("hipcc not available")
    d = tempfile.mkdtemp()
    try:
        objs = []
        for src in (os.path.join(b.CSRC, "index.hip"), os.path.join(b.CSRC, "report.hip"),
                    os.path.join(HERE, "host_checks.cpp")):
            obj = os.path.join(d, os.path.basename(src) + ".o")
            cmd = [b.HIPCC, "-O1", "-g", "-std=c++17", "--offload-arch=" + b.ARCH,
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                   "-I", os.path.join(b.ROOT, "include")] + SAN + ["-c", src, "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-2000:]
            objs.append(obj)
        exe = os.path.join(d, "host_checks")
        r = subprocess.run([b.HIPCC, "--offload-arch=" + b.ARCH, "-fsanitize=address",
                            "-fsanitize=undefined", "-o", exe] + objs,
                           capture_output=True, text=True)
        if r.returncode != 0:
            pytest.skip("sanitizer runtime not linkable here: %s" % r.stderr[-300:])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
        assert r.returncode == 0 and "host checks: ok" in r.stdout, r.stdout + r.stderr[-3000:]
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    finally:
        shutil.rmtree(d, ignore_errors=True)
