"""Host code under AddressSanitizer + UndefinedBehaviorSanitizer: the
database layout (layout.cpp), the hybrid search's host scorer
(cpu_scorer.cpp), the traceback walk (trace_walk.cpp, over codes the driver
computes from their definition) and the C oracle (sw_oracle.c), built with the sanitizers
into one driver (tests/sanitize/driver.cpp) and run on random and edge-case
inputs.  CPU only."""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(not os.path.exists(CLANG), reason="clang++ not available")
def test_host_code_under_sanitizers():
    csrc = os.path.join(ROOT, "paper_2203_11100_amd", "csrc")
    with tempfile.TemporaryDirectory() as tmp:
        objs = []
        for src, lang in ((os.path.join(csrc, "layout.cpp"), "c++"),
                          (os.path.join(csrc, "cpu_scorer.cpp"), "c++"),
                          (os.path.join(csrc, "trace_walk.cpp"), "c++"),
                          (os.path.join(ROOT, "oracle", "sw_oracle.c"), "c"),
                          (os.path.join(ROOT, "tests", "sanitize", "driver.cpp"), "c++")):
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            std = ["-std=c++17"] if lang == "c++" else ["-std=c99"]
            subprocess.check_call([CLANG, "-x", lang, "-O1", "-g", "-pthread"] + std + SAN +
                                  ["-c", src, "-o", obj])
            objs.append(obj)
        exe = os.path.join(tmp, "driver")
        subprocess.check_call([CLANG, "-pthread"] + SAN + objs + ["-o", exe])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
