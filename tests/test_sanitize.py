"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the CPU code (no GPU needed):
the FP64 oracle (gcc), and the library's host runtime (hipcc, sanitizers on the host
pass only): the Revolve schedule and its counts, the profile planner, the run-time model
and strategy choice (which replay the executor's bookkeeping on the host), and the
set-up of solo and batched calls.  Each driver prints OK; any sanitizer report aborts it."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")


def _run(cmd, **kw):
    p = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert p.returncode == 0, f"{' '.join(cmd)}\n{p.stdout[-2000:]}\n{p.stderr[-4000:]}"
    return p


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1",
          "-std=c11", "-fopenmp", "-ffp-contract=off", os.path.join(ROOT, "oracle", "wv_oracle.c"),
          os.path.join(SAN, "oracle_main.c"), "-o", exe, "-lm"])
    p = _run([exe], env=dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1"))
    assert p.stdout.strip().endswith("OK")


@pytest.mark.slow
@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_host_runtime_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1810_05268_amd", "csrc")
    srcs = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith(".hip"))
    host = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
            "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    common = ["-O1", "-g", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run(["hipcc", "-c", "--offload-arch=gfx950", *common, *host, src, "-o", obj])
        return obj
    jobs = srcs + [os.path.join(SAN, "host_main.cpp")]
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, jobs))
    exe = str(tmp_path / "host_san")
    _run(["hipcc", "--offload-arch=gfx950", "-fsanitize=address,undefined", "-fno-gpu-sanitize", *objs, "-o", exe])
    p = _run([exe], env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert p.stdout.strip().endswith("OK")
