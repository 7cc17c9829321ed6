"""Build libwv.so (all HIP sources, gfx950) in-tree with hipcc."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libwv.so")
SOURCES = sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))
HEADERS = sorted(glob.glob(os.path.join(HERE, "csrc", "*.h"))) + [os.path.join(HERE, "..", "include", "wv.h")]
ARCH = os.environ.get("WV_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions (keep scalar/float2 FP32 code on plain VALU ops)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unused-command-line-argument",
]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in SOURCES + HEADERS)


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and not stale():
        return LIB
    objs = []
    jobs = []
    for src in SOURCES:
        obj = os.path.join(HERE, "csrc", os.path.basename(src) + f".{os.getpid()}.o")
        cmd = ["hipcc", "-c", *[f for f in FLAGS if f != "-shared"], src, "-o", obj]
        jobs.append((cmd, obj))
    procs = [(subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), o, c) for c, o in jobs]
    failed = False
    for p, o, c in procs:
        out, _ = p.communicate()
        txt = out.decode(errors="replace")
        txt = "\n".join(l for l in txt.splitlines() if "packed-fp32-ops" not in l)
        if p.returncode != 0:
            failed = True
            sys.stderr.write(f"FAILED: {' '.join(c)}\n{txt}\n")
        elif verbose and txt.strip():
            sys.stderr.write(txt + "\n")
        objs.append(o)
    try:
        if failed:
            raise RuntimeError("hipcc failed")
        tmp = LIB + f".tmp{os.getpid()}"
        subprocess.run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp], check=True,
                       stderr=subprocess.PIPE)
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    build(force=True, verbose=True)
    print(LIB)
