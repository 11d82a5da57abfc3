"""Build libbinar.so (the gfx950 HIP library) in-tree with hipcc.

The host code is split into translation units (the API, and the launch
sequences of each key width with and without payload) that compile in parallel, then link into one
shared library."""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbinar.so")
SOURCES = [os.path.join(CSRC, f) for f in
           ["binar_api.hip", "binar_static.hip", "binar_stream.hip"] + ["binar_launch_%d%s.hip" % (kb, t) for kb in (4, 8, 16) for t in "pk"]]
HEADERS = [os.path.join(CSRC, f) for f in
           ("binar_host.h", "binar_kernels.h", "binar_keys.h", "binar_inplace.h", "binar_strings.h")]
DEPS = SOURCES + HEADERS + [os.path.join(ROOT, "include", "binar.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed fp32 instructions stay off (no float math here, but keep the rule)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(p) > t for p in DEPS)


def _filter(text: str) -> str:
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)


def build(force: bool = True) -> str:
    if not force and not stale():
        return LIB
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    with tempfile.TemporaryDirectory(prefix="binar_build_") as tmpdir:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            objs.append(obj)
            procs.append((src, subprocess.Popen([hipcc] + HIPCC_FLAGS + ["-c", "-o", obj, src],
                                                stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
        errors = []
        for src, p in procs:
            out, _ = p.communicate()
            if p.returncode != 0:
                errors.append("%s:\n%s" % (os.path.basename(src), _filter(out)))
        if errors:
            raise RuntimeError("hipcc failed:\n" + "\n".join(errors))
        tmp = LIB + ".tmp%d" % os.getpid()
        proc = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs,
                              stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if proc.returncode != 0:
            raise RuntimeError("hipcc link failed:\n" + _filter(proc.stdout))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
