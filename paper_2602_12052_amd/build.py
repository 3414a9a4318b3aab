"""Build libtred.so (HIP, gfx950) in-tree with hipcc.

The library carries the SHA-256 of the sources and flags it was built from
(tred_build_id()); the binding refuses a library whose id differs from the tree's.
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtred.so")
SOURCES = ["api.cpp", "effq.hip", "bin.hip", "conv.hip", "scatter.hip", "direct.hip"]
ARCH = "gfx950"


def hipcc_flags():
    return [
        "--offload-arch=" + ARCH,
        "-O3",
        "-std=c++17",
        "-fPIC",
        "-Wall",
        "-Wno-unused-function",
        "-Wno-unused-variable",
        "-Wno-unused-but-set-variable",
        "-Wno-unknown-pragmas",
        # no packed fp32 instructions in generated code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I" + os.path.join(os.path.dirname(HERE), "include"),
    ]


HEADER = os.path.join(os.path.dirname(HERE), "include", "tred.h")


def source_id(defines=()) -> str:
    """SHA-256 (hex) over the library's sources (every file in csrc/ and
    include/tred.h, by name and content), the compiler flags and the defines."""
    h = hashlib.sha256()
    files = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC)
                   if os.path.isfile(os.path.join(CSRC, f)))
    for path in files + [HEADER]:
        h.update(os.path.basename(path).encode() + b"\0")
        with open(path, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    # flags without include paths: the id must not depend on where the tree sits
    flags = [f for f in hipcc_flags() if not f.startswith("-I")]
    h.update(" ".join(flags + ["-D" + d for d in defines]).encode())
    return h.hexdigest()


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile every HIP/C++ source of the library and link libtred.so (or `out`)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    bid = source_id(defines)
    objdir = os.path.join(HERE, "_build" if out == LIB else "_build_" + os.path.basename(out))
    os.makedirs(objdir, exist_ok=True)
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [hipcc] + hipcc_flags() + ["-D" + d for d in defines] + lang + \
            ['-DTRED_BUILD_ID="%s"' % bid, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        log, _ = p.communicate()
        text = log.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 target feature: harmless
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write("\n".join(lines) + "\n")
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    tmp = out + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
