"""Builds libprocray.so (HIP kernels + host library) for gfx950 with hipcc.

Run as ``python -m paper_2012_10357_amd.build`` or call ``build()``.  The
library is built in-tree next to this file so that it travels with the
source tree.
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libprocray.so")

SOURCES = ["trace.hip", "noalloc.hip", "scene.cpp", "render.cpp", "server.cpp", "user_de.cpp"]

# Kernel sources the library carries as text, to rebuild the kernel with
# user-registered estimators at run time.
EMBEDDED = [("kEmbeddedTraceHip", os.path.join(CSRC, "trace.hip")),
            ("kEmbeddedDeH", os.path.join(CSRC, "de.h")),
            ("kEmbeddedInternalH", os.path.join(CSRC, "internal.h")),
            ("kEmbeddedProcrayH", os.path.join(HERE, "..", "include", "procray.h"))]


def _embedded_sources(path: str) -> None:
    delim = "PRSRC"
    out = ["// Generated at build time: kernel sources as text.", "namespace pr {"]
    for name, src in EMBEDDED:
        text = open(src).read()
        if ")" + delim + '"' in text:
            raise RuntimeError(f"{src} contains the raw-string delimiter")
        out.append(f'extern const char* const {name} = R"{delim}({text}){delim}";')
    out.append("}  // namespace pr")
    with open(path, "w") as f:
        f.write("\n".join(out) + "\n")

# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Wno-unused-command-line-argument"]


def build(verbose: bool = False, extra=None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tmp = LIB + ".tmp"
    gen_dir = tempfile.mkdtemp(prefix="procray_build_")
    gen = os.path.join(gen_dir, "embedded_sources.cpp")
    _embedded_sources(gen)
    cmd = [hipcc] + DEVICE_FLAGS + (extra or []) + ["-I", os.path.join(HERE, "..", "include"),
                                                    "-o", tmp] + srcs + [gen, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    try:
        r = subprocess.run(cmd, capture_output=True, text=True)
    finally:
        os.remove(gen)
        os.rmdir(gen_dir)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libprocray.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
