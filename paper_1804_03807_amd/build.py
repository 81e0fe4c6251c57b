"""Builds libhomotopy.so (HIP kernels for gfx950 + host C ABI) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libhomotopy.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["tracker.hip", "lanes.hip", "dense.hip", "dense11.hip", "dense12.hip",
           "dense_sliced.hip", "dense_wide_sliced.hip", "endgame.hip", "endgame_dense.hip",
           "endgame_dense_wide.hip",
           "dedup.hip", "dedup_static.hip", "ddtrack.hip", "serve.hip", "hp_host.cpp", "hp_jit.cpp"]
# headers the run-time specialised kernels are compiled with (hiprtc)
JIT_HEADERS = [("homotopy.h", os.path.join(ROOT, "include", "homotopy.h")),
               ("hp_internal.hpp", os.path.join(CSRC, "hp_internal.hpp")),
               ("hp_device.hpp", os.path.join(CSRC, "hp_device.hpp")),
               ("lane_track.hpp", os.path.join(CSRC, "lane_track.hpp")),
               ("spec_track.hpp", os.path.join(CSRC, "spec_track.hpp")),
               ("reg_lu.hpp", os.path.join(CSRC, "reg_lu.hpp"))]
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         # no packed FP32 instructions anywhere in device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-Wno-pass-failed"]


def write_jit_headers(path: str) -> None:
    """The JIT header texts as C++ raw string literals (hp_jit.cpp includes them)."""
    names, texts = [], []
    for name, src in JIT_HEADERS:
        with open(src) as fh:
            text = fh.read()
        if ")HPJIT\"" in text:
            raise RuntimeError(f"{src}: contains the raw-string delimiter")
        names.append(f'"{name}"')
        texts.append('R"HPJIT(' + text + ')HPJIT"')
    out = ("const char *const kJitHeaderNames[] = {" + ", ".join(names) + "};\n"
           "const char *const kJitHeaderTexts[] = {\n" + ",\n".join(texts) + "};\n")
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        fh.write(out)
    os.replace(tmp, path)


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    write_jit_headers(os.path.join(objdir, "hp_jit_headers.inc"))
    inc = ["-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-I" + objdir]
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        cmd = [HIPCC, *FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [HIPCC, "-x", "hip", *FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    tmp = SO + ".tmp"
    subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", tmp,
                    "-lhiprtc"], check=True)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
