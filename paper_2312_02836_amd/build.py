"""Build libburn.so (the HIP kernels and the C ABI) for gfx950 with hipcc.

    python -m paper_2312_02836_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libburn.so")

BUILD = os.path.join(HERE, "_build")

SOURCES = ["burn_api.cpp", "burn_codegen.cpp", "burn_multi.hip", "burn_plain_p0.hip", "burn_plain_p1.hip",
           "burn_plain_p2.hip", "burn_adjoint.hip", "burn_sdc.hip",
           "burn_screen.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++20", "-fPIC",
    # no packed-FP32 instructions anywhere (all arithmetic here is FP64)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


# headers of the generated kernels' body, embedded in the library as text
# (the per-network sources are compiled with them at run time)
GEN_HEADERS = [("BNG_BODY_H", "burn_gen_body.h"), ("BNG_ARGS_H", "burn_gen_args.h"),
               ("BNG_MATH_H", "bn_math.h")]


def write_gen_headers() -> str:
    """_build/burn_gen_headers.inc: each body header as a C string."""
    os.makedirs(BUILD, exist_ok=True)
    out = os.path.join(BUILD, "burn_gen_headers.inc")
    parts = []
    for name, fn in GEN_HEADERS:
        with open(os.path.join(CSRC, fn)) as f:
            text = f.read()
        if ")BNGSRC\"" in text:
            raise RuntimeError(fn + " contains the raw-string delimiter")
        parts.append(f'static const char {name}[] = R"BNGSRC({text})BNGSRC";\n')
    tmp = out + ".tmp"
    with open(tmp, "w") as f:
        f.write("".join(parts))
    os.replace(tmp, out)
    return out


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel, one object each) and link
    libburn.so (always recompiles)."""
    write_gen_headers()
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-I", BUILD]
    with tempfile.TemporaryDirectory(prefix="burn_build_") as tmpd:
        objs, procs = [], []
        for src in SOURCES:
            obj = os.path.join(tmpd, src + ".o")
            cmd = [hipcc()] + HIPCC_FLAGS + inc + ["-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd)))
            objs.append(obj)
        failed = [src for src, p in procs if p.wait() != 0]
        if failed:
            raise RuntimeError("hipcc failed on " + ", ".join(failed))
        tmp = LIB + ".tmp"
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + [
            "-L/opt/rocm/lib", "-lhiprtc", "-Wl,-rpath,/opt/rocm/lib", "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
