"""Build libposit32.so (HIP, gfx950 only) in-tree with hipcc."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libposit32.so")
SOURCES = ["p32_gemm.hip", "p32_elementwise.hip", "p32_lapack.hip", "p32_batched.hip", "p32_server.hip",
           "p32_api.cpp"]
ARCH = "gfx950"


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the Posit(32,2) library needs ROCm's hipcc")


def flags() -> list[str]:
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            # packed FP32 instructions are never wanted here (integer code)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-result", "-pthread", "-I", os.path.join(HERE, "..", "include")]


def build(verbose: bool = False, out: str | None = None, defines: list[str] | None = None) -> str:
    """Compile and link the library (to `out`, default in-tree); `defines`
    are extra -D options for tuning builds."""
    cc = hipcc()
    lib = out or LIB
    extra = ["-D" + d for d in (defines or [])]
    objdir = os.path.join(os.path.dirname(lib), "_build_" + os.path.basename(lib).replace(".", "_"))
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src: str) -> str:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        # every translation unit, host-only ones included, is built for gfx950 only
        cmd = [cc] + flags() + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError(f"hipcc failed on {src}")
        if verbose:
            sys.stderr.write(r.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = lib + ".tmp"
    r = subprocess.run([cc, "-shared", "-pthread", f"--offload-arch={ARCH}", "-o", tmp] + objs,
                       capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libposit32.so failed")
    os.replace(tmp, lib)
    if out is None:
        from paper_2401_14117_amd import isa_count
        isa_count.write_report(cc, flags(), os.path.join(HERE, "libposit32.isa.json"))
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
