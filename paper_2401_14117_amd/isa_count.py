"""Count the VALU instructions per multiply-add in the Rgemm kernel's ISA.

The fast path of one k step of the NN kernel is the straight-line block that
begins at the inner k-loop header and ends at the branch into the rare exact
path; it performs TM*TN multiply-adds.  Its VALU instruction count divided by
TM*TN is the kernel's cost per multiply-add in VALU issue slots (each a
64-lane wave instruction).  build.py records it next to the library so the
benchmark can express the kernel's throughput as a fraction of the VALU peak.
"""
from __future__ import annotations

import hashlib
import json
import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL = "_ZN3p3211gemm_kernelILb0ELb0ELb0ELb0EEEvlllPKjlS2_lPjljjPKi"
MADDS_PER_STEP = 8    # TM * TN of the kernel


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("p32_device.hpp", "p32_gemm_tile.hpp", "p32_gemm.hip"):
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def count(asm_text: str) -> dict:
    lines = asm_text.splitlines()
    start = next(i for i, l in enumerate(lines) if l.startswith(KERNEL + ":"))
    end = next(i for i in range(start, len(lines)) if "s_endpgm" in lines[i])
    body = lines[start:end]
    head = next(i for i, l in enumerate(body) if "Inner Loop Header: Depth=2" in l)
    stop = next(i for i in range(head + 1, len(body)) if "s_cbranch" in body[i])
    insts = [l.split()[0] for l in body[head + 1:stop] if re.match(r"\s+[vsd][a-z_0-9]+", l)]
    valu = [x for x in insts if x.startswith("v_")]
    return {"valu_per_step": len(valu), "valu_per_madd": len(valu) / MADDS_PER_STEP,
            "lds_per_step": sum(x.startswith("ds_") for x in insts),
            "salu_per_step": sum(x.startswith("s_") for x in insts)}


def write_report(hipcc: str, flags: list[str], out_path: str) -> dict:
    src = os.path.join(HERE, "csrc", "p32_gemm.hip")
    asm = subprocess.run([hipcc] + flags + ["--cuda-device-only", "-S", "-o", "-", src],
                         capture_output=True, text=True, check=True).stdout
    info = count(asm)
    info["kernel"] = KERNEL
    info["kernel_hash"] = source_hash()
    with open(out_path, "w") as f:
        json.dump(info, f, indent=1)
    return info
