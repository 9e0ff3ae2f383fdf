"""Count the VALU instructions per multiply-add in the Rgemm kernel's ISA.

The fast path of one k step of the NN kernel is a straight-line block that
ends at the branch into the rare exact path; it performs TM*TN multiply-adds
and is recognised by its TM*TN 64-bit products (v_mad_i64_i32) and TM*TN
exponent differences (v_sad_u32, used only by the unchecked sum).  The
k-steps of a proven k-tile are unrolled, so there is one such block per step;
the median VALU instruction count of these blocks divided by TM*TN is the
kernel's cost per multiply-add in VALU issue slots (each a 64-lane wave
instruction).  build.py records it next to the library so the benchmark can
express the kernel's throughput as a fraction of the VALU peak.
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
    blocks, cur = [], []
    for line in lines[start:end]:
        # a block ends at a branch and restarts where divergent paths rejoin
        if re.match(r"\s+s_cbranch", line) or re.match(r"\s+s_or_b64\s+exec, exec", line):
            blocks.append(cur)
            cur = []
        elif re.match(r"\s+[vsd][a-z_0-9]+", line):
            cur.append(line.split()[0])
    steps = [b for b in blocks
             if b.count("v_mad_i64_i32") == MADDS_PER_STEP and b.count("v_sad_u32") == MADDS_PER_STEP]
    if not steps:
        raise RuntimeError("fast k-step block not found in the Rgemm kernel's ISA")
    sizes = sorted(sum(x.startswith("v_") for x in b) for b in steps)
    step = next(b for b in steps if sum(x.startswith("v_") for x in b) == sizes[len(sizes) // 2])
    valu = [x for x in step if x.startswith("v_")]
    return {"valu_per_step": len(valu), "valu_per_madd": len(valu) / MADDS_PER_STEP,
            "lds_per_step": sum(x.startswith("ds_") for x in step),
            "salu_per_step": sum(x.startswith("s_") for x in step),
            "steps_found": len(steps)}


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
