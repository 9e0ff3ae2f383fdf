"""Build and run the exhaustive Posit(16,2) checker (tests/p16_checker.c)."""
import os
import subprocess
import tempfile

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def run_exhaustive(stride: int = 1) -> int:
    lib = oracle.build(force=False)
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "p16_checker")
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-o", exe,
                               os.path.join(HERE, "p16_checker.c"), lib, "-lm",
                               "-Wl,-rpath," + os.path.dirname(lib)])
        r = subprocess.run([exe, str(stride)], capture_output=True, text=True)
        print(r.stdout)
        return r.returncode
