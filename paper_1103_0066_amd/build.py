"""Builds libfei.so (HIP for gfx950) in-tree.

Steps: compile and run the reference-tensor table generator (g++), then
compile the device translation unit and the host layer with hipcc and link
them into paper_1103_0066_amd/libfei.so.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
GEN = os.path.join(CSRC, "_gen")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libfei.so")
ARCH = os.environ.get("FEI_OFFLOAD_ARCH", "gfx950")

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          # no packed FP32 instructions in any device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-missing-braces"]


def _run(cmd, quiet=False):
    r = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stderr or "").splitlines()
                    if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{err}")
    if err.strip() and not quiet:
        sys.stderr.write(err + "\n")
    return r.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(GEN, exist_ok=True)
    gen_exe = os.path.join(GEN, "gen_tables")
    _run(["g++", "-std=c++17", "-O1", "-DFEI_HD=", "-I", CSRC,
          os.path.join(CSRC, "gen_tables.cpp"), "-o", gen_exe])
    tables = _run([gen_exe])
    tmp = os.path.join(GEN, "tables.inc.tmp")
    with open(tmp, "w") as f:
        f.write(tables)
    os.replace(tmp, os.path.join(GEN, "tables.inc"))

    sources = ["kernels.hip", "api.cpp", "batch.cpp", "assembly.cpp", "noalloc.cpp", "forms.cpp", "tune.cpp"]
    objs = [os.path.join(GEN, os.path.splitext(s)[0] + ".o") for s in sources]

    def compile_one(args):
        src, obj = args
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        _run([HIPCC, *COMMON, *lang, "-c", os.path.join(CSRC, src), "-o", obj], quiet=not verbose)

    with ThreadPoolExecutor(max_workers=len(sources)) as ex:
        list(ex.map(compile_one, zip(sources, objs)))
    tmp_lib = LIB + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp_lib])
    os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
