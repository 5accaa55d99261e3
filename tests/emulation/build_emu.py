"""Builds the CPU emulation of libimb (test infrastructure): the kernel sources of
paper_1809_07008_amd/csrc compiled by g++ against the emulated HIP headers of this directory, with
AddressSanitizer, into _build/emu/libimb_emu.so.  The only source edits are the dynamic-LDS
declaration of the particle-phase kernel, which becomes a pointer to the emulated buffer, and
clang's four-element vector attribute, written as g++'s vector_size(16)."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1809_07008_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "emu")
LIB = os.path.join(OUT, "libimb_emu.so")
FLAGS = ["-std=c++20", "-O1", "-g", "-fPIC", "-fsanitize=address", "-fno-omit-frame-pointer",
         "-ffp-contract=off", "-Wno-unknown-pragmas", "-Wno-ignored-attributes", "-pthread"]


def build() -> str:
    src = os.path.join(OUT, "src")
    shutil.rmtree(OUT, ignore_errors=True)
    os.makedirs(src)
    for f in glob.glob(os.path.join(CSRC, "*.h")):
        shutil.copy(f, src)
    for f in glob.glob(os.path.join(CSRC, "*.hip")):
        text = open(f).read().replace("extern __shared__ double lds[];",
                                      "double* lds = (double*)emu_dyn_lds();")
        # clang's vector extension written in g++'s form
        text = text.replace("__attribute__((ext_vector_type(4)))",
                            "__attribute__((vector_size(16)))")
        with open(os.path.join(src, os.path.basename(f)[:-4] + ".cpp"), "w") as fh:
            fh.write(text)
    units = glob.glob(os.path.join(src, "*.cpp")) + [os.path.join(HERE, "emu.cpp")]
    inc = ["-I" + HERE, "-I" + src, "-I" + os.path.join(ROOT, "include")]

    def compile_one(u):
        o = os.path.join(src, os.path.basename(u)[:-4] + ".o")
        r = subprocess.run(["g++", *FLAGS, *inc, "-c", u, "-o", o], capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError("g++ failed for %s:\n%s" % (u, r.stderr[-4000:]))
        return o

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, units))
    subprocess.check_call(["g++", "-shared", "-fsanitize=address", "-pthread", *objs, "-o", LIB])
    return LIB


if __name__ == "__main__":
    print(build())
