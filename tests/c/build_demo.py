"""Compile tests/c/c_abi_demo.c against the library (libfmb.so), the oracle library and the HIP
runtime with the host C compiler.  Run after the library and the oracle are built."""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "c_abi_demo.c")
EXE = os.path.join(HERE, "c_abi_demo")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build() -> str:
    pkg = os.path.join(ROOT, "paper_2308_14737_amd")
    orc = os.path.join(ROOT, "oracle")
    tmp = EXE + ".tmp"
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
           f"-I{os.path.join(ROOT, 'include')}", SRC, "-o", tmp, f"-L{pkg}", "-lfmb", f"-L{orc}", "-lfmb_oracle",
           f"-L{ROCM}/lib", "-lamdhip64", "-lm", f"-Wl,-rpath,$ORIGIN/../../paper_2308_14737_amd:$ORIGIN/../../oracle:{ROCM}/lib"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, EXE)
    return EXE


if __name__ == "__main__":
    print(build())
