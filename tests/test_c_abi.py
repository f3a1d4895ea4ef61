"""The C ABI used from a plain C program (tests/c/c_abi_demo.c), compared with the oracle.

The program is compiled by the build step; the host checks need no GPU, the render and
backward checks run on the GPU."""

from __future__ import annotations

import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
EXE = os.path.join(HERE, "c", "c_abi_demo")


def _exe():
    if not os.path.exists(EXE):
        pytest.skip("tests/c/c_abi_demo is not built (the build step compiles it)")
    return EXE


def test_c_program_host_calls():
    r = subprocess.run([_exe(), "host"], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host checks OK" in r.stdout


@pytest.mark.gpu
def test_c_program_render_and_backward():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    r = subprocess.run([_exe(), "gpu"], capture_output=True, text=True, timeout=120)
    print(r.stdout, flush=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "gpu checks OK" in r.stdout
