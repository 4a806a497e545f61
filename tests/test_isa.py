"""Checks on the gfx950 code the compiler emits for the hot kernels (CPU only).

Two properties are enforced on the assembly of every kernel source:

* every FP32 matrix-core chain accumulates in place: an MFMA whose source C
  is a register tuple other than its destination (a chain the compiler has
  moved between tuples) is rejected. Such a move, with vector writes to the
  old tuple in between, lost one step's contribution in the last accumulator
  register of a Gram tile on gfx950; the kernels are written so that the
  compiler keeps each chain in one tuple, and this test keeps it that way.
* no kernel writes through the scalar data cache (scalar stores or atomics).
"""
import concurrent.futures
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2510_02774_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["round.hip", "round_ip.hip", "round_bf16.hip", "round_fp16.hip", "round_fp8.hip", "quant.hip", "kernels.hip", "order.hip", "search.hip"]

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None,
                                reason="hipcc not available")

MFMA = re.compile(r"^\s*(v_mfma\S*)\s+(\S+),\s*(\S+),\s*(\S+),\s*(\S+)")
SCALAR_WRITE = re.compile(r"^\s*s_(store|atomic|buffer_store|scratch_store|dcache_wb)")


def _asm(src, tmp_path):
    out = tmp_path / (src + ".s")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-x", "hip",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-S", "--cuda-device-only",
           os.path.join(CSRC, src), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out.read_text()


def _kernels(asm):
    """Yields (name, lines) per function body."""
    for m in re.finditer(r"^(_ZN5grnnd\w+):", asm, re.M):
        end = asm.index(".Lfunc_end", m.end())
        yield m.group(1), asm[m.end():end].splitlines()


def test_mfma_chains_accumulate_in_place_and_no_scalar_writes(tmp_path):
    with concurrent.futures.ThreadPoolExecutor(len(SOURCES)) as ex:
        asms = list(ex.map(lambda src: _asm(src, tmp_path), SOURCES))
    moved, scalar = [], []
    nk = 0
    for name, lines in (kl for asm in asms for kl in _kernels(asm)):
        nk += 1
        for ln in lines:
            m = MFMA.match(ln)
            if m and m.group(5) != "0" and m.group(5) != m.group(2):
                moved.append(f"{name}: {ln.strip()}")
            if SCALAR_WRITE.match(ln):
                scalar.append(f"{name}: {ln.strip()}")
    assert nk > 0
    assert not moved, "MFMA chain moved between register tuples:\n" + "\n".join(moved[:10])
    assert not scalar, "scalar-cache writes:\n" + "\n".join(scalar[:10])
