"""The double fast-path kernels keep the Jacobian row in registers that the
compiler is told it may not use (a register budget plus clobbers on every
statement that touches them).  Compile the evaluation source to gfx950
assembly and check that no compiler-generated instruction touches the
pinned registers, that nothing spills to scratch, and that the kernel
descriptor reserves the pinned registers.  The GPR indexing mode those
statements use writes M0, which the compiler reserves (a clobber of it is not
honoured): no compiler-generated instruction of these kernels may use M0."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"

KERNELS = [(r"_ZN2ph20eval_d_pinned_kernel\S*", 128, "256"),
           (r"_ZN2ph22eval_d_pinned16_kernel\S*", 64, "128")]


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    from paper_1505_00383_amd import build as B
    out = tmp_path_factory.mktemp("asm") / "eval.s"
    cmd = [HIPCC, "-x", "hip"] + B.COMMON + B.DEVICE + [
        "-S", "--cuda-device-only", os.path.join(B.CSRC, "eval.hip"), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out.read_text()


@pytest.mark.parametrize("pattern,first_pinned,vgprs", KERNELS)
def test_pinned_registers_untouched_by_compiler(asm, pattern, first_pinned, vgprs):
    name = re.search("^(" + pattern + "):", asm, re.M).group(1)
    start = asm.index(name + ":")
    end = asm.index("; -- End function", start)
    body = asm[start:end]
    tail = asm[end:end + 3000]
    outside = re.sub(r";;#ASMSTART.*?;;#ASMEND", "", body, flags=re.S)
    bad = [ln for ln in outside.split("\n")
           if any(int(m.group(2) or m.group(3)) >= first_pinned
                  for m in re.finditer(r"v\[(\d+):(\d+)\]|\bv(\d+)\b", ln))]
    assert not bad, bad[:5]
    m0 = [ln for ln in outside.split("\n") if re.search(r"\bm0\b", ln)]
    assert not m0, m0[:5]
    assert re.search(r"; ScratchSize: (\S+)", tail).group(1) == "0"
    assert re.search(r"; NumVgprs: (\S+)", tail).group(1) == vgprs
