"""The double fast-path kernels keep the Jacobian row in registers that the
compiler is told it may not use (a register budget plus clobbers on every
statement that touches them); the double-double fast path keeps it in the 256
accumulation registers (AGPRs), clobbered by every statement that touches
them.  Compile the evaluation source to gfx950
assembly and check that no compiler-generated instruction touches the
pinned registers, that nothing spills to scratch, and that the kernel
descriptor reserves the pinned registers.  The GPR indexing mode those
statements use writes M0, which the compiler reserves (a clobber of it is not
honoured): no compiler-generated instruction of these kernels may use M0.
Two properties of the compiled code that cost time when lost are checked the
same way: the pinned row store reads no spilled scalars back, and the QD
kernel's lane swap sets no zero "old" operand for its DPP moves."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"

KERNELS = [(r"_ZN2ph20eval_d_pinned_kernel\S*", 128, "256"),
           (r"_ZN2ph22eval_d_pinned16_kernel\S*", 64, "128")]


def _compile(tmp_path_factory, src):
    from paper_1505_00383_amd import build as B
    kept = B.kept_asm(src)          # the assembly the build kept, if current
    if kept:
        with open(kept) as f:
            return f.read()
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("asm") / (src + ".s")
    cmd = [HIPCC, "-x", "hip"] + B.COMMON + B.DEVICE + [
        "-S", "--cuda-device-only", os.path.join(B.CSRC, src), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out.read_text()


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    return _compile(tmp_path_factory, "eval.hip")


@pytest.fixture(scope="module", params=[("eval_dd.hip", "_ZN2ph19eval_dd_arow_kernel"),
                                        ("eval_qd.hip", "_ZN2ph19eval_qd_arow_kernel")])
def asm_acc(request, tmp_path_factory):
    src, kernel = request.param
    return _compile(tmp_path_factory, src), kernel


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


def test_accumulation_register_row_untouched_by_compiler(asm_acc):
    """eval_dd_arow_kernel and eval_qd_arow_kernel: every instruction that
    names an accumulation register sits in an inline-asm block, no compiler
    instruction uses M0, no scratch, 256 AGPRs reserved and one wave per SIMD."""
    asm_dd, kernel = asm_acc
    name = re.search("^(" + kernel + r"\S*):", asm_dd, re.M).group(1)
    start = asm_dd.index(name + ":")
    end = asm_dd.index("; -- End function", start)
    body = asm_dd[start:end]
    tail = asm_dd[end:end + 3000]
    outside = re.sub(r";;#ASMSTART.*?;;#ASMEND", "", body, flags=re.S)
    code = [ln for ln in outside.split("\n") if ln.startswith("\t") and not ln.startswith("\t.")
            and not ln.strip().startswith(";")]
    bad = [ln for ln in code if re.search(r"\ba\[?\d", ln) or "accvgpr" in ln]
    assert not bad, bad[:5]
    m0 = [ln for ln in code if re.search(r"\bm0\b", ln)]
    assert not m0, m0[:5]
    assert re.search(r"; ScratchSize: (\S+)", tail).group(1) == "0"
    assert re.search(r"; Occupancy: (\S+)", tail).group(1) == "1"
    # the kernel's metadata entry: 256 AGPRs next to its name
    meta = asm_dd[asm_dd.index(".amdgpu_metadata"):]
    entry = meta[:meta.index(".name:           " + name)]
    entry = entry[entry.rindex("- .agpr_count"):]
    assert re.search(r"\.agpr_count:\s+(\d+)", entry).group(1) == "256"
    # every indexed accumulation-register access is bracketed by the index mode
    blocks = re.findall(r";;#ASMSTART(.*?);;#ASMEND", body, flags=re.S)
    for b in blocks:
        if "accvgpr" in b and "s_set_gpr_idx_on" in b:
            assert b.strip().split("\n")[-1].strip() == "s_set_gpr_idx_off", b[-200:]


def _body(asm, pattern):
    name = re.search("^(" + pattern + r"\S*):", asm, re.M).group(1)
    start = asm.index(name + ":")
    return asm[start:asm.index("; -- End function", start)]


def test_row_store_keeps_no_per_column_scalars(asm):
    """The pinned row leaves in a loop over the equation's columns, so no
    per-column bound or offset is held in scalar registers across the term
    loop and spilled to vector-register lanes (an unrolled store read 64 such
    values back per equation); a few lane spills elsewhere are allowed."""
    for pattern, _, _ in KERNELS:
        body = _body(asm, pattern)
        assert len(re.findall(r"\bv_readlane_b32\b", body)) <= 4, pattern


def test_qd_pair_swap_sets_no_zero_old_operand(tmp_path_factory):
    """Every lane has a source in the QD kernel's adjacent-lane swap, so its DPP
    moves carry no "old" operand: no DPP move writes a register whose last
    writer (in program order) set it to zero.  With a zero "old" operand every
    one of the 2672 moves had such a writer."""
    body = _body(_compile(tmp_path_factory, "eval_qd.hip"), r"_ZN2ph19eval_qd_arow_kernel")
    last, moves = {}, 0
    for ln in body.split("\n"):
        m = re.match(r"\t(v_\w+)\s+(v\d+|v\[\d+:\d+\])", ln)
        if not m:
            continue
        op, dst = m.group(1), m.group(2)
        if op == "v_mov_b32_dpp":
            moves += 1
            assert last.get(dst) != "zero", ln
        if dst.startswith("v["):
            lo, hi = (int(x) for x in dst[2:-1].split(":"))
            regs = ["v%d" % r for r in range(lo, hi + 1)]
        else:
            regs = [dst]
        kind = "zero" if re.match(r"\tv_mov_b32_e32 v\d+, 0$", ln) else "other"
        for r in regs:
            last[r] = kind
    assert moves > 0
