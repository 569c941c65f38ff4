"""Build libph.so (HIP for gfx950) in-tree with hipcc.

    python -m paper_1505_00383_amd.build

Every source in csrc/ is compiled to an object under _build/ (in parallel) and
linked into paper_1505_00383_amd/libph.so.  Device code is built with
-ffp-contract=off (the error-free transformations need separately rounded
operations; every FMA is explicit) and with packed FP32 instructions disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libph.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("PH_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
          f"-I{os.path.join(HERE, '..', 'include')}"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


# Sources whose compiled gfx950 assembly tests/test_pinned_registers.py
# inspects: the build keeps it (-save-temps) with a fingerprint of what it was
# compiled from, so the check need not compile them a second time.
ASM_KEPT = ("eval.hip", "eval_dd.hip", "eval_qd.hip")


def asm_fingerprint(src: str) -> str:
    """sha256 of the source, every header beside it and the flags."""
    import hashlib
    h = hashlib.sha256()
    names = [src] + sorted(f for f in os.listdir(CSRC) if f.endswith(".hpp"))
    for f in names:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    h.update(" ".join(COMMON + DEVICE).encode())
    return h.hexdigest()


def kept_asm(src: str) -> str | None:
    """Path of the device assembly the last build kept for src, if it was
    compiled from the current sources, else None."""
    stem = src.rsplit(".", 1)[0]
    path = os.path.join(BUILD, f"{stem}-hip-amdgcn-amd-amdhsa-{ARCH}.s")
    fp = os.path.join(BUILD, src + ".asm.sha256")
    if not (os.path.exists(path) and os.path.exists(fp)):
        return None
    with open(fp) as fh:
        if fh.read().strip() != asm_fingerprint(src):
            return None
    return path


# track_unit.hip holds the tracker launchers for one (residual limbs, FP64
# solves) pair per compilation: six objects built in parallel.
TRACK_UNIT = "track_unit.hip"
TRACK_VARIANTS = [(L, m) for L in (1, 2, 4) for m in (1, 0)]


def sources():
    """(source, object name, extra flags) of every compilation."""
    out = []
    # the heaviest compilations first: the tracker units, then eval.hip
    for f in sorted(os.listdir(CSRC), key=lambda f: (f != TRACK_UNIT, f != "eval.hip", f)):
        if not f.endswith((".hip", ".cpp")):
            continue
        if f == TRACK_UNIT:
            for L, m in TRACK_VARIANTS:
                out.append((f, f"track_l{L}{'m' if m else 'p'}.o",
                            [f"-DPH_TRACK_L={L}", f"-DPH_TRACK_MIXED={m}"]))
        else:
            out.append((f, f + ".o", []))
    return out


def _compile(job) -> str:
    src, oname, extra = job
    obj = os.path.join(BUILD, oname)
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    keep = ["-save-temps=obj"] if src in ASM_KEPT else []
    fp = asm_fingerprint(src) if keep else None
    cmd = [HIPCC] + lang + COMMON + DEVICE + extra + keep + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=BUILD)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    if keep:
        with open(os.path.join(BUILD, src + ".asm.sha256"), "w") as fh:
            fh.write(fp + "\n")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", file=sys.stderr)
    return LIB


if __name__ == "__main__":
    build()
