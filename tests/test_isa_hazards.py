"""Checks of the gfx950 machine code of the library's kernels (CPU only).

A vector-memory store of more than 8 bytes reads its data registers after it
issues; a vector instruction that overwrites them in the next cycle corrupts
the stored data in some lanes.  The compiler inserts the wait state for
buffer stores only when they carry no scalar offset register, and on gfx950
16-byte stores with one lost their data this way (the last two colour
components of some particles).  The kernels therefore pass the whole offset
of every 16-byte store in the vector offset.  This test compiles each HIP
source to gfx950 assembly and checks that no store of more than 8 bytes has
its data registers written by the instruction that follows it, and that no
16-byte buffer store uses a scalar offset register.
"""
import concurrent.futures
import os
import re
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2307_07999_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

_STORE = re.compile(r"^\s*(buffer|global|flat|scratch)_store_(dwordx3|dwordx4|b96|b128)\s+v\[(\d+):(\d+)\],\s*(.*)$")
_VALU_DST = re.compile(r"^\s*v_\S+\s+(?:v\[(\d+):(\d+)\]|v(\d+))\b")
_SGPR_SOFFSET = re.compile(r",\s*s\d+(\s|$)")


def _asm(src, out_dir):
    # the flags the library build gives this source, so that the code checked is the code shipped
    from paper_2307_07999_amd import build
    out = os.path.join(out_dir, os.path.basename(src) + ".s")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops"] + build.PER_SOURCE.get(os.path.basename(src), []) + [
           "--cuda-device-only", "-S", "-o", out, "-I", CSRC, "-I", os.path.join(ROOT, "include"), src]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return out


def _instructions(path):
    for line in open(path):
        s = line.strip()
        if not s or s.startswith((";", ".")) or s.endswith(":"):
            continue
        yield line.rstrip("\n")


def _findings(path):
    bad = []
    ins = list(_instructions(path))
    for k, line in enumerate(ins):
        m = _STORE.match(line)
        if not m:
            continue
        data = set(range(int(m.group(3)), int(m.group(4)) + 1))
        if m.group(1) == "buffer" and _SGPR_SOFFSET.search(m.group(5)):
            bad.append("scalar soffset: " + line.strip())
        if k + 1 < len(ins):
            d = _VALU_DST.match(ins[k + 1])
            if d:
                regs = (set(range(int(d.group(1)), int(d.group(2)) + 1)) if d.group(1) else {int(d.group(3))})
                if regs & data:
                    bad.append("data overwritten: %s || %s" % (line.strip(), ins[k + 1].strip()))
    return bad


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_no_wide_store_data_hazard():
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    assert srcs
    tmp = tempfile.mkdtemp(prefix="glasma_isa_")
    try:
        with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as pool:
            outs = list(pool.map(lambda s: _asm(s, tmp), srcs))
        problems = {os.path.basename(o): _findings(o) for o in outs}
        stores = sum(1 for o in outs for l in _instructions(o) if _STORE.match(l))
        assert stores > 0, "no wide stores found: the pattern no longer matches the assembly"
        assert not any(problems.values()), problems
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
