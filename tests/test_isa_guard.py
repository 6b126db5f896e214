"""Guard against a register-allocation hazard in the integration kernel.

Copies that the register allocator places inside a region running with
part of the wavefront masked off (between `s_and_saveexec_b64` and the
matching `s_or_b64 exec, exec, ...`) only update the active lanes.  Where
the copy's destination is read after the region by every lane, the masked
lanes read stale values: this once lost the per-lane statistics of failing
cells in the one-cell-per-lane FP64 kernel (a branch to the library log
for non-positive temperatures opened such a region).  The test compiles the
kernel for gfx950 and checks every instantiation for AGPRs that are written
only inside such regions and read outside all of them.  The region
tracking follows the structured exec-mask pattern the compiler emits; it is
a screen, not a proof.
"""

import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1905_09395_amd", "csrc")
# the polynomial / MLP instantiations and the sigmoid-network ones
SOURCES = {"stev_kernel.hip": 20, "stev_kernel_ann.hip": 14}
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

AREG = re.compile(r"\ba(\d+)\b|\ba\[(\d+):(\d+)\]")


def agprs(operand):
    out = []
    for m in AREG.finditer(operand):
        if m.group(1) is not None:
            out.append(int(m.group(1)))
        else:
            out.extend(range(int(m.group(2)), int(m.group(3)) + 1))
    return out


def suspicious(body):
    """AGPRs written only inside partial-exec regions and read outside all
    of the regions that write them."""
    stack, rid = [], 0
    writes, reads = {}, {}
    for line in body.split("\n"):
        t = line.strip()
        if not t or t[0] in ";.":
            continue
        op, _, rest = t.partition(" ")
        if op.startswith("s_and_saveexec_b64"):
            rid += 1
            stack.append(rid)
        elif op == "s_or_b64" and rest.startswith("exec, exec"):
            if stack:
                stack.pop()
        if not op.startswith("v_"):
            continue
        ops = [o.strip() for o in rest.split(",")]
        if not ops:
            continue
        st = tuple(stack)
        for a in agprs(ops[0]):       # destination
            writes.setdefault(a, []).append(st)
        for o in ops[1:]:             # sources
            for a in agprs(o):
                reads.setdefault(a, []).append(st)
    bad = []
    for a, ws in writes.items():
        if not all(ws):
            continue
        for st in reads.get(a, []):
            if not any(st[:len(w)] == w for w in ws):
                bad.append(a)
                break
    return sorted(bad)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
@pytest.mark.parametrize("src", sorted(SOURCES))
def test_no_agpr_copies_escape_partial_exec_regions(tmp_path, src):
    SRC = os.path.join(CSRC, src)
    asm = tmp_path / "k.s"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=on",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "--cuda-device-only", "-S", SRC, "-o", str(asm)]
    subprocess.run(cmd, check=True, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    s = asm.read_text()
    names = re.findall(r"^(_ZN4stev15stev_persistent\S+):\s*;", s, re.M)
    assert len(names) >= SOURCES[src], "expected every kernel variant in the assembly"
    found = {}
    for nm in names:
        i = s.index(nm + ":")
        j = s.index(".Lfunc_end", i)
        bad = suspicious(s[i:j])
        if bad:
            found[nm] = bad
    assert not found, f"AGPRs written only under a partial exec mask and read outside it: {found}"
