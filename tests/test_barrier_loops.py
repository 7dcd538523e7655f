"""Every loop that passes a workgroup barrier must be lowered as a uniform
loop.  The compiler may turn a loop whose exit it believes to be lane
dependent into an exec-mask loop; a wave then keeps iterating (and passing
the barrier) for its remaining lanes, so its barrier count no longer matches
the other waves of the workgroup.  In a kernel whose waves play different
roles (walkers and contractors) that silently desynchronises the roles.

The check compiles each HIP source to gfx950 assembly with the library's own
flags and inspects the loop annotations the compiler writes: a loop whose own
blocks contain `s_andn2_b64 exec, exec, ...` (the exec-mask loop exit) must
not contain `s_barrier`.  CPU only: hipcc cross-compiles."""
import os
import re
import shutil
import subprocess
import tempfile

import pytest

from paper_2503_06161_amd import build as B

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
KERNEL_SOURCES = [s for s in B.SOURCES if s != "fe_api.hip"]


def divergent_barrier_loops(asm: str):
    """({kernel: [loop headers]}, kernel count) for barrier-carrying loops
    lowered with an exec-mask exit."""
    out, nkern = {}, 0
    for m in re.finditer(r"^(\S+):\s*; @(\S+)\n(.*?)^\.Lfunc_end", asm, re.S | re.M):
        nkern += 1
        name, body = m.group(1), m.group(3)
        blocks = []                      # [label, annotation, instructions, annotation open]
        for raw in body.split("\n"):
            line = raw.strip()
            mh = re.match(r"^(?:\.LBB(\d+_\d+)|; %bb\.(\d+)):(.*)", line)
            if mh:
                lab = "BB" + mh.group(1) if mh.group(1) else "bb" + mh.group(2)
                blocks.append([lab, mh.group(3), [], True])
            elif not blocks:
                blocks.append([None, "", [], False])
            elif line.startswith(";"):
                if blocks[-1][3]:        # annotation continued on the next line
                    blocks[-1][1] += " " + line
            elif line and not line.startswith("."):
                blocks[-1][2].append(line)
                blocks[-1][3] = False
        parent, member = {}, []
        for lab, note, ins, _ in blocks:
            hdr = None
            if "Loop Header" in note:
                hdr = lab
                mp = re.search(r"Parent Loop (BB\d+_\d+)", note)
                parent[lab] = mp.group(1) if mp else None
            else:
                mi = re.search(r"in Loop: Header=(BB\d+_\d+)", note)
                hdr = mi.group(1) if mi else None
            member.append((hdr, ins))
        loops = {}
        for hdr, ins in member:
            h, own = hdr, True
            while h is not None:
                d = loops.setdefault(h, [0, False])
                d[0] += sum(1 for x in ins if x.startswith("s_barrier"))
                if own and any(x.startswith("s_andn2_b64 exec, exec") for x in ins):
                    d[1] = True
                own = False
                h = parent.get(h)
        bad = sorted(h for h, (nb, div) in loops.items() if nb and div)
        if bad:
            out[name] = bad
    return out, nkern


def test_checker_flags_a_divergent_barrier_loop():
    """Hand-written assembly skeletons pin the checker itself."""
    bad = """k:                                      ; @k
; %bb.0:
\ts_mov_b64 s[0:1], 0
.LBB0_1:                                ; =>This Inner Loop Header: Depth=1
\ts_barrier
\tv_cmp_gt_u32_e32 vcc, 4, v0
\ts_or_b64 s[0:1], vcc, s[0:1]
\ts_andn2_b64 exec, exec, s[0:1]
\ts_cbranch_execnz .LBB0_1
; %bb.2:
\ts_endpgm
.Lfunc_end0:
"""
    good = bad.replace("\ts_andn2_b64 exec, exec, s[0:1]\n\ts_cbranch_execnz .LBB0_1",
                       "\ts_cmp_lg_u32 s2, 0\n\ts_cbranch_scc1 .LBB0_1")
    # an inner loop with an exec-mask exit and no barrier, inside a uniform
    # loop that holds the barrier: not flagged; the header annotation of a
    # nested loop spans two lines
    nested = """k:                                      ; @k
; %bb.0:
\ts_mov_b64 s[0:1], 0
.LBB0_1:                                ; =>This Loop Header: Depth=1
\ts_barrier
.LBB0_2:                                ;   Parent Loop BB0_1 Depth=1
                                        ; =>  This Inner Loop Header: Depth=2
\tv_cmp_gt_u32_e32 vcc, 4, v0
\ts_andn2_b64 exec, exec, s[0:1]
\ts_cbranch_execnz .LBB0_2
; %bb.3:                                ;   in Loop: Header=BB0_1 Depth=1
\ts_cmp_lg_u32 s2, 0
\ts_cbranch_scc1 .LBB0_1
; %bb.4:
\ts_endpgm
.Lfunc_end0:
"""
    assert divergent_barrier_loops(bad) == ({"k": ["BB0_1"]}, 1)
    assert divergent_barrier_loops(good) == ({}, 1)
    assert divergent_barrier_loops(nested) == ({}, 1)
    # the same nest with the barrier moved into the inner loop is flagged
    inner = nested.replace("\ts_barrier\n.LBB0_2", ".LBB0_2").replace(
        "Depth=2\n\tv_cmp", "Depth=2\n\ts_barrier\n\tv_cmp")
    assert divergent_barrier_loops(inner) == ({"k": ["BB0_2"]}, 1)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_barrier_loops_are_uniform_in_every_kernel():
    flags = [f for f in B.FLAGS if f != "-fPIC"]
    with tempfile.TemporaryDirectory() as tmp:
        procs = {}
        for src in KERNEL_SOURCES:
            out = os.path.join(tmp, src + ".s")
            cmd = [HIPCC, *flags, "--cuda-device-only", "-S", os.path.join(B.CSRC, src), "-o", out]
            procs[src] = (subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE), out)
        bad, total = {}, 0
        for src, (p, out) in procs.items():
            _, err = p.communicate(timeout=600)
            assert p.returncode == 0, (src, err.decode()[-2000:])
            found, n = divergent_barrier_loops(open(out).read())
            total += n
            bad.update({f"{src}:{k}": v for k, v in found.items()})
    assert total >= 100, total
    assert not bad, bad
