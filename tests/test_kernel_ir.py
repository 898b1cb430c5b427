"""Static checks of the device code (CPU only: compiles to LLVM IR with hipcc).

Lane-split loops.  A loop whose body holds a cross-lane operation (shuffle,
ballot, readfirstlane, DPP, barrier) must not have a back edge that branches on
the lane index alone.  The optimiser can produce such a back edge by threading
a loop's latch on a branch like ``if (lane == 0)`` inside the body; on the GPU
the wavefront then splits between two back edges, and the lanes of one of them
run the cross-lane operations without the others, possibly forever.  (A
persistent work loop that took its ticket with ``if (lane == 0) t =
atomicAdd(...)`` hung this way.)  The emulator-free check below finds such back
edges in the IR, and a planted snippet with the old pattern proves that it
fires.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or ("/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else None)
pytestmark = pytest.mark.skipif(HIPCC is None, reason="hipcc not available")

CONVERGENT = ("llvm.amdgcn.ds.bpermute", "llvm.amdgcn.readfirstlane", "llvm.amdgcn.icmp", "llvm.amdgcn.ballot",
              "llvm.amdgcn.update.dpp", "llvm.amdgcn.mov.dpp", "llvm.amdgcn.s.barrier", "llvm.amdgcn.wave.barrier",
              "llvm.amdgcn.permlane", "llvm.amdgcn.readlane")
LANE_SOURCES = ("llvm.amdgcn.mbcnt", "llvm.amdgcn.workitem.id")


def device_ir(src, out):
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "-S", "-emit-llvm", "--cuda-device-only",
           src, "-o", out]
    subprocess.run(cmd, check=True, stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    with open(out) as f:
        return f.read()


def _functions(ir):
    for m in re.finditer(r"^define [^@]*@(\S+)\(", ir, re.M):
        end = ir.index("\n}\n", m.start())
        yield m.group(1), ir[m.start():end].split("\n")


def lane_split_back_edges(ir):
    """(function, block) of every branch whose condition is computed from the
    lane index alone and whose two successors belong to different loops, one
    of which holds a cross-lane operation."""
    found = []
    for name, body in _functions(ir):
        defs, order, blocks, succ = {}, ["entry"], {"entry": []}, {}
        cur = "entry"
        for line in body[1:]:
            b = re.match(r"^(\d+):", line)
            if b:
                cur = b.group(1)
                order.append(cur)
                blocks[cur] = []
                continue
            blocks[cur].append(line.strip())
            d = re.match(r"\s*(%\d+) = (.*)", line)
            if d:
                defs[d.group(1)] = d.group(2)
        cond = {}
        for b in order:
            term = [x for x in blocks[b] if x.startswith(("br ", "switch ", "ret"))]
            t = term[-1] if term else ""
            succ[b] = re.findall(r"label %(\d+)", t)
            c = re.match(r"br i1 (%\d+)", t)
            cond[b] = c.group(1) if c else None
        pred = {b: [] for b in order}
        for b in order:
            for s in succ[b]:
                pred.setdefault(s, []).append(b)
        # retreating edges of a depth-first search from the entry
        back, state, stack = [], {}, [("entry", iter(succ["entry"]))]
        state["entry"] = 1
        while stack:
            node, it = stack[-1]
            nxt = next(it, None)
            if nxt is None:
                state[node] = 2
                stack.pop()
            elif state.get(nxt) == 1:
                back.append((node, nxt))
            elif nxt not in state:
                state[nxt] = 1
                stack.append((nxt, iter(succ.get(nxt, []))))

        def kind(v, depth=0):
            """'lane': varies between the lanes of a wavefront and is computed
            from the lane or work-item index and constants only; 'uni': such a
            value that is uniform in a wavefront (e.g. index >> 6, index < 64k);
            None: anything else."""
            d = defs.get(v)
            if d is None or depth > 10:
                return None
            if any(s in d for s in LANE_SOURCES):
                return "lane"
            op = re.match(r"(icmp|and|or|xor|select|zext|sext|trunc|lshr|ashr|shl|add|sub)\b", d)
            if not op:
                return None
            ops = re.findall(r"%\d+", d)
            kinds = [kind(o, depth + 1) for o in ops]
            if not ops or any(x is None for x in kinds):
                return None
            if "lane" not in kinds:
                return "uni"
            consts = [int(c) for c in re.findall(r"(?<![%\w])(-?\d+)(?=\s*$|\s*,)", d)]
            c = consts[-1] if consts else None
            name_ = op.group(1)
            if name_ in ("lshr", "ashr") and c is not None and c >= 6:
                return "uni"
            if name_ == "and" and c is not None and (c & 63) == 0:
                return "uni"
            if name_ == "icmp" and c is not None and c % 64 == 0 and re.match(r"icmp (samesign )?[us](lt|ge|gt|le)", d):
                return "uni"
            return "lane"

        def lane_only(v):
            return kind(v) == "lane"

        loops = {}  # header -> blocks of its natural loop(s)
        for latch, header in back:
            # (a self-loop's body is its header alone: never walk past it)
            body_, work = {header, latch}, ([latch] if latch != header else [])
            while work:
                n = work.pop()
                for p in pred.get(n, []):
                    if p not in body_:
                        body_.add(p)
                        work.append(p)
            loops.setdefault(header, set()).update(body_)
        conv = {h for h, bl in loops.items() if any(any(c in x for c in CONVERGENT) for lb in bl
                                                     for x in blocks.get(lb, []))}
        member = {b: frozenset(h for h, bl in loops.items() if b in bl) for b in order}
        # a branch on the lane index whose successors lie in different loops
        # (one re-enters or stays in a loop the other leaves) splits the
        # wavefront across loop iterations
        for b in order:
            if cond.get(b) is None or len(succ[b]) != 2 or not lane_only(cond[b]):
                continue
            s1, s2 = succ[b]
            differ = member.get(s1, frozenset()) ^ member.get(s2, frozenset())
            if any(h in conv for h in differ):
                found.append((name, b))
    return found


PLANTED = r'''
#include <hip/hip_runtime.h>
__global__ void planted(unsigned* head, unsigned n, const int* items, int* out) {
  for (;;) {
    unsigned it = 0;
    if (__lane_id() == 0) it = atomicAdd(head, 1u);
    it = __builtin_amdgcn_readfirstlane(__shfl((int)it, 0, 64));
    if (it >= n) break;
    int v = items[it] + threadIdx.x;
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    if (__lane_id() == 0) out[it] = v;
  }
}
'''


def test_planted_lane_split_is_detected(tmp_path):
    src = tmp_path / "planted.hip"
    src.write_text(PLANTED)
    ir = device_ir(str(src), str(tmp_path / "planted.ll"))
    assert lane_split_back_edges(ir), "the check must flag the planted lane-0 ticket loop"


def test_library_has_no_lane_split_loops(tmp_path):
    src = os.path.join(ROOT, "paper_1904_02266_amd", "csrc", "cvo_kernels.hip")
    ir = device_ir(src, str(tmp_path / "kernels.ll"))
    bad = lane_split_back_edges(ir)
    assert not bad, f"lane-split back edges in loops with cross-lane operations: {bad[:5]}"
