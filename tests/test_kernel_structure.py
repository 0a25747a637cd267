"""Structure of the compiled kernels: no barrier inside a lane-divergent loop,
and the single-shuffle kernel's partial memory wait covers its reservations.

A loop that contains a workgroup barrier must be left by all lanes of a wave
in the same iteration.  If the compiler gives such a loop a per-lane exit
(the loop latch removes lanes from the execution mask), lanes can be parked
outside the loop while the rest of the wave keeps iterating, which ends in a
kernel that never finishes.  This test compiles every HIP source of the
library to gfx950 assembly and checks, for each kernel, that no loop holding
a barrier (directly or in a nested loop) has an exec-mask latch.  It runs on
the CPU: hipcc cross-compiles without a GPU.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2103_01216_amd import build as rpbuild

HIPCC = rpbuild.HIPCC

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None,
                                reason="hipcc not available")

FUNC_RE = re.compile(r"^([A-Za-z_][\w.$]*):\s*; @\1\s*$", re.M)
BLOCK_RE = re.compile(r"^(\.LBB\d+_\d+|; %bb\.\d+):\s*(;.*)?$")


def _assembly(src, tmp_path):
    out = tmp_path / (os.path.basename(src) + ".s")
    flags = [f for f in rpbuild.FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [HIPCC, *flags, "--cuda-device-only", "-S", "-o", str(out), src]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    return out.read_text()


def _functions(asm):
    """name -> list of lines of that function's body."""
    out = {}
    for m in FUNC_RE.finditer(asm):
        end = asm.find(".Lfunc_end", m.end())
        out[m.group(1)] = asm[m.end():end].split("\n")
    return out


def _divergent_barrier_loops(lines):
    """Loops (by header) that hold a barrier and have an exec-mask latch."""
    blocks, order, cur = {}, [], None
    children = {}   # header -> all nested loop headers (from the loop comments)
    pending = None
    for ln in lines:
        m = BLOCK_RE.match(ln)
        if m:
            cur = m.group(1)
            order.append(cur)
            ann = m.group(2) or ""
            blocks[cur] = {"ann": ann, "ins": []}
            pending = cur if "Loop Header" in ann else None
            continue
        if cur is None:
            continue
        s = ln.strip()
        if s.startswith(";"):
            if "Loop Header" in s:
                pending = cur
                blocks[cur]["ann"] += " " + s
            c = re.search(r"Child Loop (BB\d+_\d+)", s)
            if c and pending:
                children.setdefault("BB" + pending.split("BB")[1], []).append(c.group(1))
            continue
        blocks[cur]["ins"].append(s)

    def innermost(b):
        ann = blocks[b]["ann"]
        if "Loop Header" in ann and b.startswith(".LBB"):
            return b[2:]
        h = re.search(r"Header=(BB\d+_\d+)", ann)
        return h.group(1) if h else None

    def ancestors(h):
        # every header that lists h among its nested loops contains it
        return [p for p, ch in children.items() if h in ch]

    with_barrier = set()
    for b in order:
        if any(i.startswith("s_barrier") for i in blocks[b]["ins"]):
            h = innermost(b)
            if h:
                with_barrier.add(h)
                with_barrier.update(ancestors(h))
    bad = []
    for b in order:
        h = innermost(b)
        if h in with_barrier and any(i.startswith("s_andn2_b64 exec, exec") for i in blocks[b]["ins"]):
            bad.append((b, h))
    return bad


@pytest.mark.parametrize("src", rpbuild.SRCS, ids=os.path.basename)
def test_no_barrier_in_divergent_loop(src, tmp_path):
    funcs = _functions(_assembly(src, tmp_path))
    kernels = {n: body for n, body in funcs.items() if "kernel" in n}
    assert kernels, "no kernels found in the assembly"
    bad = {n: _divergent_barrier_loops(body) for n, body in kernels.items()}
    bad = {n: v for n, v in bad.items() if v}
    assert not bad, bad


def test_checker_flags_a_parked_lane_loop(tmp_path):
    """The check itself: a workgroup loop whose single-lane claim step and
    single-lane publish step meet at the back edge, with the loop exit taken
    from a vector register, is compiled with an exec-mask latch."""
    src = tmp_path / "parked.hip"
    src.write_text(r'''
#include <hip/hip_runtime.h>
#include <cstdint>
__global__ __launch_bounds__(256) void parked_kernel(uint32_t *claims, uint32_t n, uint32_t *out)
{
    __shared__ uint32_t sh_claim;
    __shared__ uint32_t acc[256];
    for (;;) {
        if (threadIdx.x == 0)
            sh_claim = __hip_atomic_fetch_add(claims, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const uint32_t idx = sh_claim;
        __syncthreads();
        if (idx >= n)
            break;
        acc[threadIdx.x] = idx * threadIdx.x;
        __syncthreads();
        uint32_t t = 0;
        for (int i = 0; i < 256; i += 64)
            t += acc[(threadIdx.x + i) & 255];
        __syncthreads();
        if (threadIdx.x == 0)
            out[idx] = t;
    }
}
''')
    funcs = _functions(_assembly(str(src), tmp_path))
    body = [b for n, b in funcs.items() if "parked_kernel" in n][0]
    assert _divergent_barrier_loops(body)


# ------------------------------------------------- partial wait before the barrier

LABEL_RE = re.compile(r"^(\.LBB\d+_\d+):")
VMEM_RE = re.compile(r"^(global|buffer|flat|scratch)_(\w+)")
WAIT_RE = re.compile(r"^s_waitcnt vmcnt\((\d+)\)")


def _segments(lines):
    """Label-delimited segments: [(label, [(instruction, from_inline_asm)])]."""
    segs = [("entry", [])]
    asm = False
    for ln in lines:
        s = ln.strip()
        m = LABEL_RE.match(s)
        if m:
            segs.append((m.group(1), []))
            continue
        if s.startswith(";;#ASMSTART"):
            asm = True
            continue
        if s.startswith(";;#ASMEND"):
            asm = False
            continue
        if not s or s.startswith(";") or s.startswith("."):
            continue
        segs[-1][1].append((s.split(";")[0].strip(), asm))
    return segs


def _predecessors(segs):
    """label -> [(segment index, instruction index)] that transfer to it."""
    pred = {}
    for si, (_, ins) in enumerate(segs):
        for j, (i, _) in enumerate(ins):
            m = re.match(r"^s_(cbranch_\w+|branch)\s+(\.LBB\d+_\d+)", i)
            if m:
                pred.setdefault(m.group(2), []).append((si, j - 1))
        last = ins[-1][0] if ins else ""
        if si + 1 < len(segs) and not re.match(r"^s_(branch|endpgm|setpc)", last):
            pred.setdefault(segs[si + 1][0], []).append((si, len(ins) - 1))
    return pred


def _last_vmem_ok(segs, pred, si, j, need):
    """Walking back from instruction j of segment si along every path, are the
    `need` most recent vector memory instructions all loads?"""
    seen = set()
    stack = [(si, j, need)]
    while stack:
        si, j, need = stack.pop()
        if (si, j, need) in seen:
            continue
        seen.add((si, j, need))
        ins = segs[si][1]
        while j >= 0 and need > 0:
            m = VMEM_RE.match(ins[j][0])
            if m:
                if not m.group(2).startswith("load"):
                    return False, ins[j][0]
                need -= 1
            j -= 1
        if need == 0:
            continue
        froms = pred.get(segs[si][0], [])
        if not froms:
            return False, "reached the function entry"
        stack.extend((p, q, need) for p, q in froms)
    return True, None


def test_partial_wait_covers_reservations(tmp_path):
    """Before the round's first barrier a wave waits with vmcnt(N), leaving
    its N record loads in flight; that is only safe if, on every path, the N
    most recent vector memory instructions before the wait are those loads
    (so every reservation atomic and window clear, issued earlier, has
    completed).  Checked on every instance of the single-shuffle kernel and
    of its group form."""
    src = [s for s in rpbuild.SRCS if os.path.basename(s) == "rp.hip"][0]
    funcs = _functions(_assembly(src, tmp_path))
    kernels = {n: b for n, b in funcs.items()
               if "rp_rounds_kernel" in n or "rp_rounds_group_kernel" in n}
    assert kernels
    with_wait = 0
    for name, body in kernels.items():
        segs = _segments(body)
        pred = _predecessors(segs)
        for si, (_, ins) in enumerate(segs):
            for j, (i, from_asm) in enumerate(ins):
                m = WAIT_RE.match(i)
                if from_asm and m and int(m.group(1)) > 0:
                    with_wait += 1
                    ok, why = _last_vmem_ok(segs, pred, si, j - 1, int(m.group(1)))
                    assert ok, (name, i, why)
        # instances holding 4/8/16-byte records use the partial wait
        eb = re.search(r"ILi\d+ELi(\d+)E", name)
        if eb and eb.group(1) != "0":
            assert any(WAIT_RE.match(i) and a and not i.endswith("(0)")
                       for _, ins in segs for i, a in ins), name
    assert with_wait > 0


def test_wait_checker_flags_an_atomic_after_the_loads():
    """The check itself, on a hand-made listing: an atomic between the loads
    and the wait, or a path that skips the loads, fails it."""
    good = ["global_atomic_umax v[0:1], v2, off", "global_load_dwordx2 v[4:5], v[6:7], off",
            "global_load_dwordx2 v[8:9], v[6:7], off", ";;#ASMSTART", "s_waitcnt vmcnt(2)",
            ";;#ASMEND", "s_barrier"]
    bad1 = ["global_load_dwordx2 v[4:5], v[6:7], off", "global_atomic_umax v[0:1], v2, off",
            "global_load_dwordx2 v[8:9], v[6:7], off", ";;#ASMSTART", "s_waitcnt vmcnt(2)",
            ";;#ASMEND", "s_barrier"]
    bad2 = ["global_atomic_umax v[0:1], v2, off", "s_cbranch_vccz .LBB0_2",
            "global_load_dwordx2 v[4:5], v[6:7], off", "global_load_dwordx2 v[8:9], v[6:7], off",
            ".LBB0_2:", ";;#ASMSTART", "s_waitcnt vmcnt(2)", ";;#ASMEND", "s_barrier"]

    def check(lines):
        segs = _segments(lines)
        pred = _predecessors(segs)
        for si, (_, ins) in enumerate(segs):
            for j, (i, a) in enumerate(ins):
                if a and WAIT_RE.match(i):
                    return _last_vmem_ok(segs, pred, si, j - 1, int(WAIT_RE.match(i).group(1)))[0]
        raise AssertionError("no wait")

    assert check(good)
    assert not check(bad1)
    assert not check(bad2)
