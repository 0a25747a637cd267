"""Structure of the compiled kernels: no barrier inside a lane-divergent loop.

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
