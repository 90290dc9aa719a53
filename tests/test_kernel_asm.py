"""Assembly checks of the tiled kernels (host only: hipcc cross-compiles for gfx950).

The compute waves of the tiled solve and of the tiled factor issue no global load
inside their loop.  On this architecture vector loads and stores share one
memory counter, so a wait on that counter inside the loop stalls the wave until
its own earlier stores (the values it published) are acknowledged.  Such waits
once came back through the compiler's bookkeeping, with no load in the loop:
the poller wave's loads were carried around the pass loop, and the factor's
per-row threshold load put a full wait on every chunk.  The kernels rule both
out now; this test keeps them out.  A variant that spills to scratch needs those
waits for its scratch loads and is skipped.
"""
import os
import re
import subprocess
import tempfile

import pytest

from paper_1812_06160_amd import build as B

KERNELS = os.path.join(B.CSRC, "kernels.hip")


@pytest.fixture(scope="module")
def asm():
    try:
        hipcc = B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "kernels.s")
        cmd = [hipcc, "-x", "hip"] + B.DEVICE + B.COMMON + ["--offload-device-only", "-S", KERNELS, "-o", out]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        with open(out) as f:
            return f.read()


def functions(text, pattern):
    """(mangled name, body lines, scratch bytes) of every function matching pattern."""
    out = []
    for m in re.finditer(r"\n(_Z\w*" + pattern + r"\w*):", text):
        end = text.index(".Lfunc_end", m.end())
        body = text[m.end():end].split("\n")
        tail = text[end:end + 4000]
        sm = re.search(r"; ScratchSize: (\d+)", tail)
        out.append((m.group(1), body, int(sm.group(1)) if sm else 0))
    return out


def publish_loop(body):
    """Lines of the innermost loop that holds the first publishing store (a store
    with the coherence bit to a 64-bit address, the form only the compute waves'
    publish takes)."""
    stores = [k for k, ln in enumerate(body)
              if re.search(r"global_store_dword(x2)?\s+v\[\d+:\d+\], v(\[\d+:\d+\]|\d+), off sc1", ln)]
    assert stores, "no publishing store found"
    head = None
    for k in range(stores[0], -1, -1):
        m = re.search(r"Header=(BB\d+_\d+) Depth=\d", body[k])
        if m:
            head = m.group(1)
            break
    assert head, "publishing store outside any loop"
    marks = [k for k, ln in enumerate(body) if f"Header={head} " in ln or ln.startswith(f".L{head}:")]
    lo, hi = min(marks), max(marks)
    while hi + 1 < len(body) and not body[hi + 1].startswith((".LBB", "; %bb")):
        hi += 1
    return body[lo:hi + 1]


@pytest.mark.parametrize("kernel", ["k_solve_tiled", "k_factor_tiled"])
def test_tiled_compute_loops_hold_no_memory_waits(asm, kernel):
    fns = functions(asm, r"\d+" + kernel)
    assert fns, f"{kernel} not found in the assembly"
    checked = 0
    for name, body, scratch in fns:
        if scratch:
            continue
        loop = publish_loop(body)
        waits = [ln.strip() for ln in loop if "s_waitcnt vmcnt" in ln]
        assert not waits, f"{name}: {len(waits)} vector-memory waits in the compute loop"
        checked += 1
    assert checked >= len(fns) - 2
