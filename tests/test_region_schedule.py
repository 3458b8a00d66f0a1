"""Build check of the compact region kernel's product loop schedule (CPU, hipcc).

The solve streams every region's matrix once per sparse product, and a wave
hides the memory latency only while the 16 index and 16 value loads of an
unrolled batch of entries are all in flight before their gathers.  Under a
tighter occupancy target the compiler has scheduled the same loop as load,
wait, gather, wait, FMA for every entry (32 waits on vector memory per 16
entries) and the solve ran 2.5x slower; an LDS atomic placed between one
entry's loads and the next entry's has the same effect (loads may not pass an
atomic).  This compiles region.hip for gfx950
to assembly and checks that the kernels (FP32 and FP64, every column width,
with and without the learned preconditioner) keep their 16-deep product
loops batched.  Kernels lost that to code they never run, which only added
register pressure: the 4-column and the preconditioned 1-column FP32 kernels
to the half-layout path, the FP64 4-column kernel to the LDS-staged Lanczos
vector; those paths are now compiled only where they run.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1609_08377_amd", "csrc")
KERNEL = "_ZN5elses12_GLOBAL__N_114compact_kernelIfLi1ELi0EEEvNS_11CompactArgsE"
# every instantiation: value type (f FP32, d FP64) x columns per region x preconditioned
KERNELS = {(tv, c, pc): "_ZN5elses12_GLOBAL__N_114compact_kernelI%sLi%dELi%dEEEvNS_11CompactArgsE" % (tv, c, pc)
           for tv in "fd" for c in (1, 2, 4) for pc in (0, 1)}
# preconditioned multi-column and FP64 4-column preconditioned kernels whose product
# loops the compiler serialises under their register pressure (off the benchmark path;
# they were so before the half layout of B too)
SERIALISED = {("d", 2, 1), ("f", 4, 1), ("d", 4, 1)}


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def product_loops(asm: str, symbol: str):
    """(global loads, LDS reads, vector-memory waits, longest run of global loads
    issued with no vector-memory wait between them) of every loop of `symbol`
    without a barrier that holds at least 32 global loads and 16 LDS reads."""
    lines = asm.split("\n")
    start = next(i for i, l in enumerate(lines) if l.startswith(symbol + ":"))
    end = next(i for i in range(start, len(lines)) if lines[i].startswith(".Lfunc_end"))
    body = lines[start:end]
    labels = {}
    for k, l in enumerate(body):
        m = re.match(r"^(\.LBB\d+_\d+):", l)
        if m:
            labels[m.group(1)] = k
    out = []
    for k, l in enumerate(body):
        m = re.search(r"s_c?branch\w*\s+(\.LBB\d+_\d+)", l)
        if m and m.group(1) in labels and labels[m.group(1)] < k:
            seg = body[labels[m.group(1)]:k + 1]
            loads = sum("global_load" in x for x in seg)
            lds = sum("ds_read" in x for x in seg)
            if loads >= 32 and lds >= 16 and not any("s_barrier" in x for x in seg) and len(seg) < 800:
                run = best = 0
                for x in seg:
                    if "global_load" in x:
                        run += 1
                        best = max(best, run)
                    elif "s_waitcnt vmcnt" in x:
                        run = 0
                out.append((loads, lds, sum("s_waitcnt vmcnt" in x for x in seg), best))
    return out


def test_product_loops_keep_their_loads_in_flight(tmp_path):
    cc = hipcc()
    if cc is None:
        pytest.skip("hipcc not available")
    out = tmp_path / "region.s"
    cmd = [cc, "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-Wno-unused-command-line-argument", "-munsafe-fp-atomics",
           "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "--cuda-device-only", "-S",
           os.path.join(CSRC, "region.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, stdout=subprocess.PIPE, stderr=subprocess.PIPE, timeout=900)
    asm = out.read_text()
    for key, kernel in KERNELS.items():
        if key in SERIALISED:
            continue
        loops = product_loops(asm, kernel)
        assert loops, f"no 16-deep product loop found in {kernel}"
        # a serialised loop waits after every load or two; a batched one issues the index
        # and value loads of its 16 entries back to back before the first wait
        for loads, lds, waits, run in loops:
            assert run >= 16, (key, loads, lds, waits, run)
