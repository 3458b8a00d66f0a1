"""Host-side check of the compact layout's half layout of B (CPU, hipcc, no GPU).

The FP32 Richardson steps of 1- and 2-column regions read the symmetric B once
per off-diagonal pair and sum the transpose half in 32-bit fixed point.  This
compiles `tests/region_layout_check.cpp` against the built library, builds a
region set of a seeded synthetic box with the library's own layout builder and
checks the half layout against the full one: every pair once, in its owner row,
with the full layout's FP32 value; the diagonal; the padding; the slice
lengths; and the bound that keeps the fixed-point sums from overflowing.  The
same build's extreme Ritz values of each region's B are checked against the
dense spectrum of the oracle's carved B.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1609_08377_amd", "csrc")
LIBDIR = os.path.join(ROOT, "paper_1609_08377_amd", "_lib")


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def write_input(path, s, centres, radii):
    with open(path, "wb") as f:
        f.write(np.int32(s.n_atoms).tobytes())
        f.write(np.int64(len(s.blk_col)).tobytes())
        f.write(np.int64(len(s.B_val)).tobytes())
        f.write(np.float64(s.L).tobytes())
        f.write(np.ascontiguousarray(s.n_orb, dtype=np.int8).tobytes())
        f.write(np.ascontiguousarray(s.blk_row_ptr, dtype=np.int64).tobytes())
        f.write(np.ascontiguousarray(s.blk_col, dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(s.val_ptr, dtype=np.int64).tobytes())
        f.write(np.ascontiguousarray(s.A_val, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(s.B_val, dtype=np.float64).tobytes())
        f.write(np.ascontiguousarray(s.pos, dtype=np.float64).tobytes())
        f.write(np.int32(len(centres)).tobytes())
        f.write(np.ascontiguousarray(centres, dtype=np.int32).tobytes())
        f.write(np.ascontiguousarray(radii, dtype=np.float64).tobytes())


def test_half_layout_of_b(tmp_path):
    cc = hipcc()
    lib = os.path.join(LIBDIR, "libelses.so")
    if cc is None or not os.path.exists(lib):
        pytest.skip("hipcc or the built library is not available")
    exe = tmp_path / "region_layout_check"
    cmd = [cc, "-std=c++17", "-O1", "-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument", "-I" + CSRC,
           os.path.join(ROOT, "tests", "region_layout_check.cpp"), "-L" + LIBDIR, "-l:libelses.so",
           "-Wl,-rpath," + LIBDIR, "-o", str(exe)]
    subprocess.run(cmd, check=True, stdout=subprocess.PIPE, stderr=subprocess.PIPE, timeout=900)
    # a seeded box with regions of the benchmark's radius rule (U[6, 14] A), small and
    # large, carbon and hydrogen centres
    s = synth.make_system(3000, 2718)
    rng = np.random.default_rng(31)
    centres = np.sort(rng.choice(s.n_atoms, size=24, replace=False)).astype(np.int32)
    radii = rng.uniform(6.0, 14.0, size=len(centres))
    inp = tmp_path / "system.bin"
    write_input(inp, s, centres, radii)
    out = subprocess.run([str(exe), str(inp)], stdout=subprocess.PIPE, stderr=subprocess.PIPE, timeout=600,
                         text=True)
    print(out.stdout.strip())
    assert out.returncode == 0, out.stdout + out.stderr
    fields = out.stdout.split()
    assert fields[0] == "ok"
    # the split keeps the half rows of a slice close in length: most slots hold a pair
    fill = float(fields[fields.index("fill") + 1])
    assert fill >= 0.6, out.stdout
    # the extreme Ritz values of each region's B (40 Lanczos steps on the built layout),
    # which set the region's Chebyshev-Richardson plan, against the spectrum of the
    # oracle's carved B: inside it (Ritz values of a symmetric matrix) and close to its ends
    ritz = {}
    for line in out.stdout.splitlines():
        if line.startswith("ritz "):
            _, r, lo, hi = line.split()
            ritz[int(r)] = (float(lo), float(hi))
    assert len(ritz) == len(centres)
    sizes = [len(oracle.region_atoms(s, int(c), float(rad))) for c, rad in zip(centres, radii)]
    for r in np.argsort(sizes)[:6]:
        _, Br, _ = oracle.carve_region(s, oracle.region_atoms(s, int(centres[r]), float(radii[r])))
        ev = np.linalg.eigvalsh(Br.dense())
        lo, hi = ritz[int(r)]
        width = ev[-1] - ev[0]
        assert ev[0] - 1e-10 <= lo <= ev[0] + 0.02 * width, (r, lo, ev[0], ev[-1])
        assert ev[-1] - 0.02 * width <= hi <= ev[-1] + 1e-10, (r, hi, ev[0], ev[-1])
