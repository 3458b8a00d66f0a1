"""Host-side check of the Chebyshev-Richardson plan (CPU, hipcc, no GPU).

Every overlap solve B v = s runs the plan of an interval holding B's spectrum
(B's own, or a region's): d steps whose inverse step lengths are the roots of
T_d on the interval, in Leja order, so that the residual is multiplied by the
scaled Chebyshev polynomial, at most 1/T_d(c/h) on the interval.  This
compiles `tests/richardson_plan_check.cpp` against the built library and pins
the library's plan to that closed form: the roots, the Leja order, the
residual polynomial on a fine grid, the reported factor, the smallest degree
meeting the tolerance and the cap.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1609_08377_amd", "csrc")
LIBDIR = os.path.join(ROOT, "paper_1609_08377_amd", "_lib")

# (lo, hi, tol): B's interval of the synthetic boxes at the mixed rounds' and the FP64
# tolerances, a wider and a nearly degenerate interval, and one past the degree cap
CASES = [(0.75, 2.2, 1e-6), (0.75, 2.2, 1e-12), (0.5, 3.0, 1e-8), (1.0, 1.001, 1e-10), (1e-4, 1.0, 1e-14)]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def test_plan_matches_the_chebyshev_closed_form(tmp_path):
    cc = hipcc()
    if cc is None or not os.path.exists(os.path.join(LIBDIR, "libelses.so")):
        pytest.skip("hipcc or the built library is not available")
    exe = tmp_path / "richardson_plan_check"
    cmd = [cc, "-std=c++17", "-O1", "-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature",
           "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument", "-I" + CSRC,
           os.path.join(ROOT, "tests", "richardson_plan_check.cpp"), "-L" + LIBDIR, "-l:libelses.so",
           "-Wl,-rpath," + LIBDIR, "-o", str(exe)]
    subprocess.run(cmd, check=True, stdout=subprocess.PIPE, stderr=subprocess.PIPE, timeout=900)
    args = ["%r,%r,%r" % c for c in CASES]
    out = subprocess.run([str(exe), *args], stdout=subprocess.PIPE, stderr=subprocess.PIPE, timeout=300, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    lines = out.stdout.split("\n")
    degrees = [int(l.split()[1]) for l in lines if l.startswith("ok ")]
    assert len(degrees) == len(CASES)
    assert degrees[3] == 3  # a nearly degenerate interval still takes the minimum of three steps
    assert degrees[4] == 400  # kRichMaxDegree: capped, reports the factor it reaches
    assert degrees[0] < degrees[1]
