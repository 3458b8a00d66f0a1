"""Mixed precision (FP32-stored A and B) through the C ABI, against the CPU FP64 oracle.

Reading: the mixed-precision problem is the pencil of the FP32-rounded A and B.
Its solutions are compared element-wise with the oracle run on that rounded
pencil (tight, like the FP64 mode), and with the oracle on the original FP64
pencil within 1e-5 relative (the mixed-mode agreement bar); the audit
recomputes the FP64 residual of the rounded pencil.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rounded(s):
    """The same system with A and B rounded to FP32 (and held exactly in FP64)."""
    return dataclasses.replace(s, A_val=s.A_val.astype(np.float32).astype(np.float64),
                               B_val=s.B_val.astype(np.float32).astype(np.float64))


@pytest.fixture(scope="module")
def el():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1609_08377_amd as el
    el.lib()
    return el


@pytest.fixture(scope="module")
def ctx(el):
    return el.Context(0)


@pytest.fixture(scope="module")
def c1m(el, ctx):
    s = synth.make_system(128, synth.config_seed(1))
    s32 = rounded(s)
    mat = el.Matrix.from_system(ctx, s, precision="mixed")
    return dict(s=s, A=oracle.to_csr(s, "A"), B=oracle.to_csr(s, "B"), A32=oracle.to_csr(s32, "A"),
                B32=oracle.to_csr(s32, "B"), mat=mat)


def rel_elementwise(xg, xr):
    return np.abs(xg - xr).max() / np.abs(xr).max()


@pytest.mark.parametrize("nvec,variant", [(64, "direct"), (128, "direct"), (256, "direct"), (64, "grouped"),
                                          (128, "grouped2"), (256, "grouped"), (256, "grouped1"),
                                          (512, 0x80 | 5), (320, "auto")])
def test_spmm32_matches_oracle(el, ctx, c1m, nvec, variant):
    """FP32 products: |y - fl32(X) x| <= 8e-6 (|fl32(X)| |x|) row by row (about 70 FP32 roundings)."""
    rng = np.random.default_rng(nvec + 7)
    n = c1m["A"].n
    X = rng.standard_normal((n, nvec)).astype(np.float32)
    Xd = torch.from_numpy(X).cuda()
    for which in ("A", "B"):
        C = c1m[which + "32"]
        Y = el.spmm32(ctx, c1m["mat"], which, Xd, variant).cpu().numpy().astype(np.float64)
        X64 = X.astype(np.float64)
        ref = C.dense() @ X64
        absref = np.abs(C.dense()) @ np.abs(X64)
        assert np.all(np.abs(Y - ref) <= 8e-6 * absref), which


def test_mixed_full_mode_vs_rounded_and_fp64_oracle(el, ctx, c1m):
    z = synth.shift_grid(32)
    cols = np.array([0, 1, 3, 100, 171, 200, 256], dtype=np.int32)
    mat = c1m["mat"]
    out = el.shifted_solve(ctx, mat, cols, z, tol=1e-10, full=True, audit=True, mixed=True)
    xg = out["x"].cpu().numpy()
    res = out["resid"].cpu().numpy()
    # audit of the rounded pencil: tol plus the floor of the two-round FP32 overlap
    # solve, whose relative error is below 1e-11
    xnorm = np.linalg.norm(xg, axis=2)
    bound = 1e-10 * 1.0001 + 1e-11 * np.abs(z)[None, :] * mat.b_interval[1] * xnorm
    assert np.all(res <= bound), (res / bound).max()
    ref32 = oracle.shifted_solve(c1m["A32"], c1m["B32"], cols, z, tol=1e-11, full=True)
    ref64 = oracle.shifted_solve(c1m["A"], c1m["B"], cols, z, tol=1e-11, full=True)
    worst32 = worst64 = 0.0
    for c in range(len(cols)):
        for k in range(len(z)):
            worst32 = max(worst32, rel_elementwise(xg[c, k], ref32.x[c, k]))
            worst64 = max(worst64, rel_elementwise(xg[c, k], ref64.x[c, k]))
    assert worst32 <= 1e-7, worst32
    assert worst64 <= 1e-5, worst64


def test_mixed_all_columns_default_tol(el, ctx, c1m):
    """C1 columns at tol 1e-8 in pattern mode; sample vs the FP64 oracle within 1e-5."""
    z = synth.shift_grid(32)
    n = c1m["A"].n
    cols = np.arange(n, dtype=np.int32)
    out = el.shifted_solve(ctx, c1m["mat"], cols, z, tol=1e-8, mixed=True)
    assert np.all(out["resid"].cpu().numpy() <= 1e-8)
    pat_off = out["pat_off"]
    xg = out["x"].cpu().numpy()
    K = len(z)
    B = c1m["B"]
    sample = np.array([0, 44, 130, 256], dtype=np.int32)
    ref = oracle.shifted_solve(c1m["A"], B, sample, z, tol=1e-11, full=True)
    for c, j in enumerate(sample):
        rows = B.ci[B.rp[j]:B.rp[j + 1]]
        blk = xg[pat_off[j] * K:pat_off[j + 1] * K].reshape(K, -1)
        for k in range(K):
            assert rel_elementwise(blk[k], ref.x[c, k][rows]) <= 1e-5, (j, k)


def test_mixed_density_traces(el, ctx, c1m):
    z = synth.shift_grid(32)
    cw = oracle.fermi_weights(z, 0.0, 0.01)
    cols = np.arange(0, c1m["A"].n, 3, dtype=np.int32)
    g = el.density_matrix(ctx, c1m["mat"], cols, z, cw, tol=1e-8, mixed=True)
    ref = oracle.shifted_solve(c1m["A"], c1m["B"], cols, z, tol=1e-11, full=False)
    rho_ref, tb, ta = oracle.density_from_x(c1m["B"], c1m["A"], cols, ref.x, ref.pat_off, cw)
    rho = g["rho"].cpu().numpy()
    assert np.abs(rho - rho_ref).max() <= 1e-5 * np.abs(rho_ref).max()
    trB, trA = g["traces"]
    assert abs(trB - tb.sum()) <= 1e-5 * abs(tb.sum())
    assert abs(trA - ta.sum()) <= 1e-5 * max(1.0, abs(ta.sum()))


def test_mixed_needs_mixed_matrix(el, ctx):
    s = synth.make_system(64, 5, r_cut=3.5)
    mat = el.Matrix.from_system(ctx, s)
    with pytest.raises(el.ElsesError):
        el.shifted_solve(ctx, mat, [0], [0.1 + 0.1j], mixed=True)
    with pytest.raises(el.ElsesError):
        el.spmm32(ctx, mat, "B", torch.zeros((mat.M, 64), dtype=torch.float32, device="cuda"))


def test_mixed_slot_and_variant_agreement(el, ctx, c1m):
    """Different tilings (one, two or four columns per lane) give the same answers to rounding."""
    z = synth.shift_grid(16)
    cols = np.arange(0, 257, 2, dtype=np.int32)
    outs = [el.shifted_solve(ctx, c1m["mat"], cols, z, tol=1e-10, slots=sl, variant=v, mixed=True)
            for sl, v in ((256, "grouped"), (128, "direct"), (192, "grouped1"), (256, 0x80 | 5))]
    x0 = outs[0]["x"].cpu().numpy()
    for o in outs[1:]:
        assert rel_elementwise(o["x"].cpu().numpy(), x0) <= 1e-7
