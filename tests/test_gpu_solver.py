"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Bar (FP64 mode): for every compared (j, k) the element-wise difference
|x_gpu - x_ref| <= 1e-8 * max_i |x_ref,i| with both sides solved to a tight
residual, and at the default tolerance 1e-8 the oracle-recomputed true residual
of the GPU solution is <= 1e-8 (the residual certificate the metric is quoted at).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import dense

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


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
def c1(el, ctx):
    s = synth.make_system(128, synth.config_seed(1))
    A, B = oracle.to_csr(s, "A"), oracle.to_csr(s, "B")
    mat = el.Matrix.from_system(ctx, s)
    return s, A, B, mat


def rel_elementwise(xg, xr):
    return np.abs(xg - xr).max() / np.abs(xr).max()


def test_b_interval_brackets_spectrum(c1):
    s, A, B, mat = c1
    lam = np.linalg.eigvalsh(B.dense())
    lo, hi = mat.b_interval
    assert 0 < lo < lam[0] and hi > lam[-1]
    assert lo > 0.9 * lam[0] and hi < 1.1 * lam[-1]


@pytest.mark.parametrize("nvec,variant", [(1, "auto"), (3, "auto"), (64, "direct"), (128, "direct"),
                                          (64, "staged8"), (192, "staged4"), (64, "grouped"), (128, "grouped"),
                                          (320, "grouped"), (128, "grouped2"), (64, "grouped1")])
def test_spmm_matches_oracle_csr(el, ctx, c1, nvec, variant):
    s, A, B, mat = c1
    rng = np.random.default_rng(nvec)
    X = rng.standard_normal((A.n, nvec))
    Xd = torch.from_numpy(X).cuda()
    for which, C in (("A", A), ("B", B)):
        Y = el.spmm(ctx, mat, which, Xd, variant).cpu().numpy().reshape(A.n, nvec)
        ref = np.stack([C.matvec(X[:, v]) for v in range(nvec)], axis=1)
        assert np.abs(Y - ref).max() <= 1e-14 * np.abs(ref).max()


def test_full_mode_tight_vs_oracle_and_dense(el, ctx, c1):
    s, A, B, mat = c1
    z = synth.shift_grid(32)
    cols = np.array([0, 1, 2, 3, 100, 171, 172, 200, 256], dtype=np.int32)
    out = el.shifted_solve(ctx, mat, cols, z, tol=1e-10, full=True, audit=True)
    xg = out["x"].cpu().numpy()
    ref = oracle.shifted_solve(A, B, cols, z, tol=1e-11, full=True)
    Ad, Bd = A.dense(), B.dense()
    res = out["resid"].cpu().numpy()
    # true residual <= tol + |z| ||B - p(B)^{-1}|| ||x||: the overlap solve is the fixed
    # polynomial p(B) with ||I - p(B) B|| <= inner_tol = 1e-13
    xnorm = np.linalg.norm(xg, axis=2)
    bound = 1e-10 * 1.0001 + 2e-13 * np.abs(z)[None, :] * mat.b_interval[1] * xnorm
    assert np.all(res <= bound), (res / bound).max()
    for c, j in enumerate(cols):
        for k in range(len(z)):
            assert rel_elementwise(xg[c, k], ref.x[c, k]) <= 1e-8, (j, k)
            lu = np.linalg.solve(z[k] * Bd - Ad, np.eye(A.n)[:, j])
            assert rel_elementwise(xg[c, k], lu) <= 1e-8, (j, k)


def test_all_columns_pattern_mode_default_tol(el, ctx, c1):
    """C1 workload: all 257 columns x 32 shifts at tol 1e-8; a ragged last tile."""
    s, A, B, mat = c1
    z = synth.shift_grid(32)
    cols = np.arange(A.n, dtype=np.int32)
    out = el.shifted_solve(ctx, mat, cols, z, tol=1e-8)
    pat_off = out["pat_off"]
    xg = out["x"].cpu().numpy()
    K = len(z)
    assert np.all(out["resid"].cpu().numpy() <= 1e-8)
    iters = out["iters"].cpu().numpy()
    assert iters.min() > 100 and iters.max() < 5000
    # oracle on a sample of columns, element by element on the pattern (tight reference)
    sample = np.array([0, 5, 42, 43, 44, 130, 255, 256], dtype=np.int32)
    ref = oracle.shifted_solve(A, B, sample, z, tol=1e-11, full=True)
    lmin = np.linalg.eigvalsh(B.dense())[0]
    for c, j in enumerate(sample):
        rows = B.ci[B.rp[j]:B.rp[j + 1]]
        blk = xg[pat_off[j] * K:pat_off[j + 1] * K].reshape(K, -1)
        for k in range(K):
            # forward error bound from the residual certificate
            bound = 1e-8 / (z[k].imag * lmin)
            assert np.abs(blk[k] - ref.x[c, k][rows]).max() <= bound
            assert rel_elementwise(blk[k], ref.x[c, k][rows]) <= 5e-7
    # symmetry G_ij = G_ji across the whole pattern
    Gd = np.zeros((K, A.n, A.n), complex)
    for j in range(A.n):
        rows = B.ci[B.rp[j]:B.rp[j + 1]]
        Gd[:, rows, j] = xg[pat_off[j] * K:pat_off[j + 1] * K].reshape(K, -1)
    assert np.abs(Gd - np.transpose(Gd, (0, 2, 1))).max() <= 2e-6 * np.abs(Gd).max()


def test_pattern_mode_tight_elementwise(el, ctx, c1):
    s, A, B, mat = c1
    z = synth.shift_grid(32)
    cols = np.array([7, 8, 99, 150, 180, 181], dtype=np.int32)
    out = el.shifted_solve(ctx, mat, cols, z, tol=1e-11)
    ref = oracle.shifted_solve(A, B, cols, z, tol=1e-11, full=False)
    xg = out["x"].cpu().numpy()
    assert np.array_equal(out["pat_off"], ref.pat_off)
    K = len(z)
    for c in range(len(cols)):
        a = xg[out["pat_off"][c] * K:out["pat_off"][c + 1] * K].reshape(K, -1)
        b = ref.x[ref.pat_off[c] * K:ref.pat_off[c + 1] * K].reshape(K, -1)
        for k in range(K):
            assert rel_elementwise(a[k], b[k]) <= 1e-8


def test_density_matrix_traces_closed_form(el, ctx):
    s = synth.make_system(64, 2024, r_cut=3.5)
    A, B = oracle.to_csr(s, "A"), oracle.to_csr(s, "B")
    mat = el.Matrix.from_system(ctx, s)
    z = synth.shift_grid(16, lo=-1.0, hi=1.0, eta=0.05)
    cw = oracle.fermi_weights(z, mu=0.2, tau=0.1)
    cols = np.arange(A.n, dtype=np.int32)
    out = el.density_matrix(ctx, mat, cols, z, cw, tol=1e-11)
    refB, refA = dense.trace_closed_forms(A.dense(), B.dense(), z, cw)
    trB, trA = out["traces"]
    assert abs(trB - refB) <= 1e-9 * abs(refB)
    assert abs(trA - refA) <= 1e-9 * max(1.0, abs(refA))
    # rho element by element against the oracle's rho from its own x
    r = oracle.shifted_solve(A, B, cols, z, tol=1e-11, full=False)
    rho_ref, tb, ta = oracle.density_from_x(B, A, cols, r.x, r.pat_off, cw)
    rho = out["rho"].cpu().numpy()
    assert np.abs(rho - rho_ref).max() <= 1e-8 * np.abs(rho_ref).max()
    ct = out["col_traces"].cpu().numpy()
    assert np.abs(ct[:, 0] - tb).max() <= 1e-8 * np.abs(tb).max()


def test_overlap_interval_beyond_the_richardson_cap_is_refused(el, ctx):
    """An SPD overlap with eigenvalues 0.0201 .. 1: its widened interval (2 % of the width
    on each side, about [4.8e-4, 1.02]) needs about 700 steps of the overlap solve's
    Chebyshev-Richardson plan to reach 1e-13 (R4), beyond the 400-step cap: the solve is
    refused with what it would reach, instead of returning results of an overlap solve
    less accurate than inner_tol."""
    n_at = 6
    n_orb = np.array([1] * n_at, np.int8)
    rp = np.arange(n_at + 1, dtype=np.int64)
    bc = np.arange(n_at, dtype=np.int32)
    Av = np.linspace(-0.5, 0.5, n_at)
    Bv = np.array([0.0201, 0.3, 0.5, 0.7, 0.9, 1.0])
    mat = el.Matrix(ctx, n_orb, rp, bc, Av, Bv)
    z = synth.shift_grid(4, eta=0.05)
    lo, hi = mat.b_interval
    assert 0.0 < lo < 1e-3 and hi > 1.0
    with pytest.raises(el.ElsesError) as e:
        el.shifted_solve(ctx, mat, np.arange(n_at, dtype=np.int32), z, tol=1e-8)
    assert "Richardson steps" in str(e.value)


def test_diagonal_pencil_one_iteration(el, ctx):
    """A, B diagonal (only on-site blocks): x = e_j / (z B_jj - A_jj) after one step."""
    n_at = 10
    n_orb = np.array([4] * 3 + [1] * 7, np.int8)
    rp = np.arange(n_at + 1, dtype=np.int64)
    bc = np.arange(n_at, dtype=np.int32)
    rng = np.random.default_rng(3)
    a_vals, b_vals = [], []
    for no in n_orb:
        a_vals.append(np.diag(rng.uniform(-1, 1, no)).ravel())
        b_vals.append(np.diag(rng.uniform(0.5, 2, no)).ravel())
    Av, Bv = np.concatenate(a_vals), np.concatenate(b_vals)
    mat = el.Matrix(ctx, n_orb, rp, bc, Av, Bv)
    M = mat.M
    ad = np.concatenate([np.diag(v.reshape(int(np.sqrt(v.size)), -1)) for v in a_vals])
    bd = np.concatenate([np.diag(v.reshape(int(np.sqrt(v.size)), -1)) for v in b_vals])
    z = synth.shift_grid(5, eta=0.05)
    cols = np.arange(M, dtype=np.int32)
    out = el.shifted_solve(ctx, mat, cols, z, tol=1e-12, full=True)
    x = out["x"].cpu().numpy()
    assert np.all(out["iters"].cpu().numpy() == 1)
    for j in range(M):
        for k in range(len(z)):
            ref = np.zeros(M, complex)
            ref[j] = 1 / (z[k] * bd[j] - ad[j])
            # the overlap solve is a polynomial p(B) with |1 - p(b) b| <= 1e-13, so the
            # computed x solves z/p(b) - a: |dx| <= 1e-13 |z| b |x|^2 (+ rounding)
            bound = 2e-13 * abs(z[k]) * bd[j] * abs(ref[j]) ** 2 + 1e-15 * abs(ref[j])
            assert np.abs(x[j, k] - ref).max() <= bound


def test_single_shift_and_empty_column_list(el, ctx, c1):
    s, A, B, mat = c1
    z = np.array([0.3 + 0.01j])
    out = el.shifted_solve(ctx, mat, np.array([17], np.int32), z, tol=1e-11, full=True)
    lu = np.linalg.solve(z[0] * B.dense() - A.dense(), np.eye(A.n)[:, 17])
    assert rel_elementwise(out["x"].cpu().numpy()[0, 0], lu) <= 1e-8
    out = el.shifted_solve(ctx, mat, np.zeros(0, np.int32), z)
    assert out["iters"].numel() == 0


def test_not_converged_reports_and_writes(el, ctx, c1):
    s, A, B, mat = c1
    z = synth.shift_grid(4)
    with pytest.raises(el.NotConverged):
        el.shifted_solve(ctx, mat, np.array([3], np.int32), z, max_outer=5)
    out = el.shifted_solve(ctx, mat, np.array([3], np.int32), z, max_outer=5, allow_not_converged=True)
    assert int(out["iters"].cpu()[0]) == 5
    assert np.all(out["resid"].cpu().numpy() > 1e-8)


def test_invalid_arguments(el, ctx, c1):
    s, A, B, mat = c1
    with pytest.raises(el.ElsesError) as e:
        el.shifted_solve(ctx, mat, np.array([3], np.int32), np.array([0.1 + 0.0j]))
    assert e.value.status == el.ELSES_ERR_INVALID_ARG
    with pytest.raises(el.ElsesError):
        el.shifted_solve(ctx, mat, np.array([3, 3], np.int32), np.array([0.1 + 0.01j]))
    with pytest.raises(el.ElsesError):
        el.shifted_solve(ctx, mat, np.array([A.n], np.int32), np.array([0.1 + 0.01j]))
    bad = s.A_val.copy()
    bad[5] = np.nan
    with pytest.raises(el.ElsesError):
        el.Matrix(ctx, s.n_orb, s.blk_row_ptr, s.blk_col, bad, s.B_val)
    asym = s.A_val.copy()
    asym[s.val_ptr[1]] += 1e-3  # an off-diagonal block entry without its mirror
    with pytest.raises(el.ElsesError):
        el.Matrix(ctx, s.n_orb, s.blk_row_ptr, s.blk_col, asym, s.B_val)


def test_non_spd_overlap_rejected(el, ctx, c1):
    s, A, B, mat = c1
    negB = -s.B_val
    with pytest.raises(el.ElsesError) as e:
        el.Matrix(ctx, s.n_orb, s.blk_row_ptr, s.blk_col, s.A_val, negB)
    assert e.value.status == el.ELSES_ERR_NOT_SPD


def test_identity_overlap(el, ctx, c1):
    """B = I: the plain shifted equations (zI - A) x = e_j."""
    s, A, B, mat = c1
    Bv = np.zeros_like(s.B_val)
    for I in range(s.n_atoms):
        b = s.blk_row_ptr[I] + np.searchsorted(s.blk_col[s.blk_row_ptr[I]:s.blk_row_ptr[I + 1]], I)
        no = s.n_orb[I]
        Bv[s.val_ptr[b]:s.val_ptr[b + 1]] = np.eye(no).ravel()
    m2 = el.Matrix(ctx, s.n_orb, s.blk_row_ptr, s.blk_col, s.A_val, Bv)
    z = synth.shift_grid(8)
    cols = np.array([0, 50, 250], np.int32)
    out = el.shifted_solve(ctx, m2, cols, z, tol=1e-11, full=True)
    x = out["x"].cpu().numpy()
    Ad = A.dense()
    for c, j in enumerate(cols):
        for k in range(len(z)):
            lu = np.linalg.solve(z[k] * np.eye(A.n) - Ad, np.eye(A.n)[:, j])
            assert rel_elementwise(x[c, k], lu) <= 1e-8


def test_slot_counts_agree(el, ctx, c1):
    """Different slot counts (tile shapes, refills mid-run) give the same answers."""
    s, A, B, mat = c1
    z = synth.shift_grid(8)
    cols = np.arange(0, A.n, 2, dtype=np.int32)  # 129 columns
    outs = [el.shifted_solve(ctx, mat, cols, z, tol=1e-10, slots=sl, variant=v)["x"].cpu().numpy()
            for sl, v in ((64, "staged8"), (128, "direct"), (256, "staged4"), (256, "direct"), (192, "grouped"),
                          (128, "grouped2"), (128, "grouped1"))]
    for o in outs[1:]:
        assert np.abs(o - outs[0]).max() <= 1e-8 * np.abs(outs[0]).max()
