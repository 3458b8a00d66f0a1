"""Learned block SPAI of the overlap through the C ABI, against the CPU FP64 reference (oracle/mlp.py).

Parity: features, exact-inverse targets, the MLP loss and gradient (FP32
kernels vs FP64 backpropagation) and inference (FP32, and BF16 with FP32
accumulation).  Effect (parity unpinned: training is not unique): training
lowers the loss, the learned M is SPD and narrows the spectral interval of
the overlap iteration, and the preconditioned overlap solve gives the same
answer as the plain one.
"""
import time

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp

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
def small(el, ctx):
    s = synth.make_system(64, 2024, r_cut=3.5)
    return s, el.Matrix.from_system(ctx, s)


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype).cuda()


def test_pairs_and_features(el, ctx, small):
    s, mat = small
    P = mlp.pairs(s)
    assert np.array_equal(el.spai_pairs(mat), P)
    f = el.spai_features(ctx, mat).cpu().numpy().astype(np.float64)
    ref = mlp.features(s, P)
    assert np.abs(f - ref).max() <= 1e-6 * np.abs(ref).max()


def test_targets_are_exact_inverse_blocks(el, ctx, small):
    s, mat = small
    P = mlp.pairs(s)
    T, W = el.spai_targets(ctx, mat)
    Binv = np.linalg.inv(oracle.to_csr(s, "B").dense())
    Tr, Wr = mlp.targets(s, P, Binv)
    assert np.array_equal(W.cpu().numpy(), Wr)
    assert np.abs(T.cpu().numpy() - Tr).max() <= 2e-7 * np.abs(Tr).max()


def test_loss_and_gradient_match_oracle(el, ctx, small):
    s, mat = small
    P = mlp.pairs(s)
    X = mlp.features(s, P)
    Binv = np.linalg.inv(oracle.to_csr(s, "B").dense())
    T, W = mlp.targets(s, P, Binv)
    theta = mlp.init_params(3) + 0.02 * np.random.default_rng(4).standard_normal(mlp.N_PARAM)
    # both sides see the same FP32-rounded inputs
    th32, X32, T32 = (a.astype(np.float32) for a in (theta, X, T))
    loss_ref, g_ref = mlp.loss_grad(th32.astype(np.float64), X32.astype(np.float64), T32.astype(np.float64), W)
    loss, g = el.mlp_loss_grad(ctx, dev(th32), dev(X32), dev(T32), dev(W))
    g = g.cpu().numpy().astype(np.float64)
    assert abs(loss - loss_ref) <= 1e-5 * loss_ref
    offs = np.cumsum([0] + [int(np.prod(sh)) for sh in mlp.SHAPES])
    for i in range(len(mlp.SHAPES)):  # every weight and bias block
        gr, gg = g_ref[offs[i]:offs[i + 1]], g[offs[i]:offs[i + 1]]
        assert np.abs(gg - gr).max() <= 1e-4 * np.abs(g_ref).max(), i


def test_inference_fp32_and_bf16(el, ctx, small):
    s, mat = small
    P = mlp.pairs(s)
    X = mlp.features(s, P).astype(np.float32)
    theta = (mlp.init_params(8) + 0.05 * np.random.default_rng(9).standard_normal(mlp.N_PARAM)).astype(np.float32)
    ref, _ = mlp.forward(theta.astype(np.float64), X.astype(np.float64))
    out = el.spai_predict(ctx, dev(theta), dev(X)).cpu().numpy()
    assert np.abs(out - ref).max() <= 1e-5 * np.abs(ref).max()
    ref16 = mlp.forward_bf16(theta, X.astype(np.float64))
    out16 = el.spai_predict(ctx, dev(theta), dev(X), bf16=True).cpu().numpy()
    # FP32 accumulation order can move a BF16 rounding by one unit (2^-8 relative)
    assert np.abs(out16 - ref16).max() <= 2e-2 * np.abs(ref16).max()
    assert np.abs(out16 - ref).max() <= 5e-2 * np.abs(ref).max()


@pytest.fixture(scope="module")
def trained(el, ctx):
    """The network trained on exact inverses of three 500-atom boxes."""
    feats, targs, masks = [], [], []
    for seed in (11, 12, 13):
        s = synth.make_system(500, seed)
        m = el.Matrix.from_system(ctx, s)
        feats.append(el.spai_features(ctx, m))
        T, W = el.spai_targets(ctx, m)
        targs.append(T)
        masks.append(W)
    X, T, W = torch.cat(feats), torch.cat(targs), torch.cat(masks)
    theta = dev(mlp.init_params(synth.config_seed(4) + 5))
    loss0, _ = el.mlp_loss_grad(ctx, theta, X, T, W)
    hist = el.spai_train(ctx, theta, X, T, W, steps=1500, batch=4096, lr=2e-3, seed=1)
    loss1, _ = el.mlp_loss_grad(ctx, theta, X, T, W)
    return theta, loss0, loss1, hist


def test_training_and_preconditioned_overlap_solve(el, ctx, trained):
    """Train on exact inverses of 500-atom boxes, apply to an unseen box."""
    theta, loss0, loss1, hist = trained
    assert loss1 < 0.1 * loss0, (loss0, loss1)
    assert np.all(np.isfinite(hist))
    # unseen box
    s = synth.make_system(500, 99)
    mat = el.Matrix.from_system(ctx, s)
    Mv = el.spai_apply(ctx, mat, theta, bf16=True)
    rng = np.random.default_rng(0)
    rhs = dev(rng.standard_normal((mat.M, 64)), torch.float64)
    x0, p0, br0, u0 = el.overlap_solve(ctx, mat, rhs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x0, p0, br0, u0 = el.overlap_solve(ctx, mat, rhs)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    x1, p1, br1, u1 = el.overlap_solve(ctx, mat, rhs, Mv)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x1, p1, br1, u1 = el.overlap_solve(ctx, mat, rhs, Mv)
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t0
    assert u1 and not u0
    kappa_plain, kappa_pre = br0[1] / br0[0], br1[1] / br1[0]
    print(f"\nSPAI: loss {loss0:.3e} -> {loss1:.3e}; kappa interval {kappa_plain:.3f} -> {kappa_pre:.3f}; "
          f"passes {p0} -> {p1}; time {1e3 * t_plain:.2f} ms -> {1e3 * t_pre:.2f} ms")
    assert kappa_pre < kappa_plain
    B = oracle.to_csr(s, "B").dense()
    ref = np.linalg.solve(B, rhs.cpu().numpy())
    for x in (x0, x1):
        xx = x.cpu().numpy()
        assert np.abs(xx - ref).max() <= 1e-11 * np.abs(ref).max()


def _carved_ref(s, reg, centres, radii, c, z, tol=1e-11):
    """Oracle x of region column c on the column's global pattern (zero outside the region)."""
    r = int(reg.col_region[c])
    atoms = oracle.region_atoms(s, int(centres[r]), float(radii[r]))
    Ar, Br, omap = oracle.carve_region(s, atoms)
    loc = {int(g): l for l, g in enumerate(omap)}
    j = int(reg.cols[c])
    ref = oracle.shifted_solve(Ar, Br, np.array([loc[j]], np.int32), z, tol=tol, full=True, true_residual=False)
    B = oracle.to_csr(s, "B")
    rows = B.ci[B.rp[j]:B.rp[j + 1]]
    return np.array([[ref.x[0, k, loc[int(i)]] if int(i) in loc else 0.0 for i in rows] for k in range(len(z))])


def test_preconditioned_region_solves(el, ctx, trained):
    """The learned M on the solve path: region solves whose overlap solves are CG preconditioned by
    M (elses_mat_set_preconditioner, opts.precond), FP64 and mixed, against the oracle on the carved
    pencils and against the plain solve; M narrows the overlap solves to fewer steps."""
    import dataclasses
    theta = trained[0]
    s = synth.make_system(600, 4242)
    z = synth.shift_grid(16)
    K = len(z)
    rng = np.random.default_rng(71)
    centres = np.sort(rng.choice(s.n_atoms, size=40, replace=False)).astype(np.int32)
    radii = rng.uniform(4.0, 7.0, size=centres.size)
    for precision in ("fp64", "mixed"):
        mat = el.Matrix.from_system(ctx, s, precision=precision)
        plain_reg = el.Regions(ctx, mat, centres, radii)
        el.set_preconditioner(ctx, mat, theta, bf16=True)
        reg = el.Regions(ctx, mat, centres, radii)
        mixed = precision == "mixed"
        tol = 1e-10 if not mixed else 1e-8
        plain = el.region_solve(ctx, plain_reg, z, tol=tol, mixed=mixed)
        prod_plain, fb0 = el.solve_counts(ctx)
        pre = el.region_solve(ctx, reg, z, tol=tol, mixed=mixed, precond=True)
        prod_pre, fb = el.solve_counts(ctx)
        it_plain = plain["iters"].cpu().numpy()
        it_pre = pre["iters"].cpu().numpy()
        print(f"\n{precision}: sparse products {prod_plain} plain -> {prod_pre} preconditioned "
              f"({prod_plain / it_plain.sum():.1f} -> {prod_pre / it_pre.sum():.1f} per column-iteration), "
              f"fallbacks {fb}")
        assert fb0 == 0 and fb == 0
        assert np.all(pre["resid"].cpu().numpy() <= tol)
        xp, xq = plain["x"].cpu().numpy(), pre["x"].cpu().numpy()
        assert np.abs(xq - xp).max() <= (1e-8 if not mixed else 1e-6) * np.abs(xp).max()
        sysm = s if not mixed else dataclasses.replace(
            s, A_val=s.A_val.astype(np.float32).astype(np.float64), B_val=s.B_val.astype(np.float32).astype(np.float64))
        for c in range(0, reg.n_cols, 11):
            xr = _carved_ref(sysm, reg, centres, radii, c, z)
            blk = xq[reg.pat_off[c] * K:reg.pat_off[c + 1] * K].reshape(K, -1)
            assert np.abs(blk - xr).max() <= (1e-8 if not mixed else 5e-7) * np.abs(xr).max(), (precision, c)


def test_preconditioned_global_solves(el, ctx, trained):
    """The learned M in the global path (FP64): shifted solves and the density matrix of an
    unseen box with every overlap solve run as Richardson steps x <- x + tau_k M (s - B x)
    on the interval of M B, against the oracle (shifted COCG with CG overlap solves, tol
    1e-11, and its density assembly) and against the plain solve; mixed precision and
    graph replay are refused with M."""
    theta = trained[0]
    s = synth.make_system(300, 4343)
    mat = el.Matrix.from_system(ctx, s)
    el.set_preconditioner(ctx, mat, theta, bf16=True)
    z = synth.shift_grid(16)
    K = len(z)
    cols = np.arange(0, s.M, 5, dtype=np.int32)
    plain = el.shifted_solve(ctx, mat, cols, z, tol=1e-10)
    pre = el.shifted_solve(ctx, mat, cols, z, tol=1e-10, precond=True)
    _, fb = el.solve_counts(ctx)
    assert fb == 0
    assert np.all(pre["resid"].cpu().numpy() <= 1e-10)
    A, B = oracle.to_csr(s, "A"), oracle.to_csr(s, "B")
    ref = oracle.shifted_solve(A, B, cols, z, tol=1e-11, full=False, true_residual=False)
    xp, xq = plain["x"].cpu().numpy(), pre["x"].cpu().numpy()
    assert np.abs(xq - xp).max() <= 1e-8 * np.abs(xp).max()
    for c in range(len(cols)):
        p0, p1 = int(ref.pat_off[c]), int(ref.pat_off[c + 1])
        xr = ref.x[p0 * K:p1 * K].reshape(K, -1)
        assert np.abs(xq[p0 * K:p1 * K].reshape(K, -1) - xr).max() <= 1e-8 * np.abs(xr).max(), c
    cw = oracle.fermi_weights(z, mu=0.0, tau=0.02)
    d = el.density_matrix(ctx, mat, cols, z, cw, tol=1e-10, precond=True)
    rho_r, trB, trA = oracle.density_from_x(B, A, cols, ref.x, ref.pat_off, cw)
    assert np.abs(d["rho"].cpu().numpy() - rho_r).max() <= 1e-8 * np.abs(rho_r).max()
    ctr = d["col_traces"].cpu().numpy()
    assert np.abs(ctr[:, 0] - trB).max() <= 1e-8 * np.abs(trB).max()
    assert np.abs(ctr[:, 1] - trA).max() <= 1e-8 * np.abs(trA).max()
    with pytest.raises(el.ElsesError):
        el.shifted_solve(ctx, mat, cols, z, precond=True, graph=True)
    m32 = el.Matrix.from_system(ctx, s, precision="mixed")
    el.set_preconditioner(ctx, m32, theta, bf16=True)
    with pytest.raises(el.ElsesError):
        el.shifted_solve(ctx, m32, cols, z, mixed=True, precond=True)


def test_preconditioner_fallback(el, ctx):
    """An indefinite M (a network whose output is minus the identity blocks on every pair) is judged by
    CG's curvature test: every region falls back to the plain iteration and the answers are unchanged;
    in the global path the interval of M B has no positive lower end and the plain steps run."""
    s = synth.make_system(600, 4242)
    mat = el.Matrix.from_system(ctx, s)
    theta = np.zeros(mlp.N_PARAM, dtype=np.float32)
    theta[-16:] = -np.eye(4, dtype=np.float32).reshape(-1)  # b4: output -I for every pair
    el.set_preconditioner(ctx, mat, dev(theta), bf16=False)
    rng = np.random.default_rng(72)
    centres = np.sort(rng.choice(s.n_atoms, size=12, replace=False)).astype(np.int32)
    radii = rng.uniform(4.0, 6.0, size=centres.size)
    reg = el.Regions(ctx, mat, centres, radii)
    z = synth.shift_grid(8)
    plain = el.region_solve(ctx, reg, z, tol=1e-10)
    pre = el.region_solve(ctx, reg, z, tol=1e-10, precond=True, inner_max=40)
    _, fb = el.solve_counts(ctx)
    assert fb == centres.size
    assert np.array_equal(plain["x"].cpu().numpy(), pre["x"].cpu().numpy())
    # the global path: M B has no positive interval, the solve runs the plain steps
    cols = np.arange(0, s.M, 37, dtype=np.int32)
    gp = el.shifted_solve(ctx, mat, cols, z, tol=1e-10)
    gq = el.shifted_solve(ctx, mat, cols, z, tol=1e-10, precond=True)
    _, fb = el.solve_counts(ctx)
    assert fb == 1
    assert np.array_equal(gp["x"].cpu().numpy(), gq["x"].cpu().numpy())
    el.set_preconditioner(ctx, mat, None)
    with pytest.raises(el.ElsesError):  # M removed: the global path refuses precond too
        el.shifted_solve(ctx, mat, cols, z, precond=True)
    with pytest.raises(el.ElsesError):  # a set built without M cannot run the preconditioned path
        el.region_solve(ctx, el.Regions(ctx, mat, centres, radii), z, precond=True)
