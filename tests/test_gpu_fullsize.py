"""Parity at the full sizes of the benchmark workloads, in the launch configurations the benchmark times.

Outputs are compared on samples the CPU oracle computes one by one; the
rest is checked through properties that hold at any size (every residual
estimate <= tol, symmetry G_ij = G_ji, agreement of two solvers).
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

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


def fermi_cw(z):
    K = len(z)
    return (-(1.0 / np.pi) * (2.0 / K) * 0.5 * (1.0 - np.tanh(0.5 * z.real / 0.01))).astype(np.complex128)


def pattern_rows(s, j):
    """Rows of the pattern of column j: the orbitals of the atoms coupled to j's atom, ascending."""
    J = int(np.searchsorted(s.orb_off, j, side="right") - 1)
    nb = s.blk_col[s.blk_row_ptr[J]:s.blk_row_ptr[J + 1]]
    return np.concatenate([np.arange(s.orb_off[I], s.orb_off[I] + s.n_orb[I]) for I in nb])


def pattern_values(s, j, which):
    """X_{j,i} for i in the pattern of column j, from the atom blocks."""
    vals = s.A_val if which == "A" else s.B_val
    J = int(np.searchsorted(s.orb_off, j, side="right") - 1)
    a = int(j - s.orb_off[J])
    nJ = int(s.n_orb[J])
    out = []
    for b in range(int(s.blk_row_ptr[J]), int(s.blk_row_ptr[J + 1])):
        nI = int(s.n_orb[s.blk_col[b]])
        out.append(vals[s.val_ptr[b]:s.val_ptr[b + 1]].reshape(nJ, nI)[a])
    return np.concatenate(out)


def rounded(s):
    return dataclasses.replace(s, A_val=s.A_val.astype(np.float32).astype(np.float64),
                               B_val=s.B_val.astype(np.float32).astype(np.float64))


def test_c2_batch_of_1024_columns(el, ctx):
    """4096-atom box, FP64, first batch of 1024 columns x 64 shifts at tol 1e-8 (1024 slots, default passes)."""
    s = synth.make_system(4096, synth.config_seed(2))
    mat = el.Matrix.from_system(ctx, s)
    z = synth.shift_grid(64)
    cw = fermi_cw(z)
    cols = np.arange(1024, dtype=np.int32)
    out = el.density_matrix(ctx, mat, cols, z, cw, want_x=True)
    assert np.all(out["resid"].cpu().numpy() <= 1e-8)
    K = len(z)
    xg = out["x"].cpu().numpy()
    pat_off = out["pat_off"]
    A, B = oracle.to_csr(s, "A"), oracle.to_csr(s, "B")
    # symmetry G_ij = G_ji for pairs inside the batch
    worst, scale = 0.0, 0.0
    for j in (5, 400, 777):
        rows = B.ci[B.rp[j]:B.rp[j + 1]]
        blk = xg[pat_off[j] * K:pat_off[j + 1] * K].reshape(K, -1)
        for p, i in enumerate(rows):
            if i >= 1024:
                continue
            ri = B.ci[B.rp[i]:B.rp[i + 1]]
            q = int(np.searchsorted(ri, j))
            other = xg[pat_off[i] * K:pat_off[i + 1] * K].reshape(K, -1)[:, q]
            worst = max(worst, np.abs(blk[:, p] - other).max())
            scale = max(scale, np.abs(blk[:, p]).max())
    assert worst <= 2e-6 * scale
    # sampled columns against the oracle (shifted COCG to 1e-10, one column per thread)
    sample = np.array([0, 333, 700, 1023], dtype=np.int32)
    ref = oracle.shifted_solve(A, B, sample, z, tol=1e-10, full=False, true_residual=False)
    lo = mat.b_interval[0]
    rho = out["rho"].cpu().numpy()
    rho_ref, _, _ = oracle.density_from_x(B, A, sample, ref.x, ref.pat_off, cw)
    for c, j in enumerate(sample):
        blk = xg[pat_off[j] * K:pat_off[j + 1] * K].reshape(K, -1)
        rb = ref.x[ref.pat_off[c] * K:ref.pat_off[c + 1] * K].reshape(K, -1)
        for k in range(K):
            assert np.abs(blk[k] - rb[k]).max() <= 1e-8 / (z[k].imag * lo)
            assert np.abs(blk[k] - rb[k]).max() <= 5e-7 * np.abs(rb[k]).max()
        rg = rho[pat_off[j]:pat_off[j + 1]]
        rr = rho_ref[ref.pat_off[c]:ref.pat_off[c + 1]]
        assert np.abs(rg - rr).max() <= 1e-6 * np.abs(rr).max()


def test_c3_region_tiles(el, ctx):
    """50000-atom box, the benchmark's region sample and packing (64-slot tiles), mixed precision."""
    s = synth.make_system(50000, synth.config_seed(3))
    mat = el.Matrix.from_system(ctx, s, precision="mixed")
    centres, radii = synth.sample_regions(s, 2048, synth.config_seed(3))
    centres, radii = centres[:96], radii[:96]
    reg = el.Regions(ctx, mat, centres, radii, 64)
    z = synth.shift_grid(64)
    out = el.region_solve(ctx, reg, z, fermi_cw(z), mixed=True)
    assert np.all(out["resid"].cpu().numpy() <= 1e-8)
    xg = out["x"].cpu().numpy()
    K = len(z)
    s32 = rounded(s)
    col_region = np.repeat(np.arange(centres.size), [int(s.n_orb[c]) for c in centres])
    # one carbon-centred and one hydrogen-centred region
    picks = [int(np.nonzero(s.n_orb[centres] == 4)[0][0]), int(np.nonzero(s.n_orb[centres] == 1)[0][0])]
    for r in picks:
        atoms = oracle.region_atoms(s, int(centres[r]), float(radii[r]))
        Ar, Br, orb_map = oracle.carve_region(s32, atoms)
        Ar64, Br64, _ = oracle.carve_region(s, atoms)
        loc = {int(g): l for l, g in enumerate(orb_map)}
        cidx = np.nonzero(col_region == r)[0]
        lcols = np.array([loc[int(reg.cols[c])] for c in cidx], dtype=np.int32)
        ref32 = oracle.shifted_solve(Ar, Br, lcols, z, tol=1e-10, full=True, true_residual=False)
        ref64 = oracle.shifted_solve(Ar64, Br64, lcols, z, tol=1e-10, full=True, true_residual=False)
        for q, c in enumerate(cidx):
            j = int(reg.cols[c])
            rows = pattern_rows(s, j)
            sel = [loc.get(int(i), -1) for i in rows]
            blk = xg[reg.pat_off[c] * K:reg.pat_off[c + 1] * K].reshape(K, -1)
            for k in range(K):
                r32 = np.array([ref32.x[q, k, l] if l >= 0 else 0.0 for l in sel])
                r64 = np.array([ref64.x[q, k, l] if l >= 0 else 0.0 for l in sel])
                assert np.abs(blk[k] - r32).max() <= 5e-7 * np.abs(r32).max()
                assert np.abs(blk[k] - r64).max() <= 1e-5 * np.abs(r64).max()


def first_step_regions(s, n_sampled, seed, batch=1280):
    """The region set of the benchmark's first step: sampled columns, radius U[6,14] A,
    the columns of one atom sharing its region, consecutive regions up to `batch` columns."""
    cols = synth.sample_columns(s, n_sampled, seed)
    centres, masks, radii = synth.column_regions(s, cols, seed)
    ncol = np.array([bin(int(m)).count("1") for m in masks])
    nb = int(np.searchsorted(np.cumsum(ncol), batch, side="left")) + 1
    return centres[:nb], masks[:nb], radii[:nb], ncol[:nb]


def check_region_subsample(s, reg, centres, radii, ncol, out, z, cw, seed):
    """x, rho and the per-column traces of a seeded subsample of a mixed-precision region
    solve (the largest region, the smallest, a multi-column one and two random ones)
    against the oracle on the carved FP32-rounded pencil (what mixed precision solves,
    5e-7) and, below the largest, on the FP64 pencil (1e-5)."""
    K = len(z)
    nb = centres.size
    xg = out["x"].cpu().numpy()
    rho = out["rho"].cpu().numpy()
    ctr = out["col_traces"].cpu().numpy()
    rng = np.random.default_rng(seed)
    big = int(np.argmax(reg.region_orbitals))
    picks = [big, int(np.argmin(reg.region_orbitals))]
    multi = np.nonzero(ncol > 1)[0]
    if multi.size:
        picks.append(int(multi[0]))
    picks += [int(r) for r in rng.choice(nb, size=2, replace=False)]
    picks = list(dict.fromkeys(picks))
    s32 = rounded(s)
    jobs = []
    for r in picks:
        for c in np.nonzero(reg.col_region == r)[0]:
            jobs.append((int(r), int(c), s32, 5e-7))
            if r != big:
                jobs.append((int(r), int(c), s, 1e-5))

    def run(job):
        r, c, sysm, bound = job
        atoms = oracle.region_atoms(sysm, int(centres[r]), float(radii[r]))
        Ar, Br, orb_map = oracle.carve_region(sysm, atoms)
        loc = {int(g): l for l, g in enumerate(orb_map)}
        j = int(reg.cols[c])
        ref = oracle.shifted_solve(Ar, Br, np.array([loc[j]], dtype=np.int32), z, tol=1e-8 if r == big else 1e-9,
                                   full=False, true_residual=False, nthreads=1)
        # radius >= 6 A > the 4 A cutoff: the whole pattern of j lies inside the region, in the same order
        rows_j = pattern_rows(s, j)
        assert ref.pat_off[1] == rows_j.size
        return job, ref.x.reshape(K, rows_j.size)

    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(max_workers=min(16, len(jobs))) as ex:
        results = list(ex.map(run, jobs))
    for (r, c, sysm, bound), xr in results:
        j = int(reg.cols[c])
        blk = xg[reg.pat_off[c] * K:reg.pat_off[c + 1] * K].reshape(K, -1)
        assert np.abs(blk - xr).max() <= bound * np.abs(xr).max(), (r, c, bound)
        # rho_ij = sum_k Im(c_k x_{j,k,i}) on the pattern (Eq. 12) and e_j^T rho X e_j (Eq. 7) from the
        # oracle's x and the matrix values of row j
        rho_r = np.imag(cw[:, None] * xr).sum(axis=0)
        tb = float(rho_r @ pattern_values(s, j, "B"))
        ta = float(rho_r @ pattern_values(s, j, "A"))
        rg = rho[reg.pat_off[c]:reg.pat_off[c + 1]]
        assert np.abs(rg - rho_r).max() <= 2 * bound * np.abs(rho_r).max(), (r, c)
        assert abs(ctr[c, 0] - tb) <= 2 * bound * abs(tb) + 1e-14, (r, c)
        assert abs(ctr[c, 1] - ta) <= 2 * bound * abs(ta) + 1e-14, (r, c)
    return sorted(int(reg.region_orbitals[r]) for r in picks)


def test_c4_learned_spai_and_regions(el, ctx):
    """100000-atom box: the learned SPAI assembled into the matrix at full size
    (elses_mat_set_preconditioner, BF16 inference), the standalone preconditioned
    overlap solve against the plain one, then the benchmark's first c4 step: 1280
    sampled columns solved as mixed-precision compact regions (radius U[6,14] A,
    64 shifts) with the overlap solves preconditioned by M, x, rho and the
    per-column traces of a seeded subsample (the largest and the smallest region
    included) against the oracle on the carved pencils."""
    from oracle import mlp
    feats, targs, masks = [], [], []
    for seed in (21, 22, 23):
        m = el.Matrix.from_system(ctx, synth.make_system(500, seed))
        feats.append(el.spai_features(ctx, m))
        T, W = el.spai_targets(ctx, m)
        targs.append(T)
        masks.append(W)
    theta = torch.as_tensor(mlp.init_params(synth.config_seed(4) + 5), dtype=torch.float32).cuda()
    el.spai_train(ctx, theta, torch.cat(feats), torch.cat(targs), torch.cat(masks), steps=1500, batch=4096,
                  lr=2e-3, seed=4)
    s = synth.make_system(100000, synth.config_seed(4))
    mat = el.Matrix.from_system(ctx, s, precision="mixed")
    Mv = el.spai_apply(ctx, mat, theta, bf16=True)
    rhs = torch.as_tensor(np.random.default_rng(4).standard_normal((mat.M, 64))).cuda()
    x0, p0, br0, u0 = el.overlap_solve(ctx, mat, rhs)
    x1, p1, br1, u1 = el.overlap_solve(ctx, mat, rhs, Mv)
    assert u1 and not u0
    assert br1[1] / br1[0] < br0[1] / br0[0]
    assert (x1 - x0).abs().max().item() <= 1e-11 * x0.abs().max().item()
    res = el.spmm(ctx, mat, "B", x1) - rhs
    assert res.abs().max().item() <= 1e-11 * rhs.abs().max().item()
    print(f"\nC4 SPAI: interval ratio {br0[1] / br0[0]:.3f} -> {br1[1] / br1[0]:.3f}, passes {p0} -> {p1}")
    del Mv, rhs, x0, x1, res
    # M on the matrix, then the region set of the benchmark's first step
    el.set_preconditioner(ctx, mat, theta, bf16=True)
    centres, masks, radii, ncol = first_step_regions(s, 16384, synth.config_seed(4))
    reg = el.Regions(ctx, mat, centres, radii, orb_mask=masks)
    z = synth.shift_grid(64)
    cw = fermi_cw(z)
    el.solve_counts(ctx)
    out = el.region_solve(ctx, reg, z, cw, tol=1e-8, mixed=True, precond=True)
    products, fallbacks = el.solve_counts(ctx)
    assert np.all(out["resid"].cpu().numpy() <= 1e-8)
    print(f"C4: {reg.n_cols} sampled columns in {centres.size} regions of {reg.region_orbitals.min()}-"
          f"{reg.region_orbitals.max()} orbitals, outer iterations max {int(out['iters'].max())}, "
          f"{products} sparse products, {fallbacks} preconditioner fallbacks", flush=True)
    sizes = check_region_subsample(s, reg, centres, radii, ncol, out, z, cw, 44)
    print(f"C4 subsample against the oracle: regions of {sizes} orbitals", flush=True)


def _row_products(s, rows, x, which):
    """Exact FP64 products (X x)[r] of sampled rows r from the atom blocks (values
    rounded to FP32 first when `x` is FP32, as the FP32 product reads them)."""
    vals = s.A_val if which == "A" else s.B_val
    fp32 = x.dtype == np.float32
    atom_of = np.repeat(np.arange(s.n_atoms), s.n_orb.astype(int))
    out = np.zeros((len(rows), x.shape[1]))
    mag = np.zeros((len(rows), x.shape[1]))
    for i, r in enumerate(rows):
        I = int(atom_of[r])
        a = int(r - s.orb_off[I])
        nI = int(s.n_orb[I])
        for b in range(int(s.blk_row_ptr[I]), int(s.blk_row_ptr[I + 1])):
            J = int(s.blk_col[b])
            nJ = int(s.n_orb[J])
            v = vals[s.val_ptr[b]:s.val_ptr[b + 1]].reshape(nI, nJ)[a]
            if fp32:
                v = v.astype(np.float32).astype(np.float64)
            xs = x[s.orb_off[J]:s.orb_off[J] + nJ].astype(np.float64)
            out[i] += v @ xs
            mag[i] += np.abs(v) @ np.abs(xs)
    return out, mag


def test_c5_one_gpu_share(el, ctx):
    """10^6-atom box (M = 2.0e6, FP32-stored matrices): sampled rows of the FP32
    and FP64 products against exact products from the atom blocks; then the
    first step of `bench.py` (default c5): 1280 sampled columns solved as
    mixed-precision compact regions (radius U[6,14] A, 128 shifts), with x,
    rho and the per-column traces of a seeded subsample (the largest and the
    smallest region included) against the oracle on the carved pencils."""
    s = synth.make_system(1000000, synth.config_seed(5))
    mat = el.Matrix.from_system(ctx, s, precision="mixed")
    assert mat.M == s.M and s.M > 1_990_000
    rng = np.random.default_rng(5)
    rows = np.sort(rng.choice(s.M, size=48, replace=False))
    for which in ("A", "B"):
        x32 = torch.as_tensor(rng.standard_normal((s.M, 256)).astype(np.float32)).cuda()
        y32 = el.spmm32(ctx, mat, which, x32)
        ref, mag = _row_products(s, rows, x32.cpu().numpy(), which)
        got = y32[torch.as_tensor(rows).cuda()].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(got - ref) <= 8e-6 * mag + 1e-30)
        del x32, y32
    x64 = torch.as_tensor(rng.standard_normal((s.M, 64))).cuda()
    y64 = el.spmm(ctx, mat, "B", x64)
    ref, mag = _row_products(s, rows, x64.cpu().numpy(), "B")
    got = y64[torch.as_tensor(rows).cuda()].cpu().numpy()
    assert np.all(np.abs(got - ref) <= 1e-14 * mag + 1e-300)
    del x64, y64
    del mat
    # the benchmark's first step: its region set in the compact layout, 128 shifts, mixed precision,
    # rho and traces
    mat = el.Matrix.from_system(ctx, s, precision="mixed")
    centres, masks, radii, ncol = first_step_regions(s, 65536, synth.config_seed(5))
    reg = el.Regions(ctx, mat, centres, radii, orb_mask=masks)
    z = synth.shift_grid(128)
    cw = fermi_cw(z)
    out = el.region_solve(ctx, reg, z, cw, tol=1e-8, mixed=True)
    assert np.all(out["resid"].cpu().numpy() <= 1e-8)
    print(f"\nC5: {reg.n_cols} sampled columns in {centres.size} regions of {reg.region_orbitals.min()}-"
          f"{reg.region_orbitals.max()} orbitals, outer iterations max {int(out['iters'].max())}", flush=True)
    sizes = check_region_subsample(s, reg, centres, radii, ncol, out, z, cw, 55)
    print(f"C5 subsample against the oracle: regions of {sizes} orbitals", flush=True)
