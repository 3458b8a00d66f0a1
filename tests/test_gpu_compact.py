"""Compact region layout (one persistent launch, one workgroup per region) through the C ABI.

Every check compares with the CPU oracle on the carved region pencil (A_r, B_r)
(Sec. III-B, real-space projection) or with dense solves of it, except the
identities of the layout itself (pattern output = full output on the pattern,
orbital masks, audits) which compare the GPU with itself.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth

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
def box(el, ctx):
    s = synth.make_system(600, 4242)
    return s, el.Matrix.from_system(ctx, s), el.Matrix.from_system(ctx, s, precision="mixed")


def rounded(s):
    return dataclasses.replace(s, A_val=s.A_val.astype(np.float32).astype(np.float64),
                               B_val=s.B_val.astype(np.float32).astype(np.float64))


def sample(s, n, seed, lo=3.0, hi=7.0):
    rng = np.random.default_rng(seed)
    centres = np.sort(rng.choice(s.n_atoms, size=n, replace=False)).astype(np.int32)
    return centres, rng.uniform(lo, hi, size=n)


def carved(s, centre, radius):
    atoms = oracle.region_atoms(s, int(centre), float(radius))
    Ar, Br, orb_map = oracle.carve_region(s, atoms)
    return Ar, Br, {int(g): l for l, g in enumerate(orb_map)}


def test_compact_matches_tiles_and_oracle(el, ctx, box):
    """Compact and tile layouts solve the same region pencils: equal to 1e-8, and each column
    against the oracle's solve of its carved pencil on the column's pattern."""
    s, mat, _ = box
    centres, radii = sample(s, 50, 21)
    z = synth.shift_grid(16)
    K = len(z)
    comp = el.Regions(ctx, mat, centres, radii)
    assert comp.compact and comp.n_tiles == 0
    tile = el.Regions(ctx, mat, centres, radii, 64)
    assert np.array_equal(comp.cols, tile.cols) and np.array_equal(comp.pat_off, tile.pat_off)
    assert np.array_equal(comp.region_orbitals, tile.region_orbitals)
    xc = el.region_solve(ctx, comp, z, tol=1e-10)
    xt = el.region_solve(ctx, tile, z, tol=1e-10)["x"].cpu().numpy()
    x = xc["x"].cpu().numpy()
    assert np.all(xc["resid"].cpu().numpy() <= 1e-10)
    assert np.abs(x - xt).max() <= 1e-8 * np.abs(xt).max()
    B = oracle.to_csr(s, "B")
    for c in range(0, comp.n_cols, 7):
        r = comp.col_region[c]
        Ar, Br, loc = carved(s, centres[r], radii[r])
        j = int(comp.cols[c])
        ref = oracle.shifted_solve(Ar, Br, np.array([loc[j]], np.int32), z, tol=1e-11, full=True)
        rows = B.ci[B.rp[j]:B.rp[j + 1]]
        xr = np.zeros((K, rows.size), complex)
        for p, i in enumerate(rows):
            if int(i) in loc:
                xr[:, p] = ref.x[0, :, loc[int(i)]]
        blk = x[comp.pat_off[c] * K:comp.pat_off[c + 1] * K].reshape(K, -1)
        assert np.abs(blk - xr).max() <= 1e-8 * np.abs(xr).max(), c


def test_full_output_audit_and_pattern_identity(el, ctx, box):
    """Full region vectors: normwise against dense solves of the carved pencil, the in-kernel
    FP64 audit against the oracle's true residual of the same vectors, and the pattern-mode
    output equal to the full vectors on the pattern."""
    s, mat, _ = box
    centres, radii = sample(s, 12, 33, 3.0, 5.5)
    z = synth.shift_grid(12)
    K = len(z)
    reg = el.Regions(ctx, mat, centres, radii)
    tol = 1e-8
    full = el.region_solve(ctx, reg, z, tol=tol, full=True, audit=True)
    pat = el.region_solve(ctx, reg, z, tol=tol)
    xf = full["x"].cpu().numpy()
    xp = pat["x"].cpu().numpy()
    audit = full["resid"].cpu().numpy()
    assert np.array_equal(full["iters"].cpu().numpy(), pat["iters"].cpu().numpy())
    B = oracle.to_csr(s, "B")
    for c in range(reg.n_cols):
        r = reg.col_region[c]
        Ar, Br, loc = carved(s, centres[r], radii[r])
        m = Ar.n
        assert m == reg.region_orbitals[r]
        xv = xf[reg.full_off[c] * K:reg.full_off[c + 1] * K].reshape(K, m)
        j = int(reg.cols[c])
        Ad, Bd = Ar.dense(), Br.dense()
        e = np.zeros(m)
        e[loc[j]] = 1.0
        for k in range(K):
            tr = oracle.true_residual(Ar, Br, loc[j], z[k], xv[k])
            assert tr <= tol
            assert abs(audit[c, k] - tr) <= 1e-4 * tr + 1e-13
            xd = np.linalg.solve(z[k] * Bd - Ad, e)
            assert np.linalg.norm(xv[k] - xd) <= 1e-8 * np.linalg.norm(xd)
        rows = B.ci[B.rp[j]:B.rp[j + 1]]
        blk = xp[reg.pat_off[c] * K:reg.pat_off[c + 1] * K].reshape(K, -1)
        want = np.array([[xv[k, loc[int(i)]] if int(i) in loc else 0.0 for i in rows] for k in range(K)])
        assert np.array_equal(blk, want), c


def test_audit_every_in_pattern_mode(el, ctx, box):
    """audit_every: audited columns get their FP64 true residual, and their pattern output is
    the same as without the audit (the audit carries the full vector, the arithmetic is unchanged)."""
    s, mat, _ = box
    centres, radii = sample(s, 30, 44)
    z = synth.shift_grid(16)
    reg = el.Regions(ctx, mat, centres, radii)
    plain = el.region_solve(ctx, reg, z, tol=1e-8)
    aud = el.region_solve(ctx, reg, z, tol=1e-8, audit_every=5)
    assert np.array_equal(plain["x"].cpu().numpy(), aud["x"].cpu().numpy())
    est = plain["resid"].cpu().numpy()
    tru = aud["resid"].cpu().numpy()
    audited = np.arange(reg.n_cols) % 5 == 0
    assert np.array_equal(tru[~audited], est[~audited])
    assert np.all(tru[audited] <= 1e-8)
    # the true residual tracks the recursive estimate
    print(f"audited true / estimated residual: max {np.max(tru[audited] / est[audited]):.4f}")
    assert np.all(tru[audited] <= 2.0 * est[audited] + 1e-10)


def test_orbital_masks(el, ctx, box):
    """Columns sampled on an atom share its region: masked regions give the same columns as
    the full region (one, two or three orbitals of a carbon centre; padded vector width)."""
    s, mat, _ = box
    carbons = np.nonzero(s.n_orb == 4)[0]
    hyd = np.nonzero(s.n_orb == 1)[0]
    centres = np.sort(np.concatenate([carbons[[2, 9, 15, 30]], hyd[[4, 40]]])).astype(np.int32)
    radii = np.linspace(4.0, 6.5, centres.size)
    masks = np.zeros(centres.size, np.uint8)
    patterns = iter([0b0001, 0b0110, 0b1011, 0b1111])
    for r, cen in enumerate(centres):
        masks[r] = next(patterns) if s.n_orb[cen] == 4 else 0
    z = synth.shift_grid(8)
    K = len(z)
    allreg = el.Regions(ctx, mat, centres, radii)
    mreg = el.Regions(ctx, mat, centres, radii, orb_mask=masks)
    xa = el.region_solve(ctx, allreg, z, tol=1e-10)["x"].cpu().numpy()
    xm = el.region_solve(ctx, mreg, z, tol=1e-10)["x"].cpu().numpy()
    want = [c for c in range(allreg.n_cols)
            if masks[allreg.col_region[c]] == 0
            or (masks[allreg.col_region[c]] >> int(allreg.cols[c] - s.orb_off[centres[allreg.col_region[c]]])) & 1]
    assert mreg.n_cols == len(want)
    assert np.array_equal(mreg.cols, allreg.cols[want])
    for c_m, c_a in enumerate(want):
        a = xa[allreg.pat_off[c_a] * K:allreg.pat_off[c_a + 1] * K]
        b = xm[mreg.pat_off[c_m] * K:mreg.pat_off[c_m + 1] * K]
        assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()


def test_compact_mixed_precision(el, ctx, box):
    """FP32-stored pencils: the rounded carved pencil to 5e-7, the FP64 one to 1e-5, and the
    audit certifies the rounded pencil's true residual in FP64."""
    s, _, mat32 = box
    centres, radii = sample(s, 40, 55, 4.0, 7.0)
    z = synth.shift_grid(16)
    K = len(z)
    reg = el.Regions(ctx, mat32, centres, radii)
    out = el.region_solve(ctx, reg, z, tol=1e-8, mixed=True, audit_every=3)
    assert np.all(out["resid"].cpu().numpy() <= 1e-8)
    x = out["x"].cpu().numpy()
    s32 = rounded(s)
    B = oracle.to_csr(s, "B")
    for c in range(0, reg.n_cols, 9):
        r = reg.col_region[c]
        j = int(reg.cols[c])
        rows = B.ci[B.rp[j]:B.rp[j + 1]]
        blk = x[reg.pat_off[c] * K:reg.pat_off[c + 1] * K].reshape(K, -1)
        for sysm, bound in ((s32, 5e-7), (s, 1e-5)):
            Ar, Br, loc = carved(sysm, centres[r], radii[r])
            ref = oracle.shifted_solve(Ar, Br, np.array([loc[j]], np.int32), z, tol=1e-10, full=True)
            xr = np.array([[ref.x[0, k, loc[int(i)]] if int(i) in loc else 0.0 for i in rows] for k in range(K)])
            assert np.abs(blk - xr).max() <= bound * np.abs(xr).max(), (c, bound)


def test_compact_density_traces(el, ctx, box):
    """rho and the per-column traces from the compact solve equal the oracle's assembly of the
    GPU's own x (Eq. 12, Eq. 7)."""
    s, mat, _ = box
    centres, radii = sample(s, 24, 66)
    z = synth.shift_grid(16)
    cw = oracle.fermi_weights(z, mu=0.1, tau=0.05)
    reg = el.Regions(ctx, mat, centres, radii)
    out = el.region_solve(ctx, reg, z, cw, tol=1e-10)
    xg = out["x"].cpu().numpy()
    A, B = oracle.to_csr(s, "A"), oracle.to_csr(s, "B")
    rho_ref, tb, ta = oracle.density_from_x(B, A, reg.cols, xg, reg.pat_off, cw)
    assert np.abs(out["rho"].cpu().numpy() - rho_ref).max() <= 1e-12 * np.abs(rho_ref).max()
    ct = out["col_traces"].cpu().numpy()
    assert np.abs(ct[:, 0] - tb).max() <= 1e-12 * np.abs(tb).max()
    assert np.abs(ct[:, 1] - ta).max() <= 1e-12 * np.abs(ta).max()
    assert abs(out["traces"][0] - tb.sum()) <= 1e-12 * np.abs(tb).sum()


def test_compact_invalid_arguments(el, ctx, box):
    s, mat, mat32 = box
    reg = el.Regions(ctx, mat, [3, 10], [4.0, 5.0])
    z = synth.shift_grid(4)
    with pytest.raises(el.ElsesError):
        el.region_solve(ctx, reg, z, mixed=True)  # FP64-only matrix
    with pytest.raises(el.ElsesError):
        el.region_solve(ctx, reg, z, full=True, audit_every=2)
    with pytest.raises(el.ElsesError):
        el.region_solve(ctx, reg, z, oracle.fermi_weights(z, 0.0, 0.05), full=True)
    carbon = int(np.nonzero(s.n_orb == 4)[0][0])
    hydrogen = int(np.nonzero(s.n_orb == 1)[0][0])
    with pytest.raises(el.ElsesError):
        el.Regions(ctx, mat, [carbon], [5.0], orb_mask=[0b10000])  # selects no orbital
    ok = el.Regions(ctx, mat, [hydrogen], [5.0], orb_mask=[0b1])
    assert ok.n_cols == 1


def test_compact_edge_cases(el, ctx, box):
    """Degenerate and extreme inputs of the compact path against exact answers.

    - Regions holding only their centre atom (radius below the shortest pair distance,
      1 A): the Krylov space of a 1- or 4-orbital pencil is exhausted within its size, the
      process stops at the breakdown (R5b) and x must equal the dense solve of the carved
      pencil; one slice of 64 positions holds the 1 or 4 real rows.
    - One shift (K = 1) and the largest accepted count (K = 256).
    - A region larger than the periodic box: the whole system, equal to the global solve.
    - Column widths 1, 2 and 4 (orbital masks) and regions of very different size in one
      launch.
    - No regions, or K outside [1, 256], are refused."""
    s, mat, _ = box
    carbons = np.nonzero(s.n_orb == 4)[0]
    hyd = np.nonzero(s.n_orb == 1)[0]
    # single-atom regions: dense comparison of full vectors, FP64 audit
    centres = np.sort(np.array([carbons[5], hyd[7], hyd[8]])).astype(np.int32)
    reg = el.Regions(ctx, mat, centres, np.full(3, 0.5))
    assert sorted(reg.region_orbitals.tolist()) == [1, 1, 4]
    z = synth.shift_grid(8)
    K = len(z)
    out = el.region_solve(ctx, reg, z, tol=1e-10, full=True, audit=True)
    xf = out["x"].cpu().numpy()
    assert np.all(out["resid"].cpu().numpy() <= 1e-10)
    assert np.all(out["iters"].cpu().numpy() <= 4)
    for c in range(reg.n_cols):
        r = reg.col_region[c]
        Ar, Br, loc = carved(s, centres[r], 0.5)
        m = Ar.n
        j = int(reg.cols[c])
        e = np.zeros(m)
        e[loc[j]] = 1.0
        xv = xf[reg.full_off[c] * K:reg.full_off[c + 1] * K].reshape(K, m)
        for k in range(K):
            xd = np.linalg.solve(z[k] * Br.dense() - Ar.dense(), e)
            assert np.linalg.norm(xv[k] - xd) <= 1e-12 * np.linalg.norm(xd), (c, k)
    # K = 1 and K = 256 on the same ragged region set (radii 2.5 .. 7 A), against the oracle
    rng = np.random.default_rng(81)
    centres = np.sort(rng.choice(s.n_atoms, size=10, replace=False)).astype(np.int32)
    radii = rng.uniform(2.5, 7.0, size=10)
    reg = el.Regions(ctx, mat, centres, radii)
    B = oracle.to_csr(s, "B")
    for K in (1, 256):
        z = synth.shift_grid(K)
        out = el.region_solve(ctx, reg, z, tol=1e-9)
        assert np.all(out["resid"].cpu().numpy() <= 1e-9)
        xg = out["x"].cpu().numpy()
        for c in range(0, reg.n_cols, 3):
            r = reg.col_region[c]
            Ar, Br, loc = carved(s, centres[r], radii[r])
            j = int(reg.cols[c])
            ref = oracle.shifted_solve(Ar, Br, np.array([loc[j]], np.int32), z, tol=1e-11, full=True,
                                       true_residual=False)
            rows = B.ci[B.rp[j]:B.rp[j + 1]]
            xr = np.array([[ref.x[0, k, loc[int(i)]] if int(i) in loc else 0.0 for i in rows] for k in range(K)])
            blk = xg[reg.pat_off[c] * K:reg.pat_off[c + 1] * K].reshape(K, -1)
            assert np.abs(blk - xr).max() <= 1e-8 * np.abs(xr).max(), (K, c)
    # the whole box as one region (radius beyond the box), a carbon centre with all four
    # columns, against the global solve of the same columns
    c0 = int(carbons[11])
    whole = el.Regions(ctx, mat, [c0], [1000.0])
    assert whole.region_orbitals[0] == s.M and whole.n_cols == 4
    z = synth.shift_grid(16)
    K = len(z)
    a = el.region_solve(ctx, whole, z, tol=1e-10)
    g = el.shifted_solve(ctx, mat, whole.cols, z, tol=1e-10)
    xa, xg = a["x"].cpu().numpy(), g["x"].cpu().numpy()
    assert np.array_equal(np.asarray(g["pat_off"]), whole.pat_off)
    assert np.abs(xa - xg).max() <= 1e-8 * np.abs(xg).max()
    # widths 1, 2 and 4 in one launch, with a tiny and a large region
    centres = np.sort(np.array([carbons[20], carbons[21], carbons[22], hyd[30], hyd[31]])).astype(np.int32)
    masks = {int(carbons[20]): 0b0001, int(carbons[21]): 0b0110, int(carbons[22]): 0b1111, int(hyd[30]): 1,
             int(hyd[31]): 1}
    radii = {int(carbons[20]): 6.5, int(carbons[21]): 3.0, int(carbons[22]): 5.0, int(hyd[30]): 0.5,
             int(hyd[31]): 7.0}
    mk = np.array([masks[int(c)] for c in centres], np.uint8)
    rd = np.array([radii[int(c)] for c in centres])
    reg = el.Regions(ctx, mat, centres, rd, orb_mask=mk)
    assert reg.n_cols == 1 + 2 + 4 + 1 + 1
    z = synth.shift_grid(12)
    K = len(z)
    out = el.region_solve(ctx, reg, z, tol=1e-10)
    xg = out["x"].cpu().numpy()
    for c in range(reg.n_cols):
        r = reg.col_region[c]
        Ar, Br, loc = carved(s, centres[r], rd[r])
        j = int(reg.cols[c])
        ref = oracle.shifted_solve(Ar, Br, np.array([loc[j]], np.int32), z, tol=1e-11, full=True,
                                   true_residual=False)
        rows = B.ci[B.rp[j]:B.rp[j + 1]]
        xr = np.array([[ref.x[0, k, loc[int(i)]] if int(i) in loc else 0.0 for i in rows] for k in range(K)])
        blk = xg[reg.pat_off[c] * K:reg.pat_off[c + 1] * K].reshape(K, -1)
        assert np.abs(blk - xr).max() <= 1e-8 * np.abs(xr).max(), c
    # refusals
    with pytest.raises(el.ElsesError):
        el.Regions(ctx, mat, np.zeros(0, np.int32), np.zeros(0))
    with pytest.raises(el.ElsesError):
        el.region_solve(ctx, reg, synth.shift_grid(257))


def test_region_overlap_intervals_enclose_spectra(el, ctx, box):
    """Each compact region's overlap interval (the one its Chebyshev-Richardson plan uses:
    extreme Ritz values of its B, widened) encloses the exact spectrum of the carved B_r
    and lies inside B's interval (Cauchy interlacing); typical regions get a narrower
    interval than B's, so a lower polynomial degree."""
    s, mat, _ = box
    centres, radii = sample(s, 24, 93, 2.0, 9.0)
    reg = el.Regions(ctx, mat, centres, radii)
    lo, hi = reg.overlap_intervals()
    blo, bhi = mat.b_interval
    widths = []
    for r in range(len(centres)):
        Ar, Br, loc = carved(s, centres[r], radii[r])
        ev = np.linalg.eigvalsh(Br.dense())
        assert blo <= lo[r] <= ev[0], (r, blo, lo[r], ev[0])
        assert ev[-1] <= hi[r] <= bhi, (r, ev[-1], hi[r], bhi)
        widths.append(hi[r] / lo[r])
    assert np.median(widths) < bhi / blo
