"""Region problems (principal sub-pencils around centre atoms) through the C ABI, against the CPU oracle.

Each column's reference is the oracle's solve of the carved region pencil
(A_r, B_r) (Sec. III-B, real-space projection), mapped back to the column's
pattern in the whole box; pattern rows outside the region are zero.
"""
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


def region_reference(s, centre, radius, z, tol=1e-11):
    """Oracle x on the global pattern of each of the centre's orbitals (rows outside the region: 0)."""
    atoms = oracle.region_atoms(s, centre, radius)
    Ar, Br, orb_map = oracle.carve_region(s, atoms)
    loc = {int(g): l for l, g in enumerate(orb_map)}
    B = oracle.to_csr(s, "B")
    out = []
    for q in range(int(s.n_orb[centre])):
        j = int(s.orb_off[centre]) + q
        r = oracle.shifted_solve(Ar, Br, np.array([loc[j]], dtype=np.int32), z, tol=tol, full=True)
        rows = B.ci[B.rp[j]:B.rp[j + 1]]
        x = np.zeros((len(z), rows.size), complex)
        for p, i in enumerate(rows):
            if int(i) in loc:
                x[:, p] = r.x[0, :, loc[int(i)]]
        out.append((j, x, Ar.n))
    return out


def test_regions_match_carved_oracle(el, ctx, box):
    s, mat, _ = box
    rng = np.random.default_rng(5)
    centres = np.sort(rng.choice(s.n_atoms, size=40, replace=False)).astype(np.int32)
    radii = rng.uniform(3.0, 6.5, size=centres.size)
    reg = el.Regions(ctx, mat, centres, radii)
    assert reg.n_cols == int(sum(s.n_orb[c] for c in centres))
    z = synth.shift_grid(16)
    out = el.region_solve(ctx, reg, z, tol=1e-10)
    xg = out["x"].cpu().numpy()
    K = len(z)
    assert np.all(out["resid"].cpu().numpy() <= 1e-10)
    c = 0
    for r, (cen, rad) in enumerate(zip(centres, radii)):
        refs = region_reference(s, int(cen), float(rad), z)
        assert reg.region_orbitals[r] == refs[0][2]
        for j, xr, _ in refs:
            assert reg.cols[c] == j
            blk = xg[reg.pat_off[c] * K:reg.pat_off[c + 1] * K].reshape(K, -1)
            assert np.abs(blk - xr).max() <= 1e-8 * np.abs(xr).max(), (r, j)
            c += 1


def test_region_small_dense(el, ctx, box):
    """A 3 A region against dense solves of its sub-pencil."""
    s, mat, _ = box
    centre = int(np.nonzero(s.n_orb == 4)[0][3])
    reg = el.Regions(ctx, mat, [centre], [3.0])
    z = synth.shift_grid(8)
    out = el.region_solve(ctx, reg, z, tol=1e-11)
    xg = out["x"].cpu().numpy()
    atoms = oracle.region_atoms(s, centre, 3.0)
    Ar, Br, orb_map = oracle.carve_region(s, atoms)
    loc = {int(g): l for l, g in enumerate(orb_map)}
    Ad, Bd = Ar.dense(), Br.dense()
    B = oracle.to_csr(s, "B")
    K = len(z)
    for c, j in enumerate(reg.cols):
        rows = B.ci[B.rp[j]:B.rp[j + 1]]
        blk = xg[reg.pat_off[c] * K:reg.pat_off[c + 1] * K].reshape(K, -1)
        e = np.zeros(Ar.n)
        e[loc[int(j)]] = 1
        for k in range(K):
            xd = np.linalg.solve(z[k] * Bd - Ad, e)
            ref = np.array([xd[loc[int(i)]] if int(i) in loc else 0.0 for i in rows])
            assert np.abs(blk[k] - ref).max() <= 1e-8 * np.abs(ref).max()


def test_whole_box_region_equals_global(el, ctx):
    s = synth.make_system(128, synth.config_seed(1))
    mat = el.Matrix.from_system(ctx, s)
    centres = np.array([0, 5, 17, 64, 127], dtype=np.int32)
    radii = np.full(centres.size, s.L)  # > half the box diagonal: every atom
    reg = el.Regions(ctx, mat, centres, radii)
    assert np.all(reg.region_orbitals == s.M)
    z = synth.shift_grid(32)
    out = el.region_solve(ctx, reg, z, tol=1e-10)
    glob = el.shifted_solve(ctx, mat, reg.cols, z, tol=1e-10)
    xr, xg = out["x"].cpu().numpy(), glob["x"].cpu().numpy()
    assert np.abs(xr - xg).max() <= 1e-8 * np.abs(xg).max()


def test_region_density_and_traces(el, ctx, box):
    s, mat, _ = box
    rng = np.random.default_rng(9)
    centres = np.sort(rng.choice(s.n_atoms, size=24, replace=False)).astype(np.int32)
    radii = rng.uniform(3.0, 6.0, size=centres.size)
    reg = el.Regions(ctx, mat, centres, radii)
    z = synth.shift_grid(16)
    cw = oracle.fermi_weights(z, mu=0.1, tau=0.05)
    out = el.region_solve(ctx, reg, z, cw, tol=1e-10)
    xg = out["x"].cpu().numpy()
    A, B = oracle.to_csr(s, "A"), oracle.to_csr(s, "B")
    # rho and traces from the GPU's own x with the oracle's assembly (Eq. 12, Eq. 7)
    rho_ref, tb, ta = oracle.density_from_x(B, A, reg.cols, xg, reg.pat_off, cw)
    rho = out["rho"].cpu().numpy()
    assert np.abs(rho - rho_ref).max() <= 1e-12 * np.abs(rho_ref).max()
    ct = out["col_traces"].cpu().numpy()
    assert np.abs(ct[:, 0] - tb).max() <= 1e-12 * np.abs(tb).max()
    assert abs(out["traces"][0] - tb.sum()) <= 1e-12 * abs(tb).sum()
    # and x against the carved-region oracle on a few regions
    K = len(z)
    c = 0
    for r, (cen, rad) in enumerate(zip(centres, radii)):
        refs = region_reference(s, int(cen), float(rad), z)
        for j, xr, _ in refs:
            blk = xg[reg.pat_off[c] * K:reg.pat_off[c + 1] * K].reshape(K, -1)
            assert np.abs(blk - xr).max() <= 1e-8 * np.abs(xr).max()
            c += 1
        if r >= 5:
            break


@pytest.mark.parametrize("tile_width", [0, 64, 128])
def test_region_mixed_and_tile_width(el, ctx, box, tile_width):
    s, mat, mat32 = box
    rng = np.random.default_rng(11)
    centres = np.sort(rng.choice(s.n_atoms, size=60, replace=False)).astype(np.int32)
    radii = rng.uniform(4.0, 7.0, size=centres.size)
    z = synth.shift_grid(16)
    ref = el.region_solve(ctx, el.Regions(ctx, mat, centres, radii, 64), z, tol=1e-10)["x"].cpu().numpy()
    x64 = el.region_solve(ctx, el.Regions(ctx, mat, centres, radii, tile_width), z, tol=1e-10)["x"].cpu().numpy()
    assert np.abs(x64 - ref).max() <= 1e-8 * np.abs(ref).max()
    reg32 = el.Regions(ctx, mat32, centres, radii, tile_width)
    out = el.region_solve(ctx, reg32, z, tol=1e-8, mixed=True)
    assert np.all(out["resid"].cpu().numpy() <= 1e-8)
    xm = out["x"].cpu().numpy()
    assert np.abs(xm - ref).max() <= 1e-5 * np.abs(ref).max()


def test_region_invalid_arguments(el, ctx, box):
    s, mat, _ = box
    with pytest.raises(el.ElsesError):
        el.Regions(ctx, mat, [3, 3], [5.0, 5.0])
    with pytest.raises(el.ElsesError):
        el.Regions(ctx, mat, [3], [0.0])
    with pytest.raises(el.ElsesError):
        el.Regions(ctx, mat, [s.n_atoms], [5.0])
    with pytest.raises(el.ElsesError):
        el.Regions(ctx, mat, [3], [5.0], tile_width=96)
    nopos = el.Matrix(ctx, s.n_orb, s.blk_row_ptr, s.blk_col, s.A_val, s.B_val)
    with pytest.raises(el.ElsesError):
        el.Regions(ctx, nopos, [3], [5.0])
