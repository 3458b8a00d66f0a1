"""Multiple Arnoldi method on the GPU (Eqs. 15-18) against the oracle.

Tolerance: the reduced problems are formed in FP64 from Gram-Schmidt
coefficients and row-chunked dot products over at most a few thousand rows
(rounding ~1e-13), and B^{-1} e_j is a Richardson solve to 1e-13; moving it by
that much changes the nu = 30 sums by ~3e-13 on these pencils.  Ritz values,
the Eq. 18 sums and the density-matrix entries are compared at 1e-9 absolute
(all are O(1)); the subspace dimension must agree exactly.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import arnoldi as ma
from oracle import dense

pytestmark = pytest.mark.gpu

TOL = 1e-9
MU, KT = 0.1, 0.1


def fermi(e):
    return dense.fermi(e, MU, KT)


@pytest.fixture(scope="module")
def ctx():
    import paper_1609_08377_amd as pk
    return pk.Context(0)


@pytest.fixture(scope="module")
def c1(ctx):
    import paper_1609_08377_amd as pk
    s = synth.make_system(128, synth.config_seed(1))
    return s, pk.Matrix.from_system(ctx, s), oracle.to_csr(s, "A").dense(), oracle.to_csr(s, "B").dense()


def check_column(out, c, r, rows_local=None, rho_slice=None, dense_rho_col=None):
    n = r["eps"].size
    assert out["dim"][c] == n
    np.testing.assert_allclose(out["eps"][c, :n], r["eps"], atol=TOL)
    assert np.all(out["eps"][c, n:] == 0.0) and np.all(out["w_B"][c, n:] == 0.0)
    e = out["eps"][c, :n]
    for w in ("I", "B", "A"):
        g = out["w_" + w][c, :n]
        for f in (np.ones_like, lambda x: x, fermi):
            assert abs(np.sum(f(e) * g) - np.sum(f(r["eps"]) * r["w" + w])) < TOL
    assert abs(out["col_traces"][c, 0] - ma.projected_trace(r, fermi, "B")) < TOL
    assert abs(out["col_traces"][c, 1] - ma.projected_trace(r, fermi, "A")) < TOL
    if rho_slice is not None:
        col = ma.density_column(r, fermi)
        np.testing.assert_allclose(rho_slice, np.where(rows_local >= 0, col[np.maximum(rows_local, 0)], 0.0),
                                   atol=TOL)


@pytest.mark.parametrize("nu,slots", [(30, 64), (2, 64), (48, 128), (12, 0)])
def test_global_matches_oracle(ctx, c1, nu, slots):
    import paper_1609_08377_amd as pk
    s, mat, A, B = c1
    cols = np.arange(s.orb_off[-1], dtype=np.int32) if nu == 30 else np.arange(0, 257, 3, dtype=np.int32)
    out = pk.arnoldi(ctx, mat, cols, nu=nu, mu=MU, kT=KT, want_rho=True, slots=slots)
    off, rows = pk.pattern(mat, cols)
    for c, j in enumerate(cols):
        r = ma.column(A, B, int(j), nu)
        check_column(out, c, r, rows[off[c]:off[c + 1]], out["rho"][off[c]:off[c + 1]])


@pytest.mark.parametrize("nu", [4, 30])
def test_conservation_laws(ctx, c1, nu):
    """Closed forms from the dense inverse, independent of the oracle: with
    B^{-1} e_j in the subspace the zeroth and first moments are exact."""
    import paper_1609_08377_amd as pk
    s, mat, A, B = c1
    Binv = np.linalg.inv(B)
    cols = np.arange(0, 257, 5, dtype=np.int32)
    out = pk.arnoldi(ctx, mat, cols, nu=nu)
    for c, j in enumerate(cols):
        e, wI, wB, wA = out["eps"][c], out["w_I"][c], out["w_B"][c], out["w_A"][c]
        assert abs(wB.sum() - 1.0) < 1e-11
        assert abs(wI.sum() - Binv[j, j]) < 1e-11
        assert abs(wA.sum() - (Binv @ A)[j, j]) < 1e-11
        assert abs((e * wB).sum() - (Binv @ A)[j, j]) < 1e-11
        assert abs((e * wI).sum() - (Binv @ A @ Binv)[j, j]) < 1e-11


def kappa_radii(sysm, centres, kappa):
    """Radius of each centre's region holding its kappa nearest atoms (minimum image)."""
    out = []
    for c in centres:
        d = sysm.pos - sysm.pos[c]
        d -= sysm.L * np.rint(d / sysm.L)
        r = np.sort(np.sqrt((d * d).sum(1)))
        out.append(0.5 * (r[kappa - 1] + r[kappa]))
    return np.asarray(out)


@pytest.mark.parametrize("kappa,tile", [(100, 64), (60, 128)])
def test_regions_match_oracle(ctx, kappa, tile):
    import paper_1609_08377_amd as pk
    s = synth.make_system(1024, synth.config_seed(2))
    mat = pk.Matrix.from_system(ctx, s)
    centres = synth.sample_columns(s, 40, 77) % s.n_atoms
    centres = np.unique(centres)[:24].astype(np.int32)
    radii = kappa_radii(s, centres, kappa)
    reg = pk.Regions(ctx, mat, centres, radii, tile_width=tile)
    out = pk.region_arnoldi(ctx, reg, nu=30, mu=MU, kT=KT, want_rho=True)
    c = 0
    for ci, cen in enumerate(centres):
        atoms = oracle.region_atoms(s, int(cen), float(radii[ci]))
        assert atoms.size == kappa
        for q in range(int(s.n_orb[cen])):
            j = int(s.orb_off[cen]) + q
            assert reg.cols[c] == j
            r, omap = ma.region_column(s, atoms, j, 30)
            # pattern rows of column j as local region indices (-1 outside the region)
            p0, p1 = int(reg.pat_off[c]), int(reg.pat_off[c + 1])
            g2l = -np.ones(int(s.orb_off[-1]), dtype=np.int64)
            g2l[omap] = np.arange(omap.size)
            B = oracle.to_csr(s, "B")
            grows = B.ci[B.rp[j]:B.rp[j + 1]]
            assert grows.size == p1 - p0
            check_column(out, c, r, g2l[grows], out["rho"][p0:p1])
            c += 1
    assert c == reg.n_cols


def test_regions_smaller_than_subspace_are_exact(ctx):
    """Regions of 3-16 orbitals with nu = 30: both sequences exhaust and the sums
    equal the dense spectral result of each region's sub-pencil."""
    import paper_1609_08377_amd as pk
    s = synth.make_system(128, synth.config_seed(1))
    mat = pk.Matrix.from_system(ctx, s)
    centres = np.arange(0, 40, dtype=np.int32)
    radii = np.full(centres.size, 2.3)
    reg = pk.Regions(ctx, mat, centres, radii, tile_width=64)
    out = pk.region_arnoldi(ctx, reg, nu=30, mu=MU, kT=KT, want_rho=True)
    c = 0
    for cen in centres:
        atoms = oracle.region_atoms(s, int(cen), 2.3)
        Ar, Br, omap = oracle.carve_region(s, atoms)
        Ad, Bd = Ar.dense(), Br.dense()
        lam, _ = dense.gen_eig(Ad, Bd)
        rho = dense.exact_rho(Ad, Bd, MU, KT)
        m = Ad.shape[0]
        for q in range(int(s.n_orb[cen])):
            j = int(s.orb_off[cen]) + q
            jl = int(np.nonzero(omap == j)[0][0])
            assert out["dim"][c] == m
            np.testing.assert_allclose(out["eps"][c, :m], lam, atol=1e-10)
            assert abs(out["col_traces"][c, 0] - (rho @ Bd)[jl, jl]) < 1e-10
            assert abs(out["col_traces"][c, 1] - (rho @ Ad)[jl, jl]) < 1e-10
            c += 1


def test_bad_arguments(ctx, c1):
    import paper_1609_08377_amd as pk
    s, mat, A, B = c1
    for nu in (0, 3, 50):
        with pytest.raises(pk.ElsesError):
            pk.arnoldi(ctx, mat, [0, 1], nu=nu)
    with pytest.raises(pk.ElsesError):
        pk.arnoldi(ctx, mat, [0, 0], nu=4)
    with pytest.raises(pk.ElsesError):
        pk.arnoldi(ctx, mat, [0], nu=4, kT=-1.0)
    out = pk.arnoldi(ctx, mat, np.zeros(0, dtype=np.int32), nu=4)
    assert out["eps"].shape == (0, 4)
