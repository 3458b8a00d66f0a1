"""The ordered (diamond) input on the GPU: parity with the oracle, and equal
work for the equivalent subproblems that make the ordered case balanced."""
import numpy as np
import pytest

import oracle
import synth
from oracle import arnoldi as ma
from oracle import dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1609_08377_amd as pk
    return pk.Context(0)


def test_diamond_global_density_matches_oracle(ctx):
    import paper_1609_08377_amd as pk
    s = synth.make_diamond(2, 2001)
    mat = pk.Matrix.from_system(ctx, s)
    A, B = oracle.to_csr(s, "A"), oracle.to_csr(s, "B")
    z = synth.shift_grid(16)
    c = oracle.fermi_weights(z, 0.2, 0.05)
    cols = np.arange(s.M, dtype=np.int32)
    out = pk.density_matrix(ctx, mat, cols, z, c, tol=1e-10)
    r = oracle.shifted_solve(A, B, cols, z, tol=1e-10, full=False, true_residual=False)
    pat_off = oracle.pattern_offsets(B, cols)
    rho_o, trB_o, trA_o = oracle.density_from_x(B, A, cols, r.x, pat_off, c)
    np.testing.assert_allclose(out["rho"].cpu().numpy(), rho_o, atol=1e-8)
    ct = out["col_traces"].cpu().numpy()
    np.testing.assert_allclose(ct[:, 0], trB_o, atol=1e-8)
    np.testing.assert_allclose(ct[:, 1], trA_o, atol=1e-8)
    # equivalent columns share their residual history; near the residual floor
    # (tol 1e-10) rounding moves the crossing by up to two of ~45 iterations
    it = out["iters"].cpu().numpy().reshape(-1, 4)
    assert np.all(it.max(0) - it.min(0) <= 2)


def test_diamond_regions_are_equivalent(ctx):
    """kappa-atom regions of the crystal: the same region around every atom.

    The shifted Lanczos solves of equivalent columns differ only through
    rounding, which the loss of orthogonality amplifies into a spread of a few
    iterations.  For multiple Arnoldi the crystal's point-group symmetry keeps
    both Krylov sequences of a centre orbital inside the symmetric sector;
    rounding seeds components outside it, which the block process grows into
    further directions once the sector is used up.  Those Ritz pairs carry
    essentially no weight on e_j, so the Eq. 18 sums of equivalent columns
    agree (and match the oracle and the exact density matrix) while individual
    Ritz values need not."""
    import paper_1609_08377_amd as pk
    s = synth.make_diamond(4, 2001)
    mat = pk.Matrix.from_system(ctx, s)
    centres = np.arange(0, 48, dtype=np.int32)
    radii = synth.kappa_radii(s, centres, 40)
    assert np.ptp(radii) < 1e-9
    reg = pk.Regions(ctx, mat, centres, radii, tile_width=64)
    z = synth.shift_grid(16)
    out = pk.region_solve(ctx, reg, z, tol=1e-8)
    it = out["iters"].cpu().numpy().reshape(-1, 4)
    assert np.all(it.max(0) - it.min(0) <= 0.2 * it.mean(0))
    mo = pk.region_arnoldi(ctx, reg, nu=30, mu=0.2, kT=0.05)
    f = lambda e: dense.fermi(e, 0.2, 0.05)
    tr = mo["col_traces"].reshape(-1, 4, 2)
    assert np.abs(tr - tr[0][None]).max() < 1e-7
    sI = (f(mo["eps"]) * mo["w_I"]).sum(1).reshape(-1, 4)
    assert np.abs(sI - sI[0][None]).max() < 1e-7
    atoms = oracle.region_atoms(s, 0, float(radii[0]))
    Ar, Br, omap = oracle.carve_region(s, atoms)
    rho = dense.exact_rho(Ar.dense(), Br.dense(), 0.2, 0.05)
    for q in range(4):
        r, _ = ma.region_column(s, atoms, q, 30)
        assert abs(mo["col_traces"][q, 0] - ma.projected_trace(r, f, "B")) < 1e-7
        assert abs(mo["col_traces"][q, 1] - ma.projected_trace(r, f, "A")) < 1e-7
        jl = int(np.nonzero(omap == q)[0][0])
        assert abs(sI[0, q] - rho[jl, jl]) < 1e-6
