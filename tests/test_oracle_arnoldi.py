"""Pins of the multiple Arnoldi oracle (Eqs. 15-18) against closed forms.

Every check here is fixed by linear algebra, not by the oracle itself:
  * nu >= M: the subspace is the whole space, so Eq. 18 and Eq. 17 reproduce the
    dense generalised eigendecomposition exactly (the paper states the sum
    becomes exact when nu reaches the matrix dimension);
  * B^{-1} e_j lies in the subspace, so at ANY nu the f = 1 column is exactly
    B^{-1} e_j and the zeroth and first moments of Eq. 18 are exact
    (the conservation laws the second Krylov term is there for);
  * B = I: both sequences coincide and the sum is Gauss quadrature with nu/2
    nodes, exact for polynomials of degree <= nu - 1 (Golub-Meurant);
  * the Ritz data depend on the span only: a basis built another way (QR of
    the explicit power sequences) gives the same result.
"""
import numpy as np
import pytest

import oracle
from oracle import arnoldi as ma
from oracle import dense


def pencil(M, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    X = rng.standard_normal((M, M))
    A = 0.5 * (X + X.T) / np.sqrt(M)
    Y = rng.standard_normal((M, M))
    B = np.eye(M) + 0.15 * (Y + Y.T) / np.sqrt(M)
    assert np.linalg.eigvalsh(B).min() > 0.3
    return A, B


def fermi(mu, tau):
    return lambda e: dense.fermi(e, mu, tau)


@pytest.mark.parametrize("M,seed", [(10, 1), (12, 2), (16, 3)])
def test_full_space_is_exact(M, seed):
    A, B = pencil(M, seed)
    lam, Yd = dense.gen_eig(A, B)
    f = fermi(0.1, 0.05)
    rho = dense.exact_rho(A, B, 0.1, 0.05)
    for j in range(M):
        r = ma.column(A, B, j, M)
        assert r["eps"].size == M
        np.testing.assert_allclose(r["eps"], lam, atol=1e-12)
        np.testing.assert_allclose(ma.density_column(r, f), rho[:, j], atol=1e-12)
        for X, w in ((np.eye(M), "I"), (B, "B"), (A, "A")):
            assert abs(ma.projected_trace(r, f, w) - (rho @ X)[j, j]) < 1e-12
        z = 0.3 + 0.02j
        np.testing.assert_allclose(ma.green_column(r, z), dense.dense_G(A, B, z)[:, j], atol=1e-10)


@pytest.mark.parametrize("nu", [2, 4, 6, 30])
def test_conservation_laws_any_nu(nu):
    A, B = pencil(60, 7)
    Binv = np.linalg.inv(B)
    one = lambda e: np.ones_like(e)
    ident = lambda e: e
    for j in (0, 17, 59):
        r = ma.column(A, B, j, nu)
        assert r["eps"].size == nu
        np.testing.assert_allclose(ma.density_column(r, one), Binv[:, j], atol=1e-12)
        assert abs(ma.projected_trace(r, one, "B") - 1.0) < 1e-12
        assert abs(ma.projected_trace(r, one, "I") - Binv[j, j]) < 1e-12
        assert abs(ma.projected_trace(r, one, "A") - (Binv @ A)[j, j]) < 1e-12
        assert abs(ma.projected_trace(r, ident, "B") - (Binv @ A)[j, j]) < 1e-12
        assert abs(ma.projected_trace(r, ident, "I") - (Binv @ A @ Binv)[j, j]) < 1e-12


def test_second_sequence_is_what_conserves():
    """Without K(A; B^{-1} e_j) the f = 1 column is no longer B^{-1} e_j (a dropped
    term fails).  The X = B trace stays 1 either way: e_j alone conserves it."""
    A, B = pencil(60, 7)
    Binv = np.linalg.inv(B)
    one = lambda e: np.ones_like(e)
    Q = ma.krylov_chain(A, np.eye(60)[:, 5], 6)
    r = ma.column(A, B, 5, 6, Q=Q)
    assert np.abs(ma.density_column(r, one) - Binv[:, 5]).max() > 1e-3
    assert abs(ma.projected_trace(r, one, "I") - Binv[5, 5]) > 1e-4
    assert abs(ma.projected_trace(r, one, "B") - 1.0) < 1e-12


@pytest.mark.parametrize("nu", [4, 8, 12])
def test_identity_overlap_is_gauss_quadrature(nu):
    A, _ = pencil(50, 11)
    B = np.eye(50)
    j = 3
    r = ma.column(A, B, j, nu)
    assert r["eps"].size == nu // 2  # the two sequences coincide
    Ak = np.eye(50)
    for k in range(nu + 1):
        q = float(np.sum(r["eps"] ** k * r["wI"]))
        if k <= nu - 1:
            assert abs(q - Ak[j, j]) < 1e-11 * max(1.0, abs(Ak[j, j]))
        else:
            assert abs(q - Ak[j, j]) > 1e-8  # degree nu is no longer exact
        Ak = Ak @ A


def test_basis_independence():
    A, B = pencil(40, 5)
    j, nu = 9, 6
    e = np.eye(40)[:, j]
    u = np.linalg.solve(B, e)
    P = np.stack([e, A @ e, A @ A @ e, u, A @ u, A @ A @ u], axis=1)
    Qm, _ = np.linalg.qr(P)
    r1 = ma.column(A, B, j, nu)
    r2 = ma.column(A, B, j, nu, Q=Qm)
    np.testing.assert_allclose(r1["eps"], r2["eps"], atol=1e-10)
    f = fermi(0.0, 0.1)
    np.testing.assert_allclose(ma.density_column(r1, f), ma.density_column(r2, f), atol=1e-10)
    for w in ("I", "B", "A"):
        np.testing.assert_allclose(r1["w" + w], r2["w" + w], atol=1e-10)


def test_block_construction_spans_the_two_krylov_spaces():
    """The vector-by-vector block construction spans the same space as the union of
    the two Krylov sequences built separately (orthonormalised by an SVD) when the
    union is well conditioned."""
    A, B = pencil(80, 13)
    for j, nu in ((4, 6), (30, 10)):
        e = np.eye(80)[:, j]
        u = np.linalg.solve(B, e)
        P = np.concatenate([ma.krylov_chain(A, e, nu // 2), ma.krylov_chain(A, u, nu // 2)], axis=1)
        U, sv, _ = np.linalg.svd(P, full_matrices=False)
        assert sv[-1] > 1e-6
        Q = ma.subspace(A, B, j, nu)
        assert Q.shape[1] == nu
        np.testing.assert_allclose(Q.T @ Q, np.eye(nu), atol=1e-13)
        # same span: the projector difference vanishes
        assert np.abs(Q @ Q.T - U @ U.T).max() < 1e-9


@pytest.mark.parametrize("centre,radius", [(0, 2.5), (1, 2.5), (2, 2.0)])
def test_exhausted_sequences_small_region(c1_system, centre, radius):
    """A region smaller than nu: both sequences exhaust, the result is the dense one."""
    sysm = c1_system
    atoms = oracle.region_atoms(sysm, centre, radius)
    Ar, Br, omap = oracle.carve_region(sysm, atoms)
    Ad, Bd = Ar.dense(), Br.dense()
    m = Ad.shape[0]
    assert 2 <= m < 30
    rho = dense.exact_rho(Ad, Bd, 0.0, 0.05)
    f = fermi(0.0, 0.05)
    for jl in range(m):
        r = ma.column(Ad, Bd, jl, 30)
        assert r["eps"].size == m
        np.testing.assert_allclose(ma.density_column(r, f), rho[:, jl], atol=1e-12)


def test_region_as_whole_system_equals_global(c1_csr, c1_system):
    A, B = (x.dense() for x in c1_csr)
    sysm = c1_system
    j = int(sysm.orb_off[5])
    r_g = ma.column(A, B, j, 30)
    r_r, omap = ma.region_column(sysm, np.arange(sysm.n_atoms), j, 30)
    assert np.array_equal(omap, np.arange(A.shape[0]))
    np.testing.assert_allclose(r_g["eps"], r_r["eps"], atol=1e-12)
    f = fermi(0.2, 0.1)
    np.testing.assert_allclose(ma.density_column(r_g, f), ma.density_column(r_r, f), atol=1e-12)


def test_converges_to_dense_as_nu_grows(c1_csr):
    A, B = (x.dense() for x in c1_csr)
    rho = dense.exact_rho(A, B, 0.2, 0.1)
    f = fermi(0.2, 0.1)
    j = 40
    # At large nu the two power sequences become numerically dependent (both
    # resolve the same eigenvectors), so the error levels off near 1e-3 instead
    # of reaching zero at nu = M; exactness at nu = M is pinned on small pencils.
    errs = [np.abs(ma.density_column(ma.column(A, B, j, nu), f) - rho[:, j]).max() for nu in (10, 30, 60)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 2e-3
