"""Pins of the CPU oracle against what the mathematics fixes (no GPU).

Every check here is independent of the oracle's own recurrences: dense LU
solves (definition of G, Eq. 10), the spectral sum (Eq. 11), closed forms for
diagonal and 2x2 pencils, the symmetry of G, finite termination, and the
closed-form traces of the discretised energy integral (Eqs. 4, 7, 12).
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import dense


def csr_from_dense(D, pattern=None):
    n = D.shape[0]
    mask = (D != 0) if pattern is None else pattern
    rp = np.zeros(n + 1, dtype=np.int64)
    ci, v = [], []
    for i in range(n):
        js = np.nonzero(mask[i])[0]
        ci.extend(js.tolist())
        v.extend(D[i, js].tolist())
        rp[i + 1] = len(ci)
    return oracle.CSR(n, rp, np.asarray(ci, np.int32), np.asarray(v, np.float64))


def assemble_dense(sysm, vals):
    """The test's own dense assembly from the atom blocks."""
    M = sysm.M
    D = np.zeros((M, M))
    for I in range(sysm.n_atoms):
        for b in range(sysm.blk_row_ptr[I], sysm.blk_row_ptr[I + 1]):
            J = sysm.blk_col[b]
            ni, nj = sysm.n_orb[I], sysm.n_orb[J]
            blk = vals[sysm.val_ptr[b]:sysm.val_ptr[b + 1]].reshape(ni, nj)
            D[sysm.orb_off[I]:sysm.orb_off[I] + ni, sysm.orb_off[J]:sysm.orb_off[J] + nj] = blk
    return D


@pytest.fixture(scope="module")
def small_system():
    # 64 atoms, 3.5 A cutoff (the 4 A cutoff needs a box of side > 8 A): M = 127
    return synth.make_system(64, 2024, r_cut=3.5)


def test_generator_shapes(c1_system):
    s = c1_system
    assert s.n_c == 43 and s.n_atoms - s.n_c == 85
    assert s.M == 4 * 43 + 85 == 257
    assert abs(s.L - 10.0) < 1e-3
    assert int((s.n_orb == 4).sum()) == 43 and int((s.n_orb == 1).sum()) == 85
    assert np.array_equal(np.diff(s.orb_off), s.n_orb)
    # minimum pair distance and cutoff
    pi, pj, pr, pd = s.extra["pairs"]
    assert pr.min() >= 1.0 and pr.max() <= 4.0
    assert np.allclose(np.linalg.norm(pd, axis=1), pr)


def test_csr_matches_blocks(c1_system, c1_csr):
    A, B = c1_csr
    Ad, Bd = assemble_dense(c1_system, c1_system.A_val), assemble_dense(c1_system, c1_system.B_val)
    assert np.array_equal(A.dense(), Ad)
    assert np.array_equal(B.dense(), Bd)
    assert np.array_equal(Ad, Ad.T) and np.array_equal(Bd, Bd.T)
    assert np.all(np.diag(Bd) == 1.0)
    lam = np.linalg.eigvalsh(Bd)
    assert lam[0] > 0.5  # SPD with margin
    # the CSR pattern is the atom-block pattern for A and B alike
    assert np.array_equal(A.rp, B.rp) and np.array_equal(A.ci, B.ci)


def test_csr_matvec(c1_csr):
    A, _ = c1_csr
    x = np.random.default_rng(0).standard_normal(A.n)
    assert np.allclose(A.matvec(x), A.dense() @ x, rtol=0, atol=1e-13)
    # strided column views are copied; the copy must outlive the C call
    X = np.random.default_rng(1).standard_normal((A.n, 3))
    for v in range(3):
        assert np.allclose(A.matvec(X[:, v]), A.dense() @ X[:, v], rtol=0, atol=1e-13)


def test_cg_B(c1_csr):
    _, B = c1_csr
    s = np.random.default_rng(1).standard_normal(B.n)
    x, it = oracle.cg_B(B, s, tol=1e-13)
    assert 0 < it < 100
    ref = np.linalg.solve(B.dense(), s)
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_solve_matches_dense_lu(c1_system, c1_csr):
    A, B = c1_csr
    Ad, Bd = A.dense(), B.dense()
    z = synth.shift_grid(32)
    cols = np.array([0, 1, 5, 100, 171, 172, 200, 256], dtype=np.int32)  # C and H orbitals
    r = oracle.shifted_solve(A, B, cols, z, tol=1e-11, full=True)
    assert r.inner_failures == 0
    assert np.all(r.conv_it > 0)
    for c, j in enumerate(cols):
        e = np.zeros(A.n)
        e[j] = 1.0
        for k in range(len(z)):
            ref = np.linalg.solve(z[k] * Bd - Ad, e)
            err = np.linalg.norm(r.x[c, k] - ref) / np.linalg.norm(ref)
            assert err < 2e-10, (j, k, err)
            assert r.true_res[c, k] <= 1.05e-11


def test_default_tolerance_certificate(c1_csr):
    """At tol 1e-8: true residual <= tol and ||dx|| <= ||r|| / (Im z * lambda_min(B))."""
    A, B = c1_csr
    Ad, Bd = A.dense(), B.dense()
    lmin = np.linalg.eigvalsh(Bd)[0]
    z = synth.shift_grid(32)
    cols = np.array([3, 180], dtype=np.int32)
    r = oracle.shifted_solve(A, B, cols, z, tol=1e-8, full=True)
    assert np.all(r.true_res <= 1.0001e-8)
    # the recursive estimate tracks the true residual
    assert np.all(np.abs(r.est - r.true_res) <= 1e-3 * 1e-8 + 1e-3 * r.true_res)
    for c, j in enumerate(cols):
        e = np.zeros(A.n)
        e[j] = 1.0
        for k in range(len(z)):
            ref = np.linalg.solve(z[k] * Bd - Ad, e)
            assert np.linalg.norm(r.x[c, k] - ref) <= r.true_res[c, k] / (z[k].imag * lmin) * 1.001


def test_green_symmetry(c1_csr):
    """G(z)^T = G(z) for real symmetric A, B: x_{j}[i] = x_{i}[j]."""
    A, B = c1_csr
    z = synth.shift_grid(8)
    cols = np.array([2, 9, 60, 175, 230], dtype=np.int32)
    r = oracle.shifted_solve(A, B, cols, z, tol=1e-11, full=True)
    for a, i in enumerate(cols):
        for b, j in enumerate(cols):
            for k in range(len(z)):
                gij, gji = r.x[b, k, i], r.x[a, k, j]
                assert abs(gij - gji) <= 1e-9 * np.abs(r.x[b, k]).max()


def test_diagonal_pencil_closed_form():
    rng = np.random.default_rng(5)
    n = 12
    a = rng.uniform(-2, 2, n)
    bdiag = rng.uniform(0.5, 2.0, n)
    A = csr_from_dense(np.diag(a))
    B = csr_from_dense(np.diag(bdiag))
    z = synth.shift_grid(6, eta=0.05)
    cols = np.arange(n, dtype=np.int32)
    r = oracle.shifted_solve(A, B, cols, z, tol=1e-12, full=True)
    assert np.all(r.iters == 1)
    for j in range(n):
        for k in range(len(z)):
            ref = np.zeros(n, complex)
            ref[j] = 1.0 / (z[k] * bdiag[j] - a[j])
            assert np.allclose(r.x[j, k], ref, rtol=0, atol=1e-14 * abs(ref[j]))


def test_two_by_two_closed_form():
    a, b, d, e = 0.3, -0.7, 1.1, 0.2
    A = csr_from_dense(np.array([[a, b], [b, d]]))
    B = csr_from_dense(np.array([[1.0, e], [e, 1.0]]))
    z = np.array([0.25 + 0.03j, -0.8 + 0.01j, 2.0 + 0.5j])
    r = oracle.shifted_solve(A, B, np.array([0, 1], np.int32), z, tol=1e-13, full=True)
    for k, zk in enumerate(z):
        det = (zk - a) * (zk - d) - (zk * e - b) ** 2
        col0 = np.array([zk - d, -(zk * e - b)]) / det
        col1 = np.array([-(zk * e - b), zk - a]) / det
        assert np.allclose(r.x[0, k], col0, rtol=1e-12, atol=0)
        assert np.allclose(r.x[1, k], col1, rtol=1e-12, atol=0)
        assert r.iters[0] <= 3


def test_identity_overlap_is_plain_shifted_case():
    """B = I: (zI - A) x = e_j (paper Sec. III-A)."""
    rng = np.random.default_rng(7)
    n = 40
    R = rng.standard_normal((n, n)) * (rng.uniform(size=(n, n)) < 0.15)
    Ad = 0.5 * (R + R.T) + np.diag(rng.uniform(-1, 1, n))
    A = csr_from_dense(Ad)
    B = csr_from_dense(np.eye(n))
    z = synth.shift_grid(10, lo=-2, hi=2, eta=0.02)
    cols = np.array([0, 17, 39], np.int32)
    r = oracle.shifted_solve(A, B, cols, z, tol=1e-12, full=True)
    for c, j in enumerate(cols):
        for k in range(len(z)):
            ref = np.linalg.solve(z[k] * np.eye(n) - Ad, np.eye(n)[:, j])
            assert np.linalg.norm(r.x[c, k] - ref) <= 1e-10 * np.linalg.norm(ref)


def test_finite_termination_tiny():
    """Krylov dimension cannot exceed M: convergence within ~M steps."""
    rng = np.random.default_rng(11)
    n = 8
    R = rng.standard_normal((n, n))
    Ad = 0.5 * (R + R.T)
    Q = rng.standard_normal((n, n))
    Bd = np.eye(n) + 0.05 * (Q @ Q.T)
    A, B = csr_from_dense(Ad, np.ones((n, n), bool)), csr_from_dense(Bd, np.ones((n, n), bool))
    z = synth.shift_grid(5, lo=-1.5, hi=1.5, eta=0.1)
    cols = np.arange(n, dtype=np.int32)
    r = oracle.shifted_solve(A, B, cols, z, tol=1e-12, full=True)
    assert np.all(r.iters <= n + 2)
    G = [dense.dense_G(Ad, Bd, zk) for zk in z]
    for j in range(n):
        for k in range(len(z)):
            assert np.linalg.norm(r.x[j, k] - G[k][:, j]) <= 1e-9 * np.linalg.norm(G[k][:, j])


def test_spectral_sum_equals_inverse(c1_csr):
    """Eq. 11: G(z) = sum_k y_k y_k^T / (z - lambda_k) with B-orthonormal y (dense helpers)."""
    A, B = c1_csr
    Ad, Bd = A.dense(), B.dense()
    eig = dense.gen_eig(Ad, Bd)
    lam, Y = eig
    assert np.allclose(Y.T @ Bd @ Y, np.eye(A.n), atol=1e-12)
    for zk in (0.1 + 0.01j, -0.9 + 0.01j):
        G1 = dense.dense_G(Ad, Bd, zk)
        G2 = dense.spectral_G(Ad, Bd, zk, eig)
        assert np.abs(G1 - G2).max() <= 1e-11 * np.abs(G1).max()
        assert np.abs(G1 - G1.T).max() <= 1e-11 * np.abs(G1).max()


def test_pattern_output_matches_full(c1_csr):
    A, B = c1_csr
    z = synth.shift_grid(4)
    cols = np.array([0, 7, 190], np.int32)
    rf = oracle.shifted_solve(A, B, cols, z, tol=1e-10, full=True)
    rp = oracle.shifted_solve(A, B, cols, z, tol=1e-10, full=False)
    K = len(z)
    for c, j in enumerate(cols):
        pat = B.ci[B.rp[j]:B.rp[j + 1]]
        blk = rp.x[rp.pat_off[c] * K:rp.pat_off[c + 1] * K].reshape(K, -1)
        assert np.array_equal(blk, rf.x[c][:, pat])


@pytest.fixture(scope="module")
def small_all_columns(small_system):
    A, B = oracle.to_csr(small_system, "A"), oracle.to_csr(small_system, "B")
    z = synth.shift_grid(16, lo=-1.0, hi=1.0, eta=0.05)
    cols = np.arange(A.n, dtype=np.int32)
    r = oracle.shifted_solve(A, B, cols, z, tol=1e-11, full=False)
    return A, B, z, cols, r


def test_traces_closed_form(small_all_columns):
    """Tr[rho B] = sum_n g(lambda_n), Tr[rho A] = sum_n g(lambda_n) lambda_n (Eqs. 4, 7, 11, 12)."""
    A, B, z, cols, r = small_all_columns
    c = oracle.fermi_weights(z, mu=0.2, tau=0.1)
    rho, trB, trA = oracle.density_from_x(B, A, cols, r.x, r.pat_off, c)
    refB, refA = dense.trace_closed_forms(A.dense(), B.dense(), z, c)
    assert abs(trB.sum() - refB) <= 1e-9 * abs(refB)
    assert abs(trA.sum() - refA) <= 1e-9 * max(1.0, abs(refA))
    # rho is symmetric on the pattern: rho_ij from column j equals rho_ji from column i
    Rd = np.zeros((A.n, A.n))
    for ci_, j in enumerate(cols):
        Rd[B.ci[B.rp[j]:B.rp[j + 1]], j] = rho[r.pat_off[ci_]:r.pat_off[ci_ + 1]]
    assert np.abs(Rd - Rd.T).max() <= 1e-9 * np.abs(Rd).max()


def test_energy_integral_reproduces_fermi_occupation(small_system):
    """Eq. 12 with a fine shift grid over the whole spectrum approaches Eq. 6 (sign and 1/pi of c_k)."""
    A, B = oracle.to_csr(small_system, "A"), oracle.to_csr(small_system, "B")
    Ad, Bd = A.dense(), B.dense()
    lam, Y = dense.gen_eig(Ad, Bd)
    mu, tau = float(np.median(lam)), 0.2
    z = synth.shift_grid(6000, lo=lam.min() - 4.0, hi=lam.max() + 4.0, eta=0.01)
    c = oracle.fermi_weights(z, mu, tau)
    # occupation of each eigenstate from the quadrature: g(lambda) = sum_k Im(c_k / (z_k - lambda))
    g = np.imag(c[None, :] / (z[None, :] - lam[:, None])).sum(axis=1)
    f = dense.fermi(lam, mu, tau)
    assert np.max(np.abs(g - f)) < 0.02
    assert abs(g.sum() - f.sum()) < 0.01 * f.sum()


def test_exact_rho_electron_count(small_system):
    """Eq. 6 at the chemical potential reproducing N_e (Sec. II-B): 2 Tr[rho B] = N_e."""
    A, B = oracle.to_csr(small_system, "A"), oracle.to_csr(small_system, "B")
    Ad, Bd = A.dense(), B.dense()
    eig = dense.gen_eig(Ad, Bd)
    n_e = 4 * small_system.n_c + (small_system.n_atoms - small_system.n_c)
    tau = 0.01
    mu = dense.chemical_potential(eig[0], n_e, tau)
    rho = dense.exact_rho(Ad, Bd, mu, tau, eig)
    assert abs(2.0 * np.trace(rho @ Bd) - n_e) < 1e-8
    # and the electronic energy (Eq. 4)
    assert abs(np.trace(rho @ Ad) - (dense.fermi(eig[0], mu, tau) * eig[0]).sum()) < 1e-9


def test_region_whole_box_is_global(c1_system, c1_csr):
    A, B = c1_csr
    atoms = oracle.region_atoms(c1_system, 5, radius=1e3)
    assert atoms.size == c1_system.n_atoms
    Ar, Br, omap = oracle.carve_region(c1_system, atoms)
    assert np.array_equal(omap, np.arange(A.n))
    assert np.array_equal(Ar.rp, A.rp) and np.array_equal(Ar.ci, A.ci) and np.array_equal(Ar.v, A.v)
    assert np.array_equal(Br.v, B.v)


def test_region_small_vs_dense(c1_system, c1_csr):
    A, B = c1_csr
    centre = int(np.nonzero(c1_system.n_orb == 4)[0][3])  # a carbon atom: 4 columns
    atoms = oracle.region_atoms(c1_system, centre, radius=4.5)
    Ar, Br, omap = oracle.carve_region(c1_system, atoms)
    # the test's own principal submatrix of the global dense matrices
    Ad = A.dense()[np.ix_(omap, omap)]
    Bd = B.dense()[np.ix_(omap, omap)]
    assert np.array_equal(Ar.dense(), Ad) and np.array_equal(Br.dense(), Bd)
    loc = np.nonzero(np.isin(omap, np.arange(c1_system.orb_off[centre], c1_system.orb_off[centre + 1])))[0]
    assert loc.size == 4
    z = synth.shift_grid(8)
    r = oracle.shifted_solve(Ar, Br, loc.astype(np.int32), z, tol=1e-11, full=True)
    for c, j in enumerate(loc):
        for k in range(len(z)):
            ref = np.linalg.solve(z[k] * Bd - Ad, np.eye(Ar.n)[:, j])
            assert np.linalg.norm(r.x[c, k] - ref) <= 1e-9 * np.linalg.norm(ref)
