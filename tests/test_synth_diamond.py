"""Pins of the ordered (diamond) input: geometry, symmetry, and the equivalence
of every atom's subproblem that the ordered-versus-disordered comparison rests
on (the paper's ideal diamond crystal, whose subproblems are all equivalent)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import dense


@pytest.fixture(scope="module")
def d2():
    return synth.make_diamond(2, 2001)


def test_geometry(d2):
    s = d2
    assert s.n_atoms == 64 and s.M == 256 and np.all(s.n_orb == 4)
    a = synth.DIAMOND_A
    pi, pj, pr, _ = s.extra["pairs"]
    deg = np.bincount(np.concatenate([pi, pj]), minlength=s.n_atoms)
    assert np.all(deg == 16)
    r_nn, r_2 = a * np.sqrt(3.0) / 4.0, a / np.sqrt(2.0)
    assert np.all((np.abs(pr - r_nn) < 1e-9) | (np.abs(pr - r_2) < 1e-9))
    assert np.sum(np.abs(pr - r_nn) < 1e-9) == 2 * s.n_atoms  # 4 per atom, each pair once
    assert np.all(np.diff(s.blk_row_ptr) == 17)


def test_symmetric_spd(d2):
    A, B = oracle.to_csr(d2, "A").dense(), oracle.to_csr(d2, "B").dense()
    assert np.array_equal(A, A.T) and np.array_equal(B, B.T)
    assert np.linalg.eigvalsh(B)[0] > 0.5


def _translation_perm(s, shift):
    """Atom permutation of a lattice translation (minimum image)."""
    L = s.L
    p = np.mod(s.pos + shift, L)
    q = np.mod(s.pos, L)
    d = p[:, None, :] - q[None, :, :]
    d -= L * np.rint(d / L)
    perm = np.argmin((d * d).sum(-1), axis=1)
    assert np.sort(perm).tolist() == list(range(s.n_atoms))
    return perm


@pytest.mark.parametrize("shift", [(0.5, 0.5, 0.0), (0.25, 0.25, 0.25), (1.0, 0.0, 0.0)])
def test_translations_and_inversion_map_the_pencil_onto_itself(d2, shift):
    s = d2
    A, B = oracle.to_csr(s, "A").dense(), oracle.to_csr(s, "B").dense()
    if shift == (0.25, 0.25, 0.25):
        # inversion through a bond centre maps one sublattice onto the other
        c = 0.125 * synth.DIAMOND_A
        L = s.L
        p = np.mod(2 * c - s.pos, L)
        d = p[:, None, :] - np.mod(s.pos, L)[None, :, :]
        d -= L * np.rint(d / L)
        perm = np.argmin((d * d).sum(-1), axis=1)
        assert np.sort(perm).tolist() == list(range(s.n_atoms))
    else:
        perm = _translation_perm(s, np.asarray(shift) * synth.DIAMOND_A)
    op = (perm[:, None] * 4 + np.arange(4)[None, :]).reshape(-1)
    np.testing.assert_allclose(A[np.ix_(op, op)], A, atol=1e-15)
    np.testing.assert_allclose(B[np.ix_(op, op)], B, atol=1e-15)


def test_equivalent_columns_have_equal_density_and_iterations(d2):
    s = d2
    A, B = oracle.to_csr(s, "A"), oracle.to_csr(s, "B")
    rho = dense.exact_rho(A.dense(), B.dense(), 0.2, 0.05)
    diag = np.diag(rho).reshape(-1, 4)
    assert np.abs(diag - diag[0][None, :]).max() < 1e-12
    # the shifted solves of equivalent columns have the same residual history, so
    # their iteration counts differ at most by the rounding at the tolerance crossing
    cols = np.arange(0, 256, dtype=np.int32)
    r = oracle.shifted_solve(A, B, cols, synth.shift_grid(8), tol=1e-8, full=False, true_residual=False)
    it = np.asarray(r.iters).reshape(-1, 4)
    assert np.all(it.max(0) - it.min(0) <= 1)


def test_amorphous_columns_are_not_equivalent():
    """The disordered box's columns of one orbital type differ (contrast): their
    densities spread, and so do their iteration counts."""
    s = synth.make_system(128, synth.config_seed(1))
    A, B = oracle.to_csr(s, "A"), oracle.to_csr(s, "B")
    rho = dense.exact_rho(A.dense(), B.dense(), 0.2, 0.05)
    h = np.nonzero(s.n_orb == 1)[0]
    d = np.diag(rho)[s.orb_off[h]]
    assert d.std() > 1e-3
    cols = s.orb_off[h][:32].astype(np.int32)
    r = oracle.shifted_solve(A, B, cols, synth.shift_grid(8), tol=1e-8, full=False, true_residual=False)
    it = np.asarray(r.iters)
    assert it.max() - it.min() > 5


@pytest.mark.parametrize("kappa", [20, 100])
def test_kappa_radii_hold_kappa_atoms(kappa):
    """Amorphous box: the sphere of each radius holds exactly kappa atoms (the
    centre included), checked by brute-force minimum-image distances."""
    s = synth.make_system(1024, synth.config_seed(2))
    centres = np.arange(0, 1024, 37)
    radii = synth.kappa_radii(s, centres, kappa)
    for c, r in zip(centres, radii):
        d = s.pos - s.pos[c]
        d -= s.L * np.rint(d / s.L)
        dist = np.sqrt((d * d).sum(1))
        assert np.sum(dist <= r) == kappa
        assert np.sort(dist)[kappa - 1] < r < np.sort(dist)[kappa]


def test_kappa_radii_take_whole_shells_in_the_crystal(d2):
    """Crystal: tied distances put whole shells inside, identically for every atom."""
    s = synth.make_diamond(3, 2001)
    radii = synth.kappa_radii(s, np.arange(s.n_atoms), 20)
    assert np.ptp(radii) < 1e-9
    counts = [oracle.region_atoms(s, i, float(radii[i])).size for i in range(0, s.n_atoms, 17)]
    assert len(set(counts)) == 1 and counts[0] >= 20
    d = s.pos - s.pos[0]
    d -= s.L * np.rint(d / s.L)
    dist = np.sort(np.sqrt((d * d).sum(1)))
    # membership is robust: no atom lies just outside the cut (the tied shell is
    # inside, the next shell far beyond)
    r = radii[0]
    assert np.sum(dist <= r) == np.sum(dist <= r + 1e-6) == counts[0]
