"""Observables from stored solutions through the C ABI: re-weighting, ICOHP, chemical potential.

References: the density matrix computed inside the solve (same weights), the
oracle's own solutions with its own assembly (oracle.density_from_x), and
invariants: the ICOHP summed over all atom pairs is Tr[rho A] (Eq. 4 with
X = A), and C_IJ = C_JI when rho and A are symmetric.
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
def c1(el, ctx):
    s = synth.make_system(128, synth.config_seed(1))
    return s, el.Matrix.from_system(ctx, s), oracle.to_csr(s, "A"), oracle.to_csr(s, "B")


def test_reweight_matches_solve(el, ctx, c1):
    s, mat, A, B = c1
    z = synth.shift_grid(32)
    cw = oracle.fermi_weights(z, 0.1, 0.05)
    cols = np.arange(s.M, dtype=np.int32)
    dm = el.density_matrix(ctx, mat, cols, z, cw, tol=1e-10, want_x=True)
    rw = el.density_reweight(ctx, mat, cols, cw, dm["x"])
    a, b = dm["rho"].cpu().numpy(), rw["rho"].cpu().numpy()
    assert np.abs(a - b).max() <= 1e-14 * np.abs(a).max()
    assert np.allclose(rw["traces"], dm["traces"], rtol=1e-13, atol=0)


def test_icohp_invariants_and_oracle(el, ctx, c1):
    s, mat, A, B = c1
    z = synth.shift_grid(32)
    cw = oracle.fermi_weights(z, 0.0, 0.05)
    cols = np.arange(s.M, dtype=np.int32)
    x = el.shifted_solve(ctx, mat, cols, z, tol=1e-10)["x"]
    rw = el.density_reweight(ctx, mat, cols, cw, x)
    ic = rw["icohp"].cpu().numpy()
    assert abs(ic.sum() - rw["traces"][1]) <= 1e-12 * max(1.0, abs(rw["traces"][1]))
    atom_of = np.repeat(np.arange(s.n_atoms), s.n_orb.astype(int))
    C = {}
    for c in range(len(cols)):
        J = atom_of[cols[c]]
        for b in range(rw["blk_off"][c], rw["blk_off"][c + 1]):
            key = (int(rw["blk_atom"][b]), int(J))
            C[key] = C.get(key, 0.0) + ic[b]
    scale = max(abs(v) for v in C.values())
    assert max(abs(C[(I, J)] - C[(J, I)]) for (I, J) in C) <= 1e-6 * scale
    # against the oracle's solutions and assembly
    ref = oracle.shifted_solve(A, B, cols, z, tol=1e-11, full=False, true_residual=False)
    rho_ref, _, ta = oracle.density_from_x(B, A, cols, ref.x, ref.pat_off, cw)
    assert abs(ta.sum() - rw["traces"][1]) <= 1e-8 * max(1.0, abs(ta.sum()))
    worst = 0.0
    for c, j in enumerate(cols):
        p0 = ref.pat_off[c]
        h = rho_ref[p0:ref.pat_off[c + 1]] * A.v[A.rp[j]:A.rp[j + 1]]
        q = 0
        for b in range(rw["blk_off"][c], rw["blk_off"][c + 1]):
            n = int(s.n_orb[rw["blk_atom"][b]])
            worst = max(worst, abs(h[q:q + n].sum() - ic[b]))
            q += n
    assert worst <= 1e-8 * scale


def test_chemical_potential_bisection(el, ctx, c1):
    s, mat, A, B = c1
    z = synth.shift_grid(32)
    K = len(z)
    cols = np.arange(0, s.M, 4, dtype=np.int32)
    tau = 0.05
    x = el.shifted_solve(ctx, mat, cols, z, tol=1e-10)["x"]
    ref = oracle.shifted_solve(A, B, cols, z, tol=1e-11, full=False, true_residual=False)

    def count_ref(mu):
        _, tb, _ = oracle.density_from_x(B, A, cols, ref.x, ref.pat_off, oracle.fermi_weights(z, mu, tau))
        return tb.sum()

    target = 0.5 * (count_ref(-0.8) + count_ref(0.8))
    lo, hi = -0.8, 0.8
    while hi - lo > 1e-12:
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if count_ref(mid) < target else (lo, mid)
    mu_ref = 0.5 * (lo + hi)
    mu, cnt = el.chemical_potential(ctx, mat, cols, z, np.full(K, 2.0 / K), x, tau, target, -0.8, 0.8, 1e-12)
    slope = (count_ref(mu_ref + 1e-4) - count_ref(mu_ref - 1e-4)) / 2e-4
    assert slope > 0
    assert abs(mu - mu_ref) <= 1e-8 / slope + 1e-11
    assert abs(cnt - target) <= 1e-8 * abs(target)
    with pytest.raises(el.ElsesError):
        el.chemical_potential(ctx, mat, cols, z, np.full(K, 2.0 / K), x, tau, 1e6, -0.8, 0.8)
