"""Persistent batching: HIP-graph replay of the outer iterations, and the pass autotuner.

The graph path captures a whole number of periods of the buffer rotation (at
least 8 outer iterations) once and replays it many times, with the host's
polling (a device-to-host copy and an event wait) between replays; every
column's result is written by whichever replay finishes it.  The same kernels
run in the same order as on the eager path, so outputs must agree exactly.
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
def c1(el, ctx):
    s = synth.make_system(128, synth.config_seed(1))
    return s, el.Matrix.from_system(ctx, s), el.Matrix.from_system(ctx, s, precision="mixed")


@pytest.mark.parametrize("mixed", [False, True])
def test_graph_replay_equals_eager(el, ctx, c1, mixed):
    s, mat, mat32 = c1
    m = mat32 if mixed else mat
    z = synth.shift_grid(32)
    cols = np.arange(s.M, dtype=np.int32)  # 257 columns in 128 slots: slot refill across replays
    cw = np.full(len(z), -0.01 + 0.002j)
    kw = dict(tol=1e-9, slots=128, mixed=mixed, want_x=True)
    a = el.density_matrix(ctx, m, cols, z, cw, **kw)
    b = el.density_matrix(ctx, m, cols, z, cw, graph=True, **kw)
    assert np.array_equal(a["x"].cpu().numpy(), b["x"].cpu().numpy())
    assert np.array_equal(a["rho"].cpu().numpy(), b["rho"].cpu().numpy())
    assert np.array_equal(a["iters"].cpu().numpy(), b["iters"].cpu().numpy())
    assert np.array_equal(a["traces"], b["traces"])


@pytest.mark.parametrize("mixed", [False, True])
def test_graph_replay_against_oracle(el, ctx, c1, mixed):
    """Graph replay read against the oracle, not only against the eager path: all 257
    columns of the 128-atom box in 128 slots (columns refill slots across replays), x and
    rho on the patterns and both column traces against the oracle's shifted solves
    (tol 1e-11; on the FP32-rounded pencil in mixed mode) and its density assembly
    (Eq. 12, Eq. 7).  Two graph solves (two captures, each replayed many times with the
    host's polling between replays) around an eager solve: each must also equal the
    eager result exactly."""
    s, mat, mat32 = c1
    m = mat32 if mixed else mat
    z = synth.shift_grid(32)
    K = len(z)
    cols = np.arange(s.M, dtype=np.int32)
    cw = oracle.fermi_weights(z, mu=0.0, tau=0.02)
    sysm = s if not mixed else dataclasses.replace(s, A_val=s.A_val.astype(np.float32).astype(np.float64),
                                                   B_val=s.B_val.astype(np.float32).astype(np.float64))
    A, B = oracle.to_csr(sysm, "A"), oracle.to_csr(sysm, "B")
    ref = oracle.shifted_solve(A, B, cols, z, tol=1e-11, full=False, true_residual=False)
    rho_r, trB_r, trA_r = oracle.density_from_x(B, A, cols, ref.x, ref.pat_off, cw)
    bound = 5e-7 if mixed else 1e-8
    kw = dict(tol=1e-9, slots=128, mixed=mixed, want_x=True)
    runs = [el.density_matrix(ctx, m, cols, z, cw, graph=True, **kw)]
    eager = el.density_matrix(ctx, m, cols, z, cw, **kw)
    runs.append(el.density_matrix(ctx, m, cols, z, cw, graph=True, **kw))
    for g in runs:
        assert np.array_equal(g["x"].cpu().numpy(), eager["x"].cpu().numpy())
        assert np.array_equal(g["rho"].cpu().numpy(), eager["rho"].cpu().numpy())
        assert np.array_equal(np.asarray(g["pat_off"]), ref.pat_off)
        xg = g["x"].cpu().numpy()
        for c in range(len(cols)):
            p0, p1 = int(ref.pat_off[c]), int(ref.pat_off[c + 1])
            xr = ref.x[p0 * K:p1 * K].reshape(K, -1)
            assert np.abs(xg[p0 * K:p1 * K].reshape(K, -1) - xr).max() <= bound * np.abs(xr).max(), c
        rho = g["rho"].cpu().numpy()
        assert np.abs(rho - rho_r).max() <= bound * np.abs(rho_r).max()
        ctr = g["col_traces"].cpu().numpy()
        assert np.abs(ctr[:, 0] - trB_r).max() <= bound * np.abs(trB_r).max()
        assert np.abs(ctr[:, 1] - trA_r).max() <= bound * np.abs(trA_r).max()


def test_graph_replay_region_mode(el, ctx):
    s = synth.make_system(600, 4242)
    mat = el.Matrix.from_system(ctx, s)
    rng = np.random.default_rng(3)
    centres = np.sort(rng.choice(s.n_atoms, size=30, replace=False)).astype(np.int32)
    reg = el.Regions(ctx, mat, centres, rng.uniform(4.0, 7.0, size=30), 64)
    z = synth.shift_grid(16)
    a = el.region_solve(ctx, reg, z, tol=1e-9)
    b = el.region_solve(ctx, reg, z, tol=1e-9, graph=True)
    assert np.array_equal(a["x"].cpu().numpy(), b["x"].cpu().numpy())
    assert np.array_equal(a["iters"].cpu().numpy(), b["iters"].cpu().numpy())


def test_autotune_picks_a_timed_configuration(el, ctx):
    s = synth.make_system(128, synth.config_seed(1))
    mat = el.Matrix.from_system(ctx, s)
    z = synth.shift_grid(16)
    cols = np.arange(0, s.M, 2, dtype=np.int32)
    ref = el.shifted_solve(ctx, mat, cols, z, tol=1e-10)["x"].cpu().numpy()
    v, sl, ns = el.autotune(ctx, mat, max_slots=512)
    assert sl in (256, 512) and ns > 0
    assert (v & 15) in (1, 4, 5, 6)
    got = el.shifted_solve(ctx, mat, cols, z, tol=1e-10)["x"].cpu().numpy()  # uses the tuned configuration
    assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()
