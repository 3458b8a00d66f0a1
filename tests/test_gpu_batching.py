"""Persistent batching: HIP-graph replay of the outer iterations, and the pass autotuner.

The graph path captures a whole number of periods of the buffer rotation (at
least 8 outer iterations) once and replays it many times, with the host's
polling (a device-to-host copy and an event wait) between replays; every
column's result is written by whichever replay finishes it.  The same kernels
run in the same order as on the eager path, so outputs must agree exactly.
"""
import numpy as np
import pytest

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
