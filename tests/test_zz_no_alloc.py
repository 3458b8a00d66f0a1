"""The allocation-free region solve (elses_regions_solve_noalloc) against the allocating one.

Both run the same per-region arithmetic (one workgroup per region, fixed
reduction order), only the scratch and the scheduling differ, so every output
must be identical.  Two calls in a row, the second with a smaller input, show
that the shared scratch array carries nothing from one call into the next.
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


def test_noalloc_region_solve_matches(el):
    ctx = el.Context(0)
    s = synth.make_system(600, 4242)
    mat = el.Matrix.from_system(ctx, s, precision="mixed")
    rng = np.random.default_rng(91)
    z = synth.shift_grid(16)
    cw = oracle.fermi_weights(z, mu=0.05, tau=0.02)
    for n_regions, mixed in ((48, True), (9, False)):
        centres = np.sort(rng.choice(s.n_atoms, size=n_regions, replace=False)).astype(np.int32)
        radii = rng.uniform(3.5, 7.0, size=n_regions)
        reg = el.Regions(ctx, mat, centres, radii)
        ref = el.region_solve(ctx, reg, z, cw, tol=1e-9, mixed=mixed, audit_every=4)
        got = el.region_solve(ctx, reg, z, cw, tol=1e-9, mixed=mixed, audit_every=4, noalloc=True)
        for key in ("x", "rho", "col_traces", "iters", "resid"):
            assert torch.equal(ref[key], got[key]), (n_regions, key)
        assert np.array_equal(ref["traces"], got["traces"])
        assert np.all(got["resid"].cpu().numpy() <= 1e-9)


def test_noalloc_rejects_oversized_solves(el):
    """A solve whose per-column state exceeds the scratch array is refused with the size it needs."""
    ctx = el.Context(0)
    s = synth.make_system(600, 4242)
    mat = el.Matrix.from_system(ctx, s)
    centres = np.arange(0, 200, dtype=np.int32)
    reg = el.Regions(ctx, mat, centres, np.full(centres.size, 7.0))
    z = synth.shift_grid(256)
    with pytest.raises(el.ElsesError) as e:
        el.region_solve(ctx, reg, z, full=True, audit=True, noalloc=True)
    assert "bytes of scratch" in str(e.value)
    tiles = el.Regions(ctx, mat, centres[:4], np.full(4, 5.0), 64)
    with pytest.raises(el.ElsesError):
        el.region_solve(ctx, tiles, synth.shift_grid(4), noalloc=True)
