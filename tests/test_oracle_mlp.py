"""Pins of the CPU FP64 reference of the learned SPAI (oracle/mlp.py)."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp


@pytest.fixture(scope="module")
def small():
    s = synth.make_system(64, 2024, r_cut=3.5)
    P = mlp.pairs(s)
    return s, P


def test_parameter_count():
    assert mlp.N_PARAM == 40 * 128 + 128 + 2 * (128 * 128 + 128) + 128 * 16 + 16 == 40336


def test_gelu_closed_forms():
    x = np.array([-30.0, -1.0, 0.0, 1.0, 30.0])
    g = mlp.gelu(x)
    assert g[2] == 0.0 and abs(g[0]) < 1e-12 and abs(g[4] - 30.0) < 1e-12
    # x Phi(x) at x = 1: Phi(1) = 0.841344746068543
    assert abs(g[3] - 0.841344746068543) < 1e-14
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(x), fd, rtol=0, atol=1e-8)


def test_gradient_matches_finite_differences(small):
    s, P = small
    X = mlp.features(s, P[:7])
    Binv = np.linalg.inv(oracle.to_csr(s, "B").dense())
    T, W = mlp.targets(s, P[:7], Binv)
    theta = mlp.init_params(5) + 0.01 * np.random.default_rng(1).standard_normal(mlp.N_PARAM)
    loss, g = mlp.loss_grad(theta, X, T, W)
    rng = np.random.default_rng(2)
    # every layer's weights and biases are probed
    offs = np.cumsum([0] + [int(np.prod(sh)) for sh in mlp.SHAPES])
    idx = np.concatenate([rng.choice(np.arange(offs[i], offs[i + 1]), size=min(12, offs[i + 1] - offs[i]),
                                     replace=False) for i in range(len(mlp.SHAPES))])
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss_grad(tp, X, T, W)[0] - mlp.loss_grad(tm, X, T, W)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i


def test_features_against_dense_products(small):
    s, P = small
    X = mlp.features(s, P)
    B = oracle.to_csr(s, "B").dense()
    E = B - np.eye(s.M)
    E2 = E @ E
    for p, (I, J) in enumerate(P):
        nI, nJ = int(s.n_orb[I]), int(s.n_orb[J])
        oI, oJ = int(s.orb_off[I]), int(s.orb_off[J])
        bb = X[p, 6:22].reshape(4, 4)
        ee = X[p, 22:38].reshape(4, 4)
        assert np.allclose(bb[:nI, :nJ], 10 * B[oI:oI + nI, oJ:oJ + nJ], atol=1e-15)
        # E^2 restricted to the pattern: the two-hop paths all stay inside it
        assert np.allclose(ee[:nI, :nJ], 10 * E2[oI:oI + nI, oJ:oJ + nJ], atol=1e-12)
        assert np.all(bb[nI:, :] == 0) and np.all(bb[:, nJ:] == 0)
        assert X[p, 3] <= 3.5 / 4 + 1e-12
        assert X[p, 38] == (1.0 if I == J else 0.0)
        assert math.isclose(X[p, 3], np.linalg.norm(X[p, 0:3]), rel_tol=1e-12, abs_tol=1e-15)


def test_targets_assemble_to_inverse_on_pattern(small):
    s, P = small
    Bc = oracle.to_csr(s, "B")
    B = Bc.dense()
    Binv = np.linalg.inv(B)
    T, W = mlp.targets(s, P, Binv)
    M = mlp.assemble(s, P, T)
    pat = np.zeros_like(B, dtype=bool)  # the block pattern, structural zeros included
    for i in range(Bc.n):
        pat[i, Bc.ci[Bc.rp[i]:Bc.rp[i + 1]]] = True
    assert np.allclose(M[pat], Binv[pat], atol=1e-14)
    assert np.all(M[~pat] == 0)
    assert np.allclose(M, M.T, atol=1e-15)
    # mask counts: every valid entry of every upper block
    assert W.sum() == sum(int(s.n_orb[I]) * int(s.n_orb[J]) for I, J in P)


def test_bf16_rounding_closed_forms():
    one = 1.0
    ulp = 2.0 ** -7  # spacing of bfloat16 at 1
    x = np.array([one, one + ulp / 2, one + 3 * ulp / 2, one + ulp / 2 + 2 ** -20, -2.5, 3.0e38 * 0 + 65504.0])
    r = mlp.bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0                   # tie -> even
    assert r[2] == one + 2 * ulp         # tie -> even (upwards)
    assert r[3] == one + ulp             # above the tie -> up
    assert r[4] == -2.5                  # exactly representable
    assert r[5] == 65536.0               # 65504 rounds to 2^16 in bfloat16
