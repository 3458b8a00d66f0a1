"""Dense brute-force references for small pencils (test infrastructure).

These are the textbook definitions written out with LAPACK calls:

* `dense_G(A, B, z)`          (zB - A)^{-1} by LU (Eq. 10 definition of G).
* `spectral_G(A, B, z)`       sum_k y_k y_k^T / (z - lambda_k) from the
                              generalised eigenpairs A y = lambda B y with
                              y_k^T B y_l = delta_kl (Eqs. 1, 11).
* `trace_closed_forms`        Tr[rho B] = sum_n g(lambda_n) and
                              Tr[rho A] = sum_n g(lambda_n) lambda_n with
                              g(lambda) = sum_k Im(c_k / (z_k - lambda)), i.e.
                              the discretised energy integral (Eq. 12) pushed
                              through the spectral sum (Eq. 11) and the
                              B-orthonormality of the eigenvectors.
* `exact_rho`                 rho = sum_k f(lambda_k) y_k y_k^T (Eq. 6; the
                              eigenvalue lambda_k is what f takes, Eq. 2).
* `chemical_potential`        mu such that 2 sum_k f(lambda_k) = N_e (Sec. II-B:
                              mu reproduces the number of electrons).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl


def dense_G(A: np.ndarray, B: np.ndarray, z: complex) -> np.ndarray:
    M = A.shape[0]
    return np.linalg.solve(z * B - A, np.eye(M, dtype=np.complex128))


def gen_eig(A: np.ndarray, B: np.ndarray):
    lam, Y = sl.eigh(A, B)
    return lam, Y


def spectral_G(A: np.ndarray, B: np.ndarray, z: complex, eig=None) -> np.ndarray:
    lam, Y = eig if eig is not None else gen_eig(A, B)
    return (Y / (z - lam)[None, :]) @ Y.T


def trace_closed_forms(A: np.ndarray, B: np.ndarray, z: np.ndarray, c: np.ndarray, eig=None):
    lam, _ = eig if eig is not None else gen_eig(A, B)
    g = np.imag(c[None, :] / (z[None, :] - lam[:, None])).sum(axis=1)
    return float(g.sum()), float((g * lam).sum())


def fermi(lam, mu, tau):
    t = (np.asarray(lam) - mu) / tau
    return 0.5 * (1.0 - np.tanh(0.5 * t))


def exact_rho(A: np.ndarray, B: np.ndarray, mu: float, tau: float, eig=None) -> np.ndarray:
    lam, Y = eig if eig is not None else gen_eig(A, B)
    return (Y * fermi(lam, mu, tau)[None, :]) @ Y.T


def chemical_potential(lam: np.ndarray, n_electrons: float, tau: float, spin: float = 2.0) -> float:
    lo, hi = float(lam.min()) - 50 * tau, float(lam.max()) + 50 * tau
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if spin * fermi(lam, mid, tau).sum() < n_electrons:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)
