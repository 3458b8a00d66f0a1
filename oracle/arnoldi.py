"""CPU FP64 reference of the multiple Arnoldi method (Sec. III-B, Eqs. 15-18).

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark CPU leg).  It shares
no code with the GPU library and never imports it.

For one column j of the pencil (A, B) the method restricts the generalized
problem to the direct sum of two Krylov spaces of A (Eq. 15), nu even,

    L_nu = K_{nu/2}(A; e_j)  +  K_{nu/2}(A; B^{-1} e_j).

Rayleigh-Ritz on L_nu: with Q an orthonormal basis (M x n, n <= nu), the
reduced pencil (Q^T A Q) y = eps (Q^T B Q) y with y^T (Q^T B Q) y = 1 gives
the Ritz pairs (eps_m, v_m = Q y_m) and the column's Green's function
G^(j)(z) = sum_m v_m v_m^T / (z - eps_m) (Eqs. 16-17).  The energy integral
of a projected quantity is then a finite sum (Eq. 18):

    e_j^T rho X e_j = sum_m f(eps_m) (e_j^T v_m) (v_m^T X e_j),

and the density-matrix column is rho e_j = sum_m f(eps_m) v_m (v_m^T e_j).

Construction used here.  Only the span of L_nu enters Rayleigh-Ritz, but the
two sequences become nearly dependent on realistic pencils (at nu = 30 the
smallest singular value of the union of their orthonormal bases is ~1e-10),
so which numerically marginal directions count as new decides the result at
the level of the method's own truncation error.  The reading taken: the
basis grows vector by vector in the order e_j, B^{-1} e_j, A w_0, A w_1,
A w_2, ... where w_k is the k-th basis vector and each new vector continues
the sequence of the vector it multiplies (even positions: K(A; e_j), odd:
K(A; B^{-1} e_j)).  Every candidate is orthogonalised against all basis
vectors so far by two classical Gram-Schmidt passes and kept when what
remains exceeds 1e-10 of the candidate's norm; a dropped vector ends its
sequence (its later powers lie in the span of the rest, block Krylov
deflation).  Dense LAPACK (numpy / scipy) serves for B^{-1} e_j and the
reduced eigenproblem.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sl

DEFLATE = 1e-10


def krylov_chain(A: np.ndarray, b: np.ndarray, n: int) -> np.ndarray:
    """Orthonormal basis of K_n(A; b) (columns), fewer when the space is exhausted."""
    nb = np.linalg.norm(b)
    if n < 1 or nb == 0.0:
        return np.zeros((A.shape[0], 0))
    Q = [b / nb]
    while len(Q) < n:
        c = A @ Q[-1]
        c0 = np.linalg.norm(c)
        Qm = np.stack(Q, axis=1)
        for _ in range(2):
            c = c - Qm @ (Qm.T @ c)
        nc = np.linalg.norm(c)
        if c0 == 0.0 or nc <= DEFLATE * c0:
            break
        Q.append(c / nc)
    return np.stack(Q, axis=1)


def subspace(A: np.ndarray, B: np.ndarray, j: int, nu: int) -> np.ndarray:
    """Orthonormal basis of L_nu(A, B; e_j) (Eq. 15) as the columns of Q, built
    as described in the module docstring (at most nu vectors, nu/2 per sequence)."""
    if nu < 2 or nu % 2:
        raise ValueError("nu must be even and >= 2")
    M = A.shape[0]
    e = np.zeros(M)
    e[j] = 1.0
    u = np.linalg.solve(B, e)
    basis = []
    last = [None, None]  # latest kept vector of each sequence (None: the sequence has ended)

    def admit(c, seq):
        c0 = np.linalg.norm(c)
        if basis:
            Qm = np.stack(basis, axis=1)
            for _ in range(2):
                c = c - Qm @ (Qm.T @ c)
        nc = np.linalg.norm(c)
        if c0 > 0.0 and nc > DEFLATE * c0:
            basis.append(c / nc)
            last[seq] = basis[-1]
        else:
            last[seq] = None

    admit(e, 0)
    admit(u, 1)
    for _ in range(1, nu // 2):
        for seq in (0, 1):
            if last[seq] is not None:
                admit(A @ last[seq], seq)
    return np.stack(basis, axis=1)


def ritz(A: np.ndarray, B: np.ndarray, Q: np.ndarray):
    """Ritz values (ascending) and B-orthonormal Ritz vectors of (A, B) on span(Q)."""
    eps, Y = sl.eigh(Q.T @ A @ Q, Q.T @ B @ Q)
    return eps, Q @ Y


def column(A: np.ndarray, B: np.ndarray, j: int, nu: int, Q: np.ndarray | None = None) -> dict:
    """Ritz data of column j: eps, V, and the three weight vectors of Eq. 18

    wI_m = (e_j^T v_m)^2, wB_m = (e_j^T v_m)(v_m^T B e_j), wA_m = (e_j^T v_m)(v_m^T A e_j).
    A basis Q of the subspace may be given instead of the one of `subspace`.
    """
    if Q is None:
        Q = subspace(A, B, j, nu)
    eps, V = ritz(A, B, Q)
    a = V[j, :]
    return {"eps": eps, "V": V, "a": a, "wI": a * a, "wB": a * (V.T @ B[:, j]), "wA": a * (V.T @ A[:, j])}


def projected_trace(res: dict, f, which: str = "B") -> float:
    """e_j^T rho X e_j = sum_m f(eps_m) (e_j^T v_m)(v_m^T X e_j), X = I, B or A (Eq. 18)."""
    return float(np.sum(f(res["eps"]) * res["w" + which]))


def density_column(res: dict, f) -> np.ndarray:
    """rho e_j = sum_m f(eps_m) v_m (v_m^T e_j)."""
    return res["V"] @ (f(res["eps"]) * res["a"])


def green_column(res: dict, z: complex) -> np.ndarray:
    """x^(j)(z) = G^(j)(z) e_j = sum_m v_m (v_m^T e_j) / (z - eps_m) (Eqs. 16-17)."""
    return res["V"] @ (res["a"] / (z - res["eps"]))


def region_column(sysm, atoms: np.ndarray, j_global: int, nu: int) -> tuple[dict, np.ndarray]:
    """Column j_global on the principal sub-pencil of the atom subset (real-space
    projection): returns the column's Ritz data and the local->global orbital map."""
    from . import carve_region

    Ar, Br, omap = carve_region(sysm, atoms)
    jl = int(np.nonzero(omap == j_global)[0][0])
    return column(Ar.dense(), Br.dense(), jl, nu), omap
