"""CPU FP64 oracle for the generalized shifted equations (paper Sec. III).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg use this package.  It shares no code with the GPU library
(`paper_1609_08377_amd`) and never imports it; both only read the seeded
inputs made by `synth`.

Contents
--------
* `to_csr`            scalar CSR of A and B built from the atom-block input,
                      keeping every structurally present entry (Sec. II-C:
                      composite index i <-> (I, alpha)).
* `shifted_solve`     x_{j,k} = (z_k B - A)^{-1} e_j for many shifts sharing one
                      Krylov subspace (Eqs. 9, 13, 14) -- plain C, FP64,
                      shifted COCG with a CG inner solve on B (oracle.c).
* `density_from_x`    rho_ij = sum_k Im(c_k x_{j,k,i}) on the pattern of column
                      j, the discretised energy integral (Eq. 12), and the
                      projected traces e_j^T rho X e_j for X = B, A (Eq. 7).
* `fermi_weights`     c_k = -(1/pi) w_k f(Re z_k) with the Fermi function (Eq. 3).
* `carve_region`      principal sub-pencil of the atoms within a radius of a
                      centre atom (real-space projection, Sec. III-B).
* `dense`             brute-force dense checks (Eqs. 1, 6, 10, 11).
* `arnoldi`           the multiple Arnoldi method: Rayleigh-Ritz on the
                      direct sum of two Krylov spaces and the analytic energy
                      integration (Eqs. 15-18).
* `mlp`               the learned block sparse approximate inverse of B.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_oracle.so")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc + OpenMP (plain C, no GPU)."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _c():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        lib.oracle_shifted_solve.argtypes = [ctypes.c_int, P, P, P, P, P, P, ctypes.c_int, P, ctypes.c_int, P,
                                             ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                                             ctypes.c_int, P, P, P, P, P, P, ctypes.c_int]
        lib.oracle_shifted_solve.restype = ctypes.c_int
        lib.oracle_cg_B.argtypes = [ctypes.c_int, P, P, P, P, P, ctypes.c_double, ctypes.c_int]
        lib.oracle_cg_B.restype = ctypes.c_int
        lib.oracle_spmv.argtypes = [ctypes.c_int, P, P, P, P, P]
        lib.oracle_spmv.restype = None
        lib.oracle_true_residual.argtypes = [ctypes.c_int, P, P, P, P, P, P, ctypes.c_int, ctypes.c_double,
                                             ctypes.c_double, P]
        lib.oracle_true_residual.restype = ctypes.c_double
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


@dataclass
class CSR:
    n: int
    rp: np.ndarray   # int64 (n+1)
    ci: np.ndarray   # int32
    v: np.ndarray    # float64

    def dense(self) -> np.ndarray:
        D = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rp))
        D[rows, self.ci] = self.v
        return D

    def matvec(self, x: np.ndarray) -> np.ndarray:
        y = np.zeros(self.n)
        xc = np.ascontiguousarray(x, np.float64)  # keep the (possibly copied) input alive during the call
        _c().oracle_spmv(self.n, _p(self.rp), _p(self.ci), _p(self.v), _p(xc), _p(y))
        return y


def to_csr(sysm, which: str) -> CSR:
    """Scalar CSR (rows ascending, columns ascending) of A or B.

    Row (I, alpha) lists, for each block (I, J) of atom row I in order of J,
    the orbitals beta of J.  Entries that are zero inside a present block
    (e.g. off-diagonal on-site entries) are kept, so the row pattern equals
    the atom-block pattern.
    """
    vals = sysm.A_val if which == "A" else sysm.B_val
    n_orb = sysm.n_orb.astype(np.int64)
    off = sysm.orb_off
    M = int(off[-1])
    rowlen_atom = np.zeros(sysm.n_atoms, dtype=np.int64)
    for I in range(sysm.n_atoms):
        b0, b1 = sysm.blk_row_ptr[I], sysm.blk_row_ptr[I + 1]
        rowlen_atom[I] = int(n_orb[sysm.blk_col[b0:b1]].sum())
    rl = np.repeat(rowlen_atom, n_orb)
    rp = np.zeros(M + 1, dtype=np.int64)
    np.cumsum(rl, out=rp[1:])
    ci = np.zeros(int(rp[-1]), dtype=np.int32)
    v = np.zeros(int(rp[-1]), dtype=np.float64)
    for I in range(sysm.n_atoms):
        ni = int(n_orb[I])
        b0, b1 = int(sysm.blk_row_ptr[I]), int(sysm.blk_row_ptr[I + 1])
        for a in range(ni):
            row = int(off[I]) + a
            p = int(rp[row])
            for b in range(b0, b1):
                J = int(sysm.blk_col[b])
                nj = int(n_orb[J])
                blk = vals[sysm.val_ptr[b]:sysm.val_ptr[b + 1]].reshape(ni, nj)
                ci[p:p + nj] = np.arange(off[J], off[J] + nj)
                v[p:p + nj] = blk[a]
                p += nj
    return CSR(M, rp, ci, v)


def pattern_offsets(B: CSR, cols: np.ndarray) -> np.ndarray:
    """Offsets of each column's pattern block: pat_off[c] = sum_{c'<c} |P_j(c')|; length ncols+1."""
    lens = (B.rp[np.asarray(cols) + 1] - B.rp[np.asarray(cols)]).astype(np.int64)
    off = np.zeros(len(cols) + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return off


@dataclass
class SolveResult:
    x: np.ndarray          # complex; full: (ncols, K, M); pattern: flat, see pattern_offsets
    iters: np.ndarray      # (ncols,)
    conv_it: np.ndarray    # (ncols, K)
    est: np.ndarray        # (ncols, K) residual estimates
    true_res: np.ndarray   # (ncols, K) recomputed true residuals
    pat_off: np.ndarray | None
    inner_failures: int


def shifted_solve(A: CSR, B: CSR, cols, z, tol: float = 1e-8, max_it: int = 20000, inner_tol: float = 1e-13,
                  inner_max: int = 1000, full: bool = True, nthreads: int = 0,
                  true_residual: bool = True) -> SolveResult:
    """x_{j,k} = (z_k B - A)^{-1} e_j by shifted COCG (see oracle.c)."""
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    z = np.ascontiguousarray(np.asarray(z, dtype=np.complex128))
    K = z.shape[0]
    nc = cols.shape[0]
    n = A.n
    zri = np.ascontiguousarray(np.stack([z.real, z.imag], axis=1).reshape(-1))
    if full:
        x = np.zeros((nc, K, n), dtype=np.complex128)
        pat = None
    else:
        pat = pattern_offsets(B, cols)
        x = np.zeros(int(pat[-1]) * K, dtype=np.complex128)
    iters = np.zeros(nc, dtype=np.int32)
    conv = np.zeros((nc, K), dtype=np.int32)
    est = np.zeros((nc, K))
    tru = np.zeros((nc, K)) if true_residual else None
    fails = _c().oracle_shifted_solve(n, _p(A.rp), _p(A.ci), _p(A.v), _p(B.rp), _p(B.ci), _p(B.v), nc, _p(cols),
                                      K, _p(zri), tol, max_it, inner_tol, inner_max, 1 if full else 0,
                                      _p(pat), _p(x), _p(iters), _p(conv), _p(est), _p(tru), nthreads)
    return SolveResult(x, iters, conv, est, tru, pat, fails)


def cg_B(B: CSR, s: np.ndarray, tol: float = 1e-13, max_it: int = 1000):
    x = np.zeros(B.n)
    sc = np.ascontiguousarray(s, np.float64)
    it = _c().oracle_cg_B(B.n, _p(B.rp), _p(B.ci), _p(B.v), _p(sc), _p(x), tol, max_it)
    return x, it


def true_residual(A: CSR, B: CSR, j: int, z: complex, x: np.ndarray) -> float:
    x = np.ascontiguousarray(x, dtype=np.complex128)
    return _c().oracle_true_residual(A.n, _p(A.rp), _p(A.ci), _p(A.v), _p(B.rp), _p(B.ci), _p(B.v), int(j),
                                     float(np.real(z)), float(np.imag(z)), _p(x))


def max_threads() -> int:
    return _c().oracle_max_threads()


# ---------------------------------------------------------------------------
# Energy integral and density-matrix elements (Eqs. 3, 5-7, 12)
# ---------------------------------------------------------------------------

def fermi(eps, mu: float, tau: float):
    """f(eps) = 1 / (1 + exp((eps - mu)/tau))  (Eq. 3), overflow-safe."""
    t = (np.asarray(eps, dtype=np.float64) - mu) / tau
    return 0.5 * (1.0 - np.tanh(0.5 * t))


def fermi_weights(z, mu: float, tau: float) -> np.ndarray:
    """c_k = -(1/pi) w_k f(Re z_k), w_k the midpoint width of the grid (Eq. 12 on the shift grid)."""
    z = np.asarray(z)
    eps = z.real
    K = eps.shape[0]
    if K > 1:
        w = np.full(K, (eps.max() - eps.min()) / (K - 1))
    else:
        w = np.ones(1)
    return (-(1.0 / np.pi) * w * fermi(eps, mu, tau)).astype(np.complex128)


def density_from_x(B: CSR, A: CSR, cols, x_pattern: np.ndarray, pat_off: np.ndarray, c: np.ndarray):
    """rho_ij = sum_k Im(c_k x_{j,k,i}) for i in P_j, and per-column traces.

    Returns (rho flat [pat_off[-1]], trB [ncols], trA [ncols]) with
    trX_j = sum_{i in P_j} rho_ij X_ij = e_j^T rho X e_j for symmetric rho, X (Eq. 7).
    """
    cols = np.asarray(cols)
    K = c.shape[0]
    rho = np.zeros(int(pat_off[-1]))
    trB = np.zeros(len(cols))
    trA = np.zeros(len(cols))
    for ci_, j in enumerate(cols):
        p0, p1 = int(pat_off[ci_]), int(pat_off[ci_ + 1])
        plen = p1 - p0
        xs = x_pattern[p0 * K:p1 * K].reshape(K, plen)
        r = np.imag(c[:, None] * xs).sum(axis=0)
        rho[p0:p1] = r
        b0, b1 = int(B.rp[j]), int(B.rp[j + 1])
        trB[ci_] = float(np.dot(r, B.v[b0:b1]))
        trA[ci_] = float(np.dot(r, A.v[b0:b1]))
    return rho, trB, trA


# ---------------------------------------------------------------------------
# Real-space projection (Sec. III-B): principal sub-pencil of a sphere
# ---------------------------------------------------------------------------

def region_atoms(sysm, centre: int, radius: float) -> np.ndarray:
    """Atoms whose minimum-image distance to the centre atom is <= radius, ascending."""
    d = sysm.pos - sysm.pos[centre]
    d -= sysm.L * np.rint(d / sysm.L)
    r2 = np.einsum("ij,ij->i", d, d)
    return np.nonzero(r2 <= radius * radius)[0].astype(np.int64)


def carve_region(sysm, atoms: np.ndarray):
    """Scalar CSR of the principal submatrices A_r, B_r for the atom subset.

    Returns (A_r, B_r, orbital_index_map) where orbital_index_map[l] is the
    global orbital of local orbital l.
    """
    atoms = np.asarray(atoms, dtype=np.int64)
    n_orb = sysm.n_orb.astype(np.int64)
    glob2loc_atom = -np.ones(sysm.n_atoms, dtype=np.int64)
    glob2loc_atom[atoms] = np.arange(atoms.size)
    loc_off = np.zeros(atoms.size + 1, dtype=np.int64)
    np.cumsum(n_orb[atoms], out=loc_off[1:])
    m = int(loc_off[-1])
    orb_map = np.concatenate([np.arange(sysm.orb_off[I], sysm.orb_off[I] + n_orb[I]) for I in atoms])
    out = []
    for vals in (sysm.A_val, sysm.B_val):
        rp = [0]
        ci = []
        vv = []
        for li, I in enumerate(atoms):
            ni = int(n_orb[I])
            b0, b1 = int(sysm.blk_row_ptr[I]), int(sysm.blk_row_ptr[I + 1])
            rows_c = [[] for _ in range(ni)]
            rows_v = [[] for _ in range(ni)]
            for b in range(b0, b1):
                J = int(sysm.blk_col[b])
                lj = glob2loc_atom[J]
                if lj < 0:
                    continue
                nj = int(n_orb[J])
                blk = vals[sysm.val_ptr[b]:sysm.val_ptr[b + 1]].reshape(ni, nj)
                for a in range(ni):
                    rows_c[a].extend(range(int(loc_off[lj]), int(loc_off[lj]) + nj))
                    rows_v[a].extend(blk[a].tolist())
            for a in range(ni):
                ci.extend(rows_c[a])
                vv.extend(rows_v[a])
                rp.append(len(ci))
        out.append(CSR(m, np.asarray(rp, dtype=np.int64), np.asarray(ci, dtype=np.int32),
                       np.asarray(vv, dtype=np.float64)))
    return out[0], out[1], orb_map
