"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module makes INPUTS only: atom positions, the atom-block sparsity
pattern, the values of the Hamiltonian-like matrix A and the overlap-like
matrix B, shift grids, sampled columns and region centres/radii.  It holds
none of the shifted-solver arithmetic.

The system is an amorphous hydrocarbon box (paper Sec. II-C: H atoms carry one
s orbital, C atoms carry s, px, py, pz, so M = N_H + 4 N_C; matrix elements
vanish beyond a cutoff distance).  The paper's tight-binding parameters and
polymer structures are not available, so the values follow a synthetic
recipe with the same structure:

* N_C = round(N/3) carbons, N_H = N - N_C hydrogens (C:H = 1:2).
* Periodic cube at 1.0 g/cm^3; random sequential addition with a minimum
  pair distance of 1.0 A (minimum image); the first N_C accepted points are C.
* Atoms are emitted in Morton order of a ~2 A cell grid (spatial locality),
  C and H interleaved as they fall.
* Pairs I != J with minimum-image distance r <= 4 A are coupled.  Every
  orbital pair of a coupled atom pair gets A = exp(-r/1.5) * g and
  B = 0.1 * exp(-r/1.5) * g' with g, g' ~ N(1, 0.1) drawn independently, once
  per unordered pair, and mirrored (A_JI = A_IJ^T).
* On-site: A_II = diag(g) with g ~ N(1, 0.1) (exp(0) = 1), zero between
  different orbitals of one atom; B_II = I.

Random streams: base seed s; positions use splitmix64(s), A draws PCG64(s+1),
B draws PCG64(s+2), regions PCG64(s+3), column sampling PCG64(s+4).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "_geom.so")

AMU_G = 1.66053906660e-24  # g per atomic mass unit
MASS_C = 12.011
MASS_H = 1.008
R_CUT = 4.0      # A
D_MIN = 1.0      # A
DECAY = 1.5      # A


def build(force: bool = False) -> str:
    """Compile the geometry helper with gcc (no GPU code)."""
    src = os.path.join(_HERE, "_geom.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _geom():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        lib.rsa_place.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                  ctypes.c_int64, ctypes.c_void_p]
        lib.rsa_place.restype = ctypes.c_int
        lib.count_pairs.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_void_p]
        lib.count_pairs.restype = ctypes.c_int
        lib.fill_pairs.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        lib.fill_pairs.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def box_side(n_atoms: int, density_g_cm3: float = 1.0) -> tuple[int, int, float]:
    n_c = int(round(n_atoms / 3.0))
    n_h = n_atoms - n_c
    mass_g = (n_c * MASS_C + n_h * MASS_H) * AMU_G
    vol_A3 = mass_g / density_g_cm3 * 1e24
    return n_c, n_h, vol_A3 ** (1.0 / 3.0)


def _morton3(ix: np.ndarray, iy: np.ndarray, iz: np.ndarray) -> np.ndarray:
    def spread(v):
        v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
        v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
        v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
        v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
        v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
        return v
    return spread(ix) | (spread(iy) << np.uint64(1)) | (spread(iz) << np.uint64(2))


@dataclass
class System:
    """Atom-block description of one (A, B) pencil.

    Blocks are stored for both (I, J) and (J, I), including the diagonal
    block, rows sorted by J.  Block b of row I couples atom I with atom
    blk_col[b]; its n_orb[I] x n_orb[J] values sit row-major at
    A_val[val_ptr[b]:...] (and B_val likewise).
    """
    n_atoms: int
    n_c: int
    L: float
    pos: np.ndarray            # (N, 3) float64, A
    n_orb: np.ndarray          # (N,) int8, 4 for C, 1 for H
    orb_off: np.ndarray        # (N+1,) int64 orbital offsets
    blk_row_ptr: np.ndarray    # (N+1,) int64
    blk_col: np.ndarray        # (nnzb,) int32
    val_ptr: np.ndarray        # (nnzb+1,) int64
    A_val: np.ndarray          # (nnz,) float64
    B_val: np.ndarray          # (nnz,) float64
    seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.orb_off[-1])

    @property
    def nnzb(self) -> int:
        return int(self.blk_row_ptr[-1])

    @property
    def nnz(self) -> int:
        return int(self.val_ptr[-1])


def make_system(n_atoms: int, seed: int, r_cut: float = R_CUT, density: float = 1.0,
                b_scale: float = 0.1) -> System:
    """Generate the synthetic pencil (A, B) for `n_atoms` atoms."""
    lib = _geom()
    n_c, n_h, L = box_side(n_atoms, density)
    if r_cut >= 0.5 * L:
        raise ValueError(f"box side {L:.3f} A too small for r_cut {r_cut} A (minimum image)")
    pos = np.zeros((n_atoms, 3), dtype=np.float64)
    rc = lib.rsa_place(n_atoms, L, D_MIN, np.uint64(seed & 0xFFFFFFFFFFFFFFFF), 200 * n_atoms + 1000, _ptr(pos))
    if rc != 0:
        raise RuntimeError(f"random sequential addition failed ({rc})")
    species_c = np.zeros(n_atoms, dtype=bool)
    species_c[:n_c] = True
    # Morton order of a ~2 A cell grid over all atoms (spatial locality); the
    # placement index breaks ties
    g = max(1, int(L // 2.0))
    cell = np.minimum((pos / (L / g)).astype(np.int64), g - 1)
    code = _morton3(cell[:, 0], cell[:, 1], cell[:, 2])
    order = np.lexsort((np.arange(n_atoms), code))
    pos = np.ascontiguousarray(pos[order])
    species_c = species_c[order]
    n_orb = np.where(species_c, 4, 1).astype(np.int8)
    orb_off = np.zeros(n_atoms + 1, dtype=np.int64)
    np.cumsum(n_orb, out=orb_off[1:])

    # unordered neighbour pairs (I<J), sorted by (I, J)
    cnt = np.zeros(n_atoms, dtype=np.int64)
    if lib.count_pairs(n_atoms, _ptr(pos), L, r_cut, _ptr(cnt)) != 0:
        raise RuntimeError("count_pairs failed")
    off = np.zeros(n_atoms + 1, dtype=np.int64)
    np.cumsum(cnt, out=off[1:])
    npair = int(off[-1])
    pj = np.zeros(npair, dtype=np.int32)
    pr = np.zeros(npair, dtype=np.float64)
    pd = np.zeros((npair, 3), dtype=np.float64)
    if lib.fill_pairs(n_atoms, _ptr(pos), L, r_cut, _ptr(off), _ptr(pj), _ptr(pr), _ptr(pd)) != 0:
        raise RuntimeError("fill_pairs failed")
    pi = np.repeat(np.arange(n_atoms, dtype=np.int32), cnt)

    # draws: once per unordered pair (16 per pair, top-left n_I x n_J used), then on-site
    rngA = np.random.Generator(np.random.PCG64(seed + 1))
    rngB = np.random.Generator(np.random.PCG64(seed + 2))
    gA = rngA.normal(1.0, 0.1, size=(npair, 4, 4))
    gA_site = rngA.normal(1.0, 0.1, size=(n_atoms, 4))
    gB = rngB.normal(1.0, 0.1, size=(npair, 4, 4))
    decay = np.exp(-pr / DECAY)
    blkA = gA * decay[:, None, None]
    blkB = b_scale * gB * decay[:, None, None]

    sysm = _assemble(n_atoms, n_c, L, pos, n_orb, orb_off, pi, pj, blkA, blkB, gA_site, seed)
    sysm.extra["pairs"] = (pi, pj, pr, pd)
    return sysm


def _assemble(n_atoms, n_c, L, pos, n_orb, orb_off, pi, pj, blkA, blkB, gA_site, seed) -> System:
    """Atom-block rows (diagonal + both directions of every pair, sorted by column)
    from per-pair 4 x 4 blocks (top-left n_I x n_J used for the stored (I, J), I < J;
    the mirrored (J, I) block is its transpose), on-site A = diag(gA_site), B = I."""
    npair = pi.shape[0]
    # full block rows: diagonal + both directions, sorted by column
    rows = np.concatenate([np.arange(n_atoms, dtype=np.int32), pi, pj])
    cols = np.concatenate([np.arange(n_atoms, dtype=np.int32), pj, pi])
    kind = np.concatenate([np.zeros(n_atoms, np.int8), np.ones(npair, np.int8), np.full(npair, 2, np.int8)])
    src = np.concatenate([np.arange(n_atoms), np.arange(npair), np.arange(npair)])
    o = np.lexsort((cols, rows))
    rows, cols, kind, src = rows[o], cols[o], kind[o], src[o]
    nnzb = rows.shape[0]
    blk_row_ptr = np.zeros(n_atoms + 1, dtype=np.int64)
    np.cumsum(np.bincount(rows, minlength=n_atoms), out=blk_row_ptr[1:])
    bsz = n_orb[rows].astype(np.int64) * n_orb[cols].astype(np.int64)
    val_ptr = np.zeros(nnzb + 1, dtype=np.int64)
    np.cumsum(bsz, out=val_ptr[1:])
    nnz = int(val_ptr[-1])
    A_val = np.zeros(nnz, dtype=np.float64)
    B_val = np.zeros(nnz, dtype=np.float64)
    # fill per block-shape class (vectorised)
    for ni in (4, 1):
        for nj in (4, 1):
            sel = np.nonzero((n_orb[rows] == ni) & (n_orb[cols] == nj))[0]
            if sel.size == 0:
                continue
            k = kind[sel]
            s = src[sel]
            va = np.zeros((sel.size, ni, nj))
            vb = np.zeros((sel.size, ni, nj))
            m1 = k == 1   # stored (I,J) with I<J: top-left block as drawn
            va[m1] = blkA[s[m1], :ni, :nj]
            vb[m1] = blkB[s[m1], :ni, :nj]
            m2 = k == 2   # mirrored (J,I): transpose of the pair's block
            va[m2] = np.transpose(blkA[s[m2], :nj, :ni], (0, 2, 1))
            vb[m2] = np.transpose(blkB[s[m2], :nj, :ni], (0, 2, 1))
            m0 = k == 0   # on-site
            if np.any(m0):
                idx = np.arange(ni)
                tmp = np.zeros((int(m0.sum()), ni, ni))
                tmp[:, idx, idx] = gA_site[s[m0], :ni]
                va[m0] = tmp
                va_eye = np.zeros_like(tmp)
                va_eye[:, idx, idx] = 1.0
                vb[m0] = va_eye
            base = val_ptr[sel]
            offs = base[:, None] + np.arange(ni * nj)[None, :]
            A_val[offs] = va.reshape(sel.size, ni * nj)
            B_val[offs] = vb.reshape(sel.size, ni * nj)
    return System(n_atoms=n_atoms, n_c=n_c, L=L, pos=pos, n_orb=n_orb, orb_off=orb_off,
                  blk_row_ptr=blk_row_ptr, blk_col=cols.astype(np.int32), val_ptr=val_ptr,
                  A_val=A_val, B_val=B_val, seed=seed)


DIAMOND_A = 3.567      # cubic lattice constant of diamond, Angstrom
DIAMOND_RCUT = 2.6459  # 5 bohr: first and second neighbours (1.545 and 2.522 A)


def make_diamond(n_cells: int, seed: int, r_cut: float = DIAMOND_RCUT, b_scale: float = 0.1) -> System:
    """Ideal periodic diamond crystal of n_cells^3 conventional cells (8 carbon
    atoms, 4 orbitals each), the ordered counterpart of the amorphous boxes.

    Values follow make_system's rule, A = exp(-r/1.5) g and B = 0.1 exp(-r/1.5) g
    off site, except that the random factors g are drawn once and shared: one
    symmetric 4 x 4 factor for every A pair, one for every B pair, and one set of
    four on-site factors for every atom.  Every atom is then equivalent to every
    other under the crystal's translations and its inversion through bond
    centres, so all atoms' subproblems are the same.  Atoms are numbered along a
    Morton curve as in make_system."""
    if n_cells < 2:
        raise ValueError("need at least 2 cells per side for the minimum image at the diamond cutoff")
    lib = _geom()
    fcc = np.array([[0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0]])
    basis = np.concatenate([fcc, fcc + 0.25])
    cells = np.stack(np.meshgrid(*(np.arange(n_cells),) * 3, indexing="ij"), -1).reshape(-1, 3)
    pos = ((cells[:, None, :] + basis[None, :, :]).reshape(-1, 3) * DIAMOND_A).astype(np.float64)
    n_atoms = pos.shape[0]
    L = n_cells * DIAMOND_A
    g = max(1, int(L // 2.0))
    cell = np.minimum((pos / (L / g)).astype(np.int64), g - 1)
    order = np.lexsort((np.arange(n_atoms), _morton3(cell[:, 0], cell[:, 1], cell[:, 2])))
    pos = np.ascontiguousarray(pos[order])
    n_orb = np.full(n_atoms, 4, dtype=np.int8)
    orb_off = np.arange(n_atoms + 1, dtype=np.int64) * 4
    cnt = np.zeros(n_atoms, dtype=np.int64)
    if lib.count_pairs(n_atoms, _ptr(pos), L, r_cut, _ptr(cnt)) != 0:
        raise RuntimeError("count_pairs failed")
    off = np.zeros(n_atoms + 1, dtype=np.int64)
    np.cumsum(cnt, out=off[1:])
    npair = int(off[-1])
    pj = np.zeros(npair, dtype=np.int32)
    pr = np.zeros(npair, dtype=np.float64)
    pd = np.zeros((npair, 3), dtype=np.float64)
    if lib.fill_pairs(n_atoms, _ptr(pos), L, r_cut, _ptr(off), _ptr(pj), _ptr(pr), _ptr(pd)) != 0:
        raise RuntimeError("fill_pairs failed")
    pi = np.repeat(np.arange(n_atoms, dtype=np.int32), cnt)
    rngA = np.random.Generator(np.random.PCG64(seed + 1))
    rngB = np.random.Generator(np.random.PCG64(seed + 2))
    FA = rngA.normal(1.0, 0.1, size=(4, 4))
    FA = 0.5 * (FA + FA.T)
    site = rngA.normal(1.0, 0.1, size=4)
    FB = rngB.normal(1.0, 0.1, size=(4, 4))
    FB = 0.5 * (FB + FB.T)
    decay = np.exp(-pr / DECAY)
    blkA = FA[None, :, :] * decay[:, None, None]
    blkB = b_scale * FB[None, :, :] * decay[:, None, None]
    sysm = _assemble(n_atoms, n_atoms, L, pos, n_orb, orb_off, pi, pj, blkA, blkB,
                     np.broadcast_to(site, (n_atoms, 4)), seed)
    sysm.extra["pairs"] = (pi, pj, pr, pd)
    sysm.extra["lattice"] = "diamond"
    return sysm


def shift_grid(n_shifts: int, lo: float = -1.0, hi: float = 1.0, eta: float = 0.01) -> np.ndarray:
    """Midpoint grid eps_k = lo + (k + 1/2)(hi - lo)/K with Im z = eta; complex128."""
    k = np.arange(n_shifts, dtype=np.float64)
    eps = lo + (k + 0.5) * (hi - lo) / n_shifts
    return eps + 1j * eta


def sample_columns(sysm: System, n_cols: int, seed: int) -> np.ndarray:
    """Distinct columns sampled uniformly without replacement, sorted."""
    rng = np.random.Generator(np.random.PCG64(seed + 4))
    n_cols = min(n_cols, sysm.M)
    return np.sort(rng.choice(sysm.M, size=n_cols, replace=False)).astype(np.int32)


def sample_regions(sysm: System, n_regions: int, seed: int, r_lo: float = 6.0,
                   r_hi: float = 14.0) -> tuple[np.ndarray, np.ndarray]:
    """Region centres (distinct atoms, sorted) and radii U[r_lo, r_hi] A."""
    rng = np.random.Generator(np.random.PCG64(seed + 3))
    n_regions = min(n_regions, sysm.n_atoms)
    centres = np.sort(rng.choice(sysm.n_atoms, size=n_regions, replace=False)).astype(np.int32)
    radii = rng.uniform(r_lo, r_hi, size=n_regions)
    return centres, radii


def column_regions(sysm: System, cols: np.ndarray, seed: int, r_lo: float = 6.0,
                   r_hi: float = 14.0) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Regions of sampled columns: one region per atom that carries a sampled
    column, centred on that atom (ascending), with the sampled orbitals of the
    atom as its columns (bit q of the mask = orbital q) and a radius U[r_lo, r_hi]
    A drawn per region from the region stream (seed + 3)."""
    cols = np.asarray(cols, dtype=np.int64)
    atom = np.searchsorted(sysm.orb_off, cols, side="right") - 1
    centres = np.unique(atom)
    mask = np.zeros(centres.size, dtype=np.uint8)
    where = np.searchsorted(centres, atom)
    np.bitwise_or.at(mask, where, (1 << (cols - sysm.orb_off[atom])).astype(np.uint8))
    rng = np.random.Generator(np.random.PCG64(seed + 3))
    radii = rng.uniform(r_lo, r_hi, size=centres.size)
    return centres.astype(np.int32), mask, radii


def kappa_radii(sysm: System, centres: np.ndarray, kappa: int) -> np.ndarray:
    """Radius of each centre's sphere that holds its kappa nearest atoms (the
    centre included; minimum-image distances): the midpoint between the
    kappa-th and (kappa+1)-th nearest distances, so the sphere holds exactly
    kappa atoms unless distances tie (then the whole tied shell: kappa or more).  Cell lists (side >= 1.25 x the radius
    that kappa + 1 atoms need at the mean density) keep this linear in the
    number of centres; a centre whose (kappa+1)-th neighbour is not surely
    inside its 27 cells falls back to all atoms."""
    centres = np.asarray(centres, dtype=np.int64)
    L = float(sysm.L)
    pos = np.mod(sysm.pos, L)
    dens = sysm.n_atoms / L ** 3
    r_need = (3.0 * (kappa + 1) / (4.0 * np.pi * dens)) ** (1.0 / 3.0)
    nc = int(L // (1.25 * r_need))
    out = np.empty(centres.size)

    def kth(cidx, cand):
        d = pos[cand][None, :, :] - pos[cidx][:, None, :]
        d -= L * np.rint(d / L)
        r = np.sqrt((d * d).sum(-1))
        part = np.partition(r, (kappa - 1, kappa), axis=1)
        return part[:, kappa - 1], part[:, kappa]

    if nc < 3 or sysm.n_atoms <= kappa + 1:
        for i0 in range(0, centres.size, 256):
            a, b = kth(centres[i0:i0 + 256], np.arange(sysm.n_atoms))
            out[i0:i0 + 256] = _kappa_cut(a, b)
        return out
    side = L / nc
    cell = np.minimum((pos / side).astype(np.int64), nc - 1)
    key = (cell[:, 0] * nc + cell[:, 1]) * nc + cell[:, 2]
    order = np.argsort(key, kind="stable")
    start = np.searchsorted(key[order], np.arange(nc ** 3 + 1))
    ckey = key[centres]
    for k in np.unique(ckey):
        sel = np.nonzero(ckey == k)[0]
        cx, cy, cz = k // (nc * nc), (k // nc) % nc, k % nc
        ids = [order[start[q]:start[q + 1]]
               for q in ((((cx + dx) % nc) * nc + (cy + dy) % nc) * nc + (cz + dz) % nc
                         for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1))]
        cand = np.concatenate(ids)
        if cand.size > kappa:
            a, b = kth(centres[sel], cand)
        else:
            a = b = np.full(sel.size, np.inf)
        bad = ~(b <= side)  # beyond one cell side the 27 cells may miss nearer atoms
        if bad.any():
            a2, b2 = kth(centres[sel[bad]], np.arange(sysm.n_atoms))
            a[bad], b[bad] = a2, b2
        out[sel] = _kappa_cut(a, b)
    return out


def _kappa_cut(a, b):
    """Midpoint of the kappa-th and (kappa+1)-th distances; when they tie (a
    crystal shell) the whole shell is taken, robustly against rounding."""
    return np.where(b - a > 1e-9, 0.5 * (a + b), b + 1e-9)


def config_seed(cfg_index: int) -> int:
    """Base seed of configuration i (1-based): 1000 + i."""
    return 1000 + cfg_index


# The five workloads (sizes only; the values come from make_system).
CONFIGS = {
    "c1": dict(n_atoms=128, n_shifts=32, mode="global", columns="all"),
    "c2": dict(n_atoms=4096, n_shifts=64, mode="global", columns="all"),
    "c3": dict(n_atoms=50000, n_shifts=64, mode="region", n_regions=2048),
    "c4": dict(n_atoms=100000, n_shifts=64, mode="region", n_columns=16384),
    "c5": dict(n_atoms=1000000, n_shifts=128, mode="region", n_columns=65536),
}
