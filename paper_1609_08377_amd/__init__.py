"""Python binding of libelses.so, the gfx950 generalized shifted Krylov solver.

Argument marshalling only: every step of a solve runs in the HIP kernels of
the library.  PyTorch provides device memory (output tensors) and the HIP
stream.  The entry points mirror the C ABI in include/elses.h:

    Context(device=0, stream=None)
    Matrix(ctx, n_orb, blk_row_ptr, blk_col, A_val, B_val, pos=None, box=0.0, precision="fp64")
    shifted_solve(ctx, mat, cols, shifts, ...)     -> dict(x, iters, resid, pat_off)
    density_matrix(ctx, mat, cols, shifts, c, ...) -> dict(rho, traces, col_traces, ...)
    pattern(mat, cols)                             -> (pat_off, rows)
    spmm(ctx, mat, which, x)                       -> y = A x or B x

The library must have been built (python -m paper_1609_08377_amd.build);
importing the binding without it raises ImportError: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libelses.so")

ELSES_OK = 0
ELSES_ERR_INVALID_ARG = 1
ELSES_ERR_HIP = 2
ELSES_ERR_OOM = 3
ELSES_ERR_NOT_SPD = 4
ELSES_WARN_NOT_CONVERGED = 5
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "HIP", 3: "OOM", 4: "NOT_SPD", 5: "NOT_CONVERGED"}

ELSES_FP64 = 0
ELSES_MIXED = 1
ELSES_OUT_PATTERN = 0
ELSES_OUT_FULL = 1


class ElsesError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"elses {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class NotConverged(ElsesError):
    pass


class _System(ctypes.Structure):
    _fields_ = [("n_atoms", ctypes.c_int32), ("n_orb", ctypes.c_void_p), ("blk_row_ptr", ctypes.c_void_p),
                ("blk_col", ctypes.c_void_p), ("A_val", ctypes.c_void_p), ("B_val", ctypes.c_void_p),
                ("pos", ctypes.c_void_p), ("box", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_outer", ctypes.c_int32), ("inner_tol", ctypes.c_double),
                ("out_mode", ctypes.c_int32), ("slots", ctypes.c_int32), ("use_mixed", ctypes.c_int32),
                ("audit", ctypes.c_int32), ("variant", ctypes.c_int32), ("graph", ctypes.c_int32),
                ("audit_every", ctypes.c_int32), ("precond", ctypes.c_int32), ("inner_max", ctypes.c_int32)]


class ArnoldiOpts(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_int32), ("variant", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("mu", ctypes.c_double), ("kT", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1609_08377_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        L.elses_version.restype = ctypes.c_char_p
        L.elses_ctx_create.argtypes = [ctypes.c_int, P, ctypes.POINTER(P)]
        L.elses_ctx_create.restype = ctypes.c_int
        L.elses_ctx_destroy.argtypes = [P]
        L.elses_ctx_destroy.restype = None
        L.elses_last_error.argtypes = [P]
        L.elses_last_error.restype = ctypes.c_char_p
        L.elses_mat_create.argtypes = [P, ctypes.POINTER(_System), ctypes.c_int, ctypes.POINTER(P)]
        L.elses_mat_create.restype = ctypes.c_int
        L.elses_mat_destroy.argtypes = [P]
        L.elses_mat_destroy.restype = None
        L.elses_mat_info.argtypes = [P, P, P, P, P]
        L.elses_mat_info.restype = ctypes.c_int
        L.elses_pattern.argtypes = [P, I32, P, P, P]
        L.elses_pattern.restype = ctypes.c_int
        L.elses_opts_default.argtypes = [ctypes.POINTER(Opts)]
        L.elses_opts_default.restype = None
        L.elses_shifted_solve.argtypes = [P, P, I32, P, I32, P, ctypes.POINTER(Opts), P, P, P]
        L.elses_shifted_solve.restype = ctypes.c_int
        L.elses_density_matrix.argtypes = [P, P, I32, P, I32, P, P, ctypes.POINTER(Opts), P, P, P, P, P, P]
        L.elses_density_matrix.restype = ctypes.c_int
        L.elses_spmm.argtypes = [P, P, ctypes.c_int, I32, I32, P, P]
        L.elses_spmm.restype = ctypes.c_int
        L.elses_spmm32.argtypes = [P, P, ctypes.c_int, I32, I32, P, P]
        L.elses_spmm32.restype = ctypes.c_int
        L.elses_spai_pairs.argtypes = [P, P, P]
        L.elses_spai_features.argtypes = [P, P, P]
        L.elses_spai_targets.argtypes = [P, P, P, P]
        L.elses_mlp_loss_grad.argtypes = [P, P, ctypes.c_int64, P, P, P, P, P]
        L.elses_spai_train.argtypes = [P, P, ctypes.c_int64, P, P, P, I32, I32, ctypes.c_double, ctypes.c_uint64, P]
        L.elses_spai_predict.argtypes = [P, P, ctypes.c_int64, P, I32, P]
        L.elses_spai_apply.argtypes = [P, P, P, I32, P]
        L.elses_overlap_solve.argtypes = [P, P, P, ctypes.c_double, I32, P, P, P, P, P]
        for fn in ("elses_spai_pairs", "elses_spai_features", "elses_spai_targets", "elses_mlp_loss_grad",
                   "elses_spai_train", "elses_spai_predict", "elses_spai_apply", "elses_overlap_solve"):
            getattr(L, fn).restype = ctypes.c_int
        L.elses_pattern_blocks.argtypes = [P, I32, P, P, P]
        L.elses_pattern_blocks.restype = ctypes.c_int
        L.elses_density_reweight.argtypes = [P, P, I32, P, I32, P, P, P, P, P, P]
        L.elses_density_reweight.restype = ctypes.c_int
        L.elses_chemical_potential.argtypes = [P, P, I32, P, I32, P, P, P, D, D, D, D, D, P, P]
        L.elses_chemical_potential.restype = ctypes.c_int
        L.elses_autotune.argtypes = [P, P, I32, I32, P, P, P]
        L.elses_autotune.restype = ctypes.c_int
        L.elses_regions_create.argtypes = [P, P, I32, P, P, I32, ctypes.POINTER(P)]
        L.elses_regions_create.restype = ctypes.c_int
        L.elses_regions_create_ex.argtypes = [P, P, I32, P, P, P, I32, ctypes.POINTER(P)]
        L.elses_regions_create_ex.restype = ctypes.c_int
        L.elses_regions_columns.argtypes = [P, P]
        L.elses_regions_columns.restype = ctypes.c_int
        L.elses_regions_overlap_intervals.argtypes = [P, P, P]
        L.elses_regions_overlap_intervals.restype = ctypes.c_int
        L.elses_ctx_region_idle.argtypes = [P, P, P]
        L.elses_ctx_region_idle.restype = ctypes.c_int
        L.elses_mat_set_preconditioner.argtypes = [P, P, P, I32]
        L.elses_mat_set_preconditioner.restype = ctypes.c_int
        L.elses_ctx_solve_counts.argtypes = [P, P, P]
        L.elses_ctx_solve_counts.restype = ctypes.c_int
        L.elses_regions_destroy.argtypes = [P]
        L.elses_regions_destroy.restype = None
        L.elses_regions_info.argtypes = [P, P, P, P, P, P, P, P]
        L.elses_regions_info.restype = ctypes.c_int
        L.elses_regions_solve.argtypes = [P, P, I32, P, P, ctypes.POINTER(Opts), P, P, P, P, P, P]
        L.elses_regions_solve.restype = ctypes.c_int
        L.elses_regions_solve_noalloc.argtypes = [P, P, I32, P, P, ctypes.POINTER(Opts), P, P, P, P, P, P]
        L.elses_regions_solve_noalloc.restype = ctypes.c_int
        L.elses_arnoldi_opts_default.argtypes = [ctypes.POINTER(ArnoldiOpts)]
        L.elses_arnoldi_opts_default.restype = None
        L.elses_arnoldi.argtypes = [P, P, I32, P, ctypes.POINTER(ArnoldiOpts), P, P, P, P, P, P, P]
        L.elses_arnoldi.restype = ctypes.c_int
        L.elses_regions_arnoldi.argtypes = [P, P, ctypes.POINTER(ArnoldiOpts), P, P, P, P, P, P, P]
        L.elses_regions_arnoldi.restype = ctypes.c_int
        _lib = L
    return _lib


def version() -> str:
    return lib().elses_version().decode()


def _np_ptr(a):
    return None if a is None else a.ctypes.data


def _dev_ptr(t):
    return None if t is None else t.data_ptr()


def _torch():
    import torch
    return torch


class Context:
    """A device + HIP stream; defaults to torch's current stream on `device`."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        self.device = device
        with torch.cuda.device(device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = ctypes.c_void_p()
        st = lib().elses_ctx_create(device, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != ELSES_OK:
            raise ElsesError(st, "context creation failed")
        self._h = h

    def last_error(self) -> str:
        return lib().elses_last_error(self._h).decode()

    def check(self, st: int, allow_warn: bool = False):
        if st == ELSES_OK:
            return
        if st == ELSES_WARN_NOT_CONVERGED:
            if allow_warn:
                return
            raise NotConverged(st, self.last_error())
        raise ElsesError(st, self.last_error())

    def close(self):
        if getattr(self, "_h", None):
            lib().elses_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Matrix:
    """Device copy of one (A, B) pencil in atom-block form (see include/elses.h)."""

    def __init__(self, ctx: Context, n_orb, blk_row_ptr, blk_col, A_val, B_val, pos=None, box: float = 0.0,
                 precision: str = "fp64"):
        self.ctx = ctx
        self._keep = [np.ascontiguousarray(n_orb, dtype=np.int8), np.ascontiguousarray(blk_row_ptr, np.int64),
                      np.ascontiguousarray(blk_col, np.int32), np.ascontiguousarray(A_val, np.float64),
                      np.ascontiguousarray(B_val, np.float64),
                      None if pos is None else np.ascontiguousarray(pos, np.float64).reshape(-1)]
        no, rp, bc, av, bv, ps = self._keep
        sysd = _System(int(no.shape[0]), _np_ptr(no), _np_ptr(rp), _np_ptr(bc), _np_ptr(av), _np_ptr(bv),
                       _np_ptr(ps), float(box))
        prec = {"fp64": ELSES_FP64, "mixed": ELSES_MIXED}[precision]
        h = ctypes.c_void_p()
        st = lib().elses_mat_create(ctx._h, ctypes.byref(sysd), prec, ctypes.byref(h))
        ctx.check(st)
        self._h = h
        self.precision = precision
        M = ctypes.c_int64()
        pmax = ctypes.c_int64()
        lo = ctypes.c_double()
        hi = ctypes.c_double()
        lib().elses_mat_info(h, ctypes.byref(M), ctypes.byref(pmax), ctypes.byref(lo), ctypes.byref(hi))
        self.M = int(M.value)
        self.nnz = int(av.shape[0])  # values of A (and B): every block n_I x n_J
        self.pmax = int(pmax.value)
        self.b_interval = (lo.value, hi.value)
        self._keep = None

    @classmethod
    def from_system(cls, ctx: Context, sysm, precision: str = "fp64") -> "Matrix":
        return cls(ctx, sysm.n_orb, sysm.blk_row_ptr, sysm.blk_col, sysm.A_val, sysm.B_val, pos=sysm.pos,
                   box=sysm.L, precision=precision)

    def close(self):
        if getattr(self, "_h", None):
            lib().elses_mat_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pattern(mat: Matrix, cols) -> tuple[np.ndarray, np.ndarray]:
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    off = np.zeros(cols.shape[0] + 1, dtype=np.int64)
    mat.ctx.check(lib().elses_pattern(mat._h, cols.shape[0], _np_ptr(cols), _np_ptr(off), None))
    rows = np.zeros(int(off[-1]), dtype=np.int32)
    mat.ctx.check(lib().elses_pattern(mat._h, cols.shape[0], _np_ptr(cols), _np_ptr(off), _np_ptr(rows)))
    return off, rows


VARIANTS = {"auto": 0, "direct": 1, "staged": 2, "staged8": 2, "staged4": 3, "grouped": 4, "grouped4": 4,
            "grouped2": 5, "grouped1": 6}


def _variant(v) -> int:
    """A variant name, or an int holding the variant and its placement / column bits."""
    return VARIANTS[v] if isinstance(v, str) else int(v)


def make_opts(tol=1e-8, max_outer=20000, inner_tol=1e-13, full=False, slots=0, mixed=False, audit=False,
              variant="auto", graph=False, precond=False) -> Opts:
    o = Opts()
    lib().elses_opts_default(ctypes.byref(o))
    o.tol = tol
    o.max_outer = max_outer
    o.inner_tol = inner_tol
    o.out_mode = ELSES_OUT_FULL if full else ELSES_OUT_PATTERN
    o.slots = slots
    o.use_mixed = 1 if mixed else 0
    o.audit = 1 if audit else 0
    o.variant = _variant(variant)
    o.graph = 1 if graph else 0
    o.precond = 1 if precond else 0
    return o


def _shifts_ri(shifts) -> np.ndarray:
    z = np.asarray(shifts, dtype=np.complex128)
    return np.ascontiguousarray(np.stack([z.real, z.imag], axis=1).reshape(-1))


def shifted_solve(ctx: Context, mat: Matrix, cols, shifts, *, tol=1e-8, max_outer=20000, inner_tol=1e-13,
                  full=False, slots=0, mixed=False, audit=False, want_x=True, allow_not_converged=False,
                  variant="auto", graph=False, precond=False):
    """(z_k B - A) x = e_j for j in cols and every shift; returns torch tensors on the device."""
    torch = _torch()
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    z = _shifts_ri(shifts)
    K = z.shape[0] // 2
    nc = cols.shape[0]
    dev = torch.device("cuda", ctx.device)
    if full:
        pat_off = None
        nx = nc * K * mat.M
    else:
        pat_off, _ = pattern(mat, cols)
        nx = int(pat_off[-1]) * K
    x = torch.empty(2 * nx, dtype=torch.float64, device=dev) if want_x else None
    iters = torch.empty(nc, dtype=torch.int32, device=dev)
    resid = torch.empty(nc * K, dtype=torch.float64, device=dev)
    opts = make_opts(tol, max_outer, inner_tol, full, slots, mixed, audit, variant, graph, precond)
    st = lib().elses_shifted_solve(ctx._h, mat._h, nc, _np_ptr(cols), K, _np_ptr(z), ctypes.byref(opts),
                                   _dev_ptr(x), _dev_ptr(iters), _dev_ptr(resid))
    ctx.check(st, allow_warn=allow_not_converged)
    xc = None
    if x is not None:
        xc = torch.view_as_complex(x.view(-1, 2))
        if full:
            xc = xc.view(nc, K, mat.M)
    return dict(x=xc, iters=iters, resid=resid.view(nc, K), pat_off=pat_off, status=st)


def density_matrix(ctx: Context, mat: Matrix, cols, shifts, c, *, tol=1e-8, max_outer=20000, inner_tol=1e-13,
                   slots=0, mixed=False, want_x=False, allow_not_converged=False, variant="auto", graph=False,
                   precond=False):
    """rho_ij = sum_k Im(c_k x_{j,k,i}) on the pattern, plus the traces Tr[rho B], Tr[rho A] over cols."""
    torch = _torch()
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    z = _shifts_ri(shifts)
    cw = _shifts_ri(c)
    K = z.shape[0] // 2
    if cw.shape[0] != 2 * K:
        raise ValueError("one weight per shift")
    nc = cols.shape[0]
    dev = torch.device("cuda", ctx.device)
    pat_off, _ = pattern(mat, cols)
    rho = torch.empty(int(pat_off[-1]), dtype=torch.float64, device=dev)
    col_tr = torch.empty(2 * nc, dtype=torch.float64, device=dev)
    x = torch.empty(2 * int(pat_off[-1]) * K, dtype=torch.float64, device=dev) if want_x else None
    iters = torch.empty(nc, dtype=torch.int32, device=dev)
    resid = torch.empty(nc * K, dtype=torch.float64, device=dev)
    traces = np.zeros(2)
    opts = make_opts(tol, max_outer, inner_tol, False, slots, mixed, False, variant, graph, precond)
    st = lib().elses_density_matrix(ctx._h, mat._h, nc, _np_ptr(cols), K, _np_ptr(z), _np_ptr(cw),
                                    ctypes.byref(opts), _dev_ptr(rho), _np_ptr(traces), _dev_ptr(col_tr),
                                    _dev_ptr(x), _dev_ptr(iters), _dev_ptr(resid))
    ctx.check(st, allow_warn=allow_not_converged)
    return dict(rho=rho, traces=traces, col_traces=col_tr.view(nc, 2), pat_off=pat_off, iters=iters,
                resid=resid.view(nc, K), x=None if x is None else torch.view_as_complex(x.view(-1, 2)), status=st)


def spmm(ctx: Context, mat: Matrix, which: str, x, variant: str = "auto"):
    """y = A x or B x for x a float64 device tensor of shape (M, nvec)."""
    torch = _torch()
    x = x.contiguous()
    y = torch.empty_like(x)
    nvec = 1 if x.dim() == 1 else x.shape[1]
    st = lib().elses_spmm(ctx._h, mat._h, {"A": 0, "B": 1}[which], _variant(variant), nvec, _dev_ptr(x),
                          _dev_ptr(y))
    ctx.check(st)
    return y


def spmm32(ctx: Context, mat: Matrix, which: str, x, variant: str = "auto"):
    """y = fl32(A) x or fl32(B) x in FP32 for x a float32 device tensor (M, nvec), nvec % 64 == 0."""
    torch = _torch()
    if x.dtype != torch.float32 or x.dim() != 2:
        raise ValueError("x must be a float32 (M, nvec) tensor")
    x = x.contiguous()
    y = torch.empty_like(x)
    st = lib().elses_spmm32(ctx._h, mat._h, {"A": 0, "B": 1}[which], _variant(variant), x.shape[1], _dev_ptr(x),
                            _dev_ptr(y))
    ctx.check(st)
    return y


class Regions:
    """Region problems (principal sub-pencils around centre atoms) on the device: the compact layout
    (tile_width 0, one persistent launch) or tiles of 64 / 128 column slots.  orb_mask (one uint8 per
    region) selects the centre's orbitals solved as columns (0 = all)."""

    def __init__(self, ctx: Context, mat: Matrix, centres, radii, tile_width: int = 0, orb_mask=None):
        self.ctx = ctx
        self.mat = mat
        centres = np.ascontiguousarray(centres, dtype=np.int32)
        radii = np.ascontiguousarray(radii, dtype=np.float64)
        if centres.shape != radii.shape:
            raise ValueError("one radius per centre")
        h = ctypes.c_void_p()
        if orb_mask is not None:
            mask = np.ascontiguousarray(orb_mask, dtype=np.uint8)
            if mask.shape != centres.shape:
                raise ValueError("one orbital mask per centre")
            st = lib().elses_regions_create_ex(ctx._h, mat._h, int(centres.shape[0]), _np_ptr(centres),
                                               _np_ptr(radii), _np_ptr(mask), int(tile_width), ctypes.byref(h))
        else:
            st = lib().elses_regions_create(ctx._h, mat._h, int(centres.shape[0]), _np_ptr(centres),
                                            _np_ptr(radii), int(tile_width), ctypes.byref(h))
        ctx.check(st)
        self._h = h
        self.compact = (tile_width == 0)
        nc, nt = ctypes.c_int32(), ctypes.c_int32()
        rows, useful = ctypes.c_int64(), ctypes.c_int64()
        lib().elses_regions_info(h, ctypes.byref(nc), ctypes.byref(nt), ctypes.byref(rows), ctypes.byref(useful),
                                 None, None, None)
        self.n_cols = int(nc.value)
        self.n_tiles = int(nt.value)
        self.rows_total = int(rows.value)
        self.useful_rows = int(useful.value)
        self.cols = np.zeros(self.n_cols, dtype=np.int32)
        self.pat_off = np.zeros(self.n_cols + 1, dtype=np.int64)
        self.region_orbitals = np.zeros(centres.shape[0], dtype=np.int32)
        lib().elses_regions_info(h, None, None, None, None, _np_ptr(self.cols), _np_ptr(self.pat_off),
                                 _np_ptr(self.region_orbitals))
        self.col_region = np.zeros(self.n_cols, dtype=np.int32)
        ctx.check(lib().elses_regions_columns(h, _np_ptr(self.col_region)))
        # first entry of each column's block of full region vectors ([K][m_r] per column)
        self.full_off = np.concatenate([[0], np.cumsum(self.region_orbitals[self.col_region].astype(np.int64))])

    def overlap_intervals(self):
        """(lo, hi) per region of a compact set: the overlap interval its Richardson plan uses."""
        lo = np.zeros(self.region_orbitals.shape[0])
        hi = np.zeros_like(lo)
        self.ctx.check(lib().elses_regions_overlap_intervals(self._h, _np_ptr(lo), _np_ptr(hi)))
        return lo, hi

    def close(self):
        if getattr(self, "_h", None):
            lib().elses_regions_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_preconditioner(ctx: Context, mat: Matrix, params=None, bf16: bool = True):
    """Keep the learned M (network params: FP32 device tensor, or None to remove it) with the matrix."""
    ctx.check(lib().elses_mat_set_preconditioner(ctx._h, mat._h, _dev_ptr(params), 1 if bf16 else 0))


def region_idle(ctx: Context) -> tuple[float, int]:
    """(mean idle share of resident workgroups, profiled compact solves measured) since profiling was set."""
    v, n = ctypes.c_double(), ctypes.c_int64()
    ctx.check(lib().elses_ctx_region_idle(ctx._h, ctypes.byref(v), ctypes.byref(n)))
    return float(v.value), int(n.value)


def solve_counts(ctx: Context) -> tuple[int, int]:
    """(sparse products, preconditioner fallbacks) of the last compact region solve."""
    p, f = ctypes.c_int64(), ctypes.c_int64()
    ctx.check(lib().elses_ctx_solve_counts(ctx._h, ctypes.byref(p), ctypes.byref(f)))
    return int(p.value), int(f.value)


def region_solve(ctx: Context, reg: Regions, shifts, c=None, *, tol=1e-8, max_outer=20000, inner_tol=1e-13,
                 mixed=False, want_x=True, allow_not_converged=False, variant="auto", graph=False, full=False,
                 audit=False, audit_every=0, precond=False, inner_max=200, noalloc=False):
    """Solve every region's columns for every shift; density outputs when weights c are given.

    Compact region sets also take full=True (x holds, per column, the [K][m_r] vectors of its region in
    the region's orbital order, offsets reg.full_off), audit=True (with full: resid = FP64 true residuals)
    and audit_every=n (pattern mode: the columns c % n == 0 get their true residual in resid)."""
    torch = _torch()
    z = _shifts_ri(shifts)
    K = z.shape[0] // 2
    cw = None if c is None else _shifts_ri(c)
    if cw is not None and cw.shape[0] != 2 * K:
        raise ValueError("one weight per shift")
    nc = reg.n_cols
    npat = int(reg.pat_off[-1])
    dev = torch.device("cuda", ctx.device)
    nx = int(reg.full_off[-1]) * K if full else npat * K
    x = torch.empty(2 * nx, dtype=torch.float64, device=dev) if want_x else None
    rho = torch.empty(npat, dtype=torch.float64, device=dev) if cw is not None else None
    col_tr = torch.empty(2 * nc, dtype=torch.float64, device=dev) if cw is not None else None
    iters = torch.empty(nc, dtype=torch.int32, device=dev)
    resid = torch.empty(nc * K, dtype=torch.float64, device=dev)
    traces = np.zeros(2)
    opts = make_opts(tol, max_outer, inner_tol, full, 0, mixed, audit, variant, graph)
    opts.audit_every = int(audit_every)
    opts.precond = 1 if precond else 0
    opts.inner_max = int(inner_max)
    fn = lib().elses_regions_solve_noalloc if noalloc else lib().elses_regions_solve
    st = fn(ctx._h, reg._h, K, _np_ptr(z), None if cw is None else _np_ptr(cw),
                                   ctypes.byref(opts), _dev_ptr(x), _dev_ptr(rho),
                                   None if cw is None else _np_ptr(traces), _dev_ptr(col_tr), _dev_ptr(iters),
                                   _dev_ptr(resid))
    ctx.check(st, allow_warn=allow_not_converged)
    return dict(x=None if x is None else torch.view_as_complex(x.view(-1, 2)), rho=rho,
                traces=traces if cw is not None else None,
                col_traces=None if col_tr is None else col_tr.view(nc, 2), iters=iters, resid=resid.view(nc, K),
                pat_off=reg.pat_off, cols=reg.cols, status=st)


# ---------------------------------------------------------------------------
# Learned SPAI of the overlap
# ---------------------------------------------------------------------------
MLP_PARAMS = 40336
MLP_SHAPES = [(128, 40), (128,), (128, 128), (128,), (128, 128), (128,), (16, 128), (16,)]


def mlp_init(seed: int) -> np.ndarray:
    """Seeded initial parameters of the network (FP64 host array in the library's parameter
    order): weights uniform in +-sqrt(6 / (fan_in + fan_out)), biases zero."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for sh in MLP_SHAPES:
        if len(sh) == 2:
            lim = np.sqrt(6.0 / (sh[0] + sh[1]))
            parts.append(rng.uniform(-lim, lim, size=sh).ravel())
        else:
            parts.append(np.zeros(sh))
    return np.concatenate(parts)


def spai_pairs(mat: Matrix) -> np.ndarray:
    n = ctypes.c_int64()
    lib().elses_spai_pairs(mat._h, ctypes.byref(n), None)
    out = np.zeros((n.value, 2), dtype=np.int32)
    lib().elses_spai_pairs(mat._h, ctypes.byref(n), _np_ptr(out))
    return out


def spai_features(ctx: Context, mat: Matrix):
    torch = _torch()
    n = spai_pairs(mat).shape[0]
    f = torch.empty((n, 40), dtype=torch.float32, device=torch.device("cuda", ctx.device))
    ctx.check(lib().elses_spai_features(ctx._h, mat._h, _dev_ptr(f)))
    return f


def spai_targets(ctx: Context, mat: Matrix):
    torch = _torch()
    n = spai_pairs(mat).shape[0]
    dev = torch.device("cuda", ctx.device)
    t = torch.zeros((n, 16), dtype=torch.float32, device=dev)
    m = torch.zeros((n, 16), dtype=torch.float32, device=dev)
    ctx.check(lib().elses_spai_targets(ctx._h, mat._h, _dev_ptr(t), _dev_ptr(m)))
    return t, m


def mlp_loss_grad(ctx: Context, params, feat, target, mask):
    torch = _torch()
    g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=params.device)
    loss = ctypes.c_double()
    ctx.check(lib().elses_mlp_loss_grad(ctx._h, _dev_ptr(params), feat.shape[0], _dev_ptr(feat), _dev_ptr(target),
                                        _dev_ptr(mask), ctypes.byref(loss), _dev_ptr(g)))
    return loss.value, g


def spai_train(ctx: Context, params, feat, target, mask, steps: int, batch: int = 4096, lr: float = 1e-3,
               seed: int = 0):
    hist = np.zeros(steps)
    ctx.check(lib().elses_spai_train(ctx._h, _dev_ptr(params), feat.shape[0], _dev_ptr(feat), _dev_ptr(target),
                                     _dev_ptr(mask), steps, batch, lr, seed, _np_ptr(hist)))
    return hist


def spai_predict(ctx: Context, params, feat, bf16: bool = False):
    torch = _torch()
    out = torch.empty((feat.shape[0], 16), dtype=torch.float32, device=feat.device)
    ctx.check(lib().elses_spai_predict(ctx._h, _dev_ptr(params), feat.shape[0], _dev_ptr(feat), 1 if bf16 else 0,
                                       _dev_ptr(out)))
    return out


def spai_apply(ctx: Context, mat: Matrix, params, bf16: bool = True):
    """Device buffer of M on B's pattern (opaque internal order) for overlap_solve."""
    torch = _torch()
    n = mat.nnz
    mv = torch.zeros(n, dtype=torch.float64, device=params.device)
    ctx.check(lib().elses_spai_apply(ctx._h, mat._h, _dev_ptr(params), 1 if bf16 else 0, _dev_ptr(mv)))
    return mv


def overlap_solve(ctx: Context, mat: Matrix, s, M_vals=None, tol: float = 1e-13):
    """x = B^{-1} s for s a float64 (M, nvec) device tensor; returns (x, passes, bracket, used_precond)."""
    torch = _torch()
    s = s.contiguous()
    x = torch.empty_like(s)
    passes, used = ctypes.c_int32(), ctypes.c_int32()
    br = np.zeros(2)
    ctx.check(lib().elses_overlap_solve(ctx._h, mat._h, _dev_ptr(M_vals), tol, s.shape[1], _dev_ptr(s), _dev_ptr(x),
                                        ctypes.byref(passes), _np_ptr(br), ctypes.byref(used)))
    return x, passes.value, tuple(br), bool(used.value)


def autotune(ctx: Context, mat: Matrix, mixed: bool = False, max_slots: int = 0):
    """Time the pass configurations and keep the fastest per column in `mat`; returns (variant, slots, ns/col)."""
    v, sl, ns = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
    ctx.check(lib().elses_autotune(ctx._h, mat._h, 1 if mixed else 0, max_slots, ctypes.byref(v), ctypes.byref(sl),
                                   ctypes.byref(ns)))
    return v.value, sl.value, ns.value


# ---------------------------------------------------------------------------
# Observables from stored solutions
# ---------------------------------------------------------------------------
def pattern_blocks(mat: Matrix, cols):
    """(blk_off, blk_atom): coupled-atom blocks of each column's pattern."""
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    off = np.zeros(cols.shape[0] + 1, dtype=np.int64)
    lib().elses_pattern_blocks(mat._h, cols.shape[0], _np_ptr(cols), _np_ptr(off), None)
    atoms = np.zeros(int(off[-1]), dtype=np.int32)
    lib().elses_pattern_blocks(mat._h, cols.shape[0], _np_ptr(cols), _np_ptr(off), _np_ptr(atoms))
    return off, atoms


def density_reweight(ctx: Context, mat: Matrix, cols, c, x):
    """rho, traces, per-column traces and per-(column, coupled atom) ICOHP for weights c from stored x."""
    torch = _torch()
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    cw = _shifts_ri(c)
    K = cw.shape[0] // 2
    pat_off, _ = pattern(mat, cols)
    blk_off, blk_atom = pattern_blocks(mat, cols)
    dev = x.device
    rho = torch.empty(int(pat_off[-1]), dtype=torch.float64, device=dev)
    ctr = torch.empty(2 * cols.shape[0], dtype=torch.float64, device=dev)
    ic = torch.empty(int(blk_off[-1]), dtype=torch.float64, device=dev)
    tr = np.zeros(2)
    xr = torch.view_as_real(x).contiguous() if x.is_complex() else x
    ctx.check(lib().elses_density_reweight(ctx._h, mat._h, cols.shape[0], _np_ptr(cols), K, _np_ptr(cw),
                                           _dev_ptr(xr), _dev_ptr(rho), _np_ptr(tr), _dev_ptr(ctr), _dev_ptr(ic)))
    return dict(rho=rho, traces=tr, col_traces=ctr.view(-1, 2), icohp=ic, blk_off=blk_off, blk_atom=blk_atom)


def chemical_potential(ctx: Context, mat: Matrix, cols, shifts, w, x, tau, target, mu_lo, mu_hi, mu_tol=1e-10):
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    z = _shifts_ri(shifts)
    w = np.ascontiguousarray(w, dtype=np.float64)
    xr = _torch().view_as_real(x).contiguous() if x.is_complex() else x
    mu, cnt = ctypes.c_double(), ctypes.c_double()
    ctx.check(lib().elses_chemical_potential(ctx._h, mat._h, cols.shape[0], _np_ptr(cols), z.shape[0] // 2,
                                             _np_ptr(z), _np_ptr(w), _dev_ptr(xr), tau, target, mu_lo, mu_hi,
                                             mu_tol, ctypes.byref(mu), ctypes.byref(cnt)))
    return mu.value, cnt.value


# ---------------------------------------------------------------------------
# Multiple Arnoldi method with analytic energy integration
# ---------------------------------------------------------------------------
def _arnoldi_opts(nu, mu, kT, variant, slots, inner_tol) -> ArnoldiOpts:
    o = ArnoldiOpts()
    lib().elses_arnoldi_opts_default(ctypes.byref(o))
    o.nu, o.mu, o.kT = int(nu), float(mu), float(kT)
    o.variant, o.slots, o.inner_tol = _variant(variant), int(slots), float(inner_tol)
    return o


def _arnoldi_out(n_cols, nu, npat, want_rho):
    return dict(eps=np.zeros((n_cols, nu)), w_I=np.zeros((n_cols, nu)), w_B=np.zeros((n_cols, nu)),
                w_A=np.zeros((n_cols, nu)), dim=np.zeros(n_cols, dtype=np.int32),
                rho=np.zeros(npat) if want_rho else None, col_traces=np.zeros((n_cols, 2)))


def arnoldi(ctx: Context, mat: Matrix, cols, nu: int = 30, mu: float = 0.0, kT: float = 0.0, want_rho: bool = False,
            variant="auto", slots: int = 0, inner_tol: float = 1e-13):
    """Ritz values and Eq. 18 weights of every column on L_nu (host arrays), rho on the
    column patterns and e_j^T rho X e_j (X = B, A) for the Fermi function (mu, kT)."""
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    nc = cols.shape[0]
    off = None
    if want_rho:
        off, _ = pattern(mat, cols)
    out = _arnoldi_out(nc, nu, 0 if off is None else int(off[-1]), want_rho)
    o = _arnoldi_opts(nu, mu, kT, variant, slots, inner_tol)
    st = lib().elses_arnoldi(ctx._h, mat._h, nc, _np_ptr(cols), ctypes.byref(o), _np_ptr(out["eps"]),
                             _np_ptr(out["w_I"]), _np_ptr(out["w_B"]), _np_ptr(out["w_A"]), _np_ptr(out["dim"]),
                             _np_ptr(out["rho"]), _np_ptr(out["col_traces"]))
    ctx.check(st)
    out["pat_off"] = off
    return out


def region_arnoldi(ctx: Context, reg: Regions, nu: int = 30, mu: float = 0.0, kT: float = 0.0,
                   want_rho: bool = False, variant="auto", inner_tol: float = 1e-13):
    """The same for every column of a region set, each on its region's sub-pencil."""
    out = _arnoldi_out(reg.n_cols, nu, int(reg.pat_off[-1]), want_rho)
    o = _arnoldi_opts(nu, mu, kT, variant, 0, inner_tol)
    st = lib().elses_regions_arnoldi(ctx._h, reg._h, ctypes.byref(o), _np_ptr(out["eps"]), _np_ptr(out["w_I"]),
                                     _np_ptr(out["w_B"]), _np_ptr(out["w_A"]), _np_ptr(out["dim"]),
                                     _np_ptr(out["rho"]), _np_ptr(out["col_traces"]))
    ctx.check(st)
    out["pat_off"] = reg.pat_off
    out["cols"] = reg.cols
    return out
