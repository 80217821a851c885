"""Thin ctypes binding of libcbs.so (include/cbs.h).

Argument marshalling only: every step of the solve runs in the HIP kernels of
the library.  PyTorch supplies device memory (tensors on ``cuda``) and the
stream (``torch.cuda.current_stream()``).  The binding refuses to run
without the built library.
"""
from __future__ import annotations

import ctypes as C
import os
import sys
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcbs.so")

OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_PATTERN, ERR_SINGULAR, ERR_BREAKDOWN = -1, -2, -3, -4
ERR_NONFINITE, ERR_STATE, ERR_OOM, ERR_HIP = -5, -6, -7, -8
SOLVER_BICGSTAB, SOLVER_FGMRES, SOLVER_GMRES = 0, 1, 2
PREC_NONE, PREC_BJACOBI, PREC_AMG, PREC_SGS = 0, 1, 2, 3
SMOOTH_BJACOBI, SMOOTH_DILU, SMOOTH_SGS, SMOOTH_ILU0 = 0, 1, 2, 3
PRECISION_FP64, PRECISION_MIXED = 0, 1
LEVEL_SWEEP, LEVEL_RESIDUAL = 0, 1


class Options(C.Structure):
    _fields_ = [
        ("solver", C.c_int32), ("restart", C.c_int32), ("precond", C.c_int32),
        ("smoother", C.c_int32), ("pre_sweeps", C.c_int32), ("post_sweeps", C.c_int32),
        ("omega", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32),
        ("precision", C.c_int32), ("coarse_max", C.c_int32), ("match_passes", C.c_int32),
        ("max_levels", C.c_int32), ("reuse_aggregates", C.c_int32), ("check_every", C.c_int32),
        ("renumber", C.c_int32), ("dilu_levels", C.c_int32), ("row_split", C.c_int32),
        ("tail_rows", C.c_int32), ("schedule", C.c_int32), ("scaled_sweeps", C.c_int32),
        ("w_levels", C.c_int32), ("coarse_omega", C.c_double),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("iterations", C.c_int32), ("status", C.c_int32), ("levels", C.c_int32),
        ("precision_fallback", C.c_int32), ("rel_res_true", C.c_double),
        ("rel_res_recursive", C.c_double), ("rel_res_initial", C.c_double),
        ("t_convert_ms", C.c_double), ("t_setup_ms", C.c_double), ("t_solve_ms", C.c_double),
        ("op_complexity", C.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# (name, restype, argtypes) of every exported entry point
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    """cbs_allocator: alloc(ctx, bytes, stream), free(ctx, ptr, stream), ctx."""
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("ctx", C.c_void_p)]


def torch_allocator():
    """An Allocator that takes the library's device memory from PyTorch's
    caching allocator (torch.cuda.caching_allocator_alloc on the handle's
    stream).  Keep the returned object alive as long as the handle."""
    torch = _torch()
    dev = torch.cuda.current_device()

    def _alloc(ctx, nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), dev, int(stream or 0))
        except RuntimeError:                 # out of memory: the library reports CBS_ERR_OOM
            return None

    def _free(ctx, ptr, stream):
        torch.cuda.caching_allocator_delete(int(ptr))

    return Allocator(_ALLOC_FN(_alloc), _FREE_FN(_free), None)


_VP, _I32, _I64, _D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
SIGNATURES = [
    ("cbs_default_options", None, [C.POINTER(Options)]),
    ("cbs_create_from_ldu", C.c_int, [C.POINTER(_VP), _I32, _I32, _I32, _VP, _VP, _VP, _VP, _VP, _VP]),
    ("cbs_create_batch_from_ldu", C.c_int, [C.POINTER(_VP), _I32, C.POINTER(_I64), C.POINTER(_I64), _I32,
                                            _VP, _VP, _VP, _VP, _VP, _VP]),
    ("cbs_update_values", C.c_int, [_VP, _VP, _VP, _VP]),
    ("cbs_assemble_luo", C.c_int, [_VP, _VP, _VP, _VP, _VP, C.c_double]),
    ("cbs_assemble_luo_noalloc", C.c_int, [_VP, _VP, _VP, _VP, _VP, C.c_double]),
    ("cbs_assemble_pu", C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    ("cbs_setup", C.c_int, [_VP, C.POINTER(Options)]),
    ("cbs_solve", C.c_int, [_VP, _VP, _VP, C.POINTER(Stats)]),
    ("cbs_solve_batch", C.c_int, [_VP, _VP, _VP, C.POINTER(Stats)]),
    ("cbs_solve_transpose", C.c_int, [_VP, _VP, _VP, C.POINTER(Stats)]),
    ("cbs_gradient", C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP]),
    ("cbs_spmv", C.c_int, [_VP, _VP, _VP, _I32]),
    ("cbs_level_apply", C.c_int, [_VP, _I32, _I32, _VP, _VP, _VP, C.POINTER(_I32)]),
    ("cbs_apply_precond", C.c_int, [_VP, _VP, _VP]),
    ("cbs_apply_precond_transpose", C.c_int, [_VP, _VP, _VP]),
    ("cbs_pack_fields", C.c_int, [_I32, _I32, _VP, _VP, _VP]),
    ("cbs_unpack_fields", C.c_int, [_I32, _I32, _VP, _VP, _VP]),
    ("cbs_get_info", C.c_int, [_VP, C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I32), C.POINTER(_I64),
                               C.POINTER(_I32), C.POINTER(_I32)]),
    ("cbs_get_bcsr", C.c_int, [_VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    ("cbs_get_mirror", C.c_int, [_VP, _VP]),
    ("cbs_set_allocator", C.c_int, [_VP, C.POINTER(Allocator)]),
    ("cbs_get_level", C.c_int, [_VP, _I32, C.POINTER(_I32), C.POINTER(_I64), _VP, _VP, _VP, _VP, _VP, _VP]),
    ("cbs_destroy", C.c_int, [_VP]),
    ("cbs_error_string", C.c_char_p, [C.c_int]),
    ("cbs_last_error", C.c_char_p, []),
]

_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libcbs.so is not built (%s); run `python -m paper_2403_07882_amd.build`"
                              % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class CbsError(RuntimeError):
    def __init__(self, code: int, where: str):
        L = lib()
        msg = L.cbs_last_error().decode() if code < 0 else ""
        super().__init__("%s: %s %s" % (where, L.cbs_error_string(code).decode(), msg))
        self.code = code


def _check(code: int, where: str) -> int:
    if code < 0:
        raise CbsError(code, where)
    return code


def _torch():
    import torch
    return torch


def _stream_ptr():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(a, dtype, device="cuda"):
    """Contiguous device tensor of the given torch dtype (copies host data)."""
    torch = _torch()
    if isinstance(a, torch.Tensor):
        t = a.to(device=device, dtype=dtype)
    else:
        t = torch.as_tensor(np.ascontiguousarray(a), device=device, dtype=dtype)
    return t.contiguous()


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None and t.numel() > 0 else C.c_void_p(0)


def default_options(**kw) -> Options:
    o = Options()
    lib().cbs_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError("unknown option %r" % k)
        setattr(o, k, v)
    return o


def pack_fields(soa):
    """(n, N) per-variable fields -> (N, n) block AoS on the device."""
    torch = _torch()
    s = _dev(soa, torch.float64)
    n, N = s.shape
    out = torch.empty((N, n), dtype=torch.float64, device=s.device)
    _check(lib().cbs_pack_fields(N, n, _ptr(s), _ptr(out), _stream_ptr()), "cbs_pack_fields")
    return out


def unpack_fields(aos):
    torch = _torch()
    a = _dev(aos, torch.float64)
    N, n = a.shape
    out = torch.empty((n, N), dtype=torch.float64, device=a.device)
    _check(lib().cbs_unpack_fields(N, n, _ptr(a), _ptr(out), _stream_ptr()), "cbs_unpack_fields")
    return out


class System:
    """One coupled block system (or a batch of them) living on the GPU.

    ``System(N, n, lower_addr, upper_addr, diag, upper, lower)``: LDU arrays
    (numpy or torch; copied to the device).  Batched: pass ``cell_off`` and
    ``face_off`` (host int64 offsets) with per-system local face addresses.
    ``allocator="torch"`` takes the device memory of setup and solve from
    PyTorch's caching allocator (cbs_set_allocator) instead of hipMalloc.
    """

    def __init__(self, N, n, lower_addr, upper_addr, diag, upper, lower,
                 cell_off=None, face_off=None, allocator=None):
        torch = _torch()
        L = lib()
        self.n = int(n)
        la = _dev(lower_addr, torch.int32)
        ua = _dev(upper_addr, torch.int32)
        self.F = int(la.numel())
        self.N = int(N)
        self._la, self._ua = la, ua
        d = _dev(diag, torch.float64)
        u = _dev(upper, torch.float64)
        lo = _dev(lower, torch.float64)
        h = C.c_void_p()
        if cell_off is None:
            self.n_sys = 1
            rc = L.cbs_create_from_ldu(C.byref(h), self.N, self.F, self.n, _ptr(la), _ptr(ua),
                                       _ptr(d), _ptr(u), _ptr(lo), _stream_ptr())
        else:
            co = np.ascontiguousarray(cell_off, dtype=np.int64)
            fo = np.ascontiguousarray(face_off, dtype=np.int64)
            self.n_sys = int(co.size - 1)
            self.cell_off, self.face_off = co, fo
            rc = L.cbs_create_batch_from_ldu(C.byref(h), self.n_sys,
                                             co.ctypes.data_as(C.POINTER(C.c_int64)),
                                             fo.ctypes.data_as(C.POINTER(C.c_int64)), self.n,
                                             _ptr(la), _ptr(ua), _ptr(d), _ptr(u), _ptr(lo),
                                             _stream_ptr())
        _check(rc, "cbs_create")
        self.h = h
        self._allocator = None
        if allocator is not None:
            if allocator != "torch":
                raise ValueError("allocator must be None or 'torch'")
            self._allocator = torch_allocator()
            _check(L.cbs_set_allocator(self.h, C.byref(self._allocator)), "cbs_set_allocator")
        self.options: Optional[Options] = None
        # bumped by every call that changes the matrix or its preconditioner;
        # the autograd backward refuses a System whose generation moved
        self.generation = 0

    @classmethod
    def from_dict(cls, s, **kw):
        if "cell_off" in s:
            return cls(s["N"], s["n"], s["lower_addr"], s["upper_addr"], s["diag"], s["upper"],
                       s["lower"], cell_off=s["cell_off"], face_off=s["face_off"], **kw)
        return cls(s["N"], s["n"], s["lower_addr"], s["upper_addr"], s["diag"], s["upper"], s["lower"], **kw)

    def close(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.h = None
            lib().cbs_destroy(h)

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the module state (this module's globals, and
        # the runtime behind an allocator callback) may already be gone, so
        # the check is bound here; the process end frees the device memory
        if getattr(self, "h", None) is not None and not _finalizing():
            self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # ------------------------------------------------------------ lifecycle
    def update_values(self, diag, upper, lower):
        torch = _torch()
        d, u, lo = (_dev(a, torch.float64) for a in (diag, upper, lower))
        self.generation += 1
        _check(lib().cbs_update_values(self.h, _ptr(d), _ptr(u), _ptr(lo)), "cbs_update_values")

    def assemble_luo(self, Q, Sf, lam_visc=None, v_dt=None, gamma=1.4):
        """Assemble the density-based coupled matrix on the device from cell
        states and face area vectors (cbs_assemble_luo); then call setup."""
        torch = _torch()
        q, s = _dev(Q, torch.float64), _dev(Sf, torch.float64)
        lv = _dev(lam_visc, torch.float64) if lam_visc is not None else None
        vd = _dev(v_dt, torch.float64) if v_dt is not None else None
        self.generation += 1
        _check(lib().cbs_assemble_luo(self.h, _ptr(q), _ptr(s), None if lv is None else _ptr(lv),
                                      None if vd is None else _ptr(vd), float(gamma)), "cbs_assemble_luo")

    def assemble_luo_noalloc(self, Q, Sf, lam_visc=None, v_dt=None, gamma=1.4):
        """assemble_luo through cbs_assemble_luo_noalloc: the library's fixed
        per-device scratch instead of handle buffers (no device allocation)."""
        torch = _torch()
        q, s = _dev(Q, torch.float64), _dev(Sf, torch.float64)
        lv = _dev(lam_visc, torch.float64) if lam_visc is not None else None
        vd = _dev(v_dt, torch.float64) if v_dt is not None else None
        self.generation += 1
        _check(lib().cbs_assemble_luo_noalloc(self.h, _ptr(q), _ptr(s), None if lv is None else _ptr(lv),
                                              None if vd is None else _ptr(vd), float(gamma)),
               "cbs_assemble_luo_noalloc")

    def assemble_pu(self, Sf, fx, d, flux, nu_eff, vol, uu_add=None, pp_add=None):
        """Assemble the pressure-based (p, U) coupled matrix on the device
        from face geometry and fields (cbs_assemble_pu); then call setup."""
        torch = _torch()
        a = [_dev(x, torch.float64) for x in (Sf, fx, d, flux, nu_eff, vol)]
        opt = [None if x is None else _dev(x, torch.float64) for x in (uu_add, pp_add)]
        self.generation += 1
        _check(lib().cbs_assemble_pu(self.h, *[_ptr(x) for x in a], *[None if x is None else _ptr(x) for x in opt]),
               "cbs_assemble_pu")

    def setup(self, options: Optional[Options] = None, **kw):
        o = options if options is not None else default_options(**kw)
        self.generation += 1
        _check(lib().cbs_setup(self.h, C.byref(o)), "cbs_setup")
        self.options = o
        return self

    def _solve(self, fn, where, b, x0):
        torch = _torch()
        bb = _dev(b, torch.float64).reshape(-1)
        x = torch.zeros_like(bb) if x0 is None else _dev(x0, torch.float64).reshape(-1).clone()
        st = (Stats * self.n_sys)()
        rc = _check(fn(self.h, _ptr(bb), _ptr(x), st), where)
        stats = [s.as_dict() for s in st]
        return x.reshape(-1, self.n), (stats[0] if self.n_sys == 1 else stats), rc

    def solve(self, b, x0=None):
        """Solve A x = b; returns (x[N, n] on the device, stats dict(s))."""
        x, st, _ = self._solve(lib().cbs_solve, "cbs_solve", b, x0)
        return x, st

    def solve_batch(self, b, x0=None):
        """cbs_solve_batch: the systems' vectors concatenated; returns (x on
        the device, a list of n_sys stats dicts)."""
        x, st, _ = self._solve(lib().cbs_solve_batch, "cbs_solve_batch", b, x0)
        return x, (st if isinstance(st, list) else [st])

    def solve_transpose(self, g, x0=None):
        x, st, _ = self._solve(lib().cbs_solve_transpose, "cbs_solve_transpose", g, x0)
        return x, st

    def spmv(self, x, transpose=False):
        torch = _torch()
        xx = _dev(x, torch.float64).reshape(-1)
        y = torch.empty_like(xx)
        _check(lib().cbs_spmv(self.h, _ptr(xx), _ptr(y), 1 if transpose else 0), "cbs_spmv")
        return y.reshape(-1, self.n)

    def apply_precond(self, r, transpose=False):
        """z = M^{-1} r (transpose: the preconditioner of the transposed solve)."""
        torch = _torch()
        rr = _dev(r, torch.float64).reshape(-1)
        z = torch.empty_like(rr)
        fn = lib().cbs_apply_precond_transpose if transpose else lib().cbs_apply_precond
        _check(fn(self.h, _ptr(rr), _ptr(z)), "cbs_apply_precond")
        return z.reshape(-1, self.n)

    def level_apply(self, level, op, b, x):
        """One level kernel of the smoother (LEVEL_SWEEP or LEVEL_RESIDUAL) in
        the hierarchy's internal numbering and precision; returns y."""
        torch = _torch()
        f = C.c_int32(0)
        _check(lib().cbs_level_apply(self.h, level, op, None, None, None, C.byref(f)), "cbs_level_apply")
        dt = torch.float32 if f.value else torch.float64
        bb = _dev(b, dt).reshape(-1)
        xx = _dev(x, dt).reshape(-1)
        y = torch.empty_like(xx)
        _check(lib().cbs_level_apply(self.h, level, op, _ptr(bb), _ptr(xx), _ptr(y), None), "cbs_level_apply")
        return y.reshape(-1, self.n)

    def gradient(self, lam, x):
        torch = _torch()
        ll = _dev(lam, torch.float64).reshape(-1)
        xx = _dev(x, torch.float64).reshape(-1)
        n = self.n
        gd = torch.empty((self.N, n, n), dtype=torch.float64, device=ll.device)
        gu = torch.empty((self.F, n, n), dtype=torch.float64, device=ll.device)
        gl = torch.empty((self.F, n, n), dtype=torch.float64, device=ll.device)
        _check(lib().cbs_gradient(self.h, _ptr(ll), _ptr(xx), _ptr(gd), _ptr(gu), _ptr(gl)), "cbs_gradient")
        return gd, gu, gl

    # ------------------------------------------------------------ introspection
    def info(self):
        v = [C.c_int32(), C.c_int32(), C.c_int32(), C.c_int64(), C.c_int32(), C.c_int32()]
        _check(lib().cbs_get_info(self.h, *[C.byref(a) for a in v]), "cbs_get_info")
        return dict(zip(["n_cells", "n_faces", "bdim", "nnzb", "levels", "n_sys"], [a.value for a in v]))

    def get_bcsr(self):
        torch = _torch()
        inf = self.info()
        N, nnzb, n, F = inf["n_cells"], inf["nnzb"], inf["bdim"], inf["n_faces"]
        dev = "cuda"
        rp = torch.empty(N + 1, dtype=torch.int32, device=dev)
        col = torch.empty(nnzb, dtype=torch.int32, device=dev)
        vals = torch.empty((nnzb, n, n), dtype=torch.float64, device=dev)
        ds = torch.empty(N, dtype=torch.int32, device=dev)
        us = torch.empty(max(F, 1), dtype=torch.int32, device=dev)
        ls = torch.empty(max(F, 1), dtype=torch.int32, device=dev)
        _check(lib().cbs_get_bcsr(self.h, _ptr(rp), _ptr(col), _ptr(vals), _ptr(ds), _ptr(us), _ptr(ls)),
               "cbs_get_bcsr")
        return {"row_ptr": rp, "col": col, "vals": vals, "diag_slot": ds,
                "upper_slot": us[:F], "lower_slot": ls[:F]}

    def get_mirror(self):
        """The level-0 transpose-slot map mirror[nnzb] (device int32)."""
        torch = _torch()
        nnzb = self.info()["nnzb"]
        m = torch.empty(max(nnzb, 1), dtype=torch.int32, device="cuda")
        _check(lib().cbs_get_mirror(self.h, _ptr(m)), "cbs_get_mirror")
        return m[:nnzb]

    def get_level(self, level):
        torch = _torch()
        nr, nz = C.c_int32(), C.c_int64()
        _check(lib().cbs_get_level(self.h, level, C.byref(nr), C.byref(nz), None, None, None, None, None, None),
               "cbs_get_level")
        N, nnzb, n = nr.value, nz.value, self.n
        dev = "cuda"
        rp = torch.empty(N + 1, dtype=torch.int32, device=dev)
        col = torch.empty(max(nnzb, 1), dtype=torch.int32, device=dev)
        vals = torch.empty((max(nnzb, 1), n, n), dtype=torch.float64, device=dev)
        agg = torch.full((N,), -1, dtype=torch.int32, device=dev)
        colour = torch.full((N,), -1, dtype=torch.int32, device=dev)
        order = torch.empty((N,), dtype=torch.int32, device=dev)
        _check(lib().cbs_get_level(self.h, level, C.byref(nr), C.byref(nz), _ptr(rp), _ptr(col), _ptr(vals),
                                   _ptr(agg), _ptr(colour), _ptr(order)), "cbs_get_level")
        return {"N": N, "nnzb": nnzb, "row_ptr": rp, "col": col[:nnzb], "vals": vals[:nnzb],
                "agg": agg, "colour": colour, "order": order}


# ---------------------------------------------------------------- autograd
def _coupled_solve_cls():
    torch = _torch()

    class CoupledSolve(torch.autograd.Function):
        """x = A(diag, upper, lower)^{-1} b with the adjoint solve in backward.

        forward(system, diag, upper, lower, b): (re)loads the values into the
        given System (same pattern), sets it up with its options and solves.
        backward(g): lambda = A^{-T} g (transpose solve on the same
        aggregates); dL/db = lambda, dL/dA_ij = -lambda_i x_j^T on the pattern.
        Both raise CbsError (code NOT_CONVERGED) when a solve stops at the
        iteration cap, and backward raises RuntimeError when the System's
        values or preconditioner changed after forward (another update,
        assembly, setup or coupled_solve on it), since lambda would then be
        the adjoint of another matrix.
        """

        @staticmethod
        def forward(ctx, system, diag, upper, lower, b):
            system.update_values(diag.detach(), upper.detach(), lower.detach())
            system.setup(system.options if system.options is not None else default_options())
            x, st = system.solve(b.detach())
            _require_converged(st, "coupled_solve forward")
            ctx.system = system
            ctx.generation = system.generation
            ctx.save_for_backward(x)
            ctx.stats = st
            return x

        @staticmethod
        def backward(ctx, g):
            (x,) = ctx.saved_tensors
            system = ctx.system
            if system.generation != ctx.generation:
                raise RuntimeError("coupled_solve backward: the System was updated or set up again after "
                                   "forward; the adjoint would use another matrix")
            lam, st = system.solve_transpose(g.contiguous())
            _require_converged(st, "coupled_solve backward (transposed solve)")
            gd, gu, gl = system.gradient(lam, x)
            return None, gd, gu, gl, lam.reshape(g.shape)

    return CoupledSolve


def _require_converged(st, where):
    """Raise CbsError(NOT_CONVERGED) unless every system's status is OK."""
    for s in (st if isinstance(st, list) else [st]):
        if s["status"] != OK:
            raise CbsError(int(s["status"]), where)


_CS = None


def coupled_solve(system: System, diag, upper, lower, b):
    """Differentiable solve (torch.autograd) through the HIP library."""
    global _CS
    if _CS is None:
        _CS = _coupled_solve_cls()
    return _CS.apply(system, diag, upper, lower, b)
