"""CPU FP64 oracle for the coupled block-sparse solve (test infrastructure).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark use
this package.  The product library never imports it.  The arithmetic lives in
``oracle.c`` (plain C, FP64); this module builds it with gcc and wraps each
function with numpy arrays.  See ``oracle.c`` for the paper passages each
function follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_SANITIZE=1 builds and loads a copy instrumented with AddressSanitizer
# and UBSan (run the Python process with the two runtimes in LD_PRELOAD)
_SANITIZE = os.environ.get("ORACLE_SANITIZE") == "1"
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")

OK, NOT_CONVERGED = 0, 1
ERR_ARG, ERR_PATTERN, ERR_SINGULAR, ERR_BREAKDOWN = -1, -2, -3, -4

PREC_NONE, PREC_BJACOBI, PREC_AMG, PREC_SGS = 0, 1, 2, 3
# the AMG V-cycle in FP32 emulation (row-scaled or unscaled sweeps), with an AMG handle
PREC_AMG_FP32, PREC_AMG_FP32_UNSCALED = 4, 5
SMOOTH_BJACOBI, SMOOTH_DILU, SMOOTH_SGS, SMOOTH_ILU0 = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP); with
    ORACLE_SANITIZE=1 into liboracle_san.so with -fsanitize=address,undefined."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        opt = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer"] if _SANITIZE else ["-O2"]
        subprocess.check_call(["gcc", *opt, "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")


def _declare(L):
    ci, cl, cd, vp = C.c_int, C.c_long, C.c_double, C.c_void_p
    sig = {
        "orc_pack": (None, [ci, ci, _f64p, _f64p]),
        "orc_unpack": (None, [ci, ci, _f64p, _f64p]),
        "orc_ldu_to_bcsr": (ci, [ci, ci, ci, _i32p, _i32p, _f64p, _f64p, _f64p,
                                 _i32p, _i32p, _f64p, _i32p, _i32p, _i32p]),
        "orc_spmv_bcsr": (None, [ci, ci, _i32p, _i32p, _f64p, _f64p, _f64p]),
        "orc_spmv_bcsr_t": (None, [ci, ci, _i32p, _i32p, _f64p, _f64p, _f64p]),
        "orc_spmv_ldu": (None, [ci, ci, ci, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p]),
        "orc_transpose": (None, [ci, ci, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p]),
        "orc_blockinv": (ci, [cl, ci, _f64p, _f64p, C.POINTER(cl)]),
        "orc_dense_solve": (ci, [ci, _f64p, _f64p, _f64p]),
        "orc_bjacobi_sweep": (None, [ci, ci, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p, cd]),
        "orc_sgs_sweep": (None, [ci, ci, _i32p, _i32p, _f64p, _f64p, _i32p, _f64p, _f64p]),
        "orc_dilu_setup": (ci, [ci, ci, _i32p, _i32p, _f64p, _i32p, _f64p]),
        "orc_dilu_apply": (None, [ci, ci, _i32p, _i32p, _f64p, _i32p, _f64p, _f64p, _f64p]),
        "orc_ilu0_setup": (ci, [ci, ci, _i32p, _i32p, _f64p, _i32p, _f64p, _f64p]),
        "orc_ilu0_apply": (None, [ci, ci, _i32p, _i32p, _f64p, _i32p, _f64p, _f64p, _f64p]),
        "orc_strength": (None, [ci, ci, _i32p, _i32p, _f64p, _f64p]),
        "orc_match": (ci, [ci, _i32p, _i32p, _f64p, _i32p]),
        "orc_rap_count": (cl, [ci, _i32p, _i32p, _i32p, ci, _i32p]),
        "orc_rap_fill": (None, [ci, ci, _i32p, _i32p, _f64p, _i32p, ci, _i32p, _i32p, _f64p]),
        "orc_restrict": (None, [ci, ci, _i32p, _f64p, ci, _f64p]),
        "orc_prolong_add": (None, [ci, ci, _i32p, _f64p, _f64p]),
        "orc_amg_create": (vp, [ci, ci, _i32p, _i32p, _f64p, ci, ci, ci, ci, ci, cd,
                                vp, ci, vp, ci, ci]),
        "orc_amg_free": (None, [vp]),
        "orc_sgs_prec_create": (vp, [ci, ci, _i32p, _i32p, _f64p, _i32p, ci]),
        "orc_sgs_prec_free": (None, [vp]),
        "orc_sgs_prec_apply": (None, [vp, _f64p, _f64p]),
        "orc_amg_levels": (ci, [vp]),
        "orc_amg_level_info": (None, [vp, ci, C.POINTER(ci), C.POINTER(cl)]),
        "orc_amg_apply": (None, [vp, _f64p, _f64p]),
        "orc_amg_apply_fp32": (ci, [vp, _f64p, _f64p, ci]),
        "orc_amg_set_cycle": (ci, [vp, ci, C.c_double]),
        "orc_bicgstab": (ci, [ci, ci, _i32p, _i32p, _f64p, ci, vp, _f64p, _f64p, cd, ci,
                              C.POINTER(ci), C.POINTER(cd)]),
        "orc_fgmres": (ci, [ci, ci, _i32p, _i32p, _f64p, ci, vp, _f64p, _f64p, cd, ci, ci,
                            C.POINTER(ci), C.POINTER(cd)]),
        "orc_gmres": (ci, [ci, ci, _i32p, _i32p, _f64p, ci, vp, _f64p, _f64p, cd, ci, ci,
                           C.POINTER(ci), C.POINTER(cd)]),
        "orc_grad": (None, [ci, ci, ci, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p]),
        "orc_euler_jac": (None, [_f64p, _f64p, cd, _f64p]),
        "orc_roe_radius": (cd, [_f64p, _f64p, _f64p, cd]),
        "orc_luo_assemble": (ci, [ci, ci, _i32p, _i32p, _f64p, _f64p, vp, vp, cd, _f64p, _f64p, _f64p]),
        "orc_pu_assemble": (None, [ci, ci, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, vp, vp,
                                   _f64p, _f64p, _f64p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class OracleError(RuntimeError):
    def __init__(self, code, what=""):
        super().__init__("oracle %s failed with code %d" % (what, code))
        self.code = code


# ---------------------------------------------------------------- matrices
class BCSR:
    """Block-CSR matrix held as numpy arrays (row_ptr, col, vals[nnzb, n, n])."""

    def __init__(self, N, n, row_ptr, col, vals):
        self.N, self.n = int(N), int(n)
        self.row_ptr, self.col = _c32(row_ptr), _c32(col)
        self.vals = _c64(vals).reshape(-1, n, n)

    @property
    def nnzb(self):
        return int(self.row_ptr[-1])

    def dense(self):
        N, n = self.N, self.n
        A = np.zeros((N * n, N * n))
        rows = np.repeat(np.arange(N), np.diff(self.row_ptr))
        for k in range(self.nnzb):
            i, j = rows[k], self.col[k]
            A[i * n:(i + 1) * n, j * n:(j + 1) * n] = self.vals[k]
        return A


def pack(soa):
    """Fields (n, N) -> block AoS (N, n)."""
    soa = _c64(soa)
    n, N = soa.shape
    out = np.empty((N, n))
    lib().orc_pack(N, n, soa.ravel(), out.ravel())
    return out


def unpack(aos):
    aos = _c64(aos)
    N, n = aos.shape
    out = np.empty((n, N))
    lib().orc_unpack(N, n, aos.ravel(), out.ravel())
    return out


def ldu_to_bcsr(N, n, lower_addr, upper_addr, diag, upper, lower):
    """LDU -> (BCSR, diag_slot, upper_slot, lower_slot).  Raises OracleError."""
    la, ua = _c32(lower_addr), _c32(upper_addr)
    F = la.size
    nnzb = N + 2 * F
    rp = np.zeros(N + 1, np.int32)
    col = np.zeros(max(nnzb, 1), np.int32)
    vals = np.zeros(max(nnzb, 1) * n * n)
    ds = np.zeros(max(N, 1), np.int32)
    us = np.zeros(max(F, 1), np.int32)
    ls = np.zeros(max(F, 1), np.int32)
    d = _c64(diag).ravel(); u = _c64(upper).ravel(); l = _c64(lower).ravel()
    if u.size == 0:
        u = np.zeros(1); l = np.zeros(1)
    if la.size == 0:
        la = np.zeros(1, np.int32); ua = np.zeros(1, np.int32)
    rc = lib().orc_ldu_to_bcsr(N, F, n, la, ua, d if d.size else np.zeros(1), u, l,
                               rp, col, vals, ds, us, ls)
    if rc != OK:
        raise OracleError(rc, "ldu_to_bcsr")
    A = BCSR(N, n, rp, col[:nnzb], vals[:nnzb * n * n])
    return A, ds[:N], us[:F], ls[:F]


def from_system(s):
    """BCSR of a generated system dict."""
    return ldu_to_bcsr(s["N"], s["n"], s["lower_addr"], s["upper_addr"],
                       s["diag"], s["upper"], s["lower"])[0]


def spmv(A: BCSR, x):
    y = np.empty(A.N * A.n)
    lib().orc_spmv_bcsr(A.N, A.n, A.row_ptr, A.col, A.vals.ravel(), _c64(x).ravel(), y)
    return y.reshape(A.N, A.n)


def spmv_t(A: BCSR, x):
    y = np.empty(A.N * A.n)
    lib().orc_spmv_bcsr_t(A.N, A.n, A.row_ptr, A.col, A.vals.ravel(), _c64(x).ravel(), y)
    return y.reshape(A.N, A.n)


def spmv_ldu(s, x):
    N, n = s["N"], s["n"]
    y = np.empty(N * n)
    la, ua = _c32(s["lower_addr"]), _c32(s["upper_addr"])
    F = la.size
    up = _c64(s["upper"]).ravel(); lo = _c64(s["lower"]).ravel()
    if F == 0:
        la = ua = np.zeros(1, np.int32); up = lo = np.zeros(1)
    lib().orc_spmv_ldu(N, F, n, la, ua, _c64(s["diag"]).ravel(), up, lo,
                       _c64(x).ravel(), y)
    return y.reshape(N, n)


def transpose(A: BCSR) -> BCSR:
    rp = np.zeros(A.N + 1, np.int32)
    col = np.zeros(max(A.nnzb, 1), np.int32)
    vals = np.zeros(max(A.nnzb, 1) * A.n * A.n)
    lib().orc_transpose(A.N, A.n, A.row_ptr, A.col, A.vals.ravel(), rp, col, vals)
    return BCSR(A.N, A.n, rp, col[:A.nnzb], vals[:A.nnzb * A.n * A.n])


def blockinv(D):
    D = _c64(D)
    nb, n = D.shape[0], D.shape[1]
    out = np.empty_like(D)
    bad = C.c_long(-1)
    rc = lib().orc_blockinv(nb, n, D.ravel(), out.ravel(), C.byref(bad))
    if rc != OK:
        raise OracleError(rc, "blockinv (block %d)" % bad.value)
    return out


def dense_solve(A, b):
    A = _c64(A)
    m = A.shape[0]
    x = np.empty(m)
    rc = lib().orc_dense_solve(m, A.ravel(), _c64(b).ravel(), x)
    if rc != OK:
        raise OracleError(rc, "dense_solve")
    return x


def diag_blocks(A: BCSR):
    rows = np.repeat(np.arange(A.N), np.diff(A.row_ptr))
    k = np.nonzero(rows == A.col)[0]
    return A.vals[k]


def bjacobi_sweep(A: BCSR, Dinv, b, x, omega):
    out = np.empty(A.N * A.n)
    lib().orc_bjacobi_sweep(A.N, A.n, A.row_ptr, A.col, A.vals.ravel(), _c64(Dinv).ravel(),
                            _c64(b).ravel(), _c64(x).ravel(), out, float(omega))
    return out.reshape(A.N, A.n)


def sgs_sweep(A: BCSR, Dinv, rank, b, x):
    """One symmetric block Gauss-Seidel step from x in the order of rank."""
    out = _c64(x).ravel().copy()
    lib().orc_sgs_sweep(A.N, A.n, A.row_ptr, A.col, A.vals.ravel(), _c64(Dinv).ravel(), _c32(rank),
                        _c64(b).ravel(), out)
    return out.reshape(A.N, A.n)


def dilu_setup(A: BCSR, rank):
    Einv = np.empty((A.N, A.n, A.n))
    rc = lib().orc_dilu_setup(A.N, A.n, A.row_ptr, A.col, A.vals.ravel(), _c32(rank), Einv.ravel())
    if rc != OK:
        raise OracleError(rc, "dilu_setup")
    return Einv


def dilu_apply(A: BCSR, rank, Einv, r):
    z = np.empty(A.N * A.n)
    lib().orc_dilu_apply(A.N, A.n, A.row_ptr, A.col, A.vals.ravel(), _c32(rank),
                         _c64(Einv).ravel(), _c64(r).ravel(), z)
    return z.reshape(A.N, A.n)


def ilu0_setup(A: BCSR, rank):
    """Block ILU(0) in the order of rank: (LU factor in A's pattern, U_ii^{-1})."""
    LU = np.empty_like(A.vals)
    Uinv = np.empty((A.N, A.n, A.n))
    rc = lib().orc_ilu0_setup(A.N, A.n, A.row_ptr, A.col, A.vals.ravel(), _c32(rank), LU.ravel(), Uinv.ravel())
    if rc < 0:
        raise OracleError(rc, "ilu0_setup")
    return LU, Uinv


def ilu0_apply(A: BCSR, rank, LU, Uinv, r):
    z = np.empty(A.N * A.n)
    lib().orc_ilu0_apply(A.N, A.n, A.row_ptr, A.col, _c64(LU).ravel(), _c32(rank), _c64(Uinv).ravel(),
                         _c64(r).ravel(), z)
    return z.reshape(A.N, A.n)


def strength(A: BCSR):
    w = np.empty(max(A.nnzb, 1))
    lib().orc_strength(A.N, A.n, A.row_ptr, A.col, A.vals.ravel(), w)
    return w[:A.nnzb]


def match(N, row_ptr, col, w):
    agg = np.empty(max(N, 1), np.int32)
    nc = lib().orc_match(N, _c32(row_ptr), _c32(col), _c64(w), agg)
    return agg[:N], nc


def rap(A: BCSR, agg, nc) -> BCSR:
    agg = _c32(agg)
    rpc = np.zeros(nc + 1, np.int32)
    nz = lib().orc_rap_count(A.N, A.row_ptr, A.col, agg, nc, rpc)
    colc = np.zeros(max(nz, 1), np.int32)
    valc = np.zeros(max(nz, 1) * A.n * A.n)
    lib().orc_rap_fill(A.N, A.n, A.row_ptr, A.col, A.vals.ravel(), agg, nc, rpc, colc, valc)
    return BCSR(nc, A.n, rpc, colc[:nz], valc[:nz * A.n * A.n])


def restrict(agg, r, nc):
    r = _c64(r)
    N, n = r.shape
    out = np.empty(nc * n)
    lib().orc_restrict(N, n, _c32(agg), r.ravel(), nc, out)
    return out.reshape(nc, n)


def prolong_add(agg, e, x):
    x = _c64(x).copy()
    N, n = x.shape
    lib().orc_prolong_add(N, n, _c32(agg), _c64(e).ravel(), x.ravel())
    return x


class AMG:
    """Reference aggregation-AMG hierarchy with a V-cycle preconditioner.

    ``aggs``: optional list of aggregate maps (one per coarsened level) to
    impose a hierarchy; ``ranks``: optional DILU orderings per smoothed level;
    ``w_levels``: the coarse correction of each of the w_levels finest levels
    runs the next level's cycle twice (a W-cycle there; 0 = V-cycle);
    ``coarse_omega``: block-Jacobi damping below level 0 (0 = ``omega``).
    """

    def __init__(self, A: BCSR, coarse_max=32, passes=2, smoother=SMOOTH_BJACOBI,
                 nu1=1, nu2=1, omega=0.8, aggs=None, ranks=None, dilu_levels=-1, w_levels=0,
                 coarse_omega=0.0):
        self._keep = []
        aggp, nag = None, 0
        if aggs is not None:
            cat = np.ascontiguousarray(np.concatenate([np.asarray(a, np.int32) for a in aggs])
                                       if len(aggs) else np.zeros(1, np.int32), np.int32)
            self._keep.append(cat)
            aggp, nag = cat.ctypes.data, len(aggs)
            if nag == 0:
                aggp = cat.ctypes.data
        rk, nrk = None, 0
        if ranks is not None and len(ranks):
            catr = np.ascontiguousarray(np.concatenate([np.asarray(a, np.int32) for a in ranks]), np.int32)
            self._keep.append(catr)
            rk, nrk = catr.ctypes.data, len(ranks)
        self.A = A
        self.h = lib().orc_amg_create(A.N, A.n, A.row_ptr, A.col, A.vals.ravel(),
                                      coarse_max, passes, smoother, nu1, nu2, float(omega),
                                      aggp, nag, rk, nrk, int(dilu_levels))
        if not self.h:
            raise OracleError(ERR_SINGULAR, "amg_create")
        rc = lib().orc_amg_set_cycle(self.h, int(w_levels), float(coarse_omega))
        if rc != OK:
            raise OracleError(rc, "amg_set_cycle")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_amg_free(self.h)
            self.h = None

    @property
    def levels(self):
        return lib().orc_amg_levels(self.h)

    def level_info(self):
        out = []
        for l in range(self.levels):
            N, nz = C.c_int(), C.c_long()
            lib().orc_amg_level_info(self.h, l, C.byref(N), C.byref(nz))
            out.append((N.value, nz.value))
        return out

    def apply(self, r):
        z = np.empty(self.A.N * self.A.n)
        lib().orc_amg_apply(self.h, _c64(r).ravel(), z)
        return z.reshape(self.A.N, self.A.n)

    def apply_fp32(self, r, scaled=True):
        """The same V-cycle in FP32 emulation (orc_amg_apply_fp32): float
        level values, vectors and sums, FP64 block inverses and coarsest
        solve; ``scaled``: sweeps on the row-scaled values.  A study tool,
        not a parity target.  Block-Jacobi hierarchies only."""
        z = np.empty(self.A.N * self.A.n)
        rc = lib().orc_amg_apply_fp32(self.h, _c64(r).ravel(), z, int(bool(scaled)))
        if rc != OK:
            raise OracleError(rc, "amg_apply_fp32")
        return z.reshape(self.A.N, self.A.n)


class SGSPrec:
    """Symmetric block Gauss-Seidel preconditioner (the GMRES + SGS runs of
    Sec. 4.1): ``sweeps`` symmetric steps from zero in the order of ``rank``
    (row i is visited at position rank[i] forward and in reverse backward).
    Pass it as ``amg=`` with ``prec=PREC_SGS`` to the solvers."""

    def __init__(self, A: BCSR, rank, sweeps=1):
        self.A = A
        self._rank = _c32(rank)
        self.h = lib().orc_sgs_prec_create(A.N, A.n, A.row_ptr, A.col, A.vals.ravel(), self._rank, int(sweeps))
        if not self.h:
            raise OracleError(ERR_SINGULAR if sweeps >= 1 else ERR_ARG, "sgs_prec_create")

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_sgs_prec_free(self.h)
            self.h = None

    def apply(self, r):
        z = np.empty(self.A.N * self.A.n)
        lib().orc_sgs_prec_apply(self.h, _c64(r).ravel(), z)
        return z.reshape(self.A.N, self.A.n)


def _solve(fn, A, b, x0, prec, amg, tol, maxit, extra=()):
    x = np.zeros(A.N * A.n) if x0 is None else _c64(x0).ravel().copy()
    it, rr = C.c_int(0), C.c_double(0.0)
    h = amg.h if amg is not None else None
    rc = fn(A.N, A.n, A.row_ptr, A.col, A.vals.ravel(), prec, h, _c64(b).ravel(), x,
            float(tol), int(maxit), *extra, C.byref(it), C.byref(rr))
    if rc < 0:
        raise OracleError(rc, fn.__name__)
    return x.reshape(A.N, A.n), {"status": rc, "iterations": it.value, "relres": rr.value}


def bicgstab(A: BCSR, b, x0=None, prec=PREC_BJACOBI, amg=None, tol=1e-8, maxit=1000):
    return _solve(lib().orc_bicgstab, A, b, x0, prec, amg, tol, maxit)


def fgmres(A: BCSR, b, x0=None, prec=PREC_BJACOBI, amg=None, tol=1e-8, maxit=1000, restart=30):
    return _solve(lib().orc_fgmres, A, b, x0, prec, amg, tol, maxit, (int(restart),))


def gmres(A: BCSR, b, x0=None, prec=PREC_BJACOBI, amg=None, tol=1e-8, maxit=1000, restart=30):
    """Right-preconditioned (non-flexible) GMRES(restart)."""
    return _solve(lib().orc_gmres, A, b, x0, prec, amg, tol, maxit, (int(restart),))


def euler_jac(Q, s, gamma=1.4):
    J = np.empty(25)
    lib().orc_euler_jac(_c64(Q).ravel(), _c64(s).ravel(), float(gamma), J)
    return J.reshape(5, 5)


def roe_radius(QL, QR, s, gamma=1.4):
    return lib().orc_roe_radius(_c64(QL).ravel(), _c64(QR).ravel(), _c64(s).ravel(), float(gamma))


def luo_assemble(d, with_visc=True, with_dt=True):
    """LDU blocks of the density-based coupled matrix from ``luo_inputs``."""
    N, F = d["N"], d["F"]
    diag = np.empty((N, 5, 5)); upper = np.empty((max(F, 1), 5, 5)); lower = np.empty((max(F, 1), 5, 5))
    la, ua = _c32(d["lower_addr"]), _c32(d["upper_addr"])
    Sf = _c64(d["Sf"]).reshape(-1)
    if F == 0:
        la = ua = np.zeros(1, np.int32); Sf = np.zeros(3)
    lv = _c64(d["lam_visc"]) if with_visc else None
    vd = _c64(d["v_dt"]) if with_dt else None
    rc = lib().orc_luo_assemble(N, F, la, ua, _c64(d["Q"]).ravel(), Sf,
                                lv.ctypes.data if lv is not None else None,
                                vd.ctypes.data if vd is not None else None,
                                float(d["gamma"]), diag.ravel(), upper.ravel(), lower.ravel())
    if rc != OK:
        raise OracleError(rc, "luo_assemble: a cell state with non-positive density or pressure")
    return {"N": N, "F": F, "n": 5, "lower_addr": d["lower_addr"], "upper_addr": d["upper_addr"],
            "diag": diag, "upper": upper[:F], "lower": lower[:F]}


def pu_assemble(d, with_add=True):
    """LDU blocks of the pressure-based (p, Ux, Uy, Uz) matrix from ``pu_inputs``."""
    N, F = d["N"], d["F"]
    diag = np.empty((N, 4, 4)); upper = np.empty((max(F, 1), 4, 4)); lower = np.empty((max(F, 1), 4, 4))
    la, ua = _c32(d["lower_addr"]), _c32(d["upper_addr"])
    Sf, fx, dv, fl, nu = (_c64(d[k]).ravel() for k in ("Sf", "fx", "d", "flux", "nu"))
    if F == 0:
        la = ua = np.zeros(1, np.int32)
        Sf = dv = np.zeros(3); fx = fl = nu = np.zeros(1)
    ua_, pa_ = (_c64(d["uu_add"]), _c64(d["pp_add"])) if with_add else (None, None)
    lib().orc_pu_assemble(N, F, la, ua, Sf, fx, dv, fl, nu, _c64(d["vol"]),
                          None if ua_ is None else ua_.ctypes.data, None if pa_ is None else pa_.ctypes.data,
                          diag.ravel(), upper.ravel(), lower.ravel())
    return {"N": N, "F": F, "n": 4, "lower_addr": d["lower_addr"], "upper_addr": d["upper_addr"],
            "diag": diag, "upper": upper[:F], "lower": lower[:F]}


def grad(s, lam, x):
    N, n, F = s["N"], s["n"], s["F"]
    gd = np.empty((N, n, n)); gu = np.empty((max(F, 1), n, n)); gl = np.empty((max(F, 1), n, n))
    la, ua = _c32(s["lower_addr"]), _c32(s["upper_addr"])
    if F == 0:
        la = ua = np.zeros(1, np.int32)
    lib().orc_grad(N, F, n, la, ua, _c64(lam).ravel(), _c64(x).ravel(),
                   gd.ravel(), gu.ravel(), gl.ravel())
    return gd, gu[:F], gl[:F]


def relres(A: BCSR, b, x):
    r = _c64(b).ravel() - spmv(A, x).ravel()
    nb = np.linalg.norm(_c64(b).ravel())
    return float(np.linalg.norm(r) / nb) if nb > 0 else float(np.linalg.norm(r))
