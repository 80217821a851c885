"""The W-cycle option (w_levels): on the w_levels finest levels the coarse
correction runs the next level's cycle twice, the second run starting from
the first one's result.  The GPU cycle is compared element by element with the
oracle's cycle of the same shape on the GPU's hierarchy (level-0 numbering,
aggregates, colours), for block Jacobi in both precisions with even, odd and
zero sweep counts, with the single-workgroup tail on and off, for the
coloured smoothers (whose level-1 steps then also start from a nonzero x),
for the transposed cycle and for a batch; and the solves meet the tolerance.
"""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import concat_systems, jacobian_box, pressure_velocity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2403_07882_amd as P  # noqa: E402

ALL = 100000


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _np(t):
    return t.detach().cpu().numpy()


def _agree(z, zr, rel):
    """z against the reference zr: in norm, and element by element relative
    to the largest reference entry."""
    assert np.linalg.norm(z - zr) <= rel * np.linalg.norm(zr), (np.linalg.norm(z - zr), np.linalg.norm(zr))
    assert np.abs(z - zr).max() <= rel * np.abs(zr).max(), (np.abs(z - zr).max(), np.abs(zr).max())


def _ranks_from_colour(colour):
    N = colour.size
    key = colour.astype(np.int64) * N + np.arange(N)
    rank = np.empty(N, np.int32)
    rank[np.argsort(key, kind="stable")] = np.arange(N)
    return rank


_ORACLE_SMOOTHER = {P.SMOOTH_BJACOBI: O.SMOOTH_BJACOBI, P.SMOOTH_DILU: O.SMOOTH_DILU,
                    P.SMOOTH_SGS: O.SMOOTH_SGS, P.SMOOTH_ILU0: O.SMOOTH_ILU0}


def _cycle_pair(s, w_levels, precision=P.PRECISION_FP64, pre=2, post=2, omega=0.9, tail=0,
                smoother=P.SMOOTH_BJACOBI, dilu_levels=2, transpose=False, seed=0, coarse_omega=0.0):
    """GPU cycle z = M r (or M^T r) and the oracle's cycle of the same shape
    on the GPU's level-0 numbering, aggregates and colours (on A^T for the
    transposed one); also the oracle's V-cycle, to show the shapes differ."""
    N, n = int(s["N"]), int(s["n"])
    with P.System.from_dict(s) as sysm:
        sysm.setup(precond=P.PREC_AMG, precision=precision, coarse_max=8, pre_sweeps=pre, post_sweeps=post,
                   omega=omega, tail_rows=tail, smoother=smoother, dilu_levels=dilu_levels, w_levels=w_levels,
                   coarse_omega=coarse_omega)
        nlev = sysm.info()["levels"]
        assert nlev >= 4, nlev
        lv0 = sysm.get_level(0)
        order = _np(lv0["order"])
        A0 = O.BCSR(N, n, _np(lv0["row_ptr"]), _np(lv0["col"]), _np(lv0["vals"]))
        aggs, ranks = [], []
        ndilu = 0 if smoother == P.SMOOTH_BJACOBI else (nlev - 1 if dilu_levels < 0 else min(dilu_levels, nlev - 1))
        for l in range(nlev - 1):
            lv = sysm.get_level(l)
            aggs.append(_np(lv["agg"]))
            if l < ndilu:
                ranks.append(_ranks_from_colour(_np(lv["colour"])))
        r = np.random.default_rng(seed).standard_normal((N, n))
        z = _np(sysm.apply_precond(r, transpose=transpose))
    Aref = O.transpose(A0) if transpose else A0
    kw = dict(nu1=pre, nu2=post, omega=omega, aggs=aggs, coarse_omega=coarse_omega)
    if smoother != P.SMOOTH_BJACOBI:
        kw.update(smoother=_ORACLE_SMOOTHER[smoother], ranks=ranks, dilu_levels=ndilu)
    out = []
    for wl in (w_levels, 0):
        zr_int = O.AMG(Aref, w_levels=wl, **kw).apply(r[order])
        zr = np.empty_like(zr_int)
        zr[order] = zr_int
        out.append(zr)
    return z, out[0], out[1]


def _tol(precision):
    return 1e-11 if precision == P.PRECISION_FP64 else 1e-5


@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
@pytest.mark.parametrize("w_levels", [1, 2, 99])
def test_w_cycle_matches_oracle(w_levels, precision):
    _say("w-cycle", w_levels, "precision", precision)
    s = pressure_velocity(16, 14, 12, seed=60)
    z, zr, zv = _cycle_pair(s, w_levels, precision)
    _agree(z, zr, _tol(precision))
    assert np.linalg.norm(zr - zv) > 1e3 * _tol(precision) * np.linalg.norm(zr)     # not the V-cycle


@pytest.mark.parametrize("tail", [-1, 0, ALL])
@pytest.mark.parametrize("pre,post", [(2, 2), (1, 2), (2, 1), (0, 2), (2, 0), (3, 3)])
def test_w_cycle_sweep_counts_and_tail(pre, post, tail):
    """Even and odd numbers of sweeps (a second run with an odd count starts
    by copying x into the work vector it sweeps from), no pre- or no
    post-smoothing, and the tail off, at its default start and at the first
    level it may take (level 2, below the W level)."""
    _say("w-cycle sweeps", pre, post, "tail", tail)
    s = pressure_velocity(13, 11, 10, seed=61)
    for precision in (P.PRECISION_FP64, P.PRECISION_MIXED):
        z, zr, _ = _cycle_pair(s, 1, precision, pre=pre, post=post, omega=0.8, tail=tail)
        _agree(z, zr, _tol(precision))


@pytest.mark.parametrize("n", [1, 3, 5])
def test_w_cycle_other_block_sizes(n):
    _say("w-cycle n", n)
    s = jacobian_box(14, 12, 10, n=n, seed=62 + n)
    for precision in (P.PRECISION_FP64, P.PRECISION_MIXED):
        z, zr, _ = _cycle_pair(s, 1, precision)
        _agree(z, zr, _tol(precision))


@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
@pytest.mark.parametrize("smoother", [P.SMOOTH_DILU, P.SMOOTH_SGS, P.SMOOTH_ILU0])
def test_w_cycle_coloured_levels(smoother, precision):
    """DILU, Gauss-Seidel and ILU(0) on the two finest levels: level 1's
    second run smooths from the first run's result (two-colour form with a
    full first colour-0 update)."""
    _say("w-cycle coloured", smoother, precision)
    s = pressure_velocity(13, 11, 10, seed=63)
    for pre, post in ((2, 2), (1, 2)):
        z, zr, _ = _cycle_pair(s, 1, precision, pre=pre, post=post, omega=0.8, smoother=smoother, dilu_levels=2)
        _agree(z, zr, _tol(precision))


def test_w_cycle_coloured_random_graph():
    """Jones-Plassmann colours (more than two) on the W level: the general
    forward/backward DILU steps from a nonzero start."""
    from workloads import jacobian_graph
    _say("w-cycle coloured graph")
    s = jacobian_graph(N=3000, n=4, seed=64)
    z, zr, _ = _cycle_pair(s, 1, P.PRECISION_FP64, pre=1, post=1, omega=0.8, smoother=P.SMOOTH_DILU,
                           dilu_levels=-1)
    _agree(z, zr, 1e-11)


@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
def test_transposed_w_cycle(precision):
    _say("transposed w-cycle", precision)
    s = pressure_velocity(14, 12, 10, seed=65)
    z, zr, _ = _cycle_pair(s, 1, precision, transpose=True)
    _agree(z, zr, _tol(precision))


def test_w_cycle_batch():
    _say("w-cycle batch")
    shapes = [(12, 10, 9), (7, 6, 5), (15, 11, 8), (3, 3, 2)]
    cat = concat_systems([pressure_velocity(*sh, seed=66 + k) for k, sh in enumerate(shapes)])
    for precision in (P.PRECISION_FP64, P.PRECISION_MIXED):
        z, zr, _ = _cycle_pair(cat, 1, precision)
        _agree(z, zr, _tol(precision))


@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
def test_w_cycle_solves(precision):
    """Forward and transposed AMG-BiCGStab with the W-cycle meet the
    tolerance (residuals recomputed by the oracle) and land within 1e-6 of
    the oracle's solution, with fewer iterations than the V-cycle."""
    _say("w-cycle solves", precision)
    s = pressure_velocity(24, 22, 20, seed=67)
    A = O.from_system(s)
    At = O.transpose(A)
    xref, st = O.fgmres(A, s["b"], prec=O.PREC_BJACOBI, tol=1e-12, maxit=20000, restart=60)
    assert st["status"] == O.OK
    its = {}
    for wl in (0, 1):
        with P.System.from_dict(s) as sysm:
            sysm.setup(precond=P.PREC_AMG, precision=precision, tol=1e-8, w_levels=wl)
            x, st = sysm.solve(s["b"])
            assert st["status"] == P.OK and st["precision_fallback"] == 0
            xn = _np(x)
            assert O.relres(A, s["b"], xn) <= 1e-8 * 1.0001
            its[wl] = st["iterations"]
            if wl == 1:
                lam, stt = sysm.solve_transpose(s["b"])
                assert stt["status"] == P.OK
                assert O.relres(At, s["b"], _np(lam)) <= 1e-8 * 1.0001
                sysm.setup(precond=P.PREC_AMG, precision=precision, tol=1e-11, w_levels=1)
                xv, stv = sysm.solve(s["b"])
                assert stv["status"] == P.OK
                e = np.linalg.norm(_np(xv) - xref) / np.linalg.norm(xref)
                assert e <= 1e-6, e
    assert its[1] < its[0], its


def test_w_levels_out_of_range_is_refused():
    s = pressure_velocity(4, 4, 3, seed=68)
    with P.System.from_dict(s) as sysm:
        with pytest.raises(P.CbsError):
            sysm.setup(precond=P.PREC_AMG, w_levels=-1)


@pytest.mark.parametrize("tail", [-1, 0])
@pytest.mark.parametrize("w_levels", [0, 1])
@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
def test_coarse_damping_matches_oracle(precision, w_levels, tail):
    """coarse_omega: the block-Jacobi damping of every level below level 0
    (the per-step kernels, the zero-guess sweeps fused into the restriction
    and the one-workgroup tail), against the oracle's cycle with the same
    two dampings."""
    _say("coarse damping", precision, "w_levels", w_levels, "tail", tail)
    s = pressure_velocity(14, 12, 11, seed=69)
    z, zr, _ = _cycle_pair(s, w_levels, precision, tail=tail, coarse_omega=1.3)
    _agree(z, zr, _tol(precision))
    z1, _, _ = _cycle_pair(s, w_levels, precision, tail=tail)
    assert np.linalg.norm(z1 - zr) > 1e3 * _tol(precision) * np.linalg.norm(zr)   # the damping is applied


def test_coarse_damping_level_kernel():
    """cbs_level_apply's sweep on a coarse level uses coarse_omega, on level 0
    omega: y = x + w D^{-1} (b - A x) against the oracle's sweep."""
    s = pressure_velocity(12, 10, 9, seed=70)
    n = int(s["n"])
    with P.System.from_dict(s) as sysm:
        sysm.setup(precond=P.PREC_AMG, coarse_max=8, omega=0.8, coarse_omega=1.25)
        rng = np.random.default_rng(3)
        for lev, w in ((0, 0.8), (1, 1.25)):
            lv = sysm.get_level(lev)
            N = lv["N"]
            A = O.BCSR(N, n, _np(lv["row_ptr"]), _np(lv["col"]), _np(lv["vals"]))
            b = rng.standard_normal((N, n)); x = rng.standard_normal((N, n))
            y = _np(sysm.level_apply(lev, P.LEVEL_SWEEP, b, x))
            rows = np.repeat(np.arange(N), np.diff(A.row_ptr))
            D = A.vals.reshape(-1, n, n)[rows == A.col]
            yr = O.bjacobi_sweep(A, O.blockinv(D), b, x, w)
            _agree(y, yr.reshape(N, n), 1e-13)
        with pytest.raises(P.CbsError):
            sysm.setup(precond=P.PREC_AMG, coarse_omega=-1.0)
