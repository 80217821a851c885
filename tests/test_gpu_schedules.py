"""Every schedule of the block-row kernels (1, 2 or 4 blocks loaded per step,
normal or non-temporal matrix loads), forced through the schedule option, on a
level-0 operator of more than 65,536 block rows: at that size setup times the
six variants and keeps one, and the V-cycle prolongs level 0 in a pass of its
own instead of inside the first post-smoothing sweep.  The residual and the
block-Jacobi sweep of every smoothed level, the V-cycle and the caller-order
FP64 product are compared with the oracle element by element, in FP64 and in
mixed precision (Sec. 2.3: block smoothers, aggregation AMG; reading R11)."""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import pressure_velocity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2403_07882_amd as P  # noqa: E402

# 48 x 40 x 36 = 69,120 cells: level 0 at or above the 65,536-row threshold
SHAPE = (48, 40, 36)
OMEGA = 0.9


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def system():
    s = pressure_velocity(*SHAPE, seed=8)
    assert s["N"] >= 65536
    return s, O.from_system(s)


def _close(got, ref, rel):
    err = np.abs(got - ref).max()
    scale = np.abs(ref).max()
    assert err <= rel * scale, (err, scale, rel)


@pytest.mark.parametrize("schedule", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
def test_forced_schedule_matches_oracle_on_a_large_level(system, schedule, precision):
    s, A = system
    _say("schedule", schedule, "precision", precision)
    rng = np.random.default_rng(100 + schedule)
    mixed = precision == P.PRECISION_MIXED
    with P.System.from_dict(s) as sysm:
        sysm.setup(precond=P.PREC_AMG, precision=precision, omega=OMEGA, pre_sweeps=2, post_sweeps=2,
                   schedule=schedule)
        nlev = sysm.info()["levels"]
        assert nlev >= 3
        # caller-order FP64 product (its own sliced copy, same forced schedule)
        x = rng.standard_normal((A.N, 4))
        _close(_np(sysm.spmv(x)), O.spmv(A, x), 1e-14)
        lv0 = sysm.get_level(0)
        assert lv0["N"] >= 65536
        order = _np(lv0["order"])
        A0 = O.BCSR(A.N, 4, _np(lv0["row_ptr"]), _np(lv0["col"]), _np(lv0["vals"]))
        aggs = []
        for l in range(nlev - 1):
            lv = sysm.get_level(l)
            Al = O.BCSR(lv["N"], 4, _np(lv["row_ptr"]), _np(lv["col"]), _np(lv["vals"]))
            aggs.append(_np(lv["agg"]))
            b = rng.standard_normal((Al.N, 4))
            xl = rng.standard_normal((Al.N, 4))
            if mixed:                        # the kernels take FP32 inputs
                b, xl = b.astype(np.float32).astype(np.float64), xl.astype(np.float32).astype(np.float64)
            r = _np(sysm.level_apply(l, P.LEVEL_RESIDUAL, b, xl)).astype(np.float64)
            _close(r, b - O.spmv(Al, xl), 1e-6 if mixed else 1e-14)
            Dinv = O.blockinv(O.diag_blocks(Al))
            y = _np(sysm.level_apply(l, P.LEVEL_SWEEP, b, xl)).astype(np.float64)
            if mixed:    # row-scaled values: the right side is already Dinv b
                ref = xl + OMEGA * (b - np.einsum("kij,kj->ki", Dinv, O.spmv(Al, xl)))
            else:
                ref = O.bjacobi_sweep(Al, Dinv, b, xl, OMEGA)
            _close(y, ref, 1e-5 if mixed else 1e-13)
        rr = rng.standard_normal((A.N, 4))
        z = _np(sysm.apply_precond(rr))
    amg = O.AMG(A0, nu1=2, nu2=2, omega=OMEGA, aggs=aggs)
    zr_int = amg.apply(rr[order])
    zr = np.empty_like(zr_int)
    zr[order] = zr_int
    _close(z, zr, 1e-5 if mixed else 1e-11)
