"""Pins for the oracle's FP32 emulation of the block-Jacobi V-cycle (the
mixed-precision study tool: float level values, vectors and sums, FP64 block
inverses and coarsest solve).  It is not a parity target; these tests fix
that the casts are really applied, that the emulated cycle stays within
float rounding of the FP64 cycle, and that it serves as the preconditioner
of the FP64 Krylov loop without stagnation."""
import numpy as np
import pytest

import oracle as O
from workloads import jacobian_box, pressure_velocity

EPS32 = np.finfo(np.float32).eps


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("scaled", [True, False])
@pytest.mark.parametrize("case", ["pu", "box5"])
def test_fp32_cycle_is_within_float_rounding_of_the_fp64_cycle(case, scaled):
    """The emulated cycle is the FP64 cycle up to float rounding: away from
    it by more than FP64 rounding could explain (the casts happen) and by
    less than a few hundred float epsilons (nothing else differs: a dropped
    or sign-flipped term of a sweep, the residual or the coarse correction
    moves z by O(1))."""
    s = pressure_velocity(8, 7, 6, seed=21) if case == "pu" else jacobian_box(7, 6, 6, seed=22)
    A = O.from_system(s)
    amg = O.AMG(A, coarse_max=8, nu1=2, nu2=2, omega=0.9)
    assert amg.levels >= 3
    r = np.random.default_rng(23).standard_normal((A.N, A.n))
    z64 = amg.apply(r)
    z32 = amg.apply_fp32(r, scaled=scaled)
    d = _rel(z32, z64)
    assert 1e3 * np.finfo(np.float64).eps < d < 300 * EPS32, d
    # every entry is a float: the result was formed in single precision
    assert np.array_equal(z32, z32.astype(np.float32).astype(np.float64))


def test_the_two_sweep_forms_differ_only_by_rounding():
    """Row-scaled sweeps (S = fl(D^-1 A)) and FP64-D^-1 sweeps are the same
    smoother in exact arithmetic."""
    s = pressure_velocity(8, 7, 6, seed=24)
    A = O.from_system(s)
    amg = O.AMG(A, coarse_max=8, nu1=2, nu2=2, omega=0.9)
    r = np.random.default_rng(25).standard_normal((A.N, A.n))
    za, zb = amg.apply_fp32(r, scaled=True), amg.apply_fp32(r, scaled=False)
    assert 0.0 < _rel(za, zb) < 300 * EPS32


def test_single_level_is_the_rounded_fp64_solve():
    """With one level the emulated cycle is the FP64 dense solve of the
    float-rounded right side, rounded to float."""
    s = jacobian_box(3, 2, 2, seed=26)
    A = O.from_system(s)
    amg = O.AMG(A, coarse_max=1000)
    assert amg.levels == 1
    r = np.random.default_rng(27).standard_normal((A.N, A.n))
    r32 = r.astype(np.float32).astype(np.float64)
    x = np.linalg.solve(A.dense(), r32.ravel())
    z = amg.apply_fp32(r).ravel()
    assert np.array_equal(z, z.astype(np.float32).astype(np.float64))
    assert np.max(np.abs(z - x)) <= 2 * EPS32 * np.max(np.abs(x))


@pytest.mark.parametrize("solver", ["bicgstab", "fgmres"])
def test_fp32_preconditioner_does_not_stall_the_fp64_loop(solver):
    """FP64 BiCGStab and FGMRES(30) with the FP32-emulated V-cycle reach a
    1e-10 true residual, in about the iterations of the FP64 cycle."""
    s = pressure_velocity(10, 9, 8, seed=28)
    A = O.from_system(s)
    amg = O.AMG(A, coarse_max=8, nu1=2, nu2=2, omega=0.9)
    fn = getattr(O, solver)
    x64, st64 = fn(A, s["b"], prec=O.PREC_AMG, amg=amg, tol=1e-10, maxit=500)
    for kind in (O.PREC_AMG_FP32, O.PREC_AMG_FP32_UNSCALED):
        x32, st32 = fn(A, s["b"], prec=kind, amg=amg, tol=1e-10, maxit=500)
        assert st32["status"] == O.OK and O.relres(A, s["b"], x32) <= 1e-10 * 1.0001, st32
        assert st32["iterations"] <= st64["iterations"] + 3, (st32, st64)


def test_fp32_emulation_refuses_coloured_smoothers():
    s = pressure_velocity(6, 5, 4, seed=29)
    A = O.from_system(s)
    amg = O.AMG(A, coarse_max=8, smoother=O.SMOOTH_DILU)
    with pytest.raises(O.OracleError):
        amg.apply_fp32(np.ones((A.N, A.n)))
