"""The V-cycle tail (every level from the first small one down to the coarsest
run by one workgroup) against the oracle's V-cycle on the GPU's hierarchy,
for every block size, both precisions, uneven sweep counts and a batch of
systems; and the solves (forward and transposed) with the tail on and off.

tail_rows = -1 switches the tail off (one kernel per step, as on large
levels); 100000 starts it at level 1, so that almost the whole cycle runs in
the one workgroup.
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



def _vcycle_pair(s, tail, precision, pre, post, omega=0.9, seed=0):
    """GPU V-cycle z = M r and the oracle's V-cycle on the GPU's level-0
    numbering and aggregates."""
    N, n = int(s["N"]), int(s["n"])
    with P.System.from_dict(s) as sysm:
        sysm.setup(precond=P.PREC_AMG, precision=precision, coarse_max=8, pre_sweeps=pre, post_sweeps=post,
                   omega=omega, tail_rows=tail)
        nlev = sysm.info()["levels"]
        assert nlev >= 3
        lv0 = sysm.get_level(0)
        order = _np(lv0["order"])
        A0 = O.BCSR(N, n, _np(lv0["row_ptr"]), _np(lv0["col"]), _np(lv0["vals"]))
        aggs = [_np(sysm.get_level(l)["agg"]) for l in range(nlev - 1)]
        r = np.random.default_rng(seed).standard_normal((N, n))
        z = _np(sysm.apply_precond(r))
    amg = O.AMG(A0, nu1=pre, nu2=post, omega=omega, aggs=aggs)
    zr_int = amg.apply(r[order])
    zr = np.empty_like(zr_int)
    zr[order] = zr_int
    return z, zr


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
def test_tail_vcycle_matches_oracle_every_block_size(n, precision):
    _say("tail vcycle n", n, "precision", precision)
    s = pressure_velocity(11, 9, 8, seed=41) if n == 4 else jacobian_box(11, 9, 8, n=n, seed=40 + n)
    z, zr = _vcycle_pair(s, ALL, precision, 2, 2)
    tol = 1e-11 if precision == P.PRECISION_FP64 else 1e-5
    _agree(z, zr, tol)


@pytest.mark.parametrize("tail", [-1, 0, ALL])
@pytest.mark.parametrize("pre,post", [(1, 3), (0, 2), (3, 0), (0, 0)])
def test_tail_vcycle_uneven_sweeps(tail, pre, post):
    _say("tail vcycle sweeps", pre, post, "tail", tail)
    s = pressure_velocity(12, 10, 9, seed=42)
    z, zr = _vcycle_pair(s, tail, P.PRECISION_FP64, pre, post, omega=0.8)
    _agree(z, zr, 1e-11)
    z, zr = _vcycle_pair(s, tail, P.PRECISION_MIXED, pre, post, omega=0.8)
    _agree(z, zr, 1e-5)


@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
def test_tail_vcycle_beyond_64kb_of_lds(precision):
    """A tail whose first level holds a few hundred block rows: its staged
    vectors and patterns need more than 64 KB of LDS (a gfx950 workgroup may
    hold 160 KB)."""
    _say("tail vcycle large LDS", precision)
    s = pressure_velocity(24, 20, 18, seed=44)
    z, zr = _vcycle_pair(s, ALL, precision, 2, 2)
    _agree(z, zr, 1e-11 if precision == P.PRECISION_FP64 else 1e-5)


def test_tail_vcycle_batch_of_uneven_systems():
    """A batch: the coarsest level holds one dense inverse per system."""
    _say("tail vcycle batch")
    shapes = [(7, 6, 5), (4, 4, 3), (9, 5, 5), (3, 3, 2)]
    cat = concat_systems([pressure_velocity(*sh, seed=50 + k) for k, sh in enumerate(shapes)])
    for precision, tol in ((P.PRECISION_FP64, 1e-11), (P.PRECISION_MIXED, 1e-5)):
        z, zr = _vcycle_pair(cat, ALL, precision, 2, 2)
        _agree(z, zr, tol)


@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
def test_solves_with_and_without_tail(precision):
    """Forward and transposed AMG-BiCGStab meet the tolerance with the tail on
    and off and land on the same solution."""
    _say("tail solves", precision)
    s = pressure_velocity(14, 12, 10, seed=43)
    A = O.from_system(s)
    At = O.transpose(A)
    xs, ls = {}, {}
    for tail in (-1, ALL):
        with P.System.from_dict(s) as sysm:
            sysm.setup(precond=P.PREC_AMG, precision=precision, tol=1e-10, coarse_max=8, tail_rows=tail)
            x, st = sysm.solve(s["b"])
            lam, stt = sysm.solve_transpose(s["b"])
        assert st["status"] == P.OK and st["precision_fallback"] == 0, st
        assert stt["status"] == P.OK, stt
        xs[tail], ls[tail] = _np(x), _np(lam)
        assert O.relres(A, s["b"], xs[tail]) <= 1e-10 * 1.0001
        assert O.relres(At, s["b"], ls[tail]) <= 1e-10 * 1.0001
    for d in (xs, ls):
        assert np.linalg.norm(d[-1] - d[ALL]) <= 1e-7 * np.linalg.norm(d[-1])


@pytest.mark.parametrize("tail", [-1, ALL])
@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
@pytest.mark.parametrize("n", [4, 5])
def test_transposed_vcycle_matches_oracle_on_transposed_matrix(n, precision, tail):
    """The preconditioner of the transposed solve is the oracle's V-cycle built
    on A^T with the same aggregates (Galerkin operators of A^T, block inverses
    of A^T's diagonal); in mixed precision its sweeps run on the row-scaled
    values D^{-T} A^T."""
    _say("transposed vcycle n", n, "precision", precision, "tail", tail)
    s = pressure_velocity(11, 9, 8, seed=44) if n == 4 else jacobian_box(11, 9, 8, n=5, seed=45)
    N = int(s["N"])
    with P.System.from_dict(s) as sysm:
        sysm.setup(precond=P.PREC_AMG, precision=precision, coarse_max=8, pre_sweeps=2, post_sweeps=2,
                   omega=0.9, tail_rows=tail)
        nlev = sysm.info()["levels"]
        assert nlev >= 3
        lv0 = sysm.get_level(0)
        order = _np(lv0["order"])
        A0 = O.BCSR(N, n, _np(lv0["row_ptr"]), _np(lv0["col"]), _np(lv0["vals"]))
        aggs = [_np(sysm.get_level(l)["agg"]) for l in range(nlev - 1)]
        r = np.random.default_rng(3).standard_normal((N, n))
        z = _np(sysm.apply_precond(r, transpose=True))
        zf = _np(sysm.apply_precond(r))
    amg = O.AMG(O.transpose(A0), nu1=2, nu2=2, omega=0.9, aggs=aggs)
    zr_int = amg.apply(r[order])
    zr = np.empty_like(zr_int)
    zr[order] = zr_int
    tol = 1e-11 if precision == P.PRECISION_FP64 else 1e-5
    _agree(z, zr, tol)
    assert np.linalg.norm(zf - zr) > 1e3 * tol * np.linalg.norm(zr)     # not the forward cycle
