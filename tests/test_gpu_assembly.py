"""Device assembly of the density-based coupled matrix (cbs_assemble_luo)
against the oracle's face loop (Sec. 2.1, Eqs. discretBackward, approxJac1,
approxJac2): element by element on several mesh sizes, with and without the
optional terms, in a batch; the assembled system solves like the oracle's;
unphysical states and wrong block sizes are rejected."""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import concat_systems, luo_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2403_07882_amd as P  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _np(t):
    return t.detach().cpu().numpy()


def _blank(d):
    """An LDU system with d's faces and zero coefficients."""
    N, F = d["N"], d["F"]
    return {"N": N, "F": F, "n": 5, "lower_addr": d["lower_addr"], "upper_addr": d["upper_addr"],
            "diag": np.zeros((N, 5, 5)), "upper": np.zeros((F, 5, 5)), "lower": np.zeros((F, 5, 5)),
            "b": np.zeros((N, 5))}


def _gpu_vals(sysm):
    sysm.setup(precond=P.PREC_NONE)
    return _np(sysm.get_level(0)["vals"])


def _close(got, ref):
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max()
    assert err <= 1e-13 * scale, (err, scale)


@pytest.mark.parametrize("shape", [(12, 10, 9), (7, 1, 1), (1, 1, 1), (33, 17, 5)])
@pytest.mark.parametrize("optional", [True, False])
def test_assembly_matches_oracle(shape, optional):
    _say("assembly", shape, optional)
    d = luo_inputs(*shape, seed=sum(shape))
    ref = O.luo_assemble(d, with_visc=optional, with_dt=optional)
    A = O.from_system(ref)
    with P.System.from_dict(_blank(d)) as sysm:
        sysm.assemble_luo(d["Q"], d["Sf"], d["lam_visc"] if optional else None, d["v_dt"] if optional else None,
                          d["gamma"])
        vals = _gpu_vals(sysm)
        lv0 = sysm.get_level(0)
        assert np.array_equal(_np(lv0["row_ptr"]), A.row_ptr) and np.array_equal(_np(lv0["col"]), A.col)
    _close(vals, A.vals)


def test_assembly_in_a_batch_matches_oracle_per_system():
    _say("assembly batch")
    ds = [luo_inputs(6, 5, 4, seed=1), luo_inputs(3, 3, 2, seed=2), luo_inputs(9, 4, 3, seed=3)]
    cat = concat_systems([_blank(d) for d in ds])
    Q = np.concatenate([d["Q"] for d in ds])
    Sf = np.concatenate([d["Sf"] for d in ds])
    lv = np.concatenate([d["lam_visc"] for d in ds])
    vd = np.concatenate([d["v_dt"] for d in ds])
    with P.System.from_dict(cat) as sysm:
        sysm.assemble_luo(Q, Sf, lv, vd, 1.4)
        vals = _gpu_vals(sysm)
    # the batch is block diagonal: each system's rows and slots in order
    _close(vals, np.concatenate([O.from_system(O.luo_assemble(d)).vals for d in ds]))


@pytest.mark.parametrize("precision", [P.PRECISION_FP64, P.PRECISION_MIXED])
def test_assembled_system_solves_like_the_oracle_matrix(precision):
    """Assemble, set up AMG, solve and solve transposed: the solutions meet
    the tolerance on the oracle's matrix; re-assembling new states on the
    same handle (reuse_aggregates) solves too."""
    _say("assembly solve", precision)
    d = luo_inputs(16, 14, 12, seed=5)
    A = O.from_system(O.luo_assemble(d))
    b = np.random.default_rng(6).uniform(-1, 1, (d["N"], 5))
    with P.System.from_dict(_blank(d)) as sysm:
        sysm.assemble_luo(d["Q"], d["Sf"], d["lam_visc"], d["v_dt"], d["gamma"])
        sysm.setup(precond=P.PREC_AMG, precision=precision, tol=1e-10)
        x, st = sysm.solve(b)
        lam, stt = sysm.solve_transpose(b)
        assert st["status"] == P.OK and stt["status"] == P.OK, (st, stt)
        assert O.relres(A, b, _np(x)) <= 1e-10 * 1.0001
        assert O.relres(O.transpose(A), b, _np(lam)) <= 1e-10 * 1.0001
        d2 = luo_inputs(16, 14, 12, seed=7)
        A2 = O.from_system(O.luo_assemble(d2))
        sysm.assemble_luo(d2["Q"], d2["Sf"], d2["lam_visc"], d2["v_dt"], d2["gamma"])
        sysm.setup(precond=P.PREC_AMG, precision=precision, tol=1e-10, reuse_aggregates=1)
        x2, st2 = sysm.solve(b)
        assert st2["status"] == P.OK, st2
        assert O.relres(A2, b, _np(x2)) <= 1e-10 * 1.0001


def test_assembly_rejects_unphysical_states_and_other_block_sizes():
    _say("assembly errors")
    d = luo_inputs(4, 3, 3, seed=8)
    Q = d["Q"].copy()
    Q[5, 4] = 0.1 * Q[5, 4] - 10.0            # negative pressure in one cell
    with P.System.from_dict(_blank(d)) as sysm:
        with pytest.raises(P.CbsError) as e:
            sysm.assemble_luo(Q, d["Sf"], d["lam_visc"], d["v_dt"], d["gamma"])
        assert e.value.code == P.ERR_NONFINITE
        with pytest.raises(P.CbsError):
            sysm.assemble_luo(d["Q"], d["Sf"], None, None, 1.0)
        sysm.assemble_luo(d["Q"], d["Sf"], None, None, 1.4)      # the handle is still usable
        # a mildly negative pressure whose coefficients all stay finite (the
        # Roe average over each of its faces still has a positive c~^2)
        rho = d["Q"][5, 0]
        u = d["Q"][5, 1:4] / rho
        Q = d["Q"].copy()
        Q[5, 4] = -1e-2 / (d["gamma"] - 1.0) + 0.5 * rho * u @ u
        with pytest.raises(O.OracleError):
            O.luo_assemble(dict(d, Q=Q))
        with pytest.raises(P.CbsError) as e:
            sysm.assemble_luo(Q, d["Sf"], d["lam_visc"], d["v_dt"], d["gamma"])
        assert e.value.code == P.ERR_NONFINITE
        Q = d["Q"].copy()
        Q[7, 0] = -Q[7, 0]                        # negative density
        with pytest.raises(P.CbsError) as e:
            sysm.assemble_luo(Q, d["Sf"], d["lam_visc"], d["v_dt"], d["gamma"])
        assert e.value.code == P.ERR_NONFINITE
        sysm.assemble_luo(d["Q"], d["Sf"], d["lam_visc"], d["v_dt"], d["gamma"])
    s4 = _blank(d)
    s4.update(n=4, diag=np.zeros((d["N"], 4, 4)), upper=np.zeros((d["F"], 4, 4)), lower=np.zeros((d["F"], 4, 4)))
    with P.System.from_dict(s4) as sysm:
        with pytest.raises(P.CbsError) as e:
            sysm.assemble_luo(d["Q"], d["Sf"])
        assert e.value.code == P.ERR_ARG


# ------------------------------------------------ pressure-based (p, U) blocks
from workloads import pu_inputs  # noqa: E402


def _blank4(d):
    N, F = d["N"], d["F"]
    return {"N": N, "F": F, "n": 4, "lower_addr": d["lower_addr"], "upper_addr": d["upper_addr"],
            "diag": np.zeros((N, 4, 4)), "upper": np.zeros((F, 4, 4)), "lower": np.zeros((F, 4, 4)),
            "b": np.zeros((N, 4))}


def _pu_args(d, with_add=True):
    return (d["Sf"], d["fx"], d["d"], d["flux"], d["nu"], d["vol"],
            d["uu_add"] if with_add else None, d["pp_add"] if with_add else None)


@pytest.mark.parametrize("shape", [(12, 10, 9), (7, 1, 1), (1, 1, 1), (33, 17, 5)])
@pytest.mark.parametrize("with_add", [True, False])
def test_pu_assembly_matches_oracle(shape, with_add):
    _say("pu assembly", shape, with_add)
    d = pu_inputs(*shape, seed=sum(shape) + 1)
    A = O.from_system(O.pu_assemble(d, with_add=with_add))
    with P.System.from_dict(_blank4(d)) as sysm:
        sysm.assemble_pu(*_pu_args(d, with_add))
        vals = _gpu_vals(sysm)
        lv0 = sysm.get_level(0)
        assert np.array_equal(_np(lv0["row_ptr"]), A.row_ptr) and np.array_equal(_np(lv0["col"]), A.col)
    _close(vals, A.vals)


def test_pu_assembly_batch_solve_and_errors():
    """A batch matches the oracle system by system; an assembled system
    solves (forward and transposed, mixed AMG) to the tolerance on the
    oracle's matrix; a 5 x 5 handle is refused."""
    _say("pu assembly batch and solve")
    ds = [pu_inputs(6, 5, 4, seed=31), pu_inputs(3, 3, 2, seed=32), pu_inputs(9, 4, 3, seed=33)]
    cat = concat_systems([_blank4(d) for d in ds])
    args = [np.concatenate([a[k] for a in ds]) for k in ("Sf", "fx", "d", "flux", "nu", "vol", "uu_add", "pp_add")]
    with P.System.from_dict(cat) as sysm:
        sysm.assemble_pu(*args)
        vals = _gpu_vals(sysm)
    _close(vals, np.concatenate([O.from_system(O.pu_assemble(d)).vals for d in ds]))
    d = pu_inputs(16, 14, 12, seed=5)
    A = O.from_system(O.pu_assemble(d))
    b = np.random.default_rng(6).uniform(-1, 1, (d["N"], 4))
    with P.System.from_dict(_blank4(d)) as sysm:
        sysm.assemble_pu(*_pu_args(d))
        sysm.setup(precond=P.PREC_AMG, precision=P.PRECISION_MIXED, tol=1e-10)
        x, st = sysm.solve(b)
        lam, stt = sysm.solve_transpose(b)
    assert st["status"] == P.OK and stt["status"] == P.OK, (st, stt)
    assert O.relres(A, b, _np(x)) <= 1e-10 * 1.0001
    assert O.relres(O.transpose(A), b, _np(lam)) <= 1e-10 * 1.0001
    e = luo_inputs(3, 3, 2, seed=1)
    with P.System.from_dict(_blank(e)) as s5:
        with pytest.raises(P.CbsError) as err:
            s5.assemble_pu(*_pu_args(pu_inputs(3, 3, 2, seed=1)))
        assert err.value.code == P.ERR_ARG


def test_both_assemblies_at_full_size_match_the_oracle():
    """The 100 x 100 x 100 box that bench.py --assembly times (1M cells,
    6.94M blocks), every element of both matrices against the oracle."""
    _say("assembly full size")
    d = luo_inputs(100, 100, 100, seed=0)
    A = O.from_system(O.luo_assemble(d))
    with P.System.from_dict(_blank(d)) as sysm:
        sysm.assemble_luo(d["Q"], d["Sf"], d["lam_visc"], d["v_dt"], d["gamma"])
        vals = _gpu_vals(sysm)
    _close(vals, A.vals)
    del vals, A
    e = pu_inputs(100, 100, 100, seed=0)
    B = O.from_system(O.pu_assemble(e))
    with P.System.from_dict(_blank4(e)) as sysm:
        sysm.assemble_pu(*_pu_args(e))
        vals = _gpu_vals(sysm)
    _close(vals, B.vals)
