"""The allocation-free density-based assembly (cbs_assemble_luo_noalloc)
against the allocating entry point (cbs_assemble_luo) and the oracle's face
loop (Sec. 2.1, Eqs. discretBackward, approxJac1, approxJac2).  Calls run in a
row on the one per-device scratch array, the later ones on smaller systems, so
anything a call leaves behind there (partial results, the error flag) would
show up in the next one."""
import sys

import numpy as np
import pytest

import oracle as O
from workloads import luo_inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2403_07882_amd as P  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _np(t):
    return t.detach().cpu().numpy()


def _blank(d):
    N, F = d["N"], d["F"]
    return {"N": N, "F": F, "n": 5, "lower_addr": d["lower_addr"], "upper_addr": d["upper_addr"],
            "diag": np.zeros((N, 5, 5)), "upper": np.zeros((F, 5, 5)), "lower": np.zeros((F, 5, 5)),
            "b": np.zeros((N, 5))}


def _vals(sysm):
    return _np(sysm.get_bcsr()["vals"])


def _assemble_both(d):
    """(values from cbs_assemble_luo, values from cbs_assemble_luo_noalloc)."""
    args = (d["Q"], d["Sf"], d["lam_visc"], d["v_dt"], d["gamma"])
    with P.System.from_dict(_blank(d)) as a:
        a.assemble_luo(*args)
        ref = _vals(a)
    with P.System.from_dict(_blank(d)) as b:
        b.assemble_luo_noalloc(*args)
        got = _vals(b)
    return ref, got


def test_noalloc_assembly_matches_allocating_entry_point_on_calls_in_a_row():
    big, small = (24, 20, 18), (9, 7, 5)
    for k, shape in enumerate([big, small]):
        _say("no-alloc assembly, call", k + 1, shape)
        d = luo_inputs(*shape, seed=40 + k)
        ref, got = _assemble_both(d)
        # same kernels on other memory: identical values
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
        A = O.from_system(O.luo_assemble(d))
        assert np.abs(got - A.vals).max() <= 1e-13 * np.abs(A.vals).max()


def test_noalloc_assembly_error_flag_does_not_leak_into_the_next_call():
    _say("no-alloc assembly, error then a smaller valid call")
    bad = luo_inputs(10, 9, 8, seed=50)
    bad["Q"] = bad["Q"].copy()
    i = 17
    ke = 0.5 * (bad["Q"][i, 1:4] ** 2).sum() / bad["Q"][i, 0]
    bad["Q"][i, 4] = ke - 1e-2 / (bad["gamma"] - 1.0)     # pressure -1e-2: not physical
    with P.System.from_dict(_blank(bad)) as s1:
        with pytest.raises(P.CbsError) as ei:
            s1.assemble_luo_noalloc(bad["Q"], bad["Sf"], bad["lam_visc"], bad["v_dt"], bad["gamma"])
        assert ei.value.code == P.ERR_NONFINITE
    d = luo_inputs(6, 5, 4, seed=51)
    ref, got = _assemble_both(d)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))


def test_noalloc_assembly_refuses_a_system_beyond_its_scratch():
    _say("no-alloc assembly, oversize")
    N = 1_000_000                      # 9 N doubles of per-cell scratch > 64 MiB
    s = {"N": N, "F": 0, "n": 5, "lower_addr": np.zeros(0, np.int32), "upper_addr": np.zeros(0, np.int32),
         "diag": np.zeros((N, 5, 5)), "upper": np.zeros((0, 5, 5)), "lower": np.zeros((0, 5, 5))}
    Q = np.tile(np.array([1.0, 0.1, 0.0, 0.0, 2.5]), (N, 1))
    with P.System.from_dict(s) as sysm:
        with pytest.raises(P.CbsError) as ei:
            sysm.assemble_luo_noalloc(Q, np.zeros((0, 3)), None, None, 1.4)
        assert ei.value.code == P.ERR_ARG
        assert "scratch" in str(ei.value)
