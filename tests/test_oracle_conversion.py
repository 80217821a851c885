"""Pins for the oracle's LDU -> block-CSR conversion and field packing.

The conversion is an exact permutation (Sec. 2.3, Alg. amgxFoam, Fig.
block_amgx), so its result is unique and checked bit for bit: against
hand-derived fixtures, against a dense reconstruction from the LDU arrays,
and by the LDU -> BCSR -> LDU round trip.
"""
import json
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle as O
from workloads import jacobian_box, pressure_velocity

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _dense_from_ldu(N, n, la, ua, diag, upper, lower):
    """Brute-force dense matrix straight from the storage reading."""
    A = np.zeros((N * n, N * n))
    for i in range(N):
        A[i * n:(i + 1) * n, i * n:(i + 1) * n] = diag[i]
    for f in range(len(la)):
        l, u = la[f], ua[f]
        A[l * n:(l + 1) * n, u * n:(u + 1) * n] = upper[f]
        A[u * n:(u + 1) * n, l * n:(l + 1) * n] = lower[f]
    return A


@pytest.mark.parametrize("name", ["ldu_3cell_n2.json", "ldu_2cell_n1.json"])
def test_golden_conversion(name):
    g = _load(name)
    A, ds, us, ls = O.ldu_to_bcsr(g["N"], g["n"], g["lower_addr"], g["upper_addr"],
                                  np.array(g["diag"], float), np.array(g["upper"], float),
                                  np.array(g["lower"], float))
    assert A.row_ptr.tolist() == g["expect_row_ptr"]
    assert A.col.tolist() == g["expect_col"]
    assert A.vals.ravel().tolist() == [float(v) for v in g["expect_vals"]]
    assert ds.tolist() == g["expect_diag_slot"]
    assert us.tolist() == g["expect_upper_slot"]
    assert ls.tolist() == g["expect_lower_slot"]
    assert np.array_equal(A.dense(), np.array(g["expect_dense"], float))
    y = O.spmv(A, np.array(g["x"], float).reshape(g["N"], g["n"]))
    assert np.array_equal(y.ravel(), np.array(g["expect_Ax"], float))


def test_golden_2cell_solution():
    g = _load("ldu_2cell_n1.json")
    A = O.ldu_to_bcsr(g["N"], 1, g["lower_addr"], g["upper_addr"], np.array(g["diag"], float),
                      np.array(g["upper"], float), np.array(g["lower"], float))[0]
    x = O.dense_solve(A.dense(), np.array(g["b"], float))
    exact = np.array([a / b for a, b in g["expect_solution_fraction"]])
    assert np.allclose(x, exact, rtol=1e-15, atol=0)
    xk, st_ = O.bicgstab(A, np.array(g["b"], float).reshape(2, 1), tol=1e-14)
    assert np.allclose(xk.ravel(), exact, rtol=1e-13)


def _roundtrip_check(s):
    N, n = s["N"], s["n"]
    A, ds, us, ls = O.ldu_to_bcsr(N, n, s["lower_addr"], s["upper_addr"],
                                  s["diag"], s["upper"], s["lower"])
    # slot maps give back the LDU arrays bit for bit
    assert np.array_equal(A.vals[ds], s["diag"])
    assert np.array_equal(A.vals[us], s["upper"])
    assert np.array_equal(A.vals[ls], s["lower"])
    # every slot is hit exactly once
    allslots = np.concatenate([ds, us, ls])
    assert np.array_equal(np.sort(allslots), np.arange(A.nnzb))
    # columns strictly ascending inside each row
    for i in range(N):
        c = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0)
    return A


def test_roundtrip_density_box():
    s = jacobian_box(5, 4, 3, n=5, seed=3)
    A = _roundtrip_check(s)
    D = _dense_from_ldu(s["N"], 5, s["lower_addr"], s["upper_addr"], s["diag"], s["upper"], s["lower"])
    assert np.array_equal(A.dense(), D)


def test_roundtrip_permuted_pressure_velocity():
    s = pressure_velocity(4, 3, 5, seed=2)
    assert np.any(s["lower_addr"] > s["upper_addr"])          # both orientations occur
    A = _roundtrip_check(s)
    D = _dense_from_ldu(s["N"], 4, s["lower_addr"], s["upper_addr"], s["diag"], s["upper"], s["lower"])
    assert np.array_equal(A.dense(), D)


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 9), st.integers(1, 5), st.data())
def test_fuzz_random_face_lists(N, n, data):
    pairs = [(i, j) for i in range(N) for j in range(i + 1, N)]
    chosen = data.draw(st.lists(st.sampled_from(pairs), unique=True, max_size=len(pairs))) if pairs else []
    flips = data.draw(st.lists(st.booleans(), min_size=len(chosen), max_size=len(chosen)))
    la = np.array([b if f else a for (a, b), f in zip(chosen, flips)], np.int32)
    ua = np.array([a if f else b for (a, b), f in zip(chosen, flips)], np.int32)
    rng = np.random.default_rng(len(chosen) * 31 + N)
    F = la.size
    s = {"N": N, "n": n, "F": F, "lower_addr": la, "upper_addr": ua,
         "diag": rng.standard_normal((N, n, n)), "upper": rng.standard_normal((F, n, n)),
         "lower": rng.standard_normal((F, n, n))}
    A = _roundtrip_check(s)
    D = _dense_from_ldu(N, n, la, ua, s["diag"], s["upper"], s["lower"])
    assert np.array_equal(A.dense(), D)


@pytest.mark.parametrize("la,ua", [([0], [3]), ([-1], [1]), ([1], [1]), ([0, 1], [1, 0]), ([0, 0], [2, 2])])
def test_bad_patterns_rejected(la, ua):
    N, n = 3, 2
    F = len(la)
    with pytest.raises(O.OracleError) as e:
        O.ldu_to_bcsr(N, n, la, ua, np.ones((N, n, n)), np.ones((F, n, n)), np.ones((F, n, n)))
    assert e.value.code == O.ERR_PATTERN


def test_no_faces_is_block_diagonal():
    rng = np.random.default_rng(0)
    D = rng.standard_normal((4, 3, 3))
    A, ds, _, _ = O.ldu_to_bcsr(4, 3, [], [], D, np.zeros((0, 3, 3)), np.zeros((0, 3, 3)))
    assert A.row_ptr.tolist() == [0, 1, 2, 3, 4] and A.col.tolist() == [0, 1, 2, 3]
    assert np.array_equal(A.vals, D)


def test_pack_unpack_roundtrip_bitexact():
    rng = np.random.default_rng(5)
    soa = rng.standard_normal((5, 37))
    aos = O.pack(soa)
    assert aos.shape == (37, 5)
    for v in range(5):                      # AoS: cell-major, variable-minor
        assert np.array_equal(aos[:, v], soa[v])
    assert np.array_equal(O.unpack(aos), soa)
