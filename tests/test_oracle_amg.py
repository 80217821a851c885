"""Pins for the oracle's aggregation AMG pieces: strength weights, matching
(properties only: the heuristic has no unique answer), Galerkin coarse
operator, transfers and the V-cycle."""
import numpy as np

import oracle as O
from workloads import jacobian_box, pressure_velocity


def _P(agg, nc, n):
    """Dense piecewise-constant prolongation, block size n."""
    N = len(agg)
    P = np.zeros((N * n, nc * n))
    for i, I in enumerate(agg):
        P[i * n:(i + 1) * n, I * n:(I + 1) * n] = np.eye(n)
    return P


def test_strength_weights_brute_force():
    s = pressure_velocity(3, 3, 2, seed=0)
    A = O.from_system(s)
    w = O.strength(A)
    rows = np.repeat(np.arange(A.N), np.diff(A.row_ptr))
    Ad = A.dense(); n = 4
    blk = lambda i, j: Ad[i * n:(i + 1) * n, j * n:(j + 1) * n]
    for k in range(A.nnzb):
        i, j = rows[k], A.col[k]
        if i == j:
            assert w[k] == 0.0
            continue
        ref = 0.5 * (np.linalg.norm(blk(i, j)) + np.linalg.norm(blk(j, i))) / max(
            np.linalg.norm(blk(i, i)), np.linalg.norm(blk(j, j)))
        assert abs(w[k] - ref) <= 1e-14 * ref


def _check_aggregates(A, agg, nc, max_size):
    agg = np.asarray(agg)
    assert agg.min() == 0 and agg.max() == nc - 1
    sizes = np.bincount(agg, minlength=nc)
    assert np.all(sizes >= 1) and sizes.max() <= max_size
    # every aggregate is connected in the matrix graph
    rows = np.repeat(np.arange(A.N), np.diff(A.row_ptr))
    adj = {}
    for i, j in zip(rows, A.col):
        adj.setdefault(i, set()).add(j)
    for I in range(nc):
        mem = set(np.nonzero(agg == I)[0].tolist())
        seen, stack = set(), [next(iter(mem))]
        while stack:
            u = stack.pop()
            if u in seen:
                continue
            seen.add(u)
            stack.extend(v for v in adj[u] if v in mem and v not in seen)
        assert seen == mem


def test_matching_properties():
    s = jacobian_box(6, 6, 5, seed=1)
    A = O.from_system(s)
    agg, nc = O.match(A.N, A.row_ptr, A.col, O.strength(A))
    _check_aggregates(A, agg, nc, 3)        # pairs, plus leftovers joining a pair
    assert nc < 0.6 * A.N


def test_rap_equals_dense_galerkin_product():
    s = pressure_velocity(4, 3, 3, seed=5)
    A = O.from_system(s)
    rng = np.random.default_rng(0)
    nc = 11
    agg = np.concatenate([np.arange(nc), rng.integers(0, nc, A.N - nc)]).astype(np.int32)
    rng.shuffle(agg)
    Ac = O.rap(A, agg, nc)
    P = _P(agg, nc, 4)
    ref = P.T @ A.dense() @ P
    assert np.allclose(Ac.dense(), ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    for i in range(nc):
        assert np.all(np.diff(Ac.col[Ac.row_ptr[i]:Ac.row_ptr[i + 1]]) > 0)


def test_rap_row_sum_invariant_all_levels():
    # Variant-A Jacobian rows sum to I; Galerkin sums keep size(I) * I per coarse row.
    s = jacobian_box(8, 7, 6, seed=0)
    A = O.from_system(s)
    sizes = np.ones(A.N)
    for level in range(3):
        agg, nc = O.match(A.N, A.row_ptr, A.col, O.strength(A))
        sizes = np.bincount(agg, weights=sizes, minlength=nc)
        A = O.rap(A, agg, nc)
        rows = np.repeat(np.arange(A.N), np.diff(A.row_ptr))
        rs = np.zeros((A.N, 5, 5))
        np.add.at(rs, rows, A.vals)
        assert np.allclose(rs, sizes[:, None, None] * np.eye(5), rtol=1e-12, atol=1e-11)


def test_restrict_prolong_are_PT_and_P():
    rng = np.random.default_rng(1)
    agg = np.array([2, 0, 1, 2, 0, 1, 1], np.int32)
    r = rng.standard_normal((7, 3))
    rc = O.restrict(agg, r, 3)
    P = _P(agg, 3, 3)
    assert np.allclose(rc.ravel(), P.T @ r.ravel(), rtol=1e-15, atol=1e-15)
    e = rng.standard_normal((3, 3)); x = rng.standard_normal((7, 3))
    assert np.allclose(O.prolong_add(agg, e, x).ravel(), x.ravel() + P @ e.ravel(), rtol=1e-15)


def test_single_level_amg_is_exact_solve():
    s = jacobian_box(3, 3, 2, seed=2)
    A = O.from_system(s)
    amg = O.AMG(A, coarse_max=100)
    assert amg.levels == 1
    z = amg.apply(s["b"])
    assert np.allclose(z.ravel(), np.linalg.solve(A.dense(), s["b"].ravel()), rtol=1e-12, atol=1e-13)


def test_two_grid_without_smoothing_is_coarse_grid_correction():
    s = pressure_velocity(4, 4, 2, seed=3)
    A = O.from_system(s)
    agg, nc = O.match(A.N, A.row_ptr, A.col, O.strength(A))
    amg = O.AMG(A, nu1=0, nu2=0, aggs=[agg])
    assert amg.levels == 2
    r = np.random.default_rng(0).standard_normal((A.N, 4))
    P = _P(agg, nc, 4)
    Ac = P.T @ A.dense() @ P
    ref = P @ np.linalg.solve(Ac, P.T @ r.ravel())
    assert np.allclose(amg.apply(r).ravel(), ref, rtol=1e-11, atol=1e-12 * np.abs(ref).max())


def test_two_grid_vcycle_operator_closed_form():
    # V(1,1) with damped block Jacobi S = I - w D^{-1} A, exact coarse solve:
    # M^{-1} = [I - S (I - P Ac^{-1} P^T A) S] A^{-1} applied to r, written out densely.
    s = jacobian_box(4, 3, 2, n=3, seed=6)
    A = O.from_system(s)
    agg, nc = O.match(A.N, A.row_ptr, A.col, O.strength(A))
    w = 0.7
    amg = O.AMG(A, nu1=1, nu2=1, omega=w, aggs=[agg])
    Ad = A.dense(); n = 3
    D = np.zeros_like(Ad)
    for i in range(A.N):
        D[i * n:(i + 1) * n, i * n:(i + 1) * n] = Ad[i * n:(i + 1) * n, i * n:(i + 1) * n]
    P = _P(agg, nc, n)
    Ac = P.T @ Ad @ P
    I = np.eye(Ad.shape[0])
    S = I - w * np.linalg.solve(D, Ad)
    C = I - P @ np.linalg.solve(Ac, P.T @ Ad)
    E = S @ C @ S                          # error propagation of the cycle
    Minv = (I - E) @ np.linalg.inv(Ad)
    r = np.random.default_rng(3).standard_normal(Ad.shape[0])
    assert np.allclose(amg.apply(r.reshape(-1, n)).ravel(), Minv @ r, rtol=1e-10, atol=1e-11)


def test_amg_hierarchy_shape_and_coarse_max():
    s = pressure_velocity(12, 12, 12, seed=0)
    A = O.from_system(s)
    amg = O.AMG(A, coarse_max=32, passes=2)
    info = amg.level_info()
    assert info[0] == (A.N, A.nnzb)
    assert info[-1][0] <= 32
    for (N0, _), (N1, _) in zip(info, info[1:]):
        assert N1 < N0 / 2.5           # two passes of pairwise matching
