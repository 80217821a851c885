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


def _dense_blocks(Ad, n):
    D = np.zeros_like(Ad)
    for i in range(Ad.shape[0] // n):
        D[i * n:(i + 1) * n, i * n:(i + 1) * n] = Ad[i * n:(i + 1) * n, i * n:(i + 1) * n]
    return D


def test_three_level_w_cycle_operator_closed_form():
    # Textbook W-cycle on level 0 of a three-level hierarchy, V(1,1) with
    # damped block Jacobi and an exact solve on level 2.  The level-1 cycle
    # has error propagation E1 = S1 (I - P1 A2^{-1} P1^T A1) S1; running it
    # twice, the second from the first one's result, leaves E1^2, so the
    # level-0 coarse correction applies B1 = (I - E1^2) A1^{-1} and the cycle
    # is E0 = S0 (I - P0 B1 P0^T A0) S0, M^{-1} = (I - E0) A0^{-1}.
    s = jacobian_box(5, 4, 3, n=3, seed=7)
    A = O.from_system(s)
    n, w = 3, 0.7
    agg0, nc0 = O.match(A.N, A.row_ptr, A.col, O.strength(A))
    A1 = O.rap(A, agg0, nc0)
    agg1, nc1 = O.match(A1.N, A1.row_ptr, A1.col, O.strength(A1))
    assert 1 < nc1 < nc0 < A.N
    Ad, A1d = A.dense(), A1.dense()
    P0, P1 = _P(agg0, nc0, n), _P(agg1, nc1, n)
    assert np.allclose(A1d, P0.T @ Ad @ P0, rtol=1e-13, atol=1e-13)
    A2d = P1.T @ A1d @ P1
    I0, I1 = np.eye(Ad.shape[0]), np.eye(A1d.shape[0])
    S0 = I0 - w * np.linalg.solve(_dense_blocks(Ad, n), Ad)
    S1 = I1 - w * np.linalg.solve(_dense_blocks(A1d, n), A1d)
    E1 = S1 @ (I1 - P1 @ np.linalg.solve(A2d, P1.T @ A1d)) @ S1
    A0i, A1i = np.linalg.inv(Ad), np.linalg.inv(A1d)
    r = np.random.default_rng(5).standard_normal(Ad.shape[0])

    def cycle_op(E1k):
        B1 = (I1 - E1k) @ A1i
        E0 = S0 @ (I0 - P0 @ B1 @ P0.T @ Ad) @ S0
        return (I0 - E0) @ A0i

    zw = O.AMG(A, nu1=1, nu2=1, omega=w, aggs=[agg0, agg1], w_levels=1).apply(r.reshape(-1, n)).ravel()
    zv = O.AMG(A, nu1=1, nu2=1, omega=w, aggs=[agg0, agg1]).apply(r.reshape(-1, n)).ravel()
    refw, refv = cycle_op(E1 @ E1) @ r, cycle_op(E1) @ r
    sc = np.abs(refw).max()
    assert np.abs(zw - refw).max() <= 1e-11 * sc
    assert np.abs(zv - refv).max() <= 1e-11 * sc
    assert np.abs(refw - refv).max() > 1e-3 * sc          # the two shapes differ here
    # w_levels beyond the hierarchy changes nothing: level 1 sits above the
    # coarsest, whose exact solve is taken once
    z2 = O.AMG(A, nu1=1, nu2=1, omega=w, aggs=[agg0, agg1], w_levels=5).apply(r.reshape(-1, n)).ravel()
    assert np.array_equal(z2, zw)


def test_w_cycle_above_the_coarsest_level_is_the_v_cycle():
    s = pressure_velocity(4, 4, 2, seed=3)
    A = O.from_system(s)
    agg, nc = O.match(A.N, A.row_ptr, A.col, O.strength(A))
    r = np.random.default_rng(2).standard_normal((A.N, 4))
    zv = O.AMG(A, nu1=2, nu2=2, omega=0.9, aggs=[agg]).apply(r)
    zw = O.AMG(A, nu1=2, nu2=2, omega=0.9, aggs=[agg], w_levels=1).apply(r)
    assert np.array_equal(zv, zw)


def test_w_cycle_preconditioned_solve():
    s = pressure_velocity(16, 16, 16, seed=0)
    A = O.from_system(s)
    kw = dict(coarse_max=16, passes=2, nu1=2, nu2=2, omega=0.9)
    xv, stv = O.bicgstab(A, s["b"], prec=O.PREC_AMG, amg=O.AMG(A, **kw), tol=1e-10)
    xw, stw = O.bicgstab(A, s["b"], prec=O.PREC_AMG, amg=O.AMG(A, w_levels=1, **kw), tol=1e-10)
    assert O.relres(A, s["b"], xw) <= 1e-10
    assert stw["iterations"] <= stv["iterations"]
    assert O.AMG(A, w_levels=1, **kw).levels >= 3


def test_coarse_damping_closed_form():
    # The same three-level hierarchy with damping w0 on level 0 and w1 below
    # it: S0 = I - w0 D0^{-1} A0, S1 = I - w1 D1^{-1} A1, for the V- and the
    # W-cycle.  A cycle that used w0 everywhere (or w1 everywhere) fails it.
    s = jacobian_box(5, 4, 3, n=3, seed=9)
    A = O.from_system(s)
    n, w0, w1 = 3, 0.7, 1.2
    agg0, nc0 = O.match(A.N, A.row_ptr, A.col, O.strength(A))
    A1 = O.rap(A, agg0, nc0)
    agg1, nc1 = O.match(A1.N, A1.row_ptr, A1.col, O.strength(A1))
    Ad, A1d = A.dense(), A1.dense()
    P0, P1 = _P(agg0, nc0, n), _P(agg1, nc1, n)
    A2d = P1.T @ A1d @ P1
    I0, I1 = np.eye(Ad.shape[0]), np.eye(A1d.shape[0])
    A0i, A1i = np.linalg.inv(Ad), np.linalg.inv(A1d)
    r = np.random.default_rng(6).standard_normal(Ad.shape[0])

    def cycle_op(wa, wb, twice):
        S0 = I0 - wa * np.linalg.solve(_dense_blocks(Ad, n), Ad)
        S1 = I1 - wb * np.linalg.solve(_dense_blocks(A1d, n), A1d)
        E1 = S1 @ (I1 - P1 @ np.linalg.solve(A2d, P1.T @ A1d)) @ S1
        B1 = (I1 - (E1 @ E1 if twice else E1)) @ A1i
        E0 = S0 @ (I0 - P0 @ B1 @ P0.T @ Ad) @ S0
        return (I0 - E0) @ A0i

    for wl in (0, 1):
        z = O.AMG(A, nu1=1, nu2=1, omega=w0, aggs=[agg0, agg1], w_levels=wl,
                  coarse_omega=w1).apply(r.reshape(-1, n)).ravel()
        ref = cycle_op(w0, w1, wl == 1) @ r
        sc = np.abs(ref).max()
        assert np.abs(z - ref).max() <= 1e-11 * sc
        assert np.abs(cycle_op(w0, w0, wl == 1) @ r - ref).max() > 1e-3 * sc
        assert np.abs(cycle_op(w1, w1, wl == 1) @ r - ref).max() > 1e-3 * sc
    # coarse_omega 0 is the hierarchy's omega on every level
    z0 = O.AMG(A, nu1=1, nu2=1, omega=w0, aggs=[agg0, agg1], coarse_omega=0.0).apply(r.reshape(-1, n))
    assert np.array_equal(z0, O.AMG(A, nu1=1, nu2=1, omega=w0, aggs=[agg0, agg1]).apply(r.reshape(-1, n)))
