"""Pins for the oracle's Krylov solvers, transposed solve and LDU gradient."""
import numpy as np
import pytest

import oracle as O
from workloads import jacobian_box, pressure_velocity


@pytest.mark.parametrize("solver", ["bicgstab", "fgmres", "gmres"])
@pytest.mark.parametrize("prec", [O.PREC_NONE, O.PREC_BJACOBI, O.PREC_AMG])
def test_tiny_systems_match_dense_lu(solver, prec):
    for s in (jacobian_box(4, 3, 3, seed=1), pressure_velocity(4, 3, 3, seed=1)):
        A = O.from_system(s)
        amg = O.AMG(A, coarse_max=4) if prec == O.PREC_AMG else None
        fn = getattr(O, solver)
        x, st = fn(A, s["b"], prec=prec, amg=amg, tol=1e-10, maxit=2000)
        assert st["status"] == O.OK and st["relres"] <= 1e-10
        Ad = A.dense()
        xd = np.linalg.solve(Ad, s["b"].ravel())
        kappa = np.linalg.cond(Ad)
        assert np.linalg.norm(x.ravel() - xd) <= 10 * kappa * 1e-10 * np.linalg.norm(xd)
        # the reported residual is the true one
        assert abs(O.relres(A, s["b"], x) - st["relres"]) <= 1e-12


def test_scaled_identity_converges_in_one_iteration():
    N, n = 20, 4
    D = np.tile(3.5 * np.eye(n), (N, 1, 1))
    A = O.ldu_to_bcsr(N, n, [], [], D, np.zeros((0, n, n)), np.zeros((0, n, n)))[0]
    b = np.random.default_rng(0).standard_normal((N, n))
    for fn in (O.bicgstab, O.fgmres, O.gmres):
        x, st = fn(A, b, prec=O.PREC_NONE, tol=1e-12)
        assert st["iterations"] == 1
        assert np.allclose(x, b / 3.5, rtol=1e-14)


def test_fgmres_finite_termination():
    s = jacobian_box(3, 2, 2, n=2, seed=3)     # 24 unknowns
    A = O.from_system(s)
    m = A.N * A.n
    for fn in (O.fgmres, O.gmres):
        x, st = fn(A, s["b"], prec=O.PREC_NONE, tol=1e-13, maxit=m, restart=m)
        assert st["status"] == O.OK and st["iterations"] <= m


@pytest.mark.parametrize("prec", [O.PREC_BJACOBI, O.PREC_AMG])
def test_gmres_equals_fgmres_for_a_fixed_preconditioner(prec):
    """With a preconditioner that is one fixed linear operator, right-
    preconditioned GMRES and flexible GMRES build the same Krylov space and
    the same iterates; only rounding separates them."""
    s = pressure_velocity(6, 5, 5, seed=2)
    A = O.from_system(s)
    amg = O.AMG(A, coarse_max=8, nu1=1, nu2=1) if prec == O.PREC_AMG else None
    xf, sf = O.fgmres(A, s["b"], prec=prec, amg=amg, tol=1e-10, maxit=500, restart=12)
    xg, sg = O.gmres(A, s["b"], prec=prec, amg=amg, tol=1e-10, maxit=500, restart=12)
    assert sf["status"] == O.OK and sg["status"] == O.OK
    assert abs(sf["iterations"] - sg["iterations"]) <= 1
    assert np.linalg.norm(xf - xg) <= 1e-8 * np.linalg.norm(xf)


def test_zero_rhs_gives_zero():
    s = jacobian_box(3, 3, 3, seed=0)
    A = O.from_system(s)
    for fn in (O.bicgstab, O.fgmres, O.gmres):
        x, st = fn(A, np.zeros_like(s["b"]), x0=np.ones_like(s["b"]))
        assert st["iterations"] == 0 and np.all(x == 0)


def test_iteration_cap_reports_not_converged():
    s = pressure_velocity(6, 6, 6, seed=0)
    A = O.from_system(s)
    x, st = O.bicgstab(A, s["b"], prec=O.PREC_NONE, tol=1e-14, maxit=2)
    assert st["status"] == O.NOT_CONVERGED
    assert abs(O.relres(A, s["b"], x) - st["relres"]) <= 1e-14


def test_transposed_solve_and_gradient_by_finite_differences():
    # L = c^T x, x = A^{-1} b.  lambda = A^{-T} c; dL/db = lambda; dL/dA_ij = -lambda_i x_j^T.
    s = pressure_velocity(3, 3, 2, seed=4)
    A = O.from_system(s)
    N, n, F = s["N"], 4, s["F"]
    rng = np.random.default_rng(4)
    c = rng.standard_normal((N, n))
    x, _ = O.bicgstab(A, s["b"], tol=1e-14, maxit=5000)
    lam, st = O.bicgstab(O.transpose(A), c, tol=1e-14, maxit=5000)
    assert st["status"] == O.OK
    assert np.allclose(O.spmv_t(A, lam), c, rtol=0, atol=1e-12)
    gd, gu, gl = O.grad(s, lam, x)

    def L(diag, upper, lower, b):
        Ad = np.zeros((N * n, N * n))
        for i in range(N):
            Ad[i * n:(i + 1) * n, i * n:(i + 1) * n] = diag[i]
        for f in range(F):
            l, u = s["lower_addr"][f], s["upper_addr"][f]
            Ad[l * n:(l + 1) * n, u * n:(u + 1) * n] = upper[f]
            Ad[u * n:(u + 1) * n, l * n:(l + 1) * n] = lower[f]
        return c.ravel() @ np.linalg.solve(Ad, b.ravel())

    h = 1e-6
    base = dict(diag=s["diag"], upper=s["upper"], lower=s["lower"], b=s["b"])
    for key, g in (("diag", gd), ("upper", gu), ("lower", gl)):
        for _ in range(6):
            idx = tuple(rng.integers(0, d) for d in base[key].shape)
            p = {k: v.copy() for k, v in base.items()}; m = {k: v.copy() for k, v in base.items()}
            p[key][idx] += h; m[key][idx] -= h
            fd = (L(**p) - L(**m)) / (2 * h)
            assert abs(fd - g[idx]) <= 1e-6 * max(1.0, abs(g[idx]))
    idx = (3, 2)
    p = {k: v.copy() for k, v in base.items()}; m = {k: v.copy() for k, v in base.items()}
    p["b"][idx] += h; m["b"][idx] -= h
    assert abs((L(**p) - L(**m)) / (2 * h) - lam[idx]) <= 1e-6


def test_dilu_amg_reaches_tolerance_on_pressure_velocity():
    s = pressure_velocity(10, 10, 10, seed=0)
    A = O.from_system(s)
    amg = O.AMG(A, coarse_max=32, smoother=O.SMOOTH_DILU)
    x, st = O.bicgstab(A, s["b"], prec=O.PREC_AMG, amg=amg, tol=1e-8)
    assert st["status"] == O.OK and O.relres(A, s["b"], x) <= 1e-8


def test_sgs_amg_reaches_tolerance_and_is_exact_on_block_diagonal_levels():
    """AMG with symmetric Gauss-Seidel smoothing on the finest level solves the
    pressure-velocity system; on a block-diagonal matrix one SGS step is exact,
    so the V-cycle is the exact inverse there."""
    s = pressure_velocity(10, 10, 10, seed=0)
    A = O.from_system(s)
    amg = O.AMG(A, coarse_max=32, smoother=O.SMOOTH_SGS, dilu_levels=1)
    x, st = O.bicgstab(A, s["b"], prec=O.PREC_AMG, amg=amg, tol=1e-8)
    assert st["status"] == O.OK and O.relres(A, s["b"], x) <= 1e-8
    rng = np.random.default_rng(2)
    D = rng.standard_normal((40, 4, 4)) + 5 * np.eye(4)
    Ab = O.ldu_to_bcsr(40, 4, [], [], D, np.zeros((0, 4, 4)), np.zeros((0, 4, 4)))[0]
    agg = np.repeat(np.arange(10), 4).astype(np.int32)
    mg = O.AMG(Ab, nu1=1, nu2=0, smoother=O.SMOOTH_SGS, aggs=[agg], dilu_levels=1)
    b = rng.standard_normal((40, 4))
    assert np.allclose(mg.apply(b), np.linalg.solve(D, b[..., None])[..., 0], rtol=1e-12, atol=1e-13)


def _dense_triangles(A, rank):
    """Dense D, L (blocks of rows visited earlier in rank order) and U."""
    Ad = A.dense()
    bi = np.repeat(np.arange(A.N), A.n)
    same = bi[:, None] == bi[None, :]
    before = rank[bi][:, None] > rank[bi][None, :]
    after = rank[bi][:, None] < rank[bi][None, :]
    return Ad, Ad * same, Ad * before, Ad * after


def test_sgs_preconditioner_one_step_closed_form():
    """One symmetric step from zero: forward z1 = (D+L)^{-1} r, backward
    z = (D+U)^{-1}(r - L z1) = (D+U)^{-1} D (D+L)^{-1} r."""
    s = jacobian_box(4, 3, 3, n=3, seed=6)
    A = O.from_system(s)
    rank = np.random.default_rng(7).permutation(A.N)
    r = np.random.default_rng(8).standard_normal((A.N, A.n))
    z = O.SGSPrec(A, rank, sweeps=1).apply(r)
    _, D, L, U = _dense_triangles(A, rank)
    ref = np.linalg.solve(D + U, D @ np.linalg.solve(D + L, r.ravel()))
    assert np.allclose(z.ravel(), ref, rtol=1e-11, atol=1e-12)


def test_sgs_preconditioner_k_steps_are_the_stationary_iteration():
    """k steps from zero: z_{j+1} = z_j + M^{-1}(r - A z_j), M^{-1} the
    one-step operator of the closed form."""
    s = pressure_velocity(4, 3, 3, seed=9)
    A = O.from_system(s)
    rank = np.random.default_rng(10).permutation(A.N)
    r = np.random.default_rng(11).standard_normal((A.N, A.n)).ravel()
    Ad, D, L, U = _dense_triangles(A, rank)

    def minv(v):
        return np.linalg.solve(D + U, D @ np.linalg.solve(D + L, v))
    z = np.zeros_like(r)
    for k in range(1, 4):
        z = z + minv(r - Ad @ z)
        zk = O.SGSPrec(A, rank, sweeps=k).apply(r.reshape(A.N, A.n)).ravel()
        assert np.allclose(zk, z, rtol=1e-10, atol=1e-11), k


def test_sgs_preconditioner_is_symmetric_for_a_symmetric_matrix():
    """For symmetric A the symmetric step is a symmetric operator:
    <M^{-1} r1, r2> = <r1, M^{-1} r2> (a one-directional sweep is not)."""
    s = jacobian_box(4, 4, 3, n=3, seed=12)
    n = s["n"]
    sym = dict(s)
    sym["diag"] = s["diag"] + np.transpose(s["diag"], (0, 2, 1)) + 8 * np.eye(n)
    sym["lower"] = np.ascontiguousarray(np.transpose(s["upper"], (0, 2, 1)))
    A = O.from_system(sym)
    assert np.allclose(A.dense(), A.dense().T)
    rank = np.random.default_rng(13).permutation(A.N)
    rng = np.random.default_rng(14)
    r1, r2 = rng.standard_normal((2, A.N, n))
    P = O.SGSPrec(A, rank, sweeps=1)
    lhs, rhs = np.vdot(P.apply(r1), r2), np.vdot(r1, P.apply(r2))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # the forward half alone fails the same test
    _, D, L, U = _dense_triangles(A, rank)
    F = np.linalg.inv(D + L)
    assert abs(np.vdot(F @ r1.ravel(), r2.ravel()) - np.vdot(r1.ravel(), F @ r2.ravel())) > 1e-6


@pytest.mark.parametrize("solver", ["bicgstab", "fgmres", "gmres"])
def test_sgs_preconditioned_solvers_match_dense_lu(solver):
    for s in (jacobian_box(4, 3, 3, seed=15), pressure_velocity(5, 4, 3, seed=15)):
        A = O.from_system(s)
        rank = np.random.default_rng(16).permutation(A.N)
        P = O.SGSPrec(A, rank, sweeps=1)
        x, st = getattr(O, solver)(A, s["b"], prec=O.PREC_SGS, amg=P, tol=1e-10, maxit=2000)
        assert st["status"] == O.OK and st["relres"] <= 1e-10
        Ad = A.dense()
        xd = np.linalg.solve(Ad, s["b"].ravel())
        assert np.linalg.norm(x.ravel() - xd) <= 10 * np.linalg.cond(Ad) * 1e-10 * np.linalg.norm(xd)
        assert abs(O.relres(A, s["b"], x) - st["relres"]) <= 1e-12


def test_sgs_preconditioner_exact_on_block_diagonal_and_rejects_bad_input():
    rng = np.random.default_rng(17)
    D = rng.standard_normal((7, 4, 4)) + 4 * np.eye(4)
    A = O.ldu_to_bcsr(7, 4, [], [], D, np.zeros((0, 4, 4)), np.zeros((0, 4, 4)))[0]
    b = rng.standard_normal((7, 4))
    P = O.SGSPrec(A, rng.permutation(7))
    for fn in (O.bicgstab, O.fgmres, O.gmres):
        x, st = fn(A, b, prec=O.PREC_SGS, amg=P, tol=1e-12)
        assert st["iterations"] == 1
    with pytest.raises(O.OracleError):
        O.gmres(A, b, prec=O.PREC_SGS, amg=None)
    with pytest.raises(O.OracleError):
        O.SGSPrec(A, np.arange(7), sweeps=0)


def test_ilu0_amg_reaches_tolerance_on_a_graph_with_fill():
    from workloads import jacobian_graph
    s = jacobian_graph(N=400, n=4, hubs=4, hub_degree=20, base_degree=3, seed=30)
    A = O.from_system(s)
    its = {}
    for sm in (O.SMOOTH_BJACOBI, O.SMOOTH_DILU, O.SMOOTH_ILU0):
        amg = O.AMG(A, coarse_max=16, nu1=1, nu2=1, omega=0.8, smoother=sm, dilu_levels=-1)
        x, st = O.bicgstab(A, s["b"], prec=O.PREC_AMG, amg=amg, tol=1e-10, maxit=500)
        assert st["status"] == O.OK and O.relres(A, s["b"], x) <= 1e-10 * 1.0001
        its[sm] = st["iterations"]
    assert its[O.SMOOTH_ILU0] <= its[O.SMOOTH_BJACOBI], its
