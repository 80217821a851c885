"""Pins for the oracle's assembly of the density-based coupled matrix
(Sec. 2.1: Eq. discretBackward with the approximate Jacobian of Eqs.
approxJac1 and approxJac2)."""
import numpy as np
import pytest

import oracle as O
from workloads import luo_inputs

G = 1.4


def _flux(Q, s, g=G):
    """Euler flux F(Q) . s, written out (the textbook flux, not its Jacobian)."""
    rho, m, E = Q[0], Q[1:4], Q[4]
    u = m / rho
    p = (g - 1.0) * (E - 0.5 * rho * u @ u)
    V = u @ s
    return np.concatenate([[rho * V], m * V + p * s, [(E + p) * V]])


def _states(seed, k=6):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(k):
        rho, p = rng.uniform(0.5, 2.0), rng.uniform(0.3, 2.0)
        u = rng.normal(0.0, 0.7, 3)
        out.append(np.concatenate([[rho], rho * u, [p / (G - 1) + 0.5 * rho * u @ u]]))
    return out


def test_flux_jacobian_matches_finite_differences_of_the_flux():
    rng = np.random.default_rng(1)
    for Q in _states(2):
        s = rng.normal(size=3)
        J = O.euler_jac(Q, s, G)
        h = 1e-6
        Jfd = np.stack([(_flux(Q + h * e, s) - _flux(Q - h * e, s)) / (2 * h) for e in np.eye(5)], axis=1)
        assert np.allclose(J, Jfd, rtol=1e-7, atol=1e-7)


def test_flux_is_homogeneous_of_degree_one():
    """F(Q) . s = J(Q, s) Q for the Euler flux of an ideal gas."""
    rng = np.random.default_rng(3)
    for Q in _states(4):
        s = rng.normal(size=3)
        assert np.allclose(O.euler_jac(Q, s, G) @ Q, _flux(Q, s), rtol=1e-13, atol=1e-13)


def test_flux_jacobian_eigenvalues_are_the_wave_speeds():
    rng = np.random.default_rng(5)
    for Q in _states(6):
        n = rng.normal(size=3); n /= np.linalg.norm(n)
        rho, u = Q[0], Q[1:4] / Q[0]
        p = (G - 1) * (Q[4] - 0.5 * rho * u @ u)
        c, un = np.sqrt(G * p / rho), u @ n
        ev = np.sort(np.linalg.eigvals(O.euler_jac(Q, n, G)).real)
        assert np.allclose(ev, np.sort([un - c, un, un, un, un + c]), atol=1e-10)


def test_roe_radius_of_equal_states_and_symmetry():
    rng = np.random.default_rng(7)
    QA, QB = _states(8, 2)
    s = rng.normal(size=3)
    rho, u = QA[0], QA[1:4] / QA[0]
    p = (G - 1) * (QA[4] - 0.5 * rho * u @ u)
    assert np.isclose(O.roe_radius(QA, QA, s, G), abs(u @ s) + np.sqrt(G * p / rho) * np.linalg.norm(s), rtol=1e-14)
    # swapping the sides and the normal leaves the radius unchanged
    assert np.isclose(O.roe_radius(QA, QB, s, G), O.roe_radius(QB, QA, -s, G), rtol=1e-14)


def test_block_columns_sum_to_zero_without_the_time_term():
    """Each face adds (J_l + l I)/2 to A_ll and -(J_l + l I)/2 to A_ul: the
    linearised residual is conservative, so every block column sums to 0."""
    d = luo_inputs(5, 4, 3, seed=9)
    A = O.from_system(O.luo_assemble(d, with_dt=False))
    colsum = np.zeros((A.N, 5, 5))
    np.add.at(colsum, A.col, A.vals)
    assert np.abs(colsum).max() <= 1e-13 * np.abs(A.vals).max()
    # the time term adds V/dtau I to the diagonal only
    A2 = O.from_system(O.luo_assemble(d))
    assert np.allclose(A2.vals - A.vals, np.einsum("k,ij->kij", np.where(
        np.repeat(np.arange(A.N), np.diff(A.row_ptr)) == A.col, d["v_dt"][A.col], 0.0), np.eye(5)), atol=1e-15)


def test_uniform_state_rows_of_closed_cells_sum_to_zero():
    """For a uniform state the row sum of an interior (closed) cell is
    J(Q, sum of its outward area vectors) = 0: the face radii cancel."""
    d = luo_inputs(5, 4, 4, seed=10, uniform=True)
    A = O.from_system(O.luo_assemble(d, with_dt=False))
    rowsum = np.add.reduceat(A.vals, A.row_ptr[:-1], axis=0)
    ids = np.arange(A.N).reshape(4, 4, 5)
    inner = ids[1:-1, 1:-1, 1:-1].ravel()
    scale = np.abs(A.vals).max()
    assert np.abs(rowsum[inner]).max() <= 1e-12 * scale
    edge = ids[0, 0, 0]
    assert np.abs(rowsum[edge]).max() > 1e-3 * scale          # open (boundary) cells do not


def test_reversing_a_face_gives_the_same_matrix():
    """R_ij(n_ij) = -R_ji(n_ji): listing a face as (u, l, -S) instead of
    (l, u, S) assembles the same operator."""
    d = luo_inputs(4, 3, 3, seed=11)
    A = O.from_system(O.luo_assemble(d))
    rng = np.random.default_rng(12)
    flip = rng.random(d["F"]) < 0.5
    e = dict(d)
    e["lower_addr"] = np.where(flip, d["upper_addr"], d["lower_addr"]).astype(np.int32)
    e["upper_addr"] = np.where(flip, d["lower_addr"], d["upper_addr"]).astype(np.int32)
    e["Sf"] = np.where(flip[:, None], -d["Sf"], d["Sf"])
    B = O.from_system(O.luo_assemble(e))
    assert np.array_equal(A.row_ptr, B.row_ptr) and np.array_equal(A.col, B.col)
    assert np.allclose(A.vals, B.vals, rtol=1e-14, atol=1e-15)


def test_two_cell_blocks_by_hand():
    """One face between two cells: the four blocks from the equations."""
    Q0, Q1 = _states(13, 2)
    s = np.array([0.3, -0.1, 0.2])
    d = {"N": 2, "F": 1, "lower_addr": np.array([0], np.int32), "upper_addr": np.array([1], np.int32),
         "Q": np.stack([Q0, Q1]), "Sf": s[None], "lam_visc": np.array([0.02]), "v_dt": np.array([0.5, 0.7]),
         "gamma": G}
    L = O.luo_assemble(d)
    lam = O.roe_radius(Q0, Q1, s, G) + 0.02 * np.linalg.norm(s)
    J0, J1 = _fd_jac(Q0, s), _fd_jac(Q1, s)
    I = np.eye(5)
    assert np.allclose(L["diag"][0], 0.5 * I + 0.5 * (J0 + lam * I), atol=1e-7)
    assert np.allclose(L["upper"][0], 0.5 * (J1 - lam * I), atol=1e-7)
    assert np.allclose(L["diag"][1], 0.7 * I + 0.5 * (-J1 + lam * I), atol=1e-7)
    assert np.allclose(L["lower"][0], 0.5 * (-J0 - lam * I), atol=1e-7)


def _fd_jac(Q, s, h=1e-6):
    return np.stack([(_flux(Q + h * e, s) - _flux(Q - h * e, s)) / (2 * h) for e in np.eye(5)], axis=1)
