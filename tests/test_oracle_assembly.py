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


def _jac_uH(u, H, s, g=G):
    """The flux Jacobian as a function of velocity and total enthalpy only
    (the density cancels out of it): evaluated at the state with rho = 1,
    that velocity and rho E = (H + (g - 1)|u|^2 / 2) / g."""
    E = (H + 0.5 * (g - 1.0) * (u @ u)) / g
    return O.euler_jac(np.concatenate([[1.0], u, [E]]), s, g)


def _property_u_state(QL, QR, g=G):
    """(u~, H~) of the matrix of Jacobian form that satisfies Roe's property U,
    F(Q_R).s - F(Q_L).s = J(u~, H~, s)(Q_R - Q_L), for three independent area
    vectors at once, found by nonlinear least squares from the arithmetic
    mean of the two states.  Nothing here uses the averaging formula."""
    from scipy.optimize import least_squares
    svecs = np.eye(3) + 0.3 * np.random.default_rng(41).normal(size=(3, 3))
    dQ = QR - QL

    def res(z):
        return np.concatenate([_jac_uH(z[:3], z[3], s, g) @ dQ - (_flux(QR, s, g) - _flux(QL, s, g))
                               for s in svecs])

    def uH(Q):
        rho, u = Q[0], Q[1:4] / Q[0]
        p = (g - 1.0) * (Q[4] - 0.5 * rho * u @ u)
        return u, (Q[4] + p) / rho

    (uL, HL), (uR, HR) = uH(QL), uH(QR)
    sol = least_squares(res, np.concatenate([0.5 * (uL + uR), [0.5 * (HL + HR)]]), xtol=1e-15, ftol=1e-15,
                        gtol=1e-15)
    assert np.abs(res(sol.x)).max() <= 1e-12 * max(1.0, np.abs(_flux(QR, svecs[0], g)).max())
    return sol.x[:3], sol.x[3]


def _radius_property_u(QL, QR, s, g=G):
    """Spectral radius (largest |eigenvalue|) of the property-U matrix."""
    u, H = _property_u_state(QL, QR, g)
    return np.abs(np.linalg.eigvals(_jac_uH(u, H, s, g))).max()


def test_roe_radius_is_the_spectral_radius_of_the_property_u_matrix():
    """Sec. 2.1 takes lambda_ij from the Roe flux matrix.  Roe's matrix is the
    Jacobian evaluated at the state for which F(Q_R).s - F(Q_L).s equals the
    matrix times Q_R - Q_L for every s (property U); its spectral radius is the
    face's convective radius.  States with large density and velocity jumps
    make any other average (an arithmetic mean, swapped weights) miss."""
    rng = np.random.default_rng(40)
    for k in range(6):
        QL, QR = _states(60 + k, 2)
        QR = QR * np.array([4.0, 1.0, 1.0, 1.0, 3.0])     # density ratio of several
        s = rng.normal(size=3)
        assert np.isclose(O.roe_radius(QL, QR, s, G), _radius_property_u(QL, QR, s), rtol=1e-10, atol=0)


def test_luo_assembly_rejects_non_positive_density_or_pressure():
    """The sound speed, and with it the face radius, is undefined for a state
    with p <= 0 or rho <= 0, even where every coefficient comes out finite."""
    d = luo_inputs(4, 3, 3, seed=8)
    rho = d["Q"][5, 0]
    u = d["Q"][5, 1:4] / rho
    bad = dict(d)
    bad["Q"] = d["Q"].copy()
    bad["Q"][5, 4] = -1e-2 / (G - 1.0) + 0.5 * rho * u @ u             # p = -0.01
    with pytest.raises(O.OracleError):
        O.luo_assemble(bad)
    bad["Q"] = d["Q"].copy()
    bad["Q"][7, 0] = -bad["Q"][7, 0]
    with pytest.raises(O.OracleError):
        O.luo_assemble(bad)


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
    lam = _radius_property_u(Q0, Q1, s) + 0.02 * np.linalg.norm(s)
    J0, J1 = _fd_jac(Q0, s), _fd_jac(Q1, s)
    I = np.eye(5)
    assert np.allclose(L["diag"][0], 0.5 * I + 0.5 * (J0 + lam * I), atol=1e-7)
    assert abs(L["diag"][0][0, 0] - 0.5 - 0.5 * lam) <= 1e-12 * lam      # J has a zero (0, 0) entry
    assert np.allclose(L["upper"][0], 0.5 * (J1 - lam * I), atol=1e-7)
    assert np.allclose(L["diag"][1], 0.7 * I + 0.5 * (-J1 + lam * I), atol=1e-7)
    assert np.allclose(L["lower"][0], 0.5 * (-J0 - lam * I), atol=1e-7)


def _fd_jac(Q, s, h=1e-6):
    return np.stack([(_flux(Q + h * e, s) - _flux(Q - h * e, s)) / (2 * h) for e in np.eye(5)], axis=1)


# ------------------------------------------------ pressure-based (p, U) blocks
from workloads import pu_inputs  # noqa: E402


def _pu(d, **kw):
    return O.from_system(O.pu_assemble(d, **kw))


def test_pu_pressure_rows_are_a_laplacian():
    """Rhie-Chow pp sub-block: each row sums to pp_add (to 0 without it), off-
    diagonals are negative and the matrix of pp entries is symmetric."""
    d = pu_inputs(5, 4, 3, seed=20)
    A = _pu(d)
    rows = np.repeat(np.arange(A.N), np.diff(A.row_ptr))
    pp = A.vals[:, 0, 0]
    assert np.allclose(np.bincount(rows, pp, A.N), d["pp_add"], rtol=1e-12, atol=1e-15)
    off = rows != A.col
    assert np.all(pp[off] < 0)
    P = np.zeros((A.N, A.N)); P[rows, A.col] = pp
    assert np.allclose(P, P.T, rtol=1e-14, atol=0)


def test_pu_coupling_blocks_are_equal_and_vanish_on_closed_cells():
    """a^up = a^pu in every block; summed over a closed cell's row they give
    the sum of its outward face vectors, 0 (a constant pressure has no
    gradient and a constant velocity no divergence)."""
    d = pu_inputs(5, 5, 4, seed=21)
    A = _pu(d)
    assert np.array_equal(A.vals[:, 1:, 0], A.vals[:, 0, 1:])
    rowsum = np.add.reduceat(A.vals, A.row_ptr[:-1], axis=0)
    ids = np.arange(A.N).reshape(4, 5, 5)
    inner = ids[1:-1, 1:-1, 1:-1].ravel()
    scale = np.abs(A.vals[:, 1:, 0]).max()
    assert np.abs(rowsum[inner, 1:, 0]).max() <= 1e-13 * scale
    assert np.abs(rowsum[ids[0, 0, 0], 1:, 0]).max() > 1e-3 * scale


def test_pu_momentum_rows_of_a_divergence_free_flux_sum_to_the_additions():
    """With a uniform velocity the face fluxes of a closed cell sum to zero,
    so upwind convection plus diffusion leaves each momentum row summing to
    uu_add: max(F, 0) - max(-F, 0) = F and the diffusion cancels."""
    d = pu_inputs(5, 4, 4, seed=22)
    u = np.array([0.7, -0.3, 0.4])
    d["flux"] = d["Sf"] @ u
    A = _pu(d)
    rowsum = np.add.reduceat(A.vals, A.row_ptr[:-1], axis=0)
    ids = np.arange(A.N).reshape(4, 4, 5)
    inner = ids[1:-1, 1:-1, 1:-1].ravel()
    for c in range(1, 4):
        assert np.allclose(rowsum[inner, c, c], d["uu_add"][inner], rtol=1e-12)
        assert np.all(rowsum[inner, c, 1:][:, [k for k in range(3) if k != c - 1]] == 0)


def test_pu_reversing_a_face_gives_the_same_matrix():
    """Listing a face from its other side (neighbour first, -S, -d, -flux,
    weight 1 - f_x) assembles the same operator."""
    d = pu_inputs(4, 3, 3, seed=23)
    A = _pu(d)
    flip = np.random.default_rng(24).random(d["F"]) < 0.5
    e = dict(d)
    e["lower_addr"] = np.where(flip, d["upper_addr"], d["lower_addr"]).astype(np.int32)
    e["upper_addr"] = np.where(flip, d["lower_addr"], d["upper_addr"]).astype(np.int32)
    for k in ("Sf", "d"):
        e[k] = np.where(flip[:, None], -d[k], d[k])
    e["flux"] = np.where(flip, -d["flux"], d["flux"])
    e["fx"] = np.where(flip, 1.0 - d["fx"], d["fx"])
    B = _pu(e)
    assert np.array_equal(A.col, B.col)
    assert np.allclose(A.vals, B.vals, rtol=1e-13, atol=1e-16)


def test_pu_rhie_chow_coefficient_on_a_uniform_cube_mesh():
    """Unjittered cubes of side h, uniform inputs: D = V / a^uu for every cell
    with the same a^uu, so a_ij^pp = -D h^2 / h = -D h exactly."""
    d = pu_inputs(4, 4, 4, seed=25, jitter=0.0)
    h = d["h"]
    d["vol"] = np.full(d["N"], h ** 3)
    d["nu"] = np.full(d["F"], 0.01)
    d["flux"] = np.zeros(d["F"])
    d["uu_add"] = np.full(d["N"], 0.5)
    A = _pu(d)
    rows = np.repeat(np.arange(A.N), np.diff(A.row_ptr))
    deg = np.diff(A.row_ptr) - 1
    auu = 0.5 + deg * 0.01 * h * h / h                # diffusion k = nu |S| / (n.d) = nu h
    off = np.nonzero(rows != A.col)[0]
    Dl, Du = h ** 3 / auu[rows[off]], h ** 3 / auu[A.col[off]]
    assert np.allclose(A.vals[off, 0, 0], -0.5 * (Dl + Du) * h, rtol=1e-12)


@pytest.mark.parametrize("name", ["pu_2cell", "pu_3cell"])
def test_pu_golden_blocks_by_hand(name):
    """Two- and three-cell systems worked by hand from the coefficients after
    Eq. prb_coeff (derivations in the fixtures), with a nonzero flux, f_x away
    from 1/2 and one face listed from its neighbour's side."""
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", name + ".json")))
    d = {k: (np.array(v, dtype=np.int32) if k.endswith("_addr") else np.array(v, dtype=np.float64))
         for k, v in g.items() if not k.startswith(("_", "expect")) and k not in ("N", "F")}
    d["N"], d["F"] = g["N"], g["F"]
    L = O.pu_assemble(d)
    for k in ("diag", "upper", "lower"):
        assert np.allclose(L[k], np.array(g["expect_" + k]), rtol=0, atol=1e-14), k


def test_pu_upwind_takes_only_upstream_neighbours():
    """First-order upwind (Sec. 2.2): with no diffusion, a momentum row couples
    to a neighbour only through a face the flow enters by, i.e. the neighbour
    lies upstream; faces the flow leaves by add to the diagonal only."""
    d = pu_inputs(5, 4, 3, seed=26)
    d["nu"] = np.zeros(d["F"])
    L = O.pu_assemble(d, with_add=False)
    F = d["flux"]
    assert np.all(F != 0)
    up_lu = L["upper"][:, 1, 1]           # row owner, column neighbour
    up_ul = L["lower"][:, 1, 1]           # row neighbour, column owner
    assert np.all((up_lu != 0) == (F < 0)) and np.all(up_lu <= 0)
    assert np.all((up_ul != 0) == (F > 0)) and np.all(up_ul <= 0)
    assert np.allclose(-up_lu - up_ul, np.abs(F), rtol=1e-14)
    # the owner's diagonal collects its outflow: sum over faces of max(F, 0) seen from it
    out = np.zeros(d["N"])
    np.add.at(out, d["lower_addr"], np.maximum(F, 0))
    np.add.at(out, d["upper_addr"], np.maximum(-F, 0))
    assert np.allclose(L["diag"][:, 1, 1], out, rtol=1e-13)


def _graded_box(xs, ys, zs):
    """Inputs of the pressure-based assembly on a rectilinear mesh with
    uneven spacing, built here from the node coordinates: cell centres at
    the midpoints, face centres on the node planes, f_x the owner's linear
    weight along the cell-centre line, d = c_u - c_l, V the cell volume."""
    nx, ny, nz = len(xs) - 1, len(ys) - 1, len(zs) - 1
    cen = [0.5 * (np.asarray(a)[1:] + np.asarray(a)[:-1]) for a in (xs, ys, zs)]
    wid = [np.diff(a) for a in (xs, ys, zs)]
    cid = lambda i, j, k: i + nx * (j + ny * k)
    la, ua, S, D, FX, C = [], [], [], [], [], np.zeros((nx * ny * nz, 3))
    vol = np.zeros(nx * ny * nz)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                C[cid(i, j, k)] = (cen[0][i], cen[1][j], cen[2][k])
                vol[cid(i, j, k)] = wid[0][i] * wid[1][j] * wid[2][k]
    nodes = (xs, ys, zs)
    for ax in range(3):
        n = [nx, ny, nz]
        for k in range(nz if ax != 2 else nz - 1):
            for j in range(ny if ax != 1 else ny - 1):
                for i in range(nx if ax != 0 else nx - 1):
                    a = cid(i, j, k)
                    b = cid(i + (ax == 0), j + (ax == 1), k + (ax == 2))
                    idx = (i, j, k)[ax]
                    xf = nodes[ax][idx + 1]
                    other = [wid[q][(i, j, k)[q]] for q in range(3) if q != ax]
                    s = np.zeros(3); s[ax] = other[0] * other[1]
                    la.append(a); ua.append(b); S.append(s)
                    D.append(C[b] - C[a])
                    FX.append((C[b][ax] - xf) / (C[b][ax] - C[a][ax]))
        del n
    F = len(la)
    return {"N": nx * ny * nz, "F": F, "lower_addr": np.array(la, np.int32), "upper_addr": np.array(ua, np.int32),
            "Sf": np.array(S), "d": np.array(D), "fx": np.array(FX), "flux": np.full(F, 0.1),
            "nu": np.full(F, 0.01), "vol": vol, "uu_add": np.ones(nx * ny * nz),
            "pp_add": np.zeros(nx * ny * nz)}, C


def test_pu_coupling_is_exact_for_linear_fields_on_a_graded_mesh():
    """With linear interpolation to the face, the coupling rows are the Gauss
    theorem applied cell by cell, which is exact for linear fields: the up
    rows of a closed cell applied to p = g . x give V g, and the pu row
    applied to u = B x gives V trace(B).  The spacing is uneven, so f_x != 1/2
    and a swapped owner/neighbour weight misses."""
    xs = [0.0, 0.1, 0.35, 0.5, 1.0]
    ys = [0.0, 0.3, 0.4, 0.9]
    zs = [0.0, 0.2, 0.25, 0.6, 0.8]
    d, C = _graded_box(xs, ys, zs)
    A = O.from_system(O.pu_assemble(d))
    rng = np.random.default_rng(27)
    gvec, B = rng.normal(size=3), rng.normal(size=(3, 3))
    p = C @ gvec
    U = C @ B.T
    rows = np.repeat(np.arange(A.N), np.diff(A.row_ptr))
    grad = np.zeros((A.N, 3)); div = np.zeros(A.N)
    np.add.at(grad, rows, A.vals[:, 1:, 0] * p[A.col][:, None])
    np.add.at(div, rows, np.einsum("kc,kc->k", A.vals[:, 0, 1:], U[A.col]))
    nx, ny, nz = 4, 3, 4
    ids = np.arange(A.N).reshape(nz, ny, nx)
    inner = ids[1:-1, 1:-1, 1:-1].ravel()
    assert inner.size > 0
    assert np.allclose(grad[inner], d["vol"][inner, None] * gvec, rtol=1e-12, atol=1e-14)
    assert np.allclose(div[inner], d["vol"][inner] * np.trace(B), rtol=1e-12, atol=1e-14)
