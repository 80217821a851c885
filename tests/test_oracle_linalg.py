"""Pins for the oracle's block SpMV, transpose, block inversion, dense solve
and smoothers: closed forms, invariants and textbook special cases."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from workloads import jacobian_box, jacobian_stretched, pressure_velocity


def test_spmv_bcsr_equals_ldu_face_loop_and_dense():
    s = pressure_velocity(5, 4, 3, seed=1)
    A = O.from_system(s)
    x = np.random.default_rng(0).standard_normal((s["N"], 4))
    y1 = O.spmv(A, x)
    y2 = O.spmv_ldu(s, x)
    y3 = (A.dense() @ x.ravel()).reshape(y1.shape)
    scale = np.abs(y3).max()
    assert np.abs(y1 - y2).max() <= 1e-14 * scale
    assert np.abs(y1 - y3).max() <= 1e-14 * scale


def test_spmv_constant_vector_row_sum_invariant():
    # Variant-A Jacobian: every block row sums to (V/dtau) I, so A (v,...,v) = (V/dtau) v.
    s = jacobian_box(6, 5, 4, seed=0, vdt=1.0)
    A = O.from_system(s)
    v = np.array([0.3, -1.2, 2.0, 0.7, -0.1])
    y = O.spmv(A, np.tile(v, (s["N"], 1)))
    assert np.abs(y - v).max() <= 64 * np.finfo(float).eps * np.abs(A.vals).max()
    # stretched mesh: block rows sum to V_i I
    t = jacobian_stretched(4, 3, 6, seed=0)
    At = O.from_system(t)
    yt = O.spmv(At, np.tile(v, (t["N"], 1)))
    vol = np.repeat(np.array([1e-3 * 1.2 ** k for k in range(6)]), 12)
    assert np.allclose(yt, vol[:, None] * v, rtol=1e-12, atol=1e-15)


def test_spmv_scalar_blocks_is_textbook_csr():
    s = jacobian_box(7, 3, 2, n=1, seed=4)
    A = O.from_system(s)
    S = sp.csr_matrix((A.vals.ravel(), A.col, A.row_ptr), shape=(A.N, A.N))
    x = np.random.default_rng(2).standard_normal(A.N)
    assert np.allclose(O.spmv(A, x[:, None]).ravel(), S @ x, rtol=1e-14, atol=1e-14)


def test_transpose_dot_product_identity_and_dense():
    s = pressure_velocity(4, 4, 3, seed=3)
    A = O.from_system(s)
    rng = np.random.default_rng(9)
    x = rng.standard_normal((A.N, 4)); y = rng.standard_normal((A.N, 4))
    lhs = np.dot(y.ravel(), O.spmv(A, x).ravel())
    rhs = np.dot(O.spmv_t(A, y).ravel(), x.ravel())
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)
    AT = O.transpose(A)
    assert np.array_equal(AT.dense(), A.dense().T)
    assert np.allclose(O.spmv(AT, y), O.spmv_t(A, y), rtol=1e-13, atol=1e-13)


def test_blockinv_against_identity_and_library():
    rng = np.random.default_rng(1)
    D = rng.standard_normal((50, 5, 5)) + 3 * np.eye(5)
    Di = O.blockinv(D)
    eye = np.einsum("kij,kjl->kil", D, Di)
    cond = np.linalg.cond(D)
    err = np.abs(eye - np.eye(5)).max(axis=(1, 2))
    assert np.all(err <= 50 * cond * np.finfo(float).eps)
    assert np.allclose(Di, np.linalg.inv(D), rtol=1e-10, atol=1e-12)
    # a zero pivot column needs partial pivoting
    P = np.array([[[0.0, 1.0], [1.0, 0.0]]])
    assert np.array_equal(O.blockinv(P), P)


def test_blockinv_singular_reports_block():
    D = np.stack([np.eye(3), np.zeros((3, 3)), np.eye(3)])
    with pytest.raises(O.OracleError) as e:
        O.blockinv(D)
    assert e.value.code == O.ERR_SINGULAR and "block 1" in str(e.value)


def test_dense_solve_against_library():
    rng = np.random.default_rng(7)
    A = rng.standard_normal((40, 40)) + 10 * np.eye(40)
    b = rng.standard_normal(40)
    assert np.allclose(O.dense_solve(A, b), np.linalg.solve(A, b), rtol=1e-12, atol=1e-13)
    A[:, 3] = 0.0
    with pytest.raises(O.OracleError):
        O.dense_solve(A, b)


def test_bjacobi_block_diagonal_exact_in_one_sweep():
    rng = np.random.default_rng(0)
    D = rng.standard_normal((10, 4, 4)) + 4 * np.eye(4)
    A = O.ldu_to_bcsr(10, 4, [], [], D, np.zeros((0, 4, 4)), np.zeros((0, 4, 4)))[0]
    b = rng.standard_normal((10, 4))
    x = O.bjacobi_sweep(A, O.blockinv(D), b, np.zeros((10, 4)), 1.0)
    assert np.allclose(x, np.linalg.solve(D, b[..., None])[..., 0], rtol=1e-13, atol=1e-14)


def test_bjacobi_sweep_matches_dense_splitting():
    s = jacobian_box(4, 3, 3, seed=2)
    A = O.from_system(s)
    Dinv = O.blockinv(O.diag_blocks(A))
    rng = np.random.default_rng(3)
    x0 = rng.standard_normal((A.N, 5))
    x1 = O.bjacobi_sweep(A, Dinv, s["b"], x0, 0.8)
    # dense splitting A = D + R: x1 = x0 + w D^{-1}(b - A x0)
    Ad = A.dense()
    Dd = np.zeros_like(Ad)
    for i in range(A.N):
        Dd[i * 5:(i + 1) * 5, i * 5:(i + 1) * 5] = Ad[i * 5:(i + 1) * 5, i * 5:(i + 1) * 5]
    ref = x0.ravel() + 0.8 * np.linalg.solve(Dd, s["b"].ravel() - Ad @ x0.ravel())
    assert np.allclose(x1.ravel(), ref, rtol=1e-12, atol=1e-13)


def test_sgs_block_diagonal_exact_in_one_step():
    rng = np.random.default_rng(1)
    D = rng.standard_normal((9, 4, 4)) + 4 * np.eye(4)
    A = O.ldu_to_bcsr(9, 4, [], [], D, np.zeros((0, 4, 4)), np.zeros((0, 4, 4)))[0]
    b = rng.standard_normal((9, 4))
    x = O.sgs_sweep(A, O.blockinv(D), rng.permutation(9), b, np.ones((9, 4)))
    assert np.allclose(x, np.linalg.solve(D, b[..., None])[..., 0], rtol=1e-13, atol=1e-14)


def test_sgs_step_matches_dense_triangular_splitting():
    """For an ordering (rank), A = D + L + U with L the blocks (i, j), j before
    i, and U those after: the forward half is x' = (D + L)^{-1} (b - U x), the
    backward half x'' = (D + U)^{-1} (b - L x')."""
    s = jacobian_box(4, 3, 3, n=3, seed=4)
    A = O.from_system(s)
    n = A.n
    Dinv = O.blockinv(O.diag_blocks(A))
    rng = np.random.default_rng(5)
    rank = rng.permutation(A.N)
    x0 = rng.standard_normal((A.N, n))
    x2 = O.sgs_sweep(A, Dinv, rank, s["b"], x0)
    Ad = A.dense()
    bi = np.repeat(np.arange(A.N), n)
    before = rank[bi][:, None] > rank[bi][None, :]
    after = rank[bi][:, None] < rank[bi][None, :]
    same = bi[:, None] == bi[None, :]
    Dd, Ld, Ud = Ad * same, Ad * before, Ad * after
    b = s["b"].ravel()
    x1 = np.linalg.solve(Dd + Ld, b - Ud @ x0.ravel())
    ref = np.linalg.solve(Dd + Ud, b - Ld @ x1)
    assert np.allclose(x2.ravel(), ref, rtol=1e-11, atol=1e-12)


def _chain(N, n, seed):
    """Block-tridiagonal 1D chain: cells 0-1-2-..., natural order."""
    rng = np.random.default_rng(seed)
    la = np.arange(N - 1, dtype=np.int32); ua = la + 1
    return {"N": N, "n": n, "F": N - 1, "lower_addr": la, "upper_addr": ua.astype(np.int32),
            "diag": rng.standard_normal((N, n, n)) + 6 * np.eye(n),
            "upper": rng.standard_normal((N - 1, n, n)), "lower": rng.standard_normal((N - 1, n, n))}


def test_dilu_exact_on_block_tridiagonal_chain():
    # On a chain in natural order there is no fill-in, so DILU = exact block LU.
    s = _chain(12, 3, 0)
    A = O.from_system(s)
    rank = np.arange(12, dtype=np.int32)
    Einv = O.dilu_setup(A, rank)
    r = np.random.default_rng(1).standard_normal((12, 3))
    z = O.dilu_apply(A, rank, Einv, r)
    assert np.allclose(z.ravel(), np.linalg.solve(A.dense(), r.ravel()), rtol=1e-11, atol=1e-12)


def test_dilu_defining_property_diag_of_M_equals_diag_of_A():
    # M = (E + L) E^{-1} (E + U) with the given ordering has diag(M) = diag(A),
    # and dilu_apply solves M z = r.
    s = jacobian_box(3, 3, 2, n=2, seed=5)
    A = O.from_system(s)
    N, n = A.N, 2
    rank = np.random.default_rng(4).permutation(N).astype(np.int32)
    Einv = O.dilu_setup(A, rank)
    Ad = A.dense()
    L = np.zeros_like(Ad); U = np.zeros_like(Ad); E = np.zeros_like(Ad)
    for i in range(N):
        for j in range(N):
            blk = Ad[i * n:(i + 1) * n, j * n:(j + 1) * n]
            if i == j:
                E[i * n:(i + 1) * n, i * n:(i + 1) * n] = np.linalg.inv(Einv[i])
            elif rank[j] < rank[i]:
                L[i * n:(i + 1) * n, j * n:(j + 1) * n] = blk
            else:
                U[i * n:(i + 1) * n, j * n:(j + 1) * n] = blk
    M = (E + L) @ np.linalg.inv(E) @ (E + U)
    for i in range(N):
        sl = slice(i * n, (i + 1) * n)
        assert np.allclose(M[sl, sl], Ad[sl, sl], rtol=1e-11, atol=1e-12)
    # a hex-mesh graph has no triangles, so no fill lands on A's own pattern
    offdiag_mask = np.ones_like(Ad, bool)
    for i in range(N):
        offdiag_mask[i * n:(i + 1) * n, i * n:(i + 1) * n] = False
    assert np.allclose(M[offdiag_mask & (Ad != 0)], Ad[offdiag_mask & (Ad != 0)], rtol=1e-11, atol=1e-12)
    r = np.random.default_rng(2).standard_normal((N, n))
    z = O.dilu_apply(A, rank, Einv, r)
    assert np.allclose(M @ z.ravel(), r.ravel(), rtol=1e-10, atol=1e-11)


def _ilu_dense_factors(A, rank, LU):
    """Dense L (unit lower) and U of the ILU(0) factor, in A's numbering."""
    n = A.n
    L = np.eye(A.N * n)
    U = np.zeros((A.N * n, A.N * n))
    for i in range(A.N):
        for s in range(A.row_ptr[i], A.row_ptr[i + 1]):
            j = A.col[s]
            blk = (slice(i * n, (i + 1) * n), slice(j * n, (j + 1) * n))
            if rank[j] < rank[i]:
                L[blk] = LU[s]
            else:
                U[blk] = LU[s]
    return L, U


def _triangle_graph(seed):
    from workloads import jacobian_graph
    return jacobian_graph(N=60, n=3, hubs=3, hub_degree=10, base_degree=3, seed=seed)


def test_ilu0_defining_property_on_a_graph_with_fill():
    """ILU(0): (L U)_ij = A_ij at every block (i, j) of A's pattern; the fill
    it drops makes L U differ from A elsewhere; z = (L U)^{-1} r."""
    s = _triangle_graph(20)
    A = O.from_system(s)
    rank = np.random.default_rng(21).permutation(A.N)
    LU, Uinv = O.ilu0_setup(A, rank)
    L, U = _ilu_dense_factors(A, rank, LU)
    M, Ad = L @ U, A.dense()
    n = A.n
    inpat = np.zeros((A.N, A.N), bool)
    inpat[np.repeat(np.arange(A.N), np.diff(A.row_ptr)), A.col] = True
    mask = np.kron(inpat, np.ones((n, n), bool))
    assert np.allclose(M[mask], Ad[mask], rtol=1e-11, atol=1e-11)
    assert np.abs(M[~mask]).max() > 1e-3                  # dropped fill-in is real
    for i in range(A.N):
        assert np.allclose(Uinv[i] @ U[i * n:(i + 1) * n, i * n:(i + 1) * n], np.eye(n), atol=1e-11)
    r = np.random.default_rng(22).standard_normal((A.N, n))
    z = O.ilu0_apply(A, rank, LU, Uinv, r)
    assert np.allclose(z.ravel(), np.linalg.solve(M, r.ravel()), rtol=1e-10, atol=1e-11)


def test_ilu0_on_a_full_pattern_is_exact_block_lu():
    """Every block present: no fill is dropped, so L U = A and one apply solves."""
    N, n = 6, 3
    rng = np.random.default_rng(23)
    pairs = np.array([(i, j) for i in range(N) for j in range(i + 1, N)], np.int32)
    D = rng.standard_normal((N, n, n)) + 8 * np.eye(n)
    A = O.ldu_to_bcsr(N, n, pairs[:, 0], pairs[:, 1], D, rng.standard_normal((len(pairs), n, n)),
                      rng.standard_normal((len(pairs), n, n)))[0]
    rank = rng.permutation(N)
    LU, Uinv = O.ilu0_setup(A, rank)
    L, U = _ilu_dense_factors(A, rank, LU)
    assert np.allclose(L @ U, A.dense(), rtol=1e-12, atol=1e-12)
    b = rng.standard_normal((N, n))
    assert np.allclose(O.ilu0_apply(A, rank, LU, Uinv, b).ravel(), np.linalg.solve(A.dense(), b.ravel()),
                       rtol=1e-11, atol=1e-12)


def test_ilu0_equals_dilu_without_triangles_and_differs_with_them():
    """Without triangles in the block graph (a hex mesh) no update lands off the
    diagonal, so ILU(0) keeps A's off-diagonal blocks and its diagonal is the
    DILU one: the two preconditioners coincide.  With triangles they differ."""
    for s, same in ((jacobian_box(5, 4, 3, n=3, seed=24), True), (_triangle_graph(25), False)):
        A = O.from_system(s)
        rank = np.random.default_rng(26).permutation(A.N)
        LU, Uinv = O.ilu0_setup(A, rank)
        Einv = O.dilu_setup(A, rank)
        r = np.random.default_rng(27).standard_normal((A.N, A.n))
        zi = O.ilu0_apply(A, rank, LU, Uinv, r)
        zd = O.dilu_apply(A, rank, Einv, r)
        err = np.linalg.norm(zi - zd) / np.linalg.norm(zd)
        assert (err <= 1e-12) if same else (err > 1e-4), err


def test_ilu0_singular_pivot_is_reported():
    N, n = 3, 2
    D = np.stack([np.eye(n), np.zeros((n, n)), np.eye(n)])
    A = O.ldu_to_bcsr(N, n, [], [], D, np.zeros((0, n, n)), np.zeros((0, n, n)))[0]
    with pytest.raises(O.OracleError):
        O.ilu0_setup(A, np.arange(N))
