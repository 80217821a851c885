"""Invariants of the seeded input generators (no solver arithmetic here)."""
import numpy as np

from workloads import (batch_sizes, box_faces, concat_systems, jacobian_box, jacobian_graph,
                       jacobian_stretched, pressure_velocity, stretched_spacing)


def test_box_face_count_and_order():
    la, ua, dr = box_faces(4, 3, 2)
    assert la.size == 3 * 3 * 2 + 4 * 2 * 2 + 4 * 3 * 1
    assert np.all(la < ua)
    assert np.all(np.diff(dr) >= 0)          # x-faces, then y, then z


def test_full_size_counts_match_the_stated_workloads():
    la, _, _ = box_faces(20, 20, 20)
    assert la.size == 22800 and 8000 + 2 * la.size == 53600
    la, _, _ = box_faces(100, 100, 100)
    assert la.size == 2970000
    la, _, _ = box_faces(200, 100, 100)
    assert la.size == 5950000


def test_jacobian_is_seeded_and_positive_real():
    a = jacobian_box(5, 4, 3, seed=0)
    b = jacobian_box(5, 4, 3, seed=0)
    assert np.array_equal(a["upper"], b["upper"]) and np.array_equal(a["b"], b["b"])
    assert not np.array_equal(jacobian_box(5, 4, 3, seed=1)["b"], a["b"])
    N, n = a["N"], 5
    A = np.zeros((N * n, N * n))
    for i in range(N):
        A[i * n:(i + 1) * n, i * n:(i + 1) * n] = a["diag"][i]
    for f, (l, u) in enumerate(zip(a["lower_addr"], a["upper_addr"])):
        A[l * n:(l + 1) * n, u * n:(u + 1) * n] = a["upper"][f]
        A[u * n:(u + 1) * n, l * n:(l + 1) * n] = a["lower"][f]
    assert np.linalg.eigvalsh(0.5 * (A + A.T)).min() >= 1.0 - 1e-10


def test_stretched_mesh_spacing():
    dz = stretched_spacing(60)
    assert dz[0] == 1e-3 and abs(dz[1] / dz[0] - 1.2) < 1e-12 and dz[-1] == 1.0
    s = jacobian_stretched(3, 3, 50, seed=0)
    assert s["meta"]["max_aspect"] >= 999.0


def test_pressure_velocity_structure():
    s = pressure_velocity(5, 4, 3, seed=0)
    assert s["n"] == 4 and s["meta"]["min_volume"] > 0
    # momentum sub-block is a multiple of I3 and pp diagonal is positive
    D = s["diag"]
    uu = D[:, 1:, 1:]
    assert np.allclose(uu, uu[:, :1, :1] * np.eye(3))
    assert np.all(D[:, 0, 0] > 0)
    assert np.all(s["upper"][:, 0, 0] < 0) and np.all(s["lower"][:, 0, 0] < 0)


def test_batch_sizes_in_range_and_concat_offsets():
    shapes = batch_sizes(64, seed=0)
    sizes = np.array([a * b * c for a, b, c in shapes])
    assert len(shapes) == 64 and sizes.min() >= 5000 and sizes.max() <= 700000
    sys_ = [jacobian_box(3, 2, 2, seed=1), jacobian_box(2, 2, 2, seed=2)]
    cat = concat_systems(sys_)
    assert cat["cell_off"].tolist() == [0, 12, 20]
    assert cat["face_off"].tolist() == [0, sys_[0]["F"], sys_[0]["F"] + sys_[1]["F"]]


def test_spectral_norm_helper_matches_library_svd():
    from workloads.gen import _spectral_norms
    rng = np.random.default_rng(3)
    for n in (1, 2, 4, 5):
        J = rng.normal(0.0, 0.2, size=(500, n, n))
        ref = np.linalg.norm(J, ord=2, axis=(1, 2))
        assert np.allclose(_spectral_norms(J), ref, rtol=1e-12, atol=1e-15)


def test_graph_workload_faces_and_row_sums():
    """Random graph: faces unique and valid, both orientations present, a few
    rows far longer than a hexahedral mesh gives, seeded, and every block row
    sums to the identity (unit cell weight)."""
    s = jacobian_graph(N=600, n=3, hubs=4, hub_degree=40, base_degree=3, seed=5)
    assert np.array_equal(s["upper"], jacobian_graph(N=600, n=3, hubs=4, hub_degree=40, base_degree=3,
                                                     seed=5)["upper"])
    N, la, ua = s["N"], s["lower_addr"], s["upper_addr"]
    assert np.all((la >= 0) & (la < N) & (ua >= 0) & (ua < N)) and np.all(la != ua)
    key = np.minimum(la, ua).astype(np.int64) * N + np.maximum(la, ua)
    assert np.unique(key).size == key.size
    assert 0.3 < np.mean(la > ua) < 0.7
    deg = np.bincount(np.concatenate([la, ua]), minlength=N)
    assert deg.max() >= 35 and np.median(deg) <= 8
    rows = s["diag"].copy()
    np.add.at(rows, la, s["upper"])
    np.add.at(rows, ua, s["lower"])
    assert np.allclose(rows, np.eye(3)[None], atol=1e-12)

