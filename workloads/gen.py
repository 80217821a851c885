"""Seeded synthetic coupled block systems in face-addressed (LDU) form.

These generators produce the *inputs* of the coupled solve: a cell count N,
an internal-face list (owner ``lower_addr[f]``, neighbour ``upper_addr[f]``),
the n x n blocks ``diag[N]``, ``upper[F]``, ``lower[F]`` (each block row-major)
and a right-hand side ``b[N, n]``.  Storage convention: ``upper[f]`` is the
block at (row ``lower_addr[f]``, column ``upper_addr[f]``) and ``lower[f]`` the
block at (row ``upper_addr[f]``, column ``lower_addr[f]``).

Nothing here solves anything; both the CPU oracle and the GPU library read the
same arrays, so these constructions only set the conditioning of the
workloads.  Four families stand in for the paper's two industrial systems:

* ``jacobian_box``   -- density-based 5x5 blocks built like the approximate
  face Jacobian of Sec. 2.1 (Eqs. approxJac1/approxJac2) with a randomised
  flux Jacobian per face, plus the V/dtau identity of Eq. discretBackward.
* ``jacobian_stretched`` -- the same blocks on a boundary-layer mesh whose
  wall-normal spacing grows geometrically (face areas and volumes enter the
  block weights, as S_f does in approxJac1/2).
* ``pressure_velocity`` -- the 4x4 (p, Ux, Uy, Uz) blocks of Sec. 2.2
  (Eq. prb_coeff and the face coefficients that follow it) on a jittered,
  randomly renumbered hexahedral mesh.
* ``batch_sizes`` / ``jacobian_batch`` -- many independent density-based
  systems of log-uniform sizes concatenated with cell and face offsets
  (the offset layout of the consolidation scheme in Sec. 2.3).
* ``jacobian_graph`` -- the density-based blocks on a random face graph with
  a few very high-degree cells: an edge case for row lengths (far beyond a
  hexahedral mesh's seven blocks), random cell order and face orientation.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "box_faces", "jacobian_box", "jacobian_stretched", "pressure_velocity",
    "batch_sizes", "jacobian_batch", "concat_systems", "stretched_spacing", "jacobian_graph",
    "luo_inputs", "pu_inputs",
]


# --------------------------------------------------------------------------
# structured box topology
# --------------------------------------------------------------------------
def box_faces(nx: int, ny: int, nz: int):
    """Internal faces of an nx*ny*nz box of cells.

    Cell id = i + nx*(j + ny*k).  Faces are listed x-direction first, then y,
    then z; within a direction in cell-id order of the owner.  The owner is
    the lower id.  Returns (lower_addr, upper_addr, direction) as int32/int8.
    """
    ids = np.arange(nx * ny * nz, dtype=np.int64).reshape(nz, ny, nx)
    lo, up, dr = [], [], []
    if nx > 1:
        lo.append(ids[:, :, :-1].ravel()); up.append(ids[:, :, 1:].ravel())
        dr.append(np.zeros(lo[-1].size, np.int8))
    if ny > 1:
        lo.append(ids[:, :-1, :].ravel()); up.append(ids[:, 1:, :].ravel())
        dr.append(np.ones(lo[-1].size, np.int8))
    if nz > 1:
        lo.append(ids[:-1, :, :].ravel()); up.append(ids[1:, :, :].ravel())
        dr.append(np.full(lo[-1].size, 2, np.int8))
    if not lo:
        z = np.zeros(0, np.int32)
        return z, z.copy(), np.zeros(0, np.int8)
    return (np.concatenate(lo).astype(np.int32), np.concatenate(up).astype(np.int32),
            np.concatenate(dr))


_SPEC_LIB = None


def _spec_lib():
    """specnorm.c built with gcc on first use (input generation helper)."""
    global _SPEC_LIB
    if _SPEC_LIB is None:
        import ctypes
        import os
        import subprocess
        here = os.path.dirname(os.path.abspath(__file__))
        src, so = os.path.join(here, "specnorm.c"), os.path.join(here, "libspecnorm.so")
        if not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(src):
            tmp = so + ".tmp%d" % os.getpid()
            subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
            os.replace(tmp, so)
        lib = ctypes.CDLL(so)
        lib.spectral_norms.restype = None
        lib.spectral_norms.argtypes = [ctypes.c_long, ctypes.c_int,
                                       np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS"),
                                       np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")]
        _SPEC_LIB = lib
    return _SPEC_LIB


def _spectral_norms(J: np.ndarray) -> np.ndarray:
    """Largest singular value of each square block: sqrt(lambda_max(J^T J)),
    eigenvalues by cyclic Jacobi rotations (specnorm.c)."""
    J = np.ascontiguousarray(J, dtype=np.float64)
    out = np.empty(J.shape[0])
    if J.shape[0]:
        _spec_lib().spectral_norms(J.shape[0], J.shape[1], J.reshape(-1), out)
    return out


def _jacobian_blocks(N, lower_addr, upper_addr, J, face_w, cell_w, n, variant="A"):
    """Assemble diag/upper/lower from one random flux Jacobian per face.

    W_f = face_w[f] * 1/2 (J_f + s_f I), s_f = ||J_f||_2 (a stand-in for the
    spectral-radius term |lambda_ij| of approxJac1/2).  Variant "A": both
    off-diagonal blocks are -W_f and both diagonal blocks gain +W_f, so every
    block row sums to cell_w[i] * I.  Variant "B" flips the sign of J in the
    neighbour's row, following R_ij(n_ij) = -R_ji(n_ji).
    """
    F = lower_addr.size
    eye = np.eye(n)
    s = _spectral_norms(J)
    Wp = 0.5 * (J + s[:, None, None] * eye) * face_w[:, None, None]
    if variant == "A":
        Wn = Wp
    elif variant == "B":
        Wn = 0.5 * (-J + s[:, None, None] * eye) * face_w[:, None, None]
    else:
        raise ValueError("variant must be 'A' or 'B'")
    # Per-cell sums of the face contributions; bincount accumulates in face
    # order, so the result is reproducible.
    nn = n * n
    lanes = np.arange(nn, dtype=np.int64)

    def cell_sums(addr, W):
        idx = (addr.astype(np.int64)[:, None] * nn + lanes).reshape(-1)
        return np.bincount(idx, weights=W.reshape(-1), minlength=N * nn).reshape(N, n, n)

    diag = cell_sums(lower_addr, Wp)
    diag += cell_sums(upper_addr, Wn)
    diag += cell_w[:, None, None] * eye
    upper = -Wp          # row owner, column neighbour
    lower = -Wn          # row neighbour, column owner
    return diag, np.ascontiguousarray(upper), np.ascontiguousarray(lower)


def _pack(N, n, lower_addr, upper_addr, diag, upper, lower, b, meta):
    return {
        "N": int(N), "F": int(lower_addr.size), "n": int(n),
        "lower_addr": np.ascontiguousarray(lower_addr, dtype=np.int32),
        "upper_addr": np.ascontiguousarray(upper_addr, dtype=np.int32),
        "diag": np.ascontiguousarray(diag, dtype=np.float64),
        "upper": np.ascontiguousarray(upper, dtype=np.float64),
        "lower": np.ascontiguousarray(lower, dtype=np.float64),
        "b": np.ascontiguousarray(b, dtype=np.float64),
        "meta": meta,
    }


def jacobian_box(nx=20, ny=20, nz=20, n=5, seed=0, sigma=0.2, vdt=1.0, variant="A"):
    """Density-based coupled Jacobian on a unit-spacing box (S_f = 1, V = 1).

    Draw order from ``numpy.random.default_rng(seed)``: all J_f (faces in
    x, y, z order, each block row-major) with N(0, sigma^2) entries, then b
    with U(-1, 1) entries, cell-major / variable-minor.
    """
    N = nx * ny * nz
    la, ua, _ = box_faces(nx, ny, nz)
    rng = np.random.default_rng(seed)
    J = rng.normal(0.0, sigma, size=(la.size, n, n))
    b = rng.uniform(-1.0, 1.0, size=(N, n))
    diag, upper, lower = _jacobian_blocks(
        N, la, ua, J, np.ones(la.size), np.full(N, vdt), n, variant)
    return _pack(N, n, la, ua, diag, upper, lower, b,
                 {"kind": "jacobian_box", "shape": [nx, ny, nz], "seed": seed,
                  "sigma": sigma, "vdt": vdt, "variant": variant})


def stretched_spacing(nz: int, dz0=1e-3, ratio=1.2, dzmax=1.0) -> np.ndarray:
    """Wall-normal spacing: dz0, growing by `ratio` until it reaches dzmax."""
    dz = np.empty(nz)
    d = dz0
    for k in range(nz):
        dz[k] = min(d, dzmax)
        d *= ratio
    return dz


def jacobian_stretched(nx=200, ny=200, nz=200, n=5, seed=0, sigma=0.2,
                       dz0=1e-3, ratio=1.2, variant="A"):
    """Density-based Jacobian on a boundary-layer box (dx = dy = 1, dz graded).

    Face blocks carry the face area S_f and the diagonal the cell volume V
    (dtau = 1), as S_f and V enter approxJac1/2 and discretBackward.  Draw
    order as in :func:`jacobian_box`.
    """
    N = nx * ny * nz
    la, ua, dr = box_faces(nx, ny, nz)
    dz = stretched_spacing(nz, dz0, ratio)
    kcell = np.repeat(np.arange(nz), nx * ny)            # k of each cell id
    vol = dz[kcell]
    # x- and y-faces have area dz of the shared layer, z-faces have area 1
    area = np.where(dr == 2, 1.0, dz[kcell[la]])
    rng = np.random.default_rng(seed)
    J = rng.normal(0.0, sigma, size=(la.size, n, n))
    b = rng.uniform(-1.0, 1.0, size=(N, n))
    diag, upper, lower = _jacobian_blocks(N, la, ua, J, area, vol, n, variant)
    return _pack(N, n, la, ua, diag, upper, lower, b,
                 {"kind": "jacobian_stretched", "shape": [nx, ny, nz], "seed": seed,
                  "dz0": dz0, "ratio": ratio, "max_aspect": float(1.0 / dz.min())})


# --------------------------------------------------------------------------
# pressure-based p-U coupled system on a jittered hexahedral mesh
# --------------------------------------------------------------------------
def _quad_area(p0, p1, p2, p3):
    """Area vector of a (possibly warped) quad: half the cross product of its
    diagonals; centre = mean of the four nodes."""
    S = 0.5 * np.cross(p2 - p0, p3 - p1)
    c = 0.25 * (p0 + p1 + p2 + p3)
    return S, c


def pressure_velocity(nx=100, ny=100, nz=100, seed=0, jitter=0.2, nu=0.01,
                      permute=True, lengths=None):
    """4x4 (p, Ux, Uy, Uz) coupled system of the pressure-based solver.

    Face coefficients follow the block split of Eq. prb_coeff: upwind
    convection plus central diffusion in the uu sub-block, linear-interpolated
    face-area vectors (weights f_x, 1 - f_x) in the up and pu sub-blocks, and a
    Rhie-Chow pressure Laplacian with D = V / a_ii^uu in pp, signed so that
    the pp diagonal is positive (the sign the continuity equation with the
    Rhie-Chow flux gives).  Velocity is a uniform field u ~ U(0,1)^3.
    Boundary faces (all six sides) act on the diagonal only: Dirichlet
    velocity (diffusion and inflow convection), pressure extrapolated in the
    momentum rows, outflow velocity in continuity, and p = 0 at outflow faces
    in the Rhie-Chow Laplacian.

    Draw order from ``default_rng(seed)``: node jitter U(-jitter*h, jitter*h)
    for every node (applied to interior nodes only), the cell permutation,
    the velocity, then b ~ U(-1, 1).
    """
    n = 4
    if lengths is None:
        Lx, Ly, Lz = nx / nz, ny / nz, 1.0          # h = 1/nz in every direction
    else:
        Lx, Ly, Lz = lengths
    hx, hy, hz = Lx / nx, Ly / ny, Lz / nz
    N = nx * ny * nz
    rng = np.random.default_rng(seed)
    gx = np.linspace(0.0, Lx, nx + 1)
    gy = np.linspace(0.0, Ly, ny + 1)
    gz = np.linspace(0.0, Lz, nz + 1)
    X = np.stack(np.meshgrid(gx, gy, gz, indexing="ij"), axis=-1)  # (nx+1,ny+1,nz+1,3)
    hmin = min(hx, hy, hz)
    jit = rng.uniform(-jitter * hmin, jitter * hmin, size=X.shape)
    interior = np.zeros(X.shape[:3], bool)
    interior[1:-1, 1:-1, 1:-1] = True
    X = X + jit * interior[..., None]
    perm = rng.permutation(N) if permute else np.arange(N)
    uinf = rng.uniform(0.0, 1.0, size=3)

    # cell centres, cell (i,j,k) -> id i + nx*(j + ny*k); arrays indexed [k,j,i]
    Xk = np.transpose(X, (2, 1, 0, 3))                               # [k,j,i,3]
    C = 0.125 * (Xk[:-1, :-1, :-1] + Xk[:-1, :-1, 1:] + Xk[:-1, 1:, :-1] + Xk[:-1, 1:, 1:]
                 + Xk[1:, :-1, :-1] + Xk[1:, :-1, 1:] + Xk[1:, 1:, :-1] + Xk[1:, 1:, 1:])
    cc = C.reshape(N, 3)
    ids = np.arange(N).reshape(nz, ny, nx)

    # face node planes: x-face at node index i (between cells i-1, i)
    def xquad(kk, jj, ii):
        return (Xk[kk, jj, ii], Xk[kk, jj + 1, ii], Xk[kk + 1, jj + 1, ii], Xk[kk + 1, jj, ii])

    def yquad(kk, jj, ii):
        return (Xk[kk, jj, ii], Xk[kk + 1, jj, ii], Xk[kk + 1, jj, ii + 1], Xk[kk, jj, ii + 1])

    def zquad(kk, jj, ii):
        return (Xk[kk, jj, ii], Xk[kk, jj, ii + 1], Xk[kk, jj + 1, ii + 1], Xk[kk, jj + 1, ii])

    faces_S, faces_c, faces_P, faces_N = [], [], [], []
    bS, bc, bP = [], [], []

    def add_dir(quad, Kc, Jc, Ic, nplanes, axis):
        # internal: node plane index m = 1..nplanes-1 between cell m-1 and m
        sl_int = [slice(None)] * 3
        sl_int[axis] = slice(1, nplanes)
        kk, jj, ii = Kc[tuple(sl_int)], Jc[tuple(sl_int)], Ic[tuple(sl_int)]
        S, c = _quad_area(*quad(kk, jj, ii))
        idxP = [kk, jj, ii]; idxN = [kk, jj, ii]
        idxP[axis] = idxP[axis] - 1
        P = ids[tuple(idxP)]; Nn = ids[tuple(idxN)]
        faces_S.append(S.reshape(-1, 3)); faces_c.append(c.reshape(-1, 3))
        faces_P.append(P.ravel()); faces_N.append(Nn.ravel())
        # boundary at plane 0 (owner = cell 0) and plane nplanes (owner = last)
        for m, cellm in ((0, 0), (nplanes, nplanes - 1)):
            sl = [slice(None)] * 3
            sl[axis] = slice(m, m + 1)
            kk, jj, ii = Kc[tuple(sl)], Jc[tuple(sl)], Ic[tuple(sl)]
            S, c = _quad_area(*quad(kk, jj, ii))
            idx = [kk, jj, ii]
            idx[axis] = np.full_like(idx[axis], cellm)
            bS.append(S.reshape(-1, 3)); bc.append(c.reshape(-1, 3))
            bP.append(ids[tuple(idx)].ravel())

    # node-plane grids for each direction, array order [k, j, i]
    Kx, Jx, Ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx + 1), indexing="ij")
    add_dir(xquad, Kx, Jx, Ix, nx, 2)
    Ky, Jy, Iy = np.meshgrid(np.arange(nz), np.arange(ny + 1), np.arange(nx), indexing="ij")
    add_dir(yquad, Ky, Jy, Iy, ny, 1)
    Kz, Jz, Iz = np.meshgrid(np.arange(nz + 1), np.arange(ny), np.arange(nx), indexing="ij")
    add_dir(zquad, Kz, Jz, Iz, nz, 0)

    S = np.concatenate(faces_S); xf = np.concatenate(faces_c)
    P = np.concatenate(faces_P).astype(np.int64); Nc = np.concatenate(faces_N).astype(np.int64)
    Sb = np.concatenate(bS); xb = np.concatenate(bc); Pb = np.concatenate(bP).astype(np.int64)
    # orient: internal S from P to N; boundary S outward from P
    d = cc[Nc] - cc[P]
    sgn = np.sign(np.einsum("fi,fi->f", S, d)); sgn[sgn == 0] = 1.0
    S = S * sgn[:, None]
    db = xb - cc[Pb]
    sgnb = np.sign(np.einsum("fi,fi->f", Sb, db)); sgnb[sgnb == 0] = 1.0
    Sb = Sb * sgnb[:, None]

    # volumes: V = 1/3 sum_f x_f . S_f (outward)
    vol = np.zeros(N)
    np.add.at(vol, P, np.einsum("fi,fi->f", xf, S) / 3.0)
    np.add.at(vol, Nc, -np.einsum("fi,fi->f", xf, S) / 3.0)
    np.add.at(vol, Pb, np.einsum("fi,fi->f", xb, Sb) / 3.0)

    magS = np.linalg.norm(S, axis=1)
    nrm = S / magS[:, None]
    nd = np.einsum("fi,fi->f", nrm, d)
    fx = np.einsum("fi,fi->f", nrm, cc[Nc] - xf) / nd       # weight of the owner P
    Fl = S @ uinf
    diff = nu * magS / nd
    magSb = np.linalg.norm(Sb, axis=1)
    ndb = np.einsum("fi,fi->f", Sb / magSb[:, None], db)
    Fb = Sb @ uinf
    diffb = nu * magSb / ndb

    # momentum diagonal (scalar times I3)
    auu = np.zeros(N)
    np.add.at(auu, P, np.maximum(Fl, 0.0) + diff)
    np.add.at(auu, Nc, np.maximum(-Fl, 0.0) + diff)
    np.add.at(auu, Pb, np.maximum(Fb, 0.0) + diffb)
    Dc = vol / auu
    Df = fx * Dc[P] + (1.0 - fx) * Dc[Nc]
    g = Df * magS / nd

    F = P.size
    eye3 = np.eye(3)
    upper = np.zeros((F, 4, 4)); lower = np.zeros((F, 4, 4)); diag = np.zeros((N, 4, 4))
    # row P, column N
    upper[:, 0, 0] = -g
    upper[:, 0, 1:] = (1.0 - fx)[:, None] * S
    upper[:, 1:, 0] = (1.0 - fx)[:, None] * S
    upper[:, 1:, 1:] = -(np.maximum(-Fl, 0.0) + diff)[:, None, None] * eye3
    # row N, column P
    lower[:, 0, 0] = -g
    lower[:, 0, 1:] = -fx[:, None] * S
    lower[:, 1:, 0] = -fx[:, None] * S
    lower[:, 1:, 1:] = -(np.maximum(Fl, 0.0) + diff)[:, None, None] * eye3
    dP = np.zeros((F, 4, 4)); dN = np.zeros((F, 4, 4))
    dP[:, 0, 0] = g; dP[:, 0, 1:] = fx[:, None] * S; dP[:, 1:, 0] = fx[:, None] * S
    dP[:, 1:, 1:] = (np.maximum(Fl, 0.0) + diff)[:, None, None] * eye3
    dN[:, 0, 0] = g; dN[:, 0, 1:] = -(1.0 - fx)[:, None] * S
    dN[:, 1:, 0] = -(1.0 - fx)[:, None] * S
    dN[:, 1:, 1:] = (np.maximum(-Fl, 0.0) + diff)[:, None, None] * eye3
    np.add.at(diag, P, dP)
    np.add.at(diag, Nc, dN)
    dB = np.zeros((Pb.size, 4, 4))
    out = Fb > 0.0
    dB[:, 1:, 1:] = (np.maximum(Fb, 0.0) + diffb)[:, None, None] * eye3
    dB[:, 1:, 0] = Sb
    dB[:, 0, 1:] = Sb * out[:, None]
    dB[:, 0, 0] = np.where(out, Dc[Pb] * magSb / ndb, 0.0)
    np.add.at(diag, Pb, dB)

    # renumber cells: new id = perm[old id]; faces keep their orientation
    la = perm[P].astype(np.int32); ua = perm[Nc].astype(np.int32)
    diag_new = np.empty_like(diag); diag_new[perm] = diag
    b = rng.uniform(-1.0, 1.0, size=(N, n))
    return _pack(N, n, la, ua, diag_new, upper, lower, b,
                 {"kind": "pressure_velocity", "shape": [nx, ny, nz], "seed": seed,
                  "jitter": jitter, "nu": nu, "permuted": bool(permute),
                  "uinf": uinf.tolist(), "min_volume": float(vol.min())})


# --------------------------------------------------------------------------
# batches of uneven systems
# --------------------------------------------------------------------------
def batch_sizes(k=64, lo=1e4, hi=5e5, seed=0):
    """Box shapes for k systems of log-uniform size in [lo, hi] cells."""
    rng = np.random.default_rng(seed)
    Nk = np.round(np.exp(rng.uniform(np.log(lo), np.log(hi), size=k))).astype(np.int64)
    shapes = []
    for N in Nk:
        a = max(1, int(round(N ** (1.0 / 3.0))))
        c = max(1, int(round(N / (a * a))))
        shapes.append((a, a, c))
    return shapes


def concat_systems(systems):
    """Concatenate systems with per-system local indices and int64 offsets."""
    n = systems[0]["n"]
    cell_off = np.zeros(len(systems) + 1, np.int64)
    face_off = np.zeros(len(systems) + 1, np.int64)
    for i, s in enumerate(systems):
        assert s["n"] == n
        cell_off[i + 1] = cell_off[i] + s["N"]
        face_off[i + 1] = face_off[i] + s["F"]
    cat = lambda key: np.concatenate([s[key] for s in systems])
    return {
        "n_sys": len(systems), "n": n, "cell_off": cell_off, "face_off": face_off,
        "N": int(cell_off[-1]), "F": int(face_off[-1]),
        "lower_addr": cat("lower_addr"), "upper_addr": cat("upper_addr"),
        "diag": cat("diag"), "upper": cat("upper"), "lower": cat("lower"), "b": cat("b"),
    }


def jacobian_batch(k=64, lo=1e4, hi=5e5, seed=0, n=5):
    """k density-based box systems, system i seeded with 1 + i."""
    shapes = batch_sizes(k, lo, hi, seed)
    systems = [jacobian_box(*sh, n=n, seed=1 + i) for i, sh in enumerate(shapes)]
    out = concat_systems(systems)
    out["shapes"] = shapes
    return out


def jacobian_graph(N=3000, n=4, hubs=12, hub_degree=48, base_degree=4, seed=0, sigma=0.2):
    """Density-type blocks (as in ``jacobian_box``, unit face and cell
    weights) on a random face graph: every cell draws ``base_degree`` random
    partners and ``hubs`` cells draw ``hub_degree`` more, so a few block rows
    hold over 50 blocks.  Self pairs are dropped, repeated unordered pairs
    kept once (first draw), and each face's orientation is random, so the
    owner may be the higher cell index.

    Draw order from ``numpy.random.default_rng(seed)``: the N*base_degree base
    pairs (first cells, then second cells), the hub cells, their partners
    (hub-major), the orientation coin per kept face, J_f (N(0, sigma^2)),
    then b (U(-1, 1)).
    """
    rng = np.random.default_rng(seed)
    a = rng.integers(0, N, size=N * base_degree)
    c = rng.integers(0, N, size=N * base_degree)
    hub = rng.choice(N, size=hubs, replace=False)
    partners = rng.integers(0, N, size=(hubs, hub_degree))
    a = np.concatenate([a, np.repeat(hub, hub_degree)])
    c = np.concatenate([c, partners.reshape(-1)])
    keep = a != c
    lo, hi = np.minimum(a, c)[keep], np.maximum(a, c)[keep]
    _, first = np.unique(lo.astype(np.int64) * N + hi, return_index=True)
    first.sort()
    lo, hi = lo[first], hi[first]
    flip = rng.random(lo.size) < 0.5
    la = np.where(flip, hi, lo)
    ua = np.where(flip, lo, hi)
    F = la.size
    J = rng.normal(0.0, sigma, size=(F, n, n))
    b = rng.uniform(-1.0, 1.0, size=(N, n))
    diag, upper, lower = _jacobian_blocks(N, la, ua, J, np.ones(F), np.ones(N), n, "A")
    return _pack(N, n, la, ua, diag, upper, lower, b,
                 {"kind": "jacobian_graph", "N": N, "hubs": hubs, "hub_degree": hub_degree,
                  "base_degree": base_degree, "seed": seed, "sigma": sigma})



def luo_inputs(nx=20, ny=20, nz=20, seed=0, jitter=0.2, gamma=1.4, mach=0.5, cfl=10.0, uniform=False):
    """Inputs of the GPU assembly of the density-based coupled matrix: a
    jittered hex box of nx*ny*nz cells (unit spacing h = 1/nz), its internal
    faces in ``box_faces`` order with area vectors S_f n_f pointing from the
    owner (lower id) to the neighbour, a conservative state Q = (rho, rho u,
    rho v, rho w, rho E) per cell, a viscous spectral radius per unit area
    per face and V/dtau per cell.  Only geometry and states: no Jacobian.

    State: rho ~ U(0.8, 1.2), p ~ U(0.8, 1.2)/gamma, velocity = free stream
    (mach, 0.2 mach, 0.1 mach) + N(0, (0.1 mach)^2) per component (all
    cells equal to the first draw when ``uniform``); rho E = p/(gamma-1) +
    rho |u|^2 / 2.  lam_visc ~ U(0, 0.05); V/dtau = h^2 (|u| + c) / cfl with
    cfl ~ U(0.5, 2) * cfl per cell.

    Draw order from ``default_rng(seed)``: node jitter U(-jitter h, jitter h)
    for every node (applied to interior nodes only), rho, p, velocity
    perturbation, lam_visc, the cfl factors.
    """
    N = nx * ny * nz
    h = 1.0 / nz
    rng = np.random.default_rng(seed)
    g = [np.arange(m + 1) * h for m in (nx, ny, nz)]
    X = np.stack(np.meshgrid(*g, indexing="ij"), axis=-1)          # (nx+1, ny+1, nz+1, 3)
    jit = rng.uniform(-jitter * h, jitter * h, size=X.shape)
    interior = np.zeros(X.shape[:3], bool)
    interior[1:-1, 1:-1, 1:-1] = True
    X = X + jit * interior[..., None]
    Xk = np.transpose(X, (2, 1, 0, 3))                               # [k, j, i, 3]
    la, ua, dr = box_faces(nx, ny, nz)
    S = []
    if nx > 1:   # x faces at node plane i+1 between cells i and i+1, order [k, j, i]
        q = (Xk[:-1, :-1, 1:-1], Xk[:-1, 1:, 1:-1], Xk[1:, 1:, 1:-1], Xk[1:, :-1, 1:-1])
        S.append(_quad_area(*q)[0].reshape(-1, 3))
    if ny > 1:
        q = (Xk[:-1, 1:-1, :-1], Xk[1:, 1:-1, :-1], Xk[1:, 1:-1, 1:], Xk[:-1, 1:-1, 1:])
        S.append(_quad_area(*q)[0].reshape(-1, 3))
    if nz > 1:
        q = (Xk[1:-1, :-1, :-1], Xk[1:-1, :-1, 1:], Xk[1:-1, 1:, 1:], Xk[1:-1, 1:, :-1])
        S.append(_quad_area(*q)[0].reshape(-1, 3))
    Sf = np.concatenate(S) if S else np.zeros((0, 3))
    rho = rng.uniform(0.8, 1.2, N)
    p = rng.uniform(0.8, 1.2, N) / gamma
    vel = np.array([1.0, 0.2, 0.1]) * mach + rng.normal(0.0, 0.1 * mach, (N, 3))
    if uniform:
        rho[:] = rho[0]; p[:] = p[0]; vel[:] = vel[0]
    lam_visc = rng.uniform(0.0, 0.05, la.size)
    cfl_c = cfl * rng.uniform(0.5, 2.0, N)
    Q = np.empty((N, 5))
    Q[:, 0] = rho
    Q[:, 1:4] = rho[:, None] * vel
    Q[:, 4] = p / (gamma - 1.0) + 0.5 * rho * (vel ** 2).sum(1)
    c = np.sqrt(gamma * p / rho)
    v_dt = h * h * (np.linalg.norm(vel, axis=1) + c) / cfl_c
    return {"N": N, "F": int(la.size), "n": 5, "lower_addr": la, "upper_addr": ua, "Q": Q, "Sf": Sf,
            "lam_visc": lam_visc, "v_dt": v_dt, "gamma": float(gamma), "h": h}


def pu_inputs(nx=20, ny=20, nz=20, seed=0, jitter=0.2, nu=(0.005, 0.02)):
    """Inputs of the GPU assembly of the pressure-based (p, Ux, Uy, Uz)
    matrix: a jittered hex box (unit spacing h = 1/nz) with its internal faces
    in ``box_faces`` order, per face the area vector S_f (owner -> neighbour),
    the owner's linear-interpolation weight f_x, the centroid distance
    d = c_neighbour - c_owner, the previous-iteration volume flux u_f . S_f
    and nu_eff; per cell the volume and two diagonal additions standing in for
    boundary faces and pseudo-time relaxation (uu_add on the momentum
    diagonal, pp_add on the pressure diagonal).  Only geometry and fields.

    Velocity: u(x) = u0 (1 + 0.3 (sin 2 pi y, sin 2 pi z, sin 2 pi x)) at the
    face centre, u0 ~ U(0.2, 1)^3.  f_x = |c_u - x_f| / (|c_u - x_f| +
    |x_f - c_l|).  V = h^3 (1 + U(-0.05, 0.05)); uu_add = V |u0| / h U(0.5, 1.5);
    pp_add = 1e-3 h U(0.5, 1.5).

    Draw order from ``default_rng(seed)``: node jitter U(-jitter h, jitter h)
    for every node (applied to interior nodes only), u0, nu_eff per face
    U(nu), the volume factors, the uu_add factors, the pp_add factors.
    """
    N = nx * ny * nz
    h = 1.0 / nz
    rng = np.random.default_rng(seed)
    g = [np.arange(m + 1) * h for m in (nx, ny, nz)]
    X = np.stack(np.meshgrid(*g, indexing="ij"), axis=-1)
    jit = rng.uniform(-jitter * h, jitter * h, size=X.shape)
    interior = np.zeros(X.shape[:3], bool)
    interior[1:-1, 1:-1, 1:-1] = True
    X = X + jit * interior[..., None]
    Xk = np.transpose(X, (2, 1, 0, 3))
    C = 0.125 * (Xk[:-1, :-1, :-1] + Xk[:-1, :-1, 1:] + Xk[:-1, 1:, :-1] + Xk[:-1, 1:, 1:]
                 + Xk[1:, :-1, :-1] + Xk[1:, :-1, 1:] + Xk[1:, 1:, :-1] + Xk[1:, 1:, 1:]).reshape(N, 3)
    la, ua, _ = box_faces(nx, ny, nz)
    S, XF = [], []
    quads = []
    if nx > 1:
        quads.append((Xk[:-1, :-1, 1:-1], Xk[:-1, 1:, 1:-1], Xk[1:, 1:, 1:-1], Xk[1:, :-1, 1:-1]))
    if ny > 1:
        quads.append((Xk[:-1, 1:-1, :-1], Xk[1:, 1:-1, :-1], Xk[1:, 1:-1, 1:], Xk[:-1, 1:-1, 1:]))
    if nz > 1:
        quads.append((Xk[1:-1, :-1, :-1], Xk[1:-1, :-1, 1:], Xk[1:-1, 1:, 1:], Xk[1:-1, 1:, :-1]))
    for q in quads:
        a, c = _quad_area(*q)
        S.append(a.reshape(-1, 3)); XF.append(c.reshape(-1, 3))
    Sf = np.concatenate(S) if S else np.zeros((0, 3))
    xf = np.concatenate(XF) if XF else np.zeros((0, 3))
    d = C[ua] - C[la]
    dl = np.linalg.norm(xf - C[la], axis=1)
    du = np.linalg.norm(C[ua] - xf, axis=1)
    fx = du / (du + dl) if la.size else np.zeros(0)
    u0 = rng.uniform(0.2, 1.0, 3)
    tp = 2.0 * np.pi
    uf = u0 * (1.0 + 0.3 * np.stack([np.sin(tp * xf[:, 1]), np.sin(tp * xf[:, 2]), np.sin(tp * xf[:, 0])], axis=1))
    flux = (uf * Sf).sum(1)
    nu_f = rng.uniform(nu[0], nu[1], la.size)
    vol = h ** 3 * (1.0 + rng.uniform(-0.05, 0.05, N))
    uu_add = vol * np.linalg.norm(u0) / h * rng.uniform(0.5, 1.5, N)
    pp_add = 1e-3 * h * rng.uniform(0.5, 1.5, N)
    return {"N": N, "F": int(la.size), "n": 4, "lower_addr": la, "upper_addr": ua, "Sf": Sf, "fx": fx, "d": d,
            "flux": flux, "nu": nu_f, "vol": vol, "uu_add": uu_add, "pp_add": pp_add, "h": h}
