"""Seeded synthetic matrices and right-hand sides.

The paper's experiments use Galeri model problems (Laplace, elasticity),
SuiteSparse SPD matrices and Nalu-Wind systems (Sections 7-10).  None of those
are available here, so these generators build synthetic stand-ins with the
same shapes: 5/7-point Laplacians in natural ordering, a trilinear (Q1)
hexahedral elasticity operator with 3 dof per node, a variable-coefficient
diffusion operator and a batch of upwinded convection-diffusion operators.

Natural ordering (x fastest, then y, then z) is used everywhere and is never
permuted: Gauss-Seidel results depend on the ordering (Section 6, sequential
Gauss-Seidel).

This module contains no relaxation or Krylov arithmetic.  The only matrix
product here is b = A x_true for manufactured right-hand sides, done with
scipy.sparse.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MASTER_SEED = 2104


def rng_streams(k: int, seed: int = MASTER_SEED):
    """k independent numpy Generators spawned from one master seed."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


@dataclass
class CSR:
    n: int
    rowptr: np.ndarray  # int32, n+1
    colind: np.ndarray  # int32, nnz
    val: np.ndarray  # float64, nnz
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.colind, self.rowptr), shape=(self.n, self.n))

    def dense(self) -> np.ndarray:
        return self.to_scipy().toarray()

    def check(self) -> None:
        """Structural sanity: sorted unique columns, diagonal present."""
        rp, ci = self.rowptr, self.colind
        assert rp.dtype == np.int32 and ci.dtype == np.int32 and self.val.dtype == np.float64
        assert rp[0] == 0 and len(rp) == self.n + 1 and np.all(np.diff(rp) >= 1)
        rows = np.repeat(np.arange(self.n), np.diff(rp))
        same_row = rows[1:] == rows[:-1]
        assert np.all(ci[1:][same_row] > ci[:-1][same_row]), "columns not strictly increasing"
        assert np.all((ci >= 0) & (ci < self.n))
        has_diag = np.zeros(self.n, bool)
        has_diag[rows[ci == rows]] = True
        assert has_diag.all(), "missing diagonal"


def _from_dense_rows(cols: np.ndarray, vals: np.ndarray, mask: np.ndarray, meta=None) -> CSR:
    """Compress (n, k) candidate arrays (columns already sorted per row) into CSR."""
    n = cols.shape[0]
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colind = cols[mask].astype(np.int32)
    val = vals[mask].astype(np.float64)
    return CSR(n, rowptr.astype(np.int32), colind, val, meta or {})


def _stencil(shape, offsets, coeffs, diag):
    """Generic structured-grid operator.

    shape: (nz, ny, nx) grid; offsets: list of (dz, dy, dx) excluding (0,0,0);
    coeffs: list of arrays/scalars (one per offset, broadcast to the grid);
    diag: array/scalar diagonal.  Out-of-grid neighbours are dropped
    (homogeneous Dirichlet elimination).
    """
    nz, ny, nx = shape
    n = nz * ny * nx
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    z, y, x = z.ravel(), y.ravel(), x.ravel()
    row = np.arange(n, dtype=np.int64)
    ents = [((0, 0, 0), diag)] + list(zip(offsets, coeffs))
    ents.sort(key=lambda e: e[0][0] * ny * nx + e[0][1] * nx + e[0][2])
    k = len(ents)
    cols = np.empty((n, k), np.int64)
    vals = np.empty((n, k), np.float64)
    mask = np.empty((n, k), bool)
    for c, ((dz, dy, dx), coef) in enumerate(ents):
        cols[:, c] = row + dz * ny * nx + dy * nx + dx
        vals[:, c] = np.broadcast_to(np.asarray(coef, np.float64).ravel() if np.ndim(coef) else coef, (n,))
        mask[:, c] = (
            (z + dz >= 0) & (z + dz < nz) & (y + dy >= 0) & (y + dy < ny) & (x + dx >= 0) & (x + dx < nx)
        )
    return _from_dense_rows(cols, vals, mask)


def laplace1d(N: int) -> CSR:
    """1D 3-point Dirichlet Laplacian tridiag(-1, 2, -1), n = N."""
    A = _stencil((1, 1, N), [(0, 0, -1), (0, 0, 1)], [-1.0, -1.0], 2.0)
    A.meta = {"kind": "laplace1d", "N": N}
    return A


def poisson2d(N: int) -> CSR:
    """2D 5-point Dirichlet Laplacian (diagonal 4, off-diagonals -1), N x N
    interior points, natural x-fastest order: n = N^2, nnz = 5N^2 - 4N."""
    A = _stencil((1, N, N), [(0, -1, 0), (0, 0, -1), (0, 0, 1), (0, 1, 0)], [-1.0] * 4, 4.0)
    A.meta = {"kind": "poisson2d", "N": N}
    return A


_OFF7 = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 1), (0, 1, 0), (1, 0, 0)]


def laplace3d(N: int) -> CSR:
    """3D 7-point Dirichlet Laplacian (diagonal 6, off-diagonals -1) on N^3."""
    A = _stencil((N, N, N), _OFF7, [-1.0] * 6, 6.0)
    A.meta = {"kind": "laplace3d", "N": N}
    return A


def vardiff3d(N: int, seed: int = MASTER_SEED) -> CSR:
    """Cell-centred finite-volume -div(kappa grad u) on N^3 cells.

    kappa per cell is log-uniform over [1e-2, 1e2].  Interior face
    coefficients are the harmonic mean 2 k1 k2 / (k1 + k2); a Dirichlet
    boundary face at half a cell contributes 2 kappa_cell to the diagonal.
    Symmetric positive definite M-matrix.
    """
    (rng,) = rng_streams(1, seed)
    kap = 10.0 ** rng.uniform(-2.0, 2.0, size=(N, N, N))
    coeffs = []
    diag = np.zeros((N, N, N))
    for dz, dy, dx in _OFF7:
        nb = np.roll(kap, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
        face = 2.0 * kap * nb / (kap + nb)
        # faces on the domain boundary: Dirichlet at half a cell
        inside = np.ones((N, N, N), bool)
        for ax, d in zip((0, 1, 2), (dz, dy, dx)):
            if d == -1:
                sl = [slice(None)] * 3
                sl[ax] = 0
                inside[tuple(sl)] = False
            elif d == 1:
                sl = [slice(None)] * 3
                sl[ax] = N - 1
                inside[tuple(sl)] = False
        face = np.where(inside, face, 2.0 * kap)
        diag += face
        coeffs.append(-face)
    A = _stencil((N, N, N), _OFF7, coeffs, diag)
    A.meta = {"kind": "vardiff3d", "N": N, "seed": seed}
    return A


def convdiff2d(s: int, pe: float, theta: float) -> CSR:
    """First-order upwind -Laplace(u) + w . grad(u) on the unit square,
    s x s interior points, h = 1/(s+1), w = pe (cos theta, sin theta), rows
    scaled by h^2.  Diagonal 4 + h(|wx| + |wy|); the upwind neighbour in each
    direction gets -1 - h|w|, the downwind one -1.  Nonsymmetric M-matrix.
    """
    h = 1.0 / (s + 1)
    wx, wy = pe * np.cos(theta), pe * np.sin(theta)
    ax, ay = h * abs(wx), h * abs(wy)
    c_xm = -1.0 - (ax if wx > 0 else 0.0)
    c_xp = -1.0 - (ax if wx < 0 else 0.0)
    c_ym = -1.0 - (ay if wy > 0 else 0.0)
    c_yp = -1.0 - (ay if wy < 0 else 0.0)
    A = _stencil((1, s, s), [(0, -1, 0), (0, 0, -1), (0, 0, 1), (0, 1, 0)], [c_ym, c_xm, c_xp, c_yp], 4.0 + ax + ay)
    A.meta = {"kind": "convdiff2d", "s": s, "pe": pe, "theta": theta}
    return A


def convdiff_batch(nsys: int = 512, seed: int = MASTER_SEED, smin: int = 16, smax: int = 256, nrhs: int = 4):
    """Batch of independent convection-diffusion systems of uneven sizes.

    Grid sides s_i ~ U{smin..smax}, Peclet number ~ U(0, 50), flow angle
    ~ U(0, 2 pi), and nrhs right-hand sides per system ~ N(0, 1).
    Returns (list of CSR, list of (n_i, nrhs) arrays).
    """
    r_side, r_pe, r_th, r_b = rng_streams(4, seed)
    sides = r_side.integers(smin, smax + 1, size=nsys)
    pes = r_pe.uniform(0.0, 50.0, size=nsys)
    ths = r_th.uniform(0.0, 2 * np.pi, size=nsys)
    mats, rhs = [], []
    for s, pe, th in zip(sides, pes, ths):
        A = convdiff2d(int(s), float(pe), float(th))
        mats.append(A)
        rhs.append(r_b.standard_normal((A.n, nrhs)))
    return mats, rhs


# ---------------------------------------------------------------- elasticity

def _q1_reference(h: float):
    """Element matrices K_lambda, K_mu (24 x 24) of a trilinear cube of side h,
    2x2x2 Gauss quadrature, dof order (node a, component c) -> 3a + c with
    local node a = ax + 2 ay + 4 az.  K_e = lambda K_lambda + mu K_mu."""
    g = 1.0 / np.sqrt(3.0)
    signs = np.array([[2 * (a & 1) - 1, 2 * ((a >> 1) & 1) - 1, 2 * ((a >> 2) & 1) - 1] for a in range(8)], float)
    Cl = np.zeros((6, 6))
    Cl[:3, :3] = 1.0
    Cm = np.diag([2.0, 2.0, 2.0, 1.0, 1.0, 1.0])
    Kl = np.zeros((24, 24))
    Km = np.zeros((24, 24))
    detJ = (h / 2.0) ** 3
    for xi in (-g, g):
        for eta in (-g, g):
            for zeta in (-g, g):
                p = np.array([xi, eta, zeta])
                f = 1.0 + signs * p  # (8, 3) factors
                dN = np.empty((8, 3))
                dN[:, 0] = signs[:, 0] * f[:, 1] * f[:, 2] / 8.0
                dN[:, 1] = signs[:, 1] * f[:, 0] * f[:, 2] / 8.0
                dN[:, 2] = signs[:, 2] * f[:, 0] * f[:, 1] / 8.0
                dN *= 2.0 / h
                B = np.zeros((6, 24))
                for a in range(8):
                    dx, dy, dz = dN[a]
                    B[0, 3 * a] = dx
                    B[1, 3 * a + 1] = dy
                    B[2, 3 * a + 2] = dz
                    B[3, 3 * a] = dy
                    B[3, 3 * a + 1] = dx
                    B[4, 3 * a + 1] = dz
                    B[4, 3 * a + 2] = dy
                    B[5, 3 * a] = dz
                    B[5, 3 * a + 2] = dx
                Kl += B.T @ Cl @ B * detJ
                Km += B.T @ Cm @ B * detJ
    return Kl, Km


def elasticity_q1(Nx: int = 64, Ny: int = 64, Nz: int = 64, seed: int = MASTER_SEED) -> CSR:
    """Linear elasticity with trilinear hexahedra, 3 dof per node.

    Node grid Nx x Ny x (Nz+1), element size h = 1/Nx; the z = 0 node layer is
    Dirichlet-eliminated, leaving Nx*Ny*Nz free nodes (3 dof each, node-major
    dof order, nodes in natural order).  Per element, Young's modulus is
    log-uniform over [1, 100] and Poisson's ratio uniform over [0.2, 0.45]
    (isotropic material).  Every node pair that shares an element couples with
    a full 3x3 block; explicit zeros are kept so that the pattern is the
    structural 27-point one.
    """
    r_E, r_nu = rng_streams(2, seed)
    h = 1.0 / Nx
    ex_n, ey_n, ez_n = Nx - 1, Ny - 1, Nz
    ne = ex_n * ey_n * ez_n
    E = 10.0 ** r_E.uniform(0.0, 2.0, size=ne)
    nu = r_nu.uniform(0.2, 0.45, size=ne)
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    Kl, Km = _q1_reference(h)
    ez, ey, ex = np.meshgrid(np.arange(ez_n), np.arange(ey_n), np.arange(ex_n), indexing="ij")
    ez, ey, ex = ez.ravel(), ey.ravel(), ex.ravel()
    nnode = Nx * Ny * Nz
    Kb = np.zeros((nnode, 27, 3, 3))
    for a in range(8):
        ax, ay, az = a & 1, (a >> 1) & 1, (a >> 2) & 1
        gz = ez + az  # node-grid z of the row node (0 is eliminated)
        rfree = gz >= 1
        rnode = ((gz - 1) * Ny + (ey + ay)) * Nx + (ex + ax)
        for b in range(8):
            bx, by, bz = b & 1, (b >> 1) & 1, (b >> 2) & 1
            cfree = (ez + bz) >= 1
            m = rfree & cfree
            slot = ((bz - az) + 1) * 9 + ((by - ay) + 1) * 3 + ((bx - ax) + 1)
            blk = lam[m, None, None] * Kl[3 * a:3 * a + 3, 3 * b:3 * b + 3] + mu[m, None, None] * Km[3 * a:3 * a + 3, 3 * b:3 * b + 3]
            # rnode is injective over elements for a fixed local node a: no index collisions
            Kb[rnode[m], slot] += blk
    # structural pattern: neighbour node inside the free-node grid
    zz, yy, xx = np.meshgrid(np.arange(Nz), np.arange(Ny), np.arange(Nx), indexing="ij")
    zz, yy, xx = zz.ravel(), yy.ravel(), xx.ravel()
    node = np.arange(nnode, dtype=np.int64)
    slot_ok = np.empty((nnode, 27), bool)
    slot_col = np.empty((nnode, 27), np.int64)
    for s in range(27):
        dz, dy, dx = s // 9 - 1, (s // 3) % 3 - 1, s % 3 - 1
        slot_ok[:, s] = (zz + dz >= 0) & (zz + dz < Nz) & (yy + dy >= 0) & (yy + dy < Ny) & (xx + dx >= 0) & (xx + dx < Nx)
        slot_col[:, s] = node + (dz * Ny + dy) * Nx + dx
    # rows (node, c): columns 3*m + c' over valid slots (slot order = column order)
    cols = (3 * slot_col[:, None, :, None] + np.arange(3)[None, None, None, :])  # (nnode,1,27,3)
    cols = np.broadcast_to(cols, (nnode, 3, 27, 3)).reshape(3 * nnode, 81)
    vals = Kb.transpose(0, 2, 1, 3).reshape(3 * nnode, 81)
    mask = np.broadcast_to(slot_ok[:, None, :, None], (nnode, 3, 27, 3)).reshape(3 * nnode, 81)
    A = _from_dense_rows(cols, vals, mask)
    A.meta = {"kind": "elasticity_q1", "Nx": Nx, "Ny": Ny, "Nz": Nz, "seed": seed}
    return A


# ---------------------------------------------------------------- random tests

def random_sparse(n: int, seed: int, avg_offdiag: float = 6.0, long_rows: int = 0, long_len: int = 100,
                  diag_only_rows: int = 0, dominance: float = 1.5, neg_diag_rows: int = 0,
                  symmetric_pattern: bool = False) -> CSR:
    """Random nonsymmetric, diagonally dominant test matrix.

    Off-diagonal count per row ~ Poisson(avg_offdiag); `long_rows` rows get
    `long_len` off-diagonals (to exercise rows longer than a wavefront);
    `diag_only_rows` rows keep only their diagonal; `neg_diag_rows` rows get a
    negative diagonal.  |a_ii| = dominance * sum_j |a_ij| (or 1 if empty).
    """
    (rng,) = rng_streams(1, seed)
    rows = []
    cnt = np.minimum(rng.poisson(avg_offdiag, size=n), n - 1)
    longs = rng.choice(n, size=min(long_rows, n), replace=False) if long_rows else np.array([], int)
    cnt[longs] = min(long_len, n - 1)
    donly = rng.choice(n, size=min(diag_only_rows, n), replace=False) if diag_only_rows else np.array([], int)
    cnt[donly] = 0
    for i in range(n):
        c = rng.choice(n - 1, size=cnt[i], replace=False)
        c = np.where(c >= i, c + 1, c)
        rows.append(np.sort(c))
    if symmetric_pattern:
        import scipy.sparse as sp

        P = sp.lil_matrix((n, n), dtype=bool)
        for i, c in enumerate(rows):
            P[i, c] = True
        P = (P + P.T).tocsr()
        rows = [P.indices[P.indptr[i]:P.indptr[i + 1]] for i in range(n)]
    rp = [0]
    ci, va = [], []
    negs = set(rng.choice(n, size=min(neg_diag_rows, n), replace=False).tolist()) if neg_diag_rows else set()
    for i, c in enumerate(rows):
        v = rng.uniform(-1.0, 1.0, size=len(c))
        d = dominance * np.abs(v).sum() if len(c) else 1.0
        d = -d if i in negs else d
        allc = np.concatenate([c, [i]])
        allv = np.concatenate([v, [d]])
        o = np.argsort(allc, kind="stable")
        ci.append(allc[o])
        va.append(allv[o])
        rp.append(rp[-1] + len(allc))
    A = CSR(n, np.array(rp, np.int32), np.concatenate(ci).astype(np.int32), np.concatenate(va).astype(np.float64))
    A.meta = {"kind": "random", "seed": seed}
    return A


def make_rhs(A: CSR, dist: str = "uniform", seed: int = MASTER_SEED):
    """Manufactured solution x_true (U(-1,1) or N(0,1)) and b = A x_true."""
    (rng,) = rng_streams(1, seed + 7919)
    if dist == "uniform":
        x = rng.uniform(-1.0, 1.0, size=A.n)
    else:
        x = rng.standard_normal(A.n)
    b = A.to_scipy() @ x
    return x, b


def config_problem(k: int, size: int | None = None, seed: int = MASTER_SEED) -> dict:
    """The five workload configurations (k = 1..5) at full size, or with a
    reduced grid side `size` for quick tests.

    1: 2D 5-point Poisson 64^2, x_true ~ U(-1,1), GMRES(30).
    2: 3D 7-point Laplacian 128^3, x_true ~ N(0,1), GMRES(50).
    3: Q1 elasticity 64^3 free nodes x 3 dof, x_true ~ N(0,1), GMRES(50).
    4: variable-coefficient diffusion 192^3, x_true ~ N(0,1), GMRES(50).
    5: 512 convection-diffusion systems (sides 16..256), 4 RHS each, GMRES(20).
    """
    if k == 1:
        A = poisson2d(size or 64)
        x, b = make_rhs(A, "uniform", seed)
        return {"A": A, "b": b, "x_true": x, "restart": 30, "rtol": 1e-8}
    if k == 2:
        A = laplace3d(size or 128)
        x, b = make_rhs(A, "normal", seed)
        return {"A": A, "b": b, "x_true": x, "restart": 50, "rtol": 1e-8}
    if k == 3:
        N = size or 64
        A = elasticity_q1(N, N, N, seed)
        x, b = make_rhs(A, "normal", seed)
        return {"A": A, "b": b, "x_true": x, "restart": 50, "rtol": 1e-8}
    if k == 4:
        A = vardiff3d(size or 192, seed)
        x, b = make_rhs(A, "normal", seed)
        return {"A": A, "b": b, "x_true": x, "restart": 50, "rtol": 1e-8}
    if k == 5:
        mats, rhs = convdiff_batch(size or 512, seed)
        return {"mats": mats, "rhs": rhs, "restart": 20, "rtol": 1e-8}
    raise ValueError(k)
