"""Seeded synthetic linear systems A u = f (CSR, int32 indices, float64 values).

This module defines *inputs only*: it holds none of the solver's arithmetic, so
both the HIP path and the CPU oracle may use it.  The paper's own test matrices
(finite-element matrices from a scalar convection-diffusion-reaction equation,
Section 4.1, Table 1; SuiteSparse matrices, Section 4.6, Table 3) are not
available, so grid operators of the same size class (10^6..10^7 rows, about 7
nonzeros per row like the P1 family of Table 1) stand in for them.

Conventions shared by every generator:
  * unknowns are the interior cells/nodes of a box, ordered lexicographically
    with x fastest: index = x + nx*(y + ny*z);
  * Dirichlet boundary values are eliminated (boundary neighbours drop out of a
    row; the diagonal keeps its full value);
  * every row stores its diagonal, columns are strictly ascending;
  * the pattern is structurally symmetric.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class CSR:
    """Host CSR matrix: row_ptr int32[n+1], col int32[nnz], val float64[nnz]."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def astype32(self) -> "CSR":
        return CSR(self.n, self.row_ptr, self.col, self.val.astype(np.float32))


def _assemble(shape, offsets, coef):
    """Build a CSR matrix from a stencil on an interior grid.

    shape   -- (nx, ny, nz) grid size, x fastest.
    offsets -- list of (dx, dy, dz) neighbour offsets, (0,0,0) is the diagonal.
    coef    -- callable(k) -> float64 array of shape (nz, ny, nx) with the
               coefficient of offset k for every row (ignored where the
               neighbour lies outside the box).
    """
    nx, ny, nz = shape
    n = nx * ny * nz
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    # sort the offsets by linear displacement so each row's columns ascend
    lin = [dx + nx * (dy + ny * dz) for (dx, dy, dz) in offsets]
    order = np.argsort(lin, kind="stable")
    cols, vals, masks = [], [], []
    idx = (x + nx * (y + ny * z)).astype(np.int64)
    for k in order:
        dx, dy, dz = offsets[k]
        ok = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < ny) & (z + dz >= 0) & (z + dz < nz)
        cols.append((idx + lin[k]).reshape(-1))
        vals.append(np.broadcast_to(coef(k), (nz, ny, nx)).reshape(-1).astype(np.float64))
        masks.append(ok.reshape(-1))
    cols = np.stack(cols, axis=1)
    vals = np.stack(vals, axis=1)
    masks = np.stack(masks, axis=1)
    counts = masks.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 index range")
    return CSR(n, row_ptr.astype(np.int32), cols[masks].astype(np.int32), vals[masks].copy())


_OFF2 = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0)]
_OFF3 = _OFF2 + [(0, 0, -1), (0, 0, 1)]


def poisson2d(n: int, m: int | None = None) -> CSR:
    """5-point Laplacian on an n x m interior grid: diagonal 4, neighbours -1."""
    m = n if m is None else m
    return _assemble((n, m, 1), _OFF2, lambda k: 4.0 if k == 0 else -1.0)


def poisson3d(n: int, m: int | None = None, p: int | None = None) -> CSR:
    """7-point Laplacian on an n x m x p interior grid: diagonal 6, neighbours -1."""
    m = n if m is None else m
    p = n if p is None else p
    return _assemble((n, m, p), _OFF3, lambda k: 6.0 if k == 0 else -1.0)


def convdiff3d(n: int, velocity=(1.0, 0.5, 0.25), peclet: float = 10.0) -> CSR:
    """First-order upwind convection-diffusion, -eps*Lap(u) + b.grad(u), on n^3.

    The cell Peclet number is Pe = max|b| h / eps.  Rows are scaled by h^2/eps:
    diagonal 6 + sum_d Pe*b_d/max|b|, upwind neighbour -1 - Pe*b_d/max|b|,
    downwind neighbour -1 (velocity components must be >= 0).
    """
    bmax = max(abs(c) for c in velocity)
    c = [peclet * v / bmax for v in velocity]
    if min(c) < 0:
        raise ValueError("velocity components must be non-negative")
    diag = 6.0 + sum(c)
    table = {0: diag, 1: -1.0 - c[0], 2: -1.0, 3: -1.0 - c[1], 4: -1.0, 5: -1.0 - c[2], 6: -1.0}
    return _assemble((n, n, n), _OFF3, lambda k: table[k])


def diffusion_fv3d(tx: np.ndarray, ty: np.ndarray, tz: np.ndarray) -> CSR:
    """7-point finite-volume diffusion from face transmissibilities.

    tx has shape (nz, ny, nx+1): tx[z, y, i] is the face between cells i-1 and
    i along x, with i = 0 and i = nx the two boundary faces (Dirichlet u = 0).
    ty is (nz, ny+1, nx) and tz is (nz+1, ny, nx) likewise.  Row c gets
    a_cc = sum of its six face values and a_cd = -T_f for each interior face f
    between c and d.  The result is symmetric positive definite.
    """
    nz, ny, nxp = tx.shape
    nx = nxp - 1
    assert ty.shape == (nz, ny + 1, nx) and tz.shape == (nz + 1, ny, nx)
    diag = tx[:, :, :-1] + tx[:, :, 1:] + ty[:, :-1, :] + ty[:, 1:, :] + tz[:-1] + tz[1:]
    per = {
        0: diag,
        1: -tx[:, :, :-1],  # west face of the cell
        2: -tx[:, :, 1:],  # east
        3: -ty[:, :-1, :],  # south
        4: -ty[:, 1:, :],  # north
        5: -tz[:-1],  # down
        6: -tz[1:],  # up
    }
    return _assemble((nx, ny, nz), _OFF3, lambda k: per[k])


def gaussian_field(n: int, seed: int, std: float = 1.5, corr_len: float = 8.0) -> np.ndarray:
    """Stationary Gaussian field on an n^3 periodic grid, shape (n, n, n) [z,y,x].

    White noise is smoothed with a Gaussian kernel of width corr_len/sqrt(2),
    which gives the squared-exponential correlation exp(-r^2 / (2 corr_len^2)),
    and is then rescaled to zero mean and the requested standard deviation.
    """
    from scipy.ndimage import gaussian_filter

    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    g = gaussian_filter(w, sigma=corr_len / math.sqrt(2.0), mode="wrap")
    g -= g.mean()
    g *= std / g.std()
    return g


def vardiff3d(n: int, seed: int = 0, std: float = 1.5, corr_len: float = 8.0) -> CSR:
    """Variable-coefficient diffusion on n^3 cells, coefficient k = exp(g).

    Interior face value: exp((g_L + g_R)/2); a boundary face sits half a cell
    from the Dirichlet wall, so its value is 2*exp(g_cell).
    """
    g = gaussian_field(n, seed, std, corr_len)
    e = np.exp(g)
    tx = np.empty((n, n, n + 1))
    tx[:, :, 1:-1] = np.exp(0.5 * (g[:, :, :-1] + g[:, :, 1:]))
    tx[:, :, 0] = 2.0 * e[:, :, 0]
    tx[:, :, -1] = 2.0 * e[:, :, -1]
    ty = np.empty((n, n + 1, n))
    ty[:, 1:-1, :] = np.exp(0.5 * (g[:, :-1, :] + g[:, 1:, :]))
    ty[:, 0, :] = 2.0 * e[:, 0, :]
    ty[:, -1, :] = 2.0 * e[:, -1, :]
    tz = np.empty((n + 1, n, n))
    tz[1:-1] = np.exp(0.5 * (g[:-1] + g[1:]))
    tz[0] = 2.0 * e[0]
    tz[-1] = 2.0 * e[-1]
    return diffusion_fv3d(tx, ty, tz)


def lognormal_diffusion3d(n: int, seed: int, sigma: float = 1.0) -> CSR:
    """Diffusion on n^3 cells with iid lognormal face values exp(xi), xi ~ N(0, sigma^2).

    Boundary faces get 2*exp(xi) (half-cell distance to the wall).
    """
    rng = np.random.default_rng(seed)
    tx = np.exp(sigma * rng.standard_normal((n, n, n + 1)))
    ty = np.exp(sigma * rng.standard_normal((n, n + 1, n)))
    tz = np.exp(sigma * rng.standard_normal((n + 1, n, n)))
    tx[:, :, 0] *= 2.0
    tx[:, :, -1] *= 2.0
    ty[:, 0, :] *= 2.0
    ty[:, -1, :] *= 2.0
    tz[0] *= 2.0
    tz[-1] *= 2.0
    return diffusion_fv3d(tx, ty, tz)


def rhs_uniform(n: int, seed: int) -> np.ndarray:
    """Right-hand side with iid entries uniform on [-1, 1] (PCG64 stream of `seed`)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, n)


def random_symmetric_pattern(n: int, density: float, seed: int, weights=(1, 2, 3), nonsym_values=False,
                             explicit_zeros: float = 0.0) -> CSR:
    """Random structurally symmetric matrix with small integer weights (many ties).

    Off-diagonal magnitudes are drawn from `weights`, signs at random; the
    diagonal dominates (sum of |off-diagonal| + 1) so it is non-singular.  With
    nonsym_values the two mirror entries get independent values.  A fraction
    `explicit_zeros` of off-diagonal entries is stored as 0.0.
    """
    rng = np.random.default_rng(seed)
    upper = np.triu(rng.random((n, n)) < density, 1)
    mask = upper | upper.T
    vals = np.zeros((n, n))
    w = np.asarray(weights, dtype=np.float64)
    a = rng.choice(w, size=(n, n)) * rng.choice([-1.0, 1.0], size=(n, n))
    if nonsym_values:
        vals[mask] = a[mask]
    else:
        au = np.triu(a, 1)
        vals = au + au.T
        vals[~mask] = 0.0
    if explicit_zeros > 0:
        z = np.triu(rng.random((n, n)) < explicit_zeros, 1) & upper
        vals[z] = 0.0
        if not nonsym_values:
            vals[z.T] = 0.0
    np.fill_diagonal(vals, np.abs(vals).sum(axis=1) + 1.0)
    mask = mask | np.eye(n, dtype=bool)
    rows, cols = np.nonzero(mask)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return CSR(n, row_ptr, cols.astype(np.int32), vals[rows, cols].astype(np.float64))


def star_graph(n: int, seed: int) -> CSR:
    """Symmetric matrix whose graph is a star: row 0 is coupled to every other
    row, which are coupled to nothing else.  Off-diagonal weights -1, -2 or -3
    at random, diagonal sum of |off-diagonal| + 1.  Pairwise matching merges
    only one leaf with the hub per pass, so coarsening makes almost no progress
    (the shape high-contrast coefficients give coarse levels)."""
    rng = np.random.default_rng(seed)
    w = -rng.choice(np.array([1.0, 2.0, 3.0]), size=n - 1)
    a = np.zeros((n, n))
    a[0, 1:] = w
    a[1:, 0] = w
    np.fill_diagonal(a, np.abs(a).sum(axis=1) + 1.0)
    return from_dense(a)


def from_dense(a: np.ndarray) -> CSR:
    """CSR of the nonzero pattern of a dense square matrix plus its diagonal."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    mask = (a != 0) | np.eye(n, dtype=bool)
    rows, cols = np.nonzero(mask)
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(np.bincount(rows, minlength=n), out=row_ptr[1:])
    return CSR(n, row_ptr, cols.astype(np.int32), a[rows, cols].copy())


def diagonal(d) -> CSR:
    """Diagonal matrix: no off-diagonal couplings, so matching merges nothing."""
    d = np.asarray(d, dtype=np.float64)
    n = d.size
    return CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d.copy())


def block_diag(*mats: CSR) -> CSR:
    """Block-diagonal matrix of the given blocks, in order (columns shifted)."""
    rps, cols, vals, r0, e0 = [np.zeros(1, dtype=np.int64)], [], [], 0, 0
    for m in mats:
        rps.append(np.asarray(m.row_ptr[1:], dtype=np.int64) + e0)
        cols.append(np.asarray(m.col, dtype=np.int64) + r0)
        vals.append(np.asarray(m.val, dtype=np.float64))
        r0 += m.n
        e0 += m.nnz
    return CSR(r0, np.concatenate(rps).astype(np.int32), np.concatenate(cols).astype(np.int32),
               np.concatenate(vals))


# ---------------------------------------------------------------------------
# Named workloads (sizes of the paper-scale synthetic configurations)
# ---------------------------------------------------------------------------

WORKLOADS = {
    "poisson2d_64": dict(kind="pcg", rtol=1e-8, precond="fp64", desc="2D 5-point Poisson, 64x64 interior (N=4096)"),
    "poisson3d_128": dict(kind="pcg", rtol=1e-10, precond="fp64", desc="3D 7-point Poisson, 128^3 (N=2,097,152)"),
    "vardiff3d_160": dict(kind="pcg", rtol=1e-8, precond="fp32", desc="3D variable-coefficient FV diffusion, 160^3"),
    "convdiff3d_96": dict(kind="bicgstab", rtol=1e-8, precond="fp32",
                          desc="3D upwind convection-diffusion, 96^3, Pe=10"),
}


def make_workload(name: str, seed: int = 0):
    """Return (A, b, spec) for a named workload."""
    spec = WORKLOADS[name]
    if name == "poisson2d_64":
        a = poisson2d(64)
    elif name == "poisson3d_128":
        a = poisson3d(128)
    elif name == "vardiff3d_160":
        a = vardiff3d(160, seed=seed)
    elif name == "convdiff3d_96":
        a = convdiff3d(96)
    else:  # pragma: no cover
        raise KeyError(name)
    return a, rhs_uniform(a.n, seed), spec


def served_stream(count: int, seed: int = 0, side_min: int = 16, side_max: int = 96, sigma: float = 1.0):
    """Request sizes of a served stream: side n_i = round(exp(U(ln lo, ln hi))).

    Returns a list of (side, request_seed) pairs; request i uses seed 1000 + i
    for both its coefficients and its right-hand side.
    """
    rng = np.random.default_rng(seed)
    sides = np.rint(np.exp(rng.uniform(math.log(side_min), math.log(side_max), count))).astype(int)
    return [(int(s), 1000 + i) for i, s in enumerate(sides)]
