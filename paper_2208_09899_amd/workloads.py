"""Seeded synthetic inputs: sparse operators in CSR form and blocks of right-hand sides.

This module only builds inputs.  It holds none of the solver's arithmetic and
is shared by the GPU path, the tests and the benchmark, so that both sides of
every comparison see the very same arrays.

CSR convention used everywhere: ``row_ptr`` int64 (n+1), ``col_idx`` int32
(nnz, sorted within each row), ``values`` float64 (nnz).  Right-hand sides are
n x s float64, C-contiguous (row-major, the s entries of a row adjacent).

Operators (the problem ``A X = B`` with A large and sparse, B tall-skinny,
paper Sec. 2, eq. AX=B):

* ``tridiag_paper(n)``: the paper's ``tridiag`` test (Sec. 5.1): ones on the
  off-diagonals and -1, -2, ..., -n on the diagonal, with the two-column
  right-hand side [1/sqrt(n) * ones, (1..n)].
* ``laplace_1d(n)``: tridiag(-1, 2, -1).
* ``laplace_2d(N)``: 5-point Dirichlet Laplacian on an N x N grid (stencil
  4, -1 x 4, unscaled), x index fastest.
* ``laplace_3d(N)``: 7-point Dirichlet Laplacian on an N^3 grid.
* ``rgg_laplacian(n, seed)``: graph Laplacian of a random geometric graph in
  the unit square (expected degree 4, edge weights uniform in [0, 1)) plus a
  diagonal shift, rows ordered cell by cell for locality.
* ``convdiff_2d(N, peclet, theta)``: centred-difference -Lap(u) + w.grad(u) on
  the unit square, |w| = peclet, scaled by h^2.
* ``cyclic_shift(n)``: the permutation P e_i = e_{(i+1) mod n}.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSR:
    n: int
    row_ptr: np.ndarray   # int64 (n+1)
    col_idx: np.ndarray   # int32 (nnz)
    values: np.ndarray    # float64 (nnz)
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.values, self.col_idx, self.row_ptr), shape=(self.n, self.n))


def _from_scipy(M, name: str) -> CSR:
    M = sp.csr_matrix(M)
    M.sum_duplicates()
    M.sort_indices()
    return CSR(n=M.shape[0],
               row_ptr=np.ascontiguousarray(M.indptr, dtype=np.int64),
               col_idx=np.ascontiguousarray(M.indices, dtype=np.int32),
               values=np.ascontiguousarray(M.data, dtype=np.float64),
               name=name)


def _tri(n: int, lo: float, d, up: float):
    diag = np.broadcast_to(np.asarray(d, dtype=np.float64), (n,))
    return sp.diags([np.full(n - 1, lo), diag, np.full(n - 1, up)], [-1, 0, 1], format="csr")


def laplace_1d(n: int) -> CSR:
    return _from_scipy(_tri(n, -1.0, 2.0, -1.0), f"laplace1d_n{n}")


def tridiag_paper(n: int) -> tuple[CSR, np.ndarray]:
    """The paper's ``tridiag`` operator and its two-column right-hand side."""
    A = _tri(n, 1.0, -np.arange(1, n + 1, dtype=np.float64), 1.0)
    B = np.empty((n, 2), dtype=np.float64)
    B[:, 0] = 1.0 / math.sqrt(n)
    B[:, 1] = np.arange(1, n + 1, dtype=np.float64)
    return _from_scipy(A, f"tridiag_paper_n{n}"), B


def laplace_2d(N: int) -> CSR:
    T = _tri(N, -1.0, 2.0, -1.0)
    I = sp.identity(N, format="csr")
    return _from_scipy(sp.kron(I, T) + sp.kron(T, I), f"laplace2d_{N}x{N}")


def laplace_3d(N: int) -> CSR:
    T = _tri(N, -1.0, 2.0, -1.0)
    I = sp.identity(N, format="csr")
    A = sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I)
    return _from_scipy(A, f"laplace3d_{N}^3")


def convdiff_2d(N: int, peclet: float, theta: float) -> CSR:
    """-Lap(u) + w.grad(u) on (0,1)^2 with Dirichlet boundary, h = 1/(N+1),
    w = peclet * (cos theta, sin theta), centred differences, times h^2:
    centre 4, east/west -1 +/- h*w_x/2, north/south -1 +/- h*w_y/2."""
    h = 1.0 / (N + 1)
    wx, wy = peclet * math.cos(theta), peclet * math.sin(theta)
    Tx = _tri(N, -1.0 - 0.5 * h * wx, 2.0, -1.0 + 0.5 * h * wx)
    Ty = _tri(N, -1.0 - 0.5 * h * wy, 2.0, -1.0 + 0.5 * h * wy)
    I = sp.identity(N, format="csr")
    return _from_scipy(sp.kron(I, Tx) + sp.kron(Ty, I), f"convdiff_{N}_pe{peclet:.3f}")


def rgg_laplacian(n: int, seed: int = 3, degree: float = 4.0, shift: float = 1e-6) -> CSR:
    """Random geometric graph Laplacian + shift * I.

    n points uniform in [0,1)^2; an edge joins two points closer than
    r = sqrt(degree / (pi n)) (expected degree ``degree``); each edge gets a
    weight uniform in [0,1).  Points are renumbered cell by cell (cells of
    side >= r, row-major over the cell grid) so that neighbours sit close in
    memory.  Built with a cell grid in O(n)."""
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    r = math.sqrt(degree / (math.pi * n))
    G = max(1, int(math.floor(1.0 / r)))
    cx = np.minimum((pts[:, 0] * G).astype(np.int64), G - 1)
    cy = np.minimum((pts[:, 1] * G).astype(np.int64), G - 1)
    cell = cx + G * cy
    order = np.argsort(cell, kind="stable")
    pts = pts[order]
    cell = cell[order]
    cx, cy = cx[order], cy[order]
    start = np.searchsorted(cell, np.arange(G * G + 1))
    idx = np.arange(n, dtype=np.int64)

    I_list, J_list = [], []
    # same cell: partners j > i inside the cell
    end_i = start[cell + 1]
    cnt = end_i - idx - 1
    tot = int(cnt.sum())
    if tot:
        ii = np.repeat(idx, cnt)
        base = np.repeat(np.cumsum(cnt) - cnt, cnt)
        jj = ii + 1 + (np.arange(tot) - base)
        I_list.append(ii); J_list.append(jj)
    # half of the neighbouring cells, so every pair is visited once
    for dx, dy in ((1, 0), (-1, 1), (0, 1), (1, 1)):
        nx, ny = cx + dx, cy + dy
        ok = (nx >= 0) & (nx < G) & (ny < G)
        nc = np.where(ok, nx + G * ny, 0)
        cnt = np.where(ok, start[nc + 1] - start[nc], 0)
        tot = int(cnt.sum())
        if not tot:
            continue
        ii = np.repeat(idx, cnt)
        base = np.repeat(np.cumsum(cnt) - cnt, cnt)
        jj = np.repeat(start[nc], cnt) + (np.arange(tot) - base)
        I_list.append(ii); J_list.append(jj)
    ii = np.concatenate(I_list); jj = np.concatenate(J_list)
    d = pts[ii] - pts[jj]
    keep = (d * d).sum(axis=1) < r * r
    ii, jj = ii[keep], jj[keep]
    w = rng.random(ii.shape[0])
    rows = np.concatenate([ii, jj, idx])
    cols = np.concatenate([jj, ii, idx])
    deg = np.bincount(ii, weights=w, minlength=n) + np.bincount(jj, weights=w, minlength=n)
    vals = np.concatenate([-w, -w, deg + shift])
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n, n))
    return _from_scipy(A, f"rgg_n{n}_deg{degree:g}_shift{shift:g}")


def cyclic_shift(n: int) -> CSR:
    """The cyclic shift P e_i = e_{(i + 1) mod n} (a permutation matrix)."""
    rows = (np.arange(n) + 1) % n
    M = sp.csr_matrix((np.ones(n), (rows, np.arange(n))), shape=(n, n))
    return _from_scipy(M, f"cyclic_shift_n{n}")


def rhs(n: int, s: int, seed: int) -> np.ndarray:
    """n x s block with i.i.d. N(0,1) entries from PCG64 seeded with ``seed``."""
    return np.ascontiguousarray(np.random.default_rng(seed).standard_normal((n, s)))


def random_dense_operator(n: int, seed: int, kind: str = "spd") -> CSR:
    """Small dense test operators stored as CSR (for the dense-LU checks).

    ``spd``: Q diag(lambda) Q^T with lambda log-spaced in [1, 1e2].
    ``nonsym``: I * (2 + n^0.5) + G, G i.i.d. N(0,1) (eigenvalues well inside the right half-plane).
    """
    rng = np.random.default_rng(seed)
    if kind == "spd":
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        lam = np.logspace(0, 2, n)
        M = (Q * lam) @ Q.T
        M = 0.5 * (M + M.T)
    elif kind == "nonsym":
        M = rng.standard_normal((n, n)) + (2.0 + math.sqrt(n)) * np.eye(n)
    else:
        raise ValueError(kind)
    return _from_scipy(sp.csr_matrix(M), f"dense_{kind}_n{n}_seed{seed}")


# --------------------------------------------------------------------------------------
# Named workloads.  Each names an operator, a block of right-hand sides and solver
# parameters; sizes follow the five benchmark configurations of this project.
# --------------------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    A: CSR
    B: np.ndarray
    m: int
    tol: float
    max_cycles: int
    methods: tuple
    skeletons: tuple
    note: str = ""


def workload(name: str, scale: int | None = None) -> Workload:
    """Build a named workload.  ``scale`` shrinks the grid / node count for the
    small-size parity cases (same construction, fewer unknowns)."""
    if name == "tridiag1000":
        n = scale or 1000
        return Workload(name, laplace_1d(n), rhs(n, 4, 1), m=20, tol=1e-8, max_cycles=50,
                        methods=("gmres",), skeletons=("bcgsi_ls",),
                        note="tridiag(-1,2,-1), s=4, m=20, tol 1e-8, <=50 cycles")
    if name == "laplace2d":
        N = scale or 256
        return Workload(name, laplace_2d(N), rhs(N * N, 8, 2), m=30, tol=1e-8, max_cycles=100000,
                        methods=("fom", "gmres"), skeletons=("bcgsi_ls", "bmgs_cwy", "bmgs_icwy"),
                        note=f"2-D 5-point Laplacian {N}x{N}, s=8, m=30, tol 1e-8")
    if name == "rgg":
        n = scale or (1 << 20)
        return Workload(name, rgg_laplacian(n, seed=3), rhs(n, 16, 4), m=25, tol=1e-8,
                        max_cycles=100000, methods=("gmres",), skeletons=("bcgsi_ls",),
                        note=f"RGG Laplacian n={n} + 1e-6 I, s=16, m=25, tol 1e-8")
    if name == "convdiff2d":
        N = scale or 256
        return Workload(name, convdiff_2d(N, 10.0, 0.3), rhs(N * N, 5, 7), m=10, tol=1e-8,
                        max_cycles=100000, methods=("gmres",), skeletons=("bcgsi_ls",),
                        note=f"2-D convection-diffusion {N}x{N}, Peclet 10, s=5, m=10, tol 1e-8")
    if name == "laplace3d":
        N = scale or 128
        return Workload(name, laplace_3d(N), rhs(N ** 3, 32, 5), m=20, tol=1e-10,
                        max_cycles=100000, methods=("gmres",), skeletons=("bcgsi_ls",),
                        note=f"3-D 7-point Laplacian {N}^3, s=32, m=20, tol 1e-10")
    raise KeyError(name)


@dataclasses.dataclass
class Request:
    idx: int
    arrival: float     # seconds after stream start
    N: int
    peclet: float
    theta: float
    s: int
    seed: int


def serving_stream(count: int = 512, rate: float = 50.0, seed: int = 6,
                   side_lo: int = 64, side_hi: int = 512) -> list[Request]:
    """Poisson stream of convection-diffusion solves: grid side uniform in
    [side_lo, side_hi], Peclet uniform in [0,10], wind angle uniform in
    [0, 2 pi), s uniform in {1,4,8,16}, exponential inter-arrival times at
    ``rate`` requests per second.  Each request's RHS uses seed ``seed*100003 + idx``."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for i in range(count):
        N = int(rng.integers(side_lo, side_hi + 1))
        pe = float(rng.uniform(0.0, 10.0))
        th = float(rng.uniform(0.0, 2 * math.pi))
        s = int(rng.choice([1, 4, 8, 16]))
        out.append(Request(i, float(t[i]), N, pe, th, s, seed * 100003 + i))
    return out


def request_problem(req: Request) -> tuple[CSR, np.ndarray]:
    A = convdiff_2d(req.N, req.peclet, req.theta)
    return A, rhs(A.n, req.s, req.seed)
