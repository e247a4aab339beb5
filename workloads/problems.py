"""Problem generators: finite-difference matrices, partitions, right-hand sides.

See the package docstring for the grid conventions.  Everything here is
deterministic given its arguments (seeded with numpy's default_rng).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSR:
    """Compressed sparse rows with int64 row pointers, int32 sorted columns,
    FP64 values (complex128 for the complex families)."""

    n: int
    indptr: np.ndarray   # int64[n+1]
    indices: np.ndarray  # int32[nnz]
    data: np.ndarray     # float64[nnz] or complex128[nnz]

    @property
    def nnz(self) -> int:
        return int(self.indptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.data, self.indices, self.indptr), shape=(self.n, self.n))

    @staticmethod
    def from_scipy(M) -> "CSR":
        M = sp.csr_matrix(M)
        M.eliminate_zeros()
        M.sort_indices()
        dt = np.complex128 if np.iscomplexobj(M.data) else np.float64
        return CSR(M.shape[0], M.indptr.astype(np.int64), M.indices.astype(np.int32),
                   M.data.astype(dt))


def _assemble(n: int, entries) -> CSR:
    """entries: list of (row_idx, col_idx, values) arrays; zeros are dropped."""
    r = np.concatenate([e[0] for e in entries])
    c = np.concatenate([e[1] for e in entries])
    v = np.concatenate([e[2] for e in entries])
    keep = v != 0.0
    M = sp.csr_matrix((v[keep], (r[keep], c[keep])), shape=(n, n))
    M.sum_duplicates()
    return CSR.from_scipy(M)


def _grid2(m):
    j, i = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    return i.ravel(), j.ravel()


def _grid3(m):
    k, j, i = np.meshgrid(np.arange(m), np.arange(m), np.arange(m), indexing="ij")
    return i.ravel(), j.ravel(), k.ravel()


# ---------------------------------------------------------------------------
# Operators
# ---------------------------------------------------------------------------

def laplace2d(m: int) -> CSR:
    """5-point Laplacian [4, -1 x4] on an m x m interior grid (rows scaled by h^2)."""
    return convdiff2d(m, nu=1.0, velocity=None)


def convdiff2d(m: int, nu: float, velocity="cos-sin", neumann_x: bool = False) -> CSR:
    """-nu*Lap(u) + V.grad(u), first-order upwind, 5 points, rows scaled by h^2.

    velocity: None (pure diffusion) or "cos-sin": V(x, y) = (cos 2 pi y, sin 2 pi x)
    evaluated at the nodes.  Off-diagonals are -nu - h*max(+-V, 0), so every
    interior row sums to zero and the matrix is a nonsymmetric M-matrix.
    neumann_x: the rows at x = 0 and x = 1 drop the missing coupling from the
    diagonal (they sum to zero too), so a subdomain away from y = 0 and y = 1
    floats.
    """
    n = m * m
    h = 1.0 / (m + 1)
    i, j = _grid2(m)
    idx = i + m * j
    if velocity is None:
        vx = np.zeros(n)
        vy = np.zeros(n)
    elif velocity == "cos-sin":
        x = (i + 1) * h
        y = (j + 1) * h
        vx = np.cos(2 * np.pi * y)
        vy = np.sin(2 * np.pi * x)
    else:
        raise ValueError(velocity)
    diag = 4.0 * nu + h * (np.abs(vx) + np.abs(vy))
    west = -nu - h * np.maximum(vx, 0.0)
    east = -nu - h * np.maximum(-vx, 0.0)
    south = -nu - h * np.maximum(vy, 0.0)
    north = -nu - h * np.maximum(-vy, 0.0)
    if neumann_x:
        diag = diag + np.where(i == 0, west, 0.0) + np.where(i == m - 1, east, 0.0)
    ent = [(idx, idx, diag)]
    mk = i > 0
    ent.append((idx[mk], idx[mk] - 1, west[mk]))
    mk = i < m - 1
    ent.append((idx[mk], idx[mk] + 1, east[mk]))
    mk = j > 0
    ent.append((idx[mk], idx[mk] - m, south[mk]))
    mk = j < m - 1
    ent.append((idx[mk], idx[mk] + m, north[mk]))
    return _assemble(n, ent)


def convdiff2d_central(m: int, nu: float) -> CSR:
    """-nu*Lap(u) + V.grad(u) with central differences for the convection,
    V = (cos 2 pi y, sin 2 pi x), rows scaled by h^2: off-diagonals
    -nu -+ (h/2) V.  Where the cell Peclet number h|V|/(2 nu) exceeds 1 some
    off-diagonals are positive: a nonsymmetric matrix that is not an
    M-matrix (interior rows still sum to zero)."""
    n = m * m
    h = 1.0 / (m + 1)
    i, j = _grid2(m)
    idx = i + m * j
    x = (i + 1) * h
    y = (j + 1) * h
    vx = np.cos(2 * np.pi * y)
    vy = np.sin(2 * np.pi * x)
    diag = np.full(n, 4.0 * nu)
    west = -nu - 0.5 * h * vx
    east = -nu + 0.5 * h * vx
    south = -nu - 0.5 * h * vy
    north = -nu + 0.5 * h * vy
    ent = [(idx, idx, diag)]
    mk = i > 0
    ent.append((idx[mk], idx[mk] - 1, west[mk]))
    mk = i < m - 1
    ent.append((idx[mk], idx[mk] + 1, east[mk]))
    mk = j > 0
    ent.append((idx[mk], idx[mk] - m, south[mk]))
    mk = j < m - 1
    ent.append((idx[mk], idx[mk] + m, north[mk]))
    return _assemble(n, ent)


def convdiff2d_complex(m: int, nu: float, eta: float = 0.0, omega: float = 0.0,
                       phase_seed=None, eta_y=None, neumann_x: bool = False) -> CSR:
    """Frequency-domain convection-diffusion -nu ((1 + i eta) d_xx + (1 + i
    eta_y) d_yy) u + V.grad(u) + i omega u (eta_y defaults to eta), first-order
    upwind with V = (cos 2 pi y, sin 2 pi x), rows scaled by h^2: x-couplings
    -nu (1 + i eta) - h max(+-Vx, 0), y-couplings likewise with eta_y, the
    diagonal minus their sum plus i omega h^2.  Interior rows sum to
    i omega h^2 (to zero when omega = 0; with eta_y = 0 the y-couplings are
    real and negative, and with neumann_x the rows at x = 0 and x = 1 drop
    the missing coupling from the diagonal, so the strips that do not touch
    y = 0 or y = 1 float).  phase_seed
    applies the unitary change of variables diag(exp(i theta)) A
    diag(exp(-i theta)), theta uniform in [0, 2 pi) from that seed, which
    keeps every modulus and makes each off-diagonal entry genuinely complex
    (use it with omega > 0: it moves the null vector of a floating splitting
    off the constant)."""
    n = m * m
    h = 1.0 / (m + 1)
    i, j = _grid2(m)
    idx = i + m * j
    x = (i + 1) * h
    y = (j + 1) * h
    vx = np.cos(2 * np.pi * y)
    vy = np.sin(2 * np.pi * x)
    dx = nu * (1.0 + 1j * eta)
    dy = nu * (1.0 + 1j * (eta if eta_y is None else eta_y))
    diag = 2.0 * dx + 2.0 * dy + h * (np.abs(vx) + np.abs(vy)) + 1j * omega * h * h
    west = -dx - h * np.maximum(vx, 0.0)
    east = -dx - h * np.maximum(-vx, 0.0)
    south = -dy - h * np.maximum(vy, 0.0)
    north = -dy - h * np.maximum(-vy, 0.0)
    if neumann_x:
        diag = diag + np.where(i == 0, west, 0.0) + np.where(i == m - 1, east, 0.0)
    ent = [(idx, idx, diag)]
    mk = i > 0
    ent.append((idx[mk], idx[mk] - 1, west[mk]))
    mk = i < m - 1
    ent.append((idx[mk], idx[mk] + 1, east[mk]))
    mk = j > 0
    ent.append((idx[mk], idx[mk] - m, south[mk]))
    mk = j < m - 1
    ent.append((idx[mk], idx[mk] + m, north[mk]))
    A = _assemble(n, ent)
    if phase_seed is not None:
        ph = np.exp(1j * np.random.default_rng(phase_seed).uniform(0.0, 2 * np.pi, n))
        rows = np.repeat(np.arange(n), np.diff(A.indptr))
        A.data = A.data * ph[rows] * np.conj(ph[A.indices])
    return A


def magnetic_laplace2d(m: int, flux: float, shift: float = 0.0) -> CSR:
    """Hermitian 5-point magnetic Laplacian (Landau gauge): diagonal 4 + shift,
    -1 on x-edges, -exp(+-2 pi i flux x) on y-edges (x of the lower node),
    rows scaled by h^2.  Hermitian positive definite and diagonally dominant
    for shift >= 0 (strictly on the boundary rows)."""
    n = m * m
    h = 1.0 / (m + 1)
    i, j = _grid2(m)
    idx = i + m * j
    ph = np.exp(2j * np.pi * flux * (i + 1) * h)
    ent = [(idx, idx, np.full(n, 4.0 + shift, dtype=complex))]
    mk = i > 0
    ent.append((idx[mk], idx[mk] - 1, np.full(mk.sum(), -1.0 + 0j)))
    mk = i < m - 1
    ent.append((idx[mk], idx[mk] + 1, np.full(mk.sum(), -1.0 + 0j)))
    mk = j < m - 1
    ent.append((idx[mk], idx[mk] + m, -ph[mk]))
    mk = j > 0
    ent.append((idx[mk], idx[mk] - m, -np.conj(ph[mk])))
    return _assemble(n, ent)


def convdiff3d(m: int, nu: float) -> CSR:
    """-nu*Lap(u) + V.grad(u), upwind 7 points, with the 3D velocity of Section 4:
    V = (2x(1-x)(2y-1)z, -y(1-y)(2x-1), -z(1-z)(2x-1)(2y-1))."""
    n = m ** 3
    h = 1.0 / (m + 1)
    i, j, k = _grid3(m)
    idx = i + m * j + m * m * k
    x, y, z = (i + 1) * h, (j + 1) * h, (k + 1) * h
    vx = 2 * x * (1 - x) * (2 * y - 1) * z
    vy = -y * (1 - y) * (2 * x - 1)
    vz = -z * (1 - z) * (2 * x - 1) * (2 * y - 1)
    diag = 6.0 * nu + h * (np.abs(vx) + np.abs(vy) + np.abs(vz))
    ent = [(idx, idx, diag)]
    for coord, vel, stride in ((i, vx, 1), (j, vy, m), (k, vz, m * m)):
        lo = -nu - h * np.maximum(vel, 0.0)
        hi = -nu - h * np.maximum(-vel, 0.0)
        mk = coord > 0
        ent.append((idx[mk], idx[mk] - stride, lo[mk]))
        mk = coord < m - 1
        ent.append((idx[mk], idx[mk] + stride, hi[mk]))
    return _assemble(n, ent)


def _harmonic(a, b):
    return 2.0 * a * b / (a + b)


def gaussian_field_2d(npad: int, spacing: float, corr_len: float, seed: int) -> np.ndarray:
    """Unit-variance stationary Gaussian field on a periodic npad x npad grid with
    squared-exponential covariance exp(-r^2 / (2 l^2)).

    White noise is filtered in Fourier space by the square root of the DFT of the
    (periodised) covariance; the variance is exactly c(0) = 1 by Parseval."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((npad, npad))
    d = np.minimum(np.arange(npad), npad - np.arange(npad)) * spacing
    r2 = d[:, None] ** 2 + d[None, :] ** 2
    c = np.exp(-r2 / (2.0 * corr_len ** 2))
    S = np.maximum(np.fft.fft2(c).real, 0.0)
    g = np.fft.ifft2(np.sqrt(S) * np.fft.fft2(w)).real
    return g


def diffusion2d_lognormal(m: int, sigma: float = 2.0, corr_len: float = 0.05,
                          seed: int = 0, npad: int = 512) -> CSR:
    """-div(k grad u), 5 points, k = exp(sigma*g) at the nodes (boundary nodes
    included), face coefficients = harmonic mean of the two end nodes."""
    h = 1.0 / (m + 1)
    g = gaussian_field_2d(npad, h, corr_len, seed)[: m + 2, : m + 2]  # [j, i] incl. boundary
    kk = np.exp(sigma * g)
    n = m * m
    i, j = _grid2(m)
    idx = i + m * j
    kc = kk[j + 1, i + 1]
    kw = _harmonic(kc, kk[j + 1, i])
    ke = _harmonic(kc, kk[j + 1, i + 2])
    ks = _harmonic(kc, kk[j, i + 1])
    kn = _harmonic(kc, kk[j + 2, i + 1])
    ent = [(idx, idx, kw + ke + ks + kn)]
    mk = i > 0
    ent.append((idx[mk], idx[mk] - 1, -kw[mk]))
    mk = i < m - 1
    ent.append((idx[mk], idx[mk] + 1, -ke[mk]))
    mk = j > 0
    ent.append((idx[mk], idx[mk] - m, -ks[mk]))
    mk = j < m - 1
    ent.append((idx[mk], idx[mk] + m, -kn[mk]))
    return _assemble(n, ent)


def diffusion3d_blocks(m: int = 128, block: int = 8, log10_range=(-3.0, 3.0), seed: int = 0) -> CSR:
    """-div(k grad u), 7 points; k constant on each block^3 cell of nodes,
    log10 k ~ U[lo, hi] per cell drawn in lexicographic cell order (x fastest).
    Faces use the harmonic mean; faces to the boundary use the node's own k."""
    nb = m // block
    rng = np.random.default_rng(seed)
    logk = rng.uniform(log10_range[0], log10_range[1], size=nb ** 3)  # cell c = cx + nb*cy + nb^2*cz
    i, j, k = _grid3(m)
    idx = i + m * j + m * m * k
    cell = (i // block) + nb * (j // block) + nb * nb * (k // block)
    kc = 10.0 ** logk[cell]
    n = m ** 3
    diag = np.zeros(n)
    ent = []
    for coord, stride in ((i, 1), (j, m), (k, m * m)):
        for side in (-1, 1):
            inside = (coord > 0) if side < 0 else (coord < m - 1)
            kf = kc.copy()
            nb_idx = idx[inside] + side * stride
            kf[inside] = _harmonic(kc[inside], kc[nb_idx])
            diag += kf
            ent.append((idx[inside], nb_idx, -kf[inside]))
    ent.insert(0, (idx, idx, diag))
    return _assemble(n, ent)


# ---------------------------------------------------------------------------
# Partitions and seeds
# ---------------------------------------------------------------------------

def strip_partition(m: int, rows_per_strip: int) -> np.ndarray:
    """2D grid, part = floor(j / rows_per_strip) for grid row j."""
    i, j = _grid2(m)
    return (j // rows_per_strip).astype(np.int32)


def _splits(m: int, p: int) -> np.ndarray:
    """Owner of each of m consecutive indices when [0, m) is cut at floor(t*m/p)."""
    bounds = np.array([(t * m) // p for t in range(p + 1)])
    owner = np.zeros(m, dtype=np.int64)
    for t in range(p):
        owner[bounds[t]:bounds[t + 1]] = t
    return owner


def block_partition_2d(m: int, px: int, py: int | None = None) -> np.ndarray:
    """px x py blocks with boundaries floor(t*m/p); part = bx + px*by."""
    py = px if py is None else py
    i, j = _grid2(m)
    return (_splits(m, px)[i] + px * _splits(m, py)[j]).astype(np.int32)


def block_partition_3d(m: int, px: int, py: int, pz: int) -> np.ndarray:
    i, j, k = _grid3(m)
    return (_splits(m, px)[i] + px * (_splits(m, py)[j] + py * _splits(m, pz)[k])).astype(np.int32)


def bfs_seeds_3d(m: int, cell=(16, 8, 8), seed: int = 0) -> np.ndarray:
    """One seed vertex per lattice cell, uniform over the cell's central half.

    Cells are visited in lexicographic order (x fastest); for each, x, y and z
    offsets are drawn in that order with rng.integers over [ext/4, 3*ext/4)."""
    rng = np.random.default_rng(seed)
    cx, cy, cz = cell
    nx, ny, nz = m // cx, m // cy, m // cz
    seeds = []
    for bz in range(nz):
        for by in range(ny):
            for bx in range(nx):
                ox = rng.integers(cx // 4, 3 * cx // 4)
                oy = rng.integers(cy // 4, 3 * cy // 4)
                oz = rng.integers(cz // 4, 3 * cz // 4)
                x, y, z = bx * cx + ox, by * cy + oy, bz * cz + oz
                seeds.append(x + m * y + m * m * z)
    return np.asarray(seeds, dtype=np.int32)


def rhs(n: int, seed: int) -> np.ndarray:
    """Right-hand side ~ N(0, 1), numpy default_rng(seed).standard_normal(n)."""
    return np.random.default_rng(seed).standard_normal(n)


# ---------------------------------------------------------------------------
# Named workloads
# ---------------------------------------------------------------------------

CONFIGS = {
    "c1_laplace2d_64_strips8": dict(
        desc="2D 5-point Laplacian 64x64, 8 strips, overlap 1, nev 4, GMRES(30)",
        overlap=1, nev=4, restart=30, flexible=False, nrhs=1),
    "c2_convdiff2d_512_blocks64": dict(
        desc="2D upwind convection-diffusion 512x512, Pe 100, 8x8 blocks, overlap 2, nev 8, FGMRES(50)",
        overlap=2, nev=8, restart=50, flexible=True, nrhs=1),
    "c3a_convdiff3d_64_bfs256": dict(
        desc="3D upwind convection-diffusion 64^3, 256 BFS-grown parts, overlap 2, nev 10, FGMRES(30)",
        overlap=2, nev=10, restart=30, flexible=True, nrhs=1),
    "c4_lognormal2d_256_blocks64": dict(
        desc="2D -div(k grad u) 256x256, log-normal k (sigma 2, corr 0.05), 8x8 blocks, overlap 1, nev 8, GMRES(30)",
        overlap=1, nev=8, restart=30, flexible=False, nrhs=1),
    "c5_jump3d_128_boxes1024": dict(
        desc="3D -div(k grad u) 128^3, k jumping 1e-3..1e3 on 8^3 blocks, 1024 boxes, overlap 2, nev 12, 16 RHS",
        overlap=2, nev=12, restart=30, flexible=True, nrhs=16),
}


def c3b_sizes():
    """Grid sides of the 32 independent 2D systems: round(16 * 16^(k/31))."""
    return [int(round(16 * 16 ** (k / 31.0))) for k in range(32)]


def config(name: str, scale: int | None = None, seed: int = 0):
    """Return (A: CSR, part: int32[n], nparts, opts dict) for a named workload.

    `scale` overrides the grid side for reduced-size variants of the same
    problem family (used by the small parity cases)."""
    opts = dict(CONFIGS[name])
    if name.startswith("c1"):
        m = scale or 64
        A = laplace2d(m)
        rows = max(1, m // 8)
        part = strip_partition(m, rows)
    elif name.startswith("c2"):
        m = scale or 512
        A = convdiff2d(m, nu=0.01)
        part = block_partition_2d(m, 8)
    elif name.startswith("c3a"):
        m = scale or 64
        A = convdiff3d(m, nu=0.01)
        part = None  # BFS-grown from seeds; see bfs_seeds_3d
        opts["seeds"] = bfs_seeds_3d(m, (max(m // 4, 1), max(m // 8, 1), max(m // 8, 1)), seed)
    elif name.startswith("c4"):
        m = scale or 256
        A = diffusion2d_lognormal(m, seed=seed)
        part = block_partition_2d(m, 8)
    elif name.startswith("c5"):
        m = scale or 128
        A = diffusion3d_blocks(m, block=max(m // 16, 1), seed=seed)
        part = block_partition_3d(m, 8, 8, 16)
    else:
        raise KeyError(name)
    nparts = int(part.max()) + 1 if part is not None else len(opts["seeds"])
    return A, part, nparts, opts


def lognormal2d_values_torch(m: int, seed: int, indptr, indices, sigma: float = 2.0,
                             corr_len: float = 0.05, npad: int = 512):
    """Values of diffusion2d_lognormal(m, sigma, corr_len) for the same CSR
    pattern (indptr, indices: device tensors), drawn on the device with
    torch's generator (seed) instead of numpy's: the same recipe (white noise
    filtered by the square root of the periodised squared-exponential
    covariance, k = exp(sigma g) at the nodes, harmonic face means), a
    different sample.  Used to make many training fields quickly."""
    import torch
    dev = indptr.device
    h = 1.0 / (m + 1)
    gen = torch.Generator(device=dev).manual_seed(int(seed))
    w = torch.randn((npad, npad), generator=gen, device=dev, dtype=torch.float64)
    ar = torch.arange(npad, device=dev, dtype=torch.float64)
    d = torch.minimum(ar, npad - ar) * h
    r2 = d[:, None] ** 2 + d[None, :] ** 2
    c = torch.exp(-r2 / (2.0 * corr_len ** 2))
    S = torch.clamp(torch.fft.fft2(c).real, min=0.0)
    g = torch.fft.ifft2(torch.sqrt(S) * torch.fft.fft2(w)).real[: m + 2, : m + 2]
    kk = torch.exp(sigma * g)
    n = m * m
    deg = indptr[1:] - indptr[:-1]
    rows = torch.repeat_interleave(torch.arange(n, device=dev), deg)
    cols = indices.to(torch.int64)
    i, j = rows % m, rows // m
    harm = lambda a, b: 2.0 * a * b / (a + b)
    kc = kk[j + 1, i + 1]
    kw = harm(kc, kk[j + 1, i])
    ke = harm(kc, kk[j + 1, i + 2])
    ks = harm(kc, kk[j, i + 1])
    kn = harm(kc, kk[j + 2, i + 1])
    dlt = cols - rows
    val = torch.where(dlt == 0, kw + ke + ks + kn,
          torch.where(dlt == -1, -kw, torch.where(dlt == 1, -ke,
          torch.where(dlt == -m, -ks, -kn))))
    return val
