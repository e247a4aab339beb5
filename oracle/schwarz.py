"""Scalable FP64 oracle tier (SciPy sparse, SuperLU, ARPACK).

TEST INFRASTRUCTURE ONLY -- not part of the library's compute path.

Follows the paper section by section:

  Section 2   overlapping subdomains Omega_i = [Omega_Ii, Omega_Gamma_i] grown in
              the adjacency graph of A; restriction R_i; algebraic partition of
              unity D_i; the one-level (eq. 1, eq. 3) and two-level (eq. 2,
              eq. 4) preconditioners.
  Section 3.1 Definition 1: the local block splitting matrix obtained by
              lumping the couplings to the outside of Omega_i into the
              diagonal of the overlap rows.
  Section 3.2 eq. 5 local generalized eigenproblem and eq. 6 coarse space.
  Section 4   right-preconditioned restarted GMRES, relative tolerance, zero
              initial guess; exact LU of the local and coarse matrices.

Readings taken where the paper is silent (shared with the dense tier):
  R1  adjacency of nonsymmetric A = pattern of A + A^T, diagonal excluded.
  R2  overlap of delta layers: layer d = neighbours of (Omega_Ii + layers < d)
      not already in them; Omega_Gamma_i = union of the layers.
  R3  ascending global index inside Omega_Ii and inside Omega_Gamma_i.
  R4  Boolean partition of unity: D_i = diag(1 on Omega_Ii, 0 on Omega_Gamma_i).
  R5  s_i sums rows (not columns); sum taken in ascending column order.
  R6  kernel of the splitting: K_i is spanned by the indicator vectors of the
      connected components of the splitting's graph (stored entries of the
      splitting and its transpose) whose rows all satisfy |row sum| <= 1e-13 *
      (sum of |entries|) -- for a connected subdomain span{1} or {0}.  The
      splitting is block diagonal over the components, so its kernel is the
      sum of theirs.
  R7  eq. 5 is solved on the domain K_i^perp with codomain range(splitting);
      Pi_i = orthogonal projector onto range(splitting).
  R8  selection: finite eigenvalues by |lambda| descending; a cut that falls
      inside a cluster (|lambda| >= (1 - 1e-6) |lambda_cut|) takes the whole
      cluster (so conjugate pairs stay together); a complex eigenvector gives
      its real and imaginary parts; nev counts the kernel part; the optional
      tau filter keeps |lambda| > 1/tau.
  R9  W_i = Z_i restricted to the interior rows (D_i Z_i), orthonormalised by
      Householder QR (the span, hence M^{-1}, is unchanged).
  R10 GMRES converges when the Arnoldi estimate and the recomputed true
      residual are both <= rtol * ||b||; iterations are Arnoldi steps summed
      over restart cycles.

Complex A (the Notation paragraph takes A complex and writes adjoints): the
absolute values of Definition 1 are moduli, R_0^H and every inner product
conjugate, the selected complex eigenvectors of eq. 5 form Z_i as they are
(the real/imaginary split of R8 is for real A only), the projector of R7 uses
the left null vector of the splitting under the adjoint, and GMRES runs in
complex arithmetic with complex Givens rotations.  On real input every
operation reduces to the real one.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph
import scipy.sparse.linalg as spla

KERNEL_ROWSUM_TOL = 1e-13
CLUSTER_RTOL = 1e-6
BREAKDOWN_TOL = 1e-14

# status codes shared in meaning with the library's C interface
OK, KSP_MAXIT, KSP_BREAKDOWN = 0, 1, 2


# ---------------------------------------------------------------------------
# Section 2: graph, subdomains, restrictions, partition of unity
# ---------------------------------------------------------------------------

def validate(A: sp.csr_matrix, part, nparts: int, overlap: int, nev: int):
    """Argument checks (Section 2 assumes N non-empty disjoint subsets)."""
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("A must be square")
    part = np.asarray(part)
    if part.shape != (n,):
        raise ValueError("part must have length n")
    if part.min() < 0 or part.max() >= nparts:
        raise ValueError("part values must lie in [0, nparts)")
    if np.bincount(part, minlength=nparts).min() == 0:
        raise ValueError("every part must be non-empty")
    if overlap < 0 or nev < 0:
        raise ValueError("overlap and nev must be >= 0")


def adjacency(A: sp.csr_matrix) -> sp.csr_matrix:
    """Pattern of A + A^T without the diagonal (reading R1), as a 0/1 CSR matrix."""
    P = sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape)
    G = (P + P.T).tocsr()
    G.setdiag(0)
    G.eliminate_zeros()
    G.data[:] = 1.0
    return G


@dataclasses.dataclass
class Subdomain:
    interior: np.ndarray  # Omega_Ii, ascending
    gamma: np.ndarray     # Omega_Gamma_i, ascending
    layer: np.ndarray     # layer id (1..delta) of each gamma node

    @property
    def omega(self) -> np.ndarray:  # Omega_i = [Omega_Ii, Omega_Gamma_i]
        return np.concatenate([self.interior, self.gamma])

    @property
    def n_interior(self) -> int:
        return len(self.interior)

    @property
    def size(self) -> int:
        return len(self.interior) + len(self.gamma)


def subdomains(A: sp.csr_matrix, part, nparts: int, overlap: int, G=None) -> list[Subdomain]:
    """Section 2: grow each Omega_Ii by `overlap` graph layers (readings R2, R3)."""
    G = adjacency(A) if G is None else G
    part = np.asarray(part)
    n = A.shape[0]
    out = []
    for i in range(nparts):
        interior = np.flatnonzero(part == i)
        visited = np.zeros(n, dtype=bool)
        visited[interior] = True
        layer = np.zeros(n, dtype=np.int32)
        frontier = visited.astype(np.float64)
        for d in range(1, overlap + 1):
            reach = (G @ frontier) > 0
            new = reach & ~visited
            layer[new] = d
            visited |= new
            frontier = new.astype(np.float64)
        gamma = np.flatnonzero(visited & (part != i))
        out.append(Subdomain(interior.astype(np.int64), gamma.astype(np.int64), layer[gamma]))
    return out


def bfs_partition(A: sp.csr_matrix, seeds) -> np.ndarray:
    """Multi-source BFS partition: every vertex takes the seed with the smallest
    (graph distance, seed id).  Stand-in for the external graph partitioner of
    Section 4 (ParMETIS is not available)."""
    G = adjacency(A)
    n = A.shape[0]
    owner = np.full(n, -1, dtype=np.int64)
    seeds = np.asarray(seeds)
    owner[seeds[::-1]] = np.arange(len(seeds))[::-1]  # smallest id wins on duplicates
    frontier = np.unique(seeds)
    indptr, indices = G.indptr, G.indices
    while len(frontier):
        # candidates: (neighbour, owner of the frontier vertex)
        cnt = indptr[frontier + 1] - indptr[frontier]
        src = np.repeat(frontier, cnt)
        nb = np.concatenate([indices[indptr[v]:indptr[v + 1]] for v in frontier]) if len(frontier) else np.array([], int)
        cand_owner = owner[src]
        free = owner[nb] < 0
        nb, cand_owner = nb[free], cand_owner[free]
        if len(nb) == 0:
            break
        order = np.lexsort((cand_owner, nb))
        nb, cand_owner = nb[order], cand_owner[order]
        first = np.ones(len(nb), dtype=bool)
        first[1:] = nb[1:] != nb[:-1]
        owner[nb[first]] = cand_owner[first]
        frontier = nb[first]
    if (owner < 0).any():
        raise ValueError("graph is disconnected from the seeds")
    return owner.astype(np.int32)


def partition_of_unity(sub: Subdomain) -> np.ndarray:
    """Boolean algebraic partition of unity (reading R4): diagonal of D_i."""
    d = np.zeros(sub.size)
    d[: sub.n_interior] = 1.0
    return d


# ---------------------------------------------------------------------------
# Section 3.1: Definition 1, local block splitting
# ---------------------------------------------------------------------------

def block_splitting(A: sp.csr_matrix, sub: Subdomain):
    """Return (A_ii, s_i, Atilde_ii) in the [Omega_Ii, Omega_Gamma_i] order.

    s_i(j) is the sum of |a_jk| over k outside Omega_i for overlap row j,
    accumulated in ascending column order (reading R5); Atilde_ii equals A_ii
    except that s_i is subtracted from the overlap part of the diagonal."""
    omega = sub.omega
    n = A.shape[0]
    A_ii = A[omega][:, omega].tocsr()
    A_ii.sort_indices()
    inside = np.zeros(n, dtype=bool)
    inside[omega] = True
    g = sub.gamma
    starts, ends = A.indptr[g], A.indptr[g + 1]
    lens = ends - starts
    s = np.zeros(len(g))
    for p in range(int(lens.max()) if len(g) else 0):  # sequential left-to-right sum per row
        has = p < lens
        pos = np.where(has, starts + p, 0)
        col = A.indices[pos]
        val = np.abs(A.data[pos])
        s = s + np.where(has & ~inside[col], val, 0.0)
    At = A_ii.tolil(copy=True)
    nI = sub.n_interior
    for t in range(len(g)):
        At[nI + t, nI + t] = A_ii[nI + t, nI + t] - s[t]
    At = At.tocsr()
    At.sort_indices()
    return A_ii, s, At


def floating_components(At: sp.csr_matrix) -> list:
    """Reading R6: the connected components of the splitting's graph (stored
    entries of At and At^T) whose rows all sum to zero relative to their
    absolute row sums (floating pieces of a zero-row-sum M-matrix), as
    ascending local index arrays, ordered by their smallest index."""
    n = At.shape[0]
    rows = np.repeat(np.arange(n), np.diff(At.indptr))
    rs = np.zeros(n, dtype=At.dtype)
    ars = np.zeros(n)
    np.add.at(rs, rows, At.data)
    np.add.at(ars, rows, np.abs(At.data))
    ok = np.abs(rs) <= KERNEL_ROWSUM_TOL * ars
    G = sp.csr_matrix((np.ones(At.nnz), At.indices, At.indptr), shape=(n, n))
    ncomp, lab = csgraph.connected_components(G + G.T, directed=False)
    comps = [np.flatnonzero(lab == c) for c in range(ncomp)]
    return sorted((idx for idx in comps if ok[idx].all()), key=lambda idx: idx[0])


def kernel_dimension(At: sp.csr_matrix) -> int:
    """Reading R6: dim K_i, the number of floating components of the splitting
    (0 or 1 for a connected subdomain)."""
    return len(floating_components(At))


# ---------------------------------------------------------------------------
# Section 3.2: eq. 5 and eq. 6
# ---------------------------------------------------------------------------

def select_eigenvalues(lam: np.ndarray, count: int, tau: float = 0.0, complete: bool = True):
    """Reading R8.  Returns indices into `lam` of the selected eigenvalues
    (ordered by |lambda| descending) or raises if the cluster at the cut may be
    incomplete (complete=False means `lam` is a truncated top list)."""
    order = np.argsort(-np.abs(lam), kind="stable")
    mags = np.abs(lam[order])
    if count <= 0:
        sel = order[:0]
    else:
        if count > len(order):
            raise ValueError("not enough eigenvalues")
        cut = mags[count - 1]
        take = int(np.sum(mags >= (1.0 - CLUSTER_RTOL) * cut))
        if not complete and take >= len(order):
            raise _NeedMore()
        sel = order[:take]
    if tau > 0:
        sel = sel[np.abs(lam[sel]) > 1.0 / tau]
    return sel


class _NeedMore(Exception):
    pass


def real_basis(vecs: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """Real basis of the span of selected (possibly complex) eigenvectors: for a
    conjugate pair only the member with Im(lambda) > 0 is used, giving its real
    and imaginary parts (reading R8)."""
    cols = []
    for t in range(vecs.shape[1]):
        v = vecs[:, t]
        if abs(lam[t].imag) <= 1e-12 * max(abs(lam[t]), 1e-300):
            w = v.real if np.linalg.norm(v.real) >= np.linalg.norm(v.imag) else v.imag
            cols.append(w)
        elif lam[t].imag > 0:
            cols.append(v.real)
            cols.append(v.imag)
    return np.array(cols).T if cols else np.zeros((vecs.shape[0], 0))


def local_eigenproblem(A_ii: sp.csr_matrix, At: sp.csr_matrix, n_interior: int, nev: int,
                       tau: float = 0.0, kdim: int | None = None, tol: float = 1e-13):
    """eq. 5 on one subdomain, scalable tier (reading R7).

    T = Atilde_reg^{-1} Pi B Pi followed by the projection onto K^perp, where
    B = D A_ii D = diag(A_I, 0) under the Boolean D and Atilde_reg is the
    splitting with the last diagonal entry of each floating component doubled
    (K spanned by their indicators, reading R6; one component with the whole
    subdomain: K = span{1}).  The nonzero eigenpairs of T are exactly the
    eigenpairs of the pencil restricted to K^perp.  Returns dict(lam_all,
    lam_sel, Z, kernel) with Z = [Y, U_sel] (nev_i real columns, the kernel
    part first)."""
    ni = A_ii.shape[0]
    cplx = np.iscomplexobj(A_ii.data)
    comps = floating_components(At)
    if kdim is None:
        kdim = len(comps)
    assert kdim == len(comps)
    d = np.zeros(ni)
    d[:n_interior] = 1.0
    B = sp.diags(d) @ A_ii @ sp.diags(d)
    if kdim >= 1:
        # the splitting is block diagonal over its components, so each doubled
        # entry regularises its own component, and the solve with the unit
        # vector of that entry gives that component's left null vector (zero
        # elsewhere)
        Areg = At.tolil(copy=True)
        for idx in comps:
            Areg[idx[-1], idx[-1]] = 2.0 * At[idx[-1], idx[-1]]
        lu = spla.splu(Areg.tocsc())
        ells, ks = [], []
        for idx in comps:
            e_last = np.eye(1, ni, idx[-1]).ravel().astype(A_ii.dtype)
            ell = lu.solve(e_last, trans="H" if cplx else "T")  # null(Atilde^H)
            ell /= np.linalg.norm(ell)
            ells.append(ell)
            k = np.zeros(ni)
            k[idx] = 1.0 / np.sqrt(len(idx))
            ks.append(k)

        def Pi(x):
            for ell in ells:
                x = x - ell * (ell.conj() @ x)
            return x

        def T(x):
            y = lu.solve(Pi(B @ Pi(x)))
            for k in ks:
                y = y - k * (k @ y)
            return y
        # kernel part (L cap K)^{perp_K}: every component holds interior rows
        # (the overlap layers are grown from the interior through entries
        # inside Omega_i), B maps its indicator to a nonzero vector on it (A_I
        # is nonsingular), so L cap K = {0} and the part is K itself.
        Y = np.column_stack(ks)
    else:
        lu = spla.splu(At.tocsc())

        def T(x):
            return lu.solve(B @ x)
        Y = np.zeros((ni, 0))
    count = nev - Y.shape[1]
    if count <= 0:
        lam = np.zeros(0, complex)
        return dict(lam_all=lam, lam_sel=lam, Z=Y[:, :max(nev, 0)], kernel=kdim)
    op = spla.LinearOperator((ni, ni), matvec=T, dtype=A_ii.dtype)
    v0 = (np.ones(ni) + np.linspace(0.0, 1.0, ni)).astype(A_ii.dtype)
    for k in (ks if kdim >= 1 else []):
        v0 -= k * (k @ v0)
    extra = 6
    while True:
        kk = count + extra
        if kk + 20 >= ni:
            # small subdomain: every eigenvalue of the explicit operator
            Tm = np.column_stack([T(e) for e in np.eye(ni)])
            lam, vec = np.linalg.eig(Tm)
            sel = select_eigenvalues(lam, count, tau, complete=True)
            break
        lam, vec = spla.eigs(op, k=kk, which="LM", tol=tol, v0=v0, maxiter=100000,
                             ncv=min(ni - 1, max(2 * kk + 1, kk + 20)))
        try:
            sel = select_eigenvalues(lam, count, tau, complete=False)
            break
        except _NeedMore:
            extra *= 2
    order = np.argsort(-np.abs(lam), kind="stable")
    U = vec[:, sel] if cplx else real_basis(vec[:, sel], lam[sel])
    Z = np.hstack([Y.astype(U.dtype), U])
    return dict(lam_all=lam[order], lam_sel=lam[sel], Z=Z, kernel=kdim)


# ---------------------------------------------------------------------------
# Setup and application of eq. 4 (and the other variants of Section 2)
# ---------------------------------------------------------------------------

class TwoLevelSchwarz:
    """M^{-1} of eq. 4 (variant="deflated"), eq. 3 (variant="ras", no coarse
    space), eq. 2 (variant="additive-asm") or eq. 1 ("asm")."""

    def __init__(self, A, part, nparts: int, overlap: int, nev: int, tau: float = 0.0,
                 variant: str = "deflated", keep_local=False):
        A = sp.csr_matrix(A)
        A.sort_indices()
        validate(A, part, nparts, overlap, nev)
        self.A = A
        self.n = A.shape[0]
        self.variant = variant
        self.times = {}
        t0 = time.perf_counter()
        self.subs = subdomains(A, part, nparts, overlap)
        self.times["maps"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        self.local = []
        for sub in self.subs:
            A_ii, s, At = block_splitting(A, sub)
            self.local.append(dict(A_ii=A_ii, s=s, At=At))
        self.times["extract"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        for loc in self.local:
            loc["lu"] = spla.splu(loc["A_ii"].tocsc())
        self.times["factor"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        self.eig = []
        use_coarse = variant in ("deflated", "additive-asm", "additive-ras") and nev > 0
        W = []
        for sub, loc in zip(self.subs, self.local):
            kd = kernel_dimension(loc["At"])
            if use_coarse:
                res = local_eigenproblem(loc["A_ii"], loc["At"], sub.n_interior, nev, tau, kdim=kd)
                Wi = res["Z"][: sub.n_interior]  # D_i Z_i on the interior rows
                if Wi.shape[1]:
                    Wi, _ = np.linalg.qr(Wi)
                W.append(Wi)
                self.eig.append(res)
            else:
                self.eig.append(dict(kernel=kd, lam_sel=np.zeros(0), lam_all=np.zeros(0)))
                W.append(np.zeros((sub.n_interior, 0)))
        self.times["eig"] = time.perf_counter() - t0
        t0 = time.perf_counter()
        self.W = W
        self.nev_i = np.array([w.shape[1] for w in W], dtype=np.int64)
        self.n0 = int(self.nev_i.sum())
        if self.n0:
            rows, cols, vals = [], [], []
            off = 0
            for sub, Wi in zip(self.subs, W):
                r = np.repeat(sub.interior, Wi.shape[1])
                c = np.tile(np.arange(off, off + Wi.shape[1]), len(sub.interior))
                rows.append(r)
                cols.append(c)
                vals.append(Wi.ravel())
                off += Wi.shape[1]
            self.Z = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                   shape=(self.n, self.n0))
            self.E = (self.Z.conj().T @ (A @ self.Z)).toarray()
            self.E_lu = sla.lu_factor(self.E)
        else:
            self.Z = None
        self.times["coarse"] = time.perf_counter() - t0
        if not keep_local:
            for loc in self.local:
                loc.pop("At", None)

    # -- pieces of eq. 1-4 ---------------------------------------------------
    def coarse_correction(self, r):
        """R_0^H A_00^{-1} R_0 r."""
        if not self.n0:
            return np.zeros_like(r)
        c = self.Z.conj().T @ r
        return self.Z @ sla.lu_solve(self.E_lu, c)

    def one_level(self, t, restricted=True):
        """eq. 3 (restricted=True) or eq. 1: sum_i R_i^T [D_i] A_ii^{-1} R_i t."""
        x = np.zeros_like(t)
        for sub, loc in zip(self.subs, self.local):
            om = sub.omega
            xi = loc["lu"].solve(t[om])
            if restricted:
                x[sub.interior] += xi[: sub.n_interior]
            else:
                x[om] += xi
        return x

    def apply(self, r):
        r = np.asarray(r, dtype=np.result_type(self.A.dtype, np.asarray(r).dtype, np.float64))
        if r.ndim == 2:
            return np.stack([self.apply(r[:, j]) for j in range(r.shape[1])], axis=1)
        if self.variant == "deflated":          # eq. 4
            q = self.coarse_correction(r)
            t = r - self.A @ q
            return q + self.one_level(t, restricted=True)
        if self.variant == "ras":               # eq. 3
            return self.one_level(r, restricted=True)
        if self.variant == "asm":               # eq. 1
            return self.one_level(r, restricted=False)
        if self.variant == "additive-asm":      # eq. 2
            return self.coarse_correction(r) + self.one_level(r, restricted=False)
        if self.variant == "additive-ras":
            return self.coarse_correction(r) + self.one_level(r, restricted=True)
        raise ValueError(self.variant)

    def info(self):
        return dict(n0=self.n0, nev_i=self.nev_i.copy(),
                    kernel=np.array([e["kernel"] for e in self.eig]),
                    n_interior=np.array([s.n_interior for s in self.subs]),
                    n_i=np.array([s.size for s in self.subs]))


# ---------------------------------------------------------------------------
# Section 4: restarted right-preconditioned (F)GMRES
# ---------------------------------------------------------------------------

def gmres(A, b, M=None, restart=30, rtol=1e-8, maxit=1000, flexible=False, fixed_iters=0):
    """Restarted right-preconditioned GMRES(m) / FGMRES(m), x0 = 0, modified
    Gram-Schmidt, Givens rotations (reading R10); complex A or b run in
    complex arithmetic (conjugated inner products, rotations
    [[conj c, conj s], [-s, c]] with c = h_jj / rho, s = h_j+1,j / rho, which
    for real data are the usual [[c, s], [-s, c]]).

    fixed_iters > 0 runs exactly that many Arnoldi steps (no convergence test)
    and returns the iterate.  Returns (x, info) with info = dict(its, status,
    history) where history[k] is the Arnoldi residual estimate / ||b|| after k
    steps."""
    A = sp.csr_matrix(A) if sp.issparse(A) else A
    n = len(b)
    Mv = (lambda v: v) if M is None else M
    dt = np.result_type(A.dtype, np.asarray(b).dtype, np.float64)
    bnorm = np.linalg.norm(b)
    x = np.zeros(n, dtype=dt)
    its = 0
    hist = [1.0]
    if bnorm == 0.0:
        return x, dict(its=0, status=OK, history=hist, relres=0.0)
    status = None
    while True:
        r = b - A @ x
        beta = np.linalg.norm(r)
        if beta == 0.0 or (fixed_iters == 0 and beta <= rtol * bnorm):
            status = OK
            break
        m = restart
        V = np.zeros((m + 1, n), dtype=dt)
        Zs = np.zeros((m, n), dtype=dt) if flexible else None
        H = np.zeros((m + 1, m), dtype=dt)
        cs = np.zeros(m, dtype=dt)
        sn = np.zeros(m, dtype=dt)
        g = np.zeros(m + 1, dtype=dt)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        stop = None
        for j in range(m):
            z = Mv(V[j])
            if flexible:
                Zs[j] = z
            w = A @ z
            for i in range(j + 1):
                H[i, j] = np.conj(V[i]) @ w
                w = w - H[i, j] * V[i]
            hnext = np.linalg.norm(w)
            H[j + 1, j] = hnext
            hcol = np.linalg.norm(H[: j + 2, j])
            for i in range(j):
                t = np.conj(cs[i]) * H[i, j] + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(abs(H[j, j]), abs(H[j + 1, j]))
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            its += 1
            j_end = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            breakdown = hnext <= BREAKDOWN_TOL * hcol
            if fixed_iters:
                if its >= fixed_iters:
                    stop = "fixed"
                    break
            elif abs(g[j + 1]) <= rtol * bnorm:
                stop = "est"
                break
            elif its >= maxit:
                stop = "maxit"
                break
            if breakdown:
                stop = "breakdown"
                break
            V[j + 1] = w / hnext
        y = sla.solve_triangular(H[:j_end, :j_end], g[:j_end])
        if flexible:
            x = x + Zs[:j_end].T @ y
        else:
            x = x + Mv(V[:j_end].T @ y)
        if fixed_iters:
            if stop in ("fixed", "breakdown"):
                status = OK
                break
            continue
        true_res = np.linalg.norm(b - A @ x)
        if true_res <= rtol * bnorm:
            status = OK
            break
        if stop == "maxit" or its >= maxit:
            status = KSP_MAXIT
            break
        if stop == "breakdown":
            status = KSP_BREAKDOWN
            break
    relres = np.linalg.norm(b - A @ x) / bnorm
    return x, dict(its=its, status=status, history=hist, relres=relres)


def solve(A, b, part, nparts, overlap, nev, restart=30, rtol=1e-8, maxit=1000, flexible=False,
          fixed_iters=0, variant="deflated"):
    """Convenience: setup + GMRES; returns (x, info, preconditioner)."""
    P = TwoLevelSchwarz(A, part, nparts, overlap, nev, variant=variant)
    t0 = time.perf_counter()
    x, info = gmres(A, b, P.apply, restart, rtol, maxit, flexible, fixed_iters)
    P.times["solve"] = time.perf_counter() - t0
    return x, info, P
