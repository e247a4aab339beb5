"""Literal dense FP64 oracle tier for tiny inputs.

TEST INFRASTRUCTURE ONLY -- not part of the library's compute path.

Everything is an explicit dense matrix written in the paper's notation:
R_i = I_n(Omega_i, :) (Section 2), the permutation P_i and the 3 x 3 block
partition of P_i A P_i^T (Definition 1, Section 3.1), L_i = ker(D_i A_ii D_i)
and K_i = ker(Atilde_ii) from singular value decompositions, Pi_i the
orthogonal projector onto range(Atilde_ii), and eq. 5 solved by the QZ
algorithm on the pencil restricted to K_i^perp x range(Atilde_ii) (reading R7
of the scalable tier; the unrestricted pencil is singular whenever K_i is not
{0}).  Complex A is taken as it is (moduli in Definition 1, adjoints
throughout, complex eigenvectors as the columns of Z_i).  The explicit
preconditioner matrices of eq. 1 - eq. 4 are formed by products of these
matrices.  This tier shares no code with ``oracle.schwarz``
so that the two check each other.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

SVD_RTOL = 1e-12
CLUSTER_RTOL = 1e-6


def _graph(A):
    G = (A != 0) | (A.T != 0)
    np.fill_diagonal(G, False)
    return G


def overlapping_sets(A, part, nparts, delta):
    """Omega_Ii, Omega_Gamma_i (both ascending) and the layer of each overlap node."""
    G = _graph(A).astype(np.int64)
    n = A.shape[0]
    res = []
    for i in range(nparts):
        inside = part == i
        layer = np.full(n, -1)
        layer[inside] = 0
        for d in range(1, delta + 1):
            reach = (G @ (layer >= 0).astype(np.int64)) > 0
            layer[reach & (layer < 0)] = d
        I = np.flatnonzero(layer == 0)
        Gam = np.flatnonzero(layer > 0)
        res.append((I, Gam, layer[Gam]))
    return res


def restriction(idx, n):
    """R = I_n(idx, :)."""
    return np.eye(n)[idx, :]


def local_matrices(A, I, Gam):
    """Definition 1 with explicit blocks of P_i A P_i^T."""
    n = A.shape[0]
    c = np.setdiff1d(np.arange(n), np.concatenate([I, Gam]))
    P = restriction(np.concatenate([I, Gam, c]), n)
    PAP = P @ A @ P.T
    nI, nG = len(I), len(Gam)
    A_I = PAP[:nI, :nI]
    A_IG = PAP[:nI, nI:nI + nG]
    A_GI = PAP[nI:nI + nG, :nI]
    A_G = PAP[nI:nI + nG, nI:nI + nG]
    A_Gc = PAP[nI:nI + nG, nI + nG:]
    s = np.abs(A_Gc).sum(axis=1)
    At_G = A_G - np.diag(s)
    A_ii = np.block([[A_I, A_IG], [A_GI, A_G]])
    At_ii = np.block([[A_I, A_IG], [A_GI, At_G]])
    return A_ii, At_ii, s


def _null_and_range(M):
    U, sig, Vh = np.linalg.svd(M)
    r = int(np.sum(sig > SVD_RTOL * sig[0])) if sig[0] > 0 else 0
    return dict(right_null=Vh[r:].conj().T, right_perp=Vh[:r].conj().T,
                left_null=U[:, r:], range=U[:, :r])


def _orth(M):
    if M.size == 0:
        return M
    U, sig, _ = np.linalg.svd(M, full_matrices=False)
    r = int(np.sum(sig > SVD_RTOL * sig[0])) if sig.size and sig[0] > 0 else 0
    return U[:, :r]


def local_eig(A_ii, At_ii, nI, nev, tau=0.0):
    """eq. 5 and eq. 6 on one subdomain.  Returns dict with all finite
    eigenvalues (|lambda| descending), the selected ones, the kernel part and
    Z_i (nev_i columns, kernel part first; real for real A)."""
    cplx = np.iscomplexobj(A_ii)
    ni = A_ii.shape[0]
    D = np.diag(np.r_[np.ones(nI), np.zeros(ni - nI)])
    B = D @ A_ii @ D
    sv = _null_and_range(At_ii)
    QK, QU, Ql, QR = sv["right_null"], sv["right_perp"], sv["left_null"], sv["range"]
    Pi = np.eye(ni) - Ql @ Ql.conj().T
    lhs = QR.conj().T @ Pi @ B @ Pi @ QU
    rhs = QR.conj().T @ At_ii @ QU
    w, V = sla.eig(lhs, rhs)
    finite = np.isfinite(w)
    w, V = w[finite], V[:, finite]
    order = np.argsort(-np.abs(w), kind="stable")
    w, V = w[order], V[:, order]
    # kernel part: complement of L cap K inside K = Q_K * orth((B Q_K)^H)
    if QK.shape[1]:
        Y = QK @ _orth((B @ QK).conj().T)
    else:
        Y = np.zeros((ni, 0))
    count = nev - Y.shape[1]
    if count > 0:
        cut = np.abs(w[count - 1])
        take = int(np.sum(np.abs(w) >= (1 - CLUSTER_RTOL) * cut))
        sel = np.arange(take)
        if tau > 0:
            sel = sel[np.abs(w[sel]) > 1.0 / tau]
    else:
        sel = np.arange(0)
    cols = []
    for t in sel:
        u = QU @ V[:, t]
        if cplx:
            cols.append(u)
        elif abs(w[t].imag) <= 1e-12 * abs(w[t]):
            cols.append(u.real if np.linalg.norm(u.real) >= np.linalg.norm(u.imag) else u.imag)
        elif w[t].imag > 0:
            cols += [u.real, u.imag]
    U = np.array(cols).T if cols else np.zeros((ni, 0))
    Yk = Y if cplx else Y.real
    Z = np.hstack([Yk, U]) if count > 0 else Yk[:, :max(nev, 0)]
    return dict(lam_all=w, lam_sel=w[sel], Z=Z, kernel=QK.shape[1], B=B, Pi=Pi,
                K=QK, L=_null_and_range(B)["right_null"])


class DenseSchwarz:
    """All operators of Section 2 as explicit dense matrices."""

    def __init__(self, A, part, nparts, delta, nev, tau=0.0):
        A = np.asarray(A.toarray() if hasattr(A, "toarray") else A)
        A = A.astype(np.complex128 if np.iscomplexobj(A) else np.float64)
        part = np.asarray(part)
        self.A = A
        n = self.n = A.shape[0]
        self.sets = overlapping_sets(A, part, nparts, delta)
        self.R, self.D, self.Aii, self.Atii, self.s, self.eig = [], [], [], [], [], []
        for I, Gam, _ in self.sets:
            om = np.concatenate([I, Gam])
            R = restriction(om, n)
            A_ii, At_ii, s = local_matrices(A, I, Gam)
            assert np.allclose(A_ii, R @ A @ R.T, rtol=0, atol=0)
            self.R.append(R)
            self.D.append(np.diag(np.r_[np.ones(len(I)), np.zeros(len(Gam))]))
            self.Aii.append(A_ii)
            self.Atii.append(At_ii)
            self.s.append(s)
            self.eig.append(local_eig(A_ii, At_ii, len(I), nev, tau) if nev > 0 else None)
        # R_0^H = [R_1^T D_1 Z_1, ..., R_N^T D_N Z_N]
        blocks = [R.T @ D @ e["Z"] for R, D, e in zip(self.R, self.D, self.eig) if e is not None]
        self.R0H = np.hstack(blocks) if blocks else np.zeros((n, 0))
        self.n0 = self.R0H.shape[1]
        self.A00 = self.R0H.conj().T @ A @ self.R0H

    def M_asm(self):      # eq. 1
        return sum(R.T @ np.linalg.inv(Aii) @ R for R, Aii in zip(self.R, self.Aii))

    def M_ras(self):      # eq. 3
        return sum(R.T @ D @ np.linalg.inv(Aii) @ R for R, D, Aii in zip(self.R, self.D, self.Aii))

    def coarse(self):     # R_0^H A_00^{-1} R_0
        if self.n0 == 0:
            return np.zeros((self.n, self.n))
        return self.R0H @ np.linalg.solve(self.A00, self.R0H.conj().T)

    def M_additive(self):  # eq. 2
        return self.coarse() + self.M_asm()

    def M_deflated(self):  # eq. 4
        Q = self.coarse()
        return Q + self.M_ras() @ (np.eye(self.n) - self.A @ Q)

    def pou(self):
        return sum(R.T @ D @ R for R, D in zip(self.R, self.D))
