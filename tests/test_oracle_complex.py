"""Pins of the oracle's complex path (the paper's Notation takes A complex:
moduli in Definition 1, adjoints in R_0^H and in the inner products).

Each check ties the complex path to something other than itself: the dense
tier (explicit matrices, QZ, SVD projectors; no shared code), the real path
through a unitary diagonal change of variables (the method is invariant under
it, and the real path is pinned by the worked examples), the Section 3.2
bound on a Hermitian positive definite matrix, the deflation identity of
eq. 4 and brute-force least squares for GMRES."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import workloads as W
from oracle import dense as OD
from oracle import schwarz as OS


def same_eigs(a, b, rtol):
    a, b = np.asarray(a), list(np.asarray(b))
    assert len(a) == len(b)
    for x in a:
        j = int(np.argmin([abs(x - y) for y in b]))
        assert abs(x - b[j]) <= rtol * max(abs(x), 1e-300), (x, b[j])
        b.pop(j)


def complex_problems():
    out = []
    A = W.convdiff2d_complex(12, 0.01, eta=0.3, omega=2.0, phase_seed=7).to_scipy()
    out.append(("zcd12-3x3-d1", A, W.block_partition_2d(12, 3), 9, 1, 4))
    A = W.convdiff2d_complex(13, 0.02, eta=0.5, omega=1.0, phase_seed=3).to_scipy()
    out.append(("zcd13-3x3-d2", A, W.block_partition_2d(13, 3), 9, 2, 5))
    # omega = 0, complex x-couplings, real y-couplings, Neumann in x: the
    # middle strips float
    A = W.convdiff2d_complex(12, 0.02, eta=0.5, eta_y=0.0, neumann_x=True).to_scipy()
    out.append(("zcd12-float-strips-d1", A, W.strip_partition(12, 3), 4, 1, 3))
    A = W.magnetic_laplace2d(12, 1.7).to_scipy()
    out.append(("mag12-3x3-d1", A, W.block_partition_2d(12, 3), 9, 1, 4))
    # as the floating case with omega > 0: the real parts of the row sums of
    # the splittings vanish, the imaginary parts (omega h^2) do not: no kernel
    A = W.convdiff2d_complex(12, 0.02, eta=0.5, eta_y=0.0, omega=2.0, neumann_x=True).to_scipy()
    out.append(("zcd12-shifted-strips-d1", A, W.strip_partition(12, 3), 4, 1, 3))
    return out


PROBLEMS = complex_problems()


def _dense_variant(D, variant):
    return {"asm": D.M_asm, "ras": D.M_ras, "additive-asm": D.M_additive,
            "additive-ras": lambda: D.coarse() + D.M_ras(), "deflated": D.M_deflated}[variant]()


def _crand(n, seed, k=None):
    g = np.random.default_rng(seed)
    shape = n if k is None else (n, k)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def test_problems_are_genuinely_complex():
    """The families exercise what real input cannot: complex off-diagonal
    entries, a floating subdomain whose left null vector (adjoint) is not
    real, and a Hermitian matrix."""
    for name, A, part, N, delta, nev in PROBLEMS:
        off = A - sp.diags(A.diagonal())
        assert np.abs(off.data.imag).max() > 1e-3, name
    A = PROBLEMS[3][1]
    assert abs(A - A.conj().T).max() == 0.0
    P = OS.TwoLevelSchwarz(*PROBLEMS[2][1:], keep_local=True)
    k = [e["kernel"] for e in P.eig]
    assert k == [0, 1, 1, 0], k
    P5 = OS.TwoLevelSchwarz(*PROBLEMS[4][1:])
    assert [e["kernel"] for e in P5.eig] == [0, 0, 0, 0]
    At = P.local[1]["At"].toarray()
    U, sig, Vh = np.linalg.svd(At)
    ell = U[:, -1]
    assert sig[-1] < 1e-12 * sig[0]
    assert np.abs(ell / ell[np.argmax(np.abs(ell))]).min() > 0  # nonzero entries
    assert np.abs((ell / ell[0]).imag).max() > 1e-3  # not a real vector up to scale


@pytest.mark.parametrize("case", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_complex_tiers_agree(case):
    """QZ on the restricted pencil with SVD projectors (dense tier) against
    the scalable tier: same kernel dimension, nev_i, selected eigenvalues,
    spans, and the same M^{-1} for every variant of Section 2."""
    name, A, part, N, delta, nev = case
    D = OD.DenseSchwarz(A, part, N, delta, nev)
    P = OS.TwoLevelSchwarz(A, part, N, delta, nev)
    assert P.n0 == D.n0 and P.n0 > 0
    for i in range(N):
        e_d, e_s = D.eig[i], P.eig[i]
        assert e_d["kernel"] == e_s["kernel"]
        assert e_d["Z"].shape[1] == e_s["Z"].shape[1]
        same_eigs(e_d["lam_sel"], e_s["lam_sel"], 1e-9)
        assert sla.subspace_angles(e_d["Z"], e_s["Z"]).max() < 1e-8
    r = _crand(A.shape[0], 1, 2)
    for variant in ("deflated", "ras", "asm", "additive-asm", "additive-ras"):
        Pv = P if variant == "deflated" else OS.TwoLevelSchwarz(A, part, N, delta, nev, variant=variant)
        ref = _dense_variant(D, variant) @ r
        np.testing.assert_allclose(Pv.apply(r), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("variant", ["deflated", "additive-asm", "ras"])
def test_unitary_change_of_variables_reduces_to_real_path(variant):
    """A' = U A U^H with U = diag(exp(i theta)) keeps every modulus, so the
    splittings, the eigenvalues of eq. 5 and nev_i are those of the real A,
    the coarse space is U Z, and M'^{-1} = U M^{-1} U^H; GMRES is unitarily
    invariant: the same iterations and x' = U x.  A transposed instead of a
    conjugated product anywhere breaks this."""
    A0 = W.convdiff2d(12, 0.02).to_scipy()
    part = W.block_partition_2d(12, 2)
    th = np.random.default_rng(11).uniform(0, 2 * np.pi, A0.shape[0])
    U = sp.diags(np.exp(1j * th))
    A1 = (U @ A0 @ U.conj().T).tocsr()
    P0 = OS.TwoLevelSchwarz(A0, part, 4, 2, 5, variant=variant)
    P1 = OS.TwoLevelSchwarz(A1, part, 4, 2, 5, variant=variant)
    assert list(P1.nev_i) == list(P0.nev_i)
    for e0, e1 in zip(P0.eig, P1.eig):
        same_eigs(e1["lam_sel"], e0["lam_sel"], 1e-9)
    r = W.rhs(A0.shape[0], 3)
    z0 = P0.apply(r)
    np.testing.assert_allclose(P1.apply(U @ r), U @ z0, rtol=0, atol=1e-12 * np.abs(z0).max())
    b = W.rhs(A0.shape[0], 4)
    x0, i0 = OS.gmres(A0, b, P0.apply, restart=10, rtol=1e-9)
    x1, i1 = OS.gmres(A1, U @ b, P1.apply, restart=10, rtol=1e-9)
    assert i1["its"] == i0["its"] and i1["status"] == OS.OK
    np.testing.assert_allclose(x1, U @ x0, rtol=0, atol=1e-9 * np.abs(x0).max())


def test_hermitian_unit_eigenvalues_and_condition_bound():
    """Hermitian positive definite, diagonally dominant A (Lemma 1): every
    finite nonzero eigenvalue of eq. 5 is real and >= 1, and the Section 3.2
    bound kappa(M_additive^{-1} A) <= (k_c + 1)(2 + (2 k_c + 1) k_m / tau) holds
    with 1/tau the largest eigenvalue left out; with a weak field (close to
    the singular Neumann-like limit) the coarse space also lowers kappa."""
    A = W.magnetic_laplace2d(16, 0.25).to_scipy()  # weak field: nearly singular like the Laplacian
    part = W.block_partition_2d(16, 4)
    N, delta, nev = 16, 1, 4
    D = OD.DenseSchwarz(A, part, N, delta, nev)
    for e in D.eig:
        nz = e["lam_all"][np.abs(e["lam_all"]) > 1e-8]
        assert np.abs(nz.imag).max() < 1e-9 and nz.real.min() >= 1 - 1e-9
    Ad = A.toarray()
    ev = np.linalg.eigvals(D.M_additive() @ Ad)
    assert np.abs(ev.imag).max() < 1e-9 * np.abs(ev).max()
    kappa = ev.real.max() / ev.real.min()
    cover = np.zeros(A.shape[0], int)
    omegas = [set(np.concatenate([I, G])) for I, G, _ in D.sets]
    for om in omegas:
        cover[list(om)] += 1
    km = cover.max()
    colour = {}
    for i in range(N):
        used = {colour[j] for j in colour if omegas[i] & omegas[j]}
        colour[i] = min(set(range(N + 1)) - used)
    kc = max(colour.values()) + 1
    inv_tau = max(np.sort(np.abs(e["lam_all"]))[::-1][e["Z"].shape[1] - e["kernel"]] for e in D.eig)
    assert kappa <= (kc + 1) * (2 + (2 * kc + 1) * km * inv_tau)
    ev1 = np.linalg.eigvals(D.M_asm() @ Ad).real
    assert ev1.max() / ev1.min() > kappa


@pytest.mark.parametrize("case", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_complex_deflation_identity(case):
    """eq. 4: M^{-1} A Z = Z and Z^H (r - A R_0^H A_00^{-1} R_0 r) = 0."""
    name, A, part, N, delta, nev = case
    P = OS.TwoLevelSchwarz(A, part, N, delta, nev)
    Z = P.Z.toarray()
    np.testing.assert_allclose(P.apply(A @ Z), Z, rtol=0, atol=1e-11 * np.abs(Z).max())
    r = _crand(A.shape[0], 2)
    t = r - A @ P.coarse_correction(r)
    assert np.abs(Z.conj().T @ t).max() <= 1e-12 * np.abs(r).max() * np.sqrt(A.shape[0])


def test_complex_gmres_minimal_residual_and_direct_solve():
    """Within a cycle the complex GMRES residual equals the least-squares
    minimum over the Krylov space (brute force), FGMRES equals GMRES for a
    fixed preconditioner, and the converged x matches a dense solve within
    kappa * rtol."""
    A = W.convdiff2d_complex(9, 0.02, eta=0.4, omega=3.0, phase_seed=5).to_scipy()
    n = A.shape[0]
    part = W.block_partition_2d(9, 3)
    P = OS.TwoLevelSchwarz(A, part, 9, 1, 2)
    b = _crand(n, 6)
    Ad = A.toarray()
    AM = Ad @ np.column_stack([P.apply(e.astype(complex)) for e in np.eye(n)])
    for k in range(1, 7):
        x, info = OS.gmres(A, b, P.apply, restart=30, rtol=0.0, fixed_iters=k)
        K = np.column_stack([np.linalg.matrix_power(AM, j) @ b for j in range(k)])
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(AM @ Q, b, rcond=None)
        best = np.linalg.norm(b - AM @ Q @ y)
        assert abs(np.linalg.norm(b - Ad @ x) - best) <= 1e-10 * np.linalg.norm(b)
        assert abs(info["history"][-1] * np.linalg.norm(b) - best) <= 1e-10 * np.linalg.norm(b)
    x1, _ = OS.gmres(A, b, P.apply, restart=4, rtol=0, fixed_iters=9)
    x2, _ = OS.gmres(A, b, P.apply, restart=4, rtol=0, fixed_iters=9, flexible=True)
    np.testing.assert_allclose(x1, x2, rtol=1e-10, atol=1e-12)
    x, info = OS.gmres(A, b, P.apply, restart=30, rtol=1e-8)
    assert info["status"] == OS.OK
    xs = np.linalg.solve(Ad, b)
    assert np.linalg.norm(x - xs) <= np.linalg.cond(Ad) * 1e-8 * np.linalg.norm(xs)


def test_real_input_unchanged_by_complex_branches():
    """Real A takes the real arithmetic: real coarse space and E, and the
    same M^{-1} whether the right-hand side is real or split into parts."""
    A = W.convdiff2d(12, 0.01).to_scipy()
    part = W.block_partition_2d(12, 3)
    P = OS.TwoLevelSchwarz(A, part, 9, 1, 5)
    assert not np.iscomplexobj(P.Z.data) and not np.iscomplexobj(P.E)
    r = W.rhs(A.shape[0], 2)
    assert P.apply(r).dtype == np.float64
