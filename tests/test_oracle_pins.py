"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: hand-derived
worked examples (tests/golden), closed forms, identities implied by eq. 1-6
and Definition 1, brute force on tiny inputs, and cross-checks between the
literal dense tier and the scalable sparse tier (which share no code)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.csgraph as csg
import scipy.sparse.linalg as spla

import workloads as W
from oracle import dense as OD
from oracle import schwarz as OS


def assert_same_eigs(a, b, rtol):
    """Same multiset of (complex) eigenvalues up to rtol (nearest matching)."""
    a, b = np.asarray(a), list(np.asarray(b))
    assert len(a) == len(b)
    for x in a:
        j = int(np.argmin([abs(x - y) for y in b]))
        assert abs(x - b[j]) <= rtol * max(abs(x), 1e-300), (x, b[j])
        b.pop(j)


def lap1d(n):
    return 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)


def small_problems():
    """(name, A scipy csr, part, nparts, overlap, nev) tiny cases covering SPD,
    nonsymmetric, floating subdomains, overlap 1 and 2, ragged partitions."""
    out = []
    A = W.laplace2d(12).to_scipy()
    out.append(("lap12-3x3-d1", A, W.block_partition_2d(12, 3), 9, 1, 4))
    out.append(("lap12-strips-d2", A, W.strip_partition(12, 3), 4, 2, 3))
    A = W.convdiff2d(12, nu=0.01).to_scipy()
    out.append(("cd12-3x3-d1", A, W.block_partition_2d(12, 3), 9, 1, 5))
    A = W.convdiff2d(13, nu=0.02).to_scipy()
    out.append(("cd13-3x3-d2", A, W.block_partition_2d(13, 3), 9, 2, 4))
    A = W.diffusion2d_lognormal(12, seed=3, npad=64).to_scipy()
    out.append(("ln12-2x2-d1", A, W.block_partition_2d(12, 2), 4, 1, 3))
    A = W.convdiff3d(6, nu=0.05).to_scipy()
    out.append(("cd3d6-2x2x2-d1", A, W.block_partition_3d(6, 2, 2, 2), 8, 1, 4))
    return out


PROBLEMS = small_problems()


# ---------------------------------------------------------------------------
# worked examples
# ---------------------------------------------------------------------------

def test_golden_1d_two_parts(golden):
    g = golden("oned_two_parts.txt")
    n = int(g["n"][0])
    A = lap1d(n)
    part = np.array(g["part"], dtype=np.int32)
    P = OS.TwoLevelSchwarz(sp.csr_matrix(A), part, 2, 1, 1, keep_local=True)
    D = OD.DenseSchwarz(A, part, 2, 1, 1)
    for i in range(2):
        assert list(P.subs[i].omega) == [int(v) for v in g[f"omega{i}"]]
        np.testing.assert_array_equal(P.local[i]["s"], g[f"s{i}"])
        np.testing.assert_array_equal(D.s[i], g[f"s{i}"])
        lam = P.eig[i]["lam_sel"]
        assert np.allclose(lam, g[f"lambda{i}"], rtol=1e-12)
        assert np.allclose(D.eig[i]["lam_all"][0], g[f"lambda{i}"], rtol=1e-12)
        u = np.array(g[f"u{i}"])
        z = P.eig[i]["Z"][:, 0]
        assert abs(abs(z @ u) - np.linalg.norm(z) * np.linalg.norm(u)) < 1e-12 * np.linalg.norm(u)
    np.testing.assert_array_equal(P.local[0]["At"].toarray().ravel(), g["atilde0"])
    np.testing.assert_allclose(P.E.ravel(), g["E"], rtol=1e-14)
    Z = D.R0H / np.linalg.norm(D.R0H, axis=0)
    np.testing.assert_allclose((Z.T @ A @ Z).ravel(), g["E"], rtol=1e-14)


def test_golden_1d_three_parts_floating(golden):
    g = golden("oned_three_parts_floating.txt")
    n = int(g["n"][0])
    A = lap1d(n)
    part = np.array(g["part"], dtype=np.int32)
    P = OS.TwoLevelSchwarz(sp.csr_matrix(A), part, 3, 1, 2, keep_local=True)
    D = OD.DenseSchwarz(A, part, 3, 1, 2)
    assert list(P.subs[1].omega) == [int(v) for v in g["omega1"]]
    np.testing.assert_array_equal(P.local[1]["s"], g["s1"])
    np.testing.assert_array_equal(P.local[1]["At"].toarray().ravel(), g["atilde1"])
    np.testing.assert_array_equal(D.Atii[1].ravel(), g["atilde1"])
    assert [e["kernel"] for e in P.eig] == [int(v) for v in g["kernel"]]
    assert [e["kernel"] for e in D.eig] == [int(v) for v in g["kernel"]]
    # nev = 2 on the floating subdomain: kernel vector + top eigenvector
    assert np.allclose(P.eig[1]["lam_sel"], g["lambda1"], rtol=1e-12)
    assert np.allclose(D.eig[1]["lam_all"][0], g["lambda1"], rtol=1e-12)
    u = np.array(g["u1"])
    z = P.eig[1]["Z"][:, 1]
    assert abs(abs(z @ u) - np.linalg.norm(z) * np.linalg.norm(u)) < 1e-10 * np.linalg.norm(u)
    assert np.allclose(np.abs(P.eig[1]["Z"][:, 0]), 1 / np.sqrt(5))
    for i in (0, 2):
        assert np.allclose(P.eig[i]["lam_sel"][0], g[f"lambda{i}"], rtol=1e-12)


# ---------------------------------------------------------------------------
# Section 2: subdomains and partition of unity
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_subdomains_brute_force_distance(case):
    """Omega_Gamma_i = nodes at graph distance 1..delta from Omega_Ii (shortest
    paths in the graph of A + A^T), layer = distance; ascending order."""
    name, A, part, N, delta, nev = case
    G = sp.csr_matrix((np.abs(A) + np.abs(A.T)) != 0, dtype=float)
    G.setdiag(0)
    G.eliminate_zeros()
    dist_all = csg.shortest_path(G, unweighted=True)
    subs = OS.subdomains(A, part, N, delta)
    sets = OD.overlapping_sets(A.toarray(), part, N, delta)
    for i, sub in enumerate(subs):
        I = np.flatnonzero(part == i)
        d = dist_all[I].min(axis=0)
        gam = np.flatnonzero((d >= 1) & (d <= delta))
        np.testing.assert_array_equal(sub.interior, I)
        np.testing.assert_array_equal(sub.gamma, gam)
        np.testing.assert_array_equal(sub.layer, d[gam].astype(int))
        np.testing.assert_array_equal(sets[i][1], gam)
        np.testing.assert_array_equal(sets[i][2], d[gam].astype(int))


@pytest.mark.parametrize("case", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_partition_of_unity(case):
    """P1: sum_i R_i^T D_i R_i = I exactly (Section 2)."""
    name, A, part, N, delta, nev = case
    D = OD.DenseSchwarz(A, part, N, delta, 0)
    np.testing.assert_array_equal(D.pou(), np.eye(A.shape[0]))
    subs = OS.subdomains(A, part, N, delta)
    acc = np.zeros(A.shape[0])
    for sub in subs:
        acc[sub.omega] += OS.partition_of_unity(sub)
    np.testing.assert_array_equal(acc, 1.0)


def test_bfs_partition_brute_force():
    """Multi-source BFS owner = argmin over seeds of (graph distance, seed id)."""
    A = W.convdiff3d(8, nu=0.05).to_scipy()
    seeds = W.bfs_seeds_3d(8, (4, 4, 2), seed=5)
    part = OS.bfs_partition(A, seeds)
    G = OS.adjacency(A)
    dist = csg.shortest_path(G, unweighted=True, indices=seeds)
    key = dist * len(seeds) + np.arange(len(seeds))[:, None]
    np.testing.assert_array_equal(part, np.argmin(key, axis=0))


# ---------------------------------------------------------------------------
# Section 3.1: Definition 1 and Lemma 1
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_block_splitting_tiers_agree_bitwise(case):
    name, A, part, N, delta, nev = case
    D = OD.DenseSchwarz(A, part, N, delta, 0)
    subs = OS.subdomains(A, part, N, delta)
    for i, sub in enumerate(subs):
        A_ii, s, At = OS.block_splitting(A, sub)
        np.testing.assert_array_equal(A_ii.toarray(), D.Aii[i])
        np.testing.assert_allclose(s, D.s[i], rtol=1e-15, atol=0)
        np.testing.assert_allclose(At.toarray(), D.Atii[i], rtol=1e-15, atol=1e-300)


@pytest.mark.parametrize("seed", [0, 1])
def test_lemma1_hpsd_splitting(seed):
    """P2 (Lemma 1): for SPD diagonally dominant A, the prolonged splitting
    Atilde_i = R_i^T Atilde_ii R_i and A - Atilde_i are both PSD."""
    rng = np.random.default_rng(seed)
    n = 40
    M = sp.random(n, n, density=0.12, random_state=seed).toarray()
    M = -np.abs(M + M.T) * (rng.uniform(size=(n, n)) > 0.3)
    M = (M + M.T) / 2
    np.fill_diagonal(M, 0)
    A = M.copy()
    np.fill_diagonal(A, np.abs(M).sum(1) + rng.uniform(0, 0.3, n))
    # also flip some off-diagonal signs: Lemma 1 only needs diagonal dominance
    S = np.sign(rng.uniform(-1, 1, (n, n)))
    S = np.triu(S, 1)
    S = S + S.T + np.eye(n)
    A = A * S
    part = (np.arange(n) * 4) // n
    D = OD.DenseSchwarz(A, part, 4, 1, 0)
    eps = 1e-12 * np.abs(A).max()
    for i in range(4):
        Ati = D.R[i].T @ D.Atii[i] @ D.R[i]
        assert np.linalg.eigvalsh(Ati).min() >= -eps
        assert np.linalg.eigvalsh(A - Ati).min() >= -eps


def test_floating_rows_sum_to_zero():
    """P3: for a zero-row-sum M-matrix, the overlap rows of the splitting
    recover the full row sum, so interior (floating) subdomains satisfy
    Atilde 1 = 0 while boundary-touching ones do not (Definition 1)."""
    A = W.convdiff2d(24, nu=0.01).to_scipy()
    part = W.block_partition_2d(24, 3)
    subs = OS.subdomains(A, part, 9, 2)
    for i, sub in enumerate(subs):
        _, _, At = OS.block_splitting(A, sub)
        r = At @ np.ones(sub.size)
        floating = i == 4
        assert (np.abs(r).max() <= 1e-13 * np.abs(At).sum(1).max()) == floating
        assert OS.kernel_dimension(At) == int(floating)


# ---------------------------------------------------------------------------
# Section 3.2: eq. 5 and eq. 6
# ---------------------------------------------------------------------------

def _pencil_residual_ok(A_ii, At, nI, lam, Z, kernel):
    """P4: ||Pi B Pi u - lambda Atilde u|| <= 1e-10 (||Pi B Pi||_1 + |lambda| ||Atilde||_1) ||u||
    with Pi built here from an SVD of Atilde (not from the oracle's LU)."""
    A_ii, At = A_ii.toarray(), At.toarray()
    ni = A_ii.shape[0]
    d = np.r_[np.ones(nI), np.zeros(ni - nI)]
    B = d[:, None] * A_ii * d[None, :]
    U, sig, Vh = np.linalg.svd(At)
    r = int(np.sum(sig > 1e-12 * sig[0]))
    Ql = U[:, r:]
    Pi = np.eye(ni) - Ql @ Ql.T
    PBP = Pi @ B @ Pi
    return PBP, np.linalg.norm(PBP, 1), np.linalg.norm(At, 1), At


@pytest.mark.parametrize("case", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_eigenpair_residuals(case):
    name, A, part, N, delta, nev = case
    subs = OS.subdomains(A, part, N, delta)
    for sub in subs:
        A_ii, s, At = OS.block_splitting(A, sub)
        res = OS.local_eigenproblem(A_ii, At, sub.n_interior, nev)
        PBP, nb, na, Atd = _pencil_residual_ok(A_ii, At, sub.n_interior, None, None, None)
        # recover complex eigenvectors from the real basis: check the span is
        # invariant, i.e. PBP Z = Atilde Z Theta for a small matrix Theta
        Z = res["Z"][:, res["kernel"]:]
        if Z.shape[1] == 0:
            continue
        lhs = PBP @ Z
        rhs = Atd @ Z
        Theta, *_ = np.linalg.lstsq(rhs, lhs, rcond=None)
        resid = np.linalg.norm(lhs - rhs @ Theta, 1)
        lam_max = np.abs(res["lam_sel"]).max()
        assert resid <= 1e-10 * (nb + lam_max * na) * np.linalg.norm(Z, 1)
        assert_same_eigs(np.linalg.eigvals(Theta), res["lam_sel"], 1e-9)


@pytest.mark.parametrize("case", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_dense_and_scalable_tiers_agree(case):
    """P5: QZ on the restricted pencil (dense tier) vs ARPACK on T (scalable
    tier): same selected eigenvalues, same nev_i, same spans, same M^{-1}."""
    name, A, part, N, delta, nev = case
    D = OD.DenseSchwarz(A, part, N, delta, nev)
    P = OS.TwoLevelSchwarz(A, part, N, delta, nev)
    assert P.n0 == D.n0
    for i in range(N):
        e_d, e_s = D.eig[i], P.eig[i]
        assert e_d["kernel"] == e_s["kernel"]
        assert e_d["Z"].shape[1] == e_s["Z"].shape[1]
        assert_same_eigs(e_d["lam_sel"], e_s["lam_sel"], 1e-9)
        if e_d["Z"].shape[1]:
            ang = sla.subspace_angles(e_d["Z"], e_s["Z"])
            assert ang.max() < 1e-8
    r = np.random.default_rng(1).standard_normal(A.shape[0])
    Md = D.M_deflated()
    np.testing.assert_allclose(P.apply(r), Md @ r, rtol=0, atol=1e-12 * np.abs(Md @ r).max())


def test_unit_eigenvalue_count_and_spd_bound():
    """P6 (derived from eq. 5 under the Boolean D): when K_i = {0}, exactly
    n_I - m eigenvalues equal 1 (m = number of first-layer overlap nodes) and,
    for SPD A, every finite nonzero eigenvalue is >= 1."""
    for A, part, N, delta, spd in [
        (W.laplace2d(16).to_scipy(), W.strip_partition(16, 4), 4, 1, True),
        (W.laplace2d(16).to_scipy(), W.strip_partition(16, 4), 4, 2, True),
        (W.convdiff2d(16, 0.01).to_scipy(), W.strip_partition(16, 4), 4, 1, False),
        (W.convdiff2d(16, 0.01).to_scipy(), W.strip_partition(16, 4), 4, 2, False),
    ]:
        D = OD.DenseSchwarz(A, part, N, delta, 1)
        for i, (I, Gam, layer) in enumerate(D.sets):
            e = D.eig[i]
            assert e["kernel"] == 0
            lam = e["lam_all"]
            m = int(np.sum(layer == 1))
            n_one = int(np.sum(np.abs(lam - 1) < 1e-8))
            assert n_one == len(I) - m
            if spd:
                nz = lam[np.abs(lam) > 1e-8]
                assert np.all(np.abs(nz.imag) < 1e-10) and nz.real.min() >= 1 - 1e-10


# ---------------------------------------------------------------------------
# Section 2 eq. 1-4 and the solver
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("case", PROBLEMS[:4], ids=[p[0] for p in PROBLEMS[:4]])
def test_deflation_identity(case):
    """P7: M^{-1} A Z = Z for eq. 4, and R_0 (r - A R_0^H A_00^{-1} R_0 r) = 0."""
    name, A, part, N, delta, nev = case
    P = OS.TwoLevelSchwarz(A, part, N, delta, nev)
    Z = P.Z.toarray()
    MAZ = P.apply(A @ Z)
    np.testing.assert_allclose(MAZ, Z, rtol=0, atol=1e-12 * np.abs(Z).max())
    r = np.random.default_rng(2).standard_normal(A.shape[0])
    t = r - A @ P.coarse_correction(r)
    assert np.abs(Z.T @ t).max() <= 1e-12 * np.abs(r).max() * np.sqrt(A.shape[0])


def test_special_cases():
    """P9: N = 1 => M^{-1} = A^{-1} and GMRES takes one iteration; nev = 0 =>
    eq. 4 reduces to eq. 3 (RAS); overlap 0 => block Jacobi."""
    A = W.convdiff2d(10, 0.02).to_scipy()
    n = A.shape[0]
    r = np.random.default_rng(3).standard_normal(n)
    P = OS.TwoLevelSchwarz(A, np.zeros(n, np.int32), 1, 1, 2)
    np.testing.assert_allclose(P.apply(r), spla.spsolve(A.tocsc(), r), rtol=1e-12, atol=1e-12)
    x, info = OS.gmres(A, r, P.apply, restart=30, rtol=1e-8)
    assert info["its"] == 1
    part = W.block_partition_2d(10, 2)
    P0 = OS.TwoLevelSchwarz(A, part, 4, 2, 0)
    Pr = OS.TwoLevelSchwarz(A, part, 4, 2, 0, variant="ras")
    np.testing.assert_array_equal(P0.apply(r), Pr.apply(r))
    Pj = OS.TwoLevelSchwarz(A, part, 4, 0, 0, variant="ras")
    Ad = A.toarray()
    x = np.zeros(n)
    for i in range(4):
        I = np.flatnonzero(part == i)
        x[I] = np.linalg.solve(Ad[np.ix_(I, I)], r[I])
    np.testing.assert_allclose(Pj.apply(r), x, rtol=1e-12, atol=1e-12)


def test_spd_condition_bound():
    """P10 (Section 3.2): kappa_2(M_additive^{-1} A) <= (k_c + 1)(2 + (2 k_c + 1) k_m / tau)
    with 1/tau taken as the largest eigenvalue left out of the coarse space."""
    A = W.laplace2d(16).to_scipy()
    part = W.block_partition_2d(16, 4)
    N, delta, nev = 16, 1, 4
    D = OD.DenseSchwarz(A, part, N, delta, nev)
    Ad = A.toarray()
    M = D.M_additive()
    ev = np.linalg.eigvals(M @ Ad).real
    kappa = ev.max() / ev.min()
    # k_m: max number of subdomains sharing a row; k_c: greedy colouring of the
    # subdomain overlap graph (any valid colouring gives a valid bound)
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
    inv_tau = 0.0
    for e in D.eig:
        k = e["Z"].shape[1] - e["kernel"]
        lam = np.sort(np.abs(e["lam_all"]))[::-1]
        inv_tau = max(inv_tau, lam[k])
    bound = (kc + 1) * (2 + (2 * kc + 1) * km * inv_tau)
    assert kappa <= bound
    # and the coarse space does help: the one-level ASM is worse conditioned
    ev1 = np.linalg.eigvals(D.M_asm() @ Ad).real
    assert ev1.max() / ev1.min() > kappa


def test_gmres_minimal_residual_and_direct_solve():
    """P11: within a cycle the GMRES residual equals the least-squares minimum
    over the Krylov space (brute force), and the converged x matches a dense
    direct solve within kappa * rtol."""
    A = W.convdiff2d(9, 0.02).to_scipy()
    n = A.shape[0]
    part = W.block_partition_2d(9, 3)
    P = OS.TwoLevelSchwarz(A, part, 9, 1, 2)
    b = W.rhs(n, 0)
    Ad = A.toarray()
    Md = np.column_stack([P.apply(e) for e in np.eye(n)])
    AM = Ad @ Md
    for k in range(1, 6):
        x, info = OS.gmres(A, b, P.apply, restart=30, rtol=0.0, fixed_iters=k)
        K = np.column_stack([np.linalg.matrix_power(AM, j) @ b for j in range(k)])
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(AM @ Q, b, rcond=None)
        best = np.linalg.norm(b - AM @ Q @ y)
        assert abs(np.linalg.norm(b - Ad @ x) - best) <= 1e-10 * np.linalg.norm(b)
    x, info = OS.gmres(A, b, P.apply, restart=30, rtol=1e-8)
    assert info["status"] == OS.OK
    xs = np.linalg.solve(Ad, b)
    kappa = np.linalg.cond(Ad)
    assert np.linalg.norm(x - xs) <= kappa * 1e-8 * np.linalg.norm(xs)
    hist = info["history"]
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 1))


def test_flexible_equals_standard_for_fixed_preconditioner():
    A = W.convdiff2d(20, 0.01).to_scipy()
    part = W.block_partition_2d(20, 2)
    P = OS.TwoLevelSchwarz(A, part, 4, 2, 3)
    b = W.rhs(A.shape[0], 1)
    x1, i1 = OS.gmres(A, b, P.apply, restart=7, rtol=0, fixed_iters=12)
    x2, i2 = OS.gmres(A, b, P.apply, restart=7, rtol=0, fixed_iters=12, flexible=True)
    np.testing.assert_allclose(x1, x2, rtol=1e-10, atol=1e-12)


def test_c1_full_size_converges():
    """The 64 x 64 Laplacian in 8 strips (overlap 1, nev 4) end to end:
    converges to 1e-8, coarse size 8 x 4, solution within kappa * rtol of a
    sparse direct solve."""
    A, part, N, opts = W.config("c1_laplace2d_64_strips8")
    As = A.to_scipy()
    b = W.rhs(A.n, 0)
    x, info, P = OS.solve(As, b, part, N, opts["overlap"], opts["nev"], restart=30, rtol=1e-8)
    assert info["status"] == OS.OK and info["relres"] <= 1e-8
    assert P.n0 == 32 and all(P.nev_i == 4)
    assert all(e["kernel"] == 0 for e in P.eig)
    xs = spla.spsolve(As.tocsc(), b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-5
    # the coarse space helps: one-level RAS needs more iterations
    x1, info1, _ = OS.solve(As, b, part, N, opts["overlap"], 0, restart=30, rtol=1e-8, variant="ras")
    assert info1["its"] > info["its"]


# ---------------------------------------------------------------------------
# eq. 1 - eq. 4 as explicit matrices, and the tau rule of eq. 6
# ---------------------------------------------------------------------------

VARIANTS = [("asm", "asm"), ("ras", "ras"), ("additive-asm", "additive"),
            ("additive-ras", "additive_ras"), ("deflated", "deflated")]


def _golden_matrix(g, key):
    n = int(g["n"][0])
    return np.array(g[key]).reshape(n, n) / g[key + "_den"][0]


def _dense_variant(D, variant):
    return {"asm": D.M_asm, "ras": D.M_ras, "additive-asm": D.M_additive,
            "additive-ras": lambda: D.coarse() + D.M_ras(), "deflated": D.M_deflated}[variant]()


@pytest.mark.parametrize("variant,key", VARIANTS, ids=[v[0] for v in VARIANTS])
def test_golden_1d_variants(golden, variant, key):
    """Both tiers reproduce the hand-derived matrices of eq. 1 (ASM), eq. 3
    (RAS), eq. 2 (additive two-level), the additive restricted form and eq. 4
    (deflated) on the 1D two-part example, and the coarse correction
    R_0^H A_00^{-1} R_0 (nev = 1)."""
    g = golden("oned_two_parts_variants.txt")
    n = int(g["n"][0])
    A = sp.csr_matrix(lap1d(n))
    part = np.array(g["part"], dtype=np.int32)
    ref = _golden_matrix(g, key)
    P = OS.TwoLevelSchwarz(A, part, 2, 1, 1, variant=variant)
    np.testing.assert_allclose(P.apply(np.eye(n)), ref, rtol=0, atol=1e-14)
    D = OD.DenseSchwarz(A, part, 2, 1, 1)
    np.testing.assert_allclose(_dense_variant(D, variant), ref, rtol=0, atol=1e-14)
    Q = _golden_matrix(g, "coarse")
    np.testing.assert_allclose(D.coarse(), Q, rtol=0, atol=1e-14)
    np.testing.assert_allclose(P.coarse_correction(np.eye(n)) if P.n0 else Q, Q, rtol=0, atol=1e-14)


def test_golden_1d_tau_selection(golden):
    """eq. 6: nev caps the count (with the cluster rule), tau keeps only
    |lambda| > 1/tau.  Both tiers, all hand-derived cases; the tau = 0.3 space
    gives the nev = 1 preconditioner and an empty selection gives eq. 3."""
    g = golden("oned_two_parts_variants.txt")
    n = int(g["n"][0])
    A = sp.csr_matrix(lap1d(n))
    part = np.array(g["part"], dtype=np.int32)
    lam_all = np.array(g["lambda_all"])
    for key in ["select_a", "select_b", "select_c", "select_d", "select_e", "select_f"]:
        nev, tau, want = int(g[key][0]), g[key][1], int(g[key][2])
        P = OS.TwoLevelSchwarz(A, part, 2, 1, nev, tau=tau)
        assert list(P.nev_i) == [want, want], key
        D = OD.DenseSchwarz(A, part, 2, 1, nev, tau=tau)
        assert [e["Z"].shape[1] for e in D.eig] == [want, want], key
        assert len(OS.select_eigenvalues(lam_all, nev, tau)) == want, key
        for e in D.eig:
            assert np.abs(e["lam_all"].imag).max() < 1e-12
            np.testing.assert_allclose(np.sort(e["lam_all"].real)[::-1], lam_all, rtol=0, atol=1e-12)
            assert np.all(np.abs(e["lam_sel"]) > 1.0 / tau) if tau > 0 else True
    nev, tau, want = int(g["select_g"][0]), g["select_g"][1], int(g["select_g"][2])
    assert len(OS.select_eigenvalues(lam_all, nev, tau)) == want
    r = np.eye(n)
    P = OS.TwoLevelSchwarz(A, part, 2, 1, 3, tau=0.3)
    np.testing.assert_allclose(P.apply(r), _golden_matrix(g, "deflated"), rtol=0, atol=1e-14)
    P = OS.TwoLevelSchwarz(A, part, 2, 1, 3, tau=0.2)
    assert P.n0 == 0
    np.testing.assert_allclose(P.apply(r), _golden_matrix(g, "ras"), rtol=0, atol=1e-14)


@pytest.mark.parametrize("case", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_variants_tiers_agree(case):
    """The scalable tier's eq. 1, eq. 2 and additive restricted applies equal
    the dense tier's explicit matrices (sums of R_i^T A_ii^{-1} R_i formed with
    dense inverses) on every small problem."""
    name, A, part, N, delta, nev = case
    D = OD.DenseSchwarz(A, part, N, delta, nev)
    r = np.random.default_rng(4).standard_normal((A.shape[0], 2))
    for variant in ("asm", "additive-asm", "additive-ras"):
        P = OS.TwoLevelSchwarz(A, part, N, delta, nev, variant=variant)
        Md = _dense_variant(D, variant)
        ref = Md @ r
        np.testing.assert_allclose(P.apply(r), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def _tau_between(lam_sel, nev):
    """A threshold 1/tau halfway (in |lambda|) between two well separated
    consecutive selected eigenvalues, or None."""
    mags = np.sort(np.abs(lam_sel))[::-1]
    for k in range(1, len(mags)):
        if mags[k] < 0.9 * mags[k - 1]:
            return 2.0 / (mags[k] + mags[k - 1])
    return None


@pytest.mark.parametrize("case", PROBLEMS, ids=[p[0] for p in PROBLEMS])
def test_tau_selection_tiers_agree(case):
    """tau cut inside the selected spectrum: QZ on the restricted pencil (dense
    tier) and ARPACK on T (scalable tier) keep the same eigenvalues and span,
    all of them with |lambda| > 1/tau, and the applies of eq. 4 agree."""
    name, A, part, N, delta, nev = case
    D0 = OD.DenseSchwarz(A, part, N, delta, nev)
    taus = [t for t in (_tau_between(e["lam_sel"], nev) for e in D0.eig) if t]
    if not taus:
        pytest.skip("no well separated pair in the selected spectra")
    tau = float(np.median(taus))
    D = OD.DenseSchwarz(A, part, N, delta, nev, tau=tau)
    P = OS.TwoLevelSchwarz(A, part, N, delta, nev, tau=tau)
    assert P.n0 == D.n0 < D0.n0
    for i in range(N):
        e_d, e_s = D.eig[i], P.eig[i]
        assert e_d["Z"].shape[1] == e_s["Z"].shape[1]
        assert np.all(np.abs(e_s["lam_sel"]) > 1.0 / tau)
        lam_full = np.abs(D0.eig[i]["lam_sel"])
        assert len(e_d["lam_sel"]) == int(np.sum(lam_full > 1.0 / tau))
        assert_same_eigs(e_d["lam_sel"], e_s["lam_sel"], 1e-9)
        if e_d["Z"].shape[1]:
            assert sla.subspace_angles(e_d["Z"], e_s["Z"]).max() < 1e-8
    r = np.random.default_rng(5).standard_normal(A.shape[0])
    ref = D.M_deflated() @ r
    np.testing.assert_allclose(P.apply(r), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
