"""Parity of the complex path (ads_setup_complex, through the C interface)
with the oracle's complex path.

The library holds complex A in its real form (unknown j -> rows 2j, 2j + 1,
entry z -> [[re, -im], [im, re]]).  Compared here: the index maps and lumped
sums of Definition 1 (moduli) against the oracle's, expanded to the real
form; per subdomain twice the oracle's nev_i real coarse vectors whose span
is the real form of the oracle's complex coarse space (principal angles
<= 1e-7 rad with the eigensolver at 1e-12) and whose eigenvalues are the
oracle's with their conjugates (relative 1e-8); the apply of eq. 4 (and the
other variants) on complex vectors within 1e-9 of the oracle's; complex
GMRES iterations within +-1 and solutions within 1e-8 (or the residual
bound), fixed-iteration iterates within 1e-10."""
import re

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import workloads as W
from oracle import schwarz as OS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2201_02250_amd import ads  # noqa: E402

DEV = "cuda:0"


def real_form_cols(Wc):
    """Real form of the complex span of the columns of Wc: for each column w
    the interleaved arrays of w and i w."""
    n, m = Wc.shape
    out = np.zeros((2 * n, 2 * m))
    out[0::2, 0::2] = Wc.real
    out[1::2, 0::2] = Wc.imag
    out[0::2, 1::2] = -Wc.imag
    out[1::2, 1::2] = Wc.real
    return out


def crand(n, seed, k=None):
    g = np.random.default_rng(seed)
    shape = n if k is None else (n, k)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def inv_norm2_c(As):
    lu = spla.splu(sp.csc_matrix(As))
    n = As.shape[0]
    op = spla.LinearOperator((n, n), matvec=lambda v: lu.solve(lu.solve(np.ravel(v), trans="H")),
                             dtype=np.complex128)
    lam = spla.eigsh(op, k=1, which="LA", tol=1e-6, v0=np.ones(n, complex),
                     return_eigenvectors=False)[0]
    return 1.01 * float(np.sqrt(abs(lam)))


def solution_close(As, b, x, xo, label):
    e = float(np.linalg.norm(x - xo) / np.linalg.norm(xo))
    if e <= 1e-8:
        print(f"solution error vs oracle {label}: {e:.2e} (<= 1e-08)", flush=True)
        return
    bound = inv_norm2_c(As) * (np.linalg.norm(b - As @ x) + np.linalg.norm(b - As @ xo)) / np.linalg.norm(xo)
    print(f"solution error vs oracle {label}: {e:.2e} (residual bound {bound:.2e})", flush=True)
    assert e <= bound, (label, e, bound)


def same_eigs(a, b, rtol):
    a, b = np.asarray(a), list(np.asarray(b))
    assert len(a) == len(b), (len(a), len(b))
    for x in a:
        j = int(np.argmin([abs(x - y) for y in b]))
        assert abs(x - b[j]) <= rtol * max(abs(x), 1e-300), (x, b[j])
        b.pop(j)


CASES = [
    # name, matrix, part, nparts, overlap, nev
    ("zcd32-3x3-d2", lambda: W.convdiff2d_complex(32, 0.01, eta=0.3, omega=2.0, phase_seed=7),
     lambda: W.block_partition_2d(32, 3), 9, 2, 4),
    ("zcd40-4x4-d1", lambda: W.convdiff2d_complex(40, 0.005, eta=1.0, omega=5.0),
     lambda: W.block_partition_2d(40, 4), 16, 1, 5),
    ("mag32-3x3-d2", lambda: W.magnetic_laplace2d(32, 1.3, 0.01),
     lambda: W.block_partition_2d(32, 3), 9, 2, 4),
    ("zcd64-2x2-d2-general", lambda: W.convdiff2d_complex(64, 0.01, eta=0.5, omega=1.0,
                                                            phase_seed=2),
     lambda: W.block_partition_2d(64, 2), 4, 2, 3),
    # floating subdomains (the splitting has the complex constant as null
    # vector, span{1, i 1} in the real form): Neumann at x = 0, 1 and real
    # y-couplings, so the strips away from y = 0, 1 float (their lumped
    # couplings are real and negative); nonsymmetric, so the left null vector
    # comes from the transposed solve.  Strips m wide have real-form block
    # size 2 m + 1: 25 (two-ended register-resident factors), 97 (batched
    # block-step factors) and 265 (one-ended factors, general solves)
    ("zcd12-strips3-d1-float", lambda: W.convdiff2d_complex(12, 0.02, eta=0.5, eta_y=0.0,
                                                              neumann_x=True),
     lambda: W.strip_partition(12, 3), 4, 1, 3),
    ("zcd48-strips6-d1-float-s97", lambda: W.convdiff2d_complex(48, 0.02, eta=0.5, eta_y=0.0,
                                                                  neumann_x=True),
     lambda: W.strip_partition(48, 6), 8, 1, 3),
    # (nu 0.1: at nu 0.02 the adjoint null vector of these wide strips is
    # 4e-11 at the last unknown, where the splitting is regularised, and the
    # regularised solves of both sides keep only about 6 digits)
    ("zcd132-strips12-d1-float-s265", lambda: W.convdiff2d_complex(132, 0.1, eta=0.5, eta_y=0.0,
                                                                     neumann_x=True),
     lambda: W.strip_partition(132, 12), 11, 1, 3),
    # Hermitian (zero flux): the left null vector is the constant itself
    ("mag24-4x4-d2-float-hermitian", lambda: W.magnetic_laplace2d(24, 0.0),
     lambda: W.block_partition_2d(24, 4), 16, 2, 4),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_complex_setup_apply_solve_match_oracle(case):
    name, mk, mkp, N, delta, nev = case
    A = mk()
    part = mkp()
    As = A.to_scipy()
    n = A.n
    print(f"case {name}: n {n} complex, {N} parts, overlap {delta}, nev {nev}", flush=True)
    P = OS.TwoLevelSchwarz(As, part, N, delta, nev)
    ctx = ads.Context(A, part, N, delta, nev, eig_tol=1e-12)
    assert ctx.is_complex and ctx.n == n
    info = ctx.info
    # maps: the real form of the oracle's Omega_i, layers; lumped sums
    om, off, nI, lay = ads.ads_export_maps(ctx.ctx)
    s_gpu = ads.ads_export_splitting(ctx.ctx)
    for i, sub in enumerate(P.subs):
        omc = sub.omega
        want = np.stack([2 * omc, 2 * omc + 1], axis=1).ravel()
        got = om[off[i]:off[i + 1]]
        np.testing.assert_array_equal(got, want)
        assert nI[i] == 2 * sub.n_interior
        _, s_or, _ = OS.block_splitting(As, sub)
        s_g = s_gpu[off[i]:off[i + 1]][2 * sub.n_interior:]
        np.testing.assert_allclose(s_g[0::2], s_or, rtol=1e-15, atol=0)  # hypot rounding
        np.testing.assert_array_equal(s_g[0::2], s_g[1::2])
    # coarse space: twice the complex count, the real form of the span (a
    # floating subdomain's kernel: the real form of the constant, 2 columns)
    kd = [2 * int(e["kernel"]) for e in P.eig]
    assert list(info["kernel_dim"]) == kd
    if "float" in name:
        assert sum(kd) > 0
        blocks = sorted(set(int(b) for b in info["block"]))
        print(f"{name}: {sum(kd) // 2} floating subdomains, blocks {blocks}", flush=True)
        want = re.search(r"-s(\d+)$", name)
        if want:  # the factor / solve path the case is for
            assert max(blocks) == int(want.group(1)), blocks
    np.testing.assert_array_equal(info["nev_i"], 2 * P.nev_i)
    assert info["n0"] == 2 * P.n0
    Wg, woff, lam, _ = ads.ads_export_coarse(ctx.ctx)
    k0 = 0
    worst = 0.0
    for i in range(N):
        mi = int(info["nev_i"][i])
        Wi = Wg[woff[i]:woff[i + 1]].reshape(int(info["n_interior"][i]), mi)
        ang = sla.subspace_angles(Wi, real_form_cols(P.W[i])).max()
        worst = max(worst, ang)
        assert ang < 1e-7, (i, ang)
        lo = P.eig[i]["lam_sel"]
        assert not np.any(lam[k0:k0 + kd[i]])  # the kernel columns lead, eigenvalue 0
        same_eigs(lam[k0 + kd[i]:k0 + mi], np.concatenate([lo, lo.conj()]), 1e-8)
        k0 += mi
    print(f"{name}: n0 {info['n0']} real ({P.n0} complex), largest span angle {worst:.1e}",
          flush=True)
    # apply, two right-hand sides
    R = crand(n, 1, 2)
    Z = ctx.apply(torch.tensor(R, device=DEV)).cpu().numpy()
    Zo = P.apply(R)
    err = np.abs(Z - Zo).max() / np.abs(Zo).max()
    print(f"{name}: apply error {err:.1e}", flush=True)
    assert err <= 1e-9
    # complex GMRES: to tolerance and a fixed number of steps
    b = crand(n, 2)
    bt = torch.tensor(b, device=DEV)
    x, inf = ctx.solve(bt, restart=30, flexible=True, rtol=1e-8)
    xo, io = OS.gmres(As, b, P.apply, restart=30, rtol=1e-8, flexible=True)
    assert inf["status"] == ads.ADS_OK and abs(inf["its"][0] - io["its"]) <= 1, (inf["its"], io["its"])
    assert inf["relres"][0] <= 1e-8
    solution_close(As, b, x.cpu().numpy(), xo, name)
    k = max(2, io["its"] // 2)
    x, _ = ctx.solve(bt, restart=7, rtol=0.0, fixed_iters=k)
    xo, _ = OS.gmres(As, b, P.apply, restart=7, rtol=0.0, fixed_iters=k)
    e = np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo)
    print(f"{name}: its {inf['its'][0]} (oracle {io['its']}); fixed {k} steps, restart 7: {e:.1e}",
          flush=True)
    assert e <= 1e-10
    ctx.close()


@pytest.mark.parametrize("variant,oname", [(ads.ADS_VARIANT_RAS, "ras"), (ads.ADS_VARIANT_ASM, "asm"),
                                           (ads.ADS_VARIANT_ADDITIVE, "additive-asm"),
                                           (ads.ADS_VARIANT_ADDITIVE_RAS, "additive-ras")],
                         ids=["ras", "asm", "additive", "additive-ras"])
def test_complex_variants_match_oracle(variant, oname):
    """eq. 1, eq. 2, eq. 3 and the additive restricted form on complex A."""
    A = W.convdiff2d_complex(32, 0.01, eta=0.3, omega=2.0, phase_seed=7)
    part = W.block_partition_2d(32, 3)
    P = OS.TwoLevelSchwarz(A.to_scipy(), part, 9, 2, 4, variant=oname)
    ctx = ads.Context(A, part, 9, 2, 4, variant=variant, eig_tol=1e-12)
    R = crand(A.n, 3, 3)
    Z = ctx.apply(torch.tensor(R, device=DEV)).cpu().numpy()
    Zo = P.apply(R)
    err = np.abs(Z - Zo).max() / np.abs(Zo).max()
    print(f"complex {oname}: apply error {err:.1e}", flush=True)
    assert err <= 1e-9
    ctx.close()


@pytest.mark.parametrize("prec", [ads.ADS_PREC_FP32, ads.ADS_PREC_BF16], ids=["fp32", "bf16"])
def test_complex_low_precision_factors(prec):
    """FP32 / BF16 local factors on complex A: the solution within 1e-8 of
    the oracle's (or the residual bound), at most 2 more iterations."""
    A = W.convdiff2d_complex(48, 0.01, eta=0.5, omega=2.0, phase_seed=4)
    part = W.block_partition_2d(48, 3)
    As = A.to_scipy()
    P = OS.TwoLevelSchwarz(As, part, 9, 2, 4)
    ctx = ads.Context(A, part, 9, 2, 4, precision=prec)
    b = crand(A.n, 5)
    x, inf = ctx.solve(torch.tensor(b, device=DEV), restart=30, flexible=True, rtol=1e-8)
    xo, io = OS.gmres(As, b, P.apply, restart=30, rtol=1e-8, flexible=True)
    assert inf["status"] == ads.ADS_OK and inf["its"][0] <= io["its"] + 2, (inf["its"], io["its"])
    solution_close(As, b, x.cpu().numpy(), xo, f"complex prec {prec}")
    print(f"complex prec {prec}: its {inf['its'][0]} (oracle {io['its']}), "
          f"local resid {ctx.info['local_resid']:.1e}", flush=True)
    ctx.close()


def test_complex_batched_systems_and_sixteen_rhs():
    """Two complex systems in one context, 16 right-hand sides each: every
    (system, column) instance runs its own complex GMRES."""
    As = [W.convdiff2d_complex(24, 0.01, eta=0.4, omega=3.0, phase_seed=1),
          W.magnetic_laplace2d(20, 0.7, 0.05)]
    parts = [W.block_partition_2d(24, 2), W.block_partition_2d(20, 2)]
    ctx = ads.Context(As, parts, [4, 4], 1, 3, eig_tol=1e-12)
    Ps = [OS.TwoLevelSchwarz(A.to_scipy(), p, 4, 1, 3) for A, p in zip(As, parts)]
    ns = [A.n for A in As]
    B = np.concatenate([crand(n, 10 + k, 16) for k, n in enumerate(ns)])
    x, inf = ctx.solve(torch.tensor(B, device=DEV), restart=20, rtol=1e-8)
    X = x.cpu().numpy()
    r0 = 0
    for s, (A, P, n) in enumerate(zip(As, Ps, ns)):
        Asc = A.to_scipy()
        for j in (0, 7, 15):
            b = B[r0:r0 + n, j]
            xo, io = OS.gmres(Asc, b, P.apply, restart=20, rtol=1e-8)
            q = s * 16 + j
            assert inf["statuses"][q] == ads.ADS_OK and abs(inf["its"][q] - io["its"]) <= 1
            solution_close(Asc, b, X[r0:r0 + n, j], xo, f"batched system {s} column {j}")
        r0 += n
    ctx.close()


def test_complex_full_size_convection_diffusion():
    """256^2 complex convection-diffusion (65536 complex unknowns, real form
    131072), 8 x 8 blocks, overlap 2, nev 6 (the C2 layout): nev_i, n0,
    spans and the apply against the oracle, then FGMRES(50)."""
    m = 256
    A = W.convdiff2d_complex(m, 0.01, eta=0.25, omega=2.0, phase_seed=9)
    part = W.block_partition_2d(m, 8)
    As = A.to_scipy()
    P = OS.TwoLevelSchwarz(As, part, 64, 2, 6)
    ctx = ads.Context(A, part, 64, 2, 6, eig_tol=1e-12)
    info = ctx.info
    np.testing.assert_array_equal(info["nev_i"], 2 * P.nev_i)
    Wg, woff, _, _ = ads.ads_export_coarse(ctx.ctx)
    worst = 0.0
    for i in range(64):
        Wi = Wg[woff[i]:woff[i + 1]].reshape(int(info["n_interior"][i]), int(info["nev_i"][i]))
        worst = max(worst, sla.subspace_angles(Wi, real_form_cols(P.W[i])).max())
    assert worst < 1e-7, worst
    r = crand(A.n, 6)
    z = ctx.apply(torch.tensor(r, device=DEV)).cpu().numpy()
    zo = P.apply(r)
    assert np.abs(z - zo).max() <= 1e-9 * np.abs(zo).max()
    b = crand(A.n, 7)
    x, inf = ctx.solve(torch.tensor(b, device=DEV), restart=50, flexible=True, rtol=1e-8)
    xo, io = OS.gmres(As, b, P.apply, restart=50, rtol=1e-8, flexible=True)
    assert inf["status"] == ads.ADS_OK and abs(inf["its"][0] - io["its"]) <= 1
    solution_close(As, b, x.cpu().numpy(), xo, "complex 256^2")
    print(f"complex 256^2: n0 {P.n0} complex, span angle {worst:.1e}, its {inf['its'][0]} "
          f"(oracle {io['its']}), setup {info['t_phase_ms']}", flush=True)
    ctx.close()


def test_complex_disconnected_subdomains():
    """Disconnected subdomains of complex A (each part two strips four grid
    rows apart, overlap 1; in the real form both rows of an unknown are one
    vertex of the component search).  Dirichlet rows: nothing floats, the
    kernel dimensions are 0 as in the oracle and the apply matches it.
    Neumann rows at x = 0, 1: strips away from y = 0, 1 float, and the
    subdomains whose kernel is not the complex constant are refused."""
    part = (W.strip_partition(12, 2) % 3).astype(np.int32)
    A = W.convdiff2d_complex(12, 0.02, eta=0.5, eta_y=0.0)
    As = A.to_scipy()
    P = OS.TwoLevelSchwarz(As, part, 3, 1, 4)
    assert [e["kernel"] for e in P.eig] == [0, 0, 0]
    ctx = ads.Context(A, part, 3, 1, 4, eig_tol=1e-12)
    assert list(ctx.info["kernel_dim"]) == [0, 0, 0]
    R = crand(A.n, 5, 2)
    Z = ctx.apply(torch.tensor(R, device=DEV)).cpu().numpy()
    Zo = P.apply(R)
    err = np.abs(Z - Zo).max() / np.abs(Zo).max()
    print(f"disconnected complex apply vs oracle {err:.1e}", flush=True)
    assert err <= 1e-9
    ctx.close()
    An = W.convdiff2d_complex(12, 0.02, eta=0.5, eta_y=0.0, neumann_x=True)
    with pytest.raises(ads.AdsError) as e:
        ads.Context(An, part, 3, 1, 4)
    print(e.value, flush=True)
    assert e.value.status == ads.ADS_ERR_UNSUPPORTED and "subdomain 0" in str(e.value)
