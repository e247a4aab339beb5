"""Oracle pins for splittings whose kernel has dimension above one (reading R6:
the indicators of the floating connected components of a disconnected
subdomain).

Each part of `strip_partition(12, 2) % 3` is two strips four grid rows apart,
so with one overlap layer every subdomain has two connected components.  With
Neumann rows at x = 0, 1 the strips away from y = 0 and y = 1 float: part 0
has one floating strip (and one touching y = 0), part 1 two, part 2 one (and
one touching y = 1).  The scalable tier (components, one regularised entry
and one left null vector per floating component) is checked against the
dense tier, which takes K_i, ker Atilde_ii^H and L_i from singular value
decompositions and solves eq. 5 by QZ on the restricted pencil, sharing no
code with it."""
import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import dense as OD
from oracle import schwarz as OS

PART = (W.strip_partition(12, 2) % 3).astype(np.int32)
CASES = [
    ("upwind", lambda: W.convdiff2d(12, 0.05, neumann_x=True).to_scipy()),
    ("laplace", lambda: W.convdiff2d(12, 0.05, velocity=None, neumann_x=True).to_scipy()),
    ("complex", lambda: W.convdiff2d_complex(12, 0.02, eta=0.5, eta_y=0.0,
                                             neumann_x=True).to_scipy()),
]


def _dense_variant(D, variant):
    return {"deflated": D.M_deflated, "ras": D.M_ras, "asm": D.M_asm,
            "additive-asm": D.M_additive,
            "additive-ras": lambda: D.coarse() + D.M_ras()}[variant]()


def _same_eigs(a, b, rtol):
    a, b = np.asarray(a), list(np.asarray(b))
    assert len(a) == len(b)
    for x in a:
        j = int(np.argmin([abs(x - y) for y in b]))
        assert abs(x - b[j]) <= rtol * abs(x)
        b.pop(j)


def test_floating_components_by_hand():
    """Components and floating flags of the three splittings, counted by
    hand from the strip layout."""
    A = CASES[0][1]()
    subs = OS.subdomains(A, PART, 3, 1)
    want = [1, 2, 1]
    for sub, kd in zip(subs, want):
        _, _, At = OS.block_splitting(A, sub)
        comps = OS.floating_components(At)
        assert len(comps) == kd == OS.kernel_dimension(At)
        rows = [sorted(set(sub.omega[idx] // 12)) for idx in comps]
        for r in rows:  # whole strips plus their overlap rows, away from y = 0, 1
            assert 0 not in r and 11 not in r and len(r) == 4
    # a connected subdomain keeps the single-kernel reading
    _, _, At = OS.block_splitting(A, OS.subdomains(A, W.strip_partition(12, 4), 3, 1)[1])
    assert OS.kernel_dimension(At) == 1 and len(OS.floating_components(At)[0]) == At.shape[0]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_components_tiers_agree(case):
    """Dense tier (SVD kernels, QZ) against the scalable tier: kernel
    dimensions [1, 2, 1], nev_i, selected eigenvalues, spans of Z_i, and the
    same M^{-1} for every variant of Section 2; the two-level GMRES converges
    in as many iterations with either tier's preconditioner."""
    name, mk = case
    A = mk()
    D = OD.DenseSchwarz(A, PART, 3, 1, 4)
    P = OS.TwoLevelSchwarz(A, PART, 3, 1, 4)
    assert [e["kernel"] for e in P.eig] == [e["kernel"] for e in D.eig] == [1, 2, 1]
    assert P.n0 == D.n0
    for e_d, e_s in zip(D.eig, P.eig):
        assert e_d["Z"].shape[1] == e_s["Z"].shape[1]
        _same_eigs(e_d["lam_sel"], e_s["lam_sel"], 1e-9)
        assert sla.subspace_angles(e_d["Z"], e_s["Z"]).max() < 1e-10
    r = np.random.default_rng(3).standard_normal((A.shape[0], 2))
    for variant in ("deflated", "ras", "asm", "additive-asm", "additive-ras"):
        Pv = P if variant == "deflated" else OS.TwoLevelSchwarz(A, PART, 3, 1, 4, variant=variant)
        ref = _dense_variant(D, variant) @ r
        np.testing.assert_allclose(Pv.apply(r), ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    b = W.rhs(A.shape[0], 5).astype(A.dtype)
    x, info = OS.gmres(A, b, P.apply, restart=30, rtol=1e-10)
    xd, infod = OS.gmres(A, b, lambda v: D.M_deflated() @ v, restart=30, rtol=1e-10)
    assert info["status"] == OS.OK and abs(info["its"] - infod["its"]) <= 1
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)
