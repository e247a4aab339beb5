"""GPU tests of the learned warm start's graph network, through the C ABI:
forward, loss and backward against the FP64 CPU oracle (oracle/gnn.py) with
the same BF16-rounded parameters (the remaining difference is FP32
arithmetic: <= 1e-5 relative), the graph and targets built from a context
against their definition, and Adam."""
import numpy as np
import pytest

import workloads as W
from oracle import gnn as OG
from oracle import schwarz as OS

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2201_02250_amd import ads  # noqa: E402
from paper_2201_02250_amd import gnn as G  # noqa: E402

DEV = "cuda:0"


def sym_graph(rng, sizes, n_in):
    """Block-diagonal batch of symmetric graphs (paths with chords)."""
    rp, col, w, off = [0], [], [], [0]
    for n in sizes:
        base = off[-1]
        adj = {j: set() for j in range(n)}
        for j in range(n - 1):
            adj[j].add(j + 1)
            adj[j + 1].add(j)
        for j in range(0, n - 5, 5):
            adj[j].add(j + 5)
            adj[j + 5].add(j)
        for j in range(n):
            for k in sorted(adj[j]):
                col.append(base + k)
                w.append(0.2 + 0.1 * ((j + k) % 5))
            rp.append(len(col))
        off.append(base + n)
    N = off[-1]
    feat = rng.standard_normal((N, n_in))
    return dict(row_ptr=np.array(rp), col=np.array(col), w=np.array(w), feat=feat), np.array(off)


def to_device_graph(graph, off, mask):
    t = lambda a, dt: torch.tensor(np.asarray(a), dtype=dt, device=DEV)
    return G.Graph(t(off, torch.int64), t(graph["row_ptr"], torch.int64), t(graph["col"], torch.int32),
                   t(graph["w"], torch.float32), t(graph["feat"], torch.float32),
                   t(mask, torch.uint8))


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def test_forward_loss_backward_match_the_cpu_oracle():
    rng = np.random.default_rng(5)
    shape = G.DEFAULT_SHAPE
    graph, off = sym_graph(rng, (41, 57, 30), shape[0])
    # features rounded to FP32 on both sides
    graph["feat"] = graph["feat"].astype(np.float32).astype(np.float64)
    graph["w"] = graph["w"].astype(np.float32).astype(np.float64)
    N = off[-1]
    mask = (rng.random(N) > 0.2).astype(np.uint8)
    Z = rng.standard_normal((N, 8)).astype(np.float32)
    net = G.Net(shape, G.init_params(shape, seed=3))
    p64 = net.bf16_values()  # the BF16 parameters the kernels use
    g = to_device_graph(graph, off, mask)
    X = net.forward(g)
    L, dX = net.loss(g, X, torch.tensor(Z, device=DEV))
    net.grad.zero_()
    net.backward(g, dX)
    torch.cuda.synchronize()
    Xo, saved = OG.forward(p64, shape, graph)
    Lo, dXo = OG.loss(Xo, Z.astype(np.float64), mask, off)
    go = OG.backward(p64, shape, graph, saved, dXo)
    assert rel(X.cpu().numpy(), Xo) <= 1e-5
    assert abs(L.item() - Lo) <= 1e-5 * abs(Lo)
    assert rel(dX.cpu().numpy(), dXo) <= 1e-5
    assert rel(net.grad.cpu().numpy(), go) <= 1e-5
    # the backward accumulates: a second call doubles the gradient
    net.backward(g, dX)
    torch.cuda.synchronize()
    assert rel(net.grad.cpu().numpy(), 2 * go) <= 1e-5


def test_adam_step_and_rounding():
    shape = (4, 8, 1, 2)
    p = G.init_params(shape, seed=1)
    net = G.Net(shape, p)
    g = np.linspace(-1, 1, net.n).astype(np.float32)
    net.grad.copy_(torch.tensor(g, device=DEV))
    net.adam(1e-2)
    torch.cuda.synchronize()
    # first bias-corrected Adam step moves every parameter by lr * sign(g)
    # (up to eps), then the BF16 copy is the rounded master
    m = net.master.cpu().numpy()
    ref = p - 1e-2 * g / (np.abs(g) + 1e-8)
    assert np.abs(m - ref).max() <= 1e-6
    bf = net.bf16_values()
    assert np.abs(bf - m).max() <= np.abs(m).max() * 2.0 ** -8


def test_graph_and_targets_from_a_context():
    A, part, N, o = W.config("c4_lognormal2d_256_blocks64", scale=64)
    ctx = ads.Context(A, part, N, o["overlap"], o["nev"])
    g = G.Graph.from_context(ctx)
    Z = G.targets(ctx, 8)
    torch.cuda.synchronize()
    As = A.to_scipy()
    subs = OS.subdomains(As, part, N, o["overlap"])
    off = g.node_off.cpu().numpy()
    rp, col = g.row_ptr.cpu().numpy(), g.col.cpu().numpy()
    w, feat, mask = g.w.cpu().numpy(), g.feat.cpu().numpy(), g.mask.cpu().numpy()
    Wg, woff, lam, info = ads.ads_export_coarse(ctx.ctx)
    Zh = Z.cpu().numpy()
    for i, sub in enumerate(subs):
        om = np.sort(sub.omega)  # node order: ascending global index
        Aii = As[om][:, om].toarray()
        n = len(om)
        assert off[i + 1] - off[i] == n
        b = off[i]
        interior = np.isin(om, sub.omega[:sub.n_interior])
        np.testing.assert_array_equal(mask[b:b + n], interior.astype(np.uint8))
        d = np.abs(np.diag(Aii))
        for j in range(n):
            nb = np.nonzero(Aii[j])[0]
            nb = nb[nb != j]
            seg = slice(rp[b + j], rp[b + j + 1])
            np.testing.assert_array_equal(col[seg] - b, nb)
            ref = (np.abs(Aii[j, nb]) + np.abs(Aii[nb, j])) / (2 * np.sqrt(d[j] * d[nb]))
            np.testing.assert_allclose(w[seg], ref, rtol=1e-6)
        np.testing.assert_allclose(feat[b:b + n, 0], d / d.mean(), rtol=1e-6)
        np.testing.assert_array_equal(feat[b:b + n, 3], interior.astype(np.float32))
        # targets: interior rows carry W_i, in ascending order
        m = int(info["nev_i"][i])
        Wi = Wg[woff[i]:woff[i + 1]].reshape(-1, m)
        np.testing.assert_allclose(Zh[b:b + n][interior][:, :m], Wi, rtol=1e-6, atol=1e-7)
        assert np.all(Zh[b:b + n][~interior] == 0)
    ctx.close()
