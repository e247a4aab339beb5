"""Pins of the graph-network oracle (oracle/gnn.py) on the CPU: central
finite differences of the loss, the span properties of the projection loss,
the adjointness of the aggregation and a forward pass worked out by hand."""
import numpy as np

from oracle import gnn as OG


def small_graph(rng, sizes=(7, 9), n_in=3):
    """Block-diagonal batch of path graphs with a few chords, symmetric
    positive weights, random features."""
    rp, col, w = [0], [], []
    off = [0]
    for n in sizes:
        base = off[-1]
        adj = {j: set() for j in range(n)}
        for j in range(n - 1):
            adj[j].add(j + 1)
            adj[j + 1].add(j)
        for j in range(0, n - 3, 3):
            adj[j].add(j + 3)
            adj[j + 3].add(j)
        for j in range(n):
            for k in sorted(adj[j]):
                col.append(base + k)
                w.append(0.25 + 0.5 * ((j + k) % 3) / 2.0)
            rp.append(len(col))
        off.append(base + n)
    N = off[-1]
    feat = rng.standard_normal((N, n_in))
    return dict(row_ptr=np.array(rp), col=np.array(col), w=np.array(w), feat=feat), np.array(off)


def test_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    shape = (3, 5, 2, 2)
    graph, off = small_graph(rng)
    N = off[-1]
    mask = np.ones(N, dtype=np.uint8)
    mask[[0, 8]] = 0
    Z = rng.standard_normal((N, 3))
    p = 0.4 * rng.standard_normal(OG.nparams(*shape))
    L0, g = OG.gradient(p, shape, graph, Z, mask, off)
    h = 1e-6
    fd = np.empty_like(p)
    for k in range(p.size):
        e = np.zeros_like(p)
        e[k] = h
        fd[k] = (OG.objective(p + e, shape, graph, Z, mask, off) -
                 OG.objective(p - e, shape, graph, Z, mask, off)) / (2 * h)
    assert np.abs(fd - g).max() <= 1e-6 * max(1.0, np.abs(g).max())
    assert 0.0 < L0 < 1.0


def test_loss_is_zero_on_the_span_and_invariant_under_column_mixing():
    rng = np.random.default_rng(1)
    N = 20
    off = np.array([0, 12, 20])
    mask = np.ones(N, dtype=np.uint8)
    X = rng.standard_normal((N, 4))
    Z = X @ rng.standard_normal((4, 3))  # inside span(X) on every graph
    L, dX = OG.loss(X, Z, mask, off)
    assert L < 1e-24 and np.abs(dX).max() < 1e-12
    Z2 = rng.standard_normal((N, 3))
    M = rng.standard_normal((4, 4)) + 4 * np.eye(4)
    L1, _ = OG.loss(X, Z2, mask, off)
    L2, _ = OG.loss(X @ M, Z2, mask, off)
    assert abs(L1 - L2) <= 1e-12
    # the loss is the captured-energy complement: 1 - ||P Z||^2 / ||Z||^2 per graph
    for g in range(2):
        r = slice(off[g], off[g + 1])
        Q, _ = np.linalg.qr(X[r])
        pz = np.sum((Q.T @ Z2[r]) ** 2) / np.sum(Z2[r] ** 2)
        assert 0.0 <= 1.0 - pz <= 1.0
    Ls = np.mean([1.0 - np.sum((np.linalg.qr(X[off[g]:off[g + 1]])[0].T @ Z2[off[g]:off[g + 1]]) ** 2)
                  / np.sum(Z2[off[g]:off[g + 1]] ** 2) for g in range(2)])
    assert abs(Ls - L1) <= 1e-12


def test_aggregation_adjoint():
    rng = np.random.default_rng(2)
    graph, off = small_graph(rng, sizes=(11,))
    h = rng.standard_normal((11, 4))
    g = rng.standard_normal((11, 4))
    a = OG.aggregate(graph["row_ptr"], graph["col"], graph["w"], h)
    b = OG.aggregate_t(graph["row_ptr"], graph["col"], graph["w"], g)
    assert abs(np.sum(a * g) - np.sum(h * b)) <= 1e-12 * np.sum(np.abs(a * g))


def test_forward_by_hand():
    # one input feature, width 1, one layer, one output; two nodes joined by
    # an edge of weight 0.5 each way; features 1 and 2
    shape = (1, 1, 1, 1)
    W_in, b_in, Ws, Wn, b, W_out = 2.0, -1.0, 0.5, 1.0, 0.25, 3.0
    p = np.array([W_in, b_in, Ws, Wn, b, W_out])
    graph = dict(row_ptr=np.array([0, 1, 2]), col=np.array([1, 0]), w=np.array([0.5, 0.5]),
                 feat=np.array([[1.0], [2.0]]))
    X, _ = OG.forward(p, shape, graph)
    # h0 = (1, 3); a = (1.5, 0.5); u = (0.5+1.5+0.25, 1.5+0.5+0.25) = (2.25, 2.25)
    # h1 = (3.25, 5.25); X = 3 h1
    assert np.allclose(X[:, 0], [9.75, 15.75], rtol=0, atol=1e-14)
    # negative pre-activation is cut: with b = -10 the residual passes h0 unchanged
    p2 = p.copy()
    p2[4] = -10.0
    X2, _ = OG.forward(p2, shape, graph)
    assert np.allclose(X2[:, 0], [3.0, 9.0], rtol=0, atol=1e-14)


def test_torch_field_values_follow_the_recipe():
    """The device field generator (training data) keeps the structure of the
    numpy one: same pattern, symmetric, diagonal = sum of the face
    coefficients (zero row sums away from the boundary)."""
    import torch
    import workloads as W
    m = 24
    A = W.diffusion2d_lognormal(m, seed=0, npad=64)
    ip = torch.tensor(A.indptr)
    ix = torch.tensor(A.indices)
    v = W.lognormal2d_values_torch(m, 3, ip, ix, npad=64).numpy()
    import scipy.sparse as sp
    M = sp.csr_matrix((v, A.indices, A.indptr), shape=(A.n, A.n))
    assert abs(M - M.T).max() <= 1e-12 * abs(M).max()
    d = M.diagonal()
    assert np.all(d > 0)
    rs = np.asarray(M.sum(axis=1)).ravel()
    i, j = np.arange(A.n) % m, np.arange(A.n) // m
    inner = (i > 0) & (i < m - 1) & (j > 0) & (j < m - 1)
    assert np.abs(rs[inner]).max() <= 1e-12 * d.max()
    assert np.all(rs[~inner] > 0)
