"""FP64 CPU oracle of the learned warm start's graph network (test
infrastructure only: imported by tests/ and nowhere else).

The network is not in the paper: it predicts, per subdomain, a block whose
span approximates the coarse space of eq. 6 (the selected eigenvectors of
eq. 5, Section 3.2), as a warm start for the local eigensolves.

Definition (shape: n_in input features, width w, L layers, n_out outputs):

    h_0 = F W_in^T + 1 b_in^T                                (input layer)
    a_l = A_w h_l                                            (aggregation)
    u_l = h_l W_s,l^T + a_l W_n,l^T + 1 b_l^T                 (l = 0 .. L-1)
    h_{l+1} = h_l + relu(u_l)                                (residual)
    X = h_L W_out^T                                          (output block)

A_w is the weighted adjacency of the graph (no self loops). Parameters are
one flat vector in the order W_in (w x n_in, row-major), b_in, then per layer
W_s (w x w), W_n (w x w), b (w), then W_out (n_out x w).

Loss over a batch of graphs g (rows restricted to the mask, i.e. the interior
rows that carry the coarse basis): with C_g = (X_g^T X_g)^{-1} X_g^T Z_g the
least-squares coefficients,

    L = (1 / G) sum_g ||Z_g - X_g C_g||_F^2 / ||Z_g||_F^2,

the fraction of the target span Z_g not captured by span(X_g). Because C_g
is the minimiser, dL/dX_g = -(2 / (G ||Z_g||^2)) (Z_g - X_g C_g) C_g^T.
"""
import numpy as np


def nparams(n_in, w, L, n_out):
    return w * n_in + w + L * (2 * w * w + w) + n_out * w


def unpack(p, n_in, w, L, n_out):
    """Views of the flat parameter vector in the documented order."""
    p = np.asarray(p, dtype=np.float64)
    assert p.size == nparams(n_in, w, L, n_out)
    o = 0

    def take(shape):
        nonlocal o
        k = int(np.prod(shape))
        v = p[o:o + k].reshape(shape)
        o += k
        return v

    W_in = take((w, n_in))
    b_in = take((w,))
    layers = []
    for _ in range(L):
        layers.append((take((w, w)), take((w, w)), take((w,))))
    W_out = take((n_out, w))
    return W_in, b_in, layers, W_out


def aggregate(row_ptr, col, wgt, h):
    """a_j = sum over the edges (j, k) of w_jk h_k, rows in edge order."""
    n = len(row_ptr) - 1
    a = np.zeros_like(h)
    for j in range(n):
        for e in range(row_ptr[j], row_ptr[j + 1]):
            a[j] += wgt[e] * h[col[e]]
    return a


def aggregate_t(row_ptr, col, wgt, g):
    """Transpose of aggregate: b_k = sum over the edges (j, k) of w_jk g_j."""
    n = len(row_ptr) - 1
    b = np.zeros_like(g)
    for j in range(n):
        for e in range(row_ptr[j], row_ptr[j + 1]):
            b[col[e]] += wgt[e] * g[j]
    return b


def forward(p, shape, graph):
    """Returns X and the saved activations (h_l, a_l, u_l)."""
    n_in, w, L, n_out = shape
    W_in, b_in, layers, W_out = unpack(p, *shape)
    F = np.asarray(graph["feat"], dtype=np.float64)
    rp, col, wgt = graph["row_ptr"], graph["col"], np.asarray(graph["w"], dtype=np.float64)
    h = F @ W_in.T + b_in
    hs, As, Us = [h], [], []
    for (Ws, Wn, b) in layers:
        a = aggregate(rp, col, wgt, h)
        u = h @ Ws.T + a @ Wn.T + b
        h = h + np.maximum(u, 0.0)
        As.append(a)
        Us.append(u)
        hs.append(h)
    X = h @ W_out.T
    return X, (hs, As, Us)


def loss(X, Z, mask, node_off):
    """Loss and dL/dX (zero on unmasked rows); graphs are node ranges."""
    X = np.asarray(X, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    G = len(node_off) - 1
    dX = np.zeros_like(X)
    tot = 0.0
    for g in range(G):
        rows = np.arange(node_off[g], node_off[g + 1])
        rows = rows[np.asarray(mask)[rows] != 0]
        Xg, Zg = X[rows], Z[rows]
        zz = float(np.sum(Zg * Zg))
        C = np.linalg.solve(Xg.T @ Xg, Xg.T @ Zg)
        R = Zg - Xg @ C
        tot += float(np.sum(R * R)) / zz
        dX[rows] = -2.0 / (G * zz) * (R @ C.T)
    return tot / G, dX


def backward(p, shape, graph, saved, dX):
    """Gradient of sum(dX * X) with respect to the flat parameters."""
    n_in, w, L, n_out = shape
    W_in, b_in, layers, W_out = unpack(p, *shape)
    hs, As, Us = saved
    rp, col, wgt = graph["row_ptr"], graph["col"], np.asarray(graph["w"], dtype=np.float64)
    F = np.asarray(graph["feat"], dtype=np.float64)
    g_layers = []
    gW_out = dX.T @ hs[L]
    dh = dX @ W_out
    for l in range(L - 1, -1, -1):
        Ws, Wn, b = layers[l]
        du = dh * (Us[l] > 0.0)
        gWs = du.T @ hs[l]
        gWn = du.T @ As[l]
        gb = du.sum(axis=0)
        dh = dh + du @ Ws + aggregate_t(rp, col, wgt, du @ Wn)
        g_layers.append((gWs, gWn, gb))
    g_layers.reverse()
    gW_in = dh.T @ F
    gb_in = dh.sum(axis=0)
    parts = [gW_in.ravel(), gb_in]
    for (a, b_, c) in g_layers:
        parts += [a.ravel(), b_.ravel(), c]
    parts.append(gW_out.ravel())
    return np.concatenate(parts)


def objective(p, shape, graph, Z, mask, node_off):
    X, _ = forward(p, shape, graph)
    return loss(X, Z, mask, node_off)[0]


def gradient(p, shape, graph, Z, mask, node_off):
    """Loss and its gradient with respect to the parameters."""
    X, saved = forward(p, shape, graph)
    L_, dX = loss(X, Z, mask, node_off)
    return L_, backward(p, shape, graph, saved, dX)
