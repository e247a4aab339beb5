"""Binding of the learned warm start's graph network (argument marshalling
only: forward, loss, backward and Adam run in the library's HIP kernels).

The weights file holds the FP32 master parameters:
    8 bytes  b"ADSGNN01"
    4 x int32  n_in, width, layers, n_out
    int64      nparams
    nparams x float32 (little endian), in the order of include/ads.h
The library reads it for ads_options.warm_start and rounds to BF16.
"""
from __future__ import annotations

import ctypes as C
import struct

import numpy as np

from . import ads

MAGIC = b"ADSGNN01"
DEFAULT_SHAPE = (ads.ADS_GNN_FEATURES, 64, 4, 8)


def shape_struct(shape):
    return ads.ads_gnn_shape(*[int(v) for v in shape])


def nparams(shape):
    n = ads.lib().ads_gnn_nparams(C.byref(shape_struct(shape)))
    if n < 0:
        raise ads.AdsError(ads.ADS_ERR_ARG, ads.ads_last_error())
    return int(n)


def init_params(shape, seed=0):
    """Seeded initial FP32 parameters: weights ~ N(0, 1/fan_in), biases 0
    (the output layer 1/fan_in scaled by 0.5)."""
    n_in, w, L, n_out = shape
    rng = np.random.default_rng(seed)
    parts = [rng.standard_normal(w * n_in) / np.sqrt(n_in), np.zeros(w)]
    for _ in range(L):
        parts += [rng.standard_normal(w * w) * 0.5 / np.sqrt(w),
                  rng.standard_normal(w * w) * 0.5 / np.sqrt(w), np.zeros(w)]
    parts.append(rng.standard_normal(n_out * w) / np.sqrt(w))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == nparams(shape)
    return p


def save_weights(path, shape, master):
    master = np.ascontiguousarray(master, dtype="<f4")
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<4i", *[int(v) for v in shape]))
        f.write(struct.pack("<q", master.size))
        f.write(master.tobytes())


def load_weights(path):
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError(f"{path}: not a weights file")
        shape = struct.unpack("<4i", f.read(16))
        (n,) = struct.unpack("<q", f.read(8))
        master = np.frombuffer(f.read(4 * n), dtype="<f4").copy()
    if master.size != n or n != nparams(shape):
        raise ValueError(f"{path}: truncated or inconsistent")
    return tuple(shape), master


class Graph:
    """A graph batch in device memory (torch tensors) and its C view."""

    def __init__(self, node_off, row_ptr, col, w, feat, mask):
        import torch
        self.node_off = node_off.to(torch.int64).contiguous()
        self.row_ptr = row_ptr.to(torch.int64).contiguous()
        self.col = col.to(torch.int32).contiguous()
        self.w = w.to(torch.float32).contiguous()
        self.feat = feat.to(torch.float32).contiguous()
        self.mask = mask.to(torch.uint8).contiguous()
        self.ngraph = self.node_off.numel() - 1
        self.nnode = self.row_ptr.numel() - 1

    def view(self):
        return ads.ads_gnn_graph(self.ngraph, self.nnode, self.node_off.data_ptr(),
                                 self.row_ptr.data_ptr(), self.col.data_ptr(), self.w.data_ptr(),
                                 self.feat.data_ptr(), self.mask.data_ptr())

    @staticmethod
    def from_context(ctx, stream=None):
        """The batch of the context's subdomain graphs (ads_gnn_graph_build)."""
        import torch
        nn, ne, ng = C.c_int64(), C.c_int64(), C.c_int32()
        ads._check(ads.lib().ads_gnn_graph_size(ctx.ctx, C.byref(nn), C.byref(ne), C.byref(ng)))
        dev = torch.device("cuda:0")
        node_off = torch.empty(ng.value + 1, dtype=torch.int64, device=dev)
        row_ptr = torch.empty(nn.value + 1, dtype=torch.int64, device=dev)
        col = torch.empty(max(ne.value, 1), dtype=torch.int32, device=dev)
        w = torch.empty(max(ne.value, 1), dtype=torch.float32, device=dev)
        feat = torch.empty((nn.value, ads.ADS_GNN_FEATURES), dtype=torch.float32, device=dev)
        mask = torch.empty(nn.value, dtype=torch.uint8, device=dev)
        ads._check(ads.lib().ads_gnn_graph_build(ctx.ctx, node_off.data_ptr(), row_ptr.data_ptr(),
                                                 col.data_ptr(), w.data_ptr(), feat.data_ptr(),
                                                 mask.data_ptr(), stream))
        return Graph(node_off, row_ptr, col, w, feat, mask)


def targets(ctx, nz, stream=None):
    import torch
    nn, ne, ng = C.c_int64(), C.c_int64(), C.c_int32()
    ads._check(ads.lib().ads_gnn_graph_size(ctx.ctx, C.byref(nn), C.byref(ne), C.byref(ng)))
    Z = torch.empty((nn.value, nz), dtype=torch.float32, device="cuda:0")
    ads._check(ads.lib().ads_gnn_targets(ctx.ctx, Z.data_ptr(), nz, stream))
    return Z


class Net:
    """Parameters (FP32 master, BF16 copy, Adam moments) on the device."""

    def __init__(self, shape, master, stream=None):
        import torch
        self.shape = tuple(int(v) for v in shape)
        self.sh = shape_struct(self.shape)
        self.n = nparams(self.shape)
        dev = torch.device("cuda:0")
        self.master = torch.tensor(np.asarray(master, np.float32), device=dev)
        self.bf16 = torch.empty(self.n, dtype=torch.int16, device=dev)
        self.m = torch.zeros(self.n, dtype=torch.float32, device=dev)
        self.v = torch.zeros(self.n, dtype=torch.float32, device=dev)
        self.grad = torch.zeros(self.n, dtype=torch.float32, device=dev)
        self.step = 0
        self.stream = stream
        ads._check(ads.lib().ads_gnn_round_bf16(self.n, self.master.data_ptr(), self.bf16.data_ptr(),
                                                stream))
        self._ws = None

    def workspace(self, nnode):
        import torch
        need = ads.lib().ads_gnn_workspace_floats(C.byref(self.sh), nnode)
        if need < 0:
            raise ads.AdsError(ads.ADS_ERR_ARG, ads.ads_last_error())
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.float32, device="cuda:0")
        return self._ws

    def forward(self, g: Graph):
        import torch
        X = torch.empty((g.nnode, self.shape[3]), dtype=torch.float32, device="cuda:0")
        ws = self.workspace(g.nnode)
        gv = g.view()
        ads._check(ads.lib().ads_gnn_forward(C.byref(self.sh), self.bf16.data_ptr(), C.byref(gv),
                                             ws.data_ptr(), X.data_ptr(), self.stream))
        return X

    def loss(self, g: Graph, X, Z):
        import torch
        dX = torch.empty_like(X)
        L = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        gv = g.view()
        ads._check(ads.lib().ads_gnn_loss(C.byref(self.sh), C.byref(gv), X.data_ptr(), Z.data_ptr(),
                                          Z.shape[1], dX.data_ptr(), L.data_ptr(), self.stream))
        return L, dX

    def backward(self, g: Graph, dX):
        """grad += d(sum(dX * X))/dparams for the last forward on g."""
        gv = g.view()
        ads._check(ads.lib().ads_gnn_backward(C.byref(self.sh), self.bf16.data_ptr(), C.byref(gv),
                                              self.workspace(g.nnode).data_ptr(), dX.data_ptr(),
                                              self.grad.data_ptr(), self.stream))

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step += 1
        ads._check(ads.lib().ads_gnn_adam(self.n, self.master.data_ptr(), self.bf16.data_ptr(),
                                          self.grad.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                          self.step, lr, beta1, beta2, eps, self.stream))

    def bf16_values(self):
        """The BF16 parameters as float64 (host)."""
        b = self.bf16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        return b.view(np.float32).astype(np.float64)
