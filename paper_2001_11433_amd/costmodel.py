"""Learned scheduling cost model, driven through the library's MLP kernels.

Features come from `mce_features`, labels from the search's own per-vertex
node counts (`mce_static(per_vertex=True)`), training is full-batch Adam on
the MSE of log node counts (FP32 kernels), prediction uses the BF16 kernel.
The prediction is passed to `mce_static(sched="cost")`: largest predicted cost
first (longest-processing-time order).  It never changes the cliques.
"""

from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _as_device_graph, _check, _stream_ptr, _torch, lib, mce_features, mce_static

H = 64


def param_count() -> int:
    return int(lib().mce_mlp_param_count())


def init_params(seed: int = 0) -> np.ndarray:
    """He-style initial weights (layout of include/mce.h), identity standardisation."""
    rng = np.random.default_rng(seed)
    p = np.concatenate([
        rng.normal(0, np.sqrt(2 / 4), H * 4), np.zeros(H),
        rng.normal(0, np.sqrt(2 / H), H * H), np.zeros(H),
        rng.normal(0, np.sqrt(1 / H), H), [0.0],
        np.zeros(4), np.ones(4)]).astype(np.float32)
    assert p.size == param_count()
    return p


def labels(nodes_v, stream=None):
    """log(max(nodes, 1)) on the device (nodes_v: int64 view of uint64)."""
    torch = _torch()
    n = int(nodes_v.numel())
    out = torch.empty(max(n, 1), dtype=torch.float32, device=nodes_v.device)
    _check(lib().mce_mlp_labels(nodes_v.data_ptr(), n, out.data_ptr(), _stream_ptr(stream)))
    return out[:n]


def collect(g, rank: str = "degeneracy", sched: str = "degree"):
    """Features and labels of one graph: (feat [n,4], target [n], result)."""
    dg = _as_device_graph(g)
    feat = mce_features(dg)
    res = mce_static(dg, rank=rank, sched=sched, per_vertex=True)
    return feat, labels(res["nodes_v"]), res


class CostModel:
    def __init__(self, params: Optional[np.ndarray] = None, seed: int = 0, device: str = "cuda"):
        torch = _torch()
        p = init_params(seed) if params is None else np.asarray(params, np.float32)
        self.params = torch.from_numpy(p.copy()).to(device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.g = torch.zeros_like(self.params)
        self.loss_buf = torch.zeros(1, dtype=torch.float32, device=device)
        self.p16 = torch.zeros(self.params.numel(), dtype=torch.int16, device=device)
        self.step = 0
        self._p16_step = None  # the training step p16 was rounded at

    def bf16(self):
        """The bfloat16 parameter block (rounded again only after training steps)."""
        key = (self.step, self.params.data_ptr())
        if self._p16_step != key:
            _check(lib().mce_mlp_to_bf16(self.params.data_ptr(), self.p16.data_ptr(), _stream_ptr(None)))
            self._p16_step = key
        return self.p16

    def fit_norm(self, feat):
        self._p16_step = None
        _check(lib().mce_mlp_fit_norm(self.params.data_ptr(), feat.data_ptr(), int(feat.shape[0]),
                                      _stream_ptr(None)))

    def grad(self, feat, target):
        _check(lib().mce_mlp_grad(self.params.data_ptr(), feat.data_ptr(), target.data_ptr(), int(feat.shape[0]),
                                  self.g.data_ptr(), self.loss_buf.data_ptr(), _stream_ptr(None)))
        return self.g, float(self.loss_buf.item())

    def adam(self, lr: float):
        self.step += 1
        _check(lib().mce_mlp_adam(self.params.data_ptr(), self.m.data_ptr(), self.v.data_ptr(), self.g.data_ptr(),
                                  ctypes.c_float(lr), self.step, _stream_ptr(None)))

    def train(self, feat, target, epochs: int = 400, lr: float = 3e-3) -> List[float]:
        """Full-batch Adam on (1/n) sum (MLP(feat) - target)^2; returns the loss per epoch."""
        losses = []
        for _ in range(epochs):
            _, l = self.grad(feat, target)
            losses.append(l)
            self.adam(lr)
        return losses

    def predict(self, feat, bf16: bool = True):
        torch = _torch()
        n = int(feat.shape[0])
        out = torch.empty(max(n, 1), dtype=torch.float32, device=feat.device)
        if bf16:
            _check(lib().mce_mlp_forward_bf16(self.bf16().data_ptr(), self.params.data_ptr(), feat.data_ptr(), n,
                                              out.data_ptr(), _stream_ptr(None)))
        else:
            _check(lib().mce_mlp_forward(self.params.data_ptr(), feat.data_ptr(), n, out.data_ptr(),
                                         _stream_ptr(None)))
        return out[:n]

    def numpy(self) -> np.ndarray:
        return self.params.detach().cpu().numpy()


def train_on_graphs(graphs: Sequence, rank: str = "degeneracy", epochs: int = 400, lr: float = 3e-3,
                    seed: int = 0) -> Dict[str, object]:
    """Collects features/labels on `graphs`, fits standardisation and trains."""
    torch = _torch()
    feats, targets = [], []
    for g in graphs:
        f, t, _ = collect(g, rank)
        feats.append(f)
        targets.append(t)
    feat = torch.cat(feats).contiguous()
    target = torch.cat(targets).contiguous()
    model = CostModel(seed=seed)
    model.fit_norm(feat)
    losses = model.train(feat, target, epochs, lr)
    return {"model": model, "losses": losses, "n_train": int(feat.shape[0])}
