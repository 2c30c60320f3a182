"""Learned quintuplet scorer: training set from the chain, training on the GPU
through the library's forward / backward / Adam kernels, threshold choice and
evaluation against the plain cut chain.

Every arithmetic step of the network runs in liblst (lst_mlp_* entry points);
this module only moves data.  The standardisation constants are the mean and
inverse standard deviation of the training features (FP64 on the host,
rounded once to FP32), fixed before training starts.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

from . import lst as L


def pure_labels(tuples: np.ndarray, truth: np.ndarray) -> np.ndarray:
    """1 iff every hit of the object comes from one simulated track"""
    if len(tuples) == 0:
        return np.zeros(0, np.uint8)
    t = truth[tuples]
    return ((t[:, 0] >= 0) & np.all(t == t[:, :1], axis=1)).astype(np.uint8)


def collect(ctx: "L.Context", events, kind=L.LST_T5, stream=None):
    """Features (FP32 [N, 40], computed by the chain on the GPU) and truth
    labels of every triplet (kind LST_T3) or quintuplet (LST_T5) the chain
    stores for `events`, in a reproducible order.  The chain runs in the
    context's mode (a scored chain gives the objects that survive its
    earlier vetoes)."""
    feats, labels = [], []
    for ev in events:
        if ctx.caps is None or not ctx.caps.get("features"):
            caps = L.default_caps(1, max(ev.n_hits, 1))
            caps["features"] = 1
            ctx.reserve(caps)
        offs = np.array([0, ev.n_hits], np.int32)
        ctx.run_batch(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor, stream)
        if kind == L.LST_T3:
            ctx.run_t3_features(stream)
            f = ctx.t3_features(0, stream)
        else:
            ctx.run_t5_features(stream)
            f = ctx.t5_features(0, stream)
        obj = ctx.objects(0, kind, stream)
        # canonical order (by hit tuple): the device stores objects in
        # whatever order its blocks finish, the training set must not depend on it
        o = np.lexsort(obj.T[::-1]) if len(obj) else np.zeros(0, np.int64)
        feats.append(f[o])
        labels.append(pure_labels(obj[o], ev.truth))
    return np.concatenate(feats), np.concatenate(labels)


def standardisation(features: np.ndarray):
    """mean and 1/std per feature (std floored at 1e-6), FP32"""
    f = np.asarray(features, np.float64)
    mean = f.mean(axis=0)
    std = np.maximum(f.std(axis=0), 1e-6)
    return mean.astype(np.float32), (1.0 / std).astype(np.float32)


@dataclasses.dataclass
class TrainConfig:
    epochs: int = 8
    batch: int = 4096
    lr: float = 2e-3
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    seed: int = 0


class Trainer:
    """Mini-batch Adam on the GPU.  The training set is shuffled once on the
    host and uploaded; every epoch visits its fixed-size batches in a new
    random order."""

    def __init__(self, ctx: "L.Context", features, labels, init_params, cfg: TrainConfig,
                 mean=None, istd=None, stream=None):
        self.ctx, self.cfg = ctx, cfg
        self.stream = stream or torch.cuda.current_stream()
        dev = f"cuda:{ctx.device}"
        rng = np.random.default_rng(cfg.seed)
        n = len(labels)
        if n < 1:
            raise ValueError("empty training set")
        order = rng.permutation(n)
        if mean is None:
            mean, istd = standardisation(features)
        self.mean, self.istd = np.asarray(mean, np.float32), np.asarray(istd, np.float32)
        self.n = n
        self.rng = rng
        f_dev = torch.from_numpy(np.ascontiguousarray(features[order], np.float32)).to(dev)
        self.y = torch.from_numpy(np.ascontiguousarray(labels[order], np.uint8)).to(dev)
        self.mean_d = torch.from_numpy(self.mean).to(dev)
        self.istd_d = torch.from_numpy(self.istd).to(dev)
        self.x = torch.empty((n, 64), dtype=torch.int16, device=dev)
        ctx.mlp_prepare(f_dev, self.mean_d, self.istd_d, self.x, self.stream)
        del f_dev
        self.P = torch.from_numpy(np.ascontiguousarray(init_params, np.float32)).to(dev)
        self.m = torch.zeros_like(self.P)
        self.v = torch.zeros_like(self.P)
        self.grad = torch.zeros_like(self.P)
        b = min(cfg.batch, n)
        self.b = b
        self.logits = torch.empty(b, dtype=torch.float32, device=dev)
        self.h1 = torch.empty((b, 64), dtype=torch.int16, device=dev)
        self.h2 = torch.empty((b, 64), dtype=torch.float32, device=dev)
        self.work = torch.empty(ctx.mlp_workspace_bytes(b), dtype=torch.uint8, device=dev)
        self.n_batches = n // b          # the ragged tail of the shuffled set is left out
        self.losses = torch.zeros(max(self.n_batches, 1), dtype=torch.float32, device=dev)
        self.step_no = 0

    def step(self, k: int):
        """one Adam step on batch k"""
        c, s, b = self.ctx, self.stream, self.b
        x = self.x[k * b:(k + 1) * b]
        y = self.y[k * b:(k + 1) * b]
        c.mlp_forward(self.P, x, self.logits, self.h1, self.h2, s)
        c.mlp_backward(self.P, x, y, self.logits, self.h1, self.h2, self.work, self.grad,
                       self.losses[k:k + 1], s)
        self.step_no += 1
        cf = self.cfg
        c.mlp_adam(self.P, self.grad, self.m, self.v, self.step_no, cf.lr, cf.beta1, cf.beta2,
                   cf.eps, s)

    def epoch(self, per_step: bool = False) -> float:
        """one pass over the batches in a random order: all its steps in one
        library call (per_step: one call per step, same results)"""
        order = self.rng.permutation(self.n_batches)
        if per_step:
            for k in order:
                self.step(int(k))
        else:
            cf = self.cfg
            self.ctx.mlp_train_steps(self.P, self.x, self.y, self.b, order, self.step_no,
                                     self.logits, self.h1, self.h2, self.work, self.grad, self.m,
                                     self.v, self.losses, cf.lr, cf.beta1, cf.beta2, cf.eps,
                                     self.stream)
            self.step_no += len(order)
        self.stream.synchronize()
        return float(np.mean(self.losses.cpu().numpy()))

    def fit(self, epochs: int | None = None) -> list:
        return [self.epoch() for _ in range(epochs or self.cfg.epochs)]

    def params(self) -> np.ndarray:
        self.stream.synchronize()
        return self.P.cpu().numpy()

    def logits_all(self) -> np.ndarray:
        """logits of the whole training set under the current weights"""
        out = torch.empty(self.n, dtype=torch.float32, device=self.x.device)
        self.ctx.mlp_forward(self.P, self.x, out, stream=self.stream)
        self.stream.synchronize()
        return out.cpu().numpy()

    def labels(self) -> np.ndarray:
        return self.y.cpu().numpy()


def threshold_for(logits: np.ndarray, labels: np.ndarray, keep_true: float) -> float:
    """the largest threshold that keeps at least `keep_true` of the true
    candidates (logit >= threshold)"""
    t = np.sort(np.asarray(logits, np.float64)[np.asarray(labels) == 1])
    if len(t) == 0:
        return float("-inf")
    k = int(np.floor((1.0 - keep_true) * len(t)))
    return float(np.nextafter(np.float32(t[k]), np.float32(-np.inf)))


def training_config(base):
    """the training-set recipe (see synth.events.scorer_training_config)"""
    from synth.events import scorer_training_config
    return scorer_training_config(base)


def evaluate(ctx: "L.Context", events, geo, stream=None) -> dict:
    """Efficiency, fake and duplicate rate of the kept quintuplets (truth
    definitions of synth.truth) and the fraction of kept quintuplets whose ten
    hits all come from one track, summed over `events`, which run as one
    batched launch."""
    from synth import truth as T
    tot = dict(n_obj=0, n_findable=0, n_found=0, n_fake=0, n_dup=0, n_pure=0)
    offs = np.zeros(len(events) + 1, np.int32)
    offs[1:] = np.cumsum([ev.n_hits for ev in events])
    cat = [np.concatenate([getattr(ev, a) for ev in events]) for a in ("x", "y", "z", "module", "sensor")]
    ctx.run_batch(offs, *cat, stream)
    for e, ev in enumerate(events):
        kept = ctx.objects(e, L.LST_T5_KEPT, stream)
        m = T.metrics(kept, ev, geo)
        for k in ("n_obj", "n_findable", "n_found", "n_fake", "n_dup"):
            tot[k] += m[k]
        tot["n_pure"] += int(pure_labels(kept, ev.truth).sum())
    n = max(tot["n_obj"], 1)
    return dict(tot, eff=tot["n_found"] / max(tot["n_findable"], 1), fake=tot["n_fake"] / n,
                dup=tot["n_dup"] / n, impure=1.0 - tot["n_pure"] / n)
