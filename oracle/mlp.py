"""CPU oracle of the learned quintuplet scorer -- TEST INFRASTRUCTURE.

Plain NumPy, FP64 unless stated.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark use it; the HIP library shares no code with
it.  The scorer is not part of the paper (its Summary and Outlook section
plans to revisit the object selection for efficiency and fake rate); what it
computes is fixed here by its definition:

* network 40 -> 64 -> 64 -> 1, ReLU after both hidden layers, a logit out;
  accept a candidate iff logit >= threshold (probability = sigmoid(logit));
* inputs: the 40 FP32 features, standardised in FP32 as (f - mean) * istd and
  rounded to BF16 (round to nearest, ties to even);
* hidden weights W1, W2 rounded to BF16, biases and the last layer FP32,
  products accumulated in FP32; the first hidden layer is rounded to BF16
  again before it feeds the second (the matrix-core operand type);
* training loss: binary cross entropy on the logit, mean over the batch;
  gradients flow through the BF16 roundings unchanged (straight-through);
* optimiser: Adam with bias correction.

The oracle evaluates the network in FP64 from the BF16 operands and returns,
per candidate, a bound on how far an FP32 evaluation in any summation order
(plus the BF16 re-rounding of hidden units that such an FP32 error can flip)
can land from the FP64 logit.  A scorer decision may differ from the
oracle's only where |logit - threshold| is within that bound.

Parameter vector (FP32), in this order: W1[64][40] (row = hidden unit),
b1[64], W2[64][64], b2[64], w3[64], b3.
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 40, 64
SIZES = (("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
         ("w3", (N_H,)), ("b3", (1,)))
N_PARAM = sum(int(np.prod(s)) for _, s in SIZES)
U32 = 2.0 ** -24          # unit roundoff of FP32
U64 = 2.0 ** -53


def unpack(P):
    """named views of the flat parameter vector"""
    P = np.asarray(P)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = P[o:o + n].reshape(shape)
        o += n
    return out


def bf16(a):
    """round to the nearest BF16 value, ties to even.  FP32 input is rounded
    from its bit pattern; FP64 input is rounded from its exact value (values
    beyond the FP32 range are not expected).  Returns the rounded values in
    the input's float type."""
    a = np.asarray(a)
    if a.dtype == np.float32:
        u = a.view(np.uint32).astype(np.uint64)
        nan = np.isnan(a)
        r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
        r = np.where(nan, (u >> 16) | 0x40, r)
        return (r.astype(np.uint32) << 16).view(np.float32).reshape(a.shape)
    a = a.astype(np.float64)
    m, e = np.frexp(a)                      # a = m 2^e, 0.5 <= |m| < 1
    # BF16 keeps 8 significant bits: the grid step near a is 2^(e-8)
    step = np.ldexp(1.0, (e - 8).astype(np.int64))
    q = a / step                             # exact (power-of-two scaling)
    return np.where(a == 0.0, a, np.round(q) * step)   # np.round: ties to even


def standardise(F, mean, istd):
    """FP32 (f - mean) * istd, then BF16"""
    F = np.asarray(F, np.float32)
    x = (F - np.asarray(mean, np.float32)) * np.asarray(istd, np.float32)
    return bf16(x.astype(np.float32))


def _gamma(n, u=U32):
    return n * u / (1.0 - n * u)


def forward(P, X, exact=False):
    """logits (FP64) and the per-row error bound.

    P: the FP32 parameter vector (FP64 accepted: the rounded copies are
    taken from its exact values).  X: [n, 40] BF16-valued inputs.  With
    exact=True nothing is rounded (the smooth function the finite-difference
    checks differentiate)."""
    p = unpack(np.asarray(P, np.float64))
    X = np.asarray(X, np.float64)
    q = (lambda a: a) if exact else bf16
    W1, W2 = q(p["W1"]), q(p["W2"])
    b1, b2, w3, b3 = p["b1"], p["b2"], p["w3"], float(p["b3"][0])
    z1 = X @ W1.T + b1
    h1 = q(np.maximum(z1, 0.0))
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    logit = h2 @ w3 + b3
    if exact:
        return logit, None
    # error bound: FP32 accumulation of k terms (any order) errs by at most
    # gamma_k times the sum of magnitudes; FP64 evaluation error added on top
    g = _gamma(N_H + 2) + _gamma(N_H + 2, U64)
    e1 = g * (np.abs(X) @ np.abs(W1).T + np.abs(b1))
    lo = bf16(np.maximum(z1 - e1, 0.0))
    hi = bf16(np.maximum(z1 + e1, 0.0))
    dh1 = np.maximum(np.abs(hi - h1), np.abs(h1 - lo))   # BF16 flips within reach
    e2 = dh1 @ np.abs(W2).T + g * ((np.abs(h1) + dh1) @ np.abs(W2).T + np.abs(b2))
    bound = e2 @ np.abs(w3) + g * ((np.abs(h2) + e2) @ np.abs(w3) + abs(b3))
    return logit, bound


def bce(logit, y):
    """mean binary cross entropy on logits, FP64"""
    z = np.asarray(logit, np.float64)
    y = np.asarray(y, np.float64)
    return float(np.mean(np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def loss_and_grad(P, X, y, exact=False):
    """loss and dL/dP (flat, FP64) by backpropagation through the forward
    above; BF16 roundings pass gradients unchanged"""
    p = unpack(np.asarray(P, np.float64))
    X = np.asarray(X, np.float64)
    y = np.asarray(y, np.float64)
    n = X.shape[0]
    q = (lambda a: a) if exact else bf16
    W1, W2 = q(p["W1"]), q(p["W2"])
    b1, b2, w3, b3 = p["b1"], p["b2"], p["w3"], float(p["b3"][0])
    z1 = X @ W1.T + b1
    h1 = q(np.maximum(z1, 0.0))
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    z = h2 @ w3 + b3
    loss = bce(z, y)
    # dL/dz of the mean BCE: (sigmoid(z) - y) / n
    gz = (1.0 / (1.0 + np.exp(-z)) - y) / n
    d_w3 = h2.T @ gz
    d_b3 = np.sum(gz)
    dz2 = np.outer(gz, w3) * (z2 > 0)
    d_W2 = dz2.T @ h1
    d_b2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2) * (h1 > 0)
    d_W1 = dz1.T @ X
    d_b1 = dz1.sum(axis=0)
    grad = np.concatenate([d_W1.ravel(), d_b1, d_W2.ravel(), d_b2, d_w3, [d_b3]])
    return loss, grad


def adam(P, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """one Adam update with bias correction; returns (P, m, v) in FP64"""
    P, g = np.asarray(P, np.float64), np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return P - lr * mh / (np.sqrt(vh) + eps), m, v


def dedup(tuples, scores, veto):
    """Duplicate removal over shared hits, straight from its definition: a
    quintuplet survives iff it is not vetoed and, among the non-vetoed
    quintuplets that share any hit with it, it has the smallest key
    (score, then hit tuple lexicographically)."""
    tuples = np.asarray(tuples, np.int64)
    n = tuples.shape[0]
    keep = np.zeros(n, bool)
    live = np.flatnonzero(~np.asarray(veto, bool))
    if live.size == 0:
        return keep
    # rank of every live quintuplet under the (score, tuple) order
    keys = [tuples[live, k] for k in range(tuples.shape[1] - 1, -1, -1)]
    order = np.lexsort(keys + [np.asarray(scores, np.float32)[live]])
    rank = np.empty(live.size, np.int64)
    rank[order] = np.arange(live.size)
    best = np.full(int(tuples.max()) + 1, np.iinfo(np.int64).max)
    for k in range(tuples.shape[1]):
        np.minimum.at(best, tuples[live, k], rank)
    ok = np.all(best[tuples[live]] == rank[:, None], axis=1)
    keep[live[ok]] = True
    return keep



def score_t5(features, scores, tuples, P, mean, istd, threshold):
    """The scored chain's last two steps on the oracle's quintuplets: veto
    every quintuplet whose logit is below the threshold, then remove
    duplicates among the rest.  Returns (logit, bound, veto, keep)."""
    X = standardise(features, mean, istd)
    logit, bound = forward(P, X)
    veto = logit < threshold
    return logit, bound, veto, dedup(tuples, scores, veto)
