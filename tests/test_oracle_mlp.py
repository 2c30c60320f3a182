"""Pins of the learned-scorer oracle (FP64 network, BF16 emulation, error
bound, backpropagation, Adam, duplicate removal with vetoes).

Each check compares the oracle with something other than itself: a library
rounding routine, a closed-form network, central finite differences, an FP32
evaluation in random summation orders, the first-step identity of Adam, or
brute-force pairwise duplicate removal.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as M
from synth import events as E
from synth import geometry as G
from synth import params as PR
from synth import weights as W


# ---------------------------------------------------------------- BF16 rounding
def test_bf16_fp32_matches_library_conversion():
    rng = np.random.default_rng(1)
    a = np.concatenate([
        rng.normal(0, 1, 20000), rng.normal(0, 1e-30, 1000), rng.normal(0, 1e30, 1000),
        # exact ties: 8 significant bits + a half in the 9th
        (1.0 + (2 * rng.integers(0, 128, 2000) + 1) * 2.0 ** -8) * 2.0 ** rng.integers(-20, 20, 2000),
        [0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, 3.4e38, -3.4e38, 1e-45]]).astype(np.float32)
    ours = M.bf16(a)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(ours.view(np.uint32), ref.view(np.uint32))
    assert np.isnan(M.bf16(np.array([np.nan], np.float32)))[0]


def test_bf16_fp64_ties_and_nearest():
    # grid step at 1 is 2^-7: a half step rounds to the even neighbour
    t = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 255.5 / 128], np.float64)
    assert list(M.bf16(t)) == [1.0, 1 + 2.0 ** -6, -1.0, 2.0]
    rng = np.random.default_rng(2)
    a = rng.normal(0, 1, 5000) * 10.0 ** rng.integers(-6, 6, 5000)
    r = M.bf16(a)
    # result is representable and no other representable value is closer
    assert np.array_equal(M.bf16(r.astype(np.float32)).astype(np.float64), r)
    step = np.ldexp(1.0, np.frexp(a)[1] - 8)
    assert np.all(np.abs(a - r) <= step / 2)
    # FP32-representable inputs round as in the FP32 path
    a32 = a.astype(np.float32)
    assert np.array_equal(M.bf16(a32.astype(np.float64)), M.bf16(a32).astype(np.float64))


def test_standardise_exact_values():
    F = np.array([[3.0] * 40], np.float32)
    x = M.standardise(F, np.full(40, 1.0, np.float32), np.full(40, 0.5, np.float32))
    assert np.all(x == 1.0)
    # the FP32 subtraction happens before the multiplication
    F = np.array([[1.0 + 2.0 ** -20] * 40], np.float32)
    x = M.standardise(F, np.full(40, 1.0, np.float32), np.full(40, 2.0 ** 20, np.float32))
    assert np.all(x == 1.0)


# ---------------------------------------------------------------- forward
def _identity_net(b3):
    P = np.zeros(M.N_PARAM, np.float32)
    p = M.unpack(P)
    p["W1"][:M.N_IN, :] = np.eye(M.N_IN)
    p["W2"][:] = np.eye(M.N_H)
    p["w3"][:] = 1.0
    p["b3"][:] = b3
    return P


def test_forward_closed_form_identity_network():
    rng = np.random.default_rng(3)
    X = M.bf16(rng.normal(0, 2, (300, 40)).astype(np.float32))
    lg, bound = M.forward(_identity_net(0.25), X)
    assert np.allclose(lg, np.maximum(X.astype(np.float64), 0).sum(axis=1) + 0.25, rtol=0, atol=1e-12)
    assert np.all(bound >= 0)


def test_forward_dead_hidden_layer_gives_bias():
    P = W.random_params(np.random.default_rng(4))
    M.unpack(P)["b1"][:] = -1e6
    M.unpack(P)["b2"][:] = 0.0
    M.unpack(P)["b3"][:] = -0.75
    X = M.bf16(np.random.default_rng(5).normal(0, 1, (50, 40)).astype(np.float32))
    lg, _ = M.forward(P, X)
    assert np.all(lg == -0.75)


def _fp32_eval(P, X, rng):
    """the network in FP32 with a random summation order per dot product,
    BF16 weights and BF16 re-rounding of the first hidden layer"""
    p = M.unpack(np.asarray(P, np.float32))
    W1, W2 = M.bf16(p["W1"]), M.bf16(p["W2"])

    def dot(terms, bias):
        # terms: [n, k] FP32 products; sum them in a random order, then bias
        acc = np.zeros(terms.shape[0], np.float32)
        for j in rng.permutation(terms.shape[1]):
            acc = (acc + terms[:, j]).astype(np.float32)
        return (acc + np.float32(bias)).astype(np.float32)

    X = X.astype(np.float32)
    z1 = np.stack([dot(X * W1[j], p["b1"][j]) for j in range(M.N_H)], axis=1)
    h1 = M.bf16(np.maximum(z1, np.float32(0)))
    z2 = np.stack([dot(h1 * W2[j], p["b2"][j]) for j in range(M.N_H)], axis=1)
    h2 = np.maximum(z2, np.float32(0))
    return dot((h2 * p["w3"]).astype(np.float32), p["b3"][0])


def test_error_bound_covers_fp32_evaluation_orders():
    rng = np.random.default_rng(6)
    P = W.random_params(rng, bias=0.3)
    X = M.bf16(rng.normal(0, 1.5, (400, 40)).astype(np.float32))
    lg, bound = M.forward(P, X)
    worst = 0.0
    for _ in range(4):
        v = _fp32_eval(P, X, rng).astype(np.float64)
        assert np.all(np.abs(v - lg) <= bound)
        worst = max(worst, float(np.max(np.abs(v - lg) / bound)))
    # the bound is not vacuous: small against the logits, and actually approached
    assert np.median(bound) < 1e-3 * np.median(np.abs(lg)) + 1e-4
    assert worst > 1e-4


# ---------------------------------------------------------------- loss and gradients
def test_bce_values():
    assert M.bce([0.0, 0.0], [0, 1]) == pytest.approx(math.log(2.0), rel=1e-15)
    assert M.bce([40.0], [1]) == pytest.approx(math.exp(-40.0), rel=1e-9)
    assert M.bce([-3.0], [1]) == pytest.approx(3.0 + math.log1p(math.exp(-3.0)), rel=1e-14)


def test_gradients_match_central_finite_differences():
    rng = np.random.default_rng(7)
    P = W.random_params(rng, bias=0.2).astype(np.float64)
    X = rng.normal(0, 1, (64, 40))
    y = rng.integers(0, 2, 64)
    loss, g = M.loss_and_grad(P, X, y, exact=True)
    assert loss == pytest.approx(M.bce(M.forward(P, X, exact=True)[0], y), rel=1e-14)
    # every parameter block, including each bias and the output layer
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in M.SIZES])
    idx = np.concatenate([rng.integers(offs[i], offs[i + 1], 12) for i in range(len(M.SIZES))])
    h = 1e-6
    for i in idx:
        d = np.zeros_like(P)
        d[i] = h
        fd = (M.bce(M.forward(P + d, X, exact=True)[0], y)
              - M.bce(M.forward(P - d, X, exact=True)[0], y)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, np.max(np.abs(g))), (i, fd, g[i])


def test_rounded_gradients_use_rounded_operands():
    # with BF16-representable weights and inputs the rounding is the identity
    # (hidden re-rounding aside), so rounded and exact gradients agree closely
    rng = np.random.default_rng(8)
    P = M.bf16(W.random_params(rng).astype(np.float32))
    X = M.bf16(rng.normal(0, 1, (128, 40)).astype(np.float32))
    y = rng.integers(0, 2, 128)
    _, g_r = M.loss_and_grad(P, X, y)
    _, g_e = M.loss_and_grad(P, X, y, exact=True)
    assert np.linalg.norm(g_r - g_e) <= 2e-2 * np.linalg.norm(g_e)


def test_adam_first_steps_closed_form():
    rng = np.random.default_rng(9)
    P = rng.normal(0, 1, 100)
    g = rng.normal(0, 1e-2, 100)
    m = v = np.zeros(100)
    lr, eps = 1e-3, 1e-8
    P1, m, v = M.adam(P, g, m, v, 1, lr, eps=eps)
    assert np.allclose(P1 - P, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=0)
    # a constant gradient keeps the bias-corrected moments at g and g^2
    P2, m, v = M.adam(P1, g, m, v, 2, lr, eps=eps)
    assert np.allclose(P2 - P1, -lr * g / (np.abs(g) + eps), rtol=1e-9, atol=0)


# ---------------------------------------------------------------- duplicate removal
def _dedup_pairs(tuples, scores, veto):
    n = len(tuples)
    keep = np.zeros(n, bool)
    for t in range(n):
        if veto[t]:
            continue
        kt = (float(scores[t]), tuple(tuples[t]))
        keep[t] = not any(not veto[u] and u != t and set(tuples[u]) & set(tuples[t])
                          and (float(scores[u]), tuple(tuples[u])) < kt for u in range(n))
    return keep


def test_dedup_matches_pairwise_definition():
    rng = np.random.default_rng(10)
    for trial in range(20):
        n = int(rng.integers(1, 60))
        tuples = np.stack([rng.choice(80, 10, replace=False) for _ in range(n)])
        scores = rng.integers(0, 6, n).astype(np.float32)      # many score ties
        veto = rng.random(n) < 0.3
        assert np.array_equal(M.dedup(tuples, scores, veto), _dedup_pairs(tuples, scores, veto))
    assert not M.dedup(tuples, scores, np.ones(len(tuples), bool)).any()


@pytest.mark.parametrize("cid,geo_name", [(1, "barrel_toy"), (2, "full")])
def test_dedup_without_vetoes_equals_chain_oracle(cid, geo_name):
    geo = G.get(geo_name)
    orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    r = orc.run_event(E.generate(cid, 0))
    t5 = r.tuples[oracle.T5]
    keep = M.dedup(t5, r.t5_scores, np.zeros(len(t5), bool))
    assert np.array_equal(keep, r.t5_keep)
