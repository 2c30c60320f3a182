"""Parity of the learned scorer's kernels with the CPU oracle (-m gpu).

* preparation (standardise + BF16): bit-exact;
* forward (MFMA): every logit within the oracle's per-row error bound;
* backward: gradients against FP64 backpropagation, relative L2 error per
  parameter block <= 1e-3 (FP32 sums over <= 4096 rows plus the BF16 flips
  the forward bound allows), and bit-for-bit reproducible;
* Adam: against the FP64 update within a few FP32 ulps;
* scoring inside the chain: logits within the bound, vetoes equal (the
  threshold is put in a gap of the oracle's logits wider than the bounds),
  surviving quintuplets equal to the oracle's dedup with those vetoes, for
  the per-stage, graph and persistent launches.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as M
from synth import events as E
from synth import geometry as G
from synth import params as PR
from synth import weights as W

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _lst():
    import paper_2209_13711_amd as lst
    return lst


@pytest.fixture(scope="module")
def ctx_toy():
    lst = _lst()
    geo = G.get("barrel_toy")
    return lst.Context(PR.make(), geo.f32, geo.i32, device=0)


def _features(rng, n):
    """feature-like FP32 rows: mixed scales, some exact zeros and ones"""
    f = rng.normal(0, 1, (n, 40)) * 10.0 ** rng.integers(-2, 2, 40)
    f[:, 15:20] = rng.integers(0, 2, (n, 5))
    return f.astype(np.float32)


def _prepare(ctx, F, mean, istd):
    x = torch.empty((len(F), 64), dtype=torch.int16, device=DEV)
    ctx.mlp_prepare(torch.from_numpy(F).to(DEV), torch.from_numpy(mean).to(DEV),
                    torch.from_numpy(istd).to(DEV), x)
    return x


def _stats(F):
    return (F.mean(axis=0).astype(np.float32),
            (1.0 / np.maximum(F.std(axis=0), 1e-6)).astype(np.float32))


def _bits_to_f32(x16):
    return (x16.astype(np.uint16).astype(np.uint32) << 16).view(np.float32)


@pytest.mark.parametrize("n", [1, 597, 20000])
def test_prepare_bit_exact(ctx_toy, n):
    rng = np.random.default_rng(n)
    F = _features(rng, n)
    mean, istd = _stats(F)
    x = _prepare(ctx_toy, F, mean, istd).cpu().numpy()
    ref = M.standardise(F, mean, istd)
    assert np.array_equal(_bits_to_f32(x[:, :40]).view(np.uint32), ref.view(np.uint32))
    assert not x[:, 40:].any()


@pytest.mark.parametrize("n,bias", [(1, 0.0), (16, 0.1), (597, 0.3), (200003, 0.3)])
def test_forward_within_error_bound(ctx_toy, n, bias):
    print(f"case forward n={n}", flush=True)
    rng = np.random.default_rng(100 + n)
    F = _features(rng, n)
    mean, istd = _stats(F)
    P = W.random_params(rng, bias=bias)
    x = _prepare(ctx_toy, F, mean, istd)
    out = torch.full((n,), float("nan"), dtype=torch.float32, device=DEV)
    ctx_toy.mlp_forward(torch.from_numpy(P).to(DEV), x, out)
    got = out.cpu().numpy().astype(np.float64)
    lg, bound = M.forward(P, M.standardise(F, mean, istd))
    assert np.all(np.isfinite(got))
    bad = np.abs(got - lg) > bound
    assert not bad.any(), (np.flatnonzero(bad)[:5], got[bad][:5], lg[bad][:5], bound[bad][:5])


def test_forward_empty_is_noop(ctx_toy):
    P = torch.from_numpy(W.random_params(np.random.default_rng(1))).to(DEV)
    x = torch.empty((0, 64), dtype=torch.int16, device=DEV)
    out = torch.empty(0, dtype=torch.float32, device=DEV)
    ctx_toy.mlp_forward(P, x, out)
    torch.cuda.synchronize()


def _grads_gpu(ctx, P, x, y):
    n = x.shape[0]
    Pd = torch.from_numpy(P).to(DEV)
    yd = torch.from_numpy(y.astype(np.uint8)).to(DEV)
    lg = torch.empty(n, dtype=torch.float32, device=DEV)
    h1 = torch.empty((n, 64), dtype=torch.int16, device=DEV)
    h2 = torch.empty((n, 64), dtype=torch.float32, device=DEV)
    work = torch.empty(ctx.mlp_workspace_bytes(n), dtype=torch.uint8, device=DEV)
    grad = torch.empty(M.N_PARAM, dtype=torch.float32, device=DEV)
    loss = torch.empty(1, dtype=torch.float32, device=DEV)
    ctx.mlp_forward(Pd, x, lg, h1, h2)
    ctx.mlp_backward(Pd, x, yd, lg, h1, h2, work, grad, loss)
    torch.cuda.synchronize()
    return grad.cpu().numpy(), float(loss.cpu().numpy()[0])


# 5000 rows: 79 batches of 64 in 64 chunks of two batches each (the last
# batch ragged, the last 24 chunks empty)
@pytest.mark.parametrize("n", [1, 1000, 4096, 5000])
def test_backward_matches_oracle(ctx_toy, n):
    print(f"case backward n={n}", flush=True)
    rng = np.random.default_rng(200 + n)
    F = _features(rng, n)
    mean, istd = _stats(F) if n > 1 else (np.zeros(40, np.float32), np.ones(40, np.float32))
    P = W.random_params(rng, bias=0.2)
    y = rng.integers(0, 2, n)
    x = _prepare(ctx_toy, F, mean, istd)
    g, loss = _grads_gpu(ctx_toy, P, x, y)
    loss_ref, g_ref = M.loss_and_grad(P, M.standardise(F, mean, istd), y)
    assert loss == pytest.approx(loss_ref, rel=1e-5, abs=1e-6)
    o = 0
    for name, shape in M.SIZES:
        k = int(np.prod(shape))
        a, b = g[o:o + k].astype(np.float64), g_ref[o:o + k]
        o += k
        scale = np.linalg.norm(b)
        assert np.linalg.norm(a - b) <= 1e-3 * scale + 1e-9, (name, np.linalg.norm(a - b), scale)


def test_backward_bitwise_reproducible(ctx_toy):
    rng = np.random.default_rng(7)
    F = _features(rng, 4096)
    mean, istd = _stats(F)
    P = W.random_params(rng)
    y = rng.integers(0, 2, 4096)
    x = _prepare(ctx_toy, F, mean, istd)
    g1, l1 = _grads_gpu(ctx_toy, P, x, y)
    g2, l2 = _grads_gpu(ctx_toy, P, x, y)
    assert np.array_equal(g1.view(np.uint32), g2.view(np.uint32)) and l1 == l2


def test_adam_matches_oracle(ctx_toy):
    rng = np.random.default_rng(8)
    P = W.random_params(rng, bias=0.1)
    Pd = torch.from_numpy(P.copy()).to(DEV)
    m = torch.zeros_like(Pd)
    v = torch.zeros_like(Pd)
    Pr, mr, vr = P.astype(np.float64), np.zeros(M.N_PARAM), np.zeros(M.N_PARAM)
    lr = 1e-3
    for step in range(1, 4):
        g = (rng.normal(0, 1e-2, M.N_PARAM) * 10.0 ** rng.integers(-3, 1, M.N_PARAM)).astype(np.float32)
        ctx_toy.mlp_adam(Pd, torch.from_numpy(g).to(DEV), m, v, step, lr)
        Pr, mr, vr = M.adam(Pr, g, mr, vr, step, lr)
    got = Pd.cpu().numpy().astype(np.float64)
    ulp = np.spacing(np.abs(Pr).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(got - Pr) <= 4 * ulp + 1e-5 * lr)


def test_adam_rejects_bad_hyperparameters(ctx_toy):
    lst = _lst()
    P = torch.zeros(M.N_PARAM, dtype=torch.float32, device=DEV)
    with pytest.raises(lst.LSTError):
        ctx_toy.mlp_adam(P, P, P.clone(), P.clone(), 0, 1e-3)
    with pytest.raises(lst.LSTError):
        ctx_toy.mlp_adam(P, P, P.clone(), P.clone(), 1, -1.0)


def test_train_steps_in_one_call_equal_per_step_calls(ctx_toy):
    """lst_mlp_train_steps runs the same kernels in the same order as one
    forward, backward and Adam call per step: parameters, moments and losses
    equal bit for bit after two epochs over a ragged training set (its tail
    is left out), then the argument checks"""
    from paper_2209_13711_amd import scorer as S
    lst = _lst()
    rng = np.random.default_rng(11)
    n = 3 * 1024 + 517
    F = _features(rng, n)
    y = (rng.random(n) < 0.4).astype(np.uint8)
    P0 = W.random_params(rng, bias=0.05)
    cfg = S.TrainConfig(epochs=2, batch=1024, lr=3e-3, seed=5)
    runs = []
    for per_step in (True, False):
        tr = S.Trainer(ctx_toy, F, y, P0, cfg)
        losses = [tr.epoch(per_step=per_step) for _ in range(cfg.epochs)]
        torch.cuda.synchronize()
        runs.append((losses, tr.step_no, [t.cpu().numpy().view(np.uint32)
                                          for t in (tr.P, tr.m, tr.v, tr.losses)]))
    (l1, s1, a1), (l2, s2, a2) = runs
    assert s1 == s2 == 2 * (n // 1024)
    assert l1 == l2
    assert all(np.array_equal(a, b) for a, b in zip(a1, a2))
    assert not np.array_equal(a1[0], P0.view(np.uint32))
    # order outside the batches, empty workspace, bad hyper-parameters
    tr = S.Trainer(ctx_toy, F, y, P0, cfg)
    args = (tr.P, tr.x, tr.y, tr.b)
    rest = (tr.logits, tr.h1, tr.h2, tr.work, tr.grad, tr.m, tr.v, tr.losses)
    with pytest.raises(lst.LSTError):
        ctx_toy.mlp_train_steps(*args, [0, n // 1024], 0, *rest, 1e-3)
    with pytest.raises(lst.LSTError):
        ctx_toy.mlp_train_steps(*args, [-1], 0, *rest, 1e-3)
    with pytest.raises(lst.LSTError):
        ctx_toy.mlp_train_steps(*args, [0], 0, *rest[:3], tr.work[:16], *rest[4:], 1e-3)
    with pytest.raises(lst.LSTError):
        ctx_toy.mlp_train_steps(*args, [0], 0, *rest, -1.0)
    ctx_toy.mlp_train_steps(*args, [], 0, *rest, 1e-3)      # no step: nothing happens
    torch.cuda.synchronize()
    assert np.array_equal(tr.P.cpu().numpy(), P0)


# ---------------------------------------------------------------- scoring in the chain
def _gap_threshold(lg, bound, q=0.5):
    """a threshold near the q-quantile of the logits with no logit within
    twice its bound on either side"""
    order = np.argsort(lg)
    s = lg[order]
    mid = int(q * len(s))
    for d in range(len(s)):
        for i in (mid + d, mid - d):
            if 0 < i < len(s):
                th = float(np.float32(0.5 * (s[i - 1] + s[i])))
                if np.all(np.abs(lg - th) > 2 * bound):
                    return th
    raise AssertionError("no gap")


def _scored_case(cid, event=0, n_tracks=None, seed=0):
    lst = _lst()
    cfg = E.CONFIGS[cid]
    geo = G.get(cfg.geometry)
    params = PR.make(w=cfg.window)
    ev = E.generate(cid, event, n_tracks=n_tracks)
    ref = oracle.Oracle(params, geo.f32, geo.i32).run_event(ev)
    mean, istd = _stats(ref.t5_features)
    P = W.random_params(np.random.default_rng(seed), bias=0.2)
    lg, bound = M.forward(P, M.standardise(ref.t5_features, mean, istd))
    th = _gap_threshold(lg, bound)
    veto = lg < th
    keep = M.dedup(ref.tuples[oracle.T5], ref.t5_scores, veto)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    ctx.mlp_load(P, mean, istd, th)
    ctx.set_mode(lst.LST_MODE_MLP)
    return ctx, ev, ref, dict(lg=lg, bound=bound, veto=veto, keep=keep, th=th)


def _check_scored(ctx, ref, exp):
    lst = _lst()
    t5 = ctx.objects(0, lst.LST_T5)
    lg, veto = ctx.t5_logits(0)
    idx = {tuple(t): i for i, t in enumerate(ref.tuples[oracle.T5].tolist())}
    assert len(t5) == len(idx) and all(tuple(t) in idx for t in t5.tolist())
    j = np.array([idx[tuple(t)] for t in t5.tolist()], np.int64)
    assert np.all(np.abs(lg.astype(np.float64) - exp["lg"][j]) <= exp["bound"][j])
    assert np.array_equal(veto, exp["veto"][j])
    kept = {tuple(t) for t in ctx.objects(0, lst.LST_T5_KEPT).tolist()}
    want = {tuple(t) for t in ref.tuples[oracle.T5][exp["keep"]].tolist()}
    assert kept == want
    return len(kept)


@pytest.mark.parametrize("cid,event,n_tracks", [(1, 0, None), (2, 0, None), (5, 0, 1500)])
def test_scored_chain_matches_oracle(cid, event, n_tracks):
    print(f"case scored chain cfg{cid} event {event}", flush=True)
    ctx, ev, ref, exp = _scored_case(cid, event, n_tracks)
    offs = np.array([0, ev.n_hits], np.int32)
    ctx.run_batch(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor)
    _check_scored(ctx, ref, exp)
    assert 0 < exp["veto"].sum() < len(exp["veto"])   # the vetoes are not trivial


def test_scored_chain_stagewise_graph_and_persistent():
    lst = _lst()
    ctx, ev, ref, exp = _scored_case(2, 1, 1500, seed=3)
    offs = np.array([0, ev.n_hits], np.int32)
    ctx.run_batch(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor)
    # stage by stage, with the scoring step called explicitly
    ctx.load_hits(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor)
    for fn in (ctx.run_sort, ctx.run_md, ctx.run_segments, ctx.run_triplets, ctx.run_quintuplets,
               ctx.run_t5_score, ctx.run_dedup):
        fn()
    _check_scored(ctx, ref, exp)
    for _ in range(3):
        ctx.run_chain_graph()
        _check_scored(ctx, ref, exp)
    ctx.run_chain_persistent()
    _check_scored(ctx, ref, exp)
    # back to the plain chain: the oracle's own dedup result
    ctx.set_mode(lst.LST_MODE_CUTS)
    ctx.run_chain_graph()
    kept = {tuple(t) for t in ctx.objects(0, lst.LST_T5_KEPT).tolist()}
    assert kept == {tuple(t) for t in ref.tuples[oracle.T5_KEPT].tolist()}


def test_scorer_fallback_and_state_errors(ctx_toy):
    """scorer mode with no usable network runs the plain cut chain and says
    so in the counts; weights that are not finite are refused and unload the
    kind's earlier network"""
    lst = _lst()
    geo = G.get("barrel_toy")
    params = PR.make()
    ev = E.generate(1, 0)
    plain = oracle.Oracle(params, geo.f32, geo.i32).run_event(ev)
    kept_ref = {tuple(t) for t in plain.tuples[oracle.T5_KEPT].tolist()}
    offs = np.array([0, ev.n_hits], np.int32)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)

    def run_all(expect_fallback, expect_plain):
        for chain in (ctx.run_chain, ctx.run_chain_graph, ctx.run_chain_persistent):
            ctx.load_hits(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor)
            chain()
            assert ctx.counts(0)["mlp_fallback"] == expect_fallback
            kept = {tuple(t) for t in ctx.objects(0, lst.LST_T5_KEPT).tolist()}
            assert (kept == kept_ref) == expect_plain

    ctx.set_mode(lst.LST_MODE_MLP)           # nothing loaded
    run_all(1, True)
    P = W.random_params(np.random.default_rng(0))
    ctx.mlp_load(P, np.zeros(40), np.ones(40), 1e30)   # vetoes every quintuplet
    run_all(0, False)
    assert ctx.counts(0)["n_t5_kept"] == 0
    bad = P.copy()
    bad[5] = np.nan
    with pytest.raises(lst.LSTError) as e:
        ctx.mlp_load(bad, np.zeros(40), np.ones(40), 0.0)
    assert e.value.code == lst.lst.LST_E_INVALID
    run_all(1, True)                         # the earlier network is gone
    ctx.set_mode(lst.LST_MODE_CUTS)
    run_all(0, True)
    ctx.mlp_load(P, np.zeros(40), np.ones(40), 0.0)
    ctx.run_event(ev)
    with pytest.raises(lst.LSTError) as e:   # after dedup: out of order
        ctx.run_t5_score()
    assert e.value.code == lst.lst.LST_E_STATE


# ---------------------------------------------------------------- triplet scoring
def _scored_case_both(cid, event=0, n_tracks=None, seed=0):
    """both scorers: triplet veto before the quintuplet stage, quintuplet veto
    before dedup; expected values from the oracle's rerun with the triplet veto"""
    lst = _lst()
    cfg = E.CONFIGS[cid]
    geo = G.get(cfg.geometry)
    params = PR.make(w=cfg.window)
    ev = E.generate(cid, event, n_tracks=n_tracks)
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    ref3 = orc.run_event(ev)
    m3, s3 = _stats(ref3.t3_features)
    P3 = W.random_params(np.random.default_rng(seed + 100), bias=0.2)
    lg3, b3 = M.forward(P3, M.standardise(ref3.t3_features, m3, s3))
    th3 = _gap_threshold(lg3, b3, q=0.15)   # veto some triplets, keep most quintuplets
    veto3 = lg3 < th3
    ref = orc.rerun_t5(veto3)
    assert len(ref.tuples[oracle.T5]) > 10
    m5, s5 = _stats(ref.t5_features)
    P5 = W.random_params(np.random.default_rng(seed), bias=0.2)
    lg5, b5 = M.forward(P5, M.standardise(ref.t5_features, m5, s5))
    th5 = _gap_threshold(lg5, b5)
    veto5 = lg5 < th5
    keep = M.dedup(ref.tuples[oracle.T5], ref.t5_scores, veto5)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    ctx.mlp_load(P3, m3, s3, th3, kind=lst.LST_T3)
    ctx.mlp_load(P5, m5, s5, th5, kind=lst.LST_T5)
    ctx.set_mode(lst.LST_MODE_MLP)
    exp3 = dict(t3=ref3.tuples[oracle.T3], lg=lg3, bound=b3, veto=veto3)
    exp5 = dict(lg=lg5, bound=b5, veto=veto5, keep=keep)
    return ctx, ev, ref, exp3, exp5


def _check_t3(ctx, exp3):
    lst = _lst()
    t3 = ctx.objects(0, lst.LST_T3)
    lg, veto = ctx.t3_logits(0)
    idx = {tuple(t): i for i, t in enumerate(exp3["t3"].tolist())}
    assert len(t3) == len(idx) and all(tuple(t) in idx for t in t3.tolist())
    j = np.array([idx[tuple(t)] for t in t3.tolist()], np.int64)
    assert np.all(np.abs(lg.astype(np.float64) - exp3["lg"][j]) <= exp3["bound"][j])
    assert np.array_equal(veto, exp3["veto"][j])


@pytest.mark.parametrize("cid,event,n_tracks", [(1, 0, None), (2, 0, None), (5, 0, 1500)])
def test_triplet_and_quintuplet_scoring_match_oracle(cid, event, n_tracks):
    print(f"case scored chain (T3 + T5) cfg{cid} event {event}", flush=True)
    ctx, ev, ref, exp3, exp5 = _scored_case_both(cid, event, n_tracks)
    assert 0 < exp3["veto"].sum() < len(exp3["veto"])
    offs = np.array([0, ev.n_hits], np.int32)
    ctx.run_batch(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor)
    _check_t3(ctx, exp3)
    _check_scored(ctx, ref, exp5)


def test_triplet_scoring_stagewise_graph_and_persistent():
    ctx, ev, ref, exp3, exp5 = _scored_case_both(2, 1, 1500, seed=5)
    offs = np.array([0, ev.n_hits], np.int32)
    ctx.run_batch(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor)
    ctx.load_hits(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor)
    for fn in (ctx.run_sort, ctx.run_md, ctx.run_segments, ctx.run_triplets, ctx.run_t3_score,
               ctx.run_quintuplets, ctx.run_t5_score, ctx.run_dedup):
        fn()
    _check_t3(ctx, exp3)
    _check_scored(ctx, ref, exp5)
    for _ in range(3):
        ctx.run_chain_graph()
        _check_t3(ctx, exp3)
        _check_scored(ctx, ref, exp5)
    ctx.run_chain_persistent()
    _check_t3(ctx, exp3)
    _check_scored(ctx, ref, exp5)
    t = ctx.tuning()
    ctx.set_tuning(t["grid"], persistent=1, blocks_per_cu=1)
    ctx.run_chain_graph()                       # persistent kernel inside the graph
    _check_scored(ctx, ref, exp5)


def test_t3_features_bitwise():
    lst = _lst()
    geo = G.get("full")
    params = PR.make()
    ev = E.generate(2, 3, n_tracks=1500)
    ref = oracle.Oracle(params, geo.f32, geo.i32).run_event(ev)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    caps = lst.default_caps(1, ev.n_hits)
    caps["features"] = 1
    ctx.reserve(caps)
    ctx.run_event(ev)
    ctx.run_t3_features()
    f = ctx.t3_features(0)
    t3 = ctx.objects(0, lst.LST_T3)
    want = {tuple(t): r for t, r in zip(ref.tuples[oracle.T3].tolist(), ref.t3_features)}
    assert len(t3) == len(want)
    for t, row in zip(t3.tolist(), f):
        assert np.array_equal(row.view(np.uint32), want[tuple(t)].view(np.uint32))


# ---------------------------------------------------------------- training and gain
def _assert_gain(plain, wide, scored):
    """Three arms on the same held-out events: the plain chain at nominal
    windows, the plain chain at the widened training windows, and the widened
    chain with both learned vetoes.  Widening and the networks are told
    apart: the scored chain finds more tracks than the nominal chain, and
    against the widened chain alone the networks lower the share of kept
    quintuplets with a foreign hit and do not raise the fake rate, for at
    most 0.2 points of efficiency."""
    assert scored["eff"] >= plain["eff"] + 0.003
    assert scored["eff"] >= wide["eff"] - 0.002
    assert scored["fake"] <= wide["fake"]
    assert scored["impure"] < wide["impure"]


def test_training_on_gpu_gains_over_plain_chain():
    """Train both scorers from scratch on the GPU (triplets, then the
    quintuplets that survive the trained triplet veto, of 40 widened-window
    training events, labelled by truth) and compare, on 4 held-out 4000-helix
    events, the plain chain at the nominal windows with the widened chain plus
    the learned vetoes, with the plain chain at the widened windows as the
    third arm (see _assert_gain)."""
    lst = _lst()
    from paper_2209_13711_amd import scorer as S
    geo = G.get("barrel_toy")
    tcfg = S.training_config(E.CONFIGS[4])
    train = [E.generate(4, e, purpose=E.PURPOSE_TRAIN, cfg=tcfg) for e in range(40)]
    print("case training: events generated", flush=True)
    ctx_w = lst.Context(PR.make(w=tcfg.window), geo.f32, geo.i32, device=0)
    models = {}
    for kind in (lst.LST_T3, lst.LST_T5):
        F, y = S.collect(ctx_w, train, kind=kind)
        assert len(y) > 50000 and 0.1 < y.mean() < 0.98
        tr = S.Trainer(ctx_w, F, y, W.random_params(np.random.default_rng(kind)),
                       S.TrainConfig(epochs=8))
        losses = tr.fit()
        print("kind", kind, "losses", losses, flush=True)
        assert losses[-1] < 0.8 * losses[0]
        lg, lab = tr.logits_all(), tr.labels()
        th = S.threshold_for(lg, lab, 0.995 if kind == lst.LST_T3 else 0.99)
        assert np.mean(lg[lab == 0] < th) > 0.05     # rejects a real share of wrong ones
        models[kind] = (tr.params(), tr.mean, tr.istd, th)
        # the quintuplet scorer learns on what survives the triplet veto
        ctx_w.mlp_load(*models[kind], kind=kind)
        ctx_w.set_mode(lst.LST_MODE_MLP)
    evs = [E.generate(4, e) for e in range(4)]
    plain = S.evaluate(lst.Context(PR.make(), geo.f32, geo.i32, device=0), evs, geo)
    wide = S.evaluate(lst.Context(PR.make(w=tcfg.window), geo.f32, geo.i32, device=0), evs, geo)
    scored = S.evaluate(ctx_w, evs, geo)
    print("plain", plain, "plain widened", wide, "scored", scored, flush=True)
    _assert_gain(plain, wide, scored)


def test_training_on_full_geometry_gains_over_plain_chain():
    """The same training on the full geometry (barrel and endcap disks, PS and
    2S modules, 1 % inefficiency, 5 % noise hits): 40 widened-window training
    events, 4 held-out PU200-like events, the same three arms; the scored
    chain also has a lower fake rate than the plain chain at nominal windows."""
    lst = _lst()
    from paper_2209_13711_amd import scorer as S
    geo = G.get("full")
    tcfg = S.training_config(E.CONFIGS[2])
    train = [E.generate(2, e, purpose=E.PURPOSE_TRAIN, cfg=tcfg) for e in range(40)]
    print("case full-geometry training: events generated", flush=True)
    ctx_w = lst.Context(PR.make(w=tcfg.window), geo.f32, geo.i32, device=0)
    for kind in (lst.LST_T3, lst.LST_T5):
        F, y = S.collect(ctx_w, train, kind=kind)
        assert len(y) > 50000 and 0.1 < y.mean() < 0.98
        # endcap and 2S flags of the first MD both occur in the training set
        assert 0.0 < F[:, 3].mean() < 1.0 and 0.0 < F[:, 4].mean() < 1.0
        tr = S.Trainer(ctx_w, F, y, W.random_params(np.random.default_rng(10 + kind)),
                       S.TrainConfig(epochs=8))
        losses = tr.fit()
        print("kind", kind, "losses", losses, flush=True)
        assert losses[-1] < 0.8 * losses[0]
        lg, lab = tr.logits_all(), tr.labels()
        th = S.threshold_for(lg, lab, 0.995 if kind == lst.LST_T3 else 0.99)
        ctx_w.mlp_load(tr.params(), tr.mean, tr.istd, th, kind=kind)
        ctx_w.set_mode(lst.LST_MODE_MLP)
    evs = [E.generate(2, 200 + e) for e in range(4)]
    plain = S.evaluate(lst.Context(PR.make(), geo.f32, geo.i32, device=0), evs, geo)
    wide = S.evaluate(lst.Context(PR.make(w=tcfg.window), geo.f32, geo.i32, device=0), evs, geo)
    scored = S.evaluate(ctx_w, evs, geo)
    print("plain", plain, "plain widened", wide, "scored", scored, flush=True)
    _assert_gain(plain, wide, scored)
    assert scored["fake"] < plain["fake"]
