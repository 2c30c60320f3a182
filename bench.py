"""Benchmark of the Segment Linking hot path on one MI355X.

Default workload: one PU200-like event (about 4000 helices, full geometry with
barrel and endcap disks, 1 % hit inefficiency, 5 % noise hits) through the
plain chain: hit grouping -> mini-doublets -> segments -> triplets ->
quintuplets -> duplicate removal.  A step is one pass of that chain over the
event, whose hits are already resident in device memory (the paper's timing
also excludes the host-to-device copy of hits, Sec. 3).

Prints ONE JSON line with events/s, a roofline entry for the dominant kernel
(algorithmic bytes per launch over its HIP-event-timed duration against
8 TB/s) and the CPU oracle's own rate on the host cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
COPY_BYTES = 1 << 30
# algorithmic FLOPs of the scorer per candidate (40x64 + 64x64 + 64 multiply-adds)
MLP_FLOPS = 2 * (40 * 64 + 64 * 64 + 64)
TRAFFIC_DIR = os.path.join(ROOT, "profiles")


KERNEL_SOURCES = ("lst_kernels.hip", "lst_cuts.hpp", "lst_internal.hpp", "lst_access.hpp")


def code_digest(texts):
    """Digest of C++ sources with comments, trailing blanks and empty lines
    removed: a comment edit keeps it, any code edit changes it."""
    import hashlib
    import re
    h = hashlib.sha256()
    for text in texts:
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        code = "\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip())
        h.update(code.encode())
        h.update(b"\0")
    return h.hexdigest()[:16]


def kernel_source_digest():
    """Digest of the kernel code; counter figures taken from other kernel
    code are not reported."""
    texts = []
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2209_13711_amd", "csrc", f), encoding="utf-8") as fh:
            texts.append(fh.read())
    return code_digest(texts)


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None
    when the summary is absent or was taken from other kernel source."""
    path = os.path.join(TRAFFIC_DIR, "chain_pu200_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    key = f"hbm_bytes_per_launch[{kernel}]"
    if kv.get("source_digest") != kernel_source_digest() or key not in kv:
        return None
    return float(kv[key])


def step_done(name, t0):
    """one line on stderr per finished leg (the JSON line stays alone on stdout)"""
    print(f"bench: {name} done ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)


def assert_clean(ctx, n_events=None):
    """After a timed leg: every event's counts come back without an error
    (a time-out of a kernel-side wait raises LST_E_FAULT from the getter) and
    with no error flag raised, so no figure is taken from broken outputs."""
    for e in range(ctx.n_events if n_events is None else n_events):
        c = ctx.counts(e)
        assert c["error_flags"] == 0 and c["overflow_mask"] == 0, (e, c)


def copy_bandwidth(lst, torch, reps=10):
    """Achievable HBM bandwidth of the library's STREAM-like copy (read+write)."""
    src = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    lst.lst_stream_copy(dst, src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        lst.lst_stream_copy(dst, src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * COPY_BYTES / (ms * 1e-3) / 1e9


def algorithmic_bytes(c, n_slots, n_edges_used):
    """Minimal bytes per launch of each object kernel (every input read
    once, every output written once), from the per-unit figures of the
    method's measurement plan:
    md:  12 B per hit + 48 B per module slot + 40 B per MD written
    seg: 28 B per MD read + 12 B per map edge of a module holding an MD +
         8 B per segment written
    t3:  8 B per segment + 16 B per triplet written
    t5:  16 B per triplet + 12 B per quintuplet written"""
    H, S = c["n_hits"], n_slots
    md, seg, t3, t5 = c["n_md"], c["n_seg"], c["n_t3"], c["n_t5"]
    return {
        "md": 12 * H + 48 * S + 40 * md,
        "seg": 28 * md + 12 * n_edges_used + 8 * seg,
        "t3": 8 * seg + 16 * t3,
        "t5": 16 * t3 + 12 * t5,
    }


def layout_bytes(c, n_slots, n_edges_used):
    """The same in the library's own layouts (wider records than the
    minimal figures above; reported beside them):
    md:  sorted hit (16 B) read and its duplicate-removal state (12 B) set per
         hit; per slot two bin offsets (8 B), the module frame (52 B) and the
         slot's MD start and count (8 B); per MD its record written (85 B:
         hit pair and slot 12, three float4 48, map row 16, bend 4, S3 bound
         4, flags 1)
    seg: per MD its record read (69 B: window and cut terms, map row) and
         its segment start and count written (8 B); per slot MD start and
         count (8 B); per map edge read its column (4 B); per segment its MD
         pair written (8 B)
    t3:  per MD its record (49 B) and segment start/count (8 B) read, triplet
         start/count written (8 B); per segment its outer MD (4 B); per
         triplet its MDs and curvature (16 B) and scorer flag (1 B) written
    t5:  per MD its record (49 B) and triplet start/count (8 B); per triplet
         its MDs, curvature and flag (17 B); per quintuplet its five MDs,
         score and flag (25 B) written"""
    H, S = c["n_hits"], n_slots
    md, seg, t3, t5 = c["n_md"], c["n_seg"], c["n_t3"], c["n_t5"]
    return {
        "md": 28 * H + 68 * S + 85 * md,
        "seg": 77 * md + 8 * S + 4 * n_edges_used + 8 * seg,
        "t3": 65 * md + 4 * seg + 17 * t3,
        "t5": 57 * md + 17 * t3 + 25 * t5,
    }


def cpu_baseline(params, geo, budget_s=18.0, max_events=200):
    """The oracle chain on PU200-like events, one thread: as it runs in the
    parity tests (FP32 decisions plus the FP64 instance that records
    near-threshold candidates), and on the same events with the FP64
    instance switched off (FP32 decisions alone, same objects)."""
    import oracle
    from synth import events as E
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    fp32 = oracle.Oracle(params, geo.f32, geo.i32)
    fp32.set_margins(False)
    t_total, t_fp32, n = 0.0, 0.0, 0
    while t_total + t_fp32 < budget_s and n < max_events:
        ev = E.generate(2, 1000 + n)
        t0 = time.perf_counter()
        orc.run_event(ev)
        t1 = time.perf_counter()
        fp32.run_event(ev)
        t_total += t1 - t0
        t_fp32 += time.perf_counter() - t1
        n += 1
    return {"value": n / t_total, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} PU200-like events (config 2, seeds 1000..{999 + n}), oracle chain "
                      f"incl. hit grouping and FP64 margins, single thread, {t_total:.1f} s",
            "fp32_decisions_only": {"value": n / t_fp32, "unit": "events/s",
                                    "sample": f"same {n} events, FP64 instance off, {t_fp32:.1f} s"}}


def batched(lst, torch, E, G, PR, evs, steps=20, cache=None, compare=True):
    """64 events of uneven pileup (20 x Poisson(U(50, 250)) helices each, barrel
    toy geometry) in one launch: autotuned launch shape, then the batch timed
    as one hipGraph replay (per-stage kernels or the persistent kernel, as
    the tuner chose), the persistent kernel alone, and the same events one at
    a time through the single-event graph (compare=False: the batch alone,
    for profiles)."""
    geo = G.get("barrel_toy")
    params = PR.make()
    n_events = len(evs)
    b = E.concat(evs)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    tuned = ctx.tune(cache_path=cache, reps=3)
    stream = torch.cuda.current_stream()

    def timeit(fn, n):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    ctx.load_hits(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    t_graph = timeit(lambda: ctx.run_chain_graph(stream), steps)
    assert_clean(ctx)
    kept = sum(ctx.counts(e)["n_t5_kept"] for e in range(n_events))
    t_pers = t_single = float("nan")
    if compare:
        t_pers = timeit(lambda: ctx.run_chain_persistent(stream), steps)
        assert_clean(ctx)
        kept_p = sum(ctx.counts(e)["n_t5_kept"] for e in range(n_events))
        assert kept == kept_p, "persistent chain changed the result"
        # one event per launch, same events
        single = lst.Context(params, geo.f32, geo.i32, device=0)
        single.reserve(dict(ctx.caps, events=1))
        per_event = []
        for ev in evs[:8]:
            single.load_hits(np.array([0, ev.n_hits], np.int32), ev.x, ev.y, ev.z, ev.module,
                             ev.sensor)
            per_event.append(timeit(lambda: single.run_chain_graph(stream), 5))
            assert_clean(single)
        t_single = float(np.mean(per_event))
    # roofline of the segment stage on the batch: algorithmic bytes over the
    # tuner's per-stage median (HIP events around the stage on the stream)
    ptr, _ = ctx.module_map()
    tot = {k: 0 for k in ("n_hits", "n_md", "n_seg", "n_t3", "n_t5")}
    edges = 0
    for e, ev in enumerate(evs):
        c = ctx.counts(e)
        for k in tot:
            tot[k] += c[k]
        mods = np.unique(ev.module[ctx.objects(e, lst.LST_MD)[:, 0]])
        edges += int(np.sum(ptr[mods + 1] - ptr[mods]))
    seg_bytes = algorithmic_bytes(tot, n_events * geo.n_mod, edges)["seg"]
    # the segment stage alone: HIP events around it on the launch stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    seg_ms = []
    for _ in range(6):
        ctx.load_hits(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
        ctx.run_sort(stream)
        ctx.run_md(stream)
        e0.record(stream)
        ctx.run_segments(stream)
        e1.record(stream)
        for fn in (ctx.run_triplets, ctx.run_quintuplets, ctx.run_dedup):
            fn(stream)
        torch.cuda.synchronize()
        seg_ms.append(e0.elapsed_time(e1))
    seg_us = 1e3 * float(np.median(seg_ms[1:]))
    return {"workload": "64 uneven events (config 3): 20 x Poisson(U(50,250)) helices, "
                        "barrel toy geometry, plain chain",
            "hits": int(b.offsets[-1]), "events": n_events,
            "events_per_s": n_events / t_graph,
            "ms_per_batch": 1e3 * t_graph,
            "persistent_events_per_s": n_events / t_pers,
            "one_event_per_launch_events_per_s": 1.0 / t_single,
            "tuning": {k: tuned[k] for k in ("grid", "lanes", "persistent", "blocks_per_cu")},
            "tuner_report_us": tuned["report_us"], "t5_kept": int(kept),
            "roofline_seg": {"bound": "hbm", "achieved": seg_bytes / (seg_us * 1e-6) / 1e9,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": seg_bytes / (seg_us * 1e-6) / 1e9 / HBM_PEAK_GBS,
                             "algorithmic_bytes": int(seg_bytes), "duration_us": seg_us}}


def _gen_train(e):
    from synth import events as E
    return E.generate(4, e, purpose=E.PURPOSE_TRAIN, cfg=E.scorer_training_config(E.CONFIGS[4]))


def _gen_eval(e):
    from synth import events as E
    return E.generate(4, e)


def _gen_train_full(e):
    from synth import events as E
    return E.generate(2, e, purpose=E.PURPOSE_TRAIN, cfg=E.scorer_training_config(E.CONFIGS[2]))


def _gen_train_stress(e):
    from synth import events as E
    return E.generate(5, e, purpose=E.PURPOSE_TRAIN, cfg=E.scorer_training_config(E.CONFIGS[5]))


def _gen(args):
    from synth import events as E
    cid, e = args
    return E.generate(cid, e)


def pregenerate(scorer=True, batch=True, stress=True, pu200=True, n_train=150, n_eval=16,
                n_train_full=80, n_train_stress=100):
    """every synthetic event the side legs need, generated by a pool of CPU
    workers before this process touches the GPU"""
    import multiprocessing as mp
    out = {}
    with mp.get_context("fork").Pool(min(16, os.cpu_count() or 1)) as pool:
        if scorer:
            out["train"] = pool.map(_gen_train, range(n_train))
            out["eval"] = pool.map(_gen_eval, range(n_eval))
            out["train_full"] = pool.map(_gen_train_full, range(n_train_full))
            out["eval_full"] = pool.map(_gen, [(2, 200 + e) for e in range(n_eval)])
        if batch:
            out["batch"] = pool.map(_gen, [(3, e) for e in range(64)])
        if stress:
            out["stress"] = pool.map(_gen, [(5, e) for e in range(16)])
            if scorer:
                out["train_stress"] = pool.map(_gen_train_stress, range(n_train_stress))
        if pu200:
            out["pu200"] = pool.map(_gen, [(2, 100 + e) for e in range(16)])
    return out


def _oracle_worker(args):
    """one CPU process: the oracle on PU200-like events for `budget` seconds"""
    first, budget = args
    import oracle
    from synth import events as E, geometry as G, params as PR
    geo = G.get("full")
    orc = oracle.Oracle(PR.make(), geo.f32, geo.i32)
    n, t = 0, 0.0
    while t < budget:
        ev = E.generate(2, first + n)
        t0 = time.perf_counter()
        orc.run_event(ev)
        t += time.perf_counter() - t0
        n += 1
    return n, t


def cpu_all_cores(budget_s=8.0):
    """the oracle on every host core at once (one process per core, distinct
    events), before this process touches the GPU"""
    import multiprocessing as mp
    n_proc = min(16, os.cpu_count() or 1)
    with mp.get_context("fork").Pool(n_proc) as pool:
        res = pool.map(_oracle_worker, [(5000 + 1000 * k, budget_s) for k in range(n_proc)])
    return {"value": float(sum(n / t for n, t in res)), "unit": "events/s", "cores": n_proc,
            "kind": "oracle", "sample": f"{sum(n for n, _ in res)} PU200-like events (config 2), "
                                        f"one oracle process per core, {budget_s:.0f} s each"}


def scored(lst, torch, train, evs, steps=50, base_cfg=4):
    """Learned scorers end to end on the GPU: triplets of the training events
    (widened windows), then the quintuplets that survive the trained triplet
    veto, labelled by truth and trained by the library's kernels; thresholds
    keep 99.5 % (triplets) and 99 % (quintuplets) of the true candidates.
    Then the plain chain at nominal windows against the widened chain +
    scorers on held-out 4000-helix events (efficiency / fake rate by truth,
    events/s of one event per hipGraph replay), and the two scoring kernels
    timed with HIP events on the launch stream.  base_cfg 4: barrel toy
    geometry; 2: the full geometry (barrel and endcap disks, noise hits)."""
    from paper_2209_13711_amd import scorer as S
    from synth import events as E, geometry as G, params as PR, weights as W
    geo = G.get(E.CONFIGS[base_cfg].geometry)
    w_train = E.scorer_training_config(E.CONFIGS[base_cfg]).window
    ctx_w = lst.Context(PR.make(w=w_train), geo.f32, geo.i32, device=0)
    models, info = {}, {}
    for kind, name, keep in ((lst.LST_T3, "t3", 0.995), (lst.LST_T5, "t5", 0.99)):
        t0 = time.perf_counter()
        F, y = S.collect(ctx_w, train, kind=kind)
        t_collect = time.perf_counter() - t0
        cfg = S.TrainConfig(epochs=10)
        tr = S.Trainer(ctx_w, F, y, W.random_params(np.random.default_rng(kind)), cfg)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = tr.fit()
        t_train = time.perf_counter() - t0
        lg, lab = tr.logits_all(), tr.labels()
        th = S.threshold_for(lg, lab, keep)
        models[kind] = (tr.params(), tr.mean, tr.istd, th)
        info[name] = {"train_candidates": int(len(y)), "train_true_frac": float(y.mean()),
                      "collect_s": t_collect, "train_s": t_train, "epochs": cfg.epochs,
                      "train_candidates_per_s": tr.n_batches * tr.b * cfg.epochs / t_train,
                      "loss_first_last": [losses[0], losses[-1]], "threshold": th,
                      "true_kept": float(np.mean(lg[lab == 1] >= th)),
                      "false_vetoed": float(np.mean(lg[lab == 0] < th))}
        # the next kind learns on what survives this veto
        ctx_w.mlp_load(*models[kind], kind=kind)
        ctx_w.set_mode(lst.LST_MODE_MLP)
    # three arms on the same held-out events, each as one batched launch:
    # the plain chain at nominal windows, the plain chain at the widened
    # training windows (what widening alone does), and the widened chain with
    # both learned vetoes (what the networks add on top of the widening)
    plain_ctx = lst.Context(PR.make(), geo.f32, geo.i32, device=0)
    wide_ctx = lst.Context(PR.make(w=w_train), geo.f32, geo.i32, device=0)
    scored_ctx = lst.Context(PR.make(w=w_train), geo.f32, geo.i32, device=0)
    for kind, m in models.items():
        scored_ctx.mlp_load(*m, kind=kind)
    scored_ctx.set_mode(lst.LST_MODE_MLP)
    m_plain = S.evaluate(plain_ctx, evs, geo)
    m_wide = S.evaluate(wide_ctx, evs, geo)
    m_scored = S.evaluate(scored_ctx, evs, geo)
    for c in (plain_ctx, wide_ctx, scored_ctx):
        assert_clean(c)
    stream = torch.cuda.current_stream()

    def rate(ctx):
        per = []
        for ev in evs[:8]:
            ctx.load_hits(np.array([0, ev.n_hits], np.int32), ev.x, ev.y, ev.z, ev.module, ev.sensor)
            for _ in range(3):
                ctx.run_chain_graph(stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                ctx.run_chain_graph(stream)
            torch.cuda.synchronize()
            per.append((time.perf_counter() - t0) / steps)
            assert_clean(ctx)
        return 1.0 / float(np.mean(per))

    # scoring kernels alone: HIP events around each scoring step on the launch stream
    ev = evs[0]
    c = scored_ctx
    c.load_hits(np.array([0, ev.n_hits], np.int32), ev.x, ev.y, ev.z, ev.module, ev.sensor)
    ev3 = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ms3, ms5 = [], []
    for _ in range(20):
        for fn in (c.run_sort, c.run_md, c.run_segments, c.run_triplets):
            fn(stream)
        ev3[0].record(stream)
        c.run_t3_score(stream)
        ev3[1].record(stream)
        c.run_quintuplets(stream)
        ev3[2].record(stream)
        c.run_t5_score(stream)
        ev3[3].record(stream)
        c.run_dedup(stream)
        torch.cuda.synchronize()
        ms3.append(ev3[0].elapsed_time(ev3[1]))
        ms5.append(ev3[2].elapsed_time(ev3[3]))
    cnt = c.counts(0)

    def kern(name, ms, n):
        us = 1e3 * float(np.median(ms[5:]))
        return {"kernel": name, "duration_us": us, "objects": int(n), "bound": "mfma",
                "achieved_TFLOPs": n * MLP_FLOPS / (us * 1e-6) / 1e12, "peak_TFLOPs": 2500.0}

    model = models
    where = {4: "barrel toy", 2: "full geometry, 1 % inefficiency, 5 % noise hits",
             5: "barrel toy, 5 % displaced, 10 % noise hits"}[base_cfg]
    keys = ("eff", "fake", "dup", "impure", "n_obj")
    return {"workload": f"scorers trained on triplets and quintuplets of {len(train)} training "
                        f"events ({where}, 20 x Poisson(U(50,250)) helices, windows x1.5), "
                        f"evaluated on {len(evs)} held-out events (config {base_cfg}) in one "
                        f"batched launch per arm",
            "training": info,
            "plain_w1": {k: m_plain[k] for k in keys},
            "plain_w1.5": {k: m_wide[k] for k in keys},
            "scored_w1.5": {k: m_scored[k] for k in keys},
            "network_gain_vs_plain_w1.5": {
                "eff_points": 100 * (m_scored["eff"] - m_wide["eff"]),
                "fake_ratio": m_scored["fake"] / m_wide["fake"] if m_wide["fake"] else None,
                "impure_points": 100 * (m_scored["impure"] - m_wide["impure"])},
            "plain_events_per_s": rate(plain_ctx),
            # the widened windows alone, so that scored / this is the cost of scoring
            "plain_w1.5_events_per_s": rate(wide_ctx),
            "scored_events_per_s": rate(scored_ctx),
            "score_kernels": [kern("k_mlp_score<T3>", ms3, cnt["n_t3"]),
                              kern("k_mlp_score<T5>", ms5, cnt["n_t5"])]}, model


def multistream(lst, torch, G, PR, evs, n_streams=8, rounds=3, geometry="barrel_toy"):
    """The paper's concurrency scheme on this GPU: the same events one per
    launch, spread over n_streams HIP streams (default priority), each with
    its own context and hipGraph; hits already in device memory."""
    geo = G.get(geometry)
    params = PR.make()
    dev = []
    for ev in evs:
        t = [torch.from_numpy(np.ascontiguousarray(a)).cuda()
             for a in (ev.x, ev.y, ev.z, ev.module.astype(np.int32), ev.sensor.astype(np.uint8))]
        dev.append((np.array([0, ev.n_hits], np.int32), t))
    big = max(evs, key=lambda e: e.n_hits)
    streams = [torch.cuda.Stream() for _ in range(n_streams)]
    ctxs = []
    for k in range(n_streams):
        c = lst.Context(params, geo.f32, geo.i32, device=0)
        c.run_batch(np.array([0, big.n_hits], np.int32), big.x, big.y, big.z, big.module,
                    big.sensor)
        ctxs.append(c)

    def run_all():
        for i, (offs, t) in enumerate(dev):
            k = i % n_streams
            ctxs[k].load_hits(offs, *t, stream=streams[k])
            ctxs[k].run_chain_graph(streams[k])

    run_all()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(rounds):
        run_all()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for c in ctxs:
        assert_clean(c)
    return {"streams": n_streams, "events": len(evs), "events_per_s": rounds * len(evs) / dt}


def pu200_concurrent(lst, torch, E, G, PR, evs, steps=20):
    """Several PU200-like events in flight at once: 16 events (config 2,
    seeds 100..115) as one batched launch (tuned launch shape, one hipGraph
    replay per batch), and the same events one per launch over 8 streams."""
    geo = G.get("full")
    params = PR.make()
    b = E.concat(evs)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    tuned = ctx.tune(reps=3)
    ctx.load_hits(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
    stream = torch.cuda.current_stream()
    ctx.run_chain_graph(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.run_chain_graph(stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    assert_clean(ctx)
    kept = int(sum(ctx.counts(e)["n_t5_kept"] for e in range(len(evs))))
    del ctx
    return {"workload": f"{len(evs)} PU200-like events (config 2, seeds 100..{99 + len(evs)})",
            "hits": int(b.offsets[-1]), "t5_kept": kept,
            "batched_events_per_s": len(evs) / dt, "ms_per_batch": 1e3 * dt,
            "tuning": {k: tuned[k] for k in ("grid", "lanes", "persistent", "blocks_per_cu")},
            "multistream_8": multistream(lst, torch, G, PR, evs, geometry="full")}


def memory(lst, torch, G, PR, evs, quantiles=(0.999, 0.9999)):
    """Memory of this library's arena against the paper's layout of fixed
    per-module capacities truncated at an occupancy quantile, on PU200-like
    events.  Per object type (keyed by the module of its first hit): the
    per-module capacity at each quantile and at the maximum of the per-module
    counts over all modules of all events, the arena bytes those capacities
    imply, and the share of objects that modules above capacity would drop.
    The library itself sizes its object arrays by the event's counts and
    drops nothing; with the same capacities set in the chain
    (lst_set_capacities) each stage drops what a full module cannot hold, and
    the leg reports the resulting efficiency and fake rate (one batched
    launch of the 16 events) against the uncapped chain."""
    geo = G.get("full")
    ctx = lst.Context(PR.make(), geo.f32, geo.i32, device=0)
    kinds = {"md": lst.LST_MD, "seg": lst.LST_SEG, "t3": lst.LST_T3, "t5": lst.LST_T5}
    per_mod = {k: [] for k in kinds}
    exact = dict(events=1, hits=1, md=1, seg=1, t3=1, t5=1)
    for ev in evs:
        ctx.run_event(ev)
        exact["hits"] = max(exact["hits"], int(ev.n_hits))
        for k, kind in kinds.items():
            t = ctx.objects(0, kind)
            exact[k] = max(exact[k], len(t))
            mods = ev.module[t[:, 0]] if len(t) else np.zeros(0, np.int64)
            per_mod[k].append(np.bincount(mods, minlength=geo.n_mod))
    counts = {k: np.concatenate(v) for k, v in per_mod.items()}
    out = {"events": len(evs), "modules": int(geo.n_mod),
           "exact_arena_MB": ctx.arena_bytes(exact) / 1e6,
           "grown_arena_MB": ctx.arena_bytes(ctx.caps) / 1e6,
           "exact_caps": {k: int(exact[k]) for k in kinds}}
    from paper_2209_13711_amd import scorer as S
    keys = ("eff", "fake", "dup", "n_obj")
    m_exact = S.evaluate(ctx, evs, geo)
    out["chain_exact"] = {k: m_exact[k] for k in keys}
    stream = torch.cuda.current_stream()
    for name, q in [(f"q{100 * q:g}", q) for q in quantiles] + [("max", None)]:
        cap = {k: int(np.ceil(np.quantile(c, q))) if q is not None else int(c.max())
               for k, c in counts.items()}
        caps = dict(exact, **{k: max(1, cap[k] * geo.n_mod) for k in kinds})
        # the capacities applied in the chain (lst_set_capacities): what each
        # stage removes, and the efficiency / fake rate of what is left
        cctx = lst.Context(PR.make(), geo.f32, geo.i32, device=0)
        cctx.set_capacities([max(1, cap[k]) for k in kinds])
        m = S.evaluate(cctx, evs, geo)
        dropped = np.sum([cctx.counts(e)["dropped"] for e in range(len(evs))], axis=0)
        assert_clean(cctx)
        cctx.run_chain_graph(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(10):
            cctx.run_chain_graph(stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 10
        del cctx
        out[f"per_module_{name}"] = {
            "cap_per_module": cap,
            "arena_MB": ctx.arena_bytes(caps) / 1e6,
            "dropped_frac": {k: float(np.maximum(counts[k] - cap[k], 0).sum() /
                                      max(counts[k].sum(), 1)) for k in kinds},
            "chain_capped": dict({k: m[k] for k in keys},
                                 dropped={k: int(d) for k, d in zip(kinds, dropped)},
                                 eff_loss_points=100 * (m_exact["eff"] - m["eff"]),
                                 events_per_s=len(evs) / dt)}
    del ctx
    return out


def half_storage(lst, torch, E, G, PR, evs, steps=100):
    """Half-precision hit storage (lst_set_hit_storage): the PU200-like event
    (config 2, seed 0) and the 16-event PU200-like batch, each through the
    tuned chain as one hipGraph per step, with FP32 and with FP16 module-local
    hit storage; kept-quintuplet efficiency / fake rate by truth on the 16
    events in both modes."""
    from synth import truth as T
    geo = G.get("full")
    stream = torch.cuda.current_stream()
    out = {}
    for name, evl in (("pu200_event", [E.generate(2, 0)]), ("pu200_batch16", evs)):
        b = E.concat(evl)
        row = {}
        for mode in (0, 1):
            ctx = lst.Context(PR.make(), geo.f32, geo.i32, device=0)
            ctx.set_hit_storage(bool(mode))
            ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
            ctx.tune(reps=3)
            ctx.load_hits(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
            for _ in range(10):          # capture, then warm replays
                ctx.run_chain_graph(stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                ctx.run_chain_graph(stream)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            assert_clean(ctx)
            tot = dict(n_obj=0, n_findable=0, n_found=0, n_fake=0)
            for e, ev in enumerate(evl):
                m = T.metrics(ctx.objects(e, lst.LST_T5_KEPT), ev, geo)
                for k in tot:
                    tot[k] += m[k]
            row["fp16" if mode else "fp32"] = {
                "events_per_s": len(evl) / dt, "ms_per_step": 1e3 * dt,
                "eff": tot["n_found"] / max(tot["n_findable"], 1),
                "fake": tot["n_fake"] / max(tot["n_obj"], 1), "n_obj": tot["n_obj"],
                "hit_record_bytes": 8 if mode else 16}
            del ctx
        out[name] = row
    return out


def pixel_leg(lst, torch, E, G, PR, evs, steps=50):
    """Pixel objects and track candidates (pLS linked to quintuplets and
    triplets, cross-cleaning): one PU200-like event (config 2, seed 0) and the
    16-event PU200-like batch, chain replayed as one hipGraph then the pixel
    stage, hits and seeds resident on the device; the pixel stage alone timed
    with HIP events on the launch stream; track-candidate efficiency, fake
    and duplicate rate by truth beside the kept quintuplets'."""
    from synth import truth as T
    geo = G.get("full")
    params, pp = PR.make(), PR.make_pixel()
    stream = torch.cuda.current_stream()
    out = {}
    for name, batch in (("pu200_event", [(E.generate(2, 0), 0)]),
                        ("pu200_batch16", [(ev, 100 + e) for e, ev in enumerate(evs)])):
        evl = [ev for ev, _ in batch]
        pxs = [E.pixel_seeds(ev, 2, seed) for ev, seed in batch]
        b = E.concat(evl)
        poff = np.r_[0, np.cumsum([p.n_hits for p in pxs])].astype(np.int32)
        soff = np.r_[0, np.cumsum([p.n_seeds for p in pxs])].astype(np.int32)
        cat = lambda a: np.concatenate([getattr(p, a) for p in pxs])
        ctx = lst.Context(params, geo.f32, geo.i32, device=0)
        ctx.reserve(lst.default_caps(len(evl), int(b.offsets[-1])))
        ctx.pixel_caps(int(poff[-1]), int(soff[-1]))
        ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
        tuned = ctx.tune(reps=3)
        ctx.load_hits(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
        ctx.run_chain_graph(stream)
        ctx.load_pixel(poff, cat("x"), cat("y"), cat("z"), soff,
                       np.concatenate([p.seeds for p in pxs]), pp)
        ctx.run_pixel(stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        px_ms = []
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.run_chain_graph(stream)
            e0.record(stream)
            ctx.run_pixel(stream)
            e1.record(stream)
            e1.synchronize()
            px_ms.append(e0.elapsed_time(e1))
        dt_sync = (time.perf_counter() - t0) / steps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.run_chain_graph(stream)
            ctx.run_pixel(stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        assert_clean(ctx)
        tot = dict(n_obj=0, n_findable=0, n_found=0, n_fake=0, n_dup=0)
        t5 = dict(tot)
        types = [0, 0, 0, 0]
        for e, (ev, px) in enumerate(zip(evl, pxs)):
            m = T.tc_metrics(ctx.track_candidates(e), ev, px, geo)
            for k in tot:
                tot[k] += m[k]
            for t in range(4):
                types[t] += m["by_type"][t]
            m5 = T.metrics(ctx.objects(e, lst.LST_T5_KEPT), ev, geo)
            for k in t5:
                t5[k] += m5[k]
        rate = lambda d: {"eff": d["n_found"] / max(d["n_findable"], 1),
                          "fake": d["n_fake"] / max(d["n_obj"], 1),
                          "dup": d["n_dup"] / max(d["n_obj"], 1), "n_obj": d["n_obj"]}
        out[name] = {"events": len(evl), "seeds": int(soff[-1]),
                     "events_per_s_chain_plus_pixel": len(evl) / dt,
                     "pixel_stage_us": 1e3 * float(np.median(px_ms)),
                     "ms_per_step": 1e3 * dt,
                     "track_candidates": dict(rate(tot), by_type=dict(zip(("pT5", "pT3", "T5", "pLS"), types))),
                     "kept_quintuplets": rate(t5),
                     "tuning": {k: tuned[k] for k in ("grid", "lanes", "persistent", "blocks_per_cu")}}
        del ctx
    return out


def stress(lst, torch, E, G, PR, evs, model=None, model_transfer=None, steps=10):
    """16 PU300-like events (6000 helices, 5 % displaced, 10 % noise, windows
    x1.5) in one tuned launch: events/s and efficiency / fake / duplicate rate
    by truth, plain and (when trained scorers are given) scored: `model`
    trained on events of the stress recipe (displaced tracks and noise hits
    included), `model_transfer` trained on prompt, noise-free barrel events."""
    from paper_2209_13711_amd import scorer as S
    from synth import truth as T
    geo = G.get("barrel_toy")
    params = PR.make(w=E.CONFIGS[5].window)
    b = E.concat(evs)
    stream = torch.cuda.current_stream()

    def run(ctx):
        ctx.run_batch(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
        tuned = ctx.tune(reps=3)
        ctx.load_hits(b.offsets, b.x, b.y, b.z, b.module, b.sensor)
        ctx.run_chain_graph(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            ctx.run_chain_graph(stream)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        assert_clean(ctx)
        tot = dict(n_obj=0, n_findable=0, n_found=0, n_fake=0, n_dup=0, n_pure=0)
        for e, ev in enumerate(evs):
            kept = ctx.objects(e, lst.LST_T5_KEPT)
            m = T.metrics(kept, ev, geo)
            for k in ("n_obj", "n_findable", "n_found", "n_fake", "n_dup"):
                tot[k] += m[k]
            tot["n_pure"] += int(S.pure_labels(kept, ev.truth).sum())
        n = max(tot["n_obj"], 1)
        return {"events_per_s": len(evs) / dt, "ms_per_batch": 1e3 * dt,
                "eff": tot["n_found"] / max(tot["n_findable"], 1), "fake": tot["n_fake"] / n,
                "dup": tot["n_dup"] / n, "impure": 1.0 - tot["n_pure"] / n, "n_obj": tot["n_obj"],
                "tuning": {k: tuned[k] for k in ("grid", "lanes", "persistent", "blocks_per_cu")}}

    out = {"workload": "16 PU300-like events (config 5): 6000 helices, 5 % displaced "
                       "(d0 up to 10 cm), 10 % noise, windows x1.5, barrel toy geometry, one batch",
           "hits": int(b.offsets[-1]),
           "plain": run(lst.Context(params, geo.f32, geo.i32, device=0))}
    for name, mdl in (("scored", model), ("scored_prompt_model", model_transfer)):
        if mdl is None:
            continue
        ctx = lst.Context(params, geo.f32, geo.i32, device=0)
        for kind, m in mdl.items():
            ctx.mlp_load(*m, kind=kind)
        ctx.set_mode(lst.LST_MODE_MLP)
        out[name] = run(ctx)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-event batch figures")
    ap.add_argument("--no-scorer", action="store_true", help="skip the learned-scorer figures")
    ap.add_argument("--no-stress", action="store_true", help="skip the config-5 stress figures")
    ap.add_argument("--no-concurrent", action="store_true",
                    help="skip the figures with several PU200-like events in flight")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the 64-event batch leg and print its figures (for profiling)")
    ap.add_argument("--pixel-only", action="store_true",
                    help="run only the pixel-object leg and the half-precision storage leg "
                         "and print their figures (for profiling)")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache (JSON lines): reuse a stored launch shape for this event")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (--gpus {args.gpus} requested); events are "
              "independent, so a batch would shard across GPUs by event with no exchange", file=sys.stderr)
        sys.exit(2)

    if args.batch_only:
        pre = pregenerate(scorer=False, batch=True, stress=False, pu200=False)
        import torch
        import paper_2209_13711_amd as lst
        from synth import events as E, geometry as G, params as PR
        print(json.dumps({"batched": batched(lst, torch, E, G, PR, pre["batch"],
                                             cache=args.tune_cache, compare=False)}), flush=True)
        return
    if args.pixel_only:
        pre = pregenerate(scorer=False, batch=False, stress=False, pu200=True)
        import torch
        import paper_2209_13711_amd as lst
        from synth import events as E, geometry as G, params as PR
        print(json.dumps({"pixel": pixel_leg(lst, torch, E, G, PR, pre["pu200"], steps=20),
                          "half_storage": half_storage(lst, torch, E, G, PR, pre["pu200"],
                                                       steps=20)}), flush=True)
        return
    pre = pregenerate(scorer=not args.no_scorer, batch=not args.no_batch,
                      stress=not args.no_stress, pu200=not args.no_concurrent)
    cpu_all = None if args.no_cpu else cpu_all_cores()

    import torch
    import paper_2209_13711_amd as lst
    from synth import events as E, geometry as G, params as PR

    geo = G.get("full")
    params = PR.make()
    ev = E.generate(2, 0)
    ctx = lst.Context(params, geo.f32, geo.i32, device=0)
    stream = torch.cuda.current_stream()
    offs = np.array([0, ev.n_hits], np.int32)
    ctx.run_batch(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor)   # sizes the arena
    # launch shape for this event size (grid, lanes, persistent), tuned or cached
    tuned = ctx.tune(cache_path=args.tune_cache, reps=5)
    cnt = ctx.counts(0)
    ptr, col = ctx.module_map()
    # map edges actually read: those of modules holding at least one MD
    md_mods = np.unique(ev.module[ctx.objects(0, lst.LST_MD)[:, 0]])
    n_edges_used = int(np.sum(ptr[md_mods + 1] - ptr[md_mods]))
    n_slots = geo.n_mod

    stages = [("sort", ctx.run_sort), ("md", ctx.run_md), ("seg", ctx.run_segments),
              ("t3", ctx.run_triplets), ("t5", ctx.run_quintuplets), ("dedup", ctx.run_dedup)]

    def step(events=None):
        for i, (name, fn) in enumerate(stages):
            if events is not None:
                events[i].record(stream)
            fn(stream)
        if events is not None:
            events[-1].record(stream)

    # instrumented timed region: eager stage calls with HIP events between
    # them on the launch stream -> per-kernel durations for the roofline
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(stages) + 1)]
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    dt_eager = time.perf_counter() - t0

    # headline timed region: the same chain replayed as one hipGraph per step
    for _ in range(args.warmup):
        ctx.run_chain_graph(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ctx.run_chain_graph(stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    # the same chain with the hits handed over from host memory each step
    # (pageable numpy arrays through lst_load_hits): PCIe-inclusive rate
    n_pcie = max(args.steps // 4, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_pcie):
        ctx.load_hits(offs, ev.x, ev.y, ev.z, ev.module, ev.sensor, stream)
        ctx.run_chain_graph(stream)
    torch.cuda.synchronize()
    pcie_rate = n_pcie / (time.perf_counter() - t0)

    stage_ms = {name: float(np.mean([evs[k][i].elapsed_time(evs[k][i + 1])
                                     for k in range(args.steps)]))
                for i, (name, _) in enumerate(stages)}
    assert_clean(ctx)
    c2 = ctx.counts(0)   # after the graph replays
    assert c2["n_t5_kept"] == cnt["n_t5_kept"], "result changed between runs"

    copy_gbs = copy_bandwidth(lst, torch)
    abytes = algorithmic_bytes(cnt, n_slots, n_edges_used)
    dom = max(abytes, key=lambda k: stage_ms[k])
    achieved = abytes[dom] / (stage_ms[dom] * 1e-3) / 1e9
    lanes_of = {"md": 1, "seg": 2, "t3": 3, "t5": 4}
    dom_kernel = f"k_{dom}<{tuned['lanes'][lanes_of[dom]]}>"
    cands = cnt["cand_md"] + cnt["cand_seg"] + cnt["cand_t3"] + cnt["cand_t5"]
    value = args.steps / dt
    out = {
        "metric": "PU200 events/s on 1 MI355X (MD->T5 chain)",
        "value": value,
        "unit": "events/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "PU200-like event (config 2): ~4000 helices, pT^-3 above 0.6 GeV, "
                               "|eta|<2.4, full geometry 6 barrel layers + 2x5 disks, 1% "
                               "inefficiency, 5% noise; plain MD->segment->T3->T5 chain + dedup",
                   "events_per_step": 1, "hits": int(ev.n_hits),
                   "tuning": {k: tuned[k] for k in ("grid", "lanes", "persistent", "blocks_per_cu")}},
        "candidates_per_s": cands * value,
        "stage_ms": stage_ms,
        "eager_events_per_s": args.steps / dt_eager,
        "pcie_inclusive_events_per_s": pcie_rate,
        "objects": {k: int(cnt[k]) for k in ("n_md", "n_seg", "n_t3", "n_t5", "n_t5_kept")},
        "roofline": {"bound": "hbm", "kernel": dom_kernel, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom_kernel),
                     "algorithmic_bytes": int(abytes[dom]),
                     "layout_bytes": int(layout_bytes(cnt, n_slots, n_edges_used)[dom]),
                     "duration_us": stage_ms[dom] * 1e3,
                     "copy_GBps_measured": copy_gbs,
                     "frac_vs_copy": achieved / copy_gbs},
    }
    t0 = time.perf_counter()
    step_done("headline", t0)
    if not args.no_concurrent:
        out["pu200_concurrent"] = pu200_concurrent(lst, torch, E, G, PR, pre["pu200"])
        step_done("pu200_concurrent", t0)
        out["memory"] = memory(lst, torch, G, PR, pre["pu200"])
        step_done("memory", t0)
        out["pixel"] = pixel_leg(lst, torch, E, G, PR, pre["pu200"])
        step_done("pixel", t0)
        out["half_storage"] = half_storage(lst, torch, E, G, PR, pre["pu200"])
        step_done("half_storage", t0)
    if not args.no_batch:
        out["batched"] = batched(lst, torch, E, G, PR, pre["batch"], cache=args.tune_cache)
        out["batched"]["multistream_8"] = multistream(lst, torch, G, PR, pre["batch"])
        step_done("batched", t0)
    model = model_stress = None
    if not args.no_scorer:
        out["scored"], model = scored(lst, torch, pre["train"], pre["eval"])
        step_done("scored", t0)
        out["scored_full_geometry"], _ = scored(lst, torch, pre["train_full"], pre["eval_full"],
                                                base_cfg=2)
        step_done("scored_full_geometry", t0)
        if not args.no_stress:
            out["scored_stress"], model_stress = scored(lst, torch, pre["train_stress"],
                                                        pre["stress"], base_cfg=5)
            step_done("scored_stress", t0)
    if not args.no_stress:
        out["stress"] = stress(lst, torch, E, G, PR, pre["stress"], model_stress, model)
        step_done("stress", t0)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(params, geo)
        out["cpu_baseline_all_cores"] = cpu_all
        step_done("cpu_baseline", t0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
