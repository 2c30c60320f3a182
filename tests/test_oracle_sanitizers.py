"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The oracle's C sources are built with gcc -fsanitize=address,undefined into a
small driver (oracle/sanitize_main.c) that runs whole events through the
chain, reads every output array and reruns the quintuplets under a triplet
veto.  Events: two barrel-toy events (config 1), a PU200-like event on the
full geometry (config 2), a stress event with displaced tracks, noise and
widened windows (config 5), an empty event and one with non-finite hit
coordinates.  Every run must end cleanly with no sanitizer report, and its
object counts must equal those of the oracle built normally."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from synth import events as E
from synth import geometry as G
from synth import params as PR

ORACLE_DIR = os.path.dirname(os.path.abspath(oracle.__file__))


def _write(path, params, geo, evs):
    with open(path, "wb") as f:
        np.array([len(params), geo.n_mod, len(evs)], np.int32).tofile(f)
        np.asarray(params, np.float64).tofile(f)
        np.ascontiguousarray(geo.f32, np.float32).tofile(f)
        np.ascontiguousarray(geo.i32, np.int32).tofile(f)
        for x, y, z, mod, sen in evs:
            np.array([len(x)], np.int32).tofile(f)
            for a, t in ((x, np.float32), (y, np.float32), (z, np.float32), (mod, np.int32),
                         (sen, np.uint8)):
                np.ascontiguousarray(a, t).tofile(f)


def _expected(params, geo, evs):
    orc = oracle.Oracle(params, geo.f32, geo.i32)
    out = []
    for x, y, z, mod, sen in evs:
        r = orc.run(x, y, z, mod, sen)
        n = [len(r.tuples[k]) for k in range(5)]
        veto = np.zeros(n[2], np.uint8)
        veto[::7] = 1
        r2 = orc.rerun_t5(veto)
        out.append(n + [len(r2.tuples[3]), len(r2.tuples[4])])
    return out


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("asan") / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-I", ORACLE_DIR, "-o", exe, os.path.join(ORACLE_DIR, "sanitize_main.c"),
           os.path.join(ORACLE_DIR, "lst_oracle.c"), "-lm"]
    subprocess.run(cmd, check=True)
    return exe


def _cases(cid):
    cfg = E.CONFIGS[cid]
    geo = G.get(cfg.geometry)
    params = PR.make(w=cfg.window)
    evs = []
    for e in ((0, 1) if cid == 1 else (0,)):
        ev = E.generate(cid, e)
        evs.append((ev.x, ev.y, ev.z, ev.module, ev.sensor))
    if cid == 1:
        evs.append(tuple(np.zeros(0, t) for t in (np.float32,) * 3 + (np.int32, np.uint8)))
        ev = E.generate(1, 2)
        x, y, z = ev.x.copy(), ev.y.copy(), ev.z.copy()
        x[::17] = np.nan
        y[5::23] = np.inf
        z[7::29] = -np.inf
        evs.append((x, y, z, ev.module, ev.sensor))
    return params, geo, evs


@pytest.mark.parametrize("cid", [1, 2, 5])
def test_oracle_is_clean_under_sanitizers(cid, driver, tmp_path):
    params, geo, evs = _cases(cid)
    inp = str(tmp_path / "events.bin")
    _write(inp, params, geo, evs)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=87")
    env.pop("LD_PRELOAD", None)
    p = subprocess.run([driver, inp], capture_output=True, text=True, env=env, timeout=900)
    assert p.returncode == 0, p.stderr[-4000:]
    assert "runtime error" not in p.stderr and "Sanitizer" not in p.stderr, p.stderr[-4000:]
    got = [list(map(int, line.split())) for line in p.stdout.strip().splitlines()]
    assert got == _expected(params, geo, evs)
