"""The learned selector: the C evaluation (mlu_select) against the Python one
on the same packed model (choice and fallback flag), its argument checks, the
candidate rules, and the training machinery on synthetic timings with a known
best configuration (CPU only)."""
import ctypes
import math

import numpy as np
import pytest

from paper_1611_06365_amd import mlu
from paper_1611_06365_amd import selector as S


def random_model(seed):
    rng = np.random.default_rng(seed)
    dims = [S.N_FEATURES, S.HIDDEN, S.HIDDEN, 1]
    layers = [{"W": (rng.standard_normal((dims[i + 1], dims[i])) / math.sqrt(dims[i])).tolist(),
               "b": (0.1 * rng.standard_normal(dims[i + 1])).tolist()} for i in range(3)]
    return {"hidden": S.HIDDEN, "configs": [list(c) for c in S.CONFIGS], "layers": layers,
            "out_scale": [0.0, 0.5], "range": [S.N_LO, S.N_HI, S.BATCH_HI], "fallback_margin": 0.02}


SHAPES = [(n, b) for n in (1, 7, 8, 64, 100, 511, 512, 513, 1000, 4096, 5000, 16384, 32768, 40000)
          for b in (1, 2, 300, 20000, 30000)]


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_c_selector_matches_python(seed):
    model = random_model(seed)
    packed = S.pack(model)
    sel = S.Selector(model)
    for n, b in SHAPES:
        for p in S.PRECISIONS:
            cand = S.candidates(n, b)
            scores = np.array([sel.score(n, b, p, v, nb) for v, nb in cand])
            order = np.sort(scores)
            got = mlu.select(n, p, model=packed, batch=b, with_fallback=True)
            v, nb, fb, margin = sel.choose_model(n, b, p)
            gap = order[1] - order[0] if len(order) > 1 else np.inf
            if gap > 1e-4 * max(1.0, abs(order[0])):   # no near-tie: the choice is unique
                assert got[:2] == (v, nb), (n, b, p)
            else:
                assert got[:2] in [c for c, s in zip(cand, scores) if s <= order[0] + 1e-3]
            if abs(margin - 0.02) > 1e-3:              # the fallback flag away from its threshold
                assert got[2] == fb, (n, b, p, margin)


def test_candidates_and_fallback_rules():
    assert S.candidates(100, 50) == list(S.BATCH_CONFIGS)
    assert S.candidates(600, 50) == S.candidates(600, 1)
    assert all(v != "ll" or -(-30000 // nb) <= S.LL_MAX_PANELS for v, nb in S.candidates(30000, 1))
    sel = S.Selector(random_model(0))
    assert sel.choose_model(40000, 1, "fp64")[2]          # outside the trained range
    assert sel.choose_model(100, 30000, "fp64")[2]
    calls = []
    pick = sel.choose(40000, 1, "fp64", tuner=lambda n, b, p: calls.append((n, b, p)) or ("la", 512))
    assert pick == ("la", 512) and calls == [(40000, 1, "fp64")]


def test_select_argument_checks():
    packed = S.pack(random_model(0))
    arr = (ctypes.c_float * len(packed))(*packed)
    v, nb, fb = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    base = dict(model=ctypes.cast(arr, ctypes.c_void_p), model_len=len(packed), n=100, batch=1, precision=0,
                variant=ctypes.cast(ctypes.byref(v), ctypes.c_void_p),
                nb=ctypes.cast(ctypes.byref(nb), ctypes.c_void_p), fallback=ctypes.cast(ctypes.byref(fb),
                                                                                       ctypes.c_void_p))
    fn = mlu._call
    for key, bad, code in [("model", None, -1), ("model_len", 3, -2), ("model_len", 100, -2), ("n", 0, -3),
                           ("batch", 0, -4), ("precision", 2, -5), ("variant", None, -6), ("nb", None, -7),
                           ("fallback", None, -8)]:
        kw = dict(base)
        kw[key] = bad
        assert fn("mlu_select", *kw.values()) == code, key
    assert fn("mlu_select", *base.values()) == 0 and (v.value, nb.value) in [(i, b) for i in range(3) for b in S.NBS]
    kw = dict(base)
    kw["batch"] = 64
    assert fn("mlu_select", *kw.values()) == 0 and v.value == mlu.VARIANT_IDS.get("batched", 3) and nb.value in (16, 32)


def synthetic_records(ns, batches):
    """Timings with a known best: LA best for one matrix, its best block size
    growing with n; for batches the panel width 32 best from order 128 on."""
    recs = []
    for n in ns:
        best_nb = 64 if n < 1024 else (128 if n < 4096 else 256)
        for p in S.PRECISIONS:
            for v, nb in S.candidates(n, 1):
                t = (2 * n ** 3 / 3 / 1e9 / (40.0 if p == "fp32" else 30.0)) * \
                    (1 + 0.3 * abs(math.log2(nb / best_nb))) * {"la": 1.0, "rl": 1.2, "ll": 1.5}[v] + 1e-3
                recs.append({"n": n, "batch": 1, "precision": p, "variant": v, "nb": nb, "ms": t})
    for n, b in batches:
        for p in S.PRECISIONS:
            for v, nb in S.candidates(n, b):
                good = 32 if n >= 128 else 16
                t = b * (2 * n ** 3 / 3 / 1e9 / 8.0 + 2e-5 * n) * (1.0 if nb == good else 1.25) + 5e-3
                recs.append({"n": n, "batch": b, "precision": p, "variant": v, "nb": nb, "ms": t})
    return recs


def test_training_recovers_a_known_best():
    train = synthetic_records(S.sizes(count=24), S.batch_grid())
    hs, hb = S.held_out_shapes(singles=10, batches=10)
    held = synthetic_records(hs, hb)
    model, report = S.train(train, held, epochs=1500)
    assert report["held_out"]["mean_regret"] < 0.05
    assert report["held_out"]["mean_regret"] < report["held_out_single_fixed_la256_mean_regret"]
    assert report["held_out_with_autotuner_fallback"]["mean_regret"] <= report["held_out"]["mean_regret"] + 1e-12


def test_held_out_shapes_are_outside_the_sweep():
    hs, hb = S.held_out_shapes()
    assert not set(hs) & set(S.sizes()) and all(n % 8 for n in hs)
    assert not set(hb) & set(S.batch_grid())
