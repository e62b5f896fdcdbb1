"""The learned selector: the C evaluation (mlu_select) against the Python one
on the same packed model, its argument checks, and the training machinery on
synthetic timings with a known best configuration (CPU only)."""
import math

import numpy as np
import pytest

from paper_1611_06365_amd import mlu
from paper_1611_06365_amd import selector as S


def random_model(seed):
    rng = np.random.default_rng(seed)
    dims = [3, S.HIDDEN, S.HIDDEN, len(S.CONFIGS)]
    layers = [{"W": (rng.standard_normal((dims[i + 1], dims[i])) / math.sqrt(dims[i])).tolist(),
               "b": (0.1 * rng.standard_normal(dims[i + 1])).tolist()} for i in range(3)]
    return {"hidden": S.HIDDEN, "configs": [list(c) for c in S.CONFIGS], "layers": layers}


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_c_selector_matches_python(seed):
    model = random_model(seed)
    packed = S.pack(model)
    sel = S.Selector(model)
    for n in [1, 7, 64, 100, 1000, 4096, 5000, 16384, 32768, 40000]:
        for p in S.PRECISIONS:
            s = sel.scores(n, p)
            order = np.sort(s)
            got = mlu.select(n, p, model=packed)
            want = sel.predict(n, p)
            if order[1] - order[0] > 1e-4 * max(1.0, abs(order[0])):   # no near-tie: the choice is unique
                assert got == want, (n, p)
            else:
                assert got in [tuple(c) for c in np.array(S.CONFIGS, dtype=object)[s <= order[0] + 1e-3]]


def test_select_argument_checks():
    import ctypes

    packed = S.pack(random_model(0))
    arr = (ctypes.c_float * len(packed))(*packed)
    v, nb = ctypes.c_int(), ctypes.c_int()
    base = dict(model=ctypes.cast(arr, ctypes.c_void_p), model_len=len(packed), n=100, precision=0,
                variant=ctypes.cast(ctypes.byref(v), ctypes.c_void_p), nb=ctypes.cast(ctypes.byref(nb),
                                                                                     ctypes.c_void_p))
    fn = mlu._call
    for key, bad, code in [("model", None, -1), ("model_len", 3, -2), ("model_len", 100, -2), ("n", 0, -3),
                           ("precision", 2, -4), ("variant", None, -5), ("nb", None, -6)]:
        kw = dict(base)
        kw[key] = bad
        assert fn("mlu_select", *kw.values()) == code, key
    assert fn("mlu_select", *base.values()) == 0 and (v.value, nb.value) in [(i, b) for i in range(3) for b in S.NBS]


def test_training_recovers_a_known_best():
    # synthetic timings: LA best, with the best block size growing with n
    recs = []
    for n in S.sizes(count=24):
        best_nb = 64 if n < 1024 else (128 if n < 4096 else 256)
        for p in S.PRECISIONS:
            for v, nb in S.CONFIGS:
                t = (2 * n ** 3 / 3 / 1e9 / (40.0 if p == "fp32" else 30.0)) * \
                    (1 + 0.3 * abs(math.log2(nb / best_nb))) * {"la": 1.0, "rl": 1.2, "ll": 1.5}[v] + 1e-3
                recs.append({"n": n, "precision": p, "variant": v, "nb": nb,
                             "ms": t if S.worth_timing(n, v, nb) else None})
    model, report = S.train(recs, epochs=800)
    assert report["held_out"]["mean_regret"] < 0.1
    assert report["held_out"]["mean_regret"] < report["held_out_fixed_la256_mean_regret"]
