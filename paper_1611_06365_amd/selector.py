"""Choosing the variant and block size: an exhaustive autotuner and a learned
selector (the block-size study of Section 5.1, where the best b_o depends on the
algorithm and the problem size, turned into a model).

* The exhaustive autotuner (`time_single`, `time_batched`, `autotune`) times
  configurations on the GPU: for one matrix of order n every variant (RL, LL,
  LA) with every outer block size b of NBS through mlu_dgetrf / mlu_dsgetrf;
  for a batch of `batch` matrices of order n <= 512 the batched kernel with
  each panel width of BATCH_NBS.  Matrices are A = B B^T + n I.
* `collect` runs it over a sweep of shapes (the training set) and over shapes
  drawn outside the sweep (the held-out set) and writes the timings as JSON.
* `train` fits the selector: a multilayer perceptron in FP32 (3 layers, 64
  hidden units, ReLU) from (n, batch count, precision, variant id, block size)
  to the logarithm of the time per flop.  For a shape, every candidate
  configuration is scored and the smallest predicted time wins.  The regret
  (time of the choice / time of the autotuner's best - 1) is reported on the
  held-out shapes, with the model alone and with the autotuner as fallback.
* `Selector.choose` predicts; it defers to the autotuner (when one is given)
  for shapes outside the training range or when the best two predictions are
  within FALLBACK_MARGIN of each other.  `pack` flattens the model into the
  float array that the C entry point mlu_select evaluates (the same features,
  candidates and fallback rule).

    python -m paper_1611_06365_amd.selector collect --out timings.json
    python -m paper_1611_06365_amd.selector train timings.json --out model.json
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

VARIANTS = ("rl", "ll", "la")
VARIANT_IDS = {"rl": 0, "ll": 1, "la": 2, "batched": 3}
NBS = (64, 128, 192, 256, 384, 512)
BATCH_NBS = (16, 32)
SINGLE_CONFIGS = tuple((v, nb) for v in VARIANTS for nb in NBS)
BATCH_CONFIGS = tuple(("batched", nb) for nb in BATCH_NBS)
CONFIGS = SINGLE_CONFIGS + BATCH_CONFIGS
PRECISIONS = ("fp64", "fp32")
NB_INNER = 16
HIDDEN = 64
N_FEATURES = 9
BATCH_MAX_N = 512
# training range (shapes outside it go to the autotuner when one is given)
N_LO, N_HI, BATCH_HI = 8, 32768, 20000
FALLBACK_MARGIN = 0.005
MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_model.json")


def features(n: int, batch: int, precision: str, variant: str, nb: int) -> list[float]:
    """(log2 n scaled to about [0, 1] over 64..32768, its square, log2 of the
    batch count scaled to about [0, 1] over 1..20000, the FP32 flag, the
    variant one-hot (RL, LL, LA, batched), log2 b scaled)."""
    x = (math.log2(max(n, 1)) - 6.0) / 9.0
    bb = math.log2(max(batch, 1)) / 14.3
    onehot = [0.0] * 4
    onehot[VARIANT_IDS[variant]] = 1.0
    y = (math.log2(max(nb, 1)) - 4.0) / 5.0
    return [x, x * x, bb, 1.0 if precision == "fp32" else 0.0, *onehot, y]


LL_MAX_PANELS = 48


def worth_timing(n: int, variant: str, nb: int) -> bool:
    """The left-looking variant revisits every earlier panel for each new one
    (about p^2 / 2 solves and updates for p panels); beyond LL_MAX_PANELS
    panels it is not a candidate (far slower than the others)."""
    return variant != "ll" or -(-n // nb) <= LL_MAX_PANELS


def candidates(n: int, batch: int) -> list[tuple[str, int]]:
    """The configurations that can factor `batch` matrices of order n: the
    batched kernel's panel widths for a batch of small matrices, else every
    single-matrix variant and block size (one call per matrix)."""
    if batch > 1 and n <= BATCH_MAX_N:
        return list(BATCH_CONFIGS)
    return [c for c in SINGLE_CONFIGS if worth_timing(n, *c)]


def sizes(lo: int = 64, hi: int = 32768, count: int = 40) -> list[int]:
    """`count` orders log-uniform in [lo, hi], rounded to multiples of 8."""
    out = []
    for i in range(count):
        v = lo * (hi / lo) ** (i / (count - 1))
        out.append(int(round(v / 8.0)) * 8)
    return sorted(set(out))


BATCH_MAX_ELEMS = 1 << 28   # largest batch timed: batch x n^2 <= 2^28 (2 GiB in FP64)


def batch_grid() -> list[tuple[int, int]]:
    """The batched training sweep: (order, batch count) pairs, up to
    BATCH_MAX_ELEMS elements per batch."""
    ns = (8, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512)
    bs = (16, 128, 1024, 8192, 20000)
    return [(n, b) for n in ns for b in bs if b * n * n <= BATCH_MAX_ELEMS]


def held_out_shapes(seed: int = 7, singles: int = 24, batches: int = 24):
    """Shapes drawn outside the sweeps: orders log-uniform in [64, 32768]
    that are not multiples of 8 (the sweep's are), and batched (order, count)
    pairs with the order uniform in [9, 511] and the count log-uniform in
    [20, 20000] (up to BATCH_MAX_ELEMS elements), avoiding the sweep's
    values."""
    import numpy as np

    rng = np.random.default_rng(seed)
    grid_n = set(sizes())
    out_single = set()
    while len(out_single) < singles:
        n = int(round(64 * 512 ** rng.random()))
        if n % 8 != 0 and n not in grid_n and 64 <= n <= 32768:
            out_single.add(n)
    grid_b = set(batch_grid())
    out_batch = set()
    while len(out_batch) < batches:
        n = int(rng.integers(9, 512))
        b = int(round(20 * 1000 ** rng.random()))
        if (n, b) not in grid_b and b * n * n <= BATCH_MAX_ELEMS:
            out_batch.add((n, b))
    return sorted(out_single), sorted(out_batch)


# ---------------------------------------------------------------- autotuner
def _spd_batch(n, batch, dtype, dev, seed=0):
    """`batch` matrices B B^T + n I of order n in one buffer; returns (buffer, views)."""
    import torch

    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    b = torch.randn(batch, n, n, generator=g, dtype=torch.float64, device=dev)
    a = torch.bmm(b, b.transpose(1, 2).contiguous())
    a.diagonal(dim1=1, dim2=2).add_(float(n))
    buf = a.to(dtype).contiguous()
    del a, b
    return buf, [buf[i] for i in range(batch)]


def time_single(mlu, A, M, n, variant, nb, precision, work, ipiv, info, reps):
    """Best time (ms) of `reps` factorizations after one warm-up."""
    import torch

    best = None
    for r in range(reps + 1):   # the first run is a warm-up
        M.copy_(A)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        mlu.getrf(M, variant=variant, nb=nb, nb_inner=NB_INNER, ipiv=ipiv, info=info, work=work,
                  precision=precision)
        e1.record()
        torch.cuda.synchronize()
        if r > 0:
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
    if int(info.item()) != 0:
        raise RuntimeError(f"info {int(info.item())} for n={n} {variant} nb={nb} {precision}")
    return best


def time_batched(mlu, buf, pristine, mats, n, nb, reps):
    """Best time (ms) of `reps` batched factorizations after one warm-up."""
    import torch

    plan = mlu.BatchPlan(mats, max_n=n, nb=nb)
    best = None
    for r in range(reps + 1):
        buf.copy_(pristine)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        plan.run()
        e1.record()
        torch.cuda.synchronize()
        if r > 0:
            t = e0.elapsed_time(e1)
            best = t if best is None else min(best, t)
    if int((plan.info != 0).sum().item()) != 0:
        raise RuntimeError(f"nonzero info in a batch of order {n}")
    return best


def _reps(n, batch=1):
    work = batch * n ** 3
    return 3 if work <= 4096 ** 3 else (2 if work <= 12288 ** 3 else 1)


def time_shape(n, batch, precision, configs=None, log=None):
    """The exhaustive autotuner: time every candidate configuration for
    `batch` matrices of order n; returns [record]."""
    import torch

    import inputs.device as D
    from paper_1611_06365_amd import mlu

    mlu.load()
    dev = torch.device("cuda:0")
    configs = candidates(n, batch) if configs is None else configs
    recs = []
    if configs and configs[0][0] == "batched":
        dt = torch.float64 if precision == "fp64" else torch.float32
        buf, mats = _spd_batch(n, batch, dt, dev)
        pristine = buf.clone()
        for v, nb in configs:
            ms = time_batched(mlu, buf, pristine, mats, n, nb, _reps(n, batch))
            recs.append({"n": n, "batch": batch, "precision": precision, "variant": v, "nb": nb, "ms": ms})
        del buf, pristine, mats
    else:
        work = mlu.workspace(dev)
        A = D.spd_bbt(n, seed=0, device=dev)
        M = torch.empty_like(A)
        ipiv = torch.empty(n, dtype=torch.int32, device=dev)
        info = torch.empty(1, dtype=torch.int32, device=dev)
        for v, nb in configs:
            # one matrix per call: a batch of them takes `batch` times as long
            ms = batch * time_single(mlu, A, M, n, v, nb, precision, work, ipiv, info, _reps(n))
            recs.append({"n": n, "batch": batch, "precision": precision, "variant": v, "nb": nb, "ms": ms})
        del A, M
    torch.cuda.empty_cache()
    if log is not None and recs:
        best = min(recs, key=lambda r: r["ms"])
        log(f"[selector] n={n} batch={batch} {precision}: best {best['variant']} nb={best['nb']} "
            f"{best['ms']:.3f} ms", flush=True)
    return recs


def autotune(n, batch=1, precision="fp64", configs=None):
    """The fallback: (variant, nb) of the fastest timed candidate."""
    recs = time_shape(n, batch, precision, configs)
    best = min(recs, key=lambda r: r["ms"])
    return best["variant"], int(best["nb"])


def collect(out_path, precisions=PRECISIONS, max_n=32768, count=40, log=print):
    """Time the training sweep and the held-out shapes; write JSON."""
    import torch

    train_recs, held_recs = [], []
    for n in sizes(hi=max_n, count=count):
        for p in precisions:
            train_recs += time_shape(n, 1, p, log=log)
    for n, b in batch_grid():
        for p in precisions:
            train_recs += time_shape(n, b, p, log=log)
    hs, hb = held_out_shapes()
    for n in hs:
        if n <= max_n:
            for p in precisions:
                held_recs += time_shape(n, 1, p, log=log)
    for n, b in hb:
        for p in precisions:
            held_recs += time_shape(n, b, p, log=log)
    meta = {"what": "factorization time per configuration, A = B B^T + n I, nb_inner 16 (single matrices), "
                    "batches of equal orders (batched kernel); best of the timed runs after one warm-up, HIP events",
            "device": torch.cuda.get_device_name(0), "records": train_recs, "held_out_records": held_recs}
    with open(out_path, "w") as f:
        json.dump(meta, f)
    return train_recs, held_recs


# ---------------------------------------------------------------- model
def _gflop(n, batch):
    return batch * 2.0 * n ** 3 / 3.0 / 1e9


def _target(r):
    """log of the time per GFLOP (ms) of a record."""
    return math.log(r["ms"] / _gflop(r["n"], r["batch"]))


def _by_shape(recs):
    out = {}
    for r in recs:
        if r.get("ms") is None:
            continue
        out.setdefault((r["n"], r["batch"], r["precision"]), {})[(r["variant"], int(r["nb"]))] = r["ms"]
    return out


def regret_report(sel, recs, use_fallback=False):
    """Regret of the selector's choices on the shapes of `recs` (every
    candidate timed there: the exhaustive autotuner's best is the reference).
    With use_fallback, shapes the selector defers take the autotuner's best
    (regret 0) and are counted."""
    import numpy as np

    regrets, deferred, kinds, worst = [], 0, {"single": [], "batched": []}, None
    for (n, b, p), times in sorted(_by_shape(recs).items()):
        best = min(times.values())
        v, nb, fallback, _ = sel.choose_model(n, b, p)
        if use_fallback and fallback:
            deferred += 1
            r = 0.0
        else:
            t = times.get((v, nb))
            if t is None:
                continue
            r = t / best - 1.0
        regrets.append(r)
        kinds["batched" if v == "batched" else "single"].append(r)
        if worst is None or r > worst["regret"]:
            bv, bnb = min(times, key=times.get)
            worst = {"n": n, "batch": b, "precision": p, "chosen": [v, nb], "best": [bv, bnb], "regret": r}
    if not regrets:
        return None
    return {"cases": len(regrets), "mean_regret": float(np.mean(regrets)), "max_regret": float(np.max(regrets)),
            "share_exact": float(np.mean([r == 0.0 for r in regrets])), "deferred_to_autotuner": deferred,
            "mean_regret_by_kind": {k: (float(np.mean(x)) if x else None) for k, x in kinds.items()},
            "worst": worst}


def train(recs, held=None, epochs=4000, seed=0, lr=3e-3):
    """Fit the MLP on `recs` (all training shapes); returns (model, report)
    with the regret on the training shapes and on the held-out records."""
    import numpy as np
    import torch

    good = [r for r in recs if r.get("ms") is not None]
    X = torch.tensor([features(r["n"], r["batch"], r["precision"], r["variant"], r["nb"]) for r in good],
                     dtype=torch.float32)
    Y = torch.tensor([_target(r) for r in good], dtype=torch.float32)
    mu, sd = Y.mean(), Y.std() + 1e-6
    torch.manual_seed(seed)
    net = torch.nn.Sequential(torch.nn.Linear(N_FEATURES, HIDDEN), torch.nn.ReLU(),
                              torch.nn.Linear(HIDDEN, HIDDEN), torch.nn.ReLU(),
                              torch.nn.Linear(HIDDEN, 1))
    opt = torch.optim.Adam(net.parameters(), lr=lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, epochs)
    for _ in range(epochs):
        opt.zero_grad()
        loss = ((net(X)[:, 0] - (Y - mu) / sd) ** 2).mean()
        loss.backward()
        opt.step()
        sched.step()
    layers = [m for m in net if isinstance(m, torch.nn.Linear)]
    model = {"features": "log2 n scaled, its square, log2 batch scaled, fp32 flag, variant one-hot "
                         "(rl, ll, la, batched), log2 nb scaled", "hidden": HIDDEN,
             "configs": [list(c) for c in CONFIGS], "out_scale": [float(mu), float(sd)],
             "range": [N_LO, N_HI, BATCH_HI], "fallback_margin": FALLBACK_MARGIN,
             "layers": [{"W": l.weight.detach().numpy().tolist(), "b": l.bias.detach().numpy().tolist()}
                        for l in layers]}
    sel = Selector(model)
    report = {"training_timings": len(good), "final_train_loss": float(loss.item()),
              "train": regret_report(sel, good)}
    if held:
        report["held_out_timings"] = sum(1 for r in held if r.get("ms") is not None)
        report["held_out"] = regret_report(sel, held)
        report["held_out_with_autotuner_fallback"] = regret_report(sel, held, use_fallback=True)
        fixed = []
        for (n, b, p), times in _by_shape(held).items():
            if b == 1 and ("la", 256) in times:
                fixed.append(times[("la", 256)] / min(times.values()) - 1.0)
        report["held_out_single_fixed_la256_mean_regret"] = float(np.mean(fixed)) if fixed else None
    return model, report


class Selector:
    """The trained MLP: choose(n, batch, precision) -> (variant, nb)."""

    def __init__(self, model=None):
        if model is None:
            with open(MODEL_PATH) as f:
                model = json.load(f)
        import numpy as np

        self.model = model
        self.layers = [(np.asarray(l["W"], dtype=np.float32), np.asarray(l["b"], dtype=np.float32))
                       for l in model["layers"]]
        self.range = model.get("range", [N_LO, N_HI, BATCH_HI])
        self.margin = model.get("fallback_margin", FALLBACK_MARGIN)

    def score(self, n, batch, precision, variant, nb):
        """Predicted (scaled) log time per flop of one configuration."""
        import numpy as np

        h = np.asarray(features(n, batch, precision, variant, nb), dtype=np.float32)
        for i, (W, b) in enumerate(self.layers):
            h = W @ h + b
            if i + 1 < len(self.layers):
                h = np.maximum(h, np.float32(0.0))
        return float(h[0])

    def choose_model(self, n, batch=1, precision="fp64"):
        """(variant, nb, fallback, margin): the model's choice, whether it
        defers to the autotuner (shape outside the training range, or the
        runner-up predicted within `margin`), and the predicted margin."""
        cand = candidates(n, batch)
        scores = sorted((self.score(n, batch, precision, v, nb), i) for i, (v, nb) in enumerate(cand))
        v, nb = cand[scores[0][1]]
        # a score is (log time - mu) / sd: the runner-up's predicted relative gap
        sd = self.model.get("out_scale", [0.0, 1.0])[1]
        margin = math.exp((scores[1][0] - scores[0][0]) * sd) - 1.0 if len(scores) > 1 else float("inf")
        lo, hi, bhi = self.range
        outside = n < lo or n > hi or batch < 1 or batch > bhi
        return v, int(nb), bool(outside or margin < self.margin), margin

    def predict(self, n, precision="fp64", batch=1):
        v, nb, _, _ = self.choose_model(n, batch, precision)
        return v, nb

    def choose(self, n, batch=1, precision="fp64", tuner=None):
        """The model's choice, or the autotuner's (tuner(n, batch, precision)
        -> (variant, nb), e.g. `autotune`) when the model defers."""
        v, nb, fallback, _ = self.choose_model(n, batch, precision)
        if fallback and tuner is not None:
            return tuner(n, batch, precision)
        return v, nb


PACK_HEADER = 12


def pack(model) -> list[float]:
    """The float array mlu_select evaluates: a header [version 2, n_in,
    hidden, n_layers, n_cand, n_lo, n_hi, batch_hi, fallback margin, output
    scale sd, LL panel limit, batched order limit], per candidate its
    (variant id, nb), then per layer W row-major and b (the last layer has one
    output)."""
    layers = model["layers"]
    cfg = model["configs"]
    lo, hi, bhi = model.get("range", [N_LO, N_HI, BATCH_HI])
    out = [2.0, float(len(layers[0]["W"][0])), float(model["hidden"]), float(len(layers)), float(len(cfg)),
           float(lo), float(hi), float(bhi), float(model.get("fallback_margin", FALLBACK_MARGIN)),
           float(model.get("out_scale", [0.0, 1.0])[1]), float(LL_MAX_PANELS), float(BATCH_MAX_N)]
    assert len(out) == PACK_HEADER
    for v, nb in cfg:
        out += [float(VARIANT_IDS[v]), float(nb)]
    for l in layers:
        for row in l["W"]:
            out += [float(x) for x in row]
        out += [float(x) for x in l["b"]]
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_1611_06365_amd.selector")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect", help="time every configuration on the GPU (exhaustive autotuner)")
    c.add_argument("--out", required=True)
    c.add_argument("--count", type=int, default=40)
    c.add_argument("--max-n", type=int, default=32768)
    t = sub.add_parser("train", help="fit the selector on collected timings")
    t.add_argument("timings")
    t.add_argument("--out", default=MODEL_PATH)
    t.add_argument("--report", default=None)
    args = ap.parse_args(argv)
    if args.cmd == "collect":
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        if root not in sys.path:
            sys.path.insert(0, root)
        t0 = time.time()
        collect(args.out, max_n=args.max_n, count=args.count)
        print(f"[selector] collected in {time.time() - t0:.1f} s", flush=True)
        return 0
    with open(args.timings) as f:
        data = json.load(f)
    model, report = train(data["records"], data.get("held_out_records"))
    with open(args.out, "w") as f:
        json.dump(model, f)
    print(json.dumps(report, indent=1))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
