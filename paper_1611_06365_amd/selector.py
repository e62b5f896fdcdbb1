"""Choosing the variant and block size: an exhaustive autotuner and a learned
selector (the block-size study of Section 5.1, where the best b_o depends on the
algorithm and the problem size, turned into a model).

* `collect` is the exhaustive autotuner: it times every configuration of
  CONFIGS (variant x outer block size b, inner block size 16) for each order n
  and product precision on the GPU, through mlu_dgetrf / mlu_dsgetrf, on
  A = B B^T + n I, and writes the timings as JSON.
* `train` fits the selector, a multilayer perceptron in FP32 (3 layers, 64
  hidden units, ReLU) from features of (n, precision) to the logarithm of every
  configuration's time per flop; the configuration with the smallest
  predicted time is the choice.  Sizes alternate between a training and a
  held-out set; the regret (time of the choice / best time - 1) is reported on
  both.
* `Selector` loads the trained model (JSON) and predicts; `pack` flattens it
  into the float array that the C entry point mlu_select evaluates.

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
NBS = (64, 128, 192, 256, 384, 512)
CONFIGS = tuple((v, nb) for v in VARIANTS for nb in NBS)
PRECISIONS = ("fp64", "fp32")
NB_INNER = 16
HIDDEN = 64
MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_model.json")


def features(n: int, precision: str) -> list[float]:
    """(log2 n scaled to about [0, 1], its square, the precision flag)."""
    x = (math.log2(max(n, 1)) - 6.0) / 9.0
    return [x, x * x, 1.0 if precision == "fp32" else 0.0]


def sizes(lo: int = 64, hi: int = 32768, count: int = 40) -> list[int]:
    """`count` orders log-uniform in [lo, hi], rounded to multiples of 8."""
    out = []
    for i in range(count):
        v = lo * (hi / lo) ** (i / (count - 1))
        out.append(int(round(v / 8.0)) * 8)
    return sorted(set(out))


# ---------------------------------------------------------------- autotuner
LL_MAX_PANELS = 48


def worth_timing(n: int, variant: str, nb: int) -> bool:
    """The left-looking variant revisits every earlier panel for each new one
    (about p^2 / 2 solves and updates for p panels); beyond LL_MAX_PANELS
    panels it is not timed and counts as 4x the slowest timed configuration."""
    return variant != "ll" or -(-n // nb) <= LL_MAX_PANELS


def time_config(mlu, A, M, n, variant, nb, precision, work, ipiv, info, reps):
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


def collect(ns, out_path, precisions=PRECISIONS, log=print):
    """Time every configuration for every n and precision (the exhaustive
    autotuner); returns the records and writes them to out_path."""
    import torch

    import inputs.device as D
    from paper_1611_06365_amd import mlu

    mlu.load()
    dev = torch.device("cuda:0")
    work = mlu.workspace(dev)
    recs = []
    for n in ns:
        A = D.spd_bbt(n, seed=0, device=dev)
        M = torch.empty_like(A)
        ipiv = torch.empty(n, dtype=torch.int32, device=dev)
        info = torch.empty(1, dtype=torch.int32, device=dev)
        reps = 3 if n <= 4096 else (2 if n <= 12288 else 1)
        for precision in precisions:
            for variant, nb in CONFIGS:
                if not worth_timing(n, variant, nb):
                    recs.append({"n": n, "precision": precision, "variant": variant, "nb": nb, "ms": None})
                    continue
                ms = time_config(mlu, A, M, n, variant, nb, precision, work, ipiv, info, reps)
                recs.append({"n": n, "precision": precision, "variant": variant, "nb": nb, "ms": ms})
            best = min((r for r in recs if r["n"] == n and r["precision"] == precision and r["ms"] is not None),
                       key=lambda r: r["ms"])
            log(f"[selector] n={n} {precision}: best {best['variant']} nb={best['nb']} {best['ms']:.3f} ms",
                flush=True)
        del A, M
        torch.cuda.empty_cache()
    meta = {"what": "getrf time per configuration, A = B B^T + n I (seed 0), nb_inner 16, best of the timed "
                    "runs after one warm-up, HIP events", "configs": [list(c) for c in CONFIGS],
            "device": torch.cuda.get_device_name(0), "records": recs}
    with open(out_path, "w") as f:
        json.dump(meta, f)
    return recs


# ---------------------------------------------------------------- model
def _table(recs):
    """{(n, precision): [ms per config in CONFIGS order]}; untimed entries
    (see worth_timing) are 4x the row's slowest timed one."""
    tab = {}
    idx = {c: i for i, c in enumerate(CONFIGS)}
    seen = {}
    for r in recs:
        key = (r["n"], r["precision"])
        tab.setdefault(key, [None] * len(CONFIGS))[idx[(r["variant"], r["nb"])]] = r["ms"]
        seen.setdefault(key, set()).add(idx[(r["variant"], r["nb"])])
    out = {}
    for k, row in tab.items():
        if len(seen[k]) != len(CONFIGS) or all(x is None for x in row):
            continue
        worst = max(x for x in row if x is not None)
        out[k] = [x if x is not None else 4.0 * worst for x in row]
    return out


def _target(n, ms):
    """log of the time per 2n^3/3 flops (ms per GFLOP) of every configuration."""
    gf = 2.0 * n ** 3 / 3.0 / 1e9
    return [math.log(t / gf) for t in ms]


def train(recs, epochs=3000, seed=0, lr=3e-3):
    """Fit the MLP on the even-indexed sizes, hold out the odd-indexed ones;
    returns (model dict, report dict)."""
    import numpy as np
    import torch

    tab = _table(recs)
    ns = sorted({k[0] for k in tab})
    train_ns = set(ns[0::2])
    keys = sorted(tab)
    X = torch.tensor([features(n, p) for n, p in keys], dtype=torch.float32)
    Y = torch.tensor([_target(n, tab[(n, p)]) for n, p in keys], dtype=torch.float32)
    is_tr = torch.tensor([n in train_ns for n, _ in keys])
    mu, sd = Y[is_tr].mean(), Y[is_tr].std() + 1e-6
    torch.manual_seed(seed)
    net = torch.nn.Sequential(torch.nn.Linear(X.shape[1], HIDDEN), torch.nn.ReLU(),
                              torch.nn.Linear(HIDDEN, HIDDEN), torch.nn.ReLU(),
                              torch.nn.Linear(HIDDEN, len(CONFIGS)))
    opt = torch.optim.Adam(net.parameters(), lr=lr)
    for _ in range(epochs):
        opt.zero_grad()
        loss = ((net(X[is_tr]) - (Y[is_tr] - mu) / sd) ** 2).mean()
        loss.backward()
        opt.step()
    layers = [m for m in net if isinstance(m, torch.nn.Linear)]
    model = {"features": "log2 n scaled, its square, fp32 flag", "hidden": HIDDEN,
             "configs": [list(c) for c in CONFIGS], "out_scale": [float(mu), float(sd)],
             "layers": [{"W": l.weight.detach().numpy().tolist(), "b": l.bias.detach().numpy().tolist()}
                        for l in layers]}
    sel = Selector(model)
    report = {}
    for name, subset in (("train", [k for k in keys if k[0] in train_ns]),
                         ("held_out", [k for k in keys if k[0] not in train_ns])):
        regrets = []
        for n, p in subset:
            ms = tab[(n, p)]
            v, nb = sel.predict(n, p)
            regrets.append(ms[CONFIGS.index((v, nb))] / min(ms) - 1.0)
        report[name] = {"cases": len(subset), "mean_regret": float(np.mean(regrets)),
                        "max_regret": float(np.max(regrets)),
                        "share_exact": float(np.mean([r == 0.0 for r in regrets]))}
    # the fixed default (LA, b = 256) as a reference point
    fixed = [tab[k][CONFIGS.index(("la", 256))] / min(tab[k]) - 1.0 for k in keys if k[0] not in train_ns]
    report["held_out_fixed_la256_mean_regret"] = float(np.mean(fixed))
    report["final_train_loss"] = float(loss.item())
    return model, report


class Selector:
    """The trained MLP: predict(n, precision) -> (variant, nb)."""

    def __init__(self, model=None):
        if model is None:
            with open(MODEL_PATH) as f:
                model = json.load(f)
        import numpy as np

        self.model = model
        self.layers = [(np.asarray(l["W"], dtype=np.float32), np.asarray(l["b"], dtype=np.float32))
                       for l in model["layers"]]
        self.configs = [tuple(c) for c in model["configs"]]

    def scores(self, n, precision):
        import numpy as np

        h = np.asarray(features(n, precision), dtype=np.float32)
        for i, (W, b) in enumerate(self.layers):
            h = W @ h + b
            if i + 1 < len(self.layers):
                h = np.maximum(h, np.float32(0.0))
        return h

    def predict(self, n, precision="fp64"):
        s = self.scores(n, precision)
        v, nb = self.configs[int(s.argmin())]
        return v, int(nb)


def pack(model) -> list[float]:
    """The float array mlu_select evaluates: [n_in, hidden, n_out, n_layers,
    then per output its (variant id, nb), then per layer W row-major and b]."""
    ids = {"rl": 0, "ll": 1, "la": 2}
    layers = model["layers"]
    out = [float(len(layers[0]["W"][0])), float(model["hidden"]), float(len(model["configs"])), float(len(layers))]
    for v, nb in model["configs"]:
        out += [float(ids[v]), float(nb)]
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
        collect(sizes(hi=args.max_n, count=args.count), args.out)
        print(f"[selector] collected in {time.time() - t0:.1f} s", flush=True)
        return 0
    with open(args.timings) as f:
        recs = json.load(f)["records"]
    model, report = train(recs)
    with open(args.out, "w") as f:
        json.dump(model, f)
    print(json.dumps(report, indent=1))
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
