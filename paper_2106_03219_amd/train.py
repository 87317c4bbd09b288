"""Train the learned launch-configuration picker on the GPU.

Reads the autotuner's timing database (tune.py), labels every instance with
its fastest class, and trains the F -> 64 -> 64 -> K ReLU network with the
library's own kernels (omprt_mlp_loss_grad, omprt_mlp_adam; fp32, Adam,
mini-batches).  Evaluates on held-out instances:

  regret_i = t_i[predicted class] / min_j t_i[j] - 1   (vs the autotuner)
  gain     = geometric mean of t_i[heuristic] / t_i[predicted]

and writes the model file the runtime loads with omprt_model_load.

    python -m paper_2106_03219_amd.train --train TRAIN.jsonl --heldout HELD.jsonl \
        --out paper_2106_03219_amd/picker_model.txt
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from .tune import CLASSES

DIMS = (16, 64, 64, len(CLASSES))


def load_db(path):
    recs = [json.loads(l) for l in open(path) if l.strip()]
    recs.sort(key=lambda r: r["id"])
    return recs


def abi_chunk(r):
    """The chunk the runtime sees: an AXPY body without a user chunk runs
    schedule(static) with no chunk size (0); reductions have none (-1)."""
    return max(r["chunk"], 0) if r["body"] else -1


def feature_matrix(om, recs):
    return np.array([om.model_features(r["n"], r["dtype"], r["op"], r["body"], abi_chunk(r))
                     for r in recs], dtype=np.float32)


def init_params(seed, dims=DIMS):
    F, H1, H2, K = dims
    g = np.random.Generator(np.random.PCG64(seed))

    def he(o, i):
        return (g.uniform(-1, 1, (o, i)) * math.sqrt(6.0 / i)).astype(np.float32)
    parts = [he(H1, F), np.zeros(H1, np.float32), he(H2, H1), np.zeros(H2, np.float32),
             he(K, H2) * 0.1, np.zeros(K, np.float32)]
    return np.concatenate([p.ravel() for p in parts])


def predict(om, torch, params, X):
    Xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    Z = torch.zeros((X.shape[0], DIMS[3]), dtype=torch.float32, device="cuda")
    om.mlp_forward(DIMS, params, Xd, Z)
    torch.cuda.synchronize()
    z = Z.cpu().numpy()
    zz = z - z.max(axis=1, keepdims=True)
    p = np.exp(zz) / np.exp(zz).sum(axis=1, keepdims=True)
    return z.argmax(axis=1), p.max(axis=1)


def picked_times(recs, pred, conf, tau):
    """Time of the configuration the runtime would use: the predicted class when the
    network's softmax confidence reaches tau, else the heuristic's."""
    t = np.array([r["times_us"] for r in recs])
    th = np.array([r["heuristic_us"] for r in recs])
    tp = t[np.arange(len(recs)), pred]
    return np.where(conf >= tau, tp, th)


def choose_tau(recs, pred, conf, grid=(0.0, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7)):
    """Confidence threshold minimising the geometric-mean time on the training set."""
    best = min(grid, key=lambda tau: float(np.mean(np.log(picked_times(recs, pred, conf, tau)))))
    return float(best)


def evaluate(recs, pred, conf=None, tau=0.0):
    t = np.array([r["times_us"] for r in recs])
    best = t.min(axis=1)
    tp = t[np.arange(len(recs)), pred] if conf is None else picked_times(recs, pred, conf, tau)
    th = np.array([r["heuristic_us"] for r in recs])
    regret = tp / best - 1.0
    h_regret = th / best - 1.0
    return {
        "n": len(recs),
        "regret_mean": float(regret.mean()), "regret_p95": float(np.percentile(regret, 95)),
        "regret_median": float(np.median(regret)),
        "heuristic_regret_mean": float(h_regret.mean()),
        "heuristic_regret_p95": float(np.percentile(h_regret, 95)),
        "gain_vs_heuristic_geomean": float(np.exp(np.mean(np.log(th / tp)))),
        "top1_agreement": float(np.mean(pred == t.argmin(axis=1))),
        "total_time_ratio_vs_heuristic": float(tp.sum() / th.sum()),
        "total_time_ratio_vs_autotuner": float(tp.sum() / best.sum()),
    }


def write_model(path, mean, scale, params, tau):
    F, H1, H2, K = DIMS
    with open(path, "w") as fh:
        fh.write("omprt-mlp 1\n")
        fh.write(f"dims {F} {H1} {H2} {K}\n")
        fh.write(f"tau {tau:.6g}\n")
        fh.write("mean " + " ".join(f"{v:.9g}" for v in mean) + "\n")
        fh.write("scale " + " ".join(f"{v:.9g}" for v in scale) + "\n")
        fh.write("classes\n")
        for c in CLASSES:
            fh.write(" ".join(str(v) for v in c) + "\n")
        fh.write(f"params {params.size}\n")
        for i in range(0, params.size, 8):
            fh.write(" ".join(f"{v:.9g}" for v in params[i:i + 8]) + "\n")


def train(om, torch, X, y, epochs, batch, lr, seed, log=print, mode="graph", times=None):
    """Mini-batch Adam over the rows X (features, normalised) with labels y.

    The rows live on the GPU; every epoch permutes them there (one index_select) so that
    batch j is a fixed slice.  A step is omprt_mlp_loss_grad (forward, mean softmax
    cross-entropy into a per-batch loss slot, backward) and omprt_mlp_adam_counted (the
    step number in device memory).  mode "graph" captures one epoch's steps in a HIP graph
    after a first eager epoch and replays it; "eager" launches the steps one by one;
    "sync" is the plain loop (batches copied from the host, the loss read back every step).
    All three make the same updates in the same order.  `times`, if given, collects the
    seconds of every epoch."""
    F, H1, H2, K = DIMS
    p0 = init_params(seed)
    assert p0.size == om.mlp_param_count(*DIMS)
    params = torch.from_numpy(p0).cuda()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    grads = torch.zeros_like(params)
    N = len(y)
    starts = list(range(0, N, batch))
    sizes = torch.tensor([min(batch, N - s0) for s0 in starts], dtype=torch.float32,
                         device="cuda")
    losses = torch.zeros(len(starts), dtype=torch.float32, device="cuda")
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()
    yd = torch.from_numpy(np.ascontiguousarray(y, dtype=np.int32)).cuda()
    Xp, yp = torch.empty_like(Xd), torch.empty_like(yd)
    g = np.random.Generator(np.random.PCG64(seed + 1))

    def steps():
        for j, s0 in enumerate(starts):
            s1 = min(s0 + batch, N)
            om.mlp_loss_grad(DIMS, params, Xp[s0:s1], yp[s0:s1], losses[j:j + 1], grads)
            om.mlp_adam_counted(params, m, v, grads, step, lr=lr)

    stream = torch.cuda.Stream()
    graph = None
    with torch.cuda.stream(stream):
        for ep in range(epochs):
            t0 = time.perf_counter()
            order = g.permutation(N)
            if mode == "sync":
                tot = 0.0
                for j, s0 in enumerate(starts):
                    idx = order[s0:s0 + batch]
                    Xb = torch.from_numpy(np.ascontiguousarray(X[idx])).cuda()
                    yb = torch.from_numpy(np.ascontiguousarray(y[idx])).cuda()
                    om.mlp_loss_grad(DIMS, params, Xb, yb, losses[j:j + 1], grads)
                    om.mlp_adam_counted(params, m, v, grads, step, lr=lr)
                    tot += losses[j].item() * len(idx)
            else:
                od = torch.from_numpy(order).cuda()
                torch.index_select(Xd, 0, od, out=Xp)
                torch.index_select(yd, 0, od, out=yp)
                if mode == "graph" and ep > 0 and graph is None:
                    graph = torch.cuda.CUDAGraph()
                    with torch.cuda.graph(graph, stream=stream):
                        steps()
                if graph is not None:
                    graph.replay()
                else:
                    steps()
            if times is not None:
                stream.synchronize()
                times.append(time.perf_counter() - t0)
            if ep % 10 == 0 or ep == epochs - 1:
                if mode != "sync":
                    tot = float((losses * sizes).sum().item())
                log(f"[train] epoch {ep} mean loss {tot / N:.4f}")
    torch.cuda.synchronize()
    return params


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", required=True)
    ap.add_argument("--heldout", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--report", default=None)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tau", type=float, default=-1.0,
                    help="confidence threshold; negative = choose on the training set")
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--mode", default="graph", choices=("graph", "eager", "sync"),
                    help="how the training steps are launched (same updates in every mode)")
    args = ap.parse_args(argv)

    import torch

    import paper_2106_03219_amd as om
    om.load()
    om.model_load(None)
    tr, ho = load_db(args.train), load_db(args.heldout)
    Xtr, Xho = feature_matrix(om, tr), feature_matrix(om, ho)
    ytr = np.array([int(np.argmin(r["times_us"])) for r in tr], dtype=np.int32)
    mean = Xtr.mean(axis=0)
    std = Xtr.std(axis=0)
    scale = np.where(std > 1e-6, 1.0 / np.maximum(std, 1e-6), 1.0).astype(np.float32)
    Xn = ((Xtr - mean) * scale).astype(np.float32)
    Xhn = ((Xho - mean) * scale).astype(np.float32)
    ep_times = []
    params = train(om, torch, Xn, ytr, args.epochs, args.batch, args.lr, args.seed,
                   mode=args.mode, times=ep_times)
    pred_tr, conf_tr = predict(om, torch, params, Xn)
    pred_ho, conf_ho = predict(om, torch, params, Xhn)
    tau = choose_tau(tr, pred_tr, conf_tr) if args.tau < 0 else args.tau
    p_host = params.cpu().numpy()
    write_model(args.out, mean, scale, p_host, tau)
    report = {"train": evaluate(tr, pred_tr, conf_tr, tau),
              "heldout": evaluate(ho, pred_ho, conf_ho, tau),
              "heldout_model_only": evaluate(ho, pred_ho),
              "heldout_fallback_fraction": float(np.mean(conf_ho < tau)),
              "tau": tau, "train_label_accuracy": float(np.mean(pred_tr == ytr)),
              "classes": len(CLASSES), "epochs": args.epochs, "batch": args.batch, "lr": args.lr,
              "mode": args.mode,
              "epoch_ms_median": round(1e3 * float(np.median(ep_times[1:] or ep_times)), 3)}
    # the runtime's C++ inference must reproduce the GPU network's choice
    om.model_load(args.out)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    from .tune import class_config
    agree = 0
    for r, k, c in zip(ho, pred_ho, conf_ho):
        cfg, src = om.resolve_config(r["n"], r["dtype"], r["op"], r["body"], abi_chunk(r))
        if c < tau:
            agree += int(src != 1)
            continue
        bpi = 12 if r["body"] else {0: 4, 1: 8, 2: 4, 3: 8, 4: 2}[r["dtype"]]
        agree += int(src == 1 and cfg == class_config(CLASSES[k], r["n"], bpi, cus))
    report["host_inference_agreement"] = agree / len(ho)
    om.model_load(None)
    print(json.dumps(report, indent=1))
    if args.report:
        json.dump(report, open(args.report, "w"), indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
