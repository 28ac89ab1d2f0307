"""Train, calibrate and evaluate a learned strip selector on the GPU.

    python -m paper_2506_18003_amd.train_selector --Np 256 --N 262144 --train 16000 --val 2000 --test 2000 \
        --out paper_2506_18003_amd/models/selector_np256

Steps (each GPU step runs in the library's kernels):
  1. seeded signals (synth.workloads.cfg4_signal at a fixed N, or selector_signal with N = 2^U{14..20}),
     drawn by a pool of CPU workers started before the GPU is touched;
  2. per signal on the GPU: selector features (scd_features), the full FP32 SSCA (scd_ssca_ex) and its strip
     labels (scd_strip_labels); only features and labels are kept;
  3. feature standardisation from the training split, then mini-batch BCE training with Adam
     (scd_mlp_forward / scd_mlp_backward / scd_adam_step), checkpointing parameters and Adam state;
  4. calibration on the validation split: theta is the largest score threshold that keeps strip recall
     >= 0.99; the confidence floor is conf_min (0.9);
  5. evaluation on the test split: recall (signals below the confidence floor fall back to the full SSCA and
     count as fully recalled), the fraction of strips computed, the fallback rate, and the same for a selector
     without the network (a threshold on the ACP feature, calibrated the same way).
Outputs <out>.npz / <out>.json (the model, with the metrics under "meta") and <out>.ckpt.npz (Adam state).
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def _gen(job):
    from synth import workloads as W
    kind_fn, i, split, n = job
    if kind_fn == "cfg4":
        return W.cfg4_signal(i, n, split)[1].astype(np.complex64)
    return W.selector_signal(i, split)[1].astype(np.complex64)


def log(*a):
    print(f"[{time.strftime('%H:%M:%S')}]", *a, flush=True)


def build_split(pool, kind_fn, split, count, n, Np, dev, batch=8):
    """(features [count, 2 Np], labels [count, Np], ratios, lengths) of one split."""
    import torch

    import paper_2506_18003_amd as scd
    from paper_2506_18003_amd import selector as SEL

    feats = np.zeros((count, 2 * Np), np.float32)
    labs = np.zeros((count, Np), np.float32)
    ratios = np.zeros((count, Np), np.float32)
    lens = np.zeros(count, np.int64)
    jobs = [(kind_fn, i, split, n) for i in range(count)]
    pending = {}
    t0 = time.time()
    done = 0

    def flush(N, items):
        idx = [i for i, _ in items]
        x = torch.from_numpy(np.stack([v for _, v in items])).to(dev)
        f = SEL.features(x, Np)
        S = scd.ssca(x, Np)
        lab, rat = SEL.strip_labels(S)
        feats[idx] = f.cpu().numpy()
        labs[idx] = lab.cpu().numpy()
        ratios[idx] = rat.cpu().numpy()
        lens[idx] = N
        del S

    for i, x in enumerate(pool.imap(_gen, jobs, chunksize=4)):
        pending.setdefault(len(x), []).append((i, x))
        if len(pending[len(x)]) == batch:
            flush(len(x), pending.pop(len(x)))
            done += batch
            if done % 1000 < batch:
                log(f"{split}: {done}/{count} signals ({time.time() - t0:.0f} s)")
    for N, items in pending.items():
        flush(N, items)
    log(f"{split}: {count} signals done ({time.time() - t0:.0f} s), active strips {labs.mean():.3f}")
    return feats, labs, ratios, lens


def calibrate(scores, labels, recall=0.99):
    """Largest threshold t with recall(score >= t) >= `recall` over the positive strips."""
    pos = np.sort(scores[labels > 0.5])
    if len(pos) == 0:
        return 0.5
    k = int(np.floor((1.0 - recall) * len(pos)))
    return float(pos[k])


def evaluate(scores, labels, theta, conf_min=None):
    """Recall, fraction of strips computed and fallback rate; a signal falls back to the full SSCA when
    min_k max(s, 1 - s) < conf_min."""
    sel = scores >= theta
    fb = np.zeros(len(scores), bool)
    if conf_min is not None:
        conf = np.min(np.maximum(scores, 1 - scores), axis=1)
        fb = conf < conf_min
        sel[fb] = True
    pos = labels > 0.5
    rec = float((sel & pos).sum() / max(1, pos.sum()))
    return dict(recall=rec, work_fraction=float(sel.mean()), fallback_rate=float(fb.mean()),
                active_fraction=float(pos.mean()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--Np", type=int, required=True)
    ap.add_argument("--N", type=int, default=0, help="fixed signal length (0: 2^U{14..20})")
    ap.add_argument("--train", type=int, default=16000)
    ap.add_argument("--val", type=int, default=2000)
    ap.add_argument("--test", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--conf-min", type=float, default=0.9)
    ap.add_argument("--workers", type=int, default=16)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()

    # The worker pool starts before anything touches the GPU (workers only draw signals with numpy).
    pool = mp.get_context("spawn").Pool(args.workers)
    import torch

    from paper_2506_18003_amd import selector as SEL

    dev = torch.device("cuda:0")
    Np = args.Np
    kind_fn = "cfg4" if args.N else "mixed"
    data = {}
    for split, count in (("train", args.train), ("val", args.val), ("test", args.test)):
        data[split] = build_split(pool, kind_fn, split, count, args.N, Np, dev)
    pool.close()
    pool.join()

    Ftr, Ytr = data["train"][0], data["train"][1]
    mu = Ftr.mean(axis=0)
    sigma = Ftr.std(axis=0) + 1e-3
    std = lambda F: torch.from_numpy(((F - mu) / sigma).astype(np.float32)).to(dev)
    Xtr, Ytr_g = std(Ftr), torch.from_numpy(Ytr).to(dev)
    Xva, Yva = std(data["val"][0]), data["val"][1]
    Xte, Yte = std(data["test"][0]), data["test"][1]

    tr = SEL.Trainer(Np, dev, seed=0, lr=args.lr)
    rng = np.random.default_rng(0)
    n = len(Ftr)
    t0 = time.time()
    for ep in range(args.epochs):
        perm = torch.from_numpy(rng.permutation(n)).to(dev)
        for b0 in range(0, n - args.batch + 1, args.batch):
            idx = perm[b0:b0 + args.batch]
            tr.step(Xtr[idx].contiguous(), Ytr_g[idx].contiguous())
        if ep % 10 == 9 or ep == args.epochs - 1:
            sv = SEL.mlp_forward(tr.params, Xva, Np)[2].cpu().numpy().astype(np.float64)
            eps = 1e-7
            bce = float(-np.mean(Yva * np.log(sv + eps) + (1 - Yva) * np.log(1 - sv + eps)))
            log(f"epoch {ep + 1}: validation BCE {bce:.4f} ({time.time() - t0:.0f} s)")
    np.savez(args.out + ".ckpt.npz", params=tr.params.cpu().numpy(), m=tr.m.cpu().numpy(), v=tr.v.cpu().numpy(),
             t=np.array(tr.t))

    s_va = SEL.mlp_forward(tr.params, Xva, Np)[2].cpu().numpy()
    s_te = SEL.mlp_forward(tr.params, Xte, Np)[2].cpu().numpy()
    theta = calibrate(s_va, Yva)
    learned = evaluate(s_te, Yte, theta, args.conf_min)
    learned_no_fallback = evaluate(s_te, Yte, theta, None)
    # Without the network: threshold the raw ACP feature, calibrated the same way.
    acp_va, acp_te = data["val"][0][:, Np:], data["test"][0][:, Np:]
    tau = calibrate(acp_va, Yva)
    baseline = evaluate(acp_te, Yte, tau, None)
    meta = dict(recipe=dict(kind=kind_fn, N=args.N, train=args.train, val=args.val, test=args.test,
                            epochs=args.epochs, batch=args.batch, lr=args.lr),
                test_learned=learned, test_learned_no_fallback=learned_no_fallback,
                test_acp_threshold=dict(baseline, tau=tau), full_ssca=dict(recall=1.0, work_fraction=1.0))
    sel = SEL.Selector(Np, tr.params, torch.from_numpy(mu).to(dev), torch.from_numpy(sigma).to(dev), theta,
                       args.conf_min, meta)
    sel.save(args.out + ".npz")
    log("model", args.out, json.dumps(dict(theta=theta, **meta)))


if __name__ == "__main__":
    main()
