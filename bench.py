"""Benchmark: SSCA at N = 2^20, Np = 64 on one seeded QPSK signal (the paper's large-window workload).

One step = one full SSCA of the signal: Stage 1 (channelizer + channel-data product + M1-point DFT +
rotation) and Stage 2 (M2-point DFT), exactly the kernels scd_ssca runs, called as the two ABI stages so that
HIP events on the launch stream time each kernel inside the timed region.

Prints one JSON line. `value` is SCD points/s = Np*N / (seconds per step) with x, window and output already
resident in HBM. `roofline` reports the dominant kernel (longest average event-timed duration) against the HBM
roofline: its algorithmic bytes per launch over its average duration, against 8 TB/s; `B_2p_frac` and
`B_min_frac` give the whole step against the two byte models (x + output + one round trip of the intermediate,
and x + output), `alu` the dominant kernel's paper-convention flops against the FP32 vector peak, and
`per_kernel` both kernels both ways. `cpu_baseline` times the FP64 oracle on this host over all 64 strips of the
same signal, on every core of the host's share (a process pool over strips) and on one core; the oracle's
result also gives the error of every GPU form. A `fam` object times the FFT accumulation method on the batch
workload (16 signals of 16384 samples, Np = 256, L = 64, P = 256), a `fam_paper` object on the paper's own
FAM workload (N = 2048, Np = 256, L = 64, P = 32) as ms per estimate and input samples per second, both in
complex and power form. A `cross` object times the cross SCD of the headline signal and its delayed copy, a
`shard` object one GPU's share of the headline SSCA when its strips are split over 2, 4 or 8 GPUs, and a
`stream` object the steady-state time per block of a stream of host blocks (copies included).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--forms fp32,...] [--no-cpu-baseline] [--no-fam]
                       [--no-cross] [--cpu-workers W]
       python bench.py --write-traffic FETCH_CSV WRITE_CSV   (no GPU: summarise two rocprofv3 --pmc runs of
       `bench.py --copy-calib --forms fp32`, one with FETCH_SIZE and one with WRITE_SIZE, into the committed
       per-launch HBM traffic of the SSCA kernels)
       python bench.py --counter-table CSV [CSV ...]   (no GPU: per-kernel averages of rocprofv3 --pmc counter
       CSVs as a markdown table)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SCD pts/s, SSCA N=2^20 N'=64: FP32 vs split-BF16 vs learned strips"
PAPER_PTS_PER_S = 2 ** 26 / 0.114  # VCK5000, 114 ms per SSCA estimate at N=2^20, N_P=64 (Table III)
HBM_PEAK_GBS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak (counts packed FP32 instructions)
# What the library's code can reach: it is built without packed FP32 instructions, so one FMA per lane and
# cycle: 256 CUs x 4 SIMDs x 16 lanes x 2 flop x 2.4 GHz.
VALU_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
KERNEL_SOURCES = ("scd_device.h", "scd_launch.h", "ssca_fp32.hip")  # the FP32 SSCA kernels


def source_digest(files=KERNEL_SOURCES) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2506_18003_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, digest: str, path: str = None):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on this source."""
    path = path or os.path.join(ROOT, "profiles", "traffic_ssca_n2p20_np64.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    k = d.get("kernels", {}).get(kernel)
    if not k or d.get("source_digest") != digest:
        return None
    return k.get("bytes_per_launch")


CALIB_BYTES = 256 << 20          # the --copy-calib kernel reads and writes this many bytes
TRAFFIC_KERNELS = {"ssca_pass1": "ssca_pass1_fp32<64, true, false, false, 0>", "ssca_pass2": "ssca_pass2_fp32"}


TRAFFIC_PATH = os.path.join(ROOT, "profiles", "traffic_ssca_n2p20_np64.json")


def write_traffic(fetch_csv: str, write_csv: str, path: str = TRAFFIC_PATH) -> dict:
    """Per-launch HBM bytes of each SSCA kernel from FETCH_SIZE / WRITE_SIZE counter CSVs (KiB per dispatch),
    each counter scaled by the factor that maps its reading of the calibration kernel to the known size.
    Written to `path` (the committed summary by default) with the current source digest."""
    import csv

    def per_kernel(path):
        acc = {}
        for row in csv.DictReader(open(path)):
            acc.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]) * 1024.0)
        return {k: sum(v) / len(v) for k, v in acc.items()}

    out = {"source_digest": source_digest(), "calibration": {}, "kernels": {}}
    readings = {}
    for counter, csv_path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        pk = per_kernel(csv_path)
        calib = [v for k, v in pk.items() if "MulFunctor" in k]
        if len(calib) != 1:
            raise SystemExit(f"{csv_path}: expected one calibration kernel reading")
        factor = CALIB_BYTES / calib[0]
        out["calibration"][counter] = {"raw_bytes": calib[0], "known_bytes": CALIB_BYTES, "factor": factor}
        for name, pat in TRAFFIC_KERNELS.items():
            hits = [v for k, v in pk.items() if pat in k]
            if len(hits) != 1:
                raise SystemExit(f"{csv_path}: expected one {pat} kernel, found {len(hits)}")
            readings.setdefault(name, {})[counter] = hits[0] * factor
    for name, r in readings.items():
        out["kernels"][name] = {"fetch_bytes": round(r["FETCH_SIZE"]), "write_bytes": round(r["WRITE_SIZE"]),
                                "bytes_per_launch": round(r["FETCH_SIZE"] + r["WRITE_SIZE"])}
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out))
    return out


def counter_table(paths) -> str:
    """Markdown table of per-kernel average counter values (one row per kernel and counter) from rocprofv3
    --pmc CSVs."""
    import csv

    acc = {}
    for path in paths:
        for row in csv.DictReader(open(path)):
            acc.setdefault(row["Kernel_Name"], {}).setdefault(row["Counter_Name"], []).append(
                float(row["Counter_Value"]))
    lines = ["| kernel | counter | dispatches | average per dispatch |", "|---|---|---|---|"]
    for k in sorted(acc):
        short = k.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0].replace("scd::", "")
        for c in sorted(acc[k]):
            v = acc[k][c]
            lines.append(f"| {short} | {c} | {len(v)} | {sum(v) / len(v):.6g} |")
    return "\n".join(lines)


def shard_strips(Np: int, G: int, r: int) -> list:
    """Strips GPU r of G owns when the SSCA is split by strips: whole channel subsets (k = c mod Np/16) while
    G <= Np/16, so that no Stage 1 work is repeated; beyond that, half (or smaller) runs of one subset."""
    S = Np // 16
    if G <= S:
        return [k for k in range(Np) if (k % S) % G == r]
    per = Np // G
    ks = [k for k in range(Np) if k % S == r % S]
    h = r // S
    return ks[h * per:(h + 1) * per]


def _oracle_strips(args):
    """Pool worker: FP64 oracle strips ks of the signal (the product path never calls this)."""
    x, Np, w, ks = args
    from oracle import scd_oracle as O

    return ks, [O.ssca_strip(x, Np, w, k) for k in ks]


def cpu_oracle_ssca(x, Np, w, workers):
    """All Np strips of the FP64 oracle SSCA: in this process (workers == 1) or on a process pool over strips.
    Returns (S, seconds)."""
    import numpy as np

    t0 = time.perf_counter()
    if workers == 1:
        from oracle import scd_oracle as O

        S = np.stack([O.ssca_strip(x, Np, w, k) for k in range(Np)])
        return S, time.perf_counter() - t0
    import multiprocessing as mp

    chunks = [list(range(i, Np, workers)) for i in range(workers)]
    S = np.empty((Np, len(x)), np.complex128)
    # Spawned workers start a fresh interpreter: they never inherit this process's GPU context.
    with mp.get_context("spawn").Pool(workers) as pool:
        for ks, rows in pool.imap_unordered(_oracle_strips, [(x, Np, w, ks) for ks in chunks]):
            for k, r in zip(ks, rows):
                S[k] = r
    return S, time.perf_counter() - t0


def main():
    if len(sys.argv) == 4 and sys.argv[1] == "--write-traffic":
        write_traffic(sys.argv[2], sys.argv[3])
        return
    if len(sys.argv) >= 3 and sys.argv[1] == "--counter-table":
        print(counter_table(sys.argv[2:]))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--forms", default="fp32,split_bf16,split_fp16,bf16,learned")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fam", action="store_true", help="skip the FAM batch measurement")
    ap.add_argument("--no-cross", action="store_true", help="skip the cross-SCD and streaming measurements")
    ap.add_argument("--mix-signals", type=int, default=8,
                    help="held-out selector-recipe signals for the learned form's mixed-workload line (0: skip)")
    ap.add_argument("--combined-signals", type=int, default=64,
                    help="signals of the combined ragged workload (lengths 2^14..2^20, Np 64/128; 0: skip)")
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="processes for the oracle's all-core leg (0: min(16, os.cpu_count()), the host share of one GPU)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run one 256 MiB read + 256 MiB write elementwise kernel (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the SSCA strips would shard over GPUs by channel (scd_ssca_strips "
              "computes one GPU's share, and the `shard` line times it), but this build runs and reports a single "
              "MI355X (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2506_18003_amd as scd
    from synth import workloads as W

    dev = torch.device("cuda:0")
    c = W.cfg3()
    N, Np = c["ssca"]["N"], c["ssca"]["Np"]
    x64 = c["x"].astype(np.complex64)
    w32 = c["ssca"]["win"].astype(np.float32)
    x = torch.from_numpy(x64).to(dev)
    win = torch.from_numpy(w32).to(dev)
    inter = torch.empty(Np * N, dtype=torch.complex64, device=dev)
    out = torch.empty(Np, N, dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream(dev)

    if args.copy_calib:
        # A plain streaming kernel of known traffic (256 MiB read, 256 MiB written) to scale HBM byte counters.
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    if "learned" in forms and "fp32" not in forms:
        forms.insert(0, "fp32")  # the learned form is reported as a speedup over the plain FP32 path
    results = {}
    learned_info = None
    if "learned" in forms:
        from paper_2506_18003_amd import selector as SEL

        forms.remove("learned")
        model = os.path.join(ROOT, "paper_2506_18003_amd", "models", f"selector_np{Np}.scdm")
        with torch.cuda.device(dev):
            sel = SEL.Model.load(model)  # library-owned model loaded through the C ABI
        lout = torch.zeros(Np, N, dtype=torch.complex64, device=dev)
        for _ in range(args.warmup):
            SEL.ssca_learned(x, sel, win=win, out=lout)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, mask, _ = SEL.ssca_learned(x, sel, win=win, out=lout, want_fallback=False)
        torch.cuda.synchronize()
        lms = (time.perf_counter() - t0) * 1e3 / args.steps
        _, mask, fb = SEL.ssca_learned(x, sel, win=win, out=lout)
        m = mask.cpu().numpy().astype(bool)
        full = scd.ssca(x, Np, win=win)
        labels = SEL.strip_labels(full)[0].cpu().numpy()[0] > 0.5
        recall = float((m & labels).sum() / max(1, labels.sum()))
        learned_info = dict(ms_per_step=lms, strips=int(m.sum()), fell_back=bool(fb), recall_vs_full=recall,
                            active_strips=int(labels.sum()), out=lout.cpu().numpy(), mask=m)
        del full
        # The same comparison over held-out signals of the selector's own recipe (test-split seeds, every
        # modulation and noise, SNR in [-10, 15] dB) at N = 2^20: what the selection buys when not every strip
        # carries a cyclic feature.
        mix_full, mix_learned, mix_strips, mix_tp, mix_pos, mix_fb = [], [], 0, 0, 0, 0
        # The selector without its network: a threshold on the raw ACP feature, calibrated on the selector's
        # validation split for the same strip recall (tau, stored with the model's training metrics).
        with open(os.path.join(ROOT, "paper_2506_18003_amd", "models", f"selector_np{Np}.json")) as fh:
            meta = json.load(fh)["meta"]
        tau = meta["test_acp_threshold"]["tau"]
        acp_strips, acp_tp = 0, 0
        for i in range(args.mix_signals):
            xm = torch.from_numpy(W.selector_signal(i, "test", emin=20, emax=20)[1].astype(np.complex64)).to(dev)
            for _ in range(2):
                scd.ssca_stage1(xm, Np, inter, win=win)
                scd.ssca_stage2(inter, N, Np, out)
                SEL.ssca_learned(xm, sel, win=win, out=lout, want_fallback=False)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record(stream)
            for _ in range(5):
                scd.ssca_stage1(xm, Np, inter, win=win)
                scd.ssca_stage2(inter, N, Np, out)
            e[1].record(stream)
            for _ in range(5):
                SEL.ssca_learned(xm, sel, win=win, out=lout, want_fallback=False)
            e[2].record(stream)
            torch.cuda.synchronize()
            mix_full.append(e[0].elapsed_time(e[1]) / 5)
            mix_learned.append(e[1].elapsed_time(e[2]) / 5)
            _, mm, fbm = SEL.ssca_learned(xm, sel, win=win, out=lout)
            mm = mm.cpu().numpy().astype(bool)
            lab = SEL.strip_labels(out)[0].cpu().numpy()[0] > 0.5
            mix_strips += int(mm.sum())
            mix_tp += int((mm & lab).sum())
            mix_pos += int(lab.sum())
            mix_fb += int(bool(fbm))
            ma = SEL.features(xm, Np)[0, Np:].cpu().numpy() >= tau
            acp_strips += int(ma.sum())
            acp_tp += int((ma & lab).sum())
        if args.mix_signals:
            learned_info["mix"] = dict(
                signals=args.mix_signals, full_ms=float(np.mean(mix_full)), learned_ms=float(np.mean(mix_learned)),
                speedup_vs_fp32=float(np.mean(mix_full) / np.mean(mix_learned)),
                strip_fraction=mix_strips / (args.mix_signals * Np), recall=mix_tp / max(1, mix_pos),
                active_fraction=mix_pos / (args.mix_signals * Np), fallbacks=mix_fb,
                acp_threshold_strip_fraction=acp_strips / (args.mix_signals * Np),
                acp_threshold_recall=acp_tp / max(1, mix_pos))
        # The same comparison on the selector's own 2000-signal test split (from its training run).
        learned_info["vs_acp_threshold"] = {
            "split": f"test split of the selector recipe ({meta['recipe']['test']} signals, N = 2^U{{14..20}})",
            "learned": meta["test_learned"], "learned_no_fallback": meta["test_learned_no_fallback"],
            "acp_threshold": meta["test_acp_threshold"],
            "network_strip_saving_vs_acp": round(meta["test_acp_threshold"]["work_fraction"]
                                                 - meta["test_learned_no_fallback"]["work_fraction"], 5)}
    for form in forms:
        for _ in range(args.warmup):
            scd.ssca_stage1(x, Np, inter, win=win, precision=form)
            scd.ssca_stage2(inter, N, Np, out)
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(args.steps):
            ev[i][0].record(stream)
            scd.ssca_stage1(x, Np, inter, win=win, precision=form)
            ev[i][1].record(stream)
            scd.ssca_stage2(inter, N, Np, out)
            ev[i][2].record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p1 = sorted(e[0].elapsed_time(e[1]) for e in ev)
        p2 = sorted(e[1].elapsed_time(e[2]) for e in ev)
        tot = sorted(e[0].elapsed_time(e[2]) for e in ev)
        ms = (t1 - t0) * 1e3 / args.steps
        results[form] = dict(ms_per_step=ms, pass1_ms=float(np.mean(p1)), pass2_ms=float(np.mean(p2)),
                             step_ms_p10=tot[len(tot) // 10], step_ms_p50=tot[len(tot) // 2],
                             step_ms_p90=tot[(9 * len(tot)) // 10], out=out.cpu().numpy())

    # The combined workload: a ragged batch of signals of lengths 2^U{14..20} with Np = 64 (even index) or 128
    # (odd), one scd_ssca_batch call each way. Plain FP32 against split-BF16 + learned strips + fallback; the
    # recall is scored against the labels of the FP32 outputs.
    combined_info = None
    if args.combined_signals and "fp32" in forms and "split_bf16" in forms:
        from paper_2506_18003_amd import selector as SEL2

        models = {}
        with torch.cuda.device(dev):
            for n in (64, 128):
                models[n] = SEL2.Model.load(os.path.join(ROOT, "paper_2506_18003_amd", "models", f"selector_np{n}.scdm"))
        sigs = [W.cfg5_signal(i) for i in range(args.combined_signals)]
        xs = [torch.from_numpy(c["x"].astype(np.complex64)).to(dev) for c in sigs]
        wins = {n: torch.from_numpy(np.asarray(W.sg.hamming(n), np.float32)).to(dev) for n in (64, 128)}
        outs_f = [torch.empty(c["Np"], c["N"], dtype=torch.complex64, device=dev) for c in sigs]
        outs_l = [torch.zeros(c["Np"], c["N"], dtype=torch.complex64, device=dev) for c in sigs]
        items_f = [dict(x=x, Np=c["Np"], win=wins[c["Np"]], out=o) for x, c, o in zip(xs, sigs, outs_f)]
        items_l = [dict(x=x, Np=c["Np"], win=wins[c["Np"]], out=o, selector=models[c["Np"]])
                   for x, c, o in zip(xs, sigs, outs_l)]
        tf, tl, tl32 = [], [], []
        masks = None
        for rep in range(1 + 3):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
            e[0].record(stream)
            scd.ssca_batch(items_f)
            e[1].record(stream)
            res = scd.ssca_batch(items_l, precision="split_bf16")
            e[2].record(stream)
            scd.ssca_batch(items_l)
            e[3].record(stream)
            torch.cuda.synchronize()
            if rep:
                tf.append(e[0].elapsed_time(e[1]))
                tl.append(e[1].elapsed_time(e[2]))
                tl32.append(e[2].elapsed_time(e[3]))
            masks = [m for _, m in res]
        pts = float(sum(c["Np"] * c["N"] for c in sigs))
        strips = sum(int(m.sum().item()) for m in masks)
        nstrips = sum(c["Np"] for c in sigs)
        tp = pos = 0
        for o, m in zip(outs_f, masks):
            lab = SEL2.strip_labels(o)[0].cpu().numpy()[0] > 0.5
            mm = m.cpu().numpy().astype(bool)
            tp += int((mm & lab).sum())
            pos += int(lab.sum())
        fms, lms, l32 = float(np.median(tf)), float(np.median(tl)), float(np.median(tl32))
        combined_info = {
            "workload": f"{len(sigs)} signals of lengths 2^U{{14..20}} (cfg-5 recipe), Np 64 (even) / 128 (odd), "
                        "one scd_ssca_batch call", "scd_pts": pts,
            "fp32": {"ms_per_batch": round(fms, 4), "pts_per_s": round(pts / (fms * 1e-3), 1)},
            "split_bf16_learned": {"ms_per_batch": round(lms, 4), "pts_per_s": round(pts / (lms * 1e-3), 1),
                                   "speedup_vs_fp32": round(fms / lms, 3), "strip_fraction": round(strips / nstrips, 4),
                                   "recall_vs_fp32_labels": round(tp / max(1, pos), 5),
                                   "active_fraction": round(pos / nstrips, 4)},
            "fp32_learned": {"ms_per_batch": round(l32, 4), "pts_per_s": round(pts / (l32 * 1e-3), 1),
                             "speedup_vs_fp32": round(fms / l32, 3)}}
        for mdl in models.values():
            mdl.close()
        del outs_f, outs_l, items_f, items_l, xs

    # Split-BF16 against FP32 at Np = 128 on the same signal, where the channelizer GEMM has twice the taps
    # (interleaved trials, medians of per-step HIP event times).
    np128_info = None
    if "fp32" in forms and "split_bf16" in forms:
        Np2 = 128
        w2 = torch.from_numpy(np.hamming(Np2).astype(np.float32)).to(dev)
        inter2 = torch.empty(Np2 * N, dtype=torch.complex64, device=dev)
        out2 = torch.empty(Np2, N, dtype=torch.complex64, device=dev)
        ev2 = {f: [] for f in ("fp32", "split_bf16")}
        for rep in range(args.warmup + args.steps):
            for form in ev2:
                e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
                e[0].record(stream)
                scd.ssca_stage1(x, Np2, inter2, win=w2, precision=form)
                e[1].record(stream)
                scd.ssca_stage2(inter2, N, Np2, out2)
                e[2].record(stream)
                if rep >= args.warmup:
                    ev2[form].append(e)
        torch.cuda.synchronize()
        med = lambda v: float(np.median(v))
        t2 = {f: dict(ms_per_step=round(med([e[0].elapsed_time(e[2]) for e in v]), 5),
                      pass1_ms=round(med([e[0].elapsed_time(e[1]) for e in v]), 5)) for f, v in ev2.items()}
        np128_info = {"workload": "the headline signal at Np = 128 (N = 2^20), Hamming window", **t2,
                      "speedup_split_bf16_vs_fp32": round(t2["fp32"]["ms_per_step"] / t2["split_bf16"]["ms_per_step"], 3)}
        del inter2, out2

    # The cross SCD of x and its delayed copy y(n) = x(n + 5) (Eq. (2)'s two-input form with the paper's
    # time-delay example), one scd_ssca_cross_ex call per step on the same workload.
    cross_info = None
    if "fp32" in forms and not args.no_cross:
        yd = torch.zeros_like(x)
        yd[:-5] = x[5:]
        for _ in range(args.warmup):
            scd.ssca_cross(x, yd, Np, win=win, out=out)
        cev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        for i in range(args.steps):
            cev[i][0].record(stream)
            scd.ssca_cross(x, yd, Np, win=win, out=out)
            cev[i][1].record(stream)
        torch.cuda.synchronize()
        cms = float(np.mean([e[0].elapsed_time(e[1]) for e in cev]))
        cross_info = {"workload": "cross SCD of the headline signal x and y(n) = x(n + 5), N=2^20, Np=64",
                      "ms_per_step": round(cms, 5), "pts_per_s": round(Np * N / (cms * 1e-3), 1),
                      "speedup_vs_fp32_auto": round(results["fp32"]["ms_per_step"] / cms, 3)}
        del yd

    # One GPU's share of the headline estimate when its strips are split over G GPUs: scd_ssca_strips with the
    # strips GPU 0 would own. The broadcast of x to the other GPUs and any gather of the output are not in it.
    shard_info = None
    if "fp32" in forms and not args.no_cross:
        shard_info = {"workload": "GPU 0's strips of the headline SSCA split over G GPUs (whole channel subsets "
                                  "while G <= Np/16, half subsets beyond), scd_ssca_strips; x broadcast and output "
                                  "gather not included"}
        for G in (2, 4, 8):
            ks = shard_strips(Np, G, 0)
            for _ in range(args.warmup):
                scd.ssca_strips(x, Np, ks, win=win, out=out)
            sev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
            torch.cuda.synchronize()
            for i in range(args.steps):
                sev[i][0].record(stream)
                scd.ssca_strips(x, Np, ks, win=win, out=out)
                sev[i][1].record(stream)
            torch.cuda.synchronize()
            sms = float(np.median([e[0].elapsed_time(e[1]) for e in sev]))
            shard_info[f"G{G}"] = {"strips": len(ks), "ms": round(sms, 5),
                                   "pts_per_s": round(len(ks) * N / (sms * 1e-3), 1),
                                   "ms_vs_full_over_G": round(sms / (results["fp32"]["ms_per_step"] / G), 3)}

    # Streaming: a continuous stream of 2^20-sample blocks pushed from pinned host memory through SscaReceiver
    # (a fixed ring of 4 device slots and 2 reused output buffers; copy and estimate overlapped on two streams).
    # The initiation interval includes the host-to-device copies (PCIe), so it is reported beside `value`, never
    # as it; the host's own time inside push() and the plain copy time are given apart.
    stream_info = None
    if "fp32" in forms and not args.no_cross:
        nblk = 8     # distinct pinned host blocks, pushed round robin
        npush = 32   # blocks per timed pass (the receiver's device memory does not grow with it)
        hx = torch.from_numpy(np.tile(x64, nblk))
        blocks = []
        for b in range(nblk):
            t = torch.empty(N, dtype=torch.complex64, pin_memory=True)
            t.copy_(hx[b * N:(b + 1) * N])
            blocks.append(t)
        for rep in range(2):  # the first pass warms up
            rx = scd.SscaReceiver(N, Np, dev, win=win)
            torch.cuda.synchronize()
            host = 0.0
            t0 = time.perf_counter()
            for i in range(npush):
                h0 = time.perf_counter()
                rx.push(blocks[i % nblk])
                host += time.perf_counter() - h0
            rx.finish()
            torch.cuda.synchronize()
            sms = (time.perf_counter() - t0) * 1e3 / npush
            ring_bytes = rx.ring_bytes + sum(o.numel() * 8 for o in rx.out)
            del rx
        # push's own host cost: a ring of 64 slots never waits for a free slot over 32 pushes.
        rx = scd.SscaReceiver(N, Np, dev, win=win, slots=64)
        torch.cuda.synchronize()
        enq = 0.0
        for i in range(npush):
            h0 = time.perf_counter()
            rx.push(blocks[i % nblk])
            enq += time.perf_counter() - h0
        rx.finish()
        torch.cuda.synchronize()
        del rx
        dbuf = torch.empty(N, dtype=torch.complex64, device=dev)
        ce = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ce[0].record(stream)
        for i in range(nblk):
            dbuf.copy_(blocks[i], non_blocking=True)
        ce[1].record(stream)
        torch.cuda.synchronize()
        copy_ms = ce[0].elapsed_time(ce[1]) / nblk
        stream_info = {"workload": f"{npush} blocks of N=2^20 from pinned host memory, Np={Np}, neighbouring samples "
                                   "at block edges (host-to-device copies included)",
                       "ms_per_block": round(sms, 5), "pts_per_s": round(Np * N / (sms * 1e-3), 1),
                       "host_push_ms_per_block": round(host * 1e3 / npush, 5),
                       "host_push_note": "host time inside push, including the wait for a free ring slot (the "
                                         "estimate 3 blocks back); host_enqueue is push's own cost, measured with a "
                                         "64-slot ring that never waits",
                       "host_enqueue_ms_per_block": round(enq * 1e3 / npush, 5),
                       "h2d_copy_ms_per_block": round(copy_ms, 5),
                       "device_bytes": ring_bytes}
        del blocks, hx, dbuf

    # Algorithmic HBM bytes and flops per launch (one signal). Pass 1 reads x and writes the intermediate;
    # pass 2 reads and writes Np*N complex values. Flops follow the paper's convention (5 n log2 n per n-point
    # FFT, 6 per complex multiply, 2 per real window tap): pass 1 = the Np-point channelizer FFT of every frame,
    # the window, the down-conversion, the channel-data product, the M1-point FFTs and the rotation; pass 2 =
    # the M2-point FFTs.
    lg = lambda v: v.bit_length() - 1
    M1, M2 = 1024, N // 1024
    b1 = 8 * N + 8 * Np * N
    b2 = 2 * 8 * Np * N
    f1 = N * 5 * Np * lg(Np) + 2 * Np * N + 3 * 6 * Np * N + Np * M2 * 5 * M1 * lg(M1)
    f2 = Np * M1 * 5 * M2 * lg(M2)
    main_form = forms[0]
    r = results[main_form]
    digest = source_digest()
    kern = {"ssca_pass1": (b1, f1, r["pass1_ms"]), "ssca_pass2": (b2, f2, r["pass2_ms"])}

    def kernel_roof(name):
        """The kernel's algorithmic HBM bytes over its average duration against the 8 TB/s peak, and its
        paper-convention flops against the FP32 vector peaks (secondary)."""
        nb, nf, ms = kern[name]
        gbs = nb / (ms * 1e-3) / 1e9
        tfs = nf / (ms * 1e-3) / 1e12
        return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(gbs / HBM_PEAK_GBS, 4), "avg_ms": round(ms, 5), "algorithmic_bytes": nb,
                "alu": {"achieved": round(tfs, 2), "unit": "TFLOP/s", "algorithmic_flops": nf,
                        "peak": FP32_VECTOR_PEAK_TFLOPS, "frac": round(tfs / FP32_VECTOR_PEAK_TFLOPS, 4),
                        "peak_without_packed_fp32": VALU_PEAK_TFLOPS,
                        "frac_without_packed_fp32": round(tfs / VALU_PEAK_TFLOPS, 4)}}

    # This GPU's own device-to-device copy rate (torch's copy of 512 MiB, read + write), beside the datasheet peak.
    csrc = torch.empty(64 << 20, dtype=torch.complex64, device=dev)
    cdst = torch.empty_like(csrc)
    cdst.copy_(csrc)
    ce = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ce[0].record(stream)
    for _ in range(10):
        cdst.copy_(csrc)
    ce[1].record(stream)
    torch.cuda.synchronize()
    copy_gbs = 2 * csrc.numel() * 8 * 10 / (ce[0].elapsed_time(ce[1]) * 1e-3) / 1e9
    del csrc, cdst

    dom = max(kern, key=lambda k: kern[k][2])
    roof = dict(kernel_roof(dom), kernel=dom, traffic=measured_traffic(dom, digest))
    if roof["traffic"] is not None:
        # the HBM bytes the kernel really moves (its counters, scaled per launch) at this run's duration
        tgbs = roof["traffic"] / (kern[dom][2] * 1e-3) / 1e9
        roof.update({"traffic_GBs": round(tgbs, 1), "traffic_frac_of_peak": round(tgbs / HBM_PEAK_GBS, 4),
                     "traffic_frac_of_measured_copy": round(tgbs / copy_gbs, 4)})
    roof.update({
            "B_2p_frac": round((8 * N + 3 * 8 * Np * N) / (r["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "B_min_frac": round((8 * N + 8 * Np * N) / (r["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "per_kernel": {k: kernel_roof(k) for k in kern},
            "measured_copy_GBs": round(copy_gbs, 1),
            "B_2p_frac_of_measured_copy": round((8 * N + 3 * 8 * Np * N) / (r["ms_per_step"] * 1e-3) / 1e9 / copy_gbs, 4),
            "source_digest": digest})

    fam_line = None
    if not args.no_fam:
        # FAM on the batch workload: 16 signals of 16384 samples, Np = 256, L = 64, P = 256 (one scd_fam call:
        # channelizer + pair/P-point-DFT kernels). Algorithmic bytes: x, X_T written and read, S written.
        cf = W.cfg2()
        fp = cf["fam"]
        fNp, fL, fP = fp["Np"], fp["L"], fp["P"]
        fB = cf["x"].shape[0]
        fx = torch.from_numpy(cf["x"][:, :fP * fL].astype(np.complex64)).to(dev)
        fw = torch.from_numpy(fp["win"].astype(np.float32)).to(dev)
        fout = torch.empty(fB, fNp, fNp, fP, dtype=torch.complex64, device=dev)
        for _ in range(args.warmup):
            scd.fam(fx, fNp, fL, fP, win=fw, out=fout)
        fev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(args.steps)]
        torch.cuda.synchronize()
        for i in range(args.steps):
            fev[i][0].record(stream)
            scd.fam(fx, fNp, fL, fP, win=fw, out=fout)
            fev[i][1].record(stream)
        torch.cuda.synchronize()
        fms = float(np.mean([e[0].elapsed_time(e[1]) for e in fev]))
        fbytes = 8 * fB * fP * fL + 2 * 8 * fB * fNp * fP + 8 * fB * fNp * fNp * fP
        fam_line = {"workload": f"FAM Np={fNp} L={fL} P={fP}, {fB} signals of {fP * fL} samples (batch recipe)",
                    "ms_per_batch": round(fms, 5), "pts_per_s": round(fB * fNp * fNp * fP / (fms * 1e-3), 1),
                    "roofline": {"bound": "hbm", "achieved": round(fbytes / (fms * 1e-3) / 1e9, 1),
                                 "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                 "frac": round(fbytes / (fms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                                 "algorithmic_bytes": fbytes}}
        if not args.no_cpu_baseline:
            from oracle import scd_oracle as O

            ref = O.fam(cf["x"][0, :fP * fL].astype(np.complex64).astype(np.complex128), fNp, fL, fP,
                        fp["win"].astype(np.float32).astype(np.float64))
            fam_line["max_err_vs_oracle_signal0"] = float(np.abs(fout[0].cpu().numpy() - ref).max() / np.abs(ref).max())
        del fout
        # The paper's output form (|S|^2 over -P/4 <= q_c < P/4, scd_fam_power_ex): same kernels, a quarter of the
        # output bytes.
        pout = torch.empty(fB, fNp, fNp, fP // 2, dtype=torch.float32, device=dev)
        for _ in range(args.warmup):
            scd.fam_power(fx, fNp, fL, fP, win=fw, out=pout)
        torch.cuda.synchronize()
        for i in range(args.steps):
            fev[i][0].record(stream)
            scd.fam_power(fx, fNp, fL, fP, win=fw, out=pout)
            fev[i][1].record(stream)
        torch.cuda.synchronize()
        pms = float(np.mean([e[0].elapsed_time(e[1]) for e in fev]))
        pbytes = 8 * fB * fP * fL + 2 * 8 * fB * fNp * fP + 4 * fB * fNp * fNp * (fP // 2)
        fam_line["power_form"] = {"ms_per_batch": round(pms, 5),
                                  "pts_per_s": round(fB * fNp * fNp * (fP // 2) / (pms * 1e-3), 1),
                                  "speedup_vs_complex": round(fms / pms, 3),
                                  "achieved_GBs": round(pbytes / (pms * 1e-3) / 1e9, 1),
                                  "algorithmic_bytes": pbytes}
        del pout

    # The paper's own FAM workload (Sec. III-A worked sizes): N = 2048 samples, Np = 256, L = 64, P = 32, on the
    # paper's DSSS BPSK test signal (SNR 10 dB, processing gain 31, chip rate 0.25) with a 100 dB Chebyshev
    # window. One estimate at a time and a batch of estimates, each as the complex grid (scd_fam) and as the
    # paper's kept |S|^2 bins (scd_fam_power); ms per estimate and input samples per second.
    fam_paper = None
    if not args.no_fam:
        from scipy.signal.windows import chebwin

        from synth import signals as SG

        pNp, pL, pP = 256, 64, 32
        pN = pL * pP
        nb = 256
        xs = np.stack([SG.dsss_bpsk(pN, 10.0, SG.rng_for(8, i)) for i in range(nb)]).astype(np.complex64)
        px = torch.from_numpy(xs).to(dev)
        pw = torch.from_numpy(chebwin(pNp, at=100).astype(np.float32)).to(dev)
        fam_paper = {"workload": f"FAM N={pN} Np={pNp} L={pL} P={pP} (DSSS BPSK, 10 dB, Chebyshev window)"}
        for form, fn, shape, dt in (("complex", scd.fam, (pNp, pNp, pP), torch.complex64),
                                    ("power", scd.fam_power, (pNp, pNp, pP // 2), torch.float32)):
            o1 = torch.empty(*shape, dtype=dt, device=dev)
            ob = torch.empty(nb, *shape, dtype=dt, device=dev)
            for _ in range(args.warmup):
                fn(px[0], pNp, pL, pP, win=pw, out=o1)
                fn(px, pNp, pL, pP, win=pw, out=ob)
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            reps = max(10, args.steps)
            torch.cuda.synchronize()
            e[0].record(stream)
            for i in range(reps):
                fn(px[i % nb], pNp, pL, pP, win=pw, out=o1)
            e[1].record(stream)
            fn(px, pNp, pL, pP, win=pw, out=ob)
            e[2].record(stream)
            torch.cuda.synchronize()
            one = e[0].elapsed_time(e[1]) / reps
            bat = e[1].elapsed_time(e[2])
            outb = ob.numel() * ob.element_size() // nb
            bytes_per = 8 * pN + 2 * 8 * pNp * pP + outb
            fam_paper[form] = {
                "ms_per_estimate": round(one, 5), "input_MS_per_s": round(pN / (one * 1e-3) / 1e6, 1),
                "batch": nb, "batch_ms": round(bat, 5), "batch_ms_per_estimate": round(bat / nb, 6),
                "batch_input_MS_per_s": round(nb * pN / (bat * 1e-3) / 1e6, 1),
                "batch_hbm_GBs": round(nb * bytes_per / (bat * 1e-3) / 1e9, 1),
                "batch_hbm_frac": round(nb * bytes_per / (bat * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            del o1, ob
        fam_paper["paper_context"] = "VCK5000 0.630 ms per estimate, 3.25 MS/s (Table II/III; other hardware)"
        del px

    cpu = None
    errs = {}
    if not args.no_cpu_baseline:
        # The FP64 oracle (per-strip FIR channelizer + numpy.fft) over all 64 strips of the same signal: once on
        # a process pool over strips using the host's share of cores, once on a single core.
        ncpu = os.cpu_count() or 1
        workers = args.cpu_workers or max(1, min(16, ncpu))
        xf = x64.astype(np.complex128)
        wf = w32.astype(np.float64)
        ref, dt_all = cpu_oracle_ssca(xf, Np, wf, workers)
        _, dt_one = cpu_oracle_ssca(xf, Np, wf, 1)
        cpu = {"value": round(Np * N / dt_all, 1), "unit": "SCD pts/s", "cores": workers, "kind": "oracle",
               "sample": f"all {Np} strips of the same N=2^20 signal (FP64 numpy oracle: per-strip FIR channelizer "
                         f"+ numpy.fft) on a pool of {workers} processes over strips, {dt_all:.2f} s",
               "os_cpu_count": ncpu, "workers": workers, "seconds": round(dt_all, 3),
               "single_core": {"value": round(Np * N / dt_one, 1), "cores": 1, "seconds": round(dt_one, 3)}}
        peak = np.abs(ref).max()
        for form, rr in results.items():
            errs[form] = float(np.abs(rr["out"] - ref).max() / peak)

        if learned_info is not None:
            m = learned_info["mask"]
            errs["learned"] = (float(np.abs(learned_info["out"][m] - ref[m]).max() / np.abs(ref[m]).max())
                               if m.any() else None)

    value = Np * N / (r["ms_per_step"] * 1e-3)
    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "SCD pts/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(r["ms_per_step"], 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": round(value / PAPER_PTS_PER_S, 2),
        "vs_baseline_note": "paper's VCK5000 SSCA, 114 ms per estimate at this workload (other hardware)",
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "SSCA N=2^20 Np=64, one QPSK signal (complex carrier 0.1, 8 samples/symbol, "
                               "5 dB AWGN), Hamming window", "N": N, "Np": Np, "form": main_form},
        "roofline": roof, "cpu_baseline": cpu,
        "forms": {f: {"pts_per_s": round(Np * N / (rr["ms_per_step"] * 1e-3), 1),
                      "ms_per_step": round(rr["ms_per_step"], 5), "p10_ms": round(rr["step_ms_p10"], 5),
                      "p50_ms": round(rr["step_ms_p50"], 5), "p90_ms": round(rr["step_ms_p90"], 5),
                      "pass1_ms": round(rr["pass1_ms"], 5), "pass2_ms": round(rr["pass2_ms"], 5),
                      "speedup_vs_fp32": (round(results["fp32"]["ms_per_step"] / rr["ms_per_step"], 3)
                                          if "fp32" in results else None),
                      "max_err_vs_oracle": errs.get(f)} for f, rr in results.items()},
    }
    if fam_line is not None:
        line["fam"] = fam_line
    if fam_paper is not None:
        line["fam_paper"] = fam_paper
    if learned_info is not None:
        li = learned_info
        line["forms"]["learned"] = {
            "pts_per_s": round(Np * N / (li["ms_per_step"] * 1e-3), 1), "ms_per_step": round(li["ms_per_step"], 5),
            "speedup_vs_fp32": round(r["ms_per_step"] / li["ms_per_step"], 3), "strips_computed": li["strips"],
            "selected_pts_per_s": round(li["strips"] * N / (li["ms_per_step"] * 1e-3), 1),
            "fell_back": li["fell_back"], "active_strips": li["active_strips"],
            "recall_vs_full": li["recall_vs_full"], "max_err_vs_oracle": errs.get("learned"),
            "note": "whole scd_ssca_learned call: features, MLP + selection kernels, selected strips (asynchronous)"}
        if "vs_acp_threshold" in li:
            line["forms"]["learned"]["vs_acp_threshold"] = li["vs_acp_threshold"]
        if "mix" in li:
            line["forms"]["learned"]["mix"] = dict(
                workload=f"{li['mix']['signals']} held-out signals of the selector recipe at N=2^20, Np={Np}",
                **{k: (round(v, 4) if isinstance(v, float) else v) for k, v in li["mix"].items()})
    if np128_info is not None:
        line["split_bf16_np128"] = np128_info
    if combined_info is not None:
        line["combined"] = combined_info
    if cross_info is not None:
        line["cross"] = cross_info
    if shard_info is not None:
        line["shard"] = shard_info
    if stream_info is not None:
        line["stream"] = stream_info
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
