#!/usr/bin/env python3
"""Benchmark: decoded samples/s and site-updates/s of the message-passing
decoder on the L=256, p=0.01 toric-code workload (4096 samples per batch,
T_max = 4096, v = 3), one MI355X.

A step is one complete pass of the hot path over one batch: in-kernel noise
from the seeds, syndrome, decoder steps until no anyon is left, correction
winding and classification, final syndrome export.  Each step uses a fresh
batch of seeds (same distribution); the seeds are already in HBM when the
timed region starts.

The headline value is plain (FIFO) batching.  The learned-scheduling leg
trains the decode-time predictor on the GPU (200000 decoder-labelled L = 256
samples, p ~ U[0.005, 0.02]), picks its binning policy by timing on a
separate batch, then times the same K batches with inference and binning
inside the timed region, and checks that the results are identical.

Prints one JSON line on stdout.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

L, P, N_SAMPLES, T_MAX = 256, 0.01, 4096, 4096
BYTES_PER_SITE_UPDATE = 16.25   # 4 x int16 registers + 1 syndrome bit, read and written once per step
HBM_PEAK_GBS = 8000.0
# VALU issue of 32-bit integer / bitwise operations: 256 CUs x 4 SIMDs x 16
# lanes per clock x 2.4 GHz (a wave64 instruction every 4 clocks per SIMD)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
METRIC = "decoded samples/s & site-updates/s at L=256, p=0.01 (plain vs learned-sched)"
PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "k_bits_L256_p001.json")
CSRC = os.path.join(ROOT, "paper_2506_03266_amd", "csrc")


def kernel_source_sha():
    """sha256[:16] of the bit-sliced kernel's device code: engine.h, band.h
    (lane shifts) and bits.h, without // comments, trailing blanks and empty
    lines (so that editing a comment keeps a profile valid)."""
    import hashlib
    import re
    lines = []
    for f in ("engine.h", "band.h", "bits.h"):
        for line in open(os.path.join(CSRC, f), encoding="utf-8"):
            line = re.sub(r"//.*$", "", line.rstrip("\n")).rstrip()
            if line:
                lines.append(line)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()[:16]


def library_source_sha():
    """sha256[:16] of the library's sources (csrc/*.hip, csrc/*.h, include/mpd.h)
    and the git commit if the tree is a checkout: which code a bench line ran."""
    import glob
    import hashlib
    import subprocess
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.h")))
    for f in files + [os.path.join(ROOT, "include", "mpd.h")]:
        h.update(open(f, "rb").read())
    try:
        commit = subprocess.run(["git", "rev-parse", "--short=12", "HEAD"], cwd=ROOT, capture_output=True,
                                text=True, timeout=10).stdout.strip() or None
    except Exception:
        commit = None
    return h.hexdigest()[:16], commit


def profile_summary():
    """The committed rocprofv3 summary of k_bits on the benchmark batches
    (VALU instructions per launch from SQ_INSTS_VALU, HBM bytes per launch
    from the calibrated FETCH_SIZE / WRITE_SIZE counters), or {} if the
    kernel's code changed since the counters were taken."""
    try:
        with open(PROFILE_SUMMARY) as f:
            summ = json.load(f)
        sha = kernel_source_sha()
    except (OSError, ValueError):
        return {}
    return summ if summ.get("kernel_source_sha16") == sha else {}


def wilson(k, n, z=1.96):
    """Wilson score interval of a binomial proportion k / n."""
    if n == 0:
        return [0.0, 1.0]
    ph = k / n
    d = 1 + z * z / n
    c = (ph + z * z / (2 * n)) / d
    h = z * ((ph * (1 - ph) / n + z * z / (4 * n * n)) ** 0.5) / d
    return [max(0.0, c - h), min(1.0, c + h)]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=5120,
                    help="samples of the oracle CPU baseline (about 10 s on 16 host threads)")
    ap.add_argument("--workload", choices=["c3", "c1", "c2", "c4", "c5", "cnn", "rule", "open", "async"],
                    default="c3",
                    help="c3 (default) is the headline line; c1/c2/c4/c5 print a line for that configuration, "
                         "cnn times the predictor's kernels, rule the limited-memory variant at L = 256, open the "
                         "open lattice at L = 64 and 128, async the marching-soldiers desynchronized decoder at "
                         "L = 32 and 64")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-scheduling leg")
    ap.add_argument("--async-case", type=int, default=-1,
                    help="async workload: run only this case of its list (0: L=64 p=0.05, 1: L=64 p=0.03, "
                         "2: L=32 p=0.05); -1 runs all")
    ap.add_argument("--streams", type=int, default=None,
                    help="batches in flight, each on its own stream, host thread and workspace (default 3 for "
                         "the L = 256 workloads c3/c5, 1 for the short batches of c1/c2/c4)")
    ap.add_argument("--band-bits", type=int, default=None, metavar="K",
                    help="steps of the bit-sliced first kernel at L=256 (0: the band path's first pass)")
    ap.add_argument("--band-driver", choices=["auto", "host", "device"], default="auto",
                    help="who drives the later passes of the band path (L >= 256): the host (a survivor-count "
                         "readback per pass) or the device (one persistent launch); auto = the library's choice")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times), to calibrate HBM byte counters")
    args = ap.parse_args()
    if args.streams is None:
        args.streams = 3 if args.workload in ("c3", "c5") else (4 if args.workload == "async" else 1)
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU only (--gpus {args.gpus} requested); "
              "the decoder shards by samples, see DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2506_03266_amd.binding as b
    from paper_2506_03266_amd.workloads import seeds

    if not os.path.exists(b.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    b.set_band_driver({"auto": b.BAND_DRIVER_AUTO, "host": b.BAND_DRIVER_HOST,
                       "device": b.BAND_DRIVER_DEVICE}[args.band_driver])
    if args.band_bits is not None:
        b.set_band_bits(args.band_bits)

    if args.copy_calib:
        nbytes = args.copy_calib << 20
        src = torch.randint(0, 255, (nbytes,), dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_read": nbytes, "copy_calib_bytes_written": nbytes, "copies": 3}))
        return

    if args.workload != "c3":
        return other_workload(args, b, seeds, torch, np)

    n, K, W, S = N_SAMPLES, args.steps, args.warmup, max(1, args.streams)
    batches = [torch.from_numpy(seeds(3, i % 256, n).view(np.int64)).to(dev) for i in range(W + K)]
    outs = [(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev),
             torch.empty((n, b.syndrome_words(L)), dtype=torch.int32, device=dev)) for _ in range(W + K)]
    runner = Runner(S, torch)
    wss = [b.alloc_workspace(L, n) for _ in range(S)]

    def fifo(i, j, stream):
        b.decode_batch(L, P, batches[i], T_MAX, workspace=wss[j], out=outs[i], stream=stream)

    # one stream, with per-launch kernel timing: the roofline figures
    for i in range(W):
        fifo(i, 0, runner.streams[0])
    torch.cuda.synchronize()
    b.profile(True)
    t0 = time.perf_counter()
    for i in range(W, W + K):
        fifo(i, 0, runner.streams[0])
    torch.cuda.synchronize()
    elapsed_1 = time.perf_counter() - t0
    b.profile(False)
    bits_ms, bits_launches = b.profile_read("k_bits")
    band_ms, band_launches = b.profile_read("k_band")
    # S batches in flight: the throughput figure
    runner.run(fifo, range(W))
    elapsed = runner.run(fifo, range(W, W + K))

    device_leg = device_driven(b, batches, outs, W, K, n, wss[0], torch) if args.band_driver == "auto" else None
    learned_leg = None if args.no_learned else learned_scheduling(b, batches, outs, W, K, n, torch, np, runner)

    T_all = torch.cat([outs[i][0] for i in range(W, W + K)]).cpu().numpy().astype(np.int64)
    F_all = torch.cat([outs[i][1] for i in range(W, W + K)]).cpu().numpy()
    site_updates = float(L * L * T_all.sum())
    samples_per_s = K * n / elapsed
    su_per_s = site_updates / elapsed
    summ = profile_summary()
    lib_sha, git_commit = library_source_sha()
    avg_launch_s = bits_ms / 1e3 / max(bits_launches, 1)
    valu = summ.get("valu_insts_per_launch")
    achieved = valu * 64 / avg_launch_s / 1e12 if (valu and bits_launches) else None
    # samples that reach the band passes: T_dec above the bit-sliced steps
    k_bits = b.get_band_bits(L)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        m = args.cpu_samples
        s_cpu = seeds(3, 0, m)
        tc = time.perf_counter()
        r = oracle.decode_seeds(L, P, s_cpu, T_MAX, want_sigma=False)
        tcpu = time.perf_counter() - tc
        m1 = max(1, m // 16)
        tc = time.perf_counter()
        r1 = oracle.decode_seeds(L, P, s_cpu[:m1], T_MAX, threads=1, want_sigma=False)
        tcpu1 = time.perf_counter() - tc
        cpu = {"value": m / tcpu, "unit": "samples/s", "cores": r["threads"], "kind": "oracle",
               "sample": f"first {m} samples of batch 0 (same L, p, T_max), {tcpu:.1f} s wall",
               "site_updates_per_s": float(L * L * r["T_dec"].astype(np.int64).sum()) / tcpu,
               "one_core": {"value": m1 / tcpu1, "unit": "samples/s", "cores": r1["threads"],
                            "sample": f"first {m1} samples of batch 0, {tcpu1:.1f} s wall"}}

    line = {
        "metric": METRIC,
        "value": samples_per_s,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": elapsed / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "toric code L=256, p=0.01, 4096 seeded i.i.d. bit-flip samples per step, "
                               f"T_max=4096, v=3, plain FIFO batch, {S} batches in flight on separate streams",
                   "L": L, "p": P, "samples_per_step": n, "T_max": T_MAX, "v": 3, "scheduling": "fifo",
                   "concurrent_batches": S},
        "single_stream": {"samples_per_s": K * n / elapsed_1, "ms_per_step": elapsed_1 / K * 1e3},
        "site_updates_per_s": su_per_s,
        "mean_T_dec": float(T_all.mean()),
        "max_T_dec": int(T_all.max()),
        "T_dec_histogram": {str(int(t)): int(c) for t, c in zip(*np.unique(T_all, return_counts=True))},
        "fail_rate": float((F_all & 1).mean()),
        "fail_rate_wilson95": wilson(int((F_all & 1).sum()), int(F_all.size)),
        "timeouts": int(((F_all & 2) > 0).sum()),
        "roofline": {"bound": "alu", "kernel": "k_bits",
                     "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
                     "frac": (achieved / VALU_PEAK_TOPS) if achieved else None,
                     "traffic": summ.get("traffic_bytes_per_launch"),
                     "achieved_basis": "32-bit lane operations per launch of the bit-sliced kernel (VALU "
                                       "instructions x 64 lanes, SQ_INSTS_VALU of the committed profile on the "
                                       "benchmark batches; the count depends only on the seeds) over the live "
                                       "launch time (HIP events on the launch stream)",
                     "launches": bits_launches, "avg_launch_ms": avg_launch_s * 1e3,
                     "valu_insts_per_launch": valu,
                     "effective_state_GBps": BYTES_PER_SITE_UPDATE * site_updates / max(K, 1) / avg_launch_s / 1e9
                     if bits_launches else None,
                     "effective_state_basis": "16.25 B of u16 register and syndrome state per useful site-update "
                                              "over the k_bits launch time: the HBM traffic a decoder that kept "
                                              "its state in HBM between steps would need; the bit-sliced kernel "
                                              "keeps it on chip",
                     "band_passes": {"k_bits_steps": k_bits, "samples_beyond": int((T_all > k_bits).sum()),
                                     "launches": band_launches, "total_ms": band_ms}},
        "kernel_source_sha16": kernel_source_sha(),
        "library_source_sha16": lib_sha,
        "git_commit": git_commit,
        "cpu_baseline": cpu,
        "device_driver": device_leg,
        "learned_sched": learned_leg,
    }
    print(json.dumps(line), flush=True)


class Runner:
    """Runs batch i of a list on one of S streams (batch i on stream i mod S),
    one host thread per stream; the library calls release the interpreter
    lock, so up to S batches are in flight on the device."""

    def __init__(self, S, torch):
        self.torch = torch
        # one batch in flight: the caller's stream, no extra thread
        self.streams = [torch.cuda.current_stream()] if S == 1 else [torch.cuda.Stream() for _ in range(S)]

    def run(self, fn, idxs):
        """fn(i, j, stream) for every i in idxs; returns the wall time (s)."""
        import threading
        torch = self.torch
        idxs = list(idxs)
        S = len(self.streams)
        errs = []
        if S == 1:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in idxs:
                fn(i, 0, self.streams[0])
            torch.cuda.synchronize()
            return time.perf_counter() - t0

        def worker(j):
            try:
                with torch.cuda.stream(self.streams[j]):
                    for i in idxs[j::S]:
                        fn(i, j, self.streams[j])
            except BaseException as e:  # re-raised below
                errs.append(e)

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        threads = [threading.Thread(target=worker, args=(j,)) for j in range(S)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if errs:
            raise errs[0]
        return dt


def device_driven(b, batches, outs, W, K, n, ws, torch, rounds=5):
    """The same K batches, one stream: with the later passes driven from the
    host (a survivor-count readback per pass) and on the device (no host
    wait in a decode), and as replays of one captured HIP graph (the seeds
    copied into the graph's input before each replay), timed in alternating
    rounds so that drift of the device clock falls on all alike.  Checks
    that every output equals the plain run's."""
    dev = torch.device("cuda")
    st = torch.cuda.current_stream()
    o = (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev),
         torch.empty((n, b.syndrome_words(L)), dtype=torch.int32, device=dev))
    same = True
    s_in = batches[0].clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.decode_batch(L, P, s_in, T_MAX, workspace=ws, out=o)
    torch.cuda.synchronize()
    for i in range(W, min(W + 2, W + K)):  # a couple of replays checked against the plain run (untimed)
        s_in.copy_(batches[i])
        g.replay()
        torch.cuda.synchronize()
        same = same and all(torch.equal(x, y) for x, y in zip(o, outs[i]))

    def run(mode):
        if mode == "graph":
            for i in range(W, W + K):
                s_in.copy_(batches[i])
                g.replay()
            return
        b.set_band_driver(b.BAND_DRIVER_HOST if mode == "host" else b.BAND_DRIVER_DEVICE)
        try:
            for i in range(W, W + K):
                b.decode_batch(L, P, batches[i], T_MAX, workspace=ws, out=o, stream=st)
        finally:
            b.set_band_driver(b.BAND_DRIVER_AUTO)

    for mode in ("host", "device"):  # warm-up
        b.set_band_driver(b.BAND_DRIVER_HOST if mode == "host" else b.BAND_DRIVER_DEVICE)
        try:
            for i in range(W):
                b.decode_batch(L, P, batches[i], T_MAX, workspace=ws, out=o, stream=st)
        finally:
            b.set_band_driver(b.BAND_DRIVER_AUTO)
    el = {"host": 0.0, "device": 0.0, "graph": 0.0}
    for _ in range(rounds):
        for mode in el:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            run(mode)
            torch.cuda.synchronize()
            el[mode] += time.perf_counter() - t0
            same = same and all(torch.equal(x, y) for x, y in zip(o, outs[W + K - 1]))
    R = rounds * K
    return {"samples_per_s": R * n / el["device"], "ms_per_step": el["device"] / R * 1e3,
            "host_driver_samples_per_s": R * n / el["host"], "host_driver_ms_per_step": el["host"] / R * 1e3,
            "graph_replay_samples_per_s": R * n / el["graph"], "graph_replay_ms_per_step": el["graph"] / R * 1e3,
            "rounds": rounds, "identical_results": bool(same)}


def learned_scheduling(b, batches, outs, W, K, n, torch, np, runner, L_eval=L):
    """Train, tune and time the learned-scheduling decode on the benchmark's batches
    (same streams and batches in flight as the plain run), in rounds that
    alternate with the plain decode of the same batches."""
    from paper_2506_03266_amd import learned
    from paper_2506_03266_amd.workloads import seeds
    from scipy.stats import spearmanr
    dev = torch.device("cuda")
    t0 = time.perf_counter()
    counts, target, _, _ = learned.make_dataset(200000)
    params, hist = learned.train(counts, target, epochs=6)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    tune = torch.from_numpy(seeds(3, 201, n).view(np.int64)).to(dev)
    policy, t_best, t_single, res = learned.tune_policy(L_eval, P, tune, params, reps=2)
    lwss = [b.learned_workspace(L_eval, n) for _ in runner.streams]
    tune_set = [(torch.from_numpy(seeds(3, 201 + i, n).view(np.int64)).to(dev), P) for i in range(6)]
    policy, net_policy, in_flight = tune_in_flight(b, runner, L_eval, tune_set, params, res, lwss, torch)
    louts = [(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev),
              torch.empty((n, b.syndrome_words(L_eval)), dtype=torch.int32, device=dev), None)
             for _ in range(W + K)]
    nouts = [(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev),
              torch.empty((n, b.syndrome_words(L_eval)), dtype=torch.int32, device=dev), None)
             for _ in range(W + K)]

    def learned(i, j, stream):
        b.decode_learned(L_eval, P, batches[i], params, policy[0], policy[1], T_MAX, workspace=lwss[j],
                         out=louts[i], stream=stream)

    def net_on(i, j, stream):
        b.decode_learned(L_eval, P, batches[i], params, net_policy[0], net_policy[1], T_MAX, workspace=lwss[j],
                         out=nouts[i], stream=stream)

    def fifo(i, j, stream):
        b.decode_batch(L_eval, P, batches[i], T_MAX, workspace=fifo_ws[j], out=outs[i], stream=stream)

    fifo_ws = [b.alloc_workspace(L_eval, n) for _ in runner.streams]
    runner.run(learned, range(W))
    runner.run(net_on, range(W))
    el_fifo, el, el_net = alternate(runner, [fifo, learned, net_on], W, K)
    el_sorted = oracle_order(runner, fifo_ws, outs, batches, W, K, n, torch, P)
    # the evaluation samples' predictions (outside the timed region; a
    # one-group policy does not compute them) and the inference time per
    # batch, one stream
    b.profile(True)
    preds = [b.cnn_forward(b.syndrome_counts(L_eval, P, batches[i]), params) for i in range(W, W + K)]
    torch.cuda.synchronize()
    b.profile(False)
    cnn_ms, cnn_n = b.profile_read("k_cnn_forward")
    same = all(torch.equal(outs[i][j], louts[i][j]) and torch.equal(outs[i][j], nouts[i][j])
               for i in range(W, W + K) for j in range(3))
    T = torch.cat([outs[i][0] for i in range(W, W + K)]).cpu().numpy()
    pred = torch.cat(preds).cpu().numpy()
    y = np.log1p(T)
    mixed = learned_mixed_p(b, W, K, n, params, torch, np, runner, L_eval)
    return {"samples_per_s": K * n / el, "ms_per_step": el / K * 1e3, "ratio_vs_fifo": el_fifo / el,
            "fifo_samples_per_s": K * n / el_fifo,
            "identical_results": bool(same), "policy": {"edges": list(policy[0]), "first_pass_depth": list(policy[1])},
            "network_on": {"policy": {"edges": list(net_policy[0]), "first_pass_depth": list(net_policy[1])},
                           "samples_per_s": K * n / el_net, "ratio_vs_fifo": el_fifo / el_net},
            "oracle_order_ratio_vs_fifo": el_fifo / el_sorted,
            "cnn_forward_ms_per_step": cnn_ms / max(cnn_n, 1), "train_s": t_train,
            "train_mse_last_epoch": hist[-1], "eval_mae_ln": float(np.abs(pred - y).mean()),
            "eval_spearman": float(spearmanr(pred, T).correlation),
            "tuning_ms": {"best": t_best * 1e3, "single_bin": t_single * 1e3, "in_flight": in_flight},
            "mixed_p": mixed}


def oracle_order(runner, wss, outs, batches, W, K, n, torch, p):
    """The plain decode of the same batches with each batch's samples sorted
    by their measured T_dec, longest first: what a perfect predictor of the
    decoding time could gain by ordering (an upper bound, not a schedule)."""
    import paper_2506_03266_amd.binding as b
    dev = torch.device("cuda")
    ordered, ps = {}, {}
    for i in range(W, W + K):
        perm = torch.argsort(outs[i][0].to(torch.int64), descending=True, stable=True)
        ordered[i] = batches[i][perm].contiguous()
        ps[i] = p[i][perm].contiguous() if isinstance(p, dict) else p
    o = [(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev), None)
         for _ in range(W + K)]

    def run(i, j, stream):
        if isinstance(ps[i], float):
            b.decode_batch(L, ps[i], ordered[i], T_MAX, want_syndrome=False, workspace=wss[j], out=o[i],
                           stream=stream)
        else:
            b.decode_mixed([(L, n)], ps[i], ordered[i], T_MAX, want_syndrome=False, workspace=wss[j], out=o[i],
                           stream=stream)
    runner.run(run, range(W, W + K))
    return min(runner.run(run, range(W, W + K)) for _ in range(3))


def tune_in_flight(b, runner, L_eval, tune_set, params, res, lwss, torch, short=12):
    """Re-times the policies that were fastest one batch at a time, and the
    single-group policy, with the runner's batches in flight (the way the
    decode is used), on a set of tuning batches; returns (best policy, best
    policy that runs the network, {policy: ms per batch})."""
    n = tune_set[0][0].numel()
    dev = tune_set[0][0].device
    outs = [(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev), None,
             None) for _ in tune_set]
    cands = [res[0][1]] + [pol for _, pol in sorted(res[1:], key=lambda r: r[0])[:short]]
    times = {}
    for pol in cands:
        def run(i, j, stream, pol=pol):
            b.decode_learned(L_eval, tune_set[i][1], tune_set[i][0], params, pol[0], pol[1], T_MAX,
                             want_syndrome=False, workspace=lwss[j], out=outs[i], stream=stream)
        runner.run(run, range(len(tune_set)))
        t = min(runner.run(run, range(len(tune_set))) for _ in range(2))
        times[pol] = t / len(tune_set) * 1e3
    best = min(times, key=times.get)
    net = [p for p in times if len(p[1]) > 1]
    best_net = min(net, key=times.get) if net else best
    return best, best_net, {f"{list(p[0])}/{list(p[1])}": t for p, t in times.items()}


def alternate(runner, fns, W, K, rounds=5):
    """Times each function of `fns` over batches W..W+K-1 in alternating
    rounds (so that drift of the device clock falls on all alike); returns
    the mean wall time of one round of each."""
    tot = [0.0] * len(fns)
    for _ in range(rounds):
        for k, fn in enumerate(fns):
            tot[k] += runner.run(fn, range(W, W + K))
    return [t / rounds for t in tot]


def learned_mixed_p(b, W, K, n, params, torch, np, runner, L_eval):
    """The same comparison on batches whose samples each draw their own p from
    the training range U[0.005, 0.02], where decoding times spread from 2 to
    about 10 steps.  FIFO runs at the first-pass depth that is fastest for
    these batches (timed on a tuning batch), and the learned policy is tuned
    around that depth; both decode the same K batches, 3 in flight."""
    from paper_2506_03266_amd import learned
    from paper_2506_03266_amd.workloads import seeds
    from scipy.stats import spearmanr
    dev = torch.device("cuda")
    rng = np.random.default_rng(6)
    pr = learned.P_RANGE
    tune_s = torch.from_numpy(seeds(3, 219, n).view(np.int64)).to(dev)
    tune_p = torch.from_numpy(rng.uniform(pr[0], pr[1], n)).to(dev)
    bs = [torch.from_numpy(seeds(3, 220 + i, n).view(np.int64)).to(dev) for i in range(W + K)]
    ps = [torch.from_numpy(rng.uniform(pr[0], pr[1], n)).to(dev) for _ in range(W + K)]
    k0, kn = b.get_band_schedule(L_eval)
    k_fifo, fifo_times = learned.best_fifo_depth(L_eval, tune_p, tune_s, T_MAX)
    wss = [b.mixed_workspace([(L_eval, n)]) for _ in runner.streams]
    lwss = [b.learned_workspace(L_eval, n) for _ in runner.streams]
    fo = [(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev),
           torch.empty(n * b.syndrome_words(L_eval), dtype=torch.int32, device=dev)) for _ in range(W + K)]
    lo = [(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev),
           torch.empty((n, b.syndrome_words(L_eval)), dtype=torch.int32, device=dev), None) for _ in range(W + K)]
    no = [(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev),
           torch.empty((n, b.syndrome_words(L_eval)), dtype=torch.int32, device=dev), None) for _ in range(W + K)]
    b.set_band_schedule(k_fifo, kn, L_eval)
    try:
        policy, _, _, res = learned.tune_policy(L_eval, tune_p, tune_s, params, T_MAX, k_first=k_fifo, reps=2,
                                                wide=True)
        tune_set = [(torch.from_numpy(seeds(3, 250 + i, n).view(np.int64)).to(dev),
                     torch.from_numpy(rng.uniform(pr[0], pr[1], n)).to(dev)) for i in range(6)]
        policy, net_policy, in_flight = tune_in_flight(b, runner, L_eval, tune_set, params, res, lwss, torch)

        def fifo(i, j, stream):
            b.decode_mixed([(L_eval, n)], ps[i], bs[i], T_MAX, workspace=wss[j], out=fo[i], stream=stream)

        def lrn(i, j, stream):
            b.decode_learned(L_eval, ps[i], bs[i], params, policy[0], policy[1], T_MAX, workspace=lwss[j],
                             out=lo[i], stream=stream)

        def net_on(i, j, stream):
            b.decode_learned(L_eval, ps[i], bs[i], params, net_policy[0], net_policy[1], T_MAX, workspace=lwss[j],
                             out=no[i], stream=stream)

        runner.run(fifo, range(W))
        runner.run(lrn, range(W))
        runner.run(net_on, range(W))
        el_fifo, el_lrn, el_net = alternate(runner, [fifo, lrn, net_on], W, K)
        el_sorted = oracle_order(runner, wss, fo, bs, W, K, n, torch, {i: ps[i] for i in range(W + K)})
    finally:
        b.set_band_schedule(k0, kn, L_eval)
    same = all(torch.equal(fo[i][0], x[i][0]) and torch.equal(fo[i][1], x[i][1]) and
               torch.equal(fo[i][2], x[i][2].reshape(-1)) for i in range(W, W + K) for x in (lo, no))
    T = torch.cat([fo[i][0] for i in range(W, W + K)]).cpu().numpy()
    pred = torch.cat([b.cnn_forward(b.syndrome_counts(L_eval, ps[i], bs[i]), params)
                      for i in range(W, W + K)]).cpu().numpy()
    return {"p": "per sample U[0.005, 0.02]", "fifo_samples_per_s": K * n / el_fifo,
            "learned_samples_per_s": K * n / el_lrn, "ratio_vs_fifo": el_fifo / el_lrn,
            "fifo_first_pass_depth": k_fifo, "fifo_tuning_ms": {str(k): t * 1e3 for k, t in fifo_times.items()},
            "policy": {"edges": list(policy[0]), "first_pass_depth": list(policy[1])}, "tuning_ms_in_flight": in_flight,
            "network_on": {"policy": {"edges": list(net_policy[0]), "first_pass_depth": list(net_policy[1])},
                           "samples_per_s": K * n / el_net, "ratio_vs_fifo": el_fifo / el_net},
            "oracle_order_ratio_vs_fifo": el_fifo / el_sorted,
            "eval_spearman": float(spearmanr(pred, T).correlation), "identical_results": bool(same)}


def other_workload(args, b, seeds, torch, np):
    """Throughput of configurations 1, 2 (per p), 4 (mixed sizes) and 5 (learned
    scheduling), fresh seeds per step, --streams batches in flight."""
    from paper_2506_03266_amd.workloads import CONFIGS, mixed_batch
    dev = torch.device("cuda:0")
    K, W, S = args.steps, args.warmup, max(1, args.streams)
    runner = Runner(S, torch)
    if args.workload == "c5":
        return learned_c5(args, b, seeds, torch, np, runner)
    if args.workload == "cnn":
        return cnn_kernels(args, b, seeds, torch, np)
    if args.workload == "rule":
        return limited_memory(args, b, seeds, torch, np, runner)
    if args.workload == "open":
        return open_lattice(args, b, seeds, torch, np)
    if args.workload == "async":
        return desynchronized(args, b, seeds, torch, np)
    if args.workload == "c4":
        Ls, ps, ss = mixed_batch()
        classes = [(L, int((Ls == L).sum())) for L in dict.fromkeys(Ls.tolist())]
        nb = len(Ls)
        pt = torch.from_numpy(ps).to(dev)
        st = torch.from_numpy(ss.view(np.int64)).to(dev)
        W_syn = int(sum(c * b.syndrome_words(L) for L, c in classes))
        hL = np.ascontiguousarray([c[0] for c in classes], dtype=np.int32)
        hC = np.ascontiguousarray([c[1] for c in classes], dtype=np.int64)
        wsz = int(b.lib().mpd_mixed_workspace_bytes(len(hL), hL.ctypes.data, hC.ctypes.data))
        wss = [torch.empty(max(wsz, 1), dtype=torch.uint8, device=dev) for _ in range(S)]
        outs = [(torch.empty(nb, dtype=torch.int32, device=dev), torch.empty(nb, dtype=torch.uint8, device=dev),
                 torch.empty(W_syn, dtype=torch.int32, device=dev)) for _ in range(W + K)]

        def mixed(i, j, stream):
            b.decode_mixed(classes, pt, st, 4096, workspace=wss[j], out=outs[i], stream=stream)

        runner.run(mixed, range(W))
        dt_default = runner.run(mixed, range(W, W + K))
        T_default = [o[0].clone() for o in outs[W:]]
        # the autotuner picks each band-path class's schedule (driver, depths,
        # bit-sliced steps), timed on a probe batch of that class's size drawn
        # from other seeds at the middle of the p range
        tuned = {}
        for k, (Lc, c) in enumerate(classes):
            if Lc < 256:
                continue
            probe = torch.from_numpy(seeds(4, 100 + k, c).view(np.int64)).to(dev)
            kf, kn, ms = b.autotune_band(Lc, 0.0155, probe, 4096)
            tuned[str(Lc)] = {"k_first": kf, "k_next": kn, "k_bits": b.get_band_bits(Lc),
                              "driver": b.get_band_driver(Lc), "probe_ms": ms}
        runner.run(mixed, range(W))
        dt = runner.run(mixed, range(W, W + K))
        same = all(torch.equal(a, o[0]) for a, o in zip(T_default, outs[W:]))
        T = outs[-1][0].cpu().numpy().astype(np.int64)
        su = float((Ls.astype(np.int64) ** 2 * T).sum())
        # the figure is the default schedules'; the autotuned one is reported
        # beside it (its picks come from each class decoded alone, while the
        # mixed batch runs the classes side by side)
        print(json.dumps({"workload": "config 4: mixed L in {32,64,128,256,512}, counts ~ 1/L^2, "
                                      "p ~ U[0.001,0.03]", "samples_per_s": K * nb / dt_default,
                          "site_updates_per_s": K * su / dt_default, "ms_per_batch": dt_default / K * 1e3,
                          "autotuned": {"samples_per_s": K * nb / dt, "ms_per_batch": dt / K * 1e3,
                                        "schedules": tuned, "identical_results": bool(same)},
                          "samples": int(nb), "concurrent_batches": S}))
        return
    cfg = CONFIGS[1 if args.workload == "c1" else 2]
    L, n = cfg["L"], cfg["n"]
    for k, p in enumerate(cfg["p"]):
        batches = [torch.from_numpy(seeds(int(args.workload[1]), k, n, start=i * n).view(np.int64)).to(dev)
                   for i in range(W + K)]
        outs = [(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev), None)
                for _ in range(W + K)]

        def resident(i, j, stream):
            b.decode_batch(L, p, batches[i], cfg["T_max"], want_syndrome=False, out=outs[i], stream=stream)

        runner.run(resident, range(W))
        dt = runner.run(resident, range(W, W + K))
        T = torch.cat([outs[i][0] for i in range(W, W + K)]).cpu().numpy().astype(np.int64)
        print(json.dumps({"workload": f"config {args.workload[1]}: L={L} p={p} {n} samples",
                          "samples_per_s": K * n / dt, "site_updates_per_s": L * L * T.sum() / dt,
                          "ms_per_batch": dt / K * 1e3, "mean_T_dec": float(T.mean()), "concurrent_batches": S}))


def limited_memory(args, b, seeds, torch, np, runner):
    """The limited-memory variant (messages truncated at m_max, a random move
    of every anyon every u steps) on the L = 256, p = 0.01 batches, against
    the plain rule at the same step budget (T_max = 512, which bounds the
    cost of samples that a small m_max leaves stuck)."""
    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    n, T_max = N_SAMPLES, 512
    batches = [torch.from_numpy(seeds(3, i % 256, n).view(np.int64)).to(dev) for i in range(W + K)]
    ws = b.alloc_workspace(L, n)
    st = runner.streams[0]
    for m_max, u in ((0, 0), (16, 0), (16, 8), (6, 4)):
        outs = [(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev), None)
                for _ in range(W + K)]
        for i in range(W):
            b.decode_rule(L, P, batches[i], T_max, m_max=m_max, u=u, workspace=ws, out=outs[i], stream=st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(W, W + K):
            b.decode_rule(L, P, batches[i], T_max, m_max=m_max, u=u, workspace=ws, out=outs[i], stream=st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        T = torch.cat([outs[i][0] for i in range(W, W + K)]).cpu().numpy().astype(np.int64)
        F = torch.cat([outs[i][1] for i in range(W, W + K)]).cpu().numpy()
        print(json.dumps({"workload": f"limited memory: L={L} p={P} {n} samples, T_max={T_max}, m_max={m_max}, u={u}",
                          "samples_per_s": K * n / dt, "site_updates_per_s": L * L * T.sum() / dt,
                          "ms_per_batch": dt / K * 1e3, "mean_T_dec": float(T.mean()),
                          "fail_rate": float((F & 1).mean()), "timeouts": int(((F & 2) > 0).sum())}), flush=True)


def open_lattice(args, b, seeds, torch, np):
    """The open lattice (rough left / right boundaries) against the torus at
    the same L, p and samples: L = 64 at p = 0.01 and 0.02 and L = 128 on the
    resident kernel, L = 256 on the band path, one batch at a time."""
    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    for L, p, n in ((64, 0.01, 10000), (64, 0.02, 10000), (128, 0.01, 2500), (256, 0.01, 4096)):
        batches = [torch.from_numpy(seeds(9, int(p * 1000), n, start=i * n).view(np.int64)).to(dev)
                   for i in range(W + K)]
        line = {"workload": f"open lattice vs torus: L={L} p={p} {n} samples, T_max=4096"}
        ws = b.alloc_workspace(L, n)
        for name, fn in (("open", lambda s: b.decode_open(L, p, s, 4096, want_syndrome=False, workspace=ws)),
                         ("torus", lambda s: b.decode_batch(L, p, s, 4096, want_syndrome=False, workspace=ws))):
            outs = [None] * (W + K)
            for i in range(W):
                outs[i] = fn(batches[i])
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(W, W + K):
                outs[i] = fn(batches[i])
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            T = torch.cat([outs[i][0] for i in range(W, W + K)]).cpu().numpy().astype(np.int64)
            F = torch.cat([outs[i][1] for i in range(W, W + K)]).cpu().numpy()
            line[name] = {"samples_per_s": K * n / dt, "site_updates_per_s": L * L * T.sum() / dt,
                          "ms_per_batch": dt / K * 1e3, "mean_T_dec": float(T.mean()),
                          "fail_rate": float((F & 1).mean())}
        print(json.dumps(line), flush=True)


def desynchronized(args, b, seeds, torch, np):
    """The marching-soldiers desynchronized decoder (ring probability 1/8 per
    slot, close to independent Poisson clocks) on fresh seeded batches, timed
    with HIP events on its stream, beside the synchronous decoder on the same
    seeds (decoding-time slowdown, identical outcomes), the uncoordinated
    desynchronization on the same batches, and the oracle of each."""
    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    rho, S_max = 0.125, 20000
    st = torch.cuda.current_stream()
    # batches in flight: a sample stuck until S_max holds its compute unit for
    # the whole launch while the others finish early; other batches fill them
    runner = Runner(max(1, args.streams), torch)
    cases = ((64, 0.05, 1024), (64, 0.03, 1024), (32, 0.05, 2048))
    for L_a, p, n in (cases if args.async_case < 0 else cases[args.async_case:args.async_case + 1]):
        batches = [torch.from_numpy(seeds(11, int(p * 1000) + L_a, n, start=i * n).view(np.int64)).to(dev)
                   for i in range(W + K)]
        outs = [tuple(torch.empty(n, dtype=dt, device=dev) for dt in (torch.int32, torch.uint8, torch.int32,
                                                                        torch.int64)) + (None,)
                for _ in range(W + K)]
        for i in range(W):
            b.decode_async(L_a, p, batches[i], rho, S_max, out=outs[i], stream=st)
        torch.cuda.synchronize()
        b.profile(True)
        t0 = time.perf_counter()
        for i in range(W, W + K):
            b.decode_async(L_a, p, batches[i], rho, S_max, out=outs[i], stream=st)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        b.profile(False)
        kms, launches = b.profile_read("k_async")
        # the same batches with several in flight (one host thread and stream each)
        def run_async(i, j, stream, unc=False, sched="cyclic"):
            b.decode_async(L_a, p, batches[i], rho, S_max, out=outs[i], stream=stream, uncoordinated=unc,
                           schedule=sched)
        dt_flight = runner.run(run_async, range(W, W + K)) if len(runner.streams) > 1 else dt
        cat = lambda j: torch.cat([outs[i][j] for i in range(W, W + K)]).cpu().numpy()
        T, F, SL, U = cat(0), cat(1), cat(2).astype(np.int64), cat(3).astype(np.int64)
        # the synchronous decoder on the same seeds
        sync = [b.decode_batch(L_a, p, batches[i], 4096, want_syndrome=False) for i in range(W, W + K)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sync = [b.decode_batch(L_a, p, batches[i], 4096, want_syndrome=False) for i in range(W, W + K)]
        torch.cuda.synchronize()
        dts = time.perf_counter() - t1
        Ts = torch.cat([x[0] for x in sync]).cpu().numpy().astype(np.int64)
        Fs = torch.cat([x[1] for x in sync]).cpu().numpy()
        both = ((F & 2) == 0) & ((Fs & 2) == 0)
        line = {"workload": f"desynchronized decoder: L={L_a} p={p} {n} samples per batch, ring probability {rho} "
                            f"per slot, S_max={S_max}",
                "samples_per_s": K * n / dt_flight, "batches_in_flight": len(runner.streams),
                "single_stream_samples_per_s": K * n / dt, "ms_per_batch": dt / K * 1e3,
                "kernel": {"name": "k_async", "avg_launch_ms": kms / max(launches, 1), "launches": launches},
                "accepted_updates_per_s": float(U.sum()) / dt,
                "slots_mean": float(SL.mean()), "slots_max": int(SL.max()),
                "decoding_time_mean": float(T.mean()) * rho, "sync_T_dec_mean": float(Ts.mean()),
                "slowdown": float(T.mean()) * rho / max(float(Ts.mean()), 1e-9),
                "fail_rate": float((F & 1).mean()), "sync_fail_rate": float((Fs & 1).mean()),
                "timeouts": int(((F & 2) > 0).sum()),
                "outcomes_equal_sync": bool(np.array_equal(F[both], Fs[both])),
                "sync_samples_per_s": K * n / dts}
        # the uncoordinated desynchronization on the same batches, both schedules
        for sched in ("cyclic", "random"):
            for i in range(W):
                b.decode_async(L_a, p, batches[i], rho, S_max, out=outs[i], stream=st, uncoordinated=True,
                               schedule=sched)
            torch.cuda.synchronize()
            b.profile(True)
            t0 = time.perf_counter()
            for i in range(W, W + K):
                b.decode_async(L_a, p, batches[i], rho, S_max, out=outs[i], stream=st, uncoordinated=True,
                               schedule=sched)
            torch.cuda.synchronize()
            dtu = time.perf_counter() - t0
            b.profile(False)
            kmu, lu = b.profile_read("k_async_unc")
            dtu_flight = (runner.run(lambda i, j, stream: run_async(i, j, stream, True, sched), range(W, W + K))
                          if len(runner.streams) > 1 else dtu)
            Tu, Fu, SLu, Uu = cat(0), cat(1), cat(2).astype(np.int64), cat(3).astype(np.int64)
            key = "uncoordinated" if sched == "cyclic" else "uncoordinated_random"
            line[key] = {"samples_per_s": K * n / dtu_flight, "single_stream_samples_per_s": K * n / dtu,
                         "ms_per_batch": dtu / K * 1e3,
                         "kernel": {"name": "k_async_unc", "avg_launch_ms": kmu / max(lu, 1), "launches": lu},
                         "updates_per_s": float(Uu.sum()) / dtu, "slots_mean": float(SLu.mean()),
                         "decoding_time_mean": float(Tu.mean()) * rho, "fail_rate": float((Fu & 1).mean()),
                         "timeouts": int(((Fu & 2) > 0).sum())}
            if sched == "cyclic":
                Tc, Fc = Tu, Fu
        if not args.no_cpu_baseline:
            import oracle
            m = 256
            s_cpu = seeds(11, int(p * 1000) + L_a, m, start=W * n)
            for unc, Tg, Fg in ((False, T, F), (True, Tc, Fc)):
                tc = time.perf_counter()
                r = oracle.async_decode_seeds(L_a, p, s_cpu, rho=rho, S_max=S_max, want_sigma=False, uncoordinated=unc)
                tcpu = time.perf_counter() - tc
                cpu = {"value": m / tcpu, "unit": "samples/s", "cores": r["threads"], "kind": "oracle",
                       "sample": f"first {m} samples of the first timed batch, {tcpu:.1f} s wall"}
                if unc:
                    line["uncoordinated"]["cpu_baseline"] = cpu
                else:
                    line["cpu_baseline"] = cpu
                assert np.array_equal(r["T_async"], Tg[:m]) and np.array_equal(r["flags"], Fg[:m])
        print(json.dumps(line), flush=True)


def learned_c5(args, b, seeds, torch, np, runner):
    """Configuration 5: plain vs learned scheduling at L = 256 (4096 samples)
    and L = 1024 (1024 samples), p = 0.01, with one predictor trained at L = 256;
    policies re-timed in flight, FIFO and learned timed in alternating rounds."""
    from paper_2506_03266_amd import learned
    dev = torch.device("cuda")
    K, W = args.steps, args.warmup
    S = len(runner.streams)
    if args.no_learned:  # the plain (FIFO) decode of both sizes only
        for Lc, n, pidx in ((256, 4096, 0), (1024, 1024, 1)):
            batches = [torch.from_numpy(seeds(5, 100 + pidx, n, start=i * n).view(np.int64)).to(dev)
                       for i in range(W + K)]
            wss = [b.alloc_workspace(Lc, n) for _ in range(S)]
            outs = [(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev),
                     None) for _ in range(W + K)]

            def fifo(i, j, stream):
                b.decode_batch(Lc, P, batches[i], T_MAX, want_syndrome=False, workspace=wss[j], out=outs[i],
                               stream=stream)

            runner.run(fifo, range(W))
            dt = runner.run(fifo, range(W, W + K))
            T = torch.cat([outs[i][0] for i in range(W, W + K)]).cpu().numpy().astype(np.int64)
            print(json.dumps({"workload": f"config 5: L={Lc} p={P} {n} samples, plain decode",
                              "fifo_samples_per_s": K * n / dt, "ms_per_batch": dt / K * 1e3,
                              "mean_T_dec": float(T.mean()), "concurrent_batches": S}), flush=True)
        return
    counts, target, _, _ = learned.make_dataset(200000)
    params, _ = learned.train(counts, target, epochs=6)
    for Lc, n, pidx in ((256, 4096, 0), (1024, 1024, 1)):
        batches = [torch.from_numpy(seeds(5, 100 + pidx, n, start=i * n).view(np.int64)).to(dev)
                   for i in range(W + K)]
        tune = torch.from_numpy(seeds(5, 200 + pidx, n).view(np.int64)).to(dev)
        policy, _, _, tres = learned.tune_policy(Lc, P, tune, params, reps=2)
        wss = [b.alloc_workspace(Lc, n) for _ in range(S)]
        lwss = [b.learned_workspace(Lc, n) for _ in range(S)]
        tune_set = [(torch.from_numpy(seeds(5, 200 + pidx, n, start=i * n).view(np.int64)).to(dev), P)
                    for i in range(6)]
        policy, net_policy, _ = tune_in_flight(b, runner, Lc, tune_set, params, tres, lwss, torch)
        outs = {name: [(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev),
                        None, None) for _ in range(W + K)] for name in ("fifo", "learned", "network_on")}

        def fifo(i, j, stream):
            b.decode_batch(Lc, P, batches[i], T_MAX, want_syndrome=False, workspace=wss[j],
                           out=outs["fifo"][i][:3], stream=stream)

        def lrn(i, j, stream):
            b.decode_learned(Lc, P, batches[i], params, policy[0], policy[1], T_MAX, want_syndrome=False,
                             workspace=lwss[j], out=outs["learned"][i], stream=stream)

        def net_on(i, j, stream):
            b.decode_learned(Lc, P, batches[i], params, net_policy[0], net_policy[1], T_MAX, want_syndrome=False,
                             workspace=lwss[j], out=outs["network_on"][i], stream=stream)

        runner.run(fifo, range(W))
        runner.run(lrn, range(W))
        runner.run(net_on, range(W))
        el_fifo, el_lrn, el_net = alternate(runner, [fifo, lrn, net_on], W, K)
        res = {"fifo": (el_fifo, outs["fifo"]), "learned": (el_lrn, outs["learned"])}
        same = all(torch.equal(a[0], c[0]) and torch.equal(a[1], c[1]) and torch.equal(a[0], d[0])
                   and torch.equal(a[1], d[1])
                   for a, c, d in zip(res["fifo"][1][W:], res["learned"][1][W:], outs["network_on"][W:]))
        print(json.dumps({"workload": f"config 5: L={Lc} p={P} {n} samples, plain vs learned scheduling",
                          "fifo_samples_per_s": K * n / res["fifo"][0],
                          "learned_samples_per_s": K * n / res["learned"][0],
                          "ratio": res["fifo"][0] / res["learned"][0], "identical_results": same,
                          "policy": {"edges": list(policy[0]), "first_pass_depth": list(policy[1])},
                          "network_on": {"policy": {"edges": list(net_policy[0]),
                                                    "first_pass_depth": list(net_policy[1])},
                                         "samples_per_s": K * n / el_net, "ratio": el_fifo / el_net},
                          "concurrent_batches": S}), flush=True)


def cnn_kernels(args, b, seeds, torch, np):
    """Forward pass of the decode-time predictor on one decode batch of block-count
    maps (4096 at L = 256, 1024 at L = 1024) and training steps of 256 maps."""
    dev = torch.device("cuda")
    K, W = args.steps, args.warmup
    prm = b.cnn_init(1)
    for Lc, n in ((256, 4096), (1024, 1024)):
        c = b.syndrome_counts(Lc, P, torch.from_numpy(seeds(3, 300, n).view(np.int64)).to(dev))
        for _ in range(W):
            b.cnn_forward(c, prm)
        torch.cuda.synchronize()
        b.profile(True)
        for _ in range(K):
            b.cnn_forward(c, prm)
        torch.cuda.synchronize()
        b.profile(False)
        ms, k = b.profile_read("k_cnn_forward")
        flop = 14112.0 * (Lc // 8) ** 2 * n
        print(json.dumps({"kernel": "k_cnn_forward", "L": Lc, "maps": n, "ms": ms / k,
                          "TFLOP_per_s": flop / (ms / k) / 1e9, "bf16_dense_peak_frac": flop / (ms / k) / 1e9 / 2500}),
              flush=True)
    c = b.syndrome_counts(256, P, torch.from_numpy(seeds(3, 301, 256).view(np.int64)).to(dev))
    y = torch.full((256,), 1.6, device=dev)
    ws = b.train_workspace(32, 256)
    for _ in range(W):
        b.cnn_loss_grad(c, prm, y, workspace=ws)
    torch.cuda.synchronize()
    b.profile(True)
    t0 = time.perf_counter()
    for _ in range(K):
        b.cnn_loss_grad(c, prm, y, workspace=ws)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / K
    b.profile(False)
    print(json.dumps({"kernel": "training step (256 maps)", "ms": dt * 1e3,
                      "forward_ms": b.profile_read("k_cnn_forward")[0] / K,
                      "backward_ms": b.profile_read("k_cnn_backward")[0] / K}), flush=True)


if __name__ == "__main__":
    main()
