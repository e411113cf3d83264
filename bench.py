#!/usr/bin/env python3
"""Benchmark: decoded samples/s and site-updates/s of the message-passing
decoder on the L=256, p=0.01 toric-code workload (4096 samples per batch,
T_max = 4096, v = 3), one MI355X.

A step is one complete pass of the hot path over one batch: in-kernel noise
from the seeds, syndrome, decoder steps until no anyon is left, correction
winding and classification, final syndrome export.  Each step uses a fresh
batch of seeds (same distribution); the seeds are already in HBM when the
timed region starts.

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
METRIC = "decoded samples/s & site-updates/s at L=256, p=0.01 (plain vs learned-sched)"
PROFILE_SUMMARY = os.path.join(ROOT, "profiles", "k_band_L256_p001.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2506_03266_amd", "csrc", f) for f in ("mpd.hip", "engine.h", "band.h")]


def measured_traffic():
    """HBM bytes per k_tile launch from the committed rocprofv3 counter summary,
    or None if the kernel sources changed since the counters were taken."""
    import hashlib
    try:
        with open(PROFILE_SUMMARY) as f:
            summ = json.load(f)
        sha = hashlib.sha256(b"".join(open(p, "rb").read() for p in KERNEL_SOURCES)).hexdigest()[:16]
    except OSError:
        return None
    return summ["traffic_bytes_per_launch"] if summ.get("kernel_source_sha16") == sha else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-samples", type=int, default=1024)
    ap.add_argument("--workload", choices=["c3", "c1", "c2", "c4"], default="c3",
                    help="c3 (default) is the headline line; c1/c2/c4 print a line for that configuration")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (3 times), to calibrate HBM byte counters")
    args = ap.parse_args()
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

    n, K, W = N_SAMPLES, args.steps, args.warmup
    batches = [torch.from_numpy(seeds(3, i % 256, n).view(np.int64)).to(dev) for i in range(W + K)]
    ws = b.alloc_workspace(L, n)
    outs = [(torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev),
             torch.empty((n, b.syndrome_words(L)), dtype=torch.int32, device=dev)) for _ in range(W + K)]
    for i in range(W):
        b.decode_batch(L, P, batches[i], T_MAX, workspace=ws, out=outs[i])
    torch.cuda.synchronize()

    b.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(W, W + K):
        b.decode_batch(L, P, batches[i], T_MAX, workspace=ws, out=outs[i])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    b.profile(False)
    tile_ms, tile_launches = b.profile_read("k_band")

    T_all = torch.cat([outs[i][0] for i in range(W, W + K)]).cpu().numpy().astype(np.int64)
    F_all = torch.cat([outs[i][1] for i in range(W, W + K)]).cpu().numpy()
    site_updates = float(L * L * T_all.sum())
    samples_per_s = K * n / elapsed
    su_per_s = site_updates / elapsed
    algo_bytes_per_launch = BYTES_PER_SITE_UPDATE * site_updates / max(tile_launches, 1)
    avg_launch_s = tile_ms / 1e3 / max(tile_launches, 1)
    achieved = algo_bytes_per_launch / avg_launch_s / 1e9 if tile_launches else None

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        m = args.cpu_samples
        s_cpu = seeds(3, 0, m)
        tc = time.perf_counter()
        r = oracle.decode_seeds(L, P, s_cpu, T_MAX, want_sigma=False)
        tcpu = time.perf_counter() - tc
        cpu = {"value": m / tcpu, "unit": "samples/s", "cores": r["threads"], "kind": "oracle",
               "sample": f"first {m} samples of batch 0 (same L, p, T_max), {tcpu:.1f} s wall",
               "site_updates_per_s": float(L * L * r["T_dec"].astype(np.int64).sum()) / tcpu}

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
        "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": "toric code L=256, p=0.01, 4096 seeded i.i.d. bit-flip samples per step, "
                               "T_max=4096, v=3, plain FIFO batch",
                   "L": L, "p": P, "samples_per_step": n, "T_max": T_MAX, "v": 3, "scheduling": "fifo"},
        "site_updates_per_s": su_per_s,
        "mean_T_dec": float(T_all.mean()),
        "max_T_dec": int(T_all.max()),
        "fail_rate": float((F_all & 1).mean()),
        "timeouts": int(((F_all & 2) > 0).sum()),
        "roofline": {"bound": "hbm", "kernel": "k_band",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None, "traffic": measured_traffic(),
                     "bytes_per_site_update": BYTES_PER_SITE_UPDATE,
                     "launches": tile_launches, "avg_launch_ms": avg_launch_s * 1e3},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def other_workload(args, b, seeds, torch, np):
    """Throughput of configurations 1, 2 (per p) and 4 (mixed sizes), fresh seeds per step."""
    from paper_2506_03266_amd.workloads import CONFIGS, mixed_batch
    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    if args.workload == "c4":
        Ls, ps, ss = mixed_batch()
        classes = [(L, int((Ls == L).sum())) for L in dict.fromkeys(Ls.tolist())]
        pt = torch.from_numpy(ps).to(dev)
        st = torch.from_numpy(ss.view(np.int64)).to(dev)
        for _ in range(W):
            b.decode_mixed(classes, pt, st, 4096)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = [b.decode_mixed(classes, pt, st, 4096) for _ in range(K)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        T = outs[-1][0].cpu().numpy().astype(np.int64)
        su = float((Ls.astype(np.int64) ** 2 * T).sum())
        print(json.dumps({"workload": "config 4: mixed L in {32,64,128,256,512}, counts ~ 1/L^2, "
                                      "p ~ U[0.001,0.03]", "samples_per_s": K * len(Ls) / dt,
                          "site_updates_per_s": K * su / dt, "ms_per_batch": dt / K * 1e3,
                          "samples": int(len(Ls))}))
        return
    cfg = CONFIGS[1 if args.workload == "c1" else 2]
    L, n = cfg["L"], cfg["n"]
    for k, p in enumerate(cfg["p"]):
        batches = [torch.from_numpy(seeds(int(args.workload[1]), k, n, start=i * n).view(np.int64)).to(dev)
                   for i in range(W + K)]
        out = (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev), None)
        for i in range(W):
            b.decode_batch(L, p, batches[i], cfg["T_max"], want_syndrome=False, out=out)
        torch.cuda.synchronize()
        tsum = 0
        t0 = time.perf_counter()
        for i in range(W, W + K):
            b.decode_batch(L, p, batches[i], cfg["T_max"], want_syndrome=False, out=out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        T = out[0].cpu().numpy().astype(np.int64)
        print(json.dumps({"workload": f"config {args.workload[1]}: L={L} p={p} {n} samples",
                          "samples_per_s": K * n / dt, "site_updates_per_s_last_batch_est": L * L * T.sum() * K / dt,
                          "ms_per_batch": dt / K * 1e3, "mean_T_dec": float(T.mean())}))


if __name__ == "__main__":
    main()
