"""Monte Carlo sweeps of the 2D numerics (Sec. 7.2) on the GPU decoder.

Three measurements, all on i.i.d. bit-flip noise, periodic L x L lattices, v = 3:

* logical failure rate p_log against p at several L, and the crossing points
  of consecutive sizes (the threshold p_c);
* the slope gamma of p_log = C (p / p_c)^(gamma L) below threshold, from
  p_log at two sizes: gamma = ln(p_log(L2) / p_log(L1)) / ((L2 - L1) ln(p / p_c));
* the mean decoding time T_dec against ln L below threshold, fitted by
  T_dec = A ln L + B;
* with ``--memory``: p_log, timeouts and T_dec of the limited-memory variant
  (Sec. 5.3: messages truncated at m_max, with and without a random move of
  every anyon every u steps) against m_max at several L;
* with ``--open``: p_log against p on the open lattice (rough left and right
  boundaries, appendix on open boundaries) and its crossings;
* with ``--uncoord``: p_log against p of the uncoordinated desynchronization
  (Sec. "Uncoordinated desynchronization") beside the synchronous decoder on
  the same seeds, and the crossings of both;
* with ``--slowdown``: the marching-soldiers decoder's decoding time against
  the synchronous T_dec on the same seeds, for several L (Lemma "constant
  slowdown for desynchronization": the ratio tends to a constant).

Every sample is decoded by libmpd (noise, decoding and classification run in
the HIP kernels); this module chooses seeds, sums the per-sample results on
the device and fits the sums.  A sample that is still not anyon-free after
T_max steps is counted as a logical failure, as the decoder's flags say, and
is left out of the mean decoding time.

Run as ``python -m paper_2506_03266_amd.sweep [--quick] [--json PATH]``.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

SWEEP_CONFIG = 7    # seed stream of the sweeps (disjoint from the benchmark workloads)

# Grids: (L, samples) per size, and the noise strengths.
THRESHOLD_P = [0.06, 0.065, 0.07, 0.0725, 0.075, 0.0775, 0.08, 0.085, 0.09]
THRESHOLD_L = [(16, 200000), (32, 100000), (64, 50000), (128, 20000), (256, 8000), (512, 4000)]
SLOPE_P = [0.03, 0.04, 0.05]
SLOPE_L = [(8, 4000000), (12, 4000000), (16, 4000000), (24, 4000000), (32, 4000000)]
TDEC_P = [0.01, 0.02, 0.03, 0.05]
TDEC_L = [(16, 100000), (32, 100000), (64, 50000), (128, 20000), (256, 8000), (512, 2000), (1024, 512)]
MEMORY_P = 0.03
MEMORY_M = [2, 3, 4, 6, 8, 12, 16, 0]        # 0: no truncation
MEMORY_U = [0, 8]
MEMORY_L = [(32, 20000), (64, 10000), (128, 4000)]
MEMORY_T_MAX = 2048
OPEN_P = [0.06, 0.07, 0.075, 0.08, 0.085, 0.09, 0.1]
OPEN_L = [(16, 100000), (32, 50000), (64, 20000), (128, 5000), (256, 3000), (512, 1500)]
UNCOORD_P = [0.05, 0.06, 0.065, 0.07, 0.075, 0.08, 0.09]
UNCOORD_L = [(16, 40000), (32, 20000), (64, 8000)]
UNCOORD_RHO = 0.125     # ring probability per slot: close to independent Poisson clocks
UNCOORD_S_MAX = 20000   # slots
SLOWDOWN_P = [0.01, 0.03]
SLOWDOWN_L = [(8, 8192), (16, 8192), (32, 4096), (48, 2048), (64, 2048)]


def seed_block(L: int, p_index: int, n: int, start: int = 0) -> np.ndarray:
    """Seeds of one sweep point: stream SWEEP_CONFIG, index (L << 8) | p_index."""
    from .workloads import seeds
    return seeds(SWEEP_CONFIG, (L << 8) | p_index, n, start)


def _chunk(L: int) -> int:
    # Enough samples per call to fill the GPU; for the band path (L >= 256,
    # about 16.5 workspace bytes per site and sample) few enough to keep the
    # workspace near 8 GB.
    return 262144 if L <= 128 else int(max(64, min(8192, (8 << 30) // (17 * L * L))))


def point(L: int, p: float, n: int, p_index: int, T_max: int = 4096, m_max: int = 0, u: int = 0,
          open_bc: bool = False, uncoord: str = "") -> dict:
    """Decode n seeded samples at (L, p) (with the limited-memory variant if
    m_max or u is set, on the open lattice with open_bc, with the uncoordinated
    desynchronization under schedule `uncoord` ("cyclic" or "random") if it
    is set); returns the counts and sums of the point.

    fails counts flag bit 0 (timeouts included), timeouts flag bit 1; T_sum
    and T_sq sum T_dec over the samples that finished (for the uncoordinated
    decoder: the decoding time in slots, T_max being ignored for it).
    """
    import torch
    from . import binding as b
    dev = torch.device("cuda")
    c = min(n, _chunk(L))
    ws = b.alloc_workspace(L, c, dev)
    T = torch.empty(c, dtype=torch.int32, device=dev)
    F = torch.empty(c, dtype=torch.uint8, device=dev)
    acc = torch.zeros(5, dtype=torch.int64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a in range(0, n, c):
        m = min(c, n - a)
        s = torch.from_numpy(seed_block(L, p_index, m, a).view(np.int64)).to(dev)
        if uncoord:
            Tm, Fm, _, _, _ = b.decode_async(L, p, s, UNCOORD_RHO, UNCOORD_S_MAX, want_syndrome=False,
                                             uncoordinated=True, schedule=uncoord)
        elif open_bc:
            Tm, Fm, _ = b.decode_open(L, p, s, T_max, want_syndrome=False)
        elif m_max or u:
            Tm, Fm, _ = b.decode_rule(L, p, s, T_max, m_max=m_max, u=u, want_syndrome=False, workspace=ws,
                                      out=(T[:m], F[:m], None))
        else:
            Tm, Fm, _ = b.decode_batch(L, p, s, T_max, want_syndrome=False, workspace=ws, out=(T[:m], F[:m], None))
        Fi = Fm.to(torch.int64)
        done = (Fi & 2) == 0
        Td = torch.where(done, Tm.to(torch.int64), torch.zeros_like(Fi))
        acc += torch.stack([(Fi & 1).sum(), (Fi >> 1 & 1).sum(), Td.sum(), (Td * Td).sum(),
                            Tm.to(torch.int64).sum()])
    v = acc.cpu().tolist()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fails, timeouts, T_sum, T_sq, T_all = (int(x) for x in v)
    return dict(L=L, p=p, n=n, T_max=T_max, m_max=m_max, u=u, open=open_bc, uncoord=uncoord, fails=fails,
                timeouts=timeouts, T_sum=T_sum, T_sq=T_sq, seconds=dt, site_updates=T_all * L * L)


def p_log(r: dict) -> float:
    return r["fails"] / r["n"]


def p_log_err(r: dict) -> float:
    f = p_log(r)
    return math.sqrt(max(f * (1 - f), 1.0 / r["n"]) / r["n"])


def mean_T(r: dict):
    """(mean T_dec, its standard error) over the samples that finished."""
    k = r["n"] - r["timeouts"]
    if k == 0:
        return float("nan"), float("nan")
    m = r["T_sum"] / k
    var = max(r["T_sq"] / k - m * m, 0.0)
    return m, math.sqrt(var / k)


def crossing(ps, f1, f2):
    """First p at which p_log of the larger size stops being below that of the
    smaller one.  Between the two grid points around the sign change,
    ln(f2 / f1) is interpolated linearly in ln p, which is exact for
    p_log = C (p/p_c)^(gamma L) with a common C; None if there is no change."""
    f1 = np.asarray(f1, dtype=float)
    f2 = np.asarray(f2, dtype=float)
    for i in range(1, len(ps)):
        if f2[i - 1] < f1[i - 1] and f2[i] >= f1[i]:
            if min(f1[i - 1], f1[i], f2[i - 1], f2[i]) > 0:
                d0, d1 = math.log(f2[i - 1] / f1[i - 1]), math.log(f2[i] / f1[i])
                x0, x1 = math.log(ps[i - 1]), math.log(ps[i])
                return math.exp(x0 + (x1 - x0) * (-d0) / (d1 - d0))
            d0, d1 = f2[i - 1] - f1[i - 1], f2[i] - f1[i]
            return ps[i - 1] + (ps[i] - ps[i - 1]) * (-d0) / (d1 - d0)
    return None


def slope_gamma(L1: int, f1: float, L2: int, f2: float, p: float, p_c: float) -> float:
    """gamma of p_log = C (p/p_c)^(gamma L) from two sizes at one p."""
    return math.log(f2 / f1) / ((L2 - L1) * math.log(p / p_c))


def fit_log(Ls, T, w=None):
    """Weighted least squares of T = A ln L + B; returns (A, B)."""
    x = np.log(np.asarray(Ls, dtype=float))
    y = np.asarray(T, dtype=float)
    w = np.ones_like(x) if w is None else np.asarray(w, dtype=float)
    X = np.stack([x, np.ones_like(x)], axis=1) * np.sqrt(w)[:, None]
    A, B = np.linalg.lstsq(X, y * np.sqrt(w), rcond=None)[0]
    return float(A), float(B)


def run(quick: bool = False, T_max: int = 4096, log=print) -> dict:
    scale = 0.05 if quick else 1.0
    res = dict(T_max=T_max, threshold=[], slope=[], tdec=[])

    def go(kind, grid_L, grid_p, p_base):
        for L, n in grid_L:
            n = max(256, int(n * scale))
            for i, p in enumerate(grid_p):
                r = point(L, p, n, p_base + i, T_max)
                m, e = mean_T(r)
                log(f"{kind} L={L} p={p}: p_log={p_log(r):.5f}±{p_log_err(r):.5f} timeouts={r['timeouts']} "
                    f"T={m:.3f}±{e:.3f} n={n} {r['seconds']:.2f}s "
                    f"{r['site_updates'] / max(r['seconds'], 1e-9):.3g} site-updates/s")
                res[kind].append(r)

    go("threshold", THRESHOLD_L, THRESHOLD_P, 0)
    go("slope", SLOPE_L, SLOPE_P, 32)
    go("tdec", TDEC_L, TDEC_P, 64)
    res["summary"] = summarize(res)
    return res


TDEC_FIT_LMIN = 64   # the ln L fit uses sizes from here on (smaller ones bend below the line)


def run_memory(quick: bool = False, log=print) -> list:
    """The limited-memory grid: every (L, m_max, u) at p = MEMORY_P."""
    scale = 0.05 if quick else 1.0
    out = []
    for L, n in MEMORY_L:
        n = max(256, int(n * scale))
        for j, u in enumerate(MEMORY_U):
            for i, m in enumerate(MEMORY_M):
                r = point(L, MEMORY_P, n, 128 + 16 * j + i, MEMORY_T_MAX, m_max=m, u=u)
                mt, e = mean_T(r)
                log(f"memory L={L} m_max={m} u={u}: p_log={p_log(r):.5f} timeouts={r['timeouts']} "
                    f"T={mt:.3f}±{e:.3f} n={n} {r['seconds']:.2f}s")
                out.append(r)
    return out


def run_open(quick: bool = False, T_max: int = 4096, log=print) -> dict:
    """p_log against p on the open lattice, and the crossings of consecutive sizes."""
    scale = 0.05 if quick else 1.0
    pts = []
    for L, n in OPEN_L:
        n = max(256, int(n * scale))
        for i, p in enumerate(OPEN_P):
            r = point(L, p, n, 192 + i, T_max, open_bc=True)
            mt, e = mean_T(r)
            log(f"open L={L} p={p}: p_log={p_log(r):.5f}±{p_log_err(r):.5f} timeouts={r['timeouts']} "
                f"T={mt:.3f}±{e:.3f} n={n} {r['seconds']:.2f}s")
            pts.append(r)
    Ls = [L for L, _ in OPEN_L]
    tab = {(r["L"], r["p"]): p_log(r) for r in pts}
    cross = {f"{L1}/{L2}": crossing(OPEN_P, [tab[(L1, p)] for p in OPEN_P], [tab[(L2, p)] for p in OPEN_P])
             for L1, L2 in zip(Ls, Ls[1:])}
    return dict(points=pts, crossings=cross)


def run_uncoord(quick: bool = False, log=print) -> dict:
    """p_log against p of the uncoordinated decoder (both schedules) and of the
    synchronous one on the same seeds, and the crossings of consecutive sizes
    of each."""
    scale = 0.05 if quick else 1.0
    pts = {"cyclic": [], "random": [], "synchronous": []}
    for L, n in UNCOORD_L:
        n = max(256, int(n * scale))
        for i, p in enumerate(UNCOORD_P):
            rc = point(L, p, n, 224 + i, uncoord="cyclic")
            rr = point(L, p, n, 224 + i, uncoord="random")
            rs = point(L, p, n, 224 + i)
            log(f"uncoord L={L} p={p}: cyclic p_log={p_log(rc):.5f}±{p_log_err(rc):.5f} (timeouts {rc['timeouts']}, "
                f"time {mean_T(rc)[0] * UNCOORD_RHO:.2f}) | random p_log={p_log(rr):.5f}±{p_log_err(rr):.5f} "
                f"(timeouts {rr['timeouts']}, time {mean_T(rr)[0] * UNCOORD_RHO:.2f}) | synchronous "
                f"p_log={p_log(rs):.5f} T={mean_T(rs)[0]:.2f} n={n}")
            pts["cyclic"].append(rc)
            pts["random"].append(rr)
            pts["synchronous"].append(rs)
    Ls = [L for L, _ in UNCOORD_L]
    cross, gamma = {}, {}
    for key, rows in pts.items():
        tab = {(r["L"], r["p"]): p_log(r) for r in rows}
        cross[key] = {f"{L1}/{L2}": crossing(UNCOORD_P, [tab[(L1, p)] for p in UNCOORD_P],
                                             [tab[(L2, p)] for p in UNCOORD_P]) for L1, L2 in zip(Ls, Ls[1:])}
        # slope of p_log = C (p / p_c)^(gamma L) below threshold, from the two
        # largest sizes, against the decoder's own crossing of those sizes
        p_c = cross[key][f"{Ls[-2]}/{Ls[-1]}"]
        gamma[key] = {}
        if p_c:
            for p in UNCOORD_P:
                f1, f2 = tab[(Ls[-2], p)], tab[(Ls[-1], p)]
                if p < p_c and f1 > 0 and f2 > 0:
                    gamma[key][str(p)] = slope_gamma(Ls[-2], f1, Ls[-1], f2, p, p_c)
    return dict(points=pts, crossings=cross, gamma=gamma, rho=UNCOORD_RHO, S_max=UNCOORD_S_MAX)


def run_slowdown(quick: bool = False, log=print) -> list:
    """Mean decoding time of the marching-soldiers decoder (slots x ring
    probability) against the mean synchronous T_dec on the same seeds, over
    the samples both finish; outcomes must agree on every such sample."""
    import torch
    from . import binding as b
    scale = 0.1 if quick else 1.0
    rows = []
    for p in SLOWDOWN_P:
        for L, n in SLOWDOWN_L:
            n = max(256, int(n * scale))
            s = torch.from_numpy(seed_block(L, 240 + SLOWDOWN_P.index(p), n).view(np.int64)).cuda()
            t0 = time.perf_counter()
            Ta, Fa, _, Ua, _ = b.decode_async(L, p, s, UNCOORD_RHO, UNCOORD_S_MAX, want_syndrome=False)
            Ts, Fs, _ = b.decode_batch(L, p, s, 4096, want_syndrome=False)
            Ta, Fa, Ua = Ta.cpu().numpy(), Fa.cpu().numpy(), Ua.cpu().numpy()
            Ts, Fs = Ts.cpu().numpy(), Fs.cpu().numpy()
            dt = time.perf_counter() - t0
            both = ((Fa & 2) == 0) & ((Fs & 2) == 0) & (Ts > 0)
            ta = Ta[both].astype(np.float64) * UNCOORD_RHO
            ts = Ts[both].astype(np.float64)
            r = dict(L=L, p=p, n=n, decoded=int(both.sum()), time_async=float(ta.mean()), T_sync=float(ts.mean()),
                     ratio=float(ta.mean() / ts.mean()), ratio_median=float(np.median(ta / ts)),
                     outcomes_equal=bool(np.array_equal(Fa[both], Fs[both])), seconds=dt)
            log(f"slowdown L={L} p={p}: async time {r['time_async']:.2f} / sync T {r['T_sync']:.3f} = {r['ratio']:.2f} "
                f"(median per sample {r['ratio_median']:.2f}) over {r['decoded']} samples, outcomes equal "
                f"{r['outcomes_equal']}, {dt:.1f}s")
            rows.append(r)
    return rows


def summarize(res: dict) -> dict:
    """Crossings of consecutive sizes (all samples, and decoded samples only),
    slopes gamma against the crossing of the two largest sizes, and
    unweighted fits of mean T_dec = A ln L + B over L >= TDEC_FIT_LMIN."""
    out = {}
    th = res["threshold"]
    Ls = sorted({r["L"] for r in th})
    ps = sorted({r["p"] for r in th})
    tab = {(r["L"], r["p"]): p_log(r) for r in th}
    dec = {(r["L"], r["p"]): (r["fails"] - r["timeouts"]) / max(r["n"] - r["timeouts"], 1) for r in th}
    for key, t in (("crossings", tab), ("crossings_decoded_only", dec)):
        out[key] = {f"{L1}/{L2}": crossing(ps, [t[(L1, p)] for p in ps], [t[(L2, p)] for p in ps])
                    for L1, L2 in zip(Ls, Ls[1:])}
    pcs = [c for c in out["crossings"].values() if c is not None]
    p_c = pcs[-1] if pcs else 0.073
    out["p_c_used_for_gamma"] = p_c
    sl = res["slope"]
    sLs = sorted({r["L"] for r in sl})
    stab = {(r["L"], r["p"]): p_log(r) for r in sl}
    gam = {}
    for p in sorted({r["p"] for r in sl}):
        for L1, L2 in zip(sLs, sLs[1:]):
            f1, f2 = stab[(L1, p)], stab[(L2, p)]
            if f1 > 0 and f2 > 0:
                gam[f"p={p} L={L1}/{L2}"] = slope_gamma(L1, f1, L2, f2, p, p_c)
    out["gamma"] = gam
    td = res["tdec"]
    fits = {}
    for p in sorted({r["p"] for r in td}):
        rows = sorted((r for r in td if r["p"] == p), key=lambda r: r["L"])
        Lp = [r["L"] for r in rows]
        mT = [mean_T(r) for r in rows]
        use = [i for i, L in enumerate(Lp) if L >= TDEC_FIT_LMIN]
        A, B = fit_log([Lp[i] for i in use], [mT[i][0] for i in use])
        resid = [mT[i][0] - (A * math.log(Lp[i]) + B) for i in use]
        fits[str(p)] = dict(A=A, B=B, L=Lp, T=[m for m, _ in mT], err=[e for _, e in mT],
                            max_abs_resid=max(abs(x) for x in resid))
    out["tdec_fit"] = fits
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--quick", action="store_true", help="5%% of the samples per point")
    ap.add_argument("--T-max", type=int, default=4096)
    ap.add_argument("--json", default=None, help="write all counts and fits here")
    ap.add_argument("--memory", action="store_true", help="only the limited-memory grid")
    ap.add_argument("--open", action="store_true", help="only the open-lattice threshold grid")
    ap.add_argument("--uncoord", action="store_true", help="only the uncoordinated-desynchronization threshold grid")
    ap.add_argument("--slowdown", action="store_true", help="only the marching-soldiers slowdown against L")
    a = ap.parse_args(argv)
    import torch
    if not torch.cuda.is_available():
        sys.exit("sweep: needs a GPU (the decoder runs only in libmpd's HIP kernels)")
    if a.slowdown:
        res = run_slowdown(a.quick, log=lambda s: print(s, flush=True))
        if a.json:
            with open(a.json, "w") as f:
                json.dump(res, f, indent=1)
        return
    if a.uncoord:
        res = run_uncoord(a.quick, log=lambda s: print(s, flush=True))
        print(json.dumps({"crossings": res["crossings"], "gamma": res["gamma"]}), flush=True)
        if a.json:
            with open(a.json, "w") as f:
                json.dump(res, f, indent=1)
        return
    if a.open:
        res = run_open(a.quick, a.T_max, log=lambda s: print(s, flush=True))
        print(json.dumps(res["crossings"]), flush=True)
        if a.json:
            with open(a.json, "w") as f:
                json.dump(res, f, indent=1)
        return
    if a.memory:
        res = run_memory(a.quick, log=lambda s: print(s, flush=True))
        if a.json:
            with open(a.json, "w") as f:
                json.dump(res, f, indent=1)
        return
    res = run(a.quick, a.T_max, log=lambda s: print(s, flush=True))
    print(json.dumps(res["summary"], indent=1), flush=True)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(res, f, indent=1)


if __name__ == "__main__":
    main()
