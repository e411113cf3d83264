"""Learned scheduling on the GPU: training data from the decoder itself, training
of the decode-time predictor with the library's kernels, and the choice of a
binning policy by timing.

Every step runs in libmpd's HIP kernels (noise, decoding, block counts,
forward, loss gradient, Adam); this module only sequences the calls and
moves a few scalars.  The predictor never changes what a decode returns.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import binding as b
from .workloads import seeds as make_seeds

TRAIN_CONFIG = 5            # seed stream of the training samples (evaluation uses others)
P_RANGE = (0.005, 0.02)     # noise strengths of the training samples


def make_dataset(n: int, L: int = 256, p_range=P_RANGE, config: int = TRAIN_CONFIG, p_index: int = 1,
                 T_max: int = 4096, chunk: int = 16384, rng_seed: int = 5):
    """(counts uint8 [n, L/8, L/8], target float32 [n] = ln(1 + T_dec), T_dec int32 [n],
    p float64 [n]) on the device: p_i uniform in p_range, seeds from the
    workload generator, T_dec measured by the decoder."""
    dev = torch.device("cuda")
    p = np.random.default_rng(rng_seed).uniform(p_range[0], p_range[1], n)
    s = make_seeds(config, p_index, n)
    counts = torch.empty((n, L // 8, L // 8), dtype=torch.uint8, device=dev)
    T = torch.empty(n, dtype=torch.int32, device=dev)
    for a in range(0, n, chunk):
        e = min(n, a + chunk)
        pt = torch.from_numpy(p[a:e]).to(dev)
        st = torch.from_numpy(s[a:e].view(np.int64)).to(dev)
        b.syndrome_counts(L, pt, st, out=counts[a:e])
        Tc, _, _ = b.decode_mixed([(L, e - a)], pt, st, T_max, want_syndrome=False)
        T[a:e] = Tc
    target = torch.log1p(T.double()).float()
    return counts, target, T, p


class HipTrainOps:
    """The training step on the library's kernels: initial parameters,
    loss gradient and Adam update, all in device memory (float32)."""

    def __init__(self, M: int, batch: int, dev):
        self.ws = b.train_workspace(M, batch, dev)
        self.out = (torch.empty(1, dtype=torch.float32, device=dev),
                    torch.empty(b.CNN_PARAMS, dtype=torch.float32, device=dev),
                    torch.empty(batch, dtype=torch.float32, device=dev))
        self.dev = dev

    def init(self, seed):
        params = b.cnn_init(seed)
        return params, torch.zeros_like(params), torch.zeros_like(params)

    def loss_grad(self, c, params, y):
        loss, grad, _ = b.cnn_loss_grad(c, params, y, workspace=self.ws, out=self.out)
        return loss, grad

    def adam(self, params, grad, m, v, step, lr):
        b.cnn_adam_step(params, grad, m, v, step, lr)
        return params, m, v

    def to_device(self, t):
        return t.to(self.dev, dtype=torch.float32).contiguous()


def save_checkpoint(path: str, params, m, v, step: int, epoch: int, gen: torch.Generator, hist):
    """Training state after a whole epoch: master weights and Adam moments
    (as held, float32 on the device), the update count, the epoch count, the
    data-order generator's state and the epoch losses (safetensors: no code
    is executed when it is read back)."""
    from safetensors.torch import save_file
    t = lambda x: torch.as_tensor(x).detach().to("cpu").contiguous()
    save_file({"params": t(params), "m": t(m), "v": t(v), "step": torch.tensor([step], dtype=torch.int64),
               "epoch": torch.tensor([epoch], dtype=torch.int64), "gen_state": gen.get_state(),
               "hist": torch.tensor(hist, dtype=torch.float64)}, path)


def load_checkpoint(path: str):
    from safetensors.torch import load_file
    return load_file(path)


def train(counts, target, epochs: int = 8, batch: int = 256, lr: float = 2e-3, seed: int = 1,
          lr_final: float = 2e-4, log=None, checkpoint: str | None = None, resume: str | None = None,
          stop_after: int | None = None, ops=None):
    """Adam on the mean squared error of ln(1 + T_dec); cosine learning-rate
    decay from lr to lr_final.  Returns (params, history of epoch losses).

    checkpoint: a path rewritten after every epoch with the training state
    (save_checkpoint); resume: such a file to continue from, which gives the
    same result, bit for bit, as the run that was not interrupted (the data
    order comes from the saved generator state, the schedule from the saved
    step count); stop_after: return after this many epochs of the schedule
    (an interrupted run).  ops: the step operations (HipTrainOps by
    default)."""
    n, M = counts.shape[0], counts.shape[-1]
    dev = counts.device
    ops = HipTrainOps(M, batch, dev) if ops is None else ops
    g = torch.Generator(device="cpu").manual_seed(seed)
    steps_per_epoch = n // batch
    total = epochs * steps_per_epoch
    step = 0
    ep0 = 0
    hist = []
    if resume is not None:
        st = load_checkpoint(resume)
        params, m, v = (ops.to_device(st[k]) for k in ("params", "m", "v"))
        step, ep0 = int(st["step"][0]), int(st["epoch"][0])
        g.set_state(st["gen_state"])
        hist = [float(x) for x in st["hist"]]
    else:
        params, m, v = ops.init(seed)
    for ep in range(ep0, epochs if stop_after is None else min(epochs, stop_after)):
        perm = torch.randperm(n, generator=g).to(dev)
        acc = 0.0
        for i in range(steps_per_epoch):
            idx = perm[i * batch:(i + 1) * batch]
            c = counts.index_select(0, idx)
            y = target.index_select(0, idx)
            loss, grad = ops.loss_grad(c, params, y)
            acc = acc + loss
            step += 1
            lr_t = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * step / total))
            params, m, v = ops.adam(params, grad, m, v, step, lr_t)
        hist.append(float(acc.item() if torch.is_tensor(acc) else acc) / steps_per_epoch)
        if log:
            log(f"epoch {ep}: train mse {hist[-1]:.5f}")
        if checkpoint is not None:
            save_checkpoint(checkpoint, params, m, v, step, ep + 1, g, hist)
    return params, hist


def predict(counts, params, chunk: int = 16384):
    return torch.cat([b.cnn_forward(counts[a:a + chunk], params) for a in range(0, counts.shape[0], chunk)])


def ordering_applies(L: int) -> bool:
    """Where a bit-sliced first kernel runs (every band-path size: the whole
    lattice at L = 256, tiles above), the first pass has no depth to choose,
    so groups order the samples (longest predicted first) instead."""
    return L >= 256 and b.get_band_bits(L) > 0


def candidate_policies(pred: np.ndarray, k_first: int, wide: bool = False, order_only: bool = False):
    """Binning policies to try: one bin at the default depth (no use of the
    prediction), and splits at prediction quantiles that give the samples
    predicted shortest one step less and/or the longest one step more.  With
    `wide`, two-group splits take any pair of depths within two steps of
    k_first and three-group splits any three such depths (for batches whose
    decoding times spread widely, e.g. mixed noise strengths).  With
    `order_only` the groups only order the samples: the top decile or half
    first, or 4 or 8 groups of equal size, longest predicted first."""
    if order_only:
        pol = [((), (k_first,))]
        for qq in ([0.9], [0.5], [0.25, 0.5, 0.75], [0.125 * i for i in range(1, 8)]):
            edges = tuple(float(x) for x in np.quantile(pred, qq))
            pol.append((edges, (k_first,) * (len(edges) + 1)))
        return pol
    qs = np.quantile(pred, [0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9])
    k = k_first
    pairs = [(k - 1, k), (k, k + 1)]
    triples = [(k - 1, k, k + 1)]
    if wide:
        pairs = [(a, c) for a in range(k - 2, k + 3) for c in range(a + 1, k + 3)]
        triples = [(a, c, d) for a in range(k - 2, k + 3) for c in range(a + 1, k + 3) for d in range(c + 1, k + 3)]
    pairs = [d for d in pairs if d[0] >= 1]
    triples = [d for d in triples if d[0] >= 1]
    pol = [((), (k,))]
    for a in qs:
        for d in pairs:
            pol.append(((float(a),), d))
    for i, a in enumerate(qs):
        for c in qs[i + 1:]:
            for d in triples:
                pol.append(((float(a), float(c)), d))
    return pol


def plain_decode(L, p, seeds_t, T_max, out=None, workspace=None, stream=None):
    """The decode without a predictor (FIFO): decode_batch for one p,
    decode_mixed with the one class (L, n) for per-sample p."""
    if isinstance(p, (float, int)):
        return b.decode_batch(L, p, seeds_t, T_max, want_syndrome=out is None or out[2] is not None,
                              workspace=workspace, out=out, stream=stream)
    return b.decode_mixed([(L, seeds_t.numel())], p, seeds_t, T_max, want_syndrome=out is None or out[2] is not None,
                          workspace=workspace, out=out, stream=stream)


def best_fifo_depth(L, p, seeds_t, T_max: int = 4096, depths=range(2, 9), reps: int = 3, log=None):
    """First-pass depth that minimises the plain decode's time on a tuning
    batch (later passes at the current k_next).  Leaves the band schedule
    as it found it; returns (depth, {depth: median seconds}).  Where the
    bit-sliced first kernel runs (no first-pass depth to choose) it returns
    the current depth and no timings."""
    k0, kn = b.get_band_schedule(L)
    if ordering_applies(L):
        return k0, {}
    times = {}
    try:
        for k in depths:
            b.set_band_schedule(k, kn, L)
            plain_decode(L, p, seeds_t, T_max)
            ts = []
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plain_decode(L, p, seeds_t, T_max)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            times[k] = float(np.median(ts))
            if log:
                log(f"fifo depth {k}: {times[k] * 1e3:.3f} ms")
    finally:
        b.set_band_schedule(k0, kn, L)
    return min(times, key=times.get), times


def time_policy(L, p, seeds_t, params, policy, T_max, reps: int = 3, ws=None, out=None):
    """Median wall time (s) of decode_learned with this policy on a resident
    seed batch, predictions not copied out (so that a one-group policy times
    the FIFO fallback, which skips the network)."""
    edges, depths = policy
    if out is not None:
        out = (out[0], out[1], out[2], None)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.decode_learned(L, p, seeds_t, params, edges, depths, T_max, want_syndrome=False, workspace=ws, out=out,
                         want_pred=False)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def tune_policy(L, p, seeds_t, params, T_max: int = 4096, k_first: int | None = None, reps: int = 3, log=None,
                wide: bool = False):
    """Time every candidate policy on a tuning batch; returns (best policy,
    its time, time of the single-bin policy, all timings).  p is a number or
    per-sample values."""
    n = seeds_t.numel()
    if k_first is None:
        k_first = b.get_band_schedule(L)[0]
    dev = seeds_t.device
    ws = b.learned_workspace(L, n, dev)
    out = (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev), None,
           torch.empty(n, dtype=torch.float32, device=dev))
    b.decode_learned(L, p, seeds_t, params, (), (k_first,), T_max, want_syndrome=False, workspace=ws, out=out)
    pred = out[3].cpu().numpy()
    res = []
    for pol in candidate_policies(pred, k_first, wide, order_only=ordering_applies(L)):
        t = time_policy(L, p, seeds_t, params, pol, T_max, reps, ws, out)
        res.append((t, pol))
        if log:
            log(f"policy {pol}: {t * 1e3:.3f} ms")
    best = min(res, key=lambda r: r[0])
    return best[1], best[0], res[0][0], res
