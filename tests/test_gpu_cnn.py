"""GPU kernels of the decode-time predictor and the learned-schedule decode
(through the C ABI) against the CPU oracles.

Block counts, initial parameters and every decode result are compared
exactly; the network's floating-point outputs within the tolerances below
(float32 accumulation in a different order than the oracle's float64 sums,
with bfloat16 rounding at the same points on both sides):
  forward  |pred_gpu - pred_oracle| <= 1e-2 * max(1, |pred_oracle|)
  gradient cosine >= 0.999 and relative L2 error <= 2e-2
  Adam     parameters within 1e-6 relative (+ 1e-9 absolute)
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import cnn_oracle as co
from paper_2506_03266_amd.workloads import seeds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_03266_amd.binding as b
    b.lib()
    return b


def realistic_counts(seed, n, M, lam=2.6):
    """Block counts like an L = 8M lattice near p = 0.01 (Poisson, with a few dense blocks)."""
    r = np.random.default_rng(seed)
    c = r.poisson(lam, size=(n, M, M))
    hot = r.random((n, M, M)) < 0.01
    c[hot] += r.integers(4, 12, size=hot.sum())
    return np.minimum(c, 64).astype(np.uint8)


def trained_like_params(seed):
    """Initial parameters plus a perturbation, with a head that mixes channels."""
    p = co.init_params(seed, oracle.philox4x32_10).astype(np.float64)
    r = np.random.default_rng(seed)
    p += r.standard_normal(p.size) * 0.02
    p[co.OFF_BL] = 1.5
    return p.astype(np.float32)


@pytest.mark.parametrize("L", [16, 64, 256, 272, 1024])
def test_syndrome_counts(gpu, orc, L):
    n = 6 if L < 1024 else 2
    s = seeds(50, L, n)
    p = 0.03
    got = gpu.syndrome_counts(L, p, s).cpu().numpy()
    for i in range(n):
        ex, ey = orc.noise(L, p, int(s[i]))
        want = co.block_counts(orc.syndrome_of(L, ex, ey), 8)
        assert np.array_equal(got[i], want), (L, i)


def test_syndrome_counts_per_sample_p(gpu, orc):
    L, n = 256, 8
    s = seeds(51, 0, n)
    ps = np.linspace(0.0, 0.05, n)
    got = gpu.syndrome_counts(L, ps, s).cpu().numpy()
    for i in range(n):
        ex, ey = orc.noise(L, ps[i], int(s[i]))
        assert np.array_equal(got[i], co.block_counts(orc.syndrome_of(L, ex, ey), 8)), i
    assert got[0].sum() == 0


def test_init_matches_oracle(gpu):
    for seed in (0, 12345, 2**40 + 7):
        got = gpu.cnn_init(seed).cpu().numpy()
        want = co.init_params(seed, oracle.philox4x32_10)
        assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), seed


@pytest.mark.parametrize("M,n", [(32, 24), (8, 16), (5, 8), (2, 4), (64, 4), (34, 3), (128, 2)])
def test_forward_matches_oracle(gpu, M, n):
    """Whole-map kernel (M <= 32, incl. odd and tiny maps) and tiled kernel
    (M = 64, ragged M = 34, M = 128 as for L = 1024)."""
    counts = realistic_counts(M * 100 + n, n, M)
    params = trained_like_params(M)
    dev = torch.device("cuda")
    pred, feat, amax = gpu.cnn_forward(torch.from_numpy(counts).to(dev), torch.from_numpy(params).to(dev),
                                       want_feat=True)
    ref = co.forward(counts, params, "bf16")
    want = ref["pred"].detach().numpy()
    got = pred.cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - want) <= 1e-2 * np.maximum(1.0, np.abs(want))), (got, want)
    wf = ref["feat"].detach().numpy()
    gf = feat.cpu().numpy()
    assert np.all(np.abs(gf - wf) <= 1e-2 * np.maximum(1.0, np.abs(wf)))
    agree = (amax.cpu().numpy() == ref["argmax"]).mean()
    assert agree >= 0.9, agree


def test_forward_translation_invariance(gpu):
    """Circular convolutions and a global maximum: shifting the map leaves the
    predictions unchanged (exactly on the whole-map kernel up to summation
    order, so within float32 rounding)."""
    counts = realistic_counts(7, 4, 32)
    params = torch.from_numpy(trained_like_params(3)).cuda()
    base = gpu.cnn_forward(torch.from_numpy(counts).cuda(), params).cpu().numpy()
    sh = np.roll(counts, (5, 11), axis=(1, 2))
    got = gpu.cnn_forward(torch.from_numpy(np.ascontiguousarray(sh)).cuda(), params).cpu().numpy()
    assert np.allclose(got, base, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("M", [64, 34])
def test_forward_translation_invariance_tiled(gpu, M):
    """Wider maps run in 32 x 32 tiles from frames with a halo: a circular
    shift moves content across tile edges and the wrap seam (ragged at
    M = 34, where the last tile wraps onto the first), yet every position's
    value is computed from the same neighbourhood in the same order, so
    the predictions agree to float32 rounding."""
    counts = realistic_counts(11 + M, 3, M)
    params = torch.from_numpy(trained_like_params(5)).cuda()
    base = gpu.cnn_forward(torch.from_numpy(counts).cuda(), params).cpu().numpy()
    for dy, dx in ((5, 11), (17, 3), (M - 1, 29)):
        sh = np.ascontiguousarray(np.roll(counts, (dy, dx), axis=(1, 2)))
        got = gpu.cnn_forward(torch.from_numpy(sh).cuda(), params).cpu().numpy()
        assert np.allclose(got, base, rtol=1e-5, atol=1e-5), (dy, dx, got, base)


@pytest.mark.parametrize("M,n", [(32, 16), (8, 32), (8, 21)])
def test_gradient_matches_oracle(gpu, M, n):
    counts = realistic_counts(M + 1, n, M)
    params = trained_like_params(M + 2)
    target = np.log1p(np.random.default_rng(M).integers(2, 8, size=n)).astype(np.float32)
    dev = torch.device("cuda")
    loss, grad, pred = gpu.cnn_loss_grad(torch.from_numpy(counts).to(dev), torch.from_numpy(params).to(dev),
                                         torch.from_numpy(target).to(dev))
    wl, wg, ref = co.loss_and_grad(counts, params, target, "bf16")
    g = grad.cpu().numpy().astype(np.float64)
    cos = g @ wg / (np.linalg.norm(g) * np.linalg.norm(wg))
    rel = np.linalg.norm(g - wg) / np.linalg.norm(wg)
    assert cos >= 0.999 and rel <= 2e-2, (cos, rel)
    assert float(loss.item()) == pytest.approx(wl, rel=1e-2)
    # every layer's block individually
    for lo, hi in ((co.OFF_W1, co.OFF_W2), (co.OFF_W2, co.OFF_W3), (co.OFF_W3, co.OFF_W4), (co.OFF_W4, co.OFF_WL),
                   (co.OFF_WL, co.CNN_PARAMS)):
        a, w = g[lo:hi], wg[lo:hi]
        if np.linalg.norm(w) > 0:
            assert np.linalg.norm(a - w) / np.linalg.norm(w) <= 5e-2, (lo, hi)


def test_adam_matches_oracle(gpu):
    r = np.random.default_rng(3)
    p0 = r.standard_normal(co.CNN_PARAMS).astype(np.float32)
    dev = torch.device("cuda")
    P = torch.from_numpy(p0.copy()).to(dev)
    m = torch.zeros_like(P)
    v = torch.zeros_like(P)
    pr, mr, vr = p0.astype(np.float64), np.zeros(co.CNN_PARAMS), np.zeros(co.CNN_PARAMS)
    for t in range(1, 4):
        g = (r.standard_normal(co.CNN_PARAMS) * 10.0 ** r.integers(-6, 1, co.CNN_PARAMS)).astype(np.float32)
        gpu.cnn_adam_step(P, torch.from_numpy(g).to(dev), m, v, t, 1e-3)
        pr, mr, vr = co.adam_step(pr, g, mr, vr, t, 1e-3)
    got = P.cpu().numpy().astype(np.float64)
    assert np.allclose(got, pr, rtol=1e-6, atol=1e-9)


def test_training_lowers_loss(gpu):
    """A few hundred Adam steps on decoder-labelled L = 256 samples lower the
    training loss well below that of the initial network."""
    from paper_2506_03266_amd import learned
    counts, target, T, _ = learned.make_dataset(8192, p_range=(0.005, 0.02), p_index=9)
    params, hist = learned.train(counts, target, epochs=4, batch=256)
    assert hist[-1] < 0.5 * hist[0], hist
    assert np.isfinite(params.cpu().numpy()).all()


POLICIES = [((), (4,)), ((), (1,)), ((1.4,), (3, 4)), ((1.0, 1.6), (2, 5, 6)), ((-1e9, 1e9), (3, 6, 1)),
            ((0.0,), (7, 2))]


@pytest.mark.parametrize("policy", POLICIES)
def test_learned_decode_equals_plain(gpu, orc, policy):
    """Any binning policy returns exactly the plain decode's results (and the
    oracle's), at L = 256."""
    L, p, n = 256, 0.02, 192
    s = seeds(52, 0, n)
    params = torch.from_numpy(trained_like_params(9)).cuda()
    T0, F0, S0 = gpu.decode_batch(L, p, s, 4096)
    edges, depths = policy
    T1, F1, S1, pred = gpu.decode_learned(L, p, s, params, edges, depths, 4096)
    assert np.array_equal(T0.cpu().numpy(), T1.cpu().numpy())
    assert np.array_equal(F0.cpu().numpy(), F1.cpu().numpy())
    assert np.array_equal(S0.cpu().numpy(), S1.cpu().numpy())
    pick = np.arange(0, n, 23)
    ref = orc.decode_seeds(L, p, s[pick], 4096, threads=8)
    assert np.array_equal(T1.cpu().numpy()[pick], ref["T_dec"])
    assert np.array_equal(F1.cpu().numpy()[pick], ref["flags"])
    assert np.isfinite(pred.cpu().numpy()).all()


@pytest.mark.parametrize("k_bits", [0, 3, 10])
@pytest.mark.parametrize("p", [0.01, 0.04])
def test_learned_order_equals_plain(gpu, orc, k_bits, p):
    """At L = 256 the groups order the bit-sliced kernel's samples (longest
    predicted first; the kernel reads the syndrome the noise kernel drew),
    or, with the bit-sliced kernel off, set first-pass depths: either way
    the results are the plain decode's, and the oracle's."""
    L, n = 256, 160
    s = seeds(54, int(p * 100) * 16 + k_bits, n)
    params = torch.from_numpy(trained_like_params(11)).cuda()
    old = gpu.get_band_bits(L)
    gpu.set_band_bits(k_bits, L)
    try:
        T0, F0, S0 = gpu.decode_batch(L, p, s, 4096)
        pr = gpu.cnn_forward(gpu.syndrome_counts(L, p, s), params).cpu().numpy()
        edges = tuple(float(x) for x in np.quantile(pr, [0.25, 0.5, 0.75]))
        T1, F1, S1, _ = gpu.decode_learned(L, p, s, params, edges, (2, 3, 4, 5), 4096)
    finally:
        gpu.set_band_bits(old, L)
    ref = orc.decode_seeds(L, p, s, 4096, threads=16)
    for T, F, S in ((T0, F0, S0), (T1, F1, S1)):
        assert np.array_equal(T.cpu().numpy(), ref["T_dec"])
        assert np.array_equal(F.cpu().numpy(), ref["flags"])
        assert np.array_equal(S.cpu().numpy().view(np.uint32), ref["sigma_words"])


@pytest.mark.parametrize("L,p,n,T_max", [(256, 0.07, 8, 5), (256, 0.06, 8, 0), (512, 0.02, 4, 64),
                                         (1024, 0.01, 2, 64)])
def test_learned_decode_budgets_and_sizes(gpu, orc, L, p, n, T_max):
    """Bins deeper than T_max, timeouts, and tiled lattices (L = 512, 1024:
    the predictor's tiled kernel), against the oracle."""
    s = seeds(53, L + T_max, n)
    params = torch.from_numpy(trained_like_params(10)).cuda()
    med = float(np.median(gpu.cnn_forward(gpu.syndrome_counts(L, p, s), params).cpu().numpy()))
    T, F, S, pred = gpu.decode_learned(L, p, s, params, (med,), (2, 6), T_max)
    ref = orc.decode_seeds(L, p, s, T_max, threads=8)
    assert np.array_equal(T.cpu().numpy(), ref["T_dec"])
    assert np.array_equal(F.cpu().numpy(), ref["flags"])
    assert np.array_equal(S.cpu().numpy().view(np.uint32), ref["sigma_words"])


def test_config5_L1024_fifo_and_learned(gpu, orc):
    """The L = 1024, p = 0.01 evaluation of the learned-scheduling workload on
    64 samples: the plain (FIFO) decode and a three-group learned decode
    (the predictor's tiled kernel, groups with first passes of 2, 4 and 6
    steps) both equal the oracle on every sample."""
    L, p, n = 1024, 0.01, 64
    s = seeds(5, 201, n)
    params = torch.from_numpy(trained_like_params(14)).cuda()
    pred = gpu.cnn_forward(gpu.syndrome_counts(L, p, s), params).cpu().numpy()
    edges = tuple(float(v) for v in np.quantile(pred, [1 / 3, 2 / 3]))
    ref = orc.decode_seeds(L, p, s, 4096, threads=16)
    T0, F0, S0 = gpu.decode_batch(L, p, s, 4096)
    T1, F1, S1, _ = gpu.decode_learned(L, p, s, params, edges, (2, 4, 6), 4096)
    for tag, (T, F, S) in (("fifo", (T0, F0, S0)), ("learned", (T1, F1, S1))):
        assert np.array_equal(T.cpu().numpy(), ref["T_dec"]), tag
        assert np.array_equal(F.cpu().numpy(), ref["flags"]), tag
        assert np.array_equal(S.cpu().numpy().reshape(n, -1).view(np.uint32), ref["sigma_words"]), tag


@pytest.mark.parametrize("policy", POLICIES[:4])
def test_learned_decode_per_sample_p(gpu, orc, policy):
    """Per-sample noise strengths: any policy returns exactly what the plain
    mixed decode returns for the one class (L, n), and the oracle's results."""
    L, n = 256, 160
    s = seeds(58, 0, n)
    p = np.random.default_rng(58).uniform(0.002, 0.05, n)
    params = torch.from_numpy(trained_like_params(12)).cuda()
    T0, F0, S0 = gpu.decode_mixed([(L, n)], p, s, 4096)
    T1, F1, S1, pred = gpu.decode_learned(L, p, s, params, policy[0], policy[1], 4096)
    assert torch.equal(T0, T1) and torch.equal(F0, F1) and torch.equal(S0, S1.reshape(-1))
    pick = np.arange(0, n, 19)
    ref = orc.decode_seeds(L, p[pick], s[pick], 4096, threads=8)
    assert np.array_equal(T1.cpu().numpy()[pick], ref["T_dec"])
    assert np.array_equal(F1.cpu().numpy()[pick], ref["flags"])
    assert np.array_equal(S1.cpu().numpy()[pick].view(np.uint32), ref["sigma_words"])
    assert np.isfinite(pred.cpu().numpy()).all()


@pytest.mark.parametrize("depth,per_sample", [(4, False), (1, False), (5, True)])
def test_one_group_without_predictions_is_plain(gpu, depth, per_sample):
    """A one-group policy with no predictions asked for skips the network
    (the FIFO fallback) and returns the plain decode's results, also when
    the schedule's first-pass depth differs from the group's."""
    L, n = 256, 96
    s = seeds(59, depth, n)
    p = np.random.default_rng(59).uniform(0.005, 0.03, n) if per_sample else 0.02
    params = torch.from_numpy(trained_like_params(13)).cuda()
    if per_sample:
        T0, F0, S0 = gpu.decode_mixed([(L, n)], p, s, 4096)
    else:
        T0, F0, S0 = gpu.decode_batch(L, p, s, 4096)
    T1, F1, S1, pred = gpu.decode_learned(L, p, s, params, (), (depth,), 4096, want_pred=False)
    assert pred is None
    assert torch.equal(T0, T1) and torch.equal(F0, F1) and torch.equal(S0.reshape(-1), S1.reshape(-1))


@pytest.fixture(scope="module")
def trained(gpu):
    """The predictor as the learned schedule uses it: 200000 decoder-labelled
    L = 256 samples with p ~ U[0.005, 0.02], 6 epochs."""
    from paper_2506_03266_amd import learned
    counts, target, _, _ = learned.make_dataset(200000)
    params, hist = learned.train(counts, target, epochs=6)
    return params, target


def test_training_labels_relabelled_by_oracle(gpu, orc, trained):
    """2% of the 200000 training labels (every 50th sample of the data set
    the predictor is trained on) decoded again by the CPU oracle: the same
    T_dec for every one."""
    from paper_2506_03266_amd import learned
    _, target = trained
    n = target.numel()
    p = np.random.default_rng(5).uniform(learned.P_RANGE[0], learned.P_RANGE[1], n)  # make_dataset's draw
    s = learned.make_seeds(learned.TRAIN_CONFIG, 1, n)
    pick = np.arange(0, n, 50)
    T = np.rint(np.expm1(target.cpu().numpy().astype(np.float64))).astype(np.int64)[pick]
    ref = orc.decode_seeds(256, p[pick], s[pick], 4096, threads=16)
    assert pick.size == n // 50
    bad = np.nonzero(T != ref["T_dec"])[0]
    assert bad.size == 0, f"{bad.size} labels differ, first at sample {pick[bad[:5]]}: {T[bad[:5]]} vs {ref['T_dec'][bad[:5]]}"


def _time_batches(batches, fn):
    import time
    fn(*batches[0])
    torch.cuda.synchronize()
    t = time.perf_counter()
    outs = [fn(*x) for x in batches[1:]]
    torch.cuda.synchronize()
    return (time.perf_counter() - t) / (len(batches) - 1), outs


def test_learned_vs_fifo_L256(gpu, trained, capsys):
    """What the trained network gains (or loses) over plain FIFO batching at
    L = 256, p = 0.01 (4096 samples per batch), end to end (noise, inference,
    binning, decoding).  Picks the binning policy by timing on a tuning
    batch (a one-group policy is the FIFO fallback, without inference),
    then times both on fresh batches.  Results must be identical; the
    measured ratio is reported, and the network must beat the best constant
    predictor of the training labels on the evaluation samples."""
    from paper_2506_03266_amd import learned
    params, target = trained
    L, p, n = 256, 0.01, 4096
    tune = torch.from_numpy(seeds(3, 201, n).view(np.int64)).cuda()
    policy, _, _, _ = learned.tune_policy(L, p, tune, params, reps=2)
    batches = [torch.from_numpy(seeds(3, 210 + i, n).view(np.int64)).cuda() for i in range(6)]
    ws = gpu.alloc_workspace(L, n)
    lws = gpu.learned_workspace(L, n)

    def run(fn):
        return _time_batches([(x,) for x in batches], fn)

    t_fifo, o_fifo = run(lambda s: gpu.decode_batch(L, p, s, 4096, workspace=ws))
    t_lrn, o_lrn = run(lambda s: gpu.decode_learned(L, p, s, params, policy[0], policy[1], 4096, workspace=lws,
                                                    want_pred=False))
    for a, c in zip(o_fifo, o_lrn):
        for x, y in zip(a[:3], c[:3]):
            assert torch.equal(x, y)
    T = torch.cat([o[0] for o in o_fifo]).double()
    y = torch.log1p(T)
    pred = torch.cat([gpu.cnn_forward(gpu.syndrome_counts(L, p, s), params) for s in batches[1:]]).double()
    mse_net = float(((pred - y) ** 2).mean())
    mse_const = float(((float(target.double().mean()) - y) ** 2).mean())
    with capsys.disabled():
        print(f"\nlearned vs FIFO at L=256 p=0.01: fifo {n / t_fifo:.4g} samples/s, learned {n / t_lrn:.4g} "
              f"samples/s (ratio {t_fifo / t_lrn:.3f}), policy {policy}, mse net {mse_net:.4f} "
              f"vs training-mean constant {mse_const:.4f}")
    assert mse_net < mse_const
    assert t_lrn < 1.5 * t_fifo


def test_learned_vs_fifo_mixed_p(gpu, trained, capsys):
    """The same comparison when every sample draws its own p from the
    training range U[0.005, 0.02] (L = 256, 4096 per batch): decoding times
    spread from 2 to about 10 steps and the prediction separates them.  FIFO
    runs at its own fastest first-pass depth for these batches; results must
    be identical and the measured ratio is reported."""
    from paper_2506_03266_amd import learned
    params, _ = trained
    L, n = 256, 4096
    rng = np.random.default_rng(7)
    pr = learned.P_RANGE
    tune_s = torch.from_numpy(seeds(3, 239, n).view(np.int64)).cuda()
    tune_p = torch.from_numpy(rng.uniform(pr[0], pr[1], n)).cuda()
    k0, kn = gpu.get_band_schedule(L)
    k_fifo, _ = learned.best_fifo_depth(L, tune_p, tune_s, reps=2)
    batches = [(torch.from_numpy(seeds(3, 240 + i, n).view(np.int64)).cuda(),
                torch.from_numpy(rng.uniform(pr[0], pr[1], n)).cuda()) for i in range(6)]
    ws = gpu.mixed_workspace([(L, n)])
    lws = gpu.learned_workspace(L, n)
    gpu.set_band_schedule(k_fifo, kn, L)
    try:
        policy, _, _, _ = learned.tune_policy(L, tune_p, tune_s, params, k_first=k_fifo, reps=2, wide=True)
        t_fifo, o_fifo = _time_batches(batches, lambda s, p: gpu.decode_mixed([(L, n)], p, s, 4096, workspace=ws))
        t_lrn, o_lrn = _time_batches(batches, lambda s, p: gpu.decode_learned(L, p, s, params, policy[0],
                                                                                 policy[1], 4096, workspace=lws,
                                                                                 want_pred=False))
    finally:
        gpu.set_band_schedule(k0, kn, L)
    for a, c in zip(o_fifo, o_lrn):
        assert torch.equal(a[0], c[0]) and torch.equal(a[1], c[1]) and torch.equal(a[2], c[2].reshape(-1))
    T = torch.cat([o[0] for o in o_fifo]).cpu().numpy()
    pred = torch.cat([gpu.cnn_forward(gpu.syndrome_counts(L, p, s), params) for s, p in batches[1:]]).cpu().numpy()
    rho = float(np.corrcoef(np.argsort(np.argsort(pred)), np.argsort(np.argsort(T)))[0, 1])
    with capsys.disabled():
        print(f"\nlearned vs FIFO at L=256, p ~ U[0.005, 0.02]: fifo {n / t_fifo:.4g} samples/s (first pass "
              f"{k_fifo}), learned {n / t_lrn:.4g} samples/s (ratio {t_fifo / t_lrn:.3f}), policy {policy}, "
              f"rank correlation {rho:.3f}")
    assert rho > 0.5
    assert t_lrn < 1.5 * t_fifo


@pytest.mark.parametrize("depths,T_max", [((2, 6), 5), ((1, 7), 6), ((3, 5), 7), ((1, 2, 9), 9)])
def test_learned_timeouts_in_different_passes(gpu, orc, depths, T_max):
    """Groups of different first-pass depth reach the step budget in different
    passes, so their final states sit in different ping-pong buffers: the
    exported final syndromes of the timeouts must still be the oracle's."""
    L, p, n = 256, 0.08, 9
    s = seeds(57, 10 * T_max + len(depths), n)
    params = torch.from_numpy(trained_like_params(11)).cuda()
    pr = np.sort(gpu.cnn_forward(gpu.syndrome_counts(L, p, s), params).cpu().numpy())
    edges = tuple(float(e) for e in pr[np.linspace(0, n, len(depths) + 1).astype(int)[1:-1]])
    T, F, S, _ = gpu.decode_learned(L, p, s, params, edges, depths, T_max)
    ref = orc.decode_seeds(L, p, s, T_max, threads=8)
    assert np.array_equal(T.cpu().numpy(), ref["T_dec"])
    assert np.array_equal(F.cpu().numpy(), ref["flags"])
    assert np.array_equal(S.cpu().numpy().view(np.uint32), ref["sigma_words"])
    assert (F.cpu().numpy() & 2).sum() > 0  # some timeouts


def test_training_resume_bitwise(gpu, tmp_path):
    """Predictor training on the library's kernels, interrupted after one
    epoch and resumed from its checkpoint, ends bit for bit where the
    uninterrupted run ends (deterministic gradient reduction, saved
    moments, step count and data order)."""
    import os
    from paper_2506_03266_amd import learned
    n = 1024
    counts = gpu.syndrome_counts(256, 0.01, seeds(57, 0, n))
    target = (torch.from_numpy(np.random.default_rng(57).uniform(1.0, 2.0, n)).float()).cuda()
    kw = dict(epochs=2, batch=256, seed=2)
    p_full, h_full = learned.train(counts, target, **kw)
    ck = os.path.join(tmp_path, "train.safetensors")
    p_cut, _ = learned.train(counts, target, checkpoint=ck, stop_after=1, **kw)
    p_res, h_res = learned.train(counts, target, resume=ck, **kw)
    assert torch.equal(p_res, p_full)
    assert h_res == h_full
    assert not torch.equal(p_cut, p_full)
