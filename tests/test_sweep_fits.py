"""Host logic of the Sec. 7.2 sweeps: crossings, slope and ln L fits recover
the parameters of synthetic data built from their closed forms."""
import math

import numpy as np

from paper_2506_03266_amd import sweep
from paper_2506_03266_amd.workloads import seeds


def test_crossing_of_power_laws():
    # p_log = C (p/p_c)^(gamma L) for two sizes crosses exactly at p_c when C is shared.
    p_c, g, C = 0.0731, 0.2, 0.4
    ps = [0.06, 0.065, 0.07, 0.075, 0.08, 0.085]
    f = {L: [C * (p / p_c) ** (g * L) for p in ps] for L in (16, 32)}
    pc = sweep.crossing(ps, f[16], f[32])
    assert abs(pc - p_c) < 1e-12, pc
    assert sweep.crossing(ps, f[32], f[16]) is None      # never goes from below to above
    # With a zero count the interpolation falls back to linear in p.
    assert abs(sweep.crossing([0.1, 0.2], [0.5, 0.5], [0.0, 0.6]) - (0.1 + 0.1 * 0.5 / 0.6)) < 1e-15


def test_slope_gamma_inverts_the_scaling_form():
    p_c, g, C = 0.073, 0.21, 0.3
    for p in (0.03, 0.05):
        f = {L: C * (p / p_c) ** (g * L) for L in (8, 20)}
        assert abs(sweep.slope_gamma(8, f[8], 20, f[20], p, p_c) - g) < 1e-12


def test_fit_log_recovers_line():
    Ls = [16, 32, 64, 128, 256]
    A, B = 1.37, -0.8
    T = [A * math.log(L) + B for L in Ls]
    a, b = sweep.fit_log(Ls, T, [1, 2, 3, 4, 5])
    assert abs(a - A) < 1e-12 and abs(b - B) < 1e-12


def test_mean_and_error_from_sums():
    T = np.array([3, 4, 4, 5, 7, 4096])
    flags = np.array([0, 0, 1, 0, 0, 3])
    done = (flags & 2) == 0
    r = dict(n=6, timeouts=int((~done).sum()), fails=int((flags & 1).sum()),
             T_sum=int(T[done].sum()), T_sq=int((T[done] ** 2).sum()))
    m, e = sweep.mean_T(r)
    assert m == T[done].mean()
    assert abs(e - T[done].std() / math.sqrt(done.sum())) < 1e-12
    assert sweep.p_log(r) == 2 / 6
    assert sweep.mean_T(dict(n=2, timeouts=2, T_sum=0, T_sq=0))[0] != sweep.mean_T(dict(n=2, timeouts=2, T_sum=0, T_sq=0))[0]


def test_sweep_seeds_are_disjoint_from_the_workloads():
    a = set(sweep.seed_block(256, 3, 1000).tolist())
    assert len(a) == 1000
    for cfg in (1, 2, 3, 4, 5):
        for pi in range(4):
            assert not a & set(seeds(cfg, pi, 1000).tolist())
    assert not a & set(sweep.seed_block(512, 3, 1000).tolist())
    assert not a & set(sweep.seed_block(256, 4, 1000).tolist())


def test_summary_of_synthetic_counts():
    p_c, g, C = 0.073, 0.2, 0.4
    res = dict(threshold=[], slope=[], tdec=[])
    ps = [0.065, 0.07, 0.075, 0.08]
    n = 10 ** 9
    for L in (16, 32, 64):
        for p in ps:
            res["threshold"].append(dict(L=L, p=p, n=n, fails=round(n * C * (p / p_c) ** (g * L)), timeouts=0,
                                         T_sum=0, T_sq=0))
    for L in (8, 16):
        res["slope"].append(dict(L=L, p=0.04, n=n, fails=round(n * C * (0.04 / p_c) ** (g * L)), timeouts=0,
                                 T_sum=0, T_sq=0))
    for L in (16, 64, 256, 1024):
        m = 2.0 * math.log(L) + 1.0 - (0.5 if L < 64 else 0.0)
        k = 1000
        res["tdec"].append(dict(L=L, p=0.01, n=k, fails=0, timeouts=0, T_sum=m * k, T_sq=(m * m + 1) * k))
    s = sweep.summarize(res)
    for c in s["crossings"].values():
        assert abs(c - p_c) < 1e-4, s["crossings"]
    (gam,) = s["gamma"].values()
    assert abs(gam - g) < 0.01, gam
    fit = s["tdec_fit"]["0.01"]
    assert abs(fit["A"] - 2.0) < 1e-9 and abs(fit["B"] - 1.0) < 1e-9 and fit["max_abs_resid"] < 1e-9
    # No timeouts in these counts: both crossing tables agree.
    assert s["crossings"] == s["crossings_decoded_only"]
