"""Limited-memory variant of the rule on the GPU (messages truncated at
m_max, random moves every u steps) against the oracle, bit for bit: seeded
decodes on both decoder paths and both band drivers, explicit errors, and the
full state after a fixed number of steps."""
import numpy as np
import pytest
import torch

from paper_2506_03266_amd.workloads import seeds

pytestmark = pytest.mark.gpu

RULES = [(2, 0), (3, 4), (0, 3), (6, 1), (1, 2), (40, 5)]


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_03266_amd.binding as b
    b.lib()
    return b


def _np(t):
    return t.cpu().numpy()


def compare(tag, T, F, S, ref):
    T, F = _np(T), _np(F)
    bad = np.nonzero((T != ref["T_dec"]) | (F != ref["flags"]))[0]
    assert bad.size == 0, f"{tag}: {bad.size} mismatches, first {bad[:5]} gpu T={T[bad[:5]]} F={F[bad[:5]]} " \
                          f"oracle T={ref['T_dec'][bad[:5]]} F={ref['flags'][bad[:5]]}"
    if S is not None:
        rows = np.nonzero(np.any(_np(S).view(np.uint32) != ref["sigma_words"], axis=1))[0]
        assert rows.size == 0, f"{tag}: final syndrome differs for samples {rows[:5]}"


@pytest.mark.parametrize("m_max,u", RULES)
@pytest.mark.parametrize("L,p,n", [(8, 0.06, 300), (12, 0.05, 200), (31, 0.04, 64), (64, 0.03, 24), (128, 0.02, 6)])
def test_resident_rule_matches_oracle(gpu, orc, L, p, n, m_max, u):
    s = seeds(110, 100 * L + 10 * m_max + u, n)
    T, F, S = gpu.decode_rule(L, p, s, 150, m_max=m_max, u=u)
    ref = orc.decode_seeds(L, p, s, 150, threads=16, m_max=m_max, u=u)
    compare(f"L={L} m_max={m_max} u={u}", T, F, S, ref)


def test_plain_rule_through_the_variant_entry(gpu):
    """m_max = u = 0 through mpd_decode_rule equals mpd_decode_batch."""
    for L, n in ((16, 500), (256, 16)):
        s = seeds(111, L, n)
        a = gpu.decode_batch(L, 0.03, s, 512)
        b = gpu.decode_rule(L, 0.03, s, 512, m_max=0, u=0)
        for x, y in zip(a, b):
            assert torch.equal(x, y), L


@pytest.mark.parametrize("m_max,u", [(2, 0), (3, 2), (0, 1), (5, 3)])
@pytest.mark.parametrize("L", [7, 16])
def test_run_steps_rule_state(gpu, orc, L, m_max, u):
    """Registers (distance form, truncated ones 0), syndrome and windings after
    exactly t steps, from explicit errors with per-pattern move seeds."""
    p = 0.08
    ms = seeds(112, 10 * L + m_max, 4)
    exs, eys = zip(*[orc.noise(L, p, int(x)) for x in ms])
    links = orc.links_from_chains(L, np.stack(exs), np.stack(eys))
    for t in (1, 2, 3, 5, 8):
        M, S, W = gpu.run_steps(L, links, t, m_max=m_max, u=u, move_seeds=ms)
        M, S, W = _np(M), _np(S).view(np.uint32), _np(W)
        for k in range(len(ms)):
            m, sig, (cx, cy), _ = orc.run_steps(L, exs[k], eys[k], t, m_max=m_max, u=u, seed=int(ms[k]))
            assert np.array_equal(M[k].astype(np.int64), m.astype(np.int64)), (t, k)
            assert np.array_equal(S[k], orc.pack_bits((sig == -1).reshape(-1))), (t, k)
            wx = int(cx[:, L - 1].sum() % 2) | (int(cy[L - 1, :].sum() % 2) << 1)
            assert (int(W[k]) >> 2) == wx, (t, k)


def test_pairs_and_m_max_explicit_errors(gpu, orc):
    """Straight pairs at distance d decode with m_max = d and stay stuck with
    m_max = d - 1, on the GPU as in the oracle; random explicit errors with
    move seeds agree too."""
    L = 16
    exs, eys, cases = [], [], []
    for d in range(2, 8):
        ex = np.zeros((L, L), np.uint8)
        ex[2, 2:2 + d] = 1
        for mm in (d, d - 1):
            exs.append(ex)
            eys.append(np.zeros((L, L), np.uint8))
            cases.append(mm)
    links = orc.links_from_chains(L, np.stack(exs), np.stack(eys))
    for i, mm in enumerate(cases):
        T, F, S = gpu.decode_errors(L, links[i:i + 1], 64, m_max=mm)
        ref = orc.decode_links(L, links[i:i + 1], 64, m_max=mm)
        compare(f"pair m_max={mm}", T, F, S, ref)
    ms = seeds(113, 0, 40)
    rnd = [orc.noise(L, 0.07, int(x)) for x in ms]
    links = orc.links_from_chains(L, np.stack([a for a, _ in rnd]), np.stack([b for _, b in rnd]))
    T, F, S = gpu.decode_errors(L, links, 300, m_max=3, u=3, move_seeds=ms)
    compare("random chains", T, F, S, orc.decode_links(L, links, 300, m_max=3, u=3, seeds=ms))


@pytest.mark.parametrize("driver", ["host", "device"])
@pytest.mark.parametrize("L,p,n,T_max,m_max,u", [(256, 0.04, 12, 40, 3, 3), (256, 0.06, 8, 64, 0, 2),
                                                  (272, 0.03, 6, 48, 5, 0), (512, 0.05, 3, 24, 2, 5),
                                                  (256, 0.02, 100, 40, 4, 7)])
def test_band_rule_matches_oracle(gpu, orc, driver, L, p, n, T_max, m_max, u):
    """Band path: random-move steps and truncation across pass boundaries,
    2D tiles, small and full-size regions, both drivers."""
    gpu.set_band_driver(gpu.BAND_DRIVER_HOST if driver == "host" else gpu.BAND_DRIVER_DEVICE)
    try:
        s = seeds(114, L + T_max + u, n)
        T, F, S = gpu.decode_rule(L, p, s, T_max, m_max=m_max, u=u)
    finally:
        gpu.set_band_driver(gpu.BAND_DRIVER_AUTO)
    ref = orc.decode_seeds(L, p, s, T_max, threads=16, m_max=m_max, u=u)
    compare(f"L={L} m_max={m_max} u={u} {driver}", T, F, S, ref)
