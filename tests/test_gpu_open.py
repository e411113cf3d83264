"""Open lattice (rough left / right columns, smooth top / bottom rows) on the
GPU against the oracle, bit for bit: seeded decodes, explicit errors and the
full state after a fixed number of steps."""
import numpy as np
import pytest
import torch

from paper_2506_03266_amd.workloads import seeds

pytestmark = pytest.mark.gpu


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


@pytest.mark.parametrize("L,p,n", [(3, 0.1, 500), (4, 0.08, 500), (5, 0.1, 500), (8, 0.06, 400), (12, 0.09, 300),
                                   (16, 0.05, 300), (31, 0.07, 100), (64, 0.04, 40), (100, 0.06, 6), (128, 0.03, 6)])
def test_open_matches_oracle(gpu, orc, L, p, n):
    s = seeds(130, L, n)
    T, F, S = gpu.decode_open(L, p, s, 400)
    ref = orc.decode_seeds(L, p, s, 400, threads=16, open_bc=True)
    compare(f"open L={L} p={p}", T, F, S, ref)
    if L <= 31:
        assert int((_np(F) & 1).sum()) > 0  # failures occur and are flagged alike


def test_open_explicit_errors(gpu, orc):
    """Absorption at both boundaries, the logical row, ignored links, the
    balanced pair of L = 4, and random chains that include links which do
    not exist on the open lattice."""
    cases = []
    L = 22
    for d in range(1, 10):
        ex = np.zeros((L, L), np.uint8)
        ex[7, :d] = 1
        cases.append((ex, np.zeros((L, L), np.uint8)))
        ex = np.zeros((L, L), np.uint8)
        ex[7, L - 1 - d:L - 1] = 1
        cases.append((ex, np.zeros((L, L), np.uint8)))
    ex = np.zeros((L, L), np.uint8)
    ex[5, :] = 1  # includes the x-link of column L-1, which does not exist
    ey = np.zeros((L, L), np.uint8)
    ey[4, 0] = ey[9, L - 1] = ey[L - 1, 6] = 1  # none of these exist
    cases.append((ex, ey))
    links = orc.links_from_chains(L, np.stack([c[0] for c in cases]), np.stack([c[1] for c in cases]))
    T, F, S = gpu.decode_errors_open(L, links, 100)
    compare("hand cases", T, F, S, orc.decode_links(L, links, 100, open_bc=True))
    ex = np.zeros((4, 4), np.uint8)
    ex[2, 1] = 1
    links = orc.links_from_chains(4, ex[None], np.zeros((1, 4, 4), np.uint8))
    T, F, S = gpu.decode_errors_open(4, links, 50)
    compare("balanced pair", T, F, S, orc.decode_links(4, links, 50, open_bc=True))
    assert int(_np(F)[0]) == 3
    for L in (9, 16):
        rnd = [orc.noise(L, 0.1, int(x)) for x in seeds(131, L, 60)]
        links = orc.links_from_chains(L, np.stack([a for a, _ in rnd]), np.stack([b for _, b in rnd]))
        T, F, S = gpu.decode_errors_open(L, links, 300)
        compare(f"random chains L={L}", T, F, S, orc.decode_links(L, links, 300, open_bc=True))


@pytest.mark.parametrize("L", [5, 8, 13, 16])
def test_open_run_steps_state(gpu, orc, L):
    ms = seeds(132, L, 4)
    exs, eys = zip(*[orc.noise(L, 0.1, int(x)) for x in ms])
    links = orc.links_from_chains(L, np.stack(exs), np.stack(eys))
    for t in (0, 1, 2, 3, 5, 9):
        M, S, W = gpu.run_steps_open(L, links, t)
        M, S, W = _np(M), _np(S).view(np.uint32), _np(W)
        for k in range(len(ms)):
            m, sig, (cx, cy), _ = orc.run_steps(L, exs[k], eys[k], t, open_bc=True)
            assert np.array_equal(M[k].astype(np.int64), m.astype(np.int64)), (t, k)
            assert np.array_equal(S[k], orc.pack_bits((sig == -1).reshape(-1))), (t, k)
            assert (int(W[k]) >> 2) == int(cx[:, L - 2].sum() % 2), (t, k)
            assert int(W[k]) & 0b1010 == 0


@pytest.mark.parametrize("driver", ["host", "device"])
@pytest.mark.parametrize("L,p,n,T_max", [(256, 0.03, 8, 64), (256, 0.07, 6, 40), (256, 0.02, 100, 64),
                                         (272, 0.05, 4, 48), (320, 0.06, 3, 30), (512, 0.04, 3, 40),
                                         (256, 0.0, 4, 16), (256, 1.0, 2, 16)])
def test_open_band_matches_oracle(gpu, orc, driver, L, p, n, T_max):
    """The band path on the open lattice: full-height and 2D tiles, small and
    full-size regions, budgets ending inside passes, both drivers; p = 1
    flips every existing link (no syndrome, a crossing of every row)."""
    gpu.set_band_driver(gpu.BAND_DRIVER_HOST if driver == "host" else gpu.BAND_DRIVER_DEVICE)
    try:
        s = seeds(133, L + T_max, n)
        T, F, S = gpu.decode_open(L, p, s, T_max)
    finally:
        gpu.set_band_driver(gpu.BAND_DRIVER_AUTO)
    ref = orc.decode_seeds(L, p, s, T_max, threads=16, open_bc=True)
    compare(f"open band L={L} p={p} {driver}", T, F, S, ref)
