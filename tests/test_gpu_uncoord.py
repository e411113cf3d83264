"""Uncoordinated desynchronization on the GPU against the oracle, bit for bit:
states at any slot count (update counts, registers, syndrome, windings) and
whole decodes (decoding time in slots, outcome, slots run, updates, final
syndrome)."""
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


@pytest.mark.parametrize("schedule", ["cyclic", "random"])
@pytest.mark.parametrize("L,p", [(5, 0.12), (8, 0.08), (13, 0.06), (16, 0.05), (31, 0.05), (32, 0.04), (64, 0.03)])
@pytest.mark.parametrize("rho", [0.05, 0.3, 1.0])
def test_run_uncoord_state_matches_oracle(gpu, orc, L, p, rho, schedule):
    ms = seeds(160, 10 * L + int(100 * rho), 3)
    exs, eys = zip(*[orc.noise(L, p, int(x)) for x in ms])
    links = orc.links_from_chains(L, np.stack(exs), np.stack(eys))
    clocks = [int(x) ^ 0x3C3C for x in ms]
    for S in (7, 40, 65000):
        SL, U, M, TS, SY, W = (_np(x) for x in gpu.run_async(L, links, clocks, 6, rho, S_max=S, uncoordinated=True,
                                                             schedule=schedule))
        for k in range(len(ms)):
            r = orc.async_run(L, exs[k], eys[k], seed=clocks[k], rho=rho, t_target=6, S_max=S, uncoordinated=True,
                              schedule=schedule)
            tag = (L, rho, S, k, schedule)
            assert (int(SL[k]), int(U[k])) == (r["slots"], r["updates"]), tag
            assert np.array_equal(TS[k].view(np.uint16).astype(np.int64), r["tsim"]), tag
            assert np.array_equal(M[k].astype(np.int64), r["m"]), tag
            assert np.array_equal(SY[k].view(np.uint32), r["sigma_words"]), tag
            wc = int(r["cx"][:, L - 1].sum() % 2) | (int(r["cy"][L - 1, :].sum() % 2) << 1)
            assert (int(W[k]) >> 2) == wc, tag


@pytest.mark.parametrize("schedule", ["cyclic", "random"])
@pytest.mark.parametrize("L,p,n,rho", [(8, 0.08, 300, 0.25), (12, 0.06, 200, 0.1), (16, 0.05, 120, 0.5),
                                       (31, 0.05, 40, 0.25), (32, 0.06, 40, 1.0), (48, 0.04, 12, 0.25),
                                       (64, 0.05, 8, 0.125)])
def test_decode_uncoord_matches_oracle(gpu, orc, L, p, n, rho, schedule):
    s = seeds(161, 10 * L + int(100 * rho), n)
    T, F, SL, U, S = (_np(x) for x in gpu.decode_async(L, p, s, rho, S_max=30000, uncoordinated=True,
                                                       schedule=schedule))
    ref = orc.async_decode_seeds(L, p, s, rho=rho, S_max=30000, threads=16, uncoordinated=True, schedule=schedule)
    for key, got in (("T_async", T), ("flags", F), ("slots", SL), ("updates", U)):
        bad = np.nonzero(got != ref[key])[0]
        assert bad.size == 0, f"{key}: {bad.size} mismatches, first {bad[:4]} gpu {got[bad[:4]]} " \
                              f"oracle {ref[key][bad[:4]]}"
    assert np.array_equal(S.view(np.uint32), ref["sigma_words"])


def test_uncoord_edge_cases(gpu, orc):
    s = seeds(162, 0, 16)
    T, F, SL, U, S = (_np(x) for x in gpu.decode_async(16, 0.0, s, 0.5, uncoordinated=True))
    assert not T.any() and not F.any() and not SL.any() and not U.any() and not S.any()
    T, F, SL, U, S = (_np(x) for x in gpu.decode_async(16, 0.2, s, 0.5, S_max=0, uncoordinated=True))
    assert not T.any() and (F == 3).all() and not SL.any()
    for schedule in ("cyclic", "random"):
        ref = orc.async_decode_seeds(5, 0.15, s, rho=0.4, S_max=65000, threads=8, uncoordinated=True,
                                     schedule=schedule)
        T, F, SL, U, S = (_np(x) for x in gpu.decode_async(5, 0.15, s, 0.4, S_max=65000, uncoordinated=True,
                                                           schedule=schedule))
        assert np.array_equal(T, ref["T_async"]) and np.array_equal(F, ref["flags"])
        assert np.array_equal(SL, ref["slots"]) and np.array_equal(U, ref["updates"])
