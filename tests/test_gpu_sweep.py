"""The Sec. 7.2 sweep's per-point counts (failures, timeouts, sums of T_dec)
equal those of the oracle on the same seeds, near and above threshold and on
both decoder paths (resident L <= 128, band L >= 256)."""
import numpy as np
import pytest

from paper_2506_03266_amd import sweep

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_03266_amd.binding as b
    b.lib()
    return b


@pytest.mark.parametrize("L,p,n,T_max", [(16, 0.075, 4000, 4096), (32, 0.09, 1500, 512), (64, 0.08, 300, 1024),
                                         (256, 0.075, 24, 160)])
def test_point_counts_match_oracle(gpu, orc, L, p, n, T_max):
    r = sweep.point(L, p, n, p_index=200, T_max=T_max)
    ref = orc.decode_seeds(L, p, sweep.seed_block(L, 200, n), T_max, threads=16, want_sigma=False)
    T = ref["T_dec"].astype(np.int64)
    F = ref["flags"].astype(np.int64)
    done = (F & 2) == 0
    want = dict(fails=int((F & 1).sum()), timeouts=int((~done).sum()), T_sum=int(T[done].sum()),
                T_sq=int((T[done] ** 2).sum()), site_updates=int(T.sum()) * L * L)
    got = {k: r[k] for k in want}
    assert got == want, (L, p, got, want)
    assert want["fails"] > 0


def test_point_spans_chunks(gpu, orc):
    """A point larger than one call's chunk sums its chunks (band path, chunk
    limit forced down to two samples)."""
    L, p, n, T_max = 512, 0.07, 5, 96
    old = sweep._chunk
    try:
        sweep._chunk = lambda L: 2
        r = sweep.point(L, p, n, p_index=201, T_max=T_max)
    finally:
        sweep._chunk = old
    ref = orc.decode_seeds(L, p, sweep.seed_block(L, 201, n), T_max, threads=16, want_sigma=False)
    T = ref["T_dec"].astype(np.int64)
    F = ref["flags"].astype(np.int64)
    done = (F & 2) == 0
    assert r["fails"] == int((F & 1).sum()) and r["timeouts"] == int((~done).sum())
    assert r["T_sum"] == int(T[done].sum()) and r["T_sq"] == int((T[done] ** 2).sum())
    assert r["site_updates"] == int(T.sum()) * L * L


@pytest.mark.parametrize("L,n,m_max,u", [(32, 1000, 3, 0), (32, 1000, 4, 8), (64, 200, 2, 8)])
def test_memory_point_matches_oracle(gpu, orc, L, n, m_max, u):
    """A point of the limited-memory grid: the same counts as the oracle."""
    r = sweep.point(L, sweep.MEMORY_P, n, p_index=202, T_max=512, m_max=m_max, u=u)
    ref = orc.decode_seeds(L, sweep.MEMORY_P, sweep.seed_block(L, 202, n), 512, threads=16, want_sigma=False,
                           m_max=m_max, u=u)
    T = ref["T_dec"].astype(np.int64)
    F = ref["flags"].astype(np.int64)
    done = (F & 2) == 0
    assert (r["fails"], r["timeouts"]) == (int((F & 1).sum()), int((~done).sum()))
    assert (r["T_sum"], r["T_sq"]) == (int(T[done].sum()), int((T[done] ** 2).sum()))


@pytest.mark.parametrize("L,p,n", [(16, 0.08, 2000), (64, 0.09, 100)])
def test_open_point_matches_oracle(gpu, orc, L, p, n):
    """A point of the open-lattice grid: the same counts as the oracle."""
    r = sweep.point(L, p, n, p_index=203, T_max=1024, open_bc=True)
    ref = orc.decode_seeds(L, p, sweep.seed_block(L, 203, n), 1024, threads=16, want_sigma=False, open_bc=True)
    T = ref["T_dec"].astype(np.int64)
    F = ref["flags"].astype(np.int64)
    done = (F & 2) == 0
    assert (r["fails"], r["timeouts"]) == (int((F & 1).sum()), int((~done).sum()))
    assert (r["T_sum"], r["T_sq"]) == (int(T[done].sum()), int((T[done] ** 2).sum()))


@pytest.mark.parametrize("schedule", ["cyclic", "random"])
@pytest.mark.parametrize("L,p,n", [(16, 0.07, 1500), (32, 0.08, 200)])
def test_uncoord_point_matches_oracle(gpu, orc, L, p, n, schedule):
    """A point of the uncoordinated grid: the same counts as the oracle
    (decoding times in slots)."""
    r = sweep.point(L, p, n, p_index=204, uncoord=schedule)
    ref = orc.async_decode_seeds(L, p, sweep.seed_block(L, 204, n), rho=sweep.UNCOORD_RHO, S_max=sweep.UNCOORD_S_MAX,
                                 threads=16, want_sigma=False, uncoordinated=True, schedule=schedule)
    T = ref["T_async"].astype(np.int64)
    F = ref["flags"].astype(np.int64)
    done = (F & 2) == 0
    assert (r["fails"], r["timeouts"]) == (int((F & 1).sum()), int((~done).sum()))
    assert (r["T_sum"], r["T_sq"]) == (int(T[done].sum()), int((T[done] ** 2).sum()))


def test_slowdown_rows(gpu):
    """The slowdown sweep (quick): most samples have anyons and finish, with
    outcomes equal to the synchronous decoder's, and the ratio lies in the
    band the lag rule allows (at least v + 1 = 4 updates per step, each
    accepted at most once per ring)."""
    rows = sweep.run_slowdown(quick=True, log=lambda s: None)
    assert len(rows) == len(sweep.SLOWDOWN_P) * len(sweep.SLOWDOWN_L)
    for r in rows:
        assert r["outcomes_equal"] and r["decoded"] > 0.5 * r["n"]
        assert 4.0 <= r["ratio"] <= 40.0, r
