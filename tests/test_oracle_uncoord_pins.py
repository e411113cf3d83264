"""Pins of the uncoordinated desynchronization (Sec. "Uncoordinated
desynchronization", reading R28 of the oracle): the marching-soldiers clock
and update schedule without the lag rule or old copies.  It computes
something other than the synchronous decoder, so it is pinned by what holds
for any update order: every ring is applied, message registers settle on the
static lightfront distance of fixed anyons (the fixed point of the min-plus
rule), hand-derived pair decodes, the invariants of anyon motion, and a
threshold between low and high noise.  Both schedules of R28 are covered:
"cyclic" (every (v+1)-th update of a site is a motion) and "random" (each
update is a motion with probability 1/(v+1), drawn from Philox).
"""
import numpy as np
import pytest

from paper_2506_03266_amd.workloads import seeds
from test_oracle_pins import DIRS, boundary


def static_cone_distance(L, A):
    """m^{sa}_r for anyons A that never move: the smallest j >= 1 such that an
    anyon sits on r - j s a-hat + k b-hat for some |k| <= j (torus), 0 if
    there is none."""
    m = np.zeros((4, L, L), np.int64)
    for d, (s, ax) in enumerate(DIRS):
        for y in range(L):
            for x in range(L):
                for j in range(1, 2 * L):
                    hit = False
                    for k in range(-j, j + 1):
                        qx, qy = (x - j * s, y + k) if ax == 0 else (x + k, y - j * s)
                        if A[qy % L, qx % L]:
                            hit = True
                            break
                    if hit:
                        m[d, y, x] = j
                        break
    return m


@pytest.mark.parametrize("L,p,rho", [(6, 0.08, 1.0), (8, 0.05, 0.5), (9, 0.06, 0.25)])
def test_static_registers_settle_on_the_lightfront_distance(orc, L, p, rho):
    """With v far above the updates run, no anyon moves; in any order the
    message rule then reaches its fixed point, the static cone distance."""
    ex, ey = orc.noise(L, p, 40 + L)
    A = boundary(L, ex, ey)
    assert A.sum() > 0
    S = int(12 * L / rho)
    for clock in (1, 2, 3):
        r = orc.async_run(L, ex, ey, seed=clock, rho=rho, S_max=S, v=10 * S, uncoordinated=True)
        assert r["tsim"].max() < 10 * S and r["tsim"].min() >= 4 * L
        assert np.array_equal(r["m"], static_cone_distance(L, A)), clock


def test_every_ring_is_applied(orc):
    """No lag rule: after S slots each site has made exactly as many updates
    as it rang (R26's ring test on Philox(seed, (i >> 1, s, 0x41535943, 0)))."""
    L = 9
    ex, ey = orc.noise(L, 0.05, 7)
    for seed, rho, S in ((31, 0.3, 9), (2**35 + 3, 0.8, 5)):
        r = orc.async_run(L, ex, ey, seed=seed, rho=rho, S_max=S, t_target=1000, uncoordinated=True)
        key = [seed & 0xFFFFFFFF, seed >> 32]
        thr = orc.ring_threshold(rho)
        want = np.zeros(L * L, np.int64)
        for s in range(S):
            for i in range(L * L):
                w = orc.philox4x32_10([i >> 1, s, 0x41535943, 0], key)
                want[i] += int(w[2 * (i & 1)]) < thr
        assert np.array_equal(r["tsim"].reshape(-1), want)


@pytest.mark.parametrize("d", [1, 2])
@pytest.mark.parametrize("axis", [0, 1])
def test_close_pairs_annihilate_at_the_first_motion(orc, d, axis):
    """A pair at distance 1 or 2 with certain ringing: three message updates
    let each anyon see the other, and the fourth update of each site is its
    motion.  The first to move closes the pair (d = 1) or halves it and the
    second, moving toward where its partner was, meets it (d = 2): the decode
    ends at slot 4 for every order, and the correction is the error chain."""
    L = 12
    ex = np.zeros((L, L), np.uint8)
    ey = np.zeros((L, L), np.uint8)
    if axis == 0:
        ex[5, 4:4 + d] = 1
    else:
        ey[4:4 + d, 5] = 1
    for clock in range(16):
        r = orc.async_run(L, ex, ey, seed=clock, rho=1.0, uncoordinated=True)
        assert (r["T_async"], r["flags"], r["slots"]) == (4, 0, 4)
        assert np.array_equal(r["cx"], ex) and np.array_equal(r["cy"], ey)


@pytest.mark.parametrize("schedule", ["cyclic", "random"])
@pytest.mark.parametrize("L,p,rho", [(8, 0.06, 0.25), (10, 0.08, 1.0), (12, 0.05, 0.5)])
def test_motion_invariants(orc, L, p, rho, schedule):
    """sigma stays the boundary of E + C, anyons stay paired and never
    multiply, and a finished decode leaves no anyon."""
    for s in seeds(150, 10 * L, 4):
        ex, ey = orc.noise(L, p, int(s))
        prev = None
        for S in range(0, 120, 4):
            r = orc.async_run(L, ex, ey, seed=int(s), rho=rho, S_max=S, uncoordinated=True, schedule=schedule)
            sig = np.zeros(L * L, np.uint8)
            words = r["sigma_words"]
            for i in range(L * L):
                sig[i] = (int(words[i >> 5]) >> (i & 31)) & 1
            anyon = sig.reshape(L, L)
            assert np.array_equal(anyon, boundary(L, ex ^ r["cx"], ey ^ r["cy"]))
            assert anyon.sum() % 2 == 0
            if prev is not None:
                assert anyon.sum() <= prev
            prev = anyon.sum()
        r = orc.async_run(L, ex, ey, seed=int(s), rho=rho, S_max=30000, uncoordinated=True, schedule=schedule)
        if not r["flags"] & 2:
            assert not r["sigma_words"].any()


@pytest.mark.parametrize("schedule", ["cyclic", "random"])
def test_uncoordinated_threshold(orc, schedule):
    """The section reports a threshold for the uncoordinated decoder: larger
    lattices fail less at low noise and more at high noise."""
    res = {}
    for p in (0.03, 0.12):
        for L in (10, 20):
            r = orc.async_decode_seeds(L, p, seeds(151, 10 * L + int(100 * p), 1500), rho=0.25, S_max=30000,
                                       threads=8, want_sigma=False, uncoordinated=True, schedule=schedule)
            res[(p, L)] = float((r["flags"] & 1).mean())
    assert res[(0.03, 20)] < res[(0.03, 10)]
    assert res[(0.12, 20)] > res[(0.12, 10)]


def test_uncoordinated_batch_matches_single_runs(orc):
    L, p = 10, 0.07
    s = seeds(152, 0, 20)
    b = orc.async_decode_seeds(L, p, s, rho=0.25, S_max=20000, threads=8, uncoordinated=True)
    for k, seed in enumerate(s):
        ex, ey = orc.noise(L, p, int(seed))
        r = orc.async_run(L, ex, ey, seed=int(seed), rho=0.25, S_max=20000, uncoordinated=True)
        assert (b["T_async"][k], b["flags"][k], b["slots"][k], b["updates"][k]) == \
            (r["T_async"], r["flags"], r["slots"], r["updates"])
        assert np.array_equal(b["sigma_words"][k], r["sigma_words"])


def test_random_schedule_draws_the_update_type(orc):
    """Schedule "random" (R28): an update of site i in slot s is a motion iff
    word (i & 1) of Philox(key = seed, counter (i >> 1, s, 0x54595045, 0)) mod 4
    is 3.  For a lone pair at distance 1 with certain ringing, an endpoint's
    registers see its partner after its first message update, so the pair
    annihilates in the first slot in which an endpoint draws a motion after
    having drawn a message: T follows from the draws alone."""
    L = 12
    ex = np.zeros((L, L), np.uint8)
    ey = np.zeros((L, L), np.uint8)
    ex[5, 4] = 1
    ends = [5 * L + 4, 5 * L + 5]
    for seed in range(40):
        key = [seed & 0xFFFFFFFF, seed >> 32]
        seen = {i: False for i in ends}
        want = None
        for slot in range(200):
            for i in ends:
                w = orc.philox4x32_10([i >> 1, slot, 0x54595045, 0], key)
                motion = int(w[i & 1]) % 4 == 3
                if motion and seen[i]:
                    want = slot + 1
                if not motion:
                    seen[i] = True
            if want:
                break
        r = orc.async_run(L, ex, ey, seed=seed, rho=1.0, uncoordinated=True, schedule="random")
        assert (r["T_async"], r["flags"]) == (want, 0), seed
        assert np.array_equal(r["cx"], ex)


def test_random_schedule_applies_every_ring(orc):
    L = 9
    ex, ey = orc.noise(L, 0.05, 8)
    seed, rho, S = 77, 0.4, 7
    r = orc.async_run(L, ex, ey, seed=seed, rho=rho, S_max=S, t_target=1000, uncoordinated=True, schedule="random")
    key = [seed & 0xFFFFFFFF, seed >> 32]
    thr = orc.ring_threshold(rho)
    want = np.zeros(L * L, np.int64)
    for s_ in range(S):
        for i in range(L * L):
            w = orc.philox4x32_10([i >> 1, s_, 0x41535943, 0], key)
            want[i] += int(w[2 * (i & 1)]) < thr
    assert np.array_equal(r["tsim"].reshape(-1), want)
