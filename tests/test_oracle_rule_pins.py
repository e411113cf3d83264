"""Pins of the limited-memory variant of the rule (Sec. 5.3, the corollary on
thresholds with limited classical memory): messages that would exceed m_max
disappear (R17), and with u > 0 every u-th step moves each anyon in a random
direction (R18).  Checked against what the text and the mathematics fix:
the unbounded rule as a special case, the lightfront definition of the
messages cut at m_max, pairs that cannot see each other, the invariants of
any move pattern, uniform random directions, and the claim that random motion
removes the stuck configurations a finite m_max creates.
"""
import math

import numpy as np
import pytest

from paper_2506_03266_amd.workloads import seeds
from test_oracle_pins import DIRS, boundary, chains


def test_m_max_above_every_message_is_the_unbounded_rule(orc):
    """No register can exceed the number of updates run (3 T_max), so
    m_max = 3 T_max never truncates: results equal the unbounded rule's."""
    for L, p in [(8, 0.06), (11, 0.04), (16, 0.08)]:
        s = seeds(98, L, 40)
        a = orc.decode_seeds(L, p, s, 48, threads=8)
        b = orc.decode_seeds(L, p, s, 48, threads=8, m_max=3 * 48)
        for k in ("T_dec", "flags", "sigma_words"):
            assert np.array_equal(a[k], b[k]), (L, p, k)
    # and truncation does change results once it bites
    s = seeds(98, 99, 200)
    a = orc.decode_seeds(12, 0.05, s, 200, threads=8)
    b = orc.decode_seeds(12, 0.05, s, 200, threads=8, m_max=3)
    assert not np.array_equal(a["T_dec"], b["T_dec"])


def lightcone_messages_cut(L, hist, v, s_now, m_max):
    """Messages after sub-step s_now from the anyon history: the smallest
    j in [1, min(s_now, m_max)] such that an anyon sat, during sub-step
    s_now - j + 1, on the segment r - j s a-hat + k b-hat, |k| <= j; 0 if
    none.  A message travels one site per update and its value is its age,
    so only those younger than m_max survive."""
    m = np.zeros((4, L, L), np.int64)
    for d, (s, ax) in enumerate(DIRS):
        for y in range(L):
            for x in range(L):
                for j in range(1, min(s_now, m_max) + 1):
                    A = hist[(s_now - j) // v]
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


@pytest.mark.parametrize("L,p,seed,m_max", [(7, 0.08, 1, 2), (8, 0.06, 2, 4), (7, 0.1, 3, 1), (9, 0.05, 4, 6)])
def test_truncated_messages_match_lightcone(orc, L, p, seed, m_max):
    """The recurrence with truncation equals the lightfront definition cut at
    m_max, at every step (no random moves, so the history is the rule's own)."""
    ex, ey = orc.noise(L, p, 2000 + seed)
    T = 5
    _, _, _, hist = orc.run_steps(L, ex, ey, T, record=True, m_max=m_max)
    for t in range(1, T + 1):
        m, _, _, _ = orc.run_steps(L, ex, ey, t, m_max=m_max)
        assert m.max() <= m_max
        assert np.array_equal(m, lightcone_messages_cut(L, hist, 3, 3 * t, m_max)), f"step {t}"


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6, 7])
def test_pair_needs_m_max_at_least_its_distance(orc, d):
    """A straight pair at distance d (L = 16): with m_max = d it decodes exactly
    as with unbounded messages (T = ceil(d/3) - 1 + ceil(d/2)); with
    m_max = d - 1 no message ever reaches either anyon, nothing moves, and the
    sample times out with its two anyons in place."""
    L = 16
    ex, ey = chains(L, [[2 + k, 2] for k in range(d)], [])
    want_T = math.ceil(d / 3) - 1 + math.ceil(d / 2)
    r = orc.decode_errors(L, ex, ey, 64, m_max=d)
    assert (r["T_dec"], r["flags"]) == (want_T, 0)
    r = orc.decode_errors(L, ex, ey, 64, m_max=d - 1, want_state=True)
    assert (r["T_dec"], r["flags"]) == (64, 3)
    assert r["cx"].sum() == 0 and r["cy"].sum() == 0
    sig = np.zeros(L * L, np.uint8)
    sig[2 * L + 2] = sig[2 * L + 2 + d] = 1
    assert np.array_equal(r["sigma_words"], orc.pack_bits(sig))


@pytest.mark.parametrize("L,p,m_max,u", [(8, 0.05, 2, 1), (9, 0.08, 3, 2), (12, 0.04, 0, 3), (10, 0.1, 1, 4)])
def test_random_moves_keep_the_invariants(orc, L, p, m_max, u):
    """With random moves sigma stays the boundary of E + C, anyons stay
    paired, never multiply, and each new anyon sits within one link of an
    old one; registers stay within [0, m_max]."""
    for s in seeds(99, 10 * L + u, 4):
        ex, ey = orc.noise(L, p, int(s))
        prev = None
        for t in range(13):
            m, sig, (cx, cy), _ = orc.run_steps(L, ex, ey, t, m_max=m_max, u=u, seed=int(s))
            anyon = (sig == -1).astype(np.uint8)
            assert np.array_equal(anyon, boundary(L, ex ^ cx, ey ^ cy))
            assert anyon.sum() % 2 == 0
            assert m.min() >= 0 and m.max() <= (m_max if m_max else 3 * t)
            if prev is not None:
                assert anyon.sum() <= prev.sum()
                near = prev | np.roll(prev, 1, 0) | np.roll(prev, -1, 0) | np.roll(prev, 1, 1) \
                    | np.roll(prev, -1, 1)
                assert not np.any(anyon & (1 - near))
            prev = anyon


def test_random_directions_are_uniform(orc):
    """u = 1 and m_max = 1 on a pair 8 links apart (L = 24): in the first step
    nothing has reached either anyon, so each one takes its random step.  Over
    3000 seeds the four displacements of the left anyon are uniform (chi-square,
    3 degrees of freedom, below the 0.1% point), and the two anyons move
    independently."""
    L = 24
    ex, ey = chains(L, [[4 + k, 10] for k in range(8)], [])
    n = 3000
    cnt = np.zeros((4, 4), int)
    disp = {(1, 0): 0, (-1, 0): 1, (0, 1): 2, (0, -1): 3}
    for s in seeds(100, 0, n):
        _, sig, _, _ = orc.run_steps(L, ex, ey, 1, m_max=1, u=1, seed=int(s))
        ys, xs = np.nonzero(sig == -1)
        assert len(xs) == 2
        pts = sorted(zip(xs.tolist(), ys.tolist()))
        a = disp[(pts[0][0] - 4, pts[0][1] - 10)]
        b = disp[(pts[1][0] - 12, pts[1][1] - 10)]
        cnt[a, b] += 1
    for marg in (cnt.sum(1), cnt.sum(0)):
        chi2 = float(((marg - n / 4) ** 2 / (n / 4)).sum())
        assert chi2 < 16.27, marg
    chi2 = float(((cnt - n / 16) ** 2 / (n / 16)).sum())
    assert chi2 < 37.7, cnt  # 15 degrees of freedom, 0.1% point


def test_random_direction_table(orc):
    """R18's table, a project convention (unpinned by the paper beyond
    uniformity): word (i & 1) of Philox(key = seed, counter = (i >> 1, t,
    0x4D4F5645, 0)), mod 4, moves the anyon of site i by +x, -x, +y, -y."""
    L = 24
    ex, ey = chains(L, [[4 + k, 10] for k in range(8)], [])
    step = {0: (1, 0), 1: (-1, 0), 2: (0, 1), 3: (0, -1)}
    for s in seeds(100, 2, 64):
        s = int(s)
        key = [s & 0xFFFFFFFF, s >> 32]
        want = []
        for x in (4, 12):
            i = 10 * L + x
            w = orc.philox4x32_10([i >> 1, 1, 0x4D4F5645, 0], key)
            dx, dy = step[int(w[i & 1]) & 3]
            want.append(((x + dx) % L, (10 + dy) % L))
        _, sig, _, _ = orc.run_steps(L, ex, ey, 1, m_max=1, u=1, seed=s)
        ys, xs = np.nonzero(sig == -1)
        assert sorted(zip(xs.tolist(), ys.tolist())) == sorted(want)


def test_adjacent_sites_draw_independent_directions(orc):
    """A single flipped x-link leaves anyons on two neighbouring sites (one
    site pair of the generator's counter).  With every step random, they
    annihilate in step 1 exactly when the left one moves +x and the right one
    -x: probability 1/16 if their directions are independent and uniform."""
    L = 16
    ex, ey = chains(L, [[4, 6]], [])
    n = 4000
    gone = 0
    for s in seeds(100, 1, n):
        _, sig, _, _ = orc.run_steps(L, ex, ey, 1, m_max=1, u=1, seed=int(s))
        gone += int((sig == -1).sum() == 0)
    mu, sd = n / 16, math.sqrt(n * (1 / 16) * (15 / 16))
    assert abs(gone - mu) < 5 * sd, gone


def test_random_motion_removes_stuck_configurations(orc):
    """With m_max = 2 many samples never finish (pairs farther apart than
    m_max never see each other); moving every anyon randomly every u steps
    lets all of them annihilate (the diffusive argument of the corollary)."""
    for L, p in [(8, 0.06), (12, 0.05)]:
        s = seeds(101, L, 300)
        r0 = orc.decode_seeds(L, p, s, 3000, threads=8, want_sigma=False, m_max=2)
        assert (r0["flags"] & 2).sum() // 2 >= 20
        for u in (2, 4):
            r = orc.decode_seeds(L, p, s, 3000, threads=8, want_sigma=False, m_max=2, u=u)
            assert (r["flags"] & 2).sum() == 0, (L, u)
