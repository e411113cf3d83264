"""The C oracle against two other statements of the rule (CPU only).

1. The feedback decision of a single site, for every register pattern
   m in {0..7}^4 with and without an anyon, against a re-implementation that
   sorts the nonzero registers by (value, s a): argmin' of eq. (degbreak)
   with the readings R3-R5 (Def. "message passing automaton, general
   dimensions").
2. A pure-Python transcription of the definitions (oracle/literal.py: sets,
   dictionaries and loops) against the C oracle on every torus error pattern
   of weight <= 3 for L = 4, 5, 6 (T_dec, flags, final syndrome), and on
   random patterns step by step (registers, syndrome, correction).  The
   transcription itself is held to the hand-derived cases of
   tests/golden/hand_cases.json.
"""
from __future__ import annotations

import itertools
import json
import os
from concurrent.futures import ProcessPoolExecutor

import numpy as np
import pytest

from oracle import literal

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

# register order of the C oracle: +x, -x, +y, -y, i.e. (s, a) = (+1,1), (-1,1), (+1,2), (-1,2)
S_OF = (+1, -1, +1, -1)
A_OF = (1, 1, 2, 2)


def decision_by_sorting(m, anyon):
    """(f^x, f^y) from a sort of the nonzero registers by (m, s a)."""
    if not anyon:
        return 0, 0
    cand = sorted((m[d], S_OF[d] * A_OF[d], d) for d in range(4) if m[d] > 0)
    if not cand:
        return 0, 0
    d = cand[0][2]
    a = A_OF[d]
    plus, minus = (m[0], m[1]) if a == 1 else (m[2], m[3])
    if plus == minus:
        f = 0
    elif minus == 0 or (plus != 0 and plus < minus):
        f = +1  # nearest source on the -a side (an m^{+a} message): move along -a
    else:
        f = -1  # nearest source on the +a side: move along +a
    return (f, 0) if a == 1 else (0, f)


def test_decision_table_exhaustive(orc):
    """All 8^4 register patterns x anyon / no anyon."""
    n = 0
    for m in itertools.product(range(8), repeat=4):
        for anyon in (False, True):
            got = orc.decide(m, anyon)
            assert got == decision_by_sorting(m, anyon), (m, anyon, got)
            n += 1
            if not anyon:
                continue
            fx, fy = got
            # never two axes, and never away from the only message on an axis
            assert fx == 0 or fy == 0
            for f, (pl, mi) in ((fx, (m[0], m[1])), (fy, (m[2], m[3]))):
                if pl > 0 and mi == 0:
                    assert f in (0, +1)
                if mi > 0 and pl == 0:
                    assert f in (0, -1)
    assert n == 2 * 8 ** 4


def test_decision_examples(orc):
    """A few decisions written out by hand from the definition."""
    # the only message is m^{+x} = 3 (source 3 sites to the left): move -x (f^x = +1)
    assert orc.decide([3, 0, 0, 0], True) == (1, 0)
    # m^{-y} = 2 beats m^{+x} = 5: source above, move +y (f^y = -1)
    assert orc.decide([5, 0, 0, 2], True) == (0, -1)
    # equal smallest messages +x and +y: the tie order -y < -x < +x < +y picks +x
    assert orc.decide([2, 4, 2, 0], True) == (1, 0)
    # chosen axis tied (m^{+x} = m^{-x}): no move
    assert orc.decide([2, 2, 3, 0], True) == (0, 0)
    # not an anyon: no force whatever the registers
    assert orc.decide([1, 2, 3, 4], False) == (0, 0)
    # no message at all
    assert orc.decide([0, 0, 0, 0], True) == (0, 0)


def _chains(L, x_links, y_links):
    ex = {tuple(r): 1 for r in x_links}
    ey = {tuple(r): 1 for r in y_links}
    return ex, ey


def test_literal_reproduces_hand_cases():
    """The transcription itself against the hand-derived outcomes."""
    with open(os.path.join(GOLDEN, "hand_cases.json")) as f:
        cases = json.load(f)["cases"]
    assert len(cases) >= 20
    for c in cases:
        ex, ey = _chains(c["L"], c["x_links"], c["y_links"])
        T, fl, left, _ = literal.decode(c["L"], ex, ey, c["T_max"])
        e = c["expect"]
        assert T == e["T_dec"], c["name"]
        assert (fl & 1) == e["fail"], c["name"]
        assert ((fl >> 1) & 1) == e["timeout"], c["name"]
        assert sorted(left) == sorted(tuple(a) for a in e["final_anyons"]), c["name"]


def _link_list(L):
    return [("x", (x, y)) for y in range(L) for x in range(L)] + [("y", (x, y)) for y in range(L) for x in range(L)]


def _literal_block(args):
    """Decode patterns [lo, hi) of the weight-<=3 enumeration with the transcription."""
    L, T_max, lo, hi = args
    links = _link_list(L)
    pats = _patterns(L)[lo:hi]
    W = (L * L + 31) // 32
    T = np.zeros(len(pats), np.int32)
    F = np.zeros(len(pats), np.uint8)
    S = np.zeros((len(pats), W), np.uint32)
    for j, P in enumerate(pats):
        ex, ey = {}, {}
        for k in P:
            name, r = links[k]
            (ex if name == "x" else ey)[r] = 1
        t, fl, left, _ = literal.decode(L, ex, ey, T_max)
        T[j], F[j] = t, fl
        for (x, y) in left:
            i = y * L + x
            S[j, i >> 5] |= np.uint32(1 << (i & 31))
    return T, F, S


_PAT_CACHE = {}


def _patterns(L):
    if L not in _PAT_CACHE:
        n = 2 * L * L
        pats = [()]
        for w in (1, 2, 3):
            pats += list(itertools.combinations(range(n), w))
        _PAT_CACHE[L] = pats
    return _PAT_CACHE[L]


@pytest.mark.slow
@pytest.mark.parametrize("L", [4, 5, 6])
def test_literal_vs_c_weight_le3(orc, L):
    """Every pattern of at most three flipped links on the L x L torus."""
    T_max = 3 * L
    pats = _patterns(L)
    links = _link_list(L)
    lw = (2 * L * L + 31) // 32
    words = np.zeros((len(pats), lw), np.uint32)
    for j, P in enumerate(pats):
        for k in P:
            name, (x, y) = links[k]
            lid = 2 * (y * L + x) + (0 if name == "x" else 1)
            words[j, lid >> 5] |= np.uint32(1 << (lid & 31))
    ref = orc.decode_links(L, words, T_max, threads=4)
    chunks = 16
    bounds = np.linspace(0, len(pats), chunks + 1).astype(int)
    with ProcessPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        parts = list(ex.map(_literal_block, [(L, T_max, int(a), int(b)) for a, b in zip(bounds, bounds[1:])]))
    T = np.concatenate([p[0] for p in parts])
    F = np.concatenate([p[1] for p in parts])
    S = np.concatenate([p[2] for p in parts])
    bad = np.nonzero((T != ref["T_dec"]) | (F != ref["flags"]) | np.any(S != ref["sigma_words"], axis=1))[0]
    assert bad.size == 0, [(pats[j], int(T[j]), int(ref["T_dec"][j]), int(F[j]), int(ref["flags"][j]))
                           for j in bad[:5]]
    # every single flipped link: an adjacent pair, annihilated in one step without failure
    w1 = np.array([len(P) == 1 for P in pats])
    assert np.all(T[w1] == 1) and np.all(F[w1] == 0)
    assert T[0] == 0 and F[0] == 0


@pytest.mark.parametrize("L", [5, 6, 8])
def test_literal_vs_c_state_per_step(orc, L):
    """Registers, syndrome and correction after every step, random chains."""
    rng = np.random.default_rng(1000 + L)
    for trial in range(6):
        ex_a = (rng.random((L, L)) < 0.08).astype(np.uint8)
        ey_a = (rng.random((L, L)) < 0.08).astype(np.uint8)
        ex = {(x, y): 1 for y in range(L) for x in range(L) if ex_a[y, x]}
        ey = {(x, y): 1 for y in range(L) for x in range(L) if ey_a[y, x]}
        d = literal.Decoder(L, ex, ey)
        for t in range(0, 7):
            if t:
                d.step()
            m, sig, (cx, cy), _ = orc.run_steps(L, ex_a, ey_a, t)
            for k, (s, a) in enumerate(literal.DIRECTIONS):
                mine = np.array([[d.m[(s, a)][(x, y)] for x in range(L)] for y in range(L)])
                assert np.array_equal(mine, m[k]), (L, trial, t, (s, a))
            mine_sig = np.array([[d.sigma[(x, y)] for x in range(L)] for y in range(L)])
            assert np.array_equal(mine_sig, sig), (L, trial, t)
            mine_cx = np.array([[d.Cor[("x", (x, y))] for x in range(L)] for y in range(L)])
            mine_cy = np.array([[d.Cor[("y", (x, y))] for x in range(L)] for y in range(L)])
            assert np.array_equal(mine_cx, cx) and np.array_equal(mine_cy, cy), (L, trial, t)
