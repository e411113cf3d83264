"""Pins of the open-boundary variant (appendix on open boundaries, Def.
"message passing automaton with open boundaries"): rough boundaries B at
x = 0 and x = L - 1, smooth rows y = 0 and y = L - 1, one logical qubit.
Checked against hand-derived decoding times, the lightfront definition of
the messages with B as a permanent source, invariants, the exhaustive L = 4
lattice (a distance-3 code corrects every single error) and a threshold.
"""
import math

import numpy as np
import pytest

from paper_2506_03266_amd.workloads import seeds
from test_oracle_pins import DIRS, chains


def bulk_boundary(L, ex, ey):
    """Anyons of a chain on the open lattice: parity of the existing incident
    links at bulk sites (columns 1 .. L-2), none on B."""
    ex = ex.copy()
    ey = ey.copy()
    ex[:, L - 1] = 0
    ey[L - 1, :] = 0
    ey[:, 0] = 0
    ey[:, L - 1] = 0
    s = ex ^ np.roll(ex, 1, 1) ^ ey ^ np.roll(ey, 1, 0)
    s[:, 0] = 0
    s[:, L - 1] = 0
    return s


@pytest.mark.parametrize("d", range(1, 10))
def test_lone_anyon_is_absorbed_by_the_nearer_rough_boundary(orc, d):
    """A string from B to the site at distance d leaves one anyon.  B sources
    x-messages at every update, so the message reaches it in ceil(d/3) steps;
    it then moves one site per step onto B: T = ceil(d/3) + d - 1, no failure.
    The same at the right boundary, where error and correction each cross the
    cut once."""
    L = 22
    want = math.ceil(d / 3) + d - 1
    r = orc.decode_errors(L, *chains(L, [[k, 7] for k in range(d)], []), 100, open_bc=True)
    assert (r["T_dec"], r["flags"]) == (want, 0)
    r = orc.decode_errors(L, *chains(L, [[L - 1 - d + k, 7] for k in range(d)], []), 100, open_bc=True,
                          want_state=True)
    assert (r["T_dec"], r["flags"]) == (want, 0)
    assert r["wind"] == (1, 0, 1, 0)


def test_strings_between_and_inside_the_boundaries(orc):
    """A row of x-links from B_L to B_R has no syndrome and is the logical
    operator: T = 0, failure.  y-links inside B and links leaving the lattice
    do not exist and are ignored.  A pair far from B decodes as on the torus."""
    L = 16
    r = orc.decode_errors(L, *chains(L, [[k, 5] for k in range(L - 1)], []), 100, open_bc=True)
    assert (r["T_dec"], r["flags"]) == (0, 1)
    ghost = chains(L, [[L - 1, 3]], [[0, 4], [L - 1, 9], [6, L - 1]])
    r = orc.decode_errors(L, *ghost, 100, open_bc=True)
    assert (r["T_dec"], r["flags"]) == (0, 0)
    for d in range(2, 8):
        r = orc.decode_errors(40, *chains(40, [[15 + k, 20] for k in range(d)], []), 100, open_bc=True)
        assert (r["T_dec"], r["flags"]) == (math.ceil(d / 3) - 1 + math.ceil(d / 2), 0)


def lightcone_open(L, hist, v, s_now):
    """Messages after sub-step s_now on the open lattice from the anyon
    history: the smallest j <= s_now such that, during sub-step s_now - j + 1,
    an anyon sat on the segment r - j s a-hat + k b-hat (|k| <= j, clipped to
    the lattice, and for y-messages to the bulk columns, since B relays
    nothing) or, for x-messages, the segment's column is the rough boundary
    the message comes from; 0 if none, and 0 at B."""
    m = np.zeros((4, L, L), np.int64)
    for d, (s, ax) in enumerate(DIRS):
        for y in range(L):
            for x in range(1, L - 1):
                for j in range(1, s_now + 1):
                    A = hist[(s_now - j) // v]
                    hit = False
                    if ax == 0:
                        qx = x - j * s
                        if qx < 0 or qx > L - 1:
                            break
                        if qx == 0 or qx == L - 1:
                            hit = True
                        else:
                            hit = any(A[y + k, qx] for k in range(-j, j + 1) if 0 <= y + k < L)
                    else:
                        qy = y - j * s
                        if qy < 0 or qy > L - 1:
                            break
                        hit = any(A[qy, x + k] for k in range(-j, j + 1) if 1 <= x + k <= L - 2)
                    if hit:
                        m[d, y, x] = j
                        break
    return m


@pytest.mark.parametrize("L,p,seed", [(7, 0.08, 1), (8, 0.06, 2), (9, 0.1, 3), (6, 0.12, 4)])
def test_open_messages_match_lightcone(orc, L, p, seed):
    ex, ey = orc.noise(L, p, 3000 + seed)
    T = 5
    _, _, _, hist = orc.run_steps(L, ex, ey, T, record=True, open_bc=True)
    for t in range(1, T + 1):
        m, _, _, _ = orc.run_steps(L, ex, ey, t, open_bc=True)
        assert np.array_equal(m, lightcone_open(L, hist, 3, 3 * t)), f"step {t}"


@pytest.mark.parametrize("L,p", [(8, 0.05), (9, 0.08), (12, 0.06), (10, 0.12)])
def test_open_invariants(orc, L, p):
    """sigma is the bulk boundary of E + C; anyons never multiply and move one
    link at a time (they may vanish singly into B); on success E + C has no
    bulk boundary and crosses every vertical cut with the same parity, which
    is the reported outcome."""
    for s in seeds(121, 10 * L + int(100 * p), 5):
        ex, ey = orc.noise(L, p, int(s))
        prev = None
        for t in range(14):
            m, sig, (cx, cy), _ = orc.run_steps(L, ex, ey, t, open_bc=True)
            anyon = (sig == -1).astype(np.uint8)
            assert np.array_equal(anyon, bulk_boundary(L, ex ^ cx, ey ^ cy))
            assert not anyon[:, 0].any() and not anyon[:, L - 1].any()
            assert not m[:, :, 0].any() and not m[:, :, L - 1].any()
            if prev is not None:
                assert anyon.sum() <= prev.sum()
                near = prev.copy()
                near[:, 1:] |= prev[:, :-1]
                near[:, :-1] |= prev[:, 1:]
                near[1:, :] |= prev[:-1, :]
                near[:-1, :] |= prev[1:, :]
                assert not np.any(anyon & (1 - near))
            prev = anyon
        r = orc.decode_errors(L, ex, ey, 512, open_bc=True, want_state=True)
        if r["flags"] & 2:
            continue
        zx, zy = ex ^ r["cx"], ey ^ r["cy"]
        zx[:, L - 1] = 0
        assert bulk_boundary(L, zx, zy).sum() == 0
        cuts = {int(zx[:, c].sum() % 2) for c in range(L - 1)}
        assert len(cuts) == 1 and (r["flags"] & 1) == cuts.pop()


def open_link_ids(L):
    """Link ids (2 i + dir) of the qubits of the open lattice (R20)."""
    return [2 * (y * L + x) for y in range(L) for x in range(L - 1)] + \
           [2 * (y * L + x) + 1 for y in range(L - 1) for x in range(1, L - 1)]


def test_exhaustive_L4_open(orc):
    """All 2^18 error patterns on the 18 qubits of the L = 4 open lattice:
    successes end syndrome-free; syndrome-free patterns report T = 0 with
    failure exactly when they cross the cut an odd number of times; single
    errors decode in at most two steps without failure -- except an x-link
    between the two bulk columns: each of its anyons then sees a rough
    boundary and its partner both at distance 1, the forces along x cancel
    (sgn(0) = 0) and neither ever moves, a steady state of an even-sized
    lattice like those the paper notes for the deterministic rule."""
    L = 4
    ids = open_link_ids(L)
    assert len(ids) == 18
    n = 1 << 18
    pats = ((np.arange(n)[:, None] >> np.arange(18)[None, :]) & 1).astype(np.uint8)
    bits = np.zeros((n, 2 * L * L), np.uint8)
    bits[:, ids] = pats
    nw = (2 * L * L + 31) // 32
    wts = (bits.reshape(n, nw, 32).astype(np.uint64) << np.arange(32, dtype=np.uint64)).sum(axis=2).astype(np.uint32)
    r = orc.decode_links(L, wts, 64, threads=8, open_bc=True)
    ok = (r["flags"] & 2) == 0
    assert not np.any(r["sigma_words"][ok])
    weight = pats.sum(axis=1)
    for k in np.nonzero(weight == 1)[0]:
        lid = ids[int(np.argmax(pats[k]))]
        balanced = lid % 2 == 0 and (lid // 2) % L == 1
        got = (int(r["T_dec"][k]), int(r["flags"][k]))
        assert got == (64, 3) if balanced else (got[0] <= 2 and got[1] == 0), (lid, got)
    ex = bits[:, 0::2].reshape(n, L, L)
    ey = bits[:, 1::2].reshape(n, L, L)
    low = np.nonzero(weight <= 3)[0]
    syn = np.stack([bulk_boundary(L, ex[k], ey[k]) for k in low])
    quiet = low[syn.reshape(len(syn), -1).sum(1) == 0]
    assert len(quiet) > 0
    assert np.all(r["T_dec"][quiet] == 0)
    cross = ex[quiet][:, :, L - 2].sum(axis=1) % 2
    assert np.array_equal(r["flags"][quiet] & 1, cross.astype(np.uint8))


@pytest.mark.parametrize("L", [5, 6, 7])
def test_single_errors_decode_on_open_lattices(orc, L):
    """From L = 5 on every single error decodes within two steps without a
    logical failure."""
    ids = open_link_ids(L)
    bits = np.zeros((len(ids), 2 * L * L), np.uint8)
    bits[np.arange(len(ids)), ids] = 1
    r = orc.decode_links(L, np.stack([orc.pack_bits(b) for b in bits]), 64, open_bc=True)
    assert r["T_dec"].max() <= 2 and not np.any(r["flags"])


def test_open_threshold(orc):
    """Below threshold larger lattices fail less, above it more (the open
    lattice crosses between p = 0.07 and 0.09 on these sizes)."""
    res = {}
    for p in (0.05, 0.12):
        for L in (12, 24):
            r = orc.decode_seeds(L, p, seeds(122, 10 * L + int(100 * p), 3000), 2048, threads=8,
                                 want_sigma=False, open_bc=True)
            res[(p, L)] = float((r["flags"] & 1).mean())
    assert res[(0.05, 24)] < res[(0.05, 12)]
    assert res[(0.12, 24)] > res[(0.12, 12)]
