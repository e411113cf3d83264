"""Band path (L >= 256): full decoder state after exactly t steps, resume
from an exported state, and explicit error patterns, against the oracle
(Def. "synchronous automaton decoder"; Def. "message passing automaton,
general dimensions").  Registers are compared element by element in the
paper's distance form."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2506_03266_amd.workloads import seeds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_03266_amd.binding as b
    b.lib()
    return b


def _np(t):
    return t.cpu().numpy()


def wind_bits(L, ex, ey, cx, cy):
    wx = lambda a: int(a[:, L - 1].sum() % 2)
    wy = lambda a: int(a[L - 1, :].sum() % 2)
    return wx(ex) | (wy(ey) << 1) | (wx(cx) << 2) | (wy(cy) << 3)


def check_state(orc, L, ex, ey, t, M, S, W, k, tag, **rule):
    m, sig, (cx, cy), _ = orc.run_steps(L, ex, ey, t, **rule)
    got = M[k].astype(np.int32)
    if not np.array_equal(got, m):
        bad = np.argwhere(got != m)
        d, y, x = bad[0]
        raise AssertionError(f"{tag}: registers differ at {len(bad)} places, first d={d} (x,y)=({x},{y}): "
                             f"gpu {got[d, y, x]} oracle {m[d, y, x]}")
    want = orc.pack_bits((sig == -1).astype(np.uint8).reshape(-1))
    assert np.array_equal(S[k].view(np.uint32), want), tag
    assert int(W[k]) == wind_bits(L, ex, ey, cx, cy), tag


@pytest.mark.parametrize("L,p", [(256, 0.02), (256, 0.06), (512, 0.03)])
def test_band_run_steps_state(gpu, orc, L, p):
    """Registers, syndrome and winding bits after t = 0..9 steps: one pass
    (t <= k_first) and several passes, full-height regions (L = 256) and 2D
    tiles with row halos (L = 512)."""
    n = 2
    chains = [orc.noise(L, p, int(sd)) for sd in seeds(47, int(1000 * p) + L, n)]
    links = np.stack([orc.links_from_chains(L, ex, ey)[0] for ex, ey in chains])
    for t in range(10):
        M, S, W = gpu.run_steps_ws(L, links, t)
        M, S, W = _np(M), _np(S), _np(W)
        for k, (ex, ey) in enumerate(chains):
            check_state(orc, L, ex, ey, t, M, S, W, k, f"L={L} p={p} t={t} sample {k}")


@pytest.mark.parametrize("L", [256, 512])
def test_band_resume_equals_straight(gpu, orc, L):
    """An exported state resumed for more steps equals the straight run, in
    one resume and in chunks of 1-3 steps."""
    n = 3
    p = 0.04
    chains = [orc.noise(L, p, int(sd)) for sd in seeds(48, L, n)]
    links = np.stack([orc.links_from_chains(L, ex, ey)[0] for ex, ey in chains])
    M9, S9, W9 = gpu.run_steps_ws(L, links, 9)
    M3, S3, W3 = gpu.run_steps_ws(L, links, 3)
    Mr, Sr, Wr = gpu.run_steps_from_ws(L, M3, S3, W3, 3, 6)
    assert np.array_equal(_np(Mr), _np(M9)) and np.array_equal(_np(Sr), _np(S9)) and np.array_equal(_np(Wr), _np(W9))
    state, t = gpu.run_steps_ws(L, links, 0), 0
    for step in (1, 3, 2, 1, 2):
        state = gpu.run_steps_from_ws(L, *state, t, step)
        t += step
    assert t == 9
    assert all(np.array_equal(_np(a), _np(b)) for a, b in zip(state, (M9, S9, W9)))
    for k, (ex, ey) in enumerate(chains):
        check_state(orc, L, ex, ey, 9, _np(M9), _np(S9), _np(W9), k, f"L={L} resumed sample {k}")


def test_band_run_steps_rule(gpu, orc):
    """Limited memory (m_max) and random moves (u) on the band path, step by
    step, against the oracle's variant (R17, R18)."""
    L, p, n = 256, 0.03, 2
    chains = [orc.noise(L, p, int(sd)) for sd in seeds(49, 0, n)]
    links = np.stack([orc.links_from_chains(L, ex, ey)[0] for ex, ey in chains])
    ms = seeds(49, 1, n)
    for m_max, u in ((4, 0), (6, 3)):
        for t in (1, 4, 7):
            M, S, W = gpu.run_steps_ws(L, links, t, m_max=m_max, u=u, move_seeds=ms)
            M, S, W = _np(M), _np(S), _np(W)
            for k, (ex, ey) in enumerate(chains):
                check_state(orc, L, ex, ey, t, M, S, W, k, f"m_max={m_max} u={u} t={t} sample {k}",
                            m_max=m_max, u=u, seed=int(ms[k]))


def test_run_steps_ws_resident_sizes(gpu, orc):
    """Up to L = 128 the workspace form is the resident call."""
    L = 64
    ex, ey = orc.noise(L, 0.03, 12345)
    links = orc.links_from_chains(L, ex, ey)
    M, S, W = gpu.run_steps_ws(L, links, 5)
    M0, S0, W0 = gpu.run_steps(L, links, 5)
    assert np.array_equal(_np(M), _np(M0)) and np.array_equal(_np(S), _np(S0)) and np.array_equal(_np(W), _np(W0))


def _chain_links(orc, L, xs=(), ys=()):
    ex = np.zeros((L, L), np.uint8)
    ey = np.zeros((L, L), np.uint8)
    for x, y in xs:
        ex[y % L, x % L] ^= 1
    for x, y in ys:
        ey[y % L, x % L] ^= 1
    return ex, ey


def test_band_decode_errors(gpu, orc):
    """Explicit error patterns on the band path: chains that cross tile and
    region edges, an antipodal pair (timeout), a winding row (failure at
    T = 0), a pair closing the long way, and random patterns."""
    L = 256
    cases = [
        _chain_links(orc, L, xs=[(x, 5) for x in range(90, 97)]),            # straight chain across a tile edge
        _chain_links(orc, L, ys=[(200, y) for y in range(250, 262)]),        # chain across the row wrap
        _chain_links(orc, L, xs=[(x, 40) for x in range(0, L // 2)]),        # antipodal pair: perfect tie
        _chain_links(orc, L, xs=[(x, 9) for x in range(L)]),                 # full row: winds, no anyon
        _chain_links(orc, L, ys=[(33, y) for y in range(0, L // 2 + 1)]),    # closes the short way round
        _chain_links(orc, L, xs=[(255, 255)], ys=[(0, 255)]),                # corner of the lattice
    ]
    for sd in seeds(50, 0, 4):
        cases.append(orc.noise(L, 0.05, int(sd)))
    links = np.stack([orc.links_from_chains(L, ex, ey)[0] for ex, ey in cases])
    for T_max in (0, 3, 200):
        T, F, S = gpu.decode_errors(L, links, T_max)
        T, F, S = _np(T), _np(F), _np(S).view(np.uint32)
        for k, (ex, ey) in enumerate(cases):
            r = orc.decode_errors(L, ex, ey, T_max)
            assert (T[k], F[k]) == (r["T_dec"], r["flags"]), (k, T_max)
            assert np.array_equal(S[k], r["sigma_words"]), (k, T_max)


def test_band_state_errors(gpu):
    """Argument checks of the band state calls."""
    import torch
    L, n = 256, 1
    links = torch.zeros((n, L * L // 16), dtype=torch.int32, device="cuda")
    M = torch.empty((n, 4, L, L), dtype=torch.int16, device="cuda")
    S = torch.empty((n, L * L // 32), dtype=torch.int32, device="cuda")
    W = torch.empty(n, dtype=torch.uint8, device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    P = gpu._ptr
    rc = gpu.lib().mpd_run_steps_ws(L, P(links), None, n, 3, 0, 0, P(M), P(S), P(W), P(small), 16, None)
    assert rc == -5
    rc = gpu.lib().mpd_run_steps_ws(L, P(links), None, n, 11000, 0, 0, P(M), P(S), P(W), P(small), 16, None)
    assert rc == -3
    rc = gpu.lib().mpd_run_steps_from_ws(L, P(M), P(S), P(W), n, 10000, 1000, 0, 0, None, P(M), P(S), P(W),
                                         P(small), 16, None)
    assert rc == -3
