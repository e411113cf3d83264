"""ctypes binding of the C oracle ``mpd_oracle.c`` plus its build step.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Arrays are numpy; the
C side is plain scalar loops written from the paper's definitions:
Def. "synchronous automaton decoder" (Sec. 2.1), Def. "message passing
automaton, general dimensions" (Sec. 3.2) and Def. "logical failure rate,
expected decoding time, and thresholds" (Sec. 5.1), with i.i.d. noise as in
Sec. 7.  Direction order of register arrays: +x, -x, +y, -y.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mpd_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "libmpd_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP over samples).  Returns the .so path."""
    if not force and os.path.exists(_LIB):
        return _LIB
    os.makedirs(_BUILD, exist_ok=True)
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    lib.orc_philox4x32_10.argtypes = [P, P, P]
    lib.orc_philox4x32_10.restype = None
    lib.orc_noise.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_uint64, P, P]
    lib.orc_noise.restype = ctypes.c_int
    lib.orc_decode_errors.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int,
                                      P, P, P, P, P, P, P]
    lib.orc_decode_errors.restype = ctypes.c_int
    lib.orc_run_steps.argtypes = [ctypes.c_int, ctypes.c_int, P, P, ctypes.c_int,
                                  P, P, P, P, P]
    lib.orc_run_steps.restype = ctypes.c_int
    lib.orc_decode_seeds.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P,
                                     ctypes.c_int64, ctypes.c_int, ctypes.c_int, P, P, P, P]
    lib.orc_decode_seeds.restype = ctypes.c_int
    lib.orc_decode_links.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int64, ctypes.c_int,
                                     ctypes.c_int, P, P, P]
    I, U64 = ctypes.c_int, ctypes.c_uint64
    lib.orc_decode_errors_rule.argtypes = [I, I, I, I, U64, P, P, I, P, P, P, P, P, P, P]
    lib.orc_decode_errors_rule.restype = I
    lib.orc_run_steps_rule.argtypes = [I, I, I, I, U64, P, P, I, P, P, P, P, P]
    lib.orc_run_steps_rule.restype = I
    lib.orc_decode_seeds_rule.argtypes = [I, I, I, I, P, I, P, ctypes.c_int64, I, I, P, P, P, P]
    lib.orc_decode_seeds_rule.restype = I
    lib.orc_decode_links_rule.argtypes = [I, I, I, I, P, P, ctypes.c_int64, I, I, P, P, P]
    lib.orc_decode_links_rule.restype = I
    lib.orc_decode_errors_open.argtypes = [I, I, P, P, I, P, P, P, P, P, P, P]
    lib.orc_decode_errors_open.restype = I
    lib.orc_run_steps_open.argtypes = [I, I, P, P, I, P, P, P, P, P]
    lib.orc_run_steps_open.restype = I
    lib.orc_decode_seeds_open.argtypes = [I, I, P, I, P, ctypes.c_int64, I, I, P, P, P, P]
    lib.orc_decode_seeds_open.restype = I
    lib.orc_decode_links_open.argtypes = [I, I, P, ctypes.c_int64, I, I, P, P, P]
    lib.orc_decode_links_open.restype = I
    lib.orc_decode_links.restype = ctypes.c_int
    lib.orc_async_run.argtypes = [I, I, U64, U64, P, P, I, I, P, P, P, P, P, P, P, P, P]
    lib.orc_async_run.restype = I
    lib.orc_async_decode_seeds.argtypes = [I, I, P, I, P, ctypes.c_int64, U64, I, I, P, P, P, P, P, P]
    lib.orc_async_decode_seeds.restype = I
    lib.orc_uncoord_run.argtypes = [I, I, I] + lib.orc_async_run.argtypes[2:]
    lib.orc_uncoord_run.restype = I
    lib.orc_uncoord_decode_seeds.argtypes = [I, I, I] + lib.orc_async_decode_seeds.argtypes[2:]
    lib.orc_uncoord_decode_seeds.restype = I
    lib.orc_set_reading.argtypes = [I]
    lib.orc_set_reading.restype = I
    lib.orc_get_reading.argtypes = []
    lib.orc_get_reading.restype = I
    lib.orc_decide.argtypes = [P, I, P, P]
    lib.orc_decide.restype = I
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def philox4x32_10(ctr, key):
    """Philox4x32-10 block (Salmon et al., SC'11): 4 counter words, 2 key words."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    _load().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def noise(L: int, p: float, seed: int):
    """i.i.d. link flips (ex, ey) as uint8 [L, L] arrays indexed [y, x]."""
    ex = np.zeros(L * L, dtype=np.uint8)
    ey = np.zeros(L * L, dtype=np.uint8)
    _check(_load().orc_noise(L, float(p), int(seed) & (2**64 - 1), _ptr(ex), _ptr(ey)), "noise")
    return ex.reshape(L, L), ey.reshape(L, L)


def syndrome_of(L: int, ex, ey):
    """Anyon indicator (1 = sigma -1) of an error chain, via a zero-step run."""
    _, sig, _, _ = run_steps(L, ex, ey, 0)
    return (sig == -1).astype(np.uint8)


def pack_bits(bits):
    """Pack a flat 0/1 array as bit i%32 of uint32 word i/32."""
    b = np.asarray(bits, dtype=np.uint8).reshape(-1)
    nw = (b.size + 31) // 32
    pad = np.zeros(nw * 32, dtype=np.uint64)
    pad[: b.size] = b
    w = pad.reshape(nw, 32) << np.arange(32, dtype=np.uint64)
    return w.sum(axis=1).astype(np.uint32)


def decode_errors(L: int, ex, ey, T_max: int, v: int = 3, want_state: bool = False, m_max: int = 0,
                  u: int = 0, seed: int = 0, open_bc: bool = False):
    """Decode one explicit error chain.

    Returns dict(T_dec, flags, sigma_words) and, with want_state, also
    m [4, L, L] int32, cx, cy [L, L] and wind (Wx_E, Wy_E, Wx_C, Wy_C).
    m_max > 0 truncates messages (R17); u > 0 makes every u-th step a random
    move keyed by `seed` (R18); open_bc decodes on the lattice with rough left
    and right boundaries (R19-R22; not combined with m_max / u).
    """
    ex = np.ascontiguousarray(np.asarray(ex, dtype=np.uint8).reshape(-1))
    ey = np.ascontiguousarray(np.asarray(ey, dtype=np.uint8).reshape(-1))
    assert ex.size == L * L and ey.size == L * L
    T = np.zeros(1, dtype=np.int32)
    fl = np.zeros(1, dtype=np.uint8)
    sw = np.zeros((L * L + 31) // 32, dtype=np.uint32)
    m = np.zeros(4 * L * L, dtype=np.int32) if want_state else None
    cx = np.zeros(L * L, dtype=np.uint8) if want_state else None
    cy = np.zeros(L * L, dtype=np.uint8) if want_state else None
    wind = np.zeros(4, dtype=np.int32) if want_state else None
    if open_bc:
        assert m_max == 0 and u == 0
        _check(_load().orc_decode_errors_open(L, v, _ptr(ex), _ptr(ey), int(T_max), _ptr(T), _ptr(fl), _ptr(sw),
                                              _ptr(m), _ptr(cx), _ptr(cy), _ptr(wind)), "decode_errors")
    else:
        _check(_load().orc_decode_errors_rule(L, v, int(m_max), int(u), int(seed), _ptr(ex), _ptr(ey), int(T_max),
                                              _ptr(T), _ptr(fl), _ptr(sw), _ptr(m), _ptr(cx), _ptr(cy), _ptr(wind)),
               "decode_errors")
    out = dict(T_dec=int(T[0]), flags=int(fl[0]), sigma_words=sw)
    if want_state:
        out.update(m=m.reshape(4, L, L), cx=cx.reshape(L, L), cy=cy.reshape(L, L),
                   wind=tuple(int(w) for w in wind))
    return out


def run_steps(L: int, ex, ey, t_exact: int, v: int = 3, record: bool = False, m_max: int = 0, u: int = 0,
              seed: int = 0, open_bc: bool = False):
    """Run exactly t_exact steps.  Returns (m [4,L,L], sigma [L,L] (+1/-1),
    (cx, cy), history) with history [t_exact+1, L, L] anyon indicators or None."""
    ex = np.ascontiguousarray(np.asarray(ex, dtype=np.uint8).reshape(-1))
    ey = np.ascontiguousarray(np.asarray(ey, dtype=np.uint8).reshape(-1))
    m = np.zeros(4 * L * L, dtype=np.int32)
    sig = np.zeros(L * L, dtype=np.int8)
    cx = np.zeros(L * L, dtype=np.uint8)
    cy = np.zeros(L * L, dtype=np.uint8)
    hist = np.zeros((t_exact + 1) * L * L, dtype=np.uint8) if record else None
    if open_bc:
        assert m_max == 0 and u == 0
        _check(_load().orc_run_steps_open(L, v, _ptr(ex), _ptr(ey), int(t_exact), _ptr(m), _ptr(sig), _ptr(cx),
                                          _ptr(cy), _ptr(hist)), "run_steps")
    else:
        _check(_load().orc_run_steps_rule(L, v, int(m_max), int(u), int(seed), _ptr(ex), _ptr(ey), int(t_exact),
                                          _ptr(m), _ptr(sig), _ptr(cx), _ptr(cy), _ptr(hist)), "run_steps")
    return (m.reshape(4, L, L), sig.reshape(L, L), (cx.reshape(L, L), cy.reshape(L, L)),
            None if hist is None else hist.reshape(t_exact + 1, L, L))


def decode_seeds(L: int, p, seeds, T_max: int, v: int = 3, threads: int = 0,
                 want_sigma: bool = True, m_max: int = 0, u: int = 0, open_bc: bool = False):
    """Noise from each seed (one p, or one p per seed) and decode.

    Returns dict(T_dec int32[n], flags uint8[n], sigma_words uint32[n, W] or
    None, threads) where threads is the number of OpenMP threads used.
    """
    seeds = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64).reshape(-1))
    n = seeds.size
    pa = np.ascontiguousarray(np.atleast_1d(np.asarray(p, dtype=np.float64)))
    stride = 1 if pa.size > 1 else 0
    if stride:
        assert pa.size == n
    T = np.zeros(n, dtype=np.int32)
    fl = np.zeros(n, dtype=np.uint8)
    W = (L * L + 31) // 32
    sw = np.zeros((n, W), dtype=np.uint32) if want_sigma else None
    used = ctypes.c_int(0)
    if open_bc:
        assert m_max == 0 and u == 0
        _check(_load().orc_decode_seeds_open(L, v, _ptr(pa), stride, _ptr(seeds), n, int(T_max), int(threads),
                                             _ptr(T), _ptr(fl), _ptr(sw), ctypes.byref(used)), "decode_seeds")
    else:
        _check(_load().orc_decode_seeds_rule(L, v, int(m_max), int(u), _ptr(pa), stride, _ptr(seeds), n,
                                             int(T_max), int(threads), _ptr(T), _ptr(fl), _ptr(sw),
                                             ctypes.byref(used)), "decode_seeds")
    return dict(T_dec=T, flags=fl, sigma_words=sw, threads=int(used.value))


def links_from_chains(L: int, ex, ey):
    """Pack (ex, ey) chains of shape [..., L, L] into link words
    (link id 2*i + dir, bit l%32 of word l/32)."""
    ex = np.asarray(ex, dtype=np.uint8).reshape(-1, L * L)
    ey = np.asarray(ey, dtype=np.uint8).reshape(-1, L * L)
    n = ex.shape[0]
    bits = np.zeros((n, 2 * L * L), dtype=np.uint8)
    bits[:, 0::2] = ex
    bits[:, 1::2] = ey
    return np.stack([pack_bits(b) for b in bits]) if n else np.zeros((0, (2 * L * L + 31) // 32), np.uint32)


def decode_links(L: int, links, T_max: int, v: int = 3, threads: int = 0, m_max: int = 0, u: int = 0,
                 seeds=None, open_bc: bool = False):
    """Decode explicit error chains given as packed link words [n, W]; with
    u > 0 the random moves of chain k are keyed by seeds[k]."""
    lw = (2 * L * L + 31) // 32
    links = np.ascontiguousarray(np.asarray(links, dtype=np.uint32).reshape(-1, lw))
    n = links.shape[0]
    T = np.zeros(n, dtype=np.int32)
    fl = np.zeros(n, dtype=np.uint8)
    sw = np.zeros((n, (L * L + 31) // 32), dtype=np.uint32)
    sd = None if seeds is None else np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64).reshape(-1))
    assert sd is None or sd.size == n
    if open_bc:
        assert m_max == 0 and u == 0
        _check(_load().orc_decode_links_open(L, v, _ptr(links), n, int(T_max), int(threads), _ptr(T), _ptr(fl),
                                             _ptr(sw)), "decode_links")
    else:
        _check(_load().orc_decode_links_rule(L, v, int(m_max), int(u), _ptr(sd), _ptr(links), n, int(T_max),
                                             int(threads), _ptr(T), _ptr(fl), _ptr(sw)), "decode_links")
    return dict(T_dec=T, flags=fl, sigma_words=sw)


def ring_threshold(rho: float) -> int:
    """Ring probability per slot as the integer threshold of R26 (rho * 2^32,
    clamped to [1, 2^32])."""
    return max(1, min(1 << 32, int(rho * 4294967296.0)))


SCHEDULES = {"cyclic": 0, "random": 1}


def async_run(L: int, ex, ey, seed: int, rho: float = 1.0, t_target: int = -1, S_max: int = 100000,
              v: int = 3, uncoordinated: bool = False, schedule: str = "cyclic"):
    """Marching-soldiers desynchronization of the plain rule (R23-R27) on one
    error chain, clock keyed by `seed`.  t_target >= 0 runs until every site
    has performed (v+1) t_target updates; t_target < 0 decodes.  Returns a dict
    with slots, T_async, flags, updates, sigma_words, m (m^new, [4, L, L]),
    tsim [L, L], cx, cy.  uncoordinated=True runs the uncoordinated
    desynchronization instead (R28, with its "cyclic" or "random" schedule)."""
    n = L * L
    ex = np.ascontiguousarray(ex, dtype=np.uint8).reshape(-1)
    ey = np.ascontiguousarray(ey, dtype=np.uint8).reshape(-1)
    slots = np.zeros(1, np.int32)
    T = np.zeros(1, np.int32)
    flags = np.zeros(1, np.uint8)
    upd = np.zeros(1, np.int64)
    words = np.zeros((n + 31) // 32, np.uint32)
    m = np.zeros((4, n), np.int32)
    tsim = np.zeros(n, np.int32)
    cx = np.zeros(n, np.uint8)
    cy = np.zeros(n, np.uint8)
    if uncoordinated:
        fn = lambda L, v, *rest: _load().orc_uncoord_run(L, v, SCHEDULES[schedule], *rest)  # noqa: E731
    else:
        fn = _load().orc_async_run
    _check(fn(L, v, int(seed) & (2**64 - 1), ring_threshold(rho), _ptr(ex), _ptr(ey),
                                 int(t_target), int(S_max), _ptr(slots), _ptr(T), _ptr(flags), _ptr(upd),
                                 _ptr(words), _ptr(m), _ptr(tsim), _ptr(cx), _ptr(cy)), "async_run")
    return {"slots": int(slots[0]), "T_async": int(T[0]), "flags": int(flags[0]), "updates": int(upd[0]),
            "sigma_words": words, "m": m.reshape(4, L, L), "tsim": tsim.reshape(L, L),
            "cx": cx.reshape(L, L), "cy": cy.reshape(L, L)}


def async_decode_seeds(L: int, p, seeds, rho: float = 1.0, S_max: int = 100000, v: int = 3,
                       threads: int = 0, want_sigma: bool = True, uncoordinated: bool = False,
                       schedule: str = "cyclic"):
    """Noise + desynchronized decode per seed (R12, R23-R27; R28 with
    uncoordinated=True)."""
    s = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    n = s.size
    pa = np.ascontiguousarray(np.atleast_1d(np.asarray(p, dtype=np.float64)))
    T = np.zeros(n, np.int32)
    flags = np.zeros(n, np.uint8)
    slots = np.zeros(n, np.int32)
    upd = np.zeros(n, np.int64)
    words = np.zeros((n, (L * L + 31) // 32), np.uint32) if want_sigma else None
    used = ctypes.c_int(0)
    if uncoordinated:
        fn = lambda L, v, *rest: _load().orc_uncoord_decode_seeds(L, v, SCHEDULES[schedule], *rest)  # noqa: E731
    else:
        fn = _load().orc_async_decode_seeds
    _check(fn(L, v, _ptr(pa), 1 if pa.size > 1 else 0, _ptr(s), n,
                                          ring_threshold(rho), int(S_max), int(threads), _ptr(T), _ptr(flags),
                                          _ptr(slots), _ptr(upd), _ptr(words), ctypes.byref(used)),
           "async_decode_seeds")
    out = {"T_async": T, "flags": flags, "slots": slots, "updates": upd, "threads": used.value}
    if want_sigma:
        out["sigma_words"] = words
    return out


# Alternative readings of the garbled or ambiguous passages (bits of
# ``set_reading``); 0 is the reading every test pins (R1-R5 of the C file).
READ_LITERAL_SIGN = 1   # f^a = sgn(m^{-a} - m^{+a}) with an absent message as 0
READ_LITERAL_KEY = 2    # argmin' minimises m + s a/(D+1) as printed (eq. (degbreak))
READ_TIE_MOVES = 4      # move toward the chosen register even on an axis tie
READ_TIE_MIRROR = 8     # ties in the order +y < +x < -x < -y
READ_LINE_SITE = 16     # C^{(a)} = the single site r - s a-hat
READ_LINE_BALL = 32     # C^{(a)} = the unit infinity-ball around r - s a-hat


def set_reading(bits: int) -> None:
    """Select an alternative reading for every later decode (process-wide)."""
    _check(_load().orc_set_reading(int(bits)), "set_reading")


def get_reading() -> int:
    return int(_load().orc_get_reading())


def decide(m, anyon: bool):
    """Forces (f^x, f^y) of one site from its registers m = (m^{+x}, m^{-x},
    m^{+y}, m^{-y}) and its syndrome, as the plain-rule feedback computes them
    (argmin' of eq. (degbreak), force of Def. "message passing automaton,
    general dimensions").  An anyon moves along +a for f^a = -1 and along -a
    for f^a = +1."""
    reg = np.ascontiguousarray(np.asarray(m, dtype=np.int32).reshape(4))
    fx = ctypes.c_int(0)
    fy = ctypes.c_int(0)
    _check(_load().orc_decide(_ptr(reg), 1 if anyon else 0, ctypes.byref(fx), ctypes.byref(fy)), "decide")
    return int(fx.value), int(fy.value)
