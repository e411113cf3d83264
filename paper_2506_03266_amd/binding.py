"""ctypes binding of libmpd.so (C ABI in include/mpd.h) for torch tensors.

Argument marshalling only: every step of a decode runs in the HIP kernels of
the library.  PyTorch supplies device memory and the stream.  There is no
CPU fallback: if the library is missing, the import of a decode function
raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_build", "libmpd.so")

MPD_FLAG_FAIL = 1
MPD_FLAG_TIMEOUT = 2
MPD_T_MAX_LIMIT = 10922
BAND_DRIVER_AUTO, BAND_DRIVER_HOST, BAND_DRIVER_DEVICE = 0, 1, 2

_lib = None


class MPDError(RuntimeError):
    pass


def lib():
    """Load libmpd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise MPDError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, SZ, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
    L.mpd_version.restype = ctypes.c_char_p
    L.mpd_last_error.restype = ctypes.c_char_p
    L.mpd_workspace_bytes.argtypes = [I, I64]
    L.mpd_workspace_bytes.restype = SZ
    L.mpd_decode_batch.argtypes = [I, D, P, I64, I, P, P, P, P, SZ, P]
    L.mpd_decode_batch.restype = I
    L.mpd_decode_errors.argtypes = [I, P, I64, I, P, P, P, P, SZ, P]
    L.mpd_decode_errors.restype = I
    L.mpd_run_steps.argtypes = [I, P, I64, I, P, P, P, P]
    L.mpd_run_steps.restype = I
    L.mpd_decode_rule.argtypes = [I, D, P, I64, I, I, I, P, P, P, P, SZ, P]
    L.mpd_decode_rule.restype = I
    L.mpd_decode_errors_rule.argtypes = [I, P, P, I64, I, I, I, P, P, P, P]
    L.mpd_decode_errors_rule.restype = I
    L.mpd_run_steps_rule.argtypes = [I, P, P, I64, I, I, I, P, P, P, P]
    L.mpd_run_steps_rule.restype = I
    L.mpd_decode_open.argtypes = [I, D, P, I64, I, P, P, P, P, SZ, P]
    L.mpd_decode_open.restype = I
    L.mpd_decode_errors_open.argtypes = [I, P, I64, I, P, P, P, P]
    L.mpd_decode_errors_open.restype = I
    L.mpd_run_steps_open.argtypes = [I, P, I64, I, P, P, P, P]
    L.mpd_run_steps_open.restype = I
    L.mpd_set_band_schedule.argtypes = [I, I, I]
    L.mpd_set_band_schedule.restype = I
    L.mpd_get_band_schedule.argtypes = [I, P, P]
    L.mpd_get_band_schedule.restype = I
    L.mpd_set_band_driver.argtypes = [I, I]
    L.mpd_set_band_driver.restype = I
    L.mpd_get_band_driver.argtypes = [I, P]
    L.mpd_get_band_driver.restype = I
    L.mpd_set_band_bits.argtypes = [I, I]
    L.mpd_set_band_bits.restype = I
    L.mpd_get_band_bits.argtypes = [I, P]
    L.mpd_get_band_bits.restype = I
    L.mpd_autotune_band.argtypes = [I, D, P, I64, I, P, P, P, SZ, P, P, P, P]
    L.mpd_autotune_band.restype = I
    L.mpd_mixed_workspace_bytes.argtypes = [I, P, P]
    L.mpd_mixed_workspace_bytes.restype = SZ
    L.mpd_decode_mixed.argtypes = [I, P, P, P, P, I, P, P, P, P, SZ, P]
    L.mpd_decode_mixed.restype = I
    L.mpd_profile.argtypes = [I]
    L.mpd_profile.restype = I
    L.mpd_profile_read.argtypes = [ctypes.c_char_p, P, P]
    L.mpd_profile_read.restype = I
    L.mpd_syndrome_counts.argtypes = [I, D, P, P, I64, P, P]
    L.mpd_syndrome_counts.restype = I
    L.mpd_cnn_init.argtypes = [P, ctypes.c_uint64, P]
    L.mpd_cnn_init.restype = I
    L.mpd_cnn_forward_workspace_bytes.argtypes = [I, I64]
    L.mpd_cnn_forward_workspace_bytes.restype = SZ
    L.mpd_cnn_forward.argtypes = [P, I, I64, P, P, P, P, P, SZ, P]
    L.mpd_cnn_forward.restype = I
    L.mpd_cnn_train_workspace_bytes.argtypes = [I, I64]
    L.mpd_cnn_train_workspace_bytes.restype = SZ
    L.mpd_cnn_loss_grad.argtypes = [P, I, I64, P, P, P, P, P, P, SZ, P]
    L.mpd_cnn_loss_grad.restype = I
    F = ctypes.c_float
    L.mpd_cnn_adam_step.argtypes = [P, P, P, P, I, F, F, F, F, P]
    L.mpd_cnn_adam_step.restype = I
    L.mpd_learned_workspace_bytes.argtypes = [I, I64]
    L.mpd_learned_workspace_bytes.restype = SZ
    L.mpd_decode_learned.argtypes = [I, D, P, P, I64, I, P, I, P, P, P, P, P, P, P, SZ, P]
    L.mpd_decode_learned.restype = I
    L.mpd_run_steps_from.argtypes = [I, P, P, P, I64, I, I, I, I, P, P, P, P, P]
    L.mpd_decode_batch_static.argtypes = [I, D, P, I64, I, P, P, P, P]
    L.mpd_decode_batch_static.restype = I
    L.mpd_run_steps_ws.argtypes = [I, P, P, I64, I, I, I, P, P, P, P, SZ, P]
    L.mpd_run_steps_ws.restype = I
    L.mpd_run_steps_from_ws.argtypes = [I, P, P, P, I64, I, I, I, I, P, P, P, P, P, SZ, P]
    L.mpd_run_steps_from_ws.restype = I
    L.mpd_run_steps_from.restype = I
    L.mpd_decode_async.argtypes = [I, D, P, I64, D, I, P, P, P, P, P, P]
    L.mpd_decode_async.restype = I
    L.mpd_run_async.argtypes = [I, P, P, I64, I, D, I, P, P, P, P, P, P, P]
    L.mpd_run_async.restype = I
    L.mpd_decode_uncoord.argtypes = [I, D, P, I64, D, I, I, P, P, P, P, P, P]
    L.mpd_decode_uncoord.restype = I
    L.mpd_run_uncoord.argtypes = [I, P, P, I64, I, D, I, I, P, P, P, P, P, P, P]
    L.mpd_run_uncoord.restype = I
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != 0:
        msg = lib().mpd_last_error().decode()
        raise MPDError(f"{what} failed ({rc}): {msg}")


def _stream_ptr(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _seeds_tensor(seeds, device):
    if isinstance(seeds, torch.Tensor):
        assert seeds.dtype in (torch.int64, torch.uint64)
        return seeds.to(device).contiguous()
    a = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64)).view(np.int64)
    return torch.from_numpy(a).to(device)


def syndrome_words(L: int) -> int:
    return (L * L + 31) // 32


def link_words(L: int) -> int:
    return (2 * L * L + 31) // 32


def workspace_bytes(L: int, n: int) -> int:
    return int(lib().mpd_workspace_bytes(L, n))


def alloc_workspace(L: int, n: int, device="cuda"):
    nb = workspace_bytes(L, n)
    return torch.empty(max(nb, 1), dtype=torch.uint8, device=device)


def decode_batch(L: int, p: float, seeds, T_max: int = 4096, want_syndrome: bool = True,
                 workspace=None, out=None, stream=None):
    """Decode len(seeds) seeded noise samples.

    Returns (T_dec int32[n], flags uint8[n], syndrome int32[n, W] or None) on
    the device.  `out` may pass preallocated (T_dec, flags, syndrome).
    """
    dev = torch.device("cuda")
    s = _seeds_tensor(seeds, dev)
    n = s.numel()
    if out is None:
        T = torch.empty(n, dtype=torch.int32, device=dev)
        F = torch.empty(n, dtype=torch.uint8, device=dev)
        S = torch.empty((n, syndrome_words(L)), dtype=torch.int32, device=dev) if want_syndrome else None
    else:
        T, F, S = out
    ws = workspace if workspace is not None else alloc_workspace(L, n)
    rc = lib().mpd_decode_batch(L, float(p), _ptr(s), n, int(T_max), _ptr(T), _ptr(F), _ptr(S), _ptr(ws),
                                ws.numel(), _stream_ptr(stream))
    _check(rc, "mpd_decode_batch")
    return T, F, S


STATIC_SCRATCH_BYTES = 128 << 20


def decode_batch_static(L: int, p: float, seeds, T_max: int = 4096, want_syndrome: bool = True, out=None,
                        stream=None):
    """mpd_decode_batch_static: decode_batch without a workspace (the
    library's own scratch on the device; calls on one device must not
    overlap).  Returns (T_dec, flags, syndrome)."""
    dev = torch.device("cuda")
    s = _seeds_tensor(seeds, dev)
    n = s.numel()
    if out is None:
        T = torch.empty(n, dtype=torch.int32, device=dev)
        F = torch.empty(n, dtype=torch.uint8, device=dev)
        S = torch.empty((n, syndrome_words(L)), dtype=torch.int32, device=dev) if want_syndrome else None
    else:
        T, F, S = out
    rc = lib().mpd_decode_batch_static(L, float(p), _ptr(s), n, int(T_max), _ptr(T), _ptr(F), _ptr(S),
                                       _stream_ptr(stream))
    _check(rc, "mpd_decode_batch_static")
    return T, F, S


def _links_tensor(L, links, dev):
    if not isinstance(links, torch.Tensor):
        links = torch.from_numpy(np.ascontiguousarray(np.asarray(links, dtype=np.uint32)).view(np.int32))
    return links.to(dev).contiguous().view(-1, link_words(L))


def decode_errors(L: int, links, T_max: int = 4096, want_syndrome: bool = True, stream=None, m_max: int = 0,
                  u: int = 0, move_seeds=None):
    """Decode explicit error patterns given as link words [n, link_words(L)].
    m_max / u select the limited-memory variant (random moves keyed by
    move_seeds, one per pattern)."""
    dev = torch.device("cuda")
    links = _links_tensor(L, links, dev)
    n = links.shape[0]
    T = torch.empty(n, dtype=torch.int32, device=dev)
    F = torch.empty(n, dtype=torch.uint8, device=dev)
    S = torch.empty((n, syndrome_words(L)), dtype=torch.int32, device=dev) if want_syndrome else None
    if m_max == 0 and u == 0 and move_seeds is None:
        ws = alloc_workspace(L, n)
        rc = lib().mpd_decode_errors(L, _ptr(links), n, int(T_max), _ptr(T), _ptr(F), _ptr(S), _ptr(ws), ws.numel(),
                                     _stream_ptr(stream))
        _check(rc, "mpd_decode_errors")
    else:
        ms = None if move_seeds is None else _seeds_tensor(move_seeds, dev)
        rc = lib().mpd_decode_errors_rule(L, _ptr(links), _ptr(ms), n, int(T_max), int(m_max), int(u), _ptr(T),
                                          _ptr(F), _ptr(S), _stream_ptr(stream))
        _check(rc, "mpd_decode_errors_rule")
    return T, F, S


def run_steps(L: int, links, t_exact: int, stream=None, m_max: int = 0, u: int = 0, move_seeds=None):
    """Run exactly t_exact steps; returns (m int16[n,4,L,L], syndrome int32[n,W], wind uint8[n])."""
    dev = torch.device("cuda")
    links = _links_tensor(L, links, dev)
    n = links.shape[0]
    M = torch.empty((n, 4, L, L), dtype=torch.int16, device=dev)
    S = torch.empty((n, syndrome_words(L)), dtype=torch.int32, device=dev)
    W = torch.empty(n, dtype=torch.uint8, device=dev)
    if m_max == 0 and u == 0 and move_seeds is None:
        rc = lib().mpd_run_steps(L, _ptr(links), n, int(t_exact), _ptr(M), _ptr(S), _ptr(W), _stream_ptr(stream))
        _check(rc, "mpd_run_steps")
    else:
        ms = None if move_seeds is None else _seeds_tensor(move_seeds, dev)
        rc = lib().mpd_run_steps_rule(L, _ptr(links), _ptr(ms), n, int(t_exact), int(m_max), int(u), _ptr(M),
                                      _ptr(S), _ptr(W), _stream_ptr(stream))
        _check(rc, "mpd_run_steps_rule")
    return M, S, W


def run_steps_ws(L: int, links, t_exact: int, stream=None, m_max: int = 0, u: int = 0, move_seeds=None,
                 workspace=None):
    """mpd_run_steps_ws: exactly t_exact steps from explicit errors at any
    supported L (the band path from L = 256 on); returns (m int16[n,4,L,L],
    syndrome int32[n,W], wind uint8[n])."""
    dev = torch.device("cuda")
    links = _links_tensor(L, links, dev)
    n = links.shape[0]
    M = torch.empty((n, 4, L, L), dtype=torch.int16, device=dev)
    S = torch.empty((n, syndrome_words(L)), dtype=torch.int32, device=dev)
    W = torch.empty(n, dtype=torch.uint8, device=dev)
    ws = alloc_workspace(L, n) if workspace is None else workspace
    ms = None if move_seeds is None else _seeds_tensor(move_seeds, dev)
    rc = lib().mpd_run_steps_ws(L, _ptr(links), _ptr(ms), n, int(t_exact), int(m_max), int(u), _ptr(M), _ptr(S),
                                _ptr(W), _ptr(ws), ws.numel(), _stream_ptr(stream))
    _check(rc, "mpd_run_steps_ws")
    return M, S, W


def run_steps_from_ws(L: int, M, S, W, t_start: int, t_exact: int, stream=None, m_max: int = 0, u: int = 0,
                      move_seeds=None, workspace=None, out=None):
    """mpd_run_steps_from_ws: resume exported states at any supported L."""
    dev = torch.device("cuda")
    n = M.shape[0]
    Mo, So, Wo = (torch.empty_like(M), torch.empty_like(S), torch.empty_like(W)) if out is None else out
    ws = alloc_workspace(L, n) if workspace is None else workspace
    ms = None if move_seeds is None else _seeds_tensor(move_seeds, dev)
    rc = lib().mpd_run_steps_from_ws(L, _ptr(M), _ptr(S), _ptr(W), n, int(t_start), int(t_exact), int(m_max),
                                     int(u), _ptr(ms), _ptr(Mo), _ptr(So), _ptr(Wo), _ptr(ws), ws.numel(),
                                     _stream_ptr(stream))
    _check(rc, "mpd_run_steps_from_ws")
    return Mo, So, Wo


ASYNC_SLOT_LIMIT = 65000
UNCOORD_SCHEDULES = {"cyclic": 0, "random": 1}


def decode_async(L: int, p: float, seeds, rho: float, S_max: int = ASYNC_SLOT_LIMIT, want_syndrome: bool = True,
                 out=None, stream=None, uncoordinated: bool = False, schedule: str = "cyclic"):
    """Marching-soldiers desynchronized decode of seeded noise (5 <= L <= 64):
    the seed keys the noise and the clock, rho is the ring probability per
    slot.  Returns (T_async int32[n], flags uint8[n], slots int32[n],
    updates int64[n], syndrome int32[n, W] or None) on the device; `out` may
    pass all five preallocated.  uncoordinated=True runs the uncoordinated
    desynchronization (mpd_decode_uncoord) instead, with its "cyclic" or
    "random" schedule."""
    dev = torch.device("cuda")
    s = _seeds_tensor(seeds, dev)
    n = s.numel()
    if out is None:
        T = torch.empty(n, dtype=torch.int32, device=dev)
        F = torch.empty(n, dtype=torch.uint8, device=dev)
        SL = torch.empty(n, dtype=torch.int32, device=dev)
        U = torch.empty(n, dtype=torch.int64, device=dev)
        S = torch.empty((n, syndrome_words(L)), dtype=torch.int32, device=dev) if want_syndrome else None
    else:
        T, F, SL, U, S = out
    if uncoordinated:
        rc = lib().mpd_decode_uncoord(L, float(p), _ptr(s), n, float(rho), int(S_max), UNCOORD_SCHEDULES[schedule],
                                      _ptr(T), _ptr(F), _ptr(SL), _ptr(U), _ptr(S), _stream_ptr(stream))
        _check(rc, "mpd_decode_uncoord")
    else:
        rc = lib().mpd_decode_async(L, float(p), _ptr(s), n, float(rho), int(S_max), _ptr(T), _ptr(F), _ptr(SL),
                                    _ptr(U), _ptr(S), _stream_ptr(stream))
        _check(rc, "mpd_decode_async")
    return T, F, SL, U, S


def run_async(L: int, links, clock_seeds, t_target: int, rho: float, S_max: int = ASYNC_SLOT_LIMIT, stream=None,
              uncoordinated: bool = False, schedule: str = "cyclic"):
    """Desynchronized run of explicit error patterns until every site has
    completed t_target decoder steps (or S_max slots).  Returns (slots
    int32[n], updates int64[n], m int16[n,4,L,L], tsim int16[n,L,L] holding
    uint16 values, syndrome int32[n,W], wind uint8[n]).  uncoordinated=True
    runs mpd_run_uncoord."""
    dev = torch.device("cuda")
    links = _links_tensor(L, links, dev)
    n = links.shape[0]
    cs = _seeds_tensor(clock_seeds, dev)
    if cs.numel() != n:
        raise ValueError("one clock seed per pattern")
    SL = torch.empty(n, dtype=torch.int32, device=dev)
    U = torch.empty(n, dtype=torch.int64, device=dev)
    M = torch.empty((n, 4, L, L), dtype=torch.int16, device=dev)
    TS = torch.empty((n, L, L), dtype=torch.int16, device=dev)
    S = torch.empty((n, syndrome_words(L)), dtype=torch.int32, device=dev)
    W = torch.empty(n, dtype=torch.uint8, device=dev)
    if uncoordinated:
        rc = lib().mpd_run_uncoord(L, _ptr(links), _ptr(cs), n, int(t_target), float(rho), int(S_max),
                                   UNCOORD_SCHEDULES[schedule], _ptr(SL), _ptr(U), _ptr(M), _ptr(TS), _ptr(S), _ptr(W),
                                   _stream_ptr(stream))
        _check(rc, "mpd_run_uncoord")
    else:
        rc = lib().mpd_run_async(L, _ptr(links), _ptr(cs), n, int(t_target), float(rho), int(S_max), _ptr(SL),
                                 _ptr(U), _ptr(M), _ptr(TS), _ptr(S), _ptr(W), _stream_ptr(stream))
        _check(rc, "mpd_run_async")
    return SL, U, M, TS, S, W


def run_steps_from(L: int, M, S, W, t_start: int, t_exact: int, stream=None, m_max: int = 0, u: int = 0,
                   move_seeds=None, out=None):
    """Resume exported states (m int16[n,4,L,L], syndrome int32[n,W], wind
    uint8[n], as run_steps returns them after t_start steps) for t_exact more
    steps; returns the new (m, syndrome, wind).  `out` may pass the three
    output tensors (they may be the inputs themselves)."""
    dev = torch.device("cuda")
    n = M.shape[0]
    if out is None:
        Mo = torch.empty_like(M)
        So = torch.empty_like(S)
        Wo = torch.empty_like(W)
    else:
        Mo, So, Wo = out
    ms = None if move_seeds is None else _seeds_tensor(move_seeds, dev)
    rc = lib().mpd_run_steps_from(L, _ptr(M), _ptr(S), _ptr(W), n, int(t_start), int(t_exact), int(m_max), int(u),
                                  _ptr(ms), _ptr(Mo), _ptr(So), _ptr(Wo), _stream_ptr(stream))
    _check(rc, "mpd_run_steps_from")
    return Mo, So, Wo


def decode_open(L: int, p: float, seeds, T_max: int = 4096, want_syndrome: bool = True, workspace=None, out=None,
                stream=None):
    """Decode seeded noise on the open lattice (rough left / right columns,
    smooth top / bottom rows): L <= 128 or a multiple of 16 from 256."""
    dev = torch.device("cuda")
    s = _seeds_tensor(seeds, dev)
    n = s.numel()
    if out is None:
        T = torch.empty(n, dtype=torch.int32, device=dev)
        F = torch.empty(n, dtype=torch.uint8, device=dev)
        S = torch.empty((n, syndrome_words(L)), dtype=torch.int32, device=dev) if want_syndrome else None
    else:
        T, F, S = out
    ws = workspace if workspace is not None else alloc_workspace(L, n)
    _check(lib().mpd_decode_open(L, float(p), _ptr(s), n, int(T_max), _ptr(T), _ptr(F), _ptr(S), _ptr(ws), ws.numel(),
                                 _stream_ptr(stream)), "mpd_decode_open")
    return T, F, S


def decode_errors_open(L: int, links, T_max: int = 4096, want_syndrome: bool = True, stream=None):
    """Explicit error patterns on the open lattice."""
    dev = torch.device("cuda")
    links = _links_tensor(L, links, dev)
    n = links.shape[0]
    T = torch.empty(n, dtype=torch.int32, device=dev)
    F = torch.empty(n, dtype=torch.uint8, device=dev)
    S = torch.empty((n, syndrome_words(L)), dtype=torch.int32, device=dev) if want_syndrome else None
    _check(lib().mpd_decode_errors_open(L, _ptr(links), n, int(T_max), _ptr(T), _ptr(F), _ptr(S),
                                        _stream_ptr(stream)), "mpd_decode_errors_open")
    return T, F, S


def run_steps_open(L: int, links, t_exact: int, stream=None):
    """Exactly t_exact steps on the open lattice; returns (m, syndrome, wind)."""
    dev = torch.device("cuda")
    links = _links_tensor(L, links, dev)
    n = links.shape[0]
    M = torch.empty((n, 4, L, L), dtype=torch.int16, device=dev)
    S = torch.empty((n, syndrome_words(L)), dtype=torch.int32, device=dev)
    W = torch.empty(n, dtype=torch.uint8, device=dev)
    _check(lib().mpd_run_steps_open(L, _ptr(links), n, int(t_exact), _ptr(M), _ptr(S), _ptr(W), _stream_ptr(stream)),
           "mpd_run_steps_open")
    return M, S, W


def decode_rule(L: int, p: float, seeds, T_max: int = 4096, m_max: int = 0, u: int = 0, want_syndrome: bool = True,
                workspace=None, out=None, stream=None):
    """decode_batch with the limited-memory variant: messages truncated at
    m_max (0: none), a random move of every anyon every u steps (0: none)."""
    dev = torch.device("cuda")
    s = _seeds_tensor(seeds, dev)
    n = s.numel()
    if out is None:
        T = torch.empty(n, dtype=torch.int32, device=dev)
        F = torch.empty(n, dtype=torch.uint8, device=dev)
        S = torch.empty((n, syndrome_words(L)), dtype=torch.int32, device=dev) if want_syndrome else None
    else:
        T, F, S = out
    ws = workspace if workspace is not None else alloc_workspace(L, n)
    rc = lib().mpd_decode_rule(L, float(p), _ptr(s), n, int(T_max), int(m_max), int(u), _ptr(T), _ptr(F), _ptr(S),
                               _ptr(ws), ws.numel(), _stream_ptr(stream))
    _check(rc, "mpd_decode_rule")
    return T, F, S


def profile(enable: bool):
    """Start (clearing old records) or stop per-launch kernel timing."""
    _check(lib().mpd_profile(1 if enable else 0), "mpd_profile")


def profile_read(kernel: str):
    """(total_ms, launches) recorded for a kernel name."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(lib().mpd_profile_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)), "mpd_profile_read")
    return ms.value, cnt.value


def set_band_schedule(k_first: int, k_next: int, L: int = 0):
    """Decoder steps per pass of the band path (first pass, later passes);
    L = 0 sets the default for every L."""
    _check(lib().mpd_set_band_schedule(int(L), int(k_first), int(k_next)), "mpd_set_band_schedule")


def get_band_schedule(L: int = 0):
    a, c = ctypes.c_int(0), ctypes.c_int(0)
    _check(lib().mpd_get_band_schedule(int(L), ctypes.byref(a), ctypes.byref(c)), "mpd_get_band_schedule")
    return a.value, c.value


def set_band_driver(driver: int, L: int = 0):
    """Who drives the band path's later passes: BAND_DRIVER_AUTO, _HOST or
    _DEVICE; L = 0 sets the default and every per-L setting."""
    _check(lib().mpd_set_band_driver(int(L), int(driver)), "mpd_set_band_driver")


def get_band_driver(L: int = 0) -> int:
    d = ctypes.c_int(-1)
    _check(lib().mpd_get_band_driver(int(L), ctypes.byref(d)), "mpd_get_band_driver")
    return d.value


def set_band_bits(k_bits: int, L: int = 0):
    """Decoder steps of a plain batch at L = 64, 128 or 256 that run in the
    bit-sliced whole-lattice kernel first (0..10; 0: the band path's first
    pass, or at L = 64 and 128 the whole-lattice kernel alone); L = 0 sets the
    default and every per-L setting."""
    _check(lib().mpd_set_band_bits(int(L), int(k_bits)), "mpd_set_band_bits")


def get_band_bits(L: int = 0) -> int:
    k = ctypes.c_int(-1)
    _check(lib().mpd_get_band_bits(int(L), ctypes.byref(k)), "mpd_get_band_bits")
    return k.value


def save_band_tuning(path: str, Ls) -> dict:
    """Write the band-path settings of the lattice sizes Ls (schedule,
    driver and bit-sliced steps, as the autotuner or the setters left them) and the defaults to a
    JSON file, so that a later process can reuse them without re-tuning.
    Returns what was written."""
    import json
    state = {"default": {"k_first": get_band_schedule(0)[0], "k_next": get_band_schedule(0)[1],
                         "driver": get_band_driver(0), "k_bits": get_band_bits(0)},
             "per_L": {str(int(L)): {"k_first": get_band_schedule(int(L))[0], "k_next": get_band_schedule(int(L))[1],
                                     "driver": get_band_driver(int(L)), "k_bits": get_band_bits(int(L))}
                       for L in Ls}}
    with open(path, "w") as f:
        json.dump(state, f, indent=1)
    return state


def load_band_tuning(path: str) -> dict:
    """Apply band-path settings written by save_band_tuning: the defaults
    first, then every per-L entry.  Returns what was read."""
    import json
    with open(path) as f:
        state = json.load(f)
    d = state["default"]
    set_band_schedule(d["k_first"], d["k_next"], 0)
    set_band_driver(d["driver"], 0)
    set_band_bits(d.get("k_bits", 10), 0)
    for L, e in state["per_L"].items():
        set_band_schedule(e["k_first"], e["k_next"], int(L))
        set_band_driver(e["driver"], int(L))
        set_band_bits(e.get("k_bits", 10), int(L))
    return state


def autotune_band(L: int, p: float, seeds, T_max: int = 4096, stream=None):
    """Time the band-path schedules (driver x k_first x k_next, and the steps
    of the bit-sliced first kernel: 0, 3, 5, 8, 10 at L = 256, 0, 4, 5, 6 of
    the tiled one above) on a probe batch, time the eight fastest again in
    five interleaved rounds and keep the lowest median for L.  Returns
    (k_first, k_next, median ms); get_band_driver(L) and get_band_bits(L)
    give the chosen driver and bit-sliced steps."""
    dev = torch.device("cuda")
    s = _seeds_tensor(seeds, dev)
    n = s.numel()
    T = torch.empty(n, dtype=torch.int32, device=dev)
    F = torch.empty(n, dtype=torch.uint8, device=dev)
    ws = alloc_workspace(L, n)
    kf, kn, ms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_float(0.0)
    rc = lib().mpd_autotune_band(L, float(p), _ptr(s), n, int(T_max), _ptr(T), _ptr(F), _ptr(ws), ws.numel(),
                                 _stream_ptr(stream), ctypes.byref(kf), ctypes.byref(kn), ctypes.byref(ms))
    _check(rc, "mpd_autotune_band")
    return kf.value, kn.value, ms.value


def mixed_workspace(classes, device="cuda"):
    """Workspace for decode_mixed over classes = [(L, count), ...]."""
    hL = np.ascontiguousarray([c[0] for c in classes], dtype=np.int32)
    hC = np.ascontiguousarray([c[1] for c in classes], dtype=np.int64)
    nb = int(lib().mpd_mixed_workspace_bytes(len(hL), hL.ctypes.data_as(ctypes.c_void_p),
                                             hC.ctypes.data_as(ctypes.c_void_p)))
    return torch.empty(max(nb, 1), dtype=torch.uint8, device=device)


def decode_mixed(classes, p, seeds, T_max: int = 4096, want_syndrome: bool = True, workspace=None, out=None,
                 stream=None):
    """Decode a batch ordered by class: classes = [(L, count), ...], p and seeds
    per sample.  Returns (T_dec, flags, syndrome words concatenated by class)."""
    dev = torch.device("cuda")
    hL = np.ascontiguousarray([c[0] for c in classes], dtype=np.int32)
    hC = np.ascontiguousarray([c[1] for c in classes], dtype=np.int64)
    n = int(hC.sum())
    s = _seeds_tensor(seeds, dev)
    pt = p if isinstance(p, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(p, dtype=np.float64))
    pt = pt.to(dev, dtype=torch.float64).contiguous()
    assert s.numel() == n and pt.numel() == n
    W = int(sum(c * syndrome_words(L) for L, c in zip(hL, hC)))
    if out is None:
        T = torch.empty(n, dtype=torch.int32, device=dev)
        F = torch.empty(n, dtype=torch.uint8, device=dev)
        S = torch.empty(W, dtype=torch.int32, device=dev) if want_syndrome else None
    else:
        T, F, S = out
    nb = int(lib().mpd_mixed_workspace_bytes(len(hL), hL.ctypes.data_as(ctypes.c_void_p),
                                             hC.ctypes.data_as(ctypes.c_void_p)))
    ws = workspace if workspace is not None else torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    rc = lib().mpd_decode_mixed(len(hL), hL.ctypes.data_as(ctypes.c_void_p), hC.ctypes.data_as(ctypes.c_void_p),
                                _ptr(pt), _ptr(s), int(T_max), _ptr(T), _ptr(F), _ptr(S), _ptr(ws), ws.numel(),
                                _stream_ptr(stream))
    _check(rc, "mpd_decode_mixed")
    return T, F, S


# ---------------------------------------------------------------------------
# Learned scheduling: block counts, the decode-time predictor, scheduled decode
# ---------------------------------------------------------------------------

CNN_PARAMS = 7137


def _p_tensor(p, n, dev):
    if isinstance(p, (float, int)):
        return None
    pt = p if isinstance(p, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(p, dtype=np.float64))
    pt = pt.to(dev, dtype=torch.float64).contiguous()
    assert pt.numel() == n
    return pt


def syndrome_counts(L: int, p, seeds, out=None, stream=None):
    """Anyons per 8x8 block, uint8 [n, L/8, L/8]; p is a number or per-sample values."""
    dev = torch.device("cuda")
    s = _seeds_tensor(seeds, dev)
    n = s.numel()
    pt = _p_tensor(p, n, dev)
    c = out if out is not None else torch.empty((n, L // 8, L // 8), dtype=torch.uint8, device=dev)
    rc = lib().mpd_syndrome_counts(L, float(p) if pt is None else 0.0, _ptr(pt), _ptr(s), n, _ptr(c),
                                   _stream_ptr(stream))
    _check(rc, "mpd_syndrome_counts")
    return c


def cnn_init(seed: int, stream=None):
    """Fresh parameter vector (float32 [7137]) on the device."""
    prm = torch.empty(CNN_PARAMS, dtype=torch.float32, device="cuda")
    _check(lib().mpd_cnn_init(_ptr(prm), int(seed) & (2**64 - 1), _stream_ptr(stream)), "mpd_cnn_init")
    return prm


def cnn_forward(counts, params, want_feat: bool = False, stream=None):
    """Predictions (float32 [n]) for count maps [n, M, M]; with want_feat also
    the pooled maxima [n, 16] and their positions [n, 16]."""
    counts = counts.contiguous()
    n, M = counts.shape[0], counts.shape[-1]
    dev = counts.device
    pred = torch.empty(n, dtype=torch.float32, device=dev)
    feat = torch.empty((n, 16), dtype=torch.float32, device=dev) if want_feat else None
    amax = torch.empty((n, 16), dtype=torch.int32, device=dev) if want_feat else None
    nb = int(lib().mpd_cnn_forward_workspace_bytes(M, n))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=dev)
    rc = lib().mpd_cnn_forward(_ptr(counts), M, n, _ptr(params), _ptr(pred), _ptr(feat), _ptr(amax), _ptr(ws),
                               ws.numel(), _stream_ptr(stream))
    _check(rc, "mpd_cnn_forward")
    return (pred, feat, amax) if want_feat else pred


def train_workspace(M: int, n: int, device="cuda"):
    nb = int(lib().mpd_cnn_train_workspace_bytes(M, n))
    return torch.empty(max(nb, 1), dtype=torch.uint8, device=device)


def cnn_loss_grad(counts, params, target, workspace=None, out=None, stream=None):
    """Mean squared error and its gradient: returns (loss [1], grad [7137], pred [n])."""
    counts = counts.contiguous()
    n, M = counts.shape[0], counts.shape[-1]
    dev = counts.device
    if out is None:
        loss = torch.empty(1, dtype=torch.float32, device=dev)
        grad = torch.empty(CNN_PARAMS, dtype=torch.float32, device=dev)
        pred = torch.empty(n, dtype=torch.float32, device=dev)
    else:
        loss, grad, pred = out
    ws = workspace if workspace is not None else train_workspace(M, n, dev)
    target = target.to(dev, dtype=torch.float32).contiguous()
    rc = lib().mpd_cnn_loss_grad(_ptr(counts), M, n, _ptr(params), _ptr(target), _ptr(grad),
                                 _ptr(loss), _ptr(pred), _ptr(ws), ws.numel(), _stream_ptr(stream))
    _check(rc, "mpd_cnn_loss_grad")
    return loss, grad, pred


def cnn_adam_step(params, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8, stream=None):
    """In-place Adam update of params (and its moments m, v)."""
    rc = lib().mpd_cnn_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), int(step), float(lr), float(beta1),
                                 float(beta2), float(eps), _stream_ptr(stream))
    _check(rc, "mpd_cnn_adam_step")


def learned_workspace(L: int, n: int, device="cuda"):
    nb = int(lib().mpd_learned_workspace_bytes(L, n))
    return torch.empty(max(nb, 1), dtype=torch.uint8, device=device)


def decode_learned(L: int, p, seeds, params, edges, depths, T_max: int = 4096, want_syndrome: bool = True,
                   workspace=None, out=None, stream=None, want_pred: bool = True):
    """Decode with learned scheduling: samples with edges[b-1] <= pred < edges[b]
    start with a pass of depths[b] steps.  p is a number or per-sample values.
    Returns (T_dec, flags, syndrome, pred), results identical to decode_batch
    (decode_mixed with the one class (L, n) for per-sample p).  Without
    predictions (want_pred False, or out[3] None) a one-group policy skips
    the network: the plain decode at depths[0]."""
    dev = torch.device("cuda")
    s = _seeds_tensor(seeds, dev)
    n = s.numel()
    pt = _p_tensor(p, n, dev)
    if out is None:
        T = torch.empty(n, dtype=torch.int32, device=dev)
        F = torch.empty(n, dtype=torch.uint8, device=dev)
        S = torch.empty((n, syndrome_words(L)), dtype=torch.int32, device=dev) if want_syndrome else None
        pred = torch.empty(n, dtype=torch.float32, device=dev) if want_pred else None
    else:
        T, F, S, pred = out
    he = np.ascontiguousarray(edges, dtype=np.float32)
    hd = np.ascontiguousarray(depths, dtype=np.int32)
    assert hd.size == he.size + 1
    ws = workspace if workspace is not None else learned_workspace(L, n)
    rc = lib().mpd_decode_learned(L, float(p) if pt is None else 0.0, _ptr(pt), _ptr(s), n, int(T_max),
                                  _ptr(params), int(hd.size),
                                  he.ctypes.data_as(ctypes.c_void_p), hd.ctypes.data_as(ctypes.c_void_p), _ptr(T),
                                  _ptr(F), _ptr(S), _ptr(pred), _ptr(ws), ws.numel(), _stream_ptr(stream))
    _check(rc, "mpd_decode_learned")
    return T, F, S, pred
