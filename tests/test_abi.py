"""The C ABI library loads, exports every declared symbol and rejects bad
arguments before touching the GPU (runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    import paper_2506_03266_amd.binding as b
    if not os.path.exists(b.LIB_PATH):
        from paper_2506_03266_amd import build
        build.build()
    return b.lib()


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(mpd_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_exports_every_declared_symbol(lib):
    names = declared_symbols()
    assert "mpd_decode_batch" in names and len(names) >= 6
    for name in names:
        assert hasattr(lib, name), name


def test_version_and_workspace(lib):
    assert lib.mpd_version().startswith(b"mpd")
    assert lib.mpd_workspace_bytes(64, 10000) == 0           # on-chip path
    assert lib.mpd_workspace_bytes(256, 0) == 0
    w1 = lib.mpd_workspace_bytes(256, 1)
    w2 = lib.mpd_workspace_bytes(256, 4096)
    assert w1 > 2 * 256 * 256 * 8 and w2 > 4096 * 2 * 256 * 256 * 8


@pytest.mark.parametrize("L,p,n,T,code", [
    (2, 0.1, 1, 8, -1), (1025, 0.1, 1, 8, -1), (200, 0.1, 1, 8, -1), (127, 0.1, 1, 8, -1),
    (16400, 0.1, 1, 8, -1),
    (16, -0.1, 1, 8, -2), (16, 1.5, 1, 8, -2), (16, float("nan"), 1, 8, -2),
    (16, 0.1, 1, -1, -3), (16, 0.1, 1, 10923, -3),
    (16, 0.1, -1, 8, -7),
])
def test_bad_arguments_rejected(lib, L, p, n, T, code):
    dummy = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    rc = lib.mpd_decode_batch(L, p, dummy, n, T, dummy, dummy, None, None, 0, None)
    assert rc == code
    assert len(lib.mpd_last_error()) > 0


def test_null_pointers_rejected(lib):
    rc = lib.mpd_decode_batch(16, 0.1, None, 4, 8, None, None, None, None, 0, None)
    assert rc == -4
    dummy = ctypes.c_void_p(4096)
    rc = lib.mpd_decode_batch(256, 0.1, dummy, 4, 8, dummy, dummy, None, None, 0, None)
    assert rc == -5  # workspace missing for the tiled path


def test_empty_batch_is_a_noop(lib):
    assert lib.mpd_decode_batch(16, 0.1, None, 0, 8, None, None, None, None, 0, None) == 0


def test_counts_and_predictor_arguments(lib):
    d = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    lib.mpd_syndrome_counts.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.mpd_syndrome_counts(8, 0.1, None, d, 4, d, None) == -1
    assert lib.mpd_syndrome_counts(24, 0.1, None, d, 4, d, None) == -1
    assert lib.mpd_syndrome_counts(32, -0.5, None, d, 4, d, None) == -2
    assert lib.mpd_syndrome_counts(32, 0.1, None, d, -1, d, None) == -7
    assert lib.mpd_syndrome_counts(32, 0.1, None, None, 4, d, None) == -4
    assert lib.mpd_syndrome_counts(32, 0.1, None, d, 0, d, None) == 0
    P, I, I64, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    lib.mpd_cnn_forward.argtypes = [P, I, I64, P, P, P, P, P, SZ, P]
    lib.mpd_cnn_forward_workspace_bytes.argtypes = [I, I64]
    lib.mpd_cnn_forward_workspace_bytes.restype = SZ
    assert lib.mpd_cnn_forward(d, 1, 4, d, d, None, None, d, 1 << 20, None) == -1
    assert lib.mpd_cnn_forward(d, 32, -1, d, d, None, None, d, 1 << 20, None) == -7
    assert lib.mpd_cnn_forward(d, 32, 4, None, d, None, None, d, 1 << 20, None) == -4
    need = lib.mpd_cnn_forward_workspace_bytes(128, 4)
    assert need > lib.mpd_cnn_forward_workspace_bytes(32, 4) > 0
    assert lib.mpd_cnn_forward(d, 128, 4, d, d, None, None, d, need - 1, None) == -5
    assert lib.mpd_cnn_forward(d, 32, 0, None, None, None, None, None, 0, None) == 0
    lib.mpd_cnn_loss_grad.argtypes = [P, I, I64, P, P, P, P, P, P, SZ, P]
    lib.mpd_cnn_train_workspace_bytes.argtypes = [I, I64]
    lib.mpd_cnn_train_workspace_bytes.restype = SZ
    assert lib.mpd_cnn_train_workspace_bytes(33, 16) == 0
    assert lib.mpd_cnn_loss_grad(d, 33, 16, d, d, d, d, None, d, 1 << 30, None) == -1
    assert lib.mpd_cnn_loss_grad(d, 32, 0, d, d, d, d, None, d, 1 << 30, None) == -7
    assert lib.mpd_cnn_loss_grad(d, 32, 16, d, d, d, d, None, d, 16, None) == -5
    F = ctypes.c_float
    lib.mpd_cnn_adam_step.argtypes = [P, P, P, P, I, F, F, F, F, P]
    assert lib.mpd_cnn_adam_step(d, d, d, d, 0, 1e-3, 0.9, 0.999, 1e-8, None) == -7
    assert lib.mpd_cnn_adam_step(d, d, d, d, 1, float("nan"), 0.9, 0.999, 1e-8, None) == -2
    assert lib.mpd_cnn_adam_step(d, d, d, d, 1, 1e-3, 1.0, 0.999, 1e-8, None) == -2
    assert lib.mpd_cnn_adam_step(None, d, d, d, 1, 1e-3, 0.9, 0.999, 1e-8, None) == -4
    lib.mpd_cnn_init.argtypes = [P, ctypes.c_uint64, P]
    assert lib.mpd_cnn_init(None, 1, None) == -4


def test_learned_decode_arguments(lib):
    d = ctypes.c_void_p(4096)
    P, I, I64, SZ, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double
    lib.mpd_decode_learned.argtypes = [I, D, P, P, I64, I, P, I, P, P, P, P, P, P, P, SZ, P]
    lib.mpd_learned_workspace_bytes.argtypes = [I, I64]
    lib.mpd_learned_workspace_bytes.restype = SZ
    assert lib.mpd_learned_workspace_bytes(128, 10) == 0
    assert lib.mpd_learned_workspace_bytes(256, 10) > lib.mpd_workspace_bytes(256, 10)
    edges = (ctypes.c_float * 2)(1.0, 2.0)
    bad_edges = (ctypes.c_float * 2)(2.0, 1.0)
    depths = (ctypes.c_int * 3)(3, 4, 5)
    deep = (ctypes.c_int * 3)(3, 4, 16)

    def call(L=256, p=0.01, n=8, T=64, nb=3, e=edges, k=depths, ws_bytes=1 << 40, dp=None):
        return lib.mpd_decode_learned(L, p, dp, d, n, T, d, nb, e, k, d, d, None, None, d, ws_bytes, None)

    assert call(L=128) == -1
    assert call(p=2.0) == -2
    assert call(T=-1) == -3
    assert call(nb=0) == -7 and call(nb=9) == -7
    assert call(k=deep) == -3
    assert call(e=bad_edges) == -2
    assert call(e=None) == -4 and call(k=None) == -4
    assert call(ws_bytes=1024) == -5
    assert call(n=0) == 0
    # per-sample p: the scalar is not checked, the array's alignment is
    assert call(p=2.0, dp=ctypes.c_void_p(4097)) == -4


def test_mixed_workspace_is_per_band_class(lib):
    lib.mpd_mixed_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    lib.mpd_mixed_workspace_bytes.restype = ctypes.c_size_t
    Ls = (ctypes.c_int32 * 3)(64, 256, 256)
    cs = (ctypes.c_int64 * 3)(10, 4, 2)
    total = lib.mpd_mixed_workspace_bytes(3, Ls, cs)
    assert total >= lib.mpd_workspace_bytes(256, 4) + lib.mpd_workspace_bytes(256, 2)


def test_band_driver_setting(lib):
    """Driver of the band path's later passes: default auto, per-L settings
    kept by mpd_set_band_schedule, L = 0 applying to every L, bad values and
    NULL outputs rejected."""
    d = ctypes.c_int(-1)
    get = lambda L: (lib.mpd_get_band_driver(L, ctypes.byref(d)), d.value)[1]
    try:
        assert get(0) == 0 and get(512) == 0
        assert lib.mpd_set_band_driver(0, 3) == -7 and len(lib.mpd_last_error()) > 0
        assert lib.mpd_set_band_driver(0, -1) == -7
        assert lib.mpd_get_band_driver(0, None) == -4
        assert lib.mpd_set_band_driver(512, 2) == 0
        assert get(512) == 2 and get(256) == 0
        assert lib.mpd_set_band_schedule(512, 3, 3) == 0   # keeps the driver of L = 512
        assert get(512) == 2
        kf, kn = ctypes.c_int(0), ctypes.c_int(0)
        assert lib.mpd_get_band_schedule(512, ctypes.byref(kf), ctypes.byref(kn)) == 0 and (kf.value, kn.value) == (3, 3)
        assert lib.mpd_set_band_driver(0, 1) == 0           # default and every per-L setting
        assert get(512) == 1 and get(0) == 1 and get(256) == 1
        assert lib.mpd_set_band_schedule(0, 4, 2) == 0      # forgets per-L settings
        assert get(512) == 1
        assert lib.mpd_get_band_schedule(512, ctypes.byref(kf), ctypes.byref(kn)) == 0 and (kf.value, kn.value) == (4, 2)
    finally:
        lib.mpd_set_band_driver(0, 0)
        lib.mpd_set_band_schedule(0, 4, 2)
    assert get(0) == 0


def test_band_bits_setting(lib):
    """Steps of the bit-sliced first kernel: default 10, per-L settings, L = 0
    applying to every L, values outside [0, 10] and NULL outputs rejected."""
    k = ctypes.c_int(-1)
    get = lambda L: (lib.mpd_get_band_bits(L, ctypes.byref(k)), k.value)[1]
    try:
        assert get(0) == 10 and get(256) == 10
        assert lib.mpd_set_band_bits(256, 11) == -3 and len(lib.mpd_last_error()) > 0
        assert lib.mpd_set_band_bits(256, -1) == -3
        assert lib.mpd_get_band_bits(256, None) == -4
        assert lib.mpd_set_band_bits(256, 2) == 0
        assert get(256) == 2 and get(512) == 10
        assert lib.mpd_set_band_schedule(256, 3, 3) == 0   # keeps the setting of L = 256
        assert get(256) == 2
        assert lib.mpd_set_band_bits(0, 0) == 0             # default and every per-L setting
        assert get(256) == 0 and get(0) == 0
    finally:
        lib.mpd_set_band_bits(0, 10)
        lib.mpd_set_band_schedule(0, 4, 2)
    assert get(256) == 10


@pytest.mark.parametrize("stmt", ["from paper_2506_03266_amd import binding, sweep, learned",
                                  "import paper_2506_03266_amd as m; m.sweep.SWEEP_CONFIG; m.binding.syndrome_words(8)"])
def test_package_submodules_load_lazily(stmt):
    """Each submodule loads on first use, in a fresh interpreter (as under
    ``python -m paper_2506_03266_amd.sweep``)."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", stmt], cwd=root, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]


def test_rule_arguments_rejected(lib):
    """The limited-memory entry points reject negative m_max / u (MPD_ERR_RULE)
    and random moves without move seeds, before touching the GPU."""
    dummy = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    assert lib.mpd_decode_rule(16, 0.1, dummy, 4, 8, -1, 0, dummy, dummy, None, None, 0, None) == -8
    assert lib.mpd_decode_rule(16, 0.1, dummy, 4, 8, 0, -2, dummy, dummy, None, None, 0, None) == -8
    assert lib.mpd_decode_rule(16, 1.5, dummy, 4, 8, 2, 0, dummy, dummy, None, None, 0, None) == -2
    assert lib.mpd_decode_rule(16, 0.1, dummy, 0, 8, 2, 3, dummy, dummy, None, None, 0, None) == 0  # empty
    assert lib.mpd_decode_errors_rule(16, dummy, None, 4, 8, 2, 3, dummy, dummy, None, None) == -4
    assert lib.mpd_decode_errors_rule(16, dummy, None, 4, 8, -1, 0, dummy, dummy, None, None) == -8
    assert lib.mpd_decode_errors_rule(256, dummy, None, 4, 8, 2, 0, dummy, dummy, None, None) == -1
    assert lib.mpd_run_steps_rule(16, dummy, None, 4, 3, 2, 1, dummy, dummy, dummy, None) == -4
    assert lib.mpd_run_steps_rule(16, dummy, None, 4, 3, 2, -1, dummy, dummy, dummy, None) == -8
    assert len(lib.mpd_last_error()) > 0


def test_open_arguments_rejected(lib):
    dummy = ctypes.c_void_p(4096)  # never dereferenced: validation fails first
    assert lib.mpd_decode_open(200, 0.1, dummy, 4, 8, dummy, dummy, None, None, 0, None) == -1
    assert lib.mpd_decode_open(2, 0.1, dummy, 4, 8, dummy, dummy, None, None, 0, None) == -1
    assert lib.mpd_decode_open(16, -0.5, dummy, 4, 8, dummy, dummy, None, None, 0, None) == -2
    assert lib.mpd_decode_open(16, 0.1, None, 4, 8, dummy, dummy, None, None, 0, None) == -4
    assert lib.mpd_decode_open(16, 0.1, dummy, 0, 8, dummy, dummy, None, None, 0, None) == 0
    assert lib.mpd_decode_open(256, 0.1, dummy, 4, 8, dummy, dummy, None, None, 0, None) == -5  # workspace
    assert lib.mpd_decode_errors_open(16, None, 4, 8, dummy, dummy, None, None) == -4
    assert lib.mpd_run_steps_open(16, dummy, 4, 3, None, dummy, dummy, None) == -4
    assert lib.mpd_run_steps_open(200, dummy, 4, 3, dummy, dummy, dummy, None) == -1


def test_async_arguments_rejected(lib):
    """The desynchronized entry points check L (5..64), p, rho, the slot
    budget, t_target and pointers before any launch."""
    dummy = ctypes.c_void_p(256)
    d = lambda L=16, p=0.1, n=4, rho=0.5, S=100, T=dummy, F=dummy, sd=dummy: lib.mpd_decode_async(
        L, p, sd, n, rho, S, T, F, None, None, None, None)
    assert d(L=4) == -1 and d(L=65) == -1 and d(L=128) == -1
    assert d(p=1.5) == -2 and d(rho=0.0) == -2 and d(rho=1.01) == -2 and d(rho=float("nan")) == -2
    assert d(S=-1) == -3 and d(S=65001) == -3
    assert d(n=-1) == -7
    assert d(sd=None) == -4 and d(T=None) == -4 and d(sd=ctypes.c_void_p(260)) == -4
    assert d(n=0) == 0
    r = lambda L=16, n=4, t=3, rho=0.5, S=100, links=dummy, cs=dummy, m=dummy: lib.mpd_run_async(
        L, links, cs, n, t, rho, S, dummy, None, m, dummy, dummy, dummy, None)
    assert r(L=3) == -1 and r(rho=2.0) == -2 and r(t=-1) == -3 and r(t=16251) == -3 and r(S=70000) == -3
    assert r(links=None) == -4 and r(cs=None) == -4 and r(m=None) == -4 and r(m=ctypes.c_void_p(257)) == -4
    assert r(n=0) == 0


def test_uncoord_arguments_rejected(lib):
    """The uncoordinated entry points share the desynchronized checks and
    reject an unknown schedule."""
    dummy = ctypes.c_void_p(256)
    d = lambda L=16, rho=0.5, S=100, sch=0, sd=dummy, n=4: lib.mpd_decode_uncoord(  # noqa: E731
        L, 0.1, sd, n, rho, S, sch, dummy, dummy, None, None, None, None)
    assert d(L=4) == -1 and d(rho=0.0) == -2 and d(S=-1) == -3 and d(sd=None) == -4 and d(sch=2) == -7
    assert d(n=0) == 0 and d(n=0, sch=1) == 0
    r = lambda t=2, cs=dummy, sch=0: lib.mpd_run_uncoord(  # noqa: E731
        16, dummy, cs, 4, t, 0.5, 100, sch, dummy, None, dummy, dummy, dummy, dummy, None)
    assert r(t=-1) == -3 and r(cs=None) == -4 and r(sch=-1) == -7


def test_resume_arguments_rejected(lib):
    """mpd_run_steps_from checks L, the step range, the rule, and its state
    pointers before any launch."""
    d = ctypes.c_void_p(256)
    f = lambda L=16, t0=2, t=3, mm=0, u=0, m_in=d, s_in=d, w_in=d, ms=None, m_out=d, n=4: lib.mpd_run_steps_from(  # noqa
        L, m_in, s_in, w_in, n, t0, t, mm, u, ms, m_out, d, d, None)
    assert f(L=2) == -1 and f(L=256) == -1
    assert f(t0=-1) == -3 and f(t=-1) == -3 and f(t0=10000, t=923) == -3
    assert f(mm=-1) == -8 and f(u=-1) == -8
    assert f(m_in=None) == -4 and f(s_in=None) == -4 and f(w_in=None) == -4 and f(m_out=None) == -4
    assert f(m_in=ctypes.c_void_p(257)) == -4 and f(u=2) == -4
    assert f(n=-1) == -7 and f(n=0) == 0


def test_band_tuning_round_trip(lib, tmp_path):
    """save_band_tuning / load_band_tuning persist per-L schedules and
    drivers across processes (here: across a reset of the settings)."""
    import paper_2506_03266_amd.binding as b
    try:
        b.set_band_schedule(5, 3, 0)
        b.set_band_schedule(2, 1, 512)
        b.set_band_driver(b.BAND_DRIVER_DEVICE, 512)
        b.set_band_schedule(6, 4, 1024)
        b.set_band_bits(3, 256)
        path = str(tmp_path / "tuning.json")
        saved = b.save_band_tuning(path, [256, 512, 1024])
        assert saved["per_L"]["512"] == {"k_first": 2, "k_next": 1, "driver": b.BAND_DRIVER_DEVICE, "k_bits": 10}
        assert saved["per_L"]["256"]["k_bits"] == 3
        b.set_band_driver(b.BAND_DRIVER_AUTO, 0)
        b.set_band_schedule(4, 2, 0)
        b.set_band_bits(10, 0)
        assert b.get_band_schedule(512) == (4, 2) and b.get_band_bits(256) == 10
        b.load_band_tuning(path)
        assert b.get_band_schedule(0) == (5, 3)
        assert b.get_band_schedule(512) == (2, 1) and b.get_band_driver(512) == b.BAND_DRIVER_DEVICE
        assert b.get_band_schedule(1024) == (6, 4) and b.get_band_driver(1024) == b.get_band_driver(0)
        assert b.get_band_bits(256) == 3
    finally:
        b.set_band_driver(b.BAND_DRIVER_AUTO, 0)
        b.set_band_schedule(4, 2, 0)
        b.set_band_bits(10, 0)
