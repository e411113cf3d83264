"""Band path (L >= 256) with its later passes driven on the device: one
persistent launch in which each workgroup runs all the passes of the
surviving samples it takes.  Results must equal the oracle's bit for bit, and
the host-driven path's; a whole band-path decode can be captured into a HIP
graph and replayed."""
import numpy as np
import pytest
import torch

from paper_2506_03266_amd.workloads import seeds, CONFIGS

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_03266_amd.binding as b
    b.lib()
    return b


@pytest.fixture
def device(gpu):
    gpu.set_band_driver(gpu.BAND_DRIVER_DEVICE)
    yield gpu
    gpu.set_band_driver(gpu.BAND_DRIVER_AUTO)
    gpu.set_band_schedule(4, 2)


def _np(t):
    return t.cpu().numpy()


def compare(tag, T, F, S, ref):
    T, F = _np(T), _np(F)
    bad = np.nonzero((T != ref["T_dec"]) | (F != ref["flags"]))[0]
    assert bad.size == 0, f"{tag}: {bad.size} mismatches, first {bad[:5]} gpu T={T[bad[:5]]} F={F[bad[:5]]} " \
                          f"oracle T={ref['T_dec'][bad[:5]]} F={ref['flags'][bad[:5]]}"
    if S is not None:
        rows = np.nonzero(np.any(_np(S).view(np.uint32) != ref["sigma_words"], axis=1))[0]
        assert rows.size == 0, f"{tag}: final syndrome differs for samples {rows[:5]}"


@pytest.mark.parametrize("L,p,n,T_max", [(256, 0.06, 12, 0), (256, 0.06, 12, 1), (256, 0.06, 12, 5),
                                         (256, 0.06, 12, 7), (256, 0.07, 8, 64), (272, 0.03, 6, 64),
                                         (320, 0.06, 4, 40), (512, 0.07, 3, 9), (1024, 0.01, 3, 64),
                                         (256, 0.03, 100, 64)])
def test_device_driver_matches_oracle(device, orc, L, p, n, T_max):
    s = seeds(70, L + T_max, n)
    T, F, S = device.decode_batch(L, p, s, T_max)
    ref = orc.decode_seeds(L, p, s, T_max, threads=16)
    compare(f"L={L} p={p} T_max={T_max}", T, F, S, ref)


@pytest.mark.parametrize("k_first,k_next", [(1, 1), (2, 3), (4, 5), (6, 8), (3, 15)])
def test_device_driver_pass_depths(device, orc, k_first, k_next):
    """Tail passes of every depth, up to k = 15, whose tiles own 8 of their
    128 columns."""
    L, p, n, T_max = 256, 0.065, 6, 48
    device.set_band_schedule(k_first, k_next, L)
    s = seeds(71, 10 * k_first + k_next, n)
    T, F, S = device.decode_batch(L, p, s, T_max)
    ref = orc.decode_seeds(L, p, s, T_max, threads=16)
    compare(f"k=({k_first},{k_next})", T, F, S, ref)


def test_device_and_host_drivers_agree_on_config3(gpu, orc):
    """The benchmark batch (L = 256, p = 0.01, 4096 samples) with both drivers:
    identical outputs; a spread of samples against the oracle."""
    cfg = CONFIGS[3]
    s = seeds(3, 0, cfg["n"])
    out = {}
    try:
        for d in (gpu.BAND_DRIVER_HOST, gpu.BAND_DRIVER_DEVICE):
            gpu.set_band_driver(d)
            out[d] = [t.clone() for t in gpu.decode_batch(cfg["L"], cfg["p"][0], s, cfg["T_max"])]
    finally:
        gpu.set_band_driver(gpu.BAND_DRIVER_AUTO)
    for a, c in zip(out[gpu.BAND_DRIVER_HOST], out[gpu.BAND_DRIVER_DEVICE]):
        assert torch.equal(a, c)
    pick = np.arange(0, cfg["n"], 97)
    ref = orc.decode_seeds(cfg["L"], cfg["p"][0], s[pick], cfg["T_max"], threads=16)
    T, F, S = out[gpu.BAND_DRIVER_DEVICE]
    compare("config 3", T[pick], F[pick], S[pick], ref)


@pytest.mark.parametrize("depths,T_max", [((2, 6), 5), ((1, 7), 6), ((1, 2, 9), 9), ((3, 5), 64)])
def test_device_driver_learned_groups(device, orc, depths, T_max):
    """First passes of different depth per group, then the device-driven tail:
    samples reach the budget in different passes and buffers."""
    L, p, n = 256, 0.08, 9
    s = seeds(72, 10 * T_max + len(depths), n)
    params = device.cnn_init(13)
    pr = np.sort(device.cnn_forward(device.syndrome_counts(L, p, s), params).cpu().numpy())
    edges = tuple(float(e) for e in pr[np.linspace(0, n, len(depths) + 1).astype(int)[1:-1]])
    T, F, S, _ = device.decode_learned(L, p, s, params, edges, depths, T_max)
    ref = orc.decode_seeds(L, p, s, T_max, threads=16)
    compare(f"learned {depths} T_max={T_max}", T, F, S, ref)


def test_device_driver_mixed(device, orc):
    """A mixed call whose band classes all finish on the device, each on its
    own stream, with no host wait between passes."""
    classes = [(256, 3), (64, 5), (272, 2), (512, 1), (32, 4), (256, 1)]
    n = sum(c for _, c in classes)
    r = np.random.default_rng(12)
    ps = r.uniform(0.005, 0.06, n)
    ss = seeds(73, 0, n)
    T, F, S = device.decode_mixed(classes, ps, ss, 128)
    T, F, S = _np(T), _np(F), _np(S).view(np.uint32)
    off = woff = 0
    for L, c in classes:
        ref = orc.decode_seeds(L, ps[off:off + c], ss[off:off + c], 128, threads=16)
        W = (L * L + 31) // 32
        assert np.array_equal(T[off:off + c], ref["T_dec"]), L
        assert np.array_equal(F[off:off + c], ref["flags"]), L
        assert np.array_equal(S[woff:woff + c * W].reshape(c, W), ref["sigma_words"]), L
        off += c
        woff += c * W


@pytest.mark.parametrize("L,p,n,T_max", [(256, 0.02, 512, 4096), (512, 0.05, 16, 256)])
def test_band_decode_graph(gpu, L, p, n, T_max):
    """A whole band-path decode (noise, first pass, device-driven later
    passes, export) captured with the default driver and replayed with new
    seeds: every replay equals the eager decode."""
    dev = torch.device("cuda")
    s_in = torch.from_numpy(seeds(74, L, n).view(np.int64)).to(dev)
    ws = gpu.alloc_workspace(L, n)
    out = (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev),
           torch.empty((n, gpu.syndrome_words(L)), dtype=torch.int32, device=dev))
    gpu.decode_batch(L, p, s_in, T_max, workspace=ws, out=out)  # warm-up outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu.decode_batch(L, p, s_in, T_max, workspace=ws, out=out)
    for rep in range(3):
        fresh = torch.from_numpy(seeds(75 + rep, L, n).view(np.int64)).to(dev)
        s_in.copy_(fresh)
        g.replay()
        torch.cuda.synchronize()
        got = [t.clone() for t in out]
        T, F, S = gpu.decode_batch(L, p, fresh, T_max)
        torch.cuda.synchronize()
        assert torch.equal(got[0], T) and torch.equal(got[1], F) and torch.equal(got[2], S), rep
        assert int(T.max()) > 4  # some samples needed the later passes


def test_mixed_decode_graph(gpu):
    """The mixed-size workload (L = 32..512, per-sample p) captured as one
    graph: resident classes on a side stream and band classes on library
    streams, all forked from and joined into the captured stream."""
    from paper_2506_03266_amd.workloads import mixed_batch
    dev = torch.device("cuda")
    Ls, ps, ss = mixed_batch()
    classes = [(L, int((Ls == L).sum())) for L in dict.fromkeys(Ls.tolist())]
    n = len(Ls)
    W = sum(c * gpu.syndrome_words(L) for L, c in classes)
    p_in = torch.from_numpy(ps).to(dev)
    s_in = torch.from_numpy(ss.view(np.int64)).to(dev)
    nb = gpu.lib().mpd_mixed_workspace_bytes(len(classes), np.array([c[0] for c in classes], np.int32).ctypes.data,
                                             np.array([c[1] for c in classes], np.int64).ctypes.data)
    ws = torch.empty(nb, dtype=torch.uint8, device=dev)
    out = (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev),
           torch.empty(W, dtype=torch.int32, device=dev))
    gpu.decode_mixed(classes, p_in, s_in, 4096, workspace=ws, out=out)  # warm-up: creates the library streams
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu.decode_mixed(classes, p_in, s_in, 4096, workspace=ws, out=out)
    rng = np.random.default_rng(3)
    for rep in range(3):
        fresh_s = ss + np.uint64(1000 * (rep + 1))
        fresh_p = rng.uniform(0.001, 0.03, n)
        s_in.copy_(torch.from_numpy(fresh_s.view(np.int64)))
        p_in.copy_(torch.from_numpy(fresh_p))
        g.replay()
        torch.cuda.synchronize()
        got = [t.clone() for t in out]
        want = gpu.decode_mixed(classes, fresh_p, fresh_s, 4096)
        torch.cuda.synchronize()
        for a, c in zip(got, want):
            assert torch.equal(a, c), rep
