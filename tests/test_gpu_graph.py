"""HIP graph capture of the single-launch paths: small-lattice decodes
(L <= 128), block counts and the predictor's forward pass.  Each graph is
replayed several times with new inputs written by eager work between
replays; every replay must equal the eager result exactly."""
import numpy as np
import pytest
import torch

from paper_2506_03266_amd.workloads import seeds

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_03266_amd.binding as b
    b.lib()
    return b


@pytest.mark.parametrize("L,p,n", [(16, 0.01, 1000), (64, 0.02, 2048), (128, 0.03, 64)])
def test_resident_decode_graph(gpu, L, p, n):
    dev = torch.device("cuda")
    s_in = torch.from_numpy(seeds(60, L, n).view(np.int64)).to(dev)
    out = (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev),
           torch.empty((n, gpu.syndrome_words(L)), dtype=torch.int32, device=dev))
    gpu.decode_batch(L, p, s_in, 512, out=out)  # warm-up outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu.decode_batch(L, p, s_in, 512, out=out)
    for rep in range(4):
        fresh = torch.from_numpy(seeds(61 + rep, L, n).view(np.int64)).to(dev)
        s_in.copy_(fresh)
        g.replay()
        torch.cuda.synchronize()
        got = [t.clone() for t in out]
        T, F, S = gpu.decode_batch(L, p, fresh, 512)
        assert torch.equal(got[0], T) and torch.equal(got[1], F) and torch.equal(got[2], S), rep
        assert int(T.sum()) > 0


def test_counts_and_forward_graph(gpu):
    """Block counts of a seeded batch and the predictions, captured together
    (L = 256 maps, whole-map kernel) and for L = 1024 maps (tiled kernel,
    whose pooled maxima are cleared by a kernel inside the graph)."""
    dev = torch.device("cuda")
    params = gpu.cnn_init(3)
    for L, n in ((256, 512), (1024, 16)):
        s_in = torch.from_numpy(seeds(62, L, n).view(np.int64)).to(dev)
        counts = torch.empty((n, L // 8, L // 8), dtype=torch.uint8, device=dev)
        gpu.syndrome_counts(L, 0.01, s_in, out=counts)
        pred = gpu.cnn_forward(counts, params)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            gpu.syndrome_counts(L, 0.01, s_in, out=counts)
            pred_g = gpu.cnn_forward(counts, params)
        for rep in range(3):
            fresh = torch.from_numpy(seeds(63 + rep, L, n).view(np.int64)).to(dev)
            s_in.copy_(fresh)
            g.replay()
            torch.cuda.synchronize()
            want_c = gpu.syndrome_counts(L, 0.01, fresh)
            want_p = gpu.cnn_forward(want_c, params)
            assert torch.equal(counts, want_c), (L, rep)
            assert torch.equal(pred_g, want_p), (L, rep)


@pytest.mark.parametrize("per_sample_p", [False, True])
def test_learned_decode_graph(gpu, per_sample_p):
    """A learned-scheduling decode (noise, block counts, predictor, binning,
    group first passes sized on the device, later passes on the device) in
    one captured graph: every replay equals the plain decode of the same
    seeds and the eager learned call's predictions."""
    dev = torch.device("cuda")
    L, n, T_max = 256, 384, 4096
    rng = np.random.default_rng(64)
    p = torch.from_numpy(rng.uniform(0.005, 0.03, n)).to(dev) if per_sample_p else 0.02
    params = gpu.cnn_init(4)
    s_in = torch.from_numpy(seeds(64, int(per_sample_p), n).view(np.int64)).to(dev)
    ws = gpu.learned_workspace(L, n)
    out = (torch.empty(n, dtype=torch.int32, device=dev), torch.empty(n, dtype=torch.uint8, device=dev),
           torch.empty((n, gpu.syndrome_words(L)), dtype=torch.int32, device=dev),
           torch.empty(n, dtype=torch.float32, device=dev))
    pred0 = gpu.cnn_forward(gpu.syndrome_counts(L, p, s_in), params).cpu().numpy()
    edges = tuple(float(v) for v in np.quantile(pred0, [0.3, 0.7]))
    depths = (3, 4, 6)
    gpu.decode_learned(L, p, s_in, params, edges, depths, T_max, workspace=ws, out=out)  # warm-up
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu.decode_learned(L, p, s_in, params, edges, depths, T_max, workspace=ws, out=out)
    for rep in range(3):
        fresh = torch.from_numpy(seeds(65 + rep, int(per_sample_p), n).view(np.int64)).to(dev)
        s_in.copy_(fresh)
        g.replay()
        torch.cuda.synchronize()
        got = [t.clone() for t in out]
        if per_sample_p:
            T, F, S = gpu.decode_mixed([(L, n)], p.cpu().numpy(), fresh, T_max)
        else:
            T, F, S = gpu.decode_batch(L, p, fresh, T_max)
        _, _, _, pr = gpu.decode_learned(L, p, fresh, params, edges, depths, T_max)
        assert torch.equal(got[0], T) and torch.equal(got[1], F), rep
        assert torch.equal(got[2].reshape(-1), S.reshape(-1)), rep
        assert torch.equal(got[3], pr), rep
        assert int(T.sum()) > 0
