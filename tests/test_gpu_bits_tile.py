"""The tiled bit-sliced first pass for L > 256 (256 x 256 regions with a
halo of 4k for k <= 6 decoder steps, then the band path), against the CPU
oracle bit for bit (T_dec, flags and final syndrome): every number of tiled
steps, lattice sizes whose strips split unevenly over the tiles, budgets that
end inside the tiled steps, noise strengths from none to every link (high p
makes corrections cross the winding cuts inside the tiled steps), per-sample
noise strength, and the learned decode.  Every setting must also give the
band path's results."""
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


def compare(tag, T, F, S, ref):
    T, F = T.cpu().numpy(), F.cpu().numpy()
    S = S.cpu().numpy().view(np.uint32).reshape(T.size, -1)
    bad = np.nonzero((T != ref["T_dec"]) | (F != ref["flags"]))[0]
    assert bad.size == 0, f"{tag}: {bad.size} mismatches, first {bad[:5]} gpu T={T[bad[:5]]} F={F[bad[:5]]} " \
                          f"oracle T={ref['T_dec'][bad[:5]]} F={ref['flags'][bad[:5]]}"
    rows = np.nonzero(np.any(S != ref["sigma_words"], axis=1))[0]
    assert rows.size == 0, f"{tag}: final syndrome differs for samples {rows[:5]}"


def with_bits(gpu, L, k, fn):
    old = gpu.get_band_bits(L)
    gpu.set_band_bits(k, L)
    try:
        return fn()
    finally:
        gpu.set_band_bits(old, L)


@pytest.mark.parametrize("L", [272, 512])
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6, 10])
@pytest.mark.parametrize("p", [0.01, 0.05, 0.09])
def test_steps_against_oracle(gpu, orc, L, k, p):
    """k = 10 runs the tiled kernel's six steps; p = 0.09 (above the
    threshold) gives logical failures whose corrections cross the cuts."""
    n, T_max = 8, (1024 if p < 0.09 else 128)
    s = seeds(81, L * 100 + int(p * 1000) * 8 + k, n)
    ref = orc.decode_seeds(L, p, s, T_max, threads=16)
    T, F, S = with_bits(gpu, L, k, lambda: gpu.decode_batch(L, p, s, T_max))
    compare(f"L={L} k_bits={k} p={p}", T, F, S, ref)


@pytest.mark.parametrize("L", [288, 1024, 2048])
def test_other_sizes_against_oracle(gpu, orc, L):
    """288 = 72 groups of four rows (two tiles of 36 at six steps); 1024 over
    five tiles of 204 or 208 rows, whose edges fall inside 16-row masks;
    2048 over ten tiles per side."""
    n, p, T_max = (4, 0.03, 2048) if L < 2048 else (2, 0.02, 256)
    s = seeds(82, L, n)
    ref = orc.decode_seeds(L, p, s, T_max, threads=16)
    T, F, S = gpu.decode_batch(L, p, s, T_max)
    compare(f"L={L}", T, F, S, ref)


@pytest.mark.parametrize("T_max", [1, 2, 3, 4, 5, 6, 7, 8])
def test_budgets_inside_the_tiled_steps(gpu, orc, T_max):
    L, p, n = 272, 0.07, 8
    s = seeds(83, T_max, n)
    ref = orc.decode_seeds(L, p, s, T_max, threads=16)
    T, F, S = gpu.decode_batch(L, p, s, T_max)
    compare(f"T_max={T_max}", T, F, S, ref)


@pytest.mark.parametrize("p", [0.0, 0.5, 1.0])
def test_extreme_noise(gpu, orc, p):
    L, n, T_max = 272, 4, 64
    s = seeds(84, int(p * 10), n)
    ref = orc.decode_seeds(L, p, s, T_max, threads=8)
    T, F, S = gpu.decode_batch(L, p, s, T_max)
    compare(f"p={p}", T, F, S, ref)


def test_per_sample_noise_strength(gpu, orc):
    L, n, T_max = 512, 12, 2048
    s = seeds(85, 0, n)
    ps = np.random.default_rng(85).uniform(0.001, 0.1, n)
    ref = orc.decode_seeds(L, ps, s, T_max, threads=16)
    T, F, S = gpu.decode_mixed([(L, n)], ps, s, T_max)
    compare("per-sample p", T, F, S, ref)


@pytest.mark.parametrize("L", [272, 512])
def test_same_as_band_path_on_a_larger_batch(gpu, L):
    n, T_max = 256, 4096
    for p in (0.02, 0.08):
        s = seeds(86, L + int(p * 100), n)
        base = [x.cpu().numpy() for x in with_bits(gpu, L, 0, lambda: gpu.decode_batch(L, p, s, T_max))]
        for k in (1, 2, 3, 4, 5, 6):
            got = [x.cpu().numpy() for x in with_bits(gpu, L, k, lambda: gpu.decode_batch(L, p, s, T_max))]
            for a, b, name in zip(got, base, ("T_dec", "flags", "syndrome")):
                assert np.array_equal(a, b), f"L={L} p={p} k_bits={k}: {name} differs from the band path"


def test_learned_decode_uses_the_tiled_pass(gpu, orc):
    """A two-group policy at L = 512: the network runs, the tiled pass takes
    the samples in predicted order, and the results are the oracle's."""
    import torch
    from oracle import cnn_oracle as co
    import oracle
    L, n, p, T_max = 512, 16, 0.02, 2048
    s = seeds(87, 0, n)
    params = torch.from_numpy(co.init_params(7, oracle.philox4x32_10).astype(np.float32)).cuda()
    ref = orc.decode_seeds(L, p, s, T_max, threads=16)
    T, F, S, _ = gpu.decode_learned(L, p, s, params, [1.5], [4, 2], T_max)
    compare("learned L=512", T, F, S, ref)
