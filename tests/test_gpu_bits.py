"""The bit-sliced whole-lattice kernel that runs the first decoder steps of a
plain L = 256 batch (up to ten, on 2 to 5 bit planes), against the CPU
oracle bit for bit (T_dec, flags and
final syndrome), for every number of bit-sliced steps (0 = the band path's
first pass), budgets that end inside those steps, noise strengths from none
to every link, per-sample noise strength and both drivers of the later
passes.  Each setting must also give the same results as the band path
alone."""
import numpy as np
import pytest

from paper_2506_03266_amd.workloads import seeds

pytestmark = pytest.mark.gpu

L = 256


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


def with_bits(gpu, k, fn):
    old = gpu.get_band_bits(L)
    gpu.set_band_bits(k, L)
    try:
        return fn()
    finally:
        gpu.set_band_bits(old, L)


def test_default_is_ten_steps(gpu):
    assert gpu.get_band_bits(L) == 10


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4, 5, 6, 8, 10])
@pytest.mark.parametrize("p", [0.01, 0.03, 0.06])
def test_steps_against_oracle(gpu, orc, k, p):
    n, T_max = 24, 256
    s = seeds(61, int(p * 1000) * 8 + k, n)
    ref = orc.decode_seeds(L, p, s, T_max, threads=16)
    T, F, S = with_bits(gpu, k, lambda: gpu.decode_batch(L, p, s, T_max))
    compare(f"k_bits={k} p={p}", T, F, S, ref)


@pytest.mark.parametrize("T_max", [0, 1, 2, 3, 4, 5, 6, 9, 10, 11, 12])
def test_budgets_inside_the_bit_sliced_steps(gpu, orc, T_max):
    """Timeouts at T_max <= 10 leave their final syndrome from the bit-sliced
    kernel; T_max = 11 and 12 run band steps after it."""
    p, n = 0.05, 16
    s = seeds(62, T_max, n)
    ref = orc.decode_seeds(L, p, s, T_max, threads=16)
    T, F, S = gpu.decode_batch(L, p, s, T_max)
    compare(f"T_max={T_max}", T, F, S, ref)


@pytest.mark.parametrize("p", [0.0, 0.5, 1.0])
def test_extreme_noise(gpu, orc, p):
    n, T_max = 8, 64
    s = seeds(63, int(p * 10), n)
    ref = orc.decode_seeds(L, p, s, T_max, threads=8)
    T, F, S = gpu.decode_batch(L, p, s, T_max)
    compare(f"p={p}", T, F, S, ref)


def test_per_sample_noise_strength(gpu, orc):
    n, T_max = 48, 512
    s = seeds(64, 0, n)
    ps = np.random.default_rng(64).uniform(0.001, 0.05, n)
    ref = orc.decode_seeds(L, ps, s, T_max, threads=16)
    T, F, S = gpu.decode_mixed([(L, n)], ps, s, T_max)
    compare("per-sample p", T, F, S, ref)


def test_device_driver_after_bits(gpu, orc):
    n, p, T_max = 64, 0.04, 512
    s = seeds(65, 0, n)
    ref = orc.decode_seeds(L, p, s, T_max, threads=16)
    old = gpu.get_band_driver(L)
    gpu.set_band_driver(gpu.BAND_DRIVER_DEVICE, L)
    try:
        T, F, S = gpu.decode_batch(L, p, s, T_max)
    finally:
        gpu.set_band_driver(old, L)
    compare("device driver", T, F, S, ref)


def test_same_as_band_path_on_a_large_batch(gpu):
    """1024 samples at p = 0.02 (decodes of up to a dozen steps): every
    setting of k_bits gives the band path's results."""
    n, p, T_max = 1024, 0.02, 4096
    s = seeds(66, 0, n)
    base = [x.cpu().numpy() for x in with_bits(gpu, 0, lambda: gpu.decode_batch(L, p, s, T_max))]
    for k in (1, 3, 5, 7, 10):
        got = [x.cpu().numpy() for x in with_bits(gpu, k, lambda: gpu.decode_batch(L, p, s, T_max))]
        for a, b, name in zip(got, base, ("T_dec", "flags", "syndrome")):
            assert np.array_equal(a, b), f"k_bits={k}: {name} differs from the band path"
