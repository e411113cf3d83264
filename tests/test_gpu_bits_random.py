"""Seeded random configurations of the bit-sliced paths against the CPU
oracle, bit for bit (T_dec, flags, final syndrome): lattice size (whole
lattice at L = 64, 128, 256; tiled above, including sizes whose own parts
split unevenly), noise strength up to above the threshold, step budget, the
number of bit-sliced steps and the driver of the later band passes are
drawn per case."""
import numpy as np
import pytest

from paper_2506_03266_amd.workloads import seeds

pytestmark = pytest.mark.gpu

SIZES = [64, 128, 256, 272, 304, 320, 512]


def cases(count=120):
    r = np.random.default_rng(2506)
    out = []
    for i in range(count):
        L = int(r.choice(SIZES))
        p = float(r.uniform(0.0, 0.12))
        T_max = int(r.choice([1, 2, 3, 5, 7, 9, 11, 16, 30, 256]))
        k = int(r.integers(0, 11))
        drv = int(r.integers(0, 2))
        n = int(r.integers(2, 6) if L >= 512 else r.integers(4, 17))
        if L >= 512:
            T_max = min(T_max, 64)
        out.append((i, L, p, T_max, k, drv, n))
    return out


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_03266_amd.binding as b
    b.lib()
    return b


@pytest.mark.parametrize("case", cases(), ids=lambda c: f"{c[0]}-L{c[1]}-k{c[4]}")
def test_random_configuration(gpu, orc, case):
    i, L, p, T_max, k, drv, n = case
    s = seeds(91, i, n)
    ref = orc.decode_seeds(L, p, s, T_max, threads=16)
    old_k, old_d = gpu.get_band_bits(L), gpu.get_band_driver(L)
    gpu.set_band_bits(k, L)
    gpu.set_band_driver(gpu.BAND_DRIVER_DEVICE if drv else gpu.BAND_DRIVER_HOST, L)
    try:
        T, F, S = gpu.decode_batch(L, p, s, T_max)
    finally:
        gpu.set_band_bits(old_k, L)
        gpu.set_band_driver(old_d, L)
    T, F = T.cpu().numpy(), F.cpu().numpy()
    S = S.cpu().numpy().view(np.uint32).reshape(n, -1)
    tag = f"case {i}: L={L} p={p:.4f} T_max={T_max} k_bits={k} driver={'device' if drv else 'host'} n={n}"
    assert np.array_equal(T, ref["T_dec"]), f"{tag}: T_dec {T} vs {ref['T_dec']}"
    assert np.array_equal(F, ref["flags"]), f"{tag}: flags {F} vs {ref['flags']}"
    assert np.array_equal(S, ref["sigma_words"]), f"{tag}: final syndrome"
