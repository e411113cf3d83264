"""The bit-sliced kernel at L = 64 (one wave per sample, one column per
lane) and L = 128 (two waves, two columns per lane), against the CPU oracle
bit for bit (T_dec, flags and final syndrome): every number of bit-sliced
steps, budgets that end inside them (the final syndrome then comes from the
bit-sliced kernel), noise strengths from none to every link, per-sample
noise strength, and samples still decoding after the bit-sliced steps (the
whole-lattice kernel decodes them again from their seeds, on a resident grid
at low p and one workgroup per sample otherwise).  A batch with one p >=
0.045 skips the bit-sliced steps, so each case above that also runs as
per-sample p, which keeps them.  Every setting must give the whole-lattice
kernel's results."""
import numpy as np
import pytest

from paper_2506_03266_amd.workloads import seeds

pytestmark = pytest.mark.gpu

SIZES = [64, 128]


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


def both_forms(gpu, L, p, s, T_max):
    """The decode with one p for the batch and with the same p per sample."""
    n = len(s)
    one = gpu.decode_batch(L, p, s, T_max)
    per = gpu.decode_mixed([(L, n)], np.full(n, p), s, T_max)
    return (("one p", one), ("per-sample p", per))


def with_bits(gpu, L, k, fn):
    old = gpu.get_band_bits(L)
    gpu.set_band_bits(k, L)
    try:
        return fn()
    finally:
        gpu.set_band_bits(old, L)


@pytest.mark.parametrize("L", SIZES)
def test_default_is_ten_steps(gpu, L):
    assert gpu.get_band_bits(L) == 10


@pytest.mark.parametrize("L", SIZES)
@pytest.mark.parametrize("k", [0, 1, 2, 3, 4, 5, 6, 8, 10])
@pytest.mark.parametrize("p", [0.01, 0.05, 0.09])
def test_steps_against_oracle(gpu, orc, L, k, p):
    """p = 0.09 is above the threshold: most samples are still decoding
    after ten steps and take the whole-lattice kernel."""
    n, T_max = 48, 512
    s = seeds(71, L * 100 + int(p * 1000) * 8 + k, n)
    ref = orc.decode_seeds(L, p, s, T_max, threads=16)
    for form, (T, F, S) in with_bits(gpu, L, k, lambda: both_forms(gpu, L, p, s, T_max)):
        compare(f"L={L} k_bits={k} p={p} {form}", T, F, S, ref)


@pytest.mark.parametrize("L", SIZES)
@pytest.mark.parametrize("T_max", [0, 1, 2, 3, 4, 5, 6, 9, 10, 11, 12])
def test_budgets_inside_the_bit_sliced_steps(gpu, orc, L, T_max):
    """Timeouts at T_max <= 10 leave their final syndrome from the
    bit-sliced kernel; T_max = 11 and 12 end in the whole-lattice kernel."""
    p, n = 0.08, 32
    s = seeds(72, L * 100 + T_max, n)
    ref = orc.decode_seeds(L, p, s, T_max, threads=16)
    for form, (T, F, S) in both_forms(gpu, L, p, s, T_max):
        compare(f"L={L} T_max={T_max} {form}", T, F, S, ref)


@pytest.mark.parametrize("L", SIZES)
@pytest.mark.parametrize("p", [0.0, 0.5, 1.0])
def test_extreme_noise(gpu, orc, L, p):
    n, T_max = 8, 64
    s = seeds(73, L + int(p * 10), n)
    ref = orc.decode_seeds(L, p, s, T_max, threads=8)
    T, F, S = gpu.decode_batch(L, p, s, T_max)
    compare(f"L={L} p={p}", T, F, S, ref)


@pytest.mark.parametrize("L", SIZES)
def test_per_sample_noise_strength(gpu, orc, L):
    n, T_max = 96, 1024
    s = seeds(74, L, n)
    ps = np.random.default_rng(74 + L).uniform(0.001, 0.1, n)
    ref = orc.decode_seeds(L, ps, s, T_max, threads=16)
    T, F, S = gpu.decode_mixed([(L, n)], ps, s, T_max)
    compare(f"L={L} per-sample p", T, F, S, ref)


@pytest.mark.parametrize("L", SIZES)
def test_same_as_whole_lattice_kernel_on_a_large_batch(gpu, L):
    """4096 samples at p = 0.01 (survivors resumed on a resident grid), 0.03
    (one workgroup per survivor) and 0.07 as per-sample p (nearly every
    sample resumed): every setting of the bit-sliced steps gives the
    whole-lattice kernel's results."""
    n, T_max = 4096, 4096
    for p, per_sample in ((0.01, False), (0.03, False), (0.07, True)):
        s = seeds(75, L + int(p * 100), n)

        def run():
            if per_sample:
                return gpu.decode_mixed([(L, n)], np.full(n, p), s, T_max)
            return gpu.decode_batch(L, p, s, T_max)
        base = [x.cpu().numpy() for x in with_bits(gpu, L, 0, run)]
        for k in (1, 4, 7, 10):
            got = [x.cpu().numpy() for x in with_bits(gpu, L, k, run)]
            for a, b, name in zip(got, base, ("T_dec", "flags", "syndrome")):
                assert np.array_equal(a, b), f"L={L} p={p} k_bits={k}: {name} differs from the whole-lattice kernel"


@pytest.mark.parametrize("L", SIZES)
def test_bit_sliced_steps_skipped_at_high_one_p(gpu, L):
    """With one p for the batch the bit-sliced kernel runs below p = 0.045
    and not from there on; per-sample p always runs it."""
    n, T_max = 256, 4096
    s = seeds(77, L, n)

    def launches(fn):  # launches of the bit-sliced kernel during fn()
        import torch
        torch.cuda.synchronize()
        gpu.profile(True)
        try:
            fn()
            torch.cuda.synchronize()
        finally:
            gpu.profile(False)
        return gpu.profile_read("k_bits_small")[1]
    assert launches(lambda: gpu.decode_batch(L, 0.044, s, T_max)) == 1
    assert launches(lambda: gpu.decode_batch(L, 0.045, s, T_max)) == 0
    assert launches(lambda: gpu.decode_batch(L, 0.08, s, T_max)) == 0
    assert launches(lambda: gpu.decode_mixed([(L, n)], np.full(n, 0.08), s, T_max)) == 1


def test_mixed_classes_against_oracle(gpu, orc):
    """One mixed call over L = 64, 128 and 256 with per-sample p: the three
    bit-sliced variants side by side."""
    classes = [(64, 64), (128, 32), (256, 8)]
    n = sum(c for _, c in classes)
    s = seeds(76, 0, n)
    ps = np.random.default_rng(76).uniform(0.002, 0.06, n)
    T, F, S = gpu.decode_mixed(classes, ps, s, 2048)
    T, F = T.cpu().numpy(), F.cpu().numpy()
    S = S.cpu().numpy().view(np.uint32)
    off, woff = 0, 0
    for L, c in classes:
        ref = orc.decode_seeds(L, ps[off:off + c], s[off:off + c], 2048, threads=16)
        nw = L * L // 32
        assert np.array_equal(T[off:off + c], ref["T_dec"]), f"L={L}: T_dec"
        assert np.array_equal(F[off:off + c], ref["flags"]), f"L={L}: flags"
        assert np.array_equal(S[woff:woff + c * nw].reshape(c, nw), ref["sigma_words"]), f"L={L}: syndrome"
        off += c
        woff += c * nw
