"""The allocation-free decode (mpd_decode_batch_static) against the decode
with a caller's workspace (mpd_decode_batch): identical T_dec, flags and
final syndromes, bit for bit, on two calls in a row (the second smaller,
so that it runs on scratch still holding the first call's state), at a
resident size and at band-path sizes with one and several tiles."""
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


def _same(a, b, tag):
    for x, y, what in zip(a, b, ("T_dec", "flags", "syndrome")):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy()), f"{tag}: {what} differs"


@pytest.mark.parametrize("L,p,n1,n2,T_max", [(256, 0.01, 120, 37, 4096), (256, 0.06, 64, 9, 24),
                                             (512, 0.03, 30, 4, 4096), (1024, 0.01, 7, 2, 4096),
                                             (64, 0.02, 300, 11, 4096)])
def test_static_equals_workspace_decode(gpu, L, p, n1, n2, T_max):
    for call, n in enumerate((n1, n2)):
        s = seeds(60, 100 * L + call, n)
        ref = gpu.decode_batch(L, p, s, T_max)
        got = gpu.decode_batch_static(L, p, s, T_max)
        _same(got, ref, f"L={L} call {call} n={n}")


def test_static_rejects_oversize(gpu):
    import torch
    L = 256
    n = 200  # about 1.03 MiB of state per sample: more than the 128 MiB scratch
    assert gpu.workspace_bytes(L, n) > gpu.STATIC_SCRATCH_BYTES
    s = torch.zeros(n, dtype=torch.int64, device="cuda")
    T = torch.empty(n, dtype=torch.int32, device="cuda")
    F = torch.empty(n, dtype=torch.uint8, device="cuda")
    rc = gpu.lib().mpd_decode_batch_static(L, 0.01, gpu._ptr(s), n, 64, gpu._ptr(T), gpu._ptr(F), None, None)
    assert rc == -5
    assert b"scratch" in gpu.lib().mpd_last_error()
    # a call within the limit still works afterwards
    ss = seeds(61, 0, 5)
    _same(gpu.decode_batch_static(L, 0.01, ss, 4096), gpu.decode_batch(L, 0.01, ss, 4096), "after rejection")
