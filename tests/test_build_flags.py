"""Properties of the library's gfx950 device code (CPU only): it is built
without packed FP32 instructions, and no kernel spills registers or uses
private memory.

hipcc for gfx950 turns ordinary float2 / paired float arithmetic into
v_pk_{add,mul,fma}_f32 unless the target feature packed-fp32-ops is
switched off.  The library's build line switches it off (the host pass of
hipcc warns that it does not know the feature, which is expected: the
feature belongs to the device pass).  These tests compile device code only
(no GPU needed) and read the gfx950 assembly of our own sources."""
from __future__ import annotations

import os
import re
import subprocess

import pytest

from paper_2506_03266_amd import build

HIPCC = "/opt/rocm/bin/hipcc"
FEATURE = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
PACKED = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")

pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")


def device_asm(src_path, flags, out):
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "--cuda-device-only", "-S", "-o", out,
           "-I", os.path.join(build.ROOT, "include"), "-I", build.CSRC] + flags + [src_path]
    subprocess.run(cmd, check=True, capture_output=True)
    with open(out) as f:
        return f.read()


def test_build_line_switches_packed_fp32_off():
    flags = build.HIPCC_FLAGS
    i = flags.index("-target-feature")
    assert flags[i - 1] == "-Xclang" and flags[i + 1] == "-Xclang" and flags[i + 2] == "-packed-fp32-ops"


def test_feature_removes_packed_fp32_on_the_device(tmp_path):
    probe = os.path.join(tmp_path, "probe.hip")
    with open(probe, "w") as f:
        f.write("#include <hip/hip_runtime.h>\n"
                "__global__ void k(float2 *a, const float2 *b, float s) {\n"
                "  int i = threadIdx.x; float2 x = a[i], y = b[i];\n"
                "  x.x = x.x * s + y.x; x.y = x.y * s + y.y; a[i] = x; }\n")
    on = device_asm(probe, [], os.path.join(tmp_path, "on.s"))
    off = device_asm(probe, FEATURE, os.path.join(tmp_path, "off.s"))
    assert PACKED.search(on), "the probe no longer produces packed FP32; pick a probe that does"
    assert not PACKED.search(off)


_ASM = {}


def library_asm(tmp_path_factory, src):
    """gfx950 assembly of one library source, built with the library's flags."""
    if src not in _ASM:
        flags = [f for f in build.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
        flags = [f for f in flags if not f.startswith("--offload-arch")]
        out = os.path.join(tmp_path_factory.mktemp("asm"), src + ".s")
        _ASM[src] = device_asm(os.path.join(build.CSRC, src), flags, out)
    return _ASM[src]


@pytest.mark.slow
@pytest.mark.parametrize("src", build.SOURCES)
def test_library_has_no_packed_fp32(tmp_path_factory, src):
    asm = library_asm(tmp_path_factory, src)
    m = PACKED.search(asm)
    assert m is None, f"{src}: {m.group(0)} in the gfx950 code"


KERNEL = re.compile(r"^\s*\.amdhsa_kernel (\S+)$(.*?)^\s*\.end_amdhsa_kernel", re.M | re.S)
PRIVATE = re.compile(r"\.amdhsa_private_segment_fixed_size (\d+)")


@pytest.mark.slow
@pytest.mark.parametrize("src", build.SOURCES)
def test_library_kernels_use_no_private_memory(tmp_path_factory, src):
    """Every kernel keeps its working set in registers and LDS: no VGPR
    spill slots and no private (scratch) segment.  (SGPRs that overflow go
    to lanes of a VGPR, not to memory, and are not counted.)  Register pressure of the
    decoder kernels sits close to the budget of their launch bounds, so a
    change that hoists per-row addresses or constants out of the step loop
    shows up here before it shows up as lost throughput."""
    asm = library_asm(tmp_path_factory, src)
    kernels = KERNEL.findall(asm)
    assert kernels, f"{src}: no kernels found in the assembly"
    bad = [(name, int(PRIVATE.search(body).group(1))) for name, body in kernels
           if int(PRIVATE.search(body).group(1)) != 0]
    assert not bad, f"{src}: kernels with a private segment (bytes per lane): {bad}"
    counts = [int(c) for c in re.findall(r"\.vgpr_spill_count:\s*(\d+)", asm)]
    assert len(counts) == len(kernels) and not any(counts), f"{src}: VGPR spills {counts}"
