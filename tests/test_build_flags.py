"""The library's device code is built without packed-FP32 instructions.

build.py passes `-Xclang -target-feature -Xclang -packed-fp32-ops` to every
hipcc compile.  hipcc's host pass warns that it does not know the feature;
the device pass applies it.  This test compiles a small float2 kernel with
and without the flag to gfx950 assembly (the flag must remove the packed
instructions the compiler otherwise emits), and every library source with
the library's own flags (no v_pk_add_f32, v_pk_mul_f32 or v_pk_fma_f32)."""
import concurrent.futures as cf
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PK = re.compile(r"\bv_pk_(add|mul|fma)_f32\b")

PROBE = r"""
#include <hip/hip_runtime.h>
__global__ void probe(float2 *a, const float2 *b, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        float2 x = a[i], y = b[i];
        x.x = x.x * y.x + 1.5f; x.y = x.y * y.y + 1.5f;
        x.x += y.y; x.y += y.x;
        a[i] = x;
    }
}
"""


def device_asm(src: str, flags, out_dir: str) -> str:
    from paper_2505_07158_amd import build as B
    out = os.path.join(out_dir, os.path.basename(src) + ".s")
    cmd = [B.hipcc(), *flags, "-S", "--cuda-device-only", src, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    return open(out).read()


def test_flag_removes_packed_fp32_from_device_code():
    from paper_2505_07158_amd import build as B
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.hip")
        open(src, "w").write(PROBE)
        base = [f for f in B.FLAGS if f not in ("-fPIC",)]
        i = base.index("-packed-fp32-ops")
        without = base[:i - 3] + base[i + 1:]      # drop "-Xclang -target-feature -Xclang -packed-fp32-ops"
        assert "-packed-fp32-ops" not in without and len(without) == len(base) - 4
        assert PK.search(device_asm(src, without, d)), "probe kernel should use packed FP32 without the flag"
        assert not PK.search(device_asm(src, base, d))


def test_library_sources_have_no_packed_fp32():
    from paper_2505_07158_amd import build as B
    flags = [f for f in B.FLAGS if f != "-fPIC"]
    with tempfile.TemporaryDirectory() as d:
        with cf.ThreadPoolExecutor(len(B.SOURCES)) as ex:
            asms = list(ex.map(lambda s: device_asm(os.path.join(B.CSRC, s), flags, d), B.SOURCES))
    for s, a in zip(B.SOURCES, asms):
        assert not PK.search(a), s
