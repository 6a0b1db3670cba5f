"""The build keeps packed FP32 instructions out of the device code: the
target feature that forbids them reaches the gfx950 device pass (a float2
multiply-add compiles to v_pk_fma_f32 without it and to none with it), and
the library's own sources compile to device assembly without any."""
import os
import shutil

import pytest

from paper_2004_04080_amd import build as hb

PROBE = """#include <hip/hip_runtime.h>
__global__ void probe(float2* a, const float2* b, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    float2 x = a[i], y = b[i];
    x.x = x.x * y.x + y.y;
    x.y = x.y * y.y + y.x;
    a[i] = x;
  }
}
"""

needs_hipcc = pytest.mark.skipif(not shutil.which(hb.HIPCC) and not os.path.exists(hb.HIPCC),
                                 reason="hipcc not installed")


@needs_hipcc
def test_feature_flag_reaches_the_device_pass(tmp_path):
    src = tmp_path / "probe.hip"
    src.write_text(PROBE)
    plain = [f for f in hb.FLAGS if f not in ("-Xclang", "-target-feature", "-packed-fp32-ops")]
    assert len(plain) == len(hb.FLAGS) - 4
    without = hb.device_asm(str(src), str(tmp_path / "a.s"), plain)
    with_flag = hb.device_asm(str(src), str(tmp_path / "b.s"))
    assert hb.PACKED_FP32.search(without), "the probe no longer makes packed FP32 code"
    assert not hb.PACKED_FP32.search(with_flag)


@needs_hipcc
@pytest.mark.parametrize("src", hb.SOURCES)
def test_library_device_code_has_no_packed_fp32(src, tmp_path):
    asm = hb.device_asm(os.path.join(hb.CSRC, src), str(tmp_path / "x.s"))
    assert not hb.PACKED_FP32.search(asm)
