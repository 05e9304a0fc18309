"""Host logic of the table layouts read with paired 16-byte loads
(tests/table_layout_main.cpp): the level table of FFT twiddle powers and the
mirror-pair layout of the FP32 static phase rows, checked against the lane
slots of every plan (N, W) that the kernels use.  No GPU: the indexing is
host/device-shared constexpr code compiled here with g++."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM_INCLUDE = "/opt/rocm/include"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.isdir(ROCM_INCLUDE),
                    reason="g++ or the ROCm headers not available")
def test_paired_table_layouts(tmp_path):
    exe = str(tmp_path / "table_layout")
    cmd = ["g++", "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + ROCM_INCLUDE,
           os.path.join(HERE, "table_layout_main.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok:"), r.stdout
