"""Host build of the HIP path's per-point math (compiled with hipcc, run on
the CPU): every hand-written reverse-mode function against central finite
differences of its forward function, and the structured characteristic
projections against the explicit eigenvector rows and columns."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, 'tests', 'cpu_math', 'adjoint_check.cpp')
INC = os.path.join(ROOT, 'paper_2411_11229_amd', 'csrc')


def test_adjoint_math_against_finite_differences(tmp_path):
    hipcc = shutil.which('hipcc') or '/opt/rocm/bin/hipcc'
    if not os.path.exists(hipcc):
        pytest.skip('hipcc not available')
    exe = str(tmp_path / 'adjoint_check')
    subprocess.run([hipcc, '-O1', '-std=c++17', '--offload-arch=gfx950', f'-I{INC}', SRC, '-o', exe],
                   check=True, capture_output=True, text=True)
    res = subprocess.run([exe], capture_output=True, text=True)
    print(res.stdout)
    assert res.returncode == 0 and 'ALL OK' in res.stdout, res.stdout + res.stderr
