"""Build the HIP C-ABI library ``libhweno.so`` for gfx950, in-tree.

    python -m paper_2411_11229_amd.build            # build the library
    python -m paper_2411_11229_amd.build --asm DIR  # also keep the device assembly

hipcc cross-compiles for gfx950 without a GPU. Packed FP32 instructions are
disabled for all device code.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, 'csrc', 'hweno_kernels.hip')]
LIB = os.path.join(HERE, 'libhweno.so')
ARCH = 'gfx950'

FLAGS = [
    '-O3', '-std=c++17', '-fPIC', '-shared',
    f'--offload-arch={ARCH}',
    '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
    '-ffp-contract=fast',
    '-Wall', '-Wno-unused-function', '-Wno-unused-variable',
    f'-I{os.path.join(ROOT, "include")}',
]


def hipcc():
    for cand in (os.environ.get('HIPCC'), '/opt/rocm/bin/hipcc', shutil.which('hipcc')):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError('hipcc not found (ROCm toolchain required to build libhweno.so)')


def build(asm_dir=None, verbose=False):
    """Compile every HIP source into LIB. Always recompiles."""
    tmp = LIB + '.tmp'
    cmd = [hipcc()] + FLAGS + SRC + ['-o', tmp]
    if asm_dir:
        os.makedirs(asm_dir, exist_ok=True)
        cmd += ['-save-temps=cwd', '-Rpass-analysis=kernel-resource-usage']
    if verbose:
        print(' '.join(cmd), flush=True)
    res = subprocess.run(cmd, cwd=asm_dir or HERE, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError('hipcc failed building libhweno.so')
    if verbose and (res.stdout or res.stderr):
        sys.stderr.write(res.stdout + res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == '__main__':
    asm = None
    if '--asm' in sys.argv:
        asm = sys.argv[sys.argv.index('--asm') + 1]
    print(build(asm_dir=asm, verbose=True))
