"""Build libpse.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1709_06946_amd.build   (or build() from Python).
Every call recompiles all sources, and the host packing generator of the
synthetic inputs (libpack.so, plain C).
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
BUILD = os.path.join(HERE, '_build')
LIB = os.path.join(HERE, 'libpse.so')
PACK_SRC = os.path.join(HERE, 'packing.c')
PACK_LIB = os.path.join(HERE, 'libpack.so')
HIPCC = os.environ.get('HIPCC', '/opt/rocm/bin/hipcc')
ARCH = 'gfx950'

SOURCES = ['params.cpp', 'serve.cpp', 'fft.hip', 'grid.hip', 'real.hip', 'krylov.hip',
           'api.hip']

FLAGS = ['-O3', '-std=c++17', '-fPIC', f'--offload-arch={ARCH}',
         '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
         '-Wall', '-Wno-unused-function', '-Wno-unused-variable',
         '-Wno-unused-command-line-argument']


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + '.o')
    cmd = [HIPCC] + FLAGS + ['-c', os.path.join(CSRC, src), '-o', obj]
    if src.endswith('.cpp'):
        cmd = [HIPCC, '-O3', '-std=c++17', '-fPIC', '-Wall', '-pthread', '-c',
               os.path.join(CSRC, src), '-o', obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f'compile failed: {src}\n{r.stdout}\n{r.stderr}')
    return obj, r.stderr


def build_packing():
    """The host-only packing generator of the synthetic inputs (plain C)."""
    tmp = PACK_LIB + f'.tmp{os.getpid()}'
    cmd = ['gcc', '-O2', '-std=c99', '-fPIC', '-shared', '-Wall', '-o', tmp, PACK_SRC, '-lm']
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f'compile failed: packing.c\n{r.stdout}\n{r.stderr}')
    os.replace(tmp, PACK_LIB)
    return PACK_LIB


def build(verbose=False):
    build_packing()
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), int(os.environ.get('MAX_JOBS', os.cpu_count() or 4)))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    tmp = LIB + '.tmp'
    cmd = [HIPCC, '-shared', '-pthread', f'--offload-arch={ARCH}', '-o', tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f'link failed\n{r.stdout}\n{r.stderr}')
    os.replace(tmp, LIB)
    return LIB


if __name__ == '__main__':
    print(build(verbose=True))
