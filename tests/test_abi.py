"""Host-side checks of the C ABI (no GPU work): the library loads, exports
every function include/pse.h declares, derives parameters by the stated rules
and rejects invalid input with error codes."""
import ctypes
import math
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from oracle import params as oparams

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'pse.h')


@pytest.fixture(scope='module')
def pse():
    from paper_1709_06946_amd import pse as mod
    if not os.path.exists(mod.LIB_PATH):
        from paper_1709_06946_amd import build
        build.build()
    return mod


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r'^\s*(?:const\s+)?\w+\s*\*?\s*(pse_\w+)\s*\(', text, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ('pse_create', 'pse_destroy', 'pse_mobility_apply', 'pse_brownian_sample',
              'pse_constrained_step', 'pse_footprint_bytes', 'pse_last_error'):
        assert n in names


def test_library_exports_every_declared_symbol(pse):
    out = subprocess.run(['nm', '-D', '--defined-only', pse.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r' T (pse_\w+)', out))
    missing = set(declared_functions()) - exported
    assert not missing, missing
    lib = pse.load_library()
    for n in declared_functions():
        assert hasattr(lib, n)


def test_struct_sizes_match_header(pse):
    """Compile a tiny C program against the header and compare sizeof/offsetof
    with the ctypes mirrors used by the binding."""
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "pse.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(pse_params), sizeof(pse_derived),
         sizeof(pse_stats), sizeof(pse_step_io));
  printf("%zu %zu %zu\n", offsetof(pse_params, stream), offsetof(pse_derived, gmres_tol),
         offsetof(pse_stats, fp64_residual));
  return 0;
}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, 't.c')
        open(c, 'w').write(src)
        exe = os.path.join(d, 't')
        subprocess.run(['gcc', '-I', os.path.join(ROOT, 'include'), c, '-o', exe], check=True)
        lines = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split('\n')
    sizes = [int(v) for v in lines[0].split()]
    offs = [int(v) for v in lines[1].split()]
    assert sizes == [ctypes.sizeof(pse.pse_params), ctypes.sizeof(pse.pse_derived),
                     ctypes.sizeof(pse.pse_stats), ctypes.sizeof(pse.pse_step_io)]
    assert offs == [pse.pse_params.stream.offset, pse.pse_derived.gmres_tol.offset,
                    pse.pse_stats.fp64_residual.offset]


@pytest.mark.parametrize('eps', [1e-2, 1e-3, 1e-4, 1e-5])
def test_derive_support_and_width_rule(pse, eps):
    """Eq. bound's orthorhombic rule at the tightened quadrature tolerance
    eps/20, a Gaussian truncated at 0.85 of the balanced width, and xi placing
    exp(-u_N) = e^-9 eps at the Nyquist wave number (moment gridding)."""
    p = pse.make_params(100, 30.0, grid=64, tol=eps, deriv_gridding=1)
    d = pse.derive(p)
    assert d.deriv_gridding == 1
    assert d.support == oparams.support_orthorhombic(eps / 20)
    assert math.isclose(d.m, 0.85 * math.sqrt(math.pi * d.support))
    assert math.isclose(d.h, 30.0 / 64)
    assert math.isclose(d.eta_s, (d.h * d.support * d.xi / d.m) ** 2)
    assert d.eta_s < 1
    kn = math.pi * 64 / 30.0
    assert math.isclose(kn**2 / (4 * d.xi**2), math.log(1 / eps) + 9, rel_tol=1e-12)
    assert math.isclose(d.rcut, 2.0 + math.sqrt(math.log(1 / eps)) / d.xi)
    assert d.cells == int(30.0 // d.rcut)


@pytest.mark.parametrize('eps', [1e-2, 1e-3, 1e-4, 1e-5])
def test_derivative_gridding_takes_one_more_support_point(pse, eps):
    """The default gridding of M_ES is the derivative one with one support
    point more than the moment rule, while that stays within 10 points (else
    the moment gridding and its support are used)."""
    base = oparams.support_orthorhombic(eps / 20)
    for mode in (0, 2):
        d = pse.derive(pse.make_params(100, 30.0, grid=64, tol=eps, deriv_gridding=mode))
        if base + 1 <= 10:
            assert (d.deriv_gridding, d.support) == (2, base + 1)
        else:
            assert (d.deriv_gridding, d.support) == (1, base)
        assert math.isclose(d.m, 0.85 * math.sqrt(math.pi * d.support))
    with pytest.raises(pse.PSEError):
        pse.derive(pse.make_params(100, 30.0, grid=64, tol=eps, deriv_gridding=3))


def test_derive_support_at_1e3(pse):
    """At eps = 1e-3 the tightened rule gives P = 7 (Table 1's orthorhombic
    row, P = 5, is the untightened rule, pinned in the oracle tests)."""
    d = pse.derive(pse.make_params(100, 16.12, grid=32, tol=1e-3, deriv_gridding=1))
    assert d.support == 7
    assert pse.derive(pse.make_params(100, 16.12, grid=32, tol=1e-3)).support == 8


def test_derive_grid_from_xi(pse):
    d = pse.derive(pse.make_params(1000, 40.0, xi=1.0, tol=1e-3))
    need = 2 * 1.0 * 40.0 * math.sqrt(math.log(1e3) + 9) / math.pi
    assert d.grid >= need
    assert d.grid in (96, 128)
    assert d.xi == 1.0


@pytest.mark.parametrize('bad', [
    dict(n=0), dict(box=3.0), dict(tol=0.5), dict(grid=100), dict(grid=0, xi=0.0),
    dict(radius=-1.0), dict(precision=7), dict(grid=8, xi=5.0),
])
def test_invalid_parameters_rejected(pse, bad):
    kw = dict(n=100, box=20.0, grid=32, tol=1e-3)
    kw.update(bad)
    n, box = kw.pop('n'), kw.pop('box')
    p = pse.make_params(n, box, **kw)
    d = pse.pse_derived()
    rc = pse.lib().pse_derive(ctypes.byref(p), ctypes.byref(d))
    assert rc == -1
    assert len(pse.lib().pse_last_error(None)) > 0
    h = ctypes.c_void_p()
    assert pse.lib().pse_create(ctypes.byref(p), ctypes.byref(h)) == -1
    assert h.value is None


def test_null_arguments_rejected(pse):
    lib = pse.lib()
    assert lib.pse_derive(None, None) == -1
    assert lib.pse_mobility_apply(None, None, None, None, 3) == -1
    assert lib.pse_destroy(None) == 0


def test_footprint_grows_with_grid_and_precision(pse):
    # same cutoff for both grids, so that the pair list is the same size
    f = [pse.footprint_bytes(pse.make_params(10000, 52.0, grid=g, tol=1e-3, rcut=6.0))
         for g in (64, 128)]
    assert f[1] - f[0] >= 0.99 * 2 * 6 * (128**3 - 64**3) * 16
    fm = pse.footprint_bytes(pse.make_params(10000, 52.0, grid=128, tol=1e-3, rcut=6.0,
                                             precision=1))
    # mixed handles: FP32 grid sets (6 packed complex grids each way) plus
    # FP64 sets of 3 for the residual of the constraint solve
    assert fm > 2 * 6 * 128**3 * 8 + 2 * 3 * 128**3 * 16
    # FP64 grids dominate: 2 sets x 6 packed complex grids x 16 B
    assert f[1] > 2 * 6 * 128**3 * 16


def test_library_binds_to_torchs_hip_runtime():
    """One HIP runtime per process: after loading the binding in a fresh
    interpreter, only torch's copy of libamdhip64 is mapped."""
    code = ("from paper_1709_06946_amd import pse; pse.lib(); "
            "m = open('/proc/self/maps').read().splitlines(); "
            "print(sorted({l.split()[-1] for l in m if 'libamdhip64' in l}))")
    out = subprocess.run([sys.executable, '-c', code], capture_output=True, text=True,
                         cwd=ROOT, check=True).stdout
    paths = eval(out.strip())
    assert len(paths) == 1 and 'torch' in paths[0], paths


def test_server_error_without_server_is_empty(pse):
    """pse_server_error never returns NULL: "" for a null server or an
    unknown request (no device needed)."""
    lib = pse.load_library()
    assert lib.pse_server_error(None, 1) == b''


def test_binding_refuses_wrong_element_types(pse):
    """The kernels read each argument with one element type: float64 particle
    arrays, complex128 wave noise and FFT data.  Any other dtype is refused
    before a pointer is formed (a float64 wave noise of the complex shape
    would be read past its end)."""
    import torch
    g = 8
    with pytest.raises(TypeError, match='complex128'):
        pse._ptr(torch.zeros((3, g, g, g // 2 + 1), dtype=torch.float64), (3, g, g, g // 2 + 1),
                 'psi_wave', 'complex128')
    with pytest.raises(TypeError, match='float64'):
        pse._ptr(torch.zeros((4, 3), dtype=torch.float32), (4, 3), 'x')
    with pytest.raises(TypeError, match='float64'):
        pse._ptr(torch.zeros((4, 11), dtype=torch.complex128), (4, 11), 'in')
    # the right dtype on the host is still refused: device memory only
    with pytest.raises(TypeError, match='device'):
        pse._ptr(torch.zeros((4, 3), dtype=torch.float64), (4, 3), 'x')
