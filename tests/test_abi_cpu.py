"""C-ABI library checks that need no GPU: it loads, exports every symbol the
header declares, and rejects invalid problems before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2411_11229_amd import hweno as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'hweno.h')


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r'/\*.*?\*/', '', src, flags=re.S)
    return sorted(set(re.findall(r'\b(hweno_[a-z_]+)\s*\(', src)))


@pytest.fixture(scope='module')
def lib():
    if not os.path.exists(H.LIB_PATH):
        pytest.fail('libhweno.so is not built (run python -m paper_2411_11229_amd.build)')
    return H.load_library()


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(H.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def _prob(**kw):
    base = dict(dim=2, nx=64, ny=48, dx=0.1, dy=0.2, system='euler')
    base.update(kw)
    return H.Problem(**base).c()


def _ws_bytes(lib, p):
    n = ctypes.c_size_t(0)
    st = lib.hweno_workspace_bytes(ctypes.byref(p) if p is not None else None, ctypes.byref(n))
    return st, n.value


def test_workspace_size_valid_problem(lib):
    st, n = _ws_bytes(lib, _prob())
    assert st == 0
    # X^(1), X^(2), lambda^(2), lambda^(1): 4 states of 3 fields x 4
    # components; the RK base derivatives: 2 x 4 planes; float64, plus the
    # scalars, partial maxima and ghost buffer
    assert n >= (4 * 12 + 8) * 64 * 48 * 8
    st32, n32 = _ws_bytes(lib, _prob(precision='f32'))
    assert st32 == 0 and n32 < n


@pytest.mark.parametrize("bad", [
    dict(nx=4), dict(ny=4), dict(dim=3), dict(dim=1, ny=4), dict(dx=0.0), dict(dy=-1.0),
    dict(dx=float('nan')), dict(gas_gamma=1.0), dict(gamma0=1.0), dict(gamma0=0.0),
    dict(d0=1.5), dict(eps=0.0), dict(bc=('periodic', 'transmissive', 'periodic', 'periodic')),
    dict(bc=('periodic', 'periodic', 'transmissive', 'periodic')),
    dict(nx=40000, ny=40000),
    dict(system='burgers', bc=('reflective', 'reflective', 'periodic', 'periodic')),
    dict(system='advection', bc=('periodic', 'periodic', 'transmissive', 'reflective')),
    dict(bc=('reflective', 'periodic', 'periodic', 'periodic')),
])
def test_invalid_problems_rejected(lib, bad):
    st, _ = _ws_bytes(lib, _prob(**bad))
    assert st == -1


@pytest.mark.parametrize("bc", [('reflective',) * 4,
                                ('reflective', 'transmissive', 'periodic', 'periodic'),
                                ('transmissive', 'reflective', 'reflective', 'transmissive')])
def test_reflective_walls_accepted_for_euler(lib, bc):
    assert _ws_bytes(lib, _prob(bc=bc))[0] == 0
    assert _ws_bytes(lib, _prob(dim=1, ny=1, bc=bc))[0] == 0


def test_fixed_states_and_gravity_validated(lib):
    good = (1.0, 0.2, -0.1, 2.5)
    bc = ('dirichlet', 'transmissive', 'reflective', 'dirichlet')
    assert _ws_bytes(lib, _prob(bc=bc, bc_state=(good, None, None, good), gravity=1.0))[0] == 0
    # non-physical or non-finite fixed state, gravity outside 2D Euler
    for bad in ((-1.0, 0.0, 0.0, 2.5), (1.0, 3.0, 0.0, 1.0), (1.0, float('nan'), 0.0, 2.5)):
        assert _ws_bytes(lib, _prob(bc=bc, bc_state=(bad, None, None, good)))[0] == -1
    assert _ws_bytes(lib, _prob(dim=1, ny=1, gravity=1.0))[0] == -1
    assert _ws_bytes(lib, _prob(system='burgers', gravity=1.0))[0] == -1
    assert _ws_bytes(lib, _prob(gravity=float('inf')))[0] == -1
    # scalar laws take fixed states too (first component)
    assert _ws_bytes(lib, _prob(system='burgers', bc=('dirichlet', 'dirichlet', 'periodic', 'periodic'),
                                bc_state=((0.3,), (0.1,), None, None)))[0] == 0


def test_split_sides_validated(lib):
    st = (1.0, 0.2, -0.1, 2.5)
    sp = dict(x0=0.3, slope=0.0, speed=1.0, kinds=('dirichlet', 'reflective'), states=(st, None))
    ok = dict(bc=('transmissive', 'transmissive', 'split', 'split'), split=(sp, sp))
    assert _ws_bytes(lib, _prob(**ok))[0] == 0
    # split on an x side, in 1D, for a scalar law; bad kinds and states
    assert _ws_bytes(lib, _prob(bc=('split', 'transmissive', 'periodic', 'periodic'), split=(sp, sp)))[0] == -1
    assert _ws_bytes(lib, _prob(system='burgers', **ok))[0] == -1
    bad_kind = dict(sp, kinds=('periodic', 'reflective'))
    assert _ws_bytes(lib, _prob(bc=ok['bc'], split=(bad_kind, sp)))[0] == -1
    bad_state = dict(sp, states=((1.0, 5.0, 0.0, 1.0), None))
    assert _ws_bytes(lib, _prob(bc=ok['bc'], split=(sp, bad_state)))[0] == -1
    assert _ws_bytes(lib, _prob(bc=ok['bc'], split=(dict(sp, speed=float('nan')), sp)))[0] == -1


def test_state_array_size_limit(lib):
    # one state array must stay under 4 GiB (32-bit byte offsets)
    assert _ws_bytes(lib, _prob(nx=12000, ny=12000))[0] == -1          # 4.6 GB in FP64
    assert _ws_bytes(lib, _prob(nx=12000, ny=12000, precision='f32'))[0] == 0


def test_interface_basis_accepted(lib):
    assert _ws_bytes(lib, _prob(basis='interface'))[0] == 0
    assert _ws_bytes(lib, _prob(system='burgers', basis='interface'))[0] == 0


def test_invalid_enum_values_rejected(lib):
    for field, val in (('system', 7), ('precision', 2), ('char_basis', 2), ('char_basis', -1)):
        p = _prob()
        setattr(p, field, val)
        assert _ws_bytes(lib, p)[0] == -1
    p = _prob()
    p.bc[0] = 5
    p.bc[1] = 5
    assert _ws_bytes(lib, p)[0] == -1


def test_null_arguments_rejected(lib):
    assert _ws_bytes(lib, None)[0] == -1
    p = _prob()
    assert lib.hweno_workspace_bytes(ctypes.byref(p), None) == -1
    # entry points validate before launching anything: null buffers -> EINVAL
    assert lib.hweno_rhs(ctypes.byref(p), *([None] * 11)) == -1
    assert lib.hweno_step(ctypes.byref(p), None, None, None, 0, 0.6, 0.0, 1.0,
                          None, None, None, None, None, None) == -1
    assert lib.hweno_max_wavespeed(ctypes.byref(p), None, None, None, None) == -1
    assert lib.hweno_workspace_init(ctypes.byref(p), None, None) == -1
    assert lib.hweno_health(ctypes.byref(p), None, None, 0) == -1


def test_1d_rejects_w_buffers(lib):
    p = _prob(dim=1, ny=1)
    fake = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    assert lib.hweno_rhs(ctypes.byref(p), fake, fake, fake, fake, fake, fake, None,
                         fake, None, fake, None) == -1


def test_status_strings(lib):
    for code, text in H.STATUS.items():
        assert lib.hweno_status_string(code).decode().startswith(text.split()[0])


def test_frozen_step_output_checks(lib):
    """hweno_step_frozen's out-of-place form rejects aliasing and partial
    output sets before launching anything (distinct fake addresses, never
    dereferenced)."""
    p = _prob()
    a = [ctypes.c_void_p(0x1000 * (k + 1)) for k in range(8)]
    u, v, w, dt, rec, ws = a[0], a[1], a[2], a[3], a[4], a[5]
    f = lib.hweno_step_frozen
    # output aliases an input
    assert f(ctypes.byref(p), u, v, w, u, a[6], a[7], dt, rec, None, ws, None) == -1
    assert f(ctypes.byref(p), u, v, w, a[6], a[7], v, dt, rec, None, ws, None) == -1
    # u_out without v_out / w_out, or v_out without u_out
    assert f(ctypes.byref(p), u, v, w, a[6], None, a[7], dt, rec, None, ws, None) == -1
    assert f(ctypes.byref(p), u, v, w, a[6], a[7], None, dt, rec, None, ws, None) == -1
    assert f(ctypes.byref(p), u, v, w, None, a[6], None, dt, rec, None, ws, None) == -1


def test_multi_step_and_strip_setting_validation(lib):
    """hweno_steps rejects a non-positive step count and null buffers before
    launching anything; hweno_set_strip_rows accepts 0 (automatic) and
    positive heights, rejects negative ones."""
    p = _prob()
    a = [ctypes.c_void_p(0x1000 * (k + 1)) for k in range(5)]
    u, v, w, t, ws = a
    f = lib.hweno_steps
    assert f(ctypes.byref(p), u, v, w, 0, 0, 0.6, 0.0, 1.0, t, None, None, ws, None, None) == -1
    assert f(ctypes.byref(p), u, v, w, -3, 0, 0.6, 0.0, 1.0, t, None, None, ws, None, None) == -1
    assert f(ctypes.byref(p), None, v, w, 4, 0, 0.6, 0.0, 1.0, t, None, None, ws, None, None) == -1
    assert f(ctypes.byref(p), u, v, w, 4, 0, 0.6, 0.0, 1.0, None, None, None, ws, None, None) == -1
    assert f(ctypes.byref(p), u, v, w, 4, 9, 0.6, 0.0, 1.0, t, None, None, ws, None, None) == -1
    assert lib.hweno_set_strip_rows(-1) == -1
    assert lib.hweno_set_strip_rows(7) == 0
    assert lib.hweno_set_strip_rows(0) == 0


def test_noalloc_step_rejects_problems_beyond_its_scratch(lib):
    """hweno_step_noalloc checks the problem against its 128 MiB static
    scratch before touching a device: 2D Euler FP64 at 724^2 fits (256 bytes
    per cell), 725^2 and 1024^2 do not (HWENO_ESCRATCH); FP32 (128 bytes per
    cell) fits at 1023^2, not at 2048^2.
    Fake addresses, never dereferenced."""
    a = [ctypes.c_void_p(0x1000 * (k + 1)) for k in range(6)]
    f = lambda p: lib.hweno_step_noalloc(ctypes.byref(p), a[0], a[1], a[2], 0, 0.6, 0.0, 1.0,
                                         a[3], None, None, None)
    for n in (725, 1024):
        assert f(_prob(nx=n, ny=n)) == -6
    assert f(_prob(nx=2048, ny=2048, precision='f32')) == -6
    # within the limit, null buffers are the first error found
    p = _prob(nx=724, ny=724)
    assert lib.hweno_step_noalloc(ctypes.byref(p), None, a[1], a[2], 0, 0.6, 0.0, 1.0, a[3],
                                  None, None, None) == -1
    p = _prob(nx=1023, ny=1023, precision='f32')
    assert lib.hweno_step_noalloc(ctypes.byref(p), a[0], a[1], a[2], 0, 0.6, 0.0, 1.0, None,
                                  None, None, None) == -1
