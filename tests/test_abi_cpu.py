"""C-ABI checks that need no GPU: the library loads, exports every entry point
that include/rlb.h declares, and rejects bad arguments before any device work.
"""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_1211_3286_amd as rlb
from workloads import Params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rlb.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rlb_[a-z_]+)\s*\(", txt)))


def test_header_entry_points_exported():
    L = rlb.lib()
    names = _declared()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert sorted(rlb.ENTRY_POINTS) == names


def test_status_strings():
    for code in range(-8, 1):
        s = rlb.status_string(code)
        assert s and s != "unknown status"
    assert rlb.status_string(-99) == "unknown status"


def _p(**kw):
    base = dict(nx=8, ny=4, nz=3, bc=(0, 0, 1), tau_f=0.8, tau_v=0.8, tau_e=0.6, tau_eps=0.7)
    base.update(kw)
    return Params(**base)


def _size(members, opt):
    n = ctypes.c_size_t(0)
    arr = rlb.cparams(members)
    code = rlb.lib().rlb_workspace_size(arr, len(members), ctypes.byref(opt), ctypes.byref(n))
    return code, n.value


def test_workspace_size_scales():
    c32, b32 = _size([_p()], rlb.options(rlb.FP32))
    c64, b64 = _size([_p()], rlb.options(rlb.FP64))
    assert c32 == 0 and c64 == 0 and 0 < b32 < b64
    c, big = _size([_p(nx=256, ny=256, nz=256)], rlb.options(rlb.FP32))
    assert c == 0
    assert big >= 2 * 38 * 4 * 256 ** 3  # two population buffers
    c, tape = _size([_p(nx=64, ny=64, nz=1)], rlb.options(rlb.FP32, 50, 1000))
    c2, notape = _size([_p(nx=64, ny=64, nz=1)], rlb.options(rlb.FP32))
    assert c == 0 and tape > notape + 21 * 19 * 4 * 64 * 64


def test_workspace_size_of_the_largest_cube():
    """512^3 FP32 (about 40.8 GB of double-buffered populations) is accepted."""
    c, b = _size([_p(nx=512, ny=512, nz=512, bc=(1, 1, 1))], rlb.options(rlb.FP32))
    assert c == 0 and b > 40.8e9


@pytest.mark.parametrize("prec,nz_ok", [(rlb.FP32, 1023), (rlb.FP64, 511)])
def test_workspace_size_at_the_32_bit_plane_limit(prec, nz_ok):
    """Population byte offsets within a plane are 32-bit in the kernels: the
    largest lattices whose plane (cells rounded up to 64, plus 64) stays
    below 4 GiB are accepted, one more z-plane is refused (RLB_E_UNSUPPORTED)."""
    c, b = _size([_p(nx=1024, ny=1024, nz=nz_ok)], rlb.options(prec))
    assert c == 0 and b > 2 * 38 * 1024 * 1024 * nz_ok * (4 if prec == rlb.FP32 else 8)
    c, _ = _size([_p(nx=1024, ny=1024, nz=nz_ok + 1)], rlb.options(prec))
    assert c == -7


@pytest.mark.parametrize("kw,code", [
    (dict(nx=0), -1), (dict(nz=-3), -1), (dict(bc=(0, 2, 0)), -1),
    (dict(tau_v=0.5), -2), (dict(tau_e=0.3), -2), (dict(tau_eps=float("nan")), -2),
    (dict(tau_f=float("inf")), -2), (dict(tau_q=0.4), -2), (dict(tau_q=float("nan")), -2),
    (dict(nx=2048, ny=2048, nz=1024), -7)])
def test_workspace_size_rejects(kw, code):
    assert _size([_p(**kw)], rlb.options(rlb.FP32))[0] == code


def test_workspace_size_rejects_bad_options():
    assert _size([_p()], rlb.options(precision=7))[0] == -1
    assert _size([_p()], rlb.options(ckpt_every=-1))[0] == -1
    assert _size([_p(), _p()], rlb.options(ckpt_every=10, tape_steps=100))[0] == -7
    L = rlb.lib()
    n = ctypes.c_size_t(0)
    opt = rlb.options()
    assert L.rlb_workspace_size(None, 1, ctypes.byref(opt), ctypes.byref(n)) == -1
    assert L.rlb_workspace_size(rlb.cparams([_p()]), 0, ctypes.byref(opt), ctypes.byref(n)) == -1
    assert L.rlb_workspace_size(rlb.cparams([_p()]), 1, None, ctypes.byref(n)) == -1
    assert L.rlb_workspace_size(rlb.cparams([_p()]), 1, ctypes.byref(opt), None) == -1


def _init(members, fields, ws_ptr, ws_bytes, opt=None):
    L = rlb.lib()
    h = ctypes.c_void_p(0)
    opt = opt or rlb.options()
    arr = rlb.cparams(members)
    n, e, u = fields
    code = L.rlb_init(ctypes.byref(h), arr, len(members), ctypes.byref(opt),
                      n.ctypes.data, e.ctypes.data, u.ctypes.data, 0, ws_ptr, ws_bytes, None)
    assert h.value is None
    return code


def _fields(nc, eps=1.0, n=1.0, u=(0.0, 0.0, 0.0)):
    uu = np.zeros((3, nc))
    for c in range(3):
        uu[c] = u[c]
    return np.full(nc, n), np.full(nc, eps), uu


def test_init_validates_before_device_work():
    """Every case returns an error before the library touches a device."""
    p = _p()
    nc = p.nx * p.ny * p.nz
    _, need = _size([p], rlb.options())
    fake = 1 << 40  # aligned address, never dereferenced on these paths
    good = _fields(nc)
    assert _init([_p(tau_v=0.2)], good, fake, need) == -2
    assert _init([p], good, 0, need) == -4
    assert _init([p], good, fake + 8, need) == -4
    assert _init([p], good, fake, need - 1) == -4
    assert _init([p], _fields(nc, eps=0.0), fake, need) == -3
    assert _init([p], _fields(nc, n=-1.0), fake, need) == -3
    assert _init([p], _fields(nc, u=(0.6, 0.6, 0.6)), fake, need) == -3
    assert _init([p], _fields(nc, eps=float("nan")), fake, need) == -3
    bad = _fields(nc)
    bad[2][1, 5] = 1.0
    assert _init([p], bad, fake, need) == -3


def test_null_handles():
    L = rlb.lib()
    assert L.rlb_step(None, 1) == -1
    assert L.rlb_moments(None, None, None, None, None, None, None, None, 0) == -1
    assert L.rlb_diagnostics(None, None, None, None) == -1
    assert L.rlb_populations(None, None, None, 0) == -1
    d = (ctypes.c_double * 3)()
    assert L.rlb_grad(None, None, None, d, None, None, 0) == -1
    assert L.rlb_tune(None, 1, None, None) == -1
    assert L.rlb_info(None, None, None, 0) == -1
    L.rlb_free(None)


def test_package_fails_loudly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError):
        rlb.Simulation([_p()], *_fields(96))


def test_d2q9_options_validated():
    """D2Q9 handles: nz = 1 only, no tape, 18 population planes per buffer."""
    d2 = rlb.options(rlb.FP32, lattice=rlb.D2Q9)
    assert _size([_p(nz=3)], d2)[0] == -1
    assert _size([_p(nx=4, ny=800, nz=1)], rlb.options(rlb.FP32, 50, 100, lattice=rlb.D2Q9))[0] == -7
    assert _size([_p()], rlb.options(lattice=2))[0] == -1
    c2, b2 = _size([_p(nx=4096, ny=4096, nz=1, bc=(0, 0, 0))], d2)
    c3, b3 = _size([_p(nx=4096, ny=4096, nz=1, bc=(0, 0, 0))], rlb.options(rlb.FP32))
    assert c2 == 0 and c3 == 0
    assert 2 * 18 * 4 * 4096 ** 2 <= b2 < b3 - 2 * 19 * 4 * 4096 ** 2
    assert rlb.lattice_code("d2q9") == rlb.D2Q9 and rlb.lattice_code("D3Q19") == rlb.D3Q19


def test_d2q9_init_rejects_out_of_plane_velocity():
    p = _p(nx=6, ny=5, nz=1, bc=(0, 1, 0))
    opt = rlb.options(rlb.FP32, lattice=rlb.D2Q9)
    _, need = _size([p], opt)
    fake = 1 << 40
    assert _init([p], _fields(30, u=(0.1, 0.0, 0.05)), fake, need, opt) == -3
    assert _init([_p(nx=6, ny=5, nz=2)], _fields(60), fake, need, opt) == -1


def test_correction_option_validated():
    d2 = dict(nx=4, ny=800, nz=1, bc=(0, 1, 0))
    assert _size([_p(**d2)], rlb.options(lattice=rlb.D2Q9, correction=1))[0] == 0
    assert _size([_p(**d2)], rlb.options(lattice=rlb.D2Q9, correction=2))[0] == -1
    assert _size([_p()], rlb.options(correction=1))[0] == -7


def test_equation_of_state_parameters_validated():
    assert _size([_p(eos_gamma=5 / 3, mass=0.5)], rlb.options())[0] == 0
    assert _size([_p(eos_gamma=2.5)], rlb.options())[0] == -1
    assert _size([_p(eos_gamma=1.0)], rlb.options())[0] == -1
    assert _size([_p(mass=-1.0)], rlb.options())[0] == -1
    assert _size([_p(eos_gamma=5 / 3)], rlb.options(rlb.FP32, 10, 100))[0] == -7
    d2 = dict(nx=4, ny=8, nz=1, bc=(0, 1, 0))
    assert _size([_p(mass=0.1, **d2)], rlb.options(lattice=rlb.D2Q9, correction=1))[0] == -7
    # every input cell needs eps > m n (checked on host fields before device work)
    p = _p(eos_gamma=5 / 3, mass=2.0)
    opt = rlb.options()
    _, need = _size([p], opt)
    assert _init([p], _fields(96, eps=1.0, n=1.0), 1 << 40, need, opt) == -3


def _noalloc(member, opt, nsteps=1, fields=True):
    """rlb_run_noalloc with placeholder field pointers: every case here is
    rejected before the library touches them or the device."""
    arr = rlb.cparams([member])
    dummy = ctypes.c_void_p(0x1000) if fields else None
    bad = ctypes.c_int64(-1)
    return rlb.lib().rlb_run_noalloc(arr, ctypes.byref(opt), dummy, dummy, dummy, nsteps, None,
                                     None, None, None, None, None, ctypes.byref(bad), None)


def test_noalloc_rejects_before_device_work():
    """The allocation-free run checks what rlb_init checks, and refuses a
    lattice whose state does not fit its fixed scratch array
    (RLB_NOALLOC_SCRATCH_BYTES) with RLB_E_SCRATCH."""
    ok = _p()
    assert _noalloc(ok, rlb.options(rlb.FP32), fields=False) == -1
    assert _noalloc(ok, rlb.options(rlb.FP32), nsteps=-1) == -1
    assert _noalloc(_p(tau_v=0.5), rlb.options(rlb.FP32)) == -2
    assert _noalloc(_p(nx=0), rlb.options(rlb.FP32)) == -1
    assert _noalloc(ok, rlb.options(rlb.FP32, ckpt_every=5, tape_steps=10)) == -7
    assert _noalloc(ok, rlb.options(rlb.FP32, correction=1)) == -7
    # 64^3 FP64: 2 buffers x 38 planes x 8 B x 262,144 cells = 159 MB > 64 MiB
    assert _noalloc(_p(nx=64, ny=64, nz=64), rlb.options(rlb.FP64)) == -8
    # FP32: 61^3 (226,981 cells x 304 B = 69 MB) exceeds it as well
    assert _noalloc(_p(nx=61, ny=61, nz=61), rlb.options(rlb.FP32)) == -8
    assert rlb.status_string(-8).startswith("lattice too large")
