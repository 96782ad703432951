"""MI355X (gfx950) relativistic MRT lattice Boltzmann step - Python binding.

Thin ctypes marshalling over ``librlb.so`` (the C ABI of ``include/rlb.h``):
every step of the method runs in the HIP kernels of that library. PyTorch is
used only for device memory (the workspace and field tensors) and for the
HIP stream the library enqueues on. There is no CPU fallback: without the
built library or a GPU, constructing a :class:`Simulation` raises.

Layout conventions (same as the C ABI): a lattice of nx*ny*nz cells is
C-ordered ``(nz, ny, nx)``; velocities are ``(3, nz, ny, nx)``; a batch of
members is packed member after member along one flat cell axis. Two lattice
models: D3Q19 (default) and the D2Q9 MRT model of Sec. V.A
(``lattice=D2Q9``, nx x ny x 1 lattices with u_z = 0).
"""

from __future__ import annotations

import ctypes
import json
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librlb.so")

RLB_OK = 0
STATUS = {0: "RLB_OK", -1: "RLB_E_ARG", -2: "RLB_E_TAU", -3: "RLB_E_UNPHYSICAL",
          -4: "RLB_E_WORKSPACE", -5: "RLB_E_DEVICE", -6: "RLB_E_STATE", -7: "RLB_E_UNSUPPORTED",
          -8: "RLB_E_SCRATCH"}
NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024  # RLB_NOALLOC_SCRATCH_BYTES
FP64, FP32 = 0, 1
PERIODIC, ZERO_GRADIENT = 0, 1
D3Q19, D2Q9 = 0, 1
LATTICE_NAMES = {"d3q19": D3Q19, "d2q9": D2Q9}

# Entry points declared in include/rlb.h (checked against the header by the tests).
ENTRY_POINTS = ["rlb_workspace_size", "rlb_init", "rlb_step", "rlb_moments", "rlb_diagnostics",
                "rlb_populations", "rlb_grad", "rlb_num_variants", "rlb_variant_name",
                "rlb_set_variant", "rlb_get_variant", "rlb_tune", "rlb_info", "rlb_free",
                "rlb_status_string", "rlb_run_noalloc"]


class RLBError(RuntimeError):
    def __init__(self, code: int, call: str):
        self.code = code
        super().__init__(f"{call} failed: {STATUS.get(code, code)} ({status_string(code)})")


class CParams(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("bc", ctypes.c_int32 * 3), ("tau_f", ctypes.c_double),
                ("tau_v", ctypes.c_double), ("tau_e", ctypes.c_double),
                ("tau_eps", ctypes.c_double), ("tau_q", ctypes.c_double),
                ("eta_over_s", ctypes.c_double), ("kappa", ctypes.c_double),
                ("dof", ctypes.c_double), ("a_f", ctypes.c_double), ("a_e", ctypes.c_double),
                ("a_eps", ctypes.c_double), ("a_q", ctypes.c_double),
                ("eos_gamma", ctypes.c_double), ("mass", ctypes.c_double)]


class COptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("ckpt_every", ctypes.c_int32),
                ("tape_steps", ctypes.c_int32), ("diag_every", ctypes.c_int32),
                ("lattice", ctypes.c_int32), ("correction", ctypes.c_int32)]


_lib = None


def build_library() -> str:
    """Compile librlb.so for gfx950 (hipcc)."""
    import importlib
    return importlib.import_module("paper_1211_3286_amd.build").build()


def lib() -> ctypes.CDLL:
    """The loaded library (built first if it is not there)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build_library()
    L = ctypes.CDLL(LIB_PATH)
    vp, sz, i32, i64, dp = (ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64,
                            ctypes.POINTER(ctypes.c_double))
    P = ctypes.POINTER(CParams)
    O = ctypes.POINTER(COptions)
    H = ctypes.POINTER(ctypes.c_void_p)
    L.rlb_workspace_size.argtypes = [P, i32, O, ctypes.POINTER(sz)]
    L.rlb_init.argtypes = [H, P, i32, O, vp, vp, vp, i32, vp, sz, vp]
    L.rlb_step.argtypes = [vp, i32]
    L.rlb_moments.argtypes = [vp, vp, vp, vp, vp, vp, dp, ctypes.POINTER(i64), i32]
    L.rlb_diagnostics.argtypes = [vp, dp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.rlb_populations.argtypes = [vp, vp, vp, i32]
    L.rlb_grad.argtypes = [vp, vp, vp, dp, vp, vp, i32]
    L.rlb_num_variants.argtypes = [vp, ctypes.POINTER(i32)]
    L.rlb_variant_name.argtypes = [vp, i32, ctypes.c_char_p, sz]
    L.rlb_set_variant.argtypes = [vp, i32]
    L.rlb_get_variant.argtypes = [vp, ctypes.POINTER(i32)]
    L.rlb_tune.argtypes = [vp, i32, ctypes.POINTER(i32), dp]
    L.rlb_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.c_char_p, sz]
    L.rlb_free.argtypes = [vp]
    L.rlb_free.restype = None
    L.rlb_run_noalloc.argtypes = [P, O, vp, vp, vp, i32, vp, vp, vp, vp, vp, dp,
                                  ctypes.POINTER(i64), vp]
    L.rlb_status_string.argtypes = [i32]
    L.rlb_status_string.restype = ctypes.c_char_p
    for name in ENTRY_POINTS:
        if name not in ("rlb_free", "rlb_status_string"):
            getattr(L, name).restype = i32
    _lib = L
    return L


def status_string(code: int) -> str:
    return lib().rlb_status_string(int(code)).decode()


def _check(code: int, call: str) -> None:
    if code != RLB_OK:
        raise RLBError(code, call)


def cparams(members: Sequence) -> ctypes.Array:
    arr = (CParams * len(members))()
    for i, p in enumerate(members):
        c = arr[i]
        c.nx, c.ny, c.nz = int(p.nx), int(p.ny), int(p.nz)
        for k in range(3):
            c.bc[k] = int(p.bc[k])
        c.tau_f, c.tau_v, c.tau_e = float(p.tau_f), float(p.tau_v), float(p.tau_e)
        c.tau_eps, c.tau_q = float(p.tau_eps), float(getattr(p, "tau_q", 0.0))
        c.eta_over_s = float(getattr(p, "eta_s", 0.0))
        c.kappa = float(getattr(p, "kappa", 1.0))
        c.dof = float(getattr(p, "dof", 16.0))
        for k in ("a_f", "a_e", "a_eps", "a_q", "eos_gamma", "mass"):
            setattr(c, k, float(getattr(p, k, 0.0)))
    return arr


def lattice_code(lattice) -> int:
    """D3Q19 / D2Q9 from an int or a name ("d3q19", "d2q9")."""
    if isinstance(lattice, str):
        return LATTICE_NAMES[lattice.lower()]
    return int(lattice)


def options(precision: int = FP32, ckpt_every: int = 0, tape_steps: int = 0,
            diag_every: int = 0, lattice=D3Q19, correction: int = 0) -> COptions:
    return COptions(int(precision), int(ckpt_every), int(tape_steps), int(diag_every),
                    lattice_code(lattice), int(correction))


def workspace_size(members: Sequence, opt: COptions) -> int:
    n = ctypes.c_size_t(0)
    arr = cparams(members)
    _check(lib().rlb_workspace_size(arr, len(members), ctypes.byref(opt), ctypes.byref(n)),
           "rlb_workspace_size")
    return int(n.value)


def _dptr(t) -> int:
    return int(t.data_ptr())


class Simulation:
    """One handle of the C ABI: a lattice, or a batch of lattices.

    ``fields``: (n0, eps0, u0) as float64 torch tensors on the GPU (or numpy
    arrays, copied once). For a batch, pass flat per-member concatenations.
    ``lattice``: D3Q19 (default) or D2Q9 (or their names). ``correction``:
    1 adds the correction term of Eqs. (37)-(38) (D2Q9 only).
    """

    def __init__(self, members: Sequence, n0, eps0, u0, precision: int = FP32,
                 ckpt_every: int = 0, tape_steps: int = 0, diag_every: int = 0,
                 stream=None, device: Optional[int] = None, lattice=D3Q19,
                 correction: int = 0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("paper_1211_3286_amd needs a ROCm GPU; none is visible")
        self.torch = torch
        self.members = list(members)
        self.precision = precision
        self.ncells = sum(int(p.nx) * int(p.ny) * int(p.nz) for p in self.members)
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.device = dev
        self.lattice = lattice_code(lattice)
        self.q = 9 if self.lattice == D2Q9 else 19
        self.opt = options(precision, ckpt_every, tape_steps, diag_every, self.lattice,
                           correction)
        self._arr = cparams(self.members)
        self.ws_bytes = workspace_size(self.members, self.opt)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=dev)
        base = _dptr(self.workspace)
        self._ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        nc = self.ncells

        def dev_field(a, shape):
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
            t = t.to(device=dev, dtype=torch.float64).contiguous().reshape(shape)
            return t

        n_t = dev_field(n0, (nc,))
        e_t = dev_field(eps0, (nc,))
        u_t = dev_field(u0, (3, nc))
        h = ctypes.c_void_p(0)
        with torch.cuda.device(dev):
            code = lib().rlb_init(ctypes.byref(h), self._arr, len(self.members),
                                  ctypes.byref(self.opt), _dptr(n_t), _dptr(e_t), _dptr(u_t), 1,
                                  self._ws_ptr, self.ws_bytes, int(self.stream.cuda_stream))
        _check(code, "rlb_init")
        self.h = h

    # -- lifetime --------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "h", None) and self.h.value:
            lib().rlb_free(self.h)
            self.h = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- stepping --------------------------------------------------------
    def step(self, nsteps: int = 1) -> None:
        _check(lib().rlb_step(self.h, int(nsteps)), "rlb_step")

    @property
    def steps(self) -> int:
        s = ctypes.c_int64(0)
        _check(lib().rlb_info(self.h, ctypes.byref(s), None, 0), "rlb_info")
        return int(s.value)

    @property
    def kernel_name(self) -> str:
        buf = ctypes.create_string_buffer(128)
        _check(lib().rlb_info(self.h, None, buf, 128), "rlb_info")
        return buf.value.decode()

    # -- outputs ---------------------------------------------------------
    def moments(self, allow_unphysical: bool = False) -> Dict:
        """Fields as float64 device tensors, FP64 lattice sums, inadmissible count."""
        torch = self.torch
        nc = self.ncells
        out = {k: torch.empty(nc, dtype=torch.float64, device=self.device)
               for k in ("n", "eps", "P", "gamma")}
        out["u"] = torch.empty(3, nc, dtype=torch.float64, device=self.device)
        sums = (ctypes.c_double * 5)()
        bad = ctypes.c_int64(0)
        code = lib().rlb_moments(self.h, _dptr(out["n"]), _dptr(out["eps"]), _dptr(out["P"]),
                                 _dptr(out["gamma"]), _dptr(out["u"]), sums, ctypes.byref(bad),
                                 1)
        if code != RLB_OK and not (allow_unphysical and code == -3):
            _check(code, "rlb_moments")
        out["sums"] = np.array(sums[:])
        out["bad"] = int(bad.value)
        return out

    def sums(self) -> np.ndarray:
        s = (ctypes.c_double * 5)()
        bad = ctypes.c_int64(0)
        code = lib().rlb_moments(self.h, None, None, None, None, None, s, ctypes.byref(bad), 1)
        if code not in (RLB_OK, -3):
            _check(code, "rlb_moments")
        return np.array(s[:])

    def diagnostics(self):
        s = (ctypes.c_double * 5)()
        st = ctypes.c_int64(0)
        bad = ctypes.c_int64(0)
        _check(lib().rlb_diagnostics(self.h, s, ctypes.byref(st), ctypes.byref(bad)),
               "rlb_diagnostics")
        return np.array(s[:]), int(st.value), int(bad.value)

    def populations(self):
        """(f, g) as float64 device tensors of shape (Q, ncells), Q = 19 or 9."""
        torch = self.torch
        f = torch.empty(self.q, self.ncells, dtype=torch.float64, device=self.device)
        g = torch.empty(self.q, self.ncells, dtype=torch.float64, device=self.device)
        _check(lib().rlb_populations(self.h, _dptr(f), _dptr(g), 1), "rlb_populations")
        return f, g

    def grad(self, dL_du, dL_deps):
        """(dL/dtau[3] numpy, dL/deps0 (ncells,), dL/du0 (3, ncells)) as device tensors."""
        torch = self.torch
        nc = self.ncells
        du = dL_du.to(device=self.device, dtype=torch.float64).contiguous()
        de = dL_deps.to(device=self.device, dtype=torch.float64).contiguous()
        dtau = (ctypes.c_double * 3)()
        de0 = torch.empty(nc, dtype=torch.float64, device=self.device)
        du0 = torch.empty(3, nc, dtype=torch.float64, device=self.device)
        _check(lib().rlb_grad(self.h, _dptr(du), _dptr(de), dtau, _dptr(de0), _dptr(du0), 1),
               "rlb_grad")
        return np.array(dtau[:]), de0, du0

    # -- variants and tuning ----------------------------------------------
    def variants(self) -> List[str]:
        n = ctypes.c_int32(0)
        _check(lib().rlb_num_variants(self.h, ctypes.byref(n)), "rlb_num_variants")
        out = []
        for v in range(n.value):
            buf = ctypes.create_string_buffer(128)
            _check(lib().rlb_variant_name(self.h, v, buf, 128), "rlb_variant_name")
            out.append(buf.value.decode())
        return out

    @property
    def variant(self) -> int:
        v = ctypes.c_int32(0)
        _check(lib().rlb_get_variant(self.h, ctypes.byref(v)), "rlb_get_variant")
        return int(v.value)

    @variant.setter
    def variant(self, v: int) -> None:
        _check(lib().rlb_set_variant(self.h, int(v)), "rlb_set_variant")

    def tune(self, trial_steps: int = 5, cache: Optional[str] = None, key: Optional[str] = None):
        """Time every kernel variant (the native autotuner) and keep the fastest.

        With ``cache`` (a JSON file path), a previous choice for ``key`` is
        reused instead of timing again, and new results are stored.
        """
        key = key or self.tune_key()
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                db = json.load(fh)
            if key in db:
                self.variant = int(db[key]["variant"])
                return db[key]
        names = self.variants()
        ms = (ctypes.c_double * len(names))()
        best = ctypes.c_int32(0)
        _check(lib().rlb_tune(self.h, int(trial_steps), ctypes.byref(best), ms), "rlb_tune")
        res = {"variant": int(best.value), "name": names[best.value],
               "ms_per_step": dict(zip(names, [float(x) for x in ms]))}
        if cache:
            db = {}
            if os.path.exists(cache):
                with open(cache) as fh:
                    db = json.load(fh)
            db[key] = res
            with open(cache, "w") as fh:
                json.dump(db, fh, indent=1, sort_keys=True)
        return res

    def tune_key(self) -> str:
        torch = self.torch
        dev = torch.cuda.get_device_name(self.device)
        shapes = [(int(p.nx), int(p.ny), int(p.nz)) for p in self.members]
        shape = shapes[0] if len(shapes) == 1 else f"{len(shapes)}x{self.ncells}"
        lat = ("d2q9|" if self.lattice == D2Q9 else "") + ("c7|" if self.opt.correction else "")
        return f"{dev}|{lat}{'fp32' if self.precision == FP32 else 'fp64'}|{shape}"


def run_noalloc(params, n0, eps0, u0, nsteps: int, precision: int = FP32, lattice=D3Q19,
                correction: int = 0, stream=None, allow_unphysical: bool = False) -> Dict:
    """rlb_run_noalloc: rlb_init + rlb_step(nsteps) + rlb_moments on one
    lattice with no allocation in the library (its fixed scratch array holds
    the state). Fields are float64 device tensors; returns the rlb_moments
    outputs as Simulation.moments does."""
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("paper_1211_3286_amd needs a ROCm GPU; none is visible")
    dev = torch.device("cuda", torch.cuda.current_device())
    nc = int(params.nx) * int(params.ny) * int(params.nz)
    fields = [t.to(device=dev, dtype=torch.float64).contiguous() for t in (n0, eps0, u0)]
    out = {k: torch.empty(nc, dtype=torch.float64, device=dev) for k in ("n", "eps", "P", "gamma")}
    out["u"] = torch.empty(3, nc, dtype=torch.float64, device=dev)
    opt = options(precision, 0, 0, 0, lattice, correction)
    arr = cparams([params])
    sums = (ctypes.c_double * 5)()
    bad = ctypes.c_int64(0)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    code = lib().rlb_run_noalloc(arr, ctypes.byref(opt), *[_dptr(t) for t in fields], int(nsteps),
                                 _dptr(out["n"]), _dptr(out["eps"]), _dptr(out["P"]),
                                 _dptr(out["gamma"]), _dptr(out["u"]), sums, ctypes.byref(bad),
                                 int(st.cuda_stream))
    if code != RLB_OK and not (allow_unphysical and code == -3 and bad.value > 0):
        _check(code, "rlb_run_noalloc")
    out["sums"] = np.array(sums[:])
    out["bad"] = int(bad.value)
    return out


def problem_fields(problems) -> tuple:
    """Concatenate the (n, eps, u) fields of one or more workload problems."""
    if not isinstance(problems, (list, tuple)):
        problems = [problems]
    n = np.concatenate([p.n.ravel() for p in problems])
    e = np.concatenate([p.eps.ravel() for p in problems])
    u = np.concatenate([p.u.reshape(3, -1) for p in problems], axis=1)
    return n, e, u


def from_problems(problems, **kw) -> Simulation:
    """A Simulation of one problem or a batch of them (workloads.Problem)."""
    if not isinstance(problems, (list, tuple)):
        problems = [problems]
    lats = {getattr(p.params, "lattice", "d3q19") for p in problems}
    if len(lats) != 1:
        raise ValueError("every member of a batch uses the same lattice model")
    kw.setdefault("lattice", lats.pop())
    corr = {int(getattr(p.params, "correction", 0)) for p in problems}
    if len(corr) != 1:
        raise ValueError("every member of a batch uses the same correction setting")
    kw.setdefault("correction", corr.pop())
    n, e, u = problem_fields(problems)
    return Simulation([p.params for p in problems], n, e, u, **kw)


from paper_1211_3286_amd.autograd import RLBStep  # noqa: E402  (needs Simulation)
