"""ctypes binding of include/fdtd_rom.h: same names, argument marshalling only.

The shared library is built in-tree by ``paper_1609_07114_amd.build``.  If
it is missing, ``lib()`` raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# FDTD_ROM_LIB names another build of the same library (the sanitizer build
# of the host code that tests/test_host_sanitizers.py makes)
LIB_PATH = os.environ.get("FDTD_ROM_LIB") or os.path.join(HERE, "libfdtdrom.so")

FDTD_OK, FDTD_EINVAL, FDTD_ENOMEM, FDTD_EDEVICE = 0, -1, -2, -3
FDTD_ENOTPASSIVE, FDTD_EUNSTABLE, FDTD_ESTATE = -4, -5, -6
FDTD_F32, FDTD_F64 = 0, 1
FDTD_HZ, FDTD_EX, FDTD_EY = 0, 1, 2

_dp = C.POINTER(C.c_double)


_u8p = C.POINTER(C.c_uint8)


class fdtd_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("dx", C.c_double), ("dy", C.c_double),
                ("dt", C.c_double), ("dtype", C.c_int32), ("eps_r", _dp), ("sigma", _dp),
                ("pec", _u8p), ("pitch_pad", C.c_int32)]


class fdtd_rom(C.Structure):
    _fields_ = [("i0", C.c_int32), ("j0", C.c_int32), ("ni", C.c_int32), ("nj", C.c_int32),
                ("q", C.c_int32), ("group", C.c_int32), ("Rt", _dp), ("Ft", _dp), ("Lt", _dp),
                ("x0", _dp)]


class fdtd_source(C.Structure):
    _fields_ = [("comp", C.c_int32), ("i0", C.c_int32), ("i1", C.c_int32), ("j0", C.c_int32),
                ("j1", C.c_int32), ("nt", C.c_int32), ("incr", _dp)]


class fdtd_probe(C.Structure):
    _fields_ = [("comp", C.c_int32), ("i", C.c_int32), ("j", C.c_int32)]


class fdtd_pml(C.Structure):
    _fields_ = [("n_xlo", C.c_int32), ("n_xhi", C.c_int32), ("n_ylo", C.c_int32),
                ("n_yhi", C.c_int32), ("m", C.c_double), ("sigma_scale", C.c_double),
                ("kappa_max", C.c_double), ("alpha_max", C.c_double)]


class fdtd_problem(C.Structure):
    _fields_ = [("grid", fdtd_grid), ("roms", C.POINTER(fdtd_rom)), ("nroms", C.c_int32),
                ("sources", C.POINTER(fdtd_source)), ("nsources", C.c_int32),
                ("probes", C.POINTER(fdtd_probe)), ("nprobes", C.c_int32),
                ("max_steps", C.c_int32), ("pml", fdtd_pml)]


class fdtd_rom_build_params(C.Structure):
    _fields_ = [("ni", C.c_int32), ("nj", C.c_int32), ("r", C.c_int32), ("dx", C.c_double),
                ("dy", C.c_double), ("dt", C.c_double), ("eps_r", _dp), ("sigma", _dp),
                ("q", C.c_int32), ("f_max", C.c_double), ("theta", C.c_double),
                ("clip", C.c_int32), ("basis", C.c_int32), ("pec", _u8p)]


class fdtd_rom_build_info(C.Structure):
    _fields_ = [("q1", C.c_int32), ("q2", C.c_int32), ("p0", C.c_double),
                ("smax_before", C.c_double), ("smax_after", C.c_double),
                ("clipped", C.c_int32), ("n_fine_states", C.c_int32)]


class FdtdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_LIB = None

# name -> (restype, argtypes)
_SIGS = {
    "fdtd_rom_workspace_size": (C.c_int, [C.POINTER(fdtd_problem), C.POINTER(C.c_size_t)]),
    "fdtd_rom_create": (C.c_int, [C.POINTER(fdtd_problem), C.c_void_p, C.c_size_t, C.c_void_p,
                                  C.POINTER(C.c_void_p)]),
    "fdtd_rom_step": (C.c_int, [C.c_void_p]),
    "fdtd_rom_run": (C.c_int, [C.c_void_p, C.c_int32]),
    "fdtd_rom_prepare_run": (C.c_int, [C.c_void_p, C.c_int32]),
    "fdtd_rom_set_check_interval": (C.c_int, [C.c_void_p, C.c_int32]),
    "fdtd_rom_get_check_interval": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "fdtd_rom_steps_done": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "fdtd_rom_read_probes": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _dp]),
    "fdtd_rom_read_field": (C.c_int, [C.c_void_p, C.c_int32, _dp]),
    "fdtd_rom_probe_objective": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, _dp]),
    "fdtd_rom_read_rom_state": (C.c_int, [C.c_void_p, C.c_int32, _dp]),
    "fdtd_rom_coupled_update": (C.c_int, [C.POINTER(fdtd_problem), C.c_int32, _dp, _dp, _dp]),
    "fdtd_rom_build": (C.c_int, [C.POINTER(fdtd_rom_build_params), _dp, _dp, _dp,
                                 C.POINTER(fdtd_rom_build_info)]),
    "fdtd_rom_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "fdtd_rom_profile_read": (C.c_int, [C.c_void_p, _dp, C.POINTER(C.c_int64), _dp,
                                        C.POINTER(C.c_int64)]),
    "fdtd_rom_set_tiling": (C.c_int, [C.c_void_p, C.c_int32]),
    "fdtd_rom_set_graph": (C.c_int, [C.c_void_p, C.c_int32]),
    "fdtd_rom_get_tiling": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "fdtd_rom_set_shared_gemm": (C.c_int, [C.c_void_p, C.c_int32]),
    "fdtd_rom_set_material_mode": (C.c_int, [C.c_void_p, C.c_int32]),
    "fdtd_rom_get_material_mode": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "fdtd_rom_set_time_blocking": (C.c_int, [C.c_void_p, C.c_int32]),
    "fdtd_rom_set_pair_split": (C.c_int, [C.c_void_p, C.c_int32]),
    "fdtd_rom_get_pair_split": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "fdtd_rom_batch_set_time_blocking": (C.c_int, [C.c_void_p, C.c_int32]),
    "fdtd_rom_batch_set_pair_split": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "fdtd_rom_batch_get_time_blocking": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fdtd_rom_get_time_blocking": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fdtd_rom_adjoint_workspace_size": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32,
                                                  C.POINTER(C.c_size_t)]),
    "fdtd_rom_adjoint": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                   C.c_size_t, _dp, _dp, _dp]),
    "fdtd_rom_adjoint_plan": (C.c_int, [C.POINTER(fdtd_problem), C.c_int32, C.c_int32,
                                        C.POINTER(C.c_size_t)]),
    "fdtd_rom_adjoint_noalloc": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, _dp, _dp, _dp]),
    "fdtd_rom_adjoint_models_workspace_size": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32,
                                                         C.POINTER(C.c_size_t)]),
    "fdtd_rom_adjoint_models": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                          C.c_size_t, _dp, _dp, _dp, C.POINTER(_dp), C.POINTER(_dp),
                                          C.POINTER(_dp)]),
    "fdtd_rom_build_vjp": (C.c_int, [C.POINTER(fdtd_rom_build_params), _dp, _dp, _dp, _dp]),
    "fdtd_rom_build_keep": (C.c_int, [C.POINTER(fdtd_rom_build_params), _dp, _dp, _dp,
                                      C.POINTER(fdtd_rom_build_info), C.POINTER(C.c_void_p)]),
    "fdtd_rom_model_state_vjp": (C.c_int, [C.c_void_p, _dp, _dp, _dp, _dp]),
    "fdtd_rom_model_state_free": (None, [C.c_void_p]),
    "fdtd_rom_energy": (C.c_int, [C.c_void_p, _dp]),
    "fdtd_rom_state_size": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "fdtd_rom_get_state": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fdtd_rom_set_state": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fdtd_rom_batch_workspace_size": (C.c_int, [C.POINTER(fdtd_problem), C.c_int32,
                                                C.POINTER(C.c_size_t)]),
    "fdtd_rom_batch_create": (C.c_int, [C.POINTER(fdtd_problem), C.c_int32, C.c_void_p, C.c_size_t,
                                        C.c_void_p, C.POINTER(C.c_void_p)]),
    "fdtd_rom_batch_run": (C.c_int, [C.c_void_p, C.c_int32]),
    "fdtd_rom_batch_steps_done": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32)]),
    "fdtd_rom_batch_read_probes": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, _dp]),
    "fdtd_rom_batch_read_field": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, _dp]),
    "fdtd_rom_batch_set_tiling": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    "fdtd_rom_batch_set_graph": (C.c_int, [C.c_void_p, C.c_int32]),
    "fdtd_rom_batch_destroy": (None, [C.c_void_p]),
    "fdtd_rom_destroy": (None, [C.c_void_p]),
    "fdtd_rom_strerror": (C.c_char_p, [C.c_int]),
    "fdtd_rom_last_error": (C.c_char_p, []),
}


def lib():
    """Load the in-tree HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: run paper_1609_07114_amd.build.build() "
                               "(hipcc, gfx950) first; there is no CPU fallback")
        # PyTorch-ROCm carries its own HIP runtime, loaded under the soname
        # libamdhip64.so.7 that this library links against.  Importing torch
        # first makes the dynamic loader bind this library to that one
        # runtime; loading the library first would put a second HIP runtime
        # in the process, and device pointers from torch would be foreign to it.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _LIB = L
    return _LIB


def exported_symbols():
    return list(_SIGS)


def _check(rc):
    if rc != FDTD_OK:
        msg = lib().fdtd_rom_last_error().decode()
        raise FdtdError(rc, msg)
    return rc


def _ptr(a):
    return a.ctypes.data_as(_dp) if a is not None else None


def _mask(m, keep, shape):
    """A boolean map as a contiguous uint8 array (kept alive in ``keep``)."""
    if m is None:
        return None
    a = np.ascontiguousarray(np.asarray(m, dtype=bool).astype(np.uint8))
    assert a.shape == shape, (a.shape, shape)
    keep.append(a)
    return a.ctypes.data_as(_u8p)


# ---------------------------------------------------------------------------
# marshalling of a problem description
# ---------------------------------------------------------------------------

class ProblemStruct:
    """Owns the C structs and the contiguous float64 arrays they point to."""

    def __init__(self, nx, ny, dx, dy, dt, dtype, eps_r, sigma, roms, sources, probes,
                 max_steps, pml=None, pec=None, pitch_pad=0):
        self._keep = []

        def arr(x):
            if x is None:
                return None
            a = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
            self._keep.append(a)
            return a
        g = fdtd_grid(nx, ny, dx, dy, dt, FDTD_F64 if dtype in ("f64", FDTD_F64) else FDTD_F32,
                      _ptr(arr(eps_r)), _ptr(arr(sigma)), _mask(pec, self._keep, (ny, nx)), int(pitch_pad))
        rarr = (fdtd_rom * max(1, len(roms)))()
        for k, r in enumerate(roms):
            Rt, Ft, Lt = arr(r["Rt"]), arr(r["Ft"]), arr(r["Lt"])
            x0 = arr(r.get("x0"))
            rarr[k] = fdtd_rom(r["i0"], r["j0"], r["ni"], r["nj"], Rt.shape[0], r.get("group", -1),
                               _ptr(Rt), _ptr(Ft), _ptr(Lt), _ptr(x0))
        sarr = (fdtd_source * max(1, len(sources)))()
        for k, s in enumerate(sources):
            inc = arr(s["incr"])
            sarr[k] = fdtd_source(s["comp"], s["i0"], s["i1"], s["j0"], s["j1"], inc.size, _ptr(inc))
        parr = (fdtd_probe * max(1, len(probes)))()
        for k, p in enumerate(probes):
            parr[k] = fdtd_probe(p["comp"], p["i"], p["j"])
        self._keep += [rarr, sarr, parr]
        pm = fdtd_pml(0, 0, 0, 0, 0.0, 0.0, 0.0, 0.0)
        if pml is not None:
            pm = fdtd_pml(pml.n_xlo, pml.n_xhi, pml.n_ylo, pml.n_yhi, pml.m, pml.sigma_scale,
                          pml.kappa_max, pml.alpha_max)
        self.s = fdtd_problem(g, rarr, len(roms), sarr, len(sources), parr, len(probes), max_steps,
                              pm)

    @classmethod
    def from_workload(cls, prob, rom_mats, max_steps=None, dtype=None, x0=None):
        roms = []
        for k, (spec, m) in enumerate(zip(prob.roms, rom_mats)):
            roms.append(dict(i0=spec.i0, j0=spec.j0, ni=spec.ni, nj=spec.nj,
                             group=spec.group, Rt=m["Rt"], Ft=m["Ft"], Lt=m["Lt"],
                             x0=None if x0 is None else x0[k]))
        srcs = [dict(comp=s.comp, i0=s.i0, i1=s.i1, j0=s.j0, j1=s.j1, incr=s.incr)
                for s in prob.sources]
        prbs = [dict(comp=p.comp, i=p.i, j=p.j) for p in prob.probes]
        ms = prob.nsteps if max_steps is None else max_steps
        return cls(prob.nx, prob.ny, prob.dx, prob.dy, prob.dt, dtype or prob.dtype, prob.eps_r,
                   prob.sigma, roms, srcs, prbs, ms, getattr(prob, "pml", None),
                   getattr(prob, "pec", None), getattr(prob, "pitch_pad", 0))


# ---------------------------------------------------------------------------
# the C entry points, same names
# ---------------------------------------------------------------------------

def fdtd_rom_workspace_size(problem: ProblemStruct) -> int:
    n = C.c_size_t(0)
    _check(lib().fdtd_rom_workspace_size(C.byref(problem.s), C.byref(n)))
    return int(n.value)


def fdtd_rom_create(problem: ProblemStruct, dev_ptr: int, nbytes: int, stream: int):
    h = C.c_void_p()
    _check(lib().fdtd_rom_create(C.byref(problem.s), C.c_void_p(dev_ptr), nbytes,
                                 C.c_void_p(stream), C.byref(h)))
    return h


def fdtd_rom_step(h):
    _check(lib().fdtd_rom_step(h))


def fdtd_rom_run(h, nsteps: int):
    _check(lib().fdtd_rom_run(h, int(nsteps)))


def fdtd_rom_prepare_run(h, nsteps: int):
    _check(lib().fdtd_rom_prepare_run(h, int(nsteps)))


def fdtd_rom_set_check_interval(h, every: int):
    _check(lib().fdtd_rom_set_check_interval(h, int(every)))


def fdtd_rom_get_check_interval(h) -> int:
    n = C.c_int32(0)
    _check(lib().fdtd_rom_get_check_interval(h, C.byref(n)))
    return int(n.value)


def fdtd_rom_steps_done(h) -> int:
    n = C.c_int32(0)
    _check(lib().fdtd_rom_steps_done(h, C.byref(n)))
    return int(n.value)


def fdtd_rom_read_probes(h, first: int, count: int, nprobes: int) -> np.ndarray:
    out = np.zeros((count, nprobes), dtype=np.float64)
    _check(lib().fdtd_rom_read_probes(h, first, count, _ptr(out)))
    return out


def fdtd_rom_probe_objective(h, probe: int, first: int, count: int) -> float:
    J = C.c_double(0.0)
    _check(lib().fdtd_rom_probe_objective(h, probe, first, count, C.byref(J)))
    return float(J.value)


def fdtd_rom_read_field(h, comp: int, nx: int, ny: int) -> np.ndarray:
    shape = {FDTD_HZ: (ny, nx), FDTD_EX: (ny + 1, nx), FDTD_EY: (ny, nx + 1)}[comp]
    out = np.zeros(shape, dtype=np.float64)
    _check(lib().fdtd_rom_read_field(h, comp, _ptr(out)))
    return out


def fdtd_rom_read_rom_state(h, k: int, q: int) -> np.ndarray:
    out = np.zeros(q, dtype=np.float64)
    _check(lib().fdtd_rom_read_rom_state(h, k, _ptr(out)))
    return out


def fdtd_rom_coupled_update(problem: ProblemStruct, k: int):
    r = problem.s.roms[k]
    q, np_ = r.q, 2 * (r.ni + r.nj)
    A = np.zeros((q, q))
    B = np.zeros((q, np_))
    Cm = np.zeros((np_, q))
    _check(lib().fdtd_rom_coupled_update(C.byref(problem.s), k, _ptr(A), _ptr(B), _ptr(Cm)))
    return A, B, Cm


def fdtd_rom_build(ni, nj, r, dx, dy, dt, eps_r, sigma, q, f_max, theta=0.99, clip=True,
                   basis="sprim", pec=None):
    """Model of one refined region (host FP64 in the library).  basis
    'sprim' reduces to order q; 'identity' keeps the restricted fine model
    (q is then its state count and the argument is ignored).  pec: fine
    cells that are perfect conductors, or None."""
    er = np.ascontiguousarray(eps_r, dtype=np.float64)
    sg = np.ascontiguousarray(sigma, dtype=np.float64)
    assert er.shape == (r * nj, r * ni) and sg.shape == er.shape
    b = {"sprim": 0, "identity": 1}[basis]
    np_ = 2 * (ni + nj)
    keep = []
    prm = fdtd_rom_build_params(ni, nj, r, dx, dy, dt, _ptr(er), _ptr(sg), q, f_max, theta,
                                1 if clip else 0, b, _mask(pec, keep, er.shape))
    info = fdtd_rom_build_info()
    if b == 1:
        _check(lib().fdtd_rom_build(C.byref(prm), None, None, None, C.byref(info)))
        q = prm.q = info.n_fine_states
    Rt = np.zeros((q, q))
    Ft = np.zeros((q, q))
    Lt = np.zeros((q, np_))
    _check(lib().fdtd_rom_build(C.byref(prm), _ptr(Rt), _ptr(Ft), _ptr(Lt), C.byref(info)))
    return dict(Rt=Rt, Ft=Ft, Lt=Lt, q1=info.q1, q2=info.q2, p0=info.p0,
                smax_before=info.smax_before, smax_after=info.smax_after,
                clipped=bool(info.clipped), n_fine_states=info.n_fine_states)


def fdtd_rom_build_vjp(ni, nj, r, dx, dy, dt, eps_r, sigma, q, f_max, grad_Rt, grad_Ft, theta=0.99,
                       clip=True, basis="sprim", pec=None):
    """Fine-cell gradients (dJ/deps_r, dJ/dsigma, each [r*nj, r*ni]) from
    dJ/dR~ and dJ/dF~ of the model fdtd_rom_build makes from the same
    arguments, with its projection basis held (library, host FP64)."""
    er = np.ascontiguousarray(eps_r, dtype=np.float64)
    sg = np.ascontiguousarray(sigma, dtype=np.float64)
    assert er.shape == (r * nj, r * ni) and sg.shape == er.shape
    gR = np.ascontiguousarray(grad_Rt, dtype=np.float64)
    gF = np.ascontiguousarray(grad_Ft, dtype=np.float64)
    b = {"sprim": 0, "identity": 1}[basis]
    keep = []
    prm = fdtd_rom_build_params(ni, nj, r, dx, dy, dt, _ptr(er), _ptr(sg), q, f_max, theta,
                                1 if clip else 0, b, _mask(pec, keep, er.shape))
    if b == 1:
        info = fdtd_rom_build_info()
        _check(lib().fdtd_rom_build(C.byref(prm), None, None, None, C.byref(info)))
        prm.q = info.n_fine_states
    assert gR.shape == (prm.q, prm.q) and gF.shape == gR.shape, (gR.shape, prm.q)
    ge = np.zeros(er.shape)
    gs = np.zeros(er.shape)
    _check(lib().fdtd_rom_build_vjp(C.byref(prm), _ptr(gR), _ptr(gF), _ptr(ge), _ptr(gs)))
    return ge, gs


class ModelState:
    """The builder's state of one model (fdtd_rom_build_keep), freed with
    the object."""

    def __init__(self, ptr, q, fine_shape):
        self.ptr, self.q, self.fine_shape = ptr, q, fine_shape

    def __del__(self):
        if self.ptr is not None and _LIB is not None:
            _LIB.fdtd_rom_model_state_free(C.c_void_p(self.ptr))
            self.ptr = None


def fdtd_rom_build_keep(ni, nj, r, dx, dy, dt, eps_r, sigma, q, f_max, theta=0.99, clip=True, pec=None):
    """fdtd_rom_build (SPRIM basis) that also keeps the builder's state for
    fdtd_rom_model_state_vjp: the model dict gains 'state'."""
    er = np.ascontiguousarray(eps_r, dtype=np.float64)
    sg = np.ascontiguousarray(sigma, dtype=np.float64)
    assert er.shape == (r * nj, r * ni) and sg.shape == er.shape
    np_ = 2 * (ni + nj)
    keep = []
    prm = fdtd_rom_build_params(ni, nj, r, dx, dy, dt, _ptr(er), _ptr(sg), q, f_max, theta,
                                1 if clip else 0, 0, _mask(pec, keep, er.shape))
    info = fdtd_rom_build_info()
    Rt = np.zeros((q, q))
    Ft = np.zeros((q, q))
    Lt = np.zeros((q, np_))
    st = C.c_void_p(None)
    _check(lib().fdtd_rom_build_keep(C.byref(prm), _ptr(Rt), _ptr(Ft), _ptr(Lt), C.byref(info), C.byref(st)))
    return dict(Rt=Rt, Ft=Ft, Lt=Lt, q1=info.q1, q2=info.q2, p0=info.p0,
                smax_before=info.smax_before, smax_after=info.smax_after,
                clipped=bool(info.clipped), n_fine_states=info.n_fine_states,
                state=ModelState(st.value, q, er.shape))


def fdtd_rom_model_state_vjp(state: ModelState, grad_Rt, grad_Ft):
    """fdtd_rom_build_vjp's fine-cell gradients from a kept builder state."""
    gR = np.ascontiguousarray(grad_Rt, dtype=np.float64)
    gF = np.ascontiguousarray(grad_Ft, dtype=np.float64)
    assert gR.shape == (state.q, state.q) and gF.shape == gR.shape, (gR.shape, state.q)
    ge = np.zeros(state.fine_shape)
    gs = np.zeros(state.fine_shape)
    _check(lib().fdtd_rom_model_state_vjp(C.c_void_p(state.ptr), _ptr(gR), _ptr(gF), _ptr(ge), _ptr(gs)))
    return ge, gs


def fdtd_rom_profile_enable(h, enable: bool):
    _check(lib().fdtd_rom_profile_enable(h, 1 if enable else 0))


def fdtd_rom_profile_read(h):
    a = C.c_double(0)
    b = C.c_double(0)
    na = C.c_int64(0)
    nb = C.c_int64(0)
    _check(lib().fdtd_rom_profile_read(h, C.byref(a), C.byref(na), C.byref(b), C.byref(nb)))
    return float(a.value), int(na.value), float(b.value), int(nb.value)


def fdtd_rom_set_tiling(h, seg: int):
    _check(lib().fdtd_rom_set_tiling(h, int(seg)))


def fdtd_rom_get_tiling(h) -> int:
    n = C.c_int32(0)
    _check(lib().fdtd_rom_get_tiling(h, C.byref(n)))
    return int(n.value)


def fdtd_rom_set_shared_gemm(h, enable: bool):
    _check(lib().fdtd_rom_set_shared_gemm(h, 1 if enable else 0))


def fdtd_rom_set_material_mode(h, mode: int):
    _check(lib().fdtd_rom_set_material_mode(h, int(mode)))


def fdtd_rom_get_material_mode(h):
    """(mode, table entries): mode 1 = 16-bit index + table, 0 = per-cell arrays."""
    m = C.c_int32(0)
    n = C.c_int32(0)
    _check(lib().fdtd_rom_get_material_mode(h, C.byref(m), C.byref(n)))
    return int(m.value), int(n.value)


def fdtd_rom_set_time_blocking(h, on: bool):
    _check(lib().fdtd_rom_set_time_blocking(h, 1 if on else 0))


def fdtd_rom_set_pair_split(h, percent: int):
    _check(lib().fdtd_rom_set_pair_split(h, int(percent)))


def fdtd_rom_get_pair_split(h) -> int:
    v = C.c_int32(0)
    _check(lib().fdtd_rom_get_pair_split(h, C.byref(v)))
    return int(v.value)


def fdtd_rom_get_time_blocking(h) -> bool:
    v = C.c_int32(0)
    _check(lib().fdtd_rom_get_time_blocking(h, C.byref(v)))
    return bool(v.value)


def fdtd_rom_batch_set_pair_split(h, b: int, percent: int):
    _check(lib().fdtd_rom_batch_set_pair_split(h, int(b), int(percent)))


def fdtd_rom_batch_set_time_blocking(h, on: bool):
    _check(lib().fdtd_rom_batch_set_time_blocking(h, 1 if on else 0))


def fdtd_rom_batch_get_time_blocking(h) -> bool:
    v = C.c_int32(0)
    _check(lib().fdtd_rom_batch_get_time_blocking(h, C.byref(v)))
    return bool(v.value)


def fdtd_rom_set_graph(h, batch: int):
    _check(lib().fdtd_rom_set_graph(h, int(batch)))


def fdtd_rom_adjoint_workspace_size(h, nsteps: int, ckpt_every: int = 0) -> int:
    n = C.c_size_t(0)
    _check(lib().fdtd_rom_adjoint_workspace_size(h, int(nsteps), int(ckpt_every), C.byref(n)))
    return int(n.value)


def fdtd_rom_adjoint(h, nsteps: int, ckpt_every: int, probe: int, dev_ptr: int, nbytes: int,
                     nx: int, ny: int):
    """Returns (J, dJ/deps_r [ny, nx], dJ/dsigma [ny, nx])."""
    J = C.c_double(0)
    ge = np.zeros((ny, nx), dtype=np.float64)
    gs = np.zeros((ny, nx), dtype=np.float64)
    _check(lib().fdtd_rom_adjoint(h, int(nsteps), int(ckpt_every), int(probe), C.c_void_p(dev_ptr),
                                  nbytes, C.byref(J), _ptr(ge), _ptr(gs)))
    return float(J.value), ge, gs


def fdtd_rom_adjoint_models_workspace_size(h, nsteps: int, ckpt_every: int = 0) -> int:
    n = C.c_size_t(0)
    _check(lib().fdtd_rom_adjoint_models_workspace_size(h, int(nsteps), int(ckpt_every), C.byref(n)))
    return int(n.value)


def fdtd_rom_adjoint_models(h, nsteps: int, ckpt_every: int, probe: int, dev_ptr: int, nbytes: int,
                            nx: int, ny: int, shapes):
    """Returns (J, dJ/deps_r [ny, nx], dJ/dsigma [ny, nx], [dict(Rt, Ft, Lt)]
    per region); shapes: [(q, np)] per region."""
    J = C.c_double(0)
    ge = np.zeros((ny, nx), dtype=np.float64)
    gs = np.zeros((ny, nx), dtype=np.float64)
    outs = [dict(Rt=np.zeros((q, q)), Ft=np.zeros((q, q)), Lt=np.zeros((q, n))) for (q, n) in shapes]
    arr = (_dp * max(len(outs), 1))
    rt = arr(*[_ptr(o["Rt"]) for o in outs])
    ft = arr(*[_ptr(o["Ft"]) for o in outs])
    lt = arr(*[_ptr(o["Lt"]) for o in outs])
    _check(lib().fdtd_rom_adjoint_models(h, int(nsteps), int(ckpt_every), int(probe), C.c_void_p(dev_ptr),
                                         nbytes, C.byref(J), _ptr(ge), _ptr(gs), rt, ft, lt))
    return float(J.value), ge, gs, outs


def fdtd_rom_adjoint_plan(problem: ProblemStruct, nsteps: int, ckpt_every: int = 0) -> int:
    """Adjoint workspace bytes of a problem (host only, no handle)."""
    n = C.c_size_t(0)
    _check(lib().fdtd_rom_adjoint_plan(C.byref(problem.s), int(nsteps), int(ckpt_every), C.byref(n)))
    return int(n.value)


def fdtd_rom_adjoint_noalloc(h, nsteps: int, ckpt_every: int, probe: int, nx: int, ny: int):
    """As fdtd_rom_adjoint, with the library's static device scratch instead
    of a caller workspace.  Returns (J, dJ/deps_r [ny, nx], dJ/dsigma [ny, nx])."""
    J = C.c_double(0)
    ge = np.zeros((ny, nx), dtype=np.float64)
    gs = np.zeros((ny, nx), dtype=np.float64)
    _check(lib().fdtd_rom_adjoint_noalloc(h, int(nsteps), int(ckpt_every), int(probe), C.byref(J), _ptr(ge),
                                          _ptr(gs)))
    return float(J.value), ge, gs


def fdtd_rom_energy(h) -> float:
    e = C.c_double(0)
    _check(lib().fdtd_rom_energy(h, C.byref(e)))
    return float(e.value)


def fdtd_rom_state_size(h) -> int:
    n = C.c_size_t(0)
    _check(lib().fdtd_rom_state_size(h, C.byref(n)))
    return int(n.value)


def fdtd_rom_get_state(h, dev_ptr: int):
    _check(lib().fdtd_rom_get_state(h, C.c_void_p(dev_ptr)))


def fdtd_rom_set_state(h, dev_ptr: int):
    _check(lib().fdtd_rom_set_state(h, C.c_void_p(dev_ptr)))


def _problem_array(problems):
    arr = (fdtd_problem * len(problems))()
    for k, ps in enumerate(problems):
        arr[k] = ps.s
    return arr


def fdtd_rom_batch_workspace_size(problems) -> int:
    n = C.c_size_t(0)
    arr = _problem_array(problems)
    _check(lib().fdtd_rom_batch_workspace_size(arr, len(problems), C.byref(n)))
    return int(n.value)


def fdtd_rom_batch_create(problems, dev_ptr: int, nbytes: int, stream: int):
    h = C.c_void_p()
    arr = _problem_array(problems)
    _check(lib().fdtd_rom_batch_create(arr, len(problems), C.c_void_p(dev_ptr), nbytes,
                                       C.c_void_p(stream), C.byref(h)))
    return h


def fdtd_rom_batch_run(h, nsteps: int):
    _check(lib().fdtd_rom_batch_run(h, int(nsteps)))


def fdtd_rom_batch_steps_done(h) -> int:
    n = C.c_int32(0)
    _check(lib().fdtd_rom_batch_steps_done(h, C.byref(n)))
    return int(n.value)


def fdtd_rom_batch_read_probes(h, b: int, first: int, count: int, nprobes: int) -> np.ndarray:
    out = np.zeros((count, nprobes), dtype=np.float64)
    _check(lib().fdtd_rom_batch_read_probes(h, b, first, count, _ptr(out)))
    return out


def fdtd_rom_batch_read_field(h, b: int, comp: int, nx: int, ny: int) -> np.ndarray:
    shape = {FDTD_HZ: (ny, nx), FDTD_EX: (ny + 1, nx), FDTD_EY: (ny, nx + 1)}[comp]
    out = np.zeros(shape, dtype=np.float64)
    _check(lib().fdtd_rom_batch_read_field(h, b, comp, _ptr(out)))
    return out


def fdtd_rom_batch_set_tiling(h, b: int, seg: int):
    _check(lib().fdtd_rom_batch_set_tiling(h, int(b), int(seg)))


def fdtd_rom_batch_set_graph(h, batch: int):
    _check(lib().fdtd_rom_batch_set_graph(h, int(batch)))


def fdtd_rom_batch_destroy(h):
    lib().fdtd_rom_batch_destroy(h)


def fdtd_rom_destroy(h):
    lib().fdtd_rom_destroy(h)


def fdtd_rom_strerror(status: int) -> str:
    return lib().fdtd_rom_strerror(status).decode()


def fdtd_rom_last_error() -> str:
    return lib().fdtd_rom_last_error().decode()
