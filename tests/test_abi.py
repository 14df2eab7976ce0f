"""CPU tests of the C-ABI library: it loads, exports every entry point the
header declares, and its host-side logic (validation, the FP64 closed form
of eq. (23)) agrees with the oracle.  No device call is made here."""
import copy
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from oracle import coupling as ocp
from oracle import sim as osim
from paper_1609_07114_amd import capi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(fdtd_\w+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = capi.lib()
    decl = header_functions()
    assert len(decl) >= 10
    for name in decl:
        assert hasattr(L, name), name
    # and the binding covers all of them under the same names
    assert set(decl) == set(capi.exported_symbols())


def test_strerror():
    assert capi.fdtd_rom_strerror(capi.FDTD_ENOTPASSIVE).startswith("reduced model")


def _struct(prob, roms, **kw):
    return capi.ProblemStruct.from_workload(prob, roms, **kw)


def _create_status(ps):
    """Call create with a dummy aligned pointer: every check below fails
    before the library touches the device."""
    h = ctypes.c_void_p()
    rc = capi.lib().fdtd_rom_create(ctypes.byref(ps.s), ctypes.c_void_p(1 << 20), 1 << 40,
                                    None, ctypes.byref(h))
    return rc


@pytest.fixture(scope="module")
def small():
    p = W.random_problem(5, 24, 20, 50, nroms=2, block=(4, 3), r=2, q=10)
    roms = osim.build_roms(p)
    return p, roms


def test_workspace_size_positive(small):
    p, roms = small
    n = capi.fdtd_rom_workspace_size(_struct(p, roms))
    assert n > 6 * p.nx * p.ny * 8


def test_rejects_dt_above_cfl(small):
    import copy
    p, roms = small
    q = copy.deepcopy(p)
    q.dt = 1.01 * W.courant_dt(q.dx, q.dy, 1.0)
    assert _create_status(_struct(q, roms)) == capi.FDTD_EINVAL
    assert "CFL" in capi.fdtd_rom_last_error()


def test_rejects_region_on_wall(small):
    import copy
    p, roms = small
    q = copy.deepcopy(p)
    q.roms[0].i0 = 0
    assert _create_status(_struct(q, roms)) == capi.FDTD_EINVAL


def test_rejects_overlapping_rings(small):
    import copy
    p, roms = small
    q = copy.deepcopy(p)
    q.roms[1].i0 = q.roms[0].i0 + q.roms[0].ni
    q.roms[1].j0 = q.roms[0].j0
    assert _create_status(_struct(q, roms)) == capi.FDTD_EINVAL


def test_rejects_probe_inside_region(small):
    import copy
    p, roms = small
    q = copy.deepcopy(p)
    r = q.roms[0]
    q.probes[0] = W.Probe(W.HZ, r.i0 + 1, r.j0 + 1)
    assert _create_status(_struct(q, roms)) == capi.FDTD_EINVAL
    q.probes[0] = W.Probe(W.EX, r.i0 + 1, r.j0)   # interface edge
    assert _create_status(_struct(q, roms)) == capi.FDTD_EINVAL


def test_rejects_source_on_interface(small):
    import copy
    p, roms = small
    q = copy.deepcopy(p)
    r = q.roms[0]
    q.sources[1] = W.Source(W.EY, r.i0, r.i0 + 1, r.j0, r.j0 + 1, q.sources[1].incr)
    assert _create_status(_struct(q, roms)) == capi.FDTD_EINVAL


def test_rejects_nonpassive_model():
    """An unreduced region at 1.9x its own CFL limit violates eq. (26a) unless
    clipped (eq. (27)): create refuses it, and accepts the clipped one."""
    p = W.random_problem(11, 10, 9, 10, nroms=1, block=(3, 3), r=2, q=0,
                         dt_frac_coarse=0.95, lossy=False)
    bad = osim.build_roms(p, basis="identity", clip=False)
    assert _create_status(_struct(p, bad)) == capi.FDTD_ENOTPASSIVE
    good = osim.build_roms(p, basis="identity", clip=True)
    A, B, C = capi.fdtd_rom_coupled_update(_struct(p, good), 0)
    assert np.all(np.isfinite(A))


def test_workspace_too_small(small):
    p, roms = small
    ps = _struct(p, roms)
    h = ctypes.c_void_p()
    rc = capi.lib().fdtd_rom_create(ctypes.byref(ps.s), ctypes.c_void_p(1 << 20), 1024, None,
                                    ctypes.byref(h))
    assert rc == capi.FDTD_ENOMEM


@pytest.mark.parametrize("seed", [0, 1])
def test_closed_form_matches_oracle(seed):
    """Library FP64 closed form of eq. (23) vs the oracle's (same R~, F~, L~)."""
    p = W.random_problem(20 + seed, 26, 22, 10, nroms=2, block=(5, 4), r=2, q=14)
    roms = osim.build_roms(p)
    ps = _struct(p, roms)
    for k, (spec, m) in enumerate(zip(p.roms, roms)):
        c = ocp.RomCoupling(m["Rt"], m["Ft"], m["Lt"], spec.i0, spec.j0, spec.ni, spec.nj,
                            p.eps_r, p.sigma, p.dx, p.dy, p.dt)
        A0, B0, C0 = c.closed_form()
        A, B, C = capi.fdtd_rom_coupled_update(ps, k)
        assert np.max(np.abs(A - A0)) <= 1e-12 * np.max(np.abs(A0))
        assert np.max(np.abs(B - B0)) <= 1e-12 * np.max(np.abs(B0))
        assert np.array_equal(C, C0)


def test_absorbing_layer_validation():
    """Layer thicknesses and placement are checked on the host: negative or
    overlapping layers, and a model ring reaching into a layer, are refused."""
    import copy
    p = W.random_problem(5, 60, 50, 20, nroms=1, block=(6, 5), r=2, q=8)
    roms = [dict(Rt=np.eye(8), Ft=np.zeros((8, 8)), Lt=np.zeros((8, 22)))]
    for bad in (W.Pml(-1, 0, 0, 0), W.Pml(30, 30, 0, 0), W.Pml(0, 0, 25, 25)):
        q = copy.deepcopy(p)
        q.pml = bad
        with pytest.raises(capi.FdtdError):
            capi.fdtd_rom_workspace_size(capi.ProblemStruct.from_workload(q, roms))
    s = p.roms[0]
    q = copy.deepcopy(p)
    q.pml = W.Pml(n_xlo=s.i0, n_xhi=0, n_ylo=0, n_yhi=0)   # ring column i0-1 inside the layer
    with pytest.raises(capi.FdtdError) as e:
        capi.fdtd_rom_coupled_update(capi.ProblemStruct.from_workload(q, roms), 0)
    assert "absorbing" in str(e.value)
    q.pml = W.Pml(n_xlo=s.i0 - 1, n_xhi=2, n_ylo=2, n_yhi=2)
    capi.fdtd_rom_coupled_update(capi.ProblemStruct.from_workload(q, roms), 0)


def test_model_order_limits():
    """Orders up to what the coupling staging holds are accepted (the rods
    region of Sec. VI-C needs 1920 reduced, 6848 unreduced), larger ones are
    refused before any device work: (q + np) padded to 64 elements must fit
    64 KB (16384 FP32, 8192 FP64)."""
    import copy
    p = W.rods_reflection(nsteps=10, dtype="f32")
    np_ = p.roms[0].n_ports

    def model(q):
        return [dict(Rt=np.eye(q), Ft=np.zeros((q, q)), Lt=np.zeros((q, np_)))]

    n = capi.fdtd_rom_workspace_size(_struct(p, model(1920)))
    assert n > (1920 + np_) ** 2 * 4
    q = copy.deepcopy(p)
    q.roms[0].q = 6848
    assert capi.fdtd_rom_workspace_size(_struct(q, model(6848))) > 6848 ** 2 * 4
    q.dtype = "f64"
    q.roms[0].q = 8200
    with pytest.raises(capi.FdtdError) as e:
        capi.fdtd_rom_workspace_size(_struct(q, model(8200)))
    assert "staging" in str(e.value)


def test_closed_form_identity_basis_matches_oracle():
    """A model kept in the identity basis (clip active) makes eq. (23)'s
    matrix block upper triangular with diagonal blocks; the library solves
    it by block back substitution.  Same A~, B~' as the oracle's dense solve."""
    import copy
    p = W.random_problem(15, 20, 18, 10, nroms=1, block=(4, 3), r=3, q=0, lossy=True)
    s = p.roms[0]
    p.dt = 2.9 * W.courant_dt(p.dx / s.r, p.dy / s.r, 0.99)
    m = capi.fdtd_rom_build(s.ni, s.nj, s.r, p.dx, p.dy, p.dt, s.eps_r, s.sigma, 0, s.f_max,
                            basis="identity")
    q = copy.deepcopy(p)
    q.roms[0].q = m["Rt"].shape[0]
    roms = [dict(Rt=m["Rt"], Ft=m["Ft"], Lt=m["Lt"])]
    c = ocp.RomCoupling(m["Rt"], m["Ft"], m["Lt"], s.i0, s.j0, s.ni, s.nj, p.eps_r, p.sigma,
                        p.dx, p.dy, p.dt)
    A0, B0, C0 = c.closed_form()
    A, B, C = capi.fdtd_rom_coupled_update(_struct(q, roms), 0)
    assert np.max(np.abs(A - A0)) <= 1e-12 * np.max(np.abs(A0))
    assert np.max(np.abs(B - B0)) <= 1e-12 * np.max(np.abs(B0))
    assert np.array_equal(C, C0)


def test_pec_cells_validation():
    """PEC cells: accepted with a model that leaves the covered ports
    undriven (closed form as the oracle's); rejected inside a region, on a
    ring cell whose port the model drives, and under a source or probe."""
    p = W.pec_problem(3, r=2, q=10)
    roms = osim.build_roms(p)
    assert np.all(roms[0]["Lt"][:, [2, 9, 17]] == 0)
    spec, m = p.roms[0], roms[0]
    c = ocp.RomCoupling(m["Rt"], m["Ft"], m["Lt"], spec.i0, spec.j0, spec.ni, spec.nj,
                        p.eps_r, p.sigma, p.dx, p.dy, p.dt)
    A0, B0, _ = c.closed_form()
    A, B, _ = capi.fdtd_rom_coupled_update(_struct(p, roms), 0)
    assert np.max(np.abs(A - A0)) <= 1e-12 * np.max(np.abs(A0))
    assert np.max(np.abs(B - B0)) <= 1e-12 * np.max(np.abs(B0))
    assert not np.any(B[:, [2, 9, 17]])
    # a PEC ring cell in front of a port the model drives (South port 1)
    q = copy.deepcopy(p)
    q.pec[spec.j0 - 1, spec.i0 + 1] = True
    with pytest.raises(capi.FdtdError, match="faces PEC"):
        capi.fdtd_rom_coupled_update(_struct(q, roms), 0)
    # a PEC cell inside the region
    q = copy.deepcopy(p)
    q.pec[spec.j0 + 1, spec.i0 + 1] = True
    with pytest.raises(capi.FdtdError, match="inside the region"):
        capi.fdtd_rom_coupled_update(_struct(q, roms), 0)
    # a probe on an edge of a PEC cell, a source on a PEC cell
    q = copy.deepcopy(p)
    q.probes[0] = W.Probe(W.EY, spec.i0 + 2, 0)
    assert _create_status(_struct(q, roms)) == capi.FDTD_EINVAL
    q = copy.deepcopy(p)
    q.sources[0].i0, q.sources[0].i1 = spec.i0 + 2, spec.i0 + 3
    q.sources[0].j0, q.sources[0].j1 = 0, 1
    q.sources[0].comp = W.HZ
    assert _create_status(_struct(q, roms)) == capi.FDTD_EINVAL


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_adjoint_plan_host_only(dtype):
    """The adjoint workspace plan from a problem alone (no handle, no
    device), with models, absorbing layers and several checkpoint intervals:
    it covers at least the checkpoints, the recomputed segment and the
    adjoint sets the sweep needs (its own check keeps the parts disjoint)."""
    ts = 4 if dtype == "f32" else 8
    p = W.random_problem(81, 70, 45, 300, nroms=2, block=(5, 4), r=2, q=10, dtype=dtype)
    roms = osim.build_roms(p)
    fb = p.nx * p.ny * ts              # one field array holds at least the cells
    for K in (1, 7, 300, 0):
        nb = capi.fdtd_rom_adjoint_plan(_struct(p, roms), 300, K)
        k = K or 18
        nck = -(-300 // k)
        assert nb >= (nck + k + 2) * 3 * fb + 2 * p.nx * p.ny * 8, (K, nb)
    q = copy.deepcopy(p)
    q.pml = W.Pml(4, 4, 3, 3)
    for s in q.roms:
        s.i0 += 3
        s.j0 += 2
    nb_l = capi.fdtd_rom_adjoint_plan(_struct(q, osim.build_roms(q)), 300, 7)
    assert nb_l > capi.fdtd_rom_adjoint_plan(_struct(p, roms), 300, 7)
    with pytest.raises(capi.FdtdError):
        capi.fdtd_rom_adjoint_plan(_struct(p, roms), 301, 7)      # beyond max_steps
    with pytest.raises(capi.FdtdError):
        capi.fdtd_rom_adjoint_plan(_struct(p, roms), 300, 301)


def test_pitch_pad_checked_and_sized(small):
    """fdtd_grid.pitch_pad: multiples of 64 in [0, 1024] widen every field
    row; anything else is refused."""
    p, roms = small
    base = capi.fdtd_rom_workspace_size(_struct(p, roms))
    q = copy.copy(p)
    q.pitch_pad = 64
    assert capi.fdtd_rom_workspace_size(_struct(q, roms)) > base
    for bad in (-64, 32, 1088):
        q.pitch_pad = bad
        with pytest.raises(capi.FdtdError) as e:
            capi.fdtd_rom_workspace_size(_struct(q, roms))
        assert e.value.status == capi.FDTD_EINVAL
