"""The library's host FP64 reduced-model builder (fdtd_rom_build) against the
oracle's independent builder.  Two valid builds of the same subspace differ
by a change of reduced coordinates, so they are compared through the
coordinate-free transfer function H(p) = L^T (pR + F)^{-1} L Sc, plus
Theorem 1's invariants and the clip bound of eq. (27)."""
import numpy as np
import pytest

import workloads as W
from oracle import rom as orom
from oracle import yee
from oracle.constants import C0
from paper_1609_07114_amd import capi, romgen

PVALS = [0.3, 0.05 + 0.4j, 0.9j, 0.02]


def _both(spec, prob, **kw):
    a = capi.fdtd_rom_build(spec.ni, spec.nj, spec.r, prob.dx, prob.dy, prob.dt, spec.eps_r,
                            spec.sigma, spec.q, spec.f_max, **kw)
    b = orom.build_rom(spec.eps_r, spec.sigma, spec.r, prob.dx, prob.dy, prob.dt, spec.q,
                       spec.f_max, clip=kw.get("clip", True))
    return a, b


def _tf_err(a, b, p):
    Sc = b["Sc"]
    Ha = orom.transfer(a["Rt"], a["Ft"], a["Lt"], Sc, p)
    Hb = orom.transfer(b["Rt"], b["Ft"], b["Lt"], Sc, p)
    return np.max(np.abs(Ha - Hb)) / np.max(np.abs(Hb))


@pytest.mark.parametrize("seed,block,r,q", [(20, (5, 4), 2, 14), (21, (3, 4), 3, 11),
                                           (22, (4, 4), 2, 40)])
def test_builder_matches_oracle_transfer(seed, block, r, q):
    p = W.random_problem(seed, 26, 22, 10, nroms=1, block=block, r=r, q=q)
    a, b = _both(p.roms[0], p)
    assert (a["q1"], a["q2"]) == (b["q1"], b["q2"])
    for pv in PVALS + [b["p0"]]:
        assert _tf_err(a, b, pv) < 1e-10, pv


def test_builder_theorem1_invariants():
    p = W.random_problem(23, 26, 22, 10, nroms=1, block=(5, 5), r=2, q=20)
    s = p.roms[0]
    a = capi.fdtd_rom_build(s.ni, s.nj, s.r, p.dx, p.dy, p.dt, s.eps_r, s.sigma, s.q, s.f_max)
    Rt, Ft = a["Rt"], a["Ft"]
    assert np.array_equal(Rt, Rt.T)
    np.linalg.cholesky(Rt)
    assert np.linalg.eigvalsh(Ft + Ft.T).min() >= -1e-12 * np.abs(Ft).max()
    # only E coordinates see the ports: L~ rows of the H block are zero
    assert np.all(a["Lt"][a["q1"]:] == 0)


def test_builder_clip_active_matches_oracle():
    """dt = 1.9x the fine CFL, a nearly complete basis: the clip of eq. (27)
    is active in both builders and leaves the same model."""
    p = W.random_problem(11, 10, 9, 10, nroms=1, block=(3, 3), r=2, q=0,
                         dt_frac_coarse=0.95, lossy=True)
    s = p.roms[0]
    s.eps_r[:] = 1.0          # vacuum region: its own CFL limit is eq. (1) on the fine cells
    s.q = 64
    a, b = _both(s, p)
    assert a["clipped"] and b["clipped"]
    assert a["smax_before"] == pytest.approx(b["smax_before"], rel=1e-9)
    assert a["smax_after"] <= 0.99 * 2 / p.dt * (1 + 1e-12)
    np.linalg.cholesky(a["Rt"])
    for pv in PVALS:
        assert _tf_err(a, b, pv) < 1e-9, pv
    # without the clip the same model is not passive at this dt
    c = capi.fdtd_rom_build(s.ni, s.nj, s.r, p.dx, p.dy, p.dt, s.eps_r, s.sigma, s.q, s.f_max,
                            clip=False)
    with pytest.raises(np.linalg.LinAlgError):
        np.linalg.cholesky(c["Rt"])


def test_builder_rejects_bad_order():
    p = W.random_problem(24, 26, 22, 10, nroms=1, block=(2, 2), r=1, q=4)
    s = p.roms[0]
    with pytest.raises(capi.FdtdError):
        capi.fdtd_rom_build(s.ni, s.nj, s.r, p.dx, p.dy, p.dt, s.eps_r, s.sigma, 500, s.f_max)


def test_build_roms_groups_and_threads():
    p = W.many_copies(n=512, nsteps=10, q=16, spacing=128, block=8)
    roms = romgen.build_roms(p)
    assert len(roms) == len(p.roms) == 16
    assert all(r is roms[0] for r in roms)
    p2 = W.random_media(n=256, nsteps=10, spacing=128, offset=48, block=16, qs=(16, 24, 32, 48))
    r2 = romgen.build_roms(p2)
    assert [m["Rt"].shape[0] for m in r2] == [s.q for s in p2.roms]


def test_identity_basis_matches_oracle():
    """basis 'identity' (no reduction, the paper's "CFL extension only"
    configuration): same restricted fine model as the oracle's identity
    basis, clip of eq. (27) active at 2.9x the fine step, same transfer
    function; the size query reports the restricted state count."""
    p = W.random_problem(13, 12, 11, 10, nroms=1, block=(4, 3), r=3, q=0, lossy=True)
    s = p.roms[0]
    p.dt = 2.9 * W.courant_dt(p.dx / s.r, p.dy / s.r, 0.99)
    a = capi.fdtd_rom_build(s.ni, s.nj, s.r, p.dx, p.dy, p.dt, s.eps_r, s.sigma, 0, s.f_max,
                            basis="identity")
    b = orom.build_rom(s.eps_r, s.sigma, s.r, p.dx, p.dy, p.dt, 0, s.f_max, basis="identity")
    assert a["Rt"].shape == b["Rt"].shape == (a["n_fine_states"],) * 2
    assert (a["q1"], a["q2"]) == (b["q1"], b["q2"])
    assert a["clipped"] and b["clipped"]
    assert a["smax_before"] == pytest.approx(b["smax_before"], rel=1e-9)
    assert a["smax_after"] == pytest.approx(b["smax_after"], rel=1e-9)
    np.linalg.cholesky(a["Rt"])
    for pv in PVALS:
        assert _tf_err(a, b, pv) < 1e-9, pv
    # R~11 and R~22 stay diagonal, F~ has no H-H block
    q1 = a["q1"]
    R11 = a["Rt"][:q1, :q1]
    assert np.array_equal(R11, np.diag(np.diag(R11)))
    assert np.all(a["Ft"][q1:, q1:] == 0)


def test_identity_basis_unclipped_is_the_fine_model():
    """Below the fine CFL limit nothing is clipped: the identity-basis
    model is the restricted fine model, equal to the oracle's entry by entry
    up to the order of the states (compared through H(p) and R~ spectra)."""
    p = W.random_problem(14, 12, 11, 10, nroms=1, block=(3, 3), r=2, q=0, lossy=True)
    s = p.roms[0]
    a = capi.fdtd_rom_build(s.ni, s.nj, s.r, p.dx, p.dy, p.dt, s.eps_r, s.sigma, 0, s.f_max,
                            basis="identity")
    b = orom.build_rom(s.eps_r, s.sigma, s.r, p.dx, p.dy, p.dt, 0, s.f_max, basis="identity")
    assert not a["clipped"]
    ea, eb = np.sort(np.linalg.eigvalsh(a["Rt"])), np.sort(np.linalg.eigvalsh(b["Rt"]))
    assert np.max(np.abs(ea - eb)) <= 1e-12 * eb.max()
    for pv in PVALS:
        assert _tf_err(a, b, pv) < 1e-11, pv


@pytest.mark.parametrize("basis", ["sprim", "identity"])
def test_builder_with_pec_cells_matches_oracle(basis):
    """PEC fine cells (a plate from the South boundary, a corner cell, an
    interior cell): the library leaves their samples and the ports they
    cover out of the model like the oracle - same restricted state count,
    same dead ports (zero columns of Lt), same transfer function - and a
    port only partly on PEC cells is rejected."""
    p = W.random_problem(24, 26, 22, 10, nroms=1, block=(5, 4), r=2, q=16)
    s = p.roms[0]
    fp = np.zeros((2 * s.nj, 2 * s.ni), dtype=bool)
    fp[:4, 4:6] = True
    fp[6:, 8:] = True
    fp[2, 2] = True
    kw = dict(pec=fp, basis=basis)
    if basis == "identity":
        kw["clip"] = False
    a = capi.fdtd_rom_build(s.ni, s.nj, s.r, p.dx, p.dy, p.dt, s.eps_r, s.sigma, s.q, s.f_max, **kw)
    b = orom.build_rom(s.eps_r, s.sigma, s.r, p.dx, p.dy, p.dt, s.q, s.f_max, basis=basis,
                       clip=kw.get("clip", True), pec=fp)
    assert a["n_fine_states"] == b["model"]["n"]
    dead = b["model"]["restriction"]["dead_ports"]
    assert dead == [2, 9, 17]
    assert np.all(a["Lt"][:, dead] == 0)
    if basis == "identity":
        assert a["Rt"].shape == b["Rt"].shape
        assert np.max(np.abs(a["Rt"] - b["Rt"])) <= 1e-12 * np.abs(b["Rt"]).max()
        assert np.max(np.abs(a["Ft"] - b["Ft"])) <= 1e-12 * np.abs(b["Ft"]).max()
        assert np.array_equal(a["Lt"], b["Lt"])
    for pv in PVALS + ([b["p0"]] if basis == "sprim" else []):
        assert _tf_err(a, b, pv) < 1e-10, pv
    bad = np.zeros_like(fp)
    bad[0, 0] = True
    with pytest.raises(capi.FdtdError):
        capi.fdtd_rom_build(s.ni, s.nj, s.r, p.dx, p.dy, p.dt, s.eps_r, s.sigma, s.q, s.f_max, pec=bad)


def _port_response(Rt, Ft, Lt, Wm, p=0.3):
    """f = sum(W o H(p)), H(p) = L~^T (p R~ + F~)^{-1} L~ - a quantity of the
    model that does not depend on its basis - and its gradients with
    respect to R~ and F~."""
    X = p * Rt + Ft
    Xi = np.linalg.inv(X)
    gX = -Xi.T @ Lt @ Wm @ Lt.T @ Xi.T
    return float(np.sum(Wm * (Lt.T @ Xi @ Lt))), p * gX, gX


@pytest.mark.parametrize("r,q,basis,clipped,pec", [(2, 12, "sprim", False, False), (3, 140, "sprim", True, False),
                                                   (2, 0, "identity", True, False), (2, 16, "sprim", False, True)])
def test_build_vjp_matches_oracle(r, q, basis, clipped, pec):
    """The gradient through the builder (basis held; through the eq. (27)
    clip when it acts) of a basis-independent function of the model equals
    the oracle's (pinned by finite differences) to 1e-12: each side takes
    the function's gradient in its own basis."""
    p = W.random_problem(31, 30, 26, 10, nroms=1, block=(5, 4), r=r, q=q, dt_frac_coarse=0.9, f_bw=3e9)
    s = p.roms[0]
    fp = None
    if pec:
        fp = np.zeros((r * s.nj, r * s.ni), dtype=bool)
        fp[:4, 4:6] = True
        fp[2, 2] = True
    o = orom.build_rom(s.eps_r, s.sigma, s.r, p.dx, p.dy, p.dt, s.q, s.f_max, basis=basis, pec=fp)
    lib = capi.fdtd_rom_build(s.ni, s.nj, s.r, p.dx, p.dy, p.dt, s.eps_r, s.sigma, s.q, s.f_max, basis=basis,
                              pec=fp)
    assert o["clipped"] == clipped and lib["clipped"] == clipped
    Wm = np.random.default_rng(0).standard_normal((s.n_ports, s.n_ports))
    fo, gRo, gFo = _port_response(o["Rt"], o["Ft"], o["Lt"], Wm)
    fl, gRl, gFl = _port_response(lib["Rt"], lib["Ft"], lib["Lt"], Wm)
    assert fl == pytest.approx(fo, rel=1e-12)
    from oracle import model_grad as mg
    geo, gso = mg.build_vjp(o, gRo, gFo)
    gel, gsl = capi.fdtd_rom_build_vjp(s.ni, s.nj, s.r, p.dx, p.dy, p.dt, s.eps_r, s.sigma, s.q, s.f_max, gRl, gFl,
                                       basis=basis, pec=fp)
    assert np.linalg.norm(gel - geo) <= 1e-12 * np.linalg.norm(geo)
    assert np.linalg.norm(gsl - gso) <= 1e-12 * np.linalg.norm(gso)
    if pec:
        assert np.all(gel[fp] == 0) and np.all(gsl[fp] == 0)


@pytest.mark.parametrize("r,q,clipped,pec", [(2, 12, False, False), (3, 140, True, False), (2, 16, False, True)])
def test_kept_builder_state_gives_the_rebuilt_gradient(r, q, clipped, pec):
    """fdtd_rom_build_keep returns fdtd_rom_build's model bit for bit and a
    state whose gradient (fdtd_rom_model_state_vjp, no rebuild) is
    fdtd_rom_build_vjp's bit for bit, on every call; build_roms(keep=True)
    hands the states to build_vjps; gradients of the wrong shape are
    refused."""
    p = W.random_problem(31, 30, 26, 10, nroms=1, block=(5, 4), r=r, q=q, dt_frac_coarse=0.9, f_bw=3e9)
    s = p.roms[0]
    fp = None
    if pec:
        fp = np.zeros((r * s.nj, r * s.ni), dtype=bool)
        fp[:4, 4:6] = True
    a = capi.fdtd_rom_build(s.ni, s.nj, s.r, p.dx, p.dy, p.dt, s.eps_r, s.sigma, s.q, s.f_max, pec=fp)
    b = capi.fdtd_rom_build_keep(s.ni, s.nj, s.r, p.dx, p.dy, p.dt, s.eps_r, s.sigma, s.q, s.f_max, pec=fp)
    assert b["clipped"] == clipped
    for k in ("Rt", "Ft", "Lt"):
        assert np.array_equal(a[k], b[k]), k
    rng = np.random.default_rng(3)
    gR, gF = rng.standard_normal((s.q, s.q)), rng.standard_normal((s.q, s.q))
    want = capi.fdtd_rom_build_vjp(s.ni, s.nj, s.r, p.dx, p.dy, p.dt, s.eps_r, s.sigma, s.q, s.f_max, gR, gF,
                                   pec=fp)
    for _ in range(2):   # the state is read only: the same answer twice
        got = capi.fdtd_rom_model_state_vjp(b["state"], gR, gF)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    if fp is None:
        roms = romgen.build_roms(p, keep=True)
        got = romgen.build_vjps(p, [dict(Rt=gR, Ft=gF)], roms=roms)[0]
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
    with pytest.raises(AssertionError):
        capi.fdtd_rom_model_state_vjp(b["state"], gR[:-1, :-1], gF[:-1, :-1])
