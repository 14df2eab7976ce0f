"""Pins of the oracle's coarse Yee grid against what the mathematics fixes:
textbook discrete dispersion of a PEC cavity, the CFL boundary of eq. (1),
the PEC resonances f_mn, and the FP32 coefficient model's algebra."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import sim, yee
from oracle.constants import C0, EPS0, MU0


def _cavity(nx, ny, dx, dy, dt, eps_r=1.0):
    return W.Problem("cav", nx, ny, dx, dy, dt, np.full((ny, nx), eps_r),
                     np.zeros((ny, nx)), [], [], [], 1, "f64")


def one_step_matrix(prob, roms=()):
    """Brute force: step every unit vector of [Hz, Ex, Ey, x~...] once."""
    nx, ny = prob.nx, prob.ny
    sizes = [ny * nx, (ny + 1) * nx, ny * (nx + 1)] + [m["Rt"].shape[0] for m in roms]
    n = sum(sizes)
    M = np.zeros((n, n))
    for k in range(n):
        v = np.zeros(n)
        v[k] = 1.0
        parts = np.split(v, np.cumsum(sizes)[:-1])
        init = dict(hz=parts[0].reshape(ny, nx), ex=parts[1].reshape(ny + 1, nx),
                    ey=parts[2].reshape(ny, nx + 1), x=list(parts[3:]))
        run = sim.CoupledRun(prob, list(roms), mode="closed", init=init)
        run.step()
        M[:, k] = np.concatenate([run.f.hz.ravel(), run.f.ex.ravel(), run.f.ey.ravel()]
                                 + [x for x in run.x])
    return M


def test_dispersion_eigenvalues_pec_cavity():
    """Eigenvalues of the one-step map are exp(+-i w dt) with
    sin(w dt/2) = c dt sqrt(sin^2(m pi/2Nx)/dx^2 + sin^2(n pi/2Ny)/dy^2)
    (textbook Yee dispersion in a PEC box), plus 1 for static modes."""
    nx, ny, dx, dy = 6, 5, 0.01, 0.012
    er = 2.0
    c = C0 / math.sqrt(er)
    dt = 0.9 * yee.cfl_dt(dx, dy, c)
    M = one_step_matrix(_cavity(nx, ny, dx, dy, dt, er))
    lam = np.linalg.eigvals(M)
    # drop the structurally-zero columns (wall edges)
    lam = lam[np.abs(lam) > 1e-6]
    assert np.allclose(np.abs(lam), 1.0, atol=1e-10)
    ang = np.sort(np.abs(np.angle(lam)))
    expect = []
    for m in range(nx):
        for n in range(ny):
            if m == 0 and n == 0:
                continue
            s = c * dt * math.sqrt(math.sin(m * math.pi / (2 * nx)) ** 2 / dx ** 2
                                   + math.sin(n * math.pi / (2 * ny)) ** 2 / dy ** 2)
            w = 2 * math.asin(s)
            expect += [w, w]
    n_static = 1 + (nx - 1) * (ny - 1)
    expect += [0.0] * n_static
    expect = np.sort(np.array(expect))
    assert ang.size == expect.size
    assert np.max(np.abs(ang - expect)) < 1e-8


def test_cfl_boundary_spectral_radius():
    """Spectral radius is 1 below the discrete stability limit and > 1 above
    it; the discrete limit lies above eq. (1) and tends to it as N grows."""
    nx, ny, dx, dy = 7, 6, 0.01, 0.01
    c = C0
    smax = math.sqrt(math.sin((nx - 1) * math.pi / (2 * nx)) ** 2 / dx ** 2
                     + math.sin((ny - 1) * math.pi / (2 * ny)) ** 2 / dy ** 2)
    dt_lim = 1.0 / (c * smax)
    assert dt_lim > yee.cfl_dt(dx, dy, c)
    rho = lambda dt: np.max(np.abs(np.linalg.eigvals(one_step_matrix(_cavity(nx, ny, dx, dy, dt)))))
    assert rho(0.999 * dt_lim) < 1 + 1e-9
    assert rho(1.01 * dt_lim) > 1 + 1e-3
    # convergence of the discrete limit to eq. (1)
    for N in (10, 100, 1000):
        s = math.sqrt(2) * math.sin((N - 1) * math.pi / (2 * N)) / dx
        ratio = (1 / (c * s)) / yee.cfl_dt(dx, dx, c)
        assert ratio > 1 and ratio - 1 < 2.0 / N ** 2 * 3


def test_pec_resonances():
    """Spectral peaks of a long cavity run sit at f_mn = c/2 sqrt((m/a)^2+(n/b)^2)
    up to the O((k dx)^2) dispersion error and the FFT bin width."""
    nx, ny, dx, dy = 24, 16, 0.01, 0.01
    a, b = nx * dx, ny * dy
    dt = 0.95 * yee.cfl_dt(dx, dy, C0)
    nsteps = 8192
    rng = np.random.default_rng(0)
    incr = rng.standard_normal(nsteps) * (np.arange(nsteps) < 4)
    prob = W.Problem("res", nx, ny, dx, dy, dt, np.ones((ny, nx)), np.zeros((ny, nx)), [],
                     [W.Source(W.HZ, 3, 4, 2, 3, incr)], [W.Probe(W.HZ, 17, 11)], nsteps, "f64")
    out = sim.run(prob, [])[:, 0]
    spec = np.abs(np.fft.rfft(out * np.hanning(nsteps)))
    freqs = np.fft.rfftfreq(nsteps, dt)
    df = freqs[1]
    for (m, n) in [(1, 0), (0, 1), (1, 1), (2, 0), (2, 1)]:
        f = C0 / 2 * math.sqrt((m / a) ** 2 + (n / b) ** 2)
        # discrete Yee frequency of the same mode (slightly below f)
        s = C0 * dt * math.sqrt(math.sin(m * math.pi / (2 * nx)) ** 2 / dx ** 2
                                + math.sin(n * math.pi / (2 * ny)) ** 2 / dy ** 2)
        fd = 2 * math.asin(s) / (2 * math.pi * dt)
        lo, hi = int((f * 0.97) / df), int((f * 1.01) / df) + 2
        k = lo + int(np.argmax(spec[lo:hi]))
        # parabolic peak interpolation
        y0, y1, y2 = spec[k - 1], spec[k], spec[k + 1]
        fk = (k + 0.5 * (y0 - y2) / (y0 - 2 * y1 + y2)) * df
        assert abs(fk - fd) < 0.6 * df
        assert abs(fk - f) / f < 0.01


def test_fp32_coefficients_match_formula():
    rng = np.random.default_rng(1)
    er = rng.uniform(1, 10, (9, 11))
    sg = rng.uniform(0, 0.05, (9, 11))
    dt, dx, dy = 2e-11, 0.01, 0.013
    a = yee.edge_coefficients(er, sg, dt, dx, dy, fp32=False)
    b = yee.edge_coefficients(er, sg, dt, dx, dy, fp32=True)
    for u, v in zip(a[:4], b[:4]):
        nz = u != 0
        assert np.max(np.abs(u[nz] - v[nz]) / np.abs(u[nz])) < 3e-7
        assert np.all(v[nz] == v[nz].astype(np.float32))
    # eq. (3) by hand on one edge
    e = EPS0 * 0.5 * (er[3, 4] + er[4, 4])
    s = 0.5 * (sg[3, 4] + sg[4, 4])
    assert a[0][4, 4] == pytest.approx((e / dt - s / 2) / (e / dt + s / 2), rel=1e-14)
    assert a[1][4, 4] == pytest.approx(1 / (e / dt + s / 2) / dy, rel=1e-14)
    assert a[4] == pytest.approx(dt / (MU0 * dy), rel=1e-15)


def test_pec_column_splits_cavity_into_two():
    """A column of PEC cells across a cavity: every edge of those cells stays
    zero and their Hz too, so the one-step map falls apart into the two
    PEC cavities on either side - its non-zero eigenvalues are exactly the
    textbook Yee spectra of those two boxes (walls at the PEC cells' west
    and east faces)."""
    nx, ny, dx, dy = 13, 5, 0.01, 0.012
    c = C0
    dt = 0.9 * yee.cfl_dt(dx, dy, c)
    p = _cavity(nx, ny, dx, dy, dt)
    p.pec = np.zeros((ny, nx), dtype=bool)
    p.pec[:, 6] = True
    M = one_step_matrix(p)
    lam = np.linalg.eigvals(M)
    lam = lam[np.abs(lam) > 1e-6]
    assert np.allclose(np.abs(lam), 1.0, atol=1e-10)
    ang = np.sort(np.abs(np.angle(lam)))
    expect = []
    for sub_nx in (6, 6):
        for m in range(sub_nx):
            for n in range(ny):
                if m == 0 and n == 0:
                    continue
                s = c * dt * math.sqrt(math.sin(m * math.pi / (2 * sub_nx)) ** 2 / dx ** 2
                                       + math.sin(n * math.pi / (2 * ny)) ** 2 / dy ** 2)
                w = 2 * math.asin(s)
                expect += [w, w]
        expect += [0.0] * ((sub_nx - 1) * (ny - 1) + 1)
    expect = np.sort(np.array(expect))
    assert ang.size == expect.size
    assert np.max(np.abs(ang - expect)) < 1e-8
    # and a run keeps the PEC samples at zero
    run = sim.CoupledRun(p, [], init=dict(hz=np.ones((ny, nx)), ex=np.ones((ny + 1, nx)),
                                          ey=np.ones((ny, nx + 1)), x=[]))
    for _ in range(5):
        run.step()
    assert not np.any(run.f.hz[:, 6]) and not np.any(run.f.ey[:, 6:8]) and not np.any(run.f.ex[:, 6])
