"""Pins of the oracle's CPML layers: exact reduction to the PEC-walled Yee
update when the layers do not absorb; the reflection of a pulse against a
domain large enough that nothing comes back within the window (and, for
contrast, what PEC walls at the same place reflect); decay of the stored
energy once the pulse has left."""
import numpy as np
import pytest

import workloads as W
from oracle import cpml as ocpml
from oracle import sim as osim


def _box(n, nsteps, pml=None, f_bw=1.5e9, eps=None, sigma=None):
    dx = dy = 0.01
    dt = W.courant_dt(dx, dy, 0.99)
    c = n // 2
    src = W.Source(W.HZ, c, c + 1, c, c + 1, W.gaussian_derivative(nsteps, dt, f_bw))
    probes = [W.Probe(W.HZ, c + 15, c), W.Probe(W.HZ, c + 12, c + 12), W.Probe(W.HZ, c, c + 20)]
    eps = np.ones((n, n)) if eps is None else eps
    sigma = np.zeros((n, n)) if sigma is None else sigma
    return W.Problem("box", n, n, dx, dy, dt, eps, sigma, [], [src], probes, nsteps, "f64", pml)


@pytest.fixture(scope="module")
def reference():
    # 300^2 with PEC walls: nothing reflected reaches the probes in 320 steps
    return osim.run(_box(300, 320), [], mode="closed")


def test_non_absorbing_layers_are_the_plain_update():
    p0 = _box(80, 200, W.Pml(10, 10, 10, 10, sigma_scale=0.0, kappa_max=1.0, alpha_max=0.0))
    assert np.array_equal(osim.run(p0, [], mode="closed"), osim.run(_box(80, 200), [], mode="closed"))


def test_reflection_against_unbounded_reference(reference):
    got = osim.run(_box(80, 320, W.Pml(10, 10, 10, 10)), [], mode="closed")
    refl = np.abs(got - reference).max() / np.abs(reference).max()
    assert refl < 1e-4, refl
    pec = osim.run(_box(80, 320), [], mode="closed")
    assert np.abs(pec - reference).max() / np.abs(reference).max() > 0.5


def test_stretched_and_shifted_layers_absorb(reference):
    got = osim.run(_box(80, 320, W.Pml(10, 10, 10, 10, m=4.0, kappa_max=5.0, alpha_max=0.05)), [],
                   mode="closed")
    assert np.abs(got - reference).max() / np.abs(reference).max() < 1e-3


def test_energy_leaves_through_the_layers():
    p = _box(60, 700, W.Pml(8, 8, 8, 8))
    run = osim.CoupledRun(p, [], mode="closed")
    e = []
    for _ in range(700):
        run.step()
        e.append(run.energy())
    assert max(e) > 0 and e[-1] < 1e-6 * max(e)


def test_profiles():
    """Grading: zero outside the layers, monotone into them, a = 0 where
    sigma = 0, and the interior coefficients are exactly the identity."""
    ik_e, b_e, a_e, ik_h, b_h, a_h = ocpml.axis_profiles(50, 0.01, 1e-11, 10, 6, 3.0, 1.0, 3.0, 0.0)
    assert np.all(ik_e[10:45] == 1.0) and np.all(a_e[10:45] == 0.0) and np.all(b_e[10:45] == 1.0)
    assert np.all(ik_h[10:44] == 1.0) and np.all(a_h[10:44] == 0.0)
    assert np.all(np.diff(b_e[:10]) > 0) and np.all(np.diff(ik_e[:10]) > 0)
    assert np.all(np.diff(b_e[44:]) < 0) and np.all(np.diff(ik_e[44:]) < 0)
    assert np.all(a_e[:10] < 0) and np.all((b_e[:10] > 0) & (b_e[:10] < 1))
    assert ik_e[0] == pytest.approx(1.0 / 3.0)
