"""Inverse problem through the differentiable PISO (twin experiment): the series of inlet pressure and
the three capacitor pressures of a run with known Windkessel parameters is the target; Adam on the
log-parameters, starting 20-40 % off, must cut the misfit by two orders of magnitude and at least halve
the distance to the truth of the parameters these observations determine: each outlet's compliance C
and distal resistance Rd set its capacitor pressure's evolution, while the three proximal resistances
reach the data only through one inlet pressure and are not individually identifiable from it.  The
gradient of each iteration comes from the library's discrete adjoint through chained windows.  With the
pressure next to each outlet observed as well, all nine parameters are recovered."""
import numpy as np
import pytest

from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg
from paper_2603_15920_amd.inverse import (fit_windkessel, inlet_pressure_observer, patch_pressure_observer,
                                          simulate_series)

from gpu_util import ctx, dev, note, torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def twin():
    t = torch()
    m = mg.ybif(h=0.2, seed=2603004)
    Fi = m.n_internal_faces
    inl = m.patch("inlet")
    Ub = np.zeros((m.n_boundary_faces, 3))
    Ub[inl.start - Fi:inl.start - Fi + inl.size] = mg.parabolic_inlet(m.Cf[inl.start:inl.start + inl.size],
                                                                       (0, 0, 0), 0.5, 1.0)
    wk_nom = mg.windkessel_nominal(m, mg.inlet_flow(m, Ub))
    M = B.Mesh(ctx(), m)
    P = B.Piso(M, B.piso_params(0.01, 5e-3, tol_p=1e-12, tol_u=1e-12, maxit_p=20000, maxit_u=5000))
    P.set_boundary(dev(Ub), dev(np.zeros(m.n_boundary_faces)))
    for j in range(3):
        P.set_windkessel(j, *wk_nom[j], 0.0)
    P.set_state(dev(np.zeros((m.n_cells, 3))), dev(np.zeros(m.n_cells)), None)
    P.step(10)  # spin-up at the nominal parameters, not differentiated
    U0, p0, phi0, pc0 = P.get_state()
    state0 = (U0, p0, phi0, t.as_tensor(pc0, dtype=t.float64))
    theta_true = t.as_tensor(wk_nom * np.random.default_rng(7).uniform(0.7, 1.4, wk_nom.shape), dtype=t.float64)
    off = np.array([[1.3, 0.7, 1.25], [0.75, 1.35, 0.8], [1.2, 0.8, 1.4]])
    return m, P, state0, theta_true, theta_true.numpy() * off


def run_fit(twin, observe, label):
    t = torch()
    m, P, state0, theta_true, theta0 = twin
    n_windows, steps = 4, 3
    with t.no_grad():
        target = simulate_series(P, theta_true, state0, n_windows, steps, observe).detach()
    note(f"inverse ({label}): ybif", m.n_cells, "cells; target", target.tolist())
    note(f"inverse ({label}): truth", theta_true.numpy().ravel().tolist())
    theta, hist = fit_windkessel(P, theta0, state0, target, n_windows, steps, observe, iters=40, lr=0.05,
                                 adj_tol=1e-12)
    losses = [h[0] for h in hist]
    note(f"inverse ({label}): loss", losses[0], "->", losses[-1], "theta", theta.numpy().ravel().tolist())
    return np.log(theta_true.numpy()), np.log(theta0), np.log(theta.numpy()), losses


def test_windkessel_twin_experiment(twin):
    observe = inlet_pressure_observer(twin[0], with_capacitors=True)
    tt, t0, t1, losses = run_fit(twin, observe, "inlet + capacitors")
    d0 = np.linalg.norm(t0[:, 1:] - tt[:, 1:])
    d1 = np.linalg.norm(t1[:, 1:] - tt[:, 1:])
    note("inverse: (C, Rd) log distance", d0, "->", d1)
    assert losses[-1] <= 1e-2 * losses[0]
    assert d1 < 0.5 * d0


def test_windkessel_all_parameters_with_outlet_pressures(twin):
    """Observing the pressure next to each outlet as well (about pc + Rp Q there) brings the proximal
    resistances into the data: all nine log-parameters together must at least halve their distance
    to the truth, the three proximal resistances included."""
    observe = patch_pressure_observer(twin[0], ("inlet", "A1", "A2", "B"), with_capacitors=True)
    tt, t0, t1, losses = run_fit(twin, observe, "inlet, outlets + capacitors")
    d0, d1 = np.linalg.norm(t0 - tt), np.linalg.norm(t1 - tt)
    r0, r1 = np.linalg.norm(t0[:, 0] - tt[:, 0]), np.linalg.norm(t1[:, 0] - tt[:, 0])
    note("inverse: all-parameter log distance", d0, "->", d1, "; Rp", r0, "->", r1)
    assert losses[-1] <= 1e-2 * losses[0]
    assert d1 < 0.5 * d0
    assert r1 < 0.5 * r0
