"""Oracle tangent (forward-mode, implicitly differentiated solves; paper eqs. vjp, implicit_diff)
pinned against central finite differences of the oracle's own forward run, and the scalar Windkessel
update against its closed-form derivative."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import meshgen as mg


def wk_channel():
    m = mg.kuhn_cube(3, jitter=0.15, patches="channel", seed=21, nxyz=(5, 3, 3), hi=(2.0, 1.0, 1.0))
    Fi = m.n_internal_faces
    Ub = np.zeros((m.n_boundary_faces, 3))
    inl = m.patch("inlet")
    c = m.Cf[inl.start:inl.start + inl.size]
    Ub[inl.start - Fi:inl.start - Fi + inl.size, 0] = 16 * c[:, 1] * (1 - c[:, 1]) * c[:, 2] * (1 - c[:, 2])
    return m, Ub


def run_state(m, Ub, wk, pc0, U0, p0, phi0, nsteps, prm):
    U, p, phi, pc, it, res, st = O.piso_run(m, prm, U0, p0, phi0, Ub, np.zeros(m.n_boundary_faces), wk=wk,
                                            pc=pc0, nsteps=nsteps)
    assert st == 0
    return np.concatenate([U.ravel(), p, phi, pc])


def test_tangent_matches_central_fd():
    m, Ub = wk_channel()
    prm = O.piso_params(0.05, 0.02, tol_p=1e-13, tol_u=1e-13, maxit_p=5000, maxit_u=2000, tol_tangent=1e-13)
    rng = np.random.default_rng(7)
    U0 = np.zeros((m.n_cells, 3))
    U0[:, 0] = 0.5
    U0 += 0.05 * rng.standard_normal(U0.shape)
    p0 = 0.1 * rng.standard_normal(m.n_cells)
    phi0 = O.initial_flux(m, U0, Ub)
    wk = np.array([[0.4, 0.3, 1.5]])
    pc0 = np.array([0.2])
    nsteps = 4
    dU = rng.standard_normal((1, m.n_cells, 3))
    # directions: Rp, C, Rd, pc0, and a velocity perturbation (with its consistent flux)
    nd = 5
    dwk = np.zeros((nd, 1, 3))
    for k in range(3):
        dwk[k, 0, k] = 1.0
    dpc0 = np.zeros((nd, 1))
    dpc0[3, 0] = 1.0
    dU0 = np.zeros((nd, m.n_cells, 3))
    dU0[4] = dU[0]
    dphi0 = np.zeros((nd, m.n_faces))
    dphi0[4] = O.initial_flux(m, dU[0], np.zeros_like(Ub))   # flux is linear in U
    t = O.piso_tangent(m, prm, U0, p0, phi0, Ub, np.zeros(m.n_boundary_faces), wk, pc0, nsteps,
                       dwk=dwk, dU0=dU0, dphi0=dphi0, dpc0=dpc0)
    tang = np.concatenate([t["tU"].reshape(nd, -1), t["tp"], t["tphi"], t["tpc"]], axis=1)
    base = run_state(m, Ub, wk, pc0, U0, p0, phi0, nsteps, prm)
    np.testing.assert_allclose(np.concatenate([t["U"].ravel(), t["p"], t["phi"], t["pc"]]), base, rtol=0, atol=1e-12)
    for k in range(nd):
        h = 1e-5
        def at(s):
            return run_state(m, Ub, wk + s * h * dwk[k], pc0 + s * h * dpc0[k], U0 + s * h * dU0[k], p0,
                             phi0 + s * h * dphi0[k], nsteps, prm)
        fd = (at(1) - at(-1)) / (2 * h)
        scale = np.abs(fd).max()
        assert scale > 0
        err = np.abs(fd - tang[k]).max() / scale
        assert err < 1e-6, (k, err)


def test_windkessel_scalar_derivative():
    """d p_c(step)/d(Rp, C, Rd) for a held outlet flow Q: p_c' = p_c E + Rd Q (1-E), E = exp(-dt/(Rd C)),
    differentiated by hand, against the oracle tangent after one step from a state with known Q."""
    m, Ub = wk_channel()
    prm = O.piso_params(0.05, 0.02, tol_p=1e-13, tol_u=1e-13, tol_tangent=1e-13)
    U0 = np.zeros((m.n_cells, 3))
    U0[:, 0] = 0.3
    phi0 = O.initial_flux(m, U0, Ub)
    out = m.patch("outlet")
    Q = phi0[out.start:out.start + out.size].sum()
    Rp, Cc, Rd, pcn, dt = 0.4, 0.3, 1.5, 0.2, prm.dt
    wk = np.array([[Rp, Cc, Rd]])
    dwk = np.zeros((3, 1, 3))
    for k in range(3):
        dwk[k, 0, k] = 1.0
    t = O.piso_tangent(m, prm, U0, np.zeros(m.n_cells), phi0, Ub, np.zeros(m.n_boundary_faces), wk,
                       np.array([pcn]), 1, dwk=dwk)
    E = math.exp(-dt / (Rd * Cc))
    dE_dC = E * dt / (Rd * Cc * Cc)
    dE_dRd = E * dt / (Rd * Rd * Cc)
    expect = [0.0, pcn * dE_dC - Rd * Q * dE_dC, pcn * dE_dRd + Q * (1 - E) - Rd * Q * dE_dRd]
    np.testing.assert_allclose(t["tpc"][:, 0], expect, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(t["pc"][0], pcn * E + Rd * Q * (1 - E), rtol=1e-14)


@pytest.mark.parametrize("conv,time", [("upwind", "backward_euler"), ("sou", "crank_nicolson")])
def test_boundary_value_tangent_matches_central_fd(conv, time):
    """Tangent with respect to the fixed velocity boundary values (the inlet profile's amplitude and a
    random perturbation of all fixed faces) against central differences of the forward run."""
    m, Ub = wk_channel()
    prm = O.piso_params(0.05, 0.02, tol_p=1e-13, tol_u=1e-13, maxit_p=5000, maxit_u=2000, tol_tangent=1e-13,
                        conv=conv, time=time)
    rng = np.random.default_rng(8)
    U0 = np.zeros((m.n_cells, 3))
    U0[:, 0] = 0.5
    p0 = np.zeros(m.n_cells)
    phi0 = O.initial_flux(m, U0, Ub)
    wk = np.array([[0.4, 0.3, 1.5]])
    pc0 = np.array([0.2])
    dUb = np.stack([Ub, rng.standard_normal(Ub.shape)])
    t = O.piso_tangent(m, prm, U0, p0, phi0, Ub, np.zeros(m.n_boundary_faces), wk, pc0, 3, dUb=dUb)
    tang = np.concatenate([t["tU"].reshape(2, -1), t["tp"], t["tphi"], t["tpc"]], axis=1)
    for k in range(2):
        h = 1e-5
        fd = (run_state(m, Ub + h * dUb[k], wk, pc0, U0, p0, phi0, 3, prm)
              - run_state(m, Ub - h * dUb[k], wk, pc0, U0, p0, phi0, 3, prm)) / (2 * h)
        scale = np.abs(fd).max()
        assert scale > 0
        assert np.abs(fd - tang[k]).max() / scale < 1e-6, k
