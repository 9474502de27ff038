"""Pins of the oracle's verification step (solutions of the step's linear systems supplied instead of
solved; true residual of each system): it reproduces the solver run when fed that run's solutions,
an independent dense solve of the predictor has a residual at rounding level and leads to the same
state, a zero solution has residual exactly 1, and a one-cell perturbation of a solution raises the
residual by the closed form eps |A e_k| / |b| with A built densely in numpy."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import meshgen as mg


def _dense(m, d, u, l):
    A = np.diag(d.astype(float))
    Fi = m.n_internal_faces
    np.add.at(A, (m.owner[:Fi], m.neighbour), u)
    np.add.at(A, (m.neighbour, m.owner[:Fi]), l)
    return A


@pytest.fixture(scope="module")
def channel():
    """Windkessel channel on a small jittered Kuhn cube, advanced 3 steps from rest (a developed state
    with non-zero outlet flow, so the Windkessel update of the checked step is exercised)."""
    m = mg.kuhn_cube(5, jitter=0.15, patches="channel", seed=7)
    Fi = m.n_internal_faces
    Ub = np.zeros((m.n_boundary_faces, 3))
    inl = m.patch("inlet")
    c = m.Cf[inl.start:inl.start + inl.size]
    Ub[inl.start - Fi:inl.start - Fi + inl.size, 0] = 16 * c[:, 1] * (1 - c[:, 1]) * c[:, 2] * (1 - c[:, 2])
    pb = np.zeros(m.n_boundary_faces)
    wk = np.array([[0.3, 0.05, 2.7]])
    U0 = np.zeros((m.n_cells, 3))
    phi0 = O.initial_flux(m, U0, Ub)
    prm = O.piso_params(0.01, 1e-2, tol_p=1e-13, tol_u=1e-13, maxit_p=5000)
    U, p, phi, pc, _, _, st = O.piso_run(m, prm, U0, np.zeros(m.n_cells), phi0, Ub, pb, wk=wk, pc=np.array([0.1]),
                                         nsteps=3)
    assert st == 0
    return m, Ub, pb, wk, (U, p, phi, pc)


def test_check_step_reproduces_the_solver_run(channel):
    """Fed the solutions the solvers found, the verification step computes the run's next state bit
    for bit, and each system's true residual is the solver's stopping residual up to rounding drift."""
    m, Ub, pb, wk, (U, p, phi, pc) = channel
    for n_corr in (1, 2, 3):
        prm = O.piso_params(0.01, 1e-2, n_corr=n_corr, tol_p=1e-8, tol_u=1e-8)
        U1, p1, phi1, pc1, it, res, st, Us, pcs = O.piso_run(m, prm, U, p, phi, Ub, pb, wk=wk, pc=pc, nsteps=1,
                                                              trace=True)
        assert st == 0 and np.all(it > 0)
        U2, p2, phi2, pc2, ru, rp = O.piso_check_step(m, prm, U, p, phi, Ub, pb, Us[0], pcs[0], wk=wk, pc=pc)
        np.testing.assert_array_equal(U2, U1)
        np.testing.assert_array_equal(p2, p1)
        np.testing.assert_array_equal(phi2, phi1)
        np.testing.assert_array_equal(pc2, pc1)
        np.testing.assert_array_equal(p2, pcs[0, -1])
        assert np.all(np.concatenate([ru, rp]) <= 1e-8 * (1 + 1e-6))
        np.testing.assert_allclose(np.concatenate([ru, rp]), res[0], rtol=1e-5, atol=1e-14)


def test_dense_predictor_solution(channel):
    """An independent predictor solution (numpy dense solve of the momentum system) has a residual at
    rounding level and, with the pressure of a tightly converged single-corrector run, leads to that
    run's state."""
    m, Ub, pb, wk, (U, p, phi, pc) = channel
    prm = O.piso_params(0.01, 1e-2, n_corr=1, tol_p=1e-14, tol_u=1e-14, maxit_p=20000, maxit_u=20000)
    U1, p1, phi1, pc1, _, _, st = O.piso_run(m, prm, U, p, phi, Ub, pb, wk=wk, pc=pc, nsteps=1)
    # momentum system of the step (eq. momentum_predictor, implicit Euler), right side b - V grad p^n
    d, u, l, b = O.assemble_momentum(m, 0.01, 1e-2, phi, U, Ub)
    A = _dense(m, d, u, l)
    # boundary pressure of the step: the Windkessel update from the flux at the start of the step
    out = m.patch("outlet")
    Fi = m.n_internal_faces
    Q = phi[out.start:out.start + out.size].sum()
    Rp, Cc, Rd = wk[0]
    E = np.exp(-1e-2 / (Rd * Cc))
    pcn = pc[0] * E + Rd * Q * (1 - E)
    pbv = pb.copy()
    pbv[out.start - Fi:out.start - Fi + out.size] = pcn + Rp * Q
    assert abs(pc1[0] - pcn) <= 1e-14 * abs(pcn)
    gp = O.grad(m, p, pbv, table=O.TABLE_P)
    rhs = b - m.V[:, None] * gp
    Ud = np.linalg.solve(A, rhs)
    U2, p2, phi2, pc2, ru, rp = O.piso_check_step(m, prm, U, p, phi, Ub, pb, Ud, p1[None, :], wk=wk, pc=pc)
    assert np.all(ru <= 1e-13), ru
    assert rp[0] <= 1e-11, rp
    assert np.abs(U2 - U1).max() <= 1e-10 * np.abs(U1).max()
    assert np.abs(phi2 - phi1).max() <= 1e-10 * np.abs(phi1).max()


def test_residual_closed_forms(channel):
    m, Ub, pb, wk, (U, p, phi, pc) = channel
    prm = O.piso_params(0.01, 1e-2, n_corr=2)
    z3, z = np.zeros((m.n_cells, 3)), np.zeros((2, m.n_cells))
    *_, ru, rp = O.piso_check_step(m, prm, U, p, phi, Ub, pb, z3, z, wk=wk, pc=pc)
    np.testing.assert_array_equal(ru, 1.0)  # x = 0: r = b
    assert rp[0] == 1.0
    # one-cell perturbation eps e_k of the exact predictor solution: |r| = eps |A e_k| (+ rounding)
    d, u, l, b = O.assemble_momentum(m, 0.01, 1e-2, phi, U, Ub)
    A = _dense(m, d, u, l)
    prm_t = O.piso_params(0.01, 1e-2, n_corr=2, tol_p=1e-13, tol_u=1e-14, maxit_u=20000, maxit_p=20000)
    *_, st, Us, pcs = O.piso_run(m, prm_t, U, p, phi, Ub, pb, wk=wk, pc=pc, nsteps=1, trace=True)
    Fi = m.n_internal_faces
    out = m.patch("outlet")
    Q = phi[out.start:out.start + out.size].sum()
    Rp, Cc, Rd = wk[0]
    E = np.exp(-1e-2 / (Rd * Cc))
    pbv = pb.copy()
    pbv[out.start - Fi:out.start - Fi + out.size] = pc[0] * E + Rd * Q * (1 - E) + Rp * Q
    rhs = b - m.V[:, None] * O.grad(m, p, pbv, table=O.TABLE_P)
    for k, comp in ((0, 0), (m.n_cells // 2, 1), (m.n_cells - 1, 2)):
        eps = 1e-3 * np.abs(Us[0]).max()
        Up = Us[0].copy()
        Up[k, comp] += eps
        *_, ru, _ = O.piso_check_step(m, prm, U, p, phi, Ub, pb, Up, pcs[0], wk=wk, pc=pc)
        want = eps * np.linalg.norm(A[:, k]) / np.linalg.norm(rhs[:, comp])
        assert abs(ru[comp] - want) <= 1e-6 * want, (ru[comp], want)
        others = [c for c in range(3) if c != comp]
        assert np.all(ru[others] <= 1e-13)
