"""Validity of the benchmark's own configuration and full-size oracle parity.

* Channel on the 1,053,696-tet Kuhn cube exactly as the benchmark runs it (autotuned launch shapes,
  AMG-preconditioned pressure CG, tol 1e-8 for every solve), 5 steps from rest.  The preconditioner
  changes the iterates, so the GPU run and the oracle's Jacobi run stop at different (equally valid)
  solutions.  What is unique is checked instead: for every step, the oracle assembles each linear
  system of the step from the GPU's state before it and the GPU's own solutions (difvm_piso_step_trace)
  and recomputes the true relative residual ||b - A x||_2 / ||b||_2 of the predictor (3 components)
  and of both pressure solves; each must meet the solver tolerance, 1e-8, up to a rounding margin of
  1e-10 (the recursively updated residual the solvers test drifts from the true one by rounding only).
  The state the oracle computes from those solutions must equal the GPU's next state within 1e-9.
* The same run against the oracle's own run at tol 1e-12: the GPU with AMG at tol 1e-12 must match it
  within 1e-9 (the solution is unique up to the tolerance), and the distance of the benchmark's
  tol-1e-8 state from it is reported and bounded (1e-6 relative; it is set by the solver tolerance,
  not by the arithmetic).
* Tube (2,000,640 tets, Re 500, p = 0 outlet, Jacobi): the first 2 steps, each recomputed by the
  oracle from the GPU's solutions (1e-9, true residuals at the tolerance), equal Krylov counts and
  the solver tolerance against the oracle's own run.
* A 50,688-tet tube over 50 steps against the oracle (1e-9, equal Krylov counts)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg

from gpu_util import ctx, dev, host, note, rel_err

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL = 1e-8
RES_MARGIN = 1e-10
PISO_BAR = 1e-9


def _oracle_steps(m, prm, U0, p0, phi0, Ub, pb, nsteps, wk=None, pc=None, label="oracle"):
    """The oracle's run taken one step at a time (each step starts from the state the previous one
    left, as in one call), with a progress line per step."""
    U, p, phi = U0, p0, phi0
    pc = None if wk is None else (np.zeros(len(wk)) if pc is None else pc)
    its = []
    for k in range(nsteps):
        U, p, phi, pc_out, it, _, st = O.piso_run(m, prm, U, p, phi, Ub, pb, wk=wk, pc=pc, nsteps=1)
        if wk is not None:
            pc = pc_out
        its.append(it[0])
        note(f"{label}: oracle step {k} iterations {it[0].tolist()} status {st}")
        if st != 0:
            return U, p, phi, pc_out, np.array(its), st
    return U, p, phi, pc_out, np.array(its), 0


@pytest.fixture(scope="module")
def channel56():
    m = mg.kuhn_cube(56, jitter=0.15, patches="channel", seed=2603002)
    assert m.n_cells == 1_053_696
    Ub = mg.box_channel_inlet(m)
    q_in = mg.inlet_flow(m, Ub)
    Rd = 1.0 / q_in
    wk = np.array([[Rd / 9.0, 0.1 / Rd, Rd]])
    return m, Ub, np.zeros(m.n_boundary_faces), wk


def _channel_piso(m, Ub, pb, wk, tol, precond="amg", tune=True):
    M = B.Mesh(ctx(), m)
    if tune:
        B.difvm_tune(M.h, None)
    P = B.Piso(M, B.piso_params(0.005, 1e-3, tol_p=tol, tol_u=tol, maxit_p=5000, maxit_u=1000, precond=precond))
    P.set_boundary(dev(Ub), dev(pb))
    P.set_windkessel(0, *wk[0], 0.0)
    U0 = np.zeros((m.n_cells, 3))
    P.set_state(dev(U0), dev(np.zeros(m.n_cells)), dev(O.initial_flux(m, U0, Ub)))
    return M, P


@pytest.mark.timeout(900)
def test_headline_channel_every_solve_meets_tolerance(channel56):
    m, Ub, pb, wk = channel56
    M, P = _channel_piso(m, Ub, pb, wk, TOL)
    oprm = O.piso_params(0.005, 1e-3, tol_p=TOL, tol_u=TOL)
    worst = 0.0
    for step in range(5):
        U, p, phi, pc = (host(a) if not isinstance(a, np.ndarray) else a for a in P.get_state())
        st, it, _, Us, pcorr = P.step_trace()
        assert st == 0
        U1, p1, phi1, pc1 = (host(a) if not isinstance(a, np.ndarray) else a for a in P.get_state())
        Uo, po, phio, pco, ru, rp = O.piso_check_step(m, oprm, U, p, phi, Ub, pb, host(Us), host(pcorr), wk=wk,
                                                      pc=pc)
        note(f"headline step {step}: gpu iterations {it.tolist()}, true residuals u {ru.tolist()} p {rp.tolist()}")
        res = np.concatenate([ru, rp])
        assert np.all(res <= TOL + RES_MARGIN), res
        worst = max(worst, res.max())
        for got, ref, name in ((U1, Uo, "U"), (p1, po, "p"), (phi1, phio, "phi"), (pc1, pco, "pc")):
            e = rel_err(got, ref)
            assert e <= PISO_BAR, (step, name, e)
    note(f"headline: largest true relative residual over 5 steps x 5 solves: {worst:.3e}")
    P.close()
    M.close()


@pytest.mark.timeout(900)
def test_headline_channel_against_tight_oracle(channel56):
    m, Ub, pb, wk = channel56
    nsteps = 5
    U0 = np.zeros((m.n_cells, 3))
    phi0 = O.initial_flux(m, U0, Ub)
    note("headline: oracle 5 steps at tol 1e-12 (Jacobi)")
    ro = _oracle_steps(m, O.piso_params(0.005, 1e-3, tol_p=1e-12, tol_u=1e-12, maxit_p=20000, maxit_u=5000), U0,
                       np.zeros(m.n_cells), phi0, Ub, pb, nsteps, wk=wk, pc=np.zeros(1), label="headline")
    assert ro[5] == 0
    out = {}
    for tol in (1e-12, TOL):
        M, P = _channel_piso(m, Ub, pb, wk, tol)
        st, it, _ = P.step(nsteps)
        assert st == 0
        out[tol] = tuple(host(a) if not isinstance(a, np.ndarray) else a for a in P.get_state())
        P.close()
        M.close()
    for k, name in enumerate(("U", "p", "phi", "pc")):
        e_tight = rel_err(out[1e-12][k], ro[k])
        e_head = rel_err(out[TOL][k], ro[k])
        note(f"headline: {name} AMG tol 1e-12 vs oracle {e_tight:.3e}; benchmark (tol 1e-8) vs oracle {e_head:.3e}")
        assert e_tight <= PISO_BAR, (name, e_tight)
        assert e_head <= 1e-6, (name, e_head)


def _tube_inlet(m):
    Fi = m.n_internal_faces
    Ub = np.zeros((m.n_boundary_faces, 3))
    p = m.patch("inlet")
    Ub[p.start - Fi:p.start - Fi + p.size] = mg.parabolic_inlet(m.Cf[p.start:p.start + p.size], (0, 0, 0),
                                                                 m.meta["R"], 1.0)
    return Ub


def _tube_parity(m, nsteps, maxit_p, tol=TOL):
    Ub = _tube_inlet(m)
    pb = np.zeros(m.n_boundary_faces)
    args = dict(nu=1e-3, dt=1e-3, n_corr=2, tol_p=tol, tol_u=tol, maxit_p=maxit_p, maxit_u=2000)
    U0, p0 = np.zeros((m.n_cells, 3)), np.zeros(m.n_cells)
    phi0 = O.initial_flux(m, U0, Ub)
    M = B.Mesh(ctx(), m)
    P = B.Piso(M, B.piso_params(**args))
    P.set_boundary(dev(Ub), dev(pb))
    P.set_state(dev(U0), dev(p0), dev(phi0))
    note(f"tube {m.n_cells} cells: {nsteps} gpu steps")
    st, it, _ = P.step(nsteps)
    U, p, phi, _ = P.get_state()
    note(f"tube {m.n_cells} cells: {nsteps} oracle steps")
    ro = _oracle_steps(m, O.piso_params(**args), U0, p0, phi0, Ub, pb, nsteps, label=f"tube {m.n_cells}")
    note(f"tube {m.n_cells}: pcg counts gpu {it[:, 3:].ravel().tolist()[:8]} oracle {ro[4][:, 3:].ravel().tolist()[:8]}")
    assert st == 0 and ro[5] == 0
    np.testing.assert_array_equal(it, ro[4])
    for got, ref, name in ((host(U), ro[0], "U"), (host(p), ro[1], "p"), (host(phi), ro[2], "phi")):
        e = rel_err(got, ref)
        note(f"tube {m.n_cells}: {name} relative error {e:.3e}")
        assert e <= PISO_BAR, (name, e)


@pytest.mark.timeout(900)
def test_tube_full_size_first_two_steps_vs_oracle():
    """The tube at the configuration's own tolerance (1e-8), Jacobi, first 2 steps.  About 2,000 CG
    iterations per pressure solve amplify rounding: with equal Krylov counts the GPU's pressure and
    the oracle's differ by about 1e-9 relative (1.07e-9 measured), so the step is checked in two parts.
    Every operation of each GPU step is recomputed by the oracle from the GPU's state before it and the
    GPU's own solve solutions (difvm_piso_step_trace): the next state must match within 1e-9 and each
    solution's true relative residual must meet 1e-8 up to the rounding margin.  Against the oracle's
    own run, the Krylov counts must be equal and the states agree within the solver tolerance."""
    m = mg.tube()  # n = 16, m = 6, 521 layers
    assert m.n_cells == 2_000_640
    Ub = _tube_inlet(m)
    pb = np.zeros(m.n_boundary_faces)
    args = dict(nu=1e-3, dt=1e-3, n_corr=2, tol_p=TOL, tol_u=TOL, maxit_p=20000, maxit_u=2000)
    U0, p0 = np.zeros((m.n_cells, 3)), np.zeros(m.n_cells)
    phi0 = O.initial_flux(m, U0, Ub)
    M = B.Mesh(ctx(), m)
    P = B.Piso(M, B.piso_params(**args))
    P.set_boundary(dev(Ub), dev(pb))
    P.set_state(dev(U0), dev(p0), dev(phi0))
    oprm = O.piso_params(**args)
    its = []
    for step in range(2):
        U, p, phi, _ = (host(a) if not isinstance(a, np.ndarray) else a for a in P.get_state())
        st, it, _, Us, pcorr = P.step_trace()
        assert st == 0
        its.append(it)
        U1, p1, phi1, _ = (host(a) if not isinstance(a, np.ndarray) else a for a in P.get_state())
        Uo, po, phio, _, ru, rp = O.piso_check_step(m, oprm, U, p, phi, Ub, pb, host(Us), host(pcorr))
        res = np.concatenate([ru, rp])
        note(f"tube {m.n_cells} step {step}: gpu iterations {it.tolist()}, true residuals {res.tolist()}")
        assert np.all(res <= TOL + RES_MARGIN), res
        for got, ref, name in ((U1, Uo, "U"), (p1, po, "p"), (phi1, phio, "phi")):
            e = rel_err(got, ref)
            note(f"tube {m.n_cells} step {step}: {name} against the oracle's step from the GPU's solutions {e:.3e}")
            assert e <= PISO_BAR, (step, name, e)
    note(f"tube {m.n_cells}: 2 oracle steps")
    ro = _oracle_steps(m, oprm, U0, p0, phi0, Ub, pb, 2, label=f"tube {m.n_cells}")
    assert ro[5] == 0
    np.testing.assert_array_equal(np.array(its), ro[4])
    for got, ref, name in ((U1, ro[0], "U"), (p1, ro[1], "p"), (phi1, ro[2], "phi")):
        e = rel_err(got, ref)
        note(f"tube {m.n_cells}: {name} against the oracle's own run {e:.3e}")
        assert e <= TOL, (name, e)
    P.close()
    M.close()


@pytest.mark.timeout(600)
def test_tube_50k_fifty_steps_vs_oracle():
    # butterfly section n = 8, m = 4 (1,152 tets per layer), 44 layers over L = 2 (axial spacing near
    # the full tube's 0.046)
    m = mg.tube(n=8, m=4, layers=44, L=2.0, seed=2603013)
    assert m.n_cells == 50_688
    _tube_parity(m, 50, 20000)
