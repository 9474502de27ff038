"""GPU PISO steps against the oracle: U, p, phi (and Windkessel p_c) within 1e-9 relative (max norm)
after N steps, with equal Krylov iteration counts in every solve."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg

from gpu_util import ctx, dev, empty, host, note, rel_err, torch

pytestmark = pytest.mark.gpu

PISO_BAR = 1e-9


def inlet_values(m, patch="inlet", kind="parabolic_box"):
    Fi = m.n_internal_faces
    Ub = np.zeros((m.n_boundary_faces, 3))
    p = m.patch(patch)
    c = m.Cf[p.start:p.start + p.size]
    s = slice(p.start - Fi, p.start - Fi + p.size)
    if kind == "parabolic_box":
        Ub[s, 0] = 16 * c[:, 1] * (1 - c[:, 1]) * c[:, 2] * (1 - c[:, 2])
    elif kind == "tube":
        Ub[s] = mg.parabolic_inlet(c, (0, 0, 0), m.meta["R"], 1.0)
    elif kind == "lid":
        Ub[s, 0] = 1.0
    return Ub


def run_both(m, prm_args, Ub, pb, nsteps, wk=None, pc0=None, U0=None):
    """Run nsteps on the oracle and on the GPU from the same state; returns both final states."""
    nc = m.n_cells
    U0 = np.zeros((nc, 3)) if U0 is None else U0
    p0 = np.zeros(nc)
    phi0 = O.initial_flux(m, U0, Ub)
    oprm = O.piso_params(**prm_args)
    ro = O.piso_run(m, oprm, U0, p0, phi0, Ub, pb, wk=wk, pc=pc0, nsteps=nsteps)
    M = B.Mesh(ctx(), m)
    P = B.Piso(M, B.piso_params(**prm_args))
    P.set_boundary(dev(Ub), dev(pb))
    if wk is not None:
        for j, (Rp, Cc, Rd) in enumerate(wk):
            P.set_windkessel(j, Rp, Cc, Rd, pc0[j])
    P.set_state(dev(U0), dev(p0), dev(phi0))
    note("piso", m.name, nsteps)
    status, it, res = P.step(nsteps)
    U, p, phi, pc = P.get_state()
    return ro, (host(U), host(p), host(phi), pc, it, res, status)


def check(ro, rg, m):
    Uo, po, phio, pco, ito, reso, sto = ro
    Ug, pg, phig, pcg, itg, resg, stg = rg
    assert sto == 0 and stg == 0
    np.testing.assert_array_equal(itg, ito)
    assert rel_err(Ug, Uo) <= PISO_BAR, rel_err(Ug, Uo)
    assert rel_err(pg, po) <= PISO_BAR, rel_err(pg, po)
    assert rel_err(phig, phio) <= PISO_BAR, rel_err(phig, phio)
    if len(pco):
        assert rel_err(pcg, pco) <= PISO_BAR


def test_cavity_10_steps():
    """Lid-driven cavity, Re = 100 on 2048 jittered triangles extruded to prisms, nu = 0.01,
    dt = 1e-3, 10 steps, two correctors, tol 1e-8 (the small PISO configuration)."""
    m = mg.cavity()
    ro, rg = run_both(m, dict(nu=0.01, dt=1e-3), inlet_values(m, "lid", "lid"), np.zeros(m.n_boundary_faces), 10)
    check(ro, rg, m)
    assert np.all(rg[0][:, 2] == 0.0)


def test_channel_windkessel():
    m = mg.kuhn_cube(4, jitter=0.15, patches="channel", seed=51, nxyz=(12, 4, 4), hi=(3.0, 1.0, 1.0))
    Ub = inlet_values(m)
    wk = np.array([[0.4, 0.3, 1.5]])
    ro, rg = run_both(m, dict(nu=0.01, dt=5e-3), Ub, np.zeros(m.n_boundary_faces), 6, wk=wk, pc0=np.array([0.1]))
    check(ro, rg, m)


def test_tube_p0_outlet():
    m = mg.tube(n=8, m=4, layers=12, L=3.0)
    Ub = inlet_values(m, "inlet", "tube")
    ro, rg = run_both(m, dict(nu=1e-3, dt=1e-3), Ub, np.zeros(m.n_boundary_faces), 3)
    check(ro, rg, m)


def test_warning_not_converged():
    m = mg.cavity(8)
    Ub = inlet_values(m, "lid", "lid")
    M = B.Mesh(ctx(), m)
    P = B.Piso(M, B.piso_params(0.01, 1e-3, maxit_p=2))
    P.set_boundary(dev(Ub), dev(np.zeros(m.n_boundary_faces)))
    P.set_state(dev(np.zeros((m.n_cells, 3))), dev(np.zeros(m.n_cells)), None)
    status, it, res = P.step(1)
    assert status == B.WARN_NOT_CONVERGED and it[0, 3] == 2
