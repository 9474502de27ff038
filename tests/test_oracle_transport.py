"""Pins of the oracle's passive-scalar step (implicit Euler, upwind convection of a given face flux,
over-relaxed diffusion; the momentum predictor's discretisation with one transported scalar).
* a discretely divergence-free flux (a uniform velocity dotted with the face areas: each closed cell's
  area vectors sum to zero) keeps a constant field constant;
* with no flow and zeroGradient walls the scalar's integral is conserved and, on orthogonal hexes,
  no new extremum appears;
* pure diffusion of the box's first Dirichlet mode decays at the rate of the continuous problem,
  with the implicit-Euler factor per step, up to an error that falls at second order in h;
* with a uniform flow through a channel, the integral grows by exactly the inflow flux times the time
  until the front reaches the outlet (upwind convection conserves to the solver tolerance)."""
import math

import numpy as np

from oracle import oracle as O
from paper_2603_15920_amd import meshgen as mg


def face_flux(m, u):
    return m.Sf @ np.asarray(u, float)


def test_constant_preserved_by_divergence_free_flux():
    m = mg.kuhn_cube(6, jitter=0.15, patches="walls", seed=12)
    phi = face_flux(m, [1.0, 0.3, -0.2])
    c = np.full(m.n_cells, 2.5)
    cb = np.full(m.n_boundary_faces, 2.5)
    for table in (O.TABLE_ALL_FIXED, O.TABLE_U):
        x, it, res, st = O.transport_scalar(m, phi, c, cb, D=0.01, dt=0.05, table=table, tol=1e-13)
        assert st == 0
        assert np.abs(x - 2.5).max() < 1e-10


def test_closed_box_conserves_and_keeps_bounds():
    m = mg.hex_box(8, 7, 6, patches="walls")
    rng = np.random.default_rng(3)
    c = rng.uniform(0.0, 1.0, m.n_cells)
    phi = np.zeros(m.n_faces)
    cb = np.zeros(m.n_boundary_faces)
    mass0 = (m.V * c).sum()
    x = c
    for _ in range(5):
        x, it, res, st = O.transport_scalar(m, phi, x, cb, D=0.05, dt=0.01, table=O.TABLE_ALL_ZEROGRAD, tol=1e-14)
        assert st == 0
    assert abs((m.V * x).sum() - mass0) <= 1e-12 * mass0
    assert x.max() <= c.max() + 1e-12 and x.min() >= c.min() - 1e-12
    assert x.std() < c.std()   # diffusion smooths


def _mode_decay_error(n, D=0.1, dt=0.002, steps=10):
    m = mg.hex_box(n, n, n, patches="walls")
    s = np.sin(math.pi * m.C[:, 0]) * np.sin(math.pi * m.C[:, 1]) * np.sin(math.pi * m.C[:, 2])
    x = s.copy()
    for _ in range(steps):
        x, it, res, st = O.transport_scalar(m, np.zeros(m.n_faces), x, np.zeros(m.n_boundary_faces), D=D, dt=dt,
                                            table=O.TABLE_ALL_FIXED, tol=1e-14, maxit=2000)
        assert st == 0
    a = (m.V * x * s).sum() / (m.V * s * s).sum()
    exact = (1.0 / (1.0 + dt * 3 * math.pi ** 2 * D)) ** steps
    return abs(a - exact) / exact


def test_diffusion_mode_decay_second_order():
    e8, e16 = _mode_decay_error(8), _mode_decay_error(16)
    assert e16 < 0.01
    assert e8 / e16 > 3.0, (e8, e16)


def test_channel_discrete_mass_balance():
    """Uniform flow through an orthogonal channel (inlet fixed c = 1, zeroGradient outlet and walls):
    every step changes the integral by exactly dt times the boundary fluxes of the new field, the
    convective inflow, the diffusive flux D delta_b (c_b - c_O) at the inlet and the outflow F c_O."""
    e = ("frontAndBack", mg.U_EMPTY, mg.P_EMPTY, -1)
    sides = {"x0": ("inlet", mg.U_FIXED, mg.P_ZEROGRAD, -1), "x1": ("outlet", mg.U_ZEROGRAD, mg.P_FIXED, -1),
             "y0": ("walls", mg.U_ZEROGRAD, mg.P_ZEROGRAD, -1), "y1": ("walls", mg.U_ZEROGRAD, mg.P_ZEROGRAD, -1),
             "z0": e, "z1": e}
    m = mg.hex_box(20, 5, 1, A=np.diag([4.0, 1.0, 0.2]), patches=sides)
    Fi = m.n_internal_faces
    phi = face_flux(m, [1.0, 0.0, 0.0])
    inl, out = m.patch("inlet"), m.patch("outlet")
    cb = np.zeros(m.n_boundary_faces)
    cb[inl.start - Fi:inl.start - Fi + inl.size] = 1.0
    fi = np.arange(inl.start, inl.start + inl.size)
    fo = np.arange(out.start, out.start + out.size)
    d = m.Cf[fi] - m.C[m.owner[fi]]
    S2 = (m.Sf[fi] ** 2).sum(1)
    delta_in = S2 / np.abs((m.Sf[fi] * d).sum(1))   # |S|^2 / (S . d) on the boundary faces
    D, dt = 0.01, 0.05
    x = np.zeros(m.n_cells)
    for step in range(8):
        x0 = x
        x, it, res, st = O.transport_scalar(m, phi, x0, cb, D=D, dt=dt, table=O.TABLE_U, tol=1e-14, maxit=2000)
        if step == 0:
            assert st in (0, O.WARN_BREAKDOWN)   # from c = 0 the first step may break down (same on the GPU)
            x = x0 + 0.0
            x, it, res, st = O.transport_scalar(m, phi, np.full(m.n_cells, 1e-3), cb, D=D, dt=dt, table=O.TABLE_U,
                                                tol=1e-14, maxit=2000)
            x0 = np.full(m.n_cells, 1e-3)
        assert st == 0
        inflow = (-phi[fi] * 1.0 + D * delta_in * (1.0 - x[m.owner[fi]])).sum()
        outflow = (phi[fo] * x[m.owner[fo]]).sum()
        lhs = (m.V * (x - x0)).sum()
        rhs = dt * (inflow - outflow)
        assert abs(lhs - rhs) <= 1e-10 * abs(rhs), (step, lhs, rhs)
