"""Pins of the oracle's time schemes (scheme table: forward Euler, backward Euler, Crank-Nicolson), a
theta-method on the matrix part of the transport operator (theta = 0, 1, 1/2).
* cos(pi x) on a uniform line of cells with zeroGradient ends is an exact eigenvector of the discrete
  Laplacian (the mirror ghost equals the boundary cell), so one diffusion step multiplies it by the
  scheme's amplification factor exactly: 1/(1+z), (1-z/2)/(1+z/2), 1-z with z = D lambda dt;
* forward Euler is the explicit update of eq. momentum_predictor: one scalar step equals
  c + dt/V (-div_upwind(F, c) + D lap(c)) from the oracle's separate operators;
* advection-diffusion with steady boundary values on an orthogonal box (a fixed linear ODE system):
  Crank-Nicolson's time error falls at second order, the Euler schemes' at first;
* PISO steps of the low-amplitude Taylor-Green vortex: backward Euler first order, Crank-Nicolson
  several times more accurate, forward Euler close to backward Euler."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import meshgen as mg


@pytest.mark.parametrize("time", ["backward_euler", "crank_nicolson", "forward_euler"])
def test_cosine_mode_amplification(time):
    n, h, D = 32, 1.0 / 32, 0.3
    m = mg.hex_box(n, 1, 1, A=np.diag([1.0, h, h]), patches="walls")
    c = np.cos(math.pi * m.C[:, 0])
    lam = (2 - 2 * math.cos(math.pi * h)) / h ** 2
    dt = 0.8 / (D * lam)
    z = D * lam * dt
    R = {"backward_euler": 1 / (1 + z), "crank_nicolson": (1 - z / 2) / (1 + z / 2), "forward_euler": 1 - z}[time]
    x, it, res, st = O.transport_scalar(m, np.zeros(m.n_faces), c, np.zeros(m.n_boundary_faces), D=D, dt=dt,
                                        table=O.TABLE_ALL_ZEROGRAD, tol=1e-15, maxit=2000, time=time)
    assert st == 0
    np.testing.assert_allclose(x, R * c, rtol=0, atol=1e-12)


def test_forward_euler_is_the_explicit_update():
    m = mg.kuhn_cube(5, jitter=0.15, patches="walls", seed=21)
    rng = np.random.default_rng(2)
    Fi = m.n_internal_faces
    phi = m.Sf @ np.array([0.7, -0.4, 0.2]) + 0.1 * rng.standard_normal(m.n_faces)
    c = rng.standard_normal(m.n_cells)
    cb = rng.standard_normal(m.n_boundary_faces)
    D, dt = 0.05, 1e-3
    x, it, res, st = O.transport_scalar(m, phi, c, cb, D=D, dt=dt, table=O.TABLE_U, tol=1e-15, maxit=100,
                                        time="forward_euler")
    assert st == 0
    g = O.grad(m, c, cb, table=O.TABLE_U)
    rhs = -O.div(m, phi, c, cb, scheme=O.SCHEME_UPWIND, table=O.TABLE_U) + D * O.laplacian(m, c, g, cb,
                                                                                          table=O.TABLE_U)
    want = c + dt / m.V * rhs
    np.testing.assert_allclose(x, want, rtol=0, atol=1e-12 * np.abs(want).max())
    assert Fi > 0


def _scalar_run(time, dt, T=0.5, n=16):
    """advection-diffusion of a smooth field on an orthogonal box with steady boundary values (inflow
    c = 1 on x = 0, zeroGradient elsewhere), upwind convection of u = (1, 0.4), D = 0.02: a fixed
    linear ODE system in time"""
    e = ("frontAndBack", mg.U_EMPTY, mg.P_EMPTY, -1)
    sides = {"x0": ("in", mg.U_FIXED, mg.P_ZEROGRAD, -1), "y0": ("wall", mg.U_ZEROGRAD, mg.P_ZEROGRAD, -1),
             "x1": ("out", mg.U_ZEROGRAD, mg.P_FIXED, -1), "y1": ("out2", mg.U_ZEROGRAD, mg.P_FIXED, -1),
             "z0": e, "z1": e}
    m = mg.hex_box(n, n, 1, A=np.diag([1.0, 1.0, 1.0 / n]), patches=sides)
    Fi = m.n_internal_faces
    phi = m.Sf @ np.array([1.0, 0.4, 0.0])
    phi[Fi:][phi[Fi:] < 0] *= (m.Cf[Fi:][phi[Fi:] < 0][:, 0] < 1e-12)   # inflow only through x = 0
    cb = np.ones(m.n_boundary_faces)
    c = np.exp(-((m.C[:, 0] - 0.5) ** 2 + (m.C[:, 1] - 0.5) ** 2) / 0.05)
    for _ in range(int(round(T / dt))):
        c, it, res, st = O.transport_scalar(m, phi, c, cb, D=0.02, dt=dt, table=O.TABLE_U, tol=1e-14, maxit=2000,
                                            time=time)
        assert st == 0
    return c, m


def test_scalar_crank_nicolson_second_order_in_time():
    ref, m = _scalar_run("crank_nicolson", 0.5 / 256)

    def err(time, dt):
        c, _ = _scalar_run(time, dt)
        return math.sqrt((m.V * (c - ref) ** 2).sum() / m.V.sum())
    e_cn = [err("crank_nicolson", dt) for dt in (0.05, 0.025)]
    e_be = [err("backward_euler", dt) for dt in (0.05, 0.025)]
    assert math.log2(e_cn[0] / e_cn[1]) > 1.8, e_cn
    assert 0.8 < math.log2(e_be[0] / e_be[1]) < 1.2, e_be
    e_fe = [err("forward_euler", dt) for dt in (0.0125, 0.00625)]   # explicit: within its stability limit
    assert 0.8 < math.log2(e_fe[0] / e_fe[1]) < 1.2, e_fe


def _tg(time, dt, T=0.4, n=16, nu=0.05, amp=0.01):
    h = math.pi
    m = mg.hex_box(n, n, 1, A=np.diag([h, h, h / n]), origin=(-h / 2, -h / 2, 0.0),
                   patches={s: ("walls", mg.U_FIXED, mg.P_ZEROGRAD, -1) for s in ("x0", "x1", "y0", "y1")}
                   | {s: ("frontAndBack", mg.U_EMPTY, mg.P_EMPTY, -1) for s in ("z0", "z1")})
    Fi = m.n_internal_faces

    def exact(x, t):
        F = amp * math.exp(-2 * nu * t)
        u = np.zeros((x.shape[0], 3))
        u[:, 0] = -np.cos(x[:, 0]) * np.sin(x[:, 1]) * F
        u[:, 1] = np.sin(x[:, 0]) * np.cos(x[:, 1]) * F
        return u
    prm = O.piso_params(nu, dt, tol_p=1e-13, tol_u=1e-13, maxit_p=5000, time=time)
    U = exact(m.C, 0.0)
    p = -0.25 * amp * amp * (np.cos(2 * m.C[:, 0]) + np.cos(2 * m.C[:, 1]))
    phi = O.initial_flux(m, U, exact(m.Cf[Fi:], 0.0))
    theta = {"backward_euler": 1.0, "crank_nicolson": 0.5, "forward_euler": 0.0}[time]
    for k in range(int(round(T / dt))):
        # one set of boundary values serves a step: those at t^n + theta dt
        Ub = exact(m.Cf[Fi:], (k + theta) * dt)
        U, p, phi, pc, it, res, st = O.piso_run(m, prm, U, p, phi, Ub, np.zeros(m.n_boundary_faces), nsteps=1)
        assert st == 0
    return U, m


def test_taylor_green_time_errors():
    """PISO steps of the low-amplitude Taylor-Green vortex against a fine-step reference: backward
    Euler's error falls at first order; Crank-Nicolson's is several times smaller (its order on the full
    step is held below two by the step-size dependence of the face flux, whose 1/a_P interpolation has
    no transient term); forward Euler tracks backward Euler."""
    ref, m = _tg("crank_nicolson", 0.4 / 128)

    def err(time, dt):
        U, _ = _tg(time, dt)
        return math.sqrt((m.V * ((U - ref) ** 2).sum(1)).sum() / m.V.sum())
    e_be = [err("backward_euler", dt) for dt in (0.1, 0.05)]
    e_cn = [err("crank_nicolson", dt) for dt in (0.1, 0.05)]
    assert 0.8 < math.log2(e_be[0] / e_be[1]) < 1.2, e_be
    assert e_cn[0] < 0.25 * e_be[0] and e_cn[1] < 0.25 * e_be[1], (e_cn, e_be)
    e_fe = [err("forward_euler", dt) for dt in (0.05, 0.025)]   # stable: nu dt / h^2 <= 0.066
    assert 0.8 < math.log2(e_fe[0] / e_fe[1]) < 1.2, e_fe
    assert 0.5 < e_fe[0] / e_be[1] < 2.0, (e_fe, e_be)
