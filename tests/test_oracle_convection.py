"""Pins of the oracle's higher-order convection schemes (deferred correction, eq. deferred_correction):
linear (central), SOU (eq. sou) and QUICK on top of the implicit upwind face value.
* on a uniform line of cells with the central-difference gradient (which the Gauss gradient is there)
  the face values are the classical stencils: Fromm's phi_C + (phi_D - phi_U)/4 for SOU, Leonard's
  3/8 phi_D + 6/8 phi_C - 1/8 phi_U for QUICK, the mean for linear, for either flow direction;
* for a linear field with its exact gradient SOU reproduces the field at the face centroid and QUICK at
  the midpoint of the two cell centres, on jittered tets with random fluxes;
* linear = the difference of the linear and upwind divergences; the source sums to zero; zero flux
  and upwind add nothing;
* steady oblique advection (the scalar-transport case of Sec. 3.1.2 in miniature) and the Taylor-Green
  vortex at unit amplitude: every higher-order scheme beats first-order upwind, and SOU converges
  faster than upwind."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import meshgen as mg

HO = ["linear", "sou", "quick"]


def line(n, h=0.1):
    return mg.hex_box(n, 1, 1, A=np.diag([n * h, 1.0, 1.0]), patches="walls")


def _expected_line_source(m, conv, phi, F):
    """classical 1D face values on a uniform line; cells whose faces all have a far-upwind cell"""
    pos = np.argsort(np.argsort(m.C[:, 0]))
    cell_at = np.argsort(m.C[:, 0])
    n = m.n_cells
    Fi = m.n_internal_faces
    src = np.zeros(n)
    ok = np.ones(n, bool)
    for f in range(Fi):
        O_, N_ = m.owner[f], m.neighbour[f]
        C_, D_ = (O_, N_) if F[f] >= 0 else (N_, O_)
        u = 2 * pos[C_] - pos[D_]
        if not 0 <= u < n:
            ok[O_] = ok[N_] = False
            continue
        pU, pC, pD = phi[cell_at[u]], phi[C_], phi[D_]
        ho = {"linear": 0.5 * (pC + pD), "sou": pC + 0.25 * (pD - pU), "quick": 0.375 * pD + 0.75 * pC - 0.125 * pU}[conv]
        src[O_] -= F[f] * (ho - pC)
        src[N_] += F[f] * (ho - pC)
    return src, ok


@pytest.mark.parametrize("conv", HO)
@pytest.mark.parametrize("direction", [1.0, -1.0])
def test_uniform_line_gives_classical_stencils(conv, direction):
    m = line(24)
    rng = np.random.default_rng(5)
    phi = rng.standard_normal(m.n_cells)
    # the Gauss gradient of the oracle is the central difference on interior cells of a uniform line
    g = O.grad(m, phi, np.zeros(m.n_boundary_faces), table=O.TABLE_ALL_ZEROGRAD)
    pos = np.argsort(m.C[:, 0])
    cd = (phi[pos[2:]] - phi[pos[:-2]]) / (2 * 0.1)
    assert np.abs(g[pos[1:-1], 0] - cd).max() < 1e-12 * np.abs(cd).max()
    F = direction * (m.Sf @ np.array([1.0, 0.0, 0.0]))
    got = O.deferred_correction(m, conv, F, phi, g)
    want, ok = _expected_line_source(m, conv, phi, F)
    assert ok.sum() >= m.n_cells - 4
    np.testing.assert_allclose(got[ok], want[ok], rtol=0, atol=1e-13 * np.abs(want).max())


@pytest.mark.parametrize("conv", HO)
def test_linear_field_with_exact_gradient(conv):
    """phi = a.x: SOU hits phi(x_f), QUICK phi at the midpoint of C and D, linear the interpolate."""
    m = mg.kuhn_cube(5, jitter=0.15, patches="walls", seed=8)
    rng = np.random.default_rng(6)
    a = np.array([0.4, -1.1, 0.7])
    phi = m.C @ a
    g = np.tile(a, (m.n_cells, 1))
    Fi = m.n_internal_faces
    F = rng.standard_normal(m.n_faces)
    own, nbr = m.owner[:Fi], m.neighbour
    up = F[:Fi] >= 0
    C_ = np.where(up, own, nbr)
    D_ = np.where(up, nbr, own)
    if conv == "sou":
        ho = m.Cf[:Fi] @ a
    elif conv == "quick":
        ho = 0.5 * (m.C[C_] + m.C[D_]) @ a
    else:
        ho = m.w * phi[own] + (1 - m.w) * phi[nbr]
    t = F[:Fi] * (ho - phi[C_])
    want = np.zeros(m.n_cells)
    np.add.at(want, own, -t)
    np.add.at(want, nbr, t)
    got = O.deferred_correction(m, conv, F, phi, g)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_linear_scheme_is_linear_minus_upwind_divergence():
    m = mg.kuhn_cube(5, jitter=0.15, patches="walls", seed=9)
    rng = np.random.default_rng(7)
    F = rng.standard_normal(m.n_faces)
    phi = rng.standard_normal((m.n_cells, 3))
    phib = rng.standard_normal((m.n_boundary_faces, 3))
    g = rng.standard_normal((m.n_cells, 3, 3))
    got = O.deferred_correction(m, "linear", F, phi, g)
    want = -(O.div(m, F, phi, phib, scheme=O.SCHEME_LINEAR) - O.div(m, F, phi, phib, scheme=O.SCHEME_UPWIND))
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("conv", HO + ["upwind"])
def test_source_sums_to_zero_and_vanishes_without_flow(conv):
    m = mg.tube(n=6, m=3, layers=5)
    rng = np.random.default_rng(8)
    F = rng.standard_normal(m.n_faces)
    phi = rng.standard_normal((m.n_cells, 3))
    g = rng.standard_normal((m.n_cells, 3, 3))
    got = O.deferred_correction(m, conv, F, phi, g)
    if conv == "upwind":
        assert not got.any()
        return
    assert np.abs(got.sum(0)).max() < 1e-12 * np.abs(got).sum()
    assert np.abs(got).max() > 0
    assert not O.deferred_correction(m, conv, np.zeros(m.n_faces), phi, g).any()


def _oblique_error(n, conv, steps=60):
    """Steady oblique advection across the unit square, u = (1, 0.5), D = 1e-4: inflow faces (x = 0 and
    y = 0) carry c = g(y - x/2), the outflow is zeroGradient; the exact steady field is g(y - x/2).
    Implicit Euler with a large step marches to the steady state of the deferred-correction scheme."""
    e = ("frontAndBack", mg.U_EMPTY, mg.P_EMPTY, -1)
    sides = {"x0": ("in", mg.U_FIXED, mg.P_ZEROGRAD, -1), "y0": ("in", mg.U_FIXED, mg.P_ZEROGRAD, -1),
             "x1": ("out", mg.U_ZEROGRAD, mg.P_FIXED, -1), "y1": ("out", mg.U_ZEROGRAD, mg.P_FIXED, -1),
             "z0": e, "z1": e}
    m = mg.hex_box(n, n, 1, A=np.diag([1.0, 1.0, 1.0 / n]), patches=sides)
    Fi = m.n_internal_faces

    def g(x):
        return np.exp(-((x[:, 1] - 0.5 * x[:, 0] - 0.3) / 0.12) ** 2)
    phi = m.Sf @ np.array([1.0, 0.5, 0.0])
    cb = g(m.Cf[Fi:])
    c = np.zeros(m.n_cells)
    for _ in range(steps):
        c, it, res, st = O.transport_scalar(m, phi, c, cb, D=1e-4, dt=0.5, table=O.TABLE_U, tol=1e-12, maxit=2000,
                                            conv=conv)
        assert st == 0
    err = c - g(m.C)
    return math.sqrt((m.V * err * err).sum() / m.V.sum())


def test_oblique_advection_higher_order_beats_upwind():
    e = {conv: [_oblique_error(n, conv) for n in (20, 40)] for conv in ["upwind"] + HO}
    for conv in HO:
        assert e[conv][1] < 0.5 * e["upwind"][1], e
    p_up = math.log2(e["upwind"][0] / e["upwind"][1])
    p_sou = math.log2(e["sou"][0] / e["sou"][1])
    assert p_up < 0.9 and p_sou > p_up + 0.4, e


def _taylor_green_unit(n, conv, nu=0.05, dt=0.01, nsteps=20):
    h = math.pi
    m = mg.hex_box(n, n, 1, A=np.diag([h, h, h / n]), origin=(-h / 2, -h / 2, 0.0),
                   patches={s: ("walls", mg.U_FIXED, mg.P_ZEROGRAD, -1) for s in ("x0", "x1", "y0", "y1")}
                   | {s: ("frontAndBack", mg.U_EMPTY, mg.P_EMPTY, -1) for s in ("z0", "z1")})
    Fi = m.n_internal_faces

    def exact(x, t):
        F = math.exp(-2 * nu * t)
        u = np.zeros((x.shape[0], 3))
        u[:, 0] = -np.cos(x[:, 0]) * np.sin(x[:, 1]) * F
        u[:, 1] = np.sin(x[:, 0]) * np.cos(x[:, 1]) * F
        return u
    prm = O.piso_params(nu, dt, tol_p=1e-11, tol_u=1e-11, maxit_p=5000, conv=conv)
    U = exact(m.C, 0.0)
    p = -0.25 * (np.cos(2 * m.C[:, 0]) + np.cos(2 * m.C[:, 1]))
    phi = O.initial_flux(m, U, exact(m.Cf[Fi:], 0.0))
    for k in range(nsteps):
        Ub = exact(m.Cf[Fi:], (k + 1) * dt)
        U, p, phi, pc, it, res, st = O.piso_run(m, prm, U, p, phi, Ub, np.zeros(m.n_boundary_faces), nsteps=1)
        assert st == 0
    e = U - exact(m.C, nsteps * dt)
    return math.sqrt((m.V * (e ** 2).sum(1)).sum() / m.V.sum())


def test_taylor_green_higher_order_beats_upwind():
    """Unit amplitude (Re ~ 60 on the box): upwind's numerical viscosity dominates the error; every
    deferred-correction scheme cuts it, and SOU converges at better than first order."""
    e = {conv: [_taylor_green_unit(n, conv) for n in (16, 32)] for conv in ["upwind"] + HO}
    for conv in HO:
        assert e[conv][1] < 0.5 * e["upwind"][1], e
    assert math.log2(e["sou"][0] / e["sou"][1]) > 1.3, e
