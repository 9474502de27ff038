"""Full-size GPU checks at the workloads' own sizes.
* Channel on the 1,053,696-tet Kuhn cube (the benchmark's PISO workload, autotuned launch shapes as in
  the benchmark): the first step from rest against the oracle on the whole mesh (1e-9, equal Krylov
  counts).
* Tube (2,000,640 tets, Re 500, p = 0 outlet; one oracle step takes minutes here, so properties that
  hold at any size instead): after four steps from rest the net boundary flux vanishes and every
  cell's flux sum is at the level of the pressure solver's tolerance.
* Y-bifurcation (401,484 tets, three Windkessel outlets): gradient of a 64-probe misfit with respect
  to the 9 RCR parameters through the checkpointed window, against central finite differences of the
  GPU forward.  Bar: 1e-5 of the largest component.  The difference quotient carries the forward's
  solver noise divided by the step (tolerance 1e-12 on systems with condition numbers near 1e4 leave
  about 1e-10 relative noise in the loss, and the compliances are near 1e-2), so steps of 1e-4 of
  each parameter keep that noise near 1e-6 while the O(h^2) truncation stays below 1e-8; the exact
  dot-product checks of the adjoint against the oracle's tangent at 1e-9 are in test_gpu_adjoint.py."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg
from paper_2603_15920_amd.autograd import piso_window

from gpu_util import ctx, dev, host, note, rel_err, torch

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def cell_flux_sums(m, phi):
    div = np.bincount(m.owner, weights=phi, minlength=m.n_cells)
    div -= np.bincount(m.neighbour, weights=phi[:m.n_internal_faces], minlength=m.n_cells)
    return div


def test_channel_kuhn56_first_step_vs_oracle():
    m = mg.kuhn_cube(56, jitter=0.15, patches="channel", seed=2603002)
    assert m.n_cells == 1_053_696
    Ub = mg.box_channel_inlet(m)
    q_in = mg.inlet_flow(m, Ub)
    Rd = 1.0 / q_in
    wk = np.array([[Rd / 9.0, 0.1 / Rd, Rd]])
    args = dict(nu=0.005, dt=1e-3, n_corr=2, tol_p=1e-8, tol_u=1e-8, maxit_p=5000, maxit_u=1000)
    U0, p0 = np.zeros((m.n_cells, 3)), np.zeros(m.n_cells)
    phi0 = O.initial_flux(m, U0, Ub)
    pb = np.zeros(m.n_boundary_faces)
    M = B.Mesh(ctx(), m)
    B.difvm_tune(M.h, None)
    P = B.Piso(M, B.piso_params(**args))
    P.set_boundary(dev(Ub), dev(pb))
    P.set_windkessel(0, *wk[0], 0.0)
    P.set_state(dev(U0), dev(p0), dev(phi0))
    note("channel kuhn56: gpu step")
    st, it, _ = P.step(1)
    U, pr, phi, pc = P.get_state()
    note("channel kuhn56: oracle step")
    ro = O.piso_run(m, O.piso_params(**args), U0, p0, phi0, Ub, pb, wk=wk, pc=np.zeros(1), nsteps=1)
    assert st == 0 and ro[6] == 0
    np.testing.assert_array_equal(it, ro[4])
    assert rel_err(host(U), ro[0]) <= 1e-9
    assert rel_err(host(pr), ro[1]) <= 1e-9
    assert rel_err(host(phi), ro[2]) <= 1e-9
    assert rel_err(pc, ro[3]) <= 1e-9


def test_tube_full_size_properties():
    m = mg.tube()  # n = 16, m = 6, 521 layers
    assert m.n_cells == 2_000_640
    Fi = m.n_internal_faces
    Ub = np.zeros((m.n_boundary_faces, 3))
    p = m.patch("inlet")
    Ub[p.start - Fi:p.start - Fi + p.size] = mg.parabolic_inlet(m.Cf[p.start:p.start + p.size], (0, 0, 0), 0.5, 1.0)
    M = B.Mesh(ctx(), m)
    P = B.Piso(M, B.piso_params(1e-3, 1e-3, maxit_p=20000, maxit_u=2000))
    P.set_boundary(dev(Ub), dev(np.zeros(m.n_boundary_faces)))
    P.set_state(dev(np.zeros((m.n_cells, 3))), dev(np.zeros(m.n_cells)), None)
    note("tube", m.n_cells, "cells: 4 gpu steps")
    st, it, _ = P.step(4)
    assert st == 0
    U, pr, phi, _ = P.get_state()
    phi = host(phi)
    q_in = mg.inlet_flow(m, Ub)
    net = phi[Fi:].sum()
    note("tube: net boundary flux", net, "inlet flow", q_in, "pcg", it[-1, 3:].tolist())
    assert abs(net) <= 1e-6 * q_in
    assert np.abs(cell_flux_sums(m, phi)).max() <= 1e-6 * np.abs(phi).max()


def test_ybif_full_size_windkessel_gradient():
    m = mg.ybif(h=0.0519)
    Fi = m.n_internal_faces
    inl = m.patch("inlet")
    Ub = np.zeros((m.n_boundary_faces, 3))
    Ub[inl.start - Fi:inl.start - Fi + inl.size] = mg.parabolic_inlet(m.Cf[inl.start:inl.start + inl.size],
                                                                       (0, 0, 0), 0.5, 1.0)
    wk0 = mg.windkessel_nominal(m, mg.inlet_flow(m, Ub))
    note("ybif full", m.n_cells, "cells")
    M = B.Mesh(ctx(), m)
    P = B.Piso(M, B.piso_params(1e-3, 1e-3, tol_p=1e-12, tol_u=1e-12, maxit_p=20000, maxit_u=5000))
    P.set_boundary(dev(Ub), dev(np.zeros(m.n_boundary_faces)))
    for j in range(3):
        P.set_windkessel(j, *wk0[j], 0.0)
    P.set_state(dev(np.zeros((m.n_cells, 3))), dev(np.zeros(m.n_cells)), None)
    P.step(10)
    U0, p0, phi0, pc0 = P.get_state()
    t = torch()
    rng = np.random.default_rng(2603014)
    theta0 = wk0 * rng.uniform(0.5, 2.0, size=wk0.shape)
    interior = np.ones(m.n_cells, bool)
    interior[m.owner[Fi:]] = False
    probes = t.as_tensor(np.random.default_rng(2603024).choice(np.flatnonzero(interior), 64, replace=False),
                         device="cuda:0")
    target_U = U0[probes] * 1.05
    target_p = p0[probes] + 0.1
    nsteps, every = 6, 3

    def loss_of(theta, grad=False):
        th = t.tensor(theta, dtype=t.float64, requires_grad=grad)
        U, p, phi, pcN = piso_window(P, th, U0, p0, phi0, t.as_tensor(pc0, dtype=t.float64), nsteps, every,
                                     adj_tol=1e-12)
        L = ((U[probes] - target_U) ** 2).sum() + ((p[probes] - target_p) ** 2).sum()
        if grad:
            L.backward()
            return float(L.detach()), th.grad.numpy().copy()
        return float(L.detach()), None

    L0, g = loss_of(theta0, grad=True)
    fd = np.zeros_like(theta0)
    for j in range(3):
        for k in range(3):
            h = 1e-4 * theta0[j, k]
            tp = theta0.copy(); tp[j, k] += h
            tm = theta0.copy(); tm[j, k] -= h
            fd[j, k] = (loss_of(tp)[0] - loss_of(tm)[0]) / (2 * h)
    note("ybif full: grad", g.ravel().tolist(), "fd", fd.ravel().tolist())
    scale = np.abs(fd).max()
    assert scale > 0
    assert np.abs(g - fd).max() <= 1e-5 * scale, (g, fd)
