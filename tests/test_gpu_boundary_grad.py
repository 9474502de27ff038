"""Gradient with respect to the fixed velocity boundary values (difvm_tape_boundary_cotangent) and the
lid-velocity inverse problem built on it (Sec. 3.3.1).
* dot-product test of the window: <cotangent of the final state, oracle tangent along dU_b> equals
  <boundary cotangent from the GPU adjoint, dU_b> within 1e-9, for the inlet profile's amplitude and a
  random perturbation of every fixed face, under the default schemes and under SOU + Crank-Nicolson;
* the autograd window returns the same boundary gradient;
* lid-velocity recovery (synthetic twin): 10 random probe cells of the jittered cavity (512 cells, 30
  steps), truth U_lid = 2, start 0.5, Adam (learning rate 0.1, first-moment decay 0.7) on the lid speed,
  40 iterations; the fit must end within 1 % of the truth."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg
from paper_2603_15920_amd.autograd import piso_window
from paper_2603_15920_amd.inverse import fit_boundary_scale

from gpu_util import ctx, dev, empty, host, note, torch
from test_gpu_adjoint import channel_wk

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("conv,time", [("upwind", "backward_euler"), ("sou", "crank_nicolson")])
def test_boundary_cotangent_dot_product(conv, time):
    m, Ub = channel_wk()
    nc, nf, nfb = m.n_cells, m.n_faces, m.n_boundary_faces
    rng = np.random.default_rng(41)
    U0 = np.zeros((nc, 3)); U0[:, 0] = 0.5
    U0 += 0.05 * rng.standard_normal(U0.shape)
    p0 = 0.1 * rng.standard_normal(nc)
    phi0 = O.initial_flux(m, U0, Ub)
    wk, pc0 = np.array([[0.4, 0.3, 1.5]]), np.array([0.2])
    nu, dt, nsteps = 0.05, 0.02, 4
    cot = dict(U=rng.standard_normal((nc, 3)), p=rng.standard_normal(nc), phi=rng.standard_normal(nf),
               pc=rng.standard_normal(1))
    M = B.Mesh(ctx(), m)
    P = B.Piso(M, B.piso_params(nu, dt, tol_p=1e-13, tol_u=1e-13, maxit_p=20000, maxit_u=5000, conv=conv, time=time))
    P.set_boundary(dev(Ub), dev(np.zeros(nfb)))
    P.set_windkessel(0, *wk[0], pc0[0])
    P.set_state(dev(U0), dev(p0), dev(phi0))
    T = B.difvm_tape_create(P.h, nsteps, 3)
    with pytest.raises(B.DifvmError):
        B.difvm_tape_boundary_cotangent(T, empty((nfb, 3)))          # no adjoint yet
    st, it = B.difvm_piso_forward_record(P.h, T, nsteps)
    assert st == 0
    note("boundary adjoint", conv, time)
    st, gpc0, gwk = B.difvm_piso_adjoint(P.h, T, dev(cot["U"]), dev(cot["p"]), dev(cot["phi"]), cot["pc"], 1e-13,
                                         None, None, None, 1)
    assert st == 0
    gUb = empty((nfb, 3))
    B.difvm_tape_boundary_cotangent(T, gUb)
    B.difvm_tape_destroy(T)
    gUb = host(gUb)
    fixed = np.zeros(nfb, bool)
    for pt in m.patches:
        if pt.u_type == mg.U_FIXED:
            fixed[pt.start - m.n_internal_faces:pt.start - m.n_internal_faces + pt.size] = True
    assert not gUb[~fixed].any()
    dUb = np.stack([Ub, rng.standard_normal(Ub.shape) * fixed[:, None]])
    prm = O.piso_params(nu, dt, tol_p=1e-13, tol_u=1e-13, maxit_p=20000, maxit_u=5000, tol_tangent=1e-13,
                        conv=conv, time=time)
    t = O.piso_tangent(m, prm, U0, p0, phi0, Ub, np.zeros(nfb), wk, pc0, nsteps, dUb=dUb)
    for k in range(2):
        lhs = ((cot["U"] * t["tU"][k]).sum() + (cot["p"] * t["tp"][k]).sum() + (cot["phi"] * t["tphi"][k]).sum()
               + (cot["pc"] * t["tpc"][k]).sum())
        rhs = (gUb * dUb[k]).sum()
        assert abs(lhs - rhs) <= 1e-9 * max(abs(lhs), abs(rhs)), (k, lhs, rhs)


def cavity_case(n=32):
    m = mg.cavity(n)
    Fi = m.n_internal_faces
    lid = m.patch("lid")
    pattern = np.zeros((m.n_boundary_faces, 3))
    pattern[lid.start - Fi:lid.start - Fi + lid.size, 0] = 1.0
    return m, pattern


def test_autograd_boundary_gradient_matches_tape():
    m, pattern = cavity_case(16)
    t = torch()
    M = B.Mesh(ctx(), m)
    P = B.Piso(M, B.piso_params(0.01, 5e-3, tol_p=1e-12, tol_u=1e-12))
    U0 = t.zeros((m.n_cells, 3), dtype=t.float64, device="cuda:0")
    p0 = t.zeros(m.n_cells, dtype=t.float64, device="cuda:0")
    phi0 = dev(O.initial_flux(m, np.zeros((m.n_cells, 3)), pattern))
    s = t.tensor(1.3, dtype=t.float64, requires_grad=True)
    Ub = s.to("cuda:0") * dev(pattern)
    theta = t.zeros((0, 3), dtype=t.float64)
    pc0 = t.zeros(0, dtype=t.float64)
    U, p, phi, pc = piso_window(P, theta, U0, p0, phi0, pc0, 12, 5, 1e-12, Ub=Ub)
    w = dev(np.random.default_rng(3).standard_normal((m.n_cells, 3)))
    (U * w).sum().backward()
    g_auto = float(s.grad)
    # central difference of the same scalar through plain steps
    def J(v):
        P.set_boundary(dev(v * pattern), None)
        P.set_state(U0, p0, phi0)
        P.step(12)
        return float((P.get_state()[0] * w).sum())
    h = 1e-4
    fd = (J(1.3 + h) - J(1.3 - h)) / (2 * h)
    assert abs(g_auto - fd) <= 1e-6 * abs(fd), (g_auto, fd)


def test_lid_velocity_recovery():
    m, pattern = cavity_case(16)
    t = torch()
    M = B.Mesh(ctx(), m)
    P = B.Piso(M, B.piso_params(0.01, 5e-3, tol_p=1e-10, tol_u=1e-10))
    nsteps = 30
    U0 = t.zeros((m.n_cells, 3), dtype=t.float64, device="cuda:0")
    p0 = t.zeros(m.n_cells, dtype=t.float64, device="cuda:0")
    phi0 = dev(np.zeros(m.n_faces))           # at rest; the lid is tangential, so its flux is zero
    pc0 = t.zeros(0, dtype=t.float64)
    # synthetic truth: U_lid = 2
    P.set_boundary(dev(2.0 * pattern), dev(np.zeros(m.n_boundary_faces)))
    P.set_state(U0, p0, phi0)
    P.step(nsteps)
    U_true = host(P.get_state()[0])
    probes = np.random.default_rng(2603).choice(m.n_cells, 10, replace=False)
    target = U_true[probes]
    note("lid recovery", m.n_cells, nsteps)
    s, hist = fit_boundary_scale(P, pattern, 0.5, (U0, p0, phi0, pc0), probes, target, nsteps, iters=40, lr=0.1,
                                 ckpt_every=10, adj_tol=1e-10)
    first = next(k for k, h in enumerate(hist) if abs(h[1] - 2.0) < 0.02)
    note("lid recovery: s", s, "first within 1 % at iteration", first, "losses", hist[0][0], hist[-1][0])
    assert abs(s - 2.0) < 0.02, hist[-5:]
    assert hist[-1][0] < 1e-3 * hist[0][0], (hist[0], hist[-1])
