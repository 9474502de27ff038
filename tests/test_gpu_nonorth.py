"""GPU parity of the non-orthogonal correction schemes (minimum, orthogonal, none; the default
over-relaxed one is covered by every other GPU test) against the oracle with the same scheme: the
Laplacian operator and its assembly (FP64 1e-12, FP32 1e-5 relative), PISO steps (1e-9, equal
iteration counts) and the discrete adjoint of a window (dot-product test, 1e-9)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg

from gpu_util import ctx, empty, host, note, rel_err, to_int, to_user, torch
from test_gpu_adjoint import channel_wk, check_dot
from test_gpu_piso import check, inlet_values, run_both

pytestmark = pytest.mark.gpu

SCHEMES = ["minimum", "orthogonal", "none"]
F64_BAR, F32_BAR = 1e-12, 1e-5

MESHES = {
    "kuhn9": lambda: mg.kuhn_cube(9, jitter=0.15, patches="sides", seed=31),
    "tube": lambda: mg.tube(n=6, m=3, layers=7),
    "hex": lambda: mg.hex_box(13, 11, 7, A=np.array([[1, 0.3, 0.1], [0, 1, 0.2], [0, 0, 1.0]]), patches="sides"),
}


def fields(m, seed):
    f = mg.sinusoid_field(seed)
    return f(m.C), f(m.Cf[m.n_internal_faces:])


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("scheme", SCHEMES)
def test_laplacian_and_assembly(name, scheme):
    m = MESHES[name]()
    m.meta["nonorth"] = scheme
    note("nonorth laplacian", name, scheme, m.n_cells)
    M = B.Mesh(ctx(), m)
    phi, phib = fields(m, 410)
    g = O.grad(m, phi, phib)
    gamma = 1.0 + 0.5 * np.cos(np.arange(m.n_faces))
    ref = O.laplacian(m, phi, g, phib, gamma=gamma)
    t = torch()
    for dt, bar in ((t.float64, F64_BAR), (t.float32, F32_BAR)):
        out = empty(m.n_cells, dt)
        B.difvm_op_laplacian(M.h, B.BC_ALL_FIXED, to_int(M, gamma, B.KIND_FACE, dt), to_int(M, phi, B.KIND_CELL, dt),
                             to_int(M, g, B.KIND_CELL, dt), to_int(M, phib, B.KIND_BFACE, dt), out)
        got = to_user(M, out, B.KIND_CELL)
        assert rel_err(got, ref) <= bar, (name, scheme, dt, rel_err(got, ref))
    # implicit parts: the Laplacian matrix and the momentum matrix (viscous term) of the same scheme
    r = B.difvm_mesh_renumber_host(m)
    fl, fp = r["face_flip"].astype(bool), r["face_perm"]
    d, u, rbc = O.assemble_laplace(m, phib=phib, gamma=gamma)
    D, Up, R = empty(m.n_cells), empty(m.n_internal_faces), empty(m.n_cells)
    B.difvm_ldu_assemble_laplace(M.h, B.BC_ALL_FIXED, to_int(M, gamma, B.KIND_FACE), to_int(M, phib, B.KIND_BFACE),
                                 B.ldu(D, Up), R)
    assert rel_err(to_user(M, D, B.KIND_CELL), d) <= F64_BAR
    assert rel_err(host(Up), u[fp]) <= F64_BAR
    assert rel_err(to_user(M, R, B.KIND_CELL), rbc) <= F64_BAR
    U = np.stack([mg.sinusoid_field(420 + c)(m.C) for c in range(3)], 1)
    Ub = np.stack([mg.sinusoid_field(420 + c)(m.Cf[m.n_internal_faces:]) for c in range(3)], 1)
    flux = O.initial_flux(m, U, Ub)
    d, u, l, b = O.assemble_momentum(m, 0.01, 1e-3, flux, U, Ub)
    D, Up, Lo, Bv = empty(m.n_cells), empty(m.n_internal_faces), empty(m.n_internal_faces), empty((m.n_cells, 3))
    B.difvm_ldu_assemble_momentum(M.h, 0.01, 1e-3, to_int(M, flux, B.KIND_FACE_FLUX), to_int(M, U, B.KIND_CELL),
                                  to_int(M, Ub, B.KIND_BFACE), B.ldu(D, Up, Lo), Bv)
    assert rel_err(to_user(M, D, B.KIND_CELL), d) <= F64_BAR
    assert rel_err(host(Up), np.where(fl, l[fp], u[fp])) <= F64_BAR
    assert rel_err(host(Lo), np.where(fl, u[fp], l[fp])) <= F64_BAR
    assert rel_err(to_user(M, Bv, B.KIND_CELL), b) <= F64_BAR
    M.close()


def test_schemes_differ_on_the_gpu():
    """the flag reaches the kernels: on jittered tets the four schemes give four different Laplacians"""
    m = MESHES["kuhn9"]()
    phi, phib = fields(m, 411)
    g = O.grad(m, phi, phib)
    outs = []
    for scheme in SCHEMES + ["overrelaxed"]:
        M = B.Mesh(ctx(), m, flags=B.RENUMBER_RCM | B.NONORTH[scheme])
        out = empty(m.n_cells)
        B.difvm_op_laplacian(M.h, B.BC_ALL_FIXED, None, to_int(M, phi, B.KIND_CELL), to_int(M, g, B.KIND_CELL),
                             to_int(M, phib, B.KIND_BFACE), out)
        outs.append(to_user(M, out, B.KIND_CELL))
        M.close()
    for i in range(len(outs)):
        for j in range(i):
            assert rel_err(outs[i], outs[j]) > 1e-6


@pytest.mark.parametrize("scheme", SCHEMES)
def test_piso_channel_windkessel(scheme):
    m = mg.kuhn_cube(4, jitter=0.15, patches="channel", seed=51, nxyz=(12, 4, 4), hi=(3.0, 1.0, 1.0))
    m.meta["nonorth"] = scheme
    ro, rg = run_both(m, dict(nu=0.01, dt=5e-3), inlet_values(m), np.zeros(m.n_boundary_faces), 4,
                      wk=np.array([[0.4, 0.3, 1.5]]), pc0=np.array([0.1]))
    check(ro, rg, m)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_piso_cavity(scheme):
    m = mg.cavity(16)
    m.meta["nonorth"] = scheme
    ro, rg = run_both(m, dict(nu=0.01, dt=1e-3), inlet_values(m, "lid", "lid"), np.zeros(m.n_boundary_faces), 5)
    check(ro, rg, m)


@pytest.mark.parametrize("scheme", ["minimum", "none"])
def test_adjoint_window(scheme):
    m, Ub = channel_wk()
    m.meta["nonorth"] = scheme
    rng = np.random.default_rng(19)
    U0 = np.zeros((m.n_cells, 3)); U0[:, 0] = 0.5
    U0 += 0.05 * rng.standard_normal(U0.shape)
    p0 = 0.1 * rng.standard_normal(m.n_cells)
    phi0 = O.initial_flux(m, U0, Ub)
    check_dot(m, Ub, np.zeros(m.n_boundary_faces), [(0.4, 0.3, 1.5)], np.array([0.2]), U0, p0, phi0,
              nu=0.05, dt=0.02, nsteps=3, every=2)
