"""The smoothed-aggregation AMG preconditioner of the pressure CG.  The preconditioner changes the
iterates, not the solution, so parity is with the oracle's Jacobi-PCG solution of the same system at a
tight tolerance: the GPU solution within 1e-9 relative, the PISO state within 1e-9 (iteration counts
differ by design).  Also: the V-cycle is symmetric and positive definite, it cuts the iteration count,
the hierarchy coarsens, graph mode equals eager bit for bit, and the adjoint's transposed pressure
solves with it pass the dot-product test against the oracle's tangent."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg

from gpu_util import ctx, dev, empty, host, note, rel_err, to_int, to_user, torch
from test_gpu_adjoint import channel_wk, check_dot
from test_gpu_graph import make, run_pair
from test_gpu_piso import inlet_values

pytestmark = pytest.mark.gpu

MESHES = {
    "kuhn12": lambda: mg.kuhn_cube(12, jitter=0.15, patches="walls", seed=2603007),   # 10368 cells
    # 82,944 cells: three levels, so the coarse Chebyshev passes, the A P pass and the restriction that
    # also writes D^-1 b run (two-level hierarchies use none of them)
    "kuhn24": lambda: mg.kuhn_cube(24, jitter=0.15, patches="walls", seed=2603008),
    "tube": lambda: mg.tube(n=8, m=4, layers=12, L=3.0),
    "hex": lambda: mg.hex_box(13, 11, 7, A=np.array([[1, 0.3, 0.1], [0, 1, 0.2], [0, 0, 1.0]]), patches="walls"),
    "cavity": lambda: mg.cavity(32),
}


def laplace_system(m, seed):
    """the SPD Laplacian with Dirichlet boundaries (the pressure operator's form) and a random rhs"""
    phib = np.zeros(m.n_boundary_faces)
    d, u, rbc = O.assemble_laplace(m, phib=phib, table=O.TABLE_ALL_FIXED)
    b = np.random.default_rng(seed).standard_normal(m.n_cells)
    return d, u, b


def device_ldu(M, m, d, u):
    r = B.difvm_mesh_renumber_host(m)
    D = to_int(M, d, B.KIND_CELL)
    Up = dev(u[r["face_perm"]])
    return B.ldu(D, Up)


@pytest.mark.parametrize("name", sorted(MESHES))
def test_pcg_amg_matches_oracle_solution(name):
    m = MESHES[name]()
    M = B.Mesh(ctx(), m)
    d, u, b = laplace_system(m, 5)
    A = device_ldu(M, m, d, u)
    amg = B.difvm_amg_create(M.h, A)
    levels = B.difvm_amg_levels(amg)
    note("amg", name, m.n_cells, levels)
    assert levels[0] == m.n_cells and all(levels[i + 1] < levels[i] for i in range(len(levels) - 1))
    if name == "kuhn24":
        assert len(levels) >= 3, levels
    x = dev(np.zeros(m.n_cells))
    st, it, res = B.difvm_solve_pcg_amg(amg, A, to_int(M, b, B.KIND_CELL), x, 1e-12, 500)
    assert st == 0 and res <= 1e-12
    xo, ito, reso, sto = O.pcg(m, d, u, b, tol=1e-13, maxit=20000)
    assert sto == 0
    assert rel_err(to_user(M, x, B.KIND_CELL), xo) <= 1e-9, rel_err(to_user(M, x, B.KIND_CELL), xo)
    xj = dev(np.zeros(m.n_cells))
    stj, itj, resj = B.difvm_solve_pcg(M.h, A, to_int(M, b, B.KIND_CELL), xj, 1e-12, 20000)
    note("amg iterations", it, "jacobi", itj)
    assert 2 * it <= itj, (it, itj)
    B.difvm_amg_destroy(amg)


@pytest.mark.parametrize("name", ["kuhn12", "kuhn24"])
def test_vcycle_is_symmetric_positive_definite(name):
    m = MESHES[name]()
    M = B.Mesh(ctx(), m)
    d, u, _ = laplace_system(m, 6)
    A = device_ldu(M, m, d, u)
    amg = B.difvm_amg_create(M.h, A)
    rng = np.random.default_rng(7)
    xs = [dev(rng.standard_normal(m.n_cells)) for _ in range(3)]
    zs = []
    for x in xs:
        z = empty(m.n_cells)
        B.difvm_amg_apply(amg, x, z)
        zs.append(host(z))
    xh = [host(x) for x in xs]
    for i in range(3):
        assert (zs[i] * xh[i]).sum() > 0
        for j in range(i):
            a, b2 = (zs[i] * xh[j]).sum(), (zs[j] * xh[i]).sum()
            assert abs(a - b2) <= 1e-12 * np.sqrt((zs[i] ** 2).sum() * (xh[j] ** 2).sum()), (a, b2)
    # deterministic: the same input gives the same bits
    z2 = empty(m.n_cells)
    B.difvm_amg_apply(amg, xs[0], z2)
    assert np.array_equal(host(z2), zs[0])
    with pytest.raises(B.DifvmError):
        B.difvm_amg_apply(amg, xs[0], xs[0])
    B.difvm_amg_destroy(amg)


def test_profile_separates_idle_launches():
    """the benchmark's kernel events with every launch timed: the PCG kernels of iterations 1..k and the
    V-cycles after iterations 0..k count as active, launches queued after the stop as idle"""
    m = MESHES["kuhn12"]()
    cx = ctx()
    M = B.Mesh(cx, m)
    d, u, b = laplace_system(m, 9)
    A = device_ldu(M, m, d, u)
    amg = B.difvm_amg_create(M.h, A)
    x = dev(np.zeros(m.n_cells))
    B.difvm_ctx_profile(cx.h, 1)
    B.difvm_ctx_profile_read(cx.h)
    st, it, res = B.difvm_solve_pcg_amg(amg, A, to_int(M, b, B.KIND_CELL), x, 1e-10, 500)
    prof = B.difvm_ctx_profile_read(cx.h)
    B.difvm_ctx_profile(cx.h, 0)
    note("profile", it, prof)
    assert st == 0
    assert prof["pcg_spmv_dot"][0] == it and prof["pcg_update_dot"][0] == it
    assert prof["pcg_amg_vcycle"][0] == it + 1
    assert prof["pcg_spmv_dot (idle)"][0] >= 1   # at least the launch that finds the stop
    B.difvm_amg_destroy(amg)


def test_poisson_mms_with_amg():
    """the paper's Poisson case at 34,992 cells: the AMG-preconditioned solve reaches the same discrete
    solution (and so the same error against the manufactured solution) as Jacobi"""
    m = mg.kuhn_cube(18, jitter=0.15, patches="walls", seed=2603007)
    M = B.Mesh(ctx(), m)
    phib = mg.poisson_mms_solution(m.Cf[m.n_internal_faces:])
    d, u, rbc = O.assemble_laplace(m, phib=phib)
    N = O.laplacian(m, np.zeros(m.n_cells), mg.poisson_mms_gradient(m.C), phib) - rbc
    rhs = rbc + N - m.V * mg.poisson_mms_source(m.C)
    A = device_ldu(M, m, d, u)
    amg = B.difvm_amg_create(M.h, A)
    x = dev(np.zeros(m.n_cells))
    st, it, res = B.difvm_solve_pcg_amg(amg, A, to_int(M, rhs, B.KIND_CELL), x, 1e-12, 500)
    xo, ito, reso, sto = O.pcg(m, d, u, rhs, tol=1e-12, maxit=20000)
    note("poisson amg", it, "oracle jacobi", ito)
    assert st == 0 and sto == 0 and it * 3 <= ito
    assert rel_err(to_user(M, x, B.KIND_CELL), xo) <= 1e-9
    B.difvm_amg_destroy(amg)


def run_pair_oracle(m, prm, Ub, pb, nsteps, wk=None, pc0=None):
    nc = m.n_cells
    U0, p0 = np.zeros((nc, 3)), np.zeros(nc)
    phi0 = O.initial_flux(m, U0, Ub)
    ro = O.piso_run(m, O.piso_params(**prm), U0, p0, phi0, Ub, pb, wk=wk, pc=pc0, nsteps=nsteps)
    M = B.Mesh(ctx(), m)
    P = B.Piso(M, B.piso_params(**prm, precond="amg"))
    P.set_boundary(dev(Ub), dev(pb))
    if wk is not None:
        for j, (Rp, Cc, Rd) in enumerate(wk):
            P.set_windkessel(j, Rp, Cc, Rd, pc0[j])
    P.set_state(dev(U0), dev(p0), dev(phi0))
    note("piso amg", m.name, nsteps)
    status, it, res = P.step(nsteps)
    U, p, phi, pc = P.get_state()
    assert status == 0 and ro[6] == 0
    assert rel_err(host(U), ro[0]) <= 1e-9, rel_err(host(U), ro[0])
    assert rel_err(host(p), ro[1]) <= 1e-9, rel_err(host(p), ro[1])
    assert rel_err(host(phi), ro[2]) <= 1e-9, rel_err(host(phi), ro[2])
    if wk is not None:
        assert rel_err(pc, ro[3]) <= 1e-9
    # pressure iterations: AMG well below the oracle's Jacobi counts
    assert it[:, 3:].max() * 3 <= ro[4][:, 3:].max(), (it[:, 3:], ro[4][:, 3:])
    return P


def test_piso_cavity_reference_cell():
    m = mg.cavity(16)
    run_pair_oracle(m, dict(nu=0.01, dt=1e-3, tol_p=1e-12, tol_u=1e-12, maxit_p=5000),
                    inlet_values(m, "lid", "lid"), np.zeros(m.n_boundary_faces), 6)


def test_piso_channel_windkessel():
    m = mg.kuhn_cube(4, jitter=0.15, patches="channel", seed=51, nxyz=(12, 4, 4), hi=(3.0, 1.0, 1.0))
    run_pair_oracle(m, dict(nu=0.01, dt=5e-3, tol_p=1e-12, tol_u=1e-12, maxit_p=5000), inlet_values(m),
                    np.zeros(m.n_boundary_faces), 5, wk=np.array([[0.4, 0.3, 1.5]]), pc0=np.array([0.1]))


def test_piso_tube_and_rebuild():
    m = mg.tube(n=8, m=4, layers=12, L=3.0)
    P = run_pair_oracle(m, dict(nu=1e-3, dt=1e-3, tol_p=1e-12, tol_u=1e-12, maxit_p=5000),
                        inlet_values(m, "inlet", "tube"), np.zeros(m.n_boundary_faces), 3)
    B.difvm_piso_rebuild_preconditioner(P.h)
    status, it, res = P.step(2)
    assert status == 0


def test_adjoint_window_with_amg():
    m, Ub = channel_wk()
    rng = np.random.default_rng(37)
    U0 = np.zeros((m.n_cells, 3)); U0[:, 0] = 0.5
    U0 += 0.05 * rng.standard_normal(U0.shape)
    p0 = 0.1 * rng.standard_normal(m.n_cells)
    phi0 = O.initial_flux(m, U0, Ub)
    check_dot(m, Ub, np.zeros(m.n_boundary_faces), [(0.4, 0.3, 1.5)], np.array([0.2]), U0, p0, phi0,
              nu=0.05, dt=0.02, nsteps=4, every=3, precond="amg")


def test_graph_equals_eager_amg():
    m = mg.cavity(16)
    Ub = inlet_values(m, "lid", "lid")
    _, Pe = make(m, Ub, 0.01, 1e-3, precond="amg")
    _, Pg = make(m, Ub, 0.01, 1e-3, precond="amg")
    Pg.set_graph(True, 4)
    note("graph amg", m.n_cells)
    run_pair(Pe, Pg, 6)
    replays, redos, captures = Pg.graph_info()
    assert captures >= 1 and replays + redos == 5


def test_amg_errors():
    m = mg.cavity(8)
    M = B.Mesh(ctx(), m)
    P = B.Piso(M, B.piso_params(0.01, 1e-3))
    with pytest.raises(B.DifvmError) as e:
        B.difvm_piso_rebuild_preconditioner(P.h)
    assert e.value.status == B.ERR_INVALID_ARG
    prm = B.piso_params(0.01, 1e-3)
    prm.precond = 2
    with pytest.raises(B.DifvmError):
        B.Piso(M, prm)


def test_vcycle_is_block_diagonal_on_a_packed_mesh():
    """no aggregate crosses a member, the coarsest dense inverse keeps the blocks' exact zeros: a residual
    on one member of a packed mesh leaves the V-cycle's output exactly zero on the other"""
    a = mg.kuhn_cube(10, jitter=0.15, patches="walls", seed=61)
    b = mg.kuhn_cube(8, jitter=0.15, patches="walls", seed=62)
    packed, starts = mg.pack([a, b])
    M = B.Mesh(ctx(), packed, seg_cell_start=starts)
    d, u, _ = laplace_system(packed, 3)
    A = device_ldu(M, packed, d, u)
    amg = B.difvm_amg_create(M.h, A)
    note("packed levels", B.difvm_amg_levels(amg))
    rng = np.random.default_rng(11)
    for k in range(2):
        mb = packed.meta["members"][k]
        cs = slice(mb["cell_start"], mb["cell_start"] + mb["n_cells"])
        r = np.zeros(packed.n_cells)
        r[cs] = rng.standard_normal(mb["n_cells"])
        z = empty(packed.n_cells)
        B.difvm_amg_apply(amg, to_int(M, r, B.KIND_CELL), z)
        zu = to_user(M, z, B.KIND_CELL)
        other = np.ones(packed.n_cells, bool)
        other[cs] = False
        assert np.all(zu[other] == 0.0), k
        assert (zu[cs] * r[cs]).sum() > 0
    B.difvm_amg_destroy(amg)


def test_packed_members_with_amg():
    """a batch of three uneven members under one AMG hierarchy: each member's state after 4 steps equals
    the oracle's run of that member alone within 1e-9 (tolerances 1e-12), every member converging"""
    a = mg.cavity(16)
    b = mg.kuhn_cube(4, jitter=0.15, patches="channel", seed=51, nxyz=(12, 4, 4), hi=(3.0, 1.0, 1.0))
    c = mg.cavity(8)
    wk_b = np.array([[0.4, 0.3, 1.5]])
    members = [(a, inlet_values(a, "lid", "lid"), 0.01, None), (b, inlet_values(b), 0.02, wk_b),
               (c, inlet_values(c, "lid", "lid"), 0.005, None)]
    packed, starts = mg.pack([x[0] for x in members])
    Ub = np.concatenate([x[1] for x in members])
    M = B.Mesh(ctx(), packed, seg_cell_start=starts)
    P = B.Piso(M, B.piso_params(0.01, 1e-3, tol_p=1e-12, tol_u=1e-12, maxit_p=5000, precond="amg"))
    P.set_viscosity(np.array([x[2] for x in members]))
    P.set_boundary(dev(Ub), dev(np.zeros(packed.n_boundary_faces)))
    P.set_windkessel(0, *wk_b[0], 0.1)           # the only Windkessel of the batch (member b's)
    P.set_state(dev(np.zeros((packed.n_cells, 3))), dev(np.zeros(packed.n_cells)), None)
    note("packed amg", packed.n_cells)
    status, it, res = P.step(4)
    assert status == 0
    Ut, pt_, phit, pc = P.get_state()
    U, p = host(Ut), host(pt_)
    for k, (m, Ubm, nu, wk) in enumerate(members):
        mb = packed.meta["members"][k]
        cs = slice(mb["cell_start"], mb["cell_start"] + mb["n_cells"])
        prm = O.piso_params(nu, 1e-3, tol_p=1e-12, tol_u=1e-12, maxit_p=5000)
        U0 = np.zeros((m.n_cells, 3))
        ro = O.piso_run(m, prm, U0, np.zeros(m.n_cells), O.initial_flux(m, U0, Ubm), Ubm,
                        np.zeros(m.n_boundary_faces), wk=wk, pc=None if wk is None else np.array([0.1]), nsteps=4)
        assert ro[6] == 0
        assert rel_err(U[cs], ro[0]) <= 1e-9, (k, rel_err(U[cs], ro[0]))
        assert rel_err(p[cs], ro[1]) <= 1e-9, (k, rel_err(p[cs], ro[1]))
