"""Batched form on the GPU: several meshes packed block-diagonally into one mesh of segments.  Every
reduction is per segment, so each member must reproduce its standalone run exactly (bit for bit, with
the same Krylov iteration counts per solve), and through that the oracle's run of the member (1e-9).
Also: operators on the packed mesh, per-segment viscosity and reference cells, the adjoint of a
packed window against the members' own adjoints, and the errors of the segment entry points."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg

from gpu_util import ctx, dev, empty, host, note, rel_err

pytestmark = pytest.mark.gpu

DT = 2e-3
BAR = 1e-9


def box_inlet(m, patch="inlet"):
    Fi = m.n_internal_faces
    Ub = np.zeros((m.n_boundary_faces, 3))
    p = m.patch(patch)
    c = m.Cf[p.start:p.start + p.size]
    s = slice(p.start - Fi, p.start - Fi + p.size)
    Ub[s, 0] = 16 * c[:, 1] * (1 - c[:, 1]) * c[:, 2] * (1 - c[:, 2])
    return Ub


def lid(m):
    Fi = m.n_internal_faces
    Ub = np.zeros((m.n_boundary_faces, 3))
    p = m.patch("lid")
    Ub[p.start - Fi:p.start - Fi + p.size, 0] = 1.0
    return Ub


def cases():
    """(mesh, nu, U_b, windkessel rows, capacitor pressures) of the batch members: two cavities with
    different viscosity and jitter (reference cell), one Windkessel channel (fixed pressure)."""
    c1 = mg.cavity(8)
    ch = mg.kuhn_cube(3, jitter=0.15, patches="channel", seed=61, nxyz=(6, 3, 3), hi=(2.0, 1.0, 1.0))
    c2 = mg.cavity(8, seed=77)
    return [(c1, 0.01, lid(c1), np.zeros((0, 3)), np.zeros(0)),
            (ch, 0.01, box_inlet(ch), np.array([[0.4, 0.3, 1.5]]), np.array([0.1])),
            (c2, 0.02, lid(c2), np.zeros((0, 3)), np.zeros(0))]


def make_piso(mesh, Ub, wk, pc0, nu_seg, starts=None, **kw):
    M = B.Mesh(ctx(), mesh, seg_cell_start=starts)
    P = B.Piso(M, B.piso_params(float(nu_seg[0]), DT, **kw))
    if starts is not None:
        P.set_viscosity(nu_seg)
    P.set_boundary(dev(Ub), dev(np.zeros(mesh.n_boundary_faces)))
    for j, (Rp, Cc, Rd) in enumerate(wk):
        P.set_windkessel(j, Rp, Cc, Rd, pc0[j])
    U0 = np.zeros((mesh.n_cells, 3))
    P.set_state(dev(U0), dev(np.zeros(mesh.n_cells)), dev(O.initial_flux(mesh, U0, Ub)))
    return M, P


def packed_case():
    cs = cases()
    P, starts = mg.pack([c[0] for c in cs])
    Ub = np.concatenate([c[2] for c in cs])
    wk = np.concatenate([c[3] for c in cs])
    pc0 = np.concatenate([c[4] for c in cs])
    nu = np.array([c[1] for c in cs])
    return cs, P, starts, Ub, wk, pc0, nu


def split_state(P, k, U, p, phi):
    mb = P.meta["members"][k]
    c = slice(mb["cell_start"], mb["cell_start"] + mb["n_cells"])
    return U[c], p[c], phi[mg.member_faces(P, k)]


def test_packed_piso_equals_members():
    nsteps = 6
    cs, Pm, starts, Ub, wk, pc0, nu = packed_case()
    note("packed piso", Pm.n_cells, "cells", len(cs), "members")
    M, P = make_piso(Pm, Ub, wk, pc0, nu, starts)
    assert M.info["n_segments"] == len(cs)
    seg_its = []
    agg_its = []
    for _ in range(nsteps):
        st, it, _ = P.step(1)
        assert st == 0
        agg_its.append(it[0])
        seg_its.append(P.segment_stats()[0])
    U, p, phi, pc = P.get_state()
    U, p, phi = host(U), host(p), host(phi)
    seg_its = np.array(seg_its)  # [step, member, solve]
    np.testing.assert_array_equal(np.array(agg_its), seg_its.max(axis=1))
    for k, (m, nuk, Ubk, wkk, pck) in enumerate(cs):
        note("member", k, m.name)
        Mk, Pk = make_piso(m, Ubk, wkk, pck, [nuk])
        its = []
        for _ in range(nsteps):
            st, it, _ = Pk.step(1)
            assert st == 0
            its.append(it[0])
        Us, ps, phis, pcs = Pk.get_state()
        Uk, pk, phik = split_state(Pm, k, U, p, phi)
        np.testing.assert_array_equal(Uk, host(Us))
        np.testing.assert_array_equal(pk, host(ps))
        np.testing.assert_array_equal(phik, host(phis))
        w0 = Pm.meta["members"][k]["wk_start"]
        np.testing.assert_array_equal(pc[w0:w0 + len(wkk)], pcs)
        np.testing.assert_array_equal(seg_its[:, k], np.array(its))
        # and the oracle's run of the member
        U0 = np.zeros((m.n_cells, 3))
        ro = O.piso_run(m, O.piso_params(nu=nuk, dt=DT), U0, np.zeros(m.n_cells), O.initial_flux(m, U0, Ubk), Ubk,
                        np.zeros(m.n_boundary_faces), wk=wkk if len(wkk) else None, pc=pck if len(pck) else None,
                        nsteps=nsteps)
        assert rel_err(Uk, ro[0]) <= BAR and rel_err(pk, ro[1]) <= BAR and rel_err(phik, ro[2]) <= BAR
        np.testing.assert_array_equal(seg_its[:, k], ro[4])


def test_packed_operators_equal_members():
    cs, Pm, starts, Ub, _, _, _ = packed_case()
    M = B.Mesh(ctx(), Pm, seg_cell_start=starts)
    rng = np.random.default_rng(11)
    x = rng.standard_normal((Pm.n_cells, 3))
    xb = rng.standard_normal((Pm.n_boundary_faces, 3))
    xi, xbi = M.to_internal(dev(x), B.KIND_CELL), M.to_internal(dev(xb), B.KIND_BFACE)
    g = empty((Pm.n_cells, 9))
    B.difvm_op_grad(M.h, 3, B.BC_U, xi, xbi, g)
    g = host(M.to_user(g, B.KIND_CELL))
    for k, (m, *_r) in enumerate(cs):
        Mk = B.Mesh(ctx(), m)
        mb = Pm.meta["members"][k]
        c = slice(mb["cell_start"], mb["cell_start"] + mb["n_cells"])
        bf = slice(mb["bface_start"] - Pm.n_internal_faces, mb["bface_start"] - Pm.n_internal_faces + m.n_boundary_faces)
        gk = empty((m.n_cells, 9))
        B.difvm_op_grad(Mk.h, 3, B.BC_U, Mk.to_internal(dev(x[c]), B.KIND_CELL),
                        Mk.to_internal(dev(xb[bf]), B.KIND_BFACE), gk)
        np.testing.assert_array_equal(g[c], host(Mk.to_user(gk, B.KIND_CELL)))


def test_packed_adjoint_equals_members():
    """Reverse mode through a packed window: the packed cotangents of the inputs must equal each
    member's own adjoint (the members are independent, every solve is per segment)."""
    nsteps, every, tol = 4, 2, 1e-12
    cs, Pm, starts, Ub, wk, pc0, nu = packed_case()
    rng = np.random.default_rng(5)
    cot = dict(U=rng.standard_normal((Pm.n_cells, 3)), p=rng.standard_normal(Pm.n_cells),
               phi=rng.standard_normal(Pm.n_faces), pc=rng.standard_normal(len(wk)))

    def window(mesh, Ubx, wkx, pcx, nux, st, c):
        M, P = make_piso(mesh, Ubx, wkx, pcx, nux, st, tol_p=tol, tol_u=tol, maxit_p=20000, maxit_u=5000)
        T = B.difvm_tape_create(P.h, nsteps, every)
        s, _ = B.difvm_piso_forward_record(P.h, T, nsteps)
        assert s == 0
        gU, gp, gphi = empty((mesh.n_cells, 3)), empty(mesh.n_cells), empty(mesh.n_faces)
        s, gpc, gwk = B.difvm_piso_adjoint(P.h, T, dev(c["U"]), dev(c["p"]), dev(c["phi"]), c["pc"], tol, gU, gp,
                                           gphi, len(wkx))
        B.difvm_tape_destroy(T)
        assert s == 0
        return host(gU), host(gp), host(gphi), gpc, gwk

    note("packed adjoint", Pm.n_cells)
    gU, gp, gphi, gpc, gwk = window(Pm, Ub, wk, pc0, nu, starts, cot)
    for k, (m, nuk, Ubk, wkk, pck) in enumerate(cs):
        mb = Pm.meta["members"][k]
        c = slice(mb["cell_start"], mb["cell_start"] + mb["n_cells"])
        f = mg.member_faces(Pm, k)
        w = slice(mb["wk_start"], mb["wk_start"] + len(wkk))
        ck = dict(U=cot["U"][c], p=cot["p"][c], phi=cot["phi"][f], pc=cot["pc"][w])
        note("member adjoint", k, m.name)
        sU, sp, sphi, spc, swk = window(m, Ubk, wkk, pck, [nuk], None, ck)
        np.testing.assert_array_equal(gU[c], sU)
        np.testing.assert_array_equal(gp[c], sp)
        np.testing.assert_array_equal(gphi[f], sphi)
        np.testing.assert_array_equal(gpc[w], spc)
        np.testing.assert_array_equal(gwk[w], swk)


def test_segment_errors():
    cs, Pm, starts, Ub, wk, pc0, nu = packed_case()
    with pytest.raises(B.DifvmError) as e:
        B.Mesh(ctx(), Pm, seg_cell_start=np.array([0, 5, Pm.n_cells]))  # cuts through a member
    assert e.value.status == B.ERR_INVALID_MESH
    for bad in ([0, Pm.n_cells - 1], [1, Pm.n_cells], [0, 10, 10, Pm.n_cells]):
        with pytest.raises(B.DifvmError) as e:
            B.Mesh(ctx(), Pm, seg_cell_start=np.array(bad))
        assert e.value.status == B.ERR_INVALID_ARG
    M = B.Mesh(ctx(), Pm, seg_cell_start=starts)
    P = B.Piso(M, B.piso_params(0.01, DT))
    with pytest.raises(B.DifvmError) as e:
        P.set_viscosity([0.01, 0.02])
    assert e.value.status == B.ERR_INVALID_ARG
    with pytest.raises(B.DifvmError) as e:
        P.set_viscosity([0.01, -1.0, 0.02])
    assert e.value.status == B.ERR_INVALID_ARG
    smallest = int(np.diff(starts).min())
    with pytest.raises(B.DifvmError) as e:
        B.Piso(M, B.piso_params(0.01, DT, p_ref_cell=smallest))
    assert e.value.status == B.ERR_INVALID_ARG


def test_handles_destroy_in_any_order():
    """A PISO object keeps its mesh and context alive, a tape its PISO object: dropping the caller's
    handles first must leave the dependent objects working, and the last release frees everything."""
    m, nu, Ub, wk, pc0 = cases()[1]
    cx = B.Context(0)
    mh = B.difvm_mesh_create(cx.h, m)
    ph = B.difvm_piso_create(mh, B.piso_params(nu, DT))
    B.difvm_piso_set_boundary(ph, dev(Ub), dev(np.zeros(m.n_boundary_faces)))
    B.difvm_piso_set_windkessel(ph, 0, *wk[0], pc0[0])
    U0 = np.zeros((m.n_cells, 3))
    B.difvm_piso_set_state(ph, dev(U0), dev(np.zeros(m.n_cells)), None)
    th = B.difvm_tape_create(ph, 2, 1)
    B.difvm_mesh_destroy(mh)
    cx.close()
    st, _ = B.difvm_piso_forward_record(ph, th, 2)
    assert st == 0
    B.difvm_piso_destroy(ph)
    B.difvm_tape_destroy(th)  # last reference: frees tape, PISO object, mesh and context


def single_tet(shift=0.0):
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]]) + 0.1 + shift
    return mg.tet_mesh(P, np.array([[0, 1, 2, 3]]), lambda Cf, tri: np.zeros(Cf.shape[0], int),
                       [("walls", mg.U_FIXED, mg.P_FIXED, -1)], name="tet1")


def test_packed_with_faceless_member_solves_per_segment():
    """A one-cell member (no internal face, its tile holds one cell) packed between two meshes: each
    segment's Laplace solve equals the member's own solve bit for bit, iteration counts included."""
    from gpu_util import empty
    ms = [mg.kuhn_cube(5, jitter=0.15, patches="channel", seed=41), single_tet(),
          mg.kuhn_cube(4, jitter=0.15, patches="channel", seed=42)]
    Pm, starts = mg.pack(ms)
    pbs = [np.linspace(0.0, 1.0, m.n_boundary_faces) for m in ms]
    rhs_extra = [np.random.default_rng(k).standard_normal(m.n_cells) for k, m in enumerate(ms)]

    def solve(mesh, pb, extra, seg):
        M = B.Mesh(ctx(), mesh, seg_cell_start=seg)
        d, u, rhs = empty(mesh.n_cells), empty(max(1, mesh.n_internal_faces)), empty(mesh.n_cells)
        A = B.ldu(d, u)
        B.difvm_ldu_assemble_laplace(M.h, B.BC_P, None, M.to_internal(dev(pb), B.KIND_BFACE), A, rhs)
        b = rhs + M.to_internal(dev(extra), B.KIND_CELL)
        x = empty(mesh.n_cells).zero_()
        st = B.difvm_solve_pcg(M.h, A, b, x, 1e-11, 5000)
        return st, host(M.to_user(x, B.KIND_CELL))

    st, x = solve(Pm, np.concatenate(pbs), np.concatenate(rhs_extra), starts)
    assert st[0] == 0
    its = []
    for k, m in enumerate(ms):
        sk, xk = solve(m, pbs[k], rhs_extra[k], None)
        assert sk[0] == 0
        its.append(sk[1])
        np.testing.assert_array_equal(x[starts[k]:starts[k + 1]], xk)
    assert st[1] == max(its)
