"""GPU parity of the operator kernels against the oracle (same seeded inputs, user order on both
sides).  Bars: 1e-12 relative (max norm) in FP64, 1e-5 for FP32 kernels on FP32-rounded inputs
against the FP64 oracle on FP64 inputs; where a result cancels (divergence of a near-solenoidal flux)
the bar is 1e-12 times the per-cell sum of |terms|.  Meshes span several 256-cell tiles with a ragged
tail; the full 56^3 Kuhn cube (1,053,696 cells) is run in the launch configuration the benchmark times."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg

from gpu_util import ctx, dev, empty, host, note, rel_err, to_int, to_user, torch

pytestmark = pytest.mark.gpu

F64_BAR, F32_BAR = 1e-12, 1e-5


def single_tet():
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1.0]]) + 0.1
    return mg.tet_mesh(P, np.array([[0, 1, 2, 3]]), lambda Cf, tri: np.zeros(Cf.shape[0], int),
                       [("walls", mg.U_FIXED, mg.P_FIXED, -1)], name="tet1")


MESHES = {
    "kuhn9": lambda: mg.kuhn_cube(9, jitter=0.15, patches="sides", seed=31),        # 4374 cells: 17 tiles + tail
    "cavity": lambda: mg.cavity(),                                                   # 2048 cells, empty patch
    "tube": lambda: mg.tube(n=6, m=3, layers=7),                                    # prisms split to tets
    "hex": lambda: mg.hex_box(13, 11, 7, A=np.array([[1, 0.3, 0.1], [0, 1, 0.2], [0, 0, 1.0]]), patches="sides"),
    "tet1": single_tet,                                                              # no internal face
}
_cache = {}


def get(name):
    if name not in _cache:
        m = MESHES[name]()
        note("mesh", name, m.n_cells, "cells")
        _cache[name] = (m, B.Mesh(ctx(), m))
    return _cache[name]


def fields(m, ncomp, seed):
    fs = [mg.sinusoid_field(seed + c) for c in range(ncomp)]
    Fi = m.n_internal_faces
    phi = np.stack([f(m.C) for f in fs], 1)
    phib = np.stack([f(m.Cf[Fi:]) for f in fs], 1)
    if ncomp == 1:
        return phi[:, 0].copy(), phib[:, 0].copy()
    return phi, phib


@pytest.mark.parametrize("name", sorted(MESHES))
def test_permute_roundtrip(name):
    m, M = get(name)
    t = torch()
    rng = np.random.default_rng(1)
    for kind, n in ((B.KIND_CELL, m.n_cells), (B.KIND_FACE, m.n_faces), (B.KIND_FACE_FLUX, m.n_faces),
                    (B.KIND_BFACE, m.n_boundary_faces)):
        for nc in (1, 3):
            a = rng.standard_normal((n, nc) if nc > 1 else n)
            back = to_user(M, to_int(M, a, kind), kind)
            assert np.array_equal(back, a)
    # a flux changes sign on re-oriented faces, a value does not
    r = B.difvm_mesh_renumber_host(m)
    a = rng.standard_normal(m.n_faces)
    fi = host(M.to_internal(dev(a), B.KIND_FACE_FLUX))[:m.n_internal_faces]
    sg = np.where(r["face_flip"] > 0, -1.0, 1.0)
    assert np.array_equal(fi, sg * a[:m.n_internal_faces][r["face_perm"]])


def _run_op(M, m, op, dtype, *arrays):
    return op(*arrays)


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("ncomp", [1, 3])
@pytest.mark.parametrize("table", [B.BC_ALL_FIXED, B.BC_ALL_ZEROGRAD, B.BC_U, B.BC_P])
def test_interp_grad(name, ncomp, table):
    m, M = get(name)
    phi, phib = fields(m, ncomp, 100)
    ref_f = O.interp(m, phi, phib, table=table)
    ref_g = O.grad(m, phi, phib, table=table)
    t = torch()
    for dt, bar in ((t.float64, F64_BAR), (t.float32, F32_BAR)):
        note("interp/grad", name, ncomp, table, dt)
        p = to_int(M, phi, B.KIND_CELL, dt)
        pb = to_int(M, phib, B.KIND_BFACE, dt)
        out_f = empty(ref_f.shape, dt)
        B.difvm_op_interp(M.h, ncomp, table, p, pb, out_f)
        out_g = empty((m.n_cells, ncomp * 3) if ncomp > 1 else (m.n_cells, 3), dt)
        B.difvm_op_grad(M.h, ncomp, table, p, pb, out_g)
        got_f = to_user(M, out_f, B.KIND_FACE)
        got_g = to_user(M, out_g, B.KIND_CELL).reshape(ref_g.shape)
        assert rel_err(got_f, ref_f) <= bar, (name, dt, rel_err(got_f, ref_f))
        assert rel_err(got_g, ref_g) <= bar, (name, dt, rel_err(got_g, ref_g))


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("scheme", [B.SCHEME_ONE, B.SCHEME_UPWIND, B.SCHEME_LINEAR])
@pytest.mark.parametrize("ncomp", [1, 3])
def test_div(name, scheme, ncomp):
    m, M = get(name)
    U, Ub = fields(m, 3, 200)
    flux = O.initial_flux(m, U, Ub)             # a realistic, nearly cancelling flux
    flux[::5] += 0.01 * np.sin(np.arange(flux[::5].size))
    flux[7::11] = 0.0                          # exercise the upwind tie
    psi, psib = fields(m, ncomp, 300)
    table = B.BC_U if name == "cavity" else B.BC_ALL_FIXED
    ref = O.div(m, flux, psi, psib, scheme=scheme, table=table)
    scale = O.div(m, flux, psi, psib, scheme=scheme, table=table, absterms=True)
    t = torch()
    for dt, bar in ((t.float64, F64_BAR), (t.float32, F32_BAR)):
        note("div", name, scheme, ncomp, dt)
        F = to_int(M, flux, B.KIND_FACE_FLUX, dt)
        ps = to_int(M, psi, B.KIND_CELL, dt)
        pb = to_int(M, psib, B.KIND_BFACE, dt)
        out = empty(ref.shape, dt)
        B.difvm_op_div(M.h, scheme, ncomp, table, F, ps, pb, out)
        got = to_user(M, out, B.KIND_CELL)
        err = np.abs(got - ref) / np.maximum(scale, 1e-300)
        assert err.max() <= bar, (name, dt, err.max())


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("with_gamma", [False, True])
def test_laplacian(name, with_gamma):
    m, M = get(name)
    phi, phib = fields(m, 1, 400)
    g = O.grad(m, phi, phib)
    gamma = 1.0 + 0.5 * np.cos(np.arange(m.n_faces)) if with_gamma else None
    table = B.BC_P if name == "cavity" else B.BC_ALL_FIXED
    ref = O.laplacian(m, phi, g, phib, gamma=gamma, table=table)
    t = torch()
    for dt, bar in ((t.float64, F64_BAR), (t.float32, F32_BAR)):
        note("laplacian", name, with_gamma, dt)
        gm = to_int(M, gamma, B.KIND_FACE, dt) if with_gamma else None
        out = empty(m.n_cells, dt)
        B.difvm_op_laplacian(M.h, table, gm, to_int(M, phi, B.KIND_CELL, dt), to_int(M, g, B.KIND_CELL, dt),
                             to_int(M, phib, B.KIND_BFACE, dt), out)
        got = to_user(M, out, B.KIND_CELL)
        assert rel_err(got, ref) <= bar, (name, dt, rel_err(got, ref))


def random_ldu(m, seed, symmetric=False):
    rng = np.random.default_rng(seed)
    u = -rng.uniform(0.1, 1.0, m.n_internal_faces)
    l = u.copy() if symmetric else -rng.uniform(0.1, 1.0, m.n_internal_faces)
    d = np.zeros(m.n_cells)
    np.add.at(d, m.owner[:m.n_internal_faces], -l)
    np.add.at(d, m.neighbour, -u)
    d += rng.uniform(0.05, 0.5, m.n_cells)
    return d, u, l


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("ncomp", [1, 3])
@pytest.mark.parametrize("transpose", [0, 1])
def test_ldu_spmv(name, ncomp, transpose):
    m, M = get(name)
    d, u, l = random_ldu(m, 5)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((m.n_cells, ncomp)) if ncomp > 1 else rng.standard_normal(m.n_cells)
    ref = O.spmv(m, d, u, l, x, transpose=bool(transpose))
    t = torch()
    for dt, bar in ((t.float64, F64_BAR), (t.float32, F32_BAR)):
        note("spmv", name, ncomp, transpose, dt)
        # a re-oriented face swaps its upper and lower coefficient: permute (u, l) as a pair
        r = B.difvm_mesh_renumber_host(m)
        fl = r["face_flip"].astype(bool)
        ui = np.where(fl, l[r["face_perm"]], u[r["face_perm"]])
        li = np.where(fl, u[r["face_perm"]], l[r["face_perm"]])
        A = B.ldu(to_int(M, d, B.KIND_CELL, dt), dev(ui, dt), dev(li, dt))
        y = empty(x.shape, dt)
        B.difvm_ldu_spmv(M.h, ncomp, transpose, A, to_int(M, x, B.KIND_CELL, dt), y)
        got = to_user(M, y, B.KIND_CELL)
        assert rel_err(got, ref) <= bar, (name, dt, rel_err(got, ref))


def test_determinism_bitwise():
    m, M = get("kuhn9")
    phi, phib = fields(m, 3, 7)
    p, pb = to_int(M, phi, B.KIND_CELL), to_int(M, phib, B.KIND_BFACE)
    outs = []
    for _ in range(3):
        g = empty((m.n_cells, 9))
        B.difvm_op_grad(M.h, 3, B.BC_ALL_FIXED, p, pb, g)
        outs.append(host(g))
    assert all(np.array_equal(outs[0].view(np.uint64), o.view(np.uint64)) for o in outs[1:])


def test_invalid_arguments():
    m, M = get("kuhn9")
    t = torch()
    x = empty(m.n_cells)
    with pytest.raises(B.DifvmError) as e:
        B.difvm_op_grad(M.h, 2, B.BC_ALL_FIXED, x, x, x)
    assert e.value.status == B.ERR_INVALID_ARG
    with pytest.raises(B.DifvmError) as e:
        B.difvm_op_grad(M.h, 1, 9, x, x, x)
    assert e.value.status == B.ERR_INVALID_ARG


@pytest.fixture(scope="module")
def cube56():
    m = mg.kuhn_cube(56, jitter=0.15, patches="walls", seed=2603002)
    note("mesh kuhn56", m.n_cells)
    return m, B.Mesh(ctx(), m)


def test_full_size_operators(cube56):
    """The operator-throughput workload at full size (1,053,696 tets), every output compared."""
    m, M = cube56
    assert (m.n_cells, m.n_internal_faces, m.n_boundary_faces) == (1053696, 2088576, 37632)
    phi, phib = fields(m, 1, 2603012)
    U, Ub = fields(m, 3, 2603013)
    g = O.grad(m, phi, phib)
    flux = O.interp(m, U, Ub)
    flux = np.einsum("fi,fi->f", flux, m.Sf)
    refs = {"grad": g, "lap": O.laplacian(m, phi, g, phib),
            "div": O.div(m, flux, U, Ub, scheme=O.SCHEME_UPWIND),
            "interp": O.interp(m, phi, phib)}
    scale_div = O.div(m, flux, U, Ub, scheme=O.SCHEME_UPWIND, absterms=True)
    t = torch()
    for dt, bar in ((t.float64, F64_BAR), (t.float32, F32_BAR)):
        note("full-size operators", dt)
        p, pb = to_int(M, phi, B.KIND_CELL, dt), to_int(M, phib, B.KIND_BFACE, dt)
        out = empty((m.n_cells, 3), dt)
        B.difvm_op_grad(M.h, 1, B.BC_ALL_FIXED, p, pb, out)
        assert rel_err(to_user(M, out, B.KIND_CELL), refs["grad"]) <= bar
        out = empty(m.n_cells, dt)
        B.difvm_op_laplacian(M.h, B.BC_ALL_FIXED, None, p, to_int(M, g, B.KIND_CELL, dt), pb, out)
        assert rel_err(to_user(M, out, B.KIND_CELL), refs["lap"]) <= bar
        out = empty((m.n_cells, 3), dt)
        B.difvm_op_div(M.h, B.SCHEME_UPWIND, 3, B.BC_ALL_FIXED, to_int(M, flux, B.KIND_FACE_FLUX, dt),
                       to_int(M, U, B.KIND_CELL, dt), to_int(M, Ub, B.KIND_BFACE, dt), out)
        err = np.abs(to_user(M, out, B.KIND_CELL) - refs["div"]) / scale_div
        assert err.max() <= bar
        out = empty(m.n_faces, dt)
        B.difvm_op_interp(M.h, 1, B.BC_ALL_FIXED, p, pb, out)
        assert rel_err(to_user(M, out, B.KIND_FACE), refs["interp"]) <= bar
    # LDU products (plain and transposed, one and three components) at the same size
    d, u, l = random_ldu(m, 5)
    r = B.difvm_mesh_renumber_host(m)
    fl = r["face_flip"].astype(bool)
    ui = np.where(fl, l[r["face_perm"]], u[r["face_perm"]])
    li = np.where(fl, u[r["face_perm"]], l[r["face_perm"]])
    rng = np.random.default_rng(6)
    for ncomp, transpose in ((1, 0), (1, 1), (3, 0)):
        x = rng.standard_normal((m.n_cells, ncomp)) if ncomp > 1 else rng.standard_normal(m.n_cells)
        ref = O.spmv(m, d, u, l, x, transpose=bool(transpose))
        for dt, bar in ((t.float64, F64_BAR), (t.float32, F32_BAR)):
            note("full-size spmv", ncomp, transpose, dt)
            A = B.ldu(to_int(M, d, B.KIND_CELL, dt), dev(ui, dt), dev(li, dt))
            y = empty(x.shape, dt)
            B.difvm_ldu_spmv(M.h, ncomp, transpose, A, to_int(M, x, B.KIND_CELL, dt), y)
            assert rel_err(to_user(M, y, B.KIND_CELL), ref) <= bar, (ncomp, transpose, dt)
