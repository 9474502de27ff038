"""Halo exchange on one GPU: every part of a slab partition runs the operators on its own cells plus
ghost copies, and its owned rows must equal the whole mesh's rows bit for bit (bitwise equality of
the device results; the whole-mesh operators are pinned to the oracle in test_gpu_ops.py).

The exchange is the real pattern of one GPU per part: pack on every part (difvm_halo_pack), move
each send segment to the receiving part's receive buffer (a device copy standing in for the
transfer between GPUs), unpack (difvm_halo_unpack).  Chained as an operator sequence would be:
exchange phi -> gradient -> exchange the gradient -> Laplacian; exchange U -> interpolation,
vector upwind divergence; exchange x -> LDU products (symmetric and not, 1 and 3 components)."""
import numpy as np
import pytest

from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg

from gpu_util import ctx, note, to_int, torch

pytestmark = pytest.mark.gpu


def _fields(m, ncomp, seed):
    fs = [mg.sinusoid_field(seed + c) for c in range(ncomp)]
    Fi = m.n_internal_faces
    phi = np.stack([f(m.C) for f in fs], 1)
    phib = np.stack([f(m.Cf[Fi:]) for f in fs], 1)
    return (phi[:, 0].copy(), phib[:, 0].copy()) if ncomp == 1 else (phi, phib)


class Halo:
    """All parts of a partition on one GPU, with their exchange buffers."""

    def __init__(self, m, n_parts):
        t = torch()
        self.P = B.Partition(m, n_parts)
        self.parts = [B.PartMesh(ctx(), self.P, p) for p in range(n_parts)]
        self.idx = [{k: t.from_numpy(v.astype(np.int64)).cuda() for k, v in pm.maps.items()} for pm in self.parts]

    def local_cells(self, p, x_whole, fill_ghosts=np.nan):
        """owned rows from the whole mesh's array, ghost rows poisoned (the exchange must fill them)"""
        pm = self.parts[p]
        x = x_whole.index_select(0, self.idx[p]["cell_global"]).clone()
        x[pm.part["n_owned"]:] = fill_ghosts
        return x

    def local_faces(self, p, f_whole, nfi_whole):
        """internal then boundary faces of the part from a whole-mesh face array"""
        t = torch()
        i = self.idx[p]
        return t.cat([f_whole.index_select(0, i["face_global"]),
                      f_whole.index_select(0, i["bface_global"] + nfi_whole)]).contiguous()

    def local_bfaces(self, p, b_whole):
        return b_whole.index_select(0, self.idx[p]["bface_global"]).contiguous()

    def exchange(self, xs):
        """one exchange over every part: xs[p] is part p's local array (rows of ncomp)"""
        t = torch()
        n = len(self.parts)
        shape = xs[0].shape[1:]
        sends = [t.empty((pm.part["n_send"],) + tuple(shape), dtype=xs[0].dtype, device="cuda") for pm in self.parts]
        recvs = [t.empty((pm.part["n_ghost"],) + tuple(shape), dtype=xs[0].dtype, device="cuda") for pm in self.parts]
        for pm, x, s in zip(self.parts, xs, sends):
            pm.pack(x, s)
        for p in range(n):
            sp = self.parts[p].maps["send_start"]
            for q in range(n):
                rq = self.parts[q].maps["recv_start"]
                a, b = sp[q], sp[q + 1]
                if b > a:
                    recvs[q][rq[p]:rq[p + 1]].copy_(sends[p][a:b])
        for pm, x, r in zip(self.parts, xs, recvs):
            pm.unpack(r, x)

    def close(self):
        for pm in self.parts:
            pm.close()
        self.P.close()


def _same_owned(halo, p, got, whole, what):
    t = torch()
    info = halo.parts[p].part
    ref = whole[info["cell_lo"]:info["cell_hi"]]
    own = got[:info["n_owned"]]
    assert t.equal(own, ref), (what, p, float((own - ref).abs().max()))


CASES = {
    "tube50k_8": (lambda: mg.tube(n=8, m=4, layers=44, L=2.0, seed=2603013), 8),
    "kuhn12_3": (lambda: mg.kuhn_cube(12, jitter=0.15, patches="channel", seed=2603002), 3),
    "cavity_5": (lambda: mg.cavity(), 5),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("dtname", ["f64", "f32"])
def test_part_rows_equal_whole_mesh_rows(case, dtname):
    mesh_fn, n_parts = CASES[case]
    m = mesh_fn()
    t = torch()
    dt = t.float64 if dtname == "f64" else t.float32
    note("halo", case, n_parts, "parts", m.n_cells, "cells", dtname)
    M = B.Mesh(ctx(), m)
    H = Halo(m, n_parts)
    nfi = m.n_internal_faces
    table = B.BC_U if case == "cavity_5" else B.BC_ALL_FIXED
    phi_u, phib_u = _fields(m, 1, 100)
    U_u, Ub_u = _fields(m, 3, 200)
    phi = to_int(M, phi_u, B.KIND_CELL, dt)
    phib = to_int(M, phib_u, B.KIND_BFACE, dt)
    U = to_int(M, U_u, B.KIND_CELL, dt)
    Ub = to_int(M, Ub_u, B.KIND_BFACE, dt)
    flux = to_int(M, np.sin(np.arange(m.n_faces) * 0.37) * 0.1, B.KIND_FACE_FLUX, dt)
    # whole mesh
    g = t.empty((m.n_cells, 3), dtype=dt, device="cuda")
    B.difvm_op_grad(M.h, 1, table, phi, phib, g)
    lap = t.empty(m.n_cells, dtype=dt, device="cuda")
    B.difvm_op_laplacian(M.h, table, None, phi, g, phib, lap)
    Uf = t.empty((m.n_faces, 3), dtype=dt, device="cuda")
    B.difvm_op_interp(M.h, 3, table, U, Ub, Uf)
    dv = t.empty((m.n_cells, 3), dtype=dt, device="cuda")
    B.difvm_op_div(M.h, B.SCHEME_UPWIND, 3, table, flux, U, Ub, dv)
    rng = np.random.default_rng(7)
    diag = t.from_numpy(rng.uniform(4, 5, m.n_cells)).to("cuda", dt)
    up = t.from_numpy(rng.uniform(-1, 0, nfi)).to("cuda", dt)
    lo = t.from_numpy(rng.uniform(-1, 0, nfi)).to("cuda", dt)
    y_sym = t.empty(m.n_cells, dtype=dt, device="cuda")
    B.difvm_ldu_spmv(M.h, 1, 0, B.ldu(diag, up, up), phi, y_sym)
    y3 = t.empty((m.n_cells, 3), dtype=dt, device="cuda")
    B.difvm_ldu_spmv(M.h, 3, 0, B.ldu(diag, up, lo), U, y3)
    y3t = t.empty((m.n_cells, 3), dtype=dt, device="cuda")
    B.difvm_ldu_spmv(M.h, 3, 1, B.ldu(diag, up, lo), U, y3t)

    n = n_parts
    # exchange phi and U, check the ghost rows against the whole mesh's values
    phis = [H.local_cells(p, phi) for p in range(n)]
    Us = [H.local_cells(p, U) for p in range(n)]
    H.exchange(phis)
    H.exchange(Us)
    for p in range(n):
        cg = H.idx[p]["cell_global"]
        assert t.equal(phis[p], phi.index_select(0, cg)), ("ghost phi", p)
        assert t.equal(Us[p], U.index_select(0, cg)), ("ghost U", p)
    # gradient on every part, exchange it, then the Laplacian
    gs = []
    for p, pm in enumerate(H.parts):
        nl = pm.info["n_cells"]
        gp = t.full((nl, 3), float("nan"), dtype=dt, device="cuda")
        B.difvm_op_grad(pm.h, 1, table, phis[p], H.local_bfaces(p, phib), gp)
        _same_owned(H, p, gp, g, "grad")
        gp[pm.part["n_owned"]:] = float("nan")
        gs.append(gp)
    H.exchange(gs)
    for p, pm in enumerate(H.parts):
        nl = pm.info["n_cells"]
        pb = H.local_bfaces(p, phib)
        lp = t.empty(nl, dtype=dt, device="cuda")
        B.difvm_op_laplacian(pm.h, table, None, phis[p], gs[p], pb, lp)
        _same_owned(H, p, lp, lap, "laplacian")
        # face interpolation: every local face, internal and boundary
        nf_l = pm.info["n_internal_faces"] + pm.info["n_boundary_faces"]
        uf = t.empty((nf_l, 3), dtype=dt, device="cuda")
        B.difvm_op_interp(pm.h, 3, table, Us[p], H.local_bfaces(p, Ub), uf)
        assert t.equal(uf, H.local_faces(p, Uf, nfi)), ("interp", p)
        d = t.empty((nl, 3), dtype=dt, device="cuda")
        B.difvm_op_div(pm.h, B.SCHEME_UPWIND, 3, table, H.local_faces(p, flux, nfi), Us[p], H.local_bfaces(p, Ub), d)
        _same_owned(H, p, d, dv, "div")
        i = H.idx[p]
        dl = diag.index_select(0, i["cell_global"]).contiguous()
        ul = up.index_select(0, i["face_global"]).contiguous()
        ll = lo.index_select(0, i["face_global"]).contiguous()
        ys = t.empty(nl, dtype=dt, device="cuda")
        B.difvm_ldu_spmv(pm.h, 1, 0, B.ldu(dl, ul, ul), phis[p], ys)
        _same_owned(H, p, ys, y_sym, "spmv sym")
        y = t.empty((nl, 3), dtype=dt, device="cuda")
        B.difvm_ldu_spmv(pm.h, 3, 0, B.ldu(dl, ul, ll), Us[p], y)
        _same_owned(H, p, y, y3, "spmv 3")
        B.difvm_ldu_spmv(pm.h, 3, 1, B.ldu(dl, ul, ll), Us[p], y)
        _same_owned(H, p, y, y3t, "spmv 3 transpose")
    H.close()
    M.close()


def test_part_mesh_refuses_solvers():
    m = mg.cavity(8)
    P = B.Partition(m, 2)
    pm = B.PartMesh(ctx(), P, 0)
    t = torch()
    nl = pm.info["n_cells"]
    A = B.ldu(t.ones(nl, dtype=t.float64, device="cuda"), t.zeros(pm.info["n_internal_faces"], dtype=t.float64,
                                                                    device="cuda"))
    x = t.zeros(nl, dtype=t.float64, device="cuda")
    with pytest.raises(B.DifvmError) as e:
        B.difvm_solve_pcg(pm.h, A, x, x.clone(), 1e-8, 10)
    assert e.value.status == B.ERR_UNSUPPORTED
    with pytest.raises(B.DifvmError) as e:
        B.Piso(pm, B.piso_params(0.01, 1e-3))
    assert e.value.status == B.ERR_UNSUPPORTED
    # pack/unpack refuse a whole mesh
    M = B.Mesh(ctx(), m)
    with pytest.raises(B.DifvmError) as e:
        B.difvm_halo_pack(M.h, 1, x, x)
    assert e.value.status == B.ERR_INVALID_ARG
    pm.close()
    M.close()
    P.close()


@pytest.mark.slow
def test_full_size_tube_interior_slab():
    """The 2,000,640-tet tube in 8 slabs: an interior slab (one GPU's share, about 250k cells) and
    an end slab, chained gradient -> exchange -> Laplacian and the symmetric product, bitwise."""
    m = mg.tube()
    assert m.n_cells == 2_000_640
    t = torch()
    M = B.Mesh(ctx(), m)
    H = Halo(m, 8)
    for p in (0, 3):
        note("tube slab", p, H.parts[p].part)
    phi_u, phib_u = _fields(m, 1, 100)
    phi = to_int(M, phi_u, B.KIND_CELL)
    phib = to_int(M, phib_u, B.KIND_BFACE)
    g = t.empty((m.n_cells, 3), dtype=t.float64, device="cuda")
    B.difvm_op_grad(M.h, 1, B.BC_ALL_FIXED, phi, phib, g)
    lap = t.empty(m.n_cells, dtype=t.float64, device="cuda")
    B.difvm_op_laplacian(M.h, B.BC_ALL_FIXED, None, phi, g, phib, lap)
    phis = [H.local_cells(p, phi) for p in range(8)]
    H.exchange(phis)
    gs = []
    for p, pm in enumerate(H.parts):
        gp = t.empty((pm.info["n_cells"], 3), dtype=t.float64, device="cuda")
        B.difvm_op_grad(pm.h, 1, B.BC_ALL_FIXED, phis[p], H.local_bfaces(p, phib), gp)
        _same_owned(H, p, gp, g, "grad")
        gs.append(gp)
    H.exchange(gs)
    for p in (0, 3):
        pm = H.parts[p]
        lp = t.empty(pm.info["n_cells"], dtype=t.float64, device="cuda")
        B.difvm_op_laplacian(pm.h, B.BC_ALL_FIXED, None, phis[p], gs[p], H.local_bfaces(p, phib), lp)
        _same_owned(H, p, lp, lap, "laplacian")
    H.close()
    M.close()
