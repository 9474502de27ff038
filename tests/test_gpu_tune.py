"""Launch knobs and the autotuner: every operator's output must be bitwise the same for every
threads-per-block value, PCG results bitwise the same for every product-kernel grid (one block per
tile or persistent grids whose blocks walk several tiles, also on a packed multi-segment mesh), and
the tuner must time, cache, and on a second mesh of the same size bucket reuse its choices."""
import json

import numpy as np
import pytest

from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg

from gpu_util import ctx, dev, empty, host, note

pytestmark = pytest.mark.gpu


def fields(m, seed=4):
    rng = np.random.default_rng(seed)
    return dict(x=rng.standard_normal((m.n_cells, 3)), xb=rng.standard_normal((m.n_boundary_faces, 3)),
                F=rng.standard_normal(m.n_faces), g=rng.standard_normal((m.n_cells, 3)),
                d=4.0 + rng.random(m.n_cells), u=-rng.random(m.n_internal_faces), l=-rng.random(m.n_internal_faces))


def all_ops(M, f, torch_dtype):
    import torch
    t = lambda a: dev(a, torch_dtype)
    x = M.to_internal(t(f["x"]), B.KIND_CELL)
    x1 = M.to_internal(t(f["x"][:, 0].copy()), B.KIND_CELL)
    xb = M.to_internal(t(f["xb"]), B.KIND_BFACE)
    xb1 = M.to_internal(t(f["xb"][:, 0].copy()), B.KIND_BFACE)
    F = M.to_internal(t(f["F"]), B.KIND_FACE_FLUX)
    g = M.to_internal(t(f["g"]), B.KIND_CELL)
    nc, nf = M.src.n_cells, M.src.n_faces
    out = {}
    o = torch.empty((nf, 3), dtype=torch_dtype, device="cuda:0"); B.difvm_op_interp(M.h, 3, B.BC_U, x, xb, o); out["interp"] = host(o)
    o = torch.empty((nc, 9), dtype=torch_dtype, device="cuda:0"); B.difvm_op_grad(M.h, 3, B.BC_U, x, xb, o); out["grad"] = host(o)
    for sch in (B.SCHEME_UPWIND, B.SCHEME_LINEAR):
        o = torch.empty((nc, 3), dtype=torch_dtype, device="cuda:0"); B.difvm_op_div(M.h, sch, 3, B.BC_U, F, x, xb, o)
        out[f"div{sch}"] = host(o)
    o = torch.empty(nc, dtype=torch_dtype, device="cuda:0"); B.difvm_op_laplacian(M.h, B.BC_P, None, x1, g, xb1, o); out["lap"] = host(o)
    A = B.ldu(t(f["d"]), t(f["u"]), t(f["l"]))
    o = torch.empty((nc, 3), dtype=torch_dtype, device="cuda:0"); B.difvm_ldu_spmv(M.h, 3, 0, A, x, o); out["spmv"] = host(o)
    return out


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_operator_outputs_independent_of_block_size(dtype):
    import torch
    td = torch.float64 if dtype == "f64" else torch.float32
    m = mg.kuhn_cube(12, jitter=0.15, patches="channel", seed=8)
    M = B.Mesh(ctx(), m)
    f = fields(m)
    ref = None
    for nb in (64, 128, 256, 512):
        for k in range(10):
            B.difvm_mesh_set_launch(M.h, k, nb)
            assert B.difvm_mesh_get_launch(M.h, k) == nb
        note("ops block", dtype, nb)
        out = all_ops(M, f, td)
        if ref is None:
            ref = out
        else:
            for key in ref:
                np.testing.assert_array_equal(out[key], ref[key], err_msg=f"{key} at {nb} threads")


def pcg_solve(M, m, grid):
    B.difvm_mesh_set_launch(M.h, B.TUNE_PCG_GRID, grid)
    A, b = laplace_system(M, m)
    x = empty(m.n_cells)
    x.zero_()
    st = B.difvm_solve_pcg(M.h, A, b, x, 1e-10, 5000)
    assert st[0] == 0 and st[1] > 5
    return st, host(x)


def laplace_system(M, m):
    d, u, rhs = empty(m.n_cells), empty(max(1, m.n_internal_faces)), empty(m.n_cells)
    pb = np.zeros(m.n_boundary_faces)
    pb[: m.n_boundary_faces // 3] = 1.0
    A = B.ldu(d, u)
    B.difvm_ldu_assemble_laplace(M.h, B.BC_P, None, M.to_internal(dev(pb), B.KIND_BFACE), A, rhs)
    return A, rhs


@pytest.mark.parametrize("packed", [False, True])
def test_pcg_independent_of_grid(packed):
    if packed:
        ms = [mg.kuhn_cube(n, jitter=0.15, patches="channel", seed=20 + n) for n in (10, 7, 12, 5)]
        m, starts = mg.pack(ms)
    else:
        m, starts = mg.kuhn_cube(24, jitter=0.15, patches="channel", seed=9), None
    M = B.Mesh(ctx(), m, seg_cell_start=starts)
    ntile = sum(-(-int(c) // 1024) for c in np.diff(starts)) if packed else -(-m.n_cells // 1024)
    note("pcg grids", m.n_cells, "tiles", ntile)
    ref = None
    for grid in (0, 8, 16, 24, 32, 48, 64, 4096):
        st, x = pcg_solve(M, m, grid)
        if ref is None:
            ref = (st, x)
        else:
            assert st == ref[0]
            np.testing.assert_array_equal(x, ref[1], err_msg=f"grid {grid}")


def test_tuner_cache_roundtrip(tmp_path):
    cache = tmp_path / "tune.json"
    m = mg.kuhn_cube(16, jitter=0.15, patches="channel", seed=10)
    M = B.Mesh(ctx(), m)
    n1 = B.difvm_tune(M.h, cache)
    assert n1 == len(B.TUNE_KNOBS)
    entries = json.loads(cache.read_text())
    assert len(entries) == len(B.TUNE_KNOBS)
    got = [B.difvm_mesh_get_launch(M.h, k) for k in range(len(B.TUNE_KNOBS))]
    for k, name in enumerate(B.TUNE_KNOBS):
        (key,) = [kk for kk in entries if f"|{name}|" in kk]
        assert entries[key] == got[k]
    # a second mesh in the same size bucket reuses every choice without timing
    m2 = mg.kuhn_cube(16, jitter=0.15, patches="channel", seed=11)
    M2 = B.Mesh(ctx(), m2)
    assert B.difvm_tune(M2.h, cache) == 0
    assert [B.difvm_mesh_get_launch(M2.h, k) for k in range(len(B.TUNE_KNOBS))] == got
    # no cache: times everything, writes nothing
    assert B.difvm_tune(M2.h, None) == len(B.TUNE_KNOBS)


def test_launch_errors(tmp_path):
    m = mg.kuhn_cube(4, jitter=0.15, patches="walls", seed=3)
    M = B.Mesh(ctx(), m)
    for knob, value in ((0, 96), (0, 1024), (10, 12), (10, -8), (11, 256), (-1, 256)):
        with pytest.raises(B.DifvmError) as e:
            B.difvm_mesh_set_launch(M.h, knob, value)
        assert e.value.status == B.ERR_INVALID_ARG
    bad = tmp_path / "bad.json"
    bad.write_text('{"gfx950|grad_f64|n8|single": "x"}')
    with pytest.raises(B.DifvmError) as e:
        B.difvm_tune(M.h, bad)
    assert e.value.status == B.ERR_INVALID_ARG
