"""difvm_ldu_assemble_momentum_noalloc (the entry point that allocates nothing) against
difvm_ldu_assemble_momentum on the same inputs: bitwise equal outputs on two calls in a row, the
second on a smaller mesh (the fixed scratch keeps the first call's contents), no allocator call
during either, and a mesh above DIFVM_NOALLOC_MAX_CELLS refused with a clear error."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg

from gpu_util import note, torch

pytestmark = pytest.mark.gpu


def _inputs(m, seed):
    rng = np.random.default_rng(seed)
    U = rng.standard_normal((m.n_cells, 3))
    Ub = rng.standard_normal((m.n_boundary_faces, 3))
    return U, Ub, O.initial_flux(m, U, Ub)


def _assemble(M, m, U, Ub, flux, fn):
    t = torch()
    dev = lambda a, kind: M.to_internal(t.from_numpy(np.ascontiguousarray(a)).to("cuda:0"), kind)
    f, u, ub = dev(flux, B.KIND_FACE_FLUX), dev(U, B.KIND_CELL), dev(Ub, B.KIND_BFACE)
    e = lambda *s: t.full(s, float("nan"), dtype=t.float64, device="cuda:0")
    D, Up, Lo, b = e(m.n_cells), e(m.n_internal_faces), e(m.n_internal_faces), e(m.n_cells, 3)
    A = B.ldu(D, Up, Lo)
    t.cuda.synchronize()
    before = M.ctx.allocator.counts()
    fn(M.h, 0.01, 1e-3, f, u, ub, A, b)
    after = M.ctx.allocator.counts()
    return [x.cpu().numpy() for x in (D, Up, Lo, b)], after[0] - before[0]


def test_noalloc_momentum_assembly_matches_and_allocates_nothing():
    ctx = B.Context(0)  # torch's caching allocator, with counters
    big = mg.kuhn_cube(20, jitter=0.15, patches="channel", seed=2603002)     # 48,000 cells
    small = mg.tube(n=6, m=3, layers=7)                                        # fewer cells, prisms split to tets
    assert big.n_cells <= B.NOALLOC_MAX_CELLS and small.n_cells < big.n_cells
    for k, m in enumerate((big, small)):
        note("noalloc momentum", m.name, m.n_cells)
        M = B.Mesh(ctx, m)
        U, Ub, flux = _inputs(m, 40 + k)
        ref, _ = _assemble(M, m, U, Ub, flux, B.difvm_ldu_assemble_momentum)
        got, n_alloc = _assemble(M, m, U, Ub, flux, B.difvm_ldu_assemble_momentum_noalloc)
        assert n_alloc == 0
        for a, b, name in zip(got, ref, ("diag", "upper", "lower", "b")):
            assert np.isfinite(a).all(), name
            np.testing.assert_array_equal(a, b, err_msg=name)
        M.close()


def test_noalloc_refuses_meshes_above_the_limit():
    ctx = B.Context(0)
    m = mg.kuhn_cube(28, jitter=0.15, patches="channel", seed=2603002)        # 131,712 cells
    assert m.n_cells > B.NOALLOC_MAX_CELLS
    M = B.Mesh(ctx, m)
    U, Ub, flux = _inputs(m, 7)
    with pytest.raises(B.DifvmError) as e:
        _assemble(M, m, U, Ub, flux, B.difvm_ldu_assemble_momentum_noalloc)
    assert e.value.status == B.ERR_INVALID_ARG
    assert "DIFVM_NOALLOC_MAX_CELLS" in str(e.value)
    M.close()
