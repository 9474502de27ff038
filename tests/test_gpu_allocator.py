"""Device memory through the caller's allocator (difvm_ctx_set_allocator): every block the library
holds comes from torch's caching allocator, solves and PISO steps allocate nothing after their first
call (warm-up), results are bitwise those of a context on hipMalloc, and every block is returned."""
import gc

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg

from gpu_util import dev, host, note, to_int, torch
from test_gpu_piso import inlet_values

pytestmark = pytest.mark.gpu


def channel(n=8):
    m = mg.kuhn_cube(n, jitter=0.15, patches="channel", seed=2603002)
    Ub = inlet_values(m)
    q = -float((Ub[m.patch("inlet").start - m.n_internal_faces:][:m.patch("inlet").size]
                * m.Sf[m.patch("inlet").start:m.patch("inlet").start + m.patch("inlet").size]).sum())
    Rd = 1.0 / q
    return m, Ub, (Rd / 9.0, 0.1 / Rd, Rd)


def piso_run(ctx, m, Ub, wk, nsteps, precond, graph=False, counter=None):
    """PISO steps on a fresh mesh of ctx; with counter, asserts that steps after the first allocate
    nothing.  Returns the final state (host, user order) and the iteration counts."""
    M = B.Mesh(ctx, m)
    P = B.Piso(M, B.piso_params(0.005, 1e-3, precond=precond))
    P.set_boundary(dev(Ub), dev(np.zeros(m.n_boundary_faces)))
    P.set_windkessel(0, *wk, 0.0)
    U0 = np.zeros((m.n_cells, 3))
    P.set_state(dev(U0), dev(np.zeros(m.n_cells)), dev(O.initial_flux(m, U0, Ub)))
    if graph:
        P.set_graph(True, 4)
    its = []
    for k in range(nsteps):
        before = counter() if counter else None
        st, it, _ = P.step(1)
        assert st == 0
        its.append(it[0])
        # the first step builds the solver workspaces and the AMG hierarchy, the second captures the
        # graph in graph mode; later steps must not allocate
        if counter and k >= (2 if graph else 1):
            assert counter() == before, (k, before, counter())
    U, p, phi, pc = P.get_state()
    out = (host(U), host(p), host(phi), pc, np.array(its))
    P.close()
    M.close()
    return out


@pytest.mark.parametrize("precond,graph", [("jacobi", False), ("amg", False), ("amg", True)])
def test_piso_steps_allocate_nothing_and_match_hipmalloc(precond, graph):
    m, Ub, wk = channel()
    note("allocator piso", precond, graph)
    gc.collect()  # objects an earlier test left behind are freed now, not during this one
    tctx = B.Context(0)  # torch's caching allocator
    A = tctx.allocator
    base = torch().cuda.memory_allocated()
    r_t = piso_run(tctx, m, Ub, wk, 5, precond, graph, counter=lambda: A.counts())
    assert A.n_alloc > 0
    # everything the mesh and the PISO object held has gone back to torch
    assert A.n_free == A.n_alloc and not A.live
    assert torch().cuda.memory_allocated() == base
    hctx = B.Context(0, torch_allocator=False)  # hipMalloc
    r_h = piso_run(hctx, m, Ub, wk, 5, precond, graph)
    for a, b in zip(r_t, r_h):
        np.testing.assert_array_equal(a, b)


def test_solves_and_assembly_allocate_nothing_after_first_call():
    m = mg.kuhn_cube(6, jitter=0.15, seed=11)
    tctx = B.Context(0)
    A = tctx.allocator
    M = B.Mesh(tctx, m)
    d, u, _ = O.assemble_laplace(m, phib=np.zeros(m.n_boundary_faces), table=B.BC_ALL_FIXED)
    r = B.difvm_mesh_renumber_host(m)
    L = B.ldu(to_int(M, d, B.KIND_CELL), dev(u[r["face_perm"]]))
    b = to_int(M, np.random.default_rng(1).standard_normal(m.n_cells), B.KIND_CELL)
    rng = np.random.default_rng(2)
    U = to_int(M, rng.standard_normal((m.n_cells, 3)), B.KIND_CELL)
    Ubv = to_int(M, rng.standard_normal((m.n_boundary_faces, 3)), B.KIND_BFACE)
    flux = to_int(M, O.initial_flux(m, host(M.to_user(U, B.KIND_CELL)), host(M.to_user(Ubv, B.KIND_BFACE))),
                  B.KIND_FACE_FLUX)
    Dm, Um, Lm = (torch().empty(n, dtype=torch().float64, device="cuda:0") for n in
                  (m.n_cells, m.n_internal_faces, m.n_internal_faces))
    bm = torch().empty((m.n_cells, 3), dtype=torch().float64, device="cuda:0")
    Am = B.ldu(Dm, Um, Lm)
    x = torch().zeros(m.n_cells, dtype=torch().float64, device="cuda:0")
    X3 = torch().zeros((m.n_cells, 3), dtype=torch().float64, device="cuda:0")
    amg = B.difvm_amg_create(M.h, L)

    def calls():
        x.zero_()
        X3.zero_()
        B.difvm_solve_pcg(M.h, L, b, x, 1e-10, 2000)
        B.difvm_solve_pcg_amg(amg, L, b, x.zero_(), 1e-10, 200)
        B.difvm_ldu_assemble_momentum(M.h, 0.01, 1e-3, flux, U, Ubv, Am, bm)
        B.difvm_solve_bicgstab(M.h, Am, 3, bm, X3, 1e-10, 500)
        return host(x).copy(), host(X3).copy()

    first = calls()  # warm-up: workspaces and scratch
    n0 = A.counts()
    second = calls()
    third = calls()
    assert A.counts() == n0, (n0, A.counts())
    for a, b_ in zip(first, second):
        np.testing.assert_array_equal(a, b_)
    for a, b_ in zip(second, third):
        np.testing.assert_array_equal(a, b_)
    B.difvm_amg_destroy(amg)
    M.close()
    assert A.n_free == A.n_alloc and not A.live


def test_allocator_cannot_change_while_objects_exist():
    m = mg.kuhn_cube(3, jitter=0.1, seed=5)
    c = B.Context(0)
    M = B.Mesh(c, m)
    with pytest.raises(B.DifvmError):
        B.difvm_ctx_set_allocator(c.h, None, None)
    M.close()
    B.difvm_ctx_set_allocator(c.h, None, None)  # allowed again: back to hipMalloc
    M2 = B.Mesh(c, m)
    M2.close()
    with pytest.raises(B.DifvmError):  # exactly one of the two callbacks
        B.difvm_ctx_set_allocator(c.h, c.allocator.alloc_fn, None)


def test_allocator_failure_is_an_error_not_a_crash():
    """An allocator that returns NULL makes the call fail with DIFVM_ERR_OOM and leaks nothing."""
    m = mg.kuhn_cube(3, jitter=0.1, seed=5)
    c = B.Context(0, torch_allocator=False)
    T = B.TorchAllocator(0)
    budget = {"n": 3}
    inner_alloc = T.alloc_fn

    def alloc(nbytes, stream, user):
        if budget["n"] <= 0:
            return None
        budget["n"] -= 1
        return inner_alloc(nbytes, stream, user)

    fn = B.ALLOC_FN(alloc)
    B.difvm_ctx_set_allocator(c.h, fn, T.free_fn)
    with pytest.raises(B.DifvmError) as e:
        B.Mesh(c, m)
    assert e.value.status == B.ERR_OOM
    assert T.n_free == T.n_alloc == 3 and not T.live
