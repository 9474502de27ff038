"""Graph mode of the checkpointed reverse sweep (difvm_tape_set_graph): every full segment is
recomputed and reversed by replayed graphs; all cotangents (initial state, capacitor pressures,
Windkessel parameters, fixed velocity boundary values) must be bitwise those of the eager sweep on an
identical PISO object, with the program's own eager work between replays.  The eager sweep itself is
pinned to the oracle's tangent in test_gpu_adjoint.py."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg

from gpu_util import ctx, dev, empty, host, note

pytestmark = pytest.mark.gpu


def windkessel_channel():
    m = mg.kuhn_cube(3, jitter=0.15, patches="channel", seed=61, nxyz=(6, 3, 3), hi=(2.0, 1.0, 1.0))
    return m, mg.box_channel_inlet(m), [(0.4, 0.3, 1.5)], [0.1]


def ybif_small():
    m = mg.ybif(h=0.2)
    Ub = np.zeros((m.n_boundary_faces, 3))
    p = m.patch("inlet")
    s = slice(p.start - m.n_internal_faces, p.start - m.n_internal_faces + p.size)
    Ub[s] = mg.parabolic_inlet(m.Cf[p.start:p.start + p.size], (0.0, 0.0, 0.0), 0.5, 1.0)
    wk = mg.windkessel_nominal(m, mg.inlet_flow(m, Ub))
    return m, Ub, [tuple(r) for r in wk], [0.0] * len(wk)


def window(m, Ub, wk, pc0, nsteps, every, graph, extra, precond, reps=1, tol=1e-10, seed=5):
    M = B.Mesh(ctx(), m)
    P = B.Piso(M, B.piso_params(1e-2, 2e-3, tol_p=tol, tol_u=tol, maxit_p=20000, maxit_u=5000, precond=precond))
    P.set_boundary(dev(Ub), dev(np.zeros(m.n_boundary_faces)))
    for j, row in enumerate(wk):
        P.set_windkessel(j, *row, pc0[j])
    U0 = np.zeros((m.n_cells, 3))
    P.set_state(dev(U0), dev(np.zeros(m.n_cells)), dev(O.initial_flux(m, U0, Ub)))
    P.step(3)  # a developing flow, not the state at rest
    T = B.difvm_tape_create(P.h, nsteps, every)
    if graph:
        B.difvm_tape_set_graph(T, True, extra)
    st, _ = B.difvm_piso_forward_record(P.h, T, nsteps)
    assert st == 0
    rng = np.random.default_rng(seed)
    cot = [dev(rng.standard_normal((m.n_cells, 3))), dev(rng.standard_normal(m.n_cells)),
           dev(rng.standard_normal(m.n_faces)), rng.standard_normal(len(wk))]
    outs = []
    for r in range(reps):
        gU0, gp0, gphi0 = empty((m.n_cells, 3)), empty(m.n_cells), empty(m.n_faces)
        gUb = empty((m.n_boundary_faces, 3))
        st, gpc0, gwk = B.difvm_piso_adjoint(P.h, T, *cot, tol, gU0, gp0, gphi0, len(wk))
        assert st == 0
        B.difvm_tape_boundary_cotangent(T, gUb)
        outs.append(dict(gU0=host(gU0), gp0=host(gp0), gphi0=host(gphi0), gUb=host(gUb), gpc0=np.array(gpc0),
                         gwk=np.array(gwk)))
        P.step(1)  # eager work between sweeps: the tape's checkpoints do not move
    info = B.difvm_tape_graph_info(T) if graph else None
    B.difvm_tape_destroy(T)
    P.close()
    M.close()
    return outs, info


def same(a, b):
    for k in a:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("case,nsteps,every,precond", [
    ("channel", 12, 3, "jacobi"),   # 4 full segments: eager + capture, then 3 replays of each graph
    ("channel", 11, 3, "amg"),      # a shorter last segment (eager), then full segments replayed
    ("ybif", 9, 3, "amg"),          # three Windkessel outlets
])
def test_graph_sweep_equals_eager(case, nsteps, every, precond):
    m, Ub, wk, pc0 = windkessel_channel() if case == "channel" else ybif_small()
    note("adjoint graph", case, m.n_cells, nsteps, every, precond)
    eager, _ = window(m, Ub, wk, pc0, nsteps, every, False, 0, precond, reps=2)
    graph, info = window(m, Ub, wk, pc0, nsteps, every, True, 16, precond, reps=2)
    note("adjoint graph info (replays, redos, captures)", info)
    for e, g in zip(eager, graph):
        same(e, g)
    same(eager[0], eager[1])
    replays, redos, captures = info
    n_full = nsteps // every
    # two sweeps.  The first sweep does not recompute the window's last segment (the forward record
    # kept its steps) and runs the next one eagerly for each graph (learning the counts, then the
    # captures); every sweep reverses its first segment (the window's last) eagerly.  The second sweep
    # replays every full segment's recomputation.
    last_full = int(nsteps % every == 0)
    first = n_full - 1 - last_full
    assert replays + redos == first + n_full + first + (n_full - last_full), info
    assert replays >= 2, info


def test_graph_sweep_zero_margin():
    """No margin: later segments may outrun the first one's counts; discarded replays are redone and
    the results stay bitwise equal."""
    m, Ub, wk, pc0 = windkessel_channel()
    eager, _ = window(m, Ub, wk, pc0, 15, 3, False, 0, "jacobi")
    graph, info = window(m, Ub, wk, pc0, 15, 3, True, 0, "jacobi")
    note("adjoint graph zero margin (replays, redos, captures)", info)
    same(eager[0], graph[0])
    # 5 full segments, one sweep: the window's last segment is not recomputed and is reversed eagerly,
    # the next one runs eagerly for both graphs, the other three are replayed
    assert info[0] + info[1] == 3 + 3


def test_tape_graph_errors():
    m, Ub, wk, pc0 = windkessel_channel()
    M = B.Mesh(ctx(), m)
    P = B.Piso(M, B.piso_params(1e-2, 2e-3))
    T = B.difvm_tape_create(P.h, 4, 2)
    with pytest.raises(B.DifvmError) as e:
        B.difvm_tape_set_graph(T, True, -1)
    assert e.value.status == B.ERR_INVALID_ARG
    B.difvm_tape_set_graph(T, False, 0)
    assert B.difvm_tape_graph_info(T) == (0, 0, 0)
    B.difvm_tape_destroy(T)
