"""The all-threads timing build of the oracle (liboracle_omp.so, OpenMP in the Krylov kernels) computes
what the serial build computes: the same iteration counts and states equal within rounding (the
thread-order sums change only the order of additions)."""
import numpy as np

from oracle import oracle as O
from paper_2603_15920_amd import meshgen as mg


def test_threaded_oracle_matches_serial():
    m = mg.kuhn_cube(10, jitter=0.15, patches="channel", seed=2603002)
    Ub = mg.box_channel_inlet(m)
    Rd = 1.0 / mg.inlet_flow(m, Ub)
    wk = np.array([[Rd / 9.0, 0.1 / Rd, Rd]])
    U0 = np.zeros((m.n_cells, 3))
    phi0 = O.initial_flux(m, U0, Ub)
    prm = O.piso_params(0.005, 1e-3, maxit_p=5000)
    args = (m, prm, U0, np.zeros(m.n_cells), phi0, Ub, np.zeros(m.n_boundary_faces))
    r1 = O.piso_run(*args, wk=wk, pc=np.zeros(1), nsteps=3)
    try:
        O.use_threads(True)
        assert O.threads() >= 1
        r2 = O.piso_run(*args, wk=wk, pc=np.zeros(1), nsteps=3)
    finally:
        O.use_threads(False)
    assert r1[6] == 0 and r2[6] == 0
    np.testing.assert_array_equal(r1[4], r2[4])
    for a, b in zip(r1[:4], r2[:4]):
        assert np.abs(a - b).max() <= 1e-11 * np.abs(a).max()
