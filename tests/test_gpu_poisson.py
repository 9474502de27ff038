"""Poisson verification workload on the GPU (the paper's 3D manufactured solution, Sec. 3.1.1, on its
three mesh sizes): Laplace assembly with the exact field as Dirichlet data, the over-relaxed
correction from the exact gradient, and a Jacobi-PCG solve, all through the C-ABI.  The solution must
match the oracle's within 1e-9 with the same iteration count, and the error against the exact field
must fall at second order like the oracle's."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg

from gpu_util import ctx, dev, empty, host, note, rel_err

pytestmark = pytest.mark.gpu


def gpu_poisson(m, tol=1e-12):
    M = B.Mesh(ctx(), m)
    phib = M.to_internal(dev(mg.poisson_mms_solution(m.Cf[m.n_internal_faces:])), B.KIND_BFACE)
    d, u, rbc = empty(m.n_cells), empty(m.n_internal_faces), empty(m.n_cells)
    A = B.ldu(d, u)
    B.difvm_ldu_assemble_laplace(M.h, B.BC_ALL_FIXED, None, phib, A, rbc)
    g = M.to_internal(dev(mg.poisson_mms_gradient(m.C)), B.KIND_CELL)
    zero = empty(m.n_cells).zero_()
    lap0 = empty(m.n_cells)
    B.difvm_op_laplacian(M.h, B.BC_ALL_FIXED, None, zero, g, phib, lap0)  # = rhs_bc + correction
    rhs = lap0 - M.to_internal(dev(m.V * mg.poisson_mms_source(m.C)), B.KIND_CELL)
    x = empty(m.n_cells).zero_()
    st, it, res = B.difvm_solve_pcg(M.h, A, rhs, x, tol, 5000)
    return st, it, host(M.to_user(x, B.KIND_CELL))


def oracle_poisson(m, tol=1e-12):
    phib = mg.poisson_mms_solution(m.Cf[m.n_internal_faces:])
    d, u, rbc = O.assemble_laplace(m, phib=phib, table=O.TABLE_ALL_FIXED)
    lap0 = O.laplacian(m, np.zeros(m.n_cells), mg.poisson_mms_gradient(m.C), phib, table=O.TABLE_ALL_FIXED)
    phi, it, res, st = O.pcg(m, d, u, lap0 - m.V * mg.poisson_mms_source(m.C), tol=tol, maxit=5000)
    return st, it, phi


def l2_error(m, phi):
    e = phi - mg.poisson_mms_solution(m.C)
    return math.sqrt((m.V * e * e).sum() / m.V.sum())


def test_poisson_mms_gpu_vs_oracle_and_order():
    errs, ncell = [], []
    for n in (12, 18, 25):
        m = mg.kuhn_cube(n, jitter=0.15, patches="walls", seed=2603007)
        st, it, phi = gpu_poisson(m)
        sto, ito, phio = oracle_poisson(m)
        note("poisson", m.n_cells, "cells: gpu iters", it, "oracle", ito)
        assert st == 0 and sto == 0 and it == ito
        assert rel_err(phi, phio) <= 1e-9
        errs.append(l2_error(m, phi))
        ncell.append(m.n_cells)
    order = [math.log(errs[i] / errs[i + 1]) / math.log((ncell[i + 1] / ncell[i]) ** (1 / 3)) for i in range(2)]
    note("poisson errors", errs, "orders", order)
    assert min(order) >= 1.8
