"""Pins of the oracle's non-orthogonal correction schemes (Sec. "Diffusive flux discretization", eq.
nonortho_flux): over-relaxed, minimum, orthogonal and none.  Each scheme is pinned by the geometric
property that defines its Delta, all four by their agreement on orthogonal faces, and the corrected
ones by the exactness of the face flux for a linear field and by grid convergence."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import meshgen as mg

SCHEMES = ["overrelaxed", "minimum", "orthogonal", "none"]
SHEAR = np.array([[1.0, 0.35, 0.2], [0.0, 1.0, 0.3], [0.0, 0.0, 1.0]])


def with_scheme(mesh, scheme):
    mesh.meta["nonorth"] = scheme
    return mesh


@pytest.fixture(scope="module", params=["kuhn5", "tube", "sheared_hex"])
def mesh(request):
    if request.param == "kuhn5":
        return mg.kuhn_cube(5, patches="sides")
    if request.param == "tube":
        return mg.tube(n=6, m=3, layers=5)
    return mg.hex_box(5, 4, 3, A=SHEAR)


def _internal_d(m):
    Fi = m.n_internal_faces
    return m.Sf[:Fi], m.C[m.neighbour] - m.C[m.owner[:Fi]]


def _boundary_d(m):
    Fi = m.n_internal_faces
    return m.Sf[Fi:], m.Cf[Fi:] - m.C[m.owner[Fi:]]


def _geometry(m, scheme):
    return O.geometry(with_scheme(m, scheme))


def test_schemes_agree_on_orthogonal_faces():
    """S parallel to d: every scheme gives delta = |S|/|d| and k = 0 (eq. diff_ortho)."""
    m = mg.hex_box(4, 3, 5)
    S, d = _internal_d(m)
    Sb, db = _boundary_d(m)
    want = np.linalg.norm(S, axis=1) / np.linalg.norm(d, axis=1)
    want_b = np.linalg.norm(Sb, axis=1) / np.linalg.norm(db, axis=1)
    for s in SCHEMES:
        delta, k, deltab = _geometry(m, s)
        np.testing.assert_allclose(delta, want, rtol=1e-13)
        np.testing.assert_allclose(deltab, want_b, rtol=1e-13)
        assert np.abs(k).max() < 1e-13 * np.abs(S).max()


def test_minimum_correction_is_perpendicular_to_d(mesh):
    """minimum: Delta = (S.d^) d^ is the projection of S on d, so k = S - Delta is orthogonal to d and
    |Delta| <= |S|."""
    delta, k, deltab = _geometry(mesh, "minimum")
    S, d = _internal_d(mesh)
    dn = np.linalg.norm(d, axis=1)
    Sn = np.linalg.norm(S, axis=1)
    assert np.abs(np.einsum("ij,ij->i", k, d)).max() < 1e-12 * (Sn * dn).max()
    np.testing.assert_allclose(k, S - delta[:, None] * d, atol=1e-13 * Sn.max())
    assert np.all(delta * dn <= Sn * (1 + 1e-14))
    Sb, db = _boundary_d(mesh)
    np.testing.assert_allclose(deltab * np.einsum("ij,ij->i", db, db), np.einsum("ij,ij->i", Sb, db), rtol=1e-13)


def test_orthogonal_correction_keeps_the_length_of_s(mesh):
    """orthogonal: |Delta| = |S| along d^."""
    delta, k, deltab = _geometry(mesh, "orthogonal")
    S, d = _internal_d(mesh)
    np.testing.assert_allclose(delta * np.linalg.norm(d, axis=1), np.linalg.norm(S, axis=1), rtol=1e-13)
    np.testing.assert_allclose(k, S - delta[:, None] * d, atol=1e-13 * np.abs(S).max())
    Sb, db = _boundary_d(mesh)
    np.testing.assert_allclose(deltab * np.linalg.norm(db, axis=1), np.linalg.norm(Sb, axis=1), rtol=1e-13)


def test_overrelaxed_correction_is_perpendicular_to_s(mesh):
    """over-relaxed: |Delta| = |S|/cos(S,d), so S.Delta = |S|^2 and k is orthogonal to S; |Delta| >= |S|."""
    delta, k, _ = _geometry(mesh, "overrelaxed")
    S, d = _internal_d(mesh)
    Sn = np.linalg.norm(S, axis=1)
    assert np.abs(np.einsum("ij,ij->i", k, S)).max() < 1e-12 * (Sn * Sn).max()
    assert np.all(delta * np.linalg.norm(d, axis=1) >= Sn * (1 - 1e-14))


def test_no_correction_is_the_two_point_stencil(mesh):
    """none: delta = |S|/|d| and k = 0; the Laplacian is then sum sigma |S| (phi_N - phi_O)/|d| plus the
    boundary terms, whatever gradient is passed."""
    delta, k, deltab = _geometry(mesh, "none")
    S, d = _internal_d(mesh)
    np.testing.assert_allclose(delta, np.linalg.norm(S, axis=1) / np.linalg.norm(d, axis=1), rtol=1e-13)
    assert not k.any()
    rng = np.random.default_rng(7)
    phi = rng.standard_normal(mesh.n_cells)
    phib = rng.standard_normal(mesh.n_boundary_faces)
    g = rng.standard_normal((mesh.n_cells, 3))
    got = O.laplacian(mesh, phi, g, phib)
    Fi = mesh.n_internal_faces
    want = np.zeros(mesh.n_cells)
    t = np.linalg.norm(S, axis=1) / np.linalg.norm(d, axis=1) * (phi[mesh.neighbour] - phi[mesh.owner[:Fi]])
    np.add.at(want, mesh.owner[:Fi], t)
    np.add.at(want, mesh.neighbour, -t)
    Sb, db = _boundary_d(mesh)
    ob = mesh.owner[Fi:]
    np.add.at(want, ob, np.linalg.norm(Sb, axis=1) / np.linalg.norm(db, axis=1) * (phib - phi[ob]))
    np.testing.assert_allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("scheme", ["overrelaxed", "minimum", "orthogonal"])
def test_corrected_flux_is_exact_for_linear_fields(mesh, scheme):
    """With k = S - Delta and the exact gradient a of phi = a.x, every internal face flux equals S.a, so
    the Laplacian vanishes in each cell that has no boundary face (closed cell: sum sigma S = 0)."""
    with_scheme(mesh, scheme)
    a = np.array([0.7, -1.3, 0.4])
    phi = mesh.C @ a
    g = np.tile(a, (mesh.n_cells, 1))
    phib = mesh.Cf[mesh.n_internal_faces:] @ a
    interior = np.ones(mesh.n_cells, bool)
    interior[mesh.owner[mesh.n_internal_faces:]] = False
    assert interior.sum() > 0
    L = O.laplacian(mesh, phi, g, phib)
    scale = np.abs(mesh.Sf).max() * np.abs(a).sum() * 20
    assert np.abs(L[interior]).max() < 1e-12 * scale


def test_uncorrected_flux_is_not_exact_on_jittered_tets():
    """The two-point stencil alone misses the linear field on non-orthogonal jittered tets (on the
    uniformly sheared hexes the errors of opposite faces cancel, so those cannot show it)."""
    m = with_scheme(mg.kuhn_cube(5, patches="sides"), "none")
    a = np.array([0.7, -1.3, 0.4])
    interior = np.ones(m.n_cells, bool)
    interior[m.owner[m.n_internal_faces:]] = False
    L0 = O.laplacian(m, m.C @ a, np.tile(a, (m.n_cells, 1)), m.Cf[m.n_internal_faces:] @ a)
    assert np.abs(L0[interior]).max() > 1e-3 * np.abs(m.Sf).max()


def test_schemes_order_their_orthogonal_parts(mesh):
    """cos(S,d) <= 1 orders the orthogonal coefficients: minimum <= orthogonal <= over-relaxed."""
    dmin = _geometry(mesh, "minimum")[0]
    dort = _geometry(mesh, "orthogonal")[0]
    dovr = _geometry(mesh, "overrelaxed")[0]
    assert np.all(dmin <= dort * (1 + 1e-14)) and np.all(dort <= dovr * (1 + 1e-14))


def _poisson_error(m):
    """lap(phi) = f with phi = phi_GT on the boundary, the correction taken from the
    exact gradient: K phi = rhs_bc + N - V f with N = sum sigma k.grad(phi_GT)_f."""
    phib = mg.poisson_mms_solution(m.Cf[m.n_internal_faces:])
    d, u, rbc = O.assemble_laplace(m, phib=phib)
    N = O.laplacian(m, np.zeros(m.n_cells), mg.poisson_mms_gradient(m.C), phib) - rbc
    phi, it, res, st = O.pcg(m, d, u, rbc + N - m.V * mg.poisson_mms_source(m.C), tol=1e-12, maxit=5000)
    assert st == 0
    e = phi - mg.poisson_mms_solution(m.C)
    return math.sqrt((m.V * e * e).sum() / m.V.sum())


def test_corrected_schemes_converge_and_uncorrected_stalls():
    """Sheared hexes (constant non-orthogonality as h -> 0): every corrected scheme converges, the
    two-point stencil alone keeps an O(1) error (eq. diff_ortho is first-order inconsistent there).
    Boundary faces carry no correction, so the observed order is one."""
    meshes = [mg.hex_box(n, n, n, A=SHEAR) for n in (8, 16, 32)]
    nc = [m.n_cells for m in meshes]
    errs = {}
    for s in SCHEMES:
        errs[s] = [_poisson_error(with_scheme(m, s)) for m in meshes]
    for m in meshes:
        m.meta.pop("nonorth")
    order = {s: math.log(e[-2] / e[-1]) / math.log((nc[-1] / nc[-2]) ** (1 / 3)) for s, e in errs.items()}
    for s in ("overrelaxed", "minimum", "orthogonal"):
        assert order[s] >= 0.8, (s, errs[s])
        assert errs[s][-1] < 0.25 * errs["none"][-1], errs
    assert order["none"] < 0.2, errs["none"]
