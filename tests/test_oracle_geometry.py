"""Pins of the generated geometry and of the oracle's derived face geometry (delta, k)."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import meshgen as mg


@pytest.fixture(scope="module", params=["cavity", "kuhn5", "tube"])
def mesh(request):
    if request.param == "cavity":
        return mg.cavity(8)
    if request.param == "kuhn5":
        return mg.kuhn_cube(5, patches="sides")
    return mg.tube(n=6, m=3, layers=5)


def test_mesh_valid(mesh):
    assert mg.check_mesh(mesh)


def test_closed_cells_surface_identity(mesh):
    """Per closed cell with planar faces: sum sigma S_f = 0 and sum sigma C_f (x) S_f = V I."""
    Fi = mesh.n_internal_faces
    T = np.zeros((mesh.n_cells, 3, 3))
    np.add.at(T, mesh.owner, np.einsum("fi,fj->fij", mesh.Cf, mesh.Sf))
    np.add.at(T, mesh.neighbour, -np.einsum("fi,fj->fij", mesh.Cf[:Fi], mesh.Sf[:Fi]))
    err = np.abs(T - mesh.V[:, None, None] * np.eye(3)[None]).max()
    assert err < 1e-12 * max(1.0, np.abs(mesh.Cf).max()) * np.abs(mesh.Sf).max() * 10


def test_overrelaxed_delta_matches_paper_form(mesh):
    """delta_f |d_f| = |Delta_f| with Delta_f = (|S|/|S^.d^|) d^ (eq. nonortho_flux, over-relaxed), and
    k_f = S_f - Delta_f."""
    delta, k, _ = O.geometry(mesh)
    Fi = mesh.n_internal_faces
    S = mesh.Sf[:Fi]
    d = mesh.C[mesh.neighbour] - mesh.C[mesh.owner[:Fi]]
    Sn = np.linalg.norm(S, axis=1)
    dn = np.linalg.norm(d, axis=1)
    cosang = np.abs(np.einsum("ij,ij->i", S / Sn[:, None], d / dn[:, None]))
    Delta = (Sn / cosang)[:, None] * (d / dn[:, None])
    np.testing.assert_allclose(delta * dn, np.linalg.norm(Delta, axis=1), rtol=1e-12)
    np.testing.assert_allclose(k, S - Delta, atol=1e-12 * Sn.max())
    # the over-relaxed |Delta| is never shorter than |S|
    assert np.all(np.linalg.norm(Delta, axis=1) >= Sn * (1 - 1e-14))


def test_sizes_of_named_workloads():
    m = mg.cavity()
    assert (m.n_cells, m.n_internal_faces, m.n_boundary_faces) == (2048, 3008, 4224)
    assert [p.size for p in m.patches] == [32, 96, 4096]
