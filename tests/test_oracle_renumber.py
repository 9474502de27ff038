"""Oracle renumbering pins: hand-worked fixtures (tests/golden) and invariants on real meshes."""
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import meshgen as mg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        key, *vals = line.split()
        if key == "faces":
            out[key] = [tuple(int(t) for t in v.split(",")) for v in vals]
        else:
            out[key] = [int(v) for v in vals]
    return out


def graph_mesh(nc, faces):
    """A connectivity-only mesh (geometry is unused by renumbering)."""
    fo = np.array([f[0] for f in faces], np.int32)
    fn = np.array([f[1] for f in faces], np.int32)
    nf = len(faces)
    z = np.zeros((nf, 3))
    return mg.Mesh(owner=fo, neighbour=fn, Sf=z, Cf=z, C=np.zeros((nc, 3)), V=np.ones(nc),
                   w=np.full(nf, 0.5), patches=[])


@pytest.mark.parametrize("name", ["rcm_path5.txt", "rcm_grid3x3.txt"])
def test_rcm_golden(name):
    g = read_golden(name)
    m = graph_mesh(g["ncells"][0], g["faces"])
    r = O.renumber(m)
    for key in ("cell_perm", "face_perm", "face_flip", "owner", "neighbour", "own_start", "losort", "losort_start"):
        if key in g:
            np.testing.assert_array_equal(r[key], g[key], err_msg=key)


@pytest.mark.parametrize("maker", [lambda: mg.cavity(16), lambda: mg.kuhn_cube(8, patches="sides"),
                                   lambda: mg.tube(n=6, m=3, layers=6)])
def test_renumber_invariants(maker):
    m = maker()
    r = O.renumber(m)
    nc, nfi = m.n_cells, m.n_internal_faces
    assert np.array_equal(np.sort(r["cell_perm"]), np.arange(nc))
    assert np.array_equal(np.sort(r["face_perm"]), np.arange(nfi))
    assert np.all(r["owner"] < r["neighbour"])
    key = r["owner"].astype(np.int64) * nc + r["neighbour"]
    assert np.all(np.diff(key) >= 0)
    newof = np.empty(nc, np.int64)
    newof[r["cell_perm"]] = np.arange(nc)
    o = newof[m.owner[:nfi][r["face_perm"]]]
    n = newof[m.neighbour[r["face_perm"]]]
    flip = r["face_flip"].astype(bool)
    assert np.array_equal(np.where(flip, n, o), r["owner"])
    assert np.array_equal(np.where(flip, o, n), r["neighbour"])
    assert np.array_equal(flip, o > n)
    assert np.array_equal(r["own_start"], np.searchsorted(r["owner"], np.arange(nc + 1)))
    assert np.array_equal(r["neighbour"][r["losort"]], np.sort(r["neighbour"], kind="stable"))
    assert np.all(np.diff(r["losort"])[np.diff(r["neighbour"][r["losort"]]) == 0] > 0)  # stable
    # boundary faces: patch order kept, new owner non-decreasing inside each patch
    Fi = nfi
    for p in m.patches:
        s = slice(p.start - Fi, p.start - Fi + p.size)
        assert np.all((r["bface_perm"][s] >= p.start - Fi) & (r["bface_perm"][s] < p.start - Fi + p.size))
        assert np.all(np.diff(r["bowner"][s]) >= 0)
        assert np.array_equal(r["bowner"][s], newof[m.owner[Fi + r["bface_perm"][s]]])
    # RCM reduces the bandwidth well below the generator's ordering
    bw_new = int((r["neighbour"] - r["owner"]).max())
    assert bw_new < O.bandwidth(m)
