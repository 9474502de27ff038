"""Batched form, host side: packing several meshes block-diagonally and the renumbering of the packed
mesh.  Each member's cells must stay contiguous in the internal order, and that order restricted to
a member (with its faces and boundary faces) must be the member's own standalone order shifted by a
constant: this is what lets a batch member compute exactly what it computes alone."""
import numpy as np
import pytest

from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg


def members():
    return [mg.cavity(6), mg.kuhn_cube(3, jitter=0.15, patches="channel", seed=61, nxyz=(6, 3, 3), hi=(2.0, 1.0, 1.0)),
            mg.cavity(6, seed=77), strip4()]


def strip4():
    """four prisms in a strip: a member whose boundary is one wall patch plus the empty patch"""
    pts = np.array([[0, 0], [1, 0], [2, 0], [0, 1], [1, 1.1], [2, 1]], float)
    tris = np.array([[0, 1, 4], [0, 4, 3], [1, 2, 5], [1, 5, 4]])
    specs = [("walls", mg.U_FIXED, mg.P_ZEROGRAD, -1), ("frontAndBack", mg.U_EMPTY, mg.P_EMPTY, -1)]
    return mg.extruded_triangles(pts, tris, 0.1, lambda mid: np.zeros(len(mid), int), specs, name="strip4")


def test_pack_geometry_roundtrip():
    ms = members()
    P, starts = mg.pack(ms)
    mg.check_mesh(P)
    assert list(starts) == list(np.cumsum([0] + [m.n_cells for m in ms]))
    wk_total = 0
    for k, m in enumerate(ms):
        f = mg.member_faces(P, k)
        c = slice(starts[k], starts[k + 1])
        np.testing.assert_array_equal(P.Sf[f], m.Sf)
        np.testing.assert_array_equal(P.Cf[f], m.Cf)
        np.testing.assert_array_equal(P.owner[f] - starts[k], m.owner)
        fi = m.n_internal_faces
        np.testing.assert_array_equal(P.neighbour[f[:fi]] - starts[k], m.neighbour)
        np.testing.assert_array_equal(P.V[c], m.V)
        np.testing.assert_array_equal(P.C[c], m.C)
        for p in m.patches:
            q = P.patch(f"{k}/{p.name}")
            assert q.size == p.size and (q.u_type, q.p_type) == (p.u_type, p.p_type)
            assert q.start == P.meta["members"][k]["bface_start"] + p.start - fi
            assert q.wk_id == (p.wk_id + wk_total if p.wk_id >= 0 else -1)
        wk_total += P.meta["members"][k]["n_windkessel"]


def test_member_order_equals_standalone():
    ms = members()
    P, starts = mg.pack(ms)
    R = B.difvm_mesh_renumber_host(P, geometry=True)
    cp = R["cell_perm"]  # new -> old
    new_of = np.empty_like(cp)
    new_of[cp] = np.arange(cp.size)
    Fi = P.n_internal_faces
    for k, m in enumerate(ms):
        r = B.difvm_mesh_renumber_host(m, geometry=True)
        nk = new_of[starts[k]:starts[k + 1]]
        lo = nk.min()
        assert nk.max() - lo + 1 == m.n_cells, "member not contiguous"
        # cells: same relative order
        np.testing.assert_array_equal(cp[lo:lo + m.n_cells] - starts[k], r["cell_perm"])
        # internal faces: the member's faces form one contiguous run in the same relative order
        mb = P.meta["members"][k]
        fpos = np.flatnonzero((R["face_perm"] >= mb["face_start"]) &
                              (R["face_perm"] < mb["face_start"] + mb["n_internal_faces"]))
        if fpos.size:
            assert fpos.max() - fpos.min() + 1 == fpos.size
        np.testing.assert_array_equal(R["face_perm"][fpos] - mb["face_start"], r["face_perm"])
        np.testing.assert_array_equal(R["face_flip"][fpos], r["face_flip"])
        np.testing.assert_array_equal(R["owner"][fpos] - lo, r["owner"])
        np.testing.assert_array_equal(R["neighbour"][fpos] - lo, r["neighbour"])
        np.testing.assert_array_equal(R["w"][fpos], r["w"])
        np.testing.assert_array_equal(R["k"][fpos], r["k"])
        # boundary faces: the member's boundary block keeps its relative order
        b0 = mb["bface_start"] - Fi
        bpos = np.flatnonzero((R["bface_perm"] >= b0) & (R["bface_perm"] < b0 + mb["n_boundary_faces"]))
        np.testing.assert_array_equal(R["bface_perm"][bpos] - b0, r["bface_perm"])
        np.testing.assert_array_equal(R["bowner"][bpos] - lo, r["bowner"])
