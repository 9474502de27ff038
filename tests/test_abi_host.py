"""C-ABI checks that need no GPU: the library loads and exports every symbol the header declares; the
host renumbering matches the oracle's bit for bit (integers and permuted geometry); invalid meshes are
rejected with DIFVM_ERR_INVALID_MESH."""
import os
import re

import numpy as np
import pytest

from oracle import oracle as O
from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "difvm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:difvm_status|int|const char\*)\s+(difvm_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    lib = B.lib()
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B._SIGS), "binding signatures and header disagree"
    assert B.difvm_abi_version() == 1


MESHES = {
    "cavity": lambda: mg.cavity(12),
    "kuhn": lambda: mg.kuhn_cube(7, patches="sides", seed=5),
    "tube": lambda: mg.tube(n=6, m=3, layers=5),
    "channel_wk": lambda: mg.kuhn_cube(3, patches="channel", nxyz=(6, 3, 3), hi=(2.0, 1.0, 1.0)),
    "hex": lambda: mg.hex_box(5, 4, 3, A=np.array([[1, 0.3, 0], [0, 1, 0.2], [0, 0, 1.0]])),
}


def shuffled(m, seed):
    """Same mesh with internal and boundary faces permuted inside their blocks and random orientation
    of internal faces (exercises the flip and sort paths)."""
    rng = np.random.default_rng(seed)
    Fi = m.n_internal_faces
    perm = rng.permutation(Fi)
    flip = rng.random(Fi) < 0.5
    own = m.owner[:Fi][perm].copy()
    nbr = m.neighbour[perm].copy()
    own[flip], nbr[flip] = nbr[flip], own[flip].copy()
    S = m.Sf[:Fi][perm].copy()
    S[flip] *= -1.0
    w = m.w[perm].copy()
    w[flip] = 1.0 - w[flip]
    bperm = []
    for p in m.patches:
        bperm.append(p.start + rng.permutation(p.size))
    bperm = np.concatenate(bperm) if bperm else np.zeros(0, int)
    return mg.Mesh(owner=np.concatenate([own, m.owner[bperm]]).astype(np.int32), neighbour=nbr.astype(np.int32),
                   Sf=np.concatenate([S, m.Sf[bperm]]), Cf=np.concatenate([m.Cf[:Fi][perm], m.Cf[bperm]]), C=m.C,
                   V=m.V, w=w, patches=m.patches)


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("shuffle", [False, True])
@pytest.mark.parametrize("scheme", sorted(B.NONORTH))
def test_renumbering_bit_exact(name, shuffle, scheme):
    m = MESHES[name]()
    if shuffle:
        m = shuffled(m, 7)
    m.meta["nonorth"] = scheme
    lib = B.difvm_mesh_renumber_host(m, flags=B.RENUMBER_RCM | B.NONORTH[scheme], geometry=True)
    ora = O.renumber(m)
    for k in ("cell_perm", "face_perm", "face_flip", "owner", "neighbour", "own_start", "losort", "losort_start",
              "bface_perm", "bowner"):
        np.testing.assert_array_equal(lib[k], ora[k], err_msg=k)
    # permuted geometry: oracle geometry (user orientation) carried through the oracle's permutation
    Fi = m.n_internal_faces
    delta, kv, db = O.geometry(m)
    fp, fl = ora["face_perm"], ora["face_flip"].astype(bool)
    sgn = np.where(fl, -1.0, 1.0)[:, None]
    S_exp = np.concatenate([m.Sf[:Fi][fp] * sgn, m.Sf[Fi:][ora["bface_perm"]]])
    w_exp = np.where(fl, 1.0 - m.w[fp], m.w[fp])
    d_exp = np.concatenate([delta[fp], db[ora["bface_perm"]]])
    k_exp = kv[fp] * sgn
    # exact equality of every value; the only freedom is the sign of an exact zero, since
    # (-S) - delta (-d) rounds a vanishing component to +0 where -(S - delta d) gives -0
    for key, exp in (("S", S_exp), ("w", w_exp), ("delta", d_exp), ("k", k_exp)):
        got, exp = lib[key], np.ascontiguousarray(exp)
        assert np.array_equal(got, exp), key
        nz = exp != 0
        assert np.array_equal(got[nz].view(np.uint64), exp[nz].view(np.uint64)), key


def test_identity_order_flag():
    m = mg.kuhn_cube(4, patches="walls")
    r = B.difvm_mesh_renumber_host(m, flags=0)
    assert np.array_equal(r["cell_perm"], np.arange(m.n_cells))
    assert np.array_equal(r["cell_perm"], O.renumber(m, rcm=False)["cell_perm"])


def test_unknown_flag_bits_rejected():
    m = mg.kuhn_cube(3, patches="walls")
    for flags in (8, 16, 1 << 31):
        with pytest.raises(B.DifvmError) as e:
            B.difvm_mesh_renumber_host(m, flags=B.RENUMBER_RCM | flags)
        assert e.value.status == B.ERR_INVALID_ARG


def _expect_invalid(m, code=B.ERR_INVALID_MESH):
    with pytest.raises(B.DifvmError) as e:
        B.difvm_mesh_renumber_host(m)
    assert e.value.status == code, str(e.value)


def test_invalid_meshes_rejected():
    base = mg.kuhn_cube(3, patches="walls")
    Fi = base.n_internal_faces

    def cp():
        return mg.Mesh(base.owner.copy(), base.neighbour.copy(), base.Sf.copy(), base.Cf.copy(), base.C.copy(),
                       base.V.copy(), base.w.copy(), [mg.Patch(**vars(p)) for p in base.patches])
    m = cp(); m.V[3] = -1.0; _expect_invalid(m)
    m = cp(); m.neighbour[0] = m.owner[0]; _expect_invalid(m)
    m = cp(); m.owner[5] = m.n_cells; _expect_invalid(m)
    m = cp(); m.Sf[2] *= -1.0; _expect_invalid(m)                      # S.d <= 0 on an internal face
    m = cp(); m.Sf[Fi + 1] *= -1.0; _expect_invalid(m)                 # and on a boundary face
    m = cp(); m.patches[0].size -= 1; _expect_invalid(m)               # patches do not tile the boundary
    m = cp(); m.patches[0].p_type = 7; _expect_invalid(m)
