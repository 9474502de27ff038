"""Slab partition maps (difvm_partition_*; host only, no device): checked against a brute-force
recomputation from the whole mesh's renumbering (difvm_mesh_renumber_host)."""
import numpy as np
import pytest

from paper_2603_15920_amd import binding as B
from paper_2603_15920_amd import meshgen as mg


def brute_force(m, n_parts):
    r = B.difvm_mesh_renumber_host(m)
    nc = m.n_cells
    own, nbr, bown = r["owner"], r["neighbour"], r["bowner"]
    lo = [p * nc // n_parts for p in range(n_parts + 1)]
    part_of = np.searchsorted(np.array(lo[1:]), np.arange(nc), side="right")
    parts = []
    for p in range(n_parts):
        a, b = lo[p], lo[p + 1]
        mine_o = (own >= a) & (own < b)
        mine_n = (nbr >= a) & (nbr < b)
        ghosts = np.unique(np.concatenate([nbr[mine_o & ~mine_n], own[mine_n & ~mine_o]]))
        faces = np.nonzero(mine_o | mine_n)[0]
        bfaces = np.nonzero((bown >= a) & (bown < b))[0]
        parts.append(dict(lo=a, hi=b, ghosts=ghosts, faces=faces, bfaces=bfaces))
    return parts, part_of


@pytest.mark.parametrize("mesh_fn,n_parts", [
    (lambda: mg.tube(n=8, m=4, layers=44, L=2.0, seed=2603013), 8),
    (lambda: mg.kuhn_cube(10, jitter=0.15, patches="channel", seed=2603002), 3),
    (lambda: mg.cavity(8), 5),
    (lambda: mg.cavity(4), 1),
])
def test_partition_maps_match_brute_force(mesh_fn, n_parts):
    m = mesh_fn()
    P = B.Partition(m, n_parts)
    ref, part_of = brute_force(m, n_parts)
    total_send = total_ghost = 0
    owned = np.zeros(m.n_cells, np.int32)
    for p in range(n_parts):
        info, mp, rf = P.info[p], P.maps[p], ref[p]
        assert (info["cell_lo"], info["cell_hi"]) == (rf["lo"], rf["hi"])
        assert info["n_owned"] == rf["hi"] - rf["lo"]
        owned[rf["lo"]:rf["hi"]] += 1
        cg = mp["cell_global"]
        np.testing.assert_array_equal(cg[:info["n_owned"]], np.arange(rf["lo"], rf["hi"]))
        np.testing.assert_array_equal(cg[info["n_owned"]:], rf["ghosts"])
        np.testing.assert_array_equal(mp["face_global"], rf["faces"])
        np.testing.assert_array_equal(mp["bface_global"], rf["bfaces"])
        # ghosts grouped by owning part
        g_part = part_of[rf["ghosts"]]
        assert np.all(np.diff(g_part) >= 0)
        np.testing.assert_array_equal(mp["recv_start"], np.searchsorted(g_part, np.arange(n_parts + 1)))
        total_ghost += info["n_ghost"]
        total_send += info["n_send"]
    assert np.all(owned == 1)
    assert total_send == total_ghost
    # what p sends to q is what q receives from p, row for row
    for p in range(n_parts):
        for q in range(n_parts):
            sp, rq = P.maps[p], P.maps[q]
            sent = sp["send_cells"][sp["send_start"][q]:sp["send_start"][q + 1]] + P.info[p]["cell_lo"]
            got = rq["cell_global"][P.info[q]["n_owned"]:][rq["recv_start"][p]:rq["recv_start"][p + 1]]
            np.testing.assert_array_equal(sent, got)
    P.close()


def test_tube_slabs_have_at_most_two_neighbours():
    # RCM level sets sweep along the tube: each slab touches only the slabs before and after it
    m = mg.tube(n=8, m=4, layers=44, L=2.0, seed=2603013)
    P = B.Partition(m, 8)
    nb = [i["n_neighbours"] for i in P.info]
    assert nb[0] == 1 and nb[-1] == 1 and all(k == 2 for k in nb[1:-1]), nb


def test_partition_errors():
    m = mg.cavity(4)
    with pytest.raises(B.DifvmError) as e:
        B.Partition(m, 0)
    assert e.value.status == B.ERR_INVALID_ARG
    with pytest.raises(B.DifvmError) as e:
        B.Partition(m, m.n_cells + 1)
    assert e.value.status == B.ERR_INVALID_ARG
    P = B.Partition(m, 2)
    with pytest.raises(B.DifvmError):
        B.difvm_partition_info(P.h, 2)
    P.close()
