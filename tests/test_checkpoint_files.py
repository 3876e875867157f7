"""Host checks of checkpoint files (hm_file_info, the checks hm_load applies).

A small checkpoint is written here field by field in the documented format:
4 points on a line, leaf size 1, kmax 1; cluster tree root {0..3} with sons
{0,1} and {2,3}, each with two single-point sons; block tree root with the four
sons (t0,s0) ... (t1,s1), the diagonal ones split once more into single-point
leaves.  Each damaged copy changes one field that a valid file fixes and must
be refused; no device is used.
"""
import struct

import numpy as np
import pytest

from paper_1703_09085_amd import hm

MAGIC = b"HMATRIX1"
DENSE, RK, NONLEAF = 2, 1, 0


def layout():
    # clusters (pre-order): off, size, level, nsons, son0, son1, parent
    cl = [[0, 4, 0, 2, 1, 4, -1], [0, 2, 1, 2, 2, 3, 0], [0, 1, 2, 0, -1, -1, 1], [1, 1, 2, 0, -1, -1, 1],
          [2, 2, 1, 2, 5, 6, 0], [2, 1, 2, 0, -1, -1, 4], [3, 1, 2, 0, -1, -1, 4]]
    # blocks: t, s, kind, nt, ns, son0, parent  (sons contiguous, row-major)
    bl = [[0, 0, NONLEAF, 2, 2, 1, -1],
          [1, 1, NONLEAF, 2, 2, 5, 0], [1, 4, RK, 0, 0, -1, 0], [4, 1, RK, 0, 0, -1, 0], [4, 4, NONLEAF, 2, 2, 9, 0],
          [2, 2, DENSE, 0, 0, -1, 1], [2, 3, DENSE, 0, 0, -1, 1], [3, 2, DENSE, 0, 0, -1, 1], [3, 3, DENSE, 0, 0, -1, 1],
          [5, 5, DENSE, 0, 0, -1, 4], [5, 6, DENSE, 0, 0, -1, 4], [6, 5, DENSE, 0, 0, -1, 4], [6, 6, DENSE, 0, 0, -1, 4]]
    return dict(dim=1, kmax=1, perm=[0, 1, 2, 3], cl=cl, bl=bl, ranks=[0] * len(bl))


def values(L):
    size = [c[1] for c in L["cl"]]
    tot = 0
    for t, s, kind, *_ in L["bl"]:
        if kind == DENSE:
            tot += size[t] * size[s]
        elif kind == RK:
            tot += (size[t] + size[s]) * min(size[t], size[s], L["kmax"])
    return max(tot, 1)


def write(path, L, pool=None):
    pool = values(L) if pool is None else pool
    out = bytearray(MAGIC)
    out += struct.pack("<ii", L["dim"], L["kmax"])
    out += struct.pack("<q", len(L["perm"])) + struct.pack(f"<{len(L['perm'])}i", *L["perm"])
    out += struct.pack("<q", len(L["cl"]))
    for c in L["cl"]:
        lo, hi = float(c[0]), float(c[0] + c[1] - 1)
        out += struct.pack("<7i", *c) + struct.pack("<3d", lo, 0, 0) + struct.pack("<3d", hi, 0, 0)
    out += struct.pack("<q", len(L["bl"]))
    for b in L["bl"]:
        out += struct.pack("<7i", *b)
    out += struct.pack(f"<{len(L['ranks'])}i", *L["ranks"])
    out += struct.pack("<q", pool) + np.arange(pool, dtype=np.float64).tobytes()
    path.write_bytes(bytes(out))
    return path


def test_valid_file_is_accepted(tmp_path):
    L = layout()
    assert hm.file_info(write(tmp_path / "ok.hm", L)) == (4, 7, 13)


def damage(kind):
    L = layout()
    if kind == "perm_repeats":
        L["perm"][3] = 0
    elif kind == "perm_out_of_range":
        L["perm"][3] = 4
    elif kind == "cluster_son_negative":
        L["cl"][1][4] = -3
    elif kind == "cluster_son_cycle":
        L["cl"][4][4] = 0
    elif kind == "cluster_sons_do_not_split":
        L["cl"][6][0] = 2
    elif kind == "cluster_bad_parent":
        L["cl"][2][6] = 4
    elif kind == "block_son_self":
        L["bl"][1][5] = 1
    elif kind == "block_son_earlier":
        L["bl"][4][5] = 0
    elif kind == "block_nt_negative":
        L["bl"][0][3] = -1
    elif kind == "block_ns_mismatch":
        L["bl"][0][4] = 1
    elif kind == "block_wrong_son_cluster":
        L["bl"][2][0] = 2
    elif kind == "block_parent_unchecked":
        L["bl"][6][6] = 0
    elif kind == "nonleaf_on_leaf_cluster":
        L["bl"][5][2] = NONLEAF
    elif kind == "rank_above_capacity":
        L["ranks"][2] = 2
    elif kind == "rank_on_dense":
        L["ranks"][5] = 1
    elif kind == "root_not_whole":
        L["cl"][0][1] = 3
    return L


KINDS = ["perm_repeats", "perm_out_of_range", "cluster_son_negative", "cluster_son_cycle",
         "cluster_sons_do_not_split", "cluster_bad_parent", "block_son_self", "block_son_earlier",
         "block_nt_negative", "block_ns_mismatch", "block_wrong_son_cluster", "block_parent_unchecked",
         "nonleaf_on_leaf_cluster", "rank_above_capacity", "rank_on_dense", "root_not_whole"]


@pytest.mark.parametrize("kind", KINDS)
def test_damaged_structure_is_refused(tmp_path, kind):
    path = write(tmp_path / f"{kind}.hm", damage(kind))
    with pytest.raises(hm.HMError) as e:
        hm.file_info(path)
    assert e.value.status == 1


def test_values_must_match_the_structure(tmp_path):
    L = layout()
    for pool in (values(L) - 1, values(L) + 1):
        with pytest.raises(hm.HMError):
            hm.file_info(write(tmp_path / "v.hm", L, pool=pool))
    ok = write(tmp_path / "t.hm", L)
    data = ok.read_bytes()
    (tmp_path / "short.hm").write_bytes(data[:-8])
    with pytest.raises(hm.HMError):
        hm.file_info(tmp_path / "short.hm")
    (tmp_path / "long.hm").write_bytes(data + b"\0" * 8)
    with pytest.raises(hm.HMError):
        hm.file_info(tmp_path / "long.hm")
    with pytest.raises(hm.HMError):
        hm.file_info(tmp_path / "missing.hm")
