"""The library's TetGen reader (host code, no GPU needed) against the
reference reader and hand-written files, and its error handling."""
import os

import numpy as np
import pytest

from oracle import renumber as R
from paper_2001_08849_amd import meshgen as mg

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tetgen")


@pytest.fixture(scope="module")
def S():
    from paper_2001_08849_amd import sfem
    return sfem


def test_hand_written_cube(S):
    got = S.read_tetgen(os.path.join(GOLD, "cube"))
    ref = R.read_tetgen(os.path.join(GOLD, "cube"))
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)


@pytest.mark.parametrize("base", [0, 1])
def test_generated_files_match_reference_reader(S, tmp_path, base):
    m = mg.box_mesh(6, 3, 4, 3.0, 1.5, 2.0, jitter=0.2, seed=8)
    sh = np.random.default_rng(1).permutation(m.n_nodes)
    xyz, tets = R.apply_permutation(sh, m.xyz, m.tets)
    inv = np.empty_like(sh)
    inv[sh] = np.arange(len(sh))
    faces = inv[m.end_tris]
    marks = np.arange(len(faces)) % 4
    stem = str(tmp_path / "mesh")
    R.write_tetgen(stem, xyz, tets, faces, marks, base=base)
    got = S.read_tetgen(stem)
    ref = R.read_tetgen(stem)
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)
    assert np.array_equal(got[0], xyz) and np.array_equal(got[1], tets)


def test_without_face_file(S, tmp_path):
    m = mg.box_mesh(2, 2, 2, 1.0, 1.0, 1.0, jitter=0.0, seed=0)
    stem = str(tmp_path / "nf")
    R.write_tetgen(stem, m.xyz, m.tets)
    xyz, tets, faces, marks = S.read_tetgen(stem)
    assert faces is None and marks is None and np.array_equal(tets, m.tets)


def test_errors(S, tmp_path):
    with pytest.raises(S.SfemError, match="cannot open"):
        S.read_tetgen(str(tmp_path / "missing"))
    stem = str(tmp_path / "bad")
    m = mg.box_mesh(2, 1, 1, 1.0, 1.0, 1.0, jitter=0.0, seed=0)
    R.write_tetgen(stem, m.xyz, m.tets)
    with open(stem + ".ele") as fh:
        lines = fh.readlines()
    # a node reference past the last point
    bad = lines[:]
    bad[1] = f"  1  1 2 3 {m.n_nodes + 1}\n"
    open(stem + ".ele", "w").writelines(bad)
    with pytest.raises(S.SfemError, match="out of range"):
        S.read_tetgen(stem)
    # quadratic (10-node) tets are not T4
    bad = lines[:]
    bad[0] = f"{len(m.tets)} 10 0\n"
    open(stem + ".ele", "w").writelines(bad)
    with pytest.raises(S.SfemError, match="4-node"):
        S.read_tetgen(stem)
    # a malformed coordinate
    open(stem + ".ele", "w").writelines(lines)
    with open(stem + ".node") as fh:
        nl = fh.readlines()
    nl[3] = "2 0.5 zero 0.0\n"
    open(stem + ".node", "w").writelines(nl)
    with pytest.raises(S.SfemError, match="bad number"):
        S.read_tetgen(stem)
