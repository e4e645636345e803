"""Pins of the renumbering / TetGen-file reference (oracle/renumber.py)
against hand-derived orderings, closed forms and an independent library
routine, plus the TetGen reader on a hand-written file."""
import os

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import reverse_cuthill_mckee as scipy_rcm

from oracle import renumber as R
from paper_2001_08849_amd import meshgen as mg

GOLD = os.path.join(os.path.dirname(__file__), "golden", "tetgen")


def test_two_tets_hand_ordering():
    # tets (3,0,4,1) and (0,4,1,2): 3 and 2 have 3 neighbours, 0, 1, 4 have 4.
    # Start: least (deg, id) = 2; its levels [2] [0 1 4] [3]; the last
    # level's node 3 is no deeper, so CM starts at 2, numbers 0, 1, 4 (equal
    # degree, by id), then 0 numbers 3.  Reverse: 3 4 1 0 2.
    tets = np.array([[3, 0, 4, 1], [0, 4, 1, 2]])
    assert list(R.cuthill_mckee(5, tets)) == [2, 0, 1, 4, 3]
    assert list(R.reverse_cuthill_mckee(5, tets)) == [3, 4, 1, 0, 2]


def test_tet_chain_recovers_the_line():
    # nodes along a line, tet (i, i+1, i+2, i+3): the optimal bandwidth is 3
    # and Cuthill-McKee must walk the line from an end (each node numbers
    # exactly one new neighbour after the first level)
    n = 200
    rng = np.random.default_rng(3)
    lab = rng.permutation(n)                      # lab[line position] = label
    tets = lab[np.arange(n - 3)[:, None] + np.arange(4)]
    perm = R.reverse_cuthill_mckee(n, tets)
    pos = np.empty(n, np.int64)
    pos[perm] = np.arange(n)
    line = pos[lab]                               # new number along the line
    assert np.all(np.abs(np.diff(line)) == 1)
    # CM starts at the end with the smaller label; the reverse ends there
    start_end = 0 if lab[0] < lab[-1] else n - 1
    assert perm[-1] == lab[start_end]
    _, t2 = R.apply_permutation(perm, np.zeros((n, 3)), tets)
    assert R.bandwidth(n, t2) == 3


def test_graph_matches_tet_edges_brute_force():
    m = mg.box_mesh(3, 2, 2, 1.0, 1.0, 1.0, jitter=0.1, seed=2)
    adj = R.node_graph(m.n_nodes, m.tets)
    want = [set() for _ in range(m.n_nodes)]
    for t in m.tets:
        for a in t:
            for b in t:
                if a != b:
                    want[a].add(int(b))
    assert all(list(adj[i]) == sorted(want[i]) for i in range(m.n_nodes))


def test_bandwidth_close_to_scipy_rcm_on_shuffled_meshes():
    for dims, seed in (((12, 5, 4), 1), ((30, 4, 4), 2), ((8, 8, 8), 3)):
        m = mg.box_mesh(*dims, 1.0 * dims[0], 1.0 * dims[1], 1.0 * dims[2], jitter=0.1, seed=seed)
        rng = np.random.default_rng(seed)
        sh = rng.permutation(m.n_nodes)
        xyz, tets = R.apply_permutation(sh, m.xyz, m.tets)
        perm = R.reverse_cuthill_mckee(m.n_nodes, tets)
        assert np.array_equal(np.sort(perm), np.arange(m.n_nodes))
        _, t_ours = R.apply_permutation(perm, xyz, tets)
        adj = R.node_graph(m.n_nodes, tets)
        rows = np.repeat(np.arange(m.n_nodes), [len(a) for a in adj])
        G = sp.csr_matrix((np.ones(len(rows)), (rows, np.concatenate(adj))),
                          shape=(m.n_nodes, m.n_nodes))
        ps = scipy_rcm(G, symmetric_mode=True)
        _, t_sp = R.apply_permutation(np.asarray(ps, np.int64), xyz, tets)
        b_ours, b_sp, b_shuf = (R.bandwidth(m.n_nodes, t) for t in (t_ours, t_sp, tets))
        print(f"{dims}: bandwidth shuffled {b_shuf}, ours {b_ours}, scipy RCM {b_sp}")
        assert b_ours <= 1.25 * b_sp + 2 and b_ours < b_shuf / 3


def test_components_numbered_one_after_the_other():
    a = mg.box_mesh(4, 2, 2, 1.0, 1.0, 1.0, jitter=0.0, seed=0)
    b = mg.box_mesh(3, 3, 2, 1.0, 1.0, 1.0, jitter=0.0, seed=0)
    n = a.n_nodes + b.n_nodes
    tets = np.vstack([a.tets, b.tets + a.n_nodes])
    perm = R.reverse_cuthill_mckee(n, tets)
    comp = (perm >= a.n_nodes).astype(int)
    assert np.count_nonzero(np.diff(comp)) == 1


def test_read_hand_written_tetgen_cube():
    xyz, tets, faces, marks = R.read_tetgen(os.path.join(GOLD, "cube"))
    corners = np.array([[i & 1, (i >> 1) & 1, (i >> 2) & 1] for i in range(8)], float)
    assert np.array_equal(xyz, corners)
    assert np.array_equal(tets, [[1, 2, 4, 7], [0, 1, 2, 4], [1, 2, 3, 7], [1, 4, 5, 7],
                                 [2, 4, 6, 7]])
    P = xyz[tets]
    vol = np.abs(np.linalg.det(P[:, 1:] - P[:, :1])) / 6
    assert np.isclose(vol.sum(), 1.0)
    assert faces.shape == (12, 3) and list(marks[:4]) == [1, 1, 2, 2] and not marks[4:].any()


def test_tetgen_write_read_round_trip(tmp_path):
    m = mg.box_mesh(3, 2, 2, 1.5, 1.0, 1.0, jitter=0.2, seed=4)
    faces = m.end_tris
    marks = np.arange(len(faces)) % 3
    for base in (0, 1):
        stem = str(tmp_path / f"m{base}")
        R.write_tetgen(stem, m.xyz, m.tets, faces, marks, base=base)
        xyz, tets, f, mk = R.read_tetgen(stem)
        assert np.array_equal(xyz, m.xyz) and np.array_equal(tets, m.tets)
        assert np.array_equal(f, faces) and np.array_equal(mk, marks)
