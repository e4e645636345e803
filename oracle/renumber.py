"""Node renumbering and TetGen mesh files, plain CPU reference.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP path.

The paper builds its matrices from TetGen's node / element / face files
(Sec. 3.2) and solves with a direct solver whose cost and memory depend on
the bandwidth; the GPU path keeps its x-gathers local for the same reason.
Unstructured generators number nodes arbitrarily, so the path offers a
reverse Cuthill-McKee ordering of the mesh's node graph, defined here step
by step so that the device ordering can be compared index for index:

* graph: nodes are adjacent when they share a tetrahedron (the edges of
  the tets); deg(v) = number of distinct neighbours.
* pseudo-peripheral start (George & Liu 1979): r = the node of least
  (deg, id) among the nodes still to be numbered; repeat: build r's
  breadth-first level structure; x = the node of least (deg, id) in its
  last level; if x's level structure is deeper than r's, r = x and repeat,
  otherwise start from r.
* Cuthill-McKee (1969): number r first; then, in numbering order, each node
  numbers its not-yet-numbered neighbours in increasing (deg, id).  A node
  is thus numbered by its earliest-numbered neighbour in the previous
  level, and a level's nodes are ordered by (that neighbour's number, deg,
  id).  Components are numbered one after the other.
* reverse (George 1971): new number of the node numbered k is N - 1 - k.

TetGen files (as TetGen writes them; '#' starts a comment):
  .node: "<#points> <dim=3> <#attributes> <#markers 0|1>", then per point
         "<index> <x> <y> <z> [attributes] [marker]";
  .ele:  "<#tets> <nodes per tet> <#attributes>", then
         "<index> <n1> <n2> <n3> <n4> [more nodes] [attributes]";
  .face: "<#faces> <#markers 0|1>", then "<index> <n1> <n2> <n3> [marker]"
         (TetGen may append adjacent-tet columns; they are ignored).
The first point index (0 or 1) fixes the base of every node reference.
"""
from __future__ import annotations

from collections import deque

import numpy as np


# ----------------------------------------------------------------- the graph
def node_graph(n_nodes: int, tets: np.ndarray) -> list[np.ndarray]:
    """Sorted distinct neighbours of every node (nodes sharing a tet)."""
    tets = np.asarray(tets, np.int64)
    src = np.repeat(tets, 4, axis=1).reshape(-1)      # a a a a b b b b ...
    dst = np.tile(tets, (1, 4)).reshape(-1)           # a b c d a b c d ...
    keep = src != dst
    pairs = np.unique(src[keep] * n_nodes + dst[keep])
    s, d = pairs // n_nodes, pairs % n_nodes
    ptr = np.searchsorted(s, np.arange(n_nodes + 1))
    return [d[ptr[i]:ptr[i + 1]] for i in range(n_nodes)]


def bfs_levels(adj, start: int, allowed: np.ndarray) -> list[list[int]]:
    """Breadth-first level structure from start over the allowed nodes."""
    seen = {start}
    levels = [[start]]
    while True:
        nxt = []
        for u in levels[-1]:
            for v in adj[u]:
                v = int(v)
                if allowed[v] and v not in seen:
                    seen.add(v)
                    nxt.append(v)
        if not nxt:
            return levels
        levels.append(nxt)


def pseudo_peripheral(adj, deg: np.ndarray, allowed: np.ndarray) -> int:
    """George-Liu start node among the allowed nodes (see module doc)."""
    cand = np.flatnonzero(allowed)
    r = int(cand[np.lexsort((cand, deg[cand]))[0]])
    levels = bfs_levels(adj, r, allowed)
    while True:
        last = np.array(levels[-1])
        x = int(last[np.lexsort((last, deg[last]))[0]])
        lx = bfs_levels(adj, x, allowed)
        if len(lx) > len(levels):
            r, levels = x, lx
        else:
            return r


def cuthill_mckee(n_nodes: int, tets: np.ndarray) -> np.ndarray:
    """order[k] = old id of the node numbered k (Cuthill-McKee)."""
    adj = node_graph(n_nodes, tets)
    deg = np.array([len(a) for a in adj], np.int64)
    todo = np.ones(n_nodes, bool)
    order = []
    while todo.any():
        # the component of the least-(deg, id) node still to be numbered
        cand = np.flatnonzero(todo)
        seed = int(cand[np.lexsort((cand, deg[cand]))[0]])
        comp = np.zeros(n_nodes, bool)
        for lev in bfs_levels(adj, seed, todo):
            comp[lev] = True
        r = pseudo_peripheral(adj, deg, comp)
        todo[r] = False
        order.append(r)
        q = deque([r])
        while q:
            u = q.popleft()
            nb = [int(v) for v in adj[u] if todo[v]]
            nb.sort(key=lambda v: (deg[v], v))
            for v in nb:
                todo[v] = False
                order.append(v)
                q.append(v)
    return np.array(order, np.int64)


def reverse_cuthill_mckee(n_nodes: int, tets: np.ndarray) -> np.ndarray:
    """perm[new] = old node id of the reverse Cuthill-McKee numbering."""
    return cuthill_mckee(n_nodes, tets)[::-1].copy()


def bandwidth(n_nodes: int, tets: np.ndarray) -> int:
    """max |i - j| over nodes i, j sharing a tet."""
    t = np.asarray(tets, np.int64)
    return int((t.max(axis=1) - t.min(axis=1)).max())


def apply_permutation(perm: np.ndarray, xyz: np.ndarray, tets: np.ndarray):
    """Renumbered (xyz, tets) for perm[new] = old."""
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(perm))
    return np.asarray(xyz)[perm], inv[np.asarray(tets)]


# -------------------------------------------------------------- TetGen files
def _rows(path):
    out = []
    with open(path) as fh:
        for line in fh:
            line = line.split("#", 1)[0].split()
            if line:
                out.append(line)
    return out


def read_tetgen(stem: str):
    """(xyz [N,3], tets [T,4] 0-based, faces [F,3] 0-based or None,
    face markers [F] or None) from stem.node / stem.ele / stem.face."""
    import os
    rows = _rows(stem + ".node")
    n, dim, n_attr, n_mark = (int(v) for v in rows[0][:4])
    assert dim == 3
    pts = rows[1:1 + n]
    base = int(pts[0][0])
    idx = np.array([int(r[0]) for r in pts]) - base
    xyz = np.empty((n, 3))
    xyz[idx] = np.array([[float(v) for v in r[1:4]] for r in pts])
    rows = _rows(stem + ".ele")
    t, npt = int(rows[0][0]), int(rows[0][1])
    assert npt == 4
    ele = rows[1:1 + t]
    tets = np.array([[int(v) for v in r[1:5]] for r in ele], np.int64) - base
    faces = marks = None
    if os.path.exists(stem + ".face"):
        rows = _rows(stem + ".face")
        f, has_mark = int(rows[0][0]), int(rows[0][1])
        fr = rows[1:1 + f]
        faces = np.array([[int(v) for v in r[1:4]] for r in fr], np.int64) - base
        marks = np.array([int(r[4]) for r in fr], np.int64) if has_mark else None
    return xyz, tets, faces, marks


def write_tetgen(stem: str, xyz, tets, faces=None, marks=None, base: int = 1):
    """Writes the three files in TetGen's layout (used to make test inputs)."""
    xyz = np.asarray(xyz, float)
    with open(stem + ".node", "w") as fh:
        fh.write(f"# generated\n{len(xyz)} 3 0 0\n")
        for i, p in enumerate(xyz):
            fh.write(f"{i + base} {float(p[0])!r} {float(p[1])!r} {float(p[2])!r}\n")
    with open(stem + ".ele", "w") as fh:
        fh.write(f"{len(tets)} 4 0\n")
        for i, t in enumerate(np.asarray(tets)):
            fh.write(f"  {i + base}  {t[0] + base} {t[1] + base} {t[2] + base} {t[3] + base}\n")
    if faces is not None:
        with open(stem + ".face", "w") as fh:
            fh.write(f"{len(faces)} {1 if marks is not None else 0}\n")
            for i, f in enumerate(np.asarray(faces)):
                m = f" {int(marks[i])}" if marks is not None else ""
                fh.write(f"{i + base} {f[0] + base} {f[1] + base} {f[2] + base}{m}  # face\n")
