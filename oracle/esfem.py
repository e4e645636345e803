"""FP64 CPU oracle of the edge-based smoothed FEM (ES-FEM) with T4 elements.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP path.

The paper builds the face-based member of the S-FEM family and names the
others (Sec. 1); this is the edge-based one, defined the way the paper
defines its face domains (Sec. 2.1 STEP 2-4), with the edge in the role of
the face:

* smoothing domain of edge k = (a, b): in every tet e holding the edge, the
  part cut off by the edge, the centroids of the two faces of e through the
  edge, and the centroid of e, i.e. the two sub-tets (a, b, g_abc, g_e) and
  (a, b, g_abd, g_e), holding a sixth of e's volume; V_k = sum V_e / 6;
* smoothed gradient (the analogue of Eq. 7): b_I = (1 / V_k) * integral
  over the boundary of the domain of n N_I, evaluated exactly (N is linear
  in each tet) by the centroid rule on every triangle of every sub-tet,
  with outward normals; triangles shared by two sub-tets cancel;
* material: volume-weighted (lambda, mu) over the domain, as for faces;
* stiffness (the analogue of Eq. 9): K_k = V_k B^T c B over the support of
  the edge (all nodes of its tets), summed into the global matrix (Eq. 12)
  with the structural pattern kept.
Edges are numbered by ascending (a, b), a < b; supports ascend.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from oracle.fsfem import B_matrix, D_matrix, lame, tet_volume, tri_area

_EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def edge_table(tets: np.ndarray):
    """(edges [ne, 2] ascending, ptr [ne + 1], tet ids grouped by edge)."""
    tets = np.asarray(tets, np.int64)
    T = len(tets)
    a = np.concatenate([np.minimum(tets[:, i], tets[:, j]) for i, j in _EDGES])
    b = np.concatenate([np.maximum(tets[:, i], tets[:, j]) for i, j in _EDGES])
    t = np.tile(np.arange(T), 6)
    order = np.lexsort((t, b, a))
    a, b, t = a[order], b[order], t[order]
    first = np.ones(len(a), bool)
    first[1:] = (a[1:] != a[:-1]) | (b[1:] != b[:-1])
    starts = np.flatnonzero(first)
    ptr = np.append(starts, len(a))
    return np.stack([a[starts], b[starts]], axis=1), ptr, t


def _face_sum(P, W):
    """Sum over the 4 faces of sub-tets P [m, 4, 3] of n A N(centroid), N
    given at the 4 vertices as weights W [m, 4, n] -> [m, n, 3]."""
    out = np.zeros(W.shape[:1] + (W.shape[2], 3))
    for skip in range(4):
        idx = [i for i in range(4) if i != skip]
        A, B, C = P[:, idx[0]], P[:, idx[1]], P[:, idx[2]]
        n = np.cross(B - A, C - A)
        # orient outward: away from the sub-tet's remaining vertex
        s = np.sign(np.einsum("ij,ij->i", n, P[:, skip] - A))
        n = -s[:, None] * n                      # |n| = 2 * area
        area = tri_area(A, B, C)
        unit = n / np.linalg.norm(n, axis=1)[:, None]
        Nc = (W[:, idx[0]] + W[:, idx[1]] + W[:, idx[2]]) / 3.0   # N at the centroid
        out += Nc[:, :, None] * (unit * area[:, None])[:, None, :]
    return out


def smoothed_gradients(xyz: np.ndarray, tets: np.ndarray, edges=None):
    """Literal smoothed gradients of every edge domain.
    Returns (list of support node ids per edge, list of bbar [n_k, 3],
    V_k [ne])."""
    xyz = np.asarray(xyz, float)
    tets = np.asarray(tets, np.int64)
    E, ptr, etets = edge_table(tets) if edges is None else edges
    sup, bb = [], []
    Vk = np.zeros(len(E))
    for k in range(len(E)):
        a, b = E[k]
        tt = etets[ptr[k]:ptr[k + 1]]
        S = np.unique(tets[tt].ravel())
        loc = {int(v): i for i, v in enumerate(S)}
        n = len(S)
        Ps, Ws = [], []
        for t in tt:
            v = tets[t]
            others = [int(x) for x in v if x != a and x != b]
            X = xyz[v]
            wv = np.zeros((4, n))
            for i, x in enumerate(v):
                wv[i, loc[int(x)]] = 1.0
            pa, pb = np.flatnonzero(v == a)[0], np.flatnonzero(v == b)[0]
            g = X.mean(axis=0)
            wg = wv.mean(axis=0)
            for c in others:
                pc = np.flatnonzero(v == c)[0]
                gf = (X[pa] + X[pb] + X[pc]) / 3.0
                wf = (wv[pa] + wv[pb] + wv[pc]) / 3.0
                Ps.append(np.stack([X[pa], X[pb], gf, g]))
                Ws.append(np.stack([wv[pa], wv[pb], wf, wg]))
        Ps, Ws = np.array(Ps), np.array(Ws)
        V = tet_volume(Ps).sum()
        bk = _face_sum(Ps, Ws).sum(axis=0) / V
        sup.append(S)
        bb.append(bk)
        Vk[k] = V
    return sup, bb, Vk


def edge_material(tets, tet_vol, lam_t, mu_t, edges=None):
    """Volume-weighted (lambda, mu) of every edge domain."""
    E, ptr, etets = edge_table(tets) if edges is None else edges
    lam = np.zeros(len(E))
    mu = np.zeros(len(E))
    for k in range(len(E)):
        tt = etets[ptr[k]:ptr[k + 1]]
        w = tet_vol[tt] / 6.0
        lam[k] = np.dot(w, lam_t[tt]) / w.sum()
        mu[k] = np.dot(w, mu_t[tt]) / w.sum()
    return lam, mu


def assemble(xyz, tets, E, nu) -> sp.csr_matrix:
    """Global ES-FEM stiffness (structural pattern, sorted CSR)."""
    xyz = np.asarray(xyz, float)
    tets = np.asarray(tets, np.int64)
    T = len(tets)
    N = len(xyz)
    tv = tet_volume(xyz[tets])
    Et = np.full(T, float(E)) if np.ndim(E) == 0 else np.asarray(E, float)
    nut = np.full(T, float(nu)) if np.ndim(nu) == 0 else np.asarray(nu, float)
    lam_t, mu_t = lame(Et, nut)
    edges = edge_table(tets)
    sup, bb, Vk = smoothed_gradients(xyz, tets, edges)
    lam, mu = edge_material(tets, tv, lam_t, mu_t, edges)
    I, J, V = [], [], []
    for k in range(len(sup)):
        B = B_matrix(bb[k])
        K = Vk[k] * B.T @ D_matrix(lam[k], mu[k]) @ B
        dof = (3 * sup[k][:, None] + np.arange(3)).ravel()
        I.append(np.repeat(dof, len(dof)))
        J.append(np.tile(dof, len(dof)))
        V.append(K.ravel())
    K = sp.coo_matrix((np.concatenate(V), (np.concatenate(I), np.concatenate(J))),
                      shape=(3 * N, 3 * N)).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    return K


def assemble_rows(xyz, tets, E, nu, nodes):
    """Rows 3I..3I+2 of the global ES-FEM matrix for the given nodes, each
    as (sorted scalar columns, values [3, ncols]), from only the edges whose
    support holds I (the edges of the tets holding I)."""
    xyz = np.asarray(xyz, float)
    tets = np.asarray(tets, np.int64)
    T = len(tets)
    Et = np.full(T, float(E)) if np.ndim(E) == 0 else np.asarray(E, float)
    nut = np.full(T, float(nu)) if np.ndim(nu) == 0 else np.asarray(nu, float)
    lam_t, mu_t = lame(Et, nut)
    Ek, ptr, etets = edge_table(tets)
    key = Ek[:, 0] * len(xyz) + Ek[:, 1]
    out = {}
    for I in nodes:
        star = np.flatnonzero((tets == I).any(axis=1))
        cand = set()
        for t in star:
            v = tets[t]
            for i, j in _EDGES:
                a, b = min(v[i], v[j]), max(v[i], v[j])
                cand.add(int(np.searchsorted(key, a * len(xyz) + b)))
        acc = {}
        for k in sorted(cand):
            tt = etets[ptr[k]:ptr[k + 1]]
            sub_edges = (Ek[k:k + 1], np.array([0, len(tt)]), tt)
            sup, bb, Vk = smoothed_gradients(xyz, tets, sub_edges)
            tv = tet_volume(xyz[tets[tt]])
            w = tv / 6.0
            lam = np.dot(w, lam_t[tt]) / w.sum()
            mu = np.dot(w, mu_t[tt]) / w.sum()
            B = B_matrix(bb[0])
            K = Vk[0] * B.T @ D_matrix(lam, mu) @ B
            S = sup[0]
            p = int(np.flatnonzero(S == I)[0])
            for q, J in enumerate(S):
                blk = K[3 * p:3 * p + 3, 3 * q:3 * q + 3]
                acc[int(J)] = acc.get(int(J), 0.0) + blk
        cols = sorted(acc)
        vals = np.zeros((3, 3 * len(cols)))
        for i, J in enumerate(cols):
            vals[:, 3 * i:3 * i + 3] = acc[J]
        sc = (3 * np.array(cols)[:, None] + np.arange(3)).ravel()
        out[int(I)] = (sc, vals)
    return out
