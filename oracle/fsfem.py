"""FP64 CPU oracle of the face-based smoothed FEM (FS-FEM) with T4 elements.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It shares no code with the HIP path.

It is a plain, slow, literal reading of the paper (juSFEM, arXiv 2001.08849):

* Sec. 3.2 / Alg. 1  -- faces from the tetrahedra, split into exterior
  (one tet) and interior (two tets) rows with the opposite vertices.
* Sec. 2.1 STEP 2    -- smoothing domain of a face: the sub-tet(s) formed by
  the face and the centroid(s) of its tet(s) (Fig. 1).
* Eq. 10, Eq. 11     -- tet volume by the 4x4 determinant, triangle area by
  the cross product; STEP 3 of Sec. 3.3 -- unit normals by cross product.
* Eq. 7 + Table 1    -- smoothed gradients b_Ih from the P boundary
  triangles of the smoothing domain (P = 6 interior, 4 exterior), evaluated
  at the triangle centroids with the Table-1 shape-function values.
* Eq. 4, Eq. 9       -- B_I (6x3, Voigt rows xx,yy,zz,yz,xz,xy) and
  K_k = V_k B^T c B_k, one 12x12 (exterior) or 15x15 (interior) block per face.
* Eq. 12             -- COO triplets, exterior faces first, then interior
  faces; duplicates summed into CSR (the structural pattern is kept).
* STEP 5 (Sec. 2.1, Sec. 3.3) -- essential BCs by removing rows/columns
  (elimination; the penalty variant is an option), nodal loads.
* The solve: the paper uses a direct solver; the oracle offers a dense
  solve, a banded Cholesky solve (both exact up to rounding) and Jacobi PCG
  judged by the true residual.

Where the paper is silent or garbled this module takes these readings: an
exterior face's domain ABCF is bounded by the face ABC itself and the three
triangles through F, whose Gauss values follow the rule behind Table 1 (the
shape functions at each triangle's centroid); normals point out of the smoothing domain;
D is the standard isotropic matrix in the Voigt order of Eq. 4 (xx, yy, zz,
yz, xz, xy, engineering shears); a per-tet material enters as the
volume-weighted Lame constants of the domain; essential BCs are eliminated
by default; a uniform traction gives each node of a loaded triangle t A / 3.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

# --------------------------------------------------------------------- Table 1
# Shape-function values at the Gauss points (centroids) of the boundary
# triangles of an interior smoothing domain ABCFG, columns = nodes A,B,C,D,E
# (Table 1, rows g1..g6).  The named triangle each row belongs to follows from
# which vertices carry 5/12 and which centroid (F in ABCD, G in ABCE) appears.
TABLE1_INTERIOR = {
    "g1": ("ACF", (5 / 12, 1 / 12, 5 / 12, 1 / 12, 0.0)),
    "g2": ("ACG", (5 / 12, 1 / 12, 5 / 12, 0.0, 1 / 12)),
    "g3": ("BCG", (1 / 12, 5 / 12, 5 / 12, 0.0, 1 / 12)),
    "g4": ("BCF", (1 / 12, 5 / 12, 5 / 12, 1 / 12, 0.0)),
    "g5": ("ABF", (5 / 12, 5 / 12, 1 / 12, 1 / 12, 0.0)),
    "g6": ("ABG", (5 / 12, 5 / 12, 1 / 12, 0.0, 1 / 12)),
}
# Exterior smoothing domain ABCF (face ABC on the boundary, tet ABCD): the
# paper prints no table for it; the same rule (value of the linear shape
# functions at the triangle centroid, F carrying 1/4 of A,B,C,D) gives
TABLE1_EXTERIOR = {
    "ABC": (1 / 3, 1 / 3, 1 / 3, 0.0),
    "ACF": (5 / 12, 1 / 12, 5 / 12, 1 / 12),
    "BCF": (1 / 12, 5 / 12, 5 / 12, 1 / 12),
    "ABF": (5 / 12, 5 / 12, 1 / 12, 1 / 12),
}


# ------------------------------------------------------------- Eq. 10, Eq. 11
def tet_volume(P: np.ndarray) -> np.ndarray:
    """Eq. 10: V = |det[[x y z 1] for the 4 vertices]| / 6.  P: [...,4,3]."""
    M = np.concatenate([P, np.ones(P.shape[:-1] + (1,))], axis=-1)
    return np.abs(np.linalg.det(M)) / 6.0


def tri_area(A: np.ndarray, B: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Eq. 11: S = |AB x AC| / 2."""
    return 0.5 * np.linalg.norm(np.cross(B - A, C - A), axis=-1)


def unit_normal_away(A, B, C, away):
    """STEP 3 of the solver: unit normal of triangle ABC by the cross product
    of two edges, oriented to point away from the point `away` (the remaining
    vertex of the sub-tet the triangle bounds), i.e. outward."""
    n = np.cross(B - A, C - A)
    n = n / np.linalg.norm(n, axis=-1, keepdims=True)
    s = np.sign(np.einsum("...i,...i->...", n, away - A))
    return -s[..., None] * n


# ------------------------------------------------------------------- Alg. 1
def extract_faces(tets: np.ndarray):
    """Faces of the tetrahedra (Sec. 3.2, Alg. 1).

    Returns a dict:
      face_out : int64 [N_e, 5] = (a, b, c, tet, opp)        exterior faces
      face_in  : int64 [N_i, 7] = (a, b, c, t1, t2, o1, o2)  interior faces
      table    : int64 [N_f, 7] = all faces in ascending (a,b,c) order,
                 exterior rows carrying t2 = o2 = -1
    with a < b < c the sorted node ids of the face, t1 < t2 and o_i the vertex
    of tet t_i not on the face.  A face shared by more than two tets raises.
    """
    tets = np.asarray(tets, dtype=np.int64)
    T = tets.shape[0]
    rows = []
    for lv in range(4):  # face opposite local vertex lv
        others = np.delete(tets, lv, axis=1)
        tri = np.sort(others, axis=1)
        rows.append(np.column_stack([tri, np.arange(T), tets[:, lv]]))
    F = np.concatenate(rows, axis=0)  # (a, b, c, tet, opp)
    order = np.lexsort((F[:, 3], F[:, 2], F[:, 1], F[:, 0]))
    F = F[order]
    same = np.all(F[1:, :3] == F[:-1, :3], axis=1)
    start = np.concatenate([[True], ~same])
    gid = np.cumsum(start) - 1
    counts = np.bincount(gid)
    if counts.max(initial=0) > 2:
        raise ValueError("non-manifold mesh: a face is shared by more than two tets")
    firsts = np.flatnonzero(start)
    nf = firsts.size
    table = np.full((nf, 7), -1, dtype=np.int64)
    table[:, 0:3] = F[firsts, 0:3]
    table[:, 3] = F[firsts, 3]
    table[:, 5] = F[firsts, 4]
    two = counts == 2
    table[two, 4] = F[firsts[two] + 1, 3]
    table[two, 6] = F[firsts[two] + 1, 4]
    face_out = table[~two][:, [0, 1, 2, 3, 5]]
    face_in = table[two]
    return {"face_out": face_out, "face_in": face_in, "table": table}


# ------------------------------------------------------------------- Eq. 4 / D
def B_matrix(b: np.ndarray) -> np.ndarray:
    """Eq. 4: B for nodes with gradients b [..., n, 3] -> [..., 6, 3n],
    Voigt rows xx, yy, zz, yz, xz, xy (engineering shear)."""
    n = b.shape[-2]
    B = np.zeros(b.shape[:-2] + (6, 3 * n))
    bx, by, bz = b[..., 0], b[..., 1], b[..., 2]
    B[..., 0, 0::3] = bx
    B[..., 1, 1::3] = by
    B[..., 2, 2::3] = bz
    B[..., 3, 1::3] = bz
    B[..., 3, 2::3] = by
    B[..., 4, 0::3] = bz
    B[..., 4, 2::3] = bx
    B[..., 5, 0::3] = by
    B[..., 5, 1::3] = bx
    return B


def lame(E, nu):
    E = np.asarray(E, dtype=np.float64)
    nu = np.asarray(nu, dtype=np.float64)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def D_matrix(lam, mu) -> np.ndarray:
    """Isotropic elasticity matrix c of Eq. 9 in the Voigt order of Eq. 4."""
    lam = np.asarray(lam, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    D = np.zeros(lam.shape + (6, 6))
    for i in range(3):
        for j in range(3):
            D[..., i, j] = lam
        D[..., i, i] = lam + 2.0 * mu
        D[..., 3 + i, 3 + i] = mu
    return D


# ------------------------------------------------------- Eq. 7 + Table 1 (b)
def smoothed_gradients(xyz: np.ndarray, faces: np.ndarray):
    """Smoothed gradients and smoothing-domain volumes of a block of faces
    that are all interior or all exterior (rows of the face table).

    Interior face ABC, tets ABCD (centroid F) and ABCE (centroid G): the
    smoothing domain is ABCF u ABCG, bounded by the six triangles of
    Table 1.  Exterior face ABC of tet ABCD: the domain is ABCF, bounded by
    ABC and the three triangles through F.
    Returns (bbar [nf, n_k, 3] over nodes (A,B,C,D[,E]), V_k [nf]).
    """
    interior = faces[0, 4] >= 0
    A, Bn, C = xyz[faces[:, 0]], xyz[faces[:, 1]], xyz[faces[:, 2]]
    D = xyz[faces[:, 5]]
    F = (A + Bn + C + D) / 4.0
    pts = {"A": A, "B": Bn, "C": C, "F": F}
    V = tet_volume(np.stack([A, Bn, C, F], axis=1))
    if interior:
        Epos = xyz[faces[:, 6]]
        G = (A + Bn + C + Epos) / 4.0
        pts["G"] = G
        V = V + tet_volume(np.stack([A, Bn, C, G], axis=1))
        tris = [(name, vals) for name, vals in TABLE1_INTERIOR.values()]
        n_k = 5
    else:
        tris = list(TABLE1_EXTERIOR.items())
        n_k = 4
    bbar = np.zeros((faces.shape[0], n_k, 3))
    for name, vals in tris:
        P, Q, R = (pts[ch] for ch in name)
        # the remaining vertex of the sub-tet this triangle bounds
        if name == "ABC":
            away = F
        else:
            missing = ({"A", "B", "C"} - set(name)).pop()
            away = pts[missing]
        area = tri_area(P, Q, R)
        n = unit_normal_away(P, Q, R, away)
        for I in range(n_k):
            if vals[I] != 0.0:
                bbar[:, I, :] += n * (vals[I] * area)[:, None]
    bbar /= V[:, None, None]
    return bbar, V


def face_material(faces, tets_vol, lam_t, mu_t):
    """Constant (lambda, mu) of a smoothing domain: the volume-weighted mean
    of the tets' values (each tet contributes a quarter of its volume)."""
    t1 = faces[:, 3]
    t2 = faces[:, 4]
    w1 = tets_vol[t1] / 4.0
    lam = w1 * lam_t[t1]
    mu = w1 * mu_t[t1]
    w = w1.copy()
    inner = t2 >= 0
    w2 = tets_vol[t2[inner]] / 4.0
    lam[inner] += w2 * lam_t[t2[inner]]
    mu[inner] += w2 * mu_t[t2[inner]]
    w[inner] += w2
    return lam / w, mu / w


def _per_tet(v, T):
    v = np.asarray(v, dtype=np.float64)
    return np.full(T, float(v)) if v.ndim == 0 else v


def face_stiffness(xyz, tets, faces, E, nu, tet_vol=None):
    """Eq. 9 per face: K_k = V_k B^T c B_k for a block of same-kind faces.
    Returns (K [nf, 3n_k, 3n_k], node ids [nf, n_k])."""
    T = tets.shape[0]
    if tet_vol is None:
        tet_vol = tet_volume(xyz[tets])
    lam_t, mu_t = lame(_per_tet(E, T), _per_tet(nu, T))
    bbar, V = smoothed_gradients(xyz, faces)
    lam, mu = face_material(faces, tet_vol, lam_t, mu_t)
    B = B_matrix(bbar)
    Dm = D_matrix(lam, mu)
    K = np.einsum("fji,fjk,fkl->fil", B, Dm, B) * V[:, None, None]
    if faces[0, 4] >= 0:
        nodes = faces[:, [0, 1, 2, 5, 6]]
    else:
        nodes = faces[:, [0, 1, 2, 5]]
    return K, nodes


def _coo_block(K, nodes):
    nf, m, _ = K.shape
    dof = (3 * nodes[:, :, None] + np.arange(3)[None, None, :]).reshape(nf, m)
    I = np.broadcast_to(dof[:, :, None], (nf, m, m)).reshape(-1)
    J = np.broadcast_to(dof[:, None, :], (nf, m, m)).reshape(-1)
    return I, J, K.reshape(-1)


def assemble_coo(xyz, tets, E, nu, faces=None):
    """Eq. 12: IK, JK, VK triplets, exterior faces first, then interior."""
    if faces is None:
        faces = extract_faces(tets)
    tab = faces["table"]
    ext = tab[tab[:, 4] < 0]
    inn = tab[tab[:, 4] >= 0]
    vol = tet_volume(xyz[tets])
    parts = []
    for blk in (ext, inn):
        if blk.shape[0]:
            parts.append(_coo_block(*face_stiffness(xyz, tets, blk, E, nu, vol)))
    IK = np.concatenate([p[0] for p in parts])
    JK = np.concatenate([p[1] for p in parts])
    VK = np.concatenate([p[2] for p in parts])
    return IK, JK, VK


def assemble(xyz, tets, E, nu, faces=None) -> sp.csr_matrix:
    """Global FS-FEM stiffness as CSR (duplicates summed, structural zeros
    kept, column indices ascending).  DOF = 3*node + axis."""
    n = 3 * xyz.shape[0]
    IK, JK, VK = assemble_coo(xyz, tets, E, nu, faces)
    K = sp.coo_matrix((VK, (IK, JK)), shape=(n, n)).tocsr()
    K.sort_indices()
    return K


def assemble_rows(xyz, tets, E, nu, nodes, faces=None):
    """Rows 3I+a (a = 0..2) of K for the node ids `nodes`, computed from only
    the faces whose smoothing domain contains a node in `nodes`.  Returns a
    dict node -> (cols [m] ascending, vals [3, m])."""
    if faces is None:
        faces = extract_faces(tets)
    tab = faces["table"]
    want = np.zeros(xyz.shape[0], dtype=bool)
    want[np.asarray(nodes)] = True
    supp = tab[:, [0, 1, 2, 5, 6]]
    touch = (want[supp[:, :4]].any(axis=1)) | ((supp[:, 4] >= 0) & want[np.maximum(supp[:, 4], 0)])
    sub = tab[touch]
    vol = tet_volume(xyz[tets])
    rows = {int(I): {} for I in np.asarray(nodes)}
    for blk in (sub[sub[:, 4] < 0], sub[sub[:, 4] >= 0]):
        if blk.shape[0] == 0:
            continue
        K, nd = face_stiffness(xyz, tets, blk, E, nu, vol)
        m = nd.shape[1]
        for f in range(blk.shape[0]):
            for p in range(m):
                I = int(nd[f, p])
                if I not in rows:
                    continue
                for q in range(m):
                    J = int(nd[f, q])
                    acc = rows[I].setdefault(J, np.zeros((3, 3)))
                    acc += K[f, 3 * p:3 * p + 3, 3 * q:3 * q + 3]
    out = {}
    for I, d in rows.items():
        Js = sorted(d)
        cols = np.array([3 * J + b for J in Js for b in range(3)], dtype=np.int64)
        vals = np.zeros((3, cols.size))
        for jj, J in enumerate(Js):
            vals[:, 3 * jj:3 * jj + 3] = d[J]
        out[I] = (cols, vals)
    return out


def apply_stiffness(xyz, tets, E, nu, u, faces=None, tet_vol=None):
    """y = K u without forming K: the sum over smoothing domains of K_k u_k
    (Eq. 8 / Eq. 9), each K_k the dense 12x12 or 15x15 block of
    face_stiffness acting on the displacements of the domain's support
    nodes.  `faces` may hold any subset of the face table (a chunk of rows);
    the result is then that subset's share of K u."""
    if faces is None:
        faces = extract_faces(tets)
    tab = faces["table"]
    if tet_vol is None:
        tet_vol = tet_volume(xyz[tets])
    u = np.asarray(u, dtype=np.float64)
    y = np.zeros(u.size)
    for blk in (tab[tab[:, 4] < 0], tab[tab[:, 4] >= 0]):
        if not blk.shape[0]:
            continue
        K, nodes = face_stiffness(xyz, tets, blk, E, nu, tet_vol)
        m = nodes.shape[1]
        dof = (3 * nodes[:, :, None] + np.arange(3)).reshape(-1, 3 * m)
        yk = np.einsum("fij,fj->fi", K, u[dof])
        y += np.bincount(dof.reshape(-1), yk.reshape(-1), minlength=u.size)
    return y


# --------------------------------------------------------------- plain FEM-T4
def face_strain_stress(xyz, tets, E, nu, u, faces=None):
    """Post-processing (Sec. 3.4): the smoothed strain of every smoothing
    domain, eps_k = B_k d_k (the B of Eq. 4 built from the smoothed
    gradients of Eq. 7 and the displacements d_k of the domain's support
    nodes), and its stress sigma_k = c_k eps_k with the domain's c of Eq. 9
    (volume-weighted Lame constants, as in the stiffness).  Voigt order xx,
    yy, zz, yz, xz, xy with engineering shear strains.  Rows in face-table
    order.  Returns (eps [N_f, 6], sigma [N_f, 6])."""
    if faces is None:
        faces = extract_faces(tets)
    tab = faces["table"]
    T = tets.shape[0]
    vol = tet_volume(xyz[tets])
    lam_t, mu_t = lame(_per_tet(E, T), _per_tet(nu, T))
    U = np.asarray(u, dtype=np.float64).reshape(-1, 3)
    eps = np.zeros((tab.shape[0], 6))
    sig = np.zeros((tab.shape[0], 6))
    ext = tab[:, 4] < 0
    for mask in (ext, ~ext):
        blk = tab[mask]
        if not blk.shape[0]:
            continue
        bbar, _ = smoothed_gradients(xyz, blk)
        lam, mu = face_material(blk, vol, lam_t, mu_t)
        nodes = blk[:, [0, 1, 2, 5]] if blk[0, 4] < 0 else blk[:, [0, 1, 2, 5, 6]]
        d = U[nodes].reshape(blk.shape[0], -1)
        e = np.einsum("fij,fj->fi", B_matrix(bbar), d)
        eps[mask] = e
        sig[mask] = np.einsum("fij,fj->fi", D_matrix(lam, mu), e)
    return eps, sig


def fem_t4_assemble(xyz, tets, E, nu) -> sp.csr_matrix:
    """Conventional FEM with linear tets: K = sum_e V_e B_e^T c B_e, the
    comparison method of Sec. 4.1 (used only by the ordering test)."""
    T = tets.shape[0]
    P = xyz[tets]
    M = np.concatenate([np.ones((T, 4, 1)), P], axis=2)  # rows [1 x y z]
    Minv = np.linalg.inv(M)                              # N_a = Minv[:, a] . [1 x y z]
    grads = np.transpose(Minv[:, 1:4, :], (0, 2, 1))     # [T, 4(node), 3]
    V = tet_volume(P)
    lam, mu = lame(_per_tet(E, T), _per_tet(nu, T))
    B = B_matrix(grads)
    K = np.einsum("fji,fjk,fkl->fil", B, D_matrix(lam, mu), B) * V[:, None, None]
    I, J, VK = _coo_block(K, tets.astype(np.int64))
    n = 3 * xyz.shape[0]
    Kg = sp.coo_matrix((VK, (I, J)), shape=(n, n)).tocsr()
    Kg.sort_indices()
    return Kg


# --------------------------------------------------------------- loads, BCs
def traction_load(xyz, tris, t, n_nodes=None) -> np.ndarray:
    """Consistent nodal load of a uniform traction t [3] on triangles
    tris [n,3]: each vertex receives t * area / 3 (area by Eq. 11)."""
    n_nodes = xyz.shape[0] if n_nodes is None else n_nodes
    f = np.zeros(3 * n_nodes)
    A = tri_area(xyz[tris[:, 0]], xyz[tris[:, 1]], xyz[tris[:, 2]])
    for v in range(3):
        for a in range(3):
            np.add.at(f, 3 * tris[:, v] + a, t[a] * A / 3.0)
    return f


def apply_dirichlet(K: sp.csr_matrix, f: np.ndarray, dofs, values=None):
    """Essential BCs by elimination (STEP 5 reading): for every fixed DOF i
    the column K[:, i] * value is moved to the right-hand side, row i and
    column i are zeroed except K_ii, and f_i = K_ii * value.  The sparsity
    pattern is unchanged (zeros stay stored)."""
    dofs = np.asarray(dofs, dtype=np.int64)
    vals = np.zeros(dofs.size) if values is None else np.asarray(values, dtype=np.float64)
    n = K.shape[0]
    u_fix = np.zeros(n)
    u_fix[dofs] = vals
    f = f - K @ u_fix
    fixed = np.zeros(n, dtype=bool)
    fixed[dofs] = True
    Kb = K.copy().tocoo()
    diag = K.diagonal()
    keep = ~(fixed[Kb.row] | fixed[Kb.col]) | (Kb.row == Kb.col)
    data = np.where(keep, Kb.data, 0.0)
    Kb = sp.csr_matrix((data, (Kb.row, Kb.col)), shape=K.shape)
    Kb.sort_indices()
    f[fixed] = diag[fixed] * u_fix[fixed]
    return Kb, f


def apply_penalty(K: sp.csr_matrix, f: np.ndarray, dofs, alpha: float, values=None):
    """Penalty variant (the paper's STEP 5 choice): K_ii += alpha, f_i =
    alpha * value for fixed DOFs.  alpha must be given explicitly."""
    dofs = np.asarray(dofs, dtype=np.int64)
    vals = np.zeros(dofs.size) if values is None else np.asarray(values, dtype=np.float64)
    Kp = K.tolil(copy=True)
    for d, v in zip(dofs, vals):
        Kp[d, d] = Kp[d, d] + alpha
    f = f.copy()
    f[dofs] = alpha * vals
    Kp = Kp.tocsr()
    Kp.sort_indices()
    return Kp, f


# ------------------------------------------------------------------- solves
def rel_residual(K, u, f) -> float:
    return float(np.linalg.norm(f - K @ u) / np.linalg.norm(f))


def solve_dense(K, f) -> np.ndarray:
    return np.linalg.solve(K.toarray(), f)


def solve_banded(K: sp.csr_matrix, f: np.ndarray) -> np.ndarray:
    """Exact (up to rounding) SPD solve by banded Cholesky (LAPACK pbsv):
    the x-slowest node numbering keeps the band narrow.  The band is stored
    column-major and factorised in place, so the 1.92M-tet cantilever
    (bandwidth 5,171 DOFs, 42 GB of band) needs one copy of it."""
    C = K.tocoo()
    bw = int(np.max(np.abs(C.row.astype(np.int64) - C.col)))
    n = K.shape[0]
    ab = np.zeros((bw + 1, n), order="F")
    up = C.col >= C.row
    r, c, v = C.row[up].astype(np.int64), C.col[up].astype(np.int64), C.data[up]
    del C, up
    ab[bw + r - c, c] = v
    del r, c, v
    return solve_banded_ab(ab, f)


def solve_banded_ab(ab, f):
    from scipy.linalg import solveh_banded
    return solveh_banded(ab, f, lower=False, check_finite=False, overwrite_ab=True)


def block_row_sums(K: sp.csr_matrix) -> np.ndarray:
    """R [N, 3, 3] with R_I[a, c] = sum_J K[3I+a, 3J+c]: the 3x3 blocks of a
    node row summed, i.e. the row's response to a unit translation along c.
    Each sum is exactly rounded (math.fsum), so R is the row sum of the
    stored values to one FP64 rounding of R itself."""
    import math
    C = K.tocoo()
    n = K.shape[0]
    key = 3 * C.row.astype(np.int64) + C.col.astype(np.int64) % 3
    order = np.argsort(key, kind="stable")
    key, data = key[order], C.data[order].tolist()
    bounds = np.flatnonzero(np.concatenate([[True], key[1:] != key[:-1], [True]])).tolist()
    R = np.zeros(3 * n)
    for s, e in zip(bounds[:-1], bounds[1:]):
        R[key[s]] = math.fsum(data[s:e])
    return R.reshape(n // 3, 3, 3)


def apply_translation_form(K: sp.csr_matrix, u: np.ndarray, R=None) -> np.ndarray:
    """K u written as (K u)_{3I+a} = sum_(J,c) K[3I+a, 3J+c] (u_{3J+c} - u_{3I+c})
    + sum_c R_I[a, c] u_{3I+c} (R = block_row_sums(K)): the same number in
    exact arithmetic.  K maps rigid translations to (nearly) zero, so for a
    smooth u the plain sum cancels terms of size |K||u| down to a small
    result and keeps their rounding, eps |K| |u|; here the large terms only
    meet neighbour differences and the rounding is eps |K| |u_J - u_I|."""
    if R is None:
        R = block_row_sums(K)
    C = K.tocoo()
    n = K.shape[0]
    rows = C.row.astype(np.int64)
    own = 3 * (rows // 3) + C.col.astype(np.int64) % 3
    y = np.bincount(rows, C.data * (u[C.col] - u[own]), minlength=n)
    return y + np.einsum("iac,ic->ia", R, u.reshape(-1, 3)).reshape(-1)


def pcg_jacobi(K, f, rtol=1e-8, max_iter=100000, x0=None, check_every=50, residual=None):
    """Jacobi-preconditioned CG, x0 = 0, stopped when the TRUE relative
    residual ||f - K x|| / ||f|| <= rtol; the true residual replaces the
    recursive one every `check_every` iterations and whenever the recursive
    one claims convergence.  `residual(x)` (default f - K @ x) computes the
    true residual, e.g. with apply_translation_form.  Returns (x,
    iterations, true relres by that residual)."""
    n = K.shape[0]
    if residual is None:
        def residual(v):
            return f - K @ v
    x = np.zeros(n) if x0 is None else x0.copy()
    Dinv = 1.0 / K.diagonal()
    nf = np.linalg.norm(f)
    r = residual(x)
    z = Dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    while it < max_iter:
        q = K @ p
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        if np.linalg.norm(r) <= rtol * nf or it % check_every == 0:
            r = residual(x)
            if np.linalg.norm(r) <= rtol * nf:
                break
        z = Dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    return x, it, float(np.linalg.norm(residual(x)) / nf)


# ------------------------------------------------------------ convenience
def rigid_modes(xyz) -> np.ndarray:
    """The six rigid-body displacement fields [6, 3N]."""
    N = xyz.shape[0]
    R = np.zeros((6, N, 3))
    for a in range(3):
        R[a, :, a] = 1.0
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    R[3, :, 1], R[3, :, 2] = -z, y      # rotation about x
    R[4, :, 0], R[4, :, 2] = z, -x      # rotation about y
    R[5, :, 0], R[5, :, 1] = -y, x      # rotation about z
    return R.reshape(6, 3 * N)


def problem_system(problem, penalty=None):
    """K (BC applied), f, and the unconstrained K for a meshgen Problem."""
    m = problem.mesh
    K = assemble(m.xyz, m.tets, problem.E, problem.nu)
    f = traction_load(m.xyz, m.end_tris, np.asarray(problem.traction, dtype=np.float64))
    if penalty is None:
        Kb, fb = apply_dirichlet(K, f, problem.fixed_dofs())
    else:
        Kb, fb = apply_penalty(K, f, problem.fixed_dofs(), penalty)
    return Kb, fb, K
