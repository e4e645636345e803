"""FP64 reference of the learned preconditioner network (numpy, CPU).

TEST INFRASTRUCTURE ONLY (used by tests/ to check the GPU kernels' forward
values and gradients).  The paper has no learned component; this defines the
network the library implements, written plainly, with its gradient derived
by hand and pinned by finite differences in the tests.

Graph: nodes = mesh nodes, edges = the 3x3-block pattern of K (self edges
included), in block-CSR order.  With d = diag(K) and A = D^-1/2 K D^-1/2:
  node features x_I (8): A_II[0,1], A_II[0,2], A_II[1,2], log(d_3I+a / mean d)
                         (a = 0..2), fixed(I), 1
  edge features y_IJ (12): A_IJ (row-major 3x3), (p_J - p_I) / hbar
where hbar is the mean length of the off-diagonal edges.
Network (width H):
  h = relu(Wn x + bn),  e = relu(We y + be)
  repeat L times:  z = Wl [h_I; h_J; e] + bl,  m = relu(z),  e <- e + m,
                   a_I = mean_J m_IJ,  t = Ul [h_I; a_I] + cl,  h <- h + relu(t)
  R_IJ = Wo e_IJ (3x3, row-major);  S_IJ = (R_IJ + R_JI^T) / 2
  S'_ij = S_ij, or 0 if DOF i or j is fixed
  M = D^-1/2 (I + theta S') D^-1/2, theta = min(1, 0.9 / (1.05 |lambda_min(S')|))
      when lambda_min(S') < 0, else 1; so I + theta S' >= 0.1 I (positive
      definite; the 1.05 leaves room for an estimate of lambda_min from
      below in magnitude).  Training uses the unscaled S' (theta = 1).
Loss over pairs (r_p, e_p) with K e_p = r_p:
  L = mean_p (M r_p - e_p)^T K (M r_p - e_p) / (e_p^T K e_p)
"""
from __future__ import annotations

import dataclasses

import numpy as np

H = 64
N_LAYERS = 4
F_NODE = 8
F_EDGE = 12


@dataclasses.dataclass
class Graph:
    N: int
    bptr: np.ndarray      # [N+1]
    bcol: np.ndarray      # [nb]
    row: np.ndarray       # [nb] row node of each edge
    tr: np.ndarray        # [nb] index of the transposed edge (J,I)
    deg: np.ndarray       # [N]
    Kb: np.ndarray        # [nb, 3, 3] blocks of K (BC applied)
    d: np.ndarray         # [3N] diag(K)
    fixed: np.ndarray     # [3N] bool
    x: np.ndarray         # [N, F_NODE]
    y: np.ndarray         # [nb, F_EDGE]


def init_params(seed: int = 0, width: int = H, layers: int = N_LAYERS):
    """Glorot-uniform weights, zero biases; the decoder starts at zero so the
    untrained preconditioner is exactly Jacobi."""
    rng = np.random.default_rng(seed)

    def glorot(fan_in, fan_out):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-lim, lim, size=(fan_out, fan_in))

    P = {"Wn": glorot(F_NODE, width), "bn": np.zeros(width),
         "We": glorot(F_EDGE, width), "be": np.zeros(width)}
    for l in range(layers):
        P[f"W{l}"] = glorot(3 * width, width)
        P[f"b{l}"] = np.zeros(width)
        P[f"U{l}"] = glorot(2 * width, width)
        P[f"c{l}"] = np.zeros(width)
    P["Wo"] = np.zeros((9, width))
    return P


def build_graph(K_csr, xyz, fixed_dofs) -> Graph:
    """Block-CSR graph and input features from the BC-applied CSR matrix of
    an FS-FEM problem (scalar CSR with 3x3 node blocks, rows 3I..3I+2)."""
    n = K_csr.shape[0]
    N = n // 3
    K = K_csr.tocsr()
    K.sort_indices()
    bcols, bptr = [], [0]
    for I in range(N):
        cols = K.indices[K.indptr[3 * I]:K.indptr[3 * I + 1]]
        nodes = cols[0::3] // 3
        bcols.append(nodes)
        bptr.append(bptr[-1] + len(nodes))
    bcol = np.concatenate(bcols).astype(np.int64)
    bptr = np.array(bptr, dtype=np.int64)
    nb = bcol.size
    row = np.repeat(np.arange(N), np.diff(bptr))
    Kb = np.zeros((nb, 3, 3))
    for a in range(3):
        for c in range(3):
            Kb[:, a, c] = np.asarray(K[3 * row + a, 3 * bcol + c]).ravel()
    pos = {(int(i), int(j)): k for k, (i, j) in enumerate(zip(row, bcol))}
    tr = np.array([pos[(int(j), int(i))] for i, j in zip(row, bcol)], dtype=np.int64)
    d = K.diagonal().copy()
    fixed = np.zeros(n, dtype=bool)
    fixed[np.asarray(fixed_dofs, dtype=np.int64)] = True
    s = 1.0 / np.sqrt(d)
    A = Kb * s.reshape(N, 3)[row][:, :, None] * s.reshape(N, 3)[bcol][:, None, :]
    diag_edges = np.flatnonzero(row == bcol)
    Aii = A[diag_edges]  # one per node, rows in order
    dbar = d[~fixed].mean() if (~fixed).any() else d.mean()
    x = np.zeros((N, F_NODE))
    x[:, 0], x[:, 1], x[:, 2] = Aii[:, 0, 1], Aii[:, 0, 2], Aii[:, 1, 2]
    x[:, 3:6] = np.log(d.reshape(N, 3) / dbar)
    x[:, 6] = fixed.reshape(N, 3).any(axis=1)
    x[:, 7] = 1.0
    rel = xyz[bcol] - xyz[row]
    off = row != bcol
    hbar = np.linalg.norm(rel[off], axis=1).mean()
    y = np.concatenate([A.reshape(nb, 9), rel / hbar], axis=1)
    return Graph(N, bptr, bcol, row, tr, np.diff(bptr), Kb, d, fixed, x, y)


def relu(v):
    return np.maximum(v, 0.0)


def sum_by_row(g: Graph, v):
    """out[I] = sum of v over the edges (I, J) of node row I.  Edges are
    stored row by row (block CSR) and every row holds at least its self
    edge, so the rows are the consecutive segments starting at bptr."""
    return np.add.reduceat(v, g.bptr[:-1], axis=0)


def sum_by_col(g: Graph, v):
    """out[I] = sum of v over the edges (J, I) whose column is I: the
    transposes of row I's edges, tr[k] for k in row I."""
    return np.add.reduceat(v[g.tr], g.bptr[:-1], axis=0)


def forward(P, g: Graph, layers: int = N_LAYERS):
    """Returns S' blocks [nb,3,3] and a cache for backward."""
    c = {}
    c["h0"] = relu(g.x @ P["Wn"].T + P["bn"])
    c["e0"] = relu(g.y @ P["We"].T + P["be"])
    h, e = c["h0"], c["e0"]
    for l in range(layers):
        X = np.concatenate([h[g.row], h[g.bcol], e], axis=1)
        z = X @ P[f"W{l}"].T + P[f"b{l}"]
        m = relu(z)
        e = e + m
        a = sum_by_row(g, m) / g.deg[:, None]
        Y = np.concatenate([h, a], axis=1)
        t = Y @ P[f"U{l}"].T + P[f"c{l}"]
        h = h + relu(t)
        c[f"X{l}"], c[f"z{l}"], c[f"Y{l}"], c[f"t{l}"] = X, z, Y, t
    c["eL"] = e
    R = (e @ P["Wo"].T).reshape(-1, 3, 3)
    S = 0.5 * (R + np.transpose(R[g.tr], (0, 2, 1)))
    N = g.N
    fr = g.fixed.reshape(N, 3)
    mask = ~(fr[g.row][:, :, None] | fr[g.bcol][:, None, :])
    Sp = S * mask
    c.update(R=R, mask=mask)
    return Sp, c


def correction_matrix(g: Graph, Sp):
    """S' blocks as a scipy CSR matrix [3N, 3N]."""
    import scipy.sparse as sp
    n = 3 * g.N
    rows = (3 * g.row[:, None, None] + np.arange(3)[None, :, None]).repeat(3, 2).ravel()
    cols = (3 * g.bcol[:, None, None] + np.arange(3)[None, None, :]).repeat(3, 1).ravel()
    return sp.csr_matrix((Sp.ravel(), (rows, cols)), shape=(n, n))


def spd_theta(g: Graph, Sp):
    """(theta, lambda_min(S')) with lambda_min computed exactly (dense for
    small graphs, shift-free Lanczos to tight tolerance otherwise)."""
    S = correction_matrix(g, Sp)
    if S.shape[0] <= 4000:
        lmin = float(np.linalg.eigvalsh(S.toarray())[0])
    else:
        import scipy.sparse.linalg as sla
        lmin = float(sla.eigsh(S, k=1, which="SA", return_eigenvectors=False, tol=1e-10)[0])
    theta = 1.0 if lmin >= 0.0 else min(1.0, 0.9 / (1.05 * -lmin))
    return theta, lmin


def apply_M(g: Graph, Sp, r):
    """M r = D^-1/2 (I + S') D^-1/2 r for r [3N] or [3N, P] (pass theta S'
    for the scaled inference preconditioner)."""
    s = 1.0 / np.sqrt(g.d)
    rh = (r.T * s).T
    y = rh.copy()
    N = g.N
    rb = rh.reshape((N, 3) + rh.shape[1:])
    contrib = np.einsum("kab,kb...->ka...", Sp, rb[g.bcol])
    yb = y.reshape((N, 3) + rh.shape[1:]) + sum_by_row(g, contrib)
    return (yb.reshape(rh.shape).T * s).T


def loss(P, g: Graph, K, Rm, Em, layers: int = N_LAYERS):
    """Mean K-norm relative error of M r over pairs (columns of Rm, Em)."""
    Sp, _ = forward(P, g, layers)
    W = apply_M(g, Sp, Rm) - Em
    num = np.einsum("ip,ip->p", W, K @ W)
    den = np.einsum("ip,ip->p", Em, K @ Em)
    return float(np.mean(num / den))


def backward(P, g: Graph, K, Rm, Em, layers: int = N_LAYERS):
    """(loss, dict of gradients with the keys of P)."""
    Sp, c = forward(P, g, layers)
    Pn = Rm.shape[1]
    s = 1.0 / np.sqrt(g.d)
    W = apply_M(g, Sp, Rm) - Em
    KW = K @ W
    KE = K @ Em
    num = np.einsum("ip,ip->p", W, KW)
    den = np.einsum("ip,ip->p", Em, KE)
    L = float(np.mean(num / den))
    G = 2.0 * KW / den / Pn                    # dL / d(M r)
    gh = (G.T * s).T                           # dL / dy, y = rh + S' rh
    rh = (Rm.T * s).T
    N = g.N
    # dL/dS'_{(I,a),(J,b)} = sum_p gh[3I+a,p] rh[3J+b,p]
    ghb = gh.reshape(N, 3, Pn)
    rhb = rh.reshape(N, 3, Pn)
    dSp = np.einsum("kap,kbp->kab", ghb[g.row], rhb[g.bcol])
    dS = dSp * c["mask"]
    dR = 0.5 * (dS + np.transpose(dS[g.tr], (0, 2, 1)))
    grads = {}
    eL = c["eL"]
    dR9 = dR.reshape(-1, 9)
    grads["Wo"] = dR9.T @ eL
    de = dR9 @ P["Wo"]
    dh = np.zeros((N, P["Wn"].shape[0]))
    for l in reversed(range(layers)):
        X, z, Y, t = c[f"X{l}"], c[f"z{l}"], c[f"Y{l}"], c[f"t{l}"]
        dt = dh * (t > 0)
        grads[f"U{l}"] = dt.T @ Y
        grads[f"c{l}"] = dt.sum(axis=0)
        dY = dt @ P[f"U{l}"]
        Hw = dh.shape[1]
        dh = dh + dY[:, :Hw]
        da = dY[:, Hw:]
        dm = de + (da / g.deg[:, None])[g.row]
        dz = dm * (z > 0)
        grads[f"W{l}"] = dz.T @ X
        grads[f"b{l}"] = dz.sum(axis=0)
        dX = dz @ P[f"W{l}"]
        dh = dh + sum_by_row(g, dX[:, :Hw]) + sum_by_col(g, dX[:, Hw:2 * Hw])
        de = de + dX[:, 2 * Hw:]
    dz0 = de * (c["e0"] > 0)
    grads["We"] = dz0.T @ g.y
    grads["be"] = dz0.sum(axis=0)
    dzn = dh * (c["h0"] > 0)
    grads["Wn"] = dzn.T @ g.x
    grads["bn"] = dzn.sum(axis=0)
    return L, grads
