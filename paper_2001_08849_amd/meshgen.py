"""Seeded synthetic inputs: structured Kuhn-split T4 cantilever meshes.

This module only *generates inputs*.  It holds none of the FS-FEM arithmetic
(no volumes, normals, gradients, stiffness or loads): it emits node
coordinates, tetrahedra as node-index quadruples, the clamped-node list, the
loaded boundary triangles and the material fields.  Both the FP64 oracle
(tests only) and the HIP path consume exactly these arrays.

The paper meshes its cantilever with TetGen (Sec. 3.2, Table 3); those meshes
are not available, so the stand-in is a box of n_x x n_y x n_z hexahedral cells,
each split into six tetrahedra along its main diagonal (Kuhn/Freudenthal
split, conforming across cells), with seeded jitter of the interior nodes.

Numbering
---------
* node id  = (i*(n_y+1) + j)*(n_z+1) + k      (x slowest: small matrix band)
* cell id  = (i*n_y + j)*n_z + k
* tet id   = 6*cell + p, p indexing the axis permutations in lexicographic
  order (xyz, xzy, yxz, yzx, zxy, zyx); the tet is
  (v000, v000+e_p1, v000+e_p1+e_p2, v111).  Vertex order is left as generated,
  so half of the tetrahedra are negatively oriented; the method must not
  depend on vertex order.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import Optional

import numpy as np

PERMS = list(itertools.permutations(range(3)))  # lexicographic order


@dataclasses.dataclass
class Mesh:
    xyz: np.ndarray            # float64 [N,3]
    tets: np.ndarray           # int32   [T,4]
    grid: tuple                # (n_x, n_y, n_z)
    lengths: tuple             # (L_x, L_y, L_z)
    clamp_nodes: np.ndarray    # int32 nodes on x = 0
    end_tris: np.ndarray       # int32 [n,3] boundary triangles on x = L_x
    top_tris: np.ndarray       # int32 [n,3] boundary triangles on z = L_z

    @property
    def n_nodes(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    def clamp_dofs(self) -> np.ndarray:
        """All three DOFs (3*node + axis) of every node on x = 0."""
        n = self.clamp_nodes.astype(np.int64)
        return (3 * n[:, None] + np.arange(3)[None, :]).reshape(-1).astype(np.int32)


def node_id(i, j, k, ny, nz):
    return (i * (ny + 1) + j) * (nz + 1) + k


def box_mesh(nx: int, ny: int, nz: int, Lx: float, Ly: float, Lz: float,
             jitter: float = 0.0, seed: Optional[int] = None) -> Mesh:
    """Kuhn-split box mesh; `jitter` is the +/- fraction of the cell spacing
    applied (per axis) to nodes strictly inside the box."""
    h = np.array([Lx / nx, Ly / ny, Lz / nz])
    ii, jj, kk = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1),
                             indexing="ij")
    ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)  # node-id order
    xyz = ijk.astype(np.float64) * h[None, :]
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        d = rng.uniform(-jitter, jitter, size=xyz.shape) * h[None, :]
        inside = ((ijk > 0) & (ijk < np.array([nx, ny, nz])[None, :])).all(axis=1)
        xyz[inside] += d[inside]

    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    ci, cj, ck = ci.ravel(), cj.ravel(), ck.ravel()
    tets = np.empty((ci.size, 6, 4), dtype=np.int64)
    for p, perm in enumerate(PERMS):
        cur = np.stack([ci, cj, ck], axis=1).copy()
        tets[:, p, 0] = node_id(cur[:, 0], cur[:, 1], cur[:, 2], ny, nz)
        for s in range(3):
            cur[:, perm[s]] += 1
            tets[:, p, s + 1] = node_id(cur[:, 0], cur[:, 1], cur[:, 2], ny, nz)
    tets = tets.reshape(-1, 4).astype(np.int32)

    clamp = np.flatnonzero(ijk[:, 0] == 0).astype(np.int32)

    # the x = L_x boundary squares are cut along the (j,k)->(j+1,k+1) diagonal,
    # which is how the six-tet split of the last cell layer cuts them
    tj, tk = np.meshgrid(np.arange(ny), np.arange(nz), indexing="ij")
    tj, tk = tj.ravel(), tk.ravel()
    v00 = node_id(nx, tj, tk, ny, nz)
    v10 = node_id(nx, tj + 1, tk, ny, nz)
    v01 = node_id(nx, tj, tk + 1, ny, nz)
    v11 = node_id(nx, tj + 1, tk + 1, ny, nz)
    end_tris = np.concatenate([np.stack([v00, v10, v11], 1), np.stack([v00, v01, v11], 1)],
                              axis=0).astype(np.int32)
    # likewise the z = L_z squares, cut along (i,j)->(i+1,j+1)
    ti, tj2 = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    ti, tj2 = ti.ravel(), tj2.ravel()
    w00 = node_id(ti, tj2, nz, ny, nz)
    w10 = node_id(ti + 1, tj2, nz, ny, nz)
    w01 = node_id(ti, tj2 + 1, nz, ny, nz)
    w11 = node_id(ti + 1, tj2 + 1, nz, ny, nz)
    top_tris = np.concatenate([np.stack([w00, w10, w11], 1), np.stack([w00, w01, w11], 1)],
                              axis=0).astype(np.int32)
    return Mesh(xyz=xyz, tets=tets, grid=(nx, ny, nz), lengths=(Lx, Ly, Lz),
                clamp_nodes=clamp, end_tris=end_tris, top_tris=top_tris)


# ---------------------------------------------------------------- material fields

def blob_field(points: np.ndarray, lengths, rng, n_blobs: int = 32, width: float = 1.0):
    """Sum of `n_blobs` isotropic Gaussian bumps with N(0,1) weights and
    centres uniform in the box, evaluated at `points` [M,3]."""
    L = np.asarray(lengths, dtype=np.float64)
    centres = rng.uniform(0.0, 1.0, size=(n_blobs, 3)) * L[None, :]
    weights = rng.standard_normal(n_blobs)
    g = np.zeros(points.shape[0])
    for c, w in zip(centres, weights):
        d2 = ((points - c[None, :]) ** 2).sum(axis=1)
        g += w * np.exp(-d2 / (2.0 * width * width))
    return g


def rank_uniform(g: np.ndarray) -> np.ndarray:
    """(rank + 0.5)/M: an exactly uniform marginal that keeps g's spatial order."""
    order = np.argsort(g, kind="stable")
    r = np.empty(g.size)
    r[order] = np.arange(g.size)
    return (r + 0.5) / g.size


def blob_material(mesh: Mesh, seed: int, e_lo: float = 1e9, e_hi: float = 1e11,
                  nu_lo: float = 0.25, nu_hi: float = 0.45):
    """Per-tet E log-uniform in [e_lo, e_hi] and nu uniform in [nu_lo, nu_hi],
    both spatially correlated through independent Gaussian-blob fields sampled
    at the tet's vertex mean."""
    rng = np.random.default_rng(seed)
    pts = mesh.xyz[mesh.tets].mean(axis=1)
    u_e = rank_uniform(blob_field(pts, mesh.lengths, rng))
    u_n = rank_uniform(blob_field(pts, mesh.lengths, rng))
    E = 10.0 ** (np.log10(e_lo) + (np.log10(e_hi) - np.log10(e_lo)) * u_e)
    nu = nu_lo + (nu_hi - nu_lo) * u_n
    return E, nu


# ---------------------------------------------------------------- named workloads

@dataclasses.dataclass
class Problem:
    name: str
    mesh: Mesh
    E: object                      # float or float64 [T]
    nu: object                     # float or float64 [T]
    traction: np.ndarray           # float64 [3] (or [n_cases,3])
    rtol: float

    def fixed_dofs(self) -> np.ndarray:
        return self.mesh.clamp_dofs()


def cantilever_c0() -> Problem:
    """10x1x1 m, 10x2x2 cells (240 tets, 99 nodes), no jitter, E=210e9,
    nu=0.3, clamp x=0, traction (0,0,-1e6) Pa on x=10, rtol 1e-10."""
    m = box_mesh(10, 2, 2, 10.0, 1.0, 1.0)
    return Problem("c0_10x2x2", m, 210e9, 0.3, np.array([0.0, 0.0, -1e6]), 1e-10)


def cantilever_c1() -> Problem:
    """20x2x2 m, 100x10x10 cells (60,000 tets), +/-15% jitter, seed 1."""
    m = box_mesh(100, 10, 10, 20.0, 2.0, 2.0, jitter=0.15, seed=1)
    return Problem("c1_100x10x10", m, 210e9, 0.3, np.array([0.0, 0.0, -1e6]), 1e-8)


def cantilever_c2() -> Problem:
    """40x4x4 m, 200x40x40 cells (1.92M tets), +/-10% jitter, seed 2."""
    m = box_mesh(200, 40, 40, 40.0, 4.0, 4.0, jitter=0.10, seed=2)
    return Problem("c2_200x40x40", m, 210e9, 0.3, np.array([0.0, 0.0, -1e6]), 1e-8)


def cantilever_scaled(nx: int, ny: int, nz: int, jitter: float = 0.15, seed: int = 1,
                      L: tuple = None) -> Problem:
    """Cantilever of the c1 family (aspect 10:1:1 unless L is given) at any grid."""
    if L is None:
        L = (20.0, 2.0, 2.0)
    m = box_mesh(nx, ny, nz, *L, jitter=jitter, seed=seed)
    return Problem(f"cant_{nx}x{ny}x{nz}", m, 210e9, 0.3, np.array([0.0, 0.0, -1e6]), 1e-8)


def learned_c4(m_index: int, held_out: bool = False) -> Problem:
    """20x2x2 m, 140x14x14 cells (164,640 tets), +/-15% jitter, per-tet
    E log-uniform over [1e9, 1e11] and nu in [0.25, 0.45] in correlated blobs.
    Training meshes use seed 4000+m, held-out meshes 4900+m."""
    seed = (4900 if held_out else 4000) + m_index
    mesh = box_mesh(140, 14, 14, 20.0, 2.0, 2.0, jitter=0.15, seed=seed)
    E, nu = blob_material(mesh, seed=seed + 100000)
    return Problem(f"c4_{'held' if held_out else 'train'}{m_index}", mesh, E, nu,
                   np.array([0.0, 0.0, -1e6]), 1e-8)


def learned_small(m_index: int, grid=(40, 6, 6), held_out: bool = False) -> Problem:
    """A smaller mesh of the c4 family (same material recipe) for quick tests."""
    seed = (4900 if held_out else 4000) + m_index
    nx, ny, nz = grid
    mesh = box_mesh(nx, ny, nz, 20.0 * nx / 140.0 * 3.5, 2.0, 2.0, jitter=0.15, seed=seed)
    E, nu = blob_material(mesh, seed=seed + 100000)
    return Problem(f"c4s_{m_index}", mesh, E, nu, np.array([0.0, 0.0, -1e6]), 1e-8)


@dataclasses.dataclass
class BatchItem:
    mesh: Mesh
    E: float
    nu: float
    tractions: np.ndarray          # float64 [4,3]: +y, -y, +z, -z load cases


def batch_c3(n_meshes: int = 64, seed: int = 3, nx_range=(20, 120), nyz_range=(4, 20)):
    """64 box meshes of uneven size; mesh b draws from default_rng(seed*1000+b):
    n_x ~ U{20..120}, n_y = n_z ~ U{4..20}, spacing 0.1 m, E log-uniform in
    [1e9, 3e11], nu ~ U(0.2, 0.45), +/-15% jitter, four end-traction load
    cases (+y, -y, +z, -z) of magnitude 10^U(5,7) Pa."""
    items = []
    for b in range(n_meshes):
        rng = np.random.default_rng(seed * 1000 + b)
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        nyz = int(rng.integers(nyz_range[0], nyz_range[1] + 1))
        E = float(10.0 ** rng.uniform(9.0, np.log10(3e11)))
        nu = float(rng.uniform(0.2, 0.45))
        mag = 10.0 ** rng.uniform(5.0, 7.0, size=4)
        jseed = int(rng.integers(0, 2**31 - 1))
        mesh = box_mesh(nx, nyz, nyz, 0.1 * nx, 0.1 * nyz, 0.1 * nyz, jitter=0.15, seed=jseed)
        dirs = np.array([[0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], dtype=np.float64)
        items.append(BatchItem(mesh, E, nu, dirs * mag[:, None]))
    return items


def paper_beam(nx: int = 20, ny: int = 4, nz: int = 4) -> Problem:
    """The accuracy example of Sec. 4.1: a 1 x 0.2 x 0.2 m cantilever
    clamped at x = 0 under a uniform 12,500 N/m^2 pressure on its upper face
    in -Z, E = 2e8, nu = 0.3.  The paper's TetGen mesh (458 nodes, 1,576
    tets) is not available; a structured 20x4x4 split (1,920 tets) stands in.
    The load sits on the top face: use ``mesh.top_tris`` with ``traction``."""
    m = box_mesh(nx, ny, nz, 1.0, 0.2, 0.2)
    return Problem("paper_beam", m, 2e8, 0.3, np.array([0.0, 0.0, -12500.0]), 1e-10)


CONFIGS = {
    "c0": cantilever_c0,
    "c1": cantilever_c1,
    "c2": cantilever_c2,
}
