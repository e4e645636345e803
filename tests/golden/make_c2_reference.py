"""Writes the FP64 oracle displacements of the 1.92M-tet cantilever.

    python tests/golden/make_c2_reference.py      # ~1 h on one core, ~6 GB of memory

Calls only ``oracle/`` (and the seeded input generator).  The workload is
the paper-scale cantilever of the efficiency study (Sec. 4.2, Table 3 mesh 4
scale): 40 x 4 x 4 m, 200 x 40 x 40 cells x 6 Kuhn tets = 1,920,000 tets,
337,881 nodes, +/-10% interior jitter (seed 2), E = 210e9 Pa, nu = 0.3,
every DOF at x = 0 clamped (eliminated), uniform traction (0, 0, -1e6) Pa
on the x = 40 face.

Steps:
  1. K = sum over faces of K_k = V_k B_k^T c B_k (Eq. 9, Eq. 7 + Table 1),
     assembled in chunks of the face table and summed;
  2. f = t A / 3 per loaded-triangle vertex; BCs by elimination;
  3. the oracle's Jacobi PCG (stopped on the FP64 true residual) to 1e-8;
  4. iterative refinement: r = f - K u in the translation form of the
     product (oracle apply_translation_form: rounding eps |K| |u_J - u_I|
     instead of eps |K| |u|), K d = r by the same PCG to 1e-6 of ||r||,
     u += d; twice.  The second correction's size estimates u_ref's error.
The FP64 true residual of any FP64 vector stops near eps || |K| |u| || / ||f||
(u's own rounding, times K), 3.7e-9 here, so the residual cannot certify u
below that; the refinement corrections do.  A banded Cholesky solve (the
oracle's exact solver) would need a band of 2 x 1,723 node layers, 10,215 x
1,013,643 doubles = 77 GB: not done here.

Output: c2_u_ref.npz (u_ref float64 [3N] and the figures below) and
c2_u_ref.txt (the figures as text).
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fsfem as O  # noqa: E402
from paper_2001_08849_amd import meshgen as mg  # noqa: E402

CHUNK = 250_000


def log(*a):
    print(*a, flush=True)


def main():
    t0 = time.time()
    p = mg.cantilever_c2()
    m = p.mesh
    faces = O.extract_faces(m.tets)
    tab = faces["table"]
    n = 3 * m.n_nodes
    vol = O.tet_volume(m.xyz[m.tets])
    log(f"mesh: {m.tets.shape[0]} tets, {m.n_nodes} nodes, {tab.shape[0]} faces "
        f"({time.time() - t0:.0f} s)")

    K = sp.csr_matrix((n, n))
    for s in range(0, tab.shape[0], CHUNK):
        IK, JK, VK = [], [], []
        blk = tab[s:s + CHUNK]
        for part in (blk[blk[:, 4] < 0], blk[blk[:, 4] >= 0]):
            if part.shape[0]:
                Kf, nodes = O.face_stiffness(m.xyz, m.tets, part, p.E, p.nu, vol)
                i, j, v = O._coo_block(Kf, nodes)
                IK.append(i), JK.append(j), VK.append(v)
        Kc = sp.coo_matrix((np.concatenate(VK), (np.concatenate(IK), np.concatenate(JK))),
                           shape=(n, n)).tocsr()
        K = K + Kc
        log(f"  faces {s + blk.shape[0]}/{tab.shape[0]} ({time.time() - t0:.0f} s)")
    K.sort_indices()
    f = O.traction_load(m.xyz, m.end_tris, np.asarray(p.traction, dtype=np.float64))
    Kb, fb = O.apply_dirichlet(K, f, p.fixed_dofs())
    del K
    log(f"assembled: nnz {Kb.nnz} ({time.time() - t0:.0f} s)")

    nf = np.linalg.norm(fb)
    R = O.block_row_sums(Kb)
    u, it0, rr0 = O.pcg_jacobi(Kb, fb, rtol=1e-8, max_iter=30000)
    floor = np.finfo(np.float64).eps * np.linalg.norm(abs(Kb) @ np.abs(u)) / nf
    log(f"PCG to 1e-8: {it0} iterations, relres {rr0:.3e}; eps|K||u|/|f| {floor:.3e} "
        f"({time.time() - t0:.0f} s)")
    steps = []
    for k in range(2):
        r = fb - O.apply_translation_form(Kb, u, R)
        d, itk, rrk = O.pcg_jacobi(Kb, r, rtol=1e-6, max_iter=30000)
        u = u + d
        steps.append((float(np.linalg.norm(r) / nf), itk, float(np.linalg.norm(d) / np.linalg.norm(u))))
        log(f"refinement {k + 1}: relres before {steps[-1][0]:.3e}, {itk} iterations, "
            f"|d| / |u| {steps[-1][2]:.3e} ({time.time() - t0:.0f} s)")
    rr = float(np.linalg.norm(fb - O.apply_translation_form(Kb, u, R)) / nf)

    tip = np.flatnonzero(np.isclose(m.xyz[:, 0], m.lengths[0]))
    np.savez_compressed(os.path.join(HERE, "c2_u_ref.npz"), u=u, relres=rr, floor=floor,
                        pcg_iters=it0, correction1=steps[0][2], correction2=steps[1][2])
    with open(os.path.join(HERE, "c2_u_ref.txt"), "w") as fh:
        fh.write(
            "# FP64 oracle displacements of the 1.92M-tet cantilever (200x40x40 cells,\n"
            "# +/-10% jitter seed 2, E 210e9, nu 0.3, clamp x=0, traction (0,0,-1e6) Pa).\n"
            "# Written by tests/golden/make_c2_reference.py (oracle only); u itself is in\n"
            "# c2_u_ref.npz.\n"
            f"n_dofs {n}\nnnz {Kb.nnz}\n"
            f"eps_absK_absu_over_f {floor:.6e}\n"
            f"pcg_to_1e-8_iterations {it0}\npcg_to_1e-8_relres {rr0:.6e}\n"
            f"refinement_1 relres_before {steps[0][0]:.6e} iterations {steps[0][1]} "
            f"correction_rel_l2 {steps[0][2]:.6e}\n"
            f"refinement_2 relres_before {steps[1][0]:.6e} iterations {steps[1][1]} "
            f"correction_rel_l2 {steps[1][2]:.6e}\n"
            f"final_relres_translation_form {rr:.6e}\n"
            f"tip_uz_mean {u[3 * tip + 2].mean():.10e}\n")
    log(f"written ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
