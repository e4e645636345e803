"""The 1.92M-tet cantilever (the paper-scale workload of Sec. 4.2, Table 3):
displacements from the GPU solvers against the FP64 oracle's.

tests/golden/c2_u_ref.npz holds the oracle's displacements of this problem,
written by tests/golden/make_c2_reference.py (oracle only: PCG to 1e-8, then
two refinement steps with the translation-form residual; its last correction
is the estimate of its own error).  Each GPU solve runs to an FP64 true
relative residual of 1e-8, as the benchmark does, and must give u within
1e-8 relative L2 of it.

Beside that, the residual of the GPU's u is evaluated by the oracle itself:
K_O u as the sum of the dense per-face K_k u_k over the whole face table
(no CSR), in worker processes.  That plain FP64 sum cannot resolve a
residual below its own rounding, eps || |K| |u| || / ||f|| (the workers
return it too): the bar is 1e-8 plus twice that floor.
"""
import multiprocessing as mp
import os

import numpy as np
import pytest

from oracle import fsfem as O
from oracle import gnn_ref as G
from paper_2001_08849_amd import meshgen as mg

pytestmark = pytest.mark.gpu

REF = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_u_ref.npz")
WORKERS = 8

_W = {}


def _init(xyz, tets, E, nu):
    _W.update(xyz=xyz, tets=tets, E=E, nu=nu, vol=O.tet_volume(xyz[tets]))


def _share(args):
    """K u and |K| |u| for one chunk of the face table: the oracle's dense
    face blocks K_k (Eq. 9) applied to the support displacements."""
    tab, u = args
    w = _W
    y = np.zeros(u.size)
    ab = np.zeros(u.size)
    for blk in (tab[tab[:, 4] < 0], tab[tab[:, 4] >= 0]):
        if not blk.shape[0]:
            continue
        Kf, nodes = O.face_stiffness(w["xyz"], w["tets"], blk, w["E"], w["nu"], w["vol"])
        m = nodes.shape[1]
        dof = (3 * nodes[:, :, None] + np.arange(3)).reshape(-1, 3 * m)
        ud = u[dof]
        y += np.bincount(dof.reshape(-1), np.einsum("fij,fj->fi", Kf, ud).reshape(-1),
                         minlength=u.size)
        ab += np.bincount(dof.reshape(-1),
                          np.einsum("fij,fj->fi", np.abs(Kf), np.abs(ud)).reshape(-1),
                          minlength=u.size)
    return y, ab


@pytest.fixture(scope="module")
def c2():
    from paper_2001_08849_amd import sfem
    if not os.path.exists(REF):
        pytest.skip("reference displacements not generated (tests/golden/make_c2_reference.py)")
    p = mg.cantilever_c2()
    ctx = sfem.Context(0)
    sfem.setup_problem(ctx, p, f32_copy=True)
    ref = np.load(REF)
    faces = O.extract_faces(p.mesh.tets)
    f = O.traction_load(p.mesh.xyz, p.mesh.end_tris, np.asarray(p.traction, dtype=np.float64))
    fixed = np.zeros(f.size, dtype=bool)
    fixed[p.fixed_dofs()] = True
    f[fixed] = 0.0
    pool = mp.get_context("spawn").Pool(WORKERS, initializer=_init,
                                        initargs=(p.mesh.xyz, p.mesh.tets, p.E, p.nu))
    yield p, ctx, ref, faces["table"], f, fixed, pool
    pool.close()
    pool.join()


def oracle_relres(c2, u):
    """(||f - K_O u|| / ||f||, eps || |K_O| |u| || / ||f||) on the free DOFs
    (u must vanish on the clamped ones: elimination)."""
    p, ctx, ref, tab, f, fixed, pool = c2
    assert np.all(u[fixed] == 0.0)
    chunks = np.array_split(tab, 4 * WORKERS)
    parts = pool.map(_share, [(ch, u) for ch in chunks])
    Ku = sum(y for y, _ in parts)
    aKu = sum(a for _, a in parts)
    r = np.where(fixed, 0.0, f - Ku)
    nf = np.linalg.norm(f)
    return np.linalg.norm(r) / nf, np.finfo(float).eps * np.linalg.norm(aKu[~fixed]) / nf


def _check(c2, name, u, info):
    p, ctx, ref, *_ = c2
    u_ref = ref["u"]
    err = np.linalg.norm(u - u_ref) / np.linalg.norm(u_ref)
    rr_o, floor = oracle_relres(c2, u)
    print(f"{name}: {info['iters']} iterations, GPU true relres {info['true_relres']:.3e}; "
          f"u error vs the oracle's u {err:.3e} (its own error estimate "
          f"{float(ref['correction2']):.1e}); oracle-evaluated relres {rr_o:.3e} "
          f"(its rounding floor {floor:.2e})", flush=True)
    assert info["converged"] and info["true_relres"] <= 1e-8
    assert err <= 1e-8
    assert rr_o <= 1e-8 + 2.0 * floor


def test_c2_jacobi_f64(c2):
    from paper_2001_08849_amd import sfem
    p, ctx, *_ = c2
    u, info = ctx.solve(rtol=1e-8, mode=sfem.MODE_F64)
    _check(c2, "Jacobi PCG FP64", u, info)


def test_c2_jacobi_f32_translation_form(c2):
    from paper_2001_08849_amd import sfem
    p, ctx, *_ = c2
    u, info = ctx.solve(rtol=1e-8, mode=sfem.MODE_F32_TF)
    _check(c2, "Jacobi PCG, FP32 values in the translation form", u, info)


def _random_network(sfem, seed=3, scale_out=0.3):
    P = G.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    P["Wo"] = rng.standard_normal(P["Wo"].shape) * scale_out
    for k in P:
        if k.startswith(("b", "c")):
            P[k] = rng.standard_normal(P[k].shape) * 0.1
    net = sfem.Gnn(0, seed=1)
    net.set_params(sfem.pack_params(P))
    return net


def test_c2_learned_fixed_seed_network(c2):
    """The learned flexible PCG with a fixed-seed (untrained, nonzero
    decoder) network, FP64 and FP32-translation-form products: the
    preconditioner changes the path, not the answer."""
    from paper_2001_08849_amd import sfem
    p, ctx, *_ = c2
    net = _random_network(sfem)
    net.apply(ctx)
    for name, mode in (("learned M, FP64 products", sfem.MODE_F64),
                       ("learned M, FP32 translation-form products", sfem.MODE_F32_TF)):
        u, info = ctx.solve(rtol=1e-8, mode=mode, precond=sfem.PRECOND_LEARNED,
                            max_iter=30000)
        _check(c2, name + (" (fell back)" if info["fell_back"] else ""), u, info)
