"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: exact
rationals derived from centroid definitions (Table 1), unit-simplex values
(Eq. 10/11), an independent volume routine, brute-force face pairing,
closed-form face counts (Eq. 12), the divergence-theorem identity behind
Eq. 7, the strain energy of linear fields, rigid-body modes, the patch test,
dense and banded direct solves, Euler-Bernoulli convergence and the FEM-T4 /
FS-FEM ordering of Table 4.
"""
import os

import numpy as np
import pytest

from oracle import fsfem as O
from paper_2001_08849_amd import meshgen as mg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------- Table 1
def _bary(name, interior=True):
    """Shape values at the centroid of a named triangle, from the definition:
    a field node carries N = e_I, a tet centroid the mean of its 4 nodes."""
    e = np.eye(5)
    pt = {"A": e[0], "B": e[1], "C": e[2], "D": e[3], "E": e[4]}
    pt["F"] = (e[0] + e[1] + e[2] + e[3]) / 4
    pt["G"] = (e[0] + e[1] + e[2] + e[4]) / 4
    v = sum(pt[c] for c in name) / 3
    return v if interior else v[:4]


def test_table1_interior_from_centroids():
    for g, (name, vals) in O.TABLE1_INTERIOR.items():
        np.testing.assert_allclose(_bary(name), vals, rtol=0, atol=1e-15, err_msg=g)


def test_table1_rows_as_printed():
    # the six rows exactly as printed in Table 1 (A, B, C, D, E columns)
    printed = {
        "g1": (5, 1, 5, 1, 0), "g2": (5, 1, 5, 0, 1), "g3": (1, 5, 5, 0, 1),
        "g4": (1, 5, 5, 1, 0), "g5": (5, 5, 1, 1, 0), "g6": (5, 5, 1, 0, 1),
    }
    for g, twelfths in printed.items():
        np.testing.assert_allclose(O.TABLE1_INTERIOR[g][1], np.array(twelfths) / 12.0, atol=1e-16)


def test_exterior_gauss_values_from_centroids():
    for name, vals in O.TABLE1_EXTERIOR.items():
        np.testing.assert_allclose(_bary(name, interior=False), vals, atol=1e-15)


# ------------------------------------------------------------ Eq. 10 / 11
def test_eq10_eq11_unit_simplex():
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)
    assert O.tet_volume(P) == pytest.approx(1 / 6, abs=1e-16)
    assert O.tet_volume(P[[1, 0, 2, 3]]) == pytest.approx(1 / 6, abs=1e-16)  # orientation-free
    assert O.tri_area(P[0], P[1], P[2]) == pytest.approx(0.5, abs=1e-16)


def test_eq10_against_convex_hull():
    from scipy.spatial import ConvexHull
    rng = np.random.default_rng(0)
    for _ in range(20):
        P = rng.standard_normal((4, 3))
        assert O.tet_volume(P) == pytest.approx(ConvexHull(P).volume, rel=1e-12)


# ------------------------------------------------------------------ Alg. 1
def test_face_pairing_brute_force():
    m = mg.box_mesh(3, 2, 2, 3.0, 2.0, 2.0, jitter=0.1, seed=5).tets
    faces = O.extract_faces(m)["table"]
    brute = {}
    for t, tet in enumerate(m):
        for lv in range(4):
            key = tuple(sorted(int(v) for i, v in enumerate(tet) if i != lv))
            brute.setdefault(key, []).append((t, int(tet[lv])))
    assert len(brute) == faces.shape[0]
    keys = sorted(brute)
    for row, key in zip(faces, keys):
        assert tuple(row[:3]) == key
        owners = sorted(brute[key])
        assert row[3] == owners[0][0] and row[5] == owners[0][1]
        if len(owners) == 2:
            assert row[4] == owners[1][0] and row[6] == owners[1][1]
        else:
            assert row[4] == -1 and row[6] == -1


def test_face_counts_eq12():
    rows = np.loadtxt(os.path.join(GOLD, "eq12_coo_lengths.txt"), dtype=np.int64)
    for nx, ny, nz, ne, ni, coo in rows[:2]:
        m = mg.box_mesh(int(nx), int(ny), int(nz), 1.0, 1.0, 1.0)
        f = O.extract_faces(m.tets)
        assert f["face_out"].shape[0] == ne and f["face_in"].shape[0] == ni
        assert 144 * ne + 225 * ni == coo
    # the closed forms hold on every listed grid
    for nx, ny, nz, ne, ni, coo in rows:
        assert ne == 4 * (nx * ny + ny * nz + nz * nx)
        assert ni == (24 * nx * ny * nz - ne) // 2
        assert coo == 144 * ne + 225 * ni
    p = mg.cantilever_c0()
    IK, JK, VK = O.assemble_coo(p.mesh.xyz, p.mesh.tets, p.E, p.nu)
    assert IK.size == rows[0, 5]


def test_non_manifold_face_rejected():
    tets = np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 5]])
    with pytest.raises(ValueError):
        O.extract_faces(tets)


# -------------------------------------------------------- Eq. 7 closed form
def _grad_N(P):
    """Gradients of the 4 linear shape functions of tet P [4,3]: grad N_a =
    -(area vector of the face opposite a, pointing away from a) / (3V)."""
    g = np.zeros((4, 3))
    V = abs(np.dot(np.cross(P[1] - P[0], P[2] - P[0]), P[3] - P[0])) / 6
    for a in range(4):
        o = [i for i in range(4) if i != a]
        n = 0.5 * np.cross(P[o[1]] - P[o[0]], P[o[2]] - P[o[0]])
        if np.dot(n, P[a] - P[o[0]]) > 0:
            n = -n
        g[a] = -n / (3 * V)
    return g, V


def test_eq7_equals_volume_weighted_gradients():
    """Divergence theorem: with N linear on each tet and one-point centroid
    quadrature exact on each boundary triangle, Eq. 7 equals the average of
    the tet gradients weighted by the sub-domain volumes V_e/4."""
    p = mg.cantilever_scaled(6, 3, 3, jitter=0.15, seed=3)
    m = p.mesh
    tab = O.extract_faces(m.tets)["table"]
    worst = 0.0
    for blk in (tab[tab[:, 4] < 0], tab[tab[:, 4] >= 0]):
        bb, Vk = O.smoothed_gradients(m.xyz, blk)
        for f in range(blk.shape[0]):
            nodes = [int(v) for v in blk[f, [0, 1, 2, 5, 6]] if v >= 0]
            acc = np.zeros((len(nodes), 3))
            wsum = 0.0
            for t in blk[f, 3:5]:
                if t < 0:
                    continue
                g, V = _grad_N(m.xyz[m.tets[t]])
                for a, v in enumerate(m.tets[t]):
                    acc[nodes.index(int(v))] += (V / 4) * g[a]
                wsum += V / 4
            assert Vk[f] == pytest.approx(wsum, rel=1e-13)
            ref = acc / wsum
            worst = max(worst, np.abs(bb[f] - ref).max() / np.abs(ref).max())
    assert worst < 1e-13


def test_smoothing_volumes_sum_to_box():
    for p in (mg.cantilever_c0(), mg.cantilever_scaled(10, 3, 3, jitter=0.15, seed=2)):
        m = p.mesh
        tab = O.extract_faces(m.tets)["table"]
        tot = sum(O.smoothed_gradients(m.xyz, blk)[1].sum()
                  for blk in (tab[tab[:, 4] < 0], tab[tab[:, 4] >= 0]))
        assert tot == pytest.approx(np.prod(m.lengths), rel=1e-13)


# ----------------------------------------------------------- stiffness pins
@pytest.fixture(scope="module")
def c0_K():
    p = mg.cantilever_c0()
    return p, O.assemble(p.mesh.xyz, p.mesh.tets, p.E, p.nu)


def test_K_symmetric_and_rigid_modes(c0_K):
    p, K = c0_K
    s = abs(K).max()
    assert abs(K - K.T).max() <= 1e-14 * s
    R = O.rigid_modes(p.mesh.xyz)
    assert np.abs(K @ R.T).max() <= 1e-12 * s


def test_exactly_six_zero_eigenvalues(c0_K):
    _, K = c0_K
    ev = np.linalg.eigvalsh(K.toarray())
    lmax = ev[-1]
    assert np.sum(np.abs(ev) <= 1e-12 * lmax) == 6
    assert ev[6] > 1e-6 * lmax


def _energy_closed_form(A, Vol_lam_mu):
    eps = 0.5 * (A + A.T)
    return sum(V * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
               for V, lam, mu in Vol_lam_mu)


def test_linear_field_energy_homogeneous():
    """u = A x + c: the smoothed strain equals sym(A) in every smoothing
    domain, so u^T K u = Vol (lam tr(eps)^2 + 2 mu eps:eps) exactly.  This
    pins Eq. 4's Voigt layout (engineering shear), D and Eq. 9's sum."""
    p = mg.cantilever_scaled(5, 3, 2, jitter=0.15, seed=4)
    m = p.mesh
    K = O.assemble(m.xyz, m.tets, p.E, p.nu)
    lam, mu = O.lame(p.E, p.nu)
    rng = np.random.default_rng(7)
    for _ in range(3):
        A = rng.standard_normal((3, 3))
        u = (m.xyz @ A.T + rng.standard_normal(3)).reshape(-1)
        ref = _energy_closed_form(A, [(np.prod(m.lengths), lam, mu)])
        assert u @ (K @ u) == pytest.approx(ref, rel=1e-12)


def test_linear_field_energy_heterogeneous():
    """Per-tet (E, nu): the smoothing-domain constants are quarter-volume
    weighted means, so u^T K u = sum_e V_e (lam_e tr^2 + 2 mu_e eps:eps)."""
    p = mg.learned_small(0, grid=(6, 3, 3))
    m = p.mesh
    K = O.assemble(m.xyz, m.tets, p.E, p.nu)
    lam, mu = O.lame(p.E, p.nu)
    V = O.tet_volume(m.xyz[m.tets])
    A = np.random.default_rng(8).standard_normal((3, 3))
    u = (m.xyz @ A.T).reshape(-1)
    ref = _energy_closed_form(A, zip(V, lam, mu))
    assert u @ (K @ u) == pytest.approx(ref, rel=1e-12)


def test_single_tet_reduces_to_fem_t4():
    """One tet: every face is exterior, b = grad N exactly and the four
    domains hold V/4 each, so FS-FEM K equals the FEM-T4 element matrix."""
    P = np.array([[0, 0, 0], [1.1, 0.1, 0], [0.2, 0.9, 0.1], [0.1, 0.3, 1.2]])
    tets = np.array([[0, 1, 2, 3]])
    Kf = O.assemble(P, tets, 1e9, 0.27).toarray()
    Kt = O.fem_t4_assemble(P, tets, 1e9, 0.27).toarray()
    np.testing.assert_allclose(Kf, Kt, rtol=0, atol=1e-12 * np.abs(Kt).max())


def test_fem_t4_element_energy():
    """FEM-T4 (the comparator) pinned by the same closed-form energy."""
    P = np.array([[0, 0, 0], [1.1, 0.1, 0], [0.2, 0.9, 0.1], [0.1, 0.3, 1.2]])
    Kt = O.fem_t4_assemble(P, np.array([[0, 1, 2, 3]]), 1e9, 0.27)
    lam, mu = O.lame(1e9, 0.27)
    A = np.random.default_rng(1).standard_normal((3, 3))
    u = (P @ A.T).reshape(-1)
    ref = _energy_closed_form(A, [(O.tet_volume(P), lam, mu)])
    assert u @ (Kt @ u) == pytest.approx(ref, rel=1e-12)


def test_patch_test():
    """Linear u prescribed on every boundary node is reproduced at the
    interior nodes (no loads) to 1e-12 (elimination with nonzero values)."""
    m = mg.box_mesh(4, 4, 4, 1.0, 1.0, 1.0, jitter=0.2, seed=11)
    K = O.assemble(m.xyz, m.tets, 1e9, 0.3)
    A = np.array([[1e-3, 2e-4, -3e-4], [5e-4, -1e-3, 1e-4], [2e-4, 3e-4, 7e-4]])
    c = np.array([1e-4, -2e-4, 3e-4])
    uex = (m.xyz @ A.T + c).reshape(-1)
    on_bnd = np.any(np.isclose(m.xyz, 0.0) | np.isclose(m.xyz, 1.0), axis=1)
    bn = np.flatnonzero(on_bnd)
    dofs = (3 * bn[:, None] + np.arange(3)).reshape(-1)
    Kb, f = O.apply_dirichlet(K, np.zeros(K.shape[0]), dofs, uex[dofs])
    u = O.solve_dense(Kb, f)
    assert np.abs(u - uex).max() <= 1e-12 * np.abs(uex).max()


def test_sampled_rows_match_full(c0_K):
    p, K = c0_K
    rows = O.assemble_rows(p.mesh.xyz, p.mesh.tets, p.E, p.nu, [0, 17, 50, 98])
    for I, (cols, vals) in rows.items():
        for a in range(3):
            r = K.getrow(3 * I + a)
            assert np.array_equal(r.indices, cols)
            np.testing.assert_allclose(r.data, vals[a], rtol=0, atol=1e-14 * np.abs(vals[a]).max())


# ------------------------------------------------------------ loads / BCs
def test_traction_total_force():
    p = mg.cantilever_scaled(4, 3, 5, jitter=0.1, seed=1, L=(2.0, 0.7, 1.3))
    t = np.array([1.0, -2.0, 3.5])
    f = O.traction_load(p.mesh.xyz, p.mesh.end_tris, t)
    np.testing.assert_allclose(f.reshape(-1, 3).sum(0), t * 0.7 * 1.3, rtol=1e-13)


def test_traction_per_vertex_by_hand():
    """Consistent load t A / 3 (Eq. 11 area) on two triangles worked by hand:
    ABC with A = (0,0,0), B = (3,0,0), C = (0,4,0) has area 6; BDC with
    D = (3,8,0) has |BD x BC| / 2 = |(0,8,0) x (-3,4,0)| / 2 = 12.  So A gets
    2t, B and C 2t + 4t = 6t, D 4t, and the unused node nothing."""
    xyz = np.array([[0, 0, 0], [3, 0, 0], [0, 4, 0], [3, 8, 0], [9, 9, 9]], dtype=np.float64)
    tris = np.array([[0, 1, 2], [1, 3, 2]])
    t = np.array([1.0, -2.0, 5.0])
    f = O.traction_load(xyz, tris, t).reshape(-1, 3)
    expect = np.array([2, 6, 6, 4, 0], dtype=np.float64)[:, None] * t
    np.testing.assert_allclose(f, expect, rtol=0, atol=1e-14)


def test_penalty_nonzero_values_approach_elimination(c0_K):
    """Penalty with prescribed values ubar != 0 (K_ii += alpha, f_i = alpha
    ubar_i) tends to elimination with the same values as alpha grows, with
    an error that falls like 1/alpha; the fixed DOFs take ubar."""
    p, K = c0_K
    f = O.traction_load(p.mesh.xyz, p.mesh.end_tris, p.traction)
    dofs = p.fixed_dofs()
    ubar = np.random.default_rng(5).uniform(-1e-3, 1e-3, dofs.size)
    Kb, fb = O.apply_dirichlet(K, f, dofs, ubar)
    ue = O.solve_dense(Kb, fb)
    np.testing.assert_allclose(ue[dofs], ubar, rtol=0, atol=1e-15)
    errs = []
    for scale in (1e4, 1e6, 1e8):
        Kp, fp = O.apply_penalty(K, f, dofs, scale * K.diagonal().max(), ubar)
        up = O.solve_dense(Kp, fp)
        errs.append(np.linalg.norm(up - ue) / np.linalg.norm(ue))
    assert errs[2] < 1e-6
    assert errs[1] < 2e-2 * errs[0] and errs[2] < 2e-2 * errs[1]


def test_penalty_approaches_elimination(c0_K):
    p, K = c0_K
    f = O.traction_load(p.mesh.xyz, p.mesh.end_tris, p.traction)
    Kb, fb = O.apply_dirichlet(K, f, p.fixed_dofs())
    ue = O.solve_dense(Kb, fb)
    Kp, fp = O.apply_penalty(K, f, p.fixed_dofs(), 1e8 * K.diagonal().max())
    up = O.solve_dense(Kp, fp)
    assert np.linalg.norm(up - ue) / np.linalg.norm(ue) < 1e-6


# ----------------------------------------------------------------- solves
def test_dense_banded_pcg_agree(c0_K):
    p, K = c0_K
    f = O.traction_load(p.mesh.xyz, p.mesh.end_tris, p.traction)
    Kb, fb = O.apply_dirichlet(K, f, p.fixed_dofs())
    ud = O.solve_dense(Kb, fb)
    ub = O.solve_banded(Kb, fb)
    x, it, rr = O.pcg_jacobi(Kb, fb, rtol=1e-10)
    assert rr <= 1e-10
    assert np.linalg.norm(ub - ud) / np.linalg.norm(ud) < 1e-12
    assert np.linalg.norm(x - ud) / np.linalg.norm(ud) < 1e-9


def _tip(p, u):
    m = p.mesh
    s = np.flatnonzero(np.isclose(m.xyz[:, 0], m.lengths[0]))
    return u[3 * s + 2].mean()


@pytest.mark.slow
def test_euler_bernoulli_convergence():
    """Tip deflection of the 10x1x1 cantilever under the end traction moves
    monotonically toward P L^3 / (3 E I) as the grid is refined."""
    ratios = []
    for n in (1, 2, 4):
        m = mg.box_mesh(10 * n, 2 * n, 2 * n, 10.0, 1.0, 1.0)
        p = mg.Problem("eb", m, 210e9, 0.3, np.array([0.0, 0.0, -1e6]), 1e-10)
        Kb, fb, _ = O.problem_system(p)
        u = O.solve_banded(Kb, fb)
        eb = -1e6 * 1.0 * 10.0 ** 3 / (3 * 210e9 * (1.0 / 12.0))
        ratios.append(_tip(p, u) / eb)
    assert ratios[0] < ratios[1] < ratios[2] < 1.05
    errs = [abs(1 - r) for r in ratios]
    assert errs[2] < 0.5 * errs[1] < 0.25 * errs[0]
    assert 0.45 < ratios[0] < 0.52          # coarse FS-FEM is far from EB
    assert ratios[2] > 0.9


def test_table4_ordering_and_band():
    """Table 4: FEM-T4 is stiffer than FS-FEM, which is stiffer than the fine
    T10 reference, at every station; on the stand-in mesh the FS-FEM tip is
    within 10% of the paper's value (the paper's own mesh is not available)."""
    gold = np.loadtxt(os.path.join(GOLD, "table4_deflections.txt"))
    p = mg.paper_beam()
    m = p.mesh
    K = O.assemble(m.xyz, m.tets, p.E, p.nu)
    f = O.traction_load(m.xyz, m.top_tris, p.traction)
    Kb, fb = O.apply_dirichlet(K, f, p.fixed_dofs())
    u = O.solve_dense(Kb, fb)
    Kt = O.fem_t4_assemble(m.xyz, m.tets, p.E, p.nu)
    Ktb, ft = O.apply_dirichlet(Kt, f, p.fixed_dofs())
    ut = O.solve_dense(Ktb, ft)
    for x, t4, fs, t10 in gold:
        assert abs(t4) < abs(fs) < abs(t10)          # the paper's own ordering
        s = np.flatnonzero(np.isclose(m.xyz[:, 0], x))
        w_fs, w_t4 = u[3 * s + 2].mean(), ut[3 * s + 2].mean()
        assert abs(w_t4) < abs(w_fs) < abs(t10)
    assert abs(w_fs / gold[-1, 2] - 1) < 0.10


def test_face_strain_patch_and_rigid_motions():
    """Smoothed strains: a linear displacement field u = A x + c gives the
    exact constant strain sym(A) (Voigt, engineering shear) on every
    smoothing domain, interior and exterior, and its stress is the
    isotropic c applied to it with the domain's own material; a rigid
    motion (translation + infinitesimal rotation) gives zero strain."""
    m = mg.box_mesh(4, 3, 2, 2.0, 1.5, 1.0, jitter=0.2, seed=5)
    rng = np.random.default_rng(8)
    E = 10.0 ** rng.uniform(9, 11, size=m.n_tets)
    nu = rng.uniform(0.2, 0.45, size=m.n_tets)
    A = rng.standard_normal((3, 3))
    c = rng.standard_normal(3)
    u = (m.xyz @ A.T + c).reshape(-1)
    eps, sig = O.face_strain_stress(m.xyz, m.tets, E, nu, u)
    Sym = 0.5 * (A + A.T)
    want = np.array([Sym[0, 0], Sym[1, 1], Sym[2, 2], 2 * Sym[1, 2], 2 * Sym[0, 2], 2 * Sym[0, 1]])
    np.testing.assert_allclose(eps, np.broadcast_to(want, eps.shape), rtol=0, atol=1e-12)
    # stress: tr(eps) lambda + 2 mu eps on the diagonal, mu gamma off it, with
    # lambda, mu recovered from the stress of a pure dilatation
    ones = (m.xyz @ np.eye(3).T).reshape(-1)          # eps = (1, 1, 1, 0, 0, 0)
    _, sd = O.face_strain_stress(m.xyz, m.tets, E, nu, ones)
    three_lam_2mu = sd[:, 0]                           # 3 lambda + 2 mu
    np.testing.assert_allclose(sd[:, 0], sd[:, 1], rtol=1e-12)
    assert np.abs(sd[:, 3:]).max() <= 1e-12 * np.abs(sd).max()
    shear = np.zeros((3, 3)); shear[0, 1] = shear[1, 0] = 0.5   # gamma_xy = 1
    _, ss = O.face_strain_stress(m.xyz, m.tets, E, nu, (m.xyz @ shear.T).reshape(-1))
    mu_f = ss[:, 5]
    lam_f = (three_lam_2mu - 2 * mu_f) / 3.0
    tr = want[:3].sum()
    np.testing.assert_allclose(sig[:, 0], lam_f * tr + 2 * mu_f * want[0], rtol=1e-10)
    np.testing.assert_allclose(sig[:, 4], mu_f * want[4], rtol=1e-10)
    # the recovered constants lie between the smallest and largest tet values
    lam_t, mu_t = O.lame(E, nu)
    assert mu_f.min() >= mu_t.min() * (1 - 1e-12) and mu_f.max() <= mu_t.max() * (1 + 1e-12)
    # rigid motion
    W = rng.standard_normal((3, 3)) * 1e-3
    W = W - W.T
    ur = (m.xyz @ W.T + c).reshape(-1)
    er, sr = O.face_strain_stress(m.xyz, m.tets, E, nu, ur)
    # roundoff only: |u| ~ 1 over cells of ~0.5 gives strains ~1e-15
    assert np.abs(er).max() < 1e-13 and np.abs(sr).max() < 1e-13 * E.max()


# ------------------------------------------------- products without a CSR
def _jittered_blob():
    p = mg.cantilever_scaled(6, 3, 4, jitter=0.2, seed=11, L=(3.0, 1.0, 1.4))
    T = p.mesh.n_tets
    rng = np.random.default_rng(12)
    return p, 10.0 ** rng.uniform(9, 11, T), rng.uniform(0.25, 0.45, T)


def test_apply_stiffness_equals_assembled_product():
    """sum_k K_k u_k over the face table (no CSR) equals the assembled K u,
    also when the face table is split into chunks whose shares are summed."""
    p, E, nu = _jittered_blob()
    m = p.mesh
    faces = O.extract_faces(m.tets)
    K = O.assemble(m.xyz, m.tets, E, nu, faces)
    u = np.random.default_rng(13).standard_normal(K.shape[0])
    y = O.apply_stiffness(m.xyz, m.tets, E, nu, u, faces)
    ref = K @ u
    tab = faces["table"]
    half = tab.shape[0] // 3
    y2 = sum(O.apply_stiffness(m.xyz, m.tets, E, nu, u, {"table": t})
             for t in (tab[:half], tab[half:]))
    scale = np.abs(K) @ np.abs(u)
    assert np.abs(y - ref).max() <= 1e-13 * scale.max()
    assert np.abs(y2 - ref).max() <= 1e-13 * scale.max()


def test_block_row_sums_exact():
    """R_I[a, c] = sum_J K[3I+a, 3J+c] against exactly rounded sums (fsum)
    of the dense matrix, on the BC-applied stiffness."""
    import math
    Kb, fb, _ = O.problem_system(mg.cantilever_c0())
    R = O.block_row_sums(Kb)
    D = Kb.toarray()
    N = D.shape[0] // 3
    for I in range(N):
        for a in range(3):
            for c in range(3):
                exact = math.fsum(D[3 * I + a, c::3])
                assert R[I, a, c] == exact


def test_translation_form_equals_plain_product():
    """On a random vector the translation form of K u equals the plain
    product to within the plain product's own rounding."""
    p, E, nu = _jittered_blob()
    m = p.mesh
    K = O.assemble(m.xyz, m.tets, E, nu)
    f = O.traction_load(m.xyz, m.end_tris, p.traction)
    Kb, _ = O.apply_dirichlet(K, f, p.fixed_dofs())
    u = np.random.default_rng(14).standard_normal(K.shape[0])
    y = O.apply_translation_form(Kb, u)
    scale = (np.abs(Kb) @ np.abs(u)).max()
    assert np.abs(y - Kb @ u).max() <= 1e-14 * scale


def test_translation_form_is_accurate_on_offset_fields():
    """A linear field with a large rigid offset, u = A x + c.  The product
    of the stored K with it, computed exactly in rational arithmetic on
    interior rows, is a small difference of terms of size |K| |c|: the plain
    product's rounding is of that size, eps |K| |c|, the translation form's
    only eps |K| |A| h (neighbour differences), so it is far closer."""
    from fractions import Fraction
    p, E, nu = _jittered_blob()
    m = p.mesh
    K = O.assemble(m.xyz, m.tets, 210e9, 0.3)
    A = np.array([[1e-3, 2e-4, -3e-4], [5e-4, -1e-3, 1e-4], [2e-4, 3e-4, 7e-4]])
    u = (m.xyz @ A.T + np.array([1e3, -2e3, 5e2])).reshape(-1)
    inner = np.ones(m.n_nodes, dtype=bool)
    for ax in range(3):
        inner &= ~np.isclose(m.xyz[:, ax], 0.0) & ~np.isclose(m.xyz[:, ax], m.lengths[ax])
    rows = (3 * np.flatnonzero(inner)[:8, None] + np.arange(3)).reshape(-1)
    plain, tf = K @ u, O.apply_translation_form(K, u)
    ep = et = 0.0
    for i in rows:
        lo, hi = K.indptr[i], K.indptr[i + 1]
        exact = float(sum(Fraction(float(v)) * Fraction(float(u[j]))
                          for v, j in zip(K.data[lo:hi], K.indices[lo:hi])))
        ep = max(ep, abs(plain[i] - exact))
        et = max(et, abs(tf[i] - exact))
    scale = (np.abs(K) @ np.full(K.shape[0], np.abs(A).max())).max()   # |K| |A| (1 m)
    print(f"interior rows of K (A x + c), error vs exact: plain {ep:.2e}, "
          f"translation form {et:.2e}; |K||A| {scale:.2e}")
    assert ep > 1e3 * et
    assert et <= 1e-14 * scale
