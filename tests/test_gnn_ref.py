"""Pins of the FP64 learned-preconditioner reference: finite-difference
gradients, symmetry of M, the Jacobi limit, fixed DOFs, node-renumbering
equivariance."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fsfem as O
from oracle import gnn_ref as G
from paper_2001_08849_amd import meshgen as mg


@pytest.fixture(scope="module")
def tiny():
    p = mg.learned_small(1, grid=(4, 2, 2))
    m = p.mesh
    K = O.assemble(m.xyz, m.tets, p.E, p.nu)
    f = O.traction_load(m.xyz, m.end_tris, p.traction)
    Kb, fb = O.apply_dirichlet(K, f, p.fixed_dofs())
    g = G.build_graph(Kb, m.xyz, p.fixed_dofs())
    rng = np.random.default_rng(0)
    E = rng.standard_normal((Kb.shape[0], 3))
    E[p.fixed_dofs()] = 0.0
    R = Kb @ E
    return g, Kb, R, E


def random_params(seed, scale_out=0.05):
    P = G.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    P["Wo"] = rng.standard_normal(P["Wo"].shape) * scale_out
    for k in P:
        if k.startswith(("b", "c")):
            P[k] = rng.standard_normal(P[k].shape) * 0.1
    return P


def M_dense(g, Sp):
    n = 3 * g.N
    rows, cols, vals = [], [], []
    for k in range(len(g.row)):
        for a in range(3):
            for b in range(3):
                rows.append(3 * g.row[k] + a)
                cols.append(3 * g.bcol[k] + b)
                vals.append(Sp[k, a, b])
    S = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).toarray()
    s = 1.0 / np.sqrt(g.d)
    return (np.eye(n) + S) * s[:, None] * s[None, :], S


def test_finite_difference_gradients(tiny):
    g, K, R, E = tiny
    P = random_params(3)
    L, grads = G.backward(P, g, K, R, E)
    rng = np.random.default_rng(9)
    worst = 0.0
    for name, W in P.items():
        scale = np.abs(grads[name]).max()
        idx = [tuple(rng.integers(0, s) for s in W.shape) for _ in range(3)]
        for ix in idx:
            an = grads[name][ix]
            errs = []
            # central differences; the best of three steps (a step can cross
            # a ReLU or max() kink, a tiny one drowns in roundoff)
            for h in (1e-4, 1e-5, 1e-6):
                Wp = {k: v.copy() for k, v in P.items()}
                Wm = {k: v.copy() for k, v in P.items()}
                Wp[name][ix] += h
                Wm[name][ix] -= h
                fd = (G.loss(Wp, g, K, R, E) - G.loss(Wm, g, K, R, E)) / (2 * h)
                errs.append(abs(fd - an) / max(abs(an), 1e-3 * scale, 1e-12))
            worst = max(worst, min(errs))
    assert worst < 1e-5, worst


def test_M_symmetric_and_masked(tiny):
    g, K, R, E = tiny
    for seed in (1, 2):
        P = random_params(seed, scale_out=2.0)
        Sp, c = G.forward(P, g)
        M, S = M_dense(g, Sp)
        assert np.abs(S).max() > 0
        assert np.abs(S - S.T).max() < 1e-14
        fx = np.flatnonzero(g.fixed)
        assert np.abs(S[fx]).max() == 0.0 and np.abs(S[:, fx]).max() == 0.0
        # apply_M matches the dense matrix, for one vector and for a panel
        rng = np.random.default_rng(seed)
        r = rng.standard_normal(3 * g.N)
        np.testing.assert_allclose(G.apply_M(g, Sp, r), M @ r, rtol=1e-12, atol=1e-20)
        Rp = rng.standard_normal((3 * g.N, 4))
        np.testing.assert_allclose(G.apply_M(g, Sp, Rp), M @ Rp, rtol=1e-12, atol=1e-20)


def test_node_renumbering_equivariance():
    """Renumbering the mesh nodes permutes S' and nothing else: catches a
    transposed block, a swapped endpoint or a wrong transpose-edge index."""
    p = mg.learned_small(2, grid=(3, 2, 2))
    m = p.mesh
    P = random_params(4, scale_out=0.5)
    fixed = p.fixed_dofs()

    def run(xyz, tets, fixed_dofs):
        K = O.assemble(xyz, tets, p.E, p.nu)
        f = np.zeros(K.shape[0])
        Kb, _ = O.apply_dirichlet(K, f, fixed_dofs)
        g = G.build_graph(Kb, xyz, fixed_dofs)
        Sp, _ = G.forward(P, g)
        return g, Sp

    g0, S0 = run(m.xyz, m.tets, fixed)
    N = m.xyz.shape[0]
    perm = np.random.default_rng(5).permutation(N)       # new id of old node i
    xyz1 = np.empty_like(m.xyz)
    xyz1[perm] = m.xyz
    fixed1 = (3 * perm[np.asarray(fixed) // 3] + np.asarray(fixed) % 3)
    g1, S1 = run(xyz1, perm[m.tets], np.sort(fixed1))
    pos1 = {(int(i), int(j)): k for k, (i, j) in enumerate(zip(g1.row, g1.bcol))}
    for k, (i, j) in enumerate(zip(g0.row, g0.bcol)):
        k1 = pos1[(int(perm[i]), int(perm[j]))]
        np.testing.assert_allclose(S1[k1], S0[k], rtol=1e-9, atol=1e-12 * np.abs(S0).max())


def test_initial_network_is_jacobi(tiny):
    g, K, R, E = tiny
    P = G.init_params(0)
    Sp, _ = G.forward(P, g)
    assert np.abs(Sp).max() == 0.0
    r = np.arange(3 * g.N, dtype=float)
    np.testing.assert_allclose(G.apply_M(g, Sp, r), r / g.d, rtol=1e-15)


def test_graph_transpose_and_features(tiny):
    g, K, R, E = tiny
    assert np.array_equal(g.row[g.tr], g.bcol) and np.array_equal(g.bcol[g.tr], g.row)
    np.testing.assert_allclose(g.Kb[g.tr], np.transpose(g.Kb, (0, 2, 1)), rtol=0,
                               atol=1e-14 * np.abs(g.Kb).max())
    # Jacobi-scaled diagonal blocks have unit diagonals
    dk = g.y[g.row == g.bcol][:, [0, 4, 8]]
    np.testing.assert_allclose(dk, 1.0, rtol=1e-14)


def test_spd_theta_makes_M_positive_definite(tiny):
    g, K, R, E = tiny
    for seed, so in ((1, 0.05), (2, 3.0), (3, 30.0)):
        P = random_params(seed, scale_out=so)
        Sp, _ = G.forward(P, g)
        theta, lmin = G.spd_theta(g, Sp)
        S = G.correction_matrix(g, Sp).toarray()
        ev = np.linalg.eigvalsh(S)
        assert lmin == pytest.approx(ev[0], rel=1e-10, abs=1e-12)
        if lmin >= -0.9 / 1.05:
            assert theta == 1.0
        else:
            assert theta == pytest.approx(0.9 / (1.05 * -lmin))
        lam = np.linalg.eigvalsh(np.eye(S.shape[0]) + theta * S)
        assert lam[0] >= 0.1 - 1e-12
    # the strongest output needs the scaling
    assert theta < 1.0
