"""Pins of the FP64 learned-preconditioner reference: finite-difference
gradients, SPD-ness and symmetry of M, the Jacobi limit, fixed DOFs."""
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


def test_M_symmetric_spd_and_masked(tiny):
    g, K, R, E = tiny
    for seed in (1, 2):
        P = random_params(seed, scale_out=2.0)   # strong output: scaling is active
        Sp, c = G.forward(P, g)
        assert (c["cfac"] < 1).any()
        M, S = M_dense(g, Sp)
        assert np.abs(S - S.T).max() < 1e-14
        ev = np.linalg.eigvalsh(M * np.sqrt(g.d)[:, None] * np.sqrt(g.d)[None, :])
        assert ev.min() >= 1 - G.GAMMA - 1e-12      # Gershgorin: I + S' >= (1-gamma) I
        fx = np.flatnonzero(g.fixed)
        off = S[fx].copy()
        assert np.abs(off).max() == 0.0
        # apply_M matches the dense matrix
        r = np.random.default_rng(seed).standard_normal(3 * g.N)
        np.testing.assert_allclose(G.apply_M(g, Sp, r), M @ r, rtol=1e-12, atol=1e-20)


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
