"""Pins of the ES-FEM oracle (oracle/esfem.py) against what the
construction and the mathematics fix: sub-domain volumes (a sixth of each
tet), the divergence-theorem closed form of the smoothed gradients,
partition of unity, symmetry, rigid modes and six zero eigenvalues, the
exact energy of linear fields, the structural pattern by brute force, and
the softening against FEM-T4."""
import numpy as np

from oracle import esfem as ES
from oracle import fsfem as O
from paper_2001_08849_amd import meshgen as mg


def _mesh(jit=0.15, seed=3, dims=(4, 2, 3)):
    return mg.box_mesh(*dims, 2.0, 1.0, 1.5, jitter=jit, seed=seed)


def test_edge_table_brute_force():
    m = _mesh()
    E, ptr, et = ES.edge_table(m.tets)
    want = {}
    for t, v in enumerate(m.tets):
        for i in range(4):
            for j in range(i + 1, 4):
                want.setdefault((min(v[i], v[j]), max(v[i], v[j])), []).append(t)
    assert [tuple(e) for e in E] == sorted(want)
    for k, e in enumerate(E):
        assert list(et[ptr[k]:ptr[k + 1]]) == want[tuple(e)]


def test_volumes_and_closed_form_gradients():
    m = _mesh()
    sup, bb, Vk = ES.smoothed_gradients(m.xyz, m.tets)
    tv = O.tet_volume(m.xyz[m.tets])
    E, ptr, et = ES.edge_table(m.tets)
    assert np.isclose(Vk.sum(), 2.0 * 1.0 * 1.5, rtol=1e-13)
    P = m.xyz[m.tets]
    e1, e2, e3 = P[:, 1] - P[:, 0], P[:, 2] - P[:, 0], P[:, 3] - P[:, 0]
    det = np.einsum("ij,ij->i", e1, np.cross(e2, e3))
    G = np.stack([np.cross(e2, e3), np.cross(e3, e1), np.cross(e1, e2)], 1) / det[:, None, None]
    G = np.concatenate([-G.sum(1, keepdims=True), G], 1)          # grad N of each tet vertex
    worst = 0.0
    for k in range(len(E)):
        tt = et[ptr[k]:ptr[k + 1]]
        assert np.isclose(Vk[k], tv[tt].sum() / 6.0, rtol=1e-13)
        ref = np.zeros_like(bb[k])
        for t in tt:
            for i, v in enumerate(m.tets[t]):
                ref[np.searchsorted(sup[k], v)] += tv[t] / 6.0 * G[t, i]
        ref /= Vk[k]
        worst = max(worst, np.abs(bb[k] - ref).max() / np.abs(ref).max())
        assert np.abs(bb[k].sum(axis=0)).max() <= 1e-12 * np.abs(bb[k]).max()
    assert worst < 1e-12, worst


def test_symmetry_rigid_modes_and_spectrum():
    m = _mesh(dims=(3, 2, 2))
    K = ES.assemble(m.xyz, m.tets, 2e11, 0.3)
    Kd = K.toarray()
    assert np.abs(Kd - Kd.T).max() <= 1e-12 * np.abs(Kd).max()
    R = O.rigid_modes(m.xyz)
    assert np.abs(Kd @ R.T).max() <= 1e-10 * np.abs(Kd).max()
    ev = np.linalg.eigvalsh(Kd)
    assert np.all(np.abs(ev[:6]) <= 1e-10 * ev[-1]) and ev[6] > 1e-6 * ev[-1]


def test_linear_fields_energy_exact():
    m = _mesh()
    lam, mu = O.lame(7e10, 0.33)
    K = ES.assemble(m.xyz, m.tets, 7e10, 0.33)
    rng = np.random.default_rng(2)
    A = rng.standard_normal((3, 3))
    u = (m.xyz @ A.T).ravel()
    eps = 0.5 * (A + A.T)
    energy = 2 * mu * np.sum(eps * eps) + lam * np.trace(eps) ** 2
    assert np.isclose(u @ (K @ u), energy * 3.0, rtol=1e-12)


def test_pattern_brute_force():
    m = _mesh(dims=(3, 2, 2))
    K = ES.assemble(m.xyz, m.tets, 2e11, 0.3)
    E, ptr, et = ES.edge_table(m.tets)
    rows = [set() for _ in range(m.n_nodes)]
    for k in range(len(E)):
        S = set(np.unique(m.tets[et[ptr[k]:ptr[k + 1]]]).tolist())
        for I in S:
            rows[I] |= S
    for I in range(m.n_nodes):
        cols = K.indices[K.indptr[3 * I]:K.indptr[3 * I + 1]]
        assert sorted({c // 3 for c in cols}) == sorted(rows[I])


def test_softer_than_fem_t4():
    p = mg.cantilever_c0()
    m = p.mesh
    f = O.traction_load(m.xyz, m.end_tris, np.asarray(p.traction, float))
    tips = {}
    for name, K in (("es", ES.assemble(m.xyz, m.tets, p.E, p.nu)),
                    ("fs", O.assemble(m.xyz, m.tets, p.E, p.nu)),
                    ("fem", O.fem_t4_assemble(m.xyz, m.tets, p.E, p.nu))):
        Kb, fb = O.apply_dirichlet(K, f, p.fixed_dofs())
        u = O.solve_dense(Kb, fb)
        tips[name] = np.abs(u[2::3]).max()
    print(tips)
    assert tips["es"] > tips["fem"]


def test_rows_equal_full_assembly():
    m = mg.box_mesh(4, 3, 3, 2.0, 1.5, 1.5, jitter=0.15, seed=2)
    rng = np.random.default_rng(1)
    E = 10.0 ** rng.uniform(9, 11, m.n_tets)
    K = ES.assemble(m.xyz, m.tets, E, 0.3)
    for I, (cols, vals) in ES.assemble_rows(m.xyz, m.tets, E, 0.3, [0, 17, 40]).items():
        for a in range(3):
            r = 3 * I + a
            sl = slice(K.indptr[r], K.indptr[r + 1])
            assert np.array_equal(K.indices[sl], cols)
            assert np.abs(K.data[sl] - vals[a]).max() <= 1e-14 * np.abs(vals[a]).max()
