"""GPU parity of the post-processing step (smoothed strain and stress of
every smoothing domain) against the FP64 oracle: every face of small
meshes, sampled faces of the 1.92M-tet cantilever, and the patch test
(a linear field's exact constant strain) on every face at full size."""
import numpy as np
import pytest

from oracle import fsfem as O
from paper_2001_08849_amd import meshgen as mg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2001_08849_amd import sfem
    return sfem


def field_err(a, b):
    """Worst entry error of each Voigt column relative to that column's max."""
    return max(np.abs(a[:, k] - b[:, k]).max() / max(np.abs(b[:, k]).max(), 1e-300)
               for k in range(6))


@pytest.mark.parametrize("het", [False, True])
def test_face_stress_matches_oracle(S, het):
    m = mg.box_mesh(7, 3, 4, 3.5, 1.5, 2.0, jitter=0.2, seed=13)
    rng = np.random.default_rng(4)
    if het:
        E = 10.0 ** rng.uniform(9, 11, size=m.n_tets)
        nu = rng.uniform(0.2, 0.45, size=m.n_tets)
    else:
        E, nu = 7e10, 0.33
    u = rng.standard_normal(3 * m.n_nodes) * 1e-3
    ctx = S.Context(0)
    ctx.set_mesh(m.xyz, m.tets)
    ctx.set_material(E, nu)
    eps, sig, ms = ctx.face_stress(u)
    e_ref, s_ref = O.face_strain_stress(m.xyz, m.tets, E, nu, u)
    ee, es = field_err(eps, e_ref), field_err(sig, s_ref)
    print(f"face stress ({'per-tet' if het else 'homogeneous'} material): strain error {ee:.2e}, "
          f"stress error {es:.2e}")
    assert ee <= 1e-12 and es <= 1e-12


def test_face_stress_full_size(S):
    p = mg.cantilever_c2()
    m = p.mesh
    ctx = S.Context(0)
    ctx.set_mesh(m.xyz, m.tets)
    ctx.set_material(p.E, p.nu)
    # patch test on every face: u = A x + c has the strain sym(A) everywhere
    rng = np.random.default_rng(21)
    A = rng.standard_normal((3, 3)) * 1e-3
    c = rng.standard_normal(3)
    eps, sig, ms = ctx.face_stress((m.xyz @ A.T + c).reshape(-1))
    Sy = 0.5 * (A + A.T)
    want = np.array([Sy[0, 0], Sy[1, 1], Sy[2, 2], 2 * Sy[1, 2], 2 * Sy[0, 2], 2 * Sy[0, 1]])
    perr = np.abs(eps - want).max() / np.abs(want).max()
    # sampled faces of a random field against the oracle
    u = rng.standard_normal(3 * m.n_nodes) * 1e-3
    eps, sig, ms = ctx.face_stress(u)
    tab = O.extract_faces(m.tets)["table"]
    assert tab.shape[0] == eps.shape[0]
    pick = np.sort(rng.choice(tab.shape[0], size=4000, replace=False))
    e_ref, s_ref = O.face_strain_stress(m.xyz, m.tets, p.E, p.nu, u, faces={"table": tab[pick]})
    ee, es = field_err(eps[pick], e_ref), field_err(sig[pick], s_ref)
    print(f"c2 face stress: {eps.shape[0]} faces in {ms:.3f} ms; patch-test error {perr:.2e}; "
          f"sampled strain error {ee:.2e}, stress error {es:.2e}")
    assert perr <= 1e-10 and ee <= 1e-12 and es <= 1e-12
