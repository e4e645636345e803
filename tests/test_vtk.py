"""Host-side VTK output: files round-trip exactly (binary and ASCII), the
cell structure is what ParaView expects, and von Mises matches its closed
forms (uniaxial stress s -> |s|, pure shear t -> sqrt(3) |t|)."""
import numpy as np
import pytest

from oracle import fsfem as O
from paper_2001_08849_amd import meshgen as mg
from paper_2001_08849_amd import vtk


def test_von_mises_closed_forms():
    s = np.zeros((4, 6))
    s[0, 0] = -3.0                      # uniaxial
    s[1, 5] = 2.0                       # pure shear xy
    s[2, :3] = 5.0                      # hydrostatic
    s[3] = [1.0, -2.0, 0.5, 0.3, -0.7, 1.1]
    vm = vtk.von_mises(s)
    dev = np.array([[1.0, 1.1, -0.7], [1.1, -2.0, 0.3], [-0.7, 0.3, 0.5]])
    dev -= np.trace(dev) / 3 * np.eye(3)
    np.testing.assert_allclose(vm[:3], [3.0, 2.0 * np.sqrt(3.0), 0.0], atol=1e-15)
    np.testing.assert_allclose(vm[3], np.sqrt(1.5 * np.sum(dev * dev)), rtol=1e-14)


@pytest.mark.parametrize("binary", [True, False])
def test_round_trip(tmp_path, binary):
    m = mg.box_mesh(4, 2, 3, 2.0, 1.0, 1.5, jitter=0.15, seed=3)
    rng = np.random.default_rng(5)
    u = rng.standard_normal(3 * m.n_nodes) * 1e-3
    faces = O.extract_faces(m.tets)["table"]
    eps, sig = O.face_strain_stress(m.xyz, m.tets, 2e11, 0.3, u)
    p1, p2 = tmp_path / "u.vtk", tmp_path / "faces.vtk"
    vtk.write_solution(p1, m.xyz, m.tets, u, binary=binary)
    vtk.write_face_fields(p2, m.xyz, faces, eps, sig, binary=binary)
    a = vtk.read_legacy(p1)
    assert np.array_equal(a["points"], m.xyz)
    assert np.array_equal(a["cells"], m.tets)
    assert np.all(a["cell_types"] == vtk.VTK_TETRA)
    assert np.array_equal(a["point_data"]["displacement"], u.reshape(-1, 3))
    b = vtk.read_legacy(p2)
    assert np.array_equal(b["cells"], faces[:, :3])
    assert np.all(b["cell_types"] == vtk.VTK_TRIANGLE)
    assert np.array_equal(b["cell_data"]["strain"], eps)
    assert np.array_equal(b["cell_data"]["stress"], sig)
    assert np.array_equal(b["cell_data"]["von_mises"][:, 0], vtk.von_mises(sig))
