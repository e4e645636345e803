"""Legacy-VTK output for inspecting results in ParaView (Sec. 3.4 post-processing).

Two datasets, both VTK legacy 'UNSTRUCTURED_GRID' files (binary: big-endian,
as the legacy format requires):

- write_solution(path, xyz, tets, u): the tetrahedra (VTK_TETRA) with the
  nodal displacement as point data 'displacement' (3 components).
- write_face_fields(path, xyz, faces, strain, stress): one triangle
  (VTK_TRIANGLE) per face of the mesh, i.e. per smoothing domain, with the
  domain's smoothed strain and stress as cell data (Voigt order xx, yy, zz,
  yz, xz, xy, engineering shear) and the von Mises stress.  The smoothed
  fields are constant over a face's smoothing domain, so the face carries
  them.

read_legacy(path) parses files written here back into arrays (tests, tools).
Host code only: it takes arrays the library returned.
"""
from __future__ import annotations

import numpy as np

VTK_TRIANGLE = 5
VTK_TETRA = 10


def von_mises(stress: np.ndarray) -> np.ndarray:
    """Von Mises equivalent stress of Voigt rows (xx, yy, zz, yz, xz, xy)."""
    s = np.asarray(stress, float)
    xx, yy, zz, yz, xz, xy = (s[:, k] for k in range(6))
    return np.sqrt(0.5 * ((xx - yy) ** 2 + (yy - zz) ** 2 + (zz - xx) ** 2)
                   + 3.0 * (yz ** 2 + xz ** 2 + xy ** 2))


def _write(path, xyz, cells, ctype, point_data=(), cell_data=(), binary=True, title="sfem"):
    xyz = np.asarray(xyz, float).reshape(-1, 3)
    cells = np.asarray(cells, np.int64)
    n, k = cells.shape
    with open(path, "wb") as fh:
        def line(s):
            fh.write((s + "\n").encode("ascii"))

        def block(a, dtype, fmt):
            a = np.ascontiguousarray(a)
            if binary:
                fh.write(a.astype(dtype).tobytes())
                fh.write(b"\n")
            else:
                for row in a.reshape(len(a), -1):
                    line(" ".join(fmt % v for v in row))

        line("# vtk DataFile Version 3.0")
        line(title[:255])
        line("BINARY" if binary else "ASCII")
        line("DATASET UNSTRUCTURED_GRID")
        line(f"POINTS {len(xyz)} double")
        block(xyz, ">f8", "%.17g")
        line(f"CELLS {n} {n * (k + 1)}")
        block(np.hstack([np.full((n, 1), k, np.int64), cells]), ">i4", "%d")
        line(f"CELL_TYPES {n}")
        block(np.full((n, 1), ctype, np.int64), ">i4", "%d")
        for tag, data, count in (("POINT_DATA", point_data, len(xyz)),
                                 ("CELL_DATA", cell_data, n)):
            if not data:
                continue
            line(f"{tag} {count}")
            for name, arr in data:
                arr = np.asarray(arr, float).reshape(count, -1)
                if arr.shape[1] == 3:
                    line(f"VECTORS {name} double")
                else:
                    line(f"SCALARS {name} double {arr.shape[1]}")
                    line("LOOKUP_TABLE default")
                block(arr, ">f8", "%.17g")


def write_solution(path, xyz, tets, u=None, binary=True):
    """Tet mesh with the nodal displacement u ([3N], DOF 3*node + axis)."""
    pd = [] if u is None else [("displacement", np.asarray(u, float).reshape(-1, 3))]
    _write(path, xyz, tets, VTK_TETRA, point_data=pd, binary=binary, title="sfem displacement")


def write_face_fields(path, xyz, faces, strain, stress, binary=True):
    """One triangle per smoothing domain.  faces: [nf, >=3] with the face's
    nodes (a, b, c) in its first three columns (the face table of the
    library); strain, stress: [nf, 6] in the same order."""
    tri = np.asarray(faces)[:, :3]
    cd = [("strain", strain), ("stress", stress), ("von_mises", von_mises(stress)[:, None])]
    _write(path, xyz, tri, VTK_TRIANGLE, cell_data=cd, binary=binary,
           title="sfem smoothed strain and stress per face")


def read_legacy(path):
    """Arrays of a file written by this module: dict with 'points',
    'cells', 'cell_types', and 'point_data' / 'cell_data' name -> array."""
    raw = open(path, "rb").read()
    pos = 0

    def next_line():
        nonlocal pos
        end = raw.index(b"\n", pos)
        s = raw[pos:end].decode("ascii").strip()
        pos = end + 1
        return s

    next_line()
    next_line()
    binary = next_line() == "BINARY"
    assert next_line() == "DATASET UNSTRUCTURED_GRID"

    def read(count, dtype):
        nonlocal pos
        if binary:
            nb = count * np.dtype(dtype).itemsize
            a = np.frombuffer(raw[pos:pos + nb], dtype=dtype).copy()
            pos += nb + 1
            return a
        vals = []
        while len(vals) < count:
            vals.extend(next_line().split())
        return np.array(vals, dtype=np.dtype(dtype).newbyteorder("="))

    out = {"point_data": {}, "cell_data": {}}
    _, npts, _ = next_line().split()
    out["points"] = read(3 * int(npts), ">f8").astype(float).reshape(-1, 3)
    _, nc, size = next_line().split()
    c = read(int(size), ">i4").astype(np.int64).reshape(int(nc), -1)
    out["cells"] = c[:, 1:]
    next_line()
    out["cell_types"] = read(int(nc), ">i4").astype(np.int64)
    section = None
    count = 0
    while pos < len(raw):
        s = next_line()
        if not s:
            continue
        w = s.split()
        if w[0] in ("POINT_DATA", "CELL_DATA"):
            section = "point_data" if w[0] == "POINT_DATA" else "cell_data"
            count = int(w[1])
            continue
        if w[0] == "VECTORS":
            out[section][w[1]] = read(3 * count, ">f8").astype(float).reshape(count, 3)
        elif w[0] == "SCALARS":
            ncomp = int(w[3]) if len(w) > 3 else 1
            next_line()  # LOOKUP_TABLE
            out[section][w[1]] = read(ncomp * count, ">f8").astype(float).reshape(count, ncomp)
    return out
