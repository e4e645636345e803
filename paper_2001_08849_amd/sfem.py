"""Python binding of libsfem.so (include/sfem.h): argument marshalling only.

Every computation runs in the library's HIP kernels.  This module converts
numpy arrays (host) and torch tensors (device memory of the context's GPU)
into pointers and raises ``SfemError`` on a non-zero status.  If the library has not been built,
``lib()`` raises -- there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfem.so")

PTR_HOST, PTR_DEVICE = 0, 1
K_UNCONSTRAINED, K_WITH_BC, K_F32 = 0, 1, 2
ASM_F64, ASM_F32_COPY, ASM_F32_ARITH = 0, 1, 2
PRECOND_JACOBI, PRECOND_LEARNED = 0, 1
MODE_F64, MODE_F32_IR, MODE_F32_RR, MODE_F32_TF = 0, 1, 2, 3
NUM_SCHEDULES = 18
DOMAIN_FACE, DOMAIN_EDGE = 0, 1

STATUS = {0: "SFEM_OK", -1: "SFEM_EINVAL", -2: "SFEM_EMESH", -3: "SFEM_ENOMEM",
          -4: "SFEM_EHIP", -5: "SFEM_ENOCONV", -6: "SFEM_ESTATE"}

EXPORTS = [
    "sfem_create", "sfem_destroy", "sfem_last_error", "sfem_set_stream", "sfem_set_graph_replay",
    "sfem_set_mesh",
    "sfem_set_material", "sfem_set_material_per_tet", "sfem_set_dirichlet",
    "sfem_set_bc_penalty", "sfem_set_nodal_load", "sfem_add_traction", "sfem_assemble",
    "sfem_get_sizes", "sfem_get_faces", "sfem_get_csr", "sfem_get_rhs", "sfem_spmv",
    "sfem_solve", "sfem_get_timings", "sfem_timer_start", "sfem_timer_stop",
    "sfem_synchronize", "sfem_set_schedule", "sfem_get_schedule", "sfem_autotune",
    "sfem_gnn_num_params", "sfem_gnn_create", "sfem_gnn_destroy", "sfem_gnn_last_error",
    "sfem_gnn_get_params", "sfem_gnn_set_params", "sfem_gnn_set_pairs",
    "sfem_gnn_generate_pairs", "sfem_gnn_loss_grad", "sfem_gnn_train", "sfem_gnn_apply",
    "sfem_get_precond", "sfem_precond_apply", "sfem_get_precond_info", "sfem_face_stress",
    "sfem_set_precond_kernel", "sfem_get_precond_kernel",
    "sfem_batch_create", "sfem_batch_destroy", "sfem_batch_last_error", "sfem_batch_add_mesh",
    "sfem_batch_add_traction", "sfem_batch_build", "sfem_batch_sizes", "sfem_batch_autotune",
    "sfem_batch_get_schedule", "sfem_batch_solve", "sfem_batch_get_solution",
    "sfem_batch_get_system_info", "sfem_tetgen_read", "sfem_tetgen_last_error",
    "sfem_tetgen_sizes", "sfem_tetgen_get", "sfem_tetgen_free", "sfem_rcm_permutation",
    "sfem_permute_mesh", "sfem_set_smoothing_domain", "sfem_batch_set_schedule",
    "sfem_precond_save", "sfem_precond_load", "sfem_precond_apply_noalloc",
]


class SfemError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class SolveOpts(C.Structure):
    _fields_ = [("precond", C.c_int), ("mode", C.c_int), ("rtol", C.c_double),
                ("max_iter", C.c_int), ("check_every", C.c_int), ("inner_rtol", C.c_double),
                ("max_outer", C.c_int), ("profile", C.c_int), ("f32_until", C.c_double),
                ("f32_from", C.c_double)]


class BatchOpts(C.Structure):
    _fields_ = [("mode", C.c_int), ("rtol", C.c_double), ("max_iter", C.c_int),
                ("check_every", C.c_int), ("use_graph", C.c_int)]


class BatchInfo(C.Structure):
    _fields_ = [("ms_solve", C.c_double), ("periods", C.c_int), ("all_converged", C.c_int),
                ("max_iters", C.c_int), ("worst_relres", C.c_double),
                ("fp64_from_period", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SolveInfo(C.Structure):
    _fields_ = [("iters", C.c_int), ("outer_steps", C.c_int), ("fell_back", C.c_int),
                ("converged", C.c_int), ("true_relres", C.c_double), ("ms_solve", C.c_double),
                ("ms_spmv_avg", C.c_double), ("n_spmv", C.c_int),
                ("ms_mapply_avg", C.c_double), ("n_mapply", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_LIB = None


def lib() -> C.CDLL:
    """Load libsfem.so (once).  Raises if it is missing."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run paper_2001_08849_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int, C.c_double
        sig = {
            "sfem_create": (i32, [C.POINTER(vp), i32, vp]),
            "sfem_destroy": (None, [vp]),
            "sfem_last_error": (C.c_char_p, [vp]),
            "sfem_set_stream": (i32, [vp, vp]),
            "sfem_set_graph_replay": (i32, [vp, i32]),
            "sfem_set_mesh": (i32, [vp, i64, vp, i64, vp, i32]),
            "sfem_set_material": (i32, [vp, dbl, dbl]),
            "sfem_set_material_per_tet": (i32, [vp, vp, vp, i32]),
            "sfem_set_dirichlet": (i32, [vp, i64, vp, vp, i32]),
            "sfem_set_bc_penalty": (i32, [vp, dbl]),
            "sfem_set_nodal_load": (i32, [vp, vp, i32]),
            "sfem_add_traction": (i32, [vp, i64, vp, C.POINTER(dbl), i32]),
            "sfem_assemble": (i32, [vp, i32]),
            "sfem_get_sizes": (i32, [vp] + [C.POINTER(i64)] * 5),
            "sfem_get_faces": (i32, [vp, vp, i32]),
            "sfem_get_csr": (i32, [vp, vp, vp, vp, i32, i32]),
            "sfem_get_rhs": (i32, [vp, vp, i32]),
            "sfem_spmv": (i32, [vp, vp, vp, i32]),
            "sfem_solve": (i32, [vp, C.POINTER(SolveOpts), vp, i32, C.POINTER(SolveInfo)]),
            "sfem_get_timings": (i32, [vp, C.POINTER(dbl), C.POINTER(dbl)]),
            "sfem_timer_start": (i32, [vp]),
            "sfem_timer_stop": (i32, [vp, C.POINTER(dbl)]),
            "sfem_synchronize": (i32, [vp]),
            "sfem_set_schedule": (i32, [vp, i32, i32, i32]),
            "sfem_get_schedule": (i32, [vp, i32, C.POINTER(i32), C.POINTER(i32)]),
            "sfem_autotune": (i32, [vp, i32, C.POINTER(dbl), C.POINTER(dbl)]),
            "sfem_gnn_num_params": (i64, []),
            "sfem_gnn_create": (i32, [C.POINTER(vp), i32, C.c_uint64]),
            "sfem_gnn_destroy": (None, [vp]),
            "sfem_gnn_last_error": (C.c_char_p, [vp]),
            "sfem_gnn_get_params": (i32, [vp, vp, i64]),
            "sfem_gnn_set_params": (i32, [vp, vp, i64]),
            "sfem_precond_save": (i32, [vp, C.c_char_p]),
            "sfem_precond_load": (i32, [vp, C.c_char_p]),
            "sfem_gnn_set_pairs": (i32, [vp, i64, vp, vp, i32]),
            "sfem_gnn_generate_pairs": (i32, [vp, i32, i32, C.c_uint64, C.POINTER(i64)]),
            "sfem_gnn_loss_grad": (i32, [vp, vp, vp, i32, C.POINTER(dbl), vp]),
            "sfem_gnn_train": (i32, [vp, C.POINTER(vp), i32, i32, i32, dbl, C.c_uint64, vp]),
            "sfem_gnn_apply": (i32, [vp, vp, C.POINTER(dbl)]),
            "sfem_get_precond": (i32, [vp, vp, vp, i32]),
            "sfem_precond_apply": (i32, [vp, vp, vp, i32]),
            "sfem_precond_apply_noalloc": (i32, [vp, vp, vp]),
            "sfem_get_precond_info": (i32, [vp] + [C.POINTER(dbl)] * 3),
            "sfem_set_precond_kernel": (i32, [vp, i32]),
            "sfem_get_precond_kernel": (i32, [vp, C.POINTER(i32), C.POINTER(dbl),
                                              C.POINTER(dbl), C.POINTER(dbl)]),
            "sfem_face_stress": (i32, [vp, vp, vp, vp, i32, C.POINTER(dbl)]),
            "sfem_batch_create": (i32, [C.POINTER(vp), i32]),
            "sfem_batch_destroy": (None, [vp]),
            "sfem_batch_last_error": (C.c_char_p, [vp]),
            "sfem_batch_add_mesh": (i32, [vp, i64, vp, i64, vp, dbl, dbl, i64, vp,
                                          C.POINTER(i32)]),
            "sfem_batch_add_traction": (i32, [vp, i32, i32, i64, vp, C.POINTER(dbl)]),
            "sfem_batch_build": (i32, [vp, i32]),
            "sfem_batch_sizes": (i32, [vp, C.POINTER(i32)] + [C.POINTER(i64)] * 4),
            "sfem_batch_autotune": (i32, [vp, i32, i32, i32, C.POINTER(dbl)]),
            "sfem_batch_get_schedule": (i32, [vp, i32] + [C.POINTER(i32)] * 5),
            "sfem_batch_set_schedule": (i32, [vp, i32, i32, i32, i32]),
            "sfem_batch_solve": (i32, [vp, C.POINTER(BatchOpts), C.POINTER(BatchInfo)]),
            "sfem_batch_get_solution": (i32, [vp, i32, i32, vp, i32]),
            "sfem_batch_get_system_info": (i32, [vp, vp, vp, vp, vp]),
            "sfem_tetgen_read": (i32, [C.POINTER(vp), C.c_char_p]),
            "sfem_tetgen_last_error": (C.c_char_p, [vp]),
            "sfem_tetgen_sizes": (i32, [vp] + [C.POINTER(i64)] * 3 + [C.POINTER(i32)] * 2),
            "sfem_tetgen_get": (i32, [vp, vp, vp, vp, vp]),
            "sfem_tetgen_free": (None, [vp]),
            "sfem_rcm_permutation": (i32, [vp, i64, i64, vp, i32, vp, i32, C.POINTER(dbl)]),
            "sfem_permute_mesh": (i32, [vp, i64, i64, vp, vp, vp, vp, vp, i32]),
            "sfem_set_smoothing_domain": (i32, [vp, i32]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _arg(a, dtype):
    """(pointer, ptr_kind, keepalive) for a numpy array or a torch tensor."""
    if a is None:
        return None, PTR_HOST, None
    if _is_torch(a):
        import torch
        want = {np.float64: torch.float64, np.int32: torch.int32,
                np.float32: torch.float32}[dtype]
        if a.dtype != want:
            raise TypeError(f"expected {want}, got {a.dtype}")
        if not a.is_contiguous():
            raise ValueError("tensor must be contiguous")
        return C.c_void_p(a.data_ptr()), (PTR_DEVICE if a.is_cuda else PTR_HOST), a
    arr = np.ascontiguousarray(a, dtype=dtype)
    return arr.ctypes.data_as(C.c_void_p), PTR_HOST, arr


@dataclass
class Sizes:
    n_faces: int
    n_exterior: int
    n_rows: int
    nnz: int
    n_blocks: int


class Context:
    """One sfem_ctx on `device`.  `stream` is a hipStream_t handle (an int,
    e.g. ``torch.cuda.current_stream().cuda_stream``); by default the library
    creates and owns a stream.

    This module never imports torch itself: a process must hold a single
    HIP runtime, and torch wheels bundle their own.  Processes that use torch
    tensors with this library import torch first, and the library then runs
    on torch's runtime."""

    def __init__(self, device: int = 0, stream: int = 0):
        L = lib()
        h = C.c_void_p()
        st = L.sfem_create(C.byref(h), device, C.c_void_p(stream) if stream else None)
        if st != 0:
            raise SfemError(st, "sfem_create failed")
        self._h = h
        self._L = L

    def close(self):
        if getattr(self, "_h", None):
            self._L.sfem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st):
        if st != 0:
            raise SfemError(st, self._L.sfem_last_error(self._h).decode())
        return st

    # ------------------------------------------------------------ inputs
    def set_graph_replay(self, enabled: bool):
        """Replay full PCG check periods as a captured hipGraph (default) or
        launch every kernel one by one (same results)."""
        self._check(self._L.sfem_set_graph_replay(self._h, int(bool(enabled))))

    def set_stream(self, stream_handle: int):
        self._check(self._L.sfem_set_stream(self._h, C.c_void_p(stream_handle)))

    def set_mesh(self, xyz, tets):
        px, kx, a1 = _arg(xyz, np.float64)
        pt, kt, a2 = _arg(tets, np.int32)
        if kx != kt:
            raise ValueError("xyz and tets must both be host or both be device arrays")
        n, t = int(xyz.shape[0]), int(tets.shape[0])
        self._check(self._L.sfem_set_mesh(self._h, n, px, t, pt, kx))

    def set_material(self, E, nu):
        if np.ndim(E) == 0 and np.ndim(nu) == 0:
            self._check(self._L.sfem_set_material(self._h, float(E), float(nu)))
        else:
            pe, ke, a1 = _arg(E, np.float64)
            pn, kn, a2 = _arg(nu, np.float64)
            self._check(self._L.sfem_set_material_per_tet(self._h, pe, pn, ke))

    def set_dirichlet(self, dofs, values=None):
        pd, kd, a1 = _arg(dofs, np.int32)
        pv, kv, a2 = _arg(values, np.float64)
        self._check(self._L.sfem_set_dirichlet(self._h, int(len(dofs)), pd, pv, kd))

    def set_bc_penalty(self, alpha: float):
        self._check(self._L.sfem_set_bc_penalty(self._h, float(alpha)))

    def set_nodal_load(self, f):
        pf, kf, a = _arg(f, np.float64)
        self._check(self._L.sfem_set_nodal_load(self._h, pf, kf))

    def add_traction(self, tris, t):
        pt, kt, a = _arg(tris, np.int32)
        tv = (C.c_double * 3)(*[float(v) for v in t])
        self._check(self._L.sfem_add_traction(self._h, int(len(tris)), pt, tv, kt))

    # ------------------------------------------------------------ compute
    def assemble(self, f32_copy: bool = False, f32_arith: bool = False):
        """f32_copy: keep an FP32 copy (the FP64 values rounded); f32_arith:
        an FP32 copy from FP32 face arithmetic (a second pass)."""
        flags = ASM_F32_ARITH if f32_arith else (ASM_F32_COPY if f32_copy else ASM_F64)
        self._check(self._L.sfem_assemble(self._h, flags))

    def sizes(self) -> Sizes:
        v = [C.c_int64() for _ in range(5)]
        self._check(self._L.sfem_get_sizes(self._h, *[C.byref(x) for x in v]))
        return Sizes(*[int(x.value) for x in v])

    def faces(self) -> np.ndarray:
        s = self.sizes()
        out = np.empty((s.n_faces, 7), dtype=np.int32)
        self._check(self._L.sfem_get_faces(self._h, out.ctypes.data_as(C.c_void_p), PTR_HOST))
        return out

    def csr(self, which: int = K_WITH_BC, values: bool = True):
        s = self.sizes()
        rp = np.empty(s.n_rows + 1, dtype=np.int32)
        ci = np.empty(s.nnz, dtype=np.int32)
        va = np.empty(s.nnz, dtype=np.float64) if values else None
        self._check(self._L.sfem_get_csr(
            self._h, rp.ctypes.data_as(C.c_void_p), ci.ctypes.data_as(C.c_void_p),
            va.ctypes.data_as(C.c_void_p) if values else None, which, PTR_HOST))
        return rp, ci, va

    def csr_values_into(self, out, which: int = K_WITH_BC):
        """Copy the CSR values into a device tensor (float64, nnz)."""
        p, k, a = _arg(out, np.float64)
        self._check(self._L.sfem_get_csr(self._h, None, None, p, which, k))

    def rhs(self) -> np.ndarray:
        out = np.empty(self.sizes().n_rows, dtype=np.float64)
        self._check(self._L.sfem_get_rhs(self._h, out.ctypes.data_as(C.c_void_p), PTR_HOST))
        return out

    def spmv(self, x, y=None):
        if y is None:
            y = np.empty_like(np.asarray(x, dtype=np.float64)) if not _is_torch(x) else x.clone()
        px, kx, a1 = _arg(x, np.float64)
        py, ky, a2 = _arg(y, np.float64)
        if kx != ky:
            raise ValueError("x and y must live on the same side")
        self._check(self._L.sfem_spmv(self._h, px, py, kx))
        return y

    def solve(self, rtol: float = 1e-8, mode: int = MODE_F64, precond: int = PRECOND_JACOBI,
              max_iter: int = 0, check_every: int = 0, inner_rtol: float = 0.0,
              max_outer: int = 0, out=None, raise_on_noconv: bool = False,
              profile: bool = False, f32_until: float = 0.0, f32_from: float = 0.0):
        opts = SolveOpts(precond, mode, rtol, max_iter, check_every, inner_rtol, max_outer,
                         int(profile), f32_until, f32_from)
        info = SolveInfo()
        if out is None:
            out = np.empty(self.sizes().n_rows, dtype=np.float64)
        pu, ku, a = _arg(out, np.float64)
        st = self._L.sfem_solve(self._h, C.byref(opts), pu, ku, C.byref(info))
        if st != 0 and (st != -5 or raise_on_noconv):
            self._check(st)
        return out, info.as_dict()

    def face_stress(self, u):
        """(strain, stress) float64 [n_faces][6] of every smoothing domain and
        the kernel's device ms."""
        nf = self.sizes().n_faces
        eps = np.empty((nf, 6), dtype=np.float64)
        sig = np.empty((nf, 6), dtype=np.float64)
        pu, ku, a = _arg(u, np.float64)
        if ku != PTR_HOST:
            raise ValueError("face_stress takes a host u")
        ms = C.c_double()
        self._check(self._L.sfem_face_stress(self._h, pu, eps.ctypes.data_as(C.c_void_p),
                                             sig.ctypes.data_as(C.c_void_p), PTR_HOST,
                                             C.byref(ms)))
        return eps, sig, ms.value

    def set_smoothing_domain(self, domain: int):
        """DOMAIN_FACE (the paper's FS-FEM, default) or DOMAIN_EDGE (ES-FEM)."""
        self._check(self._L.sfem_set_smoothing_domain(self._h, int(domain)))

    def rcm_permutation(self, n_nodes: int, tets):
        """(perm, device ms): reverse Cuthill-McKee numbering of a mesh's nodes,
        perm[new] = old.  tets: int32 [n_tets, 4], host array or device
        tensor (then perm is returned on the host all the same)."""
        pt, kt, a = _arg(tets, np.int32)
        n_tets = (a.numel() if _is_torch(a) else a.size) // 4
        perm = np.empty(int(n_nodes), np.int32)
        ms = C.c_double()
        self._check(self._L.sfem_rcm_permutation(self._h, int(n_nodes), int(n_tets), pt, kt,
                                                 perm.ctypes.data_as(C.c_void_p), PTR_HOST,
                                                 C.byref(ms)))
        return perm, ms.value

    def permute_mesh(self, perm, xyz, tets):
        """Renumbered (xyz, tets) for perm[new] = old (host arrays)."""
        pp, _, p_ = _arg(perm, np.int32)
        px, _, x_ = _arg(xyz, np.float64)
        pt, _, t_ = _arg(tets, np.int32)
        xo = np.empty_like(x_).reshape(-1, 3)
        to = np.empty_like(t_).reshape(-1, 4)
        self._check(self._L.sfem_permute_mesh(self._h, p_.size, t_.size // 4, pp, px, pt,
                                              xo.ctypes.data_as(C.c_void_p),
                                              to.ctypes.data_as(C.c_void_p), PTR_HOST))
        return xo, to

    def timer_start(self):
        self._check(self._L.sfem_timer_start(self._h))

    def timer_stop(self) -> float:
        ms = C.c_double()
        self._check(self._L.sfem_timer_stop(self._h, C.byref(ms)))
        return ms.value

    def set_schedule(self, variant: int, grid_cap: int = 4096, f32: bool = False):
        self._check(self._L.sfem_set_schedule(self._h, ASM_F32_COPY if f32 else ASM_F64,
                                              int(variant), int(grid_cap)))

    def schedule(self, f32: bool = False):
        v, g = C.c_int(), C.c_int()
        self._check(self._L.sfem_get_schedule(self._h, ASM_F32_COPY if f32 else ASM_F64,
                                              C.byref(v), C.byref(g)))
        return v.value, g.value

    def autotune(self, reps: int = 10):
        a, b = C.c_double(), C.c_double()
        self._check(self._L.sfem_autotune(self._h, int(reps), C.byref(a), C.byref(b)))
        return {"f64": (self.schedule(False), a.value), "f32": (self.schedule(True), b.value)}

    def synchronize(self):
        self._check(self._L.sfem_synchronize(self._h))

    def timings(self):
        a, b = C.c_double(), C.c_double()
        self._check(self._L.sfem_get_timings(self._h, C.byref(a), C.byref(b)))
        return {"ms_topology": a.value, "ms_assemble": b.value}


    # ------------------------------------------------ learned preconditioner
    def set_pairs(self, r, e):
        """Training pairs: r, e float32 [n_pairs][3N] (r = K e)."""
        pr, kr, a1 = _arg(r, np.float32)
        pe, ke, a2 = _arg(e, np.float32)
        n_pairs = (r.shape[0] if getattr(r, "ndim", 1) == 2 else 1)
        if kr != ke:
            raise ValueError("r and e must live on the same side")
        self._check(self._L.sfem_gnn_set_pairs(self._h, int(n_pairs), pr, pe, kr))

    def generate_pairs(self, n_rhs: int, snaps_per_rhs: int, seed: int = 0) -> int:
        k = C.c_int64()
        self._check(self._L.sfem_gnn_generate_pairs(self._h, int(n_rhs), int(snaps_per_rhs),
                                                    int(seed), C.byref(k)))
        return k.value

    def precond(self):
        """(S' float32 [nnz] in CSR value order, d^-1/2 float64 [3N])."""
        sz = self.sizes()
        S = np.empty(sz.nnz, dtype=np.float32)
        s = np.empty(sz.n_rows, dtype=np.float64)
        self._check(self._L.sfem_get_precond(self._h, S.ctypes.data_as(C.c_void_p),
                                             s.ctypes.data_as(C.c_void_p), PTR_HOST))
        return S, s

    def precond_info(self):
        """{'theta', 'lambda_min', 'lambda_max'} of the last Gnn.apply."""
        t, a, b = C.c_double(), C.c_double(), C.c_double()
        self._check(self._L.sfem_get_precond_info(self._h, C.byref(t), C.byref(a), C.byref(b)))
        return {"theta": t.value, "lambda_min": a.value, "lambda_max": b.value}

    def set_precond_kernel(self, variant: int):
        """M apply kernel: 0 rows, 1 rh staged in LDS, 2 grouped layout, -1 time
        each and keep the fastest."""
        self._check(self._L.sfem_set_precond_kernel(self._h, int(variant)))

    def precond_kernel(self):
        """{'variant', 'us_rows', 'us_lds', 'us_grouped'}: the M apply kernel in use
        and the timings (0: not timed)."""
        v, a, b, g = C.c_int(), C.c_double(), C.c_double(), C.c_double()
        self._check(self._L.sfem_get_precond_kernel(self._h, C.byref(v), C.byref(a), C.byref(b),
                                                    C.byref(g)))
        return {"variant": v.value, "us_rows": a.value, "us_lds": b.value, "us_grouped": g.value}

    def precond_apply(self, r):
        z = np.empty(self.sizes().n_rows, dtype=np.float64)
        pr, kr, a = _arg(r, np.float64)
        self._check(self._L.sfem_precond_apply(self._h, pr, z.ctypes.data_as(C.c_void_p), kr))
        return z

    def precond_apply_noalloc(self, r_dev: int, z_dev: int):
        """z = M r between two device buffers (raw addresses) without any
        allocation by the library; enqueued on the context stream only."""
        self._check(self._L.sfem_precond_apply_noalloc(self._h, C.c_void_p(r_dev),
                                                       C.c_void_p(z_dev)))


class Gnn:
    """The learned preconditioner's network (sfem_gnn) on `device`."""

    def __init__(self, device: int = 0, seed: int = 0):
        L = lib()
        h = C.c_void_p()
        st = L.sfem_gnn_create(C.byref(h), device, int(seed))
        if st != 0:
            raise SfemError(st, "sfem_gnn_create failed")
        self._h = h
        self._L = L
        self.n_params = int(L.sfem_gnn_num_params())

    def close(self):
        if getattr(self, "_h", None):
            self._L.sfem_gnn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, ctx: Context | None = None):
        if st != 0:
            msg = (ctx._L.sfem_last_error(ctx._h) if ctx is not None
                   else self._L.sfem_gnn_last_error(self._h)).decode()
            raise SfemError(st, msg)

    def params(self) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        self._check(self._L.sfem_gnn_get_params(self._h, out.ctypes.data_as(C.c_void_p),
                                                self.n_params))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        self._check(self._L.sfem_gnn_set_params(self._h, p.ctypes.data_as(C.c_void_p), p.size))

    def save(self, path):
        """Writes the weights file (sfem_precond_save)."""
        self._check(self._L.sfem_precond_save(self._h, os.fsencode(path)))

    def load(self, path):
        """Reads a weights file into the network (sfem_precond_load)."""
        self._check(self._L.sfem_precond_load(self._h, os.fsencode(path)))

    def loss_grad(self, ctx: Context, ids, grad: bool = True):
        ids = np.ascontiguousarray(ids, dtype=np.int32)
        L = C.c_double()
        g = np.empty(self.n_params, dtype=np.float32) if grad else None
        st = self._L.sfem_gnn_loss_grad(self._h, ctx._h, ids.ctypes.data_as(C.c_void_p),
                                        int(ids.size), C.byref(L),
                                        g.ctypes.data_as(C.c_void_p) if grad else None)
        self._check(st, ctx)
        return (L.value, g) if grad else L.value

    def train(self, ctxs, steps: int, batch: int = 32, lr: float = 1e-3, seed: int = 0):
        arr = (C.c_void_p * len(ctxs))(*[c._h for c in ctxs])
        losses = np.empty(max(steps, 1), dtype=np.float32)
        st = self._L.sfem_gnn_train(self._h, arr, len(ctxs), int(steps), int(batch), float(lr),
                                    int(seed), losses.ctypes.data_as(C.c_void_p))
        self._check(st, ctxs[0])
        return losses[:steps]

    def apply(self, ctx: Context) -> float:
        ms = C.c_double()
        self._check(self._L.sfem_gnn_apply(self._h, ctx._h, C.byref(ms)), ctx)
        return ms.value


class Batch:
    """Many meshes x up to 4 load cases solved together (sfem_batch)."""

    def __init__(self, device: int = 0):
        L = lib()
        h = C.c_void_p()
        st = L.sfem_batch_create(C.byref(h), device)
        if st != 0:
            raise SfemError(st, "sfem_batch_create failed")
        self._h, self._L = h, L
        self.n_meshes = 0

    def close(self):
        if getattr(self, "_h", None):
            self._L.sfem_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st):
        if st != 0:
            raise SfemError(st, self._L.sfem_batch_last_error(self._h).decode())
        return st

    def add_mesh(self, xyz, tets, E, nu, fixed_dofs) -> int:
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tets = np.ascontiguousarray(tets, dtype=np.int32)
        fx = np.ascontiguousarray(fixed_dofs, dtype=np.int32)
        idx = C.c_int()
        self._check(self._L.sfem_batch_add_mesh(
            self._h, xyz.shape[0], xyz.ctypes.data_as(C.c_void_p), tets.shape[0],
            tets.ctypes.data_as(C.c_void_p), float(E), float(nu), fx.size,
            fx.ctypes.data_as(C.c_void_p), C.byref(idx)))
        self.n_meshes += 1
        return idx.value

    def add_traction(self, mesh: int, rhs: int, tris, t):
        tris = np.ascontiguousarray(tris, dtype=np.int32)
        tv = (C.c_double * 3)(*[float(v) for v in np.asarray(t).reshape(-1)[:3]])
        self._check(self._L.sfem_batch_add_traction(self._h, int(mesh), int(rhs), tris.shape[0],
                                                    tris.ctypes.data_as(C.c_void_p), tv))

    def build(self, f32_copy: bool = False):
        self._check(self._L.sfem_batch_build(self._h, ASM_F32_COPY if f32_copy else ASM_F64))

    def sizes(self):
        m = C.c_int()
        a, b, c, d = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        self._check(self._L.sfem_batch_sizes(self._h, C.byref(m), C.byref(a), C.byref(b),
                                             C.byref(c), C.byref(d)))
        return {"meshes": m.value, "nodes": a.value, "tets": b.value, "faces": c.value,
                "nnz": d.value}

    def autotune(self, reps: int = 5, use_cache: bool = True, f32: bool = False) -> float:
        us = C.c_double()
        self._check(self._L.sfem_batch_autotune(self._h, int(reps), int(use_cache),
                                                ASM_F32_COPY if f32 else ASM_F64, C.byref(us)))
        return us.value

    def set_schedule(self, bucket: int, lanes_per_row: int, rows_per_wg: int, packed: bool):
        self._check(self._L.sfem_batch_set_schedule(self._h, int(bucket), int(lanes_per_row),
                                                    int(rows_per_wg), int(bool(packed))))

    def schedule(self, bucket: int):
        v = [C.c_int() for _ in range(5)]
        self._check(self._L.sfem_batch_get_schedule(self._h, int(bucket), *[C.byref(x) for x in v]))
        return {"lanes_per_row": v[0].value, "rows_per_wg": v[1].value, "meshes": v[2].value,
                "from_cache": v[3].value, "packed": v[4].value}

    def solve(self, rtol: float = 1e-8, mode: int = MODE_F64, max_iter: int = 0,
              check_every: int = 0, use_graph: bool = True, raise_on_noconv: bool = False):
        o = BatchOpts(mode, rtol, max_iter, check_every, int(use_graph))
        info = BatchInfo()
        st = self._L.sfem_batch_solve(self._h, C.byref(o), C.byref(info))
        if st != 0 and (st != -5 or raise_on_noconv):
            self._check(st)
        return info.as_dict()

    def solution(self, mesh: int, rhs: int, n_nodes: int) -> np.ndarray:
        out = np.empty(3 * n_nodes, dtype=np.float64)
        self._check(self._L.sfem_batch_get_solution(self._h, int(mesh), int(rhs),
                                                    out.ctypes.data_as(C.c_void_p), PTR_HOST))
        return out

    def system_info(self):
        n = 4 * self.n_meshes
        it, cv, bk = (np.empty(n, np.int32) for _ in range(3))
        rr = np.empty(n, np.float64)
        self._check(self._L.sfem_batch_get_system_info(
            self._h, it.ctypes.data_as(C.c_void_p), cv.ctypes.data_as(C.c_void_p),
            rr.ctypes.data_as(C.c_void_p), bk.ctypes.data_as(C.c_void_p)))
        return {"iters": it, "converged": cv, "relres": rr, "breakdown": bk}


def read_tetgen(stem: str):
    """(xyz [N,3], tets [T,4], faces [F,3] or None, markers [F] or None),
    0-based, from TetGen's <stem>.node / .ele / .face (parsed by the
    library on the host)."""
    L = lib()
    h = C.c_void_p()
    st = L.sfem_tetgen_read(C.byref(h), str(stem).encode())
    try:
        if st != 0:
            raise SfemError(st, (L.sfem_tetgen_last_error(h) or b"").decode())
        n, t, f = C.c_int64(), C.c_int64(), C.c_int64()
        hm, base = C.c_int(), C.c_int()
        st = L.sfem_tetgen_sizes(h, C.byref(n), C.byref(t), C.byref(f), C.byref(hm),
                                 C.byref(base))
        if st != 0:
            raise SfemError(st, "sizes")
        xyz = np.empty((n.value, 3), np.float64)
        tets = np.empty((t.value, 4), np.int32)
        faces = np.empty((max(f.value, 0), 3), np.int32) if f.value >= 0 else None
        marks = np.empty(f.value, np.int32) if (f.value >= 0 and hm.value) else None
        ptr = lambda a: a.ctypes.data_as(C.c_void_p) if a is not None else None
        st = L.sfem_tetgen_get(h, ptr(xyz), ptr(tets), ptr(faces), ptr(marks))
        if st != 0:
            raise SfemError(st, "get")
        return xyz, tets, faces, marks
    finally:
        L.sfem_tetgen_free(h)


def batch_from_items(items, f32_copy: bool = False, device: int = 0) -> Batch:
    """A built Batch from meshgen.BatchItem's (clamp at x = 0, the four end
    tractions as load cases 0..3)."""
    b = Batch(device)
    for it in items:
        m = it.mesh
        idx = b.add_mesh(m.xyz, m.tets, it.E, it.nu, m.clamp_dofs())
        for k in range(it.tractions.shape[0]):
            b.add_traction(idx, k, m.end_tris, it.tractions[k])
    b.build(f32_copy=f32_copy)
    return b


def unpack_params(flat):
    """Splits the flat parameter vector into named arrays (the layout of
    sfem_gnn_get_params)."""
    flat = np.asarray(flat)
    H, out, o = 64, {}, 0

    def take(name, shape):
        nonlocal o
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n

    take("Wn", (H, 8)); take("bn", (H,)); take("We", (H, 12)); take("be", (H,))
    for l in range(4):
        take(f"W{l}", (H, 3 * H)); take(f"b{l}", (H,))
        take(f"U{l}", (H, 2 * H)); take(f"c{l}", (H,))
    take("Wo", (9, H))
    assert o == flat.size
    return out


def pack_params(P) -> np.ndarray:
    names = ["Wn", "bn", "We", "be"]
    for l in range(4):
        names += [f"W{l}", f"b{l}", f"U{l}", f"c{l}"]
    names.append("Wo")
    return np.concatenate([np.asarray(P[k], dtype=np.float32).ravel() for k in names])


def setup_problem(ctx: Context, problem, f32_copy: bool = False, load_tris=None):
    """Mesh + material + clamp + end traction of a meshgen Problem, then
    assemble.  Returns the context."""
    m = problem.mesh
    ctx.set_mesh(m.xyz, m.tets)
    ctx.set_material(problem.E, problem.nu)
    ctx.set_dirichlet(problem.fixed_dofs())
    tris = m.end_tris if load_tris is None else load_tris
    ctx.add_traction(tris, np.asarray(problem.traction, dtype=np.float64).reshape(-1)[:3])
    ctx.assemble(f32_copy=f32_copy)
    return ctx
