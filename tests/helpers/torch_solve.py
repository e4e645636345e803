"""Solves the 1.92M-tet-family cantilever (small size) from torch device
tensors on torch's current HIP stream and prints a JSON line comparing it
with the same solve from host arrays.  Run as a separate process by
tests/test_gpu_torch.py (torch must be imported before the library so that
one HIP runtime serves both)."""
import json
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from paper_2001_08849_amd import meshgen as mg  # noqa: E402
from paper_2001_08849_amd import sfem  # noqa: E402

p = mg.cantilever_scaled(30, 4, 4, jitter=0.15, seed=3)
m = p.mesh
dev = torch.device("cuda:0")
stream = torch.cuda.current_stream()
ctx = sfem.Context(0, stream=stream.cuda_stream)
ctx.set_mesh(torch.tensor(m.xyz, dtype=torch.float64, device=dev),
             torch.tensor(m.tets, dtype=torch.int32, device=dev))
ctx.set_material(p.E, p.nu)
ctx.set_dirichlet(torch.tensor(p.fixed_dofs(), dtype=torch.int32, device=dev))
ctx.add_traction(torch.tensor(m.end_tris, dtype=torch.int32, device=dev), list(p.traction))
ctx.assemble()
u_dev = torch.empty(3 * m.n_nodes, dtype=torch.float64, device=dev)
_, info = ctx.solve(rtol=1e-10, out=u_dev)
# torch work queued after the library's on the same stream sees its result
norm_dev = float(torch.linalg.vector_norm(u_dev).item())
y_dev = ctx.spmv(u_dev)                       # device in, device out
torch.cuda.synchronize()

host = sfem.Context(0)
sfem.setup_problem(host, p)
u_host, info_h = host.solve(rtol=1e-10)
print(json.dumps({
    "iters": info["iters"], "iters_host": info_h["iters"],
    "u_diff": float(np.abs(u_dev.cpu().numpy() - u_host).max() / np.abs(u_host).max()),
    "norm_dev": norm_dev, "norm_host": float(np.linalg.norm(u_host)),
    "spmv_diff": float(np.abs(y_dev.cpu().numpy() - host.spmv(u_host)).max()
                       / np.abs(host.spmv(u_host)).max()),
}))
