"""GPU tests of the learned preconditioner: forward and gradient parity with
the FP64 reference network, the solver integration (flexible PCG, Jacobi
limit, fallback), determinism, and what training gains.

Tolerances.  The dense layers take BF16 operands (unit roundoff u = 2^-9 ~
2e-3) with FP32 accumulation; everything else is FP32/FP64.  A forward pass
rounds every layer input once, so S' carries a few u of relative error
(1.8e-3 measured): the bound is 5u = 1e-2.  A gradient passes through about
twice as many rounded products plus FP32 loss panels (at most 1.6e-2
per tensor measured): the bound is 25u = 5e-2 per tensor and 1e-2 on the
whole vector, whose cosine with the reference must exceed 0.999.
"""
import numpy as np
import pytest

from oracle import fsfem as O
from oracle import gnn_ref as G
from paper_2001_08849_amd import meshgen as mg

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -9


@pytest.fixture(scope="module")
def S():
    from paper_2001_08849_amd import sfem
    return sfem


def ref_system(p):
    m = p.mesh
    K = O.assemble(m.xyz, m.tets, p.E, p.nu)
    f = O.traction_load(m.xyz, m.end_tris, p.traction)
    Kb, fb = O.apply_dirichlet(K, f, p.fixed_dofs())
    Kb = Kb.tocsr()
    Kb.sort_indices()
    return Kb, fb


def blocks_to_csr(g, Kb, Sp):
    """S' blocks [nb,3,3] -> values in the CSR order of Kb."""
    out = np.zeros(Kb.nnz)
    for k, (I, J) in enumerate(zip(g.row, g.bcol)):
        for a in range(3):
            lo, hi = Kb.indptr[3 * I + a], Kb.indptr[3 * I + a + 1]
            cols = Kb.indices[lo:hi]
            for c in range(3):
                out[lo + np.searchsorted(cols, 3 * J + c)] = Sp[k, a, c]
    return out


def random_params(seed, scale_out=0.3):
    P = G.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    P["Wo"] = rng.standard_normal(P["Wo"].shape) * scale_out
    for k in P:
        if k.startswith(("b", "c")):
            P[k] = rng.standard_normal(P[k].shape) * 0.1
    return P


@pytest.fixture(scope="module")
def small(S):
    p = mg.learned_small(1, grid=(8, 3, 3))
    ctx = S.Context(0)
    S.setup_problem(ctx, p)
    Kb, fb = ref_system(p)
    g = G.build_graph(Kb, p.mesh.xyz, p.fixed_dofs())
    return p, ctx, Kb, g


def fp32_params(S, P):
    """The reference parameters rounded to the network's FP32 master copy."""
    flat = S.pack_params(P)
    return flat, {k: v.astype(np.float64) for k, v in S.unpack_params(flat).items()}


@pytest.mark.parametrize("seed,scale_out", [(3, 0.3), (8, 3.0)])
def test_forward_parity(S, small, seed, scale_out):
    p, ctx, Kb, g = small
    rp, ci, _ = ctx.csr()
    assert np.array_equal(rp, Kb.indptr) and np.array_equal(ci, Kb.indices)
    flat, P64 = fp32_params(S, random_params(seed, scale_out))
    net = S.Gnn(0, seed=1)
    net.set_params(flat)
    net.apply(ctx)
    S_gpu, s_gpu = ctx.precond()
    info = ctx.precond_info()
    Sp_ref, _ = G.forward(P64, g)
    theta_ref, lmin_ref = G.spd_theta(g, Sp_ref)
    S_ref = blocks_to_csr(g, Kb, Sp_ref)
    raw = S_gpu.astype(np.float64) / info["theta"]
    rel = np.linalg.norm(raw - S_ref) / np.linalg.norm(S_ref)
    print(f"S relative Frobenius error {rel:.3e}; lambda_min {info['lambda_min']:.5f} "
          f"(exact {lmin_ref:.5f}), theta {info['theta']:.5f} (exact {theta_ref:.5f})")
    assert rel < 5 * U_BF16
    assert np.abs(raw - S_ref).max() <= 10 * U_BF16 * np.abs(S_ref).max()
    # the Lanczos estimate of lambda_min(S) and theta follow the exact ones
    assert info["lambda_min"] == pytest.approx(lmin_ref, rel=10 * U_BF16)
    assert info["theta"] == pytest.approx(theta_ref, rel=10 * U_BF16)
    if scale_out > 1:
        assert info["theta"] < 1.0
    # s = diag(K)^-1/2 from the GPU's K, whose entries match the oracle to the
    # assembly's row-relative bar (1e-12; diag(K) is its row's largest entry)
    np.testing.assert_allclose(s_gpu, 1.0 / np.sqrt(Kb.diagonal()), rtol=1e-12)
    # fixed DOFs: rows and columns of S' are exactly zero
    fixed = np.zeros(Kb.shape[0], bool)
    fixed[p.fixed_dofs()] = True
    rows = np.repeat(np.arange(Kb.shape[0]), np.diff(Kb.indptr))
    assert np.all(S_gpu[fixed[rows] | fixed[Kb.indices]] == 0.0)
    # z = M r against the reference M
    r = np.random.default_rng(0).standard_normal(Kb.shape[0])
    z = ctx.precond_apply(r)
    zr = G.apply_M(g, theta_ref * Sp_ref, r)
    assert np.linalg.norm(z - zr) / np.linalg.norm(zr) < 5 * U_BF16


def test_untrained_network_is_jacobi(S, small):
    p, ctx, Kb, g = small
    net = S.Gnn(0, seed=11)
    net.apply(ctx)
    S_gpu, _ = ctx.precond()
    assert np.all(S_gpu == 0.0)
    r = np.random.default_rng(1).standard_normal(Kb.shape[0])
    # D^-1 of the GPU's K: its diagonal matches the oracle to the assembly's
    # row-relative bar (1e-12)
    np.testing.assert_allclose(ctx.precond_apply(r), r / Kb.diagonal(), rtol=1e-12)
    # flexible PCG with M = D^-1 is Jacobi PCG; both reach the oracle's u
    uj, ij = ctx.solve(rtol=1e-8)
    ul, il = ctx.solve(rtol=1e-8, precond=S.PRECOND_LEARNED)
    assert ij["converged"] and il["converged"] and not il["fell_back"]
    assert abs(il["iters"] - ij["iters"]) <= max(2, 0.02 * ij["iters"])
    ud = O.solve_dense(Kb, O.apply_dirichlet(O.assemble(p.mesh.xyz, p.mesh.tets, p.E, p.nu),
                                             O.traction_load(p.mesh.xyz, p.mesh.end_tris,
                                                             p.traction), p.fixed_dofs())[1])
    el = np.linalg.norm(ul - ud) / np.linalg.norm(ud)
    print(f"untrained network: learned u vs oracle {el:.2e}")
    assert el <= 1e-8


def test_gradient_parity(S, small):
    p, ctx, Kb, g = small
    flat, P64 = fp32_params(S, random_params(4))
    rng = np.random.default_rng(7)
    n = Kb.shape[0]
    E = rng.standard_normal((n, 8))
    E[p.fixed_dofs()] = 0.0
    R = Kb @ E
    R32, E32 = np.ascontiguousarray(R.T, np.float32), np.ascontiguousarray(E.T, np.float32)
    ctx.set_pairs(R32, E32)
    net = S.Gnn(0, seed=1)
    net.set_params(flat)
    L_gpu, g_gpu = net.loss_grad(ctx, np.arange(8))
    L_ref, g_ref = G.backward(P64, g, Kb, R32.T.astype(np.float64), E32.T.astype(np.float64))
    assert abs(L_gpu - L_ref) / L_ref < 5 * U_BF16
    gg = S.unpack_params(g_gpu)
    worst = 0.0
    for k, ref in g_ref.items():
        nr = np.linalg.norm(ref)
        if nr == 0.0:            # the last node update does not reach the output
            assert np.all(gg[k] == 0.0), k
            continue
        rel = np.linalg.norm(gg[k] - ref) / nr
        worst = max(worst, rel)
        assert rel < 25 * U_BF16, (k, rel)
    flat_ref = S.pack_params(g_ref).astype(np.float64)
    tot = np.linalg.norm(g_gpu - flat_ref) / np.linalg.norm(flat_ref)
    cos = g_gpu @ flat_ref / (np.linalg.norm(g_gpu) * np.linalg.norm(flat_ref))
    print(f"gradient: worst tensor {worst:.3e}, total {tot:.3e}, cosine {cos:.6f}")
    assert tot < 1e-2 and cos > 0.999
    # loss without the gradient is the same number
    assert net.loss_grad(ctx, np.arange(8), grad=False) == pytest.approx(L_gpu, rel=1e-6)


def test_breakdown_falls_back_to_jacobi(S, small):
    p, ctx, Kb, g = small
    uj, ij = ctx.solve(rtol=1e-8)
    net = S.Gnn(0, seed=1)
    # NaN in the decoder: r.M r is not a number on the first iteration
    flat = S.pack_params(random_params(5))
    flat[-3] = np.nan
    net.set_params(flat)
    net.apply(ctx)
    u, info = ctx.solve(rtol=1e-8, precond=S.PRECOND_LEARNED)
    assert info["fell_back"] == 1 and info["converged"] == 1
    ud = O.solve_dense(Kb, ref_system(p)[1])
    e1 = np.linalg.norm(u - ud) / np.linalg.norm(ud)
    print(f"NaN network: fell back, u vs oracle {e1:.2e}")
    assert e1 <= 1e-8
    # a strongly indefinite M (huge random decoder) also ends in a converged solve
    net.set_params(S.pack_params(random_params(6, scale_out=50.0)))
    net.apply(ctx)
    u, info = ctx.solve(rtol=1e-8, precond=S.PRECOND_LEARNED)
    assert info["converged"] == 1 and info["true_relres"] <= 1e-8


def test_errors(S, small):
    p, ctx, Kb, g = small
    c2 = S.Context(0)
    S.setup_problem(c2, p)
    with pytest.raises(S.SfemError, match="ESTATE"):
        c2.solve(rtol=1e-8, precond=S.PRECOND_LEARNED, raise_on_noconv=True)
    with pytest.raises(S.SfemError, match="ESTATE"):
        c2.precond()
    net = S.Gnn(0, seed=1)
    with pytest.raises(S.SfemError, match="ESTATE"):
        net.loss_grad(c2, [0])          # no pairs yet
    e = np.ones((1, Kb.shape[0]), np.float32)
    c2.set_pairs((Kb @ e[0].astype(np.float64)).astype(np.float32)[None, :], e)
    with pytest.raises(S.SfemError, match="EINVAL"):
        net.loss_grad(c2, [1])          # index out of range
    with pytest.raises(S.SfemError, match="EINVAL"):
        net.loss_grad(c2, np.zeros(65, np.int32))
    with pytest.raises(S.SfemError, match="EINVAL"):
        net.set_params(np.zeros(3, np.float32))


def test_training_is_deterministic(S):
    p = mg.learned_small(2, grid=(10, 3, 3))
    ctx = S.Context(0)
    S.setup_problem(ctx, p)
    k = ctx.generate_pairs(3, 8, seed=3)
    assert k >= 12
    out = []
    for _ in range(2):
        net = S.Gnn(0, seed=9)
        losses = net.train([ctx], steps=20, batch=16, lr=1e-3, seed=4)
        out.append((losses, net.params()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_generated_pairs_are_consistent(S):
    """r = K e for the stored pairs (checked through the loss of the untrained
    network: with M = D^-1 the loss is an explicit function of (r, e))."""
    p = mg.learned_small(3, grid=(6, 3, 3))
    ctx = S.Context(0)
    S.setup_problem(ctx, p)
    k = ctx.generate_pairs(2, 6, seed=1)
    assert 2 <= k <= 12
    net = S.Gnn(0, seed=2)
    L = net.loss_grad(ctx, np.arange(k), grad=False)
    assert np.isfinite(L) and L > 0


def test_training_gains_on_held_out_mesh(S):
    """The headline property at test size: a network trained on three
    blob-material cantilevers cuts the PCG iterations of a fourth, unseen one
    (Jacobi: ~1,650 at 40x6x6; trained: ~650-750)."""
    grid = (30, 5, 5)
    ctxs = []
    for mi in range(3):
        c = S.Context(0)
        S.setup_problem(c, mg.learned_small(mi, grid=grid))
        assert c.generate_pairs(10, 20, seed=mi + 1) > 100
        ctxs.append(c)
    held = S.Context(0)
    S.setup_problem(held, mg.learned_small(0, grid=grid, held_out=True))
    net = S.Gnn(0, seed=5)
    losses = net.train(ctxs, steps=800, batch=32, lr=1e-3, seed=1)
    assert losses[-100:].mean() < losses[:20].mean()
    net.apply(held)
    uj, ij = held.solve(rtol=1e-8)
    ul, il = held.solve(rtol=1e-8, precond=S.PRECOND_LEARNED)
    print(f"held-out: Jacobi {ij['iters']} its {ij['ms_solve']:.1f} ms, "
          f"learned {il['iters']} its {il['ms_solve']:.1f} ms")
    assert il["converged"] and not il["fell_back"] and il["true_relres"] <= 1e-8
    assert il["iters"] <= 0.7 * ij["iters"]
    Kb, fb = ref_system(mg.learned_small(0, grid=grid, held_out=True))
    ub = O.solve_banded(Kb, fb)
    errs = {"jacobi": np.linalg.norm(uj - ub) / np.linalg.norm(ub),
            "learned": np.linalg.norm(ul - ub) / np.linalg.norm(ub)}
    # the mixed-precision modes accept the learned preconditioner too
    c32 = S.Context(0)
    S.setup_problem(c32, mg.learned_small(0, grid=grid, held_out=True), f32_copy=True)
    net.apply(c32)
    for name, mode in (("f32_ir", S.MODE_F32_IR), ("f32_rr", S.MODE_F32_RR),
                       ("f32_tf", S.MODE_F32_TF)):
        u, info = c32.solve(rtol=1e-8, mode=mode, precond=S.PRECOND_LEARNED)
        assert info["converged"] and info["true_relres"] <= 1e-8, (mode, info)
        errs[f"learned_{name} ({info['iters']} its)"] = np.linalg.norm(u - ub) / np.linalg.norm(ub)
    print("u error vs the oracle's banded solve: " +
          ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert max(errs.values()) <= 1e-8


def test_learned_graph_periods_equal_eager(S, small):
    """The learned flexible PCG replayed from hipGraph periods equals the
    eager launches bit for bit."""
    p, ctx, Kb, g = small
    flat, _ = fp32_params(S, random_params(3, 0.3))
    net = S.Gnn(0, seed=1)
    net.set_params(flat)
    net.apply(ctx)
    ug, ig = ctx.solve(rtol=1e-10, precond=S.PRECOND_LEARNED)
    ue, ie = ctx.solve(rtol=1e-10, precond=S.PRECOND_LEARNED, profile=True)
    assert ig["iters"] == ie["iters"] and np.array_equal(ug, ue)


def csr_positions(g, Kb):
    """CSR value index of every (block k, a, c): row 3I+a holds the blocks of
    node row I in ascending column order, 3 values each."""
    k = np.arange(g.bcol.size)
    jj = k - g.bptr[g.row]
    a = np.arange(3)[None, :, None]
    c = np.arange(3)[None, None, :]
    return Kb.indptr[3 * g.row[:, None, None] + a] + 3 * jj[:, None, None] + c


def test_forward_and_gradient_parity_at_learned_workload_size(S):
    """Forward S and the loss gradient at the size of the learned-workload
    meshes (140x14x14 cells, 164,640 tets, 770k graph edges): every edge
    kernel runs its multi-tile grid-stride loops (about 12k row tiles of 64
    edges), which the small parity mesh never reaches."""
    p = mg.learned_c4(0, held_out=True)
    ctx = S.Context(0)
    S.setup_problem(ctx, p)
    Kb, fb = ref_system(p)
    g = G.build_graph(Kb, p.mesh.xyz, p.fixed_dofs())
    flat, P64 = fp32_params(S, random_params(21, 0.3))
    net = S.Gnn(0, seed=1)
    net.set_params(flat)
    net.apply(ctx)
    S_gpu, _ = ctx.precond()
    info = ctx.precond_info()
    Sp_ref, _ = G.forward(P64, g)
    S_ref = np.zeros(Kb.nnz)
    S_ref[csr_positions(g, Kb)] = Sp_ref
    rel = np.linalg.norm(S_gpu / info["theta"] - S_ref) / np.linalg.norm(S_ref)
    rng = np.random.default_rng(22)
    E = rng.standard_normal((Kb.shape[0], 4))
    E[p.fixed_dofs()] = 0.0
    R32 = np.ascontiguousarray((Kb @ E).T, np.float32)
    E32 = np.ascontiguousarray(E.T, np.float32)
    ctx.set_pairs(R32, E32)
    L_gpu, g_gpu = net.loss_grad(ctx, np.arange(4))
    L_ref, g_ref = G.backward(P64, g, Kb, R32.T.astype(np.float64), E32.T.astype(np.float64))
    flat_ref = S.pack_params(g_ref).astype(np.float64)
    tot = np.linalg.norm(g_gpu - flat_ref) / np.linalg.norm(flat_ref)
    cos = g_gpu @ flat_ref / (np.linalg.norm(g_gpu) * np.linalg.norm(flat_ref))
    print(f"learned-workload size ({g.bcol.size} edges): S error {rel:.2e}, loss error "
          f"{abs(L_gpu - L_ref) / L_ref:.2e}, gradient error {tot:.2e}, cosine {cos:.6f}")
    assert rel < 5 * U_BF16
    assert abs(L_gpu - L_ref) / L_ref < 5 * U_BF16
    assert tot < 1e-2 and cos > 0.999
    # and the learned solve of this mesh reaches the oracle's displacements
    # (new pairs drop the context's M: infer it again)
    net.apply(ctx)
    ul, il = ctx.solve(rtol=1e-8, precond=S.PRECOND_LEARNED)
    ub = O.solve_banded(Kb, fb)
    eu = np.linalg.norm(ul - ub) / np.linalg.norm(ub)
    print(f"learned solve: {il['iters']} iterations, u error vs banded Cholesky {eu:.2e}")
    assert il["converged"] and eu <= 1e-8


def test_weights_file_round_trip(S, small, tmp_path):
    """sfem_precond_save -> sfem_precond_load -> inference gives the same M
    bit for bit; the file is the documented header plus FP32 parameters; bad
    files are refused and leave the network unchanged."""
    p, ctx, Kb, g = small
    flat, _ = fp32_params(S, random_params(3, 0.3))
    a = S.Gnn(0, seed=1)
    a.set_params(flat)
    a.apply(ctx)
    Sa, _ = ctx.precond()
    path = tmp_path / "net.sfgn"
    a.save(path)
    raw = path.read_bytes()
    n = flat.size
    hdr = np.frombuffer(raw[:32], "<u4")
    assert list(hdr) == [0x4E474653, 1, 64, 4, 8, 12, n, 0] and len(raw) == 32 + 4 * n
    assert np.array_equal(np.frombuffer(raw[32:], "<f4"), flat)
    b = S.Gnn(0, seed=99)
    b.load(path)
    assert np.array_equal(b.params().view(np.uint32), flat.view(np.uint32))
    b.apply(ctx)
    Sb, _ = ctx.precond()
    assert np.array_equal(Sa.view(np.uint32), Sb.view(np.uint32))
    keep = b.params()
    bad = {"truncated": raw[:-4], "oversized": raw + b"\0\0\0\0",
           "magic": b"XXXX" + raw[4:],
           "version": raw[:4] + np.uint32(2).tobytes() + raw[8:],
           "nan": raw[:32] + np.float32(np.nan).tobytes() + raw[36:]}
    for name, data in bad.items():
        q = tmp_path / f"{name}.sfgn"
        q.write_bytes(data)
        with pytest.raises(S.SfemError, match="EINVAL"):
            b.load(q)
        assert np.array_equal(b.params().view(np.uint32), keep.view(np.uint32)), name
    with pytest.raises(S.SfemError, match="EINVAL"):
        b.load(tmp_path / "missing.sfgn")


def test_m_apply_kernels(S):
    """The M apply with r_hat staged in LDS per chunk of rows and the one on
    the grouped layout give z = M r bit for bit as the row kernel; learned
    solves under each reach the oracle's u (the grouped kernel's solve is
    the row kernel's, bit for bit: same sums, same partials); sfem_gnn_apply
    timed all three."""
    p = mg.learned_small(2, grid=(40, 6, 6))
    ctx = S.Context(0)
    S.setup_problem(ctx, p)
    Kb, fb = ref_system(p)
    ub = O.solve_banded(Kb, fb)
    flat, _ = fp32_params(S, random_params(3, 0.3))
    net = S.Gnn(0, seed=1)
    net.set_params(flat)
    net.apply(ctx)
    info = ctx.precond_kernel()
    assert info["variant"] in (0, 1, 2)
    assert info["us_rows"] > 0 and info["us_lds"] > 0 and info["us_grouped"] > 0
    r = np.random.default_rng(4).standard_normal(Kb.shape[0])
    out = {}
    for v in (0, 1, 2):
        ctx.set_precond_kernel(v)
        assert ctx.precond_kernel()["variant"] == v
        z = ctx.precond_apply(r)
        u, i = ctx.solve(rtol=1e-10, precond=S.PRECOND_LEARNED)
        err = np.linalg.norm(u - ub) / np.linalg.norm(ub)
        out[v] = (z, i["iters"], err, u)
        assert i["converged"] and not i["fell_back"] and err <= 1e-8
    print(f"M apply: rows {info['us_rows']:.1f} us, LDS-staged {info['us_lds']:.1f} us, "
          f"grouped {info['us_grouped']:.1f} us (picked {info['variant']}); learned solve "
          f"iterations {out[0][1]} / {out[1][1]} / {out[2][1]}, u error vs banded "
          f"{out[0][2]:.1e} / {out[1][2]:.1e} / {out[2][2]:.1e}")
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][0], out[2][0])
    assert out[2][1] == out[0][1] and np.array_equal(out[2][3], out[0][3])
    assert abs(out[0][1] - out[1][1]) <= 0.05 * out[0][1] + 5
    with pytest.raises(S.SfemError, match="EINVAL"):
        ctx.set_precond_kernel(3)


def test_grouped_m_apply_needs_int16_offsets(S):
    """With shuffled node ids on a mesh of more than 32,768 nodes some block
    column lies beyond an int16 offset: the grouped M apply is neither timed
    nor accepted, and the row kernel applies M."""
    p = mg.learned_small(2, grid=(80, 20, 20))
    m = p.mesh
    assert m.n_nodes > 32768
    sh = np.random.default_rng(5).permutation(m.n_nodes)
    inv = np.empty_like(sh)
    inv[sh] = np.arange(m.n_nodes)
    ctx = S.Context(0)
    ctx.set_mesh(m.xyz[sh], inv[m.tets].astype(np.int32))
    ctx.set_material(p.E, p.nu)
    fd = np.asarray(p.fixed_dofs())
    ctx.set_dirichlet(3 * inv[fd // 3] + fd % 3)
    ctx.add_traction(inv[m.end_tris].astype(np.int32),
                     np.asarray(p.traction, dtype=np.float64).reshape(-1)[:3])
    ctx.assemble()
    flat, _ = fp32_params(S, random_params(3, 0.3))
    net = S.Gnn(0, seed=1)
    net.set_params(flat)
    net.apply(ctx)
    info = ctx.precond_kernel()
    print(f"shuffled {m.n_nodes} nodes: M apply kernel {info['variant']}, "
          f"us {info['us_rows']:.1f} / {info['us_lds']:.1f} / {info['us_grouped']:.1f}")
    assert info["us_grouped"] == 0.0 and info["variant"] in (0, 1)
    with pytest.raises(S.SfemError, match="EINVAL"):
        ctx.set_precond_kernel(2)
    r = np.random.default_rng(6).standard_normal(3 * m.n_nodes)
    z = ctx.precond_apply(r)
    assert np.all(np.isfinite(z)) and np.array_equal(z, ctx.precond_apply(r))
