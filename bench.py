"""Benchmark: FS-FEM stiffness assembly + PCG solve of the 1.92M-tet cantilever.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step = the whole hot path on one synthetic problem already resident in
HBM: numeric assembly of K (per-face smoothed stiffness summed into CSR, BCs
applied) and the solve of K u = f to an FP64 true relative residual of 1e-8.
Topology (faces, CSR pattern) is built once before timing, as the metric
counts assembly with cached topology.

Prints ONE JSON line.  `value` is the K-assembly throughput in faces/s
(median over the timed steps); solve seconds are reported beside it.
`roofline` covers the step's dominant kernel (the CG SpMV), with its
duration measured per launch by HIP events on the library's stream;
`roofline_assembly` covers the assembly kernel.  `cpu_baseline` times the
FP64 oracle (single thread) on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "K-assembly faces/s; solve s to 1e-8 rel-res @1.9M tets: learned vs Jacobi PCG"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
PROFILE_DIR = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(N, T, nf, nnz, nb, f32_copy=False, per_tet=False):
    """Bytes the method itself must move per launch (no re-reads, no
    intermediates).  Assembly: coordinates, tets and the face table read,
    every CSR value written once.  The CG product counted as a scalar CSR
    SpMV (12 bytes per nonzero: FP64 value + int32 column, row offsets, x
    read and y written once), the reference count the roofline uses; the
    library's block format moves less (its own count: format_bytes)."""
    n = 3 * N
    asm = 24 * N + 16 * T + 32 * nf + 8 * nnz + (4 * nnz if f32_copy else 0) + \
        (16 * T if per_tet else 0)
    spmv64 = 12 * nnz + 4 * (n + 1) + 8 * n + 8 * n
    spmv32 = 8 * nnz + 4 * (n + 1) + 4 * n + 4 * n
    return asm, spmv64, spmv32


def format_bytes(N, nnz, nb):
    """What the block-pattern product itself must read and write: each FP64
    value once, one int32 block column per 9 values, node-row offsets, x
    once and y once."""
    n = 3 * N
    return 8 * nnz + 4 * nb + 4 * (N + 1) + 8 * n + 8 * n


def mapply_bytes(N, nnz, nb):
    """Learned M apply z = s (rh + S' rh): the BF16 values of S' once, block
    columns, row offsets, then rh, r, s and z_old read and z written once per
    DOF (FP64 vectors)."""
    n = 3 * N
    return 2 * nnz + 4 * nb + 4 * (N + 1) + 5 * 8 * n


KERNEL_SOURCES = {
    "cg_spmv_f64_c2": ("k_cg_spmv<double, double, 8, 8>", "paper_2001_08849_amd/csrc/solve.hip"),
    "cg_spmv_f32_tf_c2": ("k_cg_spmv<float, double, 8, 72>",
                          "paper_2001_08849_amd/csrc/solve.hip"),
    "cg_spmv_lds_f64_c2": ("k_cg_spmv_lds<double, double, 8, false>",
                           "paper_2001_08849_amd/csrc/solve.hip"),
    "cg_spmv_lds_f32_tf_c2": ("k_cg_spmv_lds<float, double, 8, true>",
                              "paper_2001_08849_amd/csrc/solve.hip"),
    "assemble_c2": ("k_assemble<false, false>", "paper_2001_08849_amd/csrc/assemble.hip"),
    "mapply_c2": ("k_mapply<double>", "paper_2001_08849_amd/csrc/solve.hip"),
    "mapply_lds_c2": ("k_mapply_lds<double>", "paper_2001_08849_amd/csrc/solve.hip"),
    "mapply_grp_c2": ("k_mapply_grp<double>", "paper_2001_08849_amd/csrc/solve.hip"),
}
# instruction and stall counters summarised per kernel (one rocprofv3 pass:
# at most 8 SQ counters)
SQ_COUNTERS = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT",
               "SQ_WAIT_INST_ANY", "SQ_ACTIVE_INST_VALU", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES"]


def _sha(path):
    import hashlib
    return hashlib.sha256(open(os.path.join(ROOT, path), "rb").read()).hexdigest()


def read_traffic(kernel_tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary
    profiles/traffic_<tag>.txt, if its kernel source is unchanged since."""
    path = os.path.join(PROFILE_DIR, f"traffic_{kernel_tag}.txt")
    if not os.path.exists(path):
        return None
    try:
        text = open(path).read()
        # the JSON record starts at the first line that is a lone "{"
        rec = json.loads(text[text.index("\n{\n") + 1:text.rindex("}") + 1])
        if _sha(rec["source"]) != rec["source_sha256"]:
            return None
        return float(rec["bytes_per_launch"])
    except Exception:
        return None


def _demangle_nested(name):
    """Kernel name and builtin template arguments of an Itanium-mangled
    nested name (_ZN<len><id>...I<types>E...). The profiler leaves names
    with __bf16 parameters (DF16b) mangled."""
    import re
    i, ids = 3, []
    while i < len(name) and name[i].isdigit():
        n = re.match(r"\d+", name[i:]).group(0)
        i += len(n)
        ids.append(name[i:i + int(n)])
        i += int(n)
    base = ids[-1] if ids else name
    if i < len(name) and name[i] == "I":
        j = name.find("E", i)
        types = {"d": "double", "f": "float", "i": "int", "b": "bool"}
        args = [types.get(c, c) for c in name[i + 1:j]]
        base += "<" + ", ".join(args) + ">"
    return base


def _short(name):
    if name.startswith("_ZN"):
        return _demangle_nested(name)
    name = name.replace("void ", "").replace("sfem::(anonymous namespace)::", "")
    return name.split("(")[0]


def _counter_means(csv_path, counter=None):
    """Mean counter value per kernel name over its dispatches at the grid it
    was launched with most often (the solver's launches; the autotuner also
    tries other grid caps).  counter: only that counter's rows."""
    import collections
    import csv
    per = collections.defaultdict(float)
    name, grid = {}, {}
    for r in csv.DictReader(open(csv_path)):
        if counter is not None and r.get("Counter_Name") != counter:
            continue
        per[r["Dispatch_Id"]] += float(r["Counter_Value"])
        name[r["Dispatch_Id"]] = r["Kernel_Name"]
        grid[r["Dispatch_Id"]] = int(r.get("Grid_Size", 0) or 0)
    count = collections.Counter((name[d], grid[d]) for d in per)
    mode = {}
    for (nm, g), k in count.items():
        if nm not in mode or k > count[(nm, mode[nm])]:
            mode[nm] = g
    acc = collections.defaultdict(list)
    for d, v in per.items():
        if grid[d] == mode[name[d]]:
            acc[name[d]].append(v)
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def summarize_profiles(prof_dir, command_note):
    """Writes profiles/traffic_<tag>.txt from four rocprofv3 --pmc CSVs under
    prof_dir (fetch/, write/ for the benchmark; cfetch/, cwrite/ for the
    calibration copy) and profiles/kernels_c2.md from a --kernel-trace
    --stats CSV (ktrace/)."""
    import glob
    f = lambda sub: glob.glob(os.path.join(prof_dir, sub, "*counter_collection.csv"))[0]
    fetch, write = _counter_means(f("fetch")), _counter_means(f("write"))
    cfetch, cwrite = _counter_means(f("cfetch")), _counter_means(f("cwrite"))
    copy = [k for k in cfetch if "copyBuffer" in k][0]
    true_bytes = float(1 << 30)
    kf = true_bytes / (cfetch[copy][0] * 1024.0)   # FETCH_SIZE is in KiB
    kw = true_bytes / (cwrite[copy][0] * 1024.0)
    for tag, (pattern, src) in KERNEL_SOURCES.items():
        # the schedule variant launched most often at full size (the one the
        # solver ran, not the autotuner's candidates)
        kn = sorted((k for k in fetch if pattern in _short(k)), key=lambda k: -fetch[k][1])
        if not kn:
            continue
        fr, n = fetch[kn[0]]
        wr, _ = write[kn[0]]
        rec = {
            "kernel": _short(kn[0]), "dispatches": n,
            "fetch_kib_raw": fr, "write_kib_raw": wr,
            "copy_calibration": {"fetch_factor": kf, "write_factor": kw,
                                 "copy": "1 GiB device-to-device (bench.py --copy-calibration)"},
            "bytes_read": fr * 1024 * kf, "bytes_written": wr * 1024 * kw,
            "bytes_per_launch": fr * 1024 * kf + wr * 1024 * kw,
            "source": src, "source_sha256": _sha(src),
        }
        with open(os.path.join(PROFILE_DIR, f"traffic_{tag}.txt"), "w") as fh:
            fh.write(f"# HBM traffic per launch of {rec['kernel']} on the 1.92M-tet cantilever\n")
            fh.write(f"# commands: {command_note}\n")
            fh.write("# FETCH_SIZE / WRITE_SIZE (KiB per dispatch, mean) scaled by what the same\n"
                     "# counters read for a plain 1 GiB copy; stale once the source hash changes.\n")
            fh.write(json.dumps(rec, indent=1) + "\n")
    sq = glob.glob(os.path.join(prof_dir, "sq", "*counter_collection.csv"))
    if sq:
        summarize_sq(sq[0], command_note)
    tables = [("ktrace", "kernels_c2.md",
               "rocprofv3 kernel statistics, 1.92M-tet cantilever benchmark (untrained "
               "network: every launch at full size)"),
              ("ktrace_train", "kernels_training_c4.md",
               "rocprofv3 kernel statistics, benchmark with training (pairs and BF16-MFMA "
               "training on the 164,640-tet meshes, then the 1.92M-tet runs)")]
    for sub, fname, title in tables:
        stats = glob.glob(os.path.join(prof_dir, sub, "*kernel_stats.csv"))
        if not stats:
            continue
        import csv
        rows = list(csv.DictReader(open(stats[0])))
        with open(os.path.join(PROFILE_DIR, fname), "w") as fh:
            fh.write(f"# {title}\n\n")
            fh.write(f"Command: `{command_note}`\n\n")
            fh.write("| kernel | calls | total ms | average us | % |\n|---|---|---|---|---|\n")
            # the 30 largest, plus every hot-path kernel however small its share
            hot = ("k_assemble", "k_face_stress", "k_mapply", "k_cg_spmv", "k_edge_")
            sel = rows[:30] + [r for r in rows[30:] if any(h in r["Name"] for h in hot)]
            for r in sel:
                nm = _short(r["Name"])
                fh.write(f"| {nm} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                         f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |\n")


def summarize_sq(csv_path, command_note):
    """profiles/counters_c2.md: per hot kernel, the SQ counters of one pass
    (means per dispatch) and what they say: VALU instructions per wave,
    VALU busy (active VALU cycles over busy cycles x SIMDs), the share of
    wave cycles spent waiting on any outstanding instruction, LDS
    instructions per wave and LDS bank-conflict cycles per LDS instruction."""
    vals = {c: _counter_means(csv_path, c) for c in SQ_COUNTERS}
    rows = []
    for tag, (pattern, _src) in KERNEL_SOURCES.items():
        kn = sorted((k for k in vals["SQ_WAVES"] if pattern in _short(k)),
                    key=lambda k: -vals["SQ_WAVES"][k][1])
        if not kn:
            continue
        k = kn[0]
        g = {c: vals[c].get(k, (float("nan"), 0))[0] for c in SQ_COUNTERS}
        waves = g["SQ_WAVES"] or float("nan")
        rows.append((_short(k), g,
                     g["SQ_INSTS_VALU"] / waves, g["SQ_INSTS_LDS"] / waves,
                     g["SQ_LDS_BANK_CONFLICT"] / max(g["SQ_INSTS_LDS"], 1.0),
                     g["SQ_WAIT_INST_ANY"] / max(g["SQ_WAVE_CYCLES"], 1.0),
                     g["SQ_ACTIVE_INST_VALU"] / max(g["SQ_WAVE_CYCLES"], 1.0)))
    with open(os.path.join(PROFILE_DIR, "counters_c2.md"), "w") as fh:
        fh.write("# rocprofv3 SQ counters of the hot kernels, 1.92M-tet cantilever\n\n")
        fh.write(f"Command: `{command_note}`\n\n")
        fh.write("Means per dispatch at the solver's grid.  Ratios: VALU and LDS instructions "
                 "per wave; bank-conflict cycles per LDS instruction; the share of wave cycles "
                 "with a wave waiting on any outstanding instruction (SQ_WAIT_INST_ANY / "
                 "SQ_WAVE_CYCLES) and issuing VALU work (SQ_ACTIVE_INST_VALU / "
                 "SQ_WAVE_CYCLES).\n\n")
        fh.write("| kernel | " + " | ".join(SQ_COUNTERS) + " | VALU/wave | LDS/wave | "
                 "conflict cyc/LDS inst | wait share | VALU share |\n")
        fh.write("|---" * (len(SQ_COUNTERS) + 6) + "|\n")
        for nm, g, vw, lw, bc, ws, vs in rows:
            fh.write(f"| {nm} | " + " | ".join(f"{g[c]:.4g}" for c in SQ_COUNTERS) +
                     f" | {vw:.1f} | {lw:.1f} | {bc:.2f} | {ws:.2f} | {vs:.2f} |\n")


CPU_SNIPPET = r"""
import os, sys, time, json
sys.path.insert(0, {root!r})
import numpy as np
import scipy.sparse as sp
from oracle import fsfem as O
from paper_2001_08849_amd import meshgen as mg

W = {{}}

def init(xyz, tets, E, nu, vol, n):
    W.update(xyz=xyz, tets=tets, E=E, nu=nu, vol=vol, n=n)

def assemble_share(sub):
    xyz, tets, E, nu, vol, n = W["xyz"], W["tets"], W["E"], W["nu"], W["vol"], W["n"]
    parts = []
    for blk in (sub[sub[:, 4] < 0], sub[sub[:, 4] >= 0]):
        if blk.shape[0]:
            K, nodes = O.face_stiffness(xyz, tets, blk, E, nu, vol)
            parts.append(O._coo_block(K, nodes))
    I = np.concatenate([q[0] for q in parts]); J = np.concatenate([q[1] for q in parts])
    V = np.concatenate([q[2] for q in parts])
    return sp.coo_matrix((V, (I, J)), shape=(n, n)).tocsr().nnz

if __name__ == "__main__":
    what = {what!r}
    out = {{}}
    p = mg.cantilever_c2()
    m = p.mesh
    n = 3 * m.n_nodes
    faces = O.extract_faces(m.tets)["table"]          # topology, not timed
    S = {sample}
    sub = faces[:S]
    if what == "single":
        t0 = time.perf_counter()
        vol = O.tet_volume(m.xyz[m.tets])
        init(m.xyz, m.tets, p.E, p.nu, vol, n)
        assemble_share(sub)
        dt = time.perf_counter() - t0
        out = {{"faces": int(S), "seconds": dt, "faces_per_s": S / dt}}
        # Jacobi PCG of the 60k-tet cantilever, solve only (assembly untimed)
        p1 = mg.cantilever_c1()
        Kb, fb, _ = O.problem_system(p1)
        t0 = time.perf_counter()
        x, it, rr = O.pcg_jacobi(Kb, fb, rtol=1e-8)
        dt = time.perf_counter() - t0
        out["c1_jacobi"] = {{"seconds": dt, "iters": it, "true_relres": rr, "nnz": int(Kb.nnz)}}
    else:
        import multiprocessing as mpr
        w = int(what)
        vol = O.tet_volume(m.xyz[m.tets])
        chunks = np.array_split(sub, 4 * w)
        with mpr.get_context("spawn").Pool(w, initializer=init,
                                           initargs=(m.xyz, m.tets, p.E, p.nu, vol, n)) as pool:
            pool.map(assemble_share, [sub[:64]] * w)       # workers started and warm
            t0 = time.perf_counter()
            pool.map(assemble_share, chunks)
            dt = time.perf_counter() - t0
        out = {{"faces": int(S), "seconds": dt, "faces_per_s": S / dt, "workers": w}}
    print(json.dumps(out))
"""


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sample_faces: int, c2_iters=None, c2_nnz=None):
    """The FP64 oracle on the host cores: numeric assembly of a sample of
    the 1.92M-tet cantilever's faces on one thread (the reported value) and
    on every available core (one process each, face chunks), plus the
    oracle's Jacobi PCG of the 60k-tet cantilever on one thread (solve only),
    from which the 1.92M-tet solve is extrapolated by nnz and the GPU's
    iteration count (not measured: it would take the oracle ~20 minutes)."""
    one = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1",
               MKL_NUM_THREADS="1", NUMEXPR_NUM_THREADS="1")
    cores = len(os.sched_getaffinity(0))
    workers = max(1, min(16, cores))

    import tempfile

    def run(what):
        # a script file, not -c: the worker processes re-import it by path
        code = CPU_SNIPPET.format(root=ROOT, sample=sample_faces, what=what)
        with tempfile.TemporaryDirectory() as tmp:
            path = os.path.join(tmp, "oracle_cpu_baseline.py")
            with open(path, "w") as fh:
                fh.write(code)
            res = subprocess.run([sys.executable, path], capture_output=True, text=True,
                                 env=one, timeout=900)
        if res.returncode != 0:
            log("cpu baseline failed:", res.stderr[-2000:])
            return None
        return json.loads(res.stdout.strip().splitlines()[-1])

    rec = run("single")
    if rec is None:
        return None
    par = run(str(workers))
    out = {
        "value": rec["faces_per_s"], "unit": "faces/s", "cores": 1, "kind": "oracle",
        "sample": (f"FP64 oracle numeric assembly (Eq. 7 + Table 1 smoothed gradients, "
                   f"Eq. 9 face stiffness, Eq. 12 COO -> CSR) of the first {rec['faces']} "
                   f"faces of the 1.92M-tet cantilever, topology excluded; "
                   f"{rec['seconds']:.1f} s on one host thread"),
        "cpu_model": _cpu_model(), "host_cores_available": cores,
    }
    if par:
        out["all_cores"] = {"value": par["faces_per_s"], "unit": "faces/s",
                            "cores": par["workers"], "seconds": par["seconds"],
                            "how": "the same faces in chunks over one process per core"}
    j = rec["c1_jacobi"]
    out["oracle_jacobi_c1"] = dict(j, cores=1, what="scipy CSR Jacobi PCG of the 60k-tet "
                                                    "cantilever to a true relres of 1e-8, "
                                                    "solve only")
    if c2_iters and c2_nnz:
        per_it = j["seconds"] / j["iters"] * c2_nnz / j["nnz"]
        out["oracle_jacobi_c2_extrapolated"] = {
            "seconds": per_it * c2_iters, "per_iteration_s": per_it, "iters": c2_iters,
            "how": "c1 seconds per iteration x nnz ratio x the GPU's c2 iteration count"}
    return out


def copy_calibration():
    """A plain device-to-device copy of 2^27 float64 (1 GiB read + 1 GiB
    written) five times: what FETCH_SIZE / WRITE_SIZE read for known bytes.
    Runs in its own process (torch only here; the library is not loaded)."""
    import torch
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": b.numel() * 8,
                      "launches": 5}), flush=True)


GRAPH_REPLAY = True


def make_context(sfem):
    """A library context on cuda:0 with the chosen PCG period launching."""
    c = sfem.Context(0)
    if not GRAPH_REPLAY:
        c.set_graph_replay(False)
    return c


def train_network(args, mg, sfem, np):
    """Trains the learned preconditioner on blob-material cantilevers of
    140x14x14 cells (164,640 tets each): pairs from Jacobi-PCG runs, Adam on
    the device.  Returns the network and the training record."""
    if args.weights:
        net = sfem.Gnn(0, seed=5)
        net.load(args.weights)
        log(f"[bench] network loaded from {args.weights} (no pairs or training)")
        return {"net": net, "loaded_from": args.weights, "pairs": 0, "steps": 0}
    if args.train_steps <= 0:
        # untrained network (M = Jacobi exactly): exercises the learned
        # solve's kernels at full size without the training meshes
        log("[bench] --train-steps 0: untrained network, no pairs or training")
        return {"net": sfem.Gnn(0, seed=5), "pairs": 0, "train_meshes": 0, "steps": 0}
    t0 = time.time()
    ctxs, n_pairs = [], 0
    for mi in range(args.train_meshes):
        c = make_context(sfem)
        sfem.setup_problem(c, mg.learned_c4(mi))
        n_pairs += c.generate_pairs(10, 64, seed=mi + 1)
        ctxs.append(c)
    t_pairs = time.time() - t0
    log(f"[bench] training pairs: {n_pairs} from {len(ctxs)} meshes in {t_pairs:.1f}s")
    net = sfem.Gnn(0, seed=5)
    t1 = time.time()
    n1 = int(0.6 * args.train_steps)
    l1 = net.train(ctxs, steps=n1, batch=32, lr=1e-3, seed=1)
    l2 = net.train(ctxs, steps=args.train_steps - n1, batch=32, lr=5e-4, seed=2)
    losses = np.concatenate([l1, l2])
    t_train = time.time() - t1
    log(f"[bench] trained {args.train_steps} Adam steps in {t_train:.1f}s, minibatch loss "
        f"{losses[:20].mean():.4f} -> {losses[-100:].mean():.4f}")
    for c in ctxs:
        c.close()
    if args.save_weights:
        net.save(args.save_weights)
        log(f"[bench] network written to {args.save_weights}")
    held = make_context(sfem)
    sfem.setup_problem(held, mg.learned_c4(0, held_out=True))
    _, ij = held.solve(rtol=1e-8)
    net.apply(held)
    _, il = held.solve(rtol=1e-8, precond=sfem.PRECOND_LEARNED)
    held.close()
    log(f"[bench] held-out 164,640-tet blob mesh: Jacobi {ij['iters']} it {ij['ms_solve']:.1f} ms, "
        f"learned {il['iters']} it {il['ms_solve']:.1f} ms (fell back {il['fell_back']})")
    return {"net": net, "pairs": n_pairs, "train_meshes": args.train_meshes,
            "steps": args.train_steps, "batch": 32, "pairs_s": t_pairs, "train_s": t_train,
            "loss_first": float(losses[:20].mean()), "loss_last": float(losses[-100:].mean()),
            "heldout_c4": {"jacobi_iters": ij["iters"], "jacobi_ms": ij["ms_solve"],
                           "learned_iters": il["iters"], "learned_ms": il["ms_solve"],
                           "fell_back": il["fell_back"]}}


def renumbering_leg(prob, sfem, np, sched):
    """Node numbering and the CG product: the 1.92M-tet cantilever with its
    node ids shuffled (an unstructured generator's arbitrary numbering), then
    renumbered by the library's reverse Cuthill-McKee; the same row schedule
    times 300 Jacobi-PCG iterations on the generator's, the shuffled and the
    RCM numbering."""
    m = prob.mesh
    N = m.n_nodes
    sh = np.random.default_rng(12).permutation(N)
    inv = np.empty_like(sh)
    inv[sh] = np.arange(N)
    xyz_s, tets_s = m.xyz[sh], inv[m.tets].astype(np.int32)      # synthetic input
    ctx = make_context(sfem)
    ctx.rcm_permutation(N, tets_s)                                # warm-up
    perm, ms_rcm = ctx.rcm_permutation(N, tets_s)
    xyz_r, tets_r = ctx.permute_mesh(perm, xyz_s, tets_s)
    old_of = {"generator": np.arange(N), "shuffled": sh, "rcm": sh[perm]}
    meshes = {"generator": (m.xyz, m.tets), "shuffled": (xyz_s, tets_s), "rcm": (xyz_r, tets_r)}
    clamp = np.flatnonzero(m.xyz[:, 0] == 0.0)
    res = {"rcm_ms": ms_rcm, "bandwidth": {}, "topology_ms": {}, "assembly_ms": {},
           "us_per_cg_iteration": {}, "cg_spmv_us": {}}
    for name, (x, t) in meshes.items():
        new_of_old = np.empty(N, np.int64)
        new_of_old[old_of[name]] = np.arange(N)
        c = make_context(sfem)
        c.set_mesh(x, t)
        c.set_material(prob.E, prob.nu)
        c.set_dirichlet(np.sort((3 * new_of_old[clamp][:, None] + np.arange(3)).ravel()))
        c.add_traction(new_of_old[m.end_tris], np.asarray(prob.traction, float))
        c.assemble()
        c.assemble()
        c.set_schedule(*sched)
        c.solve(rtol=1e-8, max_iter=50)
        _, info = c.solve(rtol=1e-8, max_iter=300, profile=True)
        tt = np.asarray(t, np.int64)
        res["bandwidth"][name] = int((tt.max(axis=1) - tt.min(axis=1)).max())
        res["topology_ms"][name] = c.timings()["ms_topology"]
        res["assembly_ms"][name] = c.timings()["ms_assemble"]
        res["us_per_cg_iteration"][name] = info["ms_solve"] / max(info["iters"], 1) * 1e3
        res["cg_spmv_us"][name] = info["ms_spmv_avg"] * 1e3
        log(f"[bench] numbering {name}: bandwidth {res['bandwidth'][name]}, assembly "
            f"{res['assembly_ms'][name]:.3f} ms, CG product {res['cg_spmv_us'][name]:.1f} us, "
            f"iteration {res['us_per_cg_iteration'][name]:.1f} us")
    return res


def es_fem_leg(prob, sfem, np):
    """The same cantilever with edge-based smoothing domains (ES-FEM):
    topology, assembly (median of 3) and the Jacobi-PCG solve to 1e-8."""
    m = prob.mesh
    c = make_context(sfem)
    c.set_smoothing_domain(sfem.DOMAIN_EDGE)
    sfem.setup_problem(c, prob)
    ms = []
    for _ in range(3):
        c.assemble()
        ms.append(c.timings()["ms_assemble"])
    s = c.sizes()
    tuned = c.autotune(reps=10)
    _, info = c.solve(rtol=1e-8)
    asm = float(np.median(ms))
    abytes = 24 * m.n_nodes + 16 * m.n_tets + 8 * s.nnz
    res = {"nnz": s.nnz, "topology_ms": c.timings()["ms_topology"], "assembly_ms": asm,
           "algorithmic_bytes": abytes, "achieved_GBs": abytes / (asm * 1e-3) / 1e9,
           "row_schedule": list(tuned["f64"][0]), "solve_s": info["ms_solve"] / 1e3,
           "iters": info["iters"], "true_relres": info["true_relres"]}
    log(f"[bench] ES-FEM: nnz {s.nnz}, assembly {asm:.3f} ms, solve {info['ms_solve']:.0f} ms, "
        f"{info['iters']} iterations")
    return res


def mixed_precision_leg(ctx, sfem, u, inner_rtol, net, np, uref, reps=3):
    """FP32 matrix values with FP64 refinement on the same cantilever,
    outside the timed steps: K assembled again with its FP32 copy and both
    row schedules retuned; then, each judged by the FP64 true relative
    residual (1e-8):
      - FP32-inner-CG refinement (FP64 outer residuals), once;
      - CG with FP32 products and FP64 residual replacement, restarted in
        FP64 at 1e-3, once;
      - CG with FP32 values in the translation form of the product, FP64
        vectors and residual replacement, no restart: Jacobi and (with a
        network) the learned M, median of `reps` solves each (the learned
        one plus its inference)."""
    ctx.assemble(f32_copy=True)
    tuned = ctx.autotune(reps=3)
    _, ir = ctx.solve(rtol=1e-8, out=u, mode=sfem.MODE_F32_IR, inner_rtol=inner_rtol)
    _, rr = ctx.solve(rtol=1e-8, out=u, mode=sfem.MODE_F32_RR)
    log(f"[bench] FP32 + FP64 refinement: {ir['ms_solve']:.0f} ms, {ir['iters']} it, "
        f"{ir['outer_steps']} outer; FP32 products + FP64 replacement: {rr['ms_solve']:.0f} ms, "
        f"{rr['iters']} it")
    res = {"row_schedule_f32": list(tuned["f32"][0]) if tuned.get("f32") else None}
    for name, i in (("f32_inner_f64_refinement", ir), ("f32_products_f64_replacement", rr)):
        res[name] = {"solve_s": i["ms_solve"] * 1e-3, "iters": i["iters"],
                     "outer_steps": i["outer_steps"], "true_relres": i["true_relres"],
                     "converged": bool(i["converged"])}
    runs = []
    for _ in range(reps):
        _, i = ctx.solve(rtol=1e-8, out=u, mode=sfem.MODE_F32_TF)
        runs.append(i)
    i = runs[-1]
    res["f32_translation_form_jacobi"] = {
        "solve_s": float(np.median([r["ms_solve"] for r in runs])) * 1e-3, "iters": i["iters"],
        "true_relres": i["true_relres"], "converged": bool(i["converged"]),
        "u_error_vs_oracle": u_error(np, u, uref)}
    # every product launch timed (eager launches), for its roofline
    _, pi = ctx.solve(rtol=1e-8, out=u, mode=sfem.MODE_F32_TF, profile=True)
    res["f32_translation_form_jacobi"]["product_us_per_launch"] = pi["ms_spmv_avg"] * 1e3
    log(f"[bench] FP32 translation-form products, Jacobi: "
        f"{res['f32_translation_form_jacobi']['solve_s'] * 1e3:.0f} ms, "
        f"{res['f32_translation_form_jacobi']['iters']} it, relres "
        f"{res['f32_translation_form_jacobi']['true_relres']:.2e}")
    if net is not None:
        # the switch level: FP64 products until the true relres reaches
        # f32_from, FP32 translation-form products after (0: from the start)
        trial = {}
        for lvl in (0.0, 1e-1, 1e-2, 1e-3):
            net.apply(ctx)
            _, i = ctx.solve(rtol=1e-8, out=u, mode=sfem.MODE_F32_TF,
                             precond=sfem.PRECOND_LEARNED, f32_from=lvl)
            trial[lvl] = i
            log(f"[bench] learned M, FP32 translation-form products from relres {lvl:g}: "
                f"{i['ms_solve']:.0f} ms, {i['iters']} it, fell back {i['fell_back']}")
        best = min(trial, key=lambda k: trial[k]["ms_solve"] if trial[k]["converged"] else 1e30)
        runs = []
        for _ in range(reps):
            ms_inf = net.apply(ctx)
            _, i = ctx.solve(rtol=1e-8, out=u, mode=sfem.MODE_F32_TF,
                             precond=sfem.PRECOND_LEARNED, f32_from=best)
            i["ms_inference"] = ms_inf
            runs.append(i)
        i = runs[-1]
        ls = float(np.median([r["ms_solve"] for r in runs])) * 1e-3
        li = float(np.median([r["ms_inference"] for r in runs])) * 1e-3
        res["f32_translation_form_learned"] = {
            "f32_from": best, "solve_s": ls, "inference_s": li, "solve_incl_inference_s": ls + li,
            "iters": i["iters"], "true_relres": i["true_relres"],
            "converged": bool(i["converged"]), "fell_back": i["fell_back"],
            "u_error_vs_oracle": u_error(np, u, uref),
            "switch_levels_tried": {f"{k:g}": {"solve_s": v["ms_solve"] * 1e-3,
                                               "iters": v["iters"]} for k, v in trial.items()}}
        log(f"[bench] learned M, FP32 translation-form products from relres {best:g}: "
            f"{ls * 1e3:.0f} ms + inference {li * 1e3:.0f} ms, {i['iters']} it, relres "
            f"{i['true_relres']:.2e}, fell back {i['fell_back']}")
    return res


REF_U = os.path.join(ROOT, "tests", "golden", "c2_u_ref.npz")


def load_uref(np):
    """The oracle's displacements of the 1.92M-tet cantilever (written by
    tests/golden/make_c2_reference.py), if present."""
    if not os.path.exists(REF_U):
        return None
    return np.load(REF_U)["u"]


def u_error(np, u, uref):
    """Relative L2 distance of u from the oracle's displacements."""
    if uref is None:
        return None
    return float(np.linalg.norm(u - uref) / np.linalg.norm(uref))


def batch_leg(mg, sfem, np):
    """The batched workload: 64 meshes (1.9k-288k tets, 4.0M in all) x 4
    load cases, one block-diagonal system, tuned 4-RHS product, hipGraph
    replay of the check period, every system to an FP64 true residual of
    1e-8.  Roofline of the tuned 4-RHS product: values, block columns and
    row offsets once, plus x gathered and y written for the 4 right-hand
    sides."""
    t0 = time.time()
    items = mg.batch_c3()
    b = sfem.batch_from_items(items)
    sz = b.sizes()
    t_build = time.time() - t0
    us = b.autotune(reps=3)
    info = b.solve(rtol=1e-8, use_graph=True)
    n = 3 * sz["nodes"]
    nb = sz["nnz"] // 9
    mbytes = 8 * sz["nnz"] + 4 * nb + 4 * (sz["nodes"] + 1) + 4 * 2 * 8 * n
    ach = mbytes / (us * 1e-6) / 1e9
    res = {"meshes": sz["meshes"], "systems": 4 * sz["meshes"], "tets": sz["tets"],
           "nnz": sz["nnz"], "host_build_s": t_build, "solve_ms": info["ms_solve"],
           "periods": info["periods"], "max_iters": info["max_iters"],
           "worst_relres": info["worst_relres"], "all_converged": bool(info["all_converged"]),
           "spmm4": {"us": us, "bytes": mbytes, "achieved": ach, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": ach / HBM_PEAK_GBS},
           "schedules": [b.schedule(k) for k in range(3)]}
    log(f"[bench] batch: {sz['meshes']} meshes x 4 load cases, {sz['tets']} tets, solve "
        f"{info['ms_solve']:.0f} ms, max {info['max_iters']} iterations, 4-RHS product {us:.0f} us "
        f"({ach:.0f} GB/s)")
    # the stated precision of this workload: FP32 products inside FP64
    # residual replacement (every system judged by its FP64 true residual)
    b.close()
    b32 = sfem.batch_from_items(items, f32_copy=True)
    us32 = b32.autotune(reps=3, f32=True)
    i32 = b32.solve(rtol=1e-8, mode=sfem.MODE_F32_RR, use_graph=True)
    res["f32_products_f64_replacement"] = {
        "solve_ms": i32["ms_solve"], "periods": i32["periods"], "max_iters": i32["max_iters"],
        "worst_relres": i32["worst_relres"], "all_converged": bool(i32["all_converged"]),
        "spmm4_us": us32}
    log(f"[bench] batch, FP32 products + FP64 replacement: solve {i32['ms_solve']:.0f} ms, max "
        f"{i32['max_iters']} iterations, 4-RHS product {us32:.0f} us")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1000000)
    ap.add_argument("--skip-solve", action="store_true", help="assembly only (profiling)")
    ap.add_argument("--f32-ir", action="store_true", help="also time the FP32+FP64-IR solve")
    ap.add_argument("--inner-rtol", type=float, default=1e-2)
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the FP32/FP64 refinement leg")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the 64-mesh x 4-load-case batched solve")
    ap.add_argument("--no-es-fem", action="store_true",
                    help="skip the edge-based smoothing domain (ES-FEM) leg")
    ap.add_argument("--no-renumbering", action="store_true",
                    help="skip the shuffled / RCM numbering comparison")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip training and the learned-preconditioner solve")
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--train-meshes", type=int, default=4)
    ap.add_argument("--weights", default="", metavar="PATH",
                    help="load the network from this weights file instead of training it")
    ap.add_argument("--save-weights", default="", metavar="PATH",
                    help="write the trained network to this weights file")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--summarize-profiles", metavar="DIR",
                    help="write profiles/ summaries from rocprofv3 CSVs under DIR")
    ap.add_argument("--profile-command", default="", help="command line recorded in summaries")
    ap.add_argument("--schedule", default="", metavar="VARIANT,GRID_CAP",
                    help="pin the FP64 row schedule instead of autotuning it")
    ap.add_argument("--precond-kernel", type=int, default=-1, metavar="VARIANT",
                    help="pin the learned M's apply kernel (0: rows, 1: LDS-staged) instead of "
                         "the one timed fastest (counter runs, whose timings are distorted)")
    ap.add_argument("--tf-solve", action="store_true",
                    help="after the timed steps, one Jacobi solve with FP32 translation-form "
                         "products (profiling; the full leg is --no-mixed's)")
    ap.add_argument("--no-graph-replay", action="store_true",
                    help="launch every PCG kernel one by one (for tracers that cannot follow "
                         "hipGraph launches)")
    args = ap.parse_args()
    global GRAPH_REPLAY
    GRAPH_REPLAY = not args.no_graph_replay
    if args.copy_calibration:
        copy_calibration()
        return
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles, args.profile_command)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              f"design is described, not built.", flush=True)
        sys.exit(2)

    import numpy as np

    from paper_2001_08849_amd import meshgen as mg
    from paper_2001_08849_amd import sfem

    learned = None if args.no_learned else train_network(args, mg, sfem, np)

    t0 = time.time()
    prob = mg.cantilever_c2()
    m = prob.mesh
    log(f"[bench] mesh {m.grid} N={m.n_nodes} T={m.n_tets} generated in {time.time() - t0:.1f}s")
    ctx = make_context(sfem)
    ctx.set_mesh(m.xyz, m.tets)
    ctx.set_material(prob.E, prob.nu)
    ctx.set_dirichlet(prob.fixed_dofs())
    ctx.add_traction(m.end_tris, prob.traction)
    s = ctx.sizes()
    ms_topo = ctx.timings()["ms_topology"]
    log(f"[bench] topology {ms_topo:.1f} ms: faces {s.n_faces} ({s.n_exterior} ext), "
        f"nnz {s.nnz}, blocks {s.n_blocks}")

    ctx.assemble(f32_copy=args.f32_ir)
    if args.schedule:
        # pinned (counter runs: the profiler serialises kernels, which would
        # distort the autotuner's timings and change its choice)
        v, cap = (int(x) for x in args.schedule.split(","))
        ctx.set_schedule(v, cap)
        tuned = {"f64": ((v, cap), None)}
        log(f"[bench] row schedule pinned to (variant, grid cap) {(v, cap)}")
    else:
        tuned = ctx.autotune(reps=10)
        log(f"[bench] autotuned row schedule (variant, grid cap) {tuned['f64'][0]}: "
            f"{tuned['f64'][1]:.1f} us per PCG iteration")
    u = np.empty(s.n_rows)

    def step(profile=False):
        ctx.assemble(f32_copy=args.f32_ir)
        ms_asm = ctx.timings()["ms_assemble"]
        if args.skip_solve:
            return ms_asm, None
        _, info = ctx.solve(rtol=1e-8, out=u, profile=profile)
        if args.f32_ir:
            _, info32 = ctx.solve(rtol=1e-8, out=u, mode=sfem.MODE_F32_IR,
                                  inner_rtol=args.inner_rtol)
            info["ir"] = info32
            log(f"[bench]   FP32+FP64-IR: {info32['ms_solve']:.1f} ms, {info32['iters']} it, "
                f"{info32['outer_steps']} outer, relres {info32['true_relres']:.2e}")
            _, inforr = ctx.solve(rtol=1e-8, out=u, mode=sfem.MODE_F32_RR, profile=profile)
            info["rr"] = inforr
            log(f"[bench]   FP32-matrix CG + FP64 replacement: {inforr['ms_solve']:.1f} ms, "
                f"{inforr['iters']} it, relres {inforr['true_relres']:.2e}, "
                f"spmv {inforr['ms_spmv_avg'] * 1e3:.1f} us")
        return ms_asm, info

    for w in range(args.warmup):
        ms_asm, info = step()
        log(f"[bench] warmup {w}: assembly {ms_asm:.3f} ms" +
            (f", solve {info['ms_solve']:.1f} ms ({info['iters']} it)" if info else ""))

    uref = load_uref(np)
    ctx.synchronize()
    ctx.timer_start()
    asm_ms, solves = [], []
    for k in range(args.steps):
        ms_asm, info = step()
        asm_ms.append(ms_asm)
        if info:
            solves.append(info)
        log(f"[bench] step {k}: assembly {ms_asm:.3f} ms" +
            (f", solve {info['ms_solve']:.1f} ms, {info['iters']} it, relres "
             f"{info['true_relres']:.2e}" if info else ""))
    total_ms = ctx.timer_stop()
    ctx.synchronize()
    err_jacobi = u_error(np, u, uref) if solves else None
    # per-launch timing of the CG product (events around every launch, so
    # every launch is eager): one more solve, outside the timed steps
    prof = None
    if not args.skip_solve:
        _, prof = ctx.solve(rtol=1e-8, out=u, profile=True)
        log(f"[bench] profiled solve: {prof['ms_solve']:.1f} ms, CG product "
            f"{prof['ms_spmv_avg'] * 1e3:.1f} us per launch")

    if args.tf_solve and not args.skip_solve:
        ctx.assemble(f32_copy=True)
        _, itf = ctx.solve(rtol=1e-8, out=u, mode=sfem.MODE_F32_TF, profile=True)
        log(f"[bench] FP32 translation-form solve (profiled): {itf['ms_solve']:.1f} ms, "
            f"{itf['iters']} it, product {itf['ms_spmv_avg'] * 1e3:.1f} us per launch")
        ctx.assemble()

    stress = None
    if not args.skip_solve:
        # post-processing: smoothed strain and stress of every smoothing domain
        times = [ctx.face_stress(u)[2] for _ in range(3)]
        sb = 32 * s.n_faces + 48 * m.n_nodes + 96 * s.n_faces
        ms_s = float(np.median(times))
        stress = {"kernel": "k_face_stress<false>", "ms": ms_s, "faces": s.n_faces,
                  "faces_per_s": s.n_faces / (ms_s * 1e-3), "bytes": sb,
                  "achieved_GBs": sb / (ms_s * 1e-3) / 1e9,
                  "frac": sb / (ms_s * 1e-3) / 1e9 / HBM_PEAK_GBS}
        log(f"[bench] stress recovery: {ms_s:.3f} ms for {s.n_faces} faces")

    lsolves = []
    if learned is not None and not args.skip_solve:
        net = learned["net"]
        for k in range(max(1, args.steps) + 1):
            # the last solve times every launch (eager), for the M-apply roofline
            last = k == max(1, args.steps)
            ms_inf = net.apply(ctx)
            if args.precond_kernel >= 0:
                ctx.set_precond_kernel(args.precond_kernel)
            _, info = ctx.solve(rtol=1e-8, out=u, precond=sfem.PRECOND_LEARNED, profile=last)
            info["ms_inference"] = ms_inf
            if last:
                lprof = info
                log(f"[bench] profiled learned solve: {info['ms_solve']:.1f} ms, M apply "
                    f"{info['ms_mapply_avg'] * 1e3:.1f} us per launch")
                continue
            info["u_error_vs_oracle"] = u_error(np, u, uref)
            lsolves.append(info)
            pinfo = ctx.precond_info()
            log(f"[bench] learned {k}: inference {ms_inf:.1f} ms (theta {pinfo['theta']:.3f}), "
                f"solve {info['ms_solve']:.1f} ms, {info['iters']} it, relres "
                f"{info['true_relres']:.2e}, fell back {info['fell_back']}")

    # theta of the learned M, read before the refinement leg re-assembles K
    theta = ctx.precond_info()["theta"] if lsolves else None
    mixed = None
    if not args.skip_solve and not args.no_mixed and not args.f32_ir:
        mixed = mixed_precision_leg(ctx, sfem, u, args.inner_rtol,
                                    learned["net"] if learned else None, np, uref)

    asm_med = float(np.median(asm_ms))
    faces_per_s = s.n_faces / (asm_med * 1e-3)
    asm_bytes, spmv_bytes, _ = algorithmic_bytes(m.n_nodes, m.n_tets, s.n_faces, s.nnz,
                                                 s.n_blocks)
    out = {
        "metric": METRIC,
        "value": faces_per_s,
        "unit": "faces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "cantilever 40x4x4 m, 200x40x40 cells x 6 Kuhn T4 (1.92M tets), "
                        "+/-10% jitter seed 2, E=210e9, nu=0.3, clamp x=0, end traction 1e6 Pa",
            "tets": m.n_tets, "nodes": m.n_nodes, "faces": s.n_faces, "nnz": s.nnz,
            "solver": "Jacobi PCG FP64, x0=0, true relres <= 1e-8",
        },
        "row_schedule": {"variant": tuned["f64"][0][0], "grid_cap": tuned["f64"][0][1],
                         "autotuned_us_per_pcg_iteration": tuned["f64"][1]},
        "assembly_ms": asm_med,
        "topology_ms": ms_topo,
    }
    if solves:
        out["solve_s"] = {"jacobi_f64": float(np.median([i["ms_solve"] for i in solves])) / 1e3}
        out["solve_iters"] = {"jacobi_f64": solves[-1]["iters"]}
        out["solve_true_relres"] = {"jacobi_f64": solves[-1]["true_relres"]}
        out["u_error_vs_oracle"] = {
            "jacobi_f64": err_jacobi,
            "reference": "tests/golden/c2_u_ref.npz (FP64 oracle: PCG + translation-form "
                         "refinement, own error estimate in c2_u_ref.txt)"}
        if lsolves:
            ls = float(np.median([i["ms_solve"] for i in lsolves])) / 1e3
            li = float(np.median([i["ms_inference"] for i in lsolves])) / 1e3
            out["solve_s"]["learned"] = ls
            out["solve_s"]["learned_incl_inference"] = ls + li
            out["solve_iters"]["learned"] = lsolves[-1]["iters"]
            out["solve_true_relres"]["learned"] = lsolves[-1]["true_relres"]
            out["u_error_vs_oracle"]["learned"] = lsolves[-1]["u_error_vs_oracle"]
            mms = lprof["ms_mapply_avg"]
            mb = mapply_bytes(m.n_nodes, s.nnz, s.n_blocks)
            ach_m = mb / (mms * 1e-3) / 1e9 if mms > 0 else None
            mk = ctx.precond_kernel()
            kname, ktag = [("k_mapply<double>", "mapply_c2"),
                           ("k_mapply_lds<double>", "mapply_lds_c2"),
                           ("k_mapply_grp<double>", "mapply_grp_c2")][mk["variant"]]
            out["roofline_mapply"] = {
                "kernel": kname, "bound": "hbm", "achieved": ach_m,
                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach_m / HBM_PEAK_GBS if ach_m else None,
                "traffic": read_traffic(ktag),
                "bytes_per_launch": mb, "us_per_launch": mms * 1e3,
                "kernel_choice_us": {"rows": mk["us_rows"], "lds_staged": mk["us_lds"],
                                     "grouped": mk["us_grouped"]}}
            out["learned"] = {
                "solver": "flexible PCG, K FP64, learned M (S' BF16 in the padded node-row layout, network BF16-MFMA), "
                          "FP64 vectors and dots, true relres <= 1e-8",
                "inference_s": li, "theta": theta,
                "fell_back": lsolves[-1]["fell_back"],
                "speedup_vs_jacobi": out["solve_s"]["jacobi_f64"] / (ls + li),
                "training": {k: v for k, v in learned.items() if k != "net"},
            }
        spmv_ms = prof["ms_spmv_avg"]
        ach = spmv_bytes / (spmv_ms * 1e-3) / 1e9
        fb = format_bytes(m.n_nodes, s.nnz, s.n_blocks)
        out["roofline"] = {"kernel": f"k_cg_spmv<double,double> (row schedule "
                                     f"{tuned['f64'][0][0]})", "bound": "hbm",
                           "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": ach / HBM_PEAK_GBS,
                           "traffic": read_traffic("cg_spmv_f64_c2"),
                           "bytes_per_launch": spmv_bytes,
                           "bytes_note": "scalar CSR SpMV count: 12 nnz + 4 (n+1) + 16 n",
                           "format_bytes_per_launch": fb,
                           "format_frac": fb / (spmv_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                           "us_per_launch": spmv_ms * 1e3}
    ach_a = asm_bytes / (asm_med * 1e-3) / 1e9
    out["roofline_assembly"] = {"kernel": "k_assemble<false>", "bound": "hbm", "achieved": ach_a,
                                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach_a / HBM_PEAK_GBS,
                                "traffic": read_traffic("assemble_c2"),
                                "bytes_per_launch": asm_bytes, "us_per_launch": asm_med * 1e3}
    # the kernel's real limiter: one 64-bit LDS atomic per (row, face, entry)
    # contribution, 144 per exterior and 225 per interior face (the COO length
    # of Eq. 12); peaks: 16 per clock per CU without bank conflicts (128 B/clk
    # of LDS), 5.1 per clock per CU measured for random addresses
    n_atom = 144 * s.n_exterior + 225 * (s.n_faces - s.n_exterior)
    rate = n_atom / (asm_med * 1e-3)
    clk = 256 * 2.4e9
    out["roofline_assembly"]["lds_atomics"] = {
        "per_launch": n_atom, "achieved_per_s": rate,
        "peak_conflict_free_per_s": 16 * clk, "frac_conflict_free": rate / (16 * clk),
        "peak_random_measured_per_s": 5.1 * clk, "frac_random_measured": rate / (5.1 * clk)}
    if stress:
        out["stress_recovery"] = stress
    if mixed:
        out["mixed_precision"] = mixed
        pus = mixed["f32_translation_form_jacobi"].get("product_us_per_launch")
        if pus:
            _, _, sb32 = algorithmic_bytes(m.n_nodes, m.n_tets, s.n_faces, s.nnz, s.n_blocks)
            n = 3 * m.n_nodes
            # the kernel's own bytes: FP32 values (packed, padding included),
            # packed block columns, row offsets, C, x read and q written in FP64
            own = 4 * s.nnz + 4 * s.n_blocks + 4 * (m.n_nodes + 1) + 72 * m.n_nodes + 16 * n
            ach = sb32 / (pus * 1e-6) / 1e9
            out["roofline_f32_tf"] = {
                "kernel": "k_cg_spmv<float, double, 8, 72>", "bound": "hbm", "achieved": ach,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
                "traffic": read_traffic("cg_spmv_f32_tf_c2"), "bytes_per_launch": sb32,
                "bytes_note": "scalar CSR FP32 SpMV count: 8 nnz + 4 (n+1) + 8 n",
                "format_bytes_per_launch": own,
                "format_frac": own / (pus * 1e-6) / 1e9 / HBM_PEAK_GBS,
                "us_per_launch": pus}
        if solves:
            out["solve_s"]["jacobi_f32_translation_form"] = \
                mixed["f32_translation_form_jacobi"]["solve_s"]
            out["solve_iters"]["jacobi_f32_translation_form"] = \
                mixed["f32_translation_form_jacobi"]["iters"]
            ml = mixed.get("f32_translation_form_learned")
            if ml:
                out["solve_s"]["learned_f32_translation_form_incl_inference"] = \
                    ml["solve_incl_inference_s"]
                out["solve_iters"]["learned_f32_translation_form"] = ml["iters"]
    if not args.no_batch and not args.skip_solve:
        out["batch_c3"] = batch_leg(mg, sfem, np)
    if not args.no_es_fem and not args.skip_solve:
        out["es_fem"] = es_fem_leg(prob, sfem, np)
    if not args.no_renumbering and not args.skip_solve:
        out["renumbering"] = renumbering_leg(prob, sfem, np, tuned["f64"][0])
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle: 1 thread and all cores) ...")
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample,
                                           solves[-1]["iters"] if solves else None, s.nnz)
    out["context"] = {"paper_assembly_faces_per_s_24core": 4.2e5,
                      "paper_note": "derived: ~4.15M faces / ~10 s on a 24-core Xeon 5118, "
                                    "TetGen mesh of 2.08M tets, direct solver; not comparable"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
