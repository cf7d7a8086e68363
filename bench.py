"""Benchmark: space-time DOF-matvecs/s of the pFMM single-layer apply on one
MI355X, and the Dirichlet solve time against plain GMRES.

Default workload: the surface of the cube [-1,1]^3 with 16 x 16 squares per
face (3072 triangles) x 1024 uniform steps on [0, 1] (3,145,728 space-time
DOFs), alpha = 1, Chebyshev degree 6 in space, Lagrange degree 6 in time,
leaves below 64 elements, c_st = 0.9, n_tr = 5; densities i.i.d. U(-1, 1)
from seed 3.  A step is one full V_h apply (Algorithm 2) from a
device-resident density to a device-resident result, FP64 throughout; tree
build and nearfield assembly happen before the timed region and are
reported apart.  The same tree also runs the FP32 and BF16-input farfields,
whose error against the FP64 apply is measured (the "1e-6 rel err" of the
metric).  Then, unless switched off: the 3072 x 256 workload as a secondary
figure, and the Dirichlet solve on the 12,288-triangle x 512-step cube
(learned preconditioner with FP32 inner applies against plain FP64 GMRES,
both to an FP64 relative residual of 1e-8).

Prints one JSON line.  Only one GPU is used: --gpus above 1 exits with a
message.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "space-time DOF matvec/s of pFMM V_h at 1e-6 rel err; GMRES solve time vs plain"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
FP32_PEAK_TFS = 157.3     # dense FP32 matrix-core peak

# HBM bytes per apply from rocprofv3 FETCH_SIZE / WRITE_SIZE runs (all
# launches of the kernel in one apply), scaled by the same counters on a
# plain 1 GiB device copy (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000).  Each
# entry is valid only for the sources it was taken on (sha256 prefixes of the
# kernel file and of the file that plans and launches it); any change to
# them reports null.
TRAFFIC = [
    # profiles/hbm_traffic_v_apply_cube16x1024_m6.md
    {"kernel": "m2l", "config": 3, "precision": "fp64", "bytes": 229.16e9,
     "files": {"m2l_kernels.hpp": "7f71f6073bcde959", "pfmm.hip": "1c7e4fe0c9b84718"}},
    {"kernel": "k_near_apply", "config": 3, "bytes": 107.03e9,
     "files": {"near_apply.hpp": "30a329af442a5db2", "pfmm.hip": "1c7e4fe0c9b84718"}},
]


def measured_traffic(kernel, cfg, precision="fp64"):
    """HBM bytes per apply from the rocprofv3 counters, while the sources the
    counters were taken on (kernel and launch configuration) are unchanged."""
    import hashlib
    for e in TRAFFIC:
        if e["kernel"] != kernel or e["config"] != cfg or e.get("precision", precision) != precision:
            continue
        for name, prefix in e["files"].items():
            with open(os.path.join(ROOT, "paper_2106_15911_amd", "csrc", name), "rb") as fh:
                if hashlib.sha256(fh.read()).hexdigest()[:16] != prefix:
                    return None
        return e["bytes"]
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sample(tr, o, w, rng, per_level, n_leaves, n_rows):
    """One timed pass of the oracle's V_h apply on a bounded sample:
    moments of every box (the upward pass, in full), M2L + L2L of
    `per_level` random boxes per level, L2T of `n_leaves` random leaves, and
    the nearfield of `n_rows` random rows, its panel integrals (assembly)
    timed apart from the row sums (apply).  Returns the timings and the
    estimate of one full apply (each sampled part scaled by its count)."""
    import numpy as np
    N = tr.E_t * tr.E_x
    t0 = time.perf_counter()
    mu = o.moments(w)
    t_up = time.perf_counter() - t0
    est, timed, n_far = t_up, t_up, 0
    for l in range(2, tr.depth + 1):
        boxes = tr.levels[l]
        pick = rng.choice(len(boxes), min(per_level, len(boxes)), replace=False)
        t0 = time.perf_counter()
        for i in pick:
            Z = boxes[int(i)]
            lam_ = o.m2l(Z, mu)
            if l >= 3:
                lam_ = lam_ + o.l2l(Z, Z.parent, np.zeros_like(lam_))
        dt = time.perf_counter() - t0
        timed += dt
        n_far += len(pick)
        est += dt * len(boxes) / len(pick)
    pick = rng.choice(len(tr.leaves), n_leaves, replace=False)
    t0 = time.perf_counter()
    for i in pick:
        Z = tr.leaves[int(i)]
        o.l2t(Z, np.zeros((o.m_t + 1, o.Nk)))
    dt = time.perf_counter() - t0
    timed += dt
    est += dt * len(tr.leaves) / n_leaves
    # nearfield rows: entries (assembly) apart from the sums (apply)
    leaf = tr.leaf_of_element()
    by_id = {b.id: b for b in tr.leaves}
    memo = {}
    t_asm = t_near = 0.0
    n_int = 0
    for r in rng.choice(N, n_rows, replace=False):
        Z = by_id[int(leaf[r])]
        kt, kx = divmod(int(r), tr.E_x)
        srcs = [S for S in tr.nearfield(Z, memo) if S.s0 <= kt]
        dmax = kt - min(S.s0 for S in srcs)
        jx_all = np.unique(np.concatenate([S.tris for S in srcs]))
        t0 = time.perf_counter()
        ent = o.entries(np.full(len(jx_all), kx), jx_all, dmax)
        t_asm += time.perf_counter() - t0
        n_int += ent.size
        where = {int(j): i for i, j in enumerate(jx_all)}
        t0 = time.perf_counter()
        acc = 0.0
        for S in srcs:
            idx = np.array([where[int(j)] for j in S.tris])
            for jt in range(S.s0, min(S.s1, kt + 1)):
                acc += ent[idx, kt - jt] @ w[jt * tr.E_x + S.tris]
        t_near += time.perf_counter() - t0
    timed += t_near
    est += t_near * N / n_rows
    return dict(upward_s=t_up, timed_apply_s=timed, est_apply_s=est, n_far_boxes=n_far, n_leaves=int(n_leaves),
                n_rows=int(n_rows), assembly_sample_s=t_asm, assembly_integrals=int(n_int))


def cpu_baseline(cfg, w, distinct_integrals, per_level=8, leaves=8, rows=8, seed=123):
    """The CPU oracle's V_h apply on the same workload and inputs, timed on a
    bounded sample and scaled to one full apply, with all host threads and
    with one thread; its nearfield assembly (the panel integrals) is timed
    apart and scaled by the distinct integrals the tree needs, like the
    GPU's assembly, which the timed GPU apply excludes too."""
    from threadpoolctl import threadpool_info, threadpool_limits
    import numpy as np
    from oracle.fmm import FMMOracle
    from oracle.tree import Tree
    from workloads import config_problem
    v, t, tn, c, _ = config_problem(cfg)
    N = len(w)
    t0 = time.perf_counter()
    tr = Tree(v, t, tn, 1.0, c["n_max"], c["c_st"], c["n_tr"])
    t_tree = time.perf_counter() - t0
    blas = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    runs = {}
    for label, nthr in (("all_threads", blas), ("one_thread", 1)):
        o = FMMOracle(tr, c["m_t"], c["m_x"], "V")
        with threadpool_limits(limits=nthr):
            runs[label] = _oracle_sample(tr, o, w, np.random.default_rng(seed), per_level, leaves, rows)
        runs[label]["threads"] = nthr
        runs[label]["value"] = N / runs[label]["est_apply_s"]
        log(f"[bench] cpu oracle ({label}): {runs[label]}")
    a = runs["all_threads"]
    per_int = a["assembly_sample_s"] / max(a["assembly_integrals"], 1)
    return {"value": a["value"], "unit": "DOF-matvec/s", "cores": int(blas), "kind": "oracle",
            "sample": (f"oracle V_h apply on the same {N} DOFs: upward pass (moments of every box) in full "
                       f"({a['upward_s']:.1f} s); M2L+L2L of {a['n_far_boxes']} random boxes (up to {per_level} per "
                       f"level), L2T of {leaves} random leaves and the nearfield row sums of {rows} random rows, each "
                       f"scaled by its count; estimated full apply {a['est_apply_s']:.0f} s; panel integrals of the "
                       f"sampled rows timed apart (assembly)"),
            "one_thread_value": runs["one_thread"]["value"], "one_thread_est_apply_s": runs["one_thread"]["est_apply_s"],
            "timed_s": a["timed_apply_s"] + runs["one_thread"]["timed_apply_s"], "tree_s": t_tree,
            "assembly": {"sampled_integrals": a["assembly_integrals"], "sampled_s": a["assembly_sample_s"],
                         "s_per_integral": per_int, "tree_distinct_integrals": int(distinct_integrals),
                         "est_full_s": per_int * distinct_integrals},
            "host_cpus": os.cpu_count(), "cpu_model": _cpu_model(), "blas_threads": int(blas), "runs": runs}


def _dirichlet_rhs(cfg, P, torch, nf_mode, T=None):
    """Mesh, parameters and b = (1/2 M_h + K_h) g of the Dirichlet problem on
    one cube workload (g: p0 projection of G(x - (2.5,0,0), t + 0.1)), on
    [0, T] when T is given; b is formed on a tree holding only K_h, released
    before returning."""
    from workloads import config_problem, uniform_time_nodes
    from workloads.dirichlet import project_source_datum
    v, t, tn, c, _ = config_problem(cfg)
    if T is not None:
        tn = uniform_time_nodes(c["n_steps"], T)
    t0 = time.perf_counter()
    g = project_source_datum(v, t, tn, (2.5, 0.0, 0.0), -0.1, 1.0)
    t_g = time.perf_counter() - t0
    kw = dict(m_t=c["m_t"], m_x=c["m_x"], n_max=c["n_max"], c_st=c["c_st"], n_tr=c["n_tr"], nearfield_mode=nf_mode)
    gd = torch.from_numpy(g).to("cuda:0")
    t0 = time.perf_counter()
    tk = P.Tree(v, t, tn, P.default_params(operators=2, **kw), device=0)
    b = tk.dirichlet_rhs(gd)
    torch.cuda.synchronize()
    t_k = time.perf_counter() - t0
    tk.close()
    log(f"[solve] config {cfg}: datum {t_g:.1f} s, K tree + rhs {t_k:.2f} s")
    return v, t, tn, c, kw, b, dict(datum_s=t_g, build_K_and_rhs_s=t_k)


def toeplitz_roofline(st, near_ms):
    """The Toeplitz nearfield stage against the FP64 matrix peak: useful work
    2 FLOP per causal nearfield entry (the products the stored mode reads
    from HBM), over the stage's measured time."""
    flop = 2.0 * st["near_entries"]
    tf = flop / (near_ms * 1e-3) / 1e12
    return {"kernels": "k_near_gemm (GEMM groups) + k_near_toep (the rest)", "nearfield_ms": near_ms,
            "near_gemm_groups": st["near_gemm_groups"], "bound": "mfma", "useful_flop": flop, "achieved": tf,
            "peak": FP64_PEAK_TFS, "unit": "TFLOP/s", "frac": tf / FP64_PEAK_TFS}


def solve_bench(args):
    """Dirichlet solve on the 12,288-triangle x 512-step cube to a relative
    FP64 residual of 1e-8: plain FP64 GMRES against flexible GMRES with the
    learned preconditioner (trained on the 3,072-triangle x 256-step cube,
    its time interval stretched so that h_t / h_x^2 equals the target's:
    the local map from residual to error depends on that ratio),
    inner applies in FP64 and in the mixed FP32 farfield, all inside FP64
    iterative refinement and judged by the FP64 residual.  All solves run on
    one tree holding V_h (Toeplitz nearfield, FP32 farfield tables present);
    b is formed on a tree holding only K_h, released before.
    """
    import torch
    import paper_2106_15911_amd as P
    nf = P.NF_STORED if args.no_toeplitz else P.NF_TOEPLITZ
    # 1. the preconditioner, trained on the smaller problem's FP64 solves, on
    #    [0, T2] with h_t / h_x^2 equal to the target's (h_x ~ 1 / n on the cube)
    from workloads import CONFIGS
    ct, c2_ = CONFIGS[args.config], CONFIGS[2]
    T2 = c2_["n_steps"] * (1.0 / ct["n_steps"]) * (ct["n"] / c2_["n"]) ** 2
    v2, t2, tn2, c2, kw2, b2, _ = _dirichlet_rhs(2, P, torch, nf, T=T2)
    tv2 = P.Tree(v2, t2, tn2, P.default_params(operators=1, **kw2), device=0)
    seeds = [5 + i for i in range(max(1, args.pc_seeds))]
    pcs = []
    for sd in seeds:
        pc_i = P.Precond(device=0, features=args.pc_features, hidden=args.pc_hidden, seed=sd)
        t0 = time.perf_counter()
        loss_i = pc_i.train(tv2, b2, n_snap=16, steps=args.pc_steps, batch=4096, lr=1e-3)
        pcs.append((pc_i, loss_i, time.perf_counter() - t0))
    pc, loss, t_train = pcs[0]
    stencil = P.Precond(device=0, features=args.pc_features, hidden=0)
    t0 = time.perf_counter()
    loss_st = stencil.train(tv2, b2, n_snap=16, steps=0, batch=4096)
    t_train_st = time.perf_counter() - t0
    tv2.close()
    del b2
    log(f"[solve] preconditioner trained on {len(t2)} x {len(tn2) - 1} on [0, {T2:g}] in {t_train:.2f} s "
        f"(loss {loss:.3e}); stencil alone {t_train_st:.2f} s (fit residual {loss_st:.3e})")
    # 2. the solves on the large problem
    v, t, tn, c, kw, b, prep = _dirichlet_rhs(args.config, P, torch, nf)
    N = len(t) * (len(tn) - 1)
    t0 = time.perf_counter()
    tv = P.Tree(v, t, tn, P.default_params(operators=1, precision=P.MIXED_FP32, **kw), device=0)
    torch.cuda.synchronize()
    t_bv = time.perf_counter() - t0
    st = tv.stats()
    log(f"[solve] V tree {t_bv:.2f} s: {st}")
    tv.set_precision(P.FP64)
    w0, i0 = tv.solve_V(b, rtol=args.rtol, max_iter=args.max_iter)
    log(f"[solve] plain FP64 GMRES: {i0['iters']} iterations, {i0['seconds']:.3f} s, "
        f"true residual {i0['true_rel_residual']:.3e}")
    runs = {}
    for label, pcx, inner in (("learned_fp64", pc, P.FP64), ("learned_fp32", pc, P.MIXED_FP32),
                              ("stencil_fp32", stencil, P.MIXED_FP32), ("none_fp32", None, P.MIXED_FP32)):
        w, info = tv.solve_V_precond(b, precond=pcx, inner_precision=inner, rtol=args.rtol, max_iter=args.max_iter,
                                     raise_on_notconv=False)
        d = (torch.linalg.norm(w - w0) / torch.linalg.norm(w0)).item()
        runs[label] = dict(seconds=info["seconds"], iterations=info["iters"], refinement_steps=info["outer"],
                           converged=info["converged"], true_rel_residual=info["true_rel_residual"],
                           precond_fallback=info["precond_fallback"], rel_diff_to_plain=d)
        log(f"[solve] {label}: {info['iters']} iterations in {info['outer']} refinement steps, "
            f"{info['seconds']:.3f} s, true residual {info['true_rel_residual']:.3e}, "
            f"fallback {info['precond_fallback']}, diff to plain {d:.2e}")
        del w
    # the spread over training seeds (same data, different initial weights and minibatches)
    seed_runs = []
    for sd, (pc_i, loss_i, tr_i) in zip(seeds, pcs):
        _, info = tv.solve_V_precond(b, precond=pc_i, inner_precision=P.MIXED_FP32, rtol=args.rtol,
                                     max_iter=args.max_iter, raise_on_notconv=False)
        seed_runs.append(dict(seed=sd, loss=loss_i, iterations=info["iters"], seconds=info["seconds"],
                              true_rel_residual=info["true_rel_residual"]))
    log(f"[solve] learned_fp32 over seeds {seeds}: iterations {[r['iterations'] for r in seed_runs]}")
    # one application of the preconditioner (rms, packing, features, MLP), host-timed
    z = torch.empty_like(b)
    t_apply = {}
    for name, pcx in (("learned", pc), ("stencil", stencil)):
        pcx.apply(tv, b, out=z)
        t0 = time.perf_counter()
        for _ in range(5):
            pcx.apply(tv, b, out=z)
        t_apply[name] = 1e3 * (time.perf_counter() - t0) / 5
    log(f"[solve] preconditioner application: {t_apply}")
    del z
    # the nearfield stage of one FP64 apply on this tree (HIP events on the apply stream)
    near_roof = None
    if nf == P.NF_TOEPLITZ:
        tv.set_precision(P.FP64)
        y = tv.apply_V(b)
        tv.profile_enable(True)
        for _ in range(3):
            tv.apply_V(b, out=y)
        torch.cuda.synchronize()
        pr = tv.profile_read()
        tv.profile_enable(False)
        near_ms = pr["nearfield"][0] / max(pr["nearfield"][1], 1)
        near_roof = toeplitz_roofline(st, near_ms)
        log(f"[solve] Toeplitz nearfield of one apply: {near_roof}")
        del y
    tv.close()
    for pc_i, _, _ in pcs:
        pc_i.close()
    stencil.close()
    best = runs["learned_fp32"]
    out = {
        "metric": "Dirichlet GMRES solve time to FP64 relative residual 1e-8 (learned preconditioner, FP32 inner applies)",
        "value": best["seconds"], "unit": "s", "n_gpus": 1, "higher_is_better": False,
        "iterations": best["iterations"], "converged": best["converged"],
        "true_rel_residual": best["true_rel_residual"], "dtype": "f64 outer / f32 farfield inner",
        "data": "synthetic",
        "config": {"workload": (f"Dirichlet solve V_h w = (1/2 M_h + K_h) g, cube [-1,1]^3 {c['n']}x{c['n']} "
                                f"squares/face ({len(t)} triangles) x {c['n_steps']} steps on [0,1], g = p0 "
                                f"projection of G(x - (2.5,0,0), t + 0.1), alpha=1, m_t=m_x={c['m_t']}, "
                                f"n_max={c['n_max']}, c_st={c['c_st']}, n_tr={c['n_tr']}, "
                                f"{'Toeplitz' if nf == P.NF_TOEPLITZ else 'stored'} nearfield"),
                   "dofs": N,
                   "preconditioner": (f"least-squares stencil over 3x{args.pc_features} ring features plus a perceptron "
                                      f"3x{args.pc_features} -> {args.pc_hidden} -> {args.pc_hidden} -> 1 on its residual, "
                                      f"trained on the {len(t2)}-triangle x {len(tn2) - 1}-step Dirichlet problem "
                                      f"on [0, {T2:g}] (h_t / h_x^2 as in the solve) "
                                      f"({args.pc_steps} Adam steps of 4096 samples)")},
        "plain_fp64": dict(seconds=i0["seconds"], iterations=i0["iters"], converged=i0["converged"],
                           true_rel_residual=i0["true_rel_residual"]),
        "runs": runs, "speedup_vs_plain": i0["seconds"] / best["seconds"], "toeplitz_nearfield": near_roof,
        "train_s": t_train, "train_loss": loss, "precond_apply_ms": t_apply, "seed_runs": seed_runs,
        "stencil_train_s": t_train_st, "stencil_fit_residual": loss_st, "build_V_s": t_bv, **prep, "tree": st,
    }
    return out


def batch_bench(args):
    """48 independent cube problems (face grids 4..32, 32..512 steps, drawn
    from seed 4) applied together: one captured graph per batch apply, whose
    M2L of the levels with unequal intervals runs as one cross-problem launch
    per time offset; timed against the same applies one after another and
    against a graph of whole per-tree applies."""
    import numpy as np
    import torch
    import paper_2106_15911_amd as P
    from workloads import batch_sizes, cube_surface_mesh, uniform_time_nodes, densities
    prec = {"fp64": P.FP64, "fp32": P.MIXED_FP32, "bf16": P.MIXED_BF16}[args.precision]
    probs = []
    t0 = time.perf_counter()
    for i, (n, e) in enumerate(batch_sizes(4, 48)):
        v, t = cube_surface_mesh(n)
        probs.append((n, e, e, v, t, densities(e * len(t), 4000 + i)))
    probs.sort(key=lambda p: -p[2] * len(p[4]))     # largest first (graph branches)
    log(f"[batch] sampled and sized 48 problems in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    trees, ws = [], []
    t0 = time.perf_counter()
    for i, (n, e, ee, v, t, w) in enumerate(probs):
        prm = P.default_params(operators=1, nearfield_mode=P.NF_TOEPLITZ,
                               precision=P.MIXED_FP32 if args.precision != "fp64" else P.FP64)
        tr = P.Tree(v, t, uniform_time_nodes(ee), prm, device=0, stream=stream)
        tr.set_precision(prec)
        trees.append(tr)
        ws.append(torch.from_numpy(w).to(dev))
        if i % 8 == 7:
            log(f"[batch] built {i + 1} trees ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    N = int(sum(w.numel() for w in ws))
    mem = int(sum(tr.stats()["device_bytes"] for tr in trees))
    # one apply per tree on the stream, no graph: reference results and time
    outs_ref = [torch.empty_like(w) for w in ws]
    for tr, w, y in zip(trees, ws, outs_ref):
        tr.apply_V(w, out=y, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for tr, w, y in zip(trees, ws, outs_ref):
        tr.apply_V(w, out=y, stream=stream)
    torch.cuda.synchronize()
    ms_seq = 1e3 * (time.perf_counter() - t0)
    log(f"[batch] {N} DOFs, one apply per tree in sequence: {ms_seq:.1f} ms")
    b = P.Batch(trees)
    outs = [torch.empty_like(w) for w in ws]

    def run(cross):
        b.set_cross_m2l(cross)
        for _ in range(max(1, args.warmup)):
            b.apply_V(ws, outs, stream=stream)
        torch.cuda.synchronize()
        eq = all(bool(torch.equal(a, c)) for a, c in zip(outs, outs_ref))
        t0 = time.perf_counter()
        for _ in range(args.steps):
            b.apply_V(ws, outs, stream=stream)
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / args.steps, eq

    ms_branches, same_b = run(False)
    log(f"[batch] graph of whole applies per tree: {ms_branches:.1f} ms per batch apply; equal: {same_b}")
    ms_cross, same = run(True)
    same = same and same_b
    log(f"[batch] graph with the cross-problem M2L launch: {ms_cross:.1f} ms per batch apply; equal to single applies: "
        f"{same}")
    # the faster of the two batch forms (pfmm_batch_set_cross_m2l) is the timed configuration
    mode = "cross_problem_m2l" if ms_cross <= ms_branches else "graph_of_whole_applies"
    ms = min(ms_cross, ms_branches)
    out = {
        "metric": "space-time DOF matvec/s of pFMM V_h, 48 batched problems (aggregate)",
        "value": N / (ms * 1e-3), "unit": "DOF-matvec/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32 M2L + f64", "bf16": "bf16-input M2L + f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": ("48 independent V_h applies on cube surfaces, face grids n ~ U{4..32}, steps "
                                "E_t ~ U{32..512} from default_rng(4), as drawn (uneven time levels split at the "
                                "middle step); m_t = m_x = 6, n_max 64, c_st 0.9, n_tr 5, Toeplitz nearfield"),
                   "dofs": N, "problems": [[p[0], p[1]] for p in probs], "parallelism": "single GPU",
                   "time_classes": [tr.stats()["n_time_classes"] for tr in trees]},
        "batch_mode": mode, "sequential_ms": ms_seq, "graph_whole_applies_ms": ms_branches,
        "cross_problem_m2l_ms": ms_cross,
        "bitwise_equal_to_single_applies": same, "build_s": t_build, "device_bytes": mem,
    }
    print(json.dumps(out), flush=True)
    b.close()
    for tr in trees:
        tr.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=3,
                    help="2: 3072 x 256, 3: 3072 x 1024 (the default), 4: the 48-problem batch")
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16"], default="fp64",
                    help="farfield precision: fp64, or fp32 (M2L with FP32 inputs and accumulation; "
                         "the error against the FP64 apply on the same tree is measured and reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-toeplitz", action="store_true", help="skip the Toeplitz-nearfield measurement")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size first (HBM counter calibration)")
    ap.add_argument("--pc-features", type=int, default=8)
    ap.add_argument("--pc-hidden", type=int, default=256)
    ap.add_argument("--pc-steps", type=int, default=1500)
    ap.add_argument("--pc-seeds", type=int, default=3, help="training seeds whose solves are reported")
    ap.add_argument("--solve", action="store_true",
                    help="instead of the apply benchmark: Dirichlet solve on the 12,288 x 512 cube (config 5)")
    ap.add_argument("--no-secondary", action="store_true", help="skip the 3072 x 256 secondary measurement")
    ap.add_argument("--no-autotune", action="store_true", help="keep the built-in M2L launch choices")
    ap.add_argument("--autotune-cache", default=os.path.join(os.environ.get("TMPDIR", "/tmp"), "pfmm_autotune.json"),
                    help="JSON cache of the M2L autotuner")
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the Dirichlet solve measurement that follows the apply benchmark")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--max-iter", type=int, default=300)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(distributing time slices over GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    if args.solve:
        args.config = 5
        print(json.dumps(solve_bench(args)), flush=True)
        return
    if args.config == 4:
        batch_bench(args)
        return

    import numpy as np
    import torch
    import paper_2106_15911_amd as P
    from workloads import config_problem

    v, t, tn, c, w = config_problem(args.config)
    N = len(w)
    mixed = args.precision != "fp64"
    # the tree holds both farfield paths; the timed one is selected with set_precision
    prm = P.default_params(m_t=c["m_t"], m_x=c["m_x"], n_max=c["n_max"], c_st=c["c_st"], n_tr=c["n_tr"],
                           operators=1, precision=P.MIXED_FP32)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    t0 = time.perf_counter()
    tree = P.Tree(v, t, tn, prm, device=0, stream=stream)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    st = tree.stats()
    log(f"[bench] built config {args.config}: {st} in {t_build:.2f} s")
    tune = None
    if not args.no_autotune:
        t0 = time.perf_counter()
        n_t, n_c = tree.autotune(args.autotune_cache, stream=stream)
        tune = {"levels_timed": n_t, "levels_cached": n_c, "seconds": time.perf_counter() - t0,
                "cache": args.autotune_cache}
        log(f"[bench] autotune: {tune}")
    if args.copy_calibration_mib:
        n = args.copy_calibration_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: {8 * n} bytes read, {8 * n} bytes written")
        del a, b
    x = torch.from_numpy(w).to(dev)

    def timed(precision, steps, warmup):
        """warmup untimed applies, then `steps` applies bracketed by device
        synchronisation (in Toeplitz mode the nearfield runs beside the
        farfield chain); then
        stage times from HIP events on the apply stream over max(3, steps / 4)
        further applies, whose stages the library runs one after another
        while timing them"""
        tree.set_precision(precision)
        out = torch.empty_like(x)
        for _ in range(warmup):
            tree.apply_V(x, out=out, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            tree.apply_V(x, out=out, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tree.profile_enable(True)
        n_prof = max(3, steps // 4)
        t1 = time.perf_counter()
        for _ in range(n_prof):
            tree.apply_V(x, out=out, stream=stream)
        torch.cuda.synchronize()
        dt_serial = time.perf_counter() - t1
        pr = tree.profile_read()
        tree.profile_enable(False)
        pr["serial_apply_ms"] = (1e3 * dt_serial / n_prof, 1)
        return out, 1e3 * dt / steps, pr

    # timed region: the selected precision
    f, ms_per_step, prof = timed({"fp64": P.FP64, "fp32": P.MIXED_FP32, "bf16": P.MIXED_BF16}[args.precision],
                                 args.steps, args.warmup)
    log(f"[bench] {args.steps} applies ({args.precision}): {ms_per_step:.3f} ms/apply; stages {prof}")
    # the other farfield precisions on the same tree, with their measured error against FP64
    import numpy as np
    names = {"fp64": P.FP64, "fp32": P.MIXED_FP32, "bf16": P.MIXED_BF16}
    outs = {args.precision: f.cpu().numpy()}
    other_precision = {}
    for name, code in names.items():
        if name == args.precision:
            continue
        g, ms_o, prof_o = timed(code, max(3, args.steps // 2), 1)
        outs[name] = g.cpu().numpy()
        other_precision[name] = {"ms_per_step": ms_o, "value": N / (ms_o * 1e-3),
                                 "m2l_ms": prof_o["m2l"][0] / max(prof_o["m2l"][1], 1)}
    fd = outs["fp64"]
    for name in ("fp32", "bf16"):
        e = {"rel_2norm_vs_fp64": float(np.linalg.norm(outs[name] - fd) / np.linalg.norm(fd)),
             "rel_max_vs_fp64": float(np.abs(outs[name] - fd).max() / np.abs(fd).max())}
        if name in other_precision:
            other_precision[name]["error"] = e
        if name == args.precision:
            mixed_err = e
    if args.precision == "fp64":
        mixed_err = None
    other_precision["note"] = ("fp32: M2L with FP32 moments/operator entries and FP32 matrix-core accumulation; "
                               "bf16: the same with moments, table and operator entries rounded to bfloat16 and "
                               "multiplied on the BF16 matrix cores (FP32 accumulation); everything else FP64")
    log(f"[bench] other precisions: {other_precision}")
    tree.set_precision(names[args.precision])
    # the same product with the Toeplitz nearfield (no stored blocks), on a tree of its own
    toeplitz = None
    if not args.no_toeplitz:
        prm_t = P.default_params(m_t=c["m_t"], m_x=c["m_x"], n_max=c["n_max"], c_st=c["c_st"], n_tr=c["n_tr"],
                                 operators=1, precision=P.MIXED_FP32, nearfield_mode=P.NF_TOEPLITZ)
        tt = P.Tree(v, t, tn, prm_t, device=0, stream=stream)
        tt.set_precision({"fp64": P.FP64, "fp32": P.MIXED_FP32, "bf16": P.MIXED_BF16}[args.precision])
        ft = torch.empty_like(x)
        for _ in range(max(1, args.warmup)):
            tt.apply_V(x, out=ft, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nt = max(3, args.steps // 2)
        for _ in range(nt):
            tt.apply_V(x, out=ft, stream=stream)
        torch.cuda.synchronize()
        ms_t = 1e3 * (time.perf_counter() - t0) / nt
        tt.profile_enable(True)
        for _ in range(3):
            tt.apply_V(x, out=ft, stream=stream)
        torch.cuda.synchronize()
        pt = tt.profile_read()
        toeplitz = {"ms_per_step": ms_t, "value": N / (ms_t * 1e-3),
                    "nearfield_ms": pt["nearfield"][0] / max(pt["nearfield"][1], 1),
                    "roofline": toeplitz_roofline(tt.stats(), pt["nearfield"][0] / max(pt["nearfield"][1], 1)),
                    "device_bytes": tt.stats()["device_bytes"], "max_rel_diff_to_stored": float((ft - f).abs().max() / f.abs().max()),
                    "rel_2norm_diff_to_stored": float(torch.linalg.norm(ft - f) / torch.linalg.norm(f)),
                    "near_gemm_groups": tt.stats()["near_gemm_groups"],
                    "note": "nearfield entries read from the distinct integrals per (leaf spatial box, step "
                            "difference) instead of stored blocks (uniform steps); boxes whose leaves are time "
                            "translates run as GEMMs on the FP64 matrix cores"}
        if args.precision == "fp64":
            # the FP32 farfield with this nearfield, error against the FP64 stored-mode apply
            tt.set_precision(P.MIXED_FP32)
            tt.profile_enable(False)
            for _ in range(max(1, args.warmup)):
                tt.apply_V(x, out=ft, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(nt):
                tt.apply_V(x, out=ft, stream=stream)
            torch.cuda.synchronize()
            ms_t32 = 1e3 * (time.perf_counter() - t0) / nt
            fo, f64 = ft.cpu().numpy(), f.cpu().numpy()
            toeplitz["fp32"] = {"ms_per_step": ms_t32, "value": N / (ms_t32 * 1e-3),
                                "error": {"rel_2norm_vs_fp64": float(np.linalg.norm(fo - f64) / np.linalg.norm(f64)),
                                          "rel_max_vs_fp64": float(np.abs(fo - f64).max() / np.abs(f64).max())}}
        tt.close()
        log(f"[bench] toeplitz nearfield: {toeplitz}")

    # the metric's "at 1e-6 rel err": the fastest configuration (farfield
    # precision, nearfield mode) whose measured relative 2-norm error against
    # the FP64 stored-mode apply stays within 1e-6
    cands = [("fp64", "stored", N / (ms_per_step * 1e-3) if args.precision == "fp64" else other_precision["fp64"]["value"], 0.0)]
    for name in ("fp32", "bf16"):
        e = (other_precision[name]["error"] if name in other_precision else mixed_err)["rel_2norm_vs_fp64"]
        val = other_precision[name]["value"] if name in other_precision else N / (ms_per_step * 1e-3)
        if e <= 1e-6:
            cands.append((name, "stored", val, e))
    if toeplitz is not None and args.precision == "fp64":
        cands.append(("fp64", "toeplitz", toeplitz["value"], toeplitz["rel_2norm_diff_to_stored"]))
        e = toeplitz["fp32"]["error"]["rel_2norm_vs_fp64"]
        if e <= 1e-6:
            cands.append(("fp32", "toeplitz", toeplitz["fp32"]["value"], e))
    best = max(cands, key=lambda q: q[2])
    at_1e6 = {"precision": best[0], "nearfield": best[1], "value": best[2], "unit": "DOF-matvec/s",
              "rel_2norm_vs_fp64": best[3]}

    # roofline of the dominant kernel
    near_ms = prof["nearfield"][0] / max(prof["nearfield"][1], 1)
    m2l_ms = prof["m2l"][0] / max(prof["m2l"][1], 1)
    near_bytes = 8.0 * st["near_entries"] + 16.0 * N
    # algorithmic FLOP of eq. m2l: 2 (m_t+1)^2 C(m_x+6, 6) per interaction pair
    from math import comb
    m2l_flop = 2.0 * (c["m_t"] + 1) ** 2 * comb(c["m_x"] + 6, 6) * st["m2l_pairs"]
    if near_ms >= m2l_ms:
        achieved = near_bytes / (near_ms * 1e-3) / 1e9
        roof = {"kernel": "k_near_apply", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("k_near_apply", args.config),
                "launch_ms": near_ms, "algorithmic_bytes": near_bytes}
    else:
        achieved = m2l_flop / (m2l_ms * 1e-3) / 1e12
        peak = FP32_PEAK_TFS if mixed else FP64_PEAK_TFS
        roof = {"kernel": ("M2L stage: k_m2l_wide + k_m2l_mfma (all levels)" if st["m2l_matrix_cores"] == 1
                           else "k_m2l (all levels)"),
                "bound": "mfma" if st["m2l_matrix_cores"] == 1 else "alu", "achieved": achieved, "peak": peak,
                "unit": "TFLOP/s", "frac": achieved / peak,
                "traffic": (measured_traffic("m2l", args.config, args.precision)
                            if st["m2l_matrix_cores"] == 1 else None),
                "launch_ms": m2l_ms, "algorithmic_flop": m2l_flop}
    roof["traffic_note"] = "HBM bytes per apply, all launches of the kernel (rocprofv3 counters, copy-calibrated)"
    other = {"nearfield": {"ms": near_ms, "GB/s": near_bytes / (near_ms * 1e-3) / 1e9,
                           "traffic": measured_traffic("k_near_apply", args.config)},
             "m2l": {"ms": m2l_ms, "TFLOP/s": m2l_flop / (m2l_ms * 1e-3) / 1e12}}

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.config, w, st["distinct_integrals"])
        log(f"[bench] cpu baseline: {cpu}")

    out = {
        "metric": METRIC,
        "value": N / (ms_per_step * 1e-3),
        "unit": "DOF-matvec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32 M2L + f64", "bf16": "bf16-input M2L + f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": (f"V_h apply, cube [-1,1]^3 {c['n']}x{c['n']} squares/face ({len(t)} triangles) x "
                                f"{c['n_steps']} uniform steps on [0,1], alpha=1, m_t={c['m_t']}, m_x={c['m_x']}, "
                                f"n_max={c['n_max']}, c_st={c['c_st']}, n_tr={c['n_tr']}, "
                                + {"fp64": "FP64", "fp32": "M2L in FP32 (inputs and accumulation), rest FP64",
                                   "bf16": "M2L with BF16 inputs and FP32 accumulation, rest FP64"}[args.precision]),
                   "dofs": N, "parallelism": "single GPU", "precision": args.precision},
        "mixed_error": mixed_err,
        "at_1e-6_rel_err": at_1e6,
        "other_precision": other_precision,
        "toeplitz_nearfield": toeplitz,
        "roofline": roof,
        "other_kernels": other,
        "stages_ms_per_apply": {k: (vv[0] / max(vv[1], 1)) for k, vv in prof.items()},
        "build_s": t_build,
        "autotune": tune,
        "tree": st,
        "cpu_baseline": cpu,
    }
    tree.close()
    del x
    torch.cuda.empty_cache()
    if args.config == 3 and not args.no_secondary:
        # the 3072 x 256 workload (FP64, stored nearfield) as a secondary figure
        v2, t2, tn2, c2, w2 = config_problem(2)
        prm2 = P.default_params(m_t=c2["m_t"], m_x=c2["m_x"], n_max=c2["n_max"], c_st=c2["c_st"],
                                n_tr=c2["n_tr"], operators=1)
        tree2 = P.Tree(v2, t2, tn2, prm2, device=0, stream=stream)
        if not args.no_autotune:
            tree2.autotune(args.autotune_cache, stream=stream)
        x2 = torch.from_numpy(w2).to(dev)
        y2 = torch.empty_like(x2)
        for _ in range(max(1, args.warmup)):
            tree2.apply_V(x2, out=y2, stream=stream)
        torch.cuda.synchronize()
        n2 = max(3, args.steps // 2)
        t0 = time.perf_counter()
        for _ in range(n2):
            tree2.apply_V(x2, out=y2, stream=stream)
        torch.cuda.synchronize()
        ms2 = 1e3 * (time.perf_counter() - t0) / n2
        tree2.profile_enable(True)
        for _ in range(3):
            tree2.apply_V(x2, out=y2, stream=stream)
        torch.cuda.synchronize()
        p2 = tree2.profile_read()
        st2 = tree2.stats()
        m2l2 = p2["m2l"][0] / max(p2["m2l"][1], 1)
        nf2 = p2["nearfield"][0] / max(p2["nearfield"][1], 1)
        flop2 = 2.0 * (c2["m_t"] + 1) ** 2 * comb(c2["m_x"] + 6, 6) * st2["m2l_pairs"]
        out["secondary"] = {
            "workload": f"V_h apply, FP64, {len(t2)} triangles x {c2['n_steps']} steps (cube 16x16 squares/face), "
                        f"m_t = m_x = 6, stored nearfield", "dofs": len(w2), "ms_per_step": ms2,
            "value": len(w2) / (ms2 * 1e-3), "m2l_ms": m2l2, "m2l_frac_fp64_peak": flop2 / (m2l2 * 1e-3) / 1e12 / FP64_PEAK_TFS,
            "nearfield_ms": nf2, "nearfield_GBs": (8.0 * st2["near_entries"] + 16.0 * len(w2)) / (nf2 * 1e-3) / 1e9,
            "stages_ms_per_apply": {k: (vv[0] / max(vv[1], 1)) for k, vv in p2.items()}}
        log(f"[bench] secondary: {out['secondary']}")
        tree2.close()
        del x2, y2
        torch.cuda.empty_cache()
    if not args.no_solve:
        # the second half of the metric: GMRES time to solution, learned
        # preconditioner + FP32 inner applies against plain FP64 GMRES
        sargs = argparse.Namespace(**vars(args))
        sargs.config = 5
        sv = solve_bench(sargs)
        out["solve"] = {k: sv[k] for k in ("metric", "value", "unit", "iterations", "converged", "true_rel_residual",
                                           "plain_fp64", "speedup_vs_plain", "runs", "seed_runs", "train_s",
                                           "precond_apply_ms", "toeplitz_nearfield", "config")}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
