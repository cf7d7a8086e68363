"""Benchmark: space-time DOF-matvecs/s of the pFMM single-layer apply on one MI355X.

Workload: the surface of the cube [-1,1]^3 with 16 x 16 squares per face
(3072 triangles) x 256 uniform steps on [0, 1] (786,432 space-time DOFs),
alpha = 1, Chebyshev degree 6 in space, Lagrange degree 6 in time, leaves
below 64 elements, c_st = 0.9, n_tr = 5, FP64 everywhere; densities i.i.d.
U(-1, 1) from seed 2.  A step is one full V_h apply (Algorithm 2) from a
device-resident density to a device-resident result; tree build and
nearfield assembly happen before the timed region and are reported apart.

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

# HBM bytes per apply from rocprofv3 FETCH_SIZE / WRITE_SIZE runs on the
# 3072 x 256, m = 6 workload (FP64 farfield), scaled by the same counters on a
# plain 1 GiB device copy (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000).  Each entry
# is valid only for the sources it was taken on (sha256 prefixes of the
# kernel file and of the file that plans and launches it); any change to
# them reports null.
TRAFFIC = {
    "m2l": {"files": {"m2l_kernels.hpp": "e38d10d4f4c24a9f", "pfmm.hip": "fd115eecd436e06d"}, "config": 2,
            "precision": "fp64", "bytes": 39160588288.0},
    "k_near_apply": {"files": {"near_apply.hpp": "874d6bbd4da69cef", "pfmm.hip": "fd115eecd436e06d"}, "config": 2,
                     "bytes": 53940300800.0},
}


def measured_traffic(kernel, cfg, precision="fp64"):
    """HBM bytes per apply from the rocprofv3 counters, while the sources the
    counters were taken on (kernel and launch configuration) are unchanged."""
    import hashlib
    e = TRAFFIC.get(kernel)
    if e is None or e["bytes"] is None or e["config"] != cfg or e.get("precision", precision) != precision:
        return None
    for name, prefix in e["files"].items():
        with open(os.path.join(ROOT, "paper_2106_15911_amd", "csrc", name), "rb") as fh:
            if hashlib.sha256(fh.read()).hexdigest()[:16] != prefix:
                return None
    return e["bytes"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(cfg, w, per_level=12, leaves=12, seed=123):
    """The CPU oracle's full V_h apply, timed on a bounded sample and scaled.

    The oracle's apply is a loop over boxes: moments of every box (timed in
    full), then per level the M2L and L2L of each box, then per leaf the L2T
    and the nearfield blocks.  A random sample of boxes per level and of
    leaves is timed and scaled by the number of boxes.
    """
    import numpy as np
    from oracle.fmm import FMMOracle
    from oracle.tree import Tree
    from workloads import config_problem
    v, t, tn, c, _ = config_problem(cfg)
    rng = np.random.default_rng(seed)
    t0 = time.perf_counter()
    tr = Tree(v, t, tn, 1.0, c["n_max"], c["c_st"], c["n_tr"])
    o = FMMOracle(tr, c["m_t"], c["m_x"], "V")
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
    pick = rng.choice(len(tr.leaves), leaves, replace=False)
    memo = {}
    t0 = time.perf_counter()
    for i in pick:
        Z = tr.leaves[int(i)]
        rows = tr.elements(Z)
        f = o.l2t(Z, np.zeros((c["m_t"] + 1, o.Nk))).ravel()
        for S in tr.nearfield(Z, memo):
            f = f + o.near_block(Z, S) @ w[tr.elements(S)]
    dt = time.perf_counter() - t0
    timed += dt
    est += dt * len(tr.leaves) / leaves
    N = len(w)
    try:
        from threadpoolctl import threadpool_info
        blas = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        blas = 1
    return {"value": N / est, "unit": "DOF-matvec/s", "cores": int(blas), "kind": "oracle",
            "sample": (f"oracle V_h apply on {N} DOFs: tree + all moments ({t_up:.1f} s) in full; M2L+L2L of "
                       f"{n_far} sampled boxes (up to {per_level} per level) and L2T+nearfield of {leaves} "
                       f"sampled leaves ({timed - t_up:.1f} s), scaled by box counts; estimated full apply "
                       f"{est:.0f} s"),
            "timed_s": timed, "host_cpus": os.cpu_count()}


def oracle_rows(cfg, w, rows, seed=123):
    """Sampled rows of the oracle product for an accuracy check of the timed result."""
    import numpy as np
    from oracle.fmm import FMMOracle
    from oracle.tree import Tree
    from workloads import config_problem
    v, t, tn, c, _ = config_problem(cfg)
    tr = Tree(v, t, tn, 1.0, c["n_max"], c["c_st"], c["n_tr"])
    o = FMMOracle(tr, c["m_t"], c["m_x"], "V")
    sample = np.random.default_rng(seed).choice(len(w), rows, replace=False)
    vals, _ = o.apply_rows(w, sample)
    return sample, vals


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
        "runs": runs, "speedup_vs_plain": i0["seconds"] / best["seconds"],
        "train_s": t_train, "train_loss": loss, "precond_apply_ms": t_apply, "seed_runs": seed_runs,
        "stencil_train_s": t_train_st, "stencil_fit_residual": loss_st, "build_V_s": t_bv, **prep, "tree": st,
    }
    print(json.dumps(out), flush=True)


def supported_steps(v, t, e, P):
    """The step count of the batched workload's problem: the supported count
    nearest to the drawn E_t (ties to the larger).  Supported: the time
    levels of the tree split evenly (equal intervals per level) and no leaf
    holds more than 64 triangles (a time interval of one step is not
    refined further, so coarse steps on a fine mesh can leave large leaves)."""
    from workloads import uniform_time_nodes
    for dist in range(0, 4 * e):
        for ee in (e + dist, e - dist):
            if ee < 8 or (dist == 0 and ee != e + dist) or ee % 8:
                continue
            try:
                P.plan_stats(v, t, uniform_time_nodes(ee), P.default_params(operators=1))
                return ee
            except P.PfmmError:
                continue
    raise RuntimeError(f"no supported step count near {e}")


def batch_bench(args):
    """48 independent cube problems (face grids 4..32, 32..512 steps, drawn
    from seed 4) applied together: one captured graph per batch apply."""
    import numpy as np
    import torch
    import paper_2106_15911_amd as P
    from workloads import batch_sizes, cube_surface_mesh, uniform_time_nodes, densities
    prec = {"fp64": P.FP64, "fp32": P.MIXED_FP32, "bf16": P.MIXED_BF16}[args.precision]
    probs = []
    t0 = time.perf_counter()
    for i, (n, e) in enumerate(batch_sizes(4, 48)):
        v, t = cube_surface_mesh(n)
        ee = supported_steps(v, t, e, P)
        probs.append((n, e, ee, v, t, densities(ee * len(t), 4000 + i)))
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
    for _ in range(max(1, args.warmup)):
        b.apply_V(ws, outs, stream=stream)
    torch.cuda.synchronize()
    same = all(bool(torch.equal(a, c)) for a, c in zip(outs, outs_ref))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        b.apply_V(ws, outs, stream=stream)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / args.steps
    log(f"[batch] batched (captured graph): {ms:.1f} ms per batch apply; equal to single applies: {same}")
    out = {
        "metric": "space-time DOF matvec/s of pFMM V_h, 48 batched problems (aggregate)",
        "value": N / (ms * 1e-3), "unit": "DOF-matvec/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32 M2L + f64", "bf16": "bf16-input M2L + f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": ("48 independent V_h applies on cube surfaces, face grids n ~ U{4..32}, steps "
                                "E_t ~ U{32..512} from default_rng(4), E_t rounded to the nearest multiple of 2^k "
                                "whose time levels split evenly; m_t = m_x = 6, n_max 64, c_st 0.9, n_tr 5, "
                                "Toeplitz nearfield"),
                   "dofs": N, "problems": [[p[0], p[1], p[2]] for p in probs], "parallelism": "single GPU"},
        "sequential_ms": ms_seq, "bitwise_equal_to_single_applies": same, "build_s": t_build, "device_bytes": mem,
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
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16"], default="fp64",
                    help="farfield precision: fp64, or fp32 (M2L with FP32 inputs and accumulation; "
                         "the error against the FP64 apply on the same tree is measured and reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-toeplitz", action="store_true", help="skip the Toeplitz-nearfield measurement")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size first (HBM counter calibration)")
    ap.add_argument("--check-rows", type=int, default=0, help="compare this many sampled rows with the oracle")
    ap.add_argument("--pc-features", type=int, default=8)
    ap.add_argument("--pc-hidden", type=int, default=256)
    ap.add_argument("--pc-steps", type=int, default=1500)
    ap.add_argument("--pc-seeds", type=int, default=3, help="training seeds whose solves are reported")
    ap.add_argument("--solve", action="store_true",
                    help="instead of the apply benchmark: Dirichlet solve on the 12,288 x 512 cube (config 5)")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--max-iter", type=int, default=300)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(distributing time slices over GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    if args.solve:
        if args.config == 2:
            args.config = 5
        solve_bench(args)
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
                               "bf16: the same with moments, table and operator entries rounded to bfloat16 "
                               "(exact products, FP32 accumulation); everything else FP64")
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
                    "device_bytes": tt.stats()["device_bytes"], "max_rel_diff_to_stored": float((ft - f).abs().max() / f.abs().max()),
                    "near_gemm_groups": tt.stats()["near_gemm_groups"],
                    "note": "nearfield entries read from the distinct integrals per (leaf spatial box, step "
                            "difference) instead of stored blocks (uniform steps); boxes whose leaves are time "
                            "translates run as GEMMs on the FP64 matrix cores"}
        tt.close()
        log(f"[bench] toeplitz nearfield: {toeplitz}")

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

    check = None
    if args.check_rows:
        sample, vals = oracle_rows(args.config, w, args.check_rows)
        fg = f.cpu().numpy()
        err = float(np.abs(fg[sample] - vals).max() / np.abs(vals).max())
        check = {"rows": int(args.check_rows), "max_rel_err_vs_oracle": err}
        log(f"[bench] oracle rows check: {check}")
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args.config, w)
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
        "other_precision": other_precision,
        "toeplitz_nearfield": toeplitz,
        "roofline": roof,
        "other_kernels": other,
        "stages_ms_per_apply": {k: (vv[0] / max(vv[1], 1)) for k, vv in prof.items()},
        "build_s": t_build,
        "tree": st,
        "oracle_check": check,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    tree.close()


if __name__ == "__main__":
    main()
