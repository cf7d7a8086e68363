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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(cfg, rows, w):
    """The CPU oracle on a bounded sample: full upward pass plus `rows` rows."""
    import numpy as np
    from oracle.fmm import FMMOracle
    from oracle.tree import Tree
    from workloads import config_problem
    v, t, tn, c, _ = config_problem(cfg)
    t0 = time.perf_counter()
    tr = Tree(v, t, tn, 1.0, c["n_max"], c["c_st"], c["n_tr"])
    o = FMMOracle(tr, c["m_t"], c["m_x"], "V")
    mu = o.moments(w)
    t_up = time.perf_counter() - t0
    rng = np.random.default_rng(123)
    sample = rng.choice(len(w), rows, replace=False)
    t0 = time.perf_counter()
    vals, _ = o.apply_rows(w, sample, mu)
    t_rows = time.perf_counter() - t0
    N = len(w)
    est = t_up + t_rows * N / rows
    try:
        from threadpoolctl import threadpool_info
        blas = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    except Exception:
        blas = 1
    return {"value": N / est, "unit": "DOF-matvec/s", "cores": int(blas), "kind": "oracle",
            "sample": (f"tree + upward pass ({t_up:.1f} s) + {rows} random rows of V_h w "
                       f"({t_rows:.1f} s), extrapolated to all {N} rows"),
            "host_cpus": os.cpu_count()}, sample, vals


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=4)
    ap.add_argument("--check-rows", type=int, default=0, help="compare this many sampled rows with the oracle")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the time-slice distribution across GPUs is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2106_15911_amd as P
    from workloads import config_problem

    v, t, tn, c, w = config_problem(args.config)
    N = len(w)
    prm = P.default_params(m_t=c["m_t"], m_x=c["m_x"], n_max=c["n_max"], c_st=c["c_st"], n_tr=c["n_tr"],
                           operators=1)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    t0 = time.perf_counter()
    tree = P.Tree(v, t, tn, prm, device=0, stream=stream)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t0
    st = tree.stats()
    log(f"[bench] built config {args.config}: {st} in {t_build:.2f} s")
    x = torch.from_numpy(w).to(dev)
    f = torch.empty_like(x)
    for _ in range(args.warmup):
        tree.apply_V(x, out=f, stream=stream)
    torch.cuda.synchronize()
    # timed region
    tree.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        tree.apply_V(x, out=f, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = tree.profile_read()
    tree.profile_enable(False)
    ms_per_step = 1e3 * dt / args.steps
    log(f"[bench] {args.steps} applies: {ms_per_step:.3f} ms/apply; stages {prof}")

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
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                "launch_ms": near_ms, "algorithmic_bytes": near_bytes}
    else:
        achieved = m2l_flop / (m2l_ms * 1e-3) / 1e12
        roof = {"kernel": "k_m2l (all levels)", "bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFS,
                "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFS, "traffic": None,
                "launch_ms": m2l_ms, "algorithmic_flop": m2l_flop}
    other = {"nearfield": {"ms": near_ms, "GB/s": near_bytes / (near_ms * 1e-3) / 1e9},
             "m2l": {"ms": m2l_ms, "TFLOP/s": m2l_flop / (m2l_ms * 1e-3) / 1e12}}

    check = None
    cpu = None
    if not args.no_cpu_baseline or args.check_rows:
        rows = max(args.cpu_rows, args.check_rows)
        cpu, sample, vals = cpu_baseline(args.config, rows, w)
        fg = f.cpu().numpy()
        err = float(np.abs(fg[sample] - vals).max() / np.abs(vals).max())
        check = {"rows": int(rows), "max_rel_err_vs_oracle": err}
        log(f"[bench] oracle rows check: {check}")
        if args.no_cpu_baseline:
            cpu = None

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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"V_h apply, cube [-1,1]^3 {c['n']}x{c['n']} squares/face ({len(t)} triangles) x "
                                f"{c['n_steps']} uniform steps on [0,1], alpha=1, m_t={c['m_t']}, m_x={c['m_x']}, "
                                f"n_max={c['n_max']}, c_st={c['c_st']}, n_tr={c['n_tr']}, FP64"),
                   "dofs": N, "parallelism": "single GPU"},
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
