"""Benchmark: DD-alpha-AMG time to solution on one MI355X.

Workload (default): the 24^3 x 48 precision-form case - synthetic links
(spread 0.25), c_sw = 1.6, mu = 0.0015, 3-level DD-alpha-AMG (4^4 then 2^4
aggregates, N_v = 24/32, SAP 4^4 / 3^4 with 4 MR steps, 3 setup
iterations), FP32 stencil/SAP with bf16 P and D_c, FP64 outer FGMRES with
reliable updates, one Gaussian right-hand side solved to relative residual
1e-10.  A step is one full job: setup (link conversion, clover, adaptive
setup) plus the solve.  The plain FP64 DD-alpha-AMG on the same GPU is
timed alongside for the speed-up, and the fine stencil's HBM roofline is
measured with HIP events on the library's stream.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c2]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "dslash_fp32_c2_traffic.md")
STENCIL_SOURCES = ("fine_op.hip", "su3.h", "common.h")


def stencil_traffic(workload_name):
    """HBM bytes per stencil launch from the committed counter record
    (FETCH_SIZE and WRITE_SIZE, scaled by a copy kernel's readings), or
    None when the record is for another workload or the stencil sources
    changed since the counters were taken."""
    import hashlib
    if workload_name != "c2" or not os.path.exists(TRAFFIC_RECORD):
        return None
    rec = None
    for line in open(TRAFFIC_RECORD):
        if line.startswith("traffic_record:"):
            rec = json.loads(line.split(":", 1)[1])
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in STENCIL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1710_06198_amd", "csrc", f), "rb").read())
    if h.hexdigest()[:16] != rec["source_sha16"]:
        return None
    return rec["bytes_per_launch"]


MFMA_BF16_PEAK_TFS = 2500.0   # MI355X dense bf16 matrix peak


def batched_coarse(tm, solver, reps):
    """The level-1 coarse operator with 16 right-hand sides (one workgroup
    per coarse site, 16 RHS on the matrix cores) timed with HIP events.
    Executed MFMA work per launch: sites x 9 blocks x d^2 x 16 RHS complex
    products, each as 4 real products on a 2-part bf16 split of the FP32
    input, i.e. 16 flops per complex product (the useful complex arithmetic
    is half of that)."""
    nrhs = 16
    vc, d = solver.level_info(1)
    ms = solver.time_kernel(tm.K_DC1, nrhs, reps)
    sap_ms = solver.time_kernel(tm.K_SAP1, nrhs, max(2, reps // 4))
    flops = vc * 9 * d * d * nrhs * 16
    tfs = flops / (ms * 1e-3) / 1e12
    return {"kernel": f"k_coarse_apply_mf<{d}>", "rhs": nrhs, "sites": vc, "d": d, "ms": round(ms, 4),
            "flops_per_launch": flops, "achieved": round(tfs, 2), "peak": MFMA_BF16_PEAK_TFS, "unit": "TFLOP/s",
            "frac": round(tfs / MFMA_BF16_PEAK_TFS, 4), "sap1_sweep_16rhs_ms": round(sap_ms, 4)}


def autotune(tm, solver, counts, args):
    """Kernel variant tuning before the timed region: the library times
    both variants of every tunable family at these right-hand-side counts on
    the solver's own hierarchy and keeps the faster (process-wide table).
    --tune-cache loads a table written earlier instead, or saves this one."""
    import tempfile
    if args.tune_cache and os.path.exists(args.tune_cache):
        n = tm.tune_load(args.tune_cache)
        log(f"[bench] variant table: {n} entries from {args.tune_cache}")
        path = args.tune_cache
    else:
        fd, path = tempfile.mkstemp(suffix=".json")
        os.close(fd)
        t0 = time.perf_counter()
        solver.autotune(sorted(set(counts)), reps=3, json_path=path)
        log(f"[bench] autotune {sorted(set(counts))} in {time.perf_counter() - t0:.1f} s")
        if args.tune_cache:
            tm.tune_save(args.tune_cache)
    with open(path) as f:
        entries = json.load(f)["entries"]
    if not args.tune_cache:
        os.remove(path)
    for e in entries:
        log(f"[bench]   {e['family']} {e['shape']} -> {e['variant']} {e['ms']}")
    return entries


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def solver_params(tm, w, precision, graph=0):
    """The workload's hierarchy.  With three levels the intermediate FGMRES
    takes at most 6 steps and the coarsest GMRES at most 10: sweeps on the
    24^3 x 48 job (intermediate 3-15, coarsest 10-70 steps) moved the outer
    iteration count only between 14 and 26 while the coarse solves got
    several times cheaper (14 outer iterations at 10/50, 17 at 6/10).  Both
    precisions use the same hierarchy, so the FP64 comparison solver gets
    the same saving.  graph=1 replays the intermediate-level solve of each
    fine cycle from a captured HIP graph (mixed precision only; the plain FP64
    solver is the eager one)."""
    p = dict(nlevels=w.nlevels, agg=w.agg, nv=w.nv, setup_iters=w.setup_iters, init_smooth=w.init_smooth,
             sap_sweeps=w.sap_sweeps, mr_steps=w.mr_steps, restart=w.restart, precision=precision,
             storage=tm.STORE_BF16, coarsest_iters=10 if w.nlevels == 3 else 100,
             l2_iters=6 if w.nlevels == 3 else 10, use_graph=graph if precision == tm.MIXED else 0)
    if w.nlevels == 3:
        p["sap_block1"] = w.sap_block[1]
    return tm.default_params(**p)


def cpu_baseline(w, m0, budget_dims=(8, 8, 8, 8)):
    """The oracle (FP64 DD-alpha-AMG, torch-CPU) on an 8^4 lattice drawn with
    the workload's link spread, c_sw, mu and hierarchy; setup + solve time
    scaled by the volume ratio to the workload's lattice."""
    import torch
    from lattice_inputs import gauge_links, gaussian_spinor
    from oracle.dirac import WilsonClover, spinor_to_field, norm
    from oracle import mg
    U = gauge_links(budget_dims, w.eps, w.seeds["links"])
    op = WilsonClover(U, m0, w.csw)
    b = spinor_to_field(gaussian_spinor(budget_dims, w.seeds["source"])[0])
    sap = [w.sap_block[0]] + [tuple(min(a, l) for a, l in zip(w.sap_block[1], (1, 1, 1, 1)))]
    p = mg.MGParams(nlevels=w.nlevels, agg=w.agg, nv=w.nv, sap_block=tuple(sap[:w.nlevels - 1] or sap),
                    setup_iters=w.setup_iters, mr_steps=w.mr_steps, init_smooth=w.init_smooth)
    t0 = time.time()
    H = mg.Hierarchy(op, p, w.mu)
    H.setup(mg.setup_vectors(p, budget_dims, w.seeds["testvec"]))
    t1 = time.time()
    r = H.solve(b, w.tol, restart=w.restart)
    t2 = time.time()
    vol = 1
    for d in budget_dims:
        vol *= d
    scale = w.volume / vol
    res = norm(b - op.apply(r.x, w.mu)) / norm(b)
    return {
        "value": (t2 - t0) * scale,
        "unit": "s",
        "cores": torch.get_num_threads(),
        "kind": "oracle",
        "sample": (f"oracle setup+solve at {'x'.join(map(str, budget_dims))} with the workload's spread, c_sw, mu "
                   f"and hierarchy ({t1 - t0:.1f} s setup + {t2 - t1:.1f} s solve, {r.iters} iterations, "
                   f"residual {res:.1e}), scaled by the volume ratio {scale:.0f}"),
        "cpu_model": _cpu_model(),
        "os_cpu_count": os.cpu_count(),
    }


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _timed(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def bench_batched(args):
    """32^3 x 64: 12 spin-colour point sources at random sites solved as one
    batch of D(mu) x = b, plus 8 shifted systems (D D^dag + sigma_k) x = b
    (sigma_k log-spaced in [1e-5, 1]) on one Gaussian source as a second
    batch (two-step solves with mu' = sqrt(mu^2 + sigma)), mixed precision
    against the plain FP64 DD-alpha-AMG.  Restart 12 bounds the Krylov
    memory of 12-wide batches."""
    import torch
    import paper_1710_06198_amd as tm
    from lattice_inputs import workload, gauge_links, gaussian_spinor, point_sources, rational_shifts, load_m0
    w = workload("c3")
    m0 = load_m0()[w.name]
    kappa = 1.0 / (2 * m0 + 8)
    dev = torch.device("cuda:0")
    log(f"[bench] workload c3 dims {w.dims}: generating inputs")
    U = torch.as_tensor(gauge_links(w.dims, w.eps, w.seeds["links"])).to(dev)
    npt, nsh = w.extra["n_point"], w.extra["n_shift"]
    bp = torch.as_tensor(point_sources(w.dims, w.seeds["source"], npt)).to(dev)
    g1 = torch.as_tensor(gaussian_spinor(w.dims, w.seeds["source"] + 100, n=1)).to(dev)
    bs = g1.expand(nsh, *g1.shape[1:]).contiguous()
    sig = [float(x) for x in rational_shifts(nsh)]
    res = {}
    for prec, name in ((tm.MIXED, "mixed"), (tm.FP64, "fp64")):
        if name == "fp64" and args.no_fp64:
            continue
        p = solver_params(tm, w, prec, args.graph)
        p.restart = 12
        s = tm.Solver(w.dims, p)
        if name == "mixed" and args.tune:
            s.setup(U, kappa, w.csw, w.mu)
            res["autotuned_variants"] = autotune(tm, s, [1, npt, nsh] + list(w.nv), args)
        _, t_setup = _timed(lambda: s.setup(U, kappa, w.csw, w.mu))
        xp = torch.empty_like(bp)
        ip, t_pt = _timed(lambda: s.solve(bp, xp, tol=w.tol))
        xs = torch.empty_like(bs)
        ish, t_sh = _timed(lambda: s.solve_shifted(bs, xs, sig, tol=w.tol))
        res[name] = {"setup_s": t_setup, "point_sources_s": t_pt, "shifted_s": t_sh,
                     "total_s": t_setup + t_pt + t_sh, "point_outer_iters": ip.outer_iters,
                     "point_true_rel_resid": ip.true_rel_resid, "shifted_outer_iters": ish.outer_iters,
                     "shifted_true_rel_resid": ish.true_rel_resid}
        log(f"[bench]   {name}: {res[name]}")
        s.close()
        del xp, xs
        torch.cuda.empty_cache()
    tuned = res.pop("autotuned_variants", None)
    m = res["mixed"]
    out = {"metric": "batched solve time (s) @1e-10 rel. resid: 12 point sources + 8 shifted systems",
           "value": m["total_s"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": m["total_s"] * 1e3, "higher_is_better": False, "scaling": "strong",
           "vs_baseline": None, "dtype": "fp32+bf16 (fp64 outer)", "data": "synthetic",
           "config": {"workload": "c3: 32x32x32x64, 3-level DD-alpha-AMG, 12 point sources + 8 shifts, restart 12",
                      "lattice": list(w.dims), "mu": w.mu, "csw": w.csw, "shifts": sig,
                      "hip_graph_level1_solve": bool(args.graph)},
           "mixed": m, "fp64_amg": res.get("fp64"),
           "speedup_vs_fp64": (res["fp64"]["total_s"] / m["total_s"]) if "fp64" in res else None,
           "per_rhs_s": m["total_s"] / (npt + nsh), "autotuned_variants": tuned}
    print(json.dumps(out), flush=True)
    return 0


def bench_force(args):
    """16^3 x 32 force: phi = D xi, S_f = phi^dag (D D^dag)^-1 phi and its
    force through two multigrid solves and the adjoint kernels, mixed
    precision against the plain FP64 DD-alpha-AMG.  S_f(phi = D xi) equals
    |xi|^2 exactly, which checks the whole chain at full size."""
    import torch
    import paper_1710_06198_amd as tm
    from lattice_inputs import workload, gauge_links, gaussian_spinor, load_m0
    w = workload("c4")
    m0 = load_m0()[w.name]
    kappa = 1.0 / (2 * m0 + 8)
    dev = torch.device("cuda:0")
    log(f"[bench] workload c4 dims {w.dims}: generating inputs")
    U = torch.as_tensor(gauge_links(w.dims, w.eps, w.seeds["links"])).to(dev)
    xi = torch.as_tensor(gaussian_spinor(w.dims, w.seeds["xi"], n=1)).to(dev)
    xi2 = float((xi.abs() ** 2).sum())
    F = torch.empty((4,) + tuple(reversed(w.dims)) + (3, 3), dtype=torch.complex128, device=dev)
    res = {}
    for prec, name in ((tm.MIXED, "mixed"), (tm.FP64, "fp64")):
        if name == "fp64" and args.no_fp64:
            continue
        s = tm.Solver(w.dims, solver_params(tm, w, prec, args.graph))
        if name == "mixed" and args.tune:
            s.setup(U, kappa, w.csw, w.mu)
            res["autotuned_variants"] = autotune(tm, s, [1] + list(w.nv), args)
        _, t_setup = _timed(lambda: s.setup(U, kappa, w.csw, w.mu))
        phi = torch.empty_like(xi)
        s.apply(tm.OP_D64, 0, xi, phi, [w.mu])
        times = []
        for i in range(max(1, args.steps)):
            (S, info), t = _timed(lambda: s.force(phi, F, tol=1e-12))
            times.append(t)
        res[name] = {"setup_s": t_setup, "force_s": min(times), "S": S, "S_rel_err_vs_xi2": abs(S - xi2) / xi2,
                     "outer_iters": info.outer_iters, "true_rel_resid": info.true_rel_resid,
                     "F_norm": float(torch.linalg.vector_norm(F))}
        log(f"[bench]   {name}: {res[name]}")
        s.close()
    tuned = res.pop("autotuned_variants", None)
    m = res["mixed"]
    out = {"metric": "force time (s): S_f and dS_f/dU with solves to 1e-12",
           "value": m["setup_s"] + m["force_s"], "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": 0,
           "ms_per_step": (m["setup_s"] + m["force_s"]) * 1e3, "higher_is_better": False, "scaling": "strong",
           "vs_baseline": None, "dtype": "fp32+bf16 (fp64 outer, fp64 force kernels)", "data": "synthetic",
           "config": {"workload": "c4: 16x16x16x32, 3-level DD-alpha-AMG, phi = D xi", "lattice": list(w.dims),
                      "mu": w.mu, "csw": w.csw},
           "mixed": m, "fp64_amg": res.get("fp64"),
           "speedup_vs_fp64": ((res["fp64"]["setup_s"] + res["fp64"]["force_s"]) / (m["setup_s"] + m["force_s"]))
           if "fp64" in res else None, "autotuned_variants": tuned}
    print(json.dumps(out), flush=True)
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--graph", type=int, choices=(0, 1), default=None,
                    help="mixed precision: replay the intermediate-level solve from a HIP graph "
                         "(default: on for the batched 32^3x64 workload, whose definition names "
                         "graph-captured cycles; off elsewhere, where it measured no faster)")
    ap.add_argument("--tune", type=int, choices=(0, 1), default=1,
                    help="autotune the kernel variants on the workload's hierarchy before timing")
    ap.add_argument("--tune-cache", default=None, help="variant table JSON to load if present, else to write")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the stencil and copy timing loops (for hardware-counter passes)")
    args = ap.parse_args()
    if args.graph is None:
        args.graph = 1 if args.workload == "c3" else 0
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU only; --gpus must be 1 "
                                   "(sharding across GPUs is not implemented)"}))
        return 2

    import torch
    import paper_1710_06198_amd as tm
    from lattice_inputs import workload, gauge_links, gaussian_spinor, load_m0

    if args.workload == "c3":
        return bench_batched(args)
    if args.workload == "c4":
        return bench_force(args)
    w = workload(args.workload)
    m0 = load_m0()[w.name]
    kappa = 1.0 / (2 * m0 + 8)
    dev = torch.device("cuda:0")
    log(f"[bench] workload {w.name} dims {w.dims}: generating inputs")
    U_np = gauge_links(w.dims, w.eps, w.seeds["links"])
    U = torch.as_tensor(U_np).to(dev)
    b = torch.as_tensor(gaussian_spinor(w.dims, w.seeds["source"], n=1)).to(dev)
    x = torch.empty_like(b)
    stream = torch.cuda.Stream(device=dev)

    def job(solver):
        solver.setup(U, kappa, w.csw, w.mu)
        return solver.solve(b, x, tol=w.tol)

    mixed = tm.Solver(w.dims, solver_params(tm, w, tm.MIXED, args.graph), stream=stream)
    if args.kernels_only:
        mixed.setup(U, kappa, w.csw, w.mu)
        d_ms = mixed.time_kernel(tm.K_DSLASH32, 1, 10)
        c_ms = mixed.time_kernel(tm.K_COPY, 1, 10)
        mf = batched_coarse(tm, mixed, 10)
        print(json.dumps({"dslash_fp32_ms": d_ms, "copy_512MiB_ms": c_ms, "sites": w.volume, "mfma": mf}),
              flush=True)
        mixed.close()
        return 0
    tuned = None
    if args.tune:
        mixed.setup(U, kappa, w.csw, w.mu)
        tuned = autotune(tm, mixed, [1] + list(w.nv), args)
    for i in range(args.warmup):
        log(f"[bench] warmup {i}")
        info = job(mixed)
        log(f"[bench]   {info.as_dict()}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = []
    for i in range(args.steps):
        infos.append(job(mixed).as_dict())
        log(f"[bench] step {i}: {infos[-1]}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    setup_s = sum(i["t_setup_s"] for i in infos) / len(infos)
    solve_s = sum(i["t_solve_s"] for i in infos) / len(infos)

    # fine stencil roofline (FP32, the solve's operator), HIP events on the library stream
    V = w.volume
    st_ms = mixed.time_kernel(tm.K_DSLASH32, 1, 50)
    bytes_site = 768   # in 96 + out 96 + links 4*72 + clover 288 (FP32)
    achieved = bytes_site * V / (st_ms * 1e-3) / 1e9
    kern = {}
    for nm, kid in (("sap_fine_colour", tm.K_SAP0), ("restrict_fine", tm.K_RESTRICT0),
                    ("prolong_fine", tm.K_PROLONG0), ("coarse_op_l1", tm.K_DC1), ("coarse_op_l2", tm.K_DC2),
                    ("sap_coarse_colour", tm.K_SAP1), ("dslash_fp64", tm.K_DSLASH64)):
        try:
            kern[nm] = round(mixed.time_kernel(kid, 1, 20), 4)
        except tm.TmamgError:
            pass
    kern["dslash_fp32"] = round(st_ms, 4)
    mfma = batched_coarse(tm, mixed, 20)

    # setup reuse along a trajectory: the links take one random-walk step
    # (a stand-in for a molecular-dynamics update), the setup is updated with
    # one iteration on the kept test vectors, then the solve
    from lattice_inputs import md_step_links
    U1 = torch.as_tensor(md_step_links(U_np, 0.05, w.seeds["links"] + 1)).to(dev)

    def update_job(solver):
        solver.setup(U, kappa, w.csw, w.mu)
        torch.cuda.synchronize()
        u0 = time.perf_counter()
        solver.setup_update(U1, 1)
        torch.cuda.synchronize()
        u1 = time.perf_counter()
        inf = solver.solve(b, x, tol=w.tol).as_dict()
        return {"update_s": u1 - u0, "solve_s": inf["t_solve_s"], "total_s": u1 - u0 + inf["t_solve_s"],
                "outer_iters": inf["outer_iters"], "true_rel_resid": inf["true_rel_resid"]}

    upd = {"step": "U -> exp(0.05 i g.lambda/2) U, then 1 setup iteration", "mixed": update_job(mixed)}
    log(f"[bench] setup update: {upd['mixed']}")

    # non-degenerate doublet (Eq. 2) with the light sector's hierarchy (the
    # same P, as for the heavy doublet of an Nf = 2+1+1 run): setup, one
    # doublet solve that allocates its workspace, then the timed doublet
    # solve on the same two-flavour source
    nd_mu, nd_eps = 0.13, 0.11
    b2 = torch.as_tensor(gaussian_spinor(w.dims, w.seeds["source"] + 7, n=2)).to(dev)
    x2 = torch.empty_like(b2)

    def nd_job(solver):
        solver.setup(U, kappa, w.csw, w.mu)
        solver.solve_nd(b2, x2, nd_mu, nd_eps, tol=w.tol)   # allocates the two-flavour Krylov basis
        inf = solver.solve_nd(b2, x2, nd_mu, nd_eps, tol=w.tol).as_dict()
        return {"solve_s": inf["t_solve_s"], "outer_iters": inf["outer_iters"],
                "true_rel_resid": inf["true_rel_resid"]}

    nd = {"mubar": nd_mu, "epsbar": nd_eps, "hierarchy": f"setup at mu = {w.mu}", "mixed": nd_job(mixed)}
    log(f"[bench] doublet: {nd['mixed']}")

    fp64 = None
    if not args.no_fp64:
        log("[bench] plain FP64 DD-alpha-AMG")
        plain = tm.Solver(w.dims, solver_params(tm, w, tm.FP64), stream=stream)
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        fi = job(plain).as_dict()
        torch.cuda.synchronize()
        f1 = time.perf_counter()
        fp64 = {"total_s": f1 - f0, "setup_s": fi["t_setup_s"], "solve_s": fi["t_solve_s"],
                "outer_iters": fi["outer_iters"], "true_rel_resid": fi["true_rel_resid"]}
        log(f"[bench]   {fp64}")
        upd["fp64"] = update_job(plain)
        upd["speedup_vs_fp64"] = upd["fp64"]["total_s"] / upd["mixed"]["total_s"]
        log(f"[bench] setup update FP64: {upd['fp64']}")
        nd["fp64"] = nd_job(plain)
        nd["speedup_vs_fp64"] = nd["fp64"]["solve_s"] / nd["mixed"]["solve_s"]
        log(f"[bench] doublet FP64: {nd['fp64']}")
        plain.close()

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(w, m0)
        log(f"[bench]   {cpu}")

    out = {
        "metric": "solve time (s) @1e-10 rel. resid",
        "value": ms / 1e3,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "fp32+bf16 (fp64 outer)",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {'x'.join(map(str, w.dims))} twisted-mass clover, "
                               f"{w.nlevels}-level DD-alpha-AMG, mixed precision, 1 RHS, setup+solve",
                   "lattice": list(w.dims), "mu": w.mu, "csw": w.csw, "m0": m0, "nv": list(w.nv),
                   "tol": w.tol, "hip_graph_level1_solve": bool(args.graph), "parallelism": "1 GPU"},
        "setup_s": setup_s,
        "solve_s": solve_s,
        "outer_iters": infos[-1]["outer_iters"],
        "true_rel_resid": max(i["true_rel_resid"] for i in infos),
        "fp64_amg": fp64,
        "speedup_vs_fp64": (fp64["total_s"] / (ms / 1e3)) if fp64 else None,
        "kernel_ms": kern,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": stencil_traffic(w.name),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "k_dslash<float> (fine stencil)", "bytes_per_site": bytes_site, "sites": V},
        "mfma_batched_coarse": mfma,
        "autotuned_variants": tuned,
        "setup_update_step": upd,
        "nd_doublet_solve": nd,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    mixed.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
