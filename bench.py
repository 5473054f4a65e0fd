"""Benchmark: DD-alpha-AMG time to solution on one MI355X.

Workload (default, c3): the 32^3 x 64 mixed+batched job - synthetic links
(spread 0.25), c_sw = 1.6, mu = 0.0015, 3-level DD-alpha-AMG (4^4 then 2^4
aggregates, N_v = 24/32, SAP 4^4 / 2^4 with 4 MR steps, 3 setup
iterations), FP32 stencil/SAP with bf16 P and D_c on the matrix cores, FP64
outer FGMRES with reliable updates, intermediate-level solves replayed from
HIP graphs.  A step is one whole job: the setup, 12 spin-colour point
sources at random sites solved as one batch of D(mu) x = b, and 8 shifted
systems (D D^dag + sigma_k) x = b (sigma_k log-spaced in [1e-5, 1], one
Gaussian source) as a second batch of two-step solves, every result to
relative residual 1e-10.  The plain FP64 DD-alpha-AMG on the same GPU runs
the same job (warmed up and timed the same way) for the speed-up; the fine
SAP (the kernel with the largest share of the job, bound by FP32 vector
issue) is measured against the FP32 vector peak and the fine stencil
against the HBM roofline, with HIP events on the library's stream; the
oracle's cost of the job is estimated from its own timings.  Other
workloads: c2 (24^3 x 48, one right-hand side), c4 (16^3 x 32, force), c5
(64^3 x 128, the paper's volume: setup, 4 right-hand sides and a force).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c3|c2|c4|c5]
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
STENCIL_TRAFFIC = {"c2": os.path.join(ROOT, "profiles", "dslash_fp32_c2_traffic.md"),
                   "c3": os.path.join(ROOT, "profiles", "dslash_fp32_c3_traffic.md")}
STENCIL_SOURCES = ("fine_op.hip", "su3.h", "common.h")


def stencil_traffic(workload_name):
    """HBM bytes per FP32 stencil launch (one right-hand side) from the
    workload's committed counter record, or None (see kernel_traffic)."""
    rec = STENCIL_TRAFFIC.get(workload_name)
    return kernel_traffic(rec, STENCIL_SOURCES, workload_name, workload_name) if rec else None


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


def oracle_unit_costs(w, m0, sample_dims=(16, 16, 16, 32)):
    """The oracle's time for one application of each unit of work the job
    is made of, measured on a 16^3 x 32 lattice with the workload's link
    spread, c_sw, mu and exactly its hierarchy shape (4^4 then 2^4
    aggregates, N_v 24/32, SAP blocks 4^4 and 2^4, 4 MR steps, at most 6
    intermediate and 10 coarsest steps), then scaled to the workload's
    volume by the site ratio.  Units: one fine operator application D, one
    fine SAP application (k sweeps from zero), one multigrid cycle B_MG
    (Eq. (1), with the coarse solves run to their step limits).  P and D_c
    are timing stand-ins (orthonormalised random vectors, random coarse
    blocks of the Galerkin shapes): the cost of these steps does not depend
    on the numbers in them."""
    import torch
    from lattice_inputs import gauge_links, gaussian_spinor
    from oracle.dirac import WilsonClover, spinor_to_field
    from oracle import mg
    t_all = time.time()
    U = gauge_links(sample_dims, w.eps, w.seeds["links"])
    op = WilsonClover(U, m0, w.csw)
    v = spinor_to_field(gaussian_spinor(sample_dims, w.seeds["source"])[0])
    p = mg.MGParams(nlevels=3, agg=w.agg, nv=w.nv, sap_block=w.sap_block, sap_sweeps=w.sap_sweeps,
                    mr_steps=w.mr_steps, setup_iters=0, init_smooth=0, l2_restart=6, l2_maxiter=6, l2_tol=0.0,
                    coarsest_tol=0.0, coarsest_maxiter=10)
    H = mg.Hierarchy(op, p, w.mu)
    gen = torch.Generator().manual_seed(7)

    def rnd(*shape):
        return torch.complex(torch.randn(*shape, generator=gen, dtype=torch.float64),
                             torch.randn(*shape, generator=gen, dtype=torch.float64))

    def coarse_stand_in(dims, d):
        lx, ly, lz, lt = dims
        S = 0.1 * rnd(lt, lz, ly, lx, d, d) + 4.0 * torch.eye(d, dtype=torch.complex128)
        return mg.CoarseOp(S, 0.1 * rnd(4, lt, lz, ly, lx, d, d), 0.1 * rnd(4, lt, lz, ly, lx, d, d))

    fine = H.levels[0]
    fine.tv = mg.random_test_vectors(sample_dims, 12, w.nv[0], w.seeds["testvec"])
    fine.P = mg.build_prolongation(fine.tv, w.agg[0], sample_dims, 12)
    d1 = tuple(sample_dims[m] // w.agg[0][m] for m in range(4))
    lvl1 = mg.Level(coarse_stand_in(d1, 2 * w.nv[0]), 1)
    fine.nxt = lvl1
    H.levels.append(lvl1)
    lvl1.tv = mg.random_test_vectors(d1, 2 * w.nv[0], w.nv[1], w.seeds["testvec"] + 100)
    lvl1.P = mg.build_prolongation(lvl1.tv, w.agg[1], d1, 2 * w.nv[0])
    d2 = tuple(d1[m] // w.agg[1][m] for m in range(4))
    lvl1.nxt = mg.Level(coarse_stand_in(d2, 2 * w.nv[1]), 2)

    def timed(f):
        t0 = time.time()
        f()
        return time.time() - t0

    t_D = min(timed(lambda: op.apply(v, w.mu)) for _ in range(2))
    t_S = timed(lambda: mg.sap(op, v, torch.zeros_like(v), w.mu, w.sap_block[0], w.sap_sweeps[0], w.mr_steps))
    t_B = timed(lambda: H.precondition(fine, v, w.mu))
    vol = 1
    for d in sample_dims:
        vol *= d
    scale = w.volume / vol
    return {"D": t_D * scale, "SAP": t_S * scale, "B": t_B * scale, "scale": scale,
            "sample_dims": list(sample_dims), "sample_s": time.time() - t_all,
            "sample_units_s": {"D": t_D, "SAP": t_S, "B": t_B}}


def job_unit_counts(w, infos):
    """Units of oracle work in one job of the batched workload, from the
    library's own iteration counts: every outer FGMRES iteration applies
    B_MG and D once per right-hand side of its batch; the setup smooths N_v
    vectors init_smooth times, applies B_MG to them setup_iters times, and
    forms D P for 2 N_v columns at each of its 1 + setup_iters builds; each
    restart cycle adds one FP64 residual per right-hand side."""
    nv0 = w.nv[0]
    npt, nsh = w.extra["n_point"], w.extra["n_shift"]
    ip, ish = infos
    B = ip["outer_iters"] * npt + ish["outer_iters"] * nsh + w.setup_iters * nv0
    D = (ip["outer_iters"] + ip["cycles"]) * npt + (ish["outer_iters"] + ish["cycles"]) * nsh \
        + (1 + w.setup_iters) * 2 * nv0
    SAP = w.init_smooth * nv0
    return {"B": B, "D": D, "SAP": SAP}


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


SAP_BYTES_FIXED, SAP_BYTES_RHS = 576, 384
FP32_VECTOR_PEAK_TFS = 157.3     # MI355X FP32 vector peak (packed FMA)
FP32_NONPACKED_PEAK_TFS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flops (FMA) x 2.4 GHz
# Algorithmic FP32 flops of one SAP launch per site of the colour and right-
# hand side (FMA = 2 flops; a complex product 6, a complex multiply-add 8):
#   one hop: spin projection 12, two SU(3) x colour vector products 132,
#     reconstruction into the accumulator 48 -> 192
#   clover, two 6x6 Hermitian blocks 528; twisted mass 48
#   block residual eta - D z: 528 + 48 + 8 x 192 + 24 = 2136
#   MR step: D_B rho with the hops inside a 4^4 block (6 per site on
#     average) 1728, (q, q) 48, (q, rho) 96, e += alpha rho and
#     rho -= alpha q 192 -> 2064
SAP_FLOPS_RESIDUAL, SAP_FLOPS_MR_STEP = 2136, 2064
SAP_TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "sap_fine_fp32_c3_traffic.md")
SAP_SOURCES = ("fine_op.hip", "fine_site.h", "su3.h", "common.h")


def kernel_traffic(record, sources, workload_name, want_workload):
    """HBM bytes per launch from a committed counter record (FETCH_SIZE and
    WRITE_SIZE, scaled by a copy kernel's readings), or None when the record
    is for another workload or the kernel's sources changed since."""
    import hashlib
    if workload_name != want_workload or not os.path.exists(record):
        return None
    rec = None
    for line in open(record):
        if line.startswith("traffic_record:"):
            rec = json.loads(line.split(":", 1)[1])
    if rec is None:
        return None
    h = hashlib.sha256()
    for f in sources:
        h.update(open(os.path.join(ROOT, "paper_1710_06198_amd", "csrc", f), "rb").read())
    if h.hexdigest()[:16] != rec["source_sha16"]:
        return None
    return rec["bytes_per_launch"]


def sap_roofline(tm, solver, V, nrhs, reps, mr_steps=4, workload_name="c3"):
    """The fine SAP kernel (one colour of blocks, all MR steps) for nrhs
    right-hand sides, timed with HIP events on the library's stream.  It is
    bound by FP32 vector issue, not by HBM (about 24 flops per algorithmic
    byte, against the chip's 20 at the packed-FMA peak): achieved is the
    algorithmic flop rate against the FP32 vector peak; the non-packed FMA
    rate (the instructions the compiled kernels use) is given beside it, and so is
    the HBM view (algorithmic bytes per site of the colour: links and
    clover once, 576 B, and per right-hand side the source, the iterate
    read and written and the neighbouring iterate, 4 x 96 B)."""
    ms = solver.time_kernel(tm.K_SAP0, nrhs, reps)
    sites = V // 2
    flops = sites * nrhs * (SAP_FLOPS_RESIDUAL + mr_steps * SAP_FLOPS_MR_STEP)
    tfs = flops / (ms * 1e-3) / 1e12
    byts = sites * (SAP_BYTES_FIXED + SAP_BYTES_RHS * nrhs)
    gbs = byts / (ms * 1e-3) / 1e9
    return {"bound": "alu", "achieved": tfs, "peak": FP32_VECTOR_PEAK_TFS, "unit": "TFLOP/s",
            "frac": tfs / FP32_VECTOR_PEAK_TFS,
            "traffic": kernel_traffic(SAP_TRAFFIC_RECORD, SAP_SOURCES, workload_name, "c3"),
            "kernel": "k_sap_fine<float, 3, 256> (fine SAP, one colour, 4 MR steps per 4^4 block)",
            "rhs": nrhs, "sites_per_launch": sites, "flops_per_launch": flops,
            "flops_per_site_rhs": SAP_FLOPS_RESIDUAL + mr_steps * SAP_FLOPS_MR_STEP,
            "peak_nonpacked_fp32": FP32_NONPACKED_PEAK_TFS, "frac_nonpacked": tfs / FP32_NONPACKED_PEAK_TFS,
            "hbm_view": {"bytes_per_launch": byts, "bytes_per_site": f"{SAP_BYTES_FIXED} + {SAP_BYTES_RHS} x rhs",
                         "achieved_GBps": gbs, "frac": gbs / HBM_PEAK_GBS},
            "ms_per_launch": ms}


def stencil_roofline(tm, solver, V, reps, nrhs=1, workload_name=None):
    ms = solver.time_kernel(tm.K_DSLASH32, nrhs, reps)
    byts = V * (576 + 192 * nrhs)
    gbs = byts / (ms * 1e-3) / 1e9
    return {"kernel": "k_dslash<float>" + (", true" if nrhs > 1 else ""), "rhs": nrhs, "ms": ms,
            "bytes_per_launch": byts, "achieved": gbs, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
            "traffic": stencil_traffic(workload_name) if nrhs == 1 else None}


def bench_batched(args):
    """32^3 x 64 (the metric's configuration): setup, 12 spin-colour point
    sources at random sites as one batch of D(mu) x = b, and 8 shifted
    systems (D D^dag + sigma_k) x = b (sigma_k log-spaced in [1e-5, 1]) on
    one Gaussian source as a second batch of two-step solves, mixed
    precision, against the plain FP64 DD-alpha-AMG running the same job.
    Restart 12 bounds the Krylov memory of 12-wide batches."""
    import torch
    import paper_1710_06198_amd as tm
    from lattice_inputs import workload, gauge_links, point_sources, gaussian_spinor, rational_shifts, load_m0
    w = workload("c3")
    m0 = args.m0 if args.m0 is not None else load_m0()[w.name]
    kappa = 1.0 / (2 * m0 + 8)
    dev = torch.device("cuda:0")
    V = w.volume
    log(f"[bench] workload c3 dims {w.dims}: generating inputs")
    U = torch.as_tensor(gauge_links(w.dims, w.eps, w.seeds["links"])).to(dev)
    npt, nsh = w.extra["n_point"], w.extra["n_shift"]
    bp = torch.as_tensor(point_sources(w.dims, w.seeds["source"], npt)).to(dev)
    g1 = torch.as_tensor(gaussian_spinor(w.dims, w.seeds["source"] + 100, n=1)).to(dev)
    bs = g1.expand(nsh, *g1.shape[1:]).contiguous()
    sig = [float(x) for x in rational_shifts(nsh)]
    xp = torch.empty_like(bp)
    xs = torch.empty_like(bs)
    stream = torch.cuda.Stream(device=dev)

    def job(solver):
        solver.setup(U, kappa, w.csw, w.mu)
        ip = solver.solve(bp, xp, tol=w.tol).as_dict()
        ish = solver.solve_shifted(bs, xs, sig, tol=w.tol).as_dict()
        return ip, ish

    def run(solver, warmup, steps, name):
        for i in range(warmup):
            ip, ish = job(solver)
            log(f"[bench] {name} warmup {i}: sources {ip['outer_iters']} it, shifts {ish['outer_iters']} it")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        recs = []
        for i in range(steps):
            recs.append(job(solver))
            ip, ish = recs[-1]
            log(f"[bench] {name} step {i}: setup {ip['t_setup_s']:.3f} s, sources {ip['t_solve_s']:.3f} s "
                f"({ip['outer_iters']} it, {ip['true_rel_resid']:.1e}), shifts {ish['t_solve_s']:.3f} s "
                f"({ish['outer_iters']} it, {ish['true_rel_resid']:.1e})")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        n = len(recs)
        return {"s_per_step": (t1 - t0) / n, "setup_s": sum(r[0]["t_setup_s"] for r in recs) / n,
                "point_sources_s": sum(r[0]["t_solve_s"] for r in recs) / n,
                "shifted_s": sum(r[1]["t_solve_s"] for r in recs) / n, "steps": n, "warmup": warmup,
                "point_outer_iters": recs[-1][0]["outer_iters"], "point_cycles": recs[-1][0]["cycles"],
                "point_true_rel_resid": max(r[0]["true_rel_resid"] for r in recs),
                "point_level1_steps": recs[-1][0]["l2_iters_total"],
                "point_coarsest_iters": recs[-1][0]["coarsest_iters_total"],
                "shifted_outer_iters": recs[-1][1]["outer_iters"], "shifted_cycles": recs[-1][1]["cycles"],
                "shifted_true_rel_resid": max(r[1]["true_rel_resid"] for r in recs),
                "shifted_level1_steps": recs[-1][1]["l2_iters_total"],
                "shifted_coarsest_iters": recs[-1][1]["coarsest_iters_total"]}, recs[-1]

    p = solver_params(tm, w, tm.MIXED, args.graph)
    p.restart = 12
    mixed = tm.Solver(w.dims, p, stream=stream)
    tuned = None
    if args.tune:
        mixed.setup(U, kappa, w.csw, w.mu)
        tuned = autotune(tm, mixed, [1, npt, nsh] + list(w.nv), args)
    m, last = run(mixed, args.warmup, args.steps, "mixed")
    log(f"[bench] mixed: {m}")

    # kernels against their roofline (HIP events on the library stream)
    sap = sap_roofline(tm, mixed, V, npt, 10)
    log(f"[bench] fine SAP roofline (12 RHS): {sap}")
    sap_other = {n: round(mixed.time_kernel(tm.K_SAP0, n, 5), 4) for n in (1, nsh, w.nv[0])}
    sten = stencil_roofline(tm, mixed, V, 20, workload_name="c3")
    sten12 = stencil_roofline(tm, mixed, V, 5, npt)
    log(f"[bench] stencil: {sten} / 12 RHS {sten12}")
    kern = {}
    for nm, kid in (("restrict_fine", tm.K_RESTRICT0), ("prolong_fine", tm.K_PROLONG0),
                    ("coarse_op_l1", tm.K_DC1), ("coarse_op_l2", tm.K_DC2), ("sap_coarse_sweep", tm.K_SAP1)):
        kern[nm + "_12rhs"] = round(mixed.time_kernel(kid, npt, 5), 4)
    mfma = batched_coarse(tm, mixed, 20)
    mixed.close()
    torch.cuda.empty_cache()

    fp64 = None
    if not args.no_fp64:
        p64 = solver_params(tm, w, tm.FP64)
        p64.restart = 12
        plain = tm.Solver(w.dims, p64, stream=stream)
        fp64, _ = run(plain, 1, min(args.steps, 2), "fp64")
        log(f"[bench] fp64: {fp64}")
        plain.close()
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle: unit costs on a 16^3 x 32 sample")
        unit = oracle_unit_costs(w, m0)
        cnt = job_unit_counts(w, last)
        est = sum(cnt[k] * unit[k] for k in cnt)
        cpu = {"value": est, "unit": "s", "cores": torch.get_num_threads(), "kind": "oracle",
               "sample": (f"oracle time per unit measured at {'x'.join(map(str, unit['sample_dims']))} with the "
                          f"workload's parameters and hierarchy shape (D {unit['sample_units_s']['D']:.2f} s, SAP "
                          f"{unit['sample_units_s']['SAP']:.2f} s, B_MG {unit['sample_units_s']['B']:.2f} s; "
                          f"{unit['sample_s']:.0f} s in all), scaled by the site ratio {unit['scale']:.0f} and "
                          f"multiplied by the units one job uses ({cnt}) from the library's iteration counts"),
               "units_s_at_workload_volume": {k: unit[k] for k in ("D", "SAP", "B")}, "unit_counts": cnt,
               "cpu_model": _cpu_model(), "os_cpu_count": os.cpu_count()}
        log(f"[bench] cpu baseline: {cpu}")

    out = {"metric": "solve time (s) @1e-10 rel. resid & stencil HBM GB/s; mixed+batched vs FP64 AMG",
           "value": m["s_per_step"], "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": m["s_per_step"] * 1e3, "higher_is_better": False, "scaling": "strong",
           "vs_baseline": None, "dtype": "fp32+bf16 (fp64 outer)", "data": "synthetic",
           "config": {"workload": "c3: 32x32x32x64 twisted-mass clover, 3-level DD-alpha-AMG, mixed precision; "
                                  "one step = setup + 12 point sources (one batch) + 8 shifted systems "
                                  "(D D^dag + sigma) (one batch of two-step solves), all to 1e-10",
                      "lattice": list(w.dims), "mu": w.mu, "csw": w.csw, "m0": m0, "nv": list(w.nv),
                      "shifts": sig, "restart": 12, "tol": w.tol, "hip_graph_level1_solve": bool(args.graph),
                      "parallelism": "1 GPU"},
           "mixed": m, "fp64_amg": fp64,
           "speedup_vs_fp64": (fp64["s_per_step"] / m["s_per_step"]) if fp64 else None,
           "per_rhs_s": m["s_per_step"] / (npt + nsh),
           "roofline": sap,
           "stencil_roofline": {"1rhs": sten, "12rhs": sten12},
           "sap_fine_ms_by_rhs": sap_other, "kernel_ms": kern,
           "mfma_batched_coarse": mfma, "autotuned_variants": tuned, "cpu_baseline": cpu}
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


def paper_volume_params(tm, w):
    """The 64^3 x 128 memory plan on one GPU: the setup smooths and cycles
    the test vectors 8 at a time and releases them once P and D_c are built,
    the outer FGMRES restarts after 8 iterations, and right-hand sides are
    solved one after the other.  Fine fields are 6.4 GB in FP64 and 3.2 GB in
    FP32 at this volume: links and clover in both precisions take 58 GB, P
    in bf16 39 GB, a solve's FP64 vectors and FP32 Krylov space 90 GB."""
    p = solver_params(tm, w, tm.MIXED)
    p.restart = 8
    p.setup_chunk = 8
    p.keep_test_vectors = 0
    # the 8^3 x 16 coarsest lattice holds low modes that 10 GMRES steps do
    # not resolve at this volume: with 6 intermediate and 10 coarsest steps
    # the residual fell only to 5e-4 in 384 outer iterations, with 10 and 50
    # steps the solve converged in 46
    p.l2_iters = 10
    p.coarsest_iters = 50
    return p


def bench_paper_volume(args):
    """64^3 x 128, the paper's volume, with all three forms at once on one
    GPU: setup, 4 Gaussian right-hand sides solved one after the other to
    1e-10, and S_f with its force for phi = D xi (S_f = |xi|^2 exactly).
    Mixed precision only: the plain FP64 DD-alpha-AMG does not fit in one
    GPU's memory at this volume (its FP64 test vectors alone take 155 GB)."""
    import torch
    import paper_1710_06198_amd as tm
    from lattice_inputs import workload, gauge_links, gaussian_spinor, load_m0
    w = workload("c5")
    m0 = load_m0()[w.name]
    kappa = 1.0 / (2 * m0 + 8)
    dev = torch.device("cuda:0")
    nrhs = w.extra.get("nrhs", 4)
    workers = max(1, min(16, os.cpu_count() or 1))
    log(f"[bench] workload c5 dims {w.dims}: generating links ({workers} processes)")
    t0 = time.perf_counter()
    U = torch.as_tensor(gauge_links(w.dims, w.eps, w.seeds["links"], workers=workers))
    log(f"[bench]   links drawn in {time.perf_counter() - t0:.1f} s")
    Ud = U.to(dev)
    del U
    stream = torch.cuda.Stream(device=dev)
    s = tm.Solver(w.dims, paper_volume_params(tm, w), stream=stream)
    torch.cuda.synchronize()
    torch.cuda.reset_peak_memory_stats()
    _, t_setup = _timed(lambda: s.setup(Ud, kappa, w.csw, w.mu))
    mem_setup = torch.cuda.max_memory_allocated() / 1e9
    log(f"[bench]   setup {t_setup:.2f} s, peak device memory {mem_setup:.1f} GB")
    del Ud
    torch.cuda.empty_cache()
    b_all = gaussian_spinor(w.dims, w.seeds["source"], n=nrhs)
    solves = []
    x = None
    for r in range(nrhs):
        b = torch.as_tensor(b_all[r:r + 1]).to(dev)
        x = torch.empty_like(b) if x is None else x
        info, t = _timed(lambda: s.solve(b, x, tol=w.tol))
        solves.append({"s": t, "outer_iters": info.outer_iters, "true_rel_resid": info.true_rel_resid,
                       "level1_steps": info.l2_iters_total, "coarsest_iters": info.coarsest_iters_total})
        log(f"[bench]   rhs {r}: {solves[-1]}")
        del b
    del b_all
    xi = torch.as_tensor(gaussian_spinor(w.dims, w.seeds["xi"], n=1)).to(dev)
    xi2 = float((xi.abs() ** 2).sum())
    phi = torch.empty_like(xi)
    s.apply(tm.OP_D64, 0, xi, phi, [w.mu])
    del xi, x
    torch.cuda.empty_cache()
    F = torch.empty((4,) + tuple(reversed(w.dims)) + (3, 3), dtype=torch.complex128, device=dev)
    (S, finfo), t_force = _timed(lambda: s.force(phi, F, tol=w.tol))
    log(f"[bench]   force {t_force:.2f} s, S rel. error {abs(S - xi2) / xi2:.2e}")
    mem_peak = torch.cuda.max_memory_allocated() / 1e9
    del F, phi
    torch.cuda.empty_cache()
    V = w.volume
    st_ms = s.time_kernel(tm.K_DSLASH32, 1, 10)
    sap_ms = s.time_kernel(tm.K_SAP0, 1, 5)
    total = t_setup + sum(v["s"] for v in solves) + t_force
    out = {"metric": "solve time (s) @1e-10 rel. resid & stencil HBM GB/s; mixed+batched vs FP64 AMG",
           "value": total, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": total * 1e3,
           "higher_is_better": False, "scaling": "strong", "vs_baseline": None,
           "dtype": "fp32+bf16 (fp64 outer, fp64 force kernels)", "data": "synthetic",
           "config": {"workload": "c5: 64x64x64x128 (the paper's volume), 3-level DD-alpha-AMG, mixed precision; "
                                  "one step = setup + 4 Gaussian right-hand sides (solved one after the other) "
                                  "+ S_f and its force for phi = D xi, all to 1e-10",
                      "lattice": list(w.dims), "mu": w.mu, "csw": w.csw, "m0": m0, "nv": list(w.nv),
                      "restart": 8, "setup_chunk": 8, "parallelism": "1 GPU"},
           "setup_s": t_setup, "solves": solves, "force_s": t_force, "S_rel_err_vs_xi2": abs(S - xi2) / xi2,
           "force_outer_iters": finfo.outer_iters, "force_true_rel_resid": finfo.true_rel_resid,
           "peak_device_memory_gb": {"setup": mem_setup, "job": mem_peak},
           "fp64_amg": None,
           "stencil_roofline": {"kernel": "k_dslash<float>", "rhs": 1, "ms": st_ms, "bytes_per_launch": 768 * V,
                                "achieved": 768 * V / (st_ms * 1e-3) / 1e9, "unit": "GB/s",
                                "frac": 768 * V / (st_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
           "sap_fine_colour_1rhs_ms": sap_ms}
    s.close()
    print(json.dumps(out), flush=True)
    return 0


def kernels_only(args):
    """Timing loops for profiler and counter passes: a context with links
    and clover but no multigrid (so no setup kernels run), then the FP32
    stencil (1 RHS), the fine SAP for one colour at 12 right-hand sides and
    the 512 MiB copy kernel, 10 timed launches each after one warm launch."""
    import torch
    import paper_1710_06198_amd as tm
    from lattice_inputs import workload, gauge_links, load_m0
    w = workload(args.workload)
    m0 = load_m0()[w.name]
    dev = torch.device("cuda:0")
    U = torch.as_tensor(gauge_links(w.dims, w.eps, w.seeds["links"])).to(dev)
    p = tm.default_params(nlevels=1, agg=w.agg, precision=tm.MIXED, storage=tm.STORE_BF16, setup_iters=0,
                          init_smooth=0, mr_steps=w.mr_steps)
    s = tm.Solver(w.dims, p, stream=torch.cuda.Stream(device=dev))
    s.setup(U, 1.0 / (2 * m0 + 8), w.csw, w.mu)
    n = w.extra.get("n_point", 12)
    out = {"workload": w.name, "sites": w.volume, "dslash_fp32_ms": s.time_kernel(tm.K_DSLASH32, 1, 10),
           "sap_fine_rhs": n, "sap_fine_ms": s.time_kernel(tm.K_SAP0, n, 10),
           "copy_512MiB_ms": s.time_kernel(tm.K_COPY, 1, 10)}
    print(json.dumps(out), flush=True)
    s.close()
    return 0


def conditioning(args, iters=30):
    """The conditioning of the workload's problem: the smallest singular
    value of D(m0, mu = 0) on the workload's own lattice, by inverse
    iteration on D^dag D.  Each step is two solves at mu = 0 through the
    library, (D^dag D)^-1 x = D^-1 g5 D^-1 g5 x (D^dag = g5 D g5 at mu = 0);
    1 / (x^dag (D^dag D)^-1 x) for unit x converges to sigma_min^2 from
    above.  With the twisted mass, D(mu)^dag D(mu) = D(0)^dag D(0) + mu^2,
    so sigma_min(D(mu)) = sqrt(sigma_min^2 + mu^2): the problem sits in the
    twisted-mass-dominated regime of the paper's physical point when
    sigma_min is not much larger than mu."""
    import torch
    import paper_1710_06198_amd as tm
    from lattice_inputs import workload, gauge_links, gaussian_spinor, load_m0
    w = workload(args.workload)
    m0 = args.m0 if args.m0 is not None else load_m0()[w.name]
    dev = torch.device("cuda:0")
    U = torch.as_tensor(gauge_links(w.dims, w.eps, w.seeds["links"])).to(dev)
    s = tm.Solver(w.dims, solver_params(tm, w, tm.MIXED), stream=torch.cuda.Stream(device=dev))
    s.setup(U, 1.0 / (2 * m0 + 8), w.csw, w.mu)
    x = torch.as_tensor(gaussian_spinor(w.dims, w.seeds["source"] + 7, n=1)).to(dev)
    x /= torch.linalg.vector_norm(x)
    y = torch.empty_like(x)
    z = torch.empty_like(x)

    def g5(v):
        v[..., 2:, :] *= -1
        return v

    est, its = [], []
    for k in range(iters):
        i1 = s.solve(g5(x.clone()), y, mu_rhs=[0.0], tol=1e-8)
        i2 = s.solve(g5(y), z, mu_rhs=[0.0], tol=1e-8)
        rq = torch.vdot(x.flatten(), z.flatten()).real.item()
        est.append(1.0 / rq)
        its.append(i1.outer_iters + i2.outer_iters)
        x = z / torch.linalg.vector_norm(z)
        log(f"[cond] step {k}: sigma_min^2 <= {est[-1]:.4e} ({its[-1]} outer iterations)")
    smin = est[-1] ** 0.5
    # the eigenvalue of D(m0, 0) of smallest modulus, by inverse iteration on
    # D with its Rayleigh quotient; D(m0 + d) = D(m0) + d shifts every
    # eigenvalue by d, so m0 - Re(lambda) puts that eigenvalue on the
    # imaginary axis: the critical mass on this lattice by the same recipe
    # the workloads' m0 follow on the smaller proxy lattice
    x = torch.as_tensor(gaussian_spinor(w.dims, w.seeds["source"] + 8, n=1)).to(dev)
    x /= torch.linalg.vector_norm(x)
    dx = torch.empty_like(x)
    lams = []
    for k in range(iters):
        s.solve(x, y, mu_rhs=[0.0], tol=1e-8)
        x = y / torch.linalg.vector_norm(y)
        s.apply(tm.OP_D64, 0, x, dx, mu_rhs=[0.0])
        lam = torch.vdot(x.flatten(), dx.flatten()).item()
        lams.append([lam.real, lam.imag])
        eres = (torch.linalg.vector_norm(dx - lam * x) / abs(lam)).item()
        log(f"[cond] step {k}: lambda = {lam.real:.5e} {lam.imag:+.5e}i, |D x - lambda x| / |lambda| = {eres:.2e}")
    out = {"workload": w.name, "lattice": list(w.dims), "m0": m0, "mu": w.mu, "csw": w.csw,
           "sigma_min_D0": smin, "sigma_min_D0_sq_by_step": est, "outer_iters_by_step": its,
           "sigma_min_D_mu": (est[-1] + w.mu ** 2) ** 0.5, "sigma_min_over_mu": smin / w.mu,
           "lambda_min_modulus_D0": lams[-1], "lambda_by_step": lams, "lambda_eigen_residual": eres, "m0_critical_this_lattice": m0 - lams[-1][0]}
    s.close()
    print(json.dumps(out), flush=True)
    return 0


def coarse_kernels(args):
    """Timing loops of the level-1 matrix-core kernels on the workload's own
    mixed-precision hierarchy (for profiler and counter passes): the
    level-1 operator with 16 right-hand sides and one level-1 SAP sweep
    (both colours, residual and 4 MR steps) with 12, 10 timed launches each
    after one warm launch, and the level-2 operator with 12."""
    import torch
    import paper_1710_06198_amd as tm
    from lattice_inputs import workload, gauge_links, load_m0
    w = workload(args.workload)
    m0 = load_m0()[w.name]
    dev = torch.device("cuda:0")
    U = torch.as_tensor(gauge_links(w.dims, w.eps, w.seeds["links"])).to(dev)
    s = tm.Solver(w.dims, solver_params(tm, w, tm.MIXED), stream=torch.cuda.Stream(device=dev))
    s.setup(U, 1.0 / (2 * m0 + 8), w.csw, w.mu)
    vc, d = s.level_info(1)
    out = {"workload": w.name, "level1_sites": vc, "d": d,
           "coarse_op_l1_16rhs_ms": s.time_kernel(tm.K_DC1, 16, 10),
           "sap1_sweep_12rhs_ms": s.time_kernel(tm.K_SAP1, 12, 10),
           "coarse_op_l2_12rhs_ms": s.time_kernel(tm.K_DC2, 12, 10)}
    print(json.dumps(out), flush=True)
    s.close()
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--graph", type=int, choices=(0, 1), default=None,
                    help="mixed precision: replay the intermediate-level solve from a HIP graph "
                         "(default: on for the batched 32^3x64 workload, whose definition names "
                         "graph-captured cycles; off elsewhere, where it measured no faster)")
    ap.add_argument("--tune", type=int, choices=(0, 1), default=1,
                    help="autotune the kernel variants on the workload's hierarchy before timing")
    ap.add_argument("--tune-cache", default=None, help="variant table JSON to load if present, else to write")
    ap.add_argument("--m0", type=float, default=None,
                    help="c3 and --conditioning: this bare mass instead of the workload's (a measurement beside "
                         "the default line, e.g. at the critical mass of the workload's own lattice)")
    ap.add_argument("--conditioning", action="store_true",
                    help="estimate the smallest singular value of D(m0, mu=0) on the workload's lattice "
                         "(inverse iteration through the solver) instead of the benchmark")
    ap.add_argument("--coarse-kernels", action="store_true",
                    help="only the timing loops of the level-1 and level-2 matrix-core kernels on the "
                         "workload's hierarchy (for profiler passes)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the timing loops of the fine stencil, the fine SAP (12 right-hand sides) and "
                         "the copy kernel on a context without a multigrid setup (for profiler passes)")
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

    if args.kernels_only:
        return kernels_only(args)
    if args.conditioning:
        return conditioning(args)
    if args.coarse_kernels:
        return coarse_kernels(args)
    if args.workload == "c3":
        return bench_batched(args)
    if args.workload == "c4":
        return bench_force(args)
    if args.workload == "c5":
        return bench_paper_volume(args)
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
        job(plain)   # warm-up: first-call allocations, as the mixed solver had
        nf = min(args.steps, 3)
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        for _ in range(nf):
            fi = job(plain).as_dict()
        torch.cuda.synchronize()
        f1 = time.perf_counter()
        fp64 = {"total_s": (f1 - f0) / nf, "steps": nf, "warmup": 1, "setup_s": fi["t_setup_s"],
                "solve_s": fi["t_solve_s"], "outer_iters": fi["outer_iters"], "true_rel_resid": fi["true_rel_resid"]}
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
