#!/usr/bin/env python3
"""Time-to-solution benchmark of the structured-AMG preconditioned CG on one
MI355X.

Workload (default): 3D variable-coefficient diffusion on a 256^3 grid,
7-point finite-volume stencil, cell coefficients log-normal (sigma = 2) with
32 random spherical inclusions of contrast 10^U[-3,3], harmonic-mean faces,
seed 2, RHS uniform[-1,1]; FP64 PCG preconditioned by one V-cycle (forward GS
before, backward GS after the coarse correction), full coarsening to 4^3,
stencil Galerkin triple products, exact coarsest solve; stop at ||r||/||b|| <
1e-9 (true residual).

One step = the whole method on that input: hierarchy setup (triple products,
smoother data, coarsest inverse) followed by the PCG solve, inputs resident
in HBM.  The JSON line reports the mean step time (time-to-solution), the HBM
roofline of the kernel with the largest share of the solve, and the CPU oracle
timed on a bounded sample of the same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-solution @1e-9 rel resid + V-cycle HBM GB/s; mixed/batched vs FP64"
HBM_PEAK_GBS = 8000.0
KIND_NAMES = ["pre_sweep", "pre_sweep_u", "resid_restrict", "coarse_solve", "prolong_post", "post_sweep",
              "post_sweep_u", "spmv_fp64"]
KERNEL_OF_KIND = {"pre_sweep": "k_wavefront (forward)", "pre_sweep_u": "k_wavefront (ILU upper)",
                  "resid_restrict": "k_resid_restrict", "coarse_solve": "k_coarse_gemv",
                  "prolong_post": "k_prolong_post", "post_sweep": "k_wavefront (backward)",
                  "post_sweep_u": "k_wavefront (ILU upper, add)", "spmv_fp64": "k_spmv"}


def kernel_bytes(kind, S, N, Nc, w, smoother="gs", ncoarse=0, interp="vertex"):
    """Algorithmic HBM bytes of one launch: every stored coefficient and vector
    entry the kernel needs is read once, every output written once.  With the
    operator-dependent interpolation the transfers run as separate passes and
    read the weights in use (27/8 per fine point on average: 1, 2, 4 or 8 for
    coarse, edge, face and interior points)."""
    SL = S // 2
    if interp == "operator" and kind == "resid_restrict":
        return (S + 2) * w * N + (1 + 27 / 8) * w * N + w * Nc
    if interp == "operator" and kind == "prolong_post" and smoother == "gs":
        return (2 + 27 / 8) * w * N + w * Nc + (SL + 2) * w * N
    if kind == "pre_sweep":
        return (SL + 3) * w * N if smoother == "gs" else (SL + 2) * w * N
    if kind == "pre_sweep_u":
        return (SL + 3) * w * N
    if kind == "resid_restrict":
        return (S + 2) * w * N + w * Nc
    if kind == "coarse_solve":
        return 8 * ncoarse * ncoarse + 2 * w * ncoarse
    if kind == "prolong_post":
        return ((SL + 3) * w * N + w * Nc) if smoother == "gs" else ((S + 4) * w * N + w * Nc)
    if kind == "post_sweep":
        return (SL + 3) * w * N if smoother == "gs" else (SL + 2) * w * N
    if kind == "post_sweep_u":
        return (SL + 5) * w * N
    if kind == "spmv_fp64":
        return (S + 2) * 8 * N
    raise ValueError(kind)


def wavefront_src_hash():
    h = hashlib.sha256()
    for f in ("wavefront.hip", "stencil.hip", "smg_common.h", "smg_group.h", "smg_kernels.h"):
        with open(os.path.join(ROOT, "paper_2506_21932_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_key):
    """HBM bytes per launch measured with rocprofv3 counters (profiles/), only
    while the kernel sources are unchanged since the measurement."""
    p = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(p):
        return None
    try:
        with open(p) as f:
            d = json.load(f)
        if d.get("src_hash") != wavefront_src_hash():
            return None
        e = d["kernels"].get(kernel_key)
        return None if e is None else float(e["hbm_bytes_per_launch"])
    except Exception:
        return None


def make_workload(name):
    import workloads
    if name == "diffusion256":
        shape = (256, 256, 256)
        A, b = workloads.diffusion7(shape, seed=2)
        return dict(shape=shape, A=A, b=b, pattern=7, smoother="gs", coarsen="full", semi_levels=0, krylov=0,
                    interp="operator",
                    desc="3D diffusion 256^3, 7-pt, log-normal sigma=2 + 32 inclusions, FP64 PCG + V(1,1) sym GS, "
                         "operator-dependent interpolation")
    if name == "poisson32":
        shape = (32, 32, 32)
        A, b = workloads.poisson7(32)
        return dict(shape=shape, A=A, b=b, pattern=7, smoother="gs", coarsen="full", semi_levels=0, krylov=0,
                    interp="vertex", desc="3D Poisson 32^3, 7-pt, FP64 PCG + V(1,1) sym GS, trilinear P")
    raise SystemExit(f"unknown workload {name}")


def vcycle_roofline(smg, torch, dev, A, b, shape, kw, krylov, tol, w=8):
    """One solve with per-kernel event timing on every level: the V-cycle's
    algorithmic bytes (every stored coefficient and vector entry its kernels
    need, read once; outputs written once) over its kernels' summed time,
    against the HBM peak."""
    import numpy as np
    m = smg.StructMG(A, shape, device=dev, **kw)
    levels = [m.level_info(l) for l in range(m.nlev)]
    m.set_timing(True)
    x = torch.zeros_like(b)
    m.solve(b, x, rtol=tol, maxit=500, krylov=krylov)
    rep, _ = m.timing_report(m.nlev)
    m.close()
    ncoarse = int(np.prod(levels[-1]["dims"]))
    ms = byt = 0.0
    for (l, kind), (t, c) in rep.items():
        if kind == "spmv_fp64":
            continue
        N = int(np.prod(levels[l]["dims"]))
        Nc = int(np.prod(levels[l + 1]["dims"])) if l + 1 < len(levels) else 0
        ms += t
        byt += c * kernel_bytes(kind, levels[l]["S"], N, Nc, w, kw.get("smoother", "gs"), ncoarse,
                                kw.get("interp", "vertex"))
    gbs = byt / ms / 1e6
    return {"ms_total": round(ms, 3), "algorithmic_GBps": round(gbs, 1), "peak_GBps": HBM_PEAK_GBS,
            "frac": round(gbs / HBM_PEAK_GBS, 4)}


def host_cpu():
    """CPU model and the cores this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count()
    return model, ncpu


def cpu_baseline(name, interp="vertex", gpu_iters=None):
    """The oracle (single-threaded C, as committed) on a bounded sample of the
    workload: the same recipe at 1/8 of the unknowns (128^3 for the 256^3
    diffusion, with the inclusion radii halved so that the 32 inclusions
    cover the same volume fraction), full setup + PCG to 1e-9.  The setup time
    is scaled by the unknown-count ratio and the solve time by that ratio
    times the full problem's iteration count over the sample's."""
    import oracle
    import workloads
    if name == "diffusion256":
        shape = (128, 128, 128)
        A, b = workloads.diffusion7(shape, seed=2, nspheres=32, rmin=4.0, rmax=16.0)
        scale = 8.0
        sample = ("same recipe at 128^3 (32 inclusions, radii 4-16 cells: the inclusion volume fraction of the "
                  "256^3 input), oracle setup + PCG to 1e-9")
    else:
        shape = (32, 32, 32)
        A, b = workloads.poisson7(32)
        scale = 1.0
        sample = "full workload"
    t0 = time.perf_counter()
    H = oracle.Hierarchy(shape, 7, A, interp=interp)
    t1 = time.perf_counter()
    x, st, it, rel = H.pcg(b, 1e-9, 200)
    t2 = time.perf_counter()
    full_iters = gpu_iters if gpu_iters else it
    ms = ((t1 - t0) * scale + (t2 - t1) * scale * full_iters / max(it, 1)) * 1e3
    model, ncpu = host_cpu()
    info = {"value": round(ms, 1), "unit": "ms", "cores": 1, "kind": "oracle",
            "sample": f"{sample}, {interp} interpolation; measured setup {t1 - t0:.1f}s + solve {t2 - t1:.1f}s "
                      f"({it} iterations, rel resid {rel:.2e}); value = setup x{scale:g} + solve x{scale:g} x "
                      f"{full_iters}/{it} iterations",
            "cpu_model": model, "host_cpus": ncpu}
    return info, dict(shape=shape, A=A, b=b, x=x, desc=sample)


def oracle_errors(smg, torch, np, dev, sample, kw, krylov, precs=("fp64", "fp32", "fp16"), tol=1e-9):
    """Each V-cycle precision's Krylov solution on the oracle's sample against
    the FP64 oracle solution: relative 2-norm error and true residual."""
    A = torch.from_numpy(sample["A"]).to(dev)
    b = torch.from_numpy(sample["b"].ravel().copy()).to(dev)
    xo = sample["x"].ravel()
    out = {"sample": sample["desc"]}
    for prec in precs:
        m = smg.StructMG(A, sample["shape"], device=dev, prec=prec, **kw)
        x = torch.zeros_like(b)
        r = m.solve(b, x, rtol=tol, maxit=500, krylov=krylov)
        torch.cuda.synchronize()
        xg = x.cpu().numpy()
        out[prec] = {"rel_err_vs_oracle": float(np.linalg.norm(xg - xo) / np.linalg.norm(xo)),
                     "rel_resid_true": r["rel_resid_true"], "iters": r["iters"]}
        m.close()
    return out


# ---- supplementary workloads (opt-in; the default line is the 256^3 diffusion)
def _timed(fn, torch, reps):
    out, times = None, []
    for k in range(1 + reps):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        if k > 0:
            times.append((time.perf_counter() - ts) * 1e3)
    return out, sum(times) / len(times)


def _variants(args, smg, torch, np, dev, W, precs, tol, krylov, xref=None, steps=None, **kw):
    """Time-to-solution (setup + solve, inputs resident) of each V-cycle
    precision; xref: a reference solution for the relative error."""
    A = torch.from_numpy(W["A"]).to(dev)
    b = torch.from_numpy(W["b"].ravel().copy()).to(dev)
    x = torch.zeros_like(b)
    res = {}
    for prec in precs:
        m = smg.StructMG(A, W["shape"], device=dev, prec=prec, **kw)

        def step():
            m.resetup(A)
            x.zero_()
            return m.solve(b, x, rtol=tol, maxit=500, krylov=krylov)

        r, ms = _timed(step, torch, args.steps if steps is None else steps)
        res[prec] = {"ms_per_step": round(ms, 2), "iters": r["iters"], "rel_resid_true": r["rel_resid_true"],
                     "converged": r["status"] == 0 and r["rel_resid_true"] < tol,
                     "t_setup_ms": round(r["t_setup_ms"], 2), "t_solve_ms": round(r["t_solve_ms"], 2),
                     "levels": r["levels"]}
        if xref is not None:
            xg = x.cpu().numpy()
            res[prec]["rel_err_vs_oracle"] = float(np.linalg.norm(xg - xref) / np.linalg.norm(xref))
        print(f"[bench] {prec}: {res[prec]}", file=sys.stderr, flush=True)
        m.close()
        del m
    for prec in precs:
        res[prec]["speedup_vs_fp64"] = round(res["fp64"]["ms_per_step"] / res[prec]["ms_per_step"], 3)
    return res


def extra_weather(args, smg, torch, np, dev):
    import workloads
    shape = (512, 512, 64)
    A, b = workloads.weather19(shape, seed=3)
    W = dict(shape=shape, A=A, b=b)
    kw = dict(pattern=19, smoother="ilu0", coarsen="semi_xy", gmres_restart=30, ilu_mask=args.ilu_mask)
    res = _variants(args, smg, torch, np, dev, W, ("fp64", "fp32"), 1e-9, 30, **kw)
    mask = f" on a {args.ilu_mask}-point mask" if args.ilu_mask else ""
    line = {"metric": METRIC, "value": res["fp32"]["ms_per_step"], "unit": "ms", "n_gpus": 1,
            "steps": args.steps, "higher_is_better": False, "dtype": "f32 V-cycle / f64 GMRES",
            "data": "synthetic (seeded)",
            "config": {"workload": "weather-like 512x512x64, 19-pt, vertical 100x, GMRES(30) + ILU(0)"
                                   f"{mask} V-cycle, xy-semi coarsening, tol 1e-9"},
            "variants": res}
    At = torch.from_numpy(A).to(dev)
    bt = torch.from_numpy(b.ravel().copy()).to(dev)
    line["vcycle_fp64"] = vcycle_roofline(smg, torch, dev, At, bt, W["shape"], kw, 30, 1e-9)
    if not args.no_cpu_baseline:
        line["oracle_error"] = oracle_errors(smg, torch, np, dev, weather_sample(args.ilu_mask), kw, 30,
                                             precs=("fp64", "fp32"))
    print(json.dumps(line), flush=True)


def weather_sample(ilu_mask):
    """The weather recipe at 128 x 128 x 64 solved by the oracle (GMRES(30),
    same V-cycle) for the solution-error check."""
    import oracle
    import workloads
    shape = (128, 128, 64)
    A, b = workloads.weather19(shape, seed=3)
    H = oracle.Hierarchy(shape, 19, A, smoother="ilu0", coarsen="semi_xy", ilu_mask=ilu_mask)
    x, st, it, rel = H.gmres(b, 1e-9, 500, restart=30)
    return dict(shape=shape, A=A, b=b, x=x,
                desc=f"same recipe at 128x128x64, oracle GMRES(30): {it} iterations, rel resid {rel:.2e}")


def extra_weather_lgs(args, smg, torch, np, dev):
    import workloads
    shape = (512, 512, 64)
    A, b = workloads.weather19(shape, seed=3)
    W = dict(shape=shape, A=A, b=b)
    res = _variants(args, smg, torch, np, dev, W, ("fp64", "fp32"), 1e-9, 30, pattern=19, smoother="lgs",
                    coarsen="semi_xy", gmres_restart=30)
    print(json.dumps({"metric": METRIC, "value": res["fp32"]["ms_per_step"], "unit": "ms", "n_gpus": 1,
                      "steps": args.steps, "higher_is_better": False, "dtype": "f32 V-cycle / f64 GMRES",
                      "data": "synthetic (seeded)",
                      "config": {"workload": "weather-like 512x512x64, 19-pt, vertical 100x, GMRES(30) + line-GS "
                                             "V-cycle (z-columns), xy-semi coarsening, tol 1e-9"},
                      "variants": res}), flush=True)


def extra_diffusion_interp(args, smg, torch, np, dev):
    """The benchmark's diffusion workload with the four hierarchies: vertex
    trilinear (PCG), operator-dependent vertex interpolation (PCG),
    cell-centred piecewise constant (PCG) and Cell_3d8 restriction with
    cell-centred trilinear interpolation (non-symmetric cycle: GMRES(30))."""
    W = make_workload("diffusion256")
    A = torch.from_numpy(W["A"]).to(dev)
    b = torch.from_numpy(W["b"].ravel().copy()).to(dev)
    x = torch.zeros_like(b)
    res = {}
    for interp, kr in (("vertex", 0), ("operator", 0), ("cell", 0), ("cell_trilinear", 30)):
        m = smg.StructMG(A, W["shape"], device=dev, pattern=7, interp=interp, gmres_restart=kr)

        def step():
            m.resetup(A)
            x.zero_()
            return m.solve(b, x, rtol=1e-9, maxit=500, krylov=kr)

        r, ms = _timed(step, torch, args.steps)
        res[interp] = {"ms_per_step": round(ms, 2), "iters": r["iters"], "rel_resid_true": r["rel_resid_true"],
                       "converged": r["status"] == 0 and r["rel_resid_true"] < 1e-9, "solver": "GMRES(30)" if kr
                       else "PCG", "t_setup_ms": round(r["t_setup_ms"], 2), "t_solve_ms": round(r["t_solve_ms"], 2),
                       "levels": r["levels"], "op_complexity": round(r["op_complexity"], 4)}
        print(f"[bench] {interp}: {res[interp]}", file=sys.stderr, flush=True)
        m.close()
        del m
    for k in res:
        res[k]["speedup_vs_vertex"] = round(res["vertex"]["ms_per_step"] / res[k]["ms_per_step"], 3)
    print(json.dumps({"metric": METRIC, "value": res["operator"]["ms_per_step"], "unit": "ms", "n_gpus": 1,
                      "steps": args.steps, "higher_is_better": False, "dtype": "f64", "data": "synthetic (seeded)",
                      "config": {"workload": W["desc"] + "; trilinear, operator-dependent and cell-centred "
                                                         "hierarchies"},
                      "variants": res}), flush=True)


def extra_elasticity(args, smg, torch, np, dev):
    import workloads
    n = 128
    A, b = workloads.elasticity27(n, seed=4)
    W = dict(shape=(n, n, n), A=A, b=b)
    res = _variants(args, smg, torch, np, dev, W, ("fp64", "fp32", "fp16"), 1e-8, 0, pattern=27, block=3)
    line = {"metric": METRIC, "value": res["fp16"]["ms_per_step"], "unit": "ms", "n_gpus": 1,
            "steps": args.steps, "higher_is_better": False, "dtype": "f16 V-cycle / f64 PCG",
            "data": "synthetic (seeded)",
            "config": {"workload": "elasticity-like 128^3 x 3, 27-pt 3x3 blocks, Q1 FEM, log-normal "
                                   "moduli (sigma 1), nu 0.3, PCG + block-GS V-cycle, tol 1e-8"},
            "variants": res}
    if not args.no_cpu_baseline:
        line["oracle_error"] = oracle_errors(smg, torch, np, dev, elasticity_sample(), dict(pattern=27, block=3), 0,
                                             tol=1e-8)
    print(json.dumps(line), flush=True)


def elasticity_sample():
    """The elasticity recipe at 32^3 nodes solved by the oracle (PCG, same
    block V-cycle) for the solution-error check."""
    import oracle
    import workloads
    n = 32
    A, b = workloads.elasticity27(n, seed=4)
    H = oracle.Hierarchy((n, n, n), 27, A, block=3)
    x, st, it, rel = H.pcg(b, 1e-8, 500)
    return dict(shape=(n, n, n), A=A, b=b, x=x,
                desc=f"same recipe at 32^3 x 3, oracle PCG: {it} iterations, rel resid {rel:.2e}")


def extra_batch(args, smg, torch, np, dev):
    import workloads
    dims = workloads.reservoir_batch(256, seed=5)
    t0 = time.perf_counter()
    systems = [workloads.reservoir7(d, seed=1000 + k) for k, d in enumerate(dims)]
    print(f"[bench] 256 systems generated in {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    kw = dict(pattern=7, coarsen="full", semi_levels=3, max_coarse=512)
    As = [torch.from_numpy(A).to(dev) for A, _ in systems]
    bs = [torch.from_numpy(b.ravel().copy()).to(dev) for _, b in systems]
    ncells = sum(int(np.prod(d)) for d in dims)
    out = {}
    for prec in ("fp32", "fp64"):
        B = smg.StructMGBatch(As, dims, prec=prec, **kw)
        tune = B.tune()
        xs = [torch.zeros_like(b) for b in bs]

        def solve():
            for x in xs:
                x.zero_()
            return B.solve(bs, xs, rtol=1e-9, maxit=300)

        (st, res), ms = _timed(solve, torch, args.steps)
        out[f"batched_{prec}"] = {"ms": round(ms, 2), "systems_per_s": round(256 / (ms * 1e-3), 2),
                                  "all_converged": st == 0 and all(r["rel_resid_true"] < 1e-9 for r in res),
                                  "max_iters": max(r["iters"] for r in res),
                                  "mean_iters": round(float(np.mean([r["iters"] for r in res])), 2),
                                  "t_setup_ms": round(res[0]["t_setup_ms"], 1), "schedule": tune}
        print(f"[bench] batched {prec}: {out[f'batched_{prec}']}", file=sys.stderr, flush=True)
        B.close()
        del B
    # the FP64 path one system after another (single-system solver)
    hs = [smg.StructMG(A, d, device=dev, prec="fp64", **kw) for A, d in zip(As, dims)]
    xs = [torch.zeros_like(b) for b in bs]

    def seq():
        rs = []
        for m, b, x in zip(hs, bs, xs):
            x.zero_()
            rs.append(m.solve(b, x, rtol=1e-9, maxit=300))
        return rs

    rs, ms = _timed(seq, torch, args.steps)
    out["sequential_fp64"] = {"ms": round(ms, 2), "systems_per_s": round(256 / (ms * 1e-3), 2),
                              "all_converged": all(r["status"] == 0 for r in rs)}
    for k in ("batched_fp32", "batched_fp64"):
        out[k]["speedup_vs_sequential_fp64"] = round(out["sequential_fp64"]["ms"] / out[k]["ms"], 2)
    print(json.dumps({"metric": METRIC, "value": out["batched_fp32"]["systems_per_s"], "unit": "systems/s",
                      "n_gpus": 1, "steps": args.steps, "higher_is_better": True,
                      "dtype": "f32 V-cycle / f64 PCG", "data": "synthetic (seeded)",
                      "config": {"workload": f"256 reservoir-like 7-pt systems, dims uniform in [16,96]^3 "
                                             f"({ncells} cells), kz/kx = 0.01, xy-semi x3 then full, tol 1e-9"},
                      "variants": out}), flush=True)


# ---- the other configurations, as sub-objects of the default line ----------
def run_poisson32(args, smg, torch, np, dev, steps):
    """3D Poisson 32^3 (the parity configuration, cache resident): FP64, FP32
    and FP16 V-cycles in FP64 PCG, each solution against the oracle's."""
    import oracle
    import workloads
    shape = (32, 32, 32)
    A, b = workloads.poisson7(32)
    H = oracle.Hierarchy(shape, 7, A)
    xo, st, it, rel = H.pcg(b.reshape(shape), 1e-9, 200)
    W = dict(shape=shape, A=A, b=b)
    res = _variants(args, smg, torch, np, dev, W, ("fp64", "fp32", "fp16"), 1e-9, 0, xref=xo.ravel(), steps=steps,
                    pattern=7)
    return {"workload": "3D Poisson 32^3, 7-pt, PCG + V(1,1) sym GS, trilinear P, tol 1e-9", "variants": res,
            "oracle": {"iters": it, "rel_resid_true": rel}}


def run_weather(args, smg, torch, np, dev, steps):
    """Weather-like 512x512x64, 19-point, GMRES(30) with the ILU(0) V-cycle
    in FP64 and in FP32, and the FP64 V-cycle's algorithmic bandwidth."""
    import workloads
    shape = (512, 512, 64)
    A, b = workloads.weather19(shape, seed=3)
    W = dict(shape=shape, A=A, b=b)
    kw = dict(pattern=19, smoother="ilu0", coarsen="semi_xy", gmres_restart=30)
    res = _variants(args, smg, torch, np, dev, W, ("fp64", "fp32"), 1e-9, 30, steps=steps, **kw)
    At = torch.from_numpy(A).to(dev)
    bt = torch.from_numpy(b.ravel().copy()).to(dev)
    vc = vcycle_roofline(smg, torch, dev, At, bt, shape, kw, 30, 1e-9)
    return {"workload": "weather-like 512x512x64, 19-pt, vertical 100x, GMRES(30) + ILU(0) V-cycle, xy-semi "
                        "coarsening, tol 1e-9", "variants": res, "vcycle_fp64": vc}


def run_elasticity(args, smg, torch, np, dev, steps):
    """Elasticity-like 128^3 x 3 (3x3 blocks, 27-point): PCG with FP64, FP32
    and FP16 (row-scaled) block-GS V-cycles, tol 1e-8."""
    import workloads
    n = 128
    A, b = workloads.elasticity27(n, seed=4)
    W = dict(shape=(n, n, n), A=A, b=b)
    res = _variants(args, smg, torch, np, dev, W, ("fp64", "fp32", "fp16"), 1e-8, 0, steps=steps, pattern=27,
                    block=3)
    return {"workload": "elasticity-like 128^3 x 3, 27-pt 3x3 blocks, Q1 FEM, log-normal moduli (sigma 1), "
                        "nu 0.3, PCG + block-GS V-cycle, tol 1e-8", "variants": res}


def run_batch(args, smg, torch, np, dev, steps):
    """256 reservoir-like systems of uneven sizes solved together (FP32 and
    FP64 V-cycles, FP64 PCG) against the FP64 single-system solver run on
    one system after another."""
    import workloads
    dims = workloads.reservoir_batch(256, seed=5)
    systems = [workloads.reservoir7(d, seed=1000 + k) for k, d in enumerate(dims)]
    kw = dict(pattern=7, coarsen="full", semi_levels=3, max_coarse=512)
    As = [torch.from_numpy(A).to(dev) for A, _ in systems]
    bs = [torch.from_numpy(b.ravel().copy()).to(dev) for _, b in systems]
    ncells = sum(int(np.prod(d)) for d in dims)
    out = {}
    for prec in ("fp32", "fp64"):
        B = smg.StructMGBatch(As, dims, prec=prec, **kw)
        tune = B.tune()
        xs = [torch.zeros_like(b) for b in bs]

        def solve():
            for x in xs:
                x.zero_()
            return B.solve(bs, xs, rtol=1e-9, maxit=300)

        (st, res), ms = _timed(solve, torch, steps)
        out[f"batched_{prec}"] = {"ms": round(ms, 2), "systems_per_s": round(256 / (ms * 1e-3), 2),
                                  "all_converged": st == 0 and all(r["rel_resid_true"] < 1e-9 for r in res),
                                  "max_iters": max(r["iters"] for r in res),
                                  "mean_iters": round(float(np.mean([r["iters"] for r in res])), 2),
                                  "max_rel_resid_true": max(r["rel_resid_true"] for r in res),
                                  "t_setup_ms": round(res[0]["t_setup_ms"], 1), "schedule": tune}
        print(f"[bench] C5 batched {prec}: {out[f'batched_{prec}']}", file=sys.stderr, flush=True)
        B.close()
        del B
    hs = [smg.StructMG(A, d, device=dev, prec="fp64", **kw) for A, d in zip(As, dims)]
    xs = [torch.zeros_like(b) for b in bs]

    def seq():
        rs = []
        for m, b, x in zip(hs, bs, xs):
            x.zero_()
            rs.append(m.solve(b, x, rtol=1e-9, maxit=300))
        return rs

    rs, ms = _timed(seq, torch, steps)
    out["sequential_fp64"] = {"ms": round(ms, 2), "systems_per_s": round(256 / (ms * 1e-3), 2),
                              "all_converged": all(r["status"] == 0 for r in rs)}
    for k in ("batched_fp32", "batched_fp64"):
        out[k]["speedup_vs_sequential_fp64"] = round(out["sequential_fp64"]["ms"] / out[k]["ms"], 2)
    for m in hs:
        m.close()
    return {"workload": f"256 reservoir-like 7-pt systems, dims uniform in [16,96]^3 ({ncells} cells), kz/kx = "
                        f"0.01, xy-semi x3 then full, tol 1e-9", "unit": "systems/s", "variants": out}


CONFIG_RUNNERS = {"C1_poisson32": run_poisson32, "C3_weather512": run_weather, "C4_elasticity128": run_elasticity,
                  "C5_batch256": run_batch}


EXTRA = {"weather512": extra_weather, "weather512_lgs": extra_weather_lgs, "elasticity128": extra_elasticity,
         "reservoir_batch256": extra_batch, "diffusion256_interp": extra_diffusion_interp}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="diffusion256")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32 / FP16 V-cycle variants")
    ap.add_argument("--breakdown", action="store_true", help="print per-kernel table to stderr")
    ap.add_argument("--configs", default="C1,C3,C4,C5",
                    help="other configurations reported as sub-objects of the default line (comma list of "
                         "C1,C3,C4,C5, or none)")
    ap.add_argument("--ilu-mask", type=int, default=0, choices=(0, 7, 19, 27),
                    help="weather512: ILU(0) mask of the finest matrix (0: its own 19-point pattern)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2506_21932_amd as smg

    dev = torch.device("cuda:0")
    if args.workload in EXTRA:
        EXTRA[args.workload](args, smg, torch, np, dev)
        return
    t_gen = time.perf_counter()
    W = make_workload(args.workload)
    t_gen = time.perf_counter() - t_gen
    print(f"[bench] workload {args.workload} generated in {t_gen:.1f}s", file=sys.stderr, flush=True)
    shape = W["shape"]
    n = int(np.prod(shape))
    A = torch.from_numpy(W["A"]).to(dev)
    b = torch.from_numpy(W["b"].ravel().copy()).to(dev)
    x = torch.zeros(n, dtype=torch.float64, device=dev)
    kw = dict(pattern=W["pattern"], smoother=W["smoother"], coarsen=W["coarsen"], semi_levels=W["semi_levels"],
              interp=W["interp"])
    mg = smg.StructMG(A, shape, device=dev, **kw)
    levels = [mg.level_info(l) for l in range(mg.nlev)]

    # pre-run (untimed): find the kernel with the largest share of the solve
    mg.set_timing(True)
    x.zero_()
    mg.solve(b, x, rtol=1e-9, maxit=300, krylov=W["krylov"])
    rep, _ = mg.timing_report(mg.nlev)
    dom = max(rep.items(), key=lambda kv: kv[1][0])[0]

    def bytes_of(lk):
        l, kind = lk
        inf = levels[l]
        N = int(np.prod(inf["dims"]))
        Nc = int(np.prod(levels[l + 1]["dims"])) if l + 1 < len(levels) else 0
        ncoarse = int(np.prod(levels[-1]["dims"]))
        return kernel_bytes(kind, inf["S"], N, Nc, 8, W["smoother"], ncoarse, W["interp"])

    ncycles = sum(c for (l, k), (ms, c) in rep.items() if l == 0 and k == "pre_sweep")
    vc_ms = sum(ms for (l, k), (ms, c) in rep.items() if k != "spmv_fp64")
    vc_bytes = sum(bytes_of(lk) * c for lk, (ms, c) in rep.items() if lk[1] != "spmv_fp64")
    breakdown = {f"L{l}:{k}": {"ms_per_launch": round(ms / c, 4), "launches": c,
                               "GBps": round(bytes_of((l, k)) / (ms / c) / 1e6, 1)}
                 for (l, k), (ms, c) in sorted(rep.items())}
    if args.breakdown:
        for k, v in breakdown.items():
            print(f"[bench] {k:24s} {v}", file=sys.stderr)
    mg.set_timing(True, level=dom[0], kinds=[dom[1]])

    for _ in range(args.warmup):
        mg.resetup(A)
        x.zero_()
        mg.solve(b, x, rtol=1e-9, maxit=300, krylov=W["krylov"])
    mg.timing_report(mg.nlev)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(args.steps):
        ts = time.perf_counter()
        mg.resetup(A)
        x.zero_()
        r = mg.solve(b, x, rtol=1e-9, maxit=300, krylov=W["krylov"])
        torch.cuda.synchronize()
        r["step_ms"] = (time.perf_counter() - ts) * 1e3
        results.append(r)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    rep_t, _ = mg.timing_report(mg.nlev)
    d_ms, d_cnt = rep_t[dom]
    d_avg = d_ms / d_cnt
    d_bytes = bytes_of(dom)
    achieved = d_bytes / (d_avg * 1e-3) / 1e9
    kernel_key = f"L{dom[0]}:{dom[1]}"
    traffic = load_traffic(kernel_key)
    # a Gauss-Seidel / ILU sweep is a chain of dependent hyperplanes
    # wx*x + wy*y + z = const (weights of the level's pattern): its length and
    # the time per hyperplane
    chain = None
    if dom[1] in ("pre_sweep", "post_sweep", "pre_sweep_u", "post_sweep_u"):
        S = levels[dom[0]]["S"]
        wx, wy = {7: (1, 1), 19: (3, 2), 27: (4, 2)}[S]
        nx_, ny_, nz_ = levels[dom[0]]["dims"]
        hyper = wx * (nx_ - 1) + wy * (ny_ - 1) + (nz_ - 1) + 1
        chain = {"hyperplanes": hyper, "us_per_hyperplane": round(d_avg * 1e3 / hyper, 3)}
    ok = all(r["status"] == 0 and r["rel_resid_true"] < 1e-9 for r in results)
    line = {
        "metric": METRIC,
        "value": round(ms_per_step, 2),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded)",
        "config": {"workload": W["desc"], "grid": list(shape), "unknowns": n, "tol": 1e-9, "solver": "PCG",
                   "levels": mg.nlev},
        "roofline": {"bound": "hbm", "kernel": f"{KERNEL_OF_KIND[dom[1]]} level {dom[0]}",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "algorithmic_bytes_per_launch": d_bytes, "avg_launch_ms": round(d_avg, 4),
                     "launches": d_cnt, "dependence_chain": chain},
        "converged": ok,
        "iters": results[-1]["iters"],
        "host_waits": results[-1]["host_waits"],
        "rel_resid_true": results[-1]["rel_resid_true"],
        "t_setup_ms": round(float(np.mean([r["t_setup_ms"] for r in results])), 2),
        "t_solve_ms": round(float(np.mean([r["t_solve_ms"] for r in results])), 2),
        "vcycle": {"ms": round(vc_ms / max(ncycles, 1), 4), "algorithmic_GBps": round(vc_bytes / vc_ms / 1e6, 1)},
        "complexity": {"grid": round(results[-1]["grid_complexity"], 4),
                       "operator": round(results[-1]["op_complexity"], 4)},
        "kernels": breakdown,
    }
    # the same steps with the V-cycle replayed from a captured graph (kernel
    # timing off): time-to-solution only
    mg.set_timing(False)
    mg.set_graph(True)
    gtimes = []
    for k in range(1 + args.steps):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        mg.resetup(A)
        x.zero_()
        rg = mg.solve(b, x, rtol=1e-9, maxit=300, krylov=W["krylov"])
        torch.cuda.synchronize()
        if k > 0:
            gtimes.append((time.perf_counter() - ts) * 1e3)
    line["graph"] = {"ms_per_step": round(float(np.mean(gtimes)), 2), "iters": rg["iters"],
                     "converged": rg["status"] == 0 and rg["rel_resid_true"] < 1e-9}
    if W["interp"] != "vertex":
        # the same steps with the plain trilinear interpolation, for reference
        mg.set_timing(False)
        mv = smg.StructMG(A, shape, device=dev, **dict(kw, interp="vertex"))
        vtimes, rv = [], None
        for k in range(1 + args.steps):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            mv.resetup(A)
            x.zero_()
            rv = mv.solve(b, x, rtol=1e-9, maxit=300, krylov=W["krylov"])
            torch.cuda.synchronize()
            if k > 0:
                vtimes.append((time.perf_counter() - ts) * 1e3)
        vms = float(np.mean(vtimes))
        line["trilinear"] = {"ms_per_step": round(vms, 2), "iters": rv["iters"],
                             "converged": rv["status"] == 0 and rv["rel_resid_true"] < 1e-9,
                             "speedup_of_default": round(vms / ms_per_step, 3)}
        mv.close()
        del mv
    if not args.no_mixed:
        # the same workload with the V-cycle in FP32 and in FP16 (per-row
        # scaled) storage, inside the FP64 PCG: time-to-solution against FP64
        mg.set_timing(False)
        mixed = {}
        for prec in ("fp32", "fp16"):
            m2 = smg.StructMG(A, shape, device=dev, prec=prec, **kw)
            times, r = [], None
            for k in range(1 + args.steps):
                torch.cuda.synchronize()
                ts = time.perf_counter()
                m2.resetup(A)
                x.zero_()
                r = m2.solve(b, x, rtol=1e-9, maxit=300, krylov=W["krylov"])
                torch.cuda.synchronize()
                if k > 0:
                    times.append((time.perf_counter() - ts) * 1e3)
            ms = float(np.mean(times))
            mixed[prec] = {"ms_per_step": round(ms, 2), "iters": r["iters"], "rel_resid_true": r["rel_resid_true"],
                           "converged": r["status"] == 0 and r["rel_resid_true"] < 1e-9,
                           "t_setup_ms": round(r["t_setup_ms"], 2), "t_solve_ms": round(r["t_solve_ms"], 2),
                           "speedup_vs_fp64": round(ms_per_step / ms, 3)}
            m2.close()
            del m2
        line["mixed"] = mixed
    mg.close()
    del mg, A, b, x
    torch.cuda.empty_cache()
    # the other configurations of the metric, each as a sub-object
    wanted = [c.strip() for c in args.configs.split(",") if c.strip() and c.strip().lower() != "none"]
    if wanted:
        line["configs"] = {}
        for key, fn in CONFIG_RUNNERS.items():
            if key.split("_")[0] not in wanted:
                continue
            ts = time.perf_counter()
            print(f"[bench] configuration {key}", file=sys.stderr, flush=True)
            line["configs"][key] = fn(args, smg, torch, np, dev, min(args.steps, 3))
            line["configs"][key]["bench_wall_s"] = round(time.perf_counter() - ts, 1)
            print(f"[bench] {key} done in {time.perf_counter() - ts:.1f}s", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        line["cpu_baseline"], sample = cpu_baseline(args.workload, W["interp"], gpu_iters=line["iters"])
        line["oracle_error"] = oracle_errors(smg, torch, np, dev, sample, kw, W["krylov"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
