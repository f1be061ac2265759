"""Benchmark: DMRG-TDA sigma GFLOP/s and DMRG-TDA sweep time on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 4] [--M 1000]
                    [--nroots 16] [--prec fp32] [--precs fp64,fp32,bf16x3]
                    [--tda-iters 1] [--converge] [--copy-calib]
                    [--no-cpu-baseline] [--no-autotune] [--no-sweep-avg]

Workload (synthetic, seeded; the paper's molecular integrals are not
available): the [2Fe-2S]-shaped problem, L=36 orbitals, N=30 electrons,
Sz=0, a 10-orbital near-degenerate block with strong exchange (K=108
Cholesky rank), a random mixed-canonical MPS with M=1000.

A step is the full TDA sigma of Sec. III D (eq. sigv1 with Delta-sigma of
eq. sigv2) at the middle site for all nroots first-order wavefunctions at
once: the zeroth-order part H_0^[i] C^(1) plus the first-order left and right
parts, whose operators (eqs. lopr1st, ropr1st) are built beforehand, outside
the timing, from seeded random first-order tensors at every other site.
`value` is its rate in the headline precision (--prec).  Every precision
of the ladder (--precs) is timed the same way (with its own first-order
chains), together with the zeroth-order sigma alone and one DMRG-TDA
Davidson iteration (a forward and a backward sweep with l = 2 nroots trial
vectors, alg:dmrgtda), whose wall time is the "TDA sweep s" of the metric.
--converge also runs the headline precision's TDA to convergence and
reports the iteration count and the time to convergence (minutes at
M=1000).  Before timing a precision, the tile-shape autotuner picks the
stage shapes (--no-autotune keeps the planner's).  --copy-calib first runs
one 256 MiB device copy, so that a hardware-counter run of this command also
measures a transfer of known size.  One JSON line is printed.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# dense MI355X peaks; BF16x3 is priced at a third of the BF16 peak (three
# matrix-core products per algorithmic multiply-add)
PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16x3": 2.5e15 / 3}
PRECS = ("fp64", "fp32", "bf16x3")
DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16x3-f32acc"}
KERNEL_MODE = {"fp64": 0, "fp32": 1, "bf16x3": 2}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def prec_id(lib, name):
    return {"fp64": lib.FP64, "fp32": lib.FP32, "bf16x3": lib.BF16X3}[name]


def cpu_baseline(nvec):
    """The FP64 oracle's TDA sigma (oracle.firstorder.tda_sigma: the
    first-order wavefunction as an FCI vector, H applied as a sparse matrix,
    then projected on the one-site product basis) at the largest workload it
    handles in seconds: the PPP chain L=12 (3+3 electrons, 48400
    determinants), random MPS with M=400, middle site 6, first-order tensors
    at every site.  The FCI Hamiltonian and the inputs are built outside the
    timer; the rate is the library's algorithmic flop count of the same TDA
    sigma divided by the oracle's time.  The [2Fe-2S]-shaped workload itself
    (L=36) is far beyond a determinant-space oracle, so there is no CPU
    baseline at the benchmark's own size."""
    import numpy as np
    import torch

    import paper_1311_1646_amd as lib
    import synth
    from oracle import fci, firstorder
    from synth import mps_arrays

    L, Na, Nb, M, i = 12, 3, 3, 400, 6
    h, eri, _ = synth.ppp_integrals(L)
    mps = synth.random_mps(L, Na, Nb, M, seed=5)
    dets, H = fci.hamiltonian(h, eri, 0.0, Na, Nb)
    rng = np.random.default_rng(11)
    X = [rng.normal(size=(nvec, mps.site_size(j))) for j in range(L)]
    # algorithmic flops of this sigma, counted by the library's rule
    ctx = lib.Context(L, Na, Nb, h, eri, 0.0, device=0)
    ctx.import_mps(*mps_arrays(mps))
    ctx.build_ops()
    for j in range(i):
        ctx.renormalize(j, lib.DIR_LEFT, lib.FIRST, lib.FP64, A1=torch.tensor(X[j], device="cuda"))
    for j in range(L - 1, i, -1):
        ctx.renormalize(j, lib.DIR_RIGHT, lib.FIRST, lib.FP64, A1=torch.tensor(X[j], device="cuda"))
    ctx.sigma(i, torch.tensor(X[i], device="cuda"), kind=lib.SIGMA_TDA_FULL)
    flops_per_vec = ctx.stats()["sigma_flops"] / nvec
    ctx.close()
    ins = []
    for v in range(nvec):
        L1 = {j: firstorder.blocks(mps, j, X[j][v]) for j in range(i)}
        R1 = {j: firstorder.blocks(mps, j, X[j][v]) for j in range(i + 1, L)}
        ins.append((L1, firstorder.blocks(mps, i, X[i][v]), R1))
    done, t_tot = 0, 0.0
    while t_tot < 12.0 and done < 64 * nvec:
        L1, C1, R1 = ins[done % nvec]
        t0 = time.perf_counter()
        firstorder.tda_sigma(H, mps, dets, i, L1, C1, R1)
        t_tot += time.perf_counter() - t0
        done += 1
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(flops_per_vec * done / t_tot / 1e9, 4), "unit": "GFLOP/s", "cores": threads,
            "kind": "oracle",
            "sample": f"oracle TDA sigma (P_i^T H Psi1) at ppp-L12-N6 M=400 site {i}: {done} vectors in "
                      f"{t_tot:.1f} s; rate = the library's algorithmic flops of that sigma / oracle time; "
                      f"no CPU baseline at the L=36 workload (beyond a determinant-space oracle)"}


def build_chains(ctx, lib, L, site, nvec, prec, seed):
    """First-order operators for nvec seeded random first-order tensors at
    every site but `site` (left chain 0..site-1, right chain L-1..site+1)."""
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    t0 = time.perf_counter()
    for j in range(site):
        A = torch.randn(nvec, ctx.size(j), dtype=torch.float64, device="cuda", generator=g)
        ctx.renormalize(j, lib.DIR_LEFT, lib.FIRST, prec, A1=A)
    for j in range(L - 1, site, -1):
        A = torch.randn(nvec, ctx.size(j), dtype=torch.float64, device="cuda", generator=g)
        ctx.renormalize(j, lib.DIR_RIGHT, lib.FIRST, prec, A1=A)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def time_sigma(ctx, lib, site, C, S, prec, kind, steps, warmup):
    """Warm up, then time `steps` sigmas of all vectors; device times come
    from the library's events on its stream, the wall time from the host
    clock between two synchronizations."""
    import torch
    for _ in range(warmup):
        ctx.sigma(site, C, out=S, prec=prec, kind=kind)
    torch.cuda.synchronize()
    fl = ms = mms = mfl = mby = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.sigma(site, C, out=S, prec=prec, kind=kind)
        s = ctx.stats()
        fl += s["sigma_flops"]
        ms += s["sigma_ms"]
        mms += s["sigma_main_ms"]
        mfl += s["sigma_main_flops"]
        mby += s["sigma_main_bytes"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"gflops": round(fl / (ms * 1e-3) / 1e9, 2), "device_ms": round(ms / steps, 3),
            "wall_ms": round(wall / steps * 1e3, 3), "timed_s": round(wall, 3), "main_ms": mms / steps,
            "main_flops": mfl / steps, "main_bytes": mby / steps, "main_launches": s["sigma_main_launches"],
            "flops": fl / steps}


def sweep_averaged_sigma(ctx, lib, L, nvec, prec):
    """Zeroth-order sigma for nvec vectors at every site once (plans built
    first, outside the timing): total flops / total device time."""
    import torch
    bufs = []
    for i in range(L):
        C = torch.randn(nvec, ctx.size(i), dtype=torch.float64, device="cuda")
        bufs.append((C, torch.empty_like(C)))
        ctx.sigma(i, C, out=bufs[-1][1], prec=prec)  # plan + lists
    torch.cuda.synchronize()
    fl = ms = 0.0
    for i in range(L):
        ctx.sigma(i, bufs[i][0], out=bufs[i][1], prec=prec)
        s = ctx.stats()
        fl += s["sigma_flops"]
        ms += s["sigma_ms"]
    return {"GFLOP/s": round(fl / (ms * 1e-3) / 1e9, 2), "device_ms_all_sites": round(ms, 2), "sites": L}


def many_instances(lib, steps, warmup, n=64):
    """The many-instance workload: n independent seeded problems (L uniform
    in 8..16, N = L, M uniform in 32..256, random integrals as the small
    dense check), each with its own random MPS; the zeroth-order sigma of
    all n at their middle sites for nroots = 4 vectors each, FP32, as one
    grouped launch per contraction stage (dmrg_group_*) replayed from a HIP
    graph.  Compared with the same n sigmas issued context by context."""
    import torch

    import synth
    from synth import mps_arrays
    t0 = time.perf_counter()
    ctxs, sites, Cs, outs = [], [], [], []
    g = torch.Generator(device="cuda").manual_seed(33)
    for i in range(n):
        p = synth.config(3, instance=i)
        mps = synth.random_mps(p.L, p.Na, p.Nb, p.M, seed=3000 + i)
        c = lib.Context(p.L, p.Na, p.Nb, p.h, p.eri, p.ecore, device=0)
        c.import_mps(*mps_arrays(mps))
        c.build_ops(lib.FP64)
        site = p.L // 2
        ctxs.append(c)
        sites.append(site)
        Cs.append(torch.randn(p.nroots, c.size(site), dtype=torch.float64, device="cuda", generator=g))
        outs.append(torch.empty_like(Cs[-1]))
    setup = time.perf_counter() - t0
    # context by context (plans and FP32 copies built by the warm-up)
    for c, i, C, O in zip(ctxs, sites, Cs, outs):
        c.sigma(i, C, out=O, prec=lib.FP32)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev = 0.0
    for _ in range(steps):
        for c, i, C, O in zip(ctxs, sites, Cs, outs):
            c.sigma(i, C, out=O, prec=lib.FP32)
            dev += c.stats()["sigma_ms"]
    torch.cuda.synchronize()
    single_wall = (time.perf_counter() - t0) / steps * 1e3
    grp = lib.Group(ctxs, sites, 4, prec=lib.FP32)
    for _ in range(max(warmup, 2)):  # eager step, then graph capture
        grp.sigma(Cs, outs, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = 0.0
    for _ in range(steps):
        grp.sigma(Cs, outs, graph=True)
        ms += grp.stats()["ms"]
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps * 1e3
    st = grp.stats()
    grp.close()
    for c in ctxs:
        c.close()
    return {"instances": n, "prec": "fp32", "vectors_per_instance": 4,
            "aggregate_GFLOP/s": round(st["flops"] / (ms / steps * 1e-3) / 1e9, 2),
            "device_ms_per_step": round(ms / steps, 4), "wall_ms_per_step": round(wall, 4),
            "launches_per_step": st["launches"], "graph_nodes": st["graph_nodes"],
            "flops_per_step": st["flops"],
            "one_context_at_a_time": {"device_ms_per_step": round(dev / steps, 4),
                                      "wall_ms_per_step": round(single_wall, 4)},
            "setup_s": round(setup, 1)}


def measured_traffic(prec, M):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (profiles/), or None when there is none for this precision and
    workload or the kernel source changed since the counters were taken."""
    import hashlib
    f = os.path.join(ROOT, "profiles", "tda_sigma_accumulate_traffic.json")
    if not os.path.exists(f):
        return None
    d = json.load(open(f))
    src = open(os.path.join(ROOT, "paper_1311_1646_amd", "csrc", "kernels_mfma.hip"), "rb").read()
    if d.get("kernel_sha256") != hashlib.sha256(src).hexdigest() or d.get("prec") != prec or d.get("M") != M:
        return None
    return d["hbm_bytes_per_launch"], d["source"]


def roofline(r, name):
    ach = r["main_flops"] / (max(r["main_ms"], 1e-9) * 1e-3)
    return {"bound": "mfma", "achieved": round(ach / 1e12, 3), "peak": PEAK[name] / 1e12, "unit": "TFLOP/s",
            "frac": round(ach / PEAK[name], 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--M", type=int, default=1000)
    ap.add_argument("--nroots", type=int, default=16)
    ap.add_argument("--prec", default="fp32", choices=list(PRECS), help="headline precision")
    ap.add_argument("--precs", default="fp64,fp32,bf16x3", help="precision ladder (comma separated)")
    ap.add_argument("--tda-iters", type=int, default=1, help="TDA Davidson iterations to time per precision (0: none)")
    ap.add_argument("--converge", action="store_true", help="also run the headline TDA to convergence")
    ap.add_argument("--copy-calib", action="store_true", help="run one 256 MiB device copy first")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the planner's tile shapes")
    ap.add_argument("--no-sweep-avg", action="store_true", help="skip the zeroth-order sigma at every site")
    ap.add_argument("--no-group", action="store_true", help="skip the many-instance grouped sigma")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only (no multi-GPU path); --gpus must be 1"}))
        sys.exit(2)
    ladder_names = [p for p in PRECS if p in a.precs.split(",") or p == a.prec]

    import torch

    import paper_1311_1646_amd as lib
    import synth
    from synth import mps_arrays

    if a.copy_calib:
        src = torch.ones(32 << 20, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    p = synth.config(a.config, M=a.M)
    t0 = time.perf_counter()
    mps = synth.random_mps(p.L, p.Na, p.Nb, p.M, seed=1000 * a.config + 1)
    log(f"[bench] MPS L={p.L} M={p.M} generated in {time.perf_counter() - t0:.1f}s")
    ctx = lib.Context(p.L, p.Na, p.Nb, p.h, p.eri, p.ecore, device=0)
    ctx.import_mps(*mps_arrays(mps))
    t0 = time.perf_counter()
    ctx.build_ops(lib.FP64)
    st = ctx.stats()
    log(f"[bench] build_ops {time.perf_counter() - t0:.1f}s, device {st['renorm_ms']:.0f} ms, "
        f"ops {st['op_bytes'] / 2**30:.2f} GiB")
    # TDA Davidson iterations first, while no first-order chains are held
    # (an FP64 iteration at M=1000 with l=32 peaks near 210 GiB)
    tda = {}
    if a.tda_iters > 0:
        for name in ladder_names:
            t0 = time.perf_counter()
            _, _, _, its, _ = ctx.tda_roots(a.nroots, max_iter=a.tda_iters, tol=0.0, seed=7,
                                            prec=prec_id(lib, name), verbose=1, polish=False)
            wall = time.perf_counter() - t0
            s = ctx.stats()
            tda[name] = {"iteration_s": round(s["tda_iter_ms"] / 1e3, 3), "iterations": its,
                         "trial_vectors": 2 * a.nroots, "total_s_incl_setup": round(wall, 2)}
            log(f"[bench] TDA {name}: {tda[name]}")
            torch.cuda.empty_cache()
        if "fp64" in tda:
            for name in tda:
                if name != "fp64":
                    tda[name]["speedup_over_fp64"] = round(tda["fp64"]["iteration_s"] / tda[name]["iteration_s"], 3)
    site = p.L // 2
    size = ctx.size(site)
    g = torch.Generator(device="cuda").manual_seed(77)
    C = torch.randn(a.nroots, size, dtype=torch.float64, device="cuda", generator=g)
    S = torch.empty_like(C)
    ladder, tuned, res = {}, {}, {}
    for name in ladder_names:
        pr = prec_id(lib, name)
        if not a.no_autotune:
            s1, s2, ms = ctx.autotune(site, a.nroots, pr)
            names = {-1: "planner", 0: "64x64", 1: "128x64", 2: "64x128", 3: "128x128"}
            tuned[name] = {"stage1": names[s1], "stage2": names[s2]}
            log(f"[bench] autotune {name}: {tuned[name]} ({ms:.1f} ms)")
        zeroth = time_sigma(ctx, lib, site, C, S, pr, lib.SIGMA_ZEROTH_1SITE, a.steps, a.warmup)
        chain_s = build_chains(ctx, lib, p.L, site, a.nroots, pr, seed=1000 + pr)
        tdas = time_sigma(ctx, lib, site, C, S, pr, lib.SIGMA_TDA_FULL, a.steps, a.warmup)
        res[name] = tdas
        ladder[name] = {"tda_sigma_GFLOP/s": tdas["gflops"], "tda_sigma_device_ms": tdas["device_ms"],
                        "zeroth_sigma_GFLOP/s": zeroth["gflops"], "zeroth_sigma_device_ms": zeroth["device_ms"],
                        "first_order_chains_s": round(chain_s, 2), "roofline_frac": roofline(tdas, name)["frac"],
                        "dominant_kernel_TFLOP/s": roofline(tdas, name)["achieved"]}
        log(f"[bench] {name}: TDA sigma {tdas['gflops']} GFLOP/s ({tdas['device_ms']} ms), zeroth "
            f"{zeroth['gflops']} GFLOP/s, chains {chain_s:.1f}s, dominant {ladder[name]['dominant_kernel_TFLOP/s']} TF")
    head = res[a.prec]
    if "fp64" in ladder:
        for name in ladder:
            if name != "fp64":
                ladder[name]["tda_sigma_speedup_over_fp64"] = round(
                    ladder[name]["tda_sigma_GFLOP/s"] / ladder["fp64"]["tda_sigma_GFLOP/s"], 3)
    out = {
        "metric": "sigma GFLOP/s + TDA sweep s at M=1000 (FP32/BF16x3 vs FP64, 1 GPU)",
        "value": head["gflops"],
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["wall_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[a.prec],
        "data": "synthetic",
        "config": {"workload": f"{p.name} M={p.M} random mixed-canonical MPS, full TDA sigma (eq. sigv1+sigv2) "
                               f"at site {site} for {a.nroots} first-order wavefunctions, {a.prec} contractions",
                   "L": p.L, "N": p.Na + p.Nb, "M": p.M, "nroots": a.nroots, "site": site, "sigma_size": size,
                   "tda_sigma_device_ms": head["device_ms"], "tda_sigma_flops": head["flops"],
                   "op_GiB": round(st["op_bytes"] / 2**30, 2),
                   "build_ops": {"prec": "fp64", "device_ms": round(st["renorm_ms"], 1),
                                 "GFLOP/s": round(st["renorm_flops"] / max(st["renorm_ms"], 1e-9) / 1e6, 1),
                                 "host_planning_ms": round(st["plan_ms"], 1)},
                   "precision_ladder": ladder, "tile_shapes": tuned or "planner"},
    }
    # dominant kernel: the accumulation stage (grouped GEMM, role 1) of the
    # three parts of the TDA sigma; per launch = per sigma / launches
    rl = roofline(head, a.prec)
    tr = measured_traffic(a.prec, p.M)
    rl["traffic"] = tr[0] if tr else None
    rl["traffic_source"] = (f"committed rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel source, calibrated by a "
                            f"256 MiB copy ({tr[1]})" if tr else "none for this kernel source / precision / M")
    out["roofline"] = rl
    if tda:
        out["tda_sweep_s"] = tda[a.prec]["iteration_s"]
        out["tda"] = tda
    nl = max(head["main_launches"], 1)
    out["config"]["dominant_kernel"] = {
        "name": "ggemm_mfma_kernel<%d, 1, TM, TN>" % KERNEL_MODE[a.prec],
        "launches_per_sigma": nl, "avg_launch_ms": round(head["main_ms"] / nl, 4),
        "flops_per_launch": head["main_flops"] / nl, "algorithmic_bytes_per_launch": head["main_bytes"] / nl}
    if a.converge:
        t0 = time.perf_counter()
        om, et, r2, its, conv = ctx.tda_roots(a.nroots, max_iter=200, tol=1e-6, seed=7, prec=prec_id(lib, a.prec),
                                              verbose=1)
        s = ctx.stats()
        out["tda_converged"] = {"prec": a.prec, "converged": bool(conv), "iterations": its, "tol": 1e-6,
                                "time_to_convergence_s": round(time.perf_counter() - t0, 1),
                                "fp64_polish_iterations": s["tda_polish_iters"],
                                "omega_Eh": [round(float(x), 8) for x in om]}
        log(f"[bench] TDA converged: {out['tda_converged']}")
    if not a.no_sweep_avg:
        out["config"]["sweep_averaged_zeroth_sigma"] = sweep_averaged_sigma(ctx, lib, p.L, a.nroots,
                                                                            prec_id(lib, a.prec))
        log(f"[bench] sweep-averaged sigma: {out['config']['sweep_averaged_zeroth_sigma']}")
    ctx.close()
    if not a.no_group:
        out["config"]["many_instances"] = many_instances(lib, a.steps, a.warmup)
        log(f"[bench] many instances: {out['config']['many_instances']}")
    if not a.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(4)
        except Exception as e:  # reported, never fatal
            out["cpu_baseline"] = {"error": str(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
