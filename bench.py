"""Benchmark: DMRG sigma GFLOP/s and DMRG-TDA sweep time on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 4] [--M 1000]
                    [--nroots 16] [--prec fp32] [--ladder] [--tda-iters 1]
                    [--copy-calib] [--no-cpu-baseline] [--no-autotune]
                    [--no-sweep-avg]

Workload (synthetic, seeded): the [2Fe-2S]-shaped problem L=36 orbitals,
N=30 electrons, Sz=0, a 10-orbital near-degenerate block with strong
exchange (K=108 Cholesky rank), a random mixed-canonical MPS with M=1000.
A step is one sigma of the one-site effective Hamiltonian at the middle site
for all TDA roots at once (nroots vectors resident in HBM); `value` is its
rate.  After the timed steps, one DMRG-TDA Davidson iteration (a forward and
a backward sweep over all sites with l = 2 nroots trial vectors) is timed
and reported as `tda_sweep_s`, with the TDA sigma of the middle site measured
inside that iteration; then the zeroth-order sigma at every site once gives
the sweep-averaged rate.  Before timing a precision, the tile-shape
autotuner picks the stage shapes (--no-autotune keeps the planner's).
--copy-calib first runs one 256 MiB device
copy, so that a hardware-counter run of this command also measures a
transfer of known size.  One JSON line is printed.
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
HBM_PEAK = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(nvec):
    """The FP64 oracle (dense explicit H_eff = P^T H P applied to nvec vectors)
    at the L=8, N=8, M=64 middle site, timed on this host; its rate is the
    algorithmic flop count of the same block-sparse sigma divided by the
    oracle's time.  A reported baseline, not a target."""
    import numpy as np
    import torch

    import paper_1311_1646_amd as lib
    import synth
    from oracle import fci, mpsvec
    from synth import mps_arrays

    p = synth.config(0)
    mps = synth.random_mps(p.L, p.Na, p.Nb, p.M, seed=17)
    i = p.L // 2
    dets, H = fci.hamiltonian(p.h, p.eri, p.ecore, p.Na, p.Nb)
    C = np.random.default_rng(0).normal(size=(nvec, mps.site_size(i)))
    # algorithmic flops of this sigma, counted by the library's rule
    ctx = lib.Context(p.L, p.Na, p.Nb, p.h, p.eri, p.ecore, device=0)
    ctx.import_mps(*mps_arrays(mps))
    ctx.build_ops()
    ctx.sigma(i, torch.tensor(C, device="cuda"))
    flops = ctx.stats()["sigma_flops"]
    ctx.close()
    reps, t_tot = 0, 0.0
    while t_tot < 12.0 and reps < 50:
        t0 = time.perf_counter()
        P = mpsvec.site_basis(mps, dets, i)
        _ = C @ mpsvec.heff(H, P).T
        t_tot += time.perf_counter() - t0
        reps += 1
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": flops * reps / t_tot / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"dense H_eff sigma, L=8 N=8 M=64 middle site, {nvec} vectors, {reps} reps "
                      f"in {t_tot:.1f} s; rate = block-sparse algorithmic flops / oracle time"}


def time_sigma(ctx, lib, site, C, S, name, steps, warmup):
    """Warm up, then time `steps` sigmas of all vectors in precision `name`;
    device times come from the library's events on its stream."""
    import torch
    prec = {"fp64": lib.FP64, "fp32": lib.FP32, "bf16x3": lib.BF16X3}[name]
    for _ in range(warmup):
        ctx.sigma(site, C, out=S, prec=prec)
    torch.cuda.synchronize()
    fl = ms = mms = mfl = 0.0
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.sigma(site, C, out=S, prec=prec)
        s = ctx.stats()
        fl += s["sigma_flops"]
        ms += s["sigma_ms"]
        mms += s["sigma_main_ms"]
        mfl += s["sigma_main_flops"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return {"gflops": round(fl / (ms * 1e-3) / 1e9, 2), "device_ms": round(ms / steps, 3),
            "wall_ms": round(wall / steps * 1e3, 3), "main_ms": mms / steps, "main_flops": mfl / steps,
            "main_bytes": s["sigma_main_bytes"], "main_launches": s["sigma_main_launches"]}


def sweep_averaged_sigma(ctx, lib, L, nvec, name):
    """Zeroth-order sigma for nvec vectors at every site once (plans built
    first, outside the timing): total flops / total device time."""
    import torch
    prec = {"fp64": lib.FP64, "fp32": lib.FP32, "bf16x3": lib.BF16X3}[name]
    bufs = []
    for i in range(L):
        _, n = ctx.layout(i)
        C = torch.randn(nvec, n, dtype=torch.float64, device="cuda")
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


def measured_traffic(prec, M):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary, or None when there is none for this precision and workload or
    the kernel source changed since the counters were taken."""
    import hashlib
    f = os.path.join(ROOT, "profiles", "sigma_accumulate_traffic.json")
    if not os.path.exists(f):
        return None
    d = json.load(open(f))
    src = open(os.path.join(ROOT, "paper_1311_1646_amd", "csrc", "kernels_mfma.hip"), "rb").read()
    if d.get("kernel_sha256") != hashlib.sha256(src).hexdigest() or d.get("prec") != prec or d.get("M") != M:
        return None
    return d["hbm_bytes_per_launch"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--M", type=int, default=1000)
    ap.add_argument("--nroots", type=int, default=16)
    ap.add_argument("--prec", default="fp32", choices=list(PRECS))
    ap.add_argument("--ladder", action="store_true", help="also time the other precisions")
    ap.add_argument("--tda-iters", type=int, default=1, help="TDA Davidson iterations to time (0: none)")
    ap.add_argument("--copy-calib", action="store_true", help="run one 256 MiB device copy first")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the planner's tile shapes")
    ap.add_argument("--no-sweep-avg", action="store_true", help="skip the sigma at every site")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
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
    site = p.L // 2
    _, size = ctx.layout(site)
    C = torch.randn(a.nroots, size, dtype=torch.float64, device="cuda")
    S = torch.empty_like(C)
    ladder = {}
    tuned = {}
    for name in PRECS:
        if name != a.prec and not a.ladder:
            continue
        if not a.no_autotune:
            pr = {"fp64": lib.FP64, "fp32": lib.FP32, "bf16x3": lib.BF16X3}[name]
            s1, s2, ms = ctx.autotune(site, a.nroots, pr)
            names = {-1: "planner", 0: "64x64", 1: "128x64", 2: "64x128"}
            tuned[name] = {"stage1": names[s1], "stage2": names[s2]}
            log(f"[bench] autotune {name}: {tuned[name]} ({ms:.1f} ms)")
        ladder[name] = time_sigma(ctx, lib, site, C, S, name, a.steps, a.warmup)
        log(f"[bench] {name}: {ladder[name]}")
    head = ladder[a.prec]
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
        "config": {"workload": f"{p.name} M={p.M} random mixed-canonical MPS, site {site}, "
                               f"{a.nroots} vectors, zeroth-order sigma, {a.prec} contractions",
                   "L": p.L, "N": p.Na + p.Nb, "M": p.M, "nroots": a.nroots, "site": site,
                   "sigma_size": size, "sigma_device_ms": head["device_ms"],
                   "op_GiB": round(st["op_bytes"] / 2**30, 2),
                   "build_ops": {"prec": "fp64", "device_ms": round(st["renorm_ms"], 1),
                                 "GFLOP/s": round(st["renorm_flops"] / max(st["renorm_ms"], 1e-9) / 1e6, 1),
                                 "host_planning_ms": round(st["plan_ms"], 1)},
                   "precision_ladder": {k: {"GFLOP/s": v["gflops"], "device_ms": v["device_ms"]}
                                        for k, v in ladder.items()},
                   "tile_shapes": tuned or "planner"},
    }
    # dominant kernel: the accumulation stage (grouped GEMM, role 1) of the
    # sigma; per launch = per sigma / launches, so the ratio is the same
    ach = head["main_flops"] / (max(head["main_ms"], 1e-9) * 1e-3)
    nl = max(head["main_launches"], 1)
    out["roofline"] = {"bound": "mfma", "achieved": round(ach / 1e12, 3), "peak": PEAK[a.prec] / 1e12,
                       "unit": "TFLOP/s", "frac": round(ach / PEAK[a.prec], 4),
                       "traffic": measured_traffic(a.prec, p.M)}
    out["config"]["dominant_kernel"] = {
        "name": "ggemm_mfma_kernel<%d, 1, TM, TN>" % {"fp64": 0, "fp32": 1, "bf16x3": 2}[a.prec],
        "launches_per_sigma": nl, "avg_launch_ms": round(head["main_ms"] / nl, 4),
        "flops_per_launch": head["main_flops"] / nl, "algorithmic_bytes_per_launch": head["main_bytes"] / nl}
    if a.tda_iters > 0:
        prec = {"fp64": lib.FP64, "fp32": lib.FP32, "bf16x3": lib.BF16X3}[a.prec]
        t0 = time.perf_counter()
        _, _, _, its, _ = ctx.tda_roots(a.nroots, max_iter=a.tda_iters, tol=0.0, seed=7, prec=prec, verbose=1)
        wall = time.perf_counter() - t0
        s = ctx.stats()
        out["tda_sweep_s"] = round(s["tda_iter_ms"] / 1e3, 3)
        out["tda"] = {"iterations": its, "trial_vectors": 2 * a.nroots, "last_iteration_s": round(s["tda_iter_ms"] / 1e3, 3),
                      "total_s_incl_setup": round(wall, 2), "prec": a.prec}
        if s["tda_sigma_ms"] > 0:
            # TDA sigma of the middle site inside that iteration: first-order
            # left part for all trial vectors + zeroth-order part for the roots
            out["tda"]["middle_site_tda_sigma"] = {
                "GFLOP/s": round(s["tda_sigma_flops"] / (s["tda_sigma_ms"] * 1e-3) / 1e9, 2),
                "device_ms": round(s["tda_sigma_ms"], 3), "flops": s["tda_sigma_flops"]}
        log(f"[bench] TDA: {out['tda']}")
    if not a.no_sweep_avg:
        out["config"]["sweep_averaged_sigma"] = sweep_averaged_sigma(ctx, lib, p.L, a.nroots, a.prec)
        log(f"[bench] sweep-averaged sigma: {out['config']['sweep_averaged_sigma']}")
    if not a.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(a.nroots)
        except Exception as e:  # reported, never fatal
            out["cpu_baseline"] = {"error": str(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
