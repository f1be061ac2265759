"""Benchmark: DMRG sigma GFLOP/s (and, when available, the DMRG-TDA sweep
time) on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 4] [--M 1000]
                    [--nroots 16] [--prec fp64] [--no-cpu-baseline]

Workload (synthetic, seeded): the [2Fe-2S]-shaped problem L=36 orbitals,
N=30 electrons, Sz=0, a 10-orbital near-degenerate block with strong
exchange (K=108 Cholesky rank), a random mixed-canonical MPS with M=1000.
A step is one sigma of the one-site effective Hamiltonian at the middle site
for all TDA roots at once (nroots vectors resident in HBM).  One JSON line is
printed (rank 0).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16x3": 2.5e15}  # dense MI355X peaks
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
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import mps_arrays

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--M", type=int, default=1000)
    ap.add_argument("--nroots", type=int, default=16)
    ap.add_argument("--prec", default="fp64", choices=["fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    a = ap.parse_args()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1311_1646_amd as lib
    import synth
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from helpers import mps_arrays

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
    C = torch.randn(a.nroots, size, dtype=torch.float64, device="cuda", generator=None)
    S = torch.empty_like(C)
    for w in range(a.warmup):
        ctx.sigma(site, C, out=S)
        log(f"[bench] warmup {w} done")
    torch.cuda.synchronize()
    fl = ms = mms = 0.0
    t0 = time.perf_counter()
    for k in range(a.steps):
        ctx.sigma(site, C, out=S)
        s = ctx.stats()
        fl += s["sigma_flops"]
        ms += s["sigma_ms"]
        mms += s["sigma_main_ms"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    value = fl / (ms * 1e-3) / 1e9
    main_flops = None
    out = {
        "metric": "sigma GFLOP/s (TDA sigma, all roots, middle site)",
        "value": round(value, 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(wall / a.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{p.name} M={p.M} random mixed-canonical MPS, site {site}, "
                               f"{a.nroots} vectors, zeroth-order sigma",
                   "L": p.L, "N": p.Na + p.Nb, "M": p.M, "nroots": a.nroots, "site": site,
                   "sigma_size": size, "sigma_device_ms": round(ms / a.steps, 3)},
        "roofline": {"bound": "mfma", "achieved": None, "peak": PEAK[a.prec], "unit": "TFLOP/s",
                     "frac": None, "traffic": None},
    }
    # dominant kernel: the stage-2 grouped GEMM of the sigma
    s = ctx.stats()
    if s["sigma_main_ms"] > 0 and s["sigma_main_flops"] > 0:
        main_flops = s["sigma_main_flops"]
        ach = main_flops / (s["sigma_main_ms"] * 1e-3)
        out["roofline"]["achieved"] = round(ach / 1e12, 3)
        out["roofline"]["peak"] = PEAK[a.prec] / 1e12
        out["roofline"]["frac"] = round(ach / PEAK[a.prec], 4)
    else:
        ach = fl / (ms * 1e-3)
        out["roofline"]["achieved"] = round(ach / 1e12, 3)
        out["roofline"]["peak"] = PEAK[a.prec] / 1e12
        out["roofline"]["frac"] = round(ach / PEAK[a.prec], 4)
    if not a.no_cpu_baseline:
        try:
            out["cpu_baseline"] = cpu_baseline(a.nroots)
        except Exception as e:  # reported, never fatal
            out["cpu_baseline"] = {"error": str(e)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
