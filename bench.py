"""Benchmark of the Wilson-fermion HMC hot path on one MI355X.

Workload: the 16^4 lattice (eps = 0.3 links, beta = 6.0, kappa = 0.125, one
pseudofermion phi = D^dag eta from a Gaussian eta), i.e. the configuration the
headline metric is quoted on.  A step is one pseudofermion-force call
(lgt_fermion_force: two even/odd CG solves to an FP64 true residual of 1e-10,
then the adjoint kernel), with links and phi resident in HBM.  The timed K
steps use the mixed-precision solver (FP32 inner CG, FP64 reliable updates);
the same K calls in plain FP64 are timed after them and reported beside it.

Also reported: the roofline of the CG's dominant kernel (the even/odd hop),
timed with HIP events on the library's stream, and the FP64 CPU oracle timed
on a bounded sample of the same call on this host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(u, eta, kappa, target_tol, budget_s=20.0):
    """FP64 oracle on this host: a bounded run of its CG, extrapolated.

    Runs the oracle's unpreconditioned CG on D^dag D for up to budget_s
    seconds, fits the log-residual slope to predict the iterations needed for
    target_tol, and adds one full adjoint (force) evaluation, timed.
    """
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import dirac, force, solver

    with threadpool_limits(limits=1):
        phi = dirac.dslash_dag(u, eta, kappa)
        t_start = time.perf_counter()
        b = phi
        x = np.zeros_like(b)
        r = b.copy()
        p = r.copy()
        bb = solver.norm2(b)
        rr = bb
        hist = []
        t_it0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t_start < budget_s and rr > target_tol ** 2 * bb:
            q = dirac.ddag_d(u, p, kappa)
            alpha = rr / float(np.real(np.vdot(p.ravel(), q.ravel())))
            x = x + alpha * p
            r = r - alpha * q
            rr_new = solver.norm2(r)
            p = r + (rr_new / rr) * p
            rr = rr_new
            k += 1
            hist.append(rr)
        t_iter = (time.perf_counter() - t_it0) / max(k, 1)
        # predicted iterations to target from the average convergence rate
        if k >= 2 and rr > target_tol ** 2 * bb:
            rate = (np.log(hist[-1]) - np.log(bb)) / k
            n_pred = int(np.ceil(np.log(target_tol ** 2) / rate))
        else:
            n_pred = k
        t0 = time.perf_counter()
        y = dirac.dslash(u, x, kappa)
        force.fermion_force_from_solution(u, x, y, kappa)
        t_force = time.perf_counter() - t0
    total = t_iter * n_pred + t_force
    return {
        "value": total * 1e3, "unit": "ms/call", "cores": 1, "kind": "oracle",
        "sample": f"{k} unpreconditioned CG iterations on the 16^4 workload ({t_iter:.3f} s each), "
                  f"extrapolated to {n_pred} iterations for residual {target_tol:g}, plus one full "
                  f"adjoint+D ({t_force:.2f} s); NumPy FP64, BLAS limited to 1 thread; "
                  f"host has {len(os.sched_getaffinity(0))} cores",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path here is single-GPU (no collectives); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import lgt_inputs as li
    import paper_2602_20516_amd as lgt

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    c = li.config(2)
    dims, eps, beta, kappa, tol = c["dims"], c["eps"], c["beta"], c["kappa"], c["tol"]
    V = int(np.prod(dims))
    u = li.random_links(dims, eps, c["seeds"]["links"])
    eta = li.gaussian_spinor(dims, c["seeds"]["eta"])
    U = torch.from_numpy(u).to("cuda")
    E = torch.from_numpy(eta).to("cuda")
    lat = lgt.Lattice(dims)
    phi = lat.dslash(U, E, kappa, dagger=True)    # heat bath phi = D^dag eta, on the GPU
    out = lat.empty_gauge()
    p_mixed = lgt.Params(precision="mixed_fp32", tol=tol)
    p_fp64 = lgt.Params(precision="fp64", tol=tol)

    def run(params, n):
        st = None
        for _ in range(n):
            _, st = lat.fermion_force(U, phi, kappa, params, out=out)
        return st

    log(f"bench: warmup {args.warmup}")
    run(p_mixed, args.warmup)
    run(p_fp64, max(1, args.warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_mixed = run(p_mixed, args.steps)
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / args.steps
    log(f"bench: mixed {t_mixed * 1e3:.3f} ms/call {st_mixed}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_fp64 = run(p_fp64, args.steps)
    torch.cuda.synchronize()
    t_fp64 = (time.perf_counter() - t0) / args.steps
    log(f"bench: fp64 {t_fp64 * 1e3:.3f} ms/call {st_fp64}")

    # dominant kernel: the even/odd hop (FP32 in the timed mixed path), HIP
    # events on the library stream; FP64 beside it
    hop_ms32 = lat.hop_benchmark(U, E, "mixed_fp32", 200)
    hop_ms64 = lat.hop_benchmark(U, E, "fp64", 200)
    hop_bytes32 = 96 * 4 * V
    hop_bytes64 = 96 * 8 * V
    gbs32 = hop_bytes32 / (hop_ms32 * 1e-3) / 1e9
    gbs64 = hop_bytes64 / (hop_ms64 * 1e-3) / 1e9
    log(f"bench: hop fp32 {hop_ms32 * 1e3:.2f} us {gbs32:.0f} GB/s; fp64 {hop_ms64 * 1e3:.2f} us {gbs64:.0f} GB/s")

    # effective GB/s of the whole call: compulsory bytes of the CG iterations
    # (516 reals per site per e/o CGNR iteration) and of the force kernel
    def eff_gbs(st, p_bytes, t):
        byts = st["iters"] * 516 * p_bytes * V + 192 * 8 * V
        return byts / t / 1e9

    def traffic(name):
        # HBM bytes per launch from the committed counter passes of this kernel
        path = os.path.join(ROOT, "profiles", name)
        try:
            with open(path) as f:
                return json.load(f).get("bytes_per_launch")
        except (OSError, ValueError):
            return None

    rec = {
        "metric": "fermion force (CG+adjoint) ms/call & HBM GB/s, mixed vs FP64 at 16^4",
        "value": round(t_mixed * 1e3, 4),
        "unit": "ms/call",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_mixed * 1e3, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64 (mixed: FP32 inner CG, FP64 residual/force)",
        "data": "synthetic (seeded SU(3) links eps=0.3, Gaussian eta)",
        "config": {"workload": "16^4 Wilson-fermion force: phi = D^dag eta, two even/odd CG solves to "
                               "FP64 true residual 1e-10, adjoint kernel",
                   "dims": list(dims), "beta": beta, "kappa": kappa, "tol": tol, "fermion_bc": -1},
        "mixed": {"ms_per_call": round(t_mixed * 1e3, 4), "iters": st_mixed["iters"],
                  "reliable_updates": st_mixed["reliable_updates"],
                  "true_rel_residual": st_mixed["true_rel_residual"],
                  "effective_GBs": round(eff_gbs(st_mixed, 4, t_mixed), 1)},
        "fp64": {"ms_per_call": round(t_fp64 * 1e3, 4), "iters": st_fp64["iters"],
                 "true_rel_residual": st_fp64["true_rel_residual"],
                 "effective_GBs": round(eff_gbs(st_fp64, 8, t_fp64), 1)},
        "speedup_mixed_vs_fp64": round(t_fp64 / t_mixed, 3),
        "roofline": {"kernel": "even/odd hop H_eo, FP32 (k_hop<float,false,EpiAxpy<float>>)", "bound": "hbm",
                     "achieved": round(gbs32, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs32 / HBM_PEAK_GBS, 4),
                     "traffic": traffic("hop_fp32_16x16x16x16_traffic.json"),
                     "avg_launch_us": round(hop_ms32 * 1e3, 3), "algorithmic_bytes_per_launch": hop_bytes32,
                     "fp64": {"achieved": round(gbs64, 1), "frac": round(gbs64 / HBM_PEAK_GBS, 4),
                              "avg_launch_us": round(hop_ms64 * 1e3, 3),
                              "algorithmic_bytes_per_launch": hop_bytes64,
                              "traffic": traffic("hop_fp64_16x16x16x16_traffic.json")}},
    }
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        rec["cpu_baseline"] = cpu_baseline(u, eta, kappa, tol, args.cpu_budget)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
