"""Benchmark of the Wilson-fermion HMC hot path on one MI355X.

Workload: the 16^4 lattice (eps = 0.3 links, beta = 6.0, kappa = 0.125, one
pseudofermion phi = D^dag eta from a Gaussian eta), i.e. the configuration the
headline metric is quoted on.  A step is one pseudofermion-force call
(lgt_fermion_force: two even/odd CG solves to an FP64 true residual of 1e-10,
then the adjoint kernel), with links and phi resident in HBM.  The timed K
steps use the mixed-precision solver (FP32 inner CG, FP64 reliable updates);
the same K calls in plain FP64 are timed after them and reported beside it.

Also reported: the roofline of the CG's dominant kernel (the even/odd hop),
timed with HIP events on the library's stream; the staple (plaquette) force
of the same workload, with its error against the stored oracle values; and
the FP64 CPU oracle timed on a bounded sample of the same call on this host.

Other workloads (each prints its own JSON line; none is the headline):
  --config 3  24^3x48, kappa 0.13: force call, mixed (FP32 and BF16-stored
              inner vectors) against FP64, force difference, hop roofline
  --config 4  8^4, 12^4, 16^4 with 12 right-hand sides each (6 kappa x 2
              eta): 36 mixed solves in one batched call over the three
              lattices, against one call per lattice and 36 sequential
              solves, batched-hop roofline
  --config 5  32^3x64, kappa 0.135, 2 stout levels rho 0.1: one leapfrog
              trajectory (10 steps, tau 1) from the seeded links (dH,
              reversibility), then HMC trajectories at the same dt from a
              thermalised state (ms, dH, acceptance)
  --stout-depth N  32^3x64 (the config-5 lattice) with N stout levels (default
              8, rho 0.1): the reverse pass through the chain under several
              checkpoint schedules (none kept ... every level kept), and the
              whole smeared force with none and with every level kept
  --multishift  16^4 (headline links and kappa): one multi-shift CG with 12
              shifts 1e-4..10 on the even/odd normal operator (the solve
              of a rational pseudofermion action), FP64, against 12
              single-shift solves

Measurement helpers (no JSON line), for rocprofv3 kernel traces and counter
passes: --hop-probe Lx Ly Lz Lt PREC NRHS launches the even/odd hop (NRHS >
1: the batched hop over NRHS right-hand sides) as often as the bench line
times it, and a plain 512 MiB device copy that calibrates FETCH_SIZE /
WRITE_SIZE; --force-kernels launches the staple force and the fermion-force
adjoint 10 times each on 24^3x48 and 32^3x64, then one stout level forward
and backward 5 times on 32^3x64 (links tiled from seeded 8^4 fields).

Study (not a timing): --study dh-vs-dt runs HMC chains (Metropolis) for the
paper's step-size test, 8^4 leapfrog and 6^4 stout (rho 0.3) with the
Sexton-Weingarten integrator (10 inner steps), and reports <Delta H>,
rms Delta H, <exp(-Delta H)> and acceptance against dt.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--config 2|3|4|5]
                       [--multishift] [--stout-depth N] [--study dh-vs-dt] [--hop-probe Lx Ly Lz Lt PREC NRHS]
                       [--force-kernels]
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
    ap.add_argument("--config", type=int, default=2, choices=(2, 3, 4, 5))
    ap.add_argument("--multishift", action="store_true")
    ap.add_argument("--stout-depth", type=int, default=0, help="stout levels of the checkpointing benchmark")
    ap.add_argument("--hop-shapes", action="store_true",
                    help="time the two work shapes of the hop kernel (hop alone and inside the force)")
    ap.add_argument("--study", default=None, choices=("dh-vs-dt", "reliable-delta"))
    ap.add_argument("--force-kernels", action="store_true",
                    help="launch the staple-force, bilinear and stout kernels for rocprofv3 (no JSON line)")
    ap.add_argument("--hop-probe", nargs="+", default=None, metavar="ARG",
                    help="LX LY LZ LT PREC NRHS [valu|mfma]: launch the hop kernel and a calibration copy for "
                         "rocprofv3 (no JSON line)")
    ap.add_argument("--therm", type=int, default=100, help="thermalisation trajectories of the study")
    ap.add_argument("--meas", type=int, default=40, help="measured trajectories per step size in the study")
    ap.add_argument("--therm-c5", type=int, default=30, help="config 5: quenched thermalisation trajectories")
    ap.add_argument("--meas-c5", type=int, default=4, help="config 5: timed trajectories on the thermalised background")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the hot path here is single-GPU (no collectives); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.hop_probe:
        hop_probe(args.hop_probe)
        return
    if args.force_kernels:
        force_kernels_probe()
        return
    if args.study == "dh-vs-dt":
        print(json.dumps(study_dh_vs_dt(args)), flush=True)
        return
    if args.study == "reliable-delta":
        print(json.dumps(study_reliable_delta(args)), flush=True)
        return
    if args.multishift:
        print(json.dumps(bench_multishift(args)), flush=True)
        return
    if args.hop_shapes:
        print(json.dumps(bench_hop_shapes(args)), flush=True)
        return
    if args.stout_depth:
        print(json.dumps(bench_stout_depth(args)), flush=True)
        return
    if args.config != 2:
        rec = {3: bench_c3, 4: bench_c4, 5: bench_c5}[args.config](args)
        print(json.dumps(rec), flush=True)
        return

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
    # beside them (not the metric): the inner recursion with BF16-stored vectors
    p_bf16 = lgt.Params(precision="mixed_bf16", tol=tol)
    run(p_bf16, max(1, args.warmup))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st_bf16 = run(p_bf16, args.steps)
    torch.cuda.synchronize()
    t_bf16 = (time.perf_counter() - t0) / args.steps
    log(f"bench: mixed bf16 {t_bf16 * 1e3:.3f} ms/call {st_bf16}")

    # beside it (not the metric): the even/odd-preconditioned action, whose
    # force needs one Schur solve instead of two (same determinant weight)
    phi_o = lat.schur_dslash(U, E, kappa, dagger=True)
    eo_rec = {}
    for name, prm in (("mixed", p_mixed), ("fp64", p_fp64)):
        for _ in range(max(1, args.warmup)):
            lat.fermion_force_eo(U, phi_o, kappa, prm, out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            _, _, st_eo = lat.fermion_force_eo(U, phi_o, kappa, prm, out=out)
        torch.cuda.synchronize()
        eo_rec[name] = {"ms_per_call": round((time.perf_counter() - t0) / args.steps * 1e3, 4),
                        "iters": st_eo["iters"], "true_rel_residual": st_eo["true_rel_residual"]}
    log(f"bench: even/odd-preconditioned action {eo_rec}")

    # the forces of both paths against the oracle's values stored for this
    # workload (oracle CG to 1e-15; sampled links and the full-field norm)
    force_vs_oracle = _force_vs_oracle(lat, U, phi, kappa, {"mixed": p_mixed, "fp64": p_fp64, "mixed_bf16": p_bf16})
    log(f"bench: force vs oracle {force_vs_oracle}")

    # the same call at the outer tolerance where the mixed force meets 1e-9
    # against the oracle (at 1e-10 the solver error alone is ~1e-9, for FP64
    # and mixed alike): both paths timed there, equal FP64 true residual
    tol_bar = 1e-11
    bar = {"tol": tol_bar, "force_bar": 1e-9}
    for name, prec in (("mixed", "mixed_fp32"), ("fp64", "fp64"), ("mixed_bf16", "mixed_bf16")):
        prm = lgt.Params(precision=prec, tol=tol_bar)
        run(prm, max(1, args.warmup))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = run(prm, args.steps)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / args.steps
        bar[name] = {"ms_per_call": round(t * 1e3, 4), "iters": st["iters"], "reliable_updates": st["reliable_updates"],
                     "corrections": st["corrections"], "true_rel_residual": st["true_rel_residual"]}
    fo = _force_vs_oracle(lat, U, phi, kappa, {n: lgt.Params(precision=pr, tol=tol_bar) for n, pr in
                                               (("mixed", "mixed_fp32"), ("fp64", "fp64"), ("mixed_bf16", "mixed_bf16"))})
    for name in ("mixed", "fp64", "mixed_bf16"):
        if fo:
            bar[name].update(fo[name])
            bar[name]["meets_bar"] = fo[name]["sampled_rel_err"] <= 1e-9 and fo[name]["norm_rel_diff"] <= 1e-9
    bar["speedup_mixed_vs_fp64"] = round(bar["fp64"]["ms_per_call"] / bar["mixed"]["ms_per_call"], 3)
    log(f"bench: at the force bar {bar}")
    staple = _staple_force_16(lat, U, beta, V, args.steps)
    log(f"bench: staple force {staple}")
    copy_gbs = _copy_ceiling()
    log(f"bench: device copy ceiling {copy_gbs:.0f} GB/s")

    # dominant kernel: the even/odd hop (FP32 in the timed mixed path), HIP
    # events on the library stream over 200 launches; FP64 beside it, and
    # both out of the 256 MB last-level cache at 24^3x48 (FP64) and
    # 32^3x64 (FP32), the HBM-bound claim
    hop = _hop_roofline(lat, U, E, V)
    hop["measured_copy_GBs"] = round(copy_gbs, 1)
    hop["frac_of_copy"] = round(hop["achieved"] / copy_gbs, 4)
    hop["hbm_ceilings"] = _hbm_ceilings(copy_gbs)
    hop["out_of_cache"] = _hop_out_of_cache()
    for line in hop["out_of_cache"].values():
        if line.get("traffic"):
            # the bytes the kernel moved through HBM per second, against the read-only rate
            moved = line["traffic"] / (line["avg_launch_us"] * 1e-6) / 1e9
            line["measured_traffic_GBs"] = round(moved, 1)
            line["frac_of_read_ceiling"] = round(moved / hop["hbm_ceilings"]["read_GBs"], 4)
    log(f"bench: hop roofline {hop}")

    # effective GB/s of the whole call: compulsory bytes of the CG iterations
    # (516 reals per site per e/o CGNR iteration) and of the force kernel
    def eff_gbs(st, p_bytes, t):
        byts = st["iters"] * 516 * p_bytes * V + 192 * 8 * V
        return byts / t / 1e9

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
        "mixed_bf16": {"ms_per_call": round(t_bf16 * 1e3, 4), "iters": st_bf16["iters"],
                       "reliable_updates": st_bf16["reliable_updates"],
                       "true_rel_residual": st_bf16["true_rel_residual"],
                       "note": "FP32 arithmetic with BF16-stored inner vectors; not the metric"},
        "eo_preconditioned_action": dict(eo_rec, note="S_eo = phi_o^dag (Mhat^dag Mhat)^-1 phi_o, same determinant "
                                                      "weight, one Schur solve per force; not the metric"),
        "force_vs_oracle": force_vs_oracle,
        "at_force_bar": bar,
        "staple_force": staple,
        "roofline": hop,
    }
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        rec["cpu_baseline"] = cpu_baseline(u, eta, kappa, tol, args.cpu_budget)
    print(json.dumps(rec), flush=True)


def _staple_force_16(lat, U, beta, V, steps):
    """The plaquette (staple) force of the same workload, the second force of
    a molecular-dynamics step: ms per lgt_gauge_force call (HIP events over
    10 x steps calls; a call packs the links, then runs the staple kernel
    with canonical FP64 output), its bytes (pack: U read and its packed copy
    written; staple force: packed U read, F written -- 288 reals per site)
    and the staple kernel's ~10.8 kflop per site, and the force's error
    against the oracle's values stored for this workload."""
    import numpy as np
    import torch

    out = lat.empty_gauge()
    for _ in range(3):
        lat.gauge_force(U, beta, out=out)
    n = 10 * max(1, steps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(n):
        lat.gauge_force(U, beta, out=out)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / n
    byts, flops = 288 * 8 * V, 10.8e3 * V
    rec = {"ms_per_call": round(ms, 5),
           "bytes_model": "288 reals per site: link pack (U read, packed copy written) + staple kernel "
                          "(packed U read, F written)",
           "algorithmic_bytes": byts, "achieved_GBs": round(byts / ms / 1e6, 1),
           "frac_of_8TBs": round(byts / ms / 1e6 / HBM_PEAK_GBS, 4),
           "fp64_flops_model": "10.8 kflop per site (staple kernel)", "fp64_TFLOPs": round(flops / ms / 1e9, 2),
           "note": "16^4 links sit in the 256 MB last-level cache; the staple kernel alone, out of the "
                   "cache, is in profiles/force_kernels_24x24x24x48_32x32x32x64.json"}
    gold = _golden("c2_16x16x16x16.json")
    if gold is not None:
        F = out.cpu().numpy()
        links = [tuple(l) for l in gold["links"]]
        ref = np.array([[complex(*v) for v in m] for m in gold["F_gauge"]]).reshape(-1, 3, 3)
        got = np.stack([F[l] for l in links])
        rec["vs_oracle"] = {"sampled_rel_err": float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel())),
                            "norm_rel_diff": float(abs(np.linalg.norm(F.ravel()) - gold["F_gauge_fro"])
                                                   / gold["F_gauge_fro"])}
    return rec


def _golden(name):
    """Stored oracle values of a workload (tests/golden, written from the oracle alone), or None."""
    try:
        with open(os.path.join(ROOT, "tests", "golden", name)) as f:
            return json.load(f)
    except OSError:
        return None


def _vs_golden(F, gold):
    """Relative error of a fermion force (host array) against stored oracle
    values: over the sampled links, and of the full-field Frobenius norm."""
    import numpy as np

    links = [tuple(l) for l in gold["links"]]
    ref = np.array([[complex(*v) for v in m] for m in gold["F_fermion"]]).reshape(-1, 3, 3)
    got = np.stack([F[l] for l in links])
    return {"sampled_rel_err": float(np.linalg.norm((got - ref).ravel()) / np.linalg.norm(ref.ravel())),
            "norm_rel_diff": float(abs(np.linalg.norm(F.ravel()) - gold["F_fermion_fro"]) / gold["F_fermion_fro"])}


def _force_vs_oracle(lat, U, phi, kappa, params, golden="c2_16x16x16x16.json"):
    """The fermion force of each parameter set against the stored oracle values."""
    gold = _golden(golden)
    if gold is None:
        return None
    out = {"oracle_tol": gold["oracle_tol"], "sampled_links": len(gold["links"])}
    for name, prm in params.items():
        out[name] = _vs_golden(lat.fermion_force(U, phi, kappa, prm)[0].cpu().numpy(), gold)
    return out


def _copy_ceiling():
    """Device-to-device copy of 1 GiB (read + write counted), best of 10: the
    bandwidth ceiling a streaming kernel can reach on this GPU."""
    import torch

    a = torch.ones(128 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = 1e30
    for _ in range(12):
        e0.record()
        b.copy_(a)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del a, b
    return 2 * 1024 ** 3 / (best * 1e-3) / 1e9


def _hbm_ceilings(copy_gbs):
    """What plain streaming reaches on this GPU, best of 10 over 2 GiB: a
    read-only pass (sums of rows of 1024 floats, which writes 1/1024 of the
    bytes; a full sum reaches only 4 TB/s), a write-only pass (fill) and the
    1 GiB copy of _copy_ceiling.  A kernel that mostly reads (the hop reads
    7/8 of its bytes) can exceed the copy rate."""
    import torch

    a = torch.ones(512 * 1024 * 1024, dtype=torch.float32, device="cuda")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = {}
    for name, fn in (("read", lambda: a.view(-1, 1024).sum(1)), ("write", lambda: a.fill_(1.0))):
        best = 1e30
        for _ in range(10):
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            best = min(best, e0.elapsed_time(e1))
        out[f"{name}_GBs"] = round(2 * 1024 ** 3 / (best * 1e-3) / 1e9, 1)
    del a
    out["copy_GBs"] = round(copy_gbs, 1)
    return out


HOP_SOURCES = ("kernels_hop.hip", "lgt_hop.h", "lgt_device.h", "lgt_internal.h")
MHOP_SOURCES = ("kernels_mrhs.hip", "lgt_hop.h", "lgt_device.h", "lgt_mrhs.h")


def kernel_sources_sha(files):
    """SHA-256 over the sources a kernel is built from (ties counter records to a kernel version)."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2602_20516_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic_record(name, sources=HOP_SOURCES):
    """The committed counter record of a kernel (profiles/<name>), or None when
    the kernel's sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sources_sha") != kernel_sources_sha(sources):
        return None
    return rec


def _traffic(name, sources=HOP_SOURCES):
    """HBM bytes per launch from the committed counter passes of a kernel, or None."""
    rec = _traffic_record(name, sources)
    return rec.get("bytes_per_launch") if rec else None


def _with_profile(line, name):
    """Add the committed record's HBM bytes and its rocprofv3 launch time (and the
    fraction of the HBM peak that time gives) to a hop roofline line."""
    rec = _traffic_record(name)
    line["traffic"] = rec.get("bytes_per_launch") if rec else None
    if rec and rec.get("avg_duration_us"):
        t = rec["avg_duration_us"] * 1e-6
        line["profile"] = f"profiles/{name}"
        line["profiled_avg_launch_us"] = rec["avg_duration_us"]
        line["frac_profiled"] = round(line["algorithmic_bytes_per_launch"] / t / 1e9 / HBM_PEAK_GBS, 4)
    return line


HOP_REPS, HOP_REPS_LARGE = 200, 100  # timed hop launches at 16^4 and on the out-of-cache lattices
HOP_RUNS = 5  # runs of those launches; the bench line quotes the median run


def _hop_line(lat, U, E, V, prec, nrep=HOP_REPS):
    """Roofline figures of the single-field hop: algorithmic bytes are 96 reals
    per lattice site (all 4V links as full 3x3 matrices, input and output half
    spinors); the kernel reads SU(3) links as two rows (72 reals per site),
    given beside."""
    p = 8 if prec == "fp64" else 4
    # median of HOP_RUNS runs of nrep launches each: one run can catch a
    # disturbance of the GPU (its mean then sits ~10 % high); every run's
    # mean is reported beside
    runs = sorted(lat.hop_benchmark(U, E, prec, nrep) for _ in range(HOP_RUNS))
    ms = runs[len(runs) // 2]
    alg = 96 * p * V
    gbs = alg / (ms * 1e-3) / 1e9
    out = {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
           "avg_launch_us": round(ms * 1e3, 3), "run_means_us": [round(r * 1e3, 3) for r in runs],
           "algorithmic_bytes_per_launch": alg}
    out["two_row_bytes_per_launch"] = 72 * p * V
    out["frac_two_row_bytes"] = round(72 * p * V / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    return out


def _hop_roofline(lat, U, E, V):
    line = {"kernel": "even/odd hop H_eo, FP32, two-row SU(3) links (k_hop<float,false,EpiAxpy<float>>)",
            "bound": "hbm", "timing": "HIP events on the library stream: mean of 200 back-to-back launches, median of 5 such runs",
            "bytes_model": "96 reals per lattice site (4V links, input and output half spinors)"}
    line.update(_hop_line(lat, U, E, V, "mixed_fp32"))
    name = "x".join(str(d) for d in lat.dims)
    _with_profile(line, f"hop_fp32_{name}_traffic.json")
    line["fp64"] = _with_profile(_hop_line(lat, U, E, V, "fp64"), f"hop_fp64_{name}_traffic.json")
    line["note"] = ("at 16^4 the hop's 19-50 MB sit in the 256 MB last-level cache; the HBM figures are the "
                    "out_of_cache lines")
    return line


def _tiled_links(dims, base=(8, 8, 8, 8), seed=901):
    """SU(3) links of a large lattice, tiled from a seeded 8^4 field (bandwidth
    measurement only: the values do not change the traffic)."""
    import numpy as np

    import lgt_inputs as li
    u = li.random_links(base, 0.2, seed)
    reps = tuple(d // b for d, b in zip(dims[::-1], base[::-1])) + (1, 1, 1)
    return np.tile(u, reps)


def _hop_out_of_cache():
    """The hop where its data leave the cache: FP64 at 24^3x48, FP32 at 32^3x64."""
    import numpy as np
    import torch

    import lgt_inputs as li
    import paper_2602_20516_amd as lgt
    out = {}
    for dims, prec in (((24, 24, 24, 48), "fp64"), ((32, 32, 32, 64), "mixed_fp32")):
        V = int(np.prod(dims))
        U = torch.from_numpy(_tiled_links(dims)).to("cuda")
        E = torch.from_numpy(np.tile(li.gaussian_spinor((8, 8, 8, 8), 902),
                                     tuple(d // 8 for d in dims[::-1]) + (1, 1))).to("cuda")
        lat = lgt.Lattice(dims)
        name = "x".join(str(d) for d in dims)
        line = _with_profile(_hop_line(lat, U, E, V, prec, HOP_REPS_LARGE),
                             f"hop_{'fp64' if prec == 'fp64' else 'fp32'}_{name}_traffic.json")
        out[f"{prec}_{name}"] = line
        del U, E, lat
        torch.cuda.empty_cache()
    return out


def hop_probe(argv):
    """Launch the hop kernel (as often as the bench line times it; 20 times for
    the batched hop) and a 512 MiB device copy, for
    rocprofv3 kernel traces and counter passes: bytes per hop launch =
    counter(hop) / counter(copy) x 512 MiB."""
    import numpy as np
    import torch

    import lgt_inputs as li
    import paper_2602_20516_amd as lgt
    if len(argv) not in (6, 7):
        raise SystemExit("--hop-probe takes LX LY LZ LT PREC NRHS [valu|mfma]")
    dims = tuple(int(v) for v in argv[:4])
    prec, nrhs = argv[4], int(argv[5])
    kind = argv[6] if len(argv) == 7 else "auto"
    small = int(np.prod(dims)) <= 65536  # larger lattices: fields tiled from 8^4 (see _tiled_links)
    u = li.random_links(dims, 0.3, 201) if small else _tiled_links(dims)
    eta = (li.gaussian_spinor(dims, 202) if small
           else np.tile(li.gaussian_spinor((8, 8, 8, 8), 902), tuple(d // 8 for d in dims[::-1]) + (1, 1)))
    U = torch.from_numpy(u).to("cuda")
    E = torch.from_numpy(eta).to("cuda")
    lat = lgt.Lattice(dims)
    lat.set_batch_hop_kernel(kind)
    # as many launches as the bench line times, so that the profiled mean matches its HIP-event mean
    reps = 20 if nrhs > 1 else (HOP_REPS if small else HOP_REPS_LARGE)
    ms = lat.hop_benchmark_mrhs(U, E, nrhs, prec, reps) if nrhs > 1 else lat.hop_benchmark(U, E, prec, reps)
    a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    src = MHOP_SOURCES if nrhs > 1 else HOP_SOURCES
    print(f"hop {dims} {prec} nrhs {nrhs} kernel {kind}: {ms * 1e3:.2f} us per launch; copy of {a.numel() * 8 >> 20} MiB x5 done; "
          f"kernel_sources_sha {kernel_sources_sha(src)}", flush=True)


def force_kernels_probe():
    """The staple force and the fermion-force adjoint 10 times each on 24^3x48
    and 32^3x64, then one stout level (rho 0.1) forward and backward 5 times on
    32^3x64, fields tiled from seeded 8^4 ones: for rocprofv3 kernel traces
    and counter passes of these kernels."""
    import numpy as np
    import torch

    import lgt_inputs as li
    import paper_2602_20516_amd as lgt
    for dims in ((24, 24, 24, 48), (32, 32, 32, 64)):
        reps = tuple(d // 8 for d in dims[::-1])
        U = torch.from_numpy(_tiled_links(dims)).to("cuda")
        a = torch.from_numpy(np.tile(li.gaussian_spinor((8,) * 4, 902), reps + (1, 1))).to("cuda")
        b = torch.from_numpy(np.tile(li.gaussian_spinor((8,) * 4, 903), reps + (1, 1))).to("cuda")
        lat = lgt.Lattice(dims)
        out = lat.empty_gauge()
        for _ in range(10):
            lat.gauge_force(U, 6.0, out=out)
            lat.bilinear_force(U, a, b, 0.13, -2.0, out=out)
        del a, b
        if dims[3] == 64:
            G = torch.from_numpy(np.tile(li.random_links((8,) * 4, 0.5, 905), reps + (1, 1, 1))).to("cuda")
            gout = lat.empty_gauge()
            for _ in range(5):
                lat.stout_smear(U, 0.1, 1, out=out)
                lat.stout_backprop(U, G, 0.1, 1, out=gout)
            del G, gout
        torch.cuda.synchronize()
        print(f"force kernels {dims} done", flush=True)
        del U, out, lat
        torch.cuda.empty_cache()


def _rel(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def bench_c3(args):
    """24^3x48 force call: mixed FP32, mixed with BF16-stored vectors, FP64."""
    import numpy as np
    import torch

    import lgt_inputs as li
    import paper_2602_20516_amd as lgt

    c = li.config(3)
    dims, kappa, tol = c["dims"], c["kappa"], c["tol"]
    V = int(np.prod(dims))
    log("bench c3: generating inputs")
    U = torch.from_numpy(li.random_links(dims, c["eps"], c["seeds"]["links"])).to("cuda")
    E = torch.from_numpy(li.gaussian_spinor(dims, c["seeds"]["eta"])).to("cuda")
    lat = lgt.Lattice(dims)
    phi = lat.dslash(U, E, kappa, dagger=True)
    steps = max(1, min(args.steps, 5))
    res, forces = {}, {}
    for prec in ("mixed_fp32", "mixed_bf16", "fp64"):
        prm = lgt.Params(precision=prec, tol=tol)
        out = lat.empty_gauge()
        try:
            for _ in range(max(1, min(args.warmup, 2))):
                lat.fermion_force(U, phi, kappa, prm, out=out)
        except lgt.LGTError as e:
            res[prec] = {"unsupported": str(e)}
            continue
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st = lat.fermion_force(U, phi, kappa, prm, out=out)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) / steps
        forces[prec] = out.clone()
        p = 8 if prec == "fp64" else 4
        res[prec] = {"ms_per_call": round(t * 1e3, 3), "iters": st["iters"],
                     "reliable_updates": st["reliable_updates"], "true_rel_residual": st["true_rel_residual"],
                     "effective_GBs": round((st["iters"] * 516 * p * V + 192 * 8 * V) / t / 1e9, 1)}
        log(f"bench c3: {prec} {res[prec]}")
    for prec in ("mixed_fp32", "mixed_bf16"):
        if prec in forces:
            res[prec]["force_rel_diff_vs_fp64"] = _rel(forces[prec], forces["fp64"])
    gold = _golden("c3_24x24x24x48.json")
    at_bar = None
    if gold is not None:
        for prec in forces:
            res[prec]["force_vs_oracle"] = _vs_golden(forces[prec].cpu().numpy(), gold)
        # the outer tolerance at which the mixed force meets its bar of 1e-9
        at_bar = {"tol": 1e-11, "force_bar": 1e-9, "oracle_tol": gold["oracle_tol"]}
        for prec in ("mixed_fp32", "fp64", "mixed_bf16"):
            prm = lgt.Params(precision=prec, tol=1e-11)
            out = lat.empty_gauge()
            lat.fermion_force(U, phi, kappa, prm, out=out)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, st = lat.fermion_force(U, phi, kappa, prm, out=out)
            torch.cuda.synchronize()
            e = _vs_golden(out.cpu().numpy(), gold)
            at_bar[prec] = {"ms_per_call": round((time.perf_counter() - t0) * 1e3, 3), "iters": st["iters"],
                            "corrections": st["corrections"], "true_rel_residual": st["true_rel_residual"], **e,
                            "meets_bar": e["sampled_rel_err"] <= 1e-9}
            log(f"bench c3: at the force bar {prec} {at_bar[prec]}")
        at_bar["speedup_mixed_vs_fp64"] = round(at_bar["fp64"]["ms_per_call"] / at_bar["mixed_fp32"]["ms_per_call"], 3)
    hop_ms = lat.hop_benchmark(U, E, "mixed_fp32", 100)
    hop_bytes = 72 * 4 * V  # two-row FP32 links + half spinors
    gbs = hop_bytes / (hop_ms * 1e-3) / 1e9
    t_mixed = res["mixed_fp32"]["ms_per_call"]
    copy_gbs = _copy_ceiling()
    return {
        "metric": "fermion force (CG+adjoint) ms/call at 24^3x48, mixed vs FP64", "value": t_mixed,
        "unit": "ms/call", "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 2), "ms_per_step": t_mixed,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64 (FP32 inner CG, FP64 residual/force)", "data": "synthetic (seeded SU(3) links eps=0.2, "
        "Gaussian eta)",
        "config": {"workload": "24^3x48 Wilson-fermion force, kappa 0.13, FP64 true residual 1e-10",
                   "dims": list(dims), "kappa": kappa, "tol": tol},
        "results": res,
        "speedup_mixed_vs_fp64": round(res["fp64"]["ms_per_call"] / t_mixed, 3),
        "at_force_bar": at_bar,
        "roofline": {"kernel": "even/odd hop H_eo, FP32, two-row SU(3) links", "bound": "hbm",
                     "achieved": round(gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "measured_copy_GBs": round(copy_gbs, 1), "frac_of_copy": round(gbs / copy_gbs, 4),
                     "traffic": _traffic("hop_fp32_24x24x24x48_traffic.json"),
                     "avg_launch_us": round(hop_ms * 1e3, 3), "algorithmic_bytes_per_launch": hop_bytes},
    }


def bench_c4(args):
    """36 mixed solves over 3 lattices x 12 right-hand sides: one batched call
    over all three lattices, against one batched call per lattice and against
    36 sequential single solves."""
    import numpy as np
    import torch

    import lgt_inputs as li
    import paper_2602_20516_amd as lgt

    c = li.config(4)
    prm = lgt.Params(precision=c["precision"], tol=c["tol"])
    lats = []
    for dims in c["dims_list"]:
        U = torch.from_numpy(li.random_links(dims, c["eps"], c["seeds"]["links"])).to("cuda")
        lat = lgt.Lattice(dims)
        items = [(k, s) for k in c["kappas"] for s in c["eta_seeds"]]
        phis = [lat.dslash(U, torch.from_numpy(li.gaussian_spinor(dims, s)).to("cuda"), k, dagger=True)
                for k, s in items]
        lats.append((dims, lat, U, [k for k, _ in items], phis))

    batch = lgt.Batch()
    all_items = [(lat, U, phi, k) for dims, lat, U, ks, phis in lats for k, phi in zip(ks, phis)]

    def one_call():
        st = batch.cg_solve(all_items, prm)[2]
        out, i = [], 0
        for _, _, _, ks, _ in lats:
            out.append(st[i:i + len(ks)])
            i += len(ks)
        return out

    def per_lattice():
        out = []
        for dims, lat, U, ks, phis in lats:
            out.append(lat.cg_solve_batch(U, phis, ks, prm)[2])
        return out

    def sequential():
        out = []
        for dims, lat, U, ks, phis in lats:
            out.append([lat.cg_solve(U, phi, k, prm)[2] for k, phi in zip(ks, phis)])
        return out

    steps = max(1, min(args.steps, 5))
    timing = {}
    for name, fn in (("batched", one_call), ("per_lattice", per_lattice), ("sequential", sequential)):
        for _ in range(max(1, min(args.warmup, 2))):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st = fn()
        torch.cuda.synchronize()
        timing[name] = ((time.perf_counter() - t0) / steps, st)
        log(f"bench c4: {name} {timing[name][0] * 1e3:.2f} ms")
    tb, stb = timing["batched"]
    tl, _ = timing["per_lattice"]
    ts, sts = timing["sequential"]
    per_lat = []
    for (dims, *_), sb, ss in zip(lats, stb, sts):
        per_lat.append({"dims": list(dims), "batched_iters": [s["iters"] for s in sb],
                        "sequential_iters": [s["iters"] for s in ss],
                        "max_true_rel_residual": max(s["true_rel_residual"] for s in sb)})
    dims16, lat16, U16, _, _ = lats[-1]
    E16 = torch.from_numpy(li.gaussian_spinor(dims16, c["eta_seeds"][0])).to("cuda")
    V16 = int(np.prod(dims16))
    nr = 2 * len(c["kappas"])
    hop_ms = lat16.hop_benchmark_mrhs(U16, E16, nr, "mixed_fp32", 100)
    hop_bytes = (72 + 24 * nr) * 4 * V16
    gbs = hop_bytes / (hop_ms * 1e-3) / 1e9
    return {
        "metric": "36 mixed solves (3 lattices x 12 RHS) total ms, one batched call vs sequential",
        "value": round(tb * 1e3, 3),
        "unit": "ms", "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 2), "ms_per_step": round(tb * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64 (FP32 inner CG, FP64 residual)", "data": "synthetic (seeded SU(3) links eps=0.3, "
        "Gaussian eta seeds 402/403)",
        "config": {"workload": "8^4, 12^4, 16^4; kappa 0.10-0.135 x 2 eta per lattice; X = (D^dag D)^-1 phi to FP64 "
                               "true residual 1e-10", "tol": c["tol"]},
        "batched_ms": round(tb * 1e3, 3),
        "batched_note": "one lgt_cg_solve_batch call over the three lattices (their solves run concurrently, one "
                        "stream each)",
        "per_lattice_calls_ms": round(tl * 1e3, 3), "sequential_ms": round(ts * 1e3, 3),
        "speedup_batched_vs_sequential": round(ts / tb, 3), "lattices": per_lat,
        "roofline": {"kernel": f"batched even/odd hop H_eo, FP32, {nr} right-hand sides, 16^4", "bound": "hbm",
                     "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": _traffic("mhop_fp32_16x16x16x16_traffic.json", MHOP_SOURCES),
                     "avg_launch_us": round(hop_ms * 1e3, 3), "algorithmic_bytes_per_launch": hop_bytes},
    }


def bench_multishift(args):
    """Multi-shift CG at 16^4 with 12 shifts against 12 single-shift solves."""
    import numpy as np
    import torch

    import lgt_inputs as li
    import paper_2602_20516_amd as lgt

    c = li.config(2)
    dims, kappa, tol = c["dims"], c["kappa"], c["tol"]
    V = int(np.prod(dims))
    U = torch.from_numpy(li.random_links(dims, c["eps"], c["seeds"]["links"])).to("cuda")
    E = torch.from_numpy(li.gaussian_spinor(dims, c["seeds"]["eta"])).to("cuda")
    lat = lgt.Lattice(dims)
    phi_o = lat.schur_dslash(U, E, kappa, dagger=True)
    shifts = [float(v) for v in np.geomspace(1e-4, 10.0, 12)]
    prm = lgt.Params(precision="fp64", tol=tol)

    def multi():
        return [lat.cg_solve_multishift(U, phi_o, kappa, shifts, prm)[1]]

    def single():
        return [lat.cg_solve_multishift(U, phi_o, kappa, [s], prm)[1] for s in shifts]

    steps = max(1, min(args.steps, 10))
    timing = {}
    for name, fn in (("multishift", multi), ("single_shift_solves", single)):
        for _ in range(max(1, min(args.warmup, 3))):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st = fn()
        torch.cuda.synchronize()
        timing[name] = ((time.perf_counter() - t0) / steps, st)
        log(f"bench multishift: {name} {timing[name][0] * 1e3:.2f} ms")
    tm, stm = timing["multishift"]
    ts, sts = timing["single_shift_solves"]
    it = stm[0]["iters"]
    return {
        "metric": "multi-shift CG (12 shifts) ms/solve at 16^4, FP64", "value": round(tm * 1e3, 3), "unit": "ms",
        "n_gpus": 1, "steps": steps, "warmup": min(args.warmup, 3), "ms_per_step": round(tm * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded SU(3) links eps=0.3, Gaussian eta; phi_o = Mhat^dag eta_o)",
        "config": {"workload": "16^4 even/odd normal operator, X_i = (Mhat^dag Mhat + sigma_i)^-1 phi_o for 12 "
                               "shifts sigma_i geometric in [1e-4, 10], FP64 true residual 1e-10",
                   "dims": list(dims), "kappa": kappa, "tol": tol, "shifts": shifts},
        "multishift_ms": round(tm * 1e3, 3), "iters": it, "ms_per_iteration": round(tm * 1e3 / max(it, 1), 5),
        "true_rel_residual": stm[0]["true_rel_residual"],
        "single_shift_solves_ms": round(ts * 1e3, 3), "single_shift_iters": [s["iters"] for s in sts],
        "speedup_vs_single_shift_solves": round(ts / tm, 3),
        "note": "the shifted updates (x_i, p_i for every unconverged shift) move 4 x 12 V/2 x 16 B per shift "
                "and iteration; kernel durations in the committed rocprofv3 summary",
    }


def bench_hop_shapes(args):
    """The single-field hop with 32 and with 64 sites per block (lgt_set_hop_block_sites): one
    launch alone (HIP events over 300 launches), and the whole force call (10 calls), at
    lattice sizes around the automatic switch (32 up to 8192 sites per parity); and the
    64-site hop in site order and t-fastest (lgt_set_hop_block_order; automatic: t-fastest
    above 131072 sites per parity)."""
    import torch

    import lgt_inputs as li
    import paper_2602_20516_amd as lgt

    rows = []
    for dims in [(8, 8, 8, 8), (12, 12, 12, 12), (16, 16, 16, 16), (16, 16, 16, 32), (24, 24, 24, 48)]:
        U = torch.from_numpy(li.random_links(dims, 0.3, 11)).to("cuda")
        E = torch.from_numpy(li.gaussian_spinor(dims, 12)).to("cuda")
        lat = lgt.Lattice(dims)
        phi = lat.dslash(U, E, 0.125, dagger=True)
        vh = dims[0] * dims[1] * dims[2] * dims[3] // 2
        for prec in ("mixed_fp32", "fp64"):
            r = {"dims": list(dims), "sites_per_parity": vh, "precision": prec,
                 "automatic": 32 if vh <= 8192 else 64}
            for ns in (32, 64):
                lat.set_hop_block_sites(ns)
                r[f"hop_us_{ns}"] = round(1e3 * lat.hop_benchmark(U, E, prec, 300), 3)
                if vh <= 65536:
                    prm = lgt.Params(precision=prec, tol=1e-10)
                    for _ in range(2):
                        lat.fermion_force(U, phi, 0.125, prm)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    for _ in range(10):
                        _, st = lat.fermion_force(U, phi, 0.125, prm)
                    torch.cuda.synchronize()
                    r[f"force_ms_{ns}"] = round(1e3 * (time.perf_counter() - t0) / 10, 3)
                    r[f"force_iters_{ns}"] = st["iters"]
            # the 64-site kernel in site order (1) and t-fastest (2)
            lat.set_hop_block_sites(64)
            for order in (1, 2):
                lat.set_hop_block_order(order)
                r[f"hop_us_64_order{order}"] = round(1e3 * lat.hop_benchmark(U, E, prec, 300), 3)
            lat.set_hop_block_order(0)
            lat.set_hop_block_sites(0)
            log("bench hop shapes:", json.dumps(r))
            rows.append(r)
        del lat, U, E, phi
        torch.cuda.empty_cache()
    return {"metric": "hop kernel work shape: 32 vs 64 sites per block", "unit": "us (hop), ms (force)",
            "n_gpus": 1, "higher_is_better": False, "dtype": "f32 / f64",
            "data": "synthetic (seeded SU(3) links eps=0.3, Gaussian eta; phi = D^dag eta, kappa 0.125)",
            "config": {"workload": "one even/odd hop launch (two-row links, FP32 / FP64), and the force call "
                                   "(mixed FP32 / FP64 CG to 1e-10) up to 16^3x32; the 64-site hop in both "
                                   "block orders"},
            "rows": rows}


def bench_stout_depth(args):
    """Checkpoint schedules of a deep stout chain at 32^3x64: reverse pass and smeared force."""
    import numpy as np
    import torch

    import lgt_inputs as li
    import paper_2602_20516_amd as lgt

    c = li.config(5)
    dims, rho, n = c["dims"], c["rho"], args.stout_depth
    V = int(np.prod(dims))
    log("bench stout-depth: generating inputs")
    U = torch.from_numpy(li.random_links(dims, c["eps"], c["seeds"]["links"])).to("cuda")
    E = torch.from_numpy(li.gaussian_spinor(dims, c["seeds"]["eta"])).to("cuda")
    GT = torch.from_numpy(li.random_links(dims, 1.0, 7)).to("cuda")
    lat = lgt.Lattice(dims)
    slot_gb = 72 * 16 * (V // 2) / 1e9
    reps = max(1, min(args.steps, 5))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    caps = sorted({0, 1, 2, int(round(n ** 0.5)), n - 1})
    backprop = []
    out = lat.empty_gauge()
    for cap in caps:
        lat.set_stout_checkpoints(cap)
        t = timed(lambda: lat.stout_backprop(U, GT, rho, n, out=out))
        sch = lat.stout_last_schedule()
        backprop.append({"stored_levels": sch["stored_levels"], "recompute_passes": sch["recompute_passes"],
                         "extra_GB": round(sch["stored_levels"] * slot_gb, 2), "ms": round(t * 1e3, 2)})
        log(f"bench stout-depth: backprop {backprop[-1]}")
    # one level forward alone, for the per-pass cost
    t_fwd = timed(lambda: lat.stout_smear(U, rho, 1, out=out))
    phi = lat.dslash(lat.stout_smear(U, rho, n), E, c["kappa"], dagger=True)
    prm = lgt.Params(precision=c["precision"], tol=c["tol"])
    force = {}
    for name, cap in (("none_kept", 0), ("all_kept", -1)):
        lat.set_stout_checkpoints(cap)
        t = timed(lambda: lat.smeared_force(U, phi, c["beta"], c["kappa"], rho, n, prm, "force", out=out))
        st = lat.smeared_force(U, phi, c["beta"], c["kappa"], rho, n, prm, "force", out=out)[2]
        force[name] = {"ms": round(t * 1e3, 2), "iters": st["iters"],
                       "stored_levels": lat.stout_last_schedule()["stored_levels"]}
        log(f"bench stout-depth: force {name} {force[name]}")
    best, worst = backprop[-1]["ms"], backprop[0]["ms"]
    return {
        "metric": f"reverse pass through {n} stout levels at 32^3x64, ms, by checkpoint schedule",
        "value": best, "unit": "ms", "n_gpus": 1, "steps": reps, "warmup": 1, "ms_per_step": best,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded SU(3) links eps=0.2, Gaussian eta, random cotangent)",
        "config": {"workload": f"32^3x64 stout chain, rho {rho}, {n} levels: lgt_stout_backprop under checkpoint "
                               f"caps {caps}; smeared force (FP32 inner CG to FP64 true residual {c['tol']}, kappa "
                               f"{c['kappa']}) with no level and every level kept", "dims": list(dims), "nlevels": n},
        "stout_forward_level_ms": round(t_fwd * 1e3, 3), "level_field_GB": round(slot_gb, 3),
        "backprop": backprop, "speedup_all_kept_vs_none": round(worst / best, 3), "smeared_force": force,
    }


def bench_c5(args):
    """Smeared HMC trajectories at 32^3x64: one from the seeded start (dH,
    reversibility), then trajectories at the workload's dt = 0.1 on a gauge
    background thermalised at beta 6 (ms, dH, acceptance)."""
    import numpy as np
    import torch

    import lgt_inputs as li
    import paper_2602_20516_amd as lgt
    from paper_2602_20516_amd.hmc import HMC, HMCRecord

    c = li.config(5)
    dims = c["dims"]
    log("bench c5: generating inputs")
    u = li.random_links(dims, c["eps"], c["seeds"]["links"])
    U0 = torch.from_numpy(u).to("cuda")
    del u
    E = torch.from_numpy(li.gaussian_spinor(dims, c["seeds"]["eta"])).to("cuda")
    P0 = torch.from_numpy(li.random_momenta(dims, c["seeds"]["mom"])).to("cuda")
    lat = lgt.Lattice(dims)
    phi = lat.dslash(lat.stout_smear(U0, c["rho"], c["nstout"]), E, c["kappa"], dagger=True)
    prm = lgt.Params(precision=c["precision"], tol=c["tol"])
    nsteps = c["nsteps"]
    dt = c["tau"] / nsteps
    U, P = U0.clone(), P0.clone()
    torch.cuda.synchronize()
    log("bench c5: trajectory from the seeded start")
    t0 = time.perf_counter()
    dh, st = lat.md_step_smeared(U, P, phi, c["beta"], c["kappa"], c["rho"], c["nstout"], dt, nsteps, prm)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    log(f"bench c5: {t:.2f} s dH {dh} {st}")
    P.neg_()
    dh_back, st_back = lat.md_step_smeared(U, P, phi, c["beta"], c["kappa"], c["rho"], c["nstout"], dt, nsteps,
                                           prm)
    rev_u = _rel(U, U0)
    rev_p = _rel(-P, P0)
    log(f"bench c5: reversed dH {dh_back}; |U-U0|/|U0| {rev_u:.3e}, |P-P0|/|P0| {rev_p:.3e}")
    del P, E, phi

    # thermalisation of the gauge background: quenched molecular dynamics
    # (pure gauge, fast, every trajectory accepted: far from equilibrium none
    # would pass the Metropolis test) brings the plaquette from the seeded
    # 0.91 to its beta = 6 equilibrium (~0.6); the smeared trajectories of
    # the workload (dt = 0.1, 10 steps, Metropolis) are then timed on it
    plaq0 = lat.mean_plaquette(U)
    Uth = U0.clone()
    quenched = HMC(lat, c["beta"], 0.0, 0.05, 20, params=prm, seed=5001)
    rq = HMCRecord()
    for _ in range(args.therm_c5):
        Uth = quenched.update(Uth, rq, metropolis=False)
    plaq_th = lat.mean_plaquette(Uth)
    plaq_sm = lat.mean_plaquette(lat.stout_smear(Uth, c["rho"], c["nstout"]))
    # mean-field (tadpole) estimate of the critical hopping parameter of the
    # smeared operator, kappa_c ~ 1 / (8 u0), u0 = <plaquette>^(1/4)
    kappa_c = 1.0 / (8.0 * plaq_sm ** 0.25)
    log(f"bench c5: quenched background {rq.summary()}; plaquette {plaq_th:.4f}, smeared {plaq_sm:.4f}, "
        f"mean-field kappa_c of the smeared operator {kappa_c:.4f}")
    timed = HMC(lat, c["beta"], c["kappa"], dt, nsteps, rho=c["rho"], nlevels=c["nstout"], params=prm, seed=5003)
    rt = HMCRecord()
    times = []
    for _ in range(args.meas_c5):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        Uth = timed.update(Uth, rt)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t1)
    log(f"bench c5: trajectories on the thermalised background {rt.summary()} {times}")
    t_eq = float(np.median(times))
    return {
        "metric": "smeared HMC trajectory ms at 32^3x64 (10 leapfrog steps, 2 stout levels)",
        "value": round(t * 1e3, 1), "unit": "ms/trajectory", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(t * 1e3, 1), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "value_note": "the trajectory from the seeded inputs; trajectories on a thermalised background are in "
                      "thermalised_background (the smeared operator is supercritical there)",
        "dtype": "f32+f64 (FP32 inner CG, FP64 forces, smearing, integrator)",
        "data": "synthetic (seeded SU(3) links eps=0.2, Gaussian eta and momenta)",
        "config": {"workload": "32^3x64, beta 6.0, kappa 0.135, stout rho 0.1 x 2, tau 1, 10 steps, FP64 true "
                               "residual 1e-10", "dims": list(dims)},
        "thermalised_background": {"ms_per_trajectory": [round(x * 1e3, 1) for x in times],
                                   "median_ms": round(t_eq * 1e3, 1), "dH": rt.dH, "accepted": rt.accepted,
                                   "plaquette_after": rt.plaquette, "cg_iters": rt.cg_iters,
                                   "background": {"quenched_trajectories": args.therm_c5, "dt": 0.05, "steps": 20,
                                                  "summary": rq.summary(), "plaquette": plaq_th,
                                                  "smeared_plaquette": plaq_sm,
                                                  "mean_field_kappa_c_smeared": kappa_c},
                                   "note": "trajectories at dt 0.1, 10 steps, Metropolis, on a gauge background "
                                           "thermalised at beta 6 by quenched molecular dynamics from the seeded "
                                           "links; the mean-field kappa_c of the smeared operator there is below "
                                           "the workload's kappa"},
        "seeded_start": {"ms": round(t * 1e3, 1), "dH": dh, "dH_reversed": dh_back, "reversibility_rel_U": rev_u,
                         "reversibility_rel_P": rev_p, "iters": st["iters"],
                         "reliable_updates": st["reliable_updates"],
                         "max_true_rel_residual": st["true_rel_residual"], "plaquette": plaq0,
                         "note": "seeded eps = 0.2 links (plaquette ~0.91) are far from equilibrium at beta 6"},
        "V": int(np.prod(dims)),
    }


def study_reliable_delta(args):
    """The mixed-precision force call over the reliable-update threshold delta (lgt_solver_params
    reliable_delta) at 16^4 and 24^3x48: time, inner iterations, FP64 updates, true residual."""
    import torch

    import lgt_inputs as li
    import paper_2602_20516_amd as lgt

    rows = []
    for cfg in (2, 3):
        c = li.config(cfg)
        dims, kappa = c["dims"], c["kappa"]
        U = torch.from_numpy(li.random_links(dims, c["eps"], c["seeds"]["links"])).to("cuda")
        E = torch.from_numpy(li.gaussian_spinor(dims, c["seeds"]["eta"])).to("cuda")
        lat = lgt.Lattice(dims)
        phi = lat.dslash(U, E, kappa, dagger=True)
        reps = 5 if cfg == 2 else 2
        for prec in ("mixed_fp32", "mixed_bf16"):
            for d in (3e-2, 1e-2, 3e-3, 1e-3, 3e-4, 1e-4, 3e-5, 1e-5):
                prm = lgt.Params(precision=prec, tol=c["tol"], reliable_delta=d)
                lat.fermion_force(U, phi, kappa, prm)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                for _ in range(reps):
                    _, st = lat.fermion_force(U, phi, kappa, prm)
                torch.cuda.synchronize()
                r = {"dims": list(dims), "precision": prec, "delta": d,
                     "ms": round(1e3 * (time.perf_counter() - t0) / reps, 3), "iters": st["iters"],
                     "reliable_updates": st["reliable_updates"], "true_rel_residual": st["true_rel_residual"]}
                log("study reliable delta:", json.dumps(r))
                rows.append(r)
        del lat, U, E, phi
        torch.cuda.empty_cache()
    return {"metric": "mixed-precision force call vs the reliable-update threshold", "unit": "ms/call",
            "n_gpus": 1, "higher_is_better": False, "dtype": "f32+f64",
            "data": "synthetic (the 16^4 and 24^3x48 force workloads' seeded links and pseudofermions)",
            "config": {"workload": "lgt_fermion_force, FP32 inner with FP32- or BF16-stored vectors, FP64 true "
                                   "residual 1e-10, delta from 3e-2 to 1e-5"},
            "rows": rows}


def study_dh_vs_dt(args):
    """HMC step-size study (Sec. III B): Delta H against dt at tau = 1."""
    import math

    import numpy as np
    import torch

    import lgt_inputs as li
    import paper_2602_20516_amd as lgt
    from paper_2602_20516_amd.hmc import HMC, HMCRecord

    settings = [
        dict(name="8^4 Wilson fermions, leapfrog", dims=(8, 8, 8, 8), beta=5.7, kappa=0.12, n_inner=1, rho=0.0,
             nlevels=0, seed=701, therm_steps=40, steps=(20, 40, 80)),
        dict(name="6^4 Wilson fermions, stout rho 0.3 (1 level), Sexton-Weingarten 10 inner steps",
             dims=(6, 6, 6, 6), beta=5.7, kappa=0.12, n_inner=10, rho=0.3, nlevels=1, seed=702, therm_steps=10,
             steps=(5, 10, 20)),
    ]
    prm = lgt.Params(precision="mixed_fp32", tol=1e-10)
    out = []
    t_all = time.perf_counter()
    for st in settings:
        lat = lgt.Lattice(st["dims"])
        U = torch.from_numpy(li.random_links(st["dims"], 0.5, st["seed"])).to("cuda")

        def chain(nsteps, n, rec, seed):
            nonlocal U
            h = HMC(lat, st["beta"], st["kappa"], 1.0 / nsteps, nsteps, st["n_inner"], st["rho"], st["nlevels"], prm,
                    seed)
            for i in range(n):
                U = h.update(U, rec)
                if (i + 1) % 20 == 0:
                    log(f"study {st['dims']}: nsteps {nsteps}: {i + 1}/{n} trajectories")

        chain(st["therm_steps"], args.therm, None, st["seed"] * 10)
        rows = []
        for j, nsteps in enumerate(st["steps"]):
            rec = HMCRecord()
            chain(nsteps, args.meas, rec, st["seed"] * 10 + j + 1)
            r = rec.summary()
            r["dt"] = 1.0 / nsteps
            r["nsteps"] = nsteps
            rows.append(r)
            log(f"study {st['dims']}: dt {1.0 / nsteps:.3f}: {r}")
        dts = np.log([r["dt"] for r in rows])
        slope_rms = float(np.polyfit(dts, np.log([r["rms_dH"] for r in rows]), 1)[0])
        pos = [r for r in rows if r["mean_dH"] > 0]
        slope_mean = (float(np.polyfit(np.log([r["dt"] for r in pos]), np.log([r["mean_dH"] for r in pos]), 1)[0])
                      if len(pos) >= 2 else None)
        out.append({"setting": st["name"], "dims": list(st["dims"]), "beta": st["beta"], "kappa": st["kappa"],
                    "n_inner": st["n_inner"], "rho": st["rho"], "stout_levels": st["nlevels"],
                    "thermalisation_trajectories": args.therm, "measured_per_dt": args.meas, "rows": rows,
                    "slope_log_rms_dH_vs_log_dt": slope_rms, "slope_log_mean_dH_vs_log_dt": slope_mean})
    return {
        "study": "HMC Delta H vs dt (tau = 1), mixed-precision solves to FP64 true residual 1e-10",
        "expected": "rms Delta H ~ dt^2 (second-order integrator); <Delta H> ~ dt^4 and <exp(-Delta H)> = 1 "
                    "in equilibrium",
        "beta_kappa_note": "the paper does not state beta and kappa; beta 5.7, kappa 0.12 are this study's choice",
        "results": out, "seconds": round(time.perf_counter() - t_all, 1),
    }


if __name__ == "__main__":
    main()
