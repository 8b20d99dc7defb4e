"""Benchmark: DG assembly + block-Jacobi GMRES on one MI355X.

Workload (the paper's method on the 256x256 P2 boundary-layer problem):
  unit square, 256 x 256 squares cut into 131072 triangles, P2 (786432 dofs),
  SIPG sigma = 18 (36 on the Dirichlet boundary), eps = 1e-6, b = (1, 0),
  alpha = 0, f from u = x y (1 - exp((x-1)/eps)) (1 - exp((y-1)/eps)), g^D = 0.
One step = FP64 assembly of matrix + load vector, block-Jacobi setup, and a
GMRES solve to relative residual 1e-10 (true FP64 residual).  Both solve forms
are timed over the same K steps: plain FP64 cycles, and FP32 cycles with FP64
residual / update (iterative refinement).  `value` is the faster form's
solves/s; both are reported.  Inputs are resident in device memory before
timing.  The roofline entry is for the kernel class with the largest share of
the timed solves (the SpMV on this workload), timed in the timed region by the
solver's built-in HIP-event profiler on the launch stream (profile=3: the
Gram-Schmidt dot launches, and each block's run of SpMV launches under one
pair of events); both are reported under "timed_kernels".  The per-kernel
breakdown comes from one more, untimed, solve of each form with every heavy
kernel timed.  The line also carries, under "learned_c5", the
comparison the metric names (learned + mixed vs plain FP64) on the
learned-warm-start workload: 512 held-out 64 x 64 P1 instances, plain FP64,
mixed, and mixed from the network's guess, each timed over K whole batches.

Other workloads (not the default line):
  --workload c4: 4096 instances (seed 0), P1/P2 50/50, N x N grids with N ~ U{16..128},
     log10 eps ~ U[-6,-1], b angle ~ U[0, 2 pi], |b| ~ U[0.5, 2], alpha ~ U[0, 1], f = sum of 4
     Gaussians, g^D = 0, SIPG; one element-parallel assembly launch + one persistent solve
     launch per batch, launch shape picked by the autotuner; step = the whole batch.
  --workload c1: latency of one solve of the 8 x 8 P1 SIPG problem (128 triangles, sigma = 6, eps = 1e-2,
     b = (1, 1), alpha = 1, u = sin(pi x) sin(pi y)): assembly + block-Jacobi setup + GMRES(32) to 1e-12,
     the solve run by one workgroup with its Krylov state in LDS.
  --workload nl: the paper's non-linear example (r(u) = u^2, u = (1 - tanh((2x - y - 1/4)/sqrt(5 eps)))/2,
     eps = 1e-6, b = (1, 2)/sqrt(5), alpha = 1) on 256 x 256 squares, P2 SIPG: assembly + Newton from zero to
     ||Res||/||F|| <= 1e-10, each step J w = -Res by block-Jacobi GMRES(576) to 1e-10.
  --workload c3: assembly only, 512 x 512 squares jittered by +-0.2 h (seed 0, 524288 triangles), P3 IIPG
     sigma = 36 (72 on Dirichlet), rotating b = (-(y - 1/2), x - 1/2), eps = 1e-4, alpha = 1/2, f = 1,
     Dirichlet on x = 0 and y = 0, g^N = 0 elsewhere; FP64 and FP32 assembly, FP32 error vs FP64.
  --workload mlp: the warm-start perceptron alone (inference on 512 instances, one training step on 256),
     achieved TFLOP/s of its BF16 MFMA products against the 2.5 PFLOP/s peak.
  --workload c5: 512 held-out instances (seed 2) of the 64 x 64 P1 SIPG family (parameters as c4),
     zero guess vs the learned initial guess (perceptron + prolongation, model trained on 20000
     method solves of seed 1), FP64 and mixed cycles; step = the whole batch incl. the network.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--workload c1|c2|c3|c4|c5|nl|mlp]
       python bench.py --profile-run     (one FP64 step + a copy probe, for rocprofv3)
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
N_GRID, DEGREE, EPS = 256, 2, 1e-6
C1_RESTART = 32


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_workload(api, W, torch):
    import numpy as np
    m = W.structured_mesh(N_GRID)
    mesh = api.Mesh.from_arrays(m, DEGREE)
    prob = W.boundary_layer_problem(eps=EPS)
    vol = mesh.qpoints()[0].cpu().numpy()
    f = api.Field.qpoints(torch.from_numpy(np.ascontiguousarray(prob.f(vol[..., 0], vol[..., 1]))).cuda())
    sigma, _ = api.default_penalty(api.SIPG, DEGREE)
    P = api.Problem(api.SIPG, DEGREE, sigma, eps=prob.eps, bx=prob.b[0], by=prob.b[1], alpha=prob.alpha, f=f)
    return m, mesh, P, prob


def copy_probe(torch):
    """A plain copy kernel of known size for scaling HBM counters: 3 launches,
    each reading and writing 512 MiB."""
    src = torch.empty(64 << 20, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    log("profile run done")


def launched_kernel(cls, prec, block):
    """The HIP kernel behind one of the solver profiler's classes (P2: 6 basis
    functions per element) for Arnoldi blocks of `block` vectors."""
    if cls == "spmv_hat":
        return "spmv_hat_kernel<6, %s>" % prec
    if block in (8, 16, 32) and cls == "multidot":
        return "multidot_mfma_kernel<%s, %d>" % (prec, block)
    if block in (16, 32) and cls == "update":
        return "update_wide_kernel<%s, %d>" % (prec, block)
    if block > 1 and cls in ("multidot", "update"):
        return "%s_block_kernel<%s, %d>" % (cls, prec, block)
    return "%s_kernel<%s>" % (cls, prec)


def measured_traffic(kernel, form):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/traffic.json), or None when there is none for this kernel and
    solve form or its source file has changed since the counters were taken."""
    import hashlib
    try:
        entry = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))[kernel]
        src = open(os.path.join(ROOT, entry["source"]), "rb").read()
    except (OSError, ValueError, KeyError):
        return None
    if entry.get("form") != form or hashlib.sha1(src).hexdigest() != entry["sha1"]:
        return None
    return entry["bytes_per_launch"]


def assembly_bytes(mesh, prec_bytes, f_points=True):
    """Algorithmic HBM bytes of one assembly: BSR values + load vector written;
    per element its vertex coordinates (6 FP64), the neighbours' gradient maps
    on its three edges (3 x 2 FP64), neighbour table (3 int32), packed neighbour
    edge ids (int32), row pointer (int32), and the f values at the volume points
    (FP64) when f is given by point values, each read once."""
    n = mesh.n_loc
    out = mesh.nnzb * n * n * prec_bytes + mesh.n_dofs * prec_bytes
    inp = mesh.T * (6 * 8 + 3 * 2 * 8 + 3 * 4 + 4 + 4) + (mesh.T * mesh.n_q * 8 if f_points else 0)
    return out + inp


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--restart", type=int, default=2 * N_GRID + 64)
    ap.add_argument("--reorth", type=int, default=0, help="1: conditional second Gram-Schmidt pass")
    ap.add_argument("--lockstep-block", type=int, default=0, choices=(0, 1, 2, 3, 6, 8),
                    help="c4, c5: Arnoldi vectors per Gram-Schmidt pass of the lockstep solver (0: the batch's "
                         "choice, 8)")
    ap.add_argument("--block", type=int, default=0, choices=(0, 1, 2, 3, 4, 6, 8, 16, 32),
                    help="Arnoldi vectors per Gram-Schmidt pass (0: the solver's choice; 16 in FP64 cycles only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="c2", choices=("c1", "c2", "c3", "c4", "c5", "nl", "mlp"))
    ap.add_argument("--count", type=int, default=None, help="c4 / c5: number of instances (4096 / 512)")
    ap.add_argument("--profile-run", action="store_true",
                    help="one FP64 step and a 512 MiB device copy (counter scaling), no JSON baseline")
    args = ap.parse_args()
    if args.profile_run:
        args.steps, args.warmup, args.no_cpu_baseline = 1, 0, True
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: each workload is a single-GPU problem and the library has no "
              "multi-GPU path (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1502_02941_amd import api
    from paper_1502_02941_amd import workloads as W

    torch.cuda.set_device(0)
    if args.workload == "c4":
        return bench_c4(args, api, W, torch)
    if args.workload == "c5":
        return bench_c5(args, api, W, torch)
    if args.workload == "c3":
        return bench_c3(args, api, W, torch)
    if args.workload == "c1":
        return bench_c1(args, api, W, torch)
    if args.workload == "nl":
        return bench_nl(args, api, W, torch)
    if args.workload == "mlp":
        return bench_mlp(args, api, W, torch)
    log("building workload %dx%d P%d" % (N_GRID, N_GRID, DEGREE))
    m, mesh, P, prob = build_workload(api, W, torch)
    vals64, rhs64 = mesh.alloc_system(api.F64)
    vals32, rhs32 = mesh.alloc_system(api.F32)
    x = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
    forms = ("fp64",) if args.profile_run else ("mixed", "fp64")
    # the timed solvers time the Gram-Schmidt dot kernel and each block's SpMV run with HIP events
    # on the solve stream (profile=3); a per-kernel breakdown comes from one more, untimed, solve
    # with every heavy kernel timed (profile=1: about 6% slower from the events alone)
    def make_solver(form, profile):
        blk = 0 if form == "mixed" and args.block >= 16 else args.block  # sixteen or 32: FP64 cycles only
        return api.Solver(mesh, restart=args.restart, max_iters=20000, rel_tol=1e-10, mixed=form == "mixed",
                          inner_tol=1e-6, reorth=bool(args.reorth), profile=profile, block=blk)

    solvers = {f: make_solver(f, 3) for f in ("mixed", "fp64")}
    stream = torch.cuda.current_stream()

    def step(form):
        api.assemble(mesh, P, prec=api.F64, vals=vals64, rhs=rhs64)
        s = solvers[form]
        s.setup(vals64)
        x.zero_()
        return s.solve(rhs64, x)

    # warm-up
    for _ in range(args.warmup):
        for form in forms:
            r = step(form)
            log("warmup %s: iters %d cycles %d reorth %d rel_res %.3e" % (form, r.iters, r.cycles, r.reorth_passes,
                                                                          r.rel_res))
    torch.cuda.synchronize()

    for form in forms:
        solvers[form].profile(reset=True)
    results = {}
    for form in forms:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reps = [step(form) for _ in range(args.steps)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = all(r.converged and r.rel_res <= 1e-10 for r in reps)
        results[form] = dict(seconds=dt, iters=[r.iters for r in reps], cycles=[r.cycles for r in reps],
                             reorth=[r.reorth_passes for r in reps], rel_res=max(r.rel_res for r in reps),
                             converged=ok, kernels=solvers[form].profile(reset=True))
        log("%s: %.3f s for %d steps, iters %s, rel_res %.3e" % (form, dt, args.steps, results[form]["iters"],
                                                                  results[form]["rel_res"]))

    if not args.profile_run:
        for form in forms:
            sb = make_solver(form, 1)
            solvers[form] = sb
            step(form)
            torch.cuda.synchronize()
            results[form]["breakdown"] = sb.profile(reset=True)
            del sb

    # assembly kernels alone, HIP events on the launch stream
    def time_assembly(prec, vals, rhs, reps=20):
        for _ in range(3):
            api.assemble(mesh, P, prec=prec, vals=vals, rhs=rhs)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(reps):
            api.assemble(mesh, P, prec=prec, vals=vals, rhs=rhs)
        ev[1].record(stream)
        ev[1].synchronize()
        return ev[0].elapsed_time(ev[1]) / reps * 1e-3

    if args.profile_run:
        copy_probe(torch)
        return

    t_asm64 = time_assembly(api.F64, vals64, rhs64)
    t_asm32 = time_assembly(api.F32, vals32, rhs32)
    b64, b32 = assembly_bytes(mesh, 8), assembly_bytes(mesh, 4)
    asm = dict(fp64_melem_s=mesh.T / t_asm64 / 1e6, fp32_melem_s=mesh.T / t_asm32 / 1e6,
               fp64_us=t_asm64 * 1e6, fp32_us=t_asm32 * 1e6,
               fp64_gbs=b64 / t_asm64 / 1e9, fp32_gbs=b32 / t_asm32 / 1e9)
    log("assembly FP64 %.1f us (%.0f Melem/s, %.0f GB/s), FP32 %.1f us (%.0f Melem/s, %.0f GB/s)"
        % (asm["fp64_us"], asm["fp64_melem_s"], asm["fp64_gbs"], asm["fp32_us"], asm["fp32_melem_s"],
           asm["fp32_gbs"]))

    def kstats(form):
        out = {}
        for name, (launches, ms, nbytes) in results[form].get("breakdown", results[form]["kernels"]).items():
            if launches:
                out[name] = {"launches": launches, "avg_us": ms / launches * 1e3,
                             "GB_s": nbytes / (ms * 1e-3) / 1e9 if ms > 0 else None, "total_ms": ms}
        return out

    best = min(forms, key=lambda f: results[f]["seconds"] if results[f]["converged"] else 1e30)
    def block_of(form):  # the solver's automatic choice unless --block is given
        if args.reorth:
            return 1
        if args.block and not (form == "mixed" and args.block >= 16):
            return args.block
        if form == "fp64" and args.restart <= 608:
            return 32
        if form == "fp64" and args.restart <= 640:
            return 16
        return (8 if form == "fp64" else 6) if args.restart <= 2048 else 3

    block = block_of(best)
    other = [f for f in forms if f != best][0]
    kb = kstats(best)
    dom = max(kb, key=lambda k: kb[k]["total_ms"])  # in the untimed breakdown
    timed = {k: v for k, v in results[best]["kernels"].items() if v[0] > 0}  # timed live in the timed region
    rk = max(timed, key=lambda k: timed[k][1])  # the kernel class with the most time: the SpMV on this workload
    launches, ms, nbytes = timed[rk]
    achieved = nbytes / (ms * 1e-3) / 1e9
    line = {
        "metric": "DG assembly Melem/s; solves/s at rel-res 1e-10, learned+mixed vs plain FP64",
        "value": args.steps / results[best]["seconds"],
        "unit": "solves/s (assemble + block-Jacobi setup + GMRES to rel-res 1e-10)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": results[best]["seconds"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if best == "fp64" else "f32 Arnoldi cycles + f64 residual/update (f64 assembly)",
        "data": "synthetic (manufactured boundary-layer solution on a structured mesh)",
        "config": {"workload": "256x256 structured, P2 SIPG (131072 triangles, 786432 dofs), eps=1e-6, "
                               "b=(1,0), alpha=0, boundary-layer u; block-Jacobi GMRES(%d), %d Arnoldi vector(s) "
                               "per Gram-Schmidt pass" % (args.restart, block),
                   "restart": args.restart, "form": best, "reorth": args.reorth, "block": block,
                   "basis": "shifted (w_i = (A M^-1 - I) w_(i-1))"},
        "forms": {f: {"solves_per_s": args.steps / results[f]["seconds"],
                      "ms_per_step": results[f]["seconds"] / args.steps * 1e3,
                      "iters": results[f]["iters"], "cycles": results[f]["cycles"],
                      "reorth_passes": results[f]["reorth"], "rel_res": results[f]["rel_res"],
                      "converged": results[f]["converged"], "block": block_of(f), "kernels": kstats(f)}
                  for f in forms},
        "assembly": asm,
        "roofline": {"bound": "hbm", "kernel": rk, "dominant_in_breakdown": dom,
                     "launched": launched_kernel(rk, "double" if best == "fp64" else "float", block),
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(rk, best),
                     "launches": launches, "avg_us": ms / launches * 1e3,
                     "bytes_per_launch_avg": nbytes / launches,
                     "timed_kernels": {k: {"launches": v[0], "total_ms": v[1], "avg_us": v[1] / v[0] * 1e3,
                                           "GB_s": v[2] / (v[1] * 1e-3) / 1e9,
                                           "launched": launched_kernel(k, "double" if best == "fp64" else "float",
                                                                       block),
                                           "traffic": measured_traffic(k, best)}
                                       for k, v in timed.items()}},
        "assembly_roofline": {"bound": "hbm", "kernel": "assemble_tensor_kernel<2,double> (matrix and load vector)",
                              "achieved": asm["fp64_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                              "frac": asm["fp64_gbs"] / HBM_PEAK_GBS, "traffic": measured_traffic("assemble_c2", "fp64"),
                              "bytes_per_launch": b64},
        "cpu_baseline": None,
    }
    log("best form %s; dominant kernel %s (timed: %s): %d launches, avg %.1f us, %.0f GB/s" % (
        best, dom, rk, launches, ms / launches * 1e3, achieved))
    line["learned_c5"] = c5_legs(args, api, W, torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(m, prob, int(results["fp64"]["iters"][0]) if "fp64" in results else 538)
    print(json.dumps(line), flush=True)


def c5_legs(args, api, W, torch):
    """The comparison the metric names, learned + mixed against plain FP64, on
    the learned-warm-start workload (512 held-out 64 x 64 P1 instances, seed 2):
    plain FP64 from zero, mixed from zero, and mixed from the network's guess
    (network + prolongation + judge + batched assembly and solve, each form
    timed over `steps` whole batches after one untimed batch)."""
    from paper_1502_02941_amd import learned as L
    model = L.load(os.path.join(ROOT, "paper_1502_02941_amd", "data", "c5_mlp.npz"))
    t0 = time.perf_counter()
    out = L.evaluate(model, count=512, seed=2, reps=max(args.steps, 1), forms=L.HEADLINE_FORMS, log=log)
    keep = ("solves_per_s", "seconds", "iters_median", "iters_p90", "iters_mean", "rejected", "converged",
            "max_rel_res")
    forms = {k: {kk: out[k][kk] for kk in keep} for k, _, _, _ in L.HEADLINE_FORMS}
    log("learned-warm-start legs: %.1f s" % (time.perf_counter() - t0))
    return {"workload": "512 held-out instances (seed 2), 64x64 P1 SIPG (24576 dofs each), Gaussian-sum f; "
                        "batched assemble + solve to rel-res 1e-10; step = the whole batch",
            "steps": max(args.steps, 1), "forms": forms,
            "mixed_learned_vs_plain_fp64": forms["mixed+learned"]["solves_per_s"] / forms["fp64"]["solves_per_s"],
            "mixed_learned_vs_mixed": forms["mixed+learned"]["solves_per_s"] / forms["mixed"]["solves_per_s"],
            "coarse_rel_err_median": out["coarse_rel_err_median"], "guess_ms": out["guess_ms"]}


def host_info():
    """The host's CPU model and the number of logical CPUs this process may
    use (the oracle itself runs on one of them)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count()
    return {"cpu_model": model, "host_cpus": n}


def bench_c4(args, api, W, torch):
    import numpy as np
    from paper_1502_02941_amd import autotune
    insts = W.sample_instances(args.count or 4096, seed=0)
    meshes = {}
    pairs = []
    for i in insts:
        if i.N not in meshes:
            meshes[i.N] = W.structured_mesh(i.N)
        pairs.append((meshes[i.N], api.instance_problem(i)))
    n_el = sum(2 * i.N * i.N for i in insts)
    n_dofs = sum(2 * i.N * i.N * (i.k + 1) * (i.k + 2) // 2 for i in insts)
    log("c4: %d instances, %.1fM triangles, %.1fM dofs" % (len(insts), n_el / 1e6, n_dofs / 1e6))
    forms = {}
    for form in ("mixed", "fp64"):
        mixed = form == "mixed"
        t0 = time.perf_counter()
        best = autotune.tune_batch(api, pairs, mixed=mixed, log=log)
        log("%s: tuned %s in %.1f s" % (form, best, time.perf_counter() - t0))
        t0 = time.perf_counter()
        b = api.Batch(pairs, mixed=mixed, rel_tol=1e-10, inner_tol=1e-5, lockstep_block=args.lockstep_block, log=log,
                      **best)
        log("%s: batch created in %.1f s" % (form, time.perf_counter() - t0))
        x, rep = b.alloc()
        for w in range(args.warmup):
            tw = time.perf_counter()
            x.zero_()
            b.run(x, rep)
            b.wait(log)
            log("%s: warm-up batch %d: %.2f s" % (form, w + 1, time.perf_counter() - tw))
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev[0].record()
        for k in range(args.steps):
            x.zero_()
            b.run(x, rep)
            b.wait(log)
            log("%s: timed batch %d done at %.2f s" % (form, k + 1, time.perf_counter() - t0))
        ev[1].record()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        R = b.reports(rep)
        ok = bool((R["status"] == 0).all() and (R["rel_res"] <= 1e-10).all())
        its = R["iters"].astype(float)
        # algorithmic bytes of the batch: assembly output + per-iteration Krylov traffic
        ps = 4 if mixed else 8
        nbytes = 0.0
        for i, inst in enumerate(insts):
            n = 2 * inst.N * inst.N * (inst.k + 1) * (inst.k + 2) // 2
            nl = (inst.k + 1) * (inst.k + 2) // 2
            T = 2 * inst.N * inst.N
            nnzb = T + 2 * (3 * inst.N * inst.N - 2 * inst.N)
            cyc = max(int(R["cycles"][i]), 1)
            its_i = float(R["iters"][i])
            per = its_i / cyc
            # dots + updates over the basis: the lockstep path takes S Arnoldi vectors per pass
            # ((j + 1 + S) + (j + 1 + 2S) vectors per block of S steps, summed over the blocks of a
            # cycle: per^2 / S + (2 + 2S) per / S), the persistent path one ((j + 2) + (j + 3) per step)
            if n >= best["lockstep_min_dofs"]:
                lsb = args.lockstep_block or 8  # the batch's automatic choice
                orth = cyc * (per * per / lsb + (2.0 + 2.0 * lsb) * per / lsb) * n * ps
            else:
                orth = cyc * (per * (per + 1) + 4 * per) * n * ps
            spmv = its_i * ((nnzb - T) * nl * nl * ps + 2.0 * n * ps)
            resid = (cyc + 1) * (nnzb * nl * nl * 8 + 3 * n * 8)
            asm = nnzb * nl * nl * 8 + n * 8 + T * 72
            nbytes += orth + spmv + resid + asm
        gbs = nbytes / (dt / args.steps) / 1e9
        forms[form] = {"solves_per_s": len(insts) * args.steps / dt, "seconds_per_batch": dt / args.steps,
                       "gpu_ms_per_batch": ev[0].elapsed_time(ev[1]) / args.steps,
                       "iters_median": float(np.median(its)), "iters_p90": float(np.percentile(its, 90)),
                       "iters_max": int(its.max()), "rel_res_max": float(R["rel_res"].max()),
                       "all_converged": ok, "launch": best, "algorithmic_GB_per_batch": nbytes / 1e9,
                       "achieved_GB_s": gbs}
        log("%s: %.2f s per batch, %.0f solves/s, iters median %.0f p90 %.0f, max rel-res %.2e, %.0f GB/s"
            % (form, dt / args.steps, len(insts) * args.steps / dt, np.median(its), np.percentile(its, 90),
               R["rel_res"].max(), gbs))
        del b, x, rep
        torch.cuda.empty_cache()
    best_form = max(forms, key=lambda f: forms[f]["solves_per_s"] if forms[f]["all_converged"] else -1)
    F = forms[best_form]
    line = {
        "metric": "DG assembly Melem/s; solves/s at rel-res 1e-10, learned+mixed vs plain FP64",
        "value": F["solves_per_s"], "unit": "solves/s (batched: assemble + solve to rel-res 1e-10)",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": F["seconds_per_batch"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 cycles + f64 refinement" if best_form == "mixed" else "f64",
        "data": "synthetic (seeded instance sampler, seed 0)",
        "config": {"workload": "batched: %d instances, P1/P2, N~U{16..128}, Gaussian-sum f, SIPG" % len(insts),
                   "form": best_form, "triangles": n_el, "dofs": n_dofs},
        "forms": forms,
        "roofline": {"bound": "hbm", "kernel": "batch_assemble_kernel + solve kernels of the tuned split (whole batch)",
                     "achieved": F["achieved_GB_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": F["achieved_GB_s"] / HBM_PEAK_GBS,
                     # HBM bytes of one whole 4096-instance batch (the unit `achieved` is per)
                     "traffic": measured_traffic("c4_" + best_form, best_form) if len(insts) == 4096 else None,
                     "algorithmic_bytes_per_batch": F["algorithmic_GB_per_batch"] * 1e9},
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_c4(insts),
    }
    print(json.dumps(line), flush=True)
    if args.profile_run:
        copy_probe(torch)


def bench_c1(args, api, W, torch):
    import numpy as np
    m = W.structured_mesh(8)
    prob = W.sinsin_problem()
    mesh = api.Mesh.from_arrays(m, 1)
    vol = mesh.qpoints()[0].cpu().numpy()
    f = api.Field.qpoints(torch.from_numpy(np.ascontiguousarray(prob.f(vol[..., 0], vol[..., 1]))).cuda())
    gd_pts = mesh.qpoints()[1].cpu().numpy()
    gD = api.Field.qpoints(torch.from_numpy(np.ascontiguousarray(prob.u(gd_pts[..., 0], gd_pts[..., 1]))).cuda())
    sigma, _ = api.default_penalty(api.SIPG, 1)
    P = api.Problem(api.SIPG, 1, sigma, eps=prob.eps, bx=prob.b[0], by=prob.b[1], alpha=prob.alpha, f=f, gD=gD)
    vals, rhs = mesh.alloc_system(api.F64)
    x = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
    # GMRES(32): its Krylov state fits one workgroup's LDS, so the solve is one launch
    s = api.Solver(mesh, restart=C1_RESTART, max_iters=5000, rel_tol=1e-12)

    def step():
        api.assemble(mesh, P, prec=api.F64, vals=vals, rhs=rhs)
        s.setup(vals)
        x.zero_()
        return s.solve(rhs, x)  # synchronises

    for _ in range(max(args.warmup, 3)):
        step()
    reps = max(args.steps, 1) * 100
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        r = step()
        ts.append(time.perf_counter() - t0)
    ts = np.array(ts)
    l2, _ = api.l2_error(mesh, x, prob.u)
    log("c1: median %.3f ms, p90 %.3f ms, %d iterations, rel-res %.2e, L2 error %.3e"
        % (np.median(ts) * 1e3, np.percentile(ts, 90) * 1e3, r.iters, r.rel_res, l2))
    line = {
        "metric": "DG assembly Melem/s; solves/s at rel-res 1e-10, learned+mixed vs plain FP64",
        "value": float(np.median(ts) * 1e3), "unit": "ms per solve (assemble + setup + GMRES to rel-res 1e-12, "
                                                      "host-synchronised, median)",
        "n_gpus": 1, "steps": reps, "warmup": max(args.warmup, 3), "ms_per_step": float(np.median(ts) * 1e3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (manufactured solution)",
        "config": {"workload": "8x8 structured, P1 SIPG (128 triangles, 384 dofs), sigma=6, eps=1e-2, b=(1,1), "
                               "alpha=1, u=sin(pi x)sin(pi y); GMRES(%d)" % C1_RESTART,
                   "p90_ms": float(np.percentile(ts, 90) * 1e3), "iters": int(r.iters), "rel_res": float(r.rel_res),
                   "l2_error": float(l2), "one_workgroup_lds_solve": bool(r.persistent)},
        "roofline": None,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_c1(m, prob),
    }
    print(json.dumps(line), flush=True)


def nl_problem(W):
    tl = W.tanh_layer_problem()
    return tl, (lambda X, Y: tl.f(X, Y) + tl.u(X, Y) ** 2)


def bench_nl(args, api, W, torch):
    import numpy as np
    tl, fnl = nl_problem(W)
    m = W.structured_mesh(N_GRID)
    mesh = api.Mesh.from_arrays(m, DEGREE)
    vol, bnd = [t.cpu().numpy() for t in mesh.qpoints()[:2]]
    f = api.Field.qpoints(torch.from_numpy(np.ascontiguousarray(fnl(vol[..., 0], vol[..., 1]))).cuda())
    gD = api.Field.qpoints(torch.from_numpy(np.ascontiguousarray(tl.u(bnd[..., 0], bnd[..., 1]))).cuda())
    sigma, _ = api.default_penalty(api.SIPG, DEGREE)
    P = api.Problem(api.SIPG, DEGREE, sigma, eps=tl.eps, bx=tl.b[0], by=tl.b[1], alpha=tl.alpha, f=f, gD=gD)
    vals, rhs = mesh.alloc_system(api.F64)
    x = torch.zeros(mesh.n_dofs, dtype=torch.float64, device="cuda")
    # HIP events on the Gram-Schmidt dot kernel alone (profile=2), as in the default workload
    s = api.Solver(mesh, restart=args.restart, max_iters=20000, rel_tol=1e-10, profile=2)

    def step():
        api.assemble(mesh, P, prec=api.F64, vals=vals, rhs=rhs)
        x.zero_()
        return api.newton_solve(mesh, s, vals, rhs, x, [0.0, 1.0], tol=1e-10, max_newton=50)

    for _ in range(max(args.warmup, 1)):
        r = step()
        log("warmup: %s" % r)
    s.profile(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = [step() for _ in range(max(args.steps, 1))]
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / len(reps)
    r = reps[-1]
    l2, _ = api.l2_error(mesh, x, tl.u)
    kern = {k: v for k, v in s.profile(reset=True).items() if v[0] > 0}
    dom = max(kern, key=lambda k: kern[k][1])
    launches, ms, nbytes = kern[dom]
    log("nl: %.3f s per solve, %d Newton steps, %d GMRES iterations, rel-res %.2e, L2 error %.3e; %s %.0f GB/s"
        % (dt, r["newton_steps"], r["linear_iters"], r["rel_res"], l2, dom, nbytes / (ms * 1e-3) / 1e9))
    line = {
        "metric": "DG assembly Melem/s; solves/s at rel-res 1e-10, learned+mixed vs plain FP64",
        "value": 1.0 / dt, "unit": "non-linear solves/s (assembly + Newton to ||Res||/||F|| <= 1e-10)",
        "n_gpus": 1, "steps": len(reps), "warmup": max(args.warmup, 1), "ms_per_step": dt * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (the paper's manufactured tanh-layer solution)",
        "config": {"workload": "256x256 structured, P2 SIPG (131072 triangles, 786432 dofs), r(u)=u^2, eps=1e-6, "
                               "b=(1,2)/sqrt(5), alpha=1; Newton + block-Jacobi GMRES(%d)" % args.restart,
                   "newton_steps": r["newton_steps"], "gmres_iters": int(r["linear_iters"]),
                   "rel_res": r["rel_res"], "l2_error": l2},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": nbytes / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "launches": launches, "avg_us": ms / launches * 1e3},
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_nl(W),
    }
    print(json.dumps(line), flush=True)


def cpu_baseline_nl(W, n=32):
    """The CPU oracle (single thread, FP64; Newton with direct linear solves) on
    the same problem over a 32 x 32 mesh: non-linear solves/s of that size."""
    import numpy as np
    import oracle as O
    tl, fnl = nl_problem(W)
    m = W.structured_mesh(n)
    M = O.Mesh(m.nodes, m.elems, m.dirichlet, m.neumann)
    pts = M.volume_points(DEGREE + 2)
    bp, _ = M.boundary_points(DEGREE + 2)
    sigma, kappa = O.default_penalty(O.SIPG, DEGREE)
    t0 = time.perf_counter()
    B = O.assemble(M, DEGREE, sigma=sigma, kappa=kappa, eps=tl.eps, bx=tl.b[0], by=tl.b[1], alpha=tl.alpha,
                   f=O.Field.points(fnl(pts[..., 0], pts[..., 1])), gD=O.Field.points(tl.u(bp[..., 0], bp[..., 1])))
    _, its, rel, conv = O.newton(M, DEGREE, B, [0.0, 1.0], tol=1e-10, max_newton=50)
    t = time.perf_counter() - t0
    return {"value": 1.0 / t, "unit": "non-linear solves/s (32x32 instance of the same problem)", "cores": 1,
            "kind": "oracle", **host_info(), "sample": "same problem on a %dx%d mesh (%d triangles): assembly + %d Newton steps with "
                                        "direct solves, %.2f s" % (n, n, M.T, its, t)}


def cpu_baseline_c1(m, prob, reps=20):
    """The CPU oracle (single thread, FP64): assembly + GMRES(32) to 1e-12 of
    the same problem, median of `reps` runs."""
    import numpy as np
    import oracle as O
    M = O.Mesh(m.nodes, m.elems, m.dirichlet, m.neumann)
    pts = M.volume_points(3)
    bp, _ = M.boundary_points(3)
    sigma, kappa = O.default_penalty(O.SIPG, 1)
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        B = O.assemble(M, 1, sigma=sigma, kappa=kappa, eps=prob.eps, bx=prob.b[0], by=prob.b[1], alpha=prob.alpha,
                       f=O.Field.points(prob.f(pts[..., 0], pts[..., 1])),
                       gD=O.Field.points(prob.u(bp[..., 0], bp[..., 1])))
        O.gmres(B, restart=C1_RESTART, tol=1e-12, max_iters=5000)
        ts.append(time.perf_counter() - t0)
    return {"value": float(np.median(ts) * 1e3), "unit": "ms per solve", "cores": 1, "kind": "oracle", **host_info(),
            "sample": "the full problem, median of %d runs" % reps}


def build_c3(api, W, n=512):
    m = W.structured_mesh(n, dirichlet=("left", "bottom"), neumann=("right", "top"), jitter=0.2, seed=0)
    sigma, _ = api.default_penalty(api.IIPG, 3)
    prob = api.Problem(api.IIPG, 3, sigma, eps=1e-4, bx=api.Field.affine(0.5, 0.0, -1.0),
                       by=api.Field.affine(-0.5, 1.0, 0.0), alpha=0.5, f=1.0)
    return m, prob


def bench_c3(args, api, W, torch):
    m, prob = build_c3(api, W)
    mesh = api.Mesh.from_arrays(m, 3)
    log("c3: %d triangles, %d dofs, nnzb %d" % (mesh.T, mesh.n_dofs, mesh.nnzb))
    # the default vector-ALU tensor kernel, and the matrix-core (MFMA) path for comparison
    forms = (("fp64", api.F64, api.PART_ALL), ("fp32", api.F32, api.PART_ALL),
             ("fp64_matrix_core", api.F64, api.PART_ALL | api.ASM_MATRIX_CORE),
             ("fp32_matrix_core", api.F32, api.PART_ALL | api.ASM_MATRIX_CORE))
    if args.profile_run:
        for name, prec, parts in forms:
            vals, rhs = mesh.alloc_system(prec)
            for _ in range(3):
                api.assemble(mesh, prob, prec=prec, parts=parts, vals=vals, rhs=rhs)
            del vals, rhs
        torch.cuda.synchronize()
        copy_probe(torch)
        return
    stream = torch.cuda.current_stream()
    res = {}
    systems = {}
    reps = max(args.steps, 1) * 10
    for name, prec, parts in forms:
        vals, rhs = mesh.alloc_system(prec)
        for _ in range(max(args.warmup, 1)):
            api.assemble(mesh, prob, prec=prec, parts=parts, vals=vals, rhs=rhs)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(reps):
            api.assemble(mesh, prob, prec=prec, parts=parts, vals=vals, rhs=rhs)
        ev[1].record(stream)
        ev[1].synchronize()
        t = ev[0].elapsed_time(ev[1]) / reps * 1e-3
        nbytes = assembly_bytes(mesh, 8 if prec == api.F64 else 4, f_points=False)
        res[name] = {"us": t * 1e6, "melem_s": mesh.T / t / 1e6, "GB_s": nbytes / t / 1e9,
                     "algorithmic_bytes": nbytes}
        if parts == api.PART_ALL:
            systems[name] = (vals, rhs)
        else:
            v0, r0 = systems[name.replace("_matrix_core", "")]
            res[name]["rel_diff_vs_default"] = float((vals.double() - v0.double()).norm() / v0.double().norm())
            del vals, rhs
        log("%s: %.1f us, %.0f Melem/s, %.0f GB/s" % (name, t * 1e6, mesh.T / t / 1e6, nbytes / t / 1e9))
    v64, r64 = systems["fp64"]
    v32, r32 = systems["fp32"]
    err_a = float((v32.double() - v64).norm() / v64.norm())
    err_f = float((r32.double() - r64).norm() / r64.norm())
    log("FP32 vs FP64: matrix %.3e, load vector %.3e (relative Frobenius / 2-norm)" % (err_a, err_f))
    F = res["fp64"]
    line = {
        "metric": "DG assembly Melem/s; solves/s at rel-res 1e-10, learned+mixed vs plain FP64",
        "value": F["melem_s"], "unit": "Melem/s (FP64 assembly of matrix and load vector)",
        "n_gpus": 1, "steps": reps, "warmup": max(args.warmup, 1), "ms_per_step": F["us"] * 1e-3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (jittered structured mesh, seed 0)",
        "config": {"workload": "512x512 jittered (+-0.2h, seed 0), P3 IIPG (524288 triangles, 5242880 dofs), "
                               "rotating b, eps=1e-4, alpha=0.5, f=1, D on x=0,y=0, N elsewhere; assembly only"},
        "forms": res, "fp32_vs_fp64": {"matrix_rel_fro": err_a, "load_vector_rel": err_f},
        "roofline": {"bound": "hbm", "kernel": "assemble_tensor_kernel<3,double>", "achieved": F["GB_s"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": F["GB_s"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic("assemble_c3", "fp64"),
                     "bytes_per_launch": F["algorithmic_bytes"]},
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_c3(api, W),
    }
    print(json.dumps(line), flush=True)


def cpu_baseline_c3(api, W, n=128):
    """The CPU oracle (single thread, FP64) assembling the same problem on a
    128 x 128 jittered mesh (32768 triangles, same recipe); Melem/s."""
    import oracle as O
    m, _ = build_c3(api, W, n)
    M = O.Mesh(m.nodes, m.elems, m.dirichlet, m.neumann)
    sigma, kappa = O.default_penalty(O.IIPG, 3)
    t0 = time.perf_counter()
    O.assemble(M, 3, sigma=sigma, kappa=kappa, eps=1e-4, bx=O.Field.affine(0.5, 0.0, -1.0),
               by=O.Field.affine(-0.5, 1.0, 0.0), alpha=0.5, f=1.0, gD=0.0, gN=0.0)
    t = time.perf_counter() - t0
    return {"value": M.T / t / 1e6, "unit": "Melem/s (FP64 assembly)", "cores": 1, "kind": "oracle", **host_info(),
            "sample": "same problem on a %dx%d jittered mesh (%d triangles), %.2f s" % (n, n, M.T, t)}


def bench_mlp(args, api, W, torch):
    """The warm-start perceptron (23 -> 256 -> 256 -> 256 -> 1024, BF16 products
    with FP32 accumulation) on its own: inference on the 512 held-out instances
    and one training step (forward, loss, backward, Adam) on a batch of 256,
    each timed with HIP events on the launch stream over `steps` x 50 repetitions.
    Flops count the products only: 2 B sum_l w_l w_(l+1) forward, twice that
    backward (activation and weight gradients), the first layer's input
    gradient excluded (it is not formed)."""
    import numpy as np
    from paper_1502_02941_amd import learned as L
    widths = W.mlp_widths()
    model = L.load(os.path.join(ROOT, "paper_1502_02941_amd", "data", "c5_mlp.npz"))
    feats = torch.from_numpy(L.features(L.instances(512, seed=2))).cuda()
    stream = torch.cuda.current_stream()
    fwd_flops = lambda B: 2.0 * B * sum(widths[l] * widths[l + 1] for l in range(len(widths) - 1))
    bwd_flops = lambda B: 2.0 * fwd_flops(B) - 2.0 * B * widths[0] * widths[1]
    reps = max(args.steps, 1) * 50

    def timed(fn):
        for _ in range(5):
            fn()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        for _ in range(reps):
            fn()
        ev[1].record(stream)
        ev[1].synchronize()
        return ev[0].elapsed_time(ev[1]) / reps * 1e-3

    ws = L.WarmStart(model, 512)
    t_inf = timed(lambda: ws.coarse(feats))
    net = api.MLP(widths, 256, W.mlp_init(widths, 0))
    rng = np.random.default_rng(0)
    X = torch.from_numpy(rng.standard_normal((256, widths[0])).astype(np.float32)).cuda()
    T = torch.from_numpy(rng.standard_normal((256, widths[-1])).astype(np.float32)).cuda()

    def train_step():
        net.forward(X)
        _, dy = net.loss_mse(T)
        net.backward(dy)
        net.adam_step(1e-4)

    t_train = timed(train_step)
    peak = 2500.0  # TFLOP/s, dense BF16 MFMA
    inf_tf = fwd_flops(512) / t_inf / 1e12
    train_tf = (fwd_flops(256) + bwd_flops(256)) / t_train / 1e12
    log("inference (512): %.1f us, %.2f TFLOP/s; training step (256): %.1f us, %.2f TFLOP/s" % (
        t_inf * 1e6, inf_tf, t_train * 1e6, train_tf))
    line = {
        "metric": "DG assembly Melem/s; solves/s at rel-res 1e-10, learned+mixed vs plain FP64",
        "value": 512 / t_inf, "unit": "network inferences/s (batch of 512)", "n_gpus": 1, "steps": reps,
        "warmup": 5, "ms_per_step": t_inf * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 products, f32 accumulation", "data": "synthetic (held-out instance parameters, seed 2)",
        "config": {"workload": "warm-start perceptron 23-256-256-256-1024: inference on 512 instances; training "
                               "step on 256", "train_step_us": t_train * 1e6, "train_tflops": train_tf},
        "roofline": {"bound": "mfma", "kernel": "gemm_bf16_kernel (all layers, one inference)", "achieved": inf_tf,
                     "peak": peak, "unit": "TFLOP/s", "frac": inf_tf / peak, "traffic": None},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def bench_c5(args, api, W, torch):
    import numpy as np
    from paper_1502_02941_amd import learned as L
    model = L.load(os.path.join(ROOT, "paper_1502_02941_amd", "data", "c5_mlp.npz"))
    count = args.count or 512
    out = L.evaluate(model, count=count, seed=2, reps=max(args.steps, 1), log=log, lockstep_block=args.lockstep_block)
    forms = {k: {kk: vv for kk, vv in v.items() if kk != "iters"} for k, v in out.items()
             if isinstance(v, dict) and "seconds" in v}
    F = forms["mixed+learned"]
    line = {
        "metric": "DG assembly Melem/s; solves/s at rel-res 1e-10, learned+mixed vs plain FP64",
        "value": F["solves_per_s"], "unit": "solves/s (batched: network + prolongation + assemble + solve "
                                            "to rel-res 1e-10)",
        "n_gpus": 1, "steps": max(args.steps, 1), "warmup": 1, "ms_per_step": F["seconds"] * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 network; f32 cycles + f64 refinement",
        "data": "synthetic (seeded instance sampler: training seed 1, held-out seed 2)",
        "config": {"workload": "learned warm start: %d held-out instances, 64x64 P1 SIPG (8192 triangles, 24576 "
                               "dofs each), Gaussian-sum f" % count,
                   "form": "mixed+learned", "plain_fp64_solves_per_s": forms["fp64"]["solves_per_s"],
                   "speedup_vs_plain_fp64": F["solves_per_s"] / forms["fp64"]["solves_per_s"]},
        "forms": forms, "by_log10_eps": out["by_log10_eps"],
        "coarse_rel_err_median": out["coarse_rel_err_median"], "coarse_rel_err_p90": out["coarse_rel_err_p90"],
        "guess_ms": out["guess_ms"],
        "roofline": None,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline_c5(count),
    }
    print(json.dumps(line), flush=True)


def cpu_baseline_c5(count, sample=8):
    """The CPU oracle (single thread, FP64, zero guess, restart 2N + 64) on the
    first `sample` held-out instances; solves/s of the oracle itself."""
    import oracle as O
    from paper_1502_02941_amd import learned as L
    insts = L.instances(count, seed=2)[:sample]
    from paper_1502_02941_amd import workloads as W
    ma = W.structured_mesh(L.FINE)
    t0 = time.perf_counter()
    m = O.Mesh(ma.nodes, ma.elems, ma.dirichlet, ma.neumann)
    ok = 0
    for inst in insts:
        sigma, kappa = O.default_penalty(O.SIPG, 1)
        B = O.assemble(m, 1, sigma=sigma, kappa=kappa, eps=inst.eps, bx=inst.b[0], by=inst.b[1], alpha=inst.alpha,
                       f=O.Field.gauss_sum([tuple(t) for t in inst.gauss]), gD=0.0)
        _, its, rel, conv = O.gmres(B, restart=2 * L.FINE + 64, tol=1e-10, max_iters=20000)
        ok += conv
    dt = time.perf_counter() - t0
    return {"value": len(insts) / dt, "unit": "solves/s", "cores": 1, "kind": "oracle", **host_info(),
            "sample": "first %d held-out instances (assemble + GMRES from zero), %.1f s, %d converged"
                      % (len(insts), dt, ok)}


def cpu_baseline_c4(insts, sample=12):
    """The CPU oracle (single thread, FP64, GMRES with the same restart policy
    2N + 64) on a size-stratified sample of the batch; rate scaled to the
    batch by the sample's share of the batch's dofs."""
    import numpy as np
    import oracle as O
    from paper_1502_02941_amd import workloads as W
    sizes = np.array([2 * i.N * i.N * (i.k + 1) * (i.k + 2) // 2 for i in insts])
    order = np.argsort(sizes)
    pick = order[np.linspace(0, len(order) // 2, sample).round().astype(int)]  # lower half: bounded CPU time
    t0 = time.perf_counter()
    ok = 0
    for idx in pick:
        inst = insts[idx]
        m = W.structured_mesh(inst.N)
        M = O.Mesh(m.nodes, m.elems, m.dirichlet, m.neumann)
        sigma, kappa = O.default_penalty(O.SIPG, inst.k)
        B = O.assemble(M, inst.k, sigma=sigma, kappa=kappa, eps=inst.eps, bx=inst.b[0], by=inst.b[1],
                       alpha=inst.alpha, f=O.Field.gauss_sum([tuple(t) for t in inst.gauss]), gD=0.0)
        _, its, rel, conv = O.gmres(B, restart=2 * inst.N + 64, tol=1e-10, max_iters=20000)
        ok += conv
    dt = time.perf_counter() - t0
    share = sizes[pick].sum() / sizes.sum()
    return {"value": len(pick) / dt * share * len(insts) / len(pick), "unit": "solves/s (scaled to batch dofs)",
            "cores": 1, "kind": "oracle", **host_info(),
            "sample": "%d instances from the lower half of the size order (%.2f%% of the batch dofs), %.1f s, "
                      "%d converged; solves/s = batch size / (sample time / dof share)"
                      % (len(pick), 100 * share, dt, ok)}


def cpu_baseline(m, prob, iters):
    """The CPU oracle (one thread, FP64) on a bounded sample of the same
    workload: full assembly of the 256x256 P2 system, then two single-cycle
    GMRES runs of 10 and 40 iterations.  Modified Gram-Schmidt makes iteration
    j cost about alpha + beta j; the two runs fix alpha and beta, and the solve
    time is extrapolated to `iters` iterations in one cycle (the FP64 GPU
    solve's count: the oracle's GMRES spans the same Krylov space one vector
    at a time, and the two counts agree on every size both complete)."""
    import numpy as np
    import oracle as O
    M = O.Mesh(m.nodes, m.elems, m.dirichlet, m.neumann)
    pts = M.volume_points(DEGREE + 2)
    sigma, kappa = O.default_penalty(O.SIPG, DEGREE)
    t0 = time.perf_counter()
    B = O.assemble(M, DEGREE, sigma=sigma, kappa=kappa, eps=prob.eps, bx=prob.b[0], by=prob.b[1],
                   alpha=prob.alpha, f=O.Field.points(prob.f(pts[..., 0], pts[..., 1])))
    t_asm = time.perf_counter() - t0
    # modified Gram-Schmidt: iteration j costs about alpha + beta j; two short
    # single-cycle runs fix alpha and beta
    runs = {}
    for its in (10, 40):
        t0 = time.perf_counter()
        O.gmres(B, restart=its, tol=1e-30, max_iters=its)
        runs[its] = time.perf_counter() - t0
    s10, s40 = 10 * 11 / 2.0, 40 * 41 / 2.0
    beta = (runs[40] - 4.0 * runs[10]) / (s40 - 4.0 * s10)
    alpha = (runs[10] - beta * s10) / 10.0
    J = iters
    t_solve = J * alpha + beta * J * (J + 1) / 2.0
    return {"value": 1.0 / (t_asm + t_solve), "unit": "solves/s (assemble + GMRES, extrapolated)", "cores": 1,
            "kind": "oracle", **host_info(),
            "sample": "full 256x256 P2 assembly (%.2f s, %.3f Melem/s) + single-cycle GMRES runs of 10 and 40 "
                      "iterations (%.2f s, %.2f s) fitting t(j) = %.4f + %.2e j s per iteration, extrapolated to "
                      "the %d iterations of one cycle that the FP64 GPU solve takes (%.1f s)"
                      % (t_asm, M.T / t_asm / 1e6, runs[10], runs[40], alpha, beta, J, t_solve),
            "assembly_melem_s": M.T / t_asm / 1e6}


if __name__ == "__main__":
    main()
