"""Benchmark: PCG time-to-1e-8 with the nested twisted filtering preconditioner
and the preconditioner-apply bandwidth, on one MI355X.

One step = the whole hot path on one synthetic system: assemble A from kappa,
factor B (setup, plus the ILU(0) smoother of the combination preconditioner of
eq. com), and PCG to a true relative residual <= 1e-8.  Inputs are resident in
HBM before the timed region.  Prints one JSON line.

Default workload: 256^3 grid, kappa piecewise constant on 8^3 subcubes with
kappa = 10^U(-3,3) (seed 601), Dirichlet on the z = 0 face, Neumann elsewhere,
b ~ U[-1,1] (seed 602), filter t = 1; Newton Schur blocks with the ILU(0)
combination; mixed precision (float factors and sweeps, FP64 CG), next to the
same solve in FP64.

--kernels-only runs the preconditioner and the SpMV a few times plus a plain
device copy of known size (the calibration of the HBM byte counters) and exits;
it is the program the hardware-counter runs profile.

--suite paper solves the test matrices of Sec. 3 (Types 1-3 at 100^3, 200^3,
350^3, tolerances 1e-7 and 1e-10), one JSON line per case (the paper's own
preconditioner is --smoother ilu0).  --suite batch solves
many independent systems together (64 cubes of side 32..96, 4 right-hand sides
each, by default) and reports the batched sweeps' throughput.  --suite learned
trains the filter-vector network on mixture fields and compares PCG with t = 1,
with the exact lowest-eigenvector target and with the network's t.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PCG time-to-1e-8 & precond-apply GB/s, 256³ jump κ: mixed/learned vs FP64"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "apply_traffic.json")
# Sources of the sweep kernels; the recorded byte counts hold only for them.
SWEEP_SRCS = [os.path.join(ROOT, "paper_1909_09771_amd", "csrc", f)
              for f in ("ntd_sweep.h", "ntd_apply.h", "ntd_internal.h", "ntd_apply_f32.hip",
                        "ntd_apply_f64.hip", "ntd_apply_multi.h", "ntd_apply_multi_f32.hip",
                        "ntd_apply_multi_f64.hip", "ntd_vec.hip")]

# Algorithmic HBM bytes per unknown of each sweep launch (e = bytes of the
# factor precision).  Lower: the packed right-hand side, the four factor arrays
# (e1, 1/M, f2, g3) and the intermediate z written.  Upper: z read back, the
# four factor arrays and the final x written.  The FP64 right-hand side and
# output, the ILU(0) base and the r.z partials move in the pack and unpack
# kernels around the sweeps.
FACTOR_BYTES = {"mixed": 4, "fp64": 8}


def apply_bytes(prec: str, smoother: str):
    e = FACTOR_BYTES[prec]
    return {"lower": 6 * e, "upper": 6 * e}


# Algorithmic bytes per unknown of the rest of one application, outside the
# three sweep launches.  The ILU(0) forward and backward sweeps each read the
# three couplings, the inverted diagonal and their input and write their output
# (FP64).  The pack reads r (and, with the smoother, zi and the four bands for
# r - A zi) and writes the packed right-hand side; the unpack reads the packed
# result and r (and zi), and writes z.  The symmetric smoother adds a third
# stage: the SpMV into tv (48), tv = r - tv (24), both ILU(0) sweeps (96) and
# z += zi with the r.z partials (32).
def rest_bytes(prec: str, smoother: str):
    e = FACTOR_BYTES[prec]
    if smoother == "ilu0":
        return 2 * (5 * 8 + 8) + (6 * 8 + e) + (e + 3 * 8)
    if smoother == "ilu0sym":
        return 2 * (5 * 8 + 8) + (6 * 8 + e) + (e + 3 * 8) + 48 + 24 + 2 * (5 * 8 + 8) + 32
    return (8 + e) + (e + 2 * 8)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=256, help="cubic grid side")
    ap.add_argument("--prec", default="mixed", choices=["mixed", "fp64"])
    ap.add_argument("--schur", default="newton", choices=["diag", "newton"])
    ap.add_argument("--smoother", default="ilu0sym", choices=["none", "ilu0", "ilu0sym"],
                    help="ilu0sym (default): the symmetric ILU(0)-B-ILU(0) combination; ilu0: "
                         "the combination of eq. com (Sec. 3); none: B alone")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--maxit", type=int, default=5000)
    ap.add_argument("--no-compare", action="store_true", help="skip the FP64 comparison solve")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the solve with the filter network's t (trained first)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-iters", type=int, default=12, help="oracle PCG iterations sampled")
    ap.add_argument("--cpu-oracle-solve", action="store_true",
                    help="no GPU: the FP64 oracle's whole solve of the workload to --tol "
                         "(--maxit), single thread; prints its iterations, true residual, "
                         "setup and solve times as one JSON line (minutes at 256^3)")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-precond-legs", action="store_true",
                    help="skip the one-off solves with eq. com and with the diagonal block alone")
    ap.add_argument("--kernels-only", action="store_true",
                    help="run the preconditioner, the SpMV and a calibration copy, then exit")
    ap.add_argument("--reps", type=int, default=3, help="launches per kernel in --kernels-only")
    ap.add_argument("--suite", default=None, choices=["paper", "batch", "learned", "spheres"],
                    help="paper: the test matrices of Sec. 3 (Types 1-3, 100^3/200^3/350^3, "
                         "tol 1e-7 and 1e-10), one JSON line per case; batch: many independent "
                         "systems solved together, one JSON line per batch size; learned: train the "
                         "filter-vector network and compare PCG with t = 1 and with its t; spheres: "
                         "one solve of the 350^3 high-contrast inclusion field (b = 1) with its "
                         "memory footprint")
    ap.add_argument("--sizes", default="100,200,350", help="cube sides of --suite paper")
    ap.add_argument("--types", default="1,2,3",
                    help="test matrices of --suite paper: 1, 2 (as printed), 3, 2ring")
    ap.add_argument("--paper-smoothers", default="ilu0",
                    help="smoothers of --suite paper (ilu0 = the paper's eq. com)")
    ap.add_argument("--precs", default="mixed,fp64", help="precisions of --suite paper")
    ap.add_argument("--batch-counts", default="64", help="systems per batch (--suite batch)")
    ap.add_argument("--batch-rhs", type=int, default=4, help="right-hand sides per system")
    ap.add_argument("--batch-n", type=int, default=None,
                    help="one cube side for every system (default: U{32..96} per system)")
    ap.add_argument("--batch-schur", default="diag", choices=["diag", "newton"])
    ap.add_argument("--batch-seq", action="store_true",
                    help="also solve the systems one at a time (one right-hand side each)")
    ap.add_argument("--batch-tune", action="store_true",
                    help="also autotune the bandwidth kernels' launch shape (ntd_batch_tune) "
                         "and time the solve again")
    ap.add_argument("--batch-apply-only", action="store_true",
                    help="time the batched apply only (no PCG)")
    ap.add_argument("--batch-nr", type=int, default=1,
                    help="right-hand sides per wavefront pair in the line sweeps (1, 2, 4)")
    ap.add_argument("--batch-plane-lds", type=int, default=1, choices=[0, 1],
                    help="1 (default): the line sweeps keep each plane in LDS when every "
                         "workgroup fits at once (ntd_batch_set_plane_lds); 0: through memory")
    ap.add_argument("--batch-tune-sweeps", action="store_true",
                    help="autotune the right-hand sides per wavefront pair (ntd_batch_tune_sweeps)")
    ap.add_argument("--learn-train", type=int, default=32, help="training fields (--suite learned)")
    ap.add_argument("--learn-n", type=int, default=16, help="cube side of the training fields")
    ap.add_argument("--learn-epochs", type=int, default=20)
    ap.add_argument("--learn-lr", type=float, default=2e-3)
    ap.add_argument("--learn-eval", type=int, default=8, help="held-out evaluation fields")
    ap.add_argument("--learn-eval-n", type=int, default=32, help="cube side of the evaluation fields")
    ap.add_argument("--learn-maxit", type=int, default=2000, help="PCG iteration cap of the evaluation")
    ap.add_argument("--learn-target", default="binva", choices=["binva", "aeig"],
                    help="targets: the smallest eigenvector of B^-1 A (binva) or of A (aeig)")
    ap.add_argument("--learn-outer", type=int, default=8,
                    help="inverse iterations per B^-1 A target")
    ap.add_argument("--learn-inner-tol", type=float, default=1e-6,
                    help="relative tolerance of each inner solve of a B^-1 A target")
    ap.add_argument("--learn-configs", default="newton:ilu0sym,newton:ilu0,diag:none",
                    help="schur:smoother pairs of the evaluation solves")
    return ap.parse_args()


def log(msg: str):
    print("bench: " + msg, file=sys.stderr, flush=True)


def _code_only(text: str) -> str:
    """The source without comments and blank space: the recorded byte counts
    hold for the compiled code, which comments do not change."""
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def sweep_hash() -> str:
    h = hashlib.sha256()
    for path in SWEEP_SRCS:
        with open(path, encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def traffic_for(kernel: str, prec: str, smoother: str, size):
    """Measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, scaled by
    the copy-kernel calibration) if recorded for the current kernel source.
    size: the cube side, or "<side>x<systems>x<rhs>" for a batch."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    key = "%s/%s/%s/%s" % (kernel, prec, smoother, size)
    ent = rec.get("kernels", {}).get(key)
    if not ent or rec.get("sweep_sha") != sweep_hash():
        return None
    return ent.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "model unknown"


def cpu_baseline_child(args, full: bool = False):
    """The CPU baseline's own process (started by the benchmark before it
    touches the GPU; it imports no torch): the FP64 oracle, single thread, on
    the benchmark's workload -- assembly, setup and the ILU(0) factorization on
    the full grid, then --cpu-iters PCG iterations with the same
    preconditioner (full: the whole solve to --tol within --maxit, and the true
    relative residual of its solution).  Prints one JSON object."""
    import numpy as np
    import oracle as O
    import workloads as W
    n = args.n
    w = W.scaled_workload("jump", n) if n != 256 else W.workload("jump256")
    t0 = time.perf_counter()
    bands = O.assemble(w["kappa"], w["bc"])
    F = O.setup(bands, mode=args.schur)
    dt = O.ilu0(bands, 2)[0] if args.smoother != "none" else None
    t1 = time.perf_counter()
    x, it, rr, st, hist = O.pcg(bands, F, w["b"], args.tol if full else 1e-30,
                                args.maxit if full else args.cpu_iters, dt=dt,
                                smoother=args.smoother)
    t2 = time.perf_counter()
    out = {"setup_s": t1 - t0, "iters": it, "solve_s": t2 - t1,
           "s_per_iter": (t2 - t1) / max(it, 1), "status": st,
           "recursive_relres_last": float(hist[-1]) if len(hist) else None,
           "model": cpu_model(), "host_cores": os.cpu_count() or 0}
    if full:
        out.update({"workload": "jump%d" % n, "schur": args.schur, "smoother": args.smoother,
                    "tol": args.tol, "overall_s": t2 - t0, "threads": 1,
                    "true_relres": float(np.linalg.norm(w["b"] - O.spmv(bands, x))
                                         / np.linalg.norm(w["b"]))})
    print(json.dumps(out), flush=True)


def cpu_baseline_start(args):
    """Start cpu_baseline_child in its own process, before any GPU call, so the
    oracle's CPU work runs beside the GPU steps."""
    import atexit
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", "--n", str(args.n),
           "--schur", args.schur, "--smoother", args.smoother, "--cpu-iters",
           str(args.cpu_iters)]
    proc = subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)

    def reap():  # never leave the child behind, whatever ends the benchmark
        if proc.poll() is None:
            proc.kill()
            proc.wait()
    atexit.register(reap)
    return proc


def cpu_baseline_finish(proc, args, gpu_iters: int):
    """Wait for the child (it has usually finished by now), then extrapolate:
    setup + the GPU's iteration count x the oracle's time per iteration."""
    out, err = proc.communicate(timeout=900)
    if proc.returncode != 0:
        return {"error": "oracle process exited with %d: %s" % (proc.returncode, err[-400:])}
    r = json.loads(out.strip().splitlines()[-1])
    est = r["setup_s"] + gpu_iters * r["s_per_iter"]
    combo = {"ilu0": " + ILU(0) combination (eq. com)",
             "ilu0sym": " + symmetric ILU(0) combination", "none": ""}[args.smoother]
    return {"value": round(est, 3), "unit": "s", "cores": 1, "kind": "oracle",
            "setup_s": round(r["setup_s"], 3), "s_per_iter": round(r["s_per_iter"], 4),
            "iters_run": r["iters"],
            "sample": "FP64 C oracle (gcc -O3, x86-64-v3, no FP contraction), %s Schur blocks%s, "
                      "in its own process beside the GPU run: assembly + setup + ILU(0) on the "
                      "full %d^3 grid (%.2f s) and %d PCG iterations (%.3f s each), extrapolated "
                      "to the GPU's %d iterations; 1 thread of %d host cores (%s)"
                      % (args.schur, combo, args.n, r["setup_s"], r["iters"], r["s_per_iter"],
                         gpu_iters, r["host_cores"], r["model"])}


def kernels_only(args, S, b, n):
    """A short program for hardware-counter runs: the preconditioner and the
    SpMV `reps` times each, then a device copy of 2 GiB (the byte-counter
    calibration: 2 GiB read, 2 GiB written)."""
    import torch
    z = torch.empty_like(b)
    for _ in range(args.reps):
        S.apply_profile(b, z)
    q = torch.empty_like(b)
    for _ in range(args.reps):
        S.spmv(b, out=q)
    src = torch.ones(1 << 28, dtype=torch.float64, device=b.device)
    dst = torch.empty_like(src)
    for _ in range(args.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"kernels_only": True, "n": n, "prec": args.prec, "schur": args.schur,
                      "smoother": args.smoother, "reps": args.reps,
                      "copy_bytes_each_way": src.numel() * 8}), flush=True)


# Iteration counts of the paper's NTD+ILU(0) PCG (Sec. 3, Table 1), keyed by
# (type, cube side, tolerance); context for --suite paper.
TABLE1_ITERS = {(1, 100, 1e-7): 16, (1, 200, 1e-7): 22, (1, 350, 1e-7): 26,
                (2, 100, 1e-7): 16, (2, 200, 1e-7): 21, (2, 350, 1e-7): 25,
                (3, 100, 1e-7): 16, (3, 200, 1e-7): 21, (3, 350, 1e-7): 25,
                (1, 100, 1e-10): 30, (1, 200, 1e-10): 44, (1, 350, 1e-10): 55,
                (2, 100, 1e-10): 26, (2, 200, 1e-10): 35, (2, 350, 1e-10): 43,
                (3, 100, 1e-10): 26, (3, 200, 1e-10): 35, (3, 350, 1e-10): 43}


def paper_suite(args):
    """The test matrices of Sec. 3 (Types 1-3 on n^3, Dirichlet on every face;
    Type 2 as printed, whose ring is empty, and optionally the non-empty ring
    "2ring"), right-hand side b = A x* with x* ~ U[-1,1] (seed 701) formed by
    the library's SpMV, solved to the two tolerances of Table 1: setup time
    (assembly, factorization, ILU(0)), solve time, iterations and the error
    against x*, one JSON line per case."""
    import torch
    import paper_1909_09771_amd as P
    import workloads as W
    dev = torch.device("cuda:0")
    for n in [int(v) for v in args.sizes.split(",")]:
        for typ in args.types.split(","):
            w = W.scaled_workload("paper%s" % typ, n)
            kappa = torch.from_numpy(w["kappa"]).to(dev)
            xstar = torch.from_numpy(w["xstar"]).to(dev)
            del w
            for smoother in args.paper_smoothers.split(","):
                for tol in (1e-7, 1e-10):
                    for prec in args.precs.split(","):
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        S = P.Solver(kappa, P_BC_ALL, prec=prec, schur=args.schur,
                                     smoother=smoother)
                        torch.cuda.synchronize()
                        t1 = time.perf_counter()
                        b = S.spmv(xstar)
                        torch.cuda.synchronize()
                        t2 = time.perf_counter()
                        x, it, rr, st = S.pcg(b, tol=tol, maxit=args.maxit)
                        torch.cuda.synchronize()
                        t3 = time.perf_counter()
                        err = float(torch.linalg.vector_norm(x - xstar) /
                                    torch.linalg.vector_norm(xstar))
                        key = (int(typ), n, tol) if typ.isdigit() else None
                        line = {"suite": "paper", "type": typ, "n": n, "rows": n ** 3,
                                "tol": tol, "prec": prec, "schur": args.schur,
                                "smoother": smoother, "rhs": "A x*, x* ~ U[-1,1] seed 701",
                                "setup_s": round(t1 - t0, 4), "solve_s": round(t3 - t2, 4),
                                "overall_s": round(t1 - t0 + t3 - t2, 4), "iters": it,
                                "paper_iters": TABLE1_ITERS.get(key), "relres": rr,
                                "err_vs_xstar": err, "status": st,
                                "footprint_bytes": S.footprint_bytes}
                        print(json.dumps(line), flush=True)
                        del S, x, b
                        torch.cuda.empty_cache()
            del kappa, xstar


P_BC_ALL = [0, 0, 0, 0, 0, 0]


def copy_bandwidth(dev) -> float:
    """Measured device-to-device copy bandwidth (GB/s, bytes read + written) of a
    2 GiB copy, timed with events: the attainable HBM rate beside the published
    8 TB/s peak."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbps = reps * 2 * src.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbps


def batch_suite(args):
    """Many independent systems solved together: `count` cubes of side
    U{32..96} (or --batch-n), kappa constant on 8 z-slabs (10^U(-4,4)),
    Dirichlet faces, nrhs right-hand sides each (workloads.batch_systems).  Times
    the batch setup, the batched PCG to tol (the second of two solves; the first
    captures the iteration graph), and the batched preconditioner apply with the
    sweeps event-timed.  The roofline is that of the lower sweep launch:
    algorithmic bytes = per system, over the unknowns outside the twist plane,
    the four factor arrays once (4e) and the packed right-hand side and result
    of every right-hand side (2e each)."""
    import torch
    import paper_1909_09771_amd as P
    import workloads as W
    dev = torch.device("cuda:0")
    prec, schur, nrhs = args.prec, args.batch_schur, args.batch_rhs
    e = FACTOR_BYTES[prec]
    for count in [int(v) for v in args.batch_counts.split(",")]:
        systems = W.batch_systems(count, nrhs, n_fixed=args.batch_n)
        sides = [s["n"][0] for s in systems]
        kappas = [torch.from_numpy(s["kappa"]).to(dev) for s in systems]
        bs = [torch.from_numpy(b).to(dev) for s in systems for b in s["bs"]]
        del systems
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B = P.Batch(kappas, P_BC_ALL, nrhs=nrhs, prec=prec, schur=schur)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        log("batch of %d systems x %d rhs: setup %.3f s" % (count, nrhs, t1 - t0))
        sweep_group = {}
        if args.batch_tune_sweeps:
            ts0 = time.perf_counter()
            sweep_group["tuned"] = B.tune_sweeps()
            sweep_group["tune_s"] = round(time.perf_counter() - ts0, 4)
            log("line sweeps: %d right-hand sides per wavefront pair (tuned)" % sweep_group["tuned"])
        elif args.batch_nr != 1:
            B.set_sweep_group(args.batch_nr)
        sweep_group["nr"] = sweep_group.get("tuned", args.batch_nr)
        sweep_group["plane_lds"] = B.set_plane_lds(bool(args.batch_plane_lds))
        log("line sweeps: planes in %s" % ("LDS" if sweep_group["plane_lds"] else "memory"))
        if args.batch_apply_only:
            t2 = t3 = t1
            xs, its, rrs, sts = [], [0], [0.0], [0]
        else:
            B.pcg(bs, tol=args.tol, maxit=args.maxit, graph=True)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            xs, its, rrs, sts = B.pcg(bs, tol=args.tol, maxit=args.maxit, graph=True)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            passes, gap_ms, it_ms = B.solve_stats()
            log("batched PCG: %.3f s, iterations %d..%d; %d host checks, stream idle %.3f ms"
                % (t3 - t2, min(its), max(its), passes, gap_ms))
        zs = B.empty_like_entries()
        B.apply_profile(bs, zs)
        prof = [B.apply_profile(bs, zs) for _ in range(5)]
        lower_ms, twist_ms, upper_ms, rest_ms = [sorted(p[i] for p in prof)[2] for i in range(4)]
        units = sum(n ** 3 - n ** 2 for n in sides)
        kname_b = "k_apply_lower_b" + ("m" if sweep_group["nr"] != 1 else "") + \
            ("l" if sweep_group["plane_lds"] else "") + \
            ("%d" % sweep_group["nr"] if sweep_group["nr"] != 1 else "")
        by = sum((n ** 3 - n ** 2) * (4 * e + 2 * e * nrhs) for n in sides)
        achieved = by / (lower_ms * 1e-3) / 1e9
        line = {"suite": "batch" + ("-apply" if args.batch_apply_only else ""),
                "systems": count, "nrhs": nrhs, "entries": count * nrhs,
                "sides": [min(sides), max(sides)], "unknowns": sum(n ** 3 for n in sides),
                "prec": prec, "schur": schur, "tol": args.tol,
                "setup_s": round(t1 - t0, 4), "solve_s": round(t3 - t2, 4),
                "first_solve_s": round(t2 - t1, 4),
                "iters": {"min": min(its), "max": max(its),
                          "mean": round(sum(its) / len(its), 2)},
                "max_relres": max(rrs), "all_ok": all(st == 0 for st in sts),
                "apply_ms": {"lower": round(lower_ms, 4), "twist": round(twist_ms, 4),
                             "upper": round(upper_ms, 4), "rest": round(rest_ms, 4)},
                "roofline": {"kernel": kname_b, "bound": "hbm",
                             "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                             "traffic": traffic_for(kname_b, prec, "none",
                                                    "%sx%dx%d" % (args.batch_n, count, nrhs))
                             if args.batch_n else None,
                             "unknowns_per_launch": units,
                             "bytes_per_unknown": "4e + 2e x nrhs, e = %d" % e},
                "footprint_bytes": B.footprint_bytes,
                "sweep_rhs_per_wavefront_pair": sweep_group}
        if not args.batch_apply_only:
            line["host_checks"] = {"passes": passes, "stream_idle_ms": round(gap_ms, 4),
                                   "iterations_ms": round(it_ms, 3),
                                   "idle_frac": round(gap_ms / it_ms, 6) if it_ms > 0 else None}
        if args.batch_tune and not args.batch_apply_only:
            tt0 = time.perf_counter()
            g = B.tune()
            tt1 = time.perf_counter()
            B.pcg(bs, tol=args.tol, maxit=args.maxit, graph=True)   # recaptures the graph
            torch.cuda.synchronize()
            tt2 = time.perf_counter()
            xs, its2, rrs2, sts2 = B.pcg(bs, tol=args.tol, maxit=args.maxit, graph=True)
            torch.cuda.synchronize()
            tt3 = time.perf_counter()
            gmax = min(512, (max(n ** 3 for n in sides) + 1023) // 1024)
            line["tuned"] = {"gx_default": gmax, "gx": g, "tune_s": round(tt1 - tt0, 4),
                             "solve_s": round(tt3 - tt2, 4),
                             "iters_mean": round(sum(its2) / len(its2), 2),
                             "all_ok": all(st == 0 for st in sts2)}
            log("tuned launch shape: %d workgroups per entry (default %d); PCG %.3f s"
                % (g, gmax, tt3 - tt2))
        del xs, zs
        B.close()
        del B
        torch.cuda.empty_cache()
        if args.batch_seq:
            # the same systems one at a time, first right-hand side only
            t4 = time.perf_counter()
            for s, kap in enumerate(kappas):
                S = P.Solver(kap, P_BC_ALL, prec=prec, schur=schur)
                S.pcg(bs[s * nrhs], tol=args.tol, maxit=args.maxit)
                del S
            torch.cuda.synchronize()
            t5 = time.perf_counter()
            line["sequential_one_rhs_s"] = round(t5 - t4, 4)
            log("one system at a time (setup + PCG, one rhs each): %.3f s" % (t5 - t4))
        print(json.dumps(line), flush=True)
        del kappas, bs
        torch.cuda.empty_cache()


# Multiply-adds of the filter network per voxel (2 flops each): 27 x 16 for
# layer 1, 432 x 16 for layers 2 and 3, 432 for layer 4.
CNN_FLOP_PER_VOXEL = 2 * (27 * 16 + 2 * 432 * 16 + 432)
# Algorithmic HBM bytes of one prediction per voxel: kappa read twice (mean,
# feature: 16), the feature written and read (4), three hidden maps of 16 bf16
# written and read (192), y and t written (12).
CNN_BYTES_PER_VOXEL = 16 + 4 + 192 + 12


def spheres_suite(args):
    """The high-contrast inclusion workload: --n^3 (default 350^3, 42.9 M unknowns),
    200 spheres of radius U(0.02, 0.08) with kappa = 1e6 inside and 1 outside
    (seed 301), Dirichlet faces, b = 1, t = 1; one setup and one PCG solve to --tol
    per --precs entry with --schur/--smoother.  Reports setup and solve times,
    iterations, the true relative residual, ntd_footprint_bytes and the drop of
    free device memory from before the setup to after it (hipMemGetInfo)."""
    import time
    import numpy as np
    import torch
    import paper_1909_09771_amd as P
    import workloads as W
    dev = torch.device("cuda:0")
    n = args.n if args.n != 256 else 350
    w = W.workload("spheres350") if n == 350 else W.scaled_workload("spheres", n)
    kappa = torch.from_numpy(w["kappa"]).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(w["b"])).to(dev)
    log("spheres %d^3: kappa in [%g, %g], inside fraction %.4f" % (
        n, w["kappa"].min(), w["kappa"].max(), float((w["kappa"] > 1).mean())))
    for prec in args.precs.split(","):
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        free0 = torch.cuda.mem_get_info(dev)[0]
        t0 = time.perf_counter()
        S = P.Solver(kappa, w["bc"], prec=prec, schur=args.schur, smoother=args.smoother)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        free1 = torch.cuda.mem_get_info(dev)[0]
        x, it, rr, st, hist = S.pcg_history(
            b, tol=args.tol, maxit=args.maxit, every=150,
            progress=lambda i, r: log("%s: iteration %d, relres %.3e" % (prec, i, r)))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        # the recursive residual every 10 % of the run, and its smallest value
        marks = sorted(set([max(1, (it * q) // 10) for q in range(1, 11)])) if it else []
        line = {"suite": "spheres", "n": n, "prec": prec, "schur": args.schur,
                "smoother": args.smoother, "tol": args.tol, "iters": it, "relres": rr,
                "status": st, "setup_s": round(t1 - t0, 4), "solve_s": round(t2 - t1, 4),
                "overall_s": round(t2 - t0, 4), "footprint_bytes": S.footprint_bytes,
                "mem_get_info_delta_bytes": int(free0 - free1),
                "residual_trend": {str(m): float("%.3e" % hist[m - 1]) for m in marks},
                "min_recursive_relres": float("%.3e" % min(hist)) if hist else None}
        print(json.dumps(line), flush=True)
        S.close()
        del S, x
        torch.cuda.empty_cache()


def learned_suite(args):
    """The learned filter vector: targets (--learn-target: the smallest-eigenvalue
    eigenvector of B^-1 A by the library's inverse iteration, or the lowest
    eigenvector of A by inverse iteration with the batched FP64 PCG) on
    --learn-train mixture fields
    of side --learn-n (seeds 10000+i), Adam training, then PCG to --tol with
    t = 1, with the exact target and with the network's t on --learn-eval held-out
    fields of side --learn-eval-n (seeds 20000+i, b ~ U[-1,1] seed 30000+i),
    MIXED, for each --learn-configs preconditioner (default: Newton blocks with the
    symmetric and with the eq. com combination, and the diagonal blocks alone).
    One JSON line for the training, one per evaluation configuration."""
    import time
    import numpy as np
    import torch
    import paper_1909_09771_amd as P
    from paper_1909_09771_amd import learned as Lr
    import workloads as W
    dev = torch.device("cuda:0")
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    bc = W.BC_ALL_DIRICHLET
    n = args.learn_n
    kap = [g(W.kappa_mixture(n, 10000 + i)) for i in range(args.learn_train)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tgt = []
    if args.learn_target == "binva":
        starts = [g(W.filter_random(n, n, n, 40000 + i)) for i in range(len(kap))]
        tgt, lams = Lr.binva_targets(
            kap, [bc] * len(kap), starts, schur="newton", outer=args.learn_outer,
            inner_tol=args.learn_inner_tol, inner_maxit=200000,
            progress=lambda i, lam, it, sec: log("training target %d: lambda %.3e, %d inner "
                                                 "steps, %.1f s" % (i, lam, it, sec)))
    else:
        for i in range(0, len(kap), 64):
            tgt += Lr.eigen_targets(kap[i:i + 64], [bc] * len(kap[i:i + 64]))
    torch.cuda.synchronize()
    t_targets = time.perf_counter() - t0
    log("targets (%s): %d fields of %d^3 in %.2f s" % (args.learn_target, len(kap), n, t_targets))
    net = P.FilterNet(W.cnn_init_params(0))
    t0 = time.perf_counter()
    hist = Lr.train(net, kap, tgt, args.learn_epochs, args.learn_lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    for ep in range(0, len(hist), max(1, len(hist) // 10)):
        log("epoch %d: loss %.4e" % (ep, hist[ep]))
    log("training: %d steps in %.2f s, final loss %.4e" % (len(kap) * len(hist), t_train, hist[-1]))
    net.release_workspaces()
    del kap, tgt
    torch.cuda.empty_cache()

    ne = args.learn_eval_n
    evk = [W.kappa_mixture(ne, 20000 + i) for i in range(args.learn_eval)]
    # the network's forward pass at the evaluation size: event-timed median of 5
    kd = g(evk[0])
    tout = torch.empty_like(kd)
    net.predict(kd, tout)
    ms = []
    for _ in range(5):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        net.predict(kd, tout)
        b.record()
        b.synchronize()
        ms.append(a.elapsed_time(b))
    pred_ms = float(np.median(ms))
    vox = ne ** 3
    print(json.dumps({
        "suite": "learned", "phase": "train", "train_fields": args.learn_train, "train_n": n,
        "epochs": args.learn_epochs, "lr": args.learn_lr, "targets_s": round(t_targets, 3),
        "train_s": round(t_train, 3), "ms_per_train_step": round(1e3 * t_train / (len(hist) * args.learn_train), 4),
        "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1],
        "predict_ms": round(pred_ms, 4), "predict_n": ne,
        "predict_TFLOPs": round(CNN_FLOP_PER_VOXEL * vox / (pred_ms * 1e-3) / 1e12, 2),
        "predict_GBps": round(CNN_BYTES_PER_VOXEL * vox / (pred_ms * 1e-3) / 1e9, 1),
        "peak_bf16_TFLOPs": 2500.0, "peak_hbm_GBps": 8000.0}), flush=True)
    del kd, tout
    evt_cache, lam_cache = {}, {}

    def eval_targets(schur):
        if args.learn_target != "binva":
            schur = "any"
        if schur not in evt_cache:
            te = time.perf_counter()
            if args.learn_target == "binva":
                starts = [g(W.filter_random(ne, ne, ne, 50000 + i)) for i in range(len(evk))]
                evt_cache[schur], lam_cache[schur] = Lr.binva_targets(
                    [g(k) for k in evk], [bc] * len(evk), starts, schur=schur,
                    outer=args.learn_outer, inner_tol=args.learn_inner_tol, inner_maxit=200000,
                    progress=lambda i, lam, it, sec: log(
                        "evaluation target %d (%s): lambda %.3e, %d inner steps, %.1f s"
                        % (i, schur, lam, it, sec)))
            else:
                evt_cache[schur] = Lr.eigen_targets([g(k) for k in evk], [bc] * len(evk))
            log("evaluation targets (%s, %s blocks): %.1f s" % (args.learn_target, schur,
                                                               time.perf_counter() - te))
        return evt_cache[schur]

    for schur, smoother in (c.split(":") for c in args.learn_configs.split(",")):
        evt = eval_targets(schur)
        rows = []
        for i, k in enumerate(evk):
            kd = g(k)
            b = g(W.rhs_uniform(ne, ne, ne, 30000 + i))
            r = Lr.compare(net, kd, bc, b, tol=args.tol, maxit=args.learn_maxit, prec="mixed",
                           schur=schur, smoother=smoother)
            r["target"] = Lr.solve_with(kd, bc, b, evt[i], args.tol, args.learn_maxit, "mixed",
                                        schur, smoother)
            log("%s+%s field %d: iterations ones %d, target %d%s, learned %d%s" % (
                schur, smoother, i, r["ones"]["iters"], r["target"]["iters"],
                " (t=1 fallback)" if r["target"]["fallback"] else "", r["learned"]["iters"],
                " (t=1 fallback)" if r["learned"]["fallback"] else ""))
            rows.append(r)
        summ = {}
        conv = [r for r in rows if all(r[k]["status"] == 0 for k in ("ones", "target", "learned"))]
        for key in ("target", "learned"):   # against t = 1, on fields every candidate solved
            d = [r[key]["iters"] - r["ones"]["iters"] for r in conv]
            summ[key + "_vs_ones"] = dict(fewer=int(sum(x < 0 for x in d)),
                                          same=int(sum(x == 0 for x in d)),
                                          more=int(sum(x > 0 for x in d)),
                                          mean_change_pct=round(float(np.mean(
                                              [100.0 * (r[key]["iters"] / r["ones"]["iters"] - 1)
                                               for r in conv])) if conv else 0.0, 2))
        for key in ("ones", "target", "learned"):
            summ[key] = dict(
                mean_iters=round(float(np.mean([r[key]["iters"] for r in rows])), 2),
                total_s=round(float(np.sum([r[key]["seconds"] for r in rows])), 3),
                fallbacks=int(np.sum([r[key]["fallback"] for r in rows])),
                all_converged=bool(all(r[key]["status"] == 0 for r in rows)))
        print(json.dumps({
            "suite": "learned", "phase": "eval", "eval_fields": len(evk), "eval_n": ne,
            "schur": schur, "smoother": smoother, "prec": "mixed", "tol": args.tol,
            "target": args.learn_target,
            "target_lambda": lam_cache.get(schur),
            "target_frac_at_floor": [round(float((t <= 1e-3).double().mean()), 4) for t in evt],
            "iters": {k: [r[k]["iters"] for r in rows] for k in ("ones", "target", "learned")},
            "summary": summ}), flush=True)


def main():
    args = parse()
    if args.cpu_baseline_child or args.cpu_oracle_solve:
        cpu_baseline_child(args, full=args.cpu_oracle_solve)
        return
    if args.gpus != 1:
        print("bench.py: runs on one GPU only (--gpus 1); the level-3 twist split "
              "across two GPUs is a design, not built", file=sys.stderr)
        sys.exit(2)
    if args.suite == "paper":
        paper_suite(args)
        return
    if args.suite == "batch":
        batch_suite(args)
        return
    if args.suite == "learned":
        learned_suite(args)
        return
    if args.suite == "spheres":
        spheres_suite(args)
        return
    cpu_proc = None
    if not args.no_cpu and not args.kernels_only:
        cpu_proc = cpu_baseline_start(args)   # before the first GPU call
    import torch
    import paper_1909_09771_amd as P
    import workloads as W

    dev = torch.device("cuda:0")
    n = args.n
    w = W.scaled_workload("jump", n) if n != 256 else W.workload("jump256")
    kappa = torch.from_numpy(w["kappa"]).to(dev)
    b = torch.from_numpy(w["b"]).to(dev)
    bc = w["bc"]
    torch.cuda.synchronize()

    def make(prec):
        return P.Solver(kappa, bc, prec=prec, schur=args.schur, smoother=args.smoother)

    if args.kernels_only:
        kernels_only(args, make(args.prec), b, n)
        return

    split = []  # (setup s, solve s) of each step; both calls synchronize

    def step(prec):
        ta = time.perf_counter()
        S = make(prec)
        tb = time.perf_counter()
        x, it, rr, st = S.pcg(b, tol=args.tol, maxit=args.maxit)
        split.append((tb - ta, time.perf_counter() - tb))
        return S, x, it, rr, st

    for i in range(args.warmup):
        S, x, it, rr, st = step(args.prec)
        log("warmup %d: %d iterations, relres %.3e, status %d" % (i, it, rr, st))
        del S, x
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        S, x, it, rr, st = step(args.prec)
        results.append((it, rr, st))
        log("step %d: %d iterations, relres %.3e, status %d" % (i, it, rr, st))
        if i != args.steps - 1:
            del S, x
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    timed = split[-args.steps:]
    setup_s = sum(v[0] for v in timed) / len(timed)
    solve_s = sum(v[1] for v in timed) / len(timed)
    iters, relres, status = results[-1]

    # Preconditioner launches as PCG issues them, timed with HIP events on the
    # solver's stream (median of 21).
    z = torch.empty_like(b)
    S.apply_profile(b, z)
    prof = [S.apply_profile(b, z) for _ in range(21)]
    med = [sorted(p[i] for p in prof)[10] for i in range(4)]
    lower_ms, twist_ms, upper_ms, rest_ms = med
    sweeps_ms = lower_ms + twist_ms + upper_ms
    N = n ** 3
    by = apply_bytes(args.prec, args.smoother)
    units = (n - 1) * n * n  # unknowns outside the twist plane: one half chain each side
    cand = {"k_apply_lower": (lower_ms, by["lower"] * units),
            "k_apply_upper": (upper_ms, by["upper"] * units)}
    kname = max(cand, key=lambda k: cand[k][0])
    k_ms, k_bytes = cand[kname]
    achieved = k_bytes / (k_ms * 1e-3) / 1e9
    sweeps_gbs = (by["lower"] + by["upper"]) * N / (sweeps_ms * 1e-3) / 1e9
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    q = S.spmv(b)
    e0.record()
    for _ in range(10):
        S.spmv(b, out=q)
    e1.record()
    torch.cuda.synchronize()
    spmv_ms = e0.elapsed_time(e1) / 10
    footprint = S.footprint_bytes
    x_main = x.clone()
    del S, x

    extra = {}
    if not args.no_compare:
        other = "fp64" if args.prec == "mixed" else "mixed"
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        S2, x2, it2, rr2, st2 = step(other)
        torch.cuda.synchronize()
        c1 = time.perf_counter()
        diff = (torch.linalg.vector_norm(x_main - x2) / torch.linalg.vector_norm(x2)).item()
        extra["compare"] = {"prec": other, "s_to_solution": round(c1 - c0, 4), "iters": it2,
                            "relres": rr2, "status": st2,
                            "rel_diff_of_solutions": diff}
        log("comparison solve (%s): %.2f s, %d iterations" % (other, c1 - c0, it2))
        x_other = x2.cpu().numpy()
        del S2, x2

    if not args.no_precond_legs:
        # the paper's own preconditioner (eq. com) and the diagonal block alone,
        # one solve each in the benchmark's precision
        legs = []
        for schur, smoother in (("newton", "ilu0"), ("diag", "none")):
            torch.cuda.synchronize()
            p0 = time.perf_counter()
            SP = P.Solver(kappa, bc, prec=args.prec, schur=schur, smoother=smoother)
            xp, itp, rrp, stp = SP.pcg(b, tol=args.tol, maxit=args.maxit)
            torch.cuda.synchronize()
            p1 = time.perf_counter()
            legs.append({"schur": schur, "smoother": smoother, "prec": args.prec,
                         "s_to_solution": round(p1 - p0, 4), "iters": itp, "relres": rrp,
                         "status": stp})
            log("%s + %s solve: %.2f s, %d iterations" % (schur, smoother, p1 - p0, itp))
            del SP, xp
        extra["compare_preconditioners"] = legs

    if not args.no_learned:
        # The filter network (--suite learned's defaults): 32 mixture fields of
        # 16^3, all faces Dirichlet, targets from inverse iteration on B^-1 A
        # (Newton blocks, 8 steps, inner solves to 1e-6), 20 epochs; then the
        # same solve with its t.
        import numpy as np
        from paper_1909_09771_amd import learned as Lr
        torch.cuda.synchronize()
        l0 = time.perf_counter()
        g16 = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
        kap = [g16(W.kappa_mixture(16, 10000 + i)) for i in range(32)]
        starts = [g16(W.filter_random(16, 16, 16, 40000 + i)) for i in range(32)]
        net, hist, _, _ = Lr.train_on_binva_targets(kap, [W.BC_ALL_DIRICHLET] * 32, starts,
                                                    W.cnn_init_params(0))
        del kap, starts
        torch.cuda.synchronize()
        l1 = time.perf_counter()
        tl = net.predict(kappa)
        torch.cuda.synchronize()
        l2 = time.perf_counter()
        # setup with the predicted t (t = 1 if its factorization loses a positive
        # pivot), then PCG
        rl = Lr.solve_with(kappa, bc, b, tl, args.tol, args.maxit, args.prec, args.schur,
                           args.smoother)
        itl = rl["iters"]
        spread = (tl.max() / tl.min()).item()
        extra["compare_learned"] = {
            "prec": args.prec, "s_to_solution": round(l2 - l1 + rl["seconds"], 4),
            "predict_s": round(l2 - l1, 4), "train_s": round(l1 - l0, 3), "iters": itl,
            "relres": rl["relres"], "status": rl["status"], "t_fallback": rl["fallback"],
            "t_max_over_min": round(spread, 4),
            "net": "4 conv layers 3x3x3, trained on the B^-1 A targets of 32 mixture fields of "
                   "16^3 with all faces Dirichlet (this workload has Dirichlet at z=0 only), "
                   "final loss %.4g" % hist[-1]}
        log("learned-t solve: %.2f s (predict %.3f s), %d iterations; t max/min %.3f%s"
            % (l2 - l1 + rl["seconds"], l2 - l1, itl, spread,
               " (t = 1: the predicted t lost a positive pivot)" if rl["fallback"] else ""))
        del tl, net
        torch.cuda.empty_cache()

    precond_ms = sweeps_ms + rest_ms
    copy_gbps = copy_bandwidth(dev)
    line = {
        "metric": METRIC,
        "value": round(ms_per_step / 1e3, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32-precond/f64-cg" if args.prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": "jump%d" % n, "grid": [n, n, n],
                   "kappa": "8^3 subcubes, 10^U(-3,3), seed %d" % (601 if n == 256 else 201),
                   "bc": "Dirichlet z=0, Neumann else", "tol": args.tol, "prec": args.prec,
                   "schur": args.schur, "smoother": args.smoother, "filter": "t=1",
                   "learned": "compare_learned: the same solve with the filter network's t"},
        "iters": iters,
        "setup_s": round(setup_s, 4),
        "solve_s": round(solve_s, 4),
        "relres": relres,
        "status": status,
        "precond_ms": round(precond_ms, 4),
        "sweeps_ms": round(sweeps_ms, 4),
        "sweeps_GBps": round(sweeps_gbs, 2),
        "launch_ms": {"lower": round(lower_ms, 4), "twist": round(twist_ms, 4),
                      "upper": round(upper_ms, 4), "rest": round(rest_ms, 4)},
        "spmv_ms": round(spmv_ms, 4),
        "hbm_copy_GBps": round(copy_gbps, 1),
        "spmv_GBps": round(48 * N / (spmv_ms * 1e-3) / 1e9, 1),
        "footprint_bytes": footprint,
        "roofline": {"kernel": kname, "bound": "hbm", "achieved": round(achieved, 2),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5),
                     "traffic": traffic_for(kname, args.prec, args.smoother, n),
                     "measured_copy_GBps": round(copy_gbps, 1),
                     "frac_of_measured_copy": round(achieved / copy_gbps, 5),
                     # the launch is a chain of dependent line solves: the longer
                     # level-3 half walks n-1-floor((n-1)/2) planes, each plane a lower
                     # and an upper level-2 pass over about n lines in all
                     "chain_line_steps": (n - 1 - (n - 1) // 2) * n,
                     "us_per_line_step": round(k_ms * 1e3 / ((n - 1 - (n - 1) // 2) * n), 4)},
    }
    line["rest_GBps"] = round(rest_bytes(args.prec, args.smoother) * N / (rest_ms * 1e-3) / 1e9, 1)
    line.update(extra)
    if cpu_proc is not None:
        # The oracle leg, after the timed region: the FP64 oracle's own SpMV
        # recomputes the true relative residual of the GPU's solutions (the
        # error of each result against the oracle), then its timed baseline.
        import numpy as np
        import oracle as O
        bands = O.assemble(w["kappa"], w["bc"])
        bn = np.linalg.norm(w["b"])
        errs = {args.prec: float(np.linalg.norm(w["b"] - O.spmv(bands, x_main.cpu().numpy())) / bn)}
        if not args.no_compare:
            errs[other] = float(np.linalg.norm(w["b"] - O.spmv(bands, x_other)) / bn)
        line["oracle_true_relres"] = errs
        del bands
        log("collecting the CPU oracle baseline")
        line["cpu_baseline"] = cpu_baseline_finish(cpu_proc, args, iters)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
