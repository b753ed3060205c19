"""Benchmark: Stokes DOFs/s per solve at rel-res 1e-8 (mixed vs FP64) and the
HBM bandwidth of the velocity-block SpMV, on one MI355X.

Workload (default): the unit cube cut into 64^3 cells, Kuhn split into 6
tetrahedra, interior vertices jittered by +/-0.1 h (seed 1); Taylor-Hood P2/P1
(6,440,067 velocity + 274,625 pressure DOFs); mu = 1e-3, dt = 5e-3; a seeded
8-mode Fourier forcing (seed 1001).  One step = one generalized Stokes solve:
FP64 flexible GMRES on the coupled system with the upper block-triangular
preconditioner whose blocks are fixed FP32 operators (the velocity block a
degree-6 Chebyshev-Jacobi polynomial, the lumped Cahouet-Chabard pressure
block one multigrid V-cycle), iterative refinement until the true FP64
relative residual is <= 1e-8.  The
operator is assembled once, before the timed region; the forcing is resident
in HBM.

Printed: one JSON line with the mixed-precision DOFs/s as `value`, and beside
it the same solve in other arithmetic: the FP64 path, the mixed path with
every preconditioner value stored in FP32 (no half-precision or bfloat16
copies), the mixed path with FP32 inner CG solves to a tolerance (Chebyshev-
Jacobi degree 4 preconditioner), and the mixed path with the FGMRES basis in
FP32; one pressure-correction step (the comparator of Sec. 7.5, Table 8) with
the same tolerance; the roofline of the dominant kernel (the FP32
Chebyshev-Jacobi SpMV step on the velocity block, timed with HIP events on the
solver's stream during the timed solves) and the CPU oracle baseline.
"""

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Stokes DOFs/s per solve at rel-res 1e-8 (mixed vs FP64) + SpMV HBM GB/s"

WORKLOADS = {
    # name: (dim, n, mesh_seed, mu, dt, forcing seed, description)
    "cube64": (3, 64, 1, 1e-3, 5e-3, 1001,
               "3D unit cube 64^3 Kuhn tets, jitter 0.1h seed 1, P2/P1 6,714,692 DOFs, mu=1e-3, dt=5e-3"),
    "cube32": (3, 32, 0, 1e-2, 1e-2, 1000,
               "3D unit cube 32^3 Kuhn tets, jitter 0.1h seed 0, P2/P1 859,812 DOFs, mu=1e-2, dt=1e-2"),
    "cube128": (3, 128, 2, 1e-4, 2e-3, 1002,
                "3D unit cube 128^3 Kuhn tets, jitter 0.1h seed 2, P2/P1 53,070,468 DOFs per rhs, mu=1e-4, dt=2e-3"),
}
# per-workload solver overrides: the FGMRES basis (2 m + 1 vectors of
# N_c x nrhs doubles) must fit next to the operators at 128^3
WORKLOAD_SOLVER = {"cube128": dict(restart=10)}

SOLVER = dict(method="coupled", rtol=1e-8, cheb_degree=6, inner_mode=1, inner_rtol_u=1e-2, inner_rtol_p=1e-1,
              coupled_pc=1, schur_pc=1, restart=30, max_outer=500, max_refine=12, arnoldi_fp64=1)


PROFILE_DIR = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILE_DIR, "k_cheb_step_qb_cube64_hbm_traffic.txt")


# Sources that decide what one launch of the dominant kernel reads and writes:
# the kernel bodies, their launch wrappers, the shared structures, and the
# assembly that lays out the matrix (row order, slots, packed indices).
DIGEST_SOURCES = ["kernels.h", "common.h", "ops.hip", "ops.h", "assemble.hip", "mesh_host.cpp", "mesh_host.h"]


def kernel_source_digest():
    """sha256 over the library sources that decide the dominant kernel's
    per-launch traffic (file names + contents)."""
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2407_01783_amd", "csrc")
    for path in sorted(os.path.join(src, f) for f in DIGEST_SOURCES):
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, nrhs, strain=False):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE summary, or None when that summary was taken on
    other sources (any kernel changed since), another workload, or is absent."""
    if workload != "cube64" or nrhs != 1 or strain or not os.path.exists(TRAFFIC_FILE):
        return None
    fields = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line and line.split(":", 1)[0].strip() in ("source_sha256", "hbm_bytes_per_launch"):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != kernel_source_digest() or "hbm_bytes_per_launch" not in fields:
        return None
    return float(fields["hbm_bytes_per_launch"])


ORACLE_ITERS_FILE = os.path.join(ROOT, "tests", "golden", "cube64_oracle_iters.txt")
ORACLE_SOLUTION_FILE = os.path.join(ROOT, "tests", "golden", "cube64_oracle.txt")


def error_vs_stored_oracle(u, p):
    """Nodal relative l2 error of the timed solve against the stored FP64
    oracle solution of the 64^3 workload (the velocity at every P2 node and
    the pressure at every vertex of 400 seeded elements; values written by
    tests/golden/make_cube64_golden.py).  The M-norm error is checked by the
    full-size tests."""
    import numpy as np
    vel, pres = {}, {}
    with open(ORACLE_SOLUTION_FILE) as fh:
        lines = [ln.split() for ln in fh if not ln.startswith("#")]
    i = 0
    while i < len(lines):
        key = lines[i][0]
        if key in ("vel", "p"):
            n = int(lines[i][1])
            for r in lines[i + 1:i + 1 + n]:
                (vel if key == "vel" else pres)[int(r[0])] = [float(v) for v in r[1:]]
            i += n
        i += 1
    uv = u.cpu().numpy()[0]
    pv = p.cpu().numpy()[0]
    ug = np.array([vel[k] for k in sorted(vel)]).T
    pg = np.array([pres[k][0] for k in sorted(pres)])
    eu = np.linalg.norm(uv[:, sorted(vel)] - ug) / np.linalg.norm(ug)
    ep = np.linalg.norm(pv[sorted(pres)] - pg) / np.linalg.norm(pg)
    return {"nodal_rel_l2_u": float(eu), "nodal_rel_l2_p": float(ep), "nodes": len(vel), "vertices": len(pres),
            "reference": "FP64 oracle solution (rel-res 8.4e-16) on 400 seeded elements"}


def cpu_baseline_sampled(dim, n, mesh_seed, mu, alpha, fseed, iters=1):
    """The FP64 oracle (preconditioned MINRES) on the benchmark workload
    itself, timed on a bounded sample: `iters` MINRES iterations (assembly
    excluded, as on the GPU side), scaled to a full solve by the oracle's own
    iteration count to a true relative residual <= 1e-8 on this workload
    (tests/golden/cube64_oracle_iters.txt, written by an oracle-only script)."""
    from oracle import mesh as omesh
    from oracle import stokes as ostokes
    from paper_2407_01783_amd import inputs
    with open(ORACLE_ITERS_FILE) as fh:
        k_full = next(int(ln.split()[1]) for ln in fh if ln.startswith("minres_iters_1e-8"))
    t0 = time.perf_counter()
    m = omesh.KuhnMesh(dim, n, seed=mesh_seed, jitter=0.1)
    S = ostokes.StokesSystem(m, mu, alpha)
    F, g = S.rhs(inputs.fourier_forcing(m.p2coords, fseed))
    setup = time.perf_counter() - t0
    t0, c0 = time.perf_counter(), time.process_time()
    S.solve_minres(F, g, rtol=1e-30, maxiter=iters)
    dt, cpu = time.perf_counter() - t0, time.process_time() - c0
    per_it = dt / iters
    dofs = dim * m.n_p2 + m.n_p1
    return {"value": dofs / (per_it * k_full), "unit": "DOFs/s", "cores": _threads_used(cpu, dt), "kind": "oracle",
            "sample": f"{iters} iterations of the oracle's preconditioned MINRES on this workload "
                      f"({dofs} DOFs; {dt:.1f} s wall, {cpu:.1f} s CPU; oracle assembly {setup:.0f} s "
                      f"excluded), scaled to the {k_full} iterations the oracle needs for a true rel-res <= 1e-8 "
                      f"here"}


def _threads_used(cpu_s, wall_s):
    """Threads the timed oracle work kept busy on average (process CPU time
    over wall time, at least 1)."""
    return max(1, int(round(cpu_s / wall_s))) if wall_s > 0 else 1


def cpu_baseline(dim, mesh_seed, mu, alpha, fseed, n_sample):
    """The FP64 oracle (MINRES, block preconditioner) on a smaller mesh of the
    same workload family, solved to a true relative residual <= 1e-8 (used
    for the workloads whose own oracle system is too large to assemble in a
    benchmark run)."""
    from oracle import mesh as omesh
    from oracle import stokes as ostokes
    from paper_2407_01783_amd import inputs
    m = omesh.KuhnMesh(dim, n_sample, seed=mesh_seed, jitter=0.1)
    S = ostokes.StokesSystem(m, mu, alpha)
    F, g = S.rhs(inputs.fourier_forcing(m.p2coords, fseed))
    t0, c0 = time.perf_counter(), time.process_time()
    U, P, info = S.solve_minres(F, g, rtol=1e-10)
    dt, cpu = time.perf_counter() - t0, time.process_time() - c0
    res = S.residual(U, P, F, g)
    dofs = dim * m.n_p2 + m.n_p1
    return {"value": dofs / dt, "unit": "DOFs/s", "cores": _threads_used(cpu, dt), "kind": "oracle",
            "sample": f"oracle MINRES solve (solve only, {dt:.1f} s wall, {cpu:.1f} s CPU) on the same workload "
                      f"family at n={n_sample} ({dofs} DOFs), true rel-res {res:.1e}"}


def c2_sweep(steps):
    """The paper's method comparison (Sec. 5 and 6, Figs. 1, 3, 4, 6, 7) as a
    measurement on the 32^3 workload: Schur CG with the three Cahouet-Chabard
    variants and coupled FGMRES with the three block preconditioners (FP64),
    plus the mixed benchmark configuration, for mu in {1, 1e-2, 1e-4} and the
    augmented-Lagrangian weight gamma in {0, 1, 10}; every solve to a true
    relative residual of 1e-8.  One JSON line per case (time, DOFs/s,
    iterations)."""
    import numpy as np
    import torch
    from paper_2407_01783_amd import inputs
    from paper_2407_01783_amd.stokes import StokesProblem
    dim, n, seed, _, dt, fseed, _ = WORKLOADS["cube32"]
    alpha = 1.0 / dt
    cases = [("coupled", 1, dict(coupled_pc=1, inner_mode=1, cheb_degree=6), "coupled mixed upper, fixed inner"),
             ("coupled", 0, dict(coupled_pc=0), "coupled FP64 full factorisation"),
             ("coupled", 0, dict(coupled_pc=1), "coupled FP64 upper triangular"),
             ("coupled", 0, dict(coupled_pc=2), "coupled FP64 lower triangular"),
             ("schur", 0, dict(schur_pc=1), "Schur FP64 C^Lambda (lumped)"),
             ("schur", 0, dict(schur_pc=0), "Schur FP64 C^Delta (pressure Laplacian)"),
             ("schur", 0, dict(schur_pc=2), "Schur FP64 C (consistent mass)")]
    torch.cuda.set_device(0)
    for mu in (1.0, 1e-2, 1e-4):
        for gamma in (0.0, 1.0, 10.0):
            prob = StokesProblem(dim, n, mesh_seed=seed, jitter=0.1, mu=mu, alpha=alpha, gamma=gamma)
            xy, _ = prob.mesh()
            f = torch.tensor(inputs.fourier_forcing(xy, fseed)[None], device="cuda")
            dofs = prob.total_dofs()
            for method, prec, extra, name in cases:
                o = dict(rtol=1e-8, max_outer=3000, max_refine=40, **extra)
                _, _, info = prob.solve(f, method=method, precision=prec, **o)  # warm-up
                torch.cuda.synchronize()
                t = time.perf_counter()
                for _ in range(steps):
                    _, _, info = prob.solve(f, method=method, precision=prec, **o)
                torch.cuda.synchronize()
                el = (time.perf_counter() - t) / steps
                print(json.dumps({"sweep": "cube32", "mu": mu, "gamma": gamma, "case": name,
                                  "converged": info["status"] == 0, "rel_res": info["rel_res"],
                                  "ms": el * 1e3, "dofs_per_s": dofs / el, "outer_iters": info["outer_iters"],
                                  "inner_iters_u": info["inner_iters_u"], "inner_iters_p": info["inner_iters_p"],
                                  "refinements": info["refinements"]}), flush=True)
            del prob
            torch.cuda.empty_cache()


def c4_compare(steps):
    """Batching on the 128^3 workload, as the configuration states it: eight
    right-hand sides in one batched mixed solve, against one right-hand side
    mixed and eight sequential FP64 solves (the benchmark's solver options,
    FGMRES(10)).  One JSON line."""
    import numpy as np
    import torch
    from paper_2407_01783_amd import inputs
    from paper_2407_01783_amd.stokes import StokesProblem
    dim, n, seed, mu, dt, fseed, desc = WORKLOADS["cube128"]
    opts = dict(SOLVER)
    opts.update(WORKLOAD_SOLVER["cube128"])
    method = opts.pop("method")
    torch.cuda.set_device(0)
    prob = StokesProblem(dim, n, mesh_seed=seed, jitter=0.1, mu=mu, alpha=1.0 / dt)
    xy, _ = prob.mesh()
    f8 = torch.tensor(np.stack([inputs.fourier_forcing(xy, inputs.forcing_seed(seed, b)) for b in range(8)]),
                      device="cuda")
    dofs1 = prob.total_dofs()
    out = {"workload": desc, "dofs_per_rhs": dofs1, "solver": opts}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            info = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / steps, info

    el, info = timed(lambda: prob.solve(f8, method=method, precision=1, **opts)[2])
    out["mixed_nrhs8"] = {"s": el, "dofs_per_s": 8 * dofs1 / el, "rel_res": info["rel_res"],
                          "outer_iters": info["outer_iters"], "converged": info["status"] == 0}
    print(f"[c4] batched mixed x8: {el:.3f} s", file=sys.stderr, flush=True)
    el, info = timed(lambda: prob.solve(f8[:1], method=method, precision=1, **opts)[2])
    out["mixed_nrhs1"] = {"s": el, "dofs_per_s": dofs1 / el, "rel_res": info["rel_res"],
                          "outer_iters": info["outer_iters"], "converged": info["status"] == 0}
    print(f"[c4] mixed x1: {el:.3f} s", file=sys.stderr, flush=True)

    def seq64():
        infos = [prob.solve(f8[b:b + 1], method=method, precision=0, **opts)[2] for b in range(8)]
        return max(infos, key=lambda i: i["rel_res"])

    el, info = timed(seq64)
    out["fp64_8_sequential"] = {"s": el, "dofs_per_s": 8 * dofs1 / el, "rel_res": info["rel_res"],
                                "converged": info["status"] == 0}
    print(f"[c4] 8 sequential FP64: {el:.3f} s", file=sys.stderr, flush=True)
    out["batched_over_single"] = out["mixed_nrhs8"]["dofs_per_s"] / out["mixed_nrhs1"]["dofs_per_s"]
    out["batched_over_fp64_sequential"] = out["mixed_nrhs8"]["dofs_per_s"] / out["fp64_8_sequential"]["dofs_per_s"]
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cube64", choices=sorted(WORKLOADS))
    ap.add_argument("--nrhs", type=int, default=1)
    ap.add_argument("--strain", action="store_true",
                    help="strain-rate velocity matrix alpha M + mu (L + D) instead of the vector Laplacian")
    ap.add_argument("--p3", action="store_true",
                    help="Taylor-Hood P3/P2 on the workload's mesh instead of P2/P1")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison solves")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-n", type=int, default=16, help="mesh size of the CPU oracle sample")
    ap.add_argument("--opt", action="append", default=[], help="solver option override key=value")
    ap.add_argument("--no-projection", action="store_true",
                    help="skip timing one pressure-correction step (the comparator of the paper's Sec. 7.5) with "
                         "the same tolerance")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the FP32-storage and tolerance-inner mixed legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed solves, copy 1 GiB device-to-device 3 times (a kernel of known size "
                         "for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--c2-sweep", action="store_true",
                    help="instead of the benchmark line: the method / preconditioner / mu / gamma comparison on "
                         "the 32^3 workload, one JSON line per case")
    ap.add_argument("--c4-compare", action="store_true",
                    help="instead of the benchmark line: 128^3 with eight right-hand sides batched (mixed) against "
                         "one right-hand side and eight sequential FP64 solves")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)
    if args.c2_sweep:
        c2_sweep(args.steps)
        return
    if args.c4_compare:
        c4_compare(args.steps)
        return

    import ctypes

    import numpy as np
    import torch
    from paper_2407_01783_amd import _lib, inputs
    from paper_2407_01783_amd.stokes import StokesProblem

    dim, n, seed, mu, dt, fseed, desc = WORKLOADS[args.workload]
    alpha = 1.0 / dt
    opts = dict(SOLVER)
    opts.update(WORKLOAD_SOLVER.get(args.workload, {}))
    for kv in args.opt:
        k, v = kv.split("=", 1)
        opts[k] = type(opts.get(k, 0.0))(float(v)) if k != "method" else v
    method = opts.pop("method")

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    prob = StokesProblem(dim, n, mesh_seed=seed, jitter=0.1, mu=mu, alpha=alpha, strain=args.strain, p3=args.p3)
    if args.strain:
        desc += ", strain-rate form alpha M + mu (L + D)"
    if args.p3:
        desc = re.sub(r"P2/P1 [0-9,]+ DOFs", f"P3/P2 {prob.total_dofs():,} DOFs", desc)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    print(f"[bench] assembled {args.workload} in {setup_s:.2f} s", file=sys.stderr, flush=True)
    xy, _ = prob.mesh()
    f = torch.tensor(np.stack([inputs.fourier_forcing(xy, inputs.forcing_seed(seed, b) if b else fseed)
                               for b in range(args.nrhs)]), device="cuda")
    dofs = prob.total_dofs() * args.nrhs

    def run(precision, steps, warmup, profile, **over):
        o = dict(opts, **over)
        for _ in range(warmup):  # same options as the timed solves (profiling events are created here)
            prob.solve(f, method=method, precision=precision, profile=profile, **o)
        torch.cuda.synchronize()
        infos = []
        t = time.perf_counter()
        for _ in range(steps):
            u, p, info = prob.solve(f, method=method, precision=precision, profile=profile, **o)
            infos.append(info)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        last_out[:] = [u, p]
        return el, infos

    last_out = []

    el_mixed, infos = run(1, args.steps, args.warmup, 1)
    err = None
    if (args.workload == "cube64" and args.nrhs == 1 and not args.strain and not args.p3
            and os.path.exists(ORACLE_SOLUTION_FILE)):
        err = error_vs_stored_oracle(*last_out)
    print(f"[bench] mixed: {el_mixed / args.steps * 1e3:.1f} ms/solve", file=sys.stderr, flush=True)
    ok = all(i["status"] == 0 and i["rel_res"] <= opts["rtol"] for i in infos)
    launches = sum(i["spmv_launches"] for i in infos)
    kern_s = sum(i["spmv_seconds"] for i in infos)
    bytes_per = infos[-1]["spmv_bytes"]
    achieved = bytes_per / (kern_s / launches) / 1e9 if launches else None

    def solve_level(el, infos_):
        """Solve-level roofline: the algorithmic bytes the library counted
        for every kernel of the timed solves over their wall time."""
        b = sum(i["bytes_alg"] for i in infos_) / len(infos_)
        gbs = b * len(infos_) / el / 1e9
        return {"bytes_alg_per_solve": b, "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS}

    def leg(el, infos_):
        okl = all(i["status"] == 0 and i["rel_res"] <= opts["rtol"] for i in infos_)
        return {"value": dofs * args.steps / el, "ms_per_step": el / args.steps * 1e3, "converged": okl,
                "outer_iters": infos_[-1]["outer_iters"], "inner_iters_u": infos_[-1]["inner_iters_u"],
                "inner_iters_p": infos_[-1]["inner_iters_p"], "rel_res": max(i["rel_res"] for i in infos_)}

    # phase times (GPU time by HIP events) of one more mixed solve, outside
    # the timed region (its events would perturb the timed solves)
    _, pinfos = run(1, 1, 0, 2)
    pi = pinfos[-1]
    phases = {"inner_u_ms": pi["seconds_inner_u"] * 1e3, "inner_p_ms": pi["seconds_inner_p"] * 1e3,
              "orth_ms": pi["seconds_orth"] * 1e3, "total_ms": pi["seconds_total"] * 1e3}

    fp64 = None
    if not args.no_fp64:
        el64, infos64 = run(0, args.steps, args.warmup, 0)
        ok64 = all(i["status"] == 0 and i["rel_res"] <= opts["rtol"] for i in infos64)
        fp64 = {"value": dofs * args.steps / el64, "ms_per_step": el64 / args.steps * 1e3, "converged": ok64,
                "solve_roofline": solve_level(el64, infos64),
                "outer_iters": infos64[-1]["outer_iters"], "rel_res": infos64[-1]["rel_res"]}
        print(f"[bench] fp64: {el64 / args.steps * 1e3:.1f} ms/solve", file=sys.stderr, flush=True)

    # the same mixed solve with the FGMRES basis and Gram-Schmidt updates in
    # FP32 too (faster; outside the FP64-orthogonalization contract)
    fgmres_fp32 = None
    if not args.no_fp64 and method == "coupled":
        el32, infos32 = run(1, args.steps, args.warmup, 0, arnoldi_fp64=0)
        ok32 = all(i["status"] == 0 and i["rel_res"] <= opts["rtol"] for i in infos32)
        fgmres_fp32 = {"value": dofs * args.steps / el32, "ms_per_step": el32 / args.steps * 1e3, "converged": ok32,
                       "outer_iters": infos32[-1]["outer_iters"], "rel_res": infos32[-1]["rel_res"]}
        print(f"[bench] mixed, FP32 Arnoldi basis: {el32 / args.steps * 1e3:.1f} ms/solve", file=sys.stderr,
              flush=True)

    # BJ-style FP32 inner solves: inner CG to a tolerance, Chebyshev-Jacobi
    # degree 4 preconditioner (the default leg keeps the fixed inner operators)
    tol_inner = None
    fp32_storage = None
    if not args.no_variants and method == "coupled":
        el_t, infos_t = run(1, args.steps, args.warmup, 0, inner_mode=0, cheb_degree=4)
        tol_inner = leg(el_t, infos_t)
        tol_inner["options"] = "inner_mode=TOL, cheb_degree=4, inner_rtol_u=%g, inner_rtol_p=%g" % (
            opts["inner_rtol_u"], opts["inner_rtol_p"])
        print(f"[bench] mixed, FP32 inner CG to tolerance: {el_t / args.steps * 1e3:.1f} ms/solve", file=sys.stderr,
              flush=True)
        # every preconditioner value in FP32: a second context built without
        # the half-precision A D^-1 / bfloat16 direction / half pressure levels
        saved = {k: os.environ.get(k) for k in ("STOKES_VEL_HALF", "STOKES_VEL_BF", "STOKES_PMG_HALF")}
        for k in saved:
            os.environ[k] = "0"
        try:
            prob32 = StokesProblem(dim, n, mesh_seed=seed, jitter=0.1, mu=mu, alpha=alpha, strain=args.strain,
                                   p3=args.p3)
        finally:
            for k, v in saved.items():
                if v is None:
                    os.environ.pop(k, None)
                else:
                    os.environ[k] = v
        main_prob, prob = prob, prob32
        try:
            el_s, infos_s = run(1, args.steps, args.warmup, 0)
        finally:
            prob = main_prob
            del prob32
            torch.cuda.empty_cache()
        fp32_storage = leg(el_s, infos_s)
        print(f"[bench] mixed, FP32 preconditioner storage: {el_s / args.steps * 1e3:.1f} ms/solve",
              file=sys.stderr, flush=True)

    projection = None
    if not args.no_projection:
        popts = dict(precision=1, rtol=opts["rtol"], max_inner=5000, max_refine=30)

        def proj():
            return prob.projection_step(f, **popts)
        proj()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            _, _, pinfo = proj()
        torch.cuda.synchronize()
        elp = (time.perf_counter() - t) / args.steps
        projection = {"value": dofs / elp, "ms_per_step": elp * 1e3, "converged": pinfo["status"] == 0,
                      "rel_res": pinfo["rel_res"], "inner_iters_u": pinfo["inner_iters_u"],
                      "inner_iters_p": pinfo["inner_iters_p"],
                      "solve_over_projection": (el_mixed / args.steps) / elp}
        print(f"[bench] projection step: {elp * 1e3:.1f} ms", file=sys.stderr, flush=True)

    if args.copy_calibration:
        src = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # same-run bandwidth probe: a 2 GiB device copy and read stream
    gbs = (ctypes.c_double * 2)()
    _lib.check(_lib.load().stokes_bandwidth_probe(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream),
                                                  1 << 31, 10, gbs), "stokes_bandwidth_probe")
    probe = {"copy_GBs": gbs[0], "read_GBs": gbs[1], "bytes": 1 << 31}
    print(f"[bench] probe: copy {gbs[0]:.0f} GB/s, read {gbs[1]:.0f} GB/s", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        if args.workload == "cube64" and os.path.exists(ORACLE_ITERS_FILE):
            cpu = cpu_baseline_sampled(dim, n, seed, mu, alpha, fseed)
        else:
            cpu = cpu_baseline(dim, seed, mu, alpha, fseed, args.cpu_n)

    value = dofs * args.steps / el_mixed
    line = {
        "metric": METRIC,
        "value": value,
        "unit": "DOFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": el_mixed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 outer + f32 inner (fp16/bf16-stored preconditioner values)",
        "data": "synthetic",
        "config": {"workload": desc, "nrhs": args.nrhs, "method": method,
                   "solver": {k: v for k, v in opts.items()}, "converged": ok,
                   "rel_res": max(i["rel_res"] for i in infos), "outer_iters": infos[-1]["outer_iters"],
                   "inner_iters_u": infos[-1]["inner_iters_u"], "inner_iters_p": infos[-1]["inner_iters_p"],
                   "refinements": infos[-1]["refinements"], "setup_s": setup_s},
        "fp64": fp64,
        "mixed_vs_fp64": (value / fp64["value"]) if fp64 else None,
        "mixed_fgmres_fp32_basis": fgmres_fp32,
        "mixed_fp32_storage": fp32_storage,
        "mixed_tol_inner": tol_inner,
        "phases": phases,
        "error_vs_oracle": err,
        "projection": projection,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
                     "traffic": measured_traffic(args.workload, args.nrhs, args.strain or args.p3),
                     "kernel": f"k_cheb_step_qb<_Float16,{dim * args.nrhs},G,8,true,1> (velocity-block SELL SpMV: "
                               f"half-precision A_II D^-1 values and computed or packed column offsets read from eight-slot "
                               f"interleaved copies, bfloat16 direction (adjacent-node slot pairs gathered with one "
                               f"16-byte load at W = 3), FP32 residual; a Chebyshev step of the "
                               f"deferred sum (the iterate is formed by the closing step); G lanes per row, autotuned)",
                     "bytes_per_launch": bytes_per, "launches": launches,
                     "avg_us": kern_s / launches * 1e6 if launches else None,
                     "frac_of_read_probe": (achieved / probe["read_GBs"]) if achieved else None,
                     "probe": probe,
                     "solve": dict(solve_level(el_mixed, infos),
                                   frac_of_read_probe=solve_level(el_mixed, infos)["achieved_GBs"] / probe["read_GBs"])},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
