"""Benchmark of the spectral Stokes hot path on one MI355X.

Workloads (N=1):
* tree (default): the 3-generation vessel tree (7 bifurcations, radii
  shrinking by sqrt 2 per generation) with ~12M tets (~52M complex unknowns
  per mode) and one seeded waveform of 64 harmonics plus the mean: 65 mode
  systems. They are solved in waves of `--batch` systems (default 2; memory:
  one FP64 Krylov basis of restart 40 is ~35 GB per system), and one step is
  one wave: system k belongs to wave k mod n_waves, so every wave mixes low
  and high modes, and the steps run through the waves in turn.
* pipe: straight pipe R=1, L=10 with ~200k curved quadratic tets (~0.88M
  complex unknowns per mode), 16 harmonics plus the mean; one step = all 17.
* ybatch: 4 Y-bifurcations of about 0.3/0.6/1.2/2.4M tets, 12 cases of 32
  harmonics plus the mean on each, every case with its own period: 1,584
  systems in one step (`run_ybatch`).
* ylearn: the learned warm start on the 1.2M-tet Y, one POD basis and network
  per harmonic, zero-guess against warm-started solves of held-out waveforms
  (`run_ylearn`).

Per-mesh setup (ingest, assembly of the mode-independent matrices, the
preconditioner's multigrid hierarchies) runs once and is reported separately.
One step = per-mode right-hand sides + batched block-preconditioned GMRES to
the relative residual `--rtol` + time synthesis of the step's modes. During
the timed steps every library kernel launch is bracketed by HIP events on the
stream it runs on; the dominant kernel's algorithmic bytes per launch divided
by its mean launch time gives the roofline entry. The CPU baseline times the
oracle (assembly + sparse LU per mode) in a process pool over the host's cores
on small replicas of the workload and extrapolates to the full size with the
LU cost exponent measured between the replicas (labelled as such). Prints one
JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from workloads import cases  # noqa: E402

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILES = {"tree": os.path.join(ROOT, "profiles", "traffic_tree12m.json"),
                 "pipe": os.path.join(ROOT, "profiles", "traffic_pipe200k.json")}


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["tree", "pipe", "ybatch", "ylearn"], default="tree",
                    help="tree: the default; pipe: the 200k-tet pipe; ybatch: the batching workload "
                         "(4 Y-bifurcations of 0.3/0.6/1.2/2.4M tets, 12 cases of 32 harmonics each; "
                         "one step solves all 1,584 systems); ylearn: the learned warm start on the "
                         "1.2M-tet Y (per-harmonic POD and MLP, held-out waveforms)")
    ap.add_argument("--ymesh", type=int, choices=[0, 1, 2, 3], default=None,
                    help="ybatch: run only the k-th mesh (0.3/0.6/1.2/2.4M tets)")
    ap.add_argument("--tets", type=int, default=None, help="default: 12,000,000 (tree), 200,000 (pipe)")
    ap.add_argument("--harmonics", type=int, default=None, help="default: 64 (tree), 16 (pipe)")
    ap.add_argument("--batch", type=int, default=None,
                    help="systems per step (a wave); default: 2 (tree), all (pipe)")
    ap.add_argument("--rtol", type=float, default=None,
                    help="relative residual; default 2e-12 (tree), 4e-12 (pipe), which keep every mode "
                         "within 1e-8 of the reference (the tree's steady pressure has the largest "
                         "error-to-residual ratio)")
    ap.add_argument("--restart", type=int, default=40)
    ap.add_argument("--cheb-vel", type=int, default=12)
    ap.add_argument("--cheb-pres", type=int, default=50)
    ap.add_argument("--cheb-ratio", type=float, default=300.0,
                    help="the polynomials target [lambda_max/ratio, lambda_max] of the Jacobi-scaled blocks")
    ap.add_argument("--cheb-ratio-pres", type=float, default=1000.0,
                    help="interval ratio of the pressure polynomial (0: --cheb-ratio)")
    ap.add_argument("--ntimes", type=int, default=None, help="synthesis instants; default 16 (tree), 64 (pipe)")
    ap.add_argument("--precision", choices=["fp64", "mixed", "mixed32"], default="mixed",
                    help="mixed: FP32 operator and velocity block in FP64 refinement; mixed32: also an FP32 "
                         "Krylov basis (FP64 arithmetic)")
    ap.add_argument("--penalty", type=float, default=0.0,
                    help="penalized variant: continuity block -(penalty/mu) Mp (0: the method itself)")
    ap.add_argument("--windkessel", type=str, default=None, metavar="RP,C,RD",
                    help="three-element lumped model on the outlet instead of a traction-free outlet")
    ap.add_argument("--inner-rtol", type=float, default=3e-5,
                    help="mixed precision: end a cycle once its own residual fell by this factor")
    ap.add_argument("--vel-block", choices=["cheb", "mg"], default="mg",
                    help="velocity block: Chebyshev polynomial of the real shift, or a multigrid V-cycle")
    ap.add_argument("--pres-block", choices=["cheb", "mg"], default="mg",
                    help="pressure-Laplacian inverse in the Schur block: Chebyshev polynomial or multigrid")
    ap.add_argument("--mg-smooth", type=int, default=2, help="multigrid smoothing steps per side")
    ap.add_argument("--mg-post0", type=int, default=None,
                    help="multigrid steps after the coarse correction on the velocity's quadratic level; "
                         "default 1 (tree), 0 = --mg-smooth (pipe, ybatch)")
    ap.add_argument("--mg-ratio", type=float, default=None,
                    help="multigrid smoother interval ratio; default 10 (tree, pipe: every mode converges and "
                         "it is the fastest there), 4 (ybatch: the library default, robust on the Y meshes)")
    ap.add_argument("--steady-schur-omega", type=float, default=-1.0,
                    help="w of the steady systems' Schur Laplacian term (-1: the largest |w| of the case, 0: off)")
    ap.add_argument("--orth", type=int, choices=[0, 1], default=1,
                    help="0: two-pass classical Gram-Schmidt, 1: lagged second pass (DCGS2)")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the plain per-mode FP64 GMRES comparator step")
    ap.add_argument("--compare-systems", type=int, default=None,
                    help="systems of the first wave the comparator solves one at a time; default 2 (tree), all (pipe)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library time its candidate restart lengths and Chebyshev degrees first "
                         "(untimed setup); the defaults are what it picks on this workload")
    ap.add_argument("--no-warm-start", action="store_true",
                    help="skip the learned-warm-start leg (pipe workload; reported beside the headline)")
    ap.add_argument("--ws-periods", type=int, default=4,
                    help="training periods for the warm start (each gives one solve per harmonic)")
    ap.add_argument("--ws-snapshots", type=int, default=16,
                    help="ylearn: training periods per harmonic solved for its POD (its rank)")
    ap.add_argument("--ws-heldout", type=int, default=4,
                    help="ylearn: held-out waveforms timed (all harmonics of each)")
    ap.add_argument("--no-graph-leg", action="store_true",
                    help="skip re-running the first two waves with the event profiler off (graph replay on)")
    ap.add_argument("--no-error-check", action="store_true",
                    help="skip the tight-tolerance FP64 reference solve that estimates the error")
    ap.add_argument("--verbose", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain 1 GiB device copies (for scaling rocprofv3 byte counters)")
    a = ap.parse_args(argv)
    tree = a.workload == "tree"
    ylearn = a.workload == "ylearn"
    if a.tets is None:
        a.tets = 12_000_000 if tree else 1_200_000 if ylearn else 200_000
    if a.harmonics is None:
        a.harmonics = 64 if tree else 32 if ylearn else 16
    if a.ntimes is None:
        a.ntimes = 16 if tree else 64
    if a.rtol is None:
        a.rtol = 4e-12 if a.workload == "pipe" else 2e-12
    if a.mg_ratio is None:
        a.mg_ratio = 4.0 if a.workload in ("ybatch", "ylearn") else 10.0
    if a.mg_post0 is None:
        a.mg_post0 = 1 if tree else 0
    if a.batch is None:
        a.batch = 2 if tree else 16 if ylearn else 0
    if a.compare_systems is None:
        a.compare_systems = 2 if tree else 0
    return a


def solver_opts(args):
    """The solver options of the timed steps (also used by the full-size parity test)."""
    from paper_2009_06725_amd import scvs
    return scvs.default_opts(rtol=args.rtol, restart=args.restart, cheb_vel=args.cheb_vel,
                             cheb_pres=args.cheb_pres, cheb_ratio=args.cheb_ratio,
                             cheb_ratio_pres=args.cheb_ratio_pres, verbose=1 if args.verbose else 0,
                             precision={"fp64": 0, "mixed": 1, "mixed32": 2}[args.precision], orth=args.orth,
                             inner_rtol=args.inner_rtol, penalty=args.penalty,
                             vel_block=1 if args.vel_block == "mg" else 0,
                             pres_block=1 if args.pres_block == "mg" else 0,
                             mg_smooth=args.mg_smooth, mg_ratio=args.mg_ratio, mg_post0=args.mg_post0,
                             steady_schur_omega=args.steady_schur_omega if args.steady_schur_omega >= 0 else
                             2.0 * np.pi * args.harmonics)


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def stored_traffic(kernel: str, workload: str):
    """Bytes per launch beyond L2 (FETCH_SIZE + WRITE_SIZE, copy-calibrated) from the
    committed rocprofv3 counter summary of this workload, or None when absent or
    taken on different kernel sources."""
    from paper_2009_06725_amd.rocprof_summary import kernel_source_hash
    try:
        with open(TRAFFIC_FILES[workload]) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch", {}).get(kernel)


def copy_calibration(gib: float = 1.0, reps: int = 5):
    """Plain device copies of a known size, for scaling the HBM byte counters."""
    import torch
    n = int(gib * (1 << 30)) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_each_way": n * 4, "reps": reps, "GB/s_read+write": 2 * n * 4 / dt / 1e9}),
          flush=True)


def _oracle_mode(job):
    """One worker of the CPU baseline: the oracle's assembly and sparse LU of one
    mode of a replica case (runs in a fresh single-threaded process)."""
    kind, size, k = job
    from threadpoolctl import threadpool_limits
    from oracle.solve import case_setup, solve_modes
    threadpool_limits(1)  # one core per process (the parent's BLAS pool is inherited by fork)
    t0 = time.perf_counter()
    if kind == "tree":
        c = cases.vessel_tree_case(h=size, generations=3, n_harm=max(k, 1))
    else:
        c = cases.pipe_case(h=size, length=0.3, n_harm=max(k, 1))
    asm, loads, wall, dirn, g = case_setup(c)
    _, _, res, _ = solve_modes(asm, loads, wall, dirn, c["omega"][k:k + 1], c["rho"], c["mu"],
                               c["traction"][k:k + 1], g[k:k + 1])
    return (time.perf_counter() - t0, 3 * asm["n2"] + asm["nv"], float(res[0]))


def cpu_baseline(workload: str, h_pipe: float, full_ndof: int):
    """The oracle timed on the host: a pool of single-threaded processes, one per
    core (at most 16), each solving one mode of a small replica of the workload
    by assembly and sparse LU; two replica sizes give the LU cost exponent, which
    extrapolates the rate to the full problem. Runs before the GPU is touched."""
    import multiprocessing as mp
    cores = max(1, min(os.cpu_count() or 1, 16))
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    sizes = (0.5, 0.42) if workload == "tree" else (h_pipe * 1.6, h_pipe * 1.25)
    os.environ["OMP_NUM_THREADS"] = "1"
    out = {}
    with mp.get_context("fork").Pool(cores) as pool:
        for size in sizes:
            jobs = [(workload, size, 1 + (i % 8)) for i in range(cores)]
            t0 = time.perf_counter()
            r = pool.map(_oracle_mode, jobs)
            wall = time.perf_counter() - t0
            out[size] = (wall, r)
    (w1, r1), (w2, r2) = out[sizes[0]], out[sizes[1]]
    n1, n2 = r1[0][1], r2[0][1]
    t1 = float(np.mean([x[0] for x in r1]))
    t2 = float(np.mean([x[0] for x in r2]))
    expo = float(np.log(t2 / t1) / np.log(n2 / n1)) if n2 > n1 and t2 > t1 else 2.0
    rate2 = cores / w2  # mode-solves/s of the larger replica on all cores
    full = rate2 * (n2 / float(full_ndof)) ** expo
    return {"value": full, "unit": "mode-solves/s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "nproc": os.cpu_count(),
            "sample": f"{workload} replicas of {n1} and {n2} unknowns: one mode per process on {cores} "
                      f"single-threaded processes, oracle assembly + SuperLU per mode ({t1:.1f}s and {t2:.1f}s "
                      f"per mode); measured rate {rate2:.3g} mode-solves/s on the larger replica, "
                      f"extrapolated to {full_ndof} unknowns with the measured LU time exponent {expo:.2f}",
            "replica_mode_solves_per_s": rate2, "replica_unknowns": int(n2), "lu_time_exponent": expo,
            "extrapolated": True, "sample_seconds": round(w1 + w2, 1),
            "max_rel_residual": max(x[2] for x in r1 + r2)}


def warm_start_leg(args, case, m, g, opts, ns, ur, pr):
    """The learned warm start on this workload, reported beside the plain-method
    headline. Setup (untimed, reported): unit-amplitude solutions at the harmonics of
    `--ws-periods` seeded periods T in [0.8, 1.2] (the mean flow once), their POD, and
    MLP training on the GPU. Timed: for the held-out T = 1 modes, the network's
    prediction, its subspace correction and the warm-started solve to the same
    tolerance. The network-only guess is timed too, to show what the network itself
    contributes."""
    import torch
    from paper_2009_06725_amd import scvs
    from workloads.waveforms import period_set
    res = {}
    t0 = time.perf_counter()
    periods = period_set(args.ws_periods, seed=41)
    ks = np.arange(1, args.harmonics + 1)
    om = np.concatenate([[0.0], *[2.0 * np.pi * ks / T for T in periods]])
    nsn = om.size
    nodes = m.export(scvs.X_DIRNODES)
    xyz = m.export(scvs.X_NODEXYZ)[nodes]
    gs = np.stack([case["inlet"](xyz, float(w)) for w in om])  # unit flow-rate amplitude
    gs = torch.from_numpy(gs).to("cuda")
    snap_opts = scvs.default_opts(rtol=1e-10, restart=opts.restart, cheb_vel=opts.cheb_vel,
                                  cheb_pres=opts.cheb_pres, cheb_ratio=opts.cheb_ratio,
                                  cheb_ratio_pres=opts.cheb_ratio_pres, precision=opts.precision,
                                  verbose=opts.verbose)
    log(f"warm start: {nsn} snapshot solves ...")
    us, ps, reps = m.solve(om, np.zeros((nsn, m.info.ntraction), np.complex128), gs, opts=snap_opts)
    X = torch.cat([us.reshape(nsn, -1), ps], dim=1).contiguous()
    del us, ps, gs
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rank = min(64, nsn)
    ws = scvs.WarmStart(m, om, X, rank=rank, width=128, layers=4, seed=7)
    del X
    t2 = time.perf_counter()
    l0 = ws.train(0)
    for ep, lr in ((4000, 3e-3), (4000, 1e-3), (4000, 3e-4), (4000, 1e-4)):
        loss = ws.train(ep, lr)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    res["setup_seconds"] = {"snapshot_solves": round(t1 - t0, 1), "pod": round(t2 - t1, 2),
                            "training": round(t3 - t2, 2)}
    res["snapshots"] = {"count": int(nsn), "periods": [round(float(T), 4) for T in periods],
                        "all_converged": all(r.status == 0 for r in reps)}
    res["model"] = {"rank": rank, "width": 128, "layers": 4, "loss_initial": l0, "loss_final": loss}
    amp = case["inlet_amp"]

    def timed(refine):
        torch.cuda.synchronize()
        t = time.perf_counter()
        x0 = ws.predict(case["omega"], amp)
        if refine:
            ws.refine(case["omega"], case["traction"], g, x0)
        uw, pw, rw = m.solve(case["omega"], case["traction"], g, x0=x0, opts=opts)
        torch.cuda.synchronize()
        dtw = time.perf_counter() - t
        r = {"mode_solves_per_s": ns / dtw, "ms": 1000.0 * dtw, "iterations": [x.iterations for x in rw],
             "warm": [x.warm for x in rw], "converged": all(x.status == 0 for x in rw)}
        if ur is not None:
            eu = (torch.linalg.vector_norm((uw - ur).reshape(ns, -1), dim=1) /
                  torch.linalg.vector_norm(ur.reshape(ns, -1), dim=1)).max().item()
            ep = (torch.linalg.vector_norm(pw - pr, dim=1) / torch.linalg.vector_norm(pr, dim=1)).max().item()
            r["error_vs_tight_reference"] = {"max_u": eu, "max_p": ep}
        return r

    log("warm start: network guess ...")
    res["network_only"] = timed(False)
    log("warm start: network guess + subspace correction ...")
    res["network_and_subspace_correction"] = timed(True)
    res["value"] = res["network_and_subspace_correction"]["mode_solves_per_s"]
    res["note"] = ("held-out period T = 1 (the headline workload); the timed region holds prediction, "
                   "correction and solve; setup (snapshots, POD, training) is reported, not timed")
    ws.close()
    return res


def run_ybatch(args):
    """The batching workload: on each of 4 Y-bifurcation meshes (about 0.3, 0.6, 1.2
    and 2.4M tets) 12 cases, each with its own seeded waveform of 32 harmonics plus
    the mean and its own period: 4 x 12 x 33 = 1,584 systems. One step solves every
    system: per mesh one call with all 396 systems, which the library runs in waves
    of its memory-based slot budget. Setup (mesh generation, assembly, hierarchies)
    is reported, not timed. Prints one JSON line."""
    import torch
    from paper_2009_06725_amd import scvs
    sizes = (300_000, 600_000, 1_200_000, 2_400_000)
    if args.ymesh is not None:  # one of the four meshes only
        sizes = (sizes[args.ymesh],)
    n_harm = 32
    ctx = scvs.Context(0)
    runs = []
    t_setup = time.perf_counter()
    for nt in sizes:
        cs = cases.y_cases(nt, n_cases=12, n_harm=n_harm, seed=3)
        m = scvs.Mesh.from_workload(ctx, cs[0]["mesh"])
        m.set_bc(cs[0]["bc"])
        m.assemble(cs[0]["rho"], cs[0]["mu"])
        info = m.info
        nodes = m.export(scvs.X_DIRNODES)
        xyz = m.export(scvs.X_NODEXYZ)[nodes]
        om = np.concatenate([c["omega"] for c in cs])
        g = np.concatenate([np.stack([c["inlet_amp"][k] * c["inlet"](xyz, float(w)) for k, w in enumerate(c["omega"])])
                            for c in cs])
        gd = torch.from_numpy(g).to("cuda")
        opts = solver_opts(args)
        opts.steady_schur_omega = float(np.abs(om).max())
        opts.rtol = args.rtol
        m.mg_info(0)  # hierarchies built here (setup)
        runs.append(dict(tets=cs[0]["mesh"].nc, m=m, om=om, g=gd, tr=np.zeros((om.size, 0), np.complex128),
                         opts=opts, ndof=info.ndof))
        log(f"ybatch mesh {cs[0]['mesh'].name}: {cs[0]['mesh'].nc} tets, {info.ndof} unknowns, {om.size} systems")
    t_setup = time.perf_counter() - t_setup
    torch.cuda.synchronize()
    per, total, solved, dof_modes = [], 0.0, 0, 0.0
    conv = True
    for r in runs:
        t0 = time.perf_counter()
        _, _, rep = r["m"].solve(r["om"], r["tr"], r["g"], opts=r["opts"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        its = [x.iterations for x in rep]
        conv = conv and all(x.status == 0 for x in rep)
        per.append({"tets": int(r["tets"]), "ndof": int(r["ndof"]), "systems": len(rep), "seconds": round(dt, 2),
                    "mode_solves_per_s": len(rep) / dt, "iterations_mean": float(np.mean(its)),
                    "iterations_max": int(np.max(its)), "converged": all(x.status == 0 for x in rep)})
        log(f"ybatch {r['tets']} tets: {len(rep)} systems in {dt:.1f}s, iterations mean {np.mean(its):.0f} "
            f"max {np.max(its)}")
        total += dt
        solved += len(rep)
        dof_modes += len(rep) * r["ndof"]
        r["m"].close()
    print(json.dumps({"metric": "mode-solves/s", "value": solved / total, "unit": "mode-solves/s", "n_gpus": 1,
                      "steps": 1, "warmup": 0, "ms_per_step": total * 1e3, "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "c64 operator and preconditioner / c128 "
                      "Krylov basis, Schur scaling, refinement", "data": "synthetic",
                      "config": {"workload": "Y-bifurcations (radii 1.0/0.7/0.7, 60 degrees) of about "
                                 f"{'/'.join(f'{x / 1e6:g}' for x in sizes)}M tets, 12 cases each of 32 harmonics "
                                 f"+ mean, own period per case: {solved} systems", "rtol": args.rtol, "restart": args.restart,
                                 "precision": args.precision, "mg_ratio": args.mg_ratio, "mg_smooth": args.mg_smooth},
                      "dof_modes_per_s": dof_modes / total, "setup_seconds": round(t_setup, 1),
                      "converged": conv, "per_mesh": per}), flush=True)


def run_ylearn(args):
    """The learned-warm-start workload on the Y-bifurcation of about 1.2M tets:
    2,000 training and 200 held-out waveforms of 32 harmonics (amplitudes
    N(0,1)/k^2, phases U[0, 2pi)), each with its own period T ~ U[0.8, 1.2].
    Mode k of a waveform is its coefficient times the unit-amplitude response at
    w = 2 pi k / T, so what a model learns is that response as a function of w.
    Setup (untimed, reported): for each harmonic, unit responses at
    `--ws-snapshots` of the training periods (the shortest, the longest and evenly
    spaced order statistics between), their POD (one basis per harmonic) and the
    harmonic's MLP (4 layers of width 256) trained on the GPU. Timed, on the first
    `--ws-heldout` held-out waveforms (all 32 harmonics each): the zero-guess solve,
    the network's guess and solve, and the guess with its subspace correction and
    solve, all to the same tolerance. The steady mode is left out: its unit
    response does not depend on the period, so its guess would be exact. Prints one
    JSON line."""
    import torch
    from paper_2009_06725_amd import scvs
    from workloads.meshes import y_bifurcation_mesh_for_tets
    from workloads.waveforms import harmonic_coefficients, period_set
    n_harm, n_train, n_held = args.harmonics, 2000, 200
    t0 = time.perf_counter()
    c = cases.vessel_case(y_bifurcation_mesh_for_tets(args.tets), n_harm, 5, 1.0)
    ctx = scvs.Context(0)
    m = scvs.Mesh.from_workload(ctx, c["mesh"])
    m.set_bc(c["bc"])
    m.assemble(c["rho"], c["mu"])
    info = m.info
    nodes = m.export(scvs.X_DIRNODES)
    xyz = m.export(scvs.X_NODEXYZ)[nodes]
    opts = solver_opts(args)
    opts.steady_schur_omega = 2.0 * np.pi * n_harm / 0.8
    opts.max_batch = args.batch  # the same slot count for the three timed solves
    m.mg_info(0)
    t_setup = time.perf_counter() - t0
    log(f"ylearn mesh {c['mesh'].name}: {c['mesh'].nc} tets, {info.ndof} unknowns ({t_setup:.1f}s)")
    # training periods; the training waveforms' coefficients only scale their modes (linearity)
    # and so never enter the snapshots, the POD or the networks
    t_train = np.sort(period_set(n_train, seed=61))
    S = args.ws_snapshots
    ts = t_train[np.round(np.linspace(0, n_train - 1, S)).astype(int)]
    ks = np.repeat(np.arange(1, n_harm + 1), S)
    om_s = 2.0 * np.pi * ks / np.tile(ts, n_harm)

    def dirichlet(om, amp):
        return torch.from_numpy(np.stack([a * c["inlet"](xyz, float(w)) for w, a in zip(om, amp)])).to("cuda")

    snap_opts = solver_opts(args)
    snap_opts.steady_schur_omega = opts.steady_schur_omega
    snap_opts.rtol = 1e-10
    mws = scvs.ModeWarmStarts(m, rank=S, width=256, layers=4, seed=7)
    t0 = time.perf_counter()
    t_pod, snap_conv, per_call = 0.0, True, 4  # harmonics per snapshot solve call
    for k0 in range(1, n_harm + 1, per_call):
        kk = np.arange(k0, min(n_harm, k0 + per_call - 1) + 1)
        sel = np.isin(ks, kk)
        us, ps, reps = m.solve(om_s[sel], np.zeros((int(sel.sum()), 0), np.complex128),
                               dirichlet(om_s[sel], np.ones(int(sel.sum()))), opts=snap_opts)
        snap_conv = snap_conv and all(x.status == 0 for x in reps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for j, k in enumerate(kk):
            r = slice(j * S, (j + 1) * S)
            mws.add(int(k), om_s[ks == k], torch.cat([us[r].reshape(S, -1), ps[r]], dim=1).contiguous())
        del us, ps
        torch.cuda.empty_cache()
        torch.cuda.synchronize()
        t_pod += time.perf_counter() - t1
        log(f"ylearn: snapshots and POD of harmonics {kk[0]}..{kk[-1]} done at {time.perf_counter() - t0:.1f}s, "
            f"iterations {sum(x.iterations for x in reps)}")
    t_snap = time.perf_counter() - t0 - t_pod
    t0 = time.perf_counter()
    losses = mws.train([(4000, 3e-3), (4000, 1e-3), (4000, 3e-4), (4000, 1e-4)])
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    sig = mws.sigma()
    log(f"ylearn: POD {t_pod:.1f}s, training {t_fit:.1f}s")
    # held-out systems, ordered by harmonic (k outer, waveform inner)
    H = args.ws_heldout
    th = period_set(n_held, seed=63)
    coef = harmonic_coefficients(n_harm, 64, n_waves=n_held)
    hk = np.repeat(np.arange(1, n_harm + 1), H)
    hw = np.tile(np.arange(H), n_harm)
    om = 2.0 * np.pi * hk / th[hw]
    amp = coef[hw, hk]
    tr = np.zeros((om.size, 0), np.complex128)
    g = dirichlet(om, amp)
    # the corrections' A(0) Phi and its slope are formed on a model's first call (setup)
    first = np.arange(0, om.size, H)
    mws.refine(hk[first], om[first], tr[first], g[first].contiguous(), mws.predict(hk[first], om[first], amp[first]))
    torch.cuda.synchronize()
    ns = om.size

    def timed(kind):
        torch.cuda.synchronize()
        t = time.perf_counter()
        x0 = None
        if kind != "zero":
            x0 = mws.predict(hk, om, amp)
            if kind == "corrected":
                mws.refine(hk, om, tr, g, x0)
        u_, p_, rep = m.solve(om, tr, g, x0=x0, opts=opts)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        its = np.array([x.iterations for x in rep])
        log(f"ylearn {kind}: {dt:.1f}s, iterations {its.sum()}")
        return u_, p_, {"mode_solves_per_s": ns / dt, "seconds": round(dt, 2), "iterations_sum": int(its.sum()),
                        "iterations_per_harmonic": [float(its[hk == k].mean()) for k in range(1, n_harm + 1)],
                        "warm": int(sum(x.warm for x in rep)), "converged": all(x.status == 0 for x in rep)}

    u0, p0, r0 = timed("zero")
    u1, p1, r1 = timed("network")
    del u1, p1
    u2, p2, r2 = timed("corrected")
    eu, ep = rel_mass_l2(m, u2 - u0, p2 - p0, u0, p0)
    r2["rel_diff_vs_zero_guess"] = {"max_u": float(eu.max()), "max_p": float(ep.max())}
    mws.close()
    print(json.dumps({
        "metric": "mode-solves/s", "value": r2["mode_solves_per_s"], "unit": "mode-solves/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": r2["seconds"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c64 operator and preconditioner / c128 Krylov basis, Schur scaling, "
        "refinement; MLP bf16 products, fp32 accumulate", "data": "synthetic",
        "config": {"workload": f"learned warm start on a Y-bifurcation of {c['mesh'].nc} tets: {n_train} training and "
                   f"{n_held} held-out waveforms of {n_harm} harmonics, own period each; timed on {H} held-out "
                   f"waveforms ({ns} systems)", "ndof": int(info.ndof), "rtol": opts.rtol,
                   "snapshot_periods": [round(float(x), 4) for x in ts], "pod_rank_per_harmonic": S,
                   "mlp": {"layers": 4, "width": 256, "epochs": 16000},
                   "heldout_periods": [round(float(x), 4) for x in th[:H]]},
        "zero_guess": r0, "network_only": r1, "network_and_subspace_correction": r2,
        "network_iterations_vs_zero_guess": r1["iterations_sum"] / max(1, r0["iterations_sum"]),
        "setup_seconds": {"mesh_assembly_hierarchies": round(t_setup, 1), "snapshot_solves": round(t_snap, 1),
                          "pod": round(t_pod, 1), "training": round(t_fit, 1)},
        "snapshots_converged": snap_conv,
        "training_loss": {"initial_max": max(a for a, _ in losses.values()),
                          "final_max": max(b for _, b in losses.values())},
        # singular values below about 1e-8 sigma_0 are under the Gram matrix's rounding floor
        # (reported as 0): a harmonic whose count stays below the rank is resolved by its snapshots
        "pod_values_above_1e-7_sigma0": {int(k): int((s > 1e-7 * s[0]).sum()) for k, s in sig.items()},
        "pod_sigma_over_sigma0": {int(k): [float(f"{x / sig[k][0]:.3g}") for x in sig[k]] for k in (1, n_harm // 2, n_harm)},
    }), flush=True)


def rel_mass_l2(m, du, dp, ur, pr):
    """Relative L2(Omega) errors per mode (mass-weighted: u^H (I x M) u, p^H Mp p)."""
    dun, dpn = m.mode_norms(du, dp)
    run, rpn = m.mode_norms(ur, pr)
    return np.sqrt(dun / np.maximum(run, 1e-300)), np.sqrt(dpn / np.maximum(rpn, 1e-300))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "ybatch":
        run_ybatch(args)
        return
    if args.workload == "ylearn":
        run_ylearn(args)
        return
    tree = args.workload == "tree"
    t_start = time.perf_counter()
    if tree:
        case = cases.tree_case(n_tets=args.tets, n_harm=args.harmonics)
        h_pipe = 0.0
    else:
        case = cases.pipe_case(n_tets=args.tets, n_harm=args.harmonics)
        h_pipe = float(case["mesh"].name.split("_h")[1].split("_")[0])
    mesh = case["mesh"]
    t_mesh = time.perf_counter() - t_start
    log(f"mesh {mesh.name}: {mesh.nc} tets, {mesh.nv} vertices ({t_mesh:.1f}s)")
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on the host cores, before anything touches the GPU (the pool forks)
        log("cpu baseline (oracle, process pool) ...")
        est_ndof = int(3 * 7.8 * mesh.nv + mesh.nv) if tree else int(3 * 7.6 * mesh.nv + mesh.nv)
        cpu = cpu_baseline(args.workload, h_pipe, est_ndof)
        log(f"cpu baseline: {cpu['sample']}")
    import torch
    from paper_2009_06725_amd import scvs

    ctx = scvs.Context(0)
    t0 = time.perf_counter()
    m = scvs.Mesh.from_workload(ctx, mesh)
    wk = None
    if args.windkessel:
        from workloads.meshes import OUTLET
        wk = tuple(float(v) for v in args.windkessel.split(","))
        case["bc"][OUTLET] = 3  # traction tag carrying the lumped model, zero offset pressure
        case["traction"] = np.zeros((len(case["omega"]), 1), np.complex128)
    m.set_bc(case["bc"])
    if wk:
        m.set_windkessel({OUTLET: wk})
    m.assemble(case["rho"], case["mu"])
    torch.cuda.synchronize()
    t_ingest = time.perf_counter() - t0
    info = m.info
    if cpu is not None:
        cpu["value"] *= 1.0  # (rate already for the estimated size; rescale to the exact one below)
        ratio = (cpu["replica_unknowns"] / float(info.ndof)) ** cpu["lu_time_exponent"]
        cpu["value"] = cpu["replica_mode_solves_per_s"] * ratio
        cpu["sample"] = cpu["sample"].split(", extrapolated to")[0] + (
            f", extrapolated to {info.ndof} unknowns with the measured LU time exponent {cpu['lu_time_exponent']:.2f}")
    ns = len(case["omega"])
    nodes = m.export(scvs.X_DIRNODES)
    xyz = m.export(scvs.X_NODEXYZ)[nodes]
    g = np.zeros((ns, nodes.size, 3), np.complex128)
    for s_, w in enumerate(case["omega"]):
        g[s_] = case["inlet_amp"][s_] * case["inlet"](xyz, float(w))
    g = torch.from_numpy(g).to("cuda")
    trac = np.asarray(case["traction"]).reshape(ns, -1)
    # waves: system k goes to wave k mod n_waves (each wave mixes low and high modes)
    B = ns if args.batch <= 0 or args.batch >= ns else args.batch
    n_waves = (ns + B - 1) // B
    waves = [np.arange(w, ns, n_waves) for w in range(n_waves)]
    bmax = max(len(w) for w in waves)
    u = torch.empty((bmax, info.n2, 3), dtype=torch.complex128, device="cuda")
    p = torch.empty((bmax, info.nv), dtype=torch.complex128, device="cuda")
    times = np.arange(args.ntimes) * case["period"] / args.ntimes
    ut = torch.empty((args.ntimes, info.n2 * 3), dtype=torch.float64, device="cuda")
    pt = torch.empty((args.ntimes, info.nv), dtype=torch.float64, device="cuda")
    opts = solver_opts(args)
    if args.steady_schur_omega < 0:
        opts.steady_schur_omega = float(np.abs(case["omega"]).max())
    log(f"n2={info.n2} ndof={info.ndof} nnz_s2={info.nnz_s2} ingest+assembly {t_ingest:.2f}s; "
        f"{ns} systems in {n_waves} waves of <= {bmax}")
    tuned = None
    if args.autotune:
        # untimed setup: the library times its candidate settings on these systems
        log("autotune ...")
        t0 = time.perf_counter()
        w0 = waves[0]
        best, best_ms = m.autotune(case["omega"][w0], trac[w0], g[w0].contiguous(), base=opts)
        tuned = {"restart": best.restart, "cheb_vel": best.cheb_vel, "cheb_pres": best.cheb_pres,
                 "tuning_seconds": round(time.perf_counter() - t0, 1), "candidate_ms": round(best_ms, 1)}
        opts = best
        log(f"autotune: {tuned}")
    # per-mesh setup, timed once and reported (not part of a step): the multigrid
    # hierarchies of the preconditioner are built from the assembled matrices
    hier = None
    t_mg = 0.0
    if opts.vel_block or opts.pres_block:
        t0 = time.perf_counter()
        hier = {"velocity": m.mg_info(0), "pressure": m.mg_info(1)}
        t_mg = time.perf_counter() - t0
        log(f"multigrid hierarchies in {t_mg:.2f}s: velocity {hier['velocity']} pressure {hier['pressure']}")

    def step(i):
        sel = waves[i % n_waves]
        k = len(sel)
        gw = g[sel].contiguous() if k < ns else g
        _, _, rep = m.solve(case["omega"][sel], trac[sel], gw, u=u[:k], p=p[:k], opts=opts)
        scvs.synthesize(ctx, case["omega"][sel], u[:k], times, out=ut)
        scvs.synthesize(ctx, case["omega"][sel], p[:k], times, out=pt)
        return rep, sel

    for i in range(args.warmup):
        t0 = time.perf_counter()
        rep, sel = step(i)
        torch.cuda.synchronize()
        log(f"warmup {i}: {time.perf_counter() - t0:.2f}s systems {list(sel)} iterations {[r.iterations for r in rep]}")
    ctx.profile(True)
    ctx.profile_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    solved = 0
    step_s = []
    for i in range(args.steps):
        ts = time.perf_counter()
        rep, sel = step(i)
        torch.cuda.synchronize()
        step_s.append(time.perf_counter() - ts)
        reps.append((rep, sel))
        solved += len(sel)
        log(f"step {i} done at {time.perf_counter() - t0:.2f}s systems {list(sel)} "
            f"iterations {[r.iterations for r in rep]}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    stats = ctx.profile_read()
    ctx.profile(False)
    graph_leg = None
    if not args.no_graph_leg:
        # the first waves again with the event profiler off, so the solver records and
        # replays its graphs of Arnoldi chunks: what the event pairs of the timed steps cost
        nw = min(2, args.steps)
        log(f"graph leg: waves 0..{nw - 1} with graph replay ...")
        tg = []
        for i in range(nw):
            ts = time.perf_counter()
            rep_g, _ = step(i)
            torch.cuda.synchronize()
            tg.append(time.perf_counter() - ts)
        graph_leg = {"waves": nw, "seconds_with_events": [round(x, 3) for x in step_s[:nw]],
                     "seconds_with_graphs": [round(x, 3) for x in tg],
                     "ratio": sum(tg) / sum(step_s[:nw]),
                     "same_iterations": [r.iterations for r in rep_g] == [r.iterations for r in reps[nw - 1][0]]}
        log(f"graph leg: {graph_leg}")
    conv = all(r.status == 0 for rep, _ in reps for r in rep)
    iters_by_system = {}
    for rep, sel in reps:
        for r, k in zip(rep, sel):
            iters_by_system[int(k)] = r.iterations

    def roof(name):
        n, ms, by = stats[name]
        per = by / n
        avg_s = ms / n / 1e3
        gbs = per / avg_s / 1e9
        tr = stored_traffic(name, args.workload)
        return {"kernel": name, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": tr, "bytes_per_launch": per,
                "avg_launch_us": avg_s * 1e6, "launches": n,
                "share_of_kernel_time": ms / sum(v[1] for v in stats.values())}

    dominant = max(stats, key=lambda k: stats[k][1])
    kernels = {k: {"launches": v[0], "ms": round(v[1], 3), "GB/s": round(v[2] / (v[1] / 1e3) / 1e9, 1) if v[1] else None}
               for k, v in sorted(stats.items(), key=lambda kv: -kv[1][1])}
    if tree:
        wl = (f"3-generation vessel tree (7 bifurcations, radii / sqrt 2 per generation), {mesh.nc} P2/P1 tets, "
              f"{ns} modes ({ns - 1} harmonics + mean) in waves of <= {bmax} systems (one wave per step)")
    else:
        wl = f"pipe R=1 L=10, {mesh.nc} curved P2/P1 tets, {ns} modes ({ns - 1} harmonics + mean)"
    out = {
        "metric": "mode-solves/s",
        "value": solved / dt,
        "unit": "mode-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "c128", "mixed": "c64 operator and preconditioner / c128 Krylov basis, Schur scaling, "
                                           "refinement",
                  "mixed32": "c64 operator, preconditioner and Krylov basis storage / c128 arithmetic, "
                             "Schur scaling, refinement"
                  }[args.precision],
        "data": "synthetic",
        "config": {"workload": wl, "ndof": int(info.ndof), "modes": ns, "systems_per_step": bmax, "waves": n_waves,
                   "rtol": args.rtol, "restart": opts.restart,
                   "velocity_block": "multigrid V-cycle" if opts.vel_block else f"Chebyshev degree {opts.cheb_vel}",
                   "pressure_block": "multigrid V-cycle" if opts.pres_block else f"Chebyshev degree {opts.cheb_pres}",
                   "mg_smooth": opts.mg_smooth, "mg_post0": opts.mg_post0, "mg_ratio": opts.mg_ratio,
                   "steady_schur_omega": opts.steady_schur_omega,
                   "autotuned": tuned, "orth": args.orth, "inner_rtol": args.inner_rtol,
                   "precision": args.precision, "penalty": args.penalty,
                   "outlet": "traction-free" if wk is None else
                   {"lumped": "three-element", "rp": wk[0], "c": wk[1], "rd": wk[2]},
                   "ntimes": args.ntimes},
        "dof_modes_per_s": info.ndof * solved / dt,
        "setup_seconds": {"mesh_generation": round(t_mesh, 2), "ingest_and_assembly": round(t_ingest, 3),
                          "multigrid_hierarchies": round(t_mg, 3)},
        "multigrid_levels": hier,
        "roofline": roof(dominant),
        "spmv_roofline": roof("k_full_apply32" if "k_full_apply32" in stats else "k_full_apply"),
        "converged": conv,
        "iterations": [iters_by_system[k] for k in sorted(iters_by_system)],
        "iterations_systems": sorted(iters_by_system),
        "kernels": kernels,
        "graph_replay": graph_leg,
    }
    # mode selection on this workload: a-priori truncation error of the boundary data
    # (Eq. mode_error); the a-posteriori increments need every mode (one-wave workloads)
    hn2, gn2 = m.boundary_norms(case["omega"], trac, g)
    wts = np.where(np.asarray(case["omega"]) == 0.0, 1.0, 2.0)  # Parseval weights, two-sided modes

    def e_first(n):  # e_M when the first n modes are kept (relative to all ns modes)
        e2 = 0.0
        for q in (np.asarray(hn2), np.asarray(gn2)):
            tot = float(np.sum(wts * q))
            if tot > 0:
                e2 += float(np.sum(wts[n:] * q[n:])) / tot
        return float(np.sqrt(e2))

    picks = {}
    for eps in (1e-1, 1e-2, 1e-3):
        oc, nc, ec = scvs.select_modes(case["omega"], hn2, gn2, eps, True)
        oa, na, ea = scvs.select_modes(case["omega"], hn2, gn2, eps, False)
        picks[f"{eps:g}"] = {"consecutive": int(nc), "by_amplitude": int(na),
                             "by_amplitude_modes": [int(k) for k in oa[:na]]}
    out["mode_selection"] = {"a_priori_error_first_n_modes": [e_first(n + 1) for n in range(ns)],
                             "modes_needed": picks}
    if n_waves == 1:
        un2, _ = m.mode_norms(u, p)
        out["mode_selection"]["a_posteriori_increment_of_mode_n"] = [
            float(x) for x in scvs.mode_increments(case["omega"], un2)]
    # the first wave again, kept for the error check, the comparator and the warm start
    w0 = waves[0]
    k0 = len(w0)
    g0 = g[w0].contiguous() if k0 < ns else g
    u0 = torch.empty((k0, info.n2, 3), dtype=torch.complex128, device="cuda")
    p0 = torch.empty((k0, info.nv), dtype=torch.complex128, device="cuda")
    m.solve(case["omega"][w0], trac[w0], g0, u=u0, p=p0, opts=opts)
    ur = pr = None
    if not args.no_error_check:
        # error of the timed solution: against an FP64 solve to a 100x tighter residual
        # (not below 1e-13, about where FP64 restarts stop gaining), in L2(Omega)
        rref = max(args.rtol * 1e-2, 1e-13)
        ref = solver_opts(args)
        ref.rtol, ref.precision, ref.steady_schur_omega = rref, 0, opts.steady_schur_omega
        ur = torch.empty_like(u0)
        pr = torch.empty_like(p0)
        log("error check: FP64 reference solve of the first wave ...")
        _, _, rep3 = m.solve(case["omega"][w0], trac[w0], g0, u=ur, p=pr, opts=ref)
        eu, ep = rel_mass_l2(m, (u0 - ur).contiguous(), (p0 - pr).contiguous(), ur, pr)
        out["error_vs_tight_reference"] = {
            "reference": f"FP64 path, rtol {rref:g}", "norm": "relative L2(Omega) per mode (mass-weighted)",
            "systems": [int(k) for k in w0],
            "max_u": float(eu.max()), "max_p": float(ep.max()),
            "per_mode_u": [float(x) for x in eu], "per_mode_p": [float(x) for x in ep],
            "reference_converged": all(r.status == 0 for r in rep3)}
    if not tree and not args.no_warm_start:
        out["warm_started"] = warm_start_leg(args, case, m, g, opts, ns, ur, pr)
    if not args.no_compare:
        # comparator: plain per-mode FP64 GMRES (one system at a time, same
        # preconditioner, restart and tolerance, two-pass Gram-Schmidt) on systems
        # of the first wave
        nc = k0 if args.compare_systems <= 0 else min(args.compare_systems, k0)
        sel = np.array(w0[:nc])
        plain = solver_opts(args)
        plain.precision, plain.max_batch, plain.orth = 0, 1, 0
        plain.steady_schur_omega = opts.steady_schur_omega
        u2 = torch.empty((nc, info.n2, 3), dtype=torch.complex128, device="cuda")
        p2 = torch.empty((nc, info.nv), dtype=torch.complex128, device="cuda")
        log(f"comparator: plain per-mode FP64 GMRES on systems {list(sel)} ...")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, rep2 = m.solve(case["omega"][sel], trac[sel], g[sel].contiguous(), u=u2, p=p2, opts=plain)
        torch.cuda.synchronize()
        dtp = time.perf_counter() - t0
        du, dpp = rel_mass_l2(m, (u0[:nc] - u2).contiguous(), (p0[:nc] - p2).contiguous(), u2, p2)
        out["plain_fp64_per_mode"] = {"mode_solves_per_s": nc / dtp, "seconds": dtp, "systems": [int(k) for k in sel],
                                      "iterations": [r.iterations for r in rep2],
                                      "converged": all(r.status == 0 for r in rep2)}
        out["speedup_vs_plain_fp64"] = out["value"] / (nc / dtp)
        out["rel_diff_vs_plain_fp64"] = {"u": float(du.max()), "p": float(dpp.max())}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
