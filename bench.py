"""Benchmark: Poisson solves/s and GDOF/s to a 1e-10 relative residual on one MI355X.

A step is one full solve (x = 0 -> ||b - A x|| <= 1e-10 ||b||) of the synthetic wave-tank
workload (1024 x 16 elements, P = 8, 1,056,897 nodes), inputs resident in HBM.  The timed path
(``value``) is the mixed-precision p-multigrid with the learned element-local smoothing stage:
FP32 inner V-cycle (geometric factors stored in BF16; --prec f32 stores them in FP32, --prec col
forms them in registers from FP64 column records), BF16-MFMA network stage
on the fine level, FP64 outer flexible CG.  Its network is trained first, on the GPU, by the
library's own kernels from pairs that the plain p-multigrid generates (outside the timed region;
the training time is reported).  The stage's three placements (after pre-smoothing, before
post-smoothing, both) are timed and the fastest is the headline; beside it the same solver
without the stage (with the break-even cost of the stage) and with each way of holding the inner
factors, the plain FP64 p-multigrid, per-cycle
residual reduction in defect-correction (PDC) mode with and without the stage, the plain
smoother's verdict on the stage (residual reduction per cycle and per unit of time), iterations and
times on 20 unseen test surfaces (the oracle solves three of them on the host cores, in child
processes, and checks the GPU's pressure), the roofline of the dominant kernel (the fused
operator + smoother step; HBM-resident timing with rotated buffers, the cache-resident figure
and a plain device copy of the same bytes beside it), the whole solve's algorithmic bytes over its time, and the CPU oracle timed on a
bounded sample of the same workload.

A 3D time series (64 x 64 x 8, P = 6, moving surface, warm starts, frozen preconditioner) is
reported beside it (--c5-steps, 0 to skip), the stage loop around the solve on the same tank
(five-stage low-storage Runge-Kutta steps of the linear free-surface model, preconditioner frozen
or built from still water; --stage-steps), the mixed-precision error table of the 2048 x 16
tank at tolerances 1e-6, 1e-8, 1e-10 with the oracle's residual of every row (--no-c3 to skip),
the same solve with the paper's additive Schwarz smoother in place of Chebyshev (--no-schwarz),
and the paper's multigrid iteration table and scaling sweeps rerun on tank meshes with two
element layers (--no-context).

Usage: python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--workload c4] [--prec bf16]
                       [--no-learned] [--surfaces 20] [--oracle-surfaces 3] [--c5-steps 20]
                       [--no-cpu] [--no-fp64]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Poisson solves/s + GDOF/s to 1e-10 residual: FP32+learned p-MG vs plain FP64"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name, index=0):
    import workloads as W
    if name == "c2":
        return W.c2()
    if name == "c3":
        return W.c3()
    if name == "c4":
        return W.c4(index)
    raise SystemExit(f"unknown workload {name}")


def describe(wl, prec, learned, mode=0):
    where = {1: "fine level after pre-smoothing (step folded into the transfers)",
             2: "fine level before post-smoothing",
             3: "fine level after pre-smoothing and before post-smoothing"}.get(mode, "")
    return {"workload": f"{wl.name}: 2D sigma-mapped wave tank {wl.Nx}x{wl.Nz} elements, P={wl.P}, "
                        f"levels {'-'.join(map(str, wl.orders))}, Chebyshev({wl.cheb_degree}) on "
                        f"[{wl.cheb_lo}, {wl.cheb_hi}] x lambda_hat, "
                        f"trapezoidal bar 0.4-0.1-0.4 m, surface seed {wl.surface_seed}, "
                        f"rhs seed {wl.rhs_seed}",
            "n_global": wl.n_global, "elements": wl.n_elements, "order": wl.P,
            "inner": {"bf16": "fp32 compute, geometric factors bf16",
                      "f32": "fp32 compute, geometric factors fp32",
                      "col": "fp32 compute, geometric factors formed in registers from fp64 "
                             "column records (d, h_x, d_x per column node)"}[prec],
            "outer": "fp64 flexible CG, fp64 operator and inner products, fp64 P=1 coarse solve",
            "learned_stage": ("element-local MLP 405-128-128-81 (GELU), bf16 MFMA operands, fp32 "
                              f"accumulate; {where} (the fastest of the three placements); "
                              "energy-judged step") if learned else False,
            "tol": 1e-10}


def median_solve(s, rhs, tol, reps=7):
    """Median time of reps solves after one untimed solve (for the small context runs, whose
    sub-millisecond times a single host hiccup would dominate)."""
    import statistics

    import torch
    x = torch.zeros_like(rhs)
    x.zero_()
    _, info, _ = s.solve(rhs, x=x, tol=tol)
    ts = []
    for _ in range(reps):
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, _ = s.solve(rhs, x=x, tol=tol)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), info, x


def time_solves(s, rhs, steps, warmup, tol):
    import torch
    x = torch.zeros_like(rhs)
    info = None
    for _ in range(warmup):
        x.zero_()
        _, info, _ = s.solve(rhs, x=x, tol=tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x.zero_()
        _, info, _ = s.solve(rhs, x=x, tol=tol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) / steps, info, x


def train_network(args, wl, prec):
    """Harvest pairs with the plain p-multigrid and train the network on the GPU
    (sem_learned_harvest, sem_learned_train on a context of the benchmark's fine level)."""
    import struct

    from paper_2411_14977_amd import cases, learned
    t0 = time.perf_counter()
    X, T = learned.harvest(n_surfaces=args.train_surfaces)
    t1 = time.perf_counter()
    sv = cases.make_solver(wl, prec=prec)
    blob = learned.train_into(sv.ctx, X, T, epochs=args.epochs)
    sv.close()
    t2 = time.perf_counter()
    train_loss, val_loss = struct.unpack_from("<2f", blob, 40)
    rec = {"pairs": int(X.shape[0]), "surfaces": args.train_surfaces, "epochs": args.epochs,
           "harvest_s": t1 - t0, "train_s": t2 - t1,
           "final_train_batch_loss": train_loss, "final_val_loss": val_loss,
           "recipe": "64x16-element windows of the tank (dx = 0.025 m), seeded offsets and "
                     "surfaces (seeds 5000+), smooth and white-noise sources, 8 defect-correction "
                     "cycles each, plus random residuals; targets = element-block solves; "
                     "Adam, cosine lr 2e-3, batch 512"}
    log(f"[bench] trained on {rec['pairs']} pairs: harvest {rec['harvest_s']:.1f} s, "
        f"train {rec['train_s']:.1f} s, val loss {rec['final_val_loss']:.4f}")
    return blob, rec


def pdc_rates(wl, prec, blob, cycles, mode):
    """Per-cycle residual reduction rho = (||r_k|| / ||r_0||)^(1/k) of defect correction with the
    V-cycle, with and without the learned stage."""
    from paper_2411_14977_amd import cases
    out = {}
    for tag, m in (("plain", 0), ("learned", mode)):
        if m and blob is None:
            continue
        s = cases.make_solver(wl, prec=prec, outer="pdc", maxit=cycles)
        if m:
            s.learned_load(blob, m)
        rhs = cases.make_rhs(wl, s)
        try:
            _, info, _ = s.solve(rhs, tol=1e-30, check=False)
        finally:
            s.close()
        h = info.history()
        k = len(h) - 1
        out[tag] = {"cycles": k, "rho": (h[-1] / h[0]) ** (1.0 / k) if k > 0 and h[0] > 0 else None,
                    "skips": info.learned_skips}
    return out


def unseen_surfaces(args, blob, n, mode, keep=()):
    """Iterations and times to 1e-10 on test surfaces 1..n (surface seeds 1001.., rhs seeds
    2001.., never trained on), plain mixed precision and with the stage; the learned solutions of
    the indices in keep are returned (host arrays) for the oracle's check."""
    from paper_2411_14977_amd import cases
    rows, kept = [], {}
    for i in range(1, n + 1):
        wl = workload(args.workload, i)
        s = cases.make_solver(wl, prec=args.prec)
        rhs = cases.make_rhs(wl, s)
        r = {"surface_seed": wl.surface_seed, "rhs_seed": wl.rhs_seed}
        for tag, m in (("plain", 0), ("learned", mode)):
            if m:
                s.learned_load(blob, m)
            t, info, x = time_solves(s, rhs, 1, 1, 1e-10)
            r[tag] = {"iters": info.iters, "ms": t * 1e3, "skips": info.learned_skips,
                      "rel_res": info.rel_res}
            if m and i in keep:
                kept[i] = x.cpu().numpy()
        s.close()
        rows.append(r)
        log(f"[bench] surface {wl.surface_seed}: plain {r['plain']['iters']} it "
            f"{r['plain']['ms']:.2f} ms, learned {r['learned']['iters']} it {r['learned']['ms']:.2f} ms")
    return rows, kept


def start_oracle_parity(args, solutions):
    """One child process per kept surface: the oracle's own FP64 FPCG + p-multigrid solve to
    1e-12 on that surface's mesh and right-hand side, compared with the GPU's learned solution
    (runs on the host cores while the GPU parts of the benchmark continue)."""
    import subprocess
    import tempfile

    import numpy as np
    procs = []
    for i, x in sorted(solutions.items()):
        fd, path = tempfile.mkstemp(suffix=".npy", prefix="sem_gpu_x_")
        os.close(fd)
        np.save(path, x)
        cmd = [sys.executable, os.path.abspath(__file__), "--oracle-worker", args.workload, str(i),
               path]
        procs.append((i, path, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                                text=True)))
    return procs


def finish_oracle_parity(procs):
    out = []
    for i, path, pr in procs:
        so, se = pr.communicate()
        try:
            os.remove(path)
        except OSError:
            pass
        if pr.returncode != 0:
            log(f"[bench] oracle parity worker {i} failed: {se[-500:]}")
            out.append({"test_index": i, "error": se[-300:]})
            continue
        out.append(json.loads(so.strip().splitlines()[-1]))
    return out


def oracle_worker(name, index, path):
    """Child process: the oracle's solve of test surface `index` and the GPU solution's error."""
    import numpy as np

    from oracle import pmg
    from tests import oracle_cases as oc
    wl = workload(name, index)
    t0 = time.perf_counter()
    H = oc.hierarchy(wl)
    pmg.estimate_lambdas(H)
    L0 = H.levels[0]
    b = oc.rhs(wl, L0.mesh)
    xo, it, hist = pmg.fpcg(L0.A, b, np.zeros(L0.N), H.vcycle, 1e-12)
    t1 = time.perf_counter()
    xg = np.load(path)
    err = float(np.linalg.norm(xg - xo) / np.linalg.norm(xo))
    res = float(np.linalg.norm(b - L0.A @ xg) / np.linalg.norm(b))
    print(json.dumps({"test_index": index, "surface_seed": wl.surface_seed, "oracle_iters": it,
                      "oracle_rel_res": hist[-1], "oracle_s": t1 - t0,
                      "gpu_rel_error_vs_oracle": err, "gpu_oracle_rel_res": res}), flush=True)


def c5_learned_network(args):
    """Network of the 3D stage: pairs from 4 x 4 x 8 windows of the 3D tank at its element size
    (sem_learned_harvest on FP64 windows), trained on the GPU; returns (blob, record)."""
    import struct

    from paper_2411_14977_amd import learned
    t0 = time.perf_counter()
    X, T = learned.harvest3d(n_windows=args.c5_train_windows)
    t1 = time.perf_counter()
    blob, losses = learned.train(X, T, epochs=args.c5_epochs, batch=512, lr=2e-3)
    t2 = time.perf_counter()
    train_loss, val_loss = struct.unpack_from("<2f", blob, 40)
    rec = {"pairs": int(X.shape[0]), "windows": args.c5_train_windows, "epochs": args.c5_epochs,
           "inputs": int(X.shape[1]), "harvest_s": t1 - t0, "train_s": t2 - t1,
           "final_val_loss": val_loss,
           "recipe": "4x4x8-hexahedron windows of the 64x64x8 tank (0.1 m elements), seeded "
                     "offsets and surfaces (seeds 5000+), smooth and white-noise sources, 6 "
                     "defect-correction cycles each plus random residuals; element-block targets"}
    log(f"[bench] 3D network: {rec['pairs']} pairs, harvest {t1 - t0:.1f} s, train {t2 - t1:.1f} s, "
        f"val loss {val_loss:.4f}")
    return blob, rec


def c5_series(steps, log_every=5, blob3=None, mode3=1):
    """3D time series (64 x 64 x 8 hexahedra, P = 6, 7.26M nodes): each step moves the free
    surface (sem_mesh_update_surface, preconditioner frozen at t = 0), re-evaluates the drifting
    source at the moved nodes and solves to 1e-10 warm-started from the previous pressure.
    Mixed precision (FP32 inner, BF16 factors; FP32 inner with factors formed from column
    records), the same with the learned stage (when a network is given) and plain FP64; solve
    time timed per step."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2411_14977_amd import binding as B
    from paper_2411_14977_amd import cases
    wl = W.c5()
    xs = B.fine_x_nodes(wl.Nx, wl.P, wl.Lx)
    ys = B.fine_x_nodes(wl.Ny, wl.P, wl.Ly)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    hfn = lambda a, b: W.bar_depth_3d(a, b, wl.Lx, wl.surface_seed)
    out = {"workload": "c5: 3D sigma-mapped tank 64x64x8 hexahedra, P=6, levels 6-3-1 then "
                       "h-levels 32x32, 16x16, 8x8 at P=1 (dense exact), dt = 0.01 s",
           "n_global": wl.n_global, "steps": steps}
    runs = [("bf16", "bf16", 0), ("col", "col", 0)]
    if blob3 is not None:
        runs.append(("bf16_learned", "bf16", mode3))
    runs.append(("f64", "f64", 0))
    for tag, prec, mode in runs:
        t0 = time.perf_counter()
        s = cases.make_solver(wl, prec=prec)
        if mode:
            s.learned_load(blob3, mode)
        t_setup = time.perf_counter() - t0
        ms_op = B.sem_time_operator(s.ctx, 0, 0, 20, 0)
        by_op = B.sem_operator_bytes(s.ctx, 0, 0)
        ms_op_hbm = B.sem_time_operator(s.ctx, 0, 0, 20, 2)
        x = torch.zeros(s.n_global, dtype=torch.float64, device="cuda")
        solve_ms, iters, upd_ms, skips = [], [], [], 0
        verdict = None
        for k in range(steps):
            t = 0.01 * k
            eta = W.surface_3d(X, Y, t, wl.Lx, wl.surface_seed)
            torch.cuda.synchronize()
            u0 = time.perf_counter()
            s.update_surface(eta)
            upd_ms.append((time.perf_counter() - u0) * 1e3)
            xg, yg, zg = s.coords(0)
            f = W.bumps_3d(xg, yg, zg, t, wl.Lx, wl.rhs_seed, hfn,
                           lambda a, b: W.surface_3d(a, b, t, wl.Lx, wl.surface_seed))
            b = s.assemble_rhs(f=torch.tensor(f, dtype=torch.float64, device="cuda"))
            if mode and k == 0:  # the plain smoother's verdict on the stage; the series keeps it on
                verdict = s.learned_judge(b, cycles=6)
                s.learned_enable(mode)
            torch.cuda.synchronize()
            a0 = time.perf_counter()
            _, info, _ = s.solve(b, x=x, tol=1e-10)
            torch.cuda.synchronize()
            solve_ms.append((time.perf_counter() - a0) * 1e3)
            iters.append(info.iters)
            skips += info.learned_skips
            if log_every and k % log_every == 0:
                log(f"[bench] c5 {tag} step {k}: {info.iters} iterations, {solve_ms[-1]:.1f} ms")
        s.close()
        ms = float(np.mean(solve_ms[1:] if steps > 1 else solve_ms))
        out[tag] = {"setup_s": t_setup, "ms_per_solve": ms, "solves_per_s": 1e3 / ms,
                    "gdof_per_s": wl.n_global / (ms * 1e-3) / 1e9,
                    "iters_mean": float(np.mean(iters)), "iters_first": iters[0],
                    "surface_update_ms": float(np.mean(upd_ms)),
                    "operator_us": ms_op * 1e3,
                    "operator_gb_per_s": by_op / (ms_op * 1e-3) / 1e9,
                    "operator_us_hbm_resident": ms_op_hbm * 1e3,
                    "operator_gb_per_s_hbm_resident": by_op / (ms_op_hbm * 1e-3) / 1e9}
        if mode:
            out[tag]["placement"] = mode
            out[tag]["learned_skips"] = skips
            out[tag]["judge"] = verdict
    out["speedup_mixed_vs_fp64"] = out["f64"]["ms_per_solve"] / out["bf16"]["ms_per_solve"]
    if blob3 is not None:
        out["speedup_learned_vs_fp64"] = (out["f64"]["ms_per_solve"] /
                                          out["bf16_learned"]["ms_per_solve"])
    return out


def stage_loop_c5(steps, prec="bf16"):
    """The stage loop around the solve on the 3D tank (64 x 64 x 8 hexahedra, P = 6): the linear
    free-surface model (eta_t = phi_z, Phi_t = -g eta) advanced with the five-stage fourth-order
    low-storage scheme, dt = 0.01 s, from the tank's surface with Phi = 0; every stage moves the
    mesh to its surface, solves the Dirichlet problem to 1e-10 warm-started, and takes the
    surface derivative (sem_wave_step).  Preconditioner built from the initial surface and kept
    (frozen), or built from still water (the time-constant linearised form of Sec. 5.4)."""
    import numpy as np
    import torch

    import workloads as W
    from paper_2411_14977_amd import binding as B
    from paper_2411_14977_amd import cases
    wl = W.c5()
    xs = B.fine_x_nodes(wl.Nx, wl.P, wl.Lx)
    ys = B.fine_x_nodes(wl.Ny, wl.P, wl.Ly)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    eta0 = W.surface_3d(X, Y, 0.0, wl.Lx, wl.surface_seed).ravel()
    out = {"workload": "c5 tank, linear free-surface model, 5 stages per step, dt = 0.01 s, "
                       "tol 1e-10", "steps": steps, "prec": prec}
    for tag, still in (("frozen_initial_surface", False), ("still_water", True)):
        s = cases.make_solver(wl, prec=prec, precond_still_water=still)
        ns = eta0.size
        y = torch.tensor(np.concatenate([eta0, np.zeros(ns)]), dtype=torch.float64, device="cuda")
        K = torch.zeros_like(y)
        phi = torch.zeros(s.n_global, dtype=torch.float64, device="cuda")
        its, ms = [], []
        for k in range(steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            it = B.sem_wave_step(s.ctx, y, K, phi, 0.01, 9.81, 1e-10)
            torch.cuda.synchronize()
            ms.append((time.perf_counter() - t0) * 1e3)
            its.append(it)
        s.close()
        out[tag] = {"ms_per_step": float(np.mean(ms[1:] if steps > 1 else ms)),
                    "iters_per_stage": its,
                    "mean_iters_per_stage": float(np.mean(its))}
        log(f"[bench] stage loop c5 ({tag}): {out[tag]['ms_per_step']:.1f} ms per step of 5 "
            f"stages, iterations per stage {its}")
    return out


def c3_error_table():
    """Mixed-precision error table on the 2048 x 16, P = 8 tank (2.11M nodes): relative error of
    the FP32-inner solution (factors FP32 and BF16) at tolerances 1e-6, 1e-8, 1e-10 against the
    FP64 solve to 1e-12, and every row's residual evaluated by the oracle (its own right-hand side
    and matrix-free FP64 operator on the CPU)."""
    import torch

    import workloads as W
    from paper_2411_14977_amd import cases
    wl = W.c3()
    check = oracle_checker(wl)
    s64 = cases.make_solver(wl, prec="f64")
    rhs = cases.make_rhs(wl, s64)
    xr, info_r, _ = s64.solve(rhs, tol=1e-12, check=False)
    out = {"workload": f"{wl.name}: 2D tank {wl.Nx}x{wl.Nz}, P={wl.P}, {wl.n_global} nodes",
           "reference": {"prec": "f64", "tol": 1e-12, "iters": info_r.iters,
                         "rel_res": info_r.rel_res, "oracle_rel_res": check(xr)}}
    s64.close()
    nr = float(torch.linalg.norm(xr))
    for prec in ("f32", "bf16"):
        s = cases.make_solver(wl, prec=prec)
        rows = {}
        for tol in (1e-6, 1e-8, 1e-10):
            x, info, _ = s.solve(rhs, tol=tol)
            rows[f"{tol:g}"] = {"iters": info.iters, "rel_res": info.rel_res,
                                "oracle_rel_res": check(x),
                                "rel_error_vs_fp64": float(torch.linalg.norm(x - xr)) / nr}
        out[prec] = rows
        s.close()
    return out


def schwarz_rows(wl, rhs, prec, steps):
    """The paper's additive Schwarz smoother (Sec. 5.3) in place of Chebyshev on every level,
    same workload, precision and outer loop: element blocks with 1 and 2 sweeps before and
    after, and subdomains widened by one node layer (1 sweep); then a 3D tank (16 x 16 x 4
    hexahedra, P = 4) with Chebyshev(3) and with Schwarz at overlap 0 and 1."""
    import torch

    import workloads as W
    from paper_2411_14977_amd import cases

    def run(w, b, **kw):
        t0 = time.perf_counter()
        s = cases.make_solver(w, prec=prec, **kw)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        t, info, _ = time_solves(s, b, steps, 1, 1e-10)
        s.close()
        return {"ms_per_solve": t * 1e3, "iters": info.iters, "rel_res": info.rel_res,
                "setup_s": t_setup}

    out = {}
    for nu in (1, 2):
        out[f"sweeps_{nu}"] = run(wl, rhs, smoother="asm", nu_pre=nu, nu_post=nu)
    out["overlap_1_sweeps_1"] = run(wl, rhs, smoother="asm", nu_pre=1, nu_post=1,
                                    schwarz_overlap=1)
    w3 = W.tank3d(16, 16, 4, 4, L=1.6, name="tank3d_16x16x4_p4")
    s = cases.make_solver(w3, prec=prec)
    b3 = cases.make_rhs(w3, s)
    s.close()
    out["tank3d_16x16x4_p4"] = {
        "chebyshev3": run(w3, b3),
        "schwarz_overlap_0": run(w3, b3, smoother="asm", nu_pre=1, nu_post=1),
        "schwarz_overlap_1": run(w3, b3, smoother="asm", nu_pre=1, nu_post=1,
                                 schwarz_overlap=1)}
    return out


def paper_context(prec):
    """The paper's multigrid-efficiency experiments (Sec. 6, table of iterations per tolerance
    and the scaling figure) rerun with this solver on the synthetic tank: N_z = 2, P = 8,
    N_x = 102 at tolerances 1e-4, 1e-6, 1e-8 (PDC, FPCG and GMRES, the paper's two outer
    methods and this solver's default; PDC and GMRES also on the mixed-stage operator of two
    stage surfaces, the paper's operator within a stage, with the same-stage V-cycle), then at 1e-6 the iterations and time against N_x
    (P = 8, element width fixed at 0.25 m) and against the horizontal order P_x at N_x = 200
    with the vertical order fixed at P_z = 8 (semi-coarsened hierarchy, Sec. 5.1), for FPCG and
    GMRES; beside it the equal-order sweep P_x = P_z.  Inner precision as the timed path,
    Chebyshev(3) smoothing; times are medians of seven solves; context, not the headline."""
    import torch

    import workloads as W
    from paper_2411_14977_amd import cases

    def run(Nx, P, outer, tols, Pz=None):
        if Pz is None:
            wl = W.tank(Nx, 2, P, Lx=0.25 * Nx, name=f"ctx{Nx}p{P}")
        else:
            wl = W.tank_semi(Nx, 2, P, Pz, Lx=0.25 * Nx, name=f"ctx{Nx}p{P}z{Pz}")
        s = cases.make_solver(wl, prec=prec, outer=outer)
        rhs = cases.make_rhs(wl, s)
        rows = {}
        for tol in tols:
            t, info, _ = median_solve(s, rhs, tol)
            rows[f"{tol:g}"] = {"iters": info.iters, "ms": t * 1e3}
        levels = [list(s.level_orders(l)) for l in range(s.nlevels)]
        s.close()
        return wl.n_global, rows, levels

    def run_mixed(Nx, P, outer, tols):
        # the mixed-stage operator: stage k's surface is stage k-1's moved 5 cm along the tank
        # (the distance a 1.2 m/s crest travels in a 0.04 s stage)
        from paper_2411_14977_amd import binding as Bm
        wl = W.tank(Nx, 2, P, Lx=0.25 * Nx, name=f"ctx{Nx}p{P}")
        x = Bm.fine_x_nodes(wl.Nx, wl.P, wl.Lx)
        s = cases.make_solver(wl, prec=prec, outer=outer)
        s.update_surface(W.surface(x - 0.05, wl.Lx, wl.surface_seed))
        s.mixed_stage(W.surface(x, wl.Lx, wl.surface_seed))
        rhs = cases.make_rhs(wl, s)
        rows = {}
        for tol in tols:
            t, info, _ = median_solve(s, rhs, tol)
            rows[f"{tol:g}"] = {"iters": info.iters, "ms": t * 1e3}
        s.close()
        return wl.n_global, rows

    out = {"table": {}, "mixed_stage_table": {}, "scaling_nx": [], "scaling_px_pz8": [],
           "scaling_p": []}
    for outer in ("pdc", "fpcg", "gmres"):
        n, rows, _ = run(102, 8, outer, (1e-4, 1e-6, 1e-8))
        out["table"][outer] = {"n_global": n, **rows}
    for outer in ("pdc", "gmres"):
        n, rows = run_mixed(102, 8, outer, (1e-4, 1e-6, 1e-8))
        out["mixed_stage_table"][outer] = {"n_global": n, **rows}
    for outer in ("fpcg", "gmres"):
        for Nx in (25, 50, 100, 200, 400, 800):
            n, rows, _ = run(Nx, 8, outer, (1e-6,))
            out["scaling_nx"].append({"outer": outer, "Nx": Nx, "P": 8, "n_global": n,
                                      **rows["1e-06"]})
        for Px in (2, 3, 4, 5, 6, 7, 8, 10, 12):
            n, rows, levels = run(200, Px, outer, (1e-6,), Pz=8)
            out["scaling_px_pz8"].append({"outer": outer, "Nx": 200, "Px": Px, "Pz": 8,
                                          "n_global": n, "levels": levels, **rows["1e-06"]})
        for P in (2, 3, 4, 5, 6, 7, 8):
            n, rows, _ = run(200, P, outer, (1e-6,))
            out["scaling_p"].append({"outer": outer, "Nx": 200, "P": P, "n_global": n,
                                     **rows["1e-06"]})
    torch.cuda.synchronize()
    return out


def copy_reference(nbytes):
    """A plain device-to-device copy that moves the same number of bytes (half read, half
    written), timed HBM-resident the same way (rotated buffers, over 768 MiB in all): the
    bandwidth a launch of this size reaches without any arithmetic."""
    import torch
    n = max(1, int(nbytes / 8))  # float32 elements per side
    R = max(2, int(800e6 / (nbytes)) + 1)
    src = [torch.ones(n, device="cuda") for _ in range(R)]
    dst = [torch.empty(n, device="cuda") for _ in range(R)]
    for k in range(R):
        dst[k].copy_(src[k])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3 * R
    torch.cuda.synchronize()
    e0.record()
    for k in range(reps):
        dst[k % R].copy_(src[k % R])
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    ach = 8.0 * n / (ms * 1e-3) / 1e9
    return {"bytes": 8.0 * n, "avg_launch_ms": ms, "achieved": ach, "frac": ach / HBM_PEAK_GBS,
            "timing": "torch device copy, rotated buffers, CUDA events on the current stream"}


def traffic_from_profiles(kernel_tag):
    """HBM traffic per launch measured by rocprofv3 PMC passes (profiles/*.json), only if
    the kernel source is unchanged since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        src = open(os.path.join(ROOT, "paper_2411_14977_amd", "csrc", "kernels.hip"), "rb").read()
        if rec.get("kernels_hip_sha256") != hashlib.sha256(src).hexdigest():
            return None
        return rec.get("bytes_per_launch")
    except Exception:
        return None


def cpu_baseline(wl, tol):
    """Oracle (NumPy/SciPy, FP64) FPCG + p-MG on a bounded sample of the workload: a window of
    128 element columns of the same tank over the ramp and the flat top of the bar (same element
    size, order, layers, smoother, bathymetry, surface and source)."""
    import numpy as np

    import workloads as W
    from oracle import assemble, pmg
    from tests import oracle_cases as oc
    ncols = min(128, wl.Nx)
    c0 = min(wl.Nx - ncols, (6 * wl.Nx) // 16)
    dx = wl.Lx / wl.Nx
    x0 = c0 * dx
    Ls = ncols * dx
    full_h = lambda x: W.bar_depth(x, wl.Lx)
    full_eta = lambda x: W.surface(x, wl.Lx, wl.surface_seed)
    xs = oc.fine_x_nodes(ncols, wl.P, Ls)
    args = dict(dim=2, Nx=ncols, Nz=wl.Nz, Lx=Ls, h=full_h(xs + x0), eta=full_eta(xs + x0))
    t0 = time.perf_counter()
    H = pmg.Hierarchy(args, wl.orders, smoother="chebyshev", cheb_degree=wl.cheb_degree,
                      cheb_lo=wl.cheb_lo, cheb_hi=wl.cheb_hi,
                      cheb_degree_coarse=wl.cheb_degree_coarse or None)
    pmg.estimate_lambdas(H)
    t_setup = time.perf_counter() - t0
    L0 = H.levels[0]
    m = L0.mesh
    X, Z = m.node_coords()
    f = W.bumps(X + x0, Z, wl.Lx, wl.rhs_seed, full_h, full_eta)
    b = assemble.assemble_rhs(m, f=f)
    t0 = time.perf_counter()
    _, it, hist = pmg.fpcg(L0.A, b, np.zeros(L0.N), H.vcycle, tol)
    t_solve = time.perf_counter() - t0
    return {"value": L0.N / t_solve / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "sample": (f"oracle FP64 FPCG+p-MG (SciPy CSR, single-threaded sparse kernels; "
                       f"{os.cpu_count()} host cores available) on element columns {c0}..."
                       f"{c0 + ncols - 1} of {wl.Nx} (x in [{x0:.2f}, {x0 + Ls:.2f}] m: bar ramp "
                       f"and top) of the same tank, {L0.N} DOFs, {it} iterations to {tol:g}; "
                       f"solve {t_solve:.2f} s timed, set-up {t_setup:.2f} s excluded"),
            "solves_per_s_sample": 1.0 / t_solve, "iters": it}


def oracle_checker(wl):
    """x -> relative residual of a returned pressure, evaluated by the oracle (its own right-hand
    side and matrix-free FP64 operator on the CPU; mesh and right-hand side built once)."""
    import numpy as np

    from oracle import assemble
    from tests import oracle_cases as oc
    m = oc.fine_mesh(wl)
    b = oc.rhs(wl, m)
    nb = np.linalg.norm(b)

    def check(x):
        r = b - assemble.apply_matrix_free(m, x.cpu().numpy())
        return float(np.linalg.norm(r) / nb)
    return check


def oracle_check(wl, x):
    return oracle_checker(wl)(x)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--prec", default="bf16", choices=["bf16", "f32", "col"])
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-learned", action="store_true", help="time the V-cycle without the stage")
    ap.add_argument("--train-surfaces", type=int, default=40)
    ap.add_argument("--epochs", type=int, default=600)
    ap.add_argument("--surfaces", type=int, default=20, help="unseen test surfaces to report")
    ap.add_argument("--oracle-surfaces", type=int, default=3,
                    help="unseen surfaces whose learned solution the oracle solves and checks")
    ap.add_argument("--pdc-cycles", type=int, default=12)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparison")
    ap.add_argument("--op-reps", type=int, default=50)
    ap.add_argument("--c5-steps", type=int, default=20, help="3D time-series steps (0: skip)")
    ap.add_argument("--c5-train-windows", type=int, default=16,
                    help="3D training windows of the 3D learned stage (0: no 3D stage)")
    ap.add_argument("--c5-epochs", type=int, default=200)
    ap.add_argument("--stage-steps", type=int, default=3,
                    help="steps of the 3D stage loop around the solve (0: skip)")
    ap.add_argument("--no-c3", action="store_true", help="skip the c3 mixed-precision error table")
    ap.add_argument("--no-schwarz", action="store_true", help="skip the Schwarz-smoother rows")
    ap.add_argument("--no-context", action="store_true",
                    help="skip the paper-shaped iteration table and scaling sweeps")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the solver runs on one GPU (it has no multi-GPU path); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2411_14977_amd import binding as B
    from paper_2411_14977_amd import cases

    torch.cuda.set_device(0)
    wl = workload(args.workload)
    use_learned = not args.no_learned and wl.P == 8
    log(f"[bench] workload {wl.name} N={wl.n_global} prec={args.prec} learned={use_learned}")

    blob, train_rec = (None, None)
    if use_learned:
        blob, train_rec = train_network(args, wl, args.prec)

    s = cases.make_solver(wl, prec=args.prec)
    rhs = cases.make_rhs(wl, s)
    plain_mixed = None
    factor_rows = None
    placements = None
    mode = 0
    if use_learned:
        t_nl, info_nl, _ = time_solves(s, rhs, args.steps, args.warmup, args.tol)
        plain_mixed = {"ms_per_solve": t_nl * 1e3, "solves_per_s": 1.0 / t_nl,
                       "gdof_per_s": wl.n_global / t_nl / 1e9, "iters": info_nl.iters,
                       "rel_res": info_nl.rel_res}
        log(f"[bench] mixed without stage: {t_nl * 1e3:.3f} ms/solve, {info_nl.iters} iterations")
        # the other ways of holding the inner geometric factors, same solve
        factor_rows = {args.prec: dict(plain_mixed)}
        for pv in ("bf16", "f32", "col"):
            if pv == args.prec:
                continue
            sp = cases.make_solver(wl, prec=pv)
            tp, ip, _ = time_solves(sp, rhs, args.steps, args.warmup, args.tol)
            factor_rows[pv] = {"ms_per_solve": tp * 1e3, "iters": ip.iters, "rel_res": ip.rel_res}
            sp.close()
            log(f"[bench] mixed without stage, factors {pv}: {tp * 1e3:.3f} ms/solve, "
                f"{ip.iters} iterations")
        # every placement of the stage, timed the same way; the fastest is the headline
        placements = {}
        s.learned_load(blob, 1)
        for m in (1, 2, 3):
            s.learned_enable(m)
            tm, im, _ = time_solves(s, rhs, args.steps, args.warmup, args.tol)
            placements[str(m)] = {"ms_per_solve": tm * 1e3, "iters": im.iters,
                                  "skips": im.learned_skips, "rel_res": im.rel_res}
            log(f"[bench] learned placement {m}: {tm * 1e3:.3f} ms/solve, {im.iters} iterations")
        mode = min(placements, key=lambda k: placements[k]["ms_per_solve"])
        mode = int(mode)
        s.learned_enable(mode)
    t, info, x = time_solves(s, rhs, args.steps, args.warmup, args.tol)
    log(f"[bench] timed path: {t * 1e3:.3f} ms/solve, {info.iters} iterations, "
        f"rel_res {info.rel_res:.2e}, learned skips {info.learned_skips}")

    breakeven = None
    if use_learned:
        per_it_plain = t_nl / info_nl.iters
        per_it = t / info.iters
        breakeven = {
            "placement": mode,
            "iterations_saved": info_nl.iters - info.iters,
            "stage_us_per_iteration": (per_it - per_it_plain) * 1e6,
            "plain_iteration_us": per_it_plain * 1e6,
            # the stage pays for itself when its cost per iteration is below this
            "break_even_stage_us_per_iteration":
                (t_nl - per_it_plain * info.iters) / info.iters * 1e6 if info.iters else None}

    # the plain smoother as the judge of the stage: residual reduction per cycle and per unit of
    # time with the stage off and on (sem_learned_judge); where it switches the stage off, the
    # solve with its verdict is timed beside the headline (which keeps the stage on)
    judge = None
    if use_learned:
        judge = s.learned_judge(rhs, cycles=6)
        log(f"[bench] judge: {judge}")
        if not judge["enabled"]:
            tj, ij, _ = time_solves(s, rhs, args.steps, args.warmup, args.tol)
            judge["solve_with_verdict"] = {"stage": "off", "ms_per_solve": tj * 1e3,
                                           "iters": ij.iters, "rel_res": ij.rel_res}
        s.learned_enable(mode)

    # whole solve: the sum of every launch's algorithmic bytes over one solve (the same solve
    # issued without graphs) against the timed solve's duration
    xb = torch.zeros_like(rhs)
    wb, wit, wn = B.sem_solve_bytes(s.ctx, rhs, xb, args.tol)
    whole = {"bytes_per_solve": wb, "iters": wit, "kernels_per_solve": wn,
             "ms_per_solve": t * 1e3,
             "achieved": wb / t / 1e9 * (info.iters / wit if wit else 1.0),
             "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    whole["frac"] = whole["achieved"] / HBM_PEAK_GBS
    log(f"[bench] whole solve: {wb / 1e6:.1f} MB in {wn} kernels, "
        f"{whole['achieved']:.0f} GB/s ({100 * whole['frac']:.1f}% of HBM peak)")

    # dominant solver kernel: the fine level's fused smoother step (operator + Chebyshev update);
    # beside it the plain operator apply and the FP64 outer operator.  HBM-resident timing: the
    # launches take rotated copies of every buffer (> 768 MiB in all), so no launch finds its data
    # in the 256 MB Infinity Cache; the cache-resident figure (same buffers back to back) beside it
    def timed(kind):
        by = B.sem_operator_bytes(s.ctx, 0, kind)
        ms_hbm = B.sem_time_operator(s.ctx, 0, kind, args.op_reps, 2)
        ms_cache = B.sem_time_operator(s.ctx, 0, kind, args.op_reps, 0)
        return by, ms_hbm, ms_cache

    def gbs(by, ms):
        return by / (ms * 1e-3) / 1e9

    bytes_op, ms_op, ms_op_c = timed(0)
    bytes_step, ms_step, ms_step_c = timed(2)
    bytes_outer, ms_outer, ms_outer_c = timed(1)
    ach = gbs(bytes_step, ms_step)
    gname = {"bf16": "bf16", "f32": "float", "col": "column records"}[args.prec]
    kernel_tag = f"cheb2d_{wl.name}_{args.prec}"
    roof = {"bound": "hbm",
            "kernel": f"k_cheb2d<P={wl.P},float,{gname}>: fused operator + Chebyshev step "
                      f"(x, b, dinv, d read; x, d written; factors read once)",
            "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": traffic_from_profiles(kernel_tag),
            "algorithmic_bytes_per_launch": bytes_step, "avg_launch_ms": ms_step,
            "timing": "HIP events on the library stream around back-to-back launches that take "
                      "rotated copies of every buffer (over 768 MiB in all), so each launch "
                      "streams its data from HBM",
            "cache_resident": {"avg_launch_ms": ms_step_c, "achieved": gbs(bytes_step, ms_step_c),
                               "frac": gbs(bytes_step, ms_step_c) / HBM_PEAK_GBS,
                               "timing": "the same buffers back to back (33 MB working set "
                                         "served from the 256 MB Infinity Cache)"},
            "operator_apply": {"kernel": f"k_apply2d<P={wl.P},float,{gname}>",
                               "algorithmic_bytes_per_launch": bytes_op, "avg_launch_ms": ms_op,
                               "achieved": gbs(bytes_op, ms_op),
                               "frac": gbs(bytes_op, ms_op) / HBM_PEAK_GBS,
                               "cache_resident_achieved": gbs(bytes_op, ms_op_c)},
            "outer_fp64_operator": {"algorithmic_bytes_per_launch": bytes_outer,
                                    "avg_launch_ms": ms_outer,
                                    "achieved": gbs(bytes_outer, ms_outer),
                                    "frac": gbs(bytes_outer, ms_outer) / HBM_PEAK_GBS,
                                    "cache_resident_achieved": gbs(bytes_outer, ms_outer_c)},
            "whole_solve": whole}
    roof["copy_same_bytes"] = copy_reference(bytes_step)
    log(f"[bench] a plain device copy moving the fused step's bytes: "
        f"{roof['copy_same_bytes']['avg_launch_ms'] * 1e3:.2f} us HBM-resident "
        f"({100 * roof['copy_same_bytes']['frac']:.1f}% of HBM peak)")
    log(f"[bench] fused step {ms_step * 1e3:.2f} us HBM-resident ({ach:.0f} GB/s, "
        f"{100 * ach / HBM_PEAK_GBS:.1f}% of HBM peak), {ms_step_c * 1e3:.2f} us cache-resident; "
        f"operator {ms_op * 1e3:.2f} us ({100 * gbs(bytes_op, ms_op) / HBM_PEAK_GBS:.1f}%); "
        f"fp64 outer {ms_outer * 1e3:.2f} us")
    s.close()
    # calibration for hardware byte counters: three plain 256 MiB device copies (a profiler
    # reading FETCH_SIZE / WRITE_SIZE of this command scales the operator's counts by these)
    ca = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
    cb = torch.empty_like(ca)
    for _ in range(3):
        cb.copy_(ca)
    torch.cuda.synchronize()
    del ca, cb

    res_check = None
    try:
        res_check = oracle_check(wl, x)
    except Exception as e:  # pragma: no cover
        log(f"[bench] oracle residual check failed: {e}")

    plain = None
    if not args.no_fp64:
        s64 = cases.make_solver(wl, prec="f64")
        t64, info64, x64 = time_solves(s64, rhs, args.steps, args.warmup, args.tol)
        plain = {"ms_per_solve": t64 * 1e3, "solves_per_s": 1.0 / t64,
                 "gdof_per_s": wl.n_global / t64 / 1e9, "iters": info64.iters,
                 "rel_res": info64.rel_res,
                 "timed_path_vs_fp64_rel_diff": float(torch.linalg.norm(x - x64) / torch.linalg.norm(x64))}
        log(f"[bench] fp64: {t64 * 1e3:.3f} ms/solve, {info64.iters} iterations")
        s64.close()

    pdc = surf = None
    parity_procs = []
    parity_kept = None   # surfaces whose GPU pressure the oracle checks, once the GPU timing is done
    if use_learned:
        pdc = pdc_rates(wl, args.prec, blob, args.pdc_cycles, mode)
        log(f"[bench] PDC per-cycle rate: {pdc}")
        if args.surfaces > 0:
            keep = tuple(range(1, min(args.oracle_surfaces, args.surfaces) + 1))
            rows, kept = unseen_surfaces(args, blob, args.surfaces, mode, keep)
            saved = [r["plain"]["iters"] - r["learned"]["iters"] for r in rows]
            surf = {"rows": rows,
                    "iters_saved_mean": sum(saved) / len(saved),
                    "learned_faster_on": sum(r["learned"]["ms"] < r["plain"]["ms"] for r in rows),
                    "of": len(rows)}
            parity_kept = kept

    context = None
    if not args.no_context:
        context = paper_context(args.prec)
        log(f"[bench] paper-shaped runs: {context['table']}")
        log(f"[bench] mixed-stage operator: {context['mixed_stage_table']}")
        for outer in ("fpcg", "gmres"):
            sw = [r for r in context["scaling_px_pz8"] if r["outer"] == outer]
            log(f"[bench] P_x sweep at P_z = 8, N_x = 200, tol 1e-6 ({outer}): " +
                ", ".join(f"P_x={r['Px']}: {r['iters']} it {r['ms']:.2f} ms" for r in sw))

    schwarz = None
    if not args.no_schwarz:
        schwarz = schwarz_rows(wl, rhs, args.prec, max(2, args.steps))
        log(f"[bench] Schwarz smoother: {schwarz}")

    c3 = None
    if not args.no_c3:
        c3 = c3_error_table()
        log(f"[bench] c3 errors: f32 {[v['rel_error_vs_fp64'] for v in c3['f32'].values()]}, "
            f"bf16 {[v['rel_error_vs_fp64'] for v in c3['bf16'].values()]}")

    c5 = None
    if args.c5_steps > 0:
        blob3, rec3 = (None, None)
        if args.c5_train_windows > 0:
            blob3, rec3 = c5_learned_network(args)
        c5 = c5_series(args.c5_steps, blob3=blob3)
        c5["training"] = rec3
        msg = (f"[bench] c5 series: mixed {c5['bf16']['ms_per_solve']:.1f} ms "
               f"({c5['bf16']['iters_mean']:.1f} it), mixed with column-record factors "
               f"{c5['col']['ms_per_solve']:.1f} ms ({c5['col']['iters_mean']:.1f} it), "
               f"fp64 {c5['f64']['ms_per_solve']:.1f} ms ({c5['f64']['iters_mean']:.1f} it)")
        if blob3 is not None:
            msg += (f", mixed + learned {c5['bf16_learned']['ms_per_solve']:.1f} ms "
                    f"({c5['bf16_learned']['iters_mean']:.1f} it)")
        log(msg)

    stage_loop = None
    if args.stage_steps > 0:
        stage_loop = stage_loop_c5(args.stage_steps, args.prec)

    # the oracle's checks run on the host cores after every GPU timing, so that they do not
    # compete with the host side of the timed solves
    if parity_kept:
        parity_procs = start_oracle_parity(args, parity_kept)
        log(f"[bench] oracle checking surfaces {sorted(parity_kept)} in {len(parity_procs)} "
            f"background processes")
    if parity_procs:
        log("[bench] waiting for the oracle's solves of the unseen surfaces ...")
        surf["oracle_parity"] = finish_oracle_parity(parity_procs)
        log(f"[bench] oracle parity: {surf['oracle_parity']}")

    cpu = None
    if not args.no_cpu:
        log("[bench] timing the CPU oracle on a bounded sample ...")
        cpu = cpu_baseline(wl, args.tol)
        log(f"[bench] cpu oracle {cpu['value']:.3e} GDOF/s")

    out = {"metric": METRIC, "value": wl.n_global / t / 1e9, "unit": "GDOF/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": t * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"bf16": "fp32 inner (bf16 factors and network operands) / fp64 outer",
                     "f32": "fp32 inner (fp32 factors, bf16 network operands) / fp64 outer",
                     "col": "fp32 inner (factors formed from fp64 column records, bf16 network "
                            "operands) / fp64 outer"}[args.prec],
           "data": "synthetic", "config": describe(wl, args.prec, use_learned, mode),
           "solves_per_s": 1.0 / t, "iters": info.iters, "rel_res": info.rel_res,
           "learned_skips": info.learned_skips, "oracle_rel_res": res_check,
           "mixed_without_stage": plain_mixed, "mixed_factor_storage": factor_rows,
           "plain_fp64": plain,
           "speedup_vs_fp64": (plain["ms_per_solve"] / (t * 1e3)) if plain else None,
           "learned_placements": placements, "learned_break_even": breakeven,
           "learned_judge": judge,
           "training": train_rec, "pdc_rate": pdc, "unseen_surfaces": surf,
           "schwarz_smoother": schwarz, "paper_context": context, "c3_error_table": c3,
           "c5_series": c5, "stage_loop": stage_loop,
           "roofline": roof, "cpu_baseline": cpu}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--oracle-worker":
        oracle_worker(sys.argv[2], int(sys.argv[3]), sys.argv[4])
    else:
        main()
