#!/usr/bin/env python3
"""Throughput benchmark of the Jacobi-preconditioned block BiCGGR hot path.

One step = one complete solve of A X = B for one batch of L right-hand sides
(point sources) to a relative residual of 1e-12 in every column: every
kernel of the hot path (operator, clover, Jacobi sweeps, Gram products, L x L
solves, block updates, driver) runs in it.  Inputs are resident in HBM before
the timed region starts.

Printed JSON line (one, from rank 0):
  value        algorithmic GB/s of the multi-RHS operator kernel Y = A X (the
               Dslash of the metric), timed with HIP events around back-to-back
               launches on the library's stream, on block vectors in the tiled
               layout the solver runs in; pct_hbm_peak is its fraction of the
               8 TB/s HBM peak
  solve_GBs    algorithmic HBM bytes of all kernels of the timed solves / time
  s_per_rhs    seconds per right-hand side of the timed solves
  roofline     the dominant kernel (the FP64 Jacobi sweep, 2j-2 of the 2j+2
               hopping-kernel launches per outer iteration), timed with HIP
               events around back-to-back launches on the library's stream
  dslash       the same measurement for the operator kernel Y = A X
  solves       one solve per inner precision (FP64, FP32, BF16 Jacobi) for
               the time-to-solution comparison
  cpu_baseline the FP64 oracle on a bounded sample of the same workload
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=2)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--workload", default="lat32x64_L12_point")
    p.add_argument("--j", type=int, default=12)
    p.add_argument("--kappa", type=float, default=None)
    p.add_argument("--hop-reps", type=int, default=20)
    p.add_argument("--no-compare", action="store_true", help="skip the per-precision solve comparison")
    p.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner leg")
    p.add_argument("--learn-pairs", type=int, default=24)
    p.add_argument("--learn-steps", type=int, default=20)
    p.add_argument("--learn-snaps", type=int, default=3, help="solver snapshots per logging solve")
    p.add_argument("--snap-every", type=int, default=15)
    p.add_argument("--learn-solves", type=int, default=1,
                   help="solves that log snapshots: the first with the workload's sources, the rest with Z4 noise")
    p.add_argument("--learn-solver-pairs", type=int, default=0, help="cap on the solver pairs kept (0: all)")
    p.add_argument("--learn-lr", type=float, default=1e-3)
    p.add_argument("--learn-prec", default="f64", help="precisions of the solves with trained weights (f64,f32)")
    p.add_argument("--j-sweep", action="store_true",
                   help="only the Jacobi-step sweep: FP64 solves for j in 0, 4, 8, 12, 16, 24 at kappa and kappa-heavy")
    p.add_argument("--kappa-heavy", type=float, default=0.12,
                   help="second kappa (heavier quark) for the time-to-solution comparison; 0 skips it")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--ensembles", type=int, default=0,
                   help="compare the preconditioner precisions over this many link ensembles (link seeds) "
                        "at --kappa and --kappa-heavy: converged counts and mean s/RHS")
    p.add_argument("--conditioning", action="store_true",
                   help="only the conditioning probe: power iteration of kappa T^-1 H and ARPACK's leftmost "
                        "eigenvalues of A (GPU operator as the matrix-vector product) per lattice and kappa")
    p.add_argument("--learned-c3", action="store_true",
                   help="only the learned-preconditioner workload at 16^3 x 32 (L = 12, ~2000 solver pairs, "
                        "vs Jacobi j = 12) at kappa 0.130 and 0.120")
    p.add_argument("--hop-sweep", action="store_true",
                   help="only the operator and Jacobi-sweep kernel timings against the block width L "
                        "(1, 2, 3, 4, 6, 8, 12 up to the workload's L), in the layout the solver runs in")
    p.add_argument("--kernels-only", action="store_true",
                   help="only the hopping-kernel launches and a plain copy (for rocprofv3 counter runs)")
    return p.parse_args()


def src_hash():
    """Hash of the sources of the hopping kernels (the kernels whose HBM traffic is profiled)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_0907_3261_amd", "csrc")
    for f in ("wd_internal.h", "wd_dslash.hip"):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profiles(mode: int):
    """HBM bytes per launch of the FP64 hopping kernel (mode 0: A X, 1: Jacobi sweep) from
    the rocprofv3 FETCH_SIZE / WRITE_SIZE runs, if they were taken on the current sources."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        if d.get("src_hash") != src_hash():
            return None
        for k, v in d.get("bytes_per_launch", {}).items():
            # the LDS-staged FP64 kernel (three or more columns): mode, iterate format (the timed
            # sweep is the middle one, time-diagonal in and out: 3), coefficient storage, tiled vectors
            if k.startswith(f"void k_hop_f64<{mode}, {3 if mode == 1 else 0}, StF64, 1>"):
                return v
        for k, v in d.get("bytes_per_launch", {}).items():
            # template arguments of the register-tiled hop kernel: storage in, storage out, columns,
            # mode, stream policy, coefficient storage
            if k.startswith("void k_hop<StF64, StF64,"):
                args = [a.strip() for a in k[k.index("<") + 1:k.rindex(">")].split(",")]
                if len(args) >= 4 and args[3] == str(mode) and (len(args) < 6 or args[5] == "StF64"):
                    return v
    except Exception:
        return None
    return None


def time_hop(ctx, torch, V, L, mode, reps, prec="f64", layout=None):
    """Average duration of one hopping-kernel launch (mode 0: A X, 1: Jacobi sweep), from HIP
    events on the library's stream around reps and 2 reps back-to-back launches (the difference
    removes the once-per-call rounding of the inputs in FP32 / BF16).  layout: the block-vector
    layout of the launches; by default the tiled one the solver runs in when V allows it."""
    if layout is None:
        layout = "tiled" if V % 64 == 0 else "standard"
    ctx.set_layout(layout)
    try:
        return _time_hop(ctx, torch, V, L, mode, reps, prec)
    finally:
        ctx.set_layout("standard")


def _time_hop(ctx, torch, V, L, mode, reps, prec):
    g = torch.Generator(device="cuda").manual_seed(11)
    X = torch.complex(torch.randn((L, 12, V), generator=g, device="cuda", dtype=torch.float64),
                      torch.randn((L, 12, V), generator=g, device="cuda", dtype=torch.float64))
    R = torch.complex(torch.randn((L, 12, V), generator=g, device="cuda", dtype=torch.float64),
                      torch.randn((L, 12, V), generator=g, device="cuda", dtype=torch.float64))
    Y = torch.empty_like(X)
    ctx.hop_repeat(X, Y, 3, mode, R, prec)
    st = ctx.stream
    t = []
    for n in (reps, 2 * reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        ctx.hop_repeat(X, Y, n, mode, R, prec)
        e1.record(st)
        e1.synchronize()
        t.append(e0.elapsed_time(e1))
    del X, R, Y
    return (t[1] - t[0]) / reps


def time_copy(torch, V, L, reps=5):
    """Device-to-device copy of one N x L block with torch (read + write bytes per second): the
    rate a plain streaming kernel reaches on this GPU, reported beside the roofline."""
    a = torch.empty((L, 12, V), dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * L * 12 * V * 16 / (ms / 1e3) / 1e9


def solve_record(info, L, X=None, Xref=None, torch=None, np=None):
    d = {"status": info["status"], "iterations": info["total_iterations"], "cycles": info["cycles"],
         "fallback": info["fallback"], "s_per_rhs": round(info["seconds"] / L, 5),
         "true_residual_max": float(np.max(info["true_residual"])), "mvm_paper_per_col": int(info["mvm_paper"])}
    if Xref is not None:
        d["rel_diff_vs_f64"] = float(torch.linalg.vector_norm(X - Xref) / torch.linalg.vector_norm(Xref))
    return d


def compare_leg(ctx, torch, np, B, L, w, a):
    """Jacobi (j = a.j) solves from X = 0: FP64; FP32 and BF16 storage; FP64 iterates with FP32
    and BF16 links and A_D^-1."""
    out, Xref, k64 = {}, None, 0
    for prec in ("f64", "f32", "bf16", "f64c32", "f64cbf16"):
        torch.cuda.synchronize()
        # rounded coefficients give a fixed M but can stagnate near the critical kappa: one run,
        # capped at one and a half times the FP64 iterations
        cap = dict(max_iter=3 * k64 // 2 + 10, max_restarts=0) if prec.startswith("f64c") else {}
        X, info = ctx.solve(B, tol=w["tol"], j=a.j, prec_inner=prec, **cap)
        if prec == "f64":
            k64 = info["iterations"]
        torch.cuda.synchronize()
        if prec == "f64":
            Xref = X.clone()
        out[f"jacobi{a.j}_{prec}"] = solve_record(info, L, X, Xref, torch, np)
        print(f"[bench] jacobi {prec}: {out[f'jacobi{a.j}_{prec}']}", file=sys.stderr, flush=True)
    return out, Xref


def learned_setup(ctx, torch, np, B, V, L, w, a):
    """Learned preconditioner: start from the factored degree-3 Neumann series, time one
    application of M in FP64 and FP32, then train with Adam on pairs that the solver generates
    (snapshots X_k of FP64 Jacobi solves: r = B - A X_k, e = X - X_k) together with pairs
    (A e, e) for Gaussian e."""
    import wdinputs as wi
    out = {}
    g = torch.Generator(device="cuda").manual_seed(12)
    P = a.learn_pairs - a.learn_pairs % L           # Gaussian pairs
    S = a.learn_snaps                               # snapshot blocks of L columns per logging solve
    K = a.learn_solves if S > 0 else 0
    cap = K * S * L if a.learn_solver_pairs <= 0 else min(K * S * L, a.learn_solver_pairs - a.learn_solver_pairs % L)
    Ep = torch.empty((P + cap, 12, V), dtype=torch.complex128, device="cuda")
    Rp = torch.empty_like(Ep)
    Ep[:P] = torch.complex(torch.randn((P, 12, V), generator=g, device="cuda", dtype=torch.float64),
                           torch.randn((P, 12, V), generator=g, device="cuda", dtype=torch.float64))
    for i in range(0, P, L):
        ctx.apply(Ep[i:i + L], Rp[i:i + L])
    n = P
    if K > 0 and cap > 0:
        Xs = torch.empty((S * L, 12, V), dtype=torch.complex128, device="cuda")
        snaps = []
        for k in range(K):
            Bk = B if k == 0 else torch.from_numpy(wi.source_block("z4", V, L, w["source_seed"] + 100 + k)).cuda()
            X, info = ctx.solve(Bk, tol=w["tol"], j=a.j, x_snap=Xs, snap_every=a.snap_every)
            # a snapshot of the final iteration equals X (e = 0): leave it out
            ns = min(info["snapshots"], (info["total_iterations"] - 1) // a.snap_every, (P + cap - n) // L)
            snaps.append(ns)
            if ns > 0:
                r, e = ctx.learned_pairs(Bk, X, Xs[:ns * L])
                Rp[n:n + ns * L] = r
                Ep[n:n + ns * L] = e
                n += ns * L
                del r, e
            del X, Bk
            if n >= P + cap:
                break
        out["solver_pairs"] = {"solves": len(snaps), "snapshots": snaps, "every": a.snap_every, "columns": n - P}
        del Xs
    Rp, Ep = Rp[:n], Ep[:n]
    ctx.learned_init("neumann")
    Z = torch.empty((L, 12, V), dtype=torch.complex128, device="cuda")
    # timed on block vectors in the layout the solver runs in (the data are the benchmark's right-hand
    # sides read in that layout: the cost does not depend on the values)
    ctx.set_layout("tiled" if V % 64 == 0 else "standard")
    for prec, per_layer in (("f64", 576 + 384 * L), ("f32", 288 + 192 * L)):
        ctx.learned_apply(B, Z, prec=prec)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        reps = 5
        e0.record(ctx.stream)
        for _ in range(reps):
            ctx.learned_apply(B, Z, prec=prec)
        e1.record(ctx.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        b = 3 * V * per_layer + (2 * V * 96 * L if prec == "f32" else 0)
        out[f"apply_{prec}"] = {"ms": round(ms, 4), "alg_bytes": b, "GBs": round(b / (ms / 1e3) / 1e9, 1)}
    ctx.set_layout("standard")
    thetas = {"neumann3": ctx.get_learned()}
    # trainings from the Neumann start: Gaussian pairs only, solver pairs with them, and (when both
    # kinds exist) the solver pairs alone
    sets = [("trained_gauss", (Rp[:P], Ep[:P]), "error"), ("trained_solver", (Rp, Ep), "error")]
    if P > 0 and n > P and getattr(a, "learn_solver_only", False):
        sets.append(("trained_solver_only", (Rp[P:], Ep[P:]), "error"))
    if getattr(a, "learn_residual", False):
        # the residual-space loss ||r - A M r||^2 / ||r||^2 on the same pair sets
        sets += [("trained_gauss_residual", (Rp[:P], Ep[:P]), "residual")]
        if n > P:
            sets.append(("trained_solver_residual", (Rp[P:], Ep[P:]), "residual"))
    for name, (r, e), loss in sets:
        if (name == "trained_solver" and r.shape[0] == P) or r.shape[0] == 0:
            continue
        ctx.set_learned(thetas["neumann3"])
        t0 = time.time()
        hist = ctx.learned_train(r, e, L, steps=a.learn_steps, lr=a.learn_lr, loss=loss)
        torch.cuda.synchronize()
        nb = min(r.shape[0] // L, len(hist))  # batches cycle, so compare whole passes over the pairs
        out[name] = {"pairs": int(r.shape[0]), "steps": a.learn_steps, "lr": a.learn_lr, "loss": loss,
                     "seconds": round(time.time() - t0, 3),
                     "loss_first_pass": float(np.mean(hist[:nb])), "loss_last_pass": float(np.mean(hist[-nb:]))}
        thetas[name] = ctx.get_learned()
    print(f"[bench] learned setup: {out}", file=sys.stderr, flush=True)
    del Ep, Rp, Z
    return out, thetas


def learned_solves(ctx, torch, np, B, L, w, a, thetas, Xref):
    """Solves with the learned M (Neumann start and trained weights) in FP64 and FP32; FP64
    Jacobi j = a.j is the fallback of the FP32 form."""
    from paper_0907_3261_amd import WD_PRECOND_LEARNED
    out = {}
    legs = [("neumann3", thetas["neumann3"], "f64"), ("neumann3", thetas["neumann3"], "f32")]
    legs += [(k, thetas[k], p) for k in ("trained_gauss", "trained_solver", "trained_solver_only",
                                         "trained_gauss_residual", "trained_solver_residual")
             if thetas.get(k) is not None for p in a.learn_prec.split(",")]
    for name, th, prec in legs:
        if th is None:
            continue
        ctx.set_learned(th)
        torch.cuda.synchronize()
        X, info = ctx.solve(B, tol=w["tol"], j=a.j, precond=WD_PRECOND_LEARNED, prec_inner=prec)
        torch.cuda.synchronize()
        out[f"learned_{name}_{prec}"] = solve_record(info, L, X, Xref, torch, np)
        print(f"[bench] learned {name} {prec}: {out[f'learned_{name}_{prec}']}", file=sys.stderr, flush=True)
    return out


def ensemble_sweep(pkg, wi, torch, np, w, a, kappa, L, V, B):
    """Every preconditioner precision on a.ensembles link ensembles (seeds link_seed + e) with
    the workload's sources, at kappa and a.kappa_heavy, as the paper averages over gauge
    configurations (Tables 1 and 2): per precision the number of runs that reach the FP64 1e-12
    true residual and the mean iterations and seconds per RHS over those."""
    from paper_0907_3261_amd import WD_PRECOND_LEARNED
    modes = [("jacobi_f64", "f64", None), ("jacobi_f32", "f32", None), ("jacobi_bf16", "bf16", None),
             ("jacobi_f64c32", "f64c32", None), ("jacobi_f64cbf16", "f64cbf16", None),
             ("learned_neumann_f64", "f64", WD_PRECOND_LEARNED), ("learned_neumann_f32", "f32", WD_PRECOND_LEARNED)]
    runs = {}
    for e in range(a.ensembles):
        U = wi.random_links(w["dims"], w["eps"], w["link_seed"] + e)
        ctx = pkg.Context(w["dims"], bc_t=w["bc_t"], max_L=L)
        ctx.set_links(U)
        del U
        for kp in [kappa] + ([a.kappa_heavy] if a.kappa_heavy > 0 else []):
            ctx.set_params(kp, w["csw"])
            ctx.learned_init("neumann")
            k64 = 0
            for name, prec, pc in modes:
                kw = dict(precond=pc) if pc is not None else {}
                if prec.startswith("f64c"):
                    kw.update(max_iter=3 * k64 // 2 + 10, max_restarts=0)
                X, info = ctx.solve(B, tol=w["tol"], j=a.j, prec_inner=prec, **kw)
                ok = info["status"] == "converged" and float(np.max(info["true_residual"])) <= w["tol"]
                if name == "jacobi_f64":
                    k64 = info["iterations"]
                runs.setdefault(f"kappa{kp}", {}).setdefault(name, []).append(
                    {"ensemble": e, "ok": bool(ok), "iterations": int(info["total_iterations"]),
                     "fallback": bool(info["fallback"]), "s_per_rhs": info["seconds"] / L})
                print(f"[bench] ensemble {e} kappa {kp} {name}: {info['status']} k={info['total_iterations']} "
                      f"{info['seconds'] / L:.4f} s/RHS", file=sys.stderr, flush=True)
                del X
        ctx.close()
        torch.cuda.empty_cache()
    summary = {}
    for kk, per in runs.items():
        summary[kk] = {}
        base = [r["s_per_rhs"] for r in per["jacobi_f64"] if r["ok"]]
        for name, rs in per.items():
            good = [r for r in rs if r["ok"]]
            rec = {"converged": f"{len(good)}/{len(rs)}", "fallbacks": sum(r["fallback"] for r in rs)}
            if good:
                rec["mean_iterations"] = round(float(np.mean([r["iterations"] for r in good])), 1)
                rec["mean_s_per_rhs"] = round(float(np.mean([r["s_per_rhs"] for r in good])), 5)
                if base:
                    rec["speedup_vs_f64_jacobi_mean"] = round(float(np.mean(base)) / rec["mean_s_per_rhs"], 3)
            summary[kk][name] = rec
    return {"ensembles": summary, "workload": a.workload, "L": L, "j": a.j, "runs": runs}


def c3_leg(pkg, wi, torch, np, a):
    """The learned-preconditioner workload at the paper's lattice size: 16^3 x 32, twelve point
    sources, the linear gauge-covariant M trained (500 Adam steps from the Neumann start) on about
    2000 residual/correction pairs that FP64 Jacobi(12) solves of the same system generate (every
    iterate of point-source and Z4-source solves), on 240 Gaussian pairs, and on both, with the
    error loss ||M r - e||^2 / ||e||^2 and with the residual loss ||r - A M r||^2 / ||r||^2,
    against Jacobi j = 12 in FP64.  Run at the workload's kappa (0.130: the nominal 0.135 is past the
    critical kappa of this ensemble) and at 0.120."""
    import argparse as ap
    w = wi.workload("lat16x32_point")
    L = 12
    V = wi.volume(w["dims"])
    U = wi.random_links(w["dims"], w["eps"], w["link_seed"])
    ctx = pkg.Context(w["dims"], bc_t=w["bc_t"], max_L=L)
    ctx.set_links(U)
    del U
    B = torch.from_numpy(wi.source_block("point", V, L, 0)).cuda()
    la = ap.Namespace(**vars(a))
    la.learn_pairs, la.learn_snaps, la.snap_every, la.learn_solves = 240, 40, 1, 8
    la.learn_solver_pairs, la.learn_steps, la.learn_lr, la.learn_prec = 2000, 500, 1e-3, "f64,f32"
    la.learn_solver_only, la.learn_residual, la.j = True, True, 12
    wl = dict(w, source_seed=w["source_seed"], tol=w["tol"])
    out = {"workload": "lat16x32_point", "L": L, "j": 12}
    for kp in (w["kappa_solve"], 0.12):
        ctx.set_params(kp, w["csw"])
        torch.cuda.synchronize()
        X, info = ctx.solve(B, tol=w["tol"], j=12)
        Xref = X.clone()
        leg = {"jacobi12_f64": solve_record(info, L, X, Xref, torch, np)}
        learned, thetas = learned_setup(ctx, torch, np, B, V, L, wl, la)
        leg.update(learned_solves(ctx, torch, np, B, L, wl, la, thetas, Xref))
        ref = leg["jacobi12_f64"]["s_per_rhs"]
        for rec in leg.values():
            if rec.get("status") == "converged":
                rec["speedup_vs_f64_jacobi"] = round(ref / rec["s_per_rhs"], 3)
        out[f"kappa{kp}"] = {"solves": leg, "training": learned}
        print(f"[bench] c3 kappa={kp}: {leg}", file=sys.stderr, flush=True)
        del X, Xref
        torch.cuda.empty_cache()
    ctx.close()
    return out


def conditioning_probe(pkg, wi, torch, np, kappas=(0.120, 0.127, 0.130, 0.135)):
    """How close each synthetic ensemble is to its critical kappa, the analogue of the paper's
    kappa against kappa_c (Sec. 3.1).  Per lattice and kappa:
      rho   spectral radius of E = kappa T^-1 H, the Jacobi iteration matrix of the block reading
            (the sweep with zero right-hand side applies exactly E), from 300 power steps on one
            column: the geometric mean of the last 100 norm ratios;
      eig   the four eigenvalues of A with the smallest real part (ARPACK 'SR' through scipy, the
            GPU operator as its matrix-vector product) on the smallest lattice, where the host side
            of ARPACK stays cheap."""
    import scipy.sparse.linalg as sla
    out = {}
    for name in ("lat8x16_L12_point", "lat16x32_point", "lat32x64_L12_point"):
        w = wi.workload(name)
        V = wi.volume(w["dims"])
        N = 12 * V
        U = wi.random_links(w["dims"], w["eps"], w["link_seed"])
        ctx = pkg.Context(w["dims"], bc_t=w["bc_t"], max_L=1)
        ctx.set_links(U)
        del U
        g = torch.Generator(device="cuda").manual_seed(21)
        X0 = torch.complex(torch.randn((1, 12, V), generator=g, device="cuda", dtype=torch.float64),
                           torch.randn((1, 12, V), generator=g, device="cuda", dtype=torch.float64))
        Z = torch.zeros_like(X0)
        Y = torch.empty_like(X0)
        for kp in kappas:
            ctx.set_params(kp, w["csw"])
            X = X0 / torch.linalg.vector_norm(X0)
            logs = []
            for _ in range(300):
                ctx.hop_repeat(X, Y, 1, mode=1, R=Z)
                nrm = float(torch.linalg.vector_norm(Y))
                logs.append(np.log(nrm))
                X = Y / nrm
            rec = {"rho_kappaTinvH": round(float(np.exp(np.mean(logs[-100:]))), 5)}
            if N <= 200_000:
                Xd = ctx.empty_block(1)
                Yd = ctx.empty_block(1)

                count = [0]

                def mv(v):
                    Xd.copy_(torch.from_numpy(np.ascontiguousarray(v.reshape(1, 12, V))))
                    ctx.apply(Xd, Yd)
                    count[0] += 1
                    if count[0] % 1000 == 0:
                        print(f"[bench] conditioning {name} kappa={kp}: {count[0]} products", file=sys.stderr,
                              flush=True)
                    return Yd.cpu().numpy().reshape(-1)

                Aop = sla.LinearOperator((N, N), matvec=mv, dtype=np.complex128)
                t0 = time.time()
                try:
                    ev = sla.eigs(Aop, k=4, which="SR", ncv=40, tol=1e-5, maxiter=2000,
                                  return_eigenvectors=False)
                    ev = np.sort_complex(ev)
                    rec["eig_smallest_real"] = [[round(float(e.real), 5), round(float(e.imag), 5)] for e in ev]
                    rec["min_re"] = round(float(ev.real.min()), 5)
                except sla.ArpackNoConvergence as e:
                    rec["eig_smallest_real"] = "ARPACK did not converge"
                rec["arpack_s"] = round(time.time() - t0, 1)
                rec["arpack_products"] = count[0]
            out[f"{name}_kappa{kp}"] = rec
            print(f"[bench] conditioning {name} kappa={kp}: {rec}", file=sys.stderr, flush=True)
        ctx.close()
        torch.cuda.empty_cache()
    return out


def cpu_baseline(w, kappa):
    """Oracle A X on a 32 x 32 x 32 x 2 slab of the workload's ensemble, twelve columns."""
    import numpy as np
    import wdinputs as wi
    from oracle import WilsonClover
    dims = (w["dims"][0], w["dims"][1], w["dims"][2], 2)
    U = wi.random_links(dims, w["eps"], w["link_seed"])
    op = WilsonClover(dims, U, kappa, w["csw"], bc_t=w["bc_t"])
    L = 12
    X = op.from_block(wi.gaussian_block(op.V, L, 3))
    reps = 3
    c0 = time.process_time()
    t0 = time.perf_counter()
    for _ in range(reps):
        op.apply_A(X)
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    gbs = reps * op.V * (1152 + 384 * L) / wall / 1e9
    try:
        from threadpoolctl import threadpool_info
        blas = {i.get("internal_api", "?"): i.get("num_threads") for i in threadpool_info()}
    except Exception:
        blas = None
    return {"value": round(gbs, 4), "unit": "GB/s", "cores": max(1, round(cpu / wall)), "kind": "oracle",
            "sample": f"{reps} FP64 applications of A (numpy oracle) on a {dims[0]}x{dims[1]}x{dims[2]}x{dims[3]} "
                      f"slab of the same link ensemble, L={L}, {wall:.1f} s wall; algorithmic bytes per "
                      f"site as for the GPU operator kernel",
            "host_cpus": len(os.sched_getaffinity(0)), "blas_threads": blas,
            "per_config": cpu_per_config()}


def cpu_per_config():
    """Oracle time of one application of A at the configurations small enough for the host: the
    4^4 dense-LU workload (L = 4), 8^3 x 16 (L = 12) and the paper's 16^3 x 32 at L = 1, 4 and 12
    (one sample each; numpy's elementwise work runs on one core)."""
    import numpy as np
    import wdinputs as wi
    from oracle import WilsonClover
    out = {}
    for name, Ls in (("lat4_L4_z4", (4,)), ("lat8x16_L12_point", (12,)), ("lat16x32_point", (1, 4, 12))):
        w = wi.workload(name)
        kappa = w.get("kappa_solve", w["kappa"])
        kappa = kappa[0] if isinstance(kappa, tuple) else kappa
        op = WilsonClover(w["dims"], wi.random_links(w["dims"], w["eps"], w["link_seed"]), kappa, w["csw"],
                          bc_t=w["bc_t"])
        for L in Ls:
            X = op.from_block(wi.gaussian_block(op.V, L, 3))
            t0 = time.perf_counter()
            op.apply_A(X)
            dt = time.perf_counter() - t0
            out[f"{name} L={L}"] = {"s_per_apply": round(dt, 4),
                                    "GBs": round(op.V * (1152 + 384 * L) / dt / 1e9, 4)}
        print(f"[bench] cpu baseline {name}: {[out[f'{name} L={L}'] for L in Ls]}", file=sys.stderr, flush=True)
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {a.gpus} is not supported by this build "
              "(the multi-GPU domain decomposition is a design, not code).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_0907_3261_amd as pkg
    import wdinputs as wi

    pkg.load()
    if a.conditioning:
        print(json.dumps({"conditioning": conditioning_probe(pkg, wi, torch, np)}), flush=True)
        return
    if a.learned_c3:
        print(json.dumps({"learned_c3": c3_leg(pkg, wi, torch, np, a)}), flush=True)
        return
    w = wi.workload(a.workload)
    # solves run at the workload's subcritical kappa_solve when its nominal kappa is past criticality
    kappa = a.kappa if a.kappa is not None else w.get("kappa_solve", w["kappa"])
    if isinstance(kappa, tuple):
        kappa = kappa[0]
    L = w["L"] if isinstance(w["L"], int) else max(w["L"])
    V = wi.volume(w["dims"])
    t_setup = time.time()
    U = wi.random_links(w["dims"], w["eps"], w["link_seed"])
    ctx = pkg.Context(w["dims"], bc_t=w["bc_t"], max_L=L)
    ctx.set_links(U)
    ctx.set_params(kappa, w["csw"])
    del U
    B = torch.from_numpy(wi.source_block(w["source"], V, L, w["source_seed"])).cuda()
    torch.cuda.synchronize()
    print(f"[bench] setup {time.time() - t_setup:.1f}s  workload {a.workload} V={V} L={L} kappa={kappa}",
          file=sys.stderr, flush=True)

    st = ctx.stream
    if a.j_sweep:
        out = {}
        for kp in [kappa] + ([a.kappa_heavy] if a.kappa_heavy > 0 else []):
            ctx.set_params(kp, w["csw"])
            for j in (0, 4, 8, 12, 16, 24):
                # one run per j (no block splitting), as the paper's Table 2 counts iterations
                X, info = ctx.solve(B, tol=w["tol"], j=j, max_iter=3000, no_split=True)
                out[f"kappa{kp}_j{j}"] = {"status": info["status"], "iterations": info["iterations"],
                                          "mvm_paper_per_col": int(info["mvm_paper"]),
                                          "s_per_rhs": round(info["seconds"] / L, 5),
                                          "true_residual_max": float(np.max(info["true_residual"]))}
                print(f"[bench] j-sweep kappa={kp} j={j}: {out[f'kappa{kp}_j{j}']}", file=sys.stderr, flush=True)
        print(json.dumps({"j_sweep": out, "workload": a.workload, "L": L}), flush=True)
        ctx.close()
        return
    if a.hop_sweep:
        # algorithmic GB/s of the two hop kernels per block width; per-application bytes below the
        # 256 MB Infinity Cache are flagged (those inputs can stay cache-resident between launches)
        out = {}
        for l in (1, 2, 3, 4, 6, 8, 12):
            if l > L:
                continue
            row = {}
            for mode, name, per_site in ((0, "apply", 1152 + 384 * l), (1, "sweep", 1152 + 576 * l)):
                ms = time_hop(ctx, torch, V, l, mode, a.hop_reps)
                b = V * per_site
                row[name] = {"ms": round(ms, 4), "GBs": round(b / (ms / 1e3) / 1e9, 1),
                             "frac": round(b / (ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4), "alg_bytes": b,
                             "fits_in_mall": b <= 256e6}
            out[f"L{l}"] = row
            print(f"[bench] hop sweep L={l}: {row}", file=sys.stderr, flush=True)
        print(json.dumps({"hop_sweep": out, "workload": a.workload,
                          "layout": "tiled" if V % 64 == 0 else "standard"}), flush=True)
        ctx.close()
        return
    if a.ensembles > 0:
        ctx.close()
        print(json.dumps(ensemble_sweep(pkg, wi, torch, np, w, a, kappa, L, V, B)), flush=True)
        return
    if a.kernels_only:
        ms_sweep = time_hop(ctx, torch, V, L, 1, a.hop_reps)
        ms_apply = time_hop(ctx, torch, V, L, 0, a.hop_reps)
        ms_lowp = {p: time_hop(ctx, torch, V, L, 1, a.hop_reps, p) for p in ("f32", "bf16", "f64c32", "f64cbf16")}
        X = torch.empty((L, 12, V), dtype=torch.complex128, device="cuda")
        Y = torch.empty_like(X)
        X.fill_(1.0)
        for _ in range(3):
            Y.copy_(X)
        # one application of the learned M (Neumann start) in each precision, for its layer kernels,
        # in the layout the solver runs in
        ctx.learned_init("neumann")
        ctx.set_layout("tiled" if V % 64 == 0 else "standard")
        for prec in ("f64", "f32"):
            ctx.learned_apply(X, Y, prec)
        ctx.set_layout("standard")
        torch.cuda.synchronize()
        print(json.dumps({"sweep_ms": ms_sweep, "apply_ms": ms_apply, "sweep_lowp_ms": ms_lowp,
                          "copy_bytes_read": X.numel() * 16,
                          "src_hash": src_hash()}), flush=True)
        ctx.close()
        return
    for i in range(a.warmup):
        X, info = ctx.solve(B, tol=w["tol"], j=a.j)
        print(f"[bench] warmup {i}: {info['status']} k={info['iterations']} {info['seconds']:.2f}s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    infos = []
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for i in range(a.steps):
        X, info = ctx.solve(B, tol=w["tol"], j=a.j)
        infos.append(info)
        print(f"[bench] step {i}: {info['status']} k={info['iterations']} {info['seconds']:.2f}s", file=sys.stderr,
              flush=True)
    e1.record(st)
    e1.synchronize()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ok = all(i["status"] == "converged" and float(np.max(i["true_residual"])) <= w["tol"] for i in infos)
    bytes_total = sum(i["bytes_alg"] for i in infos)
    value = bytes_total / (ms / 1e3) / 1e9
    ms_step = ms / a.steps

    # dominant kernel: the Jacobi sweep; also the operator kernel
    ms_sweep = time_hop(ctx, torch, V, L, 1, a.hop_reps)
    ms_apply = time_hop(ctx, torch, V, L, 0, a.hop_reps)
    # the same kernels on block vectors in the standard layout (wd_apply / jacobi_precond of a
    # caller who keeps it), for comparison
    ms_sweep_std = time_hop(ctx, torch, V, L, 1, a.hop_reps, layout="standard")
    ms_apply_std = time_hop(ctx, torch, V, L, 0, a.hop_reps, layout="standard")
    b_sweep = V * (1152 + 576 * L)
    b_apply = V * (1152 + 384 * L)
    ach = b_sweep / (ms_sweep / 1e3) / 1e9
    copy_gbs = time_copy(torch, V, L)
    roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic_from_profiles(1),
            "kernel": (f"k_hop_f64<JBLOCK, time-diagonal in and out> (middle Jacobi sweep, L={L})" if L >= 3 else f"k_hop<StF64,StF64,CT,JBLOCK> (Jacobi sweep, L={L})"),
            "layout": "tiled" if V % 64 == 0 else "standard",
            "copy_GBs": round(copy_gbs, 1), "frac_of_copy": round(ach / copy_gbs, 4),
            "avg_launch_ms": round(ms_sweep, 4), "alg_bytes_per_launch": b_sweep,
            "standard_layout": {"avg_launch_ms": round(ms_sweep_std, 4),
                                "frac": round(b_sweep / (ms_sweep_std / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}}
    ach_a = b_apply / (ms_apply / 1e3) / 1e9
    dslash = {"achieved": round(ach_a, 1), "frac": round(ach_a / HBM_PEAK_GBS, 4), "unit": "GB/s",
              "avg_launch_ms": round(ms_apply, 4), "alg_bytes_per_launch": b_apply,
              "layout": "tiled" if V % 64 == 0 else "standard",
              "traffic": traffic_from_profiles(0),
              "standard_layout": {"avg_launch_ms": round(ms_apply_std, 4),
                                  "frac": round(b_apply / (ms_apply_std / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}}

    # time to solution per right-hand side: FP64 Jacobi (the plain form), low-precision Jacobi,
    # learned M, at the workload's kappa and at a heavier quark mass (kappa_heavy)
    # the low-precision sweep of the mixed-precision Jacobi (FP32 accumulate)
    lowp = {}
    # FP32 / BF16 links are stored as two rows (192 / 96 B per site), T^-1 in full (288 / 144 B)
    for prec, per_site in (("f32", 480 + 288 * L), ("bf16", 240 + 144 * L),
                           ("f64c32", 480 + 576 * L), ("f64cbf16", 240 + 576 * L)):
        ms_p = time_hop(ctx, torch, V, L, 1, a.hop_reps, prec)
        b_p = V * per_site
        lowp[prec] = {"avg_launch_ms": round(ms_p, 4), "alg_bytes_per_launch": b_p,
                      "achieved": round(b_p / (ms_p / 1e3) / 1e9, 1), "frac": round(b_p / (ms_p / 1e3) / 1e9 / HBM_PEAK_GBS, 4)}
    print(f"[bench] low-precision sweeps: {lowp}", file=sys.stderr, flush=True)

    solves, learned, thetas = {}, None, None
    kappas = [kappa] + ([a.kappa_heavy] if a.kappa_heavy > 0 else [])
    if not a.no_learned:
        learned, thetas = learned_setup(ctx, torch, np, B, V, L, w, a)
    if not a.no_compare:
        for kp in kappas:
            ctx.set_params(kp, w["csw"])
            leg, Xref = compare_leg(ctx, torch, np, B, L, w, a)
            if thetas is not None:
                th = thetas
                if kp != kappa:  # the Neumann start for this kappa; the weights were trained at the other
                    ctx.learned_init("neumann")
                    th = {"neumann3": ctx.get_learned()}
                leg.update(learned_solves(ctx, torch, np, B, L, w, a, th, Xref))
            ref = leg.get(f"jacobi{a.j}_f64", {}).get("s_per_rhs")
            for rec in leg.values():     # time-to-solution ratio against the plain FP64 Jacobi form
                if ref and rec.get("status") == "converged":
                    rec["speedup_vs_f64_jacobi"] = round(ref / rec["s_per_rhs"], 3)
            solves[f"kappa{kp}"] = leg
        ctx.set_params(kappa, w["csw"])

    cpu = None if a.no_cpu_baseline else cpu_baseline(w, kappa)
    ctx.close()
    line = {
        "metric": "Dslash GB/s (%HBM peak); s/RHS to 1e-12, mixed+learned vs FP64 plain",
        "value": dslash["achieved"], "unit": "GB/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": round(ms_step, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": a.workload, "dims": list(w["dims"]), "L": L, "kappa": kappa, "csw": w["csw"],
                   "eps": w["eps"], "sources": w["source"], "j": a.j, "tol": w["tol"],
                   "step": "one complete solve of the L right-hand sides"},
        "pct_hbm_peak": round(dslash["achieved"] / HBM_PEAK_GBS * 100, 2),
        "value_is": "algorithmic GB/s of the operator kernel Y = A X (FP64, L columns), HIP events over "
                    "back-to-back launches on the library stream",
        "solve_GBs": round(value, 1),
        "solve_GBs_is": "algorithmic HBM bytes of every kernel the timed solves launched / their time",
        "s_per_rhs": round(ms_step / 1e3 / L, 5),
        "converged": ok,
        "iterations": [i["iterations"] for i in infos],
        "roofline": roof, "dslash": dslash, "sweep_lowp": lowp, "solves": solves, "learned": learned, "cpu_baseline": cpu,
        "src_hash": src_hash(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
