"""Benchmark of the helical-wave Hamiltonian apply on one MI355X.

    python bench.py [--gpus 1] [--steps 20] [--warmup 30] [--workload nanowire-ecut30]

One step applies H to a block of 64 coefficient vectors of the largest
single-GPU workload (the filled nanowire, 88,951 basis functions): the whole
H*X path -- radial inverse GEMMs, angular inverse DFT / potential / forward
DFT per radius, radial forward GEMMs with the kinetic diagonal.  The block,
the potential and every table are resident in HBM before timing starts.
Rank 0 prints one JSON line with the throughput in vector applications per
second, the roofline position of the dominant kernel, the time to the lowest
eigenpairs in FP64 and along the BF16 / FP32 -> FP64 ladders on the 40 Ha
nanotube (200 pairs, per-eigenvalue errors before and after refinement), the
learned preconditioner against the plain one on the nanowire (400 pairs),
the batched Bloch-parameter solves of all eight seeded structures, and the
CPU oracle's throughput on a bounded sample of the headline workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "H·X vec-applies/s (64-vec block) + time-to-n-eigenpairs, mixed vs FP64 @1e-8Ha"
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector and FP64 matrix (dense)
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X FP32 matrix (dense)
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, published (packed FP32 counted; these kernels issue none)
BF16_MFMA_PEAK_TFLOPS = 2500.0 # MI355X BF16 matrix (dense)
STAGES = ("k_radial_inverse", "k_angular", "k_radial_forward")
KERNEL_SOURCES = ("paper_2210_12252_amd/csrc/kernels.hpp", "paper_2210_12252_amd/csrc/angular_fast.hpp",
                  "paper_2210_12252_amd/csrc/angular_split.hpp", "paper_2210_12252_amd/csrc/angular_pipe.hpp",
                  "paper_2210_12252_amd/csrc/radial_bf16.hpp",
                  "paper_2210_12252_amd/csrc/device.hip")


LOG_EVERY = 50   # eigensolver progress line (stderr) every this many iterations
PROFILE_EVERY = 10   # timed steps with per-kernel events: one in this many


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_counts(L, n_modes, n1, n2, n_r, nvec, elem):
    """Algorithmic flops and HBM bytes per launch of each stage kernel.

    Radial stages: 4 real flops per (coefficient, radius) pair (real table
    times complex value); bytes = coefficients in (16 B each, complex double)
    plus mode values out (2 * elem B each), the kinetic stage also reading X
    and writing Y.  Angular stage: nominal 5 N log2 N flops per complex 2D
    DFT of N = n1 * n2 points, two per slab, plus 2 N for the real potential;
    bytes = mode values in and out (2 * 2 * elem B each) plus the potential
    once (elem B per grid point)."""
    N = n1 * n2
    slabs = nvec * n_r
    modes_bytes = 2 * elem * n_r * n_modes * nvec
    inv = dict(flops=4.0 * n_r * L * nvec, bytes=16.0 * L * nvec + modes_bytes)
    ang = dict(flops=slabs * (2 * 5.0 * N * math.log2(N) + 2.0 * N),
               bytes=2.0 * modes_bytes + elem * N * n_r)
    fwd = dict(flops=4.0 * n_r * L * nvec + 2.0 * L * nvec, bytes=modes_bytes + 32.0 * L * nvec)
    return dict(zip(STAGES, (inv, ang, fwd)))


_CPU = {}


def _cpu_init(o, V):
    _CPU["o"], _CPU["V"] = o, V


def _cpu_apply(X):
    """Oracle H*X of one column slice (runs in a worker process)."""
    from oracle import hamiltonian as oh
    return oh.apply(_CPU["o"], _CPU["V"], X)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def host_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(w, nsample: int):
    """The CPU oracle's matrix-free H*X (unchanged, FP64 NumPy) on `nsample`
    vectors of the same workload, timed on the host: the columns are split
    over one worker process per available host core (at most 16), each
    running the oracle on its slice."""
    import concurrent.futures as cf
    import multiprocessing as mp

    import numpy as np

    import synth
    from oracle import basis as ob
    o = ob.basis_for(w)
    atoms = synth.atoms_for(w.structure, w.seed, w.tau, w.R)
    V = synth.potential_at(o.theta1, o.theta2, o.r, w.tau, w.alpha, atoms)
    X = synth.random_block(o.mnk, nsample, 1234)
    nw = min(host_cores(), nsample)
    slices = [X[:, i::nw] for i in range(nw)]
    with cf.ProcessPoolExecutor(nw, mp_context=mp.get_context("spawn"), initializer=_cpu_init,
                                initargs=(o, V)) as ex:
        list(ex.map(_cpu_apply, [s[:, :1] for s in slices]))   # workers started and warm
        t0 = time.perf_counter()
        Ys = list(ex.map(_cpu_apply, slices))
        wall = time.perf_counter() - t0
    assert all(np.all(np.isfinite(Y)) for Y in Ys)
    return dict(value=nsample / wall, unit="vec-applies/s", cores=nw, kind="oracle",
                sample=f"matrix-free oracle H*X (explicit DFT sums, FP64 NumPy) on {nsample} of the 64 block "
                f"vectors of {w.name}, one worker process per core, {wall:.1f} s wall",
                cpu_model=cpu_model(), nproc=os.cpu_count())


def _solve_record(st, status, res, wall):
    import numpy as np
    return dict(seconds=round(wall, 3), converged=bool(status == 0), iters=st["iters"], iters_low=st["iters_low"],
                iters_bf16=st["iters_bf16"], hx_columns=st["n_apply"], hx_s=round(st["t_apply_ms"] / 1e3, 3),
                rayleigh_ritz_s=round(st["t_rr_ms"] / 1e3, 3), max_resid=float(np.max(res)))


def time_to_eigenpairs(b, w, torch, tol=1e-8, solvers=("lobpcg", "chefsi"), table=None):
    """Lowest w.nev eigenpairs to ||H x - lambda x|| <= tol from the same
    seeded random start, by LOBPCG (TPA preconditioner) and by
    Chebyshev-filtered subspace iteration, each with FP64 H*X and along the
    precision ladders FP32 -> FP64 and BF16 -> FP32 -> FP64; all keep the
    FP64 Rayleigh-Ritz.  The filtered solver also runs each ladder stopped at
    its first switch (the low-precision result before refinement).  Reports
    wall time, iterations (outer filter steps for the latter), the H*X and
    Rayleigh-Ritz shares and the eigenvalue errors against the FP64 solve of
    the same solver; `table` (a path) receives the per-eigenvalue errors."""
    import numpy as np
    out = {"workload": w.name, "L": b.L, "nev": w.nev, "tol_Ha": tol}
    evs = {}
    b.eigensolve_ex(4, tol=1e-3, maxit=2)
    b.eigensolve_ex(4, tol=1e-3, maxit=1, cheb_degree=2)
    runs = []
    for solver in solvers:
        deg = None if solver == "lobpcg" else 0
        for prec in ("fp64", "fp32", "bf16"):
            runs.append((solver, deg, prec, f"{solver}_{prec}" if prec == "fp64" else f"{solver}_{prec}_ladder", False))
    if "chefsi" in solvers:
        for prec in ("fp32", "bf16"):
            runs.append(("chefsi", 0, prec, f"chefsi_{prec}_before_refinement", True))
    for solver, deg, prec, key, low in runs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, res, st, status = b.eigensolve_ex(w.nev, block=64, tol=tol, maxit=1000 if deg is None else 200,
                                              prec=prec, seed=7, log_every=LOG_EVERY, cheb_degree=deg,
                                              stop_low=low)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[key] = _solve_record(st, status, res, wall)
        evs[key] = ev
        print(f"[bench] eigensolve {key}: {wall:.2f} s, {st['iters']} iterations, converged {status == 0}",
              file=sys.stderr, flush=True)
    for solver in solvers:
        ref = evs[f"{solver}_fp64"]
        for prec in ("fp32", "bf16"):
            key = f"{solver}_{prec}_ladder"
            out[key]["max_abs_dlambda_vs_fp64_Ha"] = float(np.max(np.abs(evs[key] - ref)))
            out[key]["speedup_vs_fp64"] = round(out[f"{solver}_fp64"]["seconds"] / out[key]["seconds"], 3)
    if "lobpcg" in solvers and "chefsi" in solvers:
        out["chefsi_vs_lobpcg_max_abs_Ha"] = float(np.max(np.abs(evs["chefsi_fp64"] - evs["lobpcg_fp64"])))
        out["speedup_chefsi_vs_lobpcg_fp64"] = round(out["lobpcg_fp64"]["seconds"] / out["chefsi_fp64"]["seconds"], 3)
    if "chefsi" in solvers:
        ref = evs["chefsi_fp64"]
        per = {}
        for prec in ("fp32", "bf16"):
            before = np.abs(evs[f"chefsi_{prec}_before_refinement"] - ref)
            after = np.abs(evs[f"chefsi_{prec}_ladder"] - ref)
            per[prec] = {"before_refinement": dict(max=float(before.max()), median=float(np.median(before))),
                         "after_refinement": dict(max=float(after.max()), median=float(np.median(after)))}
        out["per_eigenvalue_error_vs_fp64_Ha"] = per
        if table:
            with open(table, "w") as fh:
                fh.write(f"# Per-eigenvalue error of the low-precision ladders, {w.name} (L = {b.L}), lowest "
                         f"{w.nev}\n\n")
                fh.write("Filtered subspace iteration from the same seeded start; |lambda - lambda_FP64| in Ha "
                         "against its FP64 solve (tol 1e-8).  'before': the ladder stopped at its first "
                         "precision switch (FP32: residual <= 1e-5, BF16: <= 1e-2); 'after': refined to 1e-8 in "
                         "FP64.\n\n")
                fh.write("Command: `python bench.py --eig-table <this file>` (the eigensolve leg).\n\n")
                fh.write("| j | lambda_FP64 (Ha) | FP32 before | FP32 after | BF16 before | BF16 after |\n")
                fh.write("|---:|---:|---:|---:|---:|---:|\n")
                for j in range(w.nev):
                    fh.write(f"| {j} | {ref[j]:.10f} | "
                             f"{abs(evs['chefsi_fp32_before_refinement'][j] - ref[j]):.2e} | "
                             f"{abs(evs['chefsi_fp32_ladder'][j] - ref[j]):.2e} | "
                             f"{abs(evs['chefsi_bf16_before_refinement'][j] - ref[j]):.2e} | "
                             f"{abs(evs['chefsi_bf16_ladder'][j] - ref[j]):.2e} |\n")
    return out


def density_leg(b, w, torch, nstates=None, reps=5):
    """Electron density (Sec. 4.2) of nstates (default: the solve's nev)
    normalised synthetic states with occupation 2, resident in HBM: wall time
    of helic_density (inverse transforms to the grid plus the weighted
    |phi|^2 accumulation) and its integral against 2 * nstates."""
    import numpy as np
    import synth
    n = nstates or w.nev
    mnk, _ = b.indices()
    X = torch.from_numpy(np.ascontiguousarray(synth.random_block(mnk, n, 41).T)).cuda()
    X /= torch.linalg.vector_norm(X, dim=1, keepdim=True)
    t1, t2, r, wts = b.grid()
    rho = torch.empty(len(t1) * len(t2) * len(r), dtype=torch.float64, device="cuda")
    occ = np.full(n, 2.0)
    b.density(X, occ, rho)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.density(X, occ, rho)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    # weight of a grid point: 2 pi tau / (N_theta1 N_theta2) (cyclic order 1) times omega_r = R^2 w_r
    cell = 2.0 * np.pi * w.tau / (len(t1) * len(t2)) * w.R ** 2 * wts
    W = torch.from_numpy(np.ascontiguousarray(np.broadcast_to(cell, (len(t1), len(t2), len(r))).reshape(-1))).cuda()
    integral = float((W * rho).sum())
    return dict(states=n, occupation=2.0, ms=round(1e3 * dt, 3), states_per_s=round(n / dt, 1),
                integral=integral, integral_rel_err=abs(integral - 2.0 * n) / (2.0 * n))


# Angular-stage kernel the library selects for a grid (its variant tables:
# convolution kernel for theta2 sizes 16, 64, 81; register-FFT kernel for the
# listed (theta1, theta2) grids; the general LDS FFT otherwise).
CONV_N2 = (16, 64, 81)
REGFFT_GRIDS = ((20, 96), (20, 120), (24, 120), (24, 135), (27, 144), (27, 180))


def angular_kernel_name(n1, n2):
    if n2 in CONV_N2:
        return "convolution"
    return "register-fft" if (n1, n2) in REGFFT_GRIDS else "general"


def batched_leg(torch, structures, nvec=8, steps=20, nev=60, tol=1e-8, extra=False, eig_every=8, prec="fp32"):
    """Many Bloch parameters of seeded structures (64 eta each, R ~ U[5, 12],
    E_cut ~ U[15, 35]), all in ONE batch: per structure a common grid (the
    largest automatic grid over its eta), so the batch holds one class per
    structure grid.  The batch is tuned per class (choices recorded),
    captured in one HIP graph and replayed (FP64; BF16 eager), and the lowest
    `nev` eigenpairs of every problem are solved by Chebyshev-filtered
    subspace iteration along the FP32 -> FP64 ladder with time-reversal
    halving of the eta points, concurrently on 8 streams.  With `extra`, every
    `eig_every`-th problem of each structure is also solved by FP64 LOBPCG with
    the plain and with a learned preconditioner (trained on another eta of
    the structure)."""
    import concurrent.futures as cf

    import numpy as np

    import synth
    from synth.configs import batched_problems
    from paper_2210_12252_amd import helic
    allp = batched_problems()
    t0 = time.perf_counter()
    bases, per = [], []
    for s in structures:
        probs = allp[64 * s: 64 * (s + 1)]
        with cf.ThreadPoolExecutor(8) as ex:
            auto = list(ex.map(lambda w: helic.Basis.from_workload(w), probs))
        n1 = max(b.n_t1 for b in auto)
        n2 = max(b.n_t2 for b in auto)
        nr = max(b.n_r for b in auto)
        for b in auto:
            b.close()
        grid_w = [w.with_(n_t1=n1, n_t2=n2, n_r=nr, m_max=(n1 - 1) // 2, n_max=(n2 - 1) // 2) for w in probs]
        with cf.ThreadPoolExecutor(8) as ex:
            sb = list(ex.map(lambda w: helic.Basis.from_workload(w), grid_w))
        t1, t2, r, _ = sb[0].grid()
        w0 = probs[0]
        V = torch.from_numpy(synth.potential_at(t1, t2, r, w0.tau, w0.alpha,
                                                synth.atoms_for(w0.structure, w0.seed, w0.tau, w0.R))).cuda()
        for b in sb:
            b.set_potential(V)
        Ls = [b.L for b in sb]
        per.append(dict(structure=s, R=round(w0.R, 3), ecut=round(w0.ecut, 3), n_eta=len(probs),
                        grid=f"{n1}x{n2}x{nr}", L_min=int(min(Ls)), L_max=int(max(Ls)),
                        kernel=angular_kernel_name(n1, n2), first=len(bases)))
        bases += sb
    batch = helic.Batch(bases)
    setup = time.perf_counter() - t0
    nclass, _ = batch.classes()
    total = nvec * int(batch.offsets[-1])
    X = torch.randn(total, dtype=torch.complex128, device="cuda")
    Y = torch.zeros_like(X)
    tuning = batch.tune_classes(X, Y, nvec)
    batch.capture(X, Y, nvec)
    batch.replay()
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(steps):
        batch.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - ta) / steps
    batch.apply(X, Y, nvec, prec="bf16")
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(steps):
        batch.apply(X, Y, nvec, prec="bf16")
    torch.cuda.synchronize()
    dt16 = (time.perf_counter() - ta) / steps
    del X, Y
    out = dict(problems=len(bases), structures=list(structures), classes=nclass, setup_s=round(setup, 2),
               tuning=tuning, ms_per_batched_apply=round(1e3 * dt, 3),
               vec_applies_per_s=round(len(bases) * nvec / dt, 1), bf16_ms_per_batched_apply=round(1e3 * dt16, 3),
               bf16_vec_applies_per_s=round(len(bases) * nvec / dt16, 1))
    # every problem: filtered solver, precision ladder from `prec`, time-reversal halving
    npairs = batch.time_reversal(True)
    torch.cuda.synchronize()
    te = time.perf_counter()
    ev, res, st, status = batch.eigensolve(nev, nstreams=8, tol=tol, maxit=200, cheb_degree=0, prec=prec)
    te = time.perf_counter() - te
    batch.time_reversal(False)
    ladder = {"fp64": "fp64", "fp32": "fp32 -> fp64 ladder", "bf16": "bf16 -> fp32 -> fp64 ladder"}[prec]
    out.update(eig_problems=len(bases), eig_nev=nev, eig_prec=ladder, time_reversal_pairs=npairs,
               eig_seconds=round(te, 2), eig_converged=int(np.sum(status == 0)), eig_max_resid=float(res.max()))
    for rec in per:
        a = rec.pop("first")
        sl = slice(a, a + rec["n_eta"])
        rec.update(eig_converged=int(np.sum(status[sl] == 0)), eig_max_resid=float(res[sl].max()),
                   eig_steps_mean=float(np.mean([x["iters"] for x in st[sl] if x["iters"] > 0])),
                   eig_solve_s=round(sum(x["t_total_ms"] for x in st[sl]) / 1e3, 2))
        if extra:
            sub = bases[a: a + rec["n_eta"]: eig_every]
            eb = helic.Batch(sub)
            tl = time.perf_counter()
            evl, _, _, statusl = eb.eigensolve(nev, nstreams=8, tol=tol, maxit=1000)
            tl = time.perf_counter() - tl
            rec.update(lobpcg_problems=len(sub), lobpcg_seconds=round(tl, 2),
                       lobpcg_converged=int(np.sum(statusl == 0)),
                       lobpcg_max_abs_dlambda=float(np.max(np.abs(evl - ev[sl][::eig_every]))))
            tb = bases[a + eig_every // 2]
            tl = time.perf_counter()
            Rh, Th, lh, ncol, _ = tb.lpc_harvest(nev, n_snap=12, tol=tol, maxit=1000, seed=3)
            net = helic.Lpc(seed=0)
            tb.lpc_train(net, Rh, Th, lh, ncol, batch=min(16, ncol), steps=400, lr=3e-3, seed=0)
            torch.cuda.synchronize()
            tl = time.perf_counter() - tl
            del Rh, Th, lh
            for sb in sub:
                sb.attach(net)
            te2 = time.perf_counter()
            evn, _, _, statusn = eb.eigensolve(nev, nstreams=8, tol=tol, maxit=1000, precond="learned")
            te2 = time.perf_counter() - te2
            for sb in sub:
                sb.attach(None)
            net.close()
            eb.close()
            rec.update(learned_train_s=round(tl, 2), learned_seconds=round(te2, 2),
                       learned_converged=int(np.sum(statusn == 0)),
                       learned_max_abs_dlambda=float(np.max(np.abs(evn - ev[sl][::eig_every]))))
        print(f"[bench] batched structure {rec['structure']}: {rec}", file=sys.stderr, flush=True)
    out["per_structure"] = per
    print(f"[bench] batched: {len(bases)} problems in {nclass} classes, {1e3 * dt:.2f} ms per replay, "
          f"eigensolve {te:.2f} s, converged {out['eig_converged']}", file=sys.stderr, flush=True)
    batch.close()
    for b in bases:
        b.close()
    return out


def learned_leg(torch, b, w, tol=1e-8, train_eta=0.25, n_snap=12, steps=400, batch=16, lr=3e-3):
    """Learned preconditioner against the plain one at equal residual: the
    network is trained on pairs harvested from one solve at another Bloch
    parameter (eta = train_eta) of the same structure, then both solve the
    benchmark problem `b` from the same seeded start."""
    import numpy as np

    import synth
    from paper_2210_12252_amd import helic
    wt = w.with_(name=f"{w.name}-eta{train_eta}", eta=train_eta)
    bt = helic.Basis.from_workload(wt)
    t1, t2, r, _ = bt.grid()
    atoms = synth.atoms_for(wt.structure, wt.seed, wt.tau, wt.R)
    bt.set_potential(torch.from_numpy(synth.potential_at(t1, t2, r, wt.tau, wt.alpha, atoms)).cuda())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    R, T, lam, ncol, hst = bt.lpc_harvest(w.nev, n_snap=n_snap, tol=tol, maxit=1000, seed=3, log_every=LOG_EVERY)
    torch.cuda.synchronize()
    t_h = time.perf_counter() - t0
    net = helic.Lpc(seed=0)
    t0 = time.perf_counter()
    losses = bt.lpc_train(net, R, T, lam, ncol, batch=min(batch, ncol), steps=steps, lr=lr, seed=0)
    torch.cuda.synchronize()
    t_t = time.perf_counter() - t0
    print(f"[bench] learned: harvested {ncol} pairs in {t_h:.2f} s, trained {steps} steps in {t_t:.2f} s, "
          f"loss {losses[:10].mean():.4f} -> {losses[-20:].mean():.4f}", file=sys.stderr, flush=True)
    del R, T, lam
    bt.close()
    b.attach(net)
    out = dict(workload=w.name, train_problem=wt.name, harvest_pairs=ncol, harvest_seconds=round(t_h, 2),
               train_steps=steps, train_batch_columns=min(batch, ncol), train_seconds=round(t_t, 2),
               ms_per_train_step=round(1e3 * t_t / max(steps, 1), 3),
               loss_first=round(float(losses[:10].mean()), 4), loss_last=round(float(losses[-20:].mean()), 4),
               tol_Ha=tol, nev=w.nev)
    evs = {}
    for pc in ("tpa", "learned"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, res, st, status = b.eigensolve_ex(w.nev, tol=tol, maxit=1000, precond=pc, seed=7, log_every=LOG_EVERY)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[pc] = dict(seconds=round(wall, 3), converged=bool(status == 0), iters=st["iters"],
                       fallback_iters=st["n_fallback"], precond_s=round(st["t_precond_ms"] / 1e3, 3),
                       max_resid=float(np.max(res)))
        evs[pc] = ev
        print(f"[bench] eigensolve precond={pc}: {wall:.2f} s, {st['iters']} iterations", file=sys.stderr,
              flush=True)
    b.attach(None)
    net.close()
    # the filtered solver on the same problem, for context (no preconditioner)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev, res, st, status = b.eigensolve_ex(w.nev, tol=tol, maxit=200, seed=7, cheb_degree=0)
    torch.cuda.synchronize()
    out["chefsi_fp64"] = _solve_record(st, status, res, time.perf_counter() - t0)
    out["chefsi_fp64"]["max_abs_dlambda_vs_tpa_Ha"] = float(np.max(np.abs(ev - evs["tpa"])))
    out["max_abs_dlambda_Ha"] = float(np.max(np.abs(evs["learned"] - evs["tpa"])))
    out["speedup_time"] = round(out["tpa"]["seconds"] / out["learned"]["seconds"], 3)
    out["iteration_ratio"] = round(out["learned"]["iters"] / max(out["tpa"]["iters"], 1), 3)
    return out


def measured_peaks(torch, dev, copy_mib=1024, n_gemm=8192, reps=5):
    """Attainable peaks on this GPU, next to the published ones: a plain
    device copy (STREAM-like; 2 x copy_mib MiB moved per copy) and a large
    FP64 GEMM on the matrix cores (rocBLAS through torch, 2 n^3 flops), each
    timed with events on torch's stream, best of `reps` after one warm-up."""
    n = copy_mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    a = torch.randn(n_gemm, n_gemm, dtype=torch.float64, device=dev)
    bm = torch.randn(n_gemm, n_gemm, dtype=torch.float64, device=dev)

    def best(fn):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            t.append(e0.elapsed_time(e1) * 1e-3)
        return min(t)

    t_copy = best(lambda: dst.copy_(src))
    t_gemm = best(lambda: torch.matmul(a, bm))
    out = dict(copy_GBs=round(2 * n * 8 / t_copy / 1e9, 1), copy_MiB=copy_mib,
               dgemm_TFLOPs=round(2 * n_gemm ** 3 / t_gemm / 1e12, 2), dgemm_n=n_gemm)
    del src, dst, a, bm
    torch.cuda.synchronize()
    return out


def load_traffic(name: str, nvec: int, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, or
    None when absent or taken on other kernel sources, block size or
    workload."""
    path = os.path.join(ROOT, "profiles", f"traffic_{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_hash") != kernel_hash() or t.get("nvec") != nvec or t.get("workload") != workload:
        return None
    return t


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--workload", default="nanowire-ecut30", help="headline H*X workload")
    ap.add_argument("--prec", default="fp64", choices=("fp64", "fp32", "bf16"))
    ap.add_argument("--cpu-sample", type=int, default=64, help="vectors for the CPU oracle leg (0: skip)")
    ap.add_argument("--eig", type=int, default=1, help="time-to-eigenpairs leg (0: skip)")
    ap.add_argument("--eig-workload", default="nanotube-ecut40",
                    help="workload of the time-to-eigenpairs leg (FP64 and the BF16 / FP32 ladders)")
    ap.add_argument("--eig-solvers", default="lobpcg,chefsi",
                    help="comma list of eigensolvers the eigensolve leg times (lobpcg, chefsi)")
    ap.add_argument("--eig-table", default="", help="write the per-eigenvalue error table to this path")
    ap.add_argument("--batched", default="all",
                    help="structures (0..7, comma list, 'all' or 'none') for the batched Bloch-parameter leg")
    ap.add_argument("--batched-prec", default="fp32", choices=("fp64", "fp32", "bf16"),
                    help="first rung of the batched leg's eigensolve ladder")
    ap.add_argument("--batched-extra", type=int, default=0,
                    help="batched leg: also LOBPCG and learned-preconditioner solves of every 8th eta")
    ap.add_argument("--learned", default="same",
                    help="learned-preconditioner leg: 'same' (the headline workload), a workload name, or 'none'")
    ap.add_argument("--density", type=int, default=1, help="electron-density leg (0: skip)")
    ap.add_argument("--other-precisions", type=int, default=1,
                    help="also time the headline block in the two other precisions")
    ap.add_argument("--measure-peaks", type=int, default=1,
                    help="time a 1 GiB device copy and an FP64 GEMM (attainable peaks; 0: skip)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this size (for counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library and this benchmark run on one GPU; the helical-wave solve would shard "
              "over Bloch parameters without communication, and no multi-GPU path is implemented.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import synth
    from paper_2210_12252_amd import helic

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")

    def load_problem(w):
        b = helic.Basis.from_workload(w)
        t1, t2, r, _ = b.grid()
        atoms = synth.atoms_for(w.structure, w.seed, w.tau, w.R)
        b.set_potential(torch.from_numpy(synth.potential_at(t1, t2, r, w.tau, w.alpha, atoms)).to(dev))
        return b

    w = synth.workload(args.workload)
    nvec = 64
    t_setup = time.perf_counter()
    b = load_problem(w)
    mnk, _ = b.indices()
    X = torch.from_numpy(np.ascontiguousarray(synth.random_block(mnk, nvec, 1234).T)).to(dev)
    Y = torch.empty_like(X)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    print(f"[bench] {w.name}: L={b.L} modes={b.n_modes} grid={b.n_t1}x{b.n_t2}x{b.n_r} "
          f"setup {t_setup:.2f} s", file=sys.stderr, flush=True)

    # the same block in the two other precisions, timed before the headline
    # (their applies also bring the clocks up before its warm-up steps)
    if args.other_precisions:
        other = {}
        for p in ("fp64", "fp32", "bf16"):
            if p == args.prec:
                continue
            for _ in range(3):
                b.apply_H(X, Y, prec=p)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            for _ in range(args.steps):
                b.apply_H(X, Y, prec=p)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - ta) / args.steps
            ms3, _ = b.profile_apply(X, Y, prec=p, nrep=3)
            other[p] = dict(ms_per_step=round(1e3 * dt, 4), vec_applies_per_s=round(nvec / dt, 1),
                            stages_ms={s: round(m, 4) for s, m in zip(STAGES, ms3)})
            print(f"[bench] {p}: {1e3 * dt:.3f} ms/step", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        b.apply_H(X, Y, prec=args.prec)
    torch.cuda.synchronize()
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # timed region: K steps bracketed by synchronisation on both sides.  Every
    # PROFILE_EVERY-th step runs with start and end events on each of its three
    # kernels (helic_profile_apply); the others run plain (helic_apply_H), so
    # the timestamps, which cost about 8 % per instrumented step, barely touch
    # the throughput while the stage durations are measured inside the region.
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_stage = np.zeros(3)
    ms_total = 0.0
    nprof = 0
    for k in range(args.steps):
        if k % PROFILE_EVERY == 0:
            ms, tot = b.profile_apply(X, Y, prec=args.prec, nrep=1)
            ms_stage += ms
            ms_total += tot
            nprof += 1
        else:
            b.apply_H(X, Y, prec=args.prec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_stage /= nprof
    ms_total /= nprof
    ms_per_step = 1e3 * wall / args.steps
    value = nvec * args.steps / wall
    print(f"[bench] {args.steps} steps: {ms_per_step:.3f} ms/step (events {ms_total:.3f} ms), stages "
          + ", ".join(f"{s} {m:.3f} ms" for s, m in zip(STAGES, ms_stage)), file=sys.stderr, flush=True)

    elem = {"fp64": 8, "fp32": 4, "bf16": 2}[args.prec]
    counts = algorithmic_counts(b.L, b.n_modes, b.n_t1, b.n_t2, b.n_r, nvec, elem)
    stage_info = {}
    for s, ms in zip(STAGES, ms_stage):
        c = counts[s]
        stage_info[s] = dict(ms=round(ms, 4), GBs=round(c["bytes"] / (ms * 1e-3) / 1e9, 1),
                             TFLOPs=round(c["flops"] / (ms * 1e-3) / 1e12, 2))
    dom = STAGES[int(np.argmax(ms_stage))]
    c = counts[dom]
    ms = float(np.max(ms_stage))
    intensity = c["flops"] / c["bytes"]
    if dom == "k_angular":
        peak_tf = FP64_PEAK_TFLOPS if elem == 8 else FP32_VALU_PEAK_TFLOPS
        compute_kind = "alu"
    else:
        peak_tf = FP64_PEAK_TFLOPS if elem == 8 else FP32_MFMA_PEAK_TFLOPS if elem == 4 else BF16_MFMA_PEAK_TFLOPS
        compute_kind = "mfma"
    ridge = peak_tf * 1e12 / (HBM_PEAK_GBS * 1e9)
    traffic = load_traffic(dom, nvec, w.name)
    if intensity >= ridge:
        achieved = c["flops"] / (ms * 1e-3) / 1e12
        roof = dict(bound=compute_kind, achieved=round(achieved, 3), peak=peak_tf, unit="TFLOP/s",
                    frac=round(achieved / peak_tf, 4))
    else:
        achieved = c["bytes"] / (ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4))
    roof["kernel"] = dom
    roof["traffic"] = None if traffic is None else traffic.get("bytes_per_launch")

    line = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "vec-applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[args.prec],
        "data": "synthetic",
        "config": {"workload": w.name, "L": b.L, "block": nvec, "grid": f"{b.n_t1}x{b.n_t2}x{b.n_r}",
                   "modes": b.n_modes, "R": w.R, "tau": w.tau, "alpha": round(w.alpha, 6), "ecut": w.ecut,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "stages": stage_info,
    }
    if args.other_precisions:
        line["hx_other_precisions"] = other
    if args.measure_peaks:
        mp = measured_peaks(torch, dev)
        if roof["unit"] == "GB/s":
            mp["dominant_frac_of_copy"] = round(roof["achieved"] / mp["copy_GBs"], 4)
        line["measured_peaks"] = mp
        print(f"[bench] measured peaks: {mp}", file=sys.stderr, flush=True)
    if args.learned != "none":
        if args.learned in ("same", w.name):
            lw, lb = w, b
        else:
            lw = synth.workload(args.learned)
            lb = load_problem(lw)
        line["learned_preconditioner"] = learned_leg(torch, lb, lw)
        if lb is not b:
            lb.close()
    if args.density:
        line["density"] = density_leg(b, w, torch)
    b.close()
    del X, Y
    if args.eig:
        ew = synth.workload(args.eig_workload)
        eb = load_problem(ew)
        line["eigensolve"] = time_to_eigenpairs(eb, ew, torch, solvers=tuple(args.eig_solvers.split(",")),
                                                table=args.eig_table or None)
        eb.close()
    if args.batched != "none":
        structs = list(range(8)) if args.batched == "all" else [int(x) for x in args.batched.split(",")]
        line["batched"] = batched_leg(torch, structs, extra=bool(args.batched_extra), prec=args.batched_prec)
    if args.cpu_sample > 0:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
