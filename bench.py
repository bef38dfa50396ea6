"""Benchmark of the helical-wave Hamiltonian apply on one MI355X.

    python bench.py [--gpus 1] [--steps 50] [--warmup 5] [--workload nanotube-ecut25]

One step applies H to a block of 64 coefficient vectors (the whole H*X path:
radial inverse GEMMs, angular inverse DFT / potential / forward DFT per
radius, radial forward GEMMs with the kinetic diagonal).  The block, the
potential and every table are resident in HBM before timing starts.  Rank 0
prints one JSON line with the throughput in vector applications per second,
the roofline position of the dominant kernel and the CPU oracle's throughput
on a bounded sample of the same workload.
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
STAGES = ("k_radial_inverse", "k_angular", "k_radial_forward")
KERNEL_SOURCES = ("paper_2210_12252_amd/csrc/kernels.hpp", "paper_2210_12252_amd/csrc/angular_fast.hpp",
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


def cpu_baseline(w, nsample: int):
    """The CPU oracle's matrix-free H*X on `nsample` vectors of the same
    workload, timed on the host."""
    import numpy as np

    import synth
    from oracle import basis as ob
    from oracle import hamiltonian as oh
    o = ob.basis_for(w)
    atoms = synth.atoms_for(w.structure, w.seed, w.tau, w.R)
    V = synth.potential_at(o.theta1, o.theta2, o.r, w.tau, w.alpha, atoms)
    X = synth.random_block(o.mnk, nsample, 1234)
    c0, t0 = time.process_time(), time.perf_counter()
    Y = oh.apply(o, V, X)
    wall = time.perf_counter() - t0
    cpu = time.process_time() - c0
    assert np.all(np.isfinite(Y))
    return dict(value=nsample / wall, unit="vec-applies/s", cores=max(1, round(cpu / wall)),
                kind="oracle", sample=f"matrix-free oracle H*X (explicit DFT sums, FP64) on {nsample} of the "
                f"64 block vectors of {w.name}, {wall:.1f} s wall on {os.cpu_count()} host cores")


def time_to_eigenpairs(b, w, torch, tol=1e-8, solvers=("lobpcg", "chefsi")):
    """Lowest w.nev eigenpairs to ||H x - lambda x|| <= tol from the same
    seeded random start, FP64 H*X and mixed (FP32 H*X, FP64 refinement); all
    keep the FP64 Rayleigh-Ritz.  Two solvers: LOBPCG with the TPA
    preconditioner and Chebyshev-filtered subspace iteration (automatic degree
    and guard).  Reports wall time, iterations (outer filter steps for the
    latter), the H*X and Rayleigh-Ritz shares and the largest eigenvalue
    difference against LOBPCG in FP64."""
    import numpy as np
    out = {"nev": w.nev, "tol_Ha": tol}
    evs = {}
    # warm-up: library handles and kernels of both solvers loaded before timing
    b.eigensolve_ex(4, tol=1e-3, maxit=2)
    b.eigensolve_ex(4, tol=1e-3, maxit=1, cheb_degree=2)
    runs = ((("fp64", None, "fp64"), ("fp32", None, "mixed_fp32_fp64")) if "lobpcg" in solvers else ()) + \
           ((("fp64", 0, "chefsi_fp64"), ("fp32", 0, "chefsi_mixed_fp32_fp64")) if "chefsi" in solvers else ())
    for prec, deg, key in runs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, res, st, status = b.eigensolve_ex(w.nev, block=64, tol=tol, maxit=1000 if deg is None else 200,
                                              prec=prec, seed=7, log_every=LOG_EVERY, cheb_degree=deg)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[key] = dict(seconds=round(wall, 3), converged=bool(status == 0), iters=st["iters"],
                        iters_fp32=st["iters_low"], hx_columns=st["n_apply"], hx_s=round(st["t_apply_ms"] / 1e3, 3),
                        rayleigh_ritz_s=round(st["t_rr_ms"] / 1e3, 3), max_resid=float(np.max(res)))
        evs[key] = ev
        print(f"[bench] eigensolve {key}: {wall:.2f} s, {st['iters']} iterations, converged {status == 0}",
              file=sys.stderr, flush=True)
    if "lobpcg" not in solvers or "chefsi" not in solvers:
        return out
    d = np.abs(evs["mixed_fp32_fp64"] - evs["fp64"])
    out["mixed_vs_fp64_max_abs_Ha"] = float(d.max())
    out["speedup_mixed"] = round(out["fp64"]["seconds"] / out["mixed_fp32_fp64"]["seconds"], 3)
    out["chefsi_vs_lobpcg_max_abs_Ha"] = float(max(np.abs(evs["chefsi_fp64"] - evs["fp64"]).max(),
                                                   np.abs(evs["chefsi_mixed_fp32_fp64"] - evs["fp64"]).max()))
    out["speedup_chefsi"] = round(out["fp64"]["seconds"] / out["chefsi_fp64"]["seconds"], 3)
    out["speedup_chefsi_mixed"] = round(out["fp64"]["seconds"] / out["chefsi_mixed_fp32_fp64"]["seconds"], 3)
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


def batched_leg(torch, structures, nvec=8, steps=20, eig_every=8, nev=60, tol=1e-8, learned=True):
    """Many Bloch parameters of seeded structures (64 eta each, R ~ U[5, 12],
    E_cut ~ U[15, 35]): per structure one batch with a common grid (the
    largest automatic grid over its eta), tuned, captured in a HIP graph and
    replayed; and the lowest `nev` eigenpairs of every `eig_every`-th eta,
    solved concurrently on 8 streams, with the plain preconditioner, by
    Chebyshev-filtered subspace iteration (also with time-reversal halving of
    the eta points), and (if `learned`) with a network trained on one other
    eta of the structure."""
    import concurrent.futures as cf

    import numpy as np

    import synth
    from synth.configs import batched_problems
    from paper_2210_12252_amd import helic
    allp = batched_problems()
    out = []
    for s in structures:
        probs = allp[64 * s: 64 * (s + 1)]
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(8) as ex:
            auto = list(ex.map(lambda w: helic.Basis.from_workload(w), probs))
        n1 = max(b.n_t1 for b in auto)
        n2 = max(b.n_t2 for b in auto)
        nr = max(b.n_r for b in auto)
        for b in auto:
            b.close()
        grid_w = [w.with_(n_t1=n1, n_t2=n2, n_r=nr, m_max=(n1 - 1) // 2, n_max=(n2 - 1) // 2) for w in probs]
        with cf.ThreadPoolExecutor(8) as ex:
            bases = list(ex.map(lambda w: helic.Basis.from_workload(w), grid_w))
        t1, t2, r, _ = bases[0].grid()
        w0 = probs[0]
        V = torch.from_numpy(synth.potential_at(t1, t2, r, w0.tau, w0.alpha,
                                                synth.atoms_for(w0.structure, w0.seed, w0.tau, w0.R))).cuda()
        for b in bases:
            b.set_potential(V)
        batch = helic.Batch(bases)
        setup = time.perf_counter() - t0
        total = nvec * int(batch.offsets[-1])
        X = torch.randn(total, dtype=torch.complex128, device="cuda")
        Y = torch.zeros_like(X)
        chosen, _ = batch.tune(X, Y, nvec)
        batch.capture(X, Y, nvec)
        batch.replay()
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(steps):
            batch.replay()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - ta) / steps
        Ls = np.diff(batch.offsets)
        rec = dict(structure=s, R=round(w0.R, 3), ecut=round(w0.ecut, 3), n_eta=len(probs),
                   grid=f"{n1}x{n2}x{nr}", L_min=int(Ls.min()), L_max=int(Ls.max()),
                   kernel=angular_kernel_name(n1, n2),
                   setup_s=round(setup, 2), tuned_items_per_wg=chosen, ms_per_batched_apply=round(1e3 * dt, 3),
                   vec_applies_per_s=round(len(probs) * nvec / dt, 1))
        sub = bases[::eig_every]
        eb = helic.Batch(sub)
        torch.cuda.synchronize()
        te = time.perf_counter()
        ev, res, st, status = eb.eigensolve(nev, nstreams=8, tol=tol, maxit=1000)
        te = time.perf_counter() - te
        rec.update(eig_problems=len(sub), eig_nev=nev, eig_seconds=round(te, 2),
                   eig_converged=int(np.sum(status == 0)), eig_iters_mean=float(np.mean([x["iters"] for x in st])))
        te = time.perf_counter()
        evc, resc, stc, statusc = eb.eigensolve(nev, nstreams=8, tol=tol, maxit=200, cheb_degree=0)
        te = time.perf_counter() - te
        rec.update(chefsi_eig_seconds=round(te, 2), chefsi_converged=int(np.sum(statusc == 0)),
                   chefsi_steps_mean=float(np.mean([x["iters"] for x in stc])),
                   chefsi_max_abs_dlambda=float(np.max(np.abs(evc - ev))))
        # time-reversal halving: eta and -eta of the subset share one solve
        npairs = eb.time_reversal(True)
        te = time.perf_counter()
        evt, _, _, statust = eb.eigensolve(nev, nstreams=8, tol=tol, maxit=200, cheb_degree=0)
        te = time.perf_counter() - te
        eb.time_reversal(False)
        rec.update(time_reversal_pairs=npairs, chefsi_tr_eig_seconds=round(te, 2),
                   chefsi_tr_converged=int(np.sum(statust == 0)),
                   chefsi_tr_max_abs_dlambda=float(np.max(np.abs(evt - ev))))
        if learned:
            # one network per structure, trained on pairs from the solve at an
            # eta outside the solved subset, attached to every solved problem
            tl = time.perf_counter()
            tb = bases[eig_every // 2]
            Rh, Th, lh, ncol, _ = tb.lpc_harvest(nev, n_snap=12, tol=tol, maxit=1000, seed=3)
            net = helic.Lpc(seed=0)
            tb.lpc_train(net, Rh, Th, lh, ncol, batch=min(16, ncol), steps=400, lr=3e-3, seed=0)
            torch.cuda.synchronize()
            tl = time.perf_counter() - tl
            del Rh, Th, lh
            for sb in sub:
                sb.attach(net)
            te = time.perf_counter()
            evl, resl, stl, statusl = eb.eigensolve(nev, nstreams=8, tol=tol, maxit=1000, precond="learned")
            te = time.perf_counter() - te
            for sb in sub:
                sb.attach(None)
            net.close()
            rec.update(learned_train_s=round(tl, 2), learned_eig_seconds=round(te, 2),
                       learned_converged=int(np.sum(statusl == 0)),
                       learned_iters_mean=float(np.mean([x["iters"] for x in stl])),
                       learned_max_abs_dlambda=float(np.max(np.abs(evl - ev))))
        print(f"[bench] batched structure {s}: {rec}", file=sys.stderr, flush=True)
        out.append(rec)
        eb.close()
        batch.close()
        for b in bases:
            b.close()
        del X, Y
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
    out["max_abs_dlambda_Ha"] = float(np.max(np.abs(evs["learned"] - evs["tpa"])))
    out["speedup_time"] = round(out["tpa"]["seconds"] / out["learned"]["seconds"], 3)
    out["iteration_ratio"] = round(out["learned"]["iters"] / max(out["tpa"]["iters"], 1), 3)
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
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="nanotube-ecut25")
    ap.add_argument("--prec", default="fp64", choices=("fp64", "fp32", "bf16"))
    ap.add_argument("--cpu-sample", type=int, default=64, help="vectors for the CPU oracle leg (0: skip)")
    ap.add_argument("--eig", type=int, default=1, help="also time the eigensolve (FP64 and mixed) (0: skip)")
    ap.add_argument("--eig-solvers", default="lobpcg,chefsi",
                    help="comma list of eigensolvers the eigensolve leg times (lobpcg, chefsi)")
    ap.add_argument("--batched", default="4",
                    help="structures (0..7, comma list, 'all' or 'none') for the batched Bloch-parameter leg")
    ap.add_argument("--learned", default="same",
                    help="learned-preconditioner leg: 'same' (the benchmark workload), a workload name, or 'none'")
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
    w = synth.workload(args.workload)
    nvec = 64
    t_setup = time.perf_counter()
    b = helic.Basis.from_workload(w)
    t1, t2, r, _ = b.grid()
    atoms = synth.atoms_for(w.structure, w.seed, w.tau, w.R)
    V = synth.potential_at(t1, t2, r, w.tau, w.alpha, atoms)
    b.set_potential(torch.from_numpy(V).to(dev))
    mnk, _ = b.indices()
    X = torch.from_numpy(np.ascontiguousarray(synth.random_block(mnk, nvec, 1234).T)).to(dev)
    Y = torch.empty_like(X)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    print(f"[bench] {w.name}: L={b.L} modes={b.n_modes} grid={b.n_t1}x{b.n_t2}x{b.n_r} "
          f"setup {t_setup:.2f} s", file=sys.stderr, flush=True)

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
        peak_tf = FP64_PEAK_TFLOPS if elem == 8 else FP32_MFMA_PEAK_TFLOPS
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
        "dtype": "f64" if args.prec == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "L": b.L, "block": nvec, "grid": f"{b.n_t1}x{b.n_t2}x{b.n_r}",
                   "modes": b.n_modes, "R": w.R, "tau": w.tau, "alpha": round(w.alpha, 6), "ecut": w.ecut,
                   "parallelism": "single GPU"},
        "roofline": roof,
        "stages": stage_info,
    }
    if args.eig:
        line["eigensolve"] = time_to_eigenpairs(b, w, torch, solvers=tuple(args.eig_solvers.split(",")))
        line["density"] = density_leg(b, w, torch)
    if args.batched != "none":
        structs = list(range(8)) if args.batched == "all" else [int(x) for x in args.batched.split(",")]
        line["batched"] = batched_leg(torch, structs)
    if args.learned != "none":
        if args.learned in ("same", w.name):
            lw, lb = w, b
        else:
            lw = synth.workload(args.learned)
            lb = helic.Basis.from_workload(lw)
            t1, t2, r, _ = lb.grid()
            lb.set_potential(torch.from_numpy(synth.potential_at(
                t1, t2, r, lw.tau, lw.alpha, synth.atoms_for(lw.structure, lw.seed, lw.tau, lw.R))).cuda())
        line["learned_preconditioner"] = learned_leg(torch, lb, lw)
        if lb is not b:
            lb.close()
    if args.cpu_sample > 0:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample)
    b.close()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
