"""Write the oracle's lowest eigenvalues of a workload to a golden file.

    python tests/golden/make_lowest.py nanotube-ecut25 120

Builds the dense FP64 Hamiltonian of the workload's seeded structure with the
oracle (mode B, one pair of angular modes at a time) and takes its lowest
eigenvalues with LAPACK (zheevr, subset by index).  Only ``oracle`` (the
method's arithmetic) and ``synth`` (the seeded inputs) are used.  For the
48 x 64 x 160 nanotube workload (31,543 functions) H takes 16 GB and the
eigensolve about an hour on 8 cores.
"""
from __future__ import annotations

import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import basis as ob  # noqa: E402
from oracle import hamiltonian as oh  # noqa: E402


def main(name: str, nev: int) -> None:
    w = synth.workload(name)
    o = ob.basis_for(w)
    atoms = synth.atoms_for(w.structure, w.seed, w.tau, w.R)
    V = synth.potential_at(o.theta1, o.theta2, o.r, w.tau, w.alpha, atoms)
    t0 = time.time()
    H = oh.dense_dft_modes(o, V)
    t1 = time.time()
    print(f"{name}: L = {o.L}, H built in {t1 - t0:.0f} s", flush=True)
    lam = oh.lowest_values(H, nev)
    t2 = time.time()
    print(f"{name}: lowest {nev} eigenvalues in {t2 - t1:.0f} s", flush=True)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{name.replace('-', '_')}_lowest{nev}.txt")
    with open(out, "w") as f:
        f.write(f"# Lowest {nev} eigenvalues (Ha) of the dense FP64 oracle Hamiltonian of workload {name}\n")
        f.write(f"# (L = {o.L}, grid {o.n_t1} x {o.n_t2} x {o.n_r}, structure {w.structure} seed {w.seed}).\n")
        f.write(f"# Written by: python tests/golden/make_lowest.py {name} {nev}\n")
        f.write(f"# (oracle.hamiltonian.dense_dft_modes + lowest_values; {platform.processor() or platform.machine()},"
                f" build {t1 - t0:.0f} s, eigensolve {t2 - t1:.0f} s)\n")
        for i, x in enumerate(lam):
            f.write(f"{i} {x:.17e}\n")
    print("wrote", out, flush=True)


if __name__ == "__main__":
    main(sys.argv[1], int(sys.argv[2]))
