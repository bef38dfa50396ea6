"""Workload descriptions for the helical-wave Hamiltonian benchmarks.

Every workload is a cylinder of radius ``R`` (Bohr, Dirichlet wall at r = R),
axial period ``tau`` (Bohr) and twist ``alpha`` (turns per period: the screw
operation rotates by 2*pi*alpha while translating by tau), a kinetic-energy
cutoff ``ecut`` (Ha), a helical Bloch parameter ``eta`` in [-1/2, 1/2), and a
real-space grid ``n_t1 x n_t2 x n_r`` (axial Fourier nodes x angular Fourier
nodes x radial Gauss-Jacobi nodes).  Index clamps of -1 and grid sizes of 0
mean "derive from the cutoff / the grid".  The cyclic order is 1 unless a
workload sets ``ncyc`` (an ncyc-fold symmetric structure, theta2 in
[0, 1/ncyc)), with cyclic Bloch index ``nu`` (0 unless set).

The index letters follow the paper: m is the Fourier index along theta1 (the
axial coordinate z / tau), n the Fourier index along theta2 (the angular
coordinate, Bessel order n) and k the radial index (k-th Bessel zero).
"""
from __future__ import annotations

import dataclasses
import math


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    R: float
    tau: float
    alpha: float
    ecut: float
    eta: float = 0.0
    m_max: int = -1
    n_max: int = -1
    k_max: int = -1
    n_t1: int = 0
    n_t2: int = 0
    n_r: int = 0
    nev: int = 8
    block: int = 64
    structure: str = "none"      # key understood by synth.structures.atoms_for
    seed: int = 0
    ncyc: int = 1                # cyclic order: theta2 spans [0, 1/ncyc)
    nu: int = 0                  # cyclic Bloch index, 0 <= nu < ncyc

    def params(self) -> dict:
        """Plain parameter dictionary in the library's parameter-struct order."""
        return dict(R=self.R, tau=self.tau, alpha=self.alpha, ncyc=self.ncyc,
                    ecut=self.ecut, eta=self.eta, nu=self.nu,
                    m_max=self.m_max, n_max=self.n_max, k_max=self.k_max,
                    n_t1=self.n_t1, n_t2=self.n_t2, n_r=self.n_r)

    def with_(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


# Tiny helix: 6 wells on a helix of radius 4 Bohr; box |n| <= 6, |m| <= 4,
# k <= 12, cut at 8 Ha (816 functions survive the cutoff), 16x16x48 grid.
TINY = Workload(name="tiny-helix", R=10.0, tau=6.0, alpha=0.0, ecut=8.0,
                m_max=4, n_max=6, k_max=12, n_t1=16, n_t2=16, n_r=48,
                nev=8, block=8, structure="helix6", seed=1)

# Nanotube-like: 52 wells (4 rings of 13) on radius 7.5 Bohr, twist 1/13 turn
# per 8 Bohr period, cut at 25 Ha on a 48 (axial) x 64 (angular) x 160 grid.
NANOTUBE = Workload(name="nanotube-ecut25", R=20.0, tau=8.0, alpha=1.0 / 13.0,
                    ecut=25.0, n_t1=48, n_t2=64, n_r=160, nev=120, block=64,
                    structure="tube52", seed=2)

# Same structure at a 40 Ha cutoff (mixed-precision workload).
NANOTUBE_HI = NANOTUBE.with_(name="nanotube-ecut40", ecut=40.0, n_r=208, nev=200)

# Filled nanowire: 180 wells inside radius 12 Bohr, R = 28, tau = 10, 30 Ha.
NANOWIRE = Workload(name="nanowire-ecut30", R=28.0, tau=10.0, alpha=0.0,
                    ecut=30.0, n_t1=32, n_t2=81, n_r=256, nev=400, block=64,
                    structure="wire180", seed=5)

WORKLOADS = {w.name: w for w in (TINY, NANOTUBE, NANOTUBE_HI, NANOWIRE)}


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def batched_problems(n_eta: int = 64, n_struct: int = 8, seed0: int = 40):
    """Many Bloch parameters over several seeded structures.

    Structure s draws R ~ U[5, 12] Bohr and ecut ~ U[15, 35] Ha from seed
    seed0 + s; tau = 10 Bohr, no twist, no clamps, automatic grid.  The Bloch
    parameters are eta_b = -1/2 + b / n_eta (b = 0..n_eta-1), a uniform
    sampling of the axial wavevector over one period.
    """
    import numpy as np
    out = []
    for s in range(n_struct):
        rng = np.random.Generator(np.random.PCG64(seed0 + s))
        R = float(rng.uniform(5.0, 12.0))
        ecut = float(rng.uniform(15.0, 35.0))
        base = Workload(name=f"batch-s{s}", R=R, tau=10.0, alpha=0.0, ecut=ecut,
                        nev=60, block=64, structure=f"blob:{s}", seed=seed0 + s)
        for b in range(n_eta):
            out.append(base.with_(name=f"batch-s{s}-e{b}", eta=-0.5 + b / n_eta))
    return out


def _check():
    assert math.isclose(NANOTUBE.alpha * 13, 1.0)


_check()
