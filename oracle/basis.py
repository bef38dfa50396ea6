"""Helical-wave basis: index set, kinetic diagonal, grid and radial functions.

Test infrastructure (see the package docstring); plain FP64 NumPy/SciPy.

Paper passages followed:
* basis functions F_{m,n,k} = c_{nk} exp(i 2 pi (m theta1 + n N theta2))
  J_{nN}(b_k^{nN} r / R), c_{nk} = sqrt(N/(pi tau)) / (R J_{nN+1}(b_k^{nN}))
  -- Sec. 2.3 and App. B (eq. Basis_fun_derived);
* the operator at cyclic index nu (eq. Simplify_2 and constants_abc): the
  terms a, b, c and the nu^2 / (2 r^2) and (i nu / (2 pi r^2)) d/dtheta2
  terms added to -(1/2) Laplacian + V;
* Laplacian eigenvalue lambda0 = (b/R)^2 + (2 pi/tau)^2 (m - alpha n N)^2
  -- eq. Laplacian_of_f_mnk;
* kinetic-energy cutoff (1/2) lambda0 <= E_cut, applied at each Bloch point
  with the kinetic energy "modified appropriately" -- Sec. 3.2;
* storage order i(m, n, k): m outermost, then n, then k -- eq.
  wavefun_storage (only functions that pass the cutoff are kept);
* grid: Fourier nodes in theta1, theta2 and N_r Gauss-Jacobi nodes on
  [0, R] -- Sec. 3.1; radial rule for int_0^1 f(q) q^sigma dq -- App. D.

Readings where the paper is silent (each listed in the design notes):
* The radial rule has sigma = 1 (the r dr Jacobian); radial weights are
  omega_l = R^2 w_l with (q_l, w_l) the rule for int_0^1 f(q) q dq.
* At Bloch parameter eta (nu = 0) the kinetic diagonal that enters the
  operator and the cutoff is kappa = (1/2)[(b/R)^2 + (2 pi/tau)^2
  (m - alpha n - eta)^2], which equals Alg. 5's (1/2)Lambda - a - b M - c N
  with the constants of eq. constants_abc (checked in the tests).
* Cyclic index nu != 0: the paper keeps J_{nN} and represents the 1/r^2
  terms by the integrals I(n, k, k') of eq. I_nkk_prime, which diverge for
  n = 0.  Acting on exp(i 2 pi n N theta2) R(r), those terms turn the Bessel
  operator of order nN into that of order nN - nu, so the radial functions
  here are J_p(b_k^p r / R) with p = nN - nu (zeros of J_|p|, the paper's
  signed normalisation with J_{p+1}): the same operator in the basis that
  diagonalises its kinetic part, kappa = (1/2)[(b^|p| / R)^2 + (2 pi/tau)^2
  (m - alpha (nN - nu) - eta)^2], and no I table.  At nu = 0 it is the
  paper's basis.
* Mode (m, n) sits at DFT bin (m mod N_theta1, n mod N_theta2).
* Index clamps default to what the grid resolves; an automatic grid uses the
  smallest 2,3,5-smooth sizes >= 2 max|m| + 2 and 2 max|n| + 2, and
  N_r = 4 K_max (the paper's radial rule).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import scipy.special as sp

TIE_TOL = 1e-10


def bessel_zeros(p: int, count: int) -> np.ndarray:
    """First ``count`` positive zeros of J_p for integer p (zeros of J_{-p}
    coincide with those of J_{|p|})."""
    if count <= 0:
        return np.zeros(0)
    return np.asarray(sp.jn_zeros(abs(int(p)), int(count)), dtype=np.float64)


def smooth_at_least(x: int) -> int:
    n = max(int(x), 1)
    while True:
        y = n
        for p in (2, 3, 5):
            while y % p == 0:
                y //= p
        if y == 1:
            return n
        n += 1


@dataclasses.dataclass
class Basis:
    R: float
    tau: float
    alpha: float
    eta: float
    ecut: float
    n_t1: int
    n_t2: int
    n_r: int
    mnk: np.ndarray          # (L, 3) int64, paper storage order
    bzero: np.ndarray        # (L,) Bessel zero b_k^{|n|}
    kappa: np.ndarray        # (L,) kinetic diagonal
    theta1: np.ndarray       # (n_t1,)
    theta2: np.ndarray       # (n_t2,)
    q: np.ndarray            # (n_r,) radial nodes on [0, 1]
    wq: np.ndarray           # (n_r,) weights for int_0^1 f(q) q dq
    ncyc: int = 1
    nu: int = 0

    def order(self, n):
        """Bessel order p = n N - nu of angular index n."""
        return n * self.ncyc - self.nu

    @property
    def L(self) -> int:
        return int(self.mnk.shape[0])

    @property
    def r(self) -> np.ndarray:
        return self.R * self.q

    @property
    def omega_r(self) -> np.ndarray:
        """Radial quadrature weights on [0, R] including the r dr Jacobian."""
        return self.R * self.R * self.wq

    @property
    def grid_weight(self) -> float:
        """2 pi tau * omega_theta1 * omega_theta2 (omega_theta1 = 1/N_theta1,
        omega_theta2 = 1/(N N_theta2)), eq. Fast_fwd_transform_cont; multiply by
        omega_r for the full weight of a grid point."""
        return 2.0 * math.pi * self.tau / (self.n_t1 * self.ncyc * self.n_t2)

    def xi(self, n: int, k: np.ndarray, r: np.ndarray | None = None) -> np.ndarray:
        """Radial functions xi_{n,k}(r) on the radial grid (or at ``r``),
        shape (len(r), len(k)), with the paper's signed normalisation
        sqrt(N/(pi tau)) J_p(b r/R) / (R J_{p+1}(b)), p = nN - nu (App. B)."""
        rr = self.r if r is None else np.asarray(r, dtype=np.float64)
        k = np.asarray(k, dtype=np.int64)
        p = self.order(n)
        b = bessel_zeros(p, int(k.max()) if k.size else 0)[k - 1] if k.size else np.zeros(0)
        c = math.sqrt(self.ncyc / (math.pi * self.tau)) / (self.R * sp.jv(p + 1, b))
        return sp.jv(p, np.outer(rr, b) / self.R) * c[None, :]


def kinetic_diagonal(bz, m, n, R, tau, alpha, eta, ncyc=1, nu=0):
    """kappa = (1/2)[(b/R)^2 + (2 pi/tau)^2 (m - alpha (n N - nu) - eta)^2]
    (cyclic order N, cyclic index nu)."""
    m = np.asarray(m, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    return 0.5 * ((np.asarray(bz) / R) ** 2 + (2.0 * math.pi / tau) ** 2 * (m - alpha * (n * ncyc - nu) - eta) ** 2)


def kinetic_alg5(bz, m, n, R, tau, alpha, eta, nu=0, ncyc=1):
    """The diagonal of Alg. 5 written as the paper states it:
    (1/2) Lambda - a - b (i 2 pi m) - c (i 2 pi N n), with Lambda the Laplacian
    eigenvalues (eq. Laplacian_of_f_mnk) and a, b, c from eq. constants_abc.
    Complex-valued; at nu = 0 its imaginary part vanishes."""
    m = np.asarray(m, dtype=np.float64)
    n = np.asarray(n, dtype=np.float64)
    lam0 = (np.asarray(bz) / R) ** 2 + ((2.0 * math.pi / tau) * (m - alpha * n * ncyc)) ** 2
    a = 2.0 * math.pi ** 2 / tau ** 2 * (nu * alpha * (2.0 * eta - nu * alpha) - eta ** 2)
    b = 2j * math.pi / tau ** 2 * (nu * alpha - eta)
    c = 2j * math.pi * alpha / tau ** 2 * (eta - nu * alpha)
    return 0.5 * lam0 - a - b * (2j * math.pi * m) - c * (2j * math.pi * ncyc * n)


def make_basis(R, tau, alpha, ecut, eta=0.0, m_max=-1, n_max=-1, k_max=-1,
               n_t1=0, n_t2=0, n_r=0, ncyc=1, nu=0) -> Basis:
    """Enumerate the cutoff-masked index set and build the grid.

    Cyclic order N >= 1 and index 0 <= nu < N (Sec. 2.3): mode (m, n) has
    the angular factor exp(i 2 pi (m theta1 + n N theta2)), the Bessel order
    |n N - nu| and its zeros, and theta2 spans [0, 1/N).  Raises ValueError
    on inconsistent parameters and on a cutoff tie (some |kappa - E_cut| <
    1e-10)."""
    if ncyc < 1 or not (0 <= nu < ncyc):
        raise ValueError("need cyclic order N >= 1 and 0 <= nu < N")
    if not (R > 0 and tau > 0 and ecut > 0 and 0.0 <= alpha < 1.0 and -0.5 <= eta < 0.5):
        raise ValueError("invalid parameters")
    grid_given = n_t1 > 0 and n_t2 > 0
    if (n_t1 > 0) != (n_t2 > 0):
        raise ValueError("give both angular grid sizes or neither")
    if grid_given:
        if m_max < 0:
            m_max = (n_t1 - 1) // 2
        if n_max < 0:
            n_max = (n_t2 - 1) // 2
    two_pi_tau = 2.0 * math.pi / tau
    # n limits from the smallest radial energy j_{|p|,1}^2 / (2 R^2) of the
    # order p = n N - nu, which grows with |n| on either side
    def admissible(n):
        return 0.5 * (bessel_zeros(n * ncyc - nu, 1)[0] / R) ** 2 <= ecut + TIE_TOL
    if n_max < 0:
        n_hi = 0
        while admissible(n_hi + 1):
            n_hi += 1
        n_lo = 0
        while admissible(n_lo - 1):
            n_lo -= 1
    else:
        n_lo, n_hi = -n_max, n_max
    rows = []
    for n in range(n_lo, n_hi + 1):
        p = n * ncyc - nu
        # enough zeros so that the radial energy alone exceeds the cutoff
        cnt = 8
        while True:
            z = bessel_zeros(p, cnt)
            if 0.5 * (z[-1] / R) ** 2 > ecut + 1.0 or (k_max > 0 and cnt >= k_max):
                break
            cnt *= 2
        if k_max > 0:
            z = z[:k_max]
        # m range allowed by the axial energy alone
        span = math.sqrt(2.0 * ecut) / two_pi_tau + 1.0
        c0 = alpha * p + eta
        m_lo, m_hi = int(math.floor(c0 - span)), int(math.ceil(c0 + span))
        if m_max >= 0:
            m_lo, m_hi = max(m_lo, -m_max), min(m_hi, m_max)
        for m in range(m_lo, m_hi + 1):
            kap = kinetic_diagonal(z, m, n, R, tau, alpha, eta, ncyc, nu)
            if np.any(np.abs(kap - ecut) < TIE_TOL):
                raise ValueError("cutoff tie: a kinetic energy equals E_cut to 1e-10")
            for k in np.nonzero(kap <= ecut)[0]:
                rows.append((m, n, int(k) + 1, z[k], kap[k]))
    if not rows:
        raise ValueError("empty basis")
    # paper storage order: m outermost, then n, then k
    rows.sort(key=lambda t: (t[0], t[1], t[2]))
    mnk = np.array([(t[0], t[1], t[2]) for t in rows], dtype=np.int64)
    bz = np.array([t[3] for t in rows])
    kap = np.array([t[4] for t in rows])
    mabs = int(np.abs(mnk[:, 0]).max())
    nabs = int(np.abs(mnk[:, 1]).max())
    kmx = int(mnk[:, 2].max())
    if not grid_given:
        n_t1 = smooth_at_least(2 * mabs + 2)
        n_t2 = smooth_at_least(2 * nabs + 2)
    if n_r <= 0:
        n_r = 4 * kmx
    if mnk[:, 0].max() - mnk[:, 0].min() + 1 > n_t1 or 2 * nabs + 1 > n_t2:
        raise ValueError("grid does not resolve the index set")
    x, w = sp.roots_jacobi(n_r, 0.0, 1.0)
    q = 0.5 * (1.0 + x)
    wq = 0.25 * w
    return Basis(R=float(R), tau=float(tau), alpha=float(alpha), eta=float(eta),
                 ecut=float(ecut), n_t1=int(n_t1), n_t2=int(n_t2), n_r=int(n_r),
                 mnk=mnk, bzero=bz, kappa=kap,
                 theta1=np.arange(n_t1) / n_t1, theta2=np.arange(n_t2) / (ncyc * n_t2),
                 q=q, wq=wq, ncyc=ncyc, nu=nu)


def basis_for(workload) -> Basis:
    """Basis of a ``synth.Workload`` (duck-typed: reads its attributes)."""
    w = workload
    return make_basis(w.R, w.tau, w.alpha, w.ecut, eta=w.eta, m_max=w.m_max, n_max=w.n_max,
                      k_max=w.k_max, n_t1=w.n_t1, n_t2=w.n_t2, n_r=w.n_r, ncyc=getattr(w, "ncyc", 1),
                      nu=getattr(w, "nu", 0))
