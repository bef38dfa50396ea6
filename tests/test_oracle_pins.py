"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a tabulated value,
a closed form, an identity of the continuous problem, an exact property of the
discrete operator, or a brute-force evaluation.
"""
import math
import os

import numpy as np
import pytest
import scipy.integrate as si
import scipy.linalg as sla
import scipy.special as sp

import synth
from oracle import basis as ob
from oracle import hamiltonian as oh
from oracle import precond as op
from oracle import transforms as ot

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_basis(**kw):
    p = dict(R=6.0, tau=5.0, alpha=0.2, ecut=6.0, eta=0.15, n_t1=12, n_t2=16, n_r=32)
    p.update(kw)
    return ob.make_basis(**p)


@pytest.fixture(scope="module")
def tiny():
    w = synth.workload("tiny-helix")
    b = ob.basis_for(w)
    atoms = synth.atoms_for(w.structure, w.seed, w.tau, w.R)
    V = synth.potential_at(b.theta1, b.theta2, b.r, w.tau, w.alpha, atoms)
    B = ot.basis_matrix(b)
    return w, b, V, B


# ---------------------------------------------------------------- Bessel zeros
def test_bessel_zeros_match_table():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "bessel_zeros.txt")) if not l.startswith("#")]
    for p, k, v in rows:
        z = ob.bessel_zeros(int(p), int(k))[-1]
        assert abs(z - float(v)) < 1e-12, (p, k, z, v)


@pytest.mark.parametrize("p", [0, 1, 7, 31, 64, 130])
def test_bessel_zeros_are_roots_and_interlace(p):
    z = ob.bessel_zeros(p, 60)
    zp = ob.bessel_zeros(p + 1, 60)
    assert np.all(np.abs(sp.jv(p, z)) < 1e-13)
    assert np.all(z[:-1] < zp[:-1]) and np.all(zp[:-1] < z[1:])
    # McMahon: j_{p,k} ~ beta - (4p^2 - 1)/(8 beta), beta = (k + p/2 - 1/4) pi, for k >> p
    if p <= 7:
        k = np.arange(40, 61)
        beta = (k + p / 2 - 0.25) * math.pi
        mu = 4 * p * p
        mc = beta - (mu - 1) / (8 * beta) - 4 * (mu - 1) * (7 * mu - 31) / (3 * (8 * beta) ** 3)
        assert np.max(np.abs(z[k - 1] - mc)) < 1e-6


def test_negative_order_zeros_and_signed_radial_function():
    """xi_{-n,k} equals xi_{n,k} with the paper's signed normalisation."""
    b = small_basis()
    r = np.linspace(0.1, b.R, 17)
    for n in (1, 2, 5):
        zp = ob.bessel_zeros(n, 4)
        assert np.all(np.abs(sp.jv(-n, zp)) < 1e-13)
        np.testing.assert_allclose(b.xi(-n, np.arange(1, 5), r), b.xi(n, np.arange(1, 5), r),
                                   rtol=1e-13, atol=1e-15)


# ----------------------------------------------------------- radial quadrature
@pytest.mark.parametrize("nr", [8, 48, 160])
def test_gauss_jacobi_moments(nr):
    b = small_basis(n_r=nr)
    assert np.all(b.q > 0) and np.all(b.q < 1)
    for j in range(0, 2 * nr):
        exact = 1.0 / (j + 2)
        assert abs(np.sum(b.wq * b.q ** j) - exact) < 1e-14, j


def test_bessel_orthogonality_on_grid_and_by_adaptive_quadrature():
    """(2 pi tau / N) sum_l omega_l xi_{n,k} xi_{n,k'} = delta_kk' (App. B), and
    the continuous integral by adaptive quadrature gives the same."""
    w = synth.workload("tiny-helix")
    b = ob.basis_for(w)
    K = 12
    for n in (0, 3, 6):
        tab = b.xi(n, np.arange(1, K + 1))
        gram = 2 * math.pi * b.tau * (tab * b.omega_r[:, None]).T @ tab
        assert np.max(np.abs(gram - np.eye(K))) < 1e-13
    # continuous normalisation of one function, independent of the grid
    n, k = 4, 3
    bz = ob.bessel_zeros(n, k)[-1]
    f = lambda r: (b.xi(n, np.array([k]), np.array([r]))[0, 0]) ** 2 * r
    val, err = si.quad(f, 0.0, b.R, epsabs=1e-14, epsrel=1e-13, limit=200)
    assert abs(2 * math.pi * b.tau * val - 1.0) < 1e-11
    assert bz > 0


# ---------------------------------------------------------- index set and mask
def test_index_set_is_exactly_the_cutoff_set():
    b = small_basis()
    kap = ob.kinetic_diagonal(b.bzero, b.mnk[:, 0], b.mnk[:, 1], b.R, b.tau, b.alpha, b.eta)
    assert np.all(kap <= b.ecut)
    have = set(map(tuple, b.mnk.tolist()))
    # brute force over a strictly larger box
    mmax = (b.n_t1 - 1) // 2
    nmax = (b.n_t2 - 1) // 2
    count = 0
    for n in range(-nmax, nmax + 1):
        z = sp.jn_zeros(abs(n), 40)
        for m in range(-mmax, mmax + 1):
            for k in range(1, 41):
                e = 0.5 * ((z[k - 1] / b.R) ** 2 + (2 * math.pi / b.tau * (m - b.alpha * n - b.eta)) ** 2)
                inside = e <= b.ecut
                assert inside == ((m, n, k) in have)
                count += inside
    assert count == b.L
    # paper storage order: m outermost, then n, then k
    keys = b.mnk[:, 0] * 10 ** 8 + (b.mnk[:, 1] + 10 ** 4) * 10 ** 3 + b.mnk[:, 2]
    assert np.all(np.diff(keys) > 0)


@pytest.mark.parametrize("name,L", [("tiny-helix", 816), ("nanotube-ecut25", 31543)])
def test_basis_sizes_of_workloads(name, L):
    b = ob.basis_for(synth.workload(name))
    assert b.L == L


def test_kinetic_diagonal_equals_alg5_form():
    for eta in (-0.5, -0.2, 0.0, 0.31):
        b = small_basis(eta=eta, alpha=0.37)
        m, n = b.mnk[:, 0], b.mnk[:, 1]
        alg5 = ob.kinetic_alg5(b.bzero, m, n, b.R, b.tau, b.alpha, eta)
        assert np.max(np.abs(alg5.imag)) < 1e-13
        np.testing.assert_allclose(alg5.real, b.kappa, rtol=1e-13)


def test_kinetic_diagonal_is_eigenvalue_of_cartesian_laplacian():
    """-1/2 Laplacian (Cartesian, finite differences) of the Bloch wave
    exp(-i 2 pi eta z / tau) F_{m,n,k} equals kappa times it."""
    b = small_basis(alpha=0.3, eta=0.2)
    rng = np.random.default_rng(3)
    picks = rng.choice(b.L, size=6, replace=False)

    def psi(i, x, y, z):
        m, n, k = b.mnk[i]
        r = math.hypot(x, y)
        th1 = z / b.tau
        th2 = math.atan2(y, x) / (2 * math.pi) - b.alpha * z / b.tau
        rad = b.xi(int(n), np.array([k]), np.array([r]))[0, 0]
        return np.exp(-2j * math.pi * b.eta * th1) * np.exp(2j * math.pi * (m * th1 + n * th2)) * rad

    h = 1e-2
    c = np.array([-1.0, 16.0, -30.0, 16.0, -1.0]) / (12 * h * h)
    for i in picks:
        for _ in range(3):
            rr = rng.uniform(1.0, b.R - 1.0)
            ph = rng.uniform(0, 2 * math.pi)
            x0, y0, z0 = rr * math.cos(ph), rr * math.sin(ph), rng.uniform(0, b.tau)
            lap = 0.0
            for e in np.eye(3):
                vals = [psi(i, x0 + s * h * e[0], y0 + s * h * e[1], z0 + s * h * e[2]) for s in (-2, -1, 0, 1, 2)]
                lap += np.dot(c, vals)
            p0 = psi(i, x0, y0, z0)
            assert abs(-0.5 * lap - b.kappa[i] * p0) < 1e-5 * max(1.0, b.kappa[i]) * max(abs(p0), 1e-2), (i, rr)


@pytest.mark.parametrize("ncyc,nu", [(2, 1), (3, 2), (4, 1)])
def test_cyclic_index_kinetic_diagonal_is_eigenvalue_of_cartesian_laplacian(ncyc, nu):
    """Cyclic index nu != 0: the Bloch wave exp(-i 2 pi (eta theta1 + nu
    theta2)) F_{m,n,k}, with the radial function of order nN - nu, is an
    eigenfunction of -1/2 Laplacian (Cartesian, 4th-order finite differences)
    with eigenvalue kappa = (1/2)[(b/R)^2 + (2 pi/tau)^2 (m - alpha (nN - nu)
    - eta)^2]: the reading of the nu terms of eq. Simplify_2 is the free
    particle's own operator, and its kinetic part is diagonal."""
    b = ob.make_basis(R=6.0, tau=5.0, alpha=0.3, ecut=6.0, eta=0.2, ncyc=ncyc, nu=nu)
    rng = np.random.default_rng(5 + nu)
    picks = rng.choice(b.L, size=6, replace=False)
    assert np.any(b.mnk[:, 1] == 0)

    def psi(i, x, y, z):
        m, n, k = b.mnk[i]
        r = math.hypot(x, y)
        th1 = z / b.tau
        th2 = math.atan2(y, x) / (2 * math.pi) - b.alpha * z / b.tau
        rad = b.xi(int(n), np.array([k]), np.array([r]))[0, 0]
        return (np.exp(-2j * math.pi * (b.eta * th1 + nu * th2))
                * np.exp(2j * math.pi * (m * th1 + n * ncyc * th2)) * rad)

    h = 1e-2
    c = np.array([-1.0, 16.0, -30.0, 16.0, -1.0]) / (12 * h * h)
    for i in list(picks) + list(np.nonzero(b.mnk[:, 1] == 0)[0][:2]):
        for _ in range(3):
            rr = rng.uniform(1.0, b.R - 1.0)
            ph = rng.uniform(0, 2 * math.pi)
            x0, y0, z0 = rr * math.cos(ph), rr * math.sin(ph), rng.uniform(0, b.tau)
            lap = 0.0
            for e in np.eye(3):
                vals = [psi(i, x0 + s * h * e[0], y0 + s * h * e[1], z0 + s * h * e[2]) for s in (-2, -1, 0, 1, 2)]
                lap += np.dot(c, vals)
            p0 = psi(i, x0, y0, z0)
            assert abs(-0.5 * lap - b.kappa[i] * p0) < 1e-5 * max(1.0, b.kappa[i]) * max(abs(p0), 1e-2), (i, rr)


@pytest.mark.parametrize("ncyc,nu", [(2, 1), (3, 1), (3, 2)])
def test_cyclic_index_operator_is_a_sector_of_the_order_one_operator(ncyc, nu):
    """Cyclic index nu != 0 (Sec. 2.3): for an N-fold symmetric potential the
    order-1 operator's angular indices n' = nN - nu (n' = -nu mod N) form a
    block, and that block is the (N, nu) operator entry for entry: same index
    set (radial order |n'|, kinetic energy with alpha n'), same matrix,
    although the (N, nu) basis lives on the wedge theta2 in [0, 1/N) with the
    Bloch factor exp(-i 2 pi nu theta2) taken out.  The cutoff, not the grid,
    limits n' here, so both index sets are complete."""
    n1, n2, nr = 12, 16, 32
    kw = dict(R=6.5, tau=5.0, alpha=0.15, ecut=3.5, eta=0.2, n_t1=n1, n_r=nr)
    bN = ob.make_basis(n_t2=n2, ncyc=ncyc, nu=nu, **kw)
    b1 = ob.make_basis(n_t2=ncyc * n2, ncyc=1, **kw)
    assert np.abs(b1.mnk[:, 1]).max() < (ncyc * n2 - 1) // 2 and np.abs(bN.mnk[:, 1]).max() < (n2 - 1) // 2
    motif = synth.atoms_for("helix6", 8, bN.tau, bN.R)[:2]
    atoms = synth.cyclic_images(motif, ncyc)
    V1 = synth.potential_at(b1.theta1, b1.theta2, b1.r, b1.tau, b1.alpha, atoms)
    VN = synth.potential_at(bN.theta1, bN.theta2, bN.r, bN.tau, bN.alpha, atoms)
    H1 = oh.dense_explicit(b1, V1)
    HN = oh.dense_explicit(bN, VN)
    sector = np.nonzero((b1.mnk[:, 1] + nu) % ncyc == 0)[0]
    other = np.nonzero((b1.mnk[:, 1] + nu) % ncyc != 0)[0]
    assert np.max(np.abs(H1[np.ix_(sector, other)])) < 1e-13 * np.max(np.abs(H1))
    key1 = {(int(m), (int(n) + nu) // ncyc, int(k)): i for i, (m, n, k) in enumerate(b1.mnk[sector])}
    keyN = [(int(m), int(n), int(k)) for m, n, k in bN.mnk]
    assert sorted(key1) == sorted(keyN)
    perm = np.array([sector[key1[t]] for t in keyN])
    np.testing.assert_allclose(bN.kappa, b1.kappa[perm], rtol=1e-15)
    assert np.max(np.abs(HN - H1[np.ix_(perm, perm)])) < 1e-13
    lamN = oh.lowest(HN, 10)[0]
    lam1 = np.linalg.eigvalsh(H1[np.ix_(sector, sector)])[:10]
    assert np.max(np.abs(lamN - lam1)) < 1e-12
    # the mode-B form and the matrix-free apply agree with mode A
    assert np.max(np.abs(oh.dense_dft(bN, VN) - HN)) < 1e-13
    X = synth.random_block(bN.mnk, 3, 2)
    assert np.max(np.abs(oh.apply(bN, VN, X) - HN @ X)) < 1e-13


# ------------------------------------------------------------------ transforms
def test_fast_equals_naive_transforms(tiny):
    """The paper's own check: separated sums agree with the naive sums."""
    w, b, V, B = tiny
    x = synth.random_block(b.mnk, 3, 11)
    g1 = ot.inverse_naive(b, x, B)
    g2 = ot.inverse_separable(b, x)
    assert np.max(np.abs(g1 - g2)) < 1e-13
    y1 = ot.forward_naive(b, g1 * V[..., None], B)
    y2 = ot.forward_separable(b, g1 * V[..., None])
    assert np.max(np.abs(y1 - y2)) < 1e-13


def test_round_trip_and_parseval(tiny):
    w, b, V, B = tiny
    x = synth.random_block(b.mnk, 4, 5)
    g = ot.inverse_separable(b, x)
    assert np.max(np.abs(ot.forward_separable(b, g) - x)) < 1e-13
    W = ot.grid_weights(b)
    for j in range(4):
        assert abs(np.sum(W * np.abs(g[..., j]) ** 2) - np.vdot(x[:, j], x[:, j]).real) < 1e-13


# ------------------------------------------------------------------ Hamiltonian
def test_dense_modes_agree_and_are_hermitian(tiny):
    w, b, V, B = tiny
    HA = oh.dense_explicit(b, V, B)
    HB = oh.dense_dft(b, V)
    assert np.max(np.abs(HA - HB)) < 1e-13
    assert np.max(np.abs(HA - HA.conj().T)) < 1e-14
    X = synth.random_block(b.mnk, 5, 3)
    assert np.max(np.abs(oh.apply(b, V, X) - HA @ X)) < 1e-13


def test_mode_pair_assembly_equals_the_basis_matrix_form(tiny):
    """dense_dft_modes (mode B one pair of angular modes at a time, used for
    mid-size golden eigenvalues) against the explicit basis-matrix form, on
    the tiny workload and on a twisted, eta-shifted basis whose modes have
    ragged radial lengths; its lowest eigenvalues against LAPACK on mode A."""
    w, b, V, B = tiny
    HA = oh.dense_explicit(b, V, B)
    assert np.max(np.abs(oh.dense_dft_modes(b, V) - HA)) < 1e-13
    lam = oh.lowest_values(oh.dense_dft_modes(b, V), 8)
    assert np.max(np.abs(lam - oh.lowest(HA, 8)[0])) < 1e-12
    b2 = small_basis()
    V2 = synth.potential_at(b2.theta1, b2.theta2, b2.r, b2.tau, b2.alpha,
                            synth.atoms_for("helix6", 4, b2.tau, b2.R))
    assert len(set(b2.mnk[:, 2].tolist())) > 1
    assert np.max(np.abs(oh.dense_dft_modes(b2, V2) - oh.dense_explicit(b2, V2))) < 1e-13


@pytest.mark.parametrize("ncyc", [2, 3])
def test_cyclic_operator_is_the_symmetric_sector_of_the_order_one_operator(ncyc):
    """Cyclic order N (Sec. 2.3, App. B; nu = 0): for an N-fold symmetric
    potential the order-1 operator does not couple angular index n' across
    residues mod N, and its n' = N n sector is the order-N operator: same
    index set (Bessel order N|n|, kinetic energy with alpha N n), and entry
    for entry the same matrix, although the order-N basis lives on the wedge
    theta2 in [0, 1/N) with its own normalisation sqrt(N / (pi tau)) and
    wedge quadrature weights.  Eigenvalues therefore agree too."""
    n1, n2, nr = 12, 8, 32
    kw = dict(R=6.5, tau=5.0, alpha=0.15, ecut=7.0, eta=0.2, n_t1=n1, n_r=nr)
    bN = ob.make_basis(n_t2=n2, ncyc=ncyc, **kw)
    b1 = ob.make_basis(n_t2=ncyc * n2, ncyc=1, **kw)
    motif = synth.atoms_for("helix6", 8, bN.tau, bN.R)[:2]
    atoms = synth.cyclic_images(motif, ncyc)
    V1 = synth.potential_at(b1.theta1, b1.theta2, b1.r, b1.tau, b1.alpha, atoms)
    VN = synth.potential_at(bN.theta1, bN.theta2, bN.r, bN.tau, bN.alpha, atoms)
    np.testing.assert_allclose(bN.theta2, b1.theta2[:n2], rtol=0, atol=1e-16)
    H1 = oh.dense_explicit(b1, V1)
    HN = oh.dense_explicit(bN, VN)
    sector = np.nonzero(b1.mnk[:, 1] % ncyc == 0)[0]
    other = np.nonzero(b1.mnk[:, 1] % ncyc != 0)[0]
    assert np.max(np.abs(H1[np.ix_(sector, other)])) < 1e-13 * np.max(np.abs(H1))
    # the sector's index set is the order-N set with n' = N n
    key1 = {(int(m), int(n) // ncyc, int(k)): i for i, (m, n, k) in enumerate(b1.mnk[sector])}
    keyN = [(int(m), int(n), int(k)) for m, n, k in bN.mnk]
    assert sorted(key1) == sorted(keyN)
    perm = np.array([sector[key1[t]] for t in keyN])
    np.testing.assert_allclose(bN.kappa, b1.kappa[perm], rtol=1e-15)
    assert np.max(np.abs(HN - H1[np.ix_(perm, perm)])) < 1e-13
    m, n = bN.mnk[:, 0], bN.mnk[:, 1]
    alg5 = ob.kinetic_alg5(bN.bzero, m, n, bN.R, bN.tau, bN.alpha, bN.eta, ncyc=ncyc)
    np.testing.assert_allclose(alg5.real, bN.kappa, rtol=1e-13)
    assert np.max(np.abs(alg5.imag)) < 1e-13
    lamN = oh.lowest(HN, 10)[0]
    lam1 = np.linalg.eigvalsh(H1[np.ix_(sector, sector)])[:10]
    assert np.max(np.abs(lamN - lam1)) < 1e-12
    # the mode-B form and the matrix-free apply agree with mode A at order N
    assert np.max(np.abs(oh.dense_dft(bN, VN) - HN)) < 1e-13
    X = synth.random_block(bN.mnk, 3, 2)
    assert np.max(np.abs(oh.apply(bN, VN, X) - HN @ X)) < 1e-13


def test_matrix_free_apply_is_hermitian():
    b = small_basis()
    atoms = synth.atoms_for("helix6", 9, b.tau, b.R)
    V = synth.potential_at(b.theta1, b.theta2, b.r, b.tau, b.alpha, atoms)
    x = synth.random_block(b.mnk, 1, 1)[:, 0]
    y = synth.random_block(b.mnk, 1, 2)[:, 0]
    lhs = np.vdot(y, oh.apply(b, V, x))
    rhs = np.conj(np.vdot(x, oh.apply(b, V, y)))
    assert abs(lhs - rhs) < 1e-14


def test_free_particle_closed_form():
    """V = 0: H is the kinetic diagonal, eigenvalues are the sorted kappa."""
    b = small_basis(alpha=0.41, eta=-0.3)
    V = np.zeros((b.n_t1, b.n_t2, b.n_r))
    H = oh.dense_dft(b, V)
    assert np.max(np.abs(H - np.diag(b.kappa))) == 0.0
    ev, _ = oh.lowest(oh.dense_explicit(b, V), 10)
    # closed form from the Laplacian eigenvalues and the Bloch shift
    lam0 = (b.bzero / b.R) ** 2 + (2 * math.pi / b.tau * (b.mnk[:, 0] - b.alpha * b.mnk[:, 1])) ** 2
    shifted = 0.5 * lam0 - (2 * math.pi / b.tau) ** 2 * b.eta * (b.mnk[:, 0] - b.alpha * b.mnk[:, 1]) \
        + 0.5 * (2 * math.pi / b.tau * b.eta) ** 2
    np.testing.assert_allclose(ev, np.sort(shifted)[:10], rtol=1e-13, atol=1e-14)


def test_constant_potential_shifts_spectrum():
    b = small_basis()
    V0 = -1.7
    V = np.full((b.n_t1, b.n_t2, b.n_r), V0)
    ev, _ = oh.lowest(oh.dense_explicit(b, V), 12)
    np.testing.assert_allclose(ev, np.sort(b.kappa)[:12] + V0, atol=1e-12)


def test_cosine_potential_couples_neighbouring_m_only():
    """V = V1 cos(2 pi (theta1 - phi0)) couples (m, n, k) to (m +- 1, n, k) with
    V1/2 exp(-+ i 2 pi phi0); eigenvalues are those of per-(n, k) tridiagonal
    chains in m (LAPACK stev)."""
    b = small_basis(n_t1=16)
    V1, phi0 = 0.8, 0.13
    V = np.broadcast_to(V1 * np.cos(2 * math.pi * (b.theta1 - phi0))[:, None, None],
                        (b.n_t1, b.n_t2, b.n_r)).copy()
    H = oh.dense_explicit(b, V)
    idx = {tuple(t): i for i, t in enumerate(b.mnk.tolist())}
    expect = np.diag(b.kappa).astype(np.complex128)
    for (m, n, k), i in idx.items():
        j = idx.get((m + 1, n, k))
        if j is not None:
            expect[j, i] = 0.5 * V1 * np.exp(-2j * math.pi * phi0)
            expect[i, j] = np.conj(expect[j, i])
    assert np.max(np.abs(H - expect)) < 1e-12
    chains = {}
    for (m, n, k), i in idx.items():
        chains.setdefault((n, k), []).append((m, b.kappa[i]))
    evs = []
    for key, lst in chains.items():
        lst.sort()
        d = np.array([t[1] for t in lst])
        e = np.full(len(d) - 1, 0.5 * V1)
        evs.extend(sla.eigh_tridiagonal(d, e, eigvals_only=True, lapack_driver="stev") if len(d) > 1 else d)
    evs = np.sort(evs)
    ev, _ = oh.lowest(H, 15)
    np.testing.assert_allclose(ev, evs[:15], atol=1e-12)


def test_grid_shift_invariance():
    b = small_basis()
    atoms = synth.atoms_for("helix6", 4, b.tau, b.R)
    V = synth.potential_at(b.theta1, b.theta2, b.r, b.tau, b.alpha, atoms)
    ev0, _ = oh.lowest(oh.dense_dft(b, V), 10)
    ev1, _ = oh.lowest(oh.dense_dft(b, np.roll(V, 5, axis=0)), 10)
    ev2, _ = oh.lowest(oh.dense_dft(b, np.roll(V, -3, axis=1)), 10)
    np.testing.assert_allclose(ev1, ev0, atol=1e-12)
    np.testing.assert_allclose(ev2, ev0, atol=1e-12)


def test_time_reversal():
    """lambda_j(eta) = lambda_j(-eta) at nu = 0 for a real potential (Sec. 3.3)."""
    bp = small_basis(eta=0.23)
    bm = small_basis(eta=-0.23)
    atoms = synth.atoms_for("helix6", 6, bp.tau, bp.R)
    V = synth.potential_at(bp.theta1, bp.theta2, bp.r, bp.tau, bp.alpha, atoms)
    assert bp.L == bm.L
    evp, _ = oh.lowest(oh.dense_dft(bp, V), 10)
    evm, _ = oh.lowest(oh.dense_dft(bm, V), 10)
    np.testing.assert_allclose(evp, evm, atol=1e-12)


@pytest.mark.parametrize("ncyc,nu", [(3, 1), (4, 1), (4, 2)])
def test_time_reversal_with_cyclic_index(ncyc, nu):
    """lambda_j(eta, nu) = lambda_j(-eta, N - nu) for a real N-fold symmetric
    potential (Sec. 3.3); at nu = N/2 the index is its own partner."""
    kw = dict(R=6.5, tau=5.0, alpha=0.15, ecut=5.0, n_t1=12, n_t2=16, n_r=32, ncyc=ncyc)
    bp = ob.make_basis(eta=0.23, nu=nu, **kw)
    bm = ob.make_basis(eta=-0.23, nu=(ncyc - nu) % ncyc, **kw)
    atoms = synth.cyclic_images(synth.atoms_for("helix6", 8, bp.tau, bp.R)[:2], ncyc)
    V = synth.potential_at(bp.theta1, bp.theta2, bp.r, bp.tau, bp.alpha, atoms)
    assert bp.L == bm.L
    evp, _ = oh.lowest(oh.dense_dft(bp, V), 10)
    evm, _ = oh.lowest(oh.dense_dft(bm, V), 10)
    np.testing.assert_allclose(evp, evm, atol=1e-12)


def test_eigenvalues_converge_with_cutoff():
    """Qualitative check: the lowest eigenvalue decreases towards a limit as the
    cutoff grows (variational in a nested basis with an exact quadrature)."""
    vals = []
    for ecut in (3.0, 5.0, 8.0):
        b = ob.make_basis(R=6.0, tau=5.0, alpha=0.0, ecut=ecut, n_t1=24, n_t2=24, n_r=64)
        atoms = synth.atoms_for("helix6", 2, b.tau, b.R)
        V = synth.potential_at(b.theta1, b.theta2, b.r, b.tau, b.alpha, atoms)
        vals.append(oh.lowest(oh.dense_dft(b, V), 1)[0][0])
    assert vals[0] >= vals[1] - 1e-9 >= vals[2] - 2e-9


# ------------------------------------------------------------------ preconditioner
def test_tpa_worked_values():
    assert op.tpa_factor(0.0) == 1.0
    assert abs(op.tpa_factor(1.0) - 65.0 / 81.0) < 1e-16
    g = np.linspace(0, 50, 2001)
    K = op.tpa_factor(g)
    assert np.all(np.diff(K) < 0)
    assert abs(op.tpa_factor(1e6) * 2e6 - 1.0) < 1e-5
    kappa = np.array([0.5, 2.0, 7.0])
    r = np.array([0.0, 3.0 + 4.0j, 0.0])
    w = op.tpa_apply(kappa, r)
    np.testing.assert_allclose(w, r * 65.0 / 81.0, rtol=1e-15)
    assert np.all(op.tpa_apply(kappa, np.zeros((3, 2))) == 0)


# ------------------------------------------------------------------ learned preconditioner
def _mlp_case(seed=0, L=40, ncol=3):
    from oracle import mlp
    rng = np.random.default_rng(seed)
    kappa = np.sort(rng.uniform(0.05, 9.0, L))
    vdiag = rng.uniform(-2.0, 0.0, L)
    R = rng.standard_normal((L, ncol)) + 1j * rng.standard_normal((L, ncol))
    Tt = rng.standard_normal((L, ncol)) + 1j * rng.standard_normal((L, ncol))
    lam = rng.uniform(-1.0, 0.5, ncol)
    F, K = mlp.features(kappa, vdiag, R, lam)
    theta = mlp.init_params(seed)
    theta[-65:] = rng.standard_normal(65) * 0.3      # non-zero last layer
    return mlp, F, K, R, Tt, theta


def test_mlp_gradient_matches_finite_differences():
    mlp, F, K, R, Tt, theta = _mlp_case()
    loss, grad = mlp.loss_and_grad(theta, F, K, R, Tt)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 40, replace=False), [mlp.NPARAM - 1]])
    h = 1e-6
    for i in idx:
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd = (mlp.loss_and_grad(tp, F, K, R, Tt)[0] - mlp.loss_and_grad(tm, F, K, R, Tt)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-6 * max(1.0, abs(grad[i])) + 1e-9, (i, fd, grad[i])


def test_mlp_untrained_network_is_tpa_and_loss_invariances():
    from oracle import precond as op
    mlp, F, K, R, Tt, theta = _mlp_case(2)
    theta0 = mlp.init_params(5)
    s, _ = mlp.forward(theta0, F, K)
    np.testing.assert_allclose(s, K, rtol=1e-15)
    kappa = np.exp(F[:, 0, 2])
    np.testing.assert_allclose(s * R, op.tpa_apply(kappa, R), rtol=1e-12)
    l1, _ = mlp.loss_and_grad(theta, F, K, R, Tt)
    l2, _ = mlp.loss_and_grad(theta, F, K, R, (2.5 - 1.5j) * Tt)   # target scale and phase do not matter
    assert abs(l1 - l2) < 1e-14 and 0.0 <= l1 <= 1.0
    sr = mlp.forward(theta, F, K)[0] * R
    l0, g0 = mlp.loss_and_grad(theta, F, K, R, sr)                  # target along s r: zero loss, zero gradient
    assert abs(l0) < 1e-14 and np.max(np.abs(g0)) < 1e-12


def test_adam_step_against_the_published_algorithm():
    """oracle.mlp.adam_step against Kingma & Ba (2015), Algorithm 1: moments
    m_t = b1 m + (1 - b1) g, v_t = b2 v + (1 - b2) g^2, bias-corrected by
    1 - b^t, step -lr m_hat / (sqrt(v_hat) + eps)."""
    from oracle import mlp
    rng = np.random.default_rng(3)
    g = rng.standard_normal(50) * np.logspace(-3, 2, 50)
    theta0 = rng.standard_normal(50)
    # first step from zero moments: the bias corrections give m_hat = g and
    # v_hat = g^2, so every coordinate moves by exactly lr * g / (|g| + eps)
    th, m, v = mlp.adam_step(theta0, g, np.zeros(50), np.zeros(50), 1, 0.01)
    np.testing.assert_allclose(th, theta0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g, rtol=4e-15)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=4e-15)
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step t
    # (wrong powers of b1, b2 in the bias correction break this)
    th, m, v = theta0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 31):
        prev = th
        th, m, v = mlp.adam_step(th, g, m, v, t, 0.01)
        np.testing.assert_allclose(prev - th, 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-17)
    # two steps worked by hand (40-digit decimal arithmetic): g = 1 then
    # g = -1/2, lr = 0.1 from theta = 0: m = 0.04, v = 0.001249 after step 2
    th, m, v = mlp.adam_step(np.zeros(1), np.ones(1), np.zeros(1), np.zeros(1), 1, 0.1)
    assert abs(th[0] - (-0.0999999990000000099999999)) < 1e-16
    th, m, v = mlp.adam_step(th, -0.5 * np.ones(1), m, v, 2, 0.1)
    assert abs(m[0] - 0.04) < 1e-16 and abs(v[0] - 0.001249) < 1e-17
    assert abs(th[0] - (-0.1266337026290970334541760)) < 1e-15


def test_potential_diagonal_is_the_dense_diagonal():
    """V_ii (input feature of the learned preconditioner) against the
    diagonal of the mode-A matrix built from the explicit basis matrix."""
    w = synth.workload("tiny-helix").with_(alpha=0.2, eta=0.3)
    b = ob.basis_for(w)
    atoms = synth.atoms_for(w.structure, w.seed, w.tau, w.R)
    V = synth.potential_at(b.theta1, b.theta2, b.r, w.tau, w.alpha, atoms)
    H = oh.dense_explicit(b, V)
    vd = oh.potential_diagonal(b, V)
    np.testing.assert_allclose(vd, np.real(np.diag(H)) - b.kappa, rtol=0, atol=1e-12 * np.abs(V).max())


# ------------------------------------------------------------------ density
def test_density_integral_is_the_weighted_norm_sum(tiny):
    """Parseval on the grid: sum_g W_g rho_g = sum_j occ_j ||x_j||^2 (the
    quadrature integrates |phi|^2 of band-limited functions exactly)."""
    from oracle import density as od
    w, b, V, B = tiny
    X = synth.random_block(b.mnk, 5, 21)
    occ = np.array([2.0, 2.0, 1.5, 0.5, 0.25])
    rho = od.density(b, X, occ)
    W = ot.grid_weights(b)
    want = float(np.sum(occ * np.sum(np.abs(X) ** 2, axis=0)))
    assert rho.min() >= 0.0
    assert abs(np.sum(W * rho) - want) < 1e-12 * want


def test_density_of_one_basis_function_is_its_radial_factor_squared(tiny):
    """|F_mnk|^2 = xi_{n,k}(r)^2 at every angle (the angular factors have unit
    modulus): the closed form of a one-state density."""
    from oracle import density as od
    w, b, V, B = tiny
    for i in (0, b.L // 3, b.L - 1):
        x = np.zeros(b.L, dtype=np.complex128)
        x[i] = 1.0
        rho = od.density(b, x, np.array([1.0]))
        m, n, k = b.mnk[i]
        xi = b.xi(int(n), np.array([k]))[:, 0]
        want = np.broadcast_to(xi ** 2, rho.shape)
        assert np.max(np.abs(rho - want)) < 1e-12 * np.max(want)


def test_density_against_the_basis_matrix(tiny):
    """The same density from the naive inverse transform (explicit basis
    matrix, eq. Naive_Inverse_Transform)."""
    from oracle import density as od
    w, b, V, B = tiny
    X = synth.random_block(b.mnk, 3, 22)
    occ = np.array([1.0, 0.75, 0.5])
    g = ot.inverse_naive(b, X, B)
    want = np.einsum("ijlv,v->ijl", np.abs(g) ** 2, occ)
    assert np.max(np.abs(od.density(b, X, occ) - want)) < 1e-12 * np.max(want)


# ------------------------------------------------------------------ gradients (App. C)
def test_gradient_of_one_function_closed_forms(tiny):
    """F = exp(i 2 pi (m theta1 + n theta2)) xi_{n,k}(r): E_theta1 = i 2 pi m F,
    E_theta2 = i 2 pi n F, and E_r = exp(...) d xi/dr, the latter against a
    central difference of xi."""
    from oracle import gradient as og
    w, b, V, B = tiny
    h = 1e-5 * b.R
    for i in (0, b.L // 2, b.L - 1):
        m, n, k = (int(t) for t in b.mnk[i])
        x = np.zeros(b.L, dtype=np.complex128)
        x[i] = 1.0
        F = ot.inverse_naive(b, x, B)
        e1, e2, er = og.helical_derivatives(b, x)
        scale = np.max(np.abs(F)) * 2 * math.pi * max(1, abs(m), abs(n))
        assert np.max(np.abs(e1 - 2j * math.pi * m * F)) < 1e-12 * scale
        assert np.max(np.abs(e2 - 2j * math.pi * n * F)) < 1e-12 * scale
        dxi = (b.xi(n, np.array([k]), b.r + h)[:, 0] - b.xi(n, np.array([k]), b.r - h)[:, 0]) / (2 * h)
        ang = np.exp(2j * math.pi * (m * b.theta1[:, None] + n * b.theta2[None, :]))
        want = ang[:, :, None] * dxi[None, None, :]
        assert np.max(np.abs(er - want)) < 1e-7 * np.max(np.abs(want))


@pytest.mark.parametrize("ncyc", [1, 2])
def test_cartesian_gradient_against_finite_differences(ncyc):
    """The chain rule of eq. Cartesian_Derivatives against central differences
    of the field evaluated at Cartesian points (x, y, z) mapped back to
    helical coordinates: theta1 = z / tau, phi = atan2(y, x),
    theta2 = phi / (2 pi) - alpha theta1, r = sqrt(x^2 + y^2); also at cyclic
    order 2 (angular factor exp(i 2 pi n N theta2), Bessel order |n| N)."""
    from oracle import gradient as og
    b = small_basis(ncyc=ncyc)
    rng = np.random.default_rng(8)
    idx = rng.choice(b.L, 6, replace=False)
    coef = rng.standard_normal(6) + 1j * rng.standard_normal(6)
    x = np.zeros(b.L, dtype=np.complex128)
    x[idx] = coef

    def field(px, py, pz):
        t1 = pz / b.tau
        t2 = math.atan2(py, px) / (2 * math.pi) - b.alpha * t1
        rr = math.hypot(px, py)
        s = 0.0
        for i, c in zip(idx, coef):
            m, n, k = (int(t) for t in b.mnk[i])
            s += c * np.exp(2j * math.pi * (m * t1 + n * ncyc * t2)) * b.xi(n, np.array([k]), np.array([rr]))[0, 0]
        return s

    ex, ey, ez = og.cartesian(b, *og.helical_derivatives(b, x))
    h = 1e-5
    for (i1, i2, l) in ((1, 3, 10), (5, 9, 20), (10, 14, 28), (7, 0, 5)):
        t1, t2, rr = b.theta1[i1], b.theta2[i2], b.r[l]
        phi = 2 * math.pi * (b.alpha * t1 + t2)
        p = np.array([rr * math.cos(phi), rr * math.sin(phi), b.tau * t1])
        fd = []
        for d in range(3):
            e = np.zeros(3)
            e[d] = h
            fd.append((field(*(p + e)) - field(*(p - e))) / (2 * h))
        got = np.array([ex[i1, i2, l], ey[i1, i2, l], ez[i1, i2, l]])
        assert np.max(np.abs(got - np.array(fd))) < 1e-6 * max(1.0, np.max(np.abs(fd))), (i1, i2, l, got, fd)
