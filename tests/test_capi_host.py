"""Host side of the C ABI (no GPU): exported symbols, the set-up's own special
functions and index set against the oracle, parameter validation."""
import math
import os
import re

import numpy as np
import pytest
import scipy.special as sp

import synth
from oracle import basis as ob

helic = pytest.importorskip("paper_2210_12252_amd.helic")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return helic.load()


def test_exports_every_declared_symbol(lib):
    text = open(os.path.join(ROOT, "include", "helic.h")).read()
    declared = set(re.findall(r"\b(helic_[a-z_0-9A-Z]+)\s*\(", text))
    assert declared, "no declarations found"
    assert declared == set(helic.EXPORTS)
    for name in declared:
        assert hasattr(lib, name), name


@pytest.mark.parametrize("p", [0, 1, 2, 7, 31, 64, 130])
def test_bessel_j_matches_scipy(p):
    x = np.concatenate([[0.0, 1e-3, 0.5], np.linspace(1.0, 250.0, 997)])
    ours = helic.util_bessel_j(p, x)
    ref = sp.jv(p, x)
    assert np.max(np.abs(ours - ref)) < 2e-14
    neg = helic.util_bessel_j(-p, x)
    assert np.max(np.abs(neg - sp.jv(-p, x))) < 2e-14


@pytest.mark.parametrize("p", [0, 1, 5, 31, 64, 100, 130])
def test_bessel_zeros_match_oracle(p):
    ours = helic.util_bessel_zeros(p, 70)
    ref = ob.bessel_zeros(p, 70)
    np.testing.assert_allclose(ours, ref, rtol=1e-13, atol=0)
    assert np.all(np.abs(sp.jv(p, ours)) < 1e-14)


def test_bessel_zeros_table():
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "bessel_zeros.txt"))
            if not l.startswith("#")]
    for p, k, v in rows:
        assert abs(helic.util_bessel_zeros(int(p), int(k))[-1] - float(v)) < 1e-13


@pytest.mark.parametrize("n", [1, 2, 8, 48, 160, 256])
def test_gauss_jacobi(n):
    q, w = helic.util_gauss_jacobi(n)
    x, wx = sp.roots_jacobi(n, 0.0, 1.0)
    np.testing.assert_allclose(q, 0.5 * (1 + x), rtol=0, atol=2e-15)
    np.testing.assert_allclose(w, 0.25 * wx, rtol=1e-10, atol=1e-17)  # scipy: moments to ~6e-15 only
    for j in range(2 * n):
        assert abs(np.sum(w * q ** j) - 1.0 / (j + 2)) < 1e-14


def _compare_with_oracle(w):
    b = helic.Basis.from_workload(w)
    o = ob.basis_for(w)
    assert (b.L, b.n_t1, b.n_t2, b.n_r) == (o.L, o.n_t1, o.n_t2, o.n_r)
    mnk, kappa = b.indices()
    ours = {tuple(t): kappa[i] for i, t in enumerate(mnk.tolist())}
    theirs = {tuple(t): o.kappa[i] for i, t in enumerate(o.mnk.tolist())}
    assert set(ours) == set(theirs)
    err = max(abs(ours[k] - theirs[k]) / theirs[k] for k in theirs)
    assert err < 1e-13
    t1, t2, r, wr = b.grid()
    assert np.array_equal(t1, o.theta1) and np.array_equal(t2, o.theta2)
    np.testing.assert_allclose(r, o.r, rtol=0, atol=1e-13 * w.R)
    np.testing.assert_allclose(wr, o.wq, rtol=1e-10, atol=1e-17)
    return b, mnk


@pytest.mark.parametrize("name", ["tiny-helix", "nanotube-ecut25"])
def test_index_set_matches_oracle(name):
    b, mnk = _compare_with_oracle(synth.workload(name))
    # compact order: |n| ascending, +n before -n, m ascending, k = 1..K
    g = np.abs(mnk[:, 1])
    assert np.all(np.diff(g) >= 0)
    key = np.stack([g, (mnk[:, 1] < 0).astype(int), mnk[:, 0], mnk[:, 2]], axis=1)
    for i in range(1, len(key)):
        assert tuple(key[i - 1]) < tuple(key[i])
    b.close()


def test_auto_grid_and_bloch_shift_match_oracle():
    for eta in (-0.5, -0.13, 0.37):
        w = synth.Workload(name="t", R=7.3, tau=6.1, alpha=0.21, ecut=9.5, eta=eta)
        b, _ = _compare_with_oracle(w)
        b.close()


@pytest.mark.parametrize("ncyc", [2, 3, 6])
def test_cyclic_index_set_grid_and_tables_match_oracle(ncyc):
    """Cyclic order N (nu = 0): the index set (Bessel order |n| N), kinetic
    energies (alpha N n), the wedge grid theta2 = j / (N n_t2) and the radial
    weights agree with the oracle, automatic grid and given grid."""
    for grid in ({}, dict(n_t1=16, n_t2=12, n_r=40)):
        w = synth.Workload(name="cyc", R=7.5, tau=5.5, alpha=0.13, ecut=9.0, eta=0.17, ncyc=ncyc, **grid)
        b, _ = _compare_with_oracle(w)
        b.close()


@pytest.mark.parametrize("ncyc,nu", [(2, 1), (3, 1), (3, 2), (4, 1)])
def test_cyclic_index_nu_index_set_matches_oracle(ncyc, nu):
    """Cyclic index nu != 0: radial order |n N - nu|, kinetic energies with
    alpha (n N - nu), groups of one Bessel order (ascending), the wedge grid
    and the radial weights agree with the oracle, automatic and given grid."""
    for grid in ({}, dict(n_t1=16, n_t2=12, n_r=40)):
        w = synth.Workload(name="cyc-nu", R=7.5, tau=5.5, alpha=0.13, ecut=9.0, eta=0.17, ncyc=ncyc, nu=nu, **grid)
        b, mnk = _compare_with_oracle(w)
        order = np.abs(mnk[:, 1] * ncyc - nu)
        assert np.all(np.diff(order) >= 0)
        b.close()


def test_parameter_errors():
    with pytest.raises(helic.HelicError) as e:
        helic.basis_create(R=-1.0, tau=5.0, alpha=0.0, ecut=5.0)
    assert e.value.status == helic.ERR_INVALID
    for nu in (-1, 2):   # the cyclic Bloch index runs over 0 .. N - 1
        with pytest.raises(helic.HelicError) as e:
            helic.basis_create(R=5.0, tau=5.0, alpha=0.0, ecut=5.0, ncyc=2, nu=nu)
        assert e.value.status == helic.ERR_INVALID
    with pytest.raises(helic.HelicError) as e:
        helic.basis_create(R=5.0, tau=5.0, alpha=0.0, ecut=5.0, ncyc=0)
    assert e.value.status == helic.ERR_INVALID
    with pytest.raises(helic.HelicError) as e:
        helic.basis_create(R=5.0, tau=5.0, alpha=0.0, ecut=5.0, eta=0.5)
    assert e.value.status == helic.ERR_INVALID
    with pytest.raises(helic.HelicError) as e:   # the box needs |m| up to 3: 4 bins cannot hold 7 values
        helic.basis_create(R=5.0, tau=5.0, alpha=0.0, ecut=5.0, m_max=3, n_t1=4, n_t2=16, n_r=16)
    assert e.value.status == helic.ERR_GRID
    with pytest.raises(helic.HelicError) as e:   # 7 is not 2,3,5-smooth
        helic.basis_create(R=5.0, tau=5.0, alpha=0.0, ecut=5.0, n_t1=7, n_t2=16, n_r=16)
    assert e.value.status == helic.ERR_GRID
    # E_cut equal to the energy of (m, n, k) = (0, 0, 1): a tie
    R = 5.0
    tie = 0.5 * (sp.jn_zeros(0, 1)[0] / R) ** 2
    with pytest.raises(helic.HelicError) as e:
        helic.basis_create(R=R, tau=5.0, alpha=0.0, ecut=tie)
    assert e.value.status == helic.ERR_CUTOFF_TIE
    with pytest.raises(ValueError):
        ob.make_basis(R=R, tau=5.0, alpha=0.0, ecut=tie)
    assert "tie" in helic.load().helic_last_error().decode()
