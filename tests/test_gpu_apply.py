"""GPU parity of the H*X path and the transforms against the CPU oracle.

Tolerances (derived from the arithmetic): every output element of the FP64
path is a sum of O(K + n_r + log(n_t1 n_t2)) rounded products of terms no
larger than max|kappa| |x| or max|V| |x|; a relative error of 1e-12 of the
column maximum leaves a margin of ~10^2 over the worst case of such sums.
The FP32 path computes the same sums with unit roundoff 6e-8: 2e-5 of the
column maximum.  The BF16 path rounds five quantities to bfloat16 (unit
roundoff u = 2^-9 for rounding to nearest) on the way through the potential
term -- coefficients, inverse table, G, H, forward table -- each a relative
error of at most u of what is rounded, and sums them in FP32; with the
kinetic term exact (FP64) the column error is at most about 5 u times the
size of the potential term's terms, bounded here by 1e-2 of the column
maximum (5 u = 1e-2; measured: 1e-4 to 4e-4 of the column maximum).  A BF16
error below 1e-5 would mean the path is not running in BF16.
"""
import math

import numpy as np
import pytest

import synth
from oracle import basis as ob
from oracle import hamiltonian as oh
from oracle import precond as op
from oracle import transforms as ot

torch = pytest.importorskip("torch")
helic = pytest.importorskip("paper_2210_12252_amd.helic")

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL32 = 2e-5
TOL16 = 1e-2
BF16_FLOOR = 1e-5


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


class Case:
    """A basis on both sides, the permutation between their row orders and a
    potential sampled on the oracle's grid."""

    def __init__(self, w, potential=True):
        self.w = w
        self.o = ob.basis_for(w)
        self.g = helic.Basis.from_workload(w)
        mnk, _ = self.g.indices()
        pos = {tuple(t): i for i, t in enumerate(self.o.mnk.tolist())}
        self.perm = np.array([pos[tuple(t)] for t in mnk.tolist()])   # gpu row -> oracle row
        self.mnk = mnk
        atoms = synth.atoms_for(w.structure, w.seed, w.tau, w.R) if potential else []
        self.V = synth.potential_at(self.o.theta1, self.o.theta2, self.o.r, w.tau, w.alpha, atoms)
        print(f"[case] {w.name} L={self.o.L} grid={self.o.n_t1}x{self.o.n_t2}x{self.o.n_r}", flush=True)

    def upload_V(self, V=None):
        V = self.V if V is None else V
        self.g.set_potential(torch.from_numpy(np.ascontiguousarray(V)).to(_dev()))

    def to_gpu_block(self, Xo, ld=None):
        """oracle-order (L, nv) -> device tensor (nv, ld) in library order"""
        L, nv = Xo.shape
        ld = L if ld is None else ld
        out = np.zeros((nv, ld), dtype=np.complex128)
        out[:, :L] = Xo[self.perm].T
        return torch.from_numpy(out).to(_dev())

    def from_gpu_block(self, Yg):
        Y = Yg.cpu().numpy()[:, :self.o.L].T
        out = np.empty_like(Y)
        out[self.perm] = Y
        return out


@pytest.fixture(scope="module")
def tiny():
    _dev()
    c = Case(synth.workload("tiny-helix"))
    c.upload_V()
    return c


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def test_inverse_transform_parity(tiny):
    X = synth.random_block(tiny.o.mnk, 5, 21)
    g = torch.empty((5, tiny.o.n_t1, tiny.o.n_t2, tiny.o.n_r), dtype=torch.complex128, device=_dev())
    tiny.g.transform_inverse(tiny.to_gpu_block(X), g)
    ref = np.moveaxis(ot.inverse_separable(tiny.o, X), -1, 0)
    assert _rel(g.cpu().numpy(), ref) < TOL64


def test_forward_transform_parity(tiny):
    rng = np.random.default_rng(4)
    shape = (3, tiny.o.n_t1, tiny.o.n_t2, tiny.o.n_r)
    gr = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    Xg = torch.zeros((3, tiny.o.L), dtype=torch.complex128, device=_dev())
    tiny.g.transform_forward(torch.from_numpy(gr).to(_dev()), Xg)
    ref = ot.forward_separable(tiny.o, np.moveaxis(gr, 0, -1))
    assert _rel(tiny.from_gpu_block(Xg), ref) < TOL64


@pytest.mark.parametrize("nvec,ld_pad", [(1, 0), (8, 0), (67, 5)])
def test_apply_H_parity_tiny(tiny, nvec, ld_pad):
    HA = oh.dense_explicit(tiny.o, tiny.V)
    X = synth.random_block(tiny.o.mnk, nvec, 100 + nvec)
    ld = tiny.o.L + ld_pad
    Xg = tiny.to_gpu_block(X, ld)
    Yg = torch.full((nvec, ld), 7.0 + 0j, dtype=torch.complex128, device=_dev())
    tiny.g.apply_H(Xg, Yg)
    torch.cuda.synchronize()
    ref = HA @ X
    Y = tiny.from_gpu_block(Yg)
    for j in range(nvec):
        assert np.max(np.abs(Y[:, j] - ref[:, j])) <= TOL64 * np.max(np.abs(ref[:, j])), j
    if ld_pad:   # padding rows beyond L untouched
        assert torch.all(Yg[:, tiny.o.L:] == 7.0)


def test_apply_H_fp32_parity_tiny(tiny):
    HA = oh.dense_explicit(tiny.o, tiny.V)
    X = synth.random_block(tiny.o.mnk, 16, 5)
    Yg = torch.zeros((16, tiny.o.L), dtype=torch.complex128, device=_dev())
    tiny.g.apply_H(tiny.to_gpu_block(X), Yg, prec="fp32")
    ref = HA @ X
    Y = tiny.from_gpu_block(Yg)
    for j in range(16):
        assert np.max(np.abs(Y[:, j] - ref[:, j])) <= TOL32 * np.max(np.abs(ref[:, j])), j


def test_apply_H_bf16_parity_tiny(tiny):
    """BF16 radial contractions and slabs, FP32 angular stage: every column
    against the dense oracle at the BF16 bound."""
    HA = oh.dense_explicit(tiny.o, tiny.V)
    X = synth.random_block(tiny.o.mnk, 16, 5)
    Yg = torch.zeros((16, tiny.o.L), dtype=torch.complex128, device=_dev())
    tiny.g.apply_H(tiny.to_gpu_block(X), Yg, prec="bf16")
    ref = HA @ X
    Y = tiny.from_gpu_block(Yg)
    errs = [np.max(np.abs(Y[:, j] - ref[:, j])) / np.max(np.abs(ref[:, j])) for j in range(16)]
    print(f"[tiny bf16] column errors max {max(errs):.2e} min {min(errs):.2e}", flush=True)
    assert max(errs) <= TOL16 and min(errs) > BF16_FLOOR


def test_apply_H_free_particle_and_constant_potential():
    w = synth.Workload(name="ragged", R=7.0, tau=5.5, alpha=0.3, ecut=11.0, eta=0.21,
                       n_t1=20, n_t2=30, n_r=52)
    c = Case(w, potential=False)
    X = synth.random_block(c.o.mnk, 9, 3)
    Xg = c.to_gpu_block(X)
    Yg = torch.zeros_like(Xg)
    c.upload_V(np.zeros_like(c.V))
    c.g.apply_H(Xg, Yg)
    ref = c.o.kappa[:, None] * X
    assert _rel(c.from_gpu_block(Yg), ref) < TOL64
    c.upload_V(np.full_like(c.V, -1.25))
    c.g.apply_H(Xg, Yg)
    ref = (c.o.kappa[:, None] - 1.25) * X
    assert _rel(c.from_gpu_block(Yg), ref) < 1e-11   # radial orthogonality holds to ~1e-13 at n_r = 52


def test_apply_H_is_hermitian_and_deterministic(tiny):
    x = synth.random_block(tiny.o.mnk, 2, 8)
    Xg = tiny.to_gpu_block(x)
    Yg = torch.zeros_like(Xg)
    tiny.g.apply_H(Xg, Yg)
    Y2 = torch.zeros_like(Xg)
    tiny.g.apply_H(Xg, Y2)
    assert torch.equal(Yg, Y2)
    Y = tiny.from_gpu_block(Yg)
    lhs = np.vdot(x[:, 1], Y[:, 0])
    rhs = np.conj(np.vdot(x[:, 0], Y[:, 1]))
    assert abs(lhs - rhs) < 1e-13


def test_apply_H_empty_and_errors(tiny):
    Xg = torch.zeros((0, tiny.o.L), dtype=torch.complex128, device=_dev())
    tiny.g.apply_H(Xg, Xg.clone())
    bad = torch.zeros((2, tiny.o.L - 1), dtype=torch.complex128, device=_dev())
    with pytest.raises(helic.HelicError) as e:
        tiny.g.apply_H(bad, bad.clone())
    assert e.value.status == helic.ERR_INVALID
    fresh = helic.Basis.from_workload(tiny.w)
    X = torch.zeros((1, tiny.o.L), dtype=torch.complex128, device=_dev())
    with pytest.raises(helic.HelicError) as e:
        fresh.apply_H(X, X.clone())
    assert e.value.status == helic.ERR_STATE


def test_precondition_parity(tiny):
    Rr = synth.random_block(tiny.o.mnk, 6, 17, normalize=False)
    Rr[:, 2] = 0.0
    Rg = tiny.to_gpu_block(Rr)
    Wg = torch.zeros_like(Rg)
    tiny.g.precondition(Rg, Wg)
    ref = op.tpa_apply(tiny.o.kappa, Rr)
    assert _rel(tiny.from_gpu_block(Wg), ref) < 1e-14
    tiny.g.precondition(Rg, Rg)   # in place
    assert _rel(tiny.from_gpu_block(Rg), ref) < 1e-14


@pytest.mark.parametrize("name", ["nanotube-ecut25", "nanotube-ecut40", "nanowire-ecut30"])
def test_apply_H_full_size_sampled(name):
    """Full workload size in the launch configuration of the benchmark (one
    64-vector block); columns 0, 31 and 63 checked against the matrix-free
    oracle, the rest through Hermiticity of sampled pairs."""
    w = synth.workload(name)
    c = Case(w)
    c.upload_V()
    X = synth.random_block(c.o.mnk, 64, 1234)
    Xg = c.to_gpu_block(X)
    for prec, tol in (("fp64", TOL64), ("fp32", TOL32), ("bf16", TOL16)):
        Yg = torch.zeros_like(Xg)
        c.g.apply_H(Xg, Yg, prec=prec)
        Y = c.from_gpu_block(Yg)
        cols = [0, 31, 63]
        ref = oh.apply(c.o, c.V, X[:, cols])
        for i, j in enumerate(cols):
            err = np.max(np.abs(Y[:, j] - ref[:, i])) / np.max(np.abs(ref[:, i]))
            print(f"[{name} {prec}] column {j} rel err {err:.2e}", flush=True)
            assert err <= tol
        G = X.conj().T @ Y
        herm = np.max(np.abs(G - G.conj().T)) / np.max(np.abs(G))
        assert herm < {"fp64": 1e-12, "fp32": 1e-5, "bf16": 1e-1}[prec]


def test_apply_H_parity_64_column_block():
    """Nanotube geometry at a reduced cutoff on the 48 x 64 grid with 40
    radii: the specialised angular kernel on 64-column blocks (FP64 moves the
    slab straight between global memory and the row transforms' registers,
    FP32 through LDS), a ragged block of 37 vectors spread evenly over the
    resident workgroups (work segments start and end inside radii); every
    output element against the oracle."""
    w = synth.workload("nanotube-ecut25").with_(name="nanotube-ecut10", ecut=10.0, n_t1=48, n_t2=64, n_r=40)
    c = Case(w)
    c.upload_V()
    X = synth.random_block(c.o.mnk, 37, 4242)
    ref = oh.apply(c.o, c.V, X)
    for prec, tol in (("fp64", TOL64), ("fp32", TOL32), ("bf16", TOL16)):
        Yg = torch.zeros((37, c.o.L), dtype=torch.complex128, device=_dev())
        c.g.apply_H(c.to_gpu_block(X), Yg, prec=prec)
        err = _rel(c.from_gpu_block(Yg), ref)
        print(f"[64-column block {prec}] rel err {err:.2e}", flush=True)
        assert err < tol


@pytest.mark.parametrize("workload,n1,n2,ecut", [("nanowire-ecut30", 32, 81, 30.0), ("nanotube-ecut25", 48, 64, 34.0)])
def test_split_angular_kernel_parity(workload, n1, n2, ecut, monkeypatch):
    """Grids served by the split theta1-FFT angular kernel in the FP32 and
    BF16 modes (32 x 81 with all 25 m rows in use, 48 x 64 with 25 of 28
    padded rows), 40 radii, a ragged block of 21 vectors: every output element
    against the oracle, and against the convolution kernel
    (HELIC_ANGULAR_SPLIT=0) on the same inputs (FP64 runs the convolution
    kernel in both)."""
    w = synth.workload(workload).with_(name=f"{workload}-split", ecut=ecut, n_t1=n1, n_t2=n2, n_r=40)
    c = Case(w)
    c.upload_V()
    monkeypatch.setenv("HELIC_ANGULAR_SPLIT", "0")
    conv = helic.Basis.from_workload(w)
    conv.set_potential(torch.from_numpy(c.V).to(_dev()))
    monkeypatch.delenv("HELIC_ANGULAR_SPLIT")
    X = synth.random_block(c.o.mnk, 21, 4243)
    ref = oh.apply(c.o, c.V, X)
    Xg = c.to_gpu_block(X)
    for prec, tol in (("fp64", TOL64), ("fp32", TOL32), ("bf16", TOL16)):
        Yg = torch.zeros((21, c.o.L), dtype=torch.complex128, device=_dev())
        Yc = torch.zeros_like(Yg)
        c.g.apply_H(Xg, Yg, prec=prec)
        conv.apply_H(Xg, Yc, prec=prec)
        err = _rel(c.from_gpu_block(Yg), ref)
        agree = (torch.abs(Yg - Yc).max() / torch.abs(Yc).max()).item()
        print(f"[split {n1}x{n2} {prec}] rel err {err:.2e}, vs convolution kernel {agree:.2e}", flush=True)
        assert err < tol
        assert agree < tol
    conv.close()


@pytest.mark.parametrize("workload,n1,n2,ecut,vchunk", [
    ("nanowire-ecut30", 32, 81, 30.0, 0), ("nanowire-ecut30", 32, 81, 30.0, 1), ("nanowire-ecut30", 32, 81, 30.0, 3),
    ("nanowire-ecut30", 32, 81, 14.0, 0), ("nanowire-ecut30", 32, 81, 14.0, 2),
    ("nanotube-ecut25", 48, 64, 25.0, 0), ("nanotube-ecut25", 48, 64, 34.0, 0), ("nanotube-ecut25", 48, 64, 34.0, 3)])
def test_pipelined_angular_kernel_parity(workload, n1, n2, ecut, vchunk, monkeypatch):
    """FP64 blocks served by the wave-specialised angular kernel (row waves
    move the slab straight through the theta2 transforms, convolution waves
    convolve the vector between): 32 x 81 blocks of 25 rows (every position
    holding a mode at 30 Ha; some rows and positions empty at 14 Ha) and
    48 x 64 blocks of 24 rows (25 Ha) and 28 rows (34 Ha, 25 in use).  Work
    split even over the resident workgroups (segments start and end inside
    radii), or 1, 2 or 3 items per workgroup (one- to three-vector segments,
    each drained on its own).  Every output element against the oracle, and
    against the one-vector convolution kernel (HELIC_ANGULAR_PIPE=0) on the
    same inputs."""
    w = synth.workload(workload).with_(name=f"{workload}-pipe-{ecut:g}", ecut=ecut, n_t1=n1, n_t2=n2, n_r=40)
    if vchunk:
        monkeypatch.setenv("HELIC_VCHUNK", str(vchunk))
    c = Case(w)
    c.upload_V()
    monkeypatch.setenv("HELIC_ANGULAR_PIPE", "0")
    one = helic.Basis.from_workload(w)
    one.set_potential(torch.from_numpy(c.V).to(_dev()))
    monkeypatch.delenv("HELIC_ANGULAR_PIPE")
    ms = sorted({int(m) for m in c.o.mnk[:, 0]})
    tag = f"[pipe {n1}x{n2} ecut={ecut:g} vchunk={vchunk}]"
    print(f"{tag} L={c.o.L}, m rows {len(ms)}", flush=True)
    X = synth.random_block(c.o.mnk, 21, 4244)
    ref = oh.apply(c.o, c.V, X)
    Xg = c.to_gpu_block(X)
    Yg = torch.zeros((21, c.o.L), dtype=torch.complex128, device=_dev())
    Y1 = torch.zeros_like(Yg)
    c.g.apply_H(Xg, Yg, prec="fp64")
    one.apply_H(Xg, Y1, prec="fp64")
    err = _rel(c.from_gpu_block(Yg), ref)
    agree = (torch.abs(Yg - Y1).max() / torch.abs(Y1).max()).item()
    print(f"{tag} rel err {err:.2e}, vs one-vector kernel {agree:.2e}", flush=True)
    assert err < TOL64
    assert agree < 1e-14
    one.close()


def test_radial_forward_nine_tiles_per_wave(monkeypatch):
    """FP64 radial forward on groups of 35 tiles (nanowire geometry, 40
    radii): 9 output tiles per wave (one pass over the slab, the default
    there) against 8 (a second pass for the widest groups), bit-identical
    since every tile's sums are formed in the same order, and the oracle."""
    w = synth.workload("nanowire-ecut30").with_(name="nanowire-fwd9", n_r=40)
    c = Case(w)
    c.upload_V()
    X = synth.random_block(c.o.mnk, 9, 4245)
    Xg = c.to_gpu_block(X)
    Y9 = torch.zeros_like(Xg)
    Y8 = torch.zeros_like(Xg)
    c.g.apply_H(Xg, Y9, prec="fp64")
    monkeypatch.setenv("HELIC_FWD_PF_TILES", "8")
    c.g.apply_H(Xg, Y8, prec="fp64")
    monkeypatch.delenv("HELIC_FWD_PF_TILES")
    assert torch.equal(Y9, Y8)
    err = _rel(c.from_gpu_block(Y9), oh.apply(c.o, c.V, X))
    print(f"[forward 9 tiles] rel err {err:.2e}", flush=True)
    assert err < TOL64


def test_general_and_specialised_angular_kernels_agree(tiny, monkeypatch):
    """The general LDS-FFT angular kernel and the specialised convolution
    kernel compute the same operator (both are checked against the oracle
    elsewhere; here on the same inputs, FP64 and FP32)."""
    monkeypatch.setenv("HELIC_GENERIC_ANGULAR", "1")
    gen = helic.Basis.from_workload(tiny.w)
    gen.set_potential(torch.from_numpy(tiny.V).to(_dev()))
    monkeypatch.delenv("HELIC_GENERIC_ANGULAR")
    X = tiny.to_gpu_block(synth.random_block(tiny.o.mnk, 12, 77))
    for prec, tol in (("fp64", TOL64), ("fp32", TOL32), ("bf16", TOL16)):
        Y1 = torch.zeros_like(X)
        Y2 = torch.zeros_like(X)
        gen.apply_H(X, Y1, prec=prec)
        tiny.g.apply_H(X, Y2, prec=prec)
        err = (torch.abs(Y1 - Y2).max() / torch.abs(Y1).max()).item()
        assert err < tol, (prec, err)
    gen.close()


@pytest.mark.parametrize("generic", [False, True])
def test_apply_H_parity_radix2_grid(generic, monkeypatch):
    """Nanotube geometry at a reduced cutoff on a 24 x 32 x 64 grid (radix-2
    passes in both angular directions, general angular kernel), and the tiny
    workload forced onto the general kernel."""
    if generic:
        monkeypatch.setenv("HELIC_GENERIC_ANGULAR", "1")
        w = synth.workload("tiny-helix")
    else:
        w = synth.workload("nanotube-ecut25").with_(name="nanotube-ecut6", ecut=6.0, n_t1=24, n_t2=32, n_r=64)
    c = Case(w)
    c.upload_V()
    X = synth.random_block(c.o.mnk, 5, 9)
    ref = oh.apply(c.o, c.V, X)
    for prec, tol in (("fp64", TOL64), ("bf16", TOL16)):
        Yg = torch.zeros((5, c.o.L), dtype=torch.complex128, device=_dev())
        c.g.apply_H(c.to_gpu_block(X), Yg, prec=prec)
        err = _rel(c.from_gpu_block(Yg), ref)
        print(f"[radix2 generic={generic} {prec}] rel err {err:.2e}", flush=True)
        assert err < tol


@pytest.mark.parametrize("grid", [(20, 96, 24), (20, 120, 24), (24, 120, 24), (24, 135, 24), (27, 144, 24),
                                  (27, 180, 24)])
def test_register_fft_angular_kernel_parity(grid, monkeypatch):
    """Grids of the batched workload served by the register-FFT angular
    kernel (theta1 column DFTs in registers, non-square theta2 four-step):
    against the oracle (FP64) and against the general LDS-FFT kernel on the
    same inputs (FP64 and FP32)."""
    n1, n2, nr = grid
    w = synth.Workload(name=f"blob-{n1}x{n2}", R=6.0, tau=10.0, alpha=0.0, ecut=6.0, n_t1=n1, n_t2=n2, n_r=nr,
                       m_max=(n1 - 1) // 2, n_max=(n2 - 1) // 2, structure="blob:1", seed=41, nev=4)
    c = Case(w)
    c.upload_V()
    X = synth.random_block(c.o.mnk, 6, 21)
    Yg = torch.zeros((6, c.o.L), dtype=torch.complex128, device=_dev())
    c.g.apply_H(c.to_gpu_block(X), Yg)
    ref = oh.apply(c.o, c.V, X)
    err = _rel(c.from_gpu_block(Yg), ref)
    print(f"[grid kernel {grid}] L={c.o.L} rel err vs oracle {err:.2e}", flush=True)
    assert err < TOL64
    monkeypatch.setenv("HELIC_GENERIC_ANGULAR", "1")
    gen = helic.Basis.from_workload(w)
    gen.set_potential(torch.from_numpy(c.V).to(_dev()))
    monkeypatch.delenv("HELIC_GENERIC_ANGULAR")
    Xd = c.to_gpu_block(X)
    for prec, tol in (("fp64", TOL64), ("fp32", TOL32), ("bf16", TOL16)):
        Y1 = torch.zeros_like(Xd)
        Y2 = torch.zeros_like(Xd)
        gen.apply_H(Xd, Y1, prec=prec)
        c.g.apply_H(Xd, Y2, prec=prec)
        e2 = (torch.abs(Y1 - Y2).max() / torch.abs(Y1).max()).item()
        assert e2 < tol, (prec, e2)
    gen.close()


def test_apply_H_widest_radial_groups_and_ragged_block():
    """The widest radial group the kernels take (K = 96 per |n|: 24 k steps in
    the inverse stage, 6 k tiles in the forward stage), 24 radial tiles, and a
    ragged block of 67 vectors (one 64-vector launch and a 3-vector tail),
    FP64 and FP32, against the oracle."""
    w = synth.Workload(name="wide-K", R=40.0, tau=6.0, alpha=0.0, ecut=60.0, m_max=1, n_max=2, k_max=96,
                       n_t1=8, n_t2=8, n_r=384, structure="blob:2", seed=43, nev=4)
    c = Case(w)
    assert int(c.o.mnk[:, 2].max()) == 96
    c.upload_V()
    X = synth.random_block(c.o.mnk, 67, 5)
    ref = oh.apply(c.o, c.V, X)
    for prec, tol in (("fp64", TOL64), ("fp32", TOL32), ("bf16", TOL16)):
        Yg = torch.zeros((67, c.o.L), dtype=torch.complex128, device=_dev())
        c.g.apply_H(c.to_gpu_block(X), Yg, prec=prec)
        err = _rel(c.from_gpu_block(Yg), ref)
        print(f"[wide K {prec}] L={c.o.L} rel err {err:.2e}", flush=True)
        assert err < tol


def test_profile_apply_matches_apply_and_times_each_stage(tiny):
    """The timing path (start and end events carried by the three stage
    kernels) computes the same block as helic_apply_H; the stage durations
    are positive and fit inside the whole application's span."""
    X = tiny.to_gpu_block(synth.random_block(tiny.o.mnk, 8, 61))
    Y0 = torch.empty_like(X)
    Y1 = torch.empty_like(X)
    tiny.g.apply_H(X, Y0)
    ms, tot = tiny.g.profile_apply(X, Y1, nrep=3)
    torch.cuda.synchronize()
    assert torch.equal(Y0, Y1)
    assert all(m > 0 for m in ms) and tot > 0
    assert sum(ms) <= tot * 1.001
