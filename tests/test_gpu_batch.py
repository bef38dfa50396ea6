"""Batched problems (Bloch parameters of one or several structures): one
launch per H*X stage over all problems of a grid class, HIP-graph capture and
replay, the per-class tuner, and the concurrent batched eigensolve -- each
problem checked against the CPU oracle.
Tolerances as in test_gpu_apply.py / test_gpu_eigensolve.py."""
import numpy as np
import pytest

import synth
from oracle import basis as ob
from oracle import hamiltonian as oh

torch = pytest.importorskip("torch")
helic = pytest.importorskip("paper_2210_12252_amd.helic")

pytestmark = pytest.mark.gpu
TOL64 = 1e-12
TOL32 = 2e-5


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


class Problem:
    def __init__(self, w, V=None):
        self.w = w
        self.o = ob.basis_for(w)
        self.g = helic.Basis.from_workload(w)
        mnk, _ = self.g.indices()
        pos = {tuple(t): i for i, t in enumerate(self.o.mnk.tolist())}
        self.perm = np.array([pos[tuple(t)] for t in mnk.tolist()])
        if V is None:
            atoms = synth.atoms_for(w.structure, w.seed, w.tau, w.R)
            V = synth.potential_at(self.o.theta1, self.o.theta2, self.o.r, w.tau, w.alpha, atoms)
        self.V = V
        self.g.set_potential(torch.from_numpy(V).to(_dev()))


def make_batch(base, etas):
    probs = [Problem(base.with_(name=f"{base.name}-eta{e:+.3f}", eta=e)) for e in etas]
    print(f"[batch] {base.name} L = {[p.o.L for p in probs]}", flush=True)
    return probs, helic.Batch([p.g for p in probs])


def pack(batch, probs, nvec, seed):
    """Concatenated device block and the per-problem oracle-order inputs."""
    xs = [synth.random_block(p.o.mnk, nvec, seed + i) for i, p in enumerate(probs)]
    total = nvec * int(batch.offsets[-1])
    X = torch.zeros(total, dtype=torch.complex128, device=_dev())
    for i, (p, x) in enumerate(zip(probs, xs)):
        batch.view(X, nvec, i).copy_(torch.from_numpy(np.ascontiguousarray(x[p.perm].T)))
    return X, xs


def unpack(batch, probs, Y, nvec, i):
    y = batch.view(Y, nvec, i).cpu().numpy().T
    out = np.empty_like(y)
    out[probs[i].perm] = y
    return out


TINY = synth.workload("tiny-helix")
# a structure on a grid without a specialised angular kernel (general LDS FFT)
GENERAL = synth.Workload(name="blob-20x30", R=7.0, tau=6.0, alpha=0.0, ecut=9.0, n_t1=20, n_t2=30, n_r=40,
                         structure="blob:0", seed=40, nev=6)


@pytest.mark.parametrize("base,etas", [(TINY, (-0.5, -0.2, 0.0, 0.13, 0.41)), (GENERAL, (-0.3, 0.0, 0.25))])
def test_batched_apply_matches_oracle_per_problem(base, etas):
    probs, batch = make_batch(base, etas)
    nvec = 7
    X, xs = pack(batch, probs, nvec, 300)
    for prec, tol in (("fp64", TOL64), ("fp32", TOL32), ("bf16", 1e-2)):
        Y = torch.full_like(X, 3.0)
        batch.apply(X, Y, nvec, prec=prec)
        for i, p in enumerate(probs):
            ref = oh.apply(p.o, p.V, xs[i])
            y = unpack(batch, probs, Y, nvec, i)
            for j in range(nvec):
                err = np.max(np.abs(y[:, j] - ref[:, j])) / np.max(np.abs(ref[:, j]))
                assert err <= tol, (prec, i, j, err)
    batch.close()


@pytest.mark.parametrize("base", [
    synth.workload("nanotube-ecut25").with_(name="tube-batch", ecut=12.0, n_t1=48, n_t2=64, n_r=40),
    synth.workload("nanowire-ecut30").with_(name="wire-batch", ecut=14.0, n_t1=32, n_t2=81, n_r=40)])
def test_batched_apply_on_wave_specialised_angular_grids(base, monkeypatch):
    """Grid classes whose FP64 angular stage runs the wave-specialised kernel
    (48 x 64 and 32 x 81 blocks): three Bloch parameters in one launch per
    stage, work segments crossing problem boundaries, every problem's output
    against the oracle, and the whole batch against the one-vector kernel
    (HELIC_ANGULAR_PIPE=0) on the same inputs."""
    etas = (-0.3, 0.0, 0.25)
    probs, batch = make_batch(base, etas)
    monkeypatch.setenv("HELIC_ANGULAR_PIPE", "0")
    ones = [Problem(base.with_(name=f"{base.name}-one{e:+.3f}", eta=e), V=p.V) for e, p in zip(etas, probs)]
    batch1 = helic.Batch([q.g for q in ones])
    monkeypatch.delenv("HELIC_ANGULAR_PIPE")
    nvec = 5
    X, xs = pack(batch, probs, nvec, 500)
    Y = torch.full_like(X, 3.0)
    Y1 = torch.full_like(X, 3.0)
    batch.apply(X, Y, nvec, prec="fp64")
    batch1.apply(X, Y1, nvec, prec="fp64")
    agree = (torch.abs(Y - Y1).max() / torch.abs(Y1).max()).item()
    print(f"[batch {base.name}] vs one-vector kernel {agree:.2e}", flush=True)
    assert agree < 1e-14
    for i, p in enumerate(probs):
        ref = oh.apply(p.o, p.V, xs[i])
        y = unpack(batch, probs, Y, nvec, i)
        err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
        print(f"[batch {base.name}] problem {i} rel err {err:.2e}", flush=True)
        assert err <= TOL64, (i, err)
    batch.close()
    batch1.close()


def test_graph_replay_matches_eager_apply():
    probs, batch = make_batch(TINY, (-0.25, 0.0, 0.25, 0.375))
    nvec = 16
    X, _ = pack(batch, probs, nvec, 11)
    Y_eager = torch.zeros_like(X)
    batch.apply(X, Y_eager, nvec)
    torch.cuda.synchronize()
    Y = torch.zeros_like(X)
    batch.capture(X, Y, nvec)
    scratch = torch.zeros_like(X)
    for rep in range(4):
        Y.zero_()
        batch.replay()
        torch.cuda.synchronize()
        assert torch.equal(Y, Y_eager), rep
        # eager work between replays on the same buffers' neighbours
        batch.apply(X, scratch, nvec)
        torch.cuda.synchronize()
        assert torch.equal(scratch, Y_eager)
    batch.close()


def test_tuner_keeps_results_exact():
    probs, batch = make_batch(TINY, (-0.1, 0.2))
    nvec = 32
    X, _ = pack(batch, probs, nvec, 5)
    Y0 = torch.zeros_like(X)
    batch.apply(X, Y0, nvec)
    chosen, ms = batch.tune(X, torch.zeros_like(X), nvec)
    print(f"[tune] items per angular workgroup {chosen} (0: even split), {ms:.3f} ms", flush=True)
    assert chosen in (0, 2, 4, 8, 16) and ms > 0
    Y1 = torch.zeros_like(X)
    batch.apply(X, Y1, nvec)
    torch.cuda.synchronize()
    assert (torch.abs(Y1 - Y0).max() / torch.abs(Y0).max()).item() < 1e-14
    batch.close()


def test_batched_eigensolve_matches_lapack_per_problem():
    etas = (-0.5, -0.25, 0.0, 0.25)
    probs, batch = make_batch(TINY, etas)
    ev, res, stats, status = batch.eigensolve(TINY.nev, nstreams=3, tol=1e-9, maxit=400)
    assert np.all(status == helic.OK), status
    for i, p in enumerate(probs):
        ref, _ = oh.lowest(oh.dense_explicit(p.o, p.V), TINY.nev)
        assert np.max(np.abs(ev[i] - ref)) < 1e-8, (i, ev[i] - ref)
    # time reversal across the batch: lambda(eta) = lambda(-eta)
    np.testing.assert_allclose(ev[1], ev[3], atol=1e-8)
    batch.close()


@pytest.mark.parametrize("base,etas", [(TINY, (-0.5, -0.25, 0.0, 0.25)), (GENERAL, (-0.3, 0.0, 0.25))])
def test_batched_filtered_eigensolve_matches_lapack_per_problem(base, etas):
    probs, batch = make_batch(base, etas)
    ev, res, stats, status = batch.eigensolve(base.nev, nstreams=3, tol=1e-9, maxit=200, cheb_degree=0)
    assert np.all(status == helic.OK), status
    for i, p in enumerate(probs):
        ref, _ = oh.lowest(oh.dense_explicit(p.o, p.V), base.nev)
        assert np.max(np.abs(ev[i] - ref)) < 1e-8, (i, ev[i] - ref)
    with pytest.raises(helic.HelicError):
        batch.eigensolve(TINY.nev, cheb_degree=-1)
    batch.close()


def test_time_reversal_halving_of_batched_eigensolves():
    etas = (-0.25, 0.0, 0.25, 0.125)
    probs, batch = make_batch(TINY, etas)
    assert batch.time_reversal(True) == 1                  # eta = 0.25 takes eta = -0.25's results
    for deg in (None, 0):
        ev, res, stats, status = batch.eigensolve(TINY.nev, nstreams=2, tol=1e-9, maxit=400, cheb_degree=deg)
        assert np.all(status == helic.OK), status
        assert stats[2]["iters"] == 0 and stats[2]["n_apply"] == 0 and stats[0]["n_apply"] > 0
        np.testing.assert_array_equal(ev[2], ev[0])
        ref, _ = oh.lowest(oh.dense_explicit(probs[2].o, probs[2].V), TINY.nev)
        assert np.max(np.abs(ev[2] - ref)) < 1e-8
    assert batch.time_reversal(False) == 0
    batch.close()
    # same geometry and opposite eta but another potential: not paired
    a = Problem(TINY.with_(eta=-0.25))
    b = Problem(TINY.with_(eta=0.25), V=0.5 * a.V)
    other = helic.Batch([a.g, b.g])
    assert other.time_reversal(True) == 0
    other.close()


def test_batches_across_structures_and_grids():
    """Problems of different structures, grids and angular kernels in one
    batch (one class per grid): every problem against the oracle, the same
    blocks as a single-problem apply (to rounding order), one captured graph over all
    classes replayed several times (eager work in between), and the per-class
    tuner, whose choices are recorded and leave the results unchanged."""
    probs = [Problem(TINY.with_(name="tiny-a", eta=0.1)), Problem(GENERAL.with_(name="gen-a", eta=-0.3)),
             Problem(TINY.with_(name="tiny-b", eta=-0.2)), Problem(TINY.with_(name="tiny-r40", n_r=40)),
             Problem(GENERAL.with_(name="gen-b", eta=0.25))]
    batch = helic.Batch([p.g for p in probs])
    n, cls = batch.classes()
    print(f"[multi] classes {n}: {cls.tolist()}", flush=True)
    assert n == 3 and cls[0] == cls[2] and cls[1] == cls[4] and len({cls[0], cls[1], cls[3]}) == 3
    nvec = 6
    X, xs = pack(batch, probs, nvec, 70)
    for prec, tol in (("fp64", TOL64), ("fp32", TOL32), ("bf16", 1e-2)):
        Y = torch.full_like(X, 3.0)
        batch.apply(X, Y, nvec, prec=prec)
        for i, p in enumerate(probs):
            ref = oh.apply(p.o, p.V, xs[i])
            y = unpack(batch, probs, Y, nvec, i)
            err = max(np.max(np.abs(y[:, j] - ref[:, j])) / np.max(np.abs(ref[:, j])) for j in range(nvec))
            assert err <= tol, (prec, i, err)
            single = torch.zeros((nvec, p.o.L), dtype=torch.complex128, device=_dev())
            p.g.apply_H(batch.view(X, nvec, i).contiguous(), single, prec=prec)
            d = (torch.abs(single - batch.view(Y, nvec, i)).max() / torch.abs(single).max()).item()
            assert d < {"fp64": 1e-14, "fp32": 1e-6, "bf16": 1e-2}[prec], (prec, i, d)
    Y_eager = torch.zeros_like(X)
    batch.apply(X, Y_eager, nvec)
    tuning = batch.tune_classes(X, torch.zeros_like(X), nvec)
    print(f"[multi] tuning {tuning}", flush=True)
    assert len(tuning) == 3 and all(t["ms"] > 0 and t["nprob"] >= 1 for t in tuning)
    assert sorted(t["nprob"] for t in tuning) == [1, 2, 2]
    Y1 = torch.zeros_like(X)
    batch.apply(X, Y1, nvec)
    torch.cuda.synchronize()
    assert (torch.abs(Y1 - Y_eager).max() / torch.abs(Y_eager).max()).item() < 1e-14
    Y = torch.zeros_like(X)
    batch.capture(X, Y, nvec)
    scratch = torch.zeros_like(X)
    for rep in range(3):
        Y.zero_()
        batch.replay()
        torch.cuda.synchronize()
        assert torch.equal(Y, Y1), rep
        batch.apply(X, scratch, nvec)
        torch.cuda.synchronize()
    batch.close()


def test_batched_mixed_precision_eigensolve_across_structures():
    """The FP32 -> FP64 ladder of the filtered solver over a batch of two
    structures on two grids, with time-reversal halving: every problem's
    eigenvalues against LAPACK on the dense oracle (1e-8 Ha)."""
    probs = [Problem(TINY.with_(name="t-a", eta=0.2)), Problem(TINY.with_(name="t-b", eta=-0.2)),
             Problem(GENERAL.with_(name="g-a", eta=0.0)), Problem(GENERAL.with_(name="g-b", eta=0.3))]
    batch = helic.Batch([p.g for p in probs])
    npairs = batch.time_reversal(True)
    assert npairs == 1
    nev = 6
    ev, res, st, status = batch.eigensolve(nev, tol=1e-9, maxit=300, cheb_degree=0, prec="fp32")
    for i, p in enumerate(probs):
        ref, _ = oh.lowest(oh.dense_explicit(p.o, p.V), nev)
        err = np.max(np.abs(ev[i] - ref))
        print(f"[batched mixed] problem {i} status {status[i]} max|dlambda| {err:.2e}", flush=True)
        assert status[i] == helic.OK and err < 1e-8
    batch.close()
