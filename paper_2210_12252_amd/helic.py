"""ctypes binding of libhelic (the C ABI declared in include/helic.h).

Argument marshalling only: every computation runs in the HIP library.  Device
blocks are torch tensors on the current HIP device; a block of nvec complex
columns of leading dimension ld is a C-contiguous complex128 tensor of shape
(nvec, ld) (row j of the tensor is column j of the column-major block).
Streams default to torch's current stream.  Importing this module does not
need a GPU; loading the library requires it to have been built
(``python -m paper_2210_12252_amd.build``) and raises otherwise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libhelic.so")

OK, ERR_INVALID, ERR_UNSUPPORTED, ERR_GRID, ERR_NOMEM, ERR_HIP, ERR_NOCONV, ERR_CUTOFF_TIE, ERR_STATE = range(9)
FP64, FP32, BF16 = 0, 1, 2
LPC_NPARAM = 4801
PREC = {"fp64": FP64, "fp32": FP32, "bf16": BF16}

# every function declared in include/helic.h
EXPORTS = ("helic_basis_create", "helic_basis_destroy", "helic_basis_info", "helic_basis_indices",
           "helic_grid", "helic_set_potential", "helic_apply_H", "helic_apply_H_noalloc", "helic_transform_inverse",
           "helic_transform_forward", "helic_gradient", "helic_density", "helic_profile_apply", "helic_precondition", "helic_eigensolve",
           "helic_eigensolve_ex", "helic_eigensolve_chefsi", "helic_batch_create", "helic_batch_destroy", "helic_batch_info",
           "helic_batch_classes", "helic_batch_tune_classes", "helic_batch_apply", "helic_batch_capture", "helic_batch_replay", "helic_batch_tune",
           "helic_batch_eigensolve", "helic_batch_eigensolve_chefsi",
           "helic_batch_time_reversal",
           "helic_lpc_create", "helic_lpc_destroy", "helic_lpc_get_params", "helic_lpc_set_params",
           "helic_lpc_save", "helic_lpc_load",
           "helic_lpc_attach", "helic_lpc_vdiag", "helic_lpc_apply", "helic_lpc_loss_grad", "helic_lpc_adam_step",
           "helic_lpc_train", "helic_lpc_harvest",
           "helic_util_bessel_j", "helic_util_bessel_zeros", "helic_util_gauss_jacobi",
           "helic_last_error")


class HelicError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"helic status {status}: {msg}")
        self.status = status


class SolveOpts(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int32), ("block", ctypes.c_int32), ("tol", ctypes.c_double),
                ("maxit", ctypes.c_int32), ("prec", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("precond", ctypes.c_int32), ("guard", ctypes.c_int32), ("switch_tol", ctypes.c_double),
                ("log_every", ctypes.c_int32), ("switch_tol_bf16", ctypes.c_double), ("stop_low", ctypes.c_int32)]


class ClassTuning(ctypes.Structure):
    _fields_ = [("n_t1", ctypes.c_int32), ("n_t2", ctypes.c_int32), ("n_r", ctypes.c_int32),
                ("nprob", ctypes.c_int32), ("items_per_wg", ctypes.c_int32), ("inv_ksteps", ctypes.c_int32),
                ("fwd_pipelined", ctypes.c_int32), ("fwd_tiles", ctypes.c_int32), ("ms", ctypes.c_double)]


class SolveStats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("iters_low", ctypes.c_int32), ("n_apply", ctypes.c_int64),
                ("n_fallback", ctypes.c_int32), ("t_apply_ms", ctypes.c_double), ("t_rr_ms", ctypes.c_double),
                ("t_precond_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double), ("iters_bf16", ctypes.c_int32),
                ("n_graphs", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


PRECOND = {"tpa": 0, "none": 1, "learned": 2}


class Params(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double), ("tau", ctypes.c_double), ("alpha", ctypes.c_double),
                ("ncyc", ctypes.c_int32), ("ecut", ctypes.c_double), ("eta", ctypes.c_double),
                ("nu", ctypes.c_int32), ("m_max", ctypes.c_int32), ("n_max", ctypes.c_int32),
                ("k_max", ctypes.c_int32), ("n_t1", ctypes.c_int32), ("n_t2", ctypes.c_int32),
                ("n_r", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double
_PD = ctypes.POINTER(ctypes.c_double)
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PI64 = ctypes.POINTER(ctypes.c_int64)


def load() -> ctypes.CDLL:
    """Load libhelic.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise RuntimeError(f"{LIBPATH} is not built; run python -m paper_2210_12252_amd.build")
    lib = ctypes.CDLL(LIBPATH)
    sig = {
        "helic_basis_create": [ctypes.POINTER(Params), ctypes.POINTER(_P)],
        "helic_basis_destroy": [_P],
        "helic_basis_info": [_P, _PI64, _PI32, _PI32, _PI32, _PI32],
        "helic_basis_indices": [_P, _PI32, _PD],
        "helic_grid": [_P, _PD, _PD, _PD, _PD],
        "helic_set_potential": [_P, _P, _P],
        "helic_apply_H": [_P, _P, _I64, _P, _I64, _I32, _I32, _P],
        "helic_apply_H_noalloc": [_P, _P, _I64, _P, _I64, _I32, _I32, _P],
        "helic_transform_inverse": [_P, _P, _I64, _P, _I32, _P],
        "helic_transform_forward": [_P, _P, _P, _I64, _I32, _P],
        "helic_density": [_P, _P, _I64, _I32, _PD, _P, _I32, _P],
        "helic_gradient": [_P, _P, _I64, _I32, _P, _I32, _P],
        "helic_precondition": [_P, _P, _I64, _P, _I64, _I32, _P],
        "helic_profile_apply": [_P, _P, _I64, _P, _I64, _I32, _I32, _I32, _P, _PD, _PD],
        "helic_eigensolve": [_P, _I32, _I32, _D, _I32, _I32, ctypes.c_uint64, _PD, _PD, _P, _I64,
                             _PI32, _P],
        "helic_eigensolve_ex": [_P, ctypes.POINTER(SolveOpts), _PD, _PD, _P, _I64, ctypes.POINTER(SolveStats), _P],
        "helic_eigensolve_chefsi": [_P, ctypes.POINTER(SolveOpts), _I32, _PD, _PD, _P, _I64,
                                    ctypes.POINTER(SolveStats), _P],
        "helic_batch_create": [ctypes.POINTER(_P), _I32, ctypes.POINTER(_P)],
        "helic_batch_destroy": [_P],
        "helic_batch_info": [_P, _PI64],
        "helic_batch_classes": [_P, _PI32, _PI32],
        "helic_batch_tune_classes": [_P, _P, _P, _I32, _I32, _P, ctypes.POINTER(ClassTuning), _I32, _PI32],
        "helic_batch_apply": [_P, _P, _P, _I32, _I32, _P],
        "helic_batch_capture": [_P, _P, _P, _I32, _I32],
        "helic_batch_replay": [_P, _P],
        "helic_batch_tune": [_P, _P, _P, _I32, _I32, _P, _PI32, _PD],
        "helic_batch_eigensolve": [_P, ctypes.POINTER(SolveOpts), _I32, _PD, _PD, ctypes.POINTER(SolveStats),
                                   _PI32],
        "helic_batch_time_reversal": [_P, _I32, _PI32],
        "helic_batch_eigensolve_chefsi": [_P, ctypes.POINTER(SolveOpts), _I32, _I32, _PD, _PD, ctypes.POINTER(SolveStats),
                                          _PI32],
        "helic_lpc_create": [ctypes.c_uint64, ctypes.POINTER(_P)],
        "helic_lpc_destroy": [_P],
        "helic_lpc_get_params": [_P, ctypes.POINTER(ctypes.c_float)],
        "helic_lpc_set_params": [_P, ctypes.POINTER(ctypes.c_float)],
        "helic_lpc_save": [_P, ctypes.c_char_p],
        "helic_lpc_load": [_P, ctypes.c_char_p],
        "helic_lpc_attach": [_P, _P],
        "helic_lpc_vdiag": [_P, _PD],
        "helic_lpc_apply": [_P, _P, _P, _I64, _P, _P, _I64, _I32, _P],
        "helic_lpc_loss_grad": [_P, _P, _P, _I64, _P, _I64, _P, _I32, _PD, _PD, _P],
        "helic_lpc_adam_step": [_P, _D, _P],
        "helic_lpc_train": [_P, _P, _P, _I64, _P, _I64, _P, _I32, _I32, _I32, _D, ctypes.c_uint64, _PD, _P],
        "helic_lpc_harvest": [_P, ctypes.POINTER(SolveOpts), _I32, _I32, _P, _P, _P, _PI32,
                              ctypes.POINTER(SolveStats), _P],
        "helic_util_bessel_j": [_I32, _I32, _PD, _PD],
        "helic_util_bessel_zeros": [_I32, _I32, _PD],
        "helic_util_gauss_jacobi": [_I32, _PD, _PD],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.helic_last_error.argtypes = []
    lib.helic_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status: int):
    if status != OK:
        raise HelicError(status, load().helic_last_error().decode())


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _block(t, name):
    import torch
    if not (t.is_cuda and t.dtype == torch.complex128 and t.dim() == 2 and t.stride(1) == 1):
        raise ValueError(f"{name} must be a complex128 HIP tensor of shape (nvec, ld), unit stride")
    # a single column's leading dimension is immaterial (and torch may report any stride for it)
    return t.shape[0], (t.shape[1] if t.shape[0] <= 1 else t.stride(0))


# ------------------------------------------------------------------ host calls
def basis_create(R, tau, alpha, ecut, eta=0.0, m_max=-1, n_max=-1, k_max=-1, n_t1=0, n_t2=0, n_r=0,
                 ncyc=1, nu=0) -> ctypes.c_void_p:
    p = Params(R=R, tau=tau, alpha=alpha, ncyc=ncyc, ecut=ecut, eta=eta, nu=nu, m_max=m_max,
               n_max=n_max, k_max=k_max, n_t1=n_t1, n_t2=n_t2, n_r=n_r)
    h = ctypes.c_void_p()
    _check(load().helic_basis_create(ctypes.byref(p), ctypes.byref(h)))
    return h


def basis_destroy(h):
    _check(load().helic_basis_destroy(h))


def basis_info(h) -> dict:
    L = ctypes.c_int64()
    n1, n2, nr, nm = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().helic_basis_info(h, ctypes.byref(L), ctypes.byref(n1), ctypes.byref(n2),
                                   ctypes.byref(nr), ctypes.byref(nm)))
    return dict(L=L.value, n_t1=n1.value, n_t2=n2.value, n_r=nr.value, n_modes=nm.value)


def basis_indices(h):
    L = basis_info(h)["L"]
    mnk = np.empty((L, 3), dtype=np.int32)
    kappa = np.empty(L, dtype=np.float64)
    _check(load().helic_basis_indices(h, _ptr(mnk, ctypes.c_int32), _ptr(kappa, ctypes.c_double)))
    return mnk, kappa


def grid(h):
    i = basis_info(h)
    t1, t2 = np.empty(i["n_t1"]), np.empty(i["n_t2"])
    r, w = np.empty(i["n_r"]), np.empty(i["n_r"])
    _check(load().helic_grid(h, _ptr(t1, ctypes.c_double), _ptr(t2, ctypes.c_double),
                             _ptr(r, ctypes.c_double), _ptr(w, ctypes.c_double)))
    return t1, t2, r, w


def util_bessel_j(p: int, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    _check(load().helic_util_bessel_j(p, x.size, _ptr(x, ctypes.c_double), _ptr(out, ctypes.c_double)))
    return out


def util_bessel_zeros(p: int, count: int) -> np.ndarray:
    out = np.empty(count)
    _check(load().helic_util_bessel_zeros(p, count, _ptr(out, ctypes.c_double)))
    return out


def util_gauss_jacobi(n: int):
    q, w = np.empty(n), np.empty(n)
    _check(load().helic_util_gauss_jacobi(n, _ptr(q, ctypes.c_double), _ptr(w, ctypes.c_double)))
    return q, w


# ------------------------------------------------------------------ device calls
def set_potential(h, V, stream=None):
    import torch
    if not (V.is_cuda and V.dtype == torch.float64 and V.is_contiguous()):
        raise ValueError("V must be a contiguous float64 HIP tensor in real-space order")
    i = basis_info(h)
    if V.numel() != i["n_t1"] * i["n_t2"] * i["n_r"]:
        raise ValueError("V has the wrong number of grid points")
    _check(load().helic_set_potential(h, ctypes.c_void_p(V.data_ptr()), _stream(stream)))


def apply_H(h, X, Y, prec="fp64", stream=None):
    nx, ldx = _block(X, "X")
    ny, ldy = _block(Y, "Y")
    if ny < nx:
        raise ValueError("Y has fewer columns than X")
    _check(load().helic_apply_H(h, ctypes.c_void_p(X.data_ptr()), ldx, ctypes.c_void_p(Y.data_ptr()), ldy,
                                nx, PREC[prec], _stream(stream)))


def apply_H_noalloc(h, X, Y, prec="fp64", stream=None):
    """helic_apply_H with the intermediate slabs in the library's fixed
    per-device scratch array (no device allocation in the call)."""
    nx, ldx = _block(X, "X")
    ny, ldy = _block(Y, "Y")
    if ny < nx:
        raise ValueError("Y has fewer columns than X")
    _check(load().helic_apply_H_noalloc(h, ctypes.c_void_p(X.data_ptr()), ldx, ctypes.c_void_p(Y.data_ptr()),
                                        ldy, nx, PREC[prec], _stream(stream)))


def transform_inverse(h, X, g, stream=None):
    nx, ldx = _block(X, "X")
    i = basis_info(h)
    if g.numel() < nx * i["n_t1"] * i["n_t2"] * i["n_r"] or not g.is_contiguous():
        raise ValueError("g too small or not contiguous")
    _check(load().helic_transform_inverse(h, ctypes.c_void_p(X.data_ptr()), ldx, ctypes.c_void_p(g.data_ptr()),
                                          nx, _stream(stream)))


def gradient(h, X, grad, cartesian=False, stream=None):
    """grad (complex128 HIP tensor of shape (3, nvec, n_t1, n_t2, n_r) or as
    many elements) receives (E_theta1, E_theta2, E_r), or (E_x, E_y, E_z)."""
    nx, ldx = _block(X, "X")
    i = basis_info(h)
    if not (grad.is_cuda and grad.is_contiguous() and str(grad.dtype) == "torch.complex128"
            and grad.numel() >= 3 * nx * i["n_t1"] * i["n_t2"] * i["n_r"]):
        raise ValueError("grad must be a contiguous complex128 HIP tensor of 3 * nvec grids")
    _check(load().helic_gradient(h, ctypes.c_void_p(X.data_ptr()), ldx, nx, ctypes.c_void_p(grad.data_ptr()),
                                 1 if cartesian else 0, _stream(stream)))


def density(h, X, occ, rho, accumulate=False, stream=None):
    """rho (float64 HIP tensor, n_t1*n_t2*n_r values) = or += sum_j occ[j]
    |inverse transform of X's column j|^2; occ: one weight per column."""
    nx, ldx = _block(X, "X")
    i = basis_info(h)
    occ = np.ascontiguousarray(occ, dtype=np.float64)
    if occ.size != nx:
        raise ValueError("occ needs one weight per column of X")
    if not (rho.is_cuda and rho.is_contiguous() and str(rho.dtype) == "torch.float64"
            and rho.numel() >= i["n_t1"] * i["n_t2"] * i["n_r"]):
        raise ValueError("rho must be a contiguous float64 HIP tensor of n_t1*n_t2*n_r values")
    _check(load().helic_density(h, ctypes.c_void_p(X.data_ptr()), ldx, nx, _ptr(occ, ctypes.c_double),
                                ctypes.c_void_p(rho.data_ptr()), 1 if accumulate else 0, _stream(stream)))


def transform_forward(h, g, X, stream=None):
    nx, ldx = _block(X, "X")
    i = basis_info(h)
    if g.numel() < nx * i["n_t1"] * i["n_t2"] * i["n_r"] or not g.is_contiguous():
        raise ValueError("g too small or not contiguous")
    _check(load().helic_transform_forward(h, ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(X.data_ptr()), ldx,
                                          nx, _stream(stream)))


def profile_apply(h, X, Y, prec="fp64", nrep=1, stream=None):
    """Mean per-stage and total durations (ms) of `nrep` applications."""
    nx, ldx = _block(X, "X")
    ny, ldy = _block(Y, "Y")
    if ny < nx:
        raise ValueError("Y has fewer columns than X")
    ms = np.zeros(3)
    tot = ctypes.c_double(0.0)
    _check(load().helic_profile_apply(h, ctypes.c_void_p(X.data_ptr()), ldx, ctypes.c_void_p(Y.data_ptr()), ldy,
                                      nx, PREC[prec], nrep, _stream(stream), _ptr(ms, ctypes.c_double),
                                      ctypes.byref(tot)))
    return ms, tot.value


def precondition(h, R, W, stream=None):
    nr_, ldr = _block(R, "R")
    nw, ldw = _block(W, "W")
    if nw < nr_:
        raise ValueError("W has fewer columns than R")
    _check(load().helic_precondition(h, ctypes.c_void_p(R.data_ptr()), ldr, ctypes.c_void_p(W.data_ptr()), ldw,
                                     nr_, _stream(stream)))


def eigensolve(h, nev, block=64, tol=1e-8, maxit=500, prec="fp64", seed=7, evecs=None, stream=None):
    """Returns (evals, resid, iters, status); raises on errors other than
    non-convergence."""
    evals = np.zeros(nev)
    resid = np.zeros(nev)
    iters = ctypes.c_int32(0)
    if evecs is not None:
        nv, ldv = _block(evecs, "evecs")
        if nv < nev:
            raise ValueError("evecs has fewer than nev columns")
        vptr = ctypes.c_void_p(evecs.data_ptr())
    else:
        ldv, vptr = 0, ctypes.c_void_p(0)
    st = load().helic_eigensolve(h, nev, block, tol, maxit, PREC[prec], seed, _ptr(evals, ctypes.c_double),
                                 _ptr(resid, ctypes.c_double), vptr, ldv, ctypes.byref(iters), _stream(stream))
    if st not in (OK, ERR_NOCONV):
        _check(st)
    return evals, resid, iters.value, st


def eigensolve_ex(h, nev, block=64, tol=1e-8, maxit=500, prec="fp64", seed=7, precond="tpa", guard=-1,
                  switch_tol=0.0, evecs=None, log_every=0, stream=None, cheb_degree=None, switch_tol_bf16=0.0,
                  stop_low=False):
    """Returns (evals, resid, stats dict, status); raises on errors other
    than non-convergence.  cheb_degree (an int, 0 = automatic) selects the
    Chebyshev-filtered subspace iteration instead of LOBPCG; stop_low ends a
    low-precision solve at its first precision switch."""
    o = SolveOpts(nev=nev, block=block, tol=tol, maxit=maxit, prec=PREC[prec], seed=seed,
                  precond=PRECOND[precond], guard=guard, switch_tol=switch_tol, log_every=log_every,
                  switch_tol_bf16=switch_tol_bf16, stop_low=int(bool(stop_low)))
    evals = np.zeros(nev)
    resid = np.zeros(nev)
    st = SolveStats()
    if evecs is not None:
        nv, ldv = _block(evecs, "evecs")
        if nv < nev:
            raise ValueError("evecs has fewer than nev columns")
        vptr = ctypes.c_void_p(evecs.data_ptr())
    else:
        ldv, vptr = 0, ctypes.c_void_p(0)
    if cheb_degree is None:
        status = load().helic_eigensolve_ex(h, ctypes.byref(o), _ptr(evals, ctypes.c_double),
                                            _ptr(resid, ctypes.c_double), vptr, ldv, ctypes.byref(st),
                                            _stream(stream))
    else:
        status = load().helic_eigensolve_chefsi(h, ctypes.byref(o), int(cheb_degree), _ptr(evals, ctypes.c_double),
                                                _ptr(resid, ctypes.c_double), vptr, ldv, ctypes.byref(st),
                                                _stream(stream))
    if status not in (OK, ERR_NOCONV):
        _check(status)
    stats = st.as_dict()
    stats["message"] = load().helic_last_error().decode() if status != OK else ""
    return evals, resid, stats, status


def _lam(lam, n):
    import torch
    if not (lam.is_cuda and lam.dtype == torch.float64 and lam.is_contiguous() and lam.numel() >= n):
        raise ValueError("lam must be a contiguous float64 HIP tensor with one value per column")
    return ctypes.c_void_p(lam.data_ptr())


class Lpc:
    """Learned diagonal preconditioner network (device-resident parameters
    and Adam state)."""

    def __init__(self, seed=0):
        self.h = ctypes.c_void_p()
        _check(load().helic_lpc_create(seed, ctypes.byref(self.h)))

    def close(self):
        if self.h is not None:
            load().helic_lpc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def params(self) -> np.ndarray:
        p = np.empty(LPC_NPARAM, dtype=np.float32)
        _check(load().helic_lpc_get_params(self.h, _ptr(p, ctypes.c_float)))
        return p

    @params.setter
    def params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        if p.size != LPC_NPARAM:
            raise ValueError(f"expected {LPC_NPARAM} parameters")
        _check(load().helic_lpc_set_params(self.h, _ptr(p, ctypes.c_float)))

    def adam_step(self, lr, stream=None):
        _check(load().helic_lpc_adam_step(self.h, lr, _stream(stream)))

    def save(self, path):
        _check(load().helic_lpc_save(self.h, os.fsencode(path)))

    def load(self, path):
        _check(load().helic_lpc_load(self.h, os.fsencode(path)))


class Batch:
    """A batch of problems (borrows the Basis objects, which must stay
    alive), grouped internally into classes of equal grid and angular kernel.
    Batched blocks are complex128 device tensors of nvec * offsets[-1]
    elements: problem p's block is the slice [nvec * offsets[p],
    nvec * offsets[p + 1]) viewed as (nvec, L_p)."""

    def __init__(self, bases):
        self.bases = list(bases)
        arr = (_P * len(self.bases))(*[b.h for b in self.bases])
        self.h = ctypes.c_void_p()
        _check(load().helic_batch_create(arr, len(self.bases), ctypes.byref(self.h)))
        off = np.zeros(len(self.bases) + 1, dtype=np.int64)
        _check(load().helic_batch_info(self.h, _ptr(off, ctypes.c_int64)))
        self.offsets = off

    def close(self):
        if self.h is not None:
            load().helic_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def view(self, buf, nvec, p):
        """(nvec, L_p) view of problem p in a concatenated buffer."""
        a, b = nvec * int(self.offsets[p]), nvec * int(self.offsets[p + 1])
        return buf[a:b].view(nvec, int(self.offsets[p + 1] - self.offsets[p]))

    @staticmethod
    def _flat(t, name):
        import torch
        if not (t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous complex128 HIP tensor")
        return ctypes.c_void_p(t.data_ptr())

    def apply(self, X, Y, nvec, prec="fp64", stream=None):
        _check(load().helic_batch_apply(self.h, self._flat(X, "X"), self._flat(Y, "Y"), nvec, PREC[prec],
                                        _stream(stream)))

    def capture(self, X, Y, nvec, prec="fp64"):
        _check(load().helic_batch_capture(self.h, self._flat(X, "X"), self._flat(Y, "Y"), nvec, PREC[prec]))

    def replay(self, stream=None):
        _check(load().helic_batch_replay(self.h, _stream(stream)))

    def classes(self):
        """(number of classes, class index of every problem)."""
        n = ctypes.c_int32(0)
        cls = np.zeros(len(self.bases), dtype=np.int32)
        _check(load().helic_batch_classes(self.h, ctypes.byref(n), _ptr(cls, ctypes.c_int32)))
        return n.value, cls

    def tune_classes(self, X, Y, nvec, prec="fp64", stream=None):
        """Tune every class; returns one dict of choices per class."""
        nmax = len(self.bases)
        out = (ClassTuning * nmax)()
        n = ctypes.c_int32(0)
        _check(load().helic_batch_tune_classes(self.h, self._flat(X, "X"), self._flat(Y, "Y"), nvec, PREC[prec],
                                               _stream(stream), out, nmax, ctypes.byref(n)))
        return [{f: getattr(out[i], f) for f, _ in ClassTuning._fields_} for i in range(n.value)]

    def tune(self, X, Y, nvec, prec="fp64", stream=None):
        chosen = ctypes.c_int32(0)
        ms = ctypes.c_double(0)
        _check(load().helic_batch_tune(self.h, self._flat(X, "X"), self._flat(Y, "Y"), nvec, PREC[prec],
                                       _stream(stream), ctypes.byref(chosen), ctypes.byref(ms)))
        return chosen.value, ms.value

    def time_reversal(self, enable=True):
        """Pair problems at eta and -eta (same structure) so that the batched
        eigensolvers solve one of each pair; returns the number of pairs."""
        n = ctypes.c_int32(0)
        _check(load().helic_batch_time_reversal(self.h, 1 if enable else 0, ctypes.byref(n)))
        return n.value

    def eigensolve(self, nev, nstreams=8, block=64, tol=1e-8, maxit=500, prec="fp64", seed=7, precond="tpa",
                   guard=-1, switch_tol=0.0, log_every=0, cheb_degree=None):
        """cheb_degree (an int, 0 = automatic) selects the Chebyshev-filtered
        subspace iteration instead of LOBPCG."""
        n = len(self.bases)
        o = SolveOpts(nev=nev, block=block, tol=tol, maxit=maxit, prec=PREC[prec], seed=seed,
                      precond=PRECOND[precond], guard=guard, switch_tol=switch_tol, log_every=log_every)
        evals = np.zeros((n, nev))
        resid = np.zeros((n, nev))
        stats = (SolveStats * n)()
        status = np.zeros(n, dtype=np.int32)
        if cheb_degree is None:
            st = load().helic_batch_eigensolve(self.h, ctypes.byref(o), nstreams, _ptr(evals, ctypes.c_double),
                                               _ptr(resid, ctypes.c_double), stats, _ptr(status, ctypes.c_int32))
        else:
            st = load().helic_batch_eigensolve_chefsi(self.h, ctypes.byref(o), int(cheb_degree), nstreams,
                                                      _ptr(evals, ctypes.c_double), _ptr(resid, ctypes.c_double),
                                                      stats, _ptr(status, ctypes.c_int32))
        if st not in (OK, ERR_NOCONV):
            _check(st)
        return evals, resid, [s.as_dict() for s in stats], status


class Basis:
    """Owning wrapper of a basis handle."""

    def __init__(self, **params):
        self.h = basis_create(**params)
        info = basis_info(self.h)
        self.L = info["L"]
        self.n_t1, self.n_t2, self.n_r, self.n_modes = info["n_t1"], info["n_t2"], info["n_r"], info["n_modes"]

    @classmethod
    def from_workload(cls, w, **over):
        p = dict(R=w.R, tau=w.tau, alpha=w.alpha, ecut=w.ecut, eta=w.eta, m_max=w.m_max, n_max=w.n_max,
                 k_max=w.k_max, n_t1=w.n_t1, n_t2=w.n_t2, n_r=w.n_r, ncyc=getattr(w, "ncyc", 1),
                 nu=getattr(w, "nu", 0))
        p.update(over)
        return cls(**p)

    def close(self):
        if self.h is not None:
            basis_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def indices(self):
        return basis_indices(self.h)

    def grid(self):
        return grid(self.h)

    def set_potential(self, V, stream=None):
        set_potential(self.h, V, stream)

    def apply_H(self, X, Y, prec="fp64", stream=None):
        apply_H(self.h, X, Y, prec, stream)

    def apply_H_noalloc(self, X, Y, prec="fp64", stream=None):
        apply_H_noalloc(self.h, X, Y, prec, stream)

    def transform_inverse(self, X, g, stream=None):
        transform_inverse(self.h, X, g, stream)

    def transform_forward(self, g, X, stream=None):
        transform_forward(self.h, g, X, stream)

    def density(self, X, occ, rho, accumulate=False, stream=None):
        density(self.h, X, occ, rho, accumulate, stream)

    def gradient(self, X, grad, cartesian=False, stream=None):
        gradient(self.h, X, grad, cartesian, stream)

    def precondition(self, R, W, stream=None):
        precondition(self.h, R, W, stream)

    def profile_apply(self, X, Y, prec="fp64", nrep=1, stream=None):
        return profile_apply(self.h, X, Y, prec, nrep, stream)

    def eigensolve(self, nev, **kw):
        return eigensolve(self.h, nev, **kw)

    def eigensolve_ex(self, nev, **kw):
        return eigensolve_ex(self.h, nev, **kw)

    # ---- learned preconditioner
    def attach(self, net):
        _check(load().helic_lpc_attach(self.h, net.h if net is not None else None))
        self._lpc = net   # keep the network alive while attached

    def lpc_vdiag(self):
        out = np.empty(self.L)
        _check(load().helic_lpc_vdiag(self.h, _ptr(out, ctypes.c_double)))
        return out

    def lpc_apply(self, net, R, lam, W, stream=None):
        nr_, ldr = _block(R, "R")
        nw, ldw = _block(W, "W")
        if nw < nr_:
            raise ValueError("W has fewer columns than R")
        _check(load().helic_lpc_apply(self.h, net.h, ctypes.c_void_p(R.data_ptr()), ldr, _lam(lam, nr_),
                                      ctypes.c_void_p(W.data_ptr()), ldw, nr_, _stream(stream)))

    def lpc_loss_grad(self, net, R, T, lam, stream=None):
        """(mean loss, gradient as a float64 array)."""
        nr_, ldr = _block(R, "R")
        nt, ldt = _block(T, "T")
        if nt != nr_:
            raise ValueError("R and T differ in column count")
        loss = ctypes.c_double(0.0)
        grad = np.empty(LPC_NPARAM)
        _check(load().helic_lpc_loss_grad(self.h, net.h, ctypes.c_void_p(R.data_ptr()), ldr,
                                          ctypes.c_void_p(T.data_ptr()), ldt, _lam(lam, nr_), nr_,
                                          ctypes.byref(loss), _ptr(grad, ctypes.c_double), _stream(stream)))
        return loss.value, grad

    def lpc_train(self, net, R, T, lam, ncol, batch, steps, lr=3e-3, seed=0, stream=None):
        """Adam steps on column batches of the first ncol training columns;
        returns the per-step losses."""
        nr_, ldr = _block(R, "R")
        nt, ldt = _block(T, "T")
        if min(nr_, nt) < ncol:
            raise ValueError("fewer stored columns than ncol")
        losses = np.zeros(max(steps, 1))
        _check(load().helic_lpc_train(self.h, net.h, ctypes.c_void_p(R.data_ptr()), ldr,
                                      ctypes.c_void_p(T.data_ptr()), ldt, _lam(lam, ncol), ncol, batch, steps, lr,
                                      seed, _ptr(losses, ctypes.c_double), _stream(stream)))
        return losses[:steps]

    def lpc_harvest(self, nev, n_snap=12, max_cols=None, block=64, tol=1e-8, maxit=500, seed=7, precond="tpa",
                    guard=-1, log_every=0, stream=None):
        """Training pairs from one FP64 eigensolve: (R, T, lam, ncol, stats)
        with R, T of shape (max_cols, L) and the first ncol rows filled."""
        import torch
        max_cols = max_cols or n_snap * nev
        dev = torch.device("cuda", torch.cuda.current_device())
        R = torch.zeros((max_cols, self.L), dtype=torch.complex128, device=dev)
        T = torch.zeros_like(R)
        lam = torch.zeros(max_cols, dtype=torch.float64, device=dev)
        o = SolveOpts(nev=nev, block=block, tol=tol, maxit=maxit, prec=FP64, seed=seed,
                      precond=PRECOND[precond], guard=guard, switch_tol=0.0, log_every=log_every)
        ncol = ctypes.c_int32(0)
        st = SolveStats()
        _check(load().helic_lpc_harvest(self.h, ctypes.byref(o), n_snap, max_cols, ctypes.c_void_p(R.data_ptr()),
                                        ctypes.c_void_p(T.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
                                        ctypes.byref(ncol), ctypes.byref(st), _stream(stream)))
        return R, T, lam, ncol.value, st.as_dict()
