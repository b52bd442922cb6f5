"""Python binding of libtrbl (thick-restart block Lanczos shell-model eigensolver on MI355X).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libtrbl.so`` behind the C ABI declared in ``include/trbl.h``.
PyTorch supplies device memory and the current HIP stream. There is no CPU
fallback: if the library is missing, loading fails with an error.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtrbl.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "trbl.h")

TRBL_FP64, TRBL_MIXED = 0, 1
TRBL_NOT_CONVERGED = 1


class TrblError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libtrbl error {code}: {msg}")
        self.code = code


class Orbit(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("l", ctypes.c_int), ("twoj", ctypes.c_int)]


class Tbme(ctypes.Structure):
    _fields_ = [("channel", ctypes.c_int), ("a", ctypes.c_int), ("b", ctypes.c_int), ("c", ctypes.c_int),
                ("d", ctypes.c_int), ("twoJ", ctypes.c_int), ("v", ctypes.c_double)]


class Opts(ctypes.Structure):
    _fields_ = [("nb", ctypes.c_int), ("n_eig", ctypes.c_int), ("l_s", ctypes.c_int), ("l_m", ctypes.c_int),
                ("max_iter", ctypes.c_int), ("tol", ctypes.c_double), ("precision", ctypes.c_int),
                ("refine", ctypes.c_int), ("seed", ctypes.c_uint64), ("v0", ctypes.c_void_p),
                ("stream", ctypes.c_void_p), ("check_every", ctypes.c_int), ("criterion", ctypes.c_int),
                ("mask", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("restarts", ctypes.c_int), ("n_converged", ctypes.c_int),
                ("breakdowns", ctypes.c_int), ("t_total", ctypes.c_double), ("t_hv", ctypes.c_double),
                ("t_orth", ctypes.c_double), ("t_qr", ctypes.c_double), ("t_eig", ctypes.c_double),
                ("t_restart", ctypes.c_double), ("t_refine", ctypes.c_double),
                ("resid", ctypes.POINTER(ctypes.c_double))]


_lib = None


def load():
    """Load libtrbl.so (built by ``build.py``); raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built; run paper_1902_02064_amd/build.py")
    # torch first: the library must bind to the HIP runtime that owns torch's device memory and streams
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    sig = {
        "trbl_model_create": ([ctypes.POINTER(Orbit), I, I, I, I, I, ctypes.POINTER(P)], I),
        "trbl_model_destroy": ([P], None),
        "trbl_model_dim": ([P, ctypes.POINTER(I64)], I),
        "trbl_basis_unrank": ([P, I64, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)], I),
        "trbl_basis_rank": ([P, ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(I64)], I),
        "trbl_basis_unrank_dev": ([P, P, I64, P, P, P], I),
        "trbl_basis_rank_dev": ([P, P, P, I64, P, P], I),
        "trbl_set_hamiltonian": ([P, P, P, ctypes.POINTER(Tbme), I64], I),
        "trbl_apply": ([P, I, I, P, P, P], I),
        "trbl_solve": ([P, ctypes.POINTER(Opts), P, P, ctypes.POINTER(Info)], I),
        "trbl_tbme_grad": ([P, ctypes.POINTER(Opts), I, P, P, P, P], I),
        "trbl_expect": ([P, I, P, P, P], I),
        "trbl_expect_noalloc": ([P, I, P, P, P], I),
        "trbl_occupation_mask": ([P, P, I, I, P, P], I),
        "trbl_random_tbme": ([ctypes.POINTER(Orbit), I, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(Tbme), I64,
                              ctypes.POINTER(I64)], I),
        "trbl_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def random_tbme(orbits, seed, sigma=1.0):
    """The library's seeded synthetic interaction (trbl_random_tbme): a list of
    (channel, a, b, c, d, 2J, v) in the library's drawing order."""
    lib = load()
    arr = (Orbit * len(orbits))(*[Orbit(*o) for o in orbits])
    n = ctypes.c_int64()
    _check(lib.trbl_random_tbme(arr, len(orbits), int(seed), float(sigma), None, 0, ctypes.byref(n)))
    out = (Tbme * max(1, n.value))()
    _check(lib.trbl_random_tbme(arr, len(orbits), int(seed), float(sigma), out, n.value, ctypes.byref(n)))
    return [(t.channel, t.a, t.b, t.c, t.d, t.twoJ, t.v) for t in out[:n.value]]


def header_symbols():
    """Names of the functions declared in include/trbl.h."""
    import re
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(trbl_[a-z_]+)\s*\(", text)))


def torch_float64():
    import torch
    return torch.float64


def _check(rc):
    if rc < 0:
        raise TrblError(rc, load().trbl_last_error().decode())
    return rc


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class SolveInfo:
    iterations: int
    restarts: int
    n_converged: int
    breakdowns: int
    t_total: float
    t_hv: float
    t_orth: float
    t_qr: float
    t_eig: float
    t_restart: float
    t_refine: float
    resid: np.ndarray
    converged: bool


class Model:
    """M-scheme model space (Sec. 2, App. A) with its Hamiltonian, on the current HIP device."""

    def __init__(self, orbits, n_prot, n_neut, twoM, parity=0):
        lib = load()
        arr = (Orbit * len(orbits))(*[Orbit(*o) for o in orbits])
        h = ctypes.c_void_p()
        _check(lib.trbl_model_create(arr, len(orbits), n_prot, n_neut, twoM, parity, ctypes.byref(h)))
        self._h = h
        self.orbits = tuple(tuple(o) for o in orbits)
        d = ctypes.c_int64()
        _check(lib.trbl_model_dim(h, ctypes.byref(d)))
        self.dim = int(d.value)
        self.n_tbme = 0
        self.h_version = 0  # incremented by every set_hamiltonian

    def close(self):
        if self._h:
            load().trbl_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- basis
    def unrank(self, i):
        p, n = ctypes.c_uint64(), ctypes.c_uint64()
        _check(load().trbl_basis_unrank(self._h, int(i), ctypes.byref(p), ctypes.byref(n)))
        return int(p.value), int(n.value)

    def rank(self, pbits, nbits):
        i = ctypes.c_int64()
        _check(load().trbl_basis_rank(self._h, int(pbits), int(nbits), ctypes.byref(i)))
        return int(i.value)

    def unrank_dev(self, idx):
        import torch
        idx = idx.to(torch.int64).contiguous()
        p = torch.empty_like(idx)
        n = torch.empty_like(idx)
        _check(load().trbl_basis_unrank_dev(self._h, _ptr(idx), idx.numel(), _ptr(p), _ptr(n), _stream()))
        return p, n

    def occupation_mask(self, orbit_set, max_particles):
        """Device [D] FP64 mask of the basis states with at most max_particles nucleons in the
        given orbits (the particle-hole truncation of Sec. 4.2)."""
        import torch
        orb = (ctypes.c_int * max(1, len(orbit_set)))(*orbit_set)
        mask = torch.empty(self.dim, dtype=torch.float64, device="cuda")
        _check(load().trbl_occupation_mask(self._h, orb, len(orbit_set), max_particles, _ptr(mask), _stream()))
        return mask

    def rank_dev(self, pbits, nbits):
        import torch
        pbits = pbits.to(torch.int64).contiguous()
        nbits = nbits.to(torch.int64).contiguous()
        out = torch.empty_like(pbits)
        _check(load().trbl_basis_rank_dev(self._h, _ptr(pbits), _ptr(nbits), pbits.numel(), _ptr(out),
                                          _stream()))
        return out

    # -- Hamiltonian
    def set_hamiltonian(self, spe_p, spe_n, tbme):
        norb = len(self.orbits)
        sp = (ctypes.c_double * norb)(*[float(x) for x in spe_p[:norb]])
        sn = (ctypes.c_double * norb)(*[float(x) for x in spe_n[:norb]])
        arr = (Tbme * max(1, len(tbme)))(*[Tbme(int(t[0]), int(t[1]), int(t[2]), int(t[3]), int(t[4]),
                                                 int(t[5]), float(t[6])) for t in tbme])
        _check(load().trbl_set_hamiltonian(self._h, sp, sn, arr, len(tbme)))
        self.n_tbme = len(tbme)
        self.h_version += 1

    def apply(self, V, W=None):
        """W = H V on the device; V is [D, nb] float64 (FP64) or float32 (mixed precision)."""
        import torch
        assert V.is_cuda and V.dim() == 2 and V.shape[0] == self.dim and V.is_contiguous()
        prec = TRBL_FP64 if V.dtype == torch.float64 else TRBL_MIXED
        if V.dtype not in (torch.float64, torch.float32):
            raise TypeError("V must be float64 or float32")
        if W is None:
            W = torch.empty_like(V)
        assert W.shape == V.shape and W.dtype == V.dtype and W.is_contiguous()
        _check(load().trbl_apply(self._h, prec, V.shape[1], _ptr(V), _ptr(W), _stream()))
        return W

    def expect(self, X):
        """<x_c|H|x_c> for the columns of X (device [D][n] float64), computed on the device."""
        import torch
        assert X.is_cuda and X.dtype == torch.float64 and X.dim() == 2 and X.shape[0] == self.dim
        X = X.contiguous()
        out = np.zeros(X.shape[1])
        _check(load().trbl_expect(self._h, X.shape[1], _ptr(X), out.ctypes.data_as(ctypes.c_void_p), _stream()))
        return out

    def expect_noalloc(self, X, out):
        """<x_c|H|x_c> into the device tensor out (float64, n) without any device allocation by the
        library (trbl_expect_noalloc); X is device [D][n] float64, contiguous."""
        import torch
        assert X.is_cuda and X.dtype == torch.float64 and X.dim() == 2 and X.shape[0] == self.dim
        assert X.is_contiguous() and out.is_cuda and out.dtype == torch.float64 and out.numel() >= X.shape[1]
        _check(load().trbl_expect_noalloc(self._h, X.shape[1], _ptr(X), _ptr(out), _stream()))
        return out

    # -- eigensolver
    def _opts(self, nb, n_eig, l_s, l_m, tol, precision, max_iter, seed, v0, refine, check_every=1,
              criterion="residual", mask=None):
        o = Opts()
        o.nb, o.n_eig, o.l_s, o.l_m, o.max_iter = nb, n_eig, l_s, l_m, max_iter
        o.tol = tol
        o.precision = TRBL_FP64 if precision == "fp64" else TRBL_MIXED
        o.refine = 1 if refine else 0
        o.seed = seed
        o.v0 = None if v0 is None else v0.data_ptr()
        o.stream = _stream().value
        o.check_every = check_every
        o.criterion = {"residual": 0, "ritz_change": 1}[criterion]
        if mask is not None:
            assert mask.is_cuda and mask.dtype == torch_float64() and mask.numel() == self.dim and mask.is_contiguous()
        o.mask = None if mask is None else mask.data_ptr()
        return o

    def solve(self, nb, n_eig, l_s, l_m, tol, precision="fp64", max_iter=5000, seed=1000, v0=None,
              refine=True, vectors=False, check_every=1, criterion="residual", mask=None):
        """Lowest eigenpairs by TRBL (Alg. 4). Returns (evals, evecs or None, SolveInfo).
        mask: optional device [D] 0/1 FP64 (occupation_mask): solve in that truncated subspace."""
        import torch
        o = self._opts(nb, n_eig, l_s, l_m, tol, precision, max_iter, seed, v0, refine, check_every, criterion,
                       mask)
        ev = (ctypes.c_double * n_eig)()
        res = (ctypes.c_double * n_eig)()
        info = Info()
        info.resid = ctypes.cast(res, ctypes.POINTER(ctypes.c_double))
        X = torch.empty((self.dim, n_eig), dtype=torch.float64, device="cuda") if vectors else None
        rc = _check(load().trbl_solve(self._h, ctypes.byref(o), ev, None if X is None else _ptr(X),
                                      ctypes.byref(info)))
        si = SolveInfo(info.iterations, info.restarts, info.n_converged, info.breakdowns, info.t_total,
                       info.t_hv, info.t_orth, info.t_qr, info.t_eig, info.t_restart, info.t_refine,
                       np.array(res[:]), rc == 0)
        return np.array(ev[:]), X, si

    def tbme_grad(self, weights, evecs=None, nb=8, l_s=None, l_m=None, tol=1e-10, max_iter=5000, seed=1000,
                  spe=True, n_solve=None):
        """d(sum_k w_k E_k)/dV for every element given to set_hamiltonian (and the spe if asked).

        evecs: device [D][len(weights)] FP64 eigenvectors, or None to recompute them with a TRBL
        solve for n_solve (default len(weights)) eigenpairs."""
        w = np.ascontiguousarray(weights, dtype=np.float64)
        n = len(w)
        ns = n_solve or n
        l_s = l_s or max(2 * ns, ns + nb)
        l_m = l_m or min(self.dim, l_s + 6 * nb)
        o = self._opts(nb, ns, l_s, l_m, tol, "fp64", max_iter, seed, None, True)
        gv = np.zeros(max(1, self.n_tbme))
        gs = np.zeros(2 * len(self.orbits)) if spe else None
        _check(load().trbl_tbme_grad(self._h, ctypes.byref(o), n, w.ctypes.data_as(ctypes.c_void_p),
                                     None if evecs is None else _ptr(evecs),
                                     gv.ctypes.data_as(ctypes.c_void_p),
                                     None if gs is None else gs.ctypes.data_as(ctypes.c_void_p)))
        return gv[:self.n_tbme], gs


def _autograd_fn():
    import torch

    class _Eigenvalues(torch.autograd.Function):
        """E(V, e): lowest eigenvalues as a differentiable function of the J-coupled elements and the
        single-particle energies. The backward pass is the Hellmann-Feynman density kernel of
        trbl_tbme_grad: dL/dtheta = sum_k (dL/dE_k) <psi_k| dH/dtheta |psi_k>."""

        @staticmethod
        def forward(ctx, v, spe_p, spe_n, model, structure, solver, keep_vectors):
            tb = [tuple(s) + (float(x),) for s, x in zip(structure, v.detach().cpu().tolist())]
            sp, sn = spe_p.detach().cpu().tolist(), spe_n.detach().cpu().tolist()
            model.set_hamiltonian(sp, sn, tb)
            ev, X, info = model.solve(vectors=keep_vectors, **solver)
            if not info.converged:
                raise TrblError(TRBL_NOT_CONVERGED, "TRBL did not converge in forward")
            ctx.model, ctx.solver, ctx.X = model, solver, X
            # the Hamiltonian of this forward pass: the backward pass restores it if the model has
            # been given another one since (a later forward pass, a finite-difference evaluation)
            ctx.h = (sp, sn, tb)
            ctx.h_version = model.h_version
            ctx.norb = len(model.orbits)
            return torch.from_numpy(ev).to(v.dtype)

        @staticmethod
        def backward(ctx, gE):
            w = gE.detach().cpu().numpy().astype(np.float64)
            s = ctx.solver
            if ctx.model.h_version != ctx.h_version:
                ctx.model.set_hamiltonian(*ctx.h)
                ctx.h_version = ctx.model.h_version
            gv, gs = ctx.model.tbme_grad(w, evecs=ctx.X, nb=s["nb"], l_s=s.get("l_s"), l_m=s.get("l_m"),
                                         tol=s["tol"], max_iter=s.get("max_iter", 5000), seed=s.get("seed", 1000),
                                         n_solve=s["n_eig"])
            gv = torch.from_numpy(gv).to(gE.dtype)
            gp = torch.from_numpy(gs[:ctx.norb].copy()).to(gE.dtype)
            gn = torch.from_numpy(gs[ctx.norb:].copy()).to(gE.dtype)
            return gv, gp, gn, None, None, None, None

    return _Eigenvalues


def eigenvalues(model, structure, v, spe_p, spe_n, nb, n_eig, l_s, l_m, tol, max_iter=5000, seed=1000,
                keep_vectors=True):
    """Differentiable lowest eigenvalues (torch autograd). structure: (channel, a, b, c, d, 2J) per element;
    v, spe_p, spe_n: CPU float64 tensors. keep_vectors=False recomputes the eigenvectors in the backward
    pass instead of holding D x n_eig doubles on the device between the passes."""
    solver = dict(nb=nb, n_eig=n_eig, l_s=l_s, l_m=l_m, tol=tol, max_iter=max_iter, seed=seed)
    return _autograd_fn().apply(v, spe_p, spe_n, model, [tuple(s[:6]) for s in structure], solver, keep_vectors)
