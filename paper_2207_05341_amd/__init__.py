"""MI355X (gfx950) likelihood path of neural-network maximum-likelihood
quantum state tomography (Wang, Cheng, Li, Chen): T -> rho = T T^dagger /
Tr -> p_k = Tr(rho M_k) over the per-qubit tetrahedral product POVM ->
L = -sum f_k ln p_k, and the hand-written adjoint back to dL/dT.

This module only marshals torch tensors into the C ABI of libqst.so
(include/qst.h); every step of the path runs in the library's HIP kernels on
torch's current stream.  torch supplies device memory and streams.
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import (QST_BF16GEMM, QST_F32, QST_F32X6, QST_F64, QST_MAX_QUBITS, QST_OP_ABS_MAP, QST_OP_GRAD_PRODUCT, QST_OP_LIKELIHOOD,
                   QST_OP_LIKELIHOOD_GRAD,
                   QST_FIDELITY_MAX_RANK, QST_OP_FIDELITY, QST_OP_FNN, QST_OP_NLL, QST_OP_NLL_BACKWARD, QST_OP_POVM_PROBS,
                   QST_OP_STATE_MAP, QST_PREMAP_HERMITIAN, QST_PREMAP_LOWER, QstError, workspace_bytes)

__all__ = [
    "PRECISIONS", "STATE_MAPS", "state_premap", "state_map", "povm_probs", "nll", "nll_backward",
    "likelihood_forward", "likelihood_grad", "likelihood_forward_noalloc", "likelihood_forward_fc", "povm_probs_general",
    "likelihood_forward_general", "likelihood_general", "GeneralLikelihoodFn", "grad_product", "likelihood", "LikelihoodFn", "StatePremapFn", "abs_map",
    "abs_map_backward", "abs_map_async", "AbsMapFn", "AbsProjection", "fidelity_lowrank", "fidelity_general",
    "fidelity_general_async",
    "fidelity_classical", "fnn_forward", "fnn_backward", "FnnFn", "MappingNetwork", "Rprop",
    "workspace_bytes", "QstError", "QST_F64", "QST_F32", "QST_BF16GEMM", "QST_F32X6", "QST_MAX_QUBITS",
]

PRECISIONS = {"f64": QST_F64, "f32": QST_F32, "bf16": QST_BF16GEMM, "f32x6": QST_F32X6}
_NAMES = {v: k for k, v in PRECISIONS.items()}


def _prec(dtype: torch.dtype, prec) -> int:
    if prec is None:
        if dtype == torch.complex128:
            return QST_F64
        if dtype == torch.complex64:
            return QST_F32
        raise TypeError(f"T must be complex128 or complex64, got {dtype}")
    p = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    want = torch.complex128 if p == QST_F64 else torch.complex64
    if dtype != want:
        raise TypeError(f"precision {_NAMES.get(p, p)} needs {want} storage, got {dtype}")
    return p


def real_dtype(prec: int) -> torch.dtype:
    return torch.float64 if prec == QST_F64 else torch.float32


def complex_dtype(prec: int) -> torch.dtype:
    return torch.complex128 if prec == QST_F64 else torch.complex64


def _qubits(d: int) -> int:
    n = d.bit_length() - 1
    if d != 1 << n or not 1 <= n <= QST_MAX_QUBITS:
        raise ValueError(f"matrix side {d} is not 2^N with 1 <= N <= {QST_MAX_QUBITS}")
    return n


def _matrix(x: torch.Tensor, name: str) -> tuple[int, int]:
    if x.dim() != 2 or x.shape[0] != x.shape[1]:
        raise ValueError(f"{name} must be a square matrix, got shape {tuple(x.shape)}")
    if not x.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if x.stride(1) != 1 or x.stride(0) < x.shape[1]:
        raise ValueError(f"{name} must be row-major with unit column stride")
    return _qubits(x.shape[0]), x.stride(0)


def _vector(x: torch.Tensor, name: str, n: int, dtype: torch.dtype) -> None:
    if not x.is_cuda or x.dtype != dtype or not x.is_contiguous() or x.numel() != 4 ** n:
        raise ValueError(f"{name} must be a contiguous GPU {dtype} vector of 4^{n} entries")


def _stream(dev: torch.device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)


def _workspace(n: int, prec: int, op: int, dev: torch.device):
    nbytes = workspace_bytes(n, prec, op)
    if nbytes == 0:
        return None, 0
    return torch.empty(nbytes, dtype=torch.uint8, device=dev), nbytes


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


def _povm_arg(povm):
    """None (tetrahedral) or a host array of 32 doubles from a (4, 2, 2) complex array."""
    if povm is None:
        return None
    m = torch.as_tensor(povm).to(torch.complex128).reshape(4, 2, 2)
    flat = torch.view_as_real(m.contiguous()).reshape(-1).tolist()
    return (ctypes.c_double * 32)(*flat)


#: State-map modes: the pre-map applied to T before rho = T' T'^dagger / Tr.
#: "plain" (none), "hermitian" (Chol_H: (T + T^dagger)/2, the paper's
#: default), "lower" (Chol_Delta: lower triangle of T), "abs" (the P-order
#: absolute map, T' = Q |Lambda|^(P/2) Q^dagger of the Hermitian part).
STATE_MAPS = {"plain": 0, "hermitian": QST_PREMAP_HERMITIAN, "lower": QST_PREMAP_LOWER, "abs": -1}


def state_premap(X: torch.Tensor, mode: str, prec=None, out: torch.Tensor | None = None) -> torch.Tensor:
    """Y = P(X) for the pre-map of a state-map mode ("hermitian" or "lower");
    out=X works in place.  P is self-adjoint, so it also maps dL/dT' to dL/dT."""
    if mode not in ("hermitian", "lower"):
        raise ValueError(f"unknown pre-map {mode!r}")
    n, ld = _matrix(X, "X")
    p = _prec(X.dtype, prec)
    if out is None:
        out = torch.empty(X.shape, dtype=X.dtype, device=X.device)
    else:
        n2, _ = _matrix(out, "out")
        if n2 != n or out.dtype != X.dtype:
            raise ValueError("out must match X in size and dtype")
    _lib.check(_lib.lib().qst_state_premap(n, p, STATE_MAPS[mode], X.data_ptr(), ld, out.data_ptr(), out.stride(0),
                                           _stream(X.device)), "qst_state_premap")
    return out


def abs_map(T: torch.Tensor, P: float, prec=None, out: torch.Tensor | None = None, Q0: torch.Tensor | None = None):
    """A = Q |Lambda|^(P/2) Q^dagger for the Hermitian part of T (qst_abs_map;
    the state map of A is the P-order absolute projection).  Returns
    (A, Q, lam, sweeps): Q d x d complex128, lam d float64, both on T's
    device, and the Jacobi sweeps taken (0: the direct solver, which runs
    without Q0).  Q0: optional warm start for the Jacobi solver (a unitary Q
    from an earlier call on a nearby T).  Synchronises the stream."""
    n, ld = _matrix(T, "T")
    p = _prec(T.dtype, prec)
    d = 1 << n
    if Q0 is not None and (Q0.shape != (d, d) or Q0.dtype != torch.complex128 or not Q0.is_contiguous()
                           or Q0.device != T.device):
        raise ValueError("Q0 must be a d x d contiguous complex128 matrix on T's device")
    if out is None:
        out = torch.empty((d, d), dtype=T.dtype, device=T.device)
    else:
        n2, _ = _matrix(out, "out")
        if n2 != n or out.dtype != T.dtype:
            raise ValueError("out must match T in size and dtype")
    Q = torch.empty((d, d), dtype=torch.complex128, device=T.device)
    lam = torch.empty(d, dtype=torch.float64, device=T.device)
    sweeps = ctypes.c_int(-1)
    ws, nb = _workspace(n, p, QST_OP_ABS_MAP, T.device)
    _lib.check(_lib.lib().qst_abs_map(n, p, float(P), T.data_ptr(), ld, _ptr(Q0), out.data_ptr(), out.stride(0),
                                      Q.data_ptr(), lam.data_ptr(), ctypes.byref(sweeps), _ptr(ws), nb,
                                      _stream(T.device)), "qst_abs_map")
    return out, Q, lam, sweeps.value


def abs_map_async(T: torch.Tensor, P: float, prec=None, max_sweeps: int = 16, out: torch.Tensor | None = None,
                  Q0: torch.Tensor | None = None, Q: torch.Tensor | None = None, lam: torch.Tensor | None = None,
                  sweeps: torch.Tensor | None = None, ws: torch.Tensor | None = None):
    """abs_map without synchronisation (qst_abs_map_async): the direct solver
    without Q0; with Q0, at most max_sweeps warm-started Jacobi sweeps, the
    stopping rule applied on the device.
    Returns (A, Q, lam, sweeps) with sweeps a 0-dim int32 device tensor
    (the sweeps taken, -1 when not converged: then A, Q and lam are not
    valid).  Every output and the workspace may be passed in, so that the
    call can be captured in a HIP graph without allocating."""
    n, ld = _matrix(T, "T")
    p = _prec(T.dtype, prec)
    d = 1 << n
    if Q0 is not None and (Q0.shape != (d, d) or Q0.dtype != torch.complex128 or not Q0.is_contiguous()
                           or Q0.device != T.device):
        raise ValueError("Q0 must be a d x d contiguous complex128 matrix on T's device")
    out = torch.empty((d, d), dtype=T.dtype, device=T.device) if out is None else out
    Q = torch.empty((d, d), dtype=torch.complex128, device=T.device) if Q is None else Q
    lam = torch.empty(d, dtype=torch.float64, device=T.device) if lam is None else lam
    sweeps = torch.empty((), dtype=torch.int32, device=T.device) if sweeps is None else sweeps
    nb = workspace_bytes(n, p, QST_OP_ABS_MAP)
    if ws is None:
        ws, nb = _workspace(n, p, QST_OP_ABS_MAP, T.device)
    _lib.check(_lib.lib().qst_abs_map_async(n, p, float(P), T.data_ptr(), ld, _ptr(Q0), out.data_ptr(), out.stride(0),
                                            Q.data_ptr(), lam.data_ptr(), int(max_sweeps), sweeps.data_ptr(),
                                            _ptr(ws), nb, _stream(T.device)), "qst_abs_map_async")
    return out, Q, lam, sweeps


def abs_map_backward(Q: torch.Tensor, lam: torch.Tensor, P: float, GA: torch.Tensor, prec=None,
                     out: torch.Tensor | None = None) -> torch.Tensor:
    """dL/dT from dL/dA through the absolute map (qst_abs_map_backward)."""
    n, ld = _matrix(GA, "GA")
    p = _prec(GA.dtype, prec)
    d = 1 << n
    if Q.shape != (d, d) or Q.dtype != torch.complex128 or not Q.is_contiguous() or Q.device != GA.device:
        raise ValueError("Q must be the d x d complex128 matrix returned by abs_map")
    if lam.shape != (d,) or lam.dtype != torch.float64 or not lam.is_contiguous() or lam.device != GA.device:
        raise ValueError("lam must be the d float64 eigenvalues returned by abs_map")
    if out is None:
        out = torch.empty((d, d), dtype=GA.dtype, device=GA.device)
    ws, nb = _workspace(n, p, QST_OP_ABS_MAP, GA.device)
    _lib.check(_lib.lib().qst_abs_map_backward(n, p, float(P), Q.data_ptr(), lam.data_ptr(), GA.data_ptr(), ld,
                                               out.data_ptr(), out.stride(0), _ptr(ws), nb, _stream(GA.device)),
               "qst_abs_map_backward")
    return out


class AbsMapFn(torch.autograd.Function):
    """T' = Q |Lambda|^(P/2) Q^dagger of the Hermitian part of T, backward by
    qst_abs_map_backward (saves Q and the eigenvalues).  state: None, or a
    dict that receives this call's Q and sweeps; with state["warm"] its "Q"
    (if present) warm-starts the Jacobi eigensolver, otherwise the direct
    solver runs.  With state["max_sweeps"] set the call is the
    unsynchronised qst_abs_map_async (with that bound on the warm-started
    Jacobi sweeps; its sweeps a device tensor)."""

    @staticmethod
    def forward(ctx, T, P, prec, state=None):
        Q0 = state.get("Q") if state is not None and state.get("warm") else None
        bound = None if state is None else state.get("max_sweeps")
        if bound:
            prev = state.get("sweeps")
            if isinstance(prev, torch.Tensor) and int(prev.item()) < 0:
                raise QstError(1, "qst_abs_map_async", "the previous call had failed (not finite, or not "
                                                       "converged within max_sweeps)")
            A, Q, lam, sweeps = abs_map_async(T, P, prec, max_sweeps=bound, Q0=Q0)
        else:
            A, Q, lam, sweeps = abs_map(T, P, prec, Q0=Q0)
        if state is not None:
            state["Q"], state["sweeps"] = Q, sweeps
        ctx.P, ctx.prec = P, prec
        ctx.save_for_backward(Q, lam)
        return A

    @staticmethod
    def backward(ctx, g):
        Q, lam = ctx.saved_tensors
        return abs_map_backward(Q, lam, ctx.P, g.contiguous(), ctx.prec), None, None, None


class AbsProjection:
    """The P-order absolute map for a training loop: each call returns
    T' = Q |Lambda|^(P/2) Q^dagger (differentiable).  Use as
    likelihood(proj(T), f).

    warm: False -- every call runs the direct eigensolver (a fixed sequence
    of launches); True -- each call keeps Q to warm-start the next call's
    Jacobi eigensolver.  max_sweeps: None -- synchronous calls (one
    synchronisation per call, or per Jacobi sweep when warm); an int -- the
    calls run without any synchronisation (the warm ones with at most that
    many sweeps), and a call that failed is reported by the next one
    (QstError)."""

    def __init__(self, P: float, prec=None, max_sweeps: int | None = None, warm: bool = False):
        self.P, self.prec = float(P), prec
        self.max_sweeps = max_sweeps
        self.warm = bool(warm)
        self.state: dict = {}

    def __call__(self, T: torch.Tensor) -> torch.Tensor:
        Q = self.state.get("Q")
        if Q is not None and (Q.shape != (T.shape[0], T.shape[0]) or Q.device != T.device):
            self.state = {}
        self.state["max_sweeps"] = self.max_sweeps
        self.state["warm"] = self.warm
        return AbsMapFn.apply(T, self.P, self.prec, self.state)

    @property
    def sweeps(self) -> int | None:
        s = self.state.get("sweeps")
        return int(s.item()) if isinstance(s, torch.Tensor) else s


class StatePremapFn(torch.autograd.Function):
    """T' = P(T) with backward dL/dT = P(dL/dT') (P self-adjoint)."""

    @staticmethod
    def forward(ctx, T, mode, prec):
        ctx.mode, ctx.prec = mode, prec
        return state_premap(T, mode, prec)

    @staticmethod
    def backward(ctx, g):
        return state_premap(g.contiguous(), ctx.mode, ctx.prec), None, None


def state_map(T: torch.Tensor, prec=None):
    """rho = T T^dagger / tau and tau (a 0-dim float64 device tensor)."""
    n, ld = _matrix(T, "T")
    p = _prec(T.dtype, prec)
    rho = torch.empty(T.shape, dtype=T.dtype, device=T.device)
    tau = torch.empty((), dtype=torch.float64, device=T.device)
    ws, nb = _workspace(n, p, QST_OP_STATE_MAP, T.device)
    _lib.check(_lib.lib().qst_state_map(n, p, T.data_ptr(), ld, rho.data_ptr(), rho.stride(0), tau.data_ptr(),
                                        _ptr(ws), nb, _stream(T.device)), "qst_state_map")
    return rho, tau


def povm_probs(rho: torch.Tensor, prec=None, povm=None) -> torch.Tensor:
    """p_k = Tr(rho M_k) for all 4^N outcomes (lower triangle of rho read)."""
    n, ld = _matrix(rho, "rho")
    p = _prec(rho.dtype, prec)
    out = torch.empty(4 ** n, dtype=real_dtype(p), device=rho.device)
    ws, nb = _workspace(n, p, QST_OP_POVM_PROBS, rho.device)
    _lib.check(_lib.lib().qst_povm_probs(n, p, rho.data_ptr(), ld, _povm_arg(povm), out.data_ptr(), _ptr(ws), nb,
                                         _stream(rho.device)), "qst_povm_probs")
    return out


def nll(p: torch.Tensor, f: torch.Tensor, prec=None):
    """(out, bad): out[0] = L, out[1] = F = sum f (float64); bad = uint64 counts
    [f>0 with p<=0, NaN entries] stored as int64."""
    n = (p.numel().bit_length() - 1) // 2
    pr = QST_F64 if (prec is None and p.dtype == torch.float64) else (
        QST_F32 if prec is None else (PRECISIONS[prec] if isinstance(prec, str) else int(prec)))
    _vector(p, "p", n, real_dtype(pr))
    _vector(f, "f", n, real_dtype(pr))
    out = torch.empty(2, dtype=torch.float64, device=p.device)
    bad = torch.empty(2, dtype=torch.int64, device=p.device)
    ws, nb = _workspace(n, pr, QST_OP_NLL, p.device)
    _lib.check(_lib.lib().qst_nll(n, pr, p.data_ptr(), f.data_ptr(), out.data_ptr(), bad.data_ptr(), _ptr(ws), nb,
                                  _stream(p.device)), "qst_nll")
    return out, bad


def nll_backward(T: torch.Tensor, f: torch.Tensor, p: torch.Tensor | None, tau: torch.Tensor | None, prec=None,
                 povm=None, upstream: torch.Tensor | None = None, nll_out: torch.Tensor | None = None) -> torch.Tensor:
    """dL/dRe T + i dL/dIm T (times *upstream).  p=None recomputes rho and p;
    nll_out (the [L, F] tensor of nll()) supplies F = sum f."""
    n, ld = _matrix(T, "T")
    pr = _prec(T.dtype, prec)
    _vector(f, "f", n, real_dtype(pr))
    if p is not None:
        _vector(p, "p", n, real_dtype(pr))
        if tau is None:
            raise ValueError("tau is required when p is given")
    _scalar(tau, "tau")
    _scalar(upstream, "upstream")
    if nll_out is not None and (nll_out.dtype != torch.float64 or nll_out.numel() != 2 or not nll_out.is_cuda
                                or not nll_out.is_contiguous()):
        raise ValueError("nll_out must be the contiguous two-element float64 GPU tensor returned by nll()")
    grad = torch.empty(T.shape, dtype=T.dtype, device=T.device)
    ws, nb = _workspace(n, pr, QST_OP_NLL_BACKWARD, T.device)
    _lib.check(_lib.lib().qst_nll_backward(n, pr, T.data_ptr(), ld, f.data_ptr(), _ptr(p), _ptr(tau),
                                           _ptr(nll_out), _povm_arg(povm), _ptr(upstream), grad.data_ptr(),
                                           grad.stride(0), _ptr(ws), nb, _stream(T.device)), "qst_nll_backward")
    return grad


def _scalar(t, name):
    if t is not None and (t.dtype != torch.float64 or t.numel() != 1 or not t.is_cuda):
        raise ValueError(f"{name} must be a one-element float64 GPU tensor")


def likelihood_forward(T: torch.Tensor, f: torch.Tensor, prec=None, povm=None, with_grad_matrix: bool = True):
    """One library call for L and the adjoint matrix: returns (out, tau, G, bad)
    with out = [L, F] (float64), tau (0-dim float64), G = G' = sum_k (F -
    f_k/p_k) M_k as a d x d matrix of T's dtype (None when with_grad_matrix is
    False) and bad = [f>0 with p<=0, NaN] counts.  rho and p never leave the
    library's workspace."""
    n, ld = _matrix(T, "T")
    pr = _prec(T.dtype, prec)
    _vector(f, "f", n, real_dtype(pr))
    out = torch.empty(2, dtype=torch.float64, device=T.device)
    bad = torch.empty(2, dtype=torch.int64, device=T.device)
    tau = torch.empty((), dtype=torch.float64, device=T.device)
    G = torch.empty(T.shape, dtype=T.dtype, device=T.device) if with_grad_matrix else None
    ws, nb = _workspace(n, pr, QST_OP_LIKELIHOOD, T.device)
    _lib.check(_lib.lib().qst_likelihood(n, pr, T.data_ptr(), ld, f.data_ptr(), _povm_arg(povm), tau.data_ptr(),
                                         out.data_ptr(), bad.data_ptr(), _ptr(G), 0 if G is None else G.stride(0),
                                         _ptr(ws), nb, _stream(T.device)), "qst_likelihood")
    return out, tau, G, bad


def likelihood_grad(T: torch.Tensor, f: torch.Tensor, prec=None, povm=None):
    """L and its gradient in one library call (qst_likelihood_grad): returns
    (out, tau, grad, bad) with out = [L, F] (float64), tau (0-dim float64),
    grad = dL/dRe T + i dL/dIm T (T's dtype and shape) and bad as
    likelihood_forward -- the results of likelihood_forward followed by
    grad_product, bitwise, without G'."""
    n, ld = _matrix(T, "T")
    pr = _prec(T.dtype, prec)
    _vector(f, "f", n, real_dtype(pr))
    out = torch.empty(2, dtype=torch.float64, device=T.device)
    bad = torch.empty(2, dtype=torch.int64, device=T.device)
    tau = torch.empty((), dtype=torch.float64, device=T.device)
    grad = torch.empty(T.shape, dtype=T.dtype, device=T.device)
    ws, nb = _workspace(n, pr, QST_OP_LIKELIHOOD_GRAD, T.device)
    _lib.check(_lib.lib().qst_likelihood_grad(n, pr, T.data_ptr(), ld, f.data_ptr(), _povm_arg(povm), tau.data_ptr(),
                                              out.data_ptr(), bad.data_ptr(), grad.data_ptr(), grad.stride(0),
                                              _ptr(ws), nb, _stream(T.device)), "qst_likelihood_grad")
    return out, tau, grad, bad


def likelihood_forward_noalloc(T: torch.Tensor, f: torch.Tensor, prec=None, povm=None, G: torch.Tensor | None = None,
                               out: torch.Tensor | None = None, tau: torch.Tensor | None = None,
                               bad: torch.Tensor | None = None):
    """likelihood_forward through qst_likelihood_noalloc: the library's static
    device scratch serves as the workspace (N <= 9), so the library call
    allocates nothing.  Output tensors may be passed in (then this wrapper
    allocates nothing either); returns (out, tau, G, bad) as
    likelihood_forward."""
    n, ld = _matrix(T, "T")
    pr = _prec(T.dtype, prec)
    _vector(f, "f", n, real_dtype(pr))
    out = torch.empty(2, dtype=torch.float64, device=T.device) if out is None else out
    bad = torch.empty(2, dtype=torch.int64, device=T.device) if bad is None else bad
    tau = torch.empty((), dtype=torch.float64, device=T.device) if tau is None else tau
    if G is not None:
        n2, ldg = _matrix(G, "G")
        if n2 != n or G.dtype != T.dtype:
            raise ValueError("G must match T in size and dtype")
    _lib.check(_lib.lib().qst_likelihood_noalloc(n, pr, T.data_ptr(), ld, f.data_ptr(), _povm_arg(povm),
                                                 tau.data_ptr(), out.data_ptr(), bad.data_ptr(), _ptr(G),
                                                 0 if G is None else G.stride(0), _stream(T.device)),
               "qst_likelihood_noalloc")
    return out, tau, G, bad


def likelihood_forward_fc(T: torch.Tensor, f: torch.Tensor, p_target: torch.Tensor, prec=None, povm=None,
                          with_grad_matrix: bool = True):
    """likelihood_forward plus F_c = (sum_k sqrt(p_k p_target_k))^2 of the
    model's distribution against p_target (qst_likelihood_fc; in the fused
    last pass where the plan has one).  Returns (out, tau, G, bad, fc), fc a
    0-dim float64 device tensor."""
    n, ld = _matrix(T, "T")
    pr = _prec(T.dtype, prec)
    _vector(f, "f", n, real_dtype(pr))
    _vector(p_target, "p_target", n, real_dtype(pr))
    out = torch.empty(2, dtype=torch.float64, device=T.device)
    bad = torch.empty(2, dtype=torch.int64, device=T.device)
    tau = torch.empty((), dtype=torch.float64, device=T.device)
    fc = torch.empty((), dtype=torch.float64, device=T.device)
    G = torch.empty(T.shape, dtype=T.dtype, device=T.device) if with_grad_matrix else None
    ws, nb = _workspace(n, pr, QST_OP_LIKELIHOOD, T.device)
    _lib.check(_lib.lib().qst_likelihood_fc(n, pr, T.data_ptr(), ld, f.data_ptr(), p_target.data_ptr(),
                                            _povm_arg(povm), tau.data_ptr(), out.data_ptr(), fc.data_ptr(),
                                            bad.data_ptr(), _ptr(G), 0 if G is None else G.stride(0), _ptr(ws), nb,
                                            _stream(T.device)), "qst_likelihood_fc")
    return out, tau, G, bad, fc


def grad_product(G: torch.Tensor, T: torch.Tensor, tau: torch.Tensor, prec=None,
                 upstream: torch.Tensor | None = None) -> torch.Tensor:
    """dL/dRe T + i dL/dIm T = (2 s / tau) G' T, s = *upstream (1 if None)."""
    n, ldt = _matrix(T, "T")
    n2, ldg = _matrix(G, "G")
    if n2 != n or G.dtype != T.dtype:
        raise ValueError("G must match T in size and dtype")
    pr = _prec(T.dtype, prec)
    _scalar(tau, "tau")
    _scalar(upstream, "upstream")
    grad = torch.empty(T.shape, dtype=T.dtype, device=T.device)
    ws, nb = _workspace(n, pr, QST_OP_GRAD_PRODUCT, T.device)
    _lib.check(_lib.lib().qst_grad_product(n, pr, G.data_ptr(), ldg, T.data_ptr(), ldt, tau.data_ptr(),
                                           _ptr(upstream), grad.data_ptr(), grad.stride(0), _ptr(ws), nb,
                                           _stream(T.device)), "qst_grad_product")
    return grad


def fidelity_lowrank(T: torch.Tensor, W: torch.Tensor, prec=None) -> torch.Tensor:
    """F_q(T T^dagger / Tr, W W^dagger / Tr) for a d x r target factor W
    (r <= QST_FIDELITY_MAX_RANK; a pure state is a d x 1 W), as a 0-dim
    float64 device tensor."""
    n, ld = _matrix(T, "T")
    if W.dim() != 2 or W.shape[0] != T.shape[0] or W.dtype != T.dtype or not W.is_cuda or W.stride(1) != 1:
        raise ValueError("W must be a d x r row-major GPU matrix of T's dtype")
    r = W.shape[1]
    pr = _prec(T.dtype, prec)
    F = torch.empty((), dtype=torch.float64, device=T.device)
    ws, nb = _workspace(n, pr, QST_OP_FIDELITY, T.device)
    _lib.check(_lib.lib().qst_fidelity_lowrank(n, pr, T.data_ptr(), ld, W.data_ptr(), W.stride(0), r, F.data_ptr(),
                                               _ptr(ws), nb, _stream(T.device)), "qst_fidelity_lowrank")
    return F


def fidelity_general_async(T: torch.Tensor, rho: torch.Tensor, prec=None, max_sweeps: int = 16):
    """fidelity_general without synchronisation (qst_fidelity_general_async):
    returns (F, sweeps), a 0-dim float64 and a 0-dim int32 device tensor
    (sweeps 0; -1: the input was not finite, F not valid)."""
    n, ld = _matrix(T, "T")
    n2, ldr = _matrix(rho, "rho")
    if n2 != n or rho.dtype != T.dtype:
        raise ValueError("rho must match T in size and dtype")
    pr = _prec(T.dtype, prec)
    F = torch.empty((), dtype=torch.float64, device=T.device)
    sweeps = torch.empty((), dtype=torch.int32, device=T.device)
    ws, nb = _workspace(n, pr, QST_OP_ABS_MAP, T.device)
    _lib.check(_lib.lib().qst_fidelity_general_async(n, pr, T.data_ptr(), ld, rho.data_ptr(), ldr, F.data_ptr(),
                                                     int(max_sweeps), sweeps.data_ptr(), _ptr(ws), nb,
                                                     _stream(T.device)), "qst_fidelity_general_async")
    return F, sweeps


def fidelity_general(T: torch.Tensor, rho: torch.Tensor, prec=None):
    """F_q(T T^dagger / Tr, rho) for any target density matrix rho (d x d,
    T's dtype) by one eigensolve of T^dagger rho T (qst_fidelity_general).
    Returns (F as a 0-dim float64 device tensor, 0 -- no Jacobi sweeps run).
    Synchronises the stream."""
    n, ld = _matrix(T, "T")
    n2, ldr = _matrix(rho, "rho")
    if n2 != n or rho.dtype != T.dtype:
        raise ValueError("rho must match T in size and dtype")
    pr = _prec(T.dtype, prec)
    F = torch.empty((), dtype=torch.float64, device=T.device)
    sweeps = ctypes.c_int(-1)
    ws, nb = _workspace(n, pr, QST_OP_ABS_MAP, T.device)
    _lib.check(_lib.lib().qst_fidelity_general(n, pr, T.data_ptr(), ld, rho.data_ptr(), ldr, F.data_ptr(),
                                               ctypes.byref(sweeps), _ptr(ws), nb, _stream(T.device)),
               "qst_fidelity_general")
    return F, sweeps.value


def fidelity_classical(p_hat: torch.Tensor, p: torch.Tensor, prec=None) -> torch.Tensor:
    """F_c = (sum_k sqrt(p_hat_k p_k))^2 as a 0-dim float64 device tensor."""
    n = (p.numel().bit_length() - 1) // 2
    pr = QST_F64 if (prec is None and p.dtype == torch.float64) else (
        QST_F32 if prec is None else (PRECISIONS[prec] if isinstance(prec, str) else int(prec)))
    _vector(p_hat, "p_hat", n, real_dtype(pr))
    _vector(p, "p", n, real_dtype(pr))
    F = torch.empty((), dtype=torch.float64, device=p.device)
    ws, nb = _workspace(n, pr, QST_OP_FIDELITY, p.device)
    _lib.check(_lib.lib().qst_fidelity_classical(n, pr, p_hat.data_ptr(), p.data_ptr(), F.data_ptr(), _ptr(ws), nb,
                                                 _stream(p.device)), "qst_fidelity_classical")
    return F


def _fnn_args(W2: torch.Tensor, x: torch.Tensor):
    D = x.numel()
    n = (D.bit_length() - 1) // 2
    if 4 ** n != D or not 1 <= n <= QST_MAX_QUBITS:
        raise ValueError(f"x must have 4^N entries, got {D}")
    return n, D, 2 * n


def _check_real(t: torch.Tensor, name: str, shape, dtype):
    if tuple(t.shape) != tuple(shape) or t.dtype != dtype or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous GPU {dtype} tensor of shape {tuple(shape)}")


def fnn_forward(W1, b1, W2, b2, x, prec=None):
    """The mapping network (Sec. 3.1): returns (T, h_pre) with T the d x d
    Hermitian matrix filled from the 4^N outputs and h_pre the 2N hidden
    pre-activations (input of fnn_backward)."""
    n, D, H = _fnn_args(W2, x)
    rt = x.dtype
    for t, name, shape in ((W1, "W1", (H, D)), (b1, "b1", (H,)), (W2, "W2", (D, H)), (b2, "b2", (D,)), (x, "x", (D,))):
        _check_real(t, name, shape, rt)
    pr = QST_F64 if rt == torch.float64 else (QST_F32 if prec is None else _prec(torch.complex64, prec))
    d = 1 << n
    T = torch.empty((d, d), dtype=torch.complex128 if rt == torch.float64 else torch.complex64, device=x.device)
    h_pre = torch.empty(H, dtype=rt, device=x.device)
    ws, nb = _workspace(n, pr, QST_OP_FNN, x.device)
    _lib.check(_lib.lib().qst_fnn_forward(n, pr, W1.data_ptr(), b1.data_ptr(), W2.data_ptr(), b2.data_ptr(),
                                          x.data_ptr(), h_pre.data_ptr(), T.data_ptr(), T.stride(0), _ptr(ws), nb,
                                          _stream(x.device)), "qst_fnn_forward")
    return T, h_pre


def fnn_backward(W2, x, h_pre, G, prec=None):
    """Parameter gradients (dW1, db1, dW2, db2) from G = dL/dT."""
    n, D, H = _fnn_args(W2, x)
    rt = x.dtype
    _check_real(W2, "W2", (D, H), rt)
    _check_real(h_pre, "h_pre", (H,), rt)
    n2, ldg = _matrix(G, "G")
    if n2 != n:
        raise ValueError("G must be d x d")
    pr = QST_F64 if rt == torch.float64 else (QST_F32 if prec is None else _prec(torch.complex64, prec))
    dW1 = torch.empty((H, D), dtype=rt, device=x.device)
    db1 = torch.empty(H, dtype=rt, device=x.device)
    dW2 = torch.empty((D, H), dtype=rt, device=x.device)
    db2 = torch.empty(D, dtype=rt, device=x.device)
    ws, nb = _workspace(n, pr, QST_OP_FNN, x.device)
    _lib.check(_lib.lib().qst_fnn_backward(n, pr, W2.data_ptr(), x.data_ptr(), h_pre.data_ptr(), G.data_ptr(), ldg,
                                           dW1.data_ptr(), db1.data_ptr(), dW2.data_ptr(), db2.data_ptr(), _ptr(ws),
                                           nb, _stream(x.device)), "qst_fnn_backward")
    return dW1, db1, dW2, db2


class FnnFn(torch.autograd.Function):
    """T = fill(W2 leaky(W1 x + b1) + b2) with the library's backward."""

    @staticmethod
    def forward(ctx, W1, b1, W2, b2, x, prec):
        T, h_pre = fnn_forward(W1, b1, W2, b2, x, prec)
        ctx.save_for_backward(W2, x, h_pre)
        ctx.prec = prec
        return T

    @staticmethod
    def backward(ctx, g):
        W2, x, h_pre = ctx.saved_tensors
        dW1, db1, dW2, db2 = fnn_backward(W2, x, h_pre, g.contiguous(), ctx.prec)
        return dW1, db1, dW2, db2, None, None


class MappingNetwork(torch.nn.Module):
    """The 3-layer network of Sec. 3.1 for N qubits: 4^N inputs (the
    measured distribution), 2N hidden units (leaky ReLU), 4^N outputs filling
    the Hermitian T.  Parameters start uniform in +-1/sqrt(fan_in), the
    usual initialisation of a linear layer."""

    def __init__(self, n_qubits: int, dtype=torch.float32, device="cuda", generator=None):
        super().__init__()
        D, H = 4 ** n_qubits, 2 * n_qubits

        def uni(shape, fan_in):
            b = 1.0 / fan_in ** 0.5
            return torch.nn.Parameter((torch.rand(shape, generator=generator, dtype=torch.float64) * 2 - 1).mul(b)
                                      .to(device=device, dtype=dtype))

        self.W1, self.b1 = uni((H, D), D), uni((H,), D)
        self.W2, self.b2 = uni((D, H), H), uni((D,), H)

    def forward(self, x, prec=None):
        return FnnFn.apply(self.W1, self.b1, self.W2, self.b2, x, prec)


class Rprop(torch.optim.Optimizer):
    """Rprop (iRprop-, the optimiser of the paper's setup) with each tensor's
    step done by one library call (qst_rprop_step): param, grad, previous
    gradient and step size streamed once."""

    def __init__(self, params, lr=1e-3, etas=(0.5, 1.2), step_sizes=(1e-6, 50.0)):
        super().__init__(params, dict(lr=lr, etas=etas, step_sizes=step_sizes))

    @torch.no_grad()
    def step(self, closure=None):
        loss = closure() if closure is not None else None
        for group in self.param_groups:
            em, ep = group["etas"]
            smin, smax = group["step_sizes"]
            for p in group["params"]:
                if p.grad is None:
                    continue
                if p.dtype not in (torch.float32, torch.float64) or not p.is_cuda or not p.is_contiguous():
                    raise ValueError("Rprop takes contiguous float32 / float64 GPU parameters")
                st = self.state[p]
                if not st:
                    st["prev"] = torch.zeros_like(p)
                    st["step"] = torch.full_like(p, group["lr"])
                g = p.grad.contiguous()
                pr = QST_F64 if p.dtype == torch.float64 else QST_F32
                _lib.check(_lib.lib().qst_rprop_step(p.numel(), pr, p.data_ptr(), g.data_ptr(), st["prev"].data_ptr(),
                                                     st["step"].data_ptr(), em, ep, smin, smax, _stream(p.device)),
                           "qst_rprop_step")
        return loss


class LikelihoodFn(torch.autograd.Function):
    """L(T) = -sum_k f_k ln Tr(M_k T T^dagger / Tr(T T^dagger)) with the
    hand-written adjoint.  Modes:
      "fused"     forward = qst_likelihood (L and G'), backward = qst_grad_product;
                  kept between them: T, G' and tau (nothing of length 4^N);
      "stored"    forward keeps p; backward = qst_nll_backward(p);
      "recompute" forward keeps T, f, tau; backward rebuilds rho and p."""

    @staticmethod
    def forward(ctx, T, f, prec, mode, povm):
        ctx.prec, ctx.povm, ctx.mode = prec, povm, mode
        if mode == "fused":
            need = ctx.needs_input_grad[0]
            out, tau, G, _ = likelihood_forward(T, f, prec, povm, with_grad_matrix=need)
            ctx.save_for_backward(T, G, tau)
            return out[0].clone()
        rho, tau = state_map(T, prec)
        p = povm_probs(rho, prec, povm)
        del rho
        out, _ = nll(p, f, _prec(T.dtype, prec))
        if mode == "recompute":
            ctx.save_for_backward(T, f, tau, out)
        else:
            ctx.save_for_backward(T, f, tau, out, p)
        return out[0].clone()

    @staticmethod
    def backward(ctx, g):
        up = g.detach().to(torch.float64).reshape(1).contiguous()
        if ctx.mode == "fused":
            T, G, tau = ctx.saved_tensors
            return grad_product(G, T, tau, ctx.prec, up), None, None, None, None
        saved = ctx.saved_tensors
        T, f, tau, out = saved[0], saved[1], saved[2], saved[3]
        p = None if ctx.mode == "recompute" else saved[4]
        grad = nll_backward(T, f, p, None if p is None else tau, ctx.prec, ctx.povm, up, out)
        return grad, None, None, None, None


def _general_povm_arg(povms, n: int):
    """(settings, K, host array) from general product POVMs: (K, 2, 2) (one
    POVM on every qubit), (N, K, 2, 2) (a POVM per qubit) or
    (S, N, K, 2, 2) (S settings), complex."""
    m = torch.as_tensor(povms).to(torch.complex128)
    if m.dim() == 3:
        m = m.unsqueeze(0).expand(n, *m.shape)
    if m.dim() == 4:
        m = m.unsqueeze(0)
    if m.dim() != 5 or m.shape[1] != n or tuple(m.shape[3:]) != (2, 2):
        raise ValueError(f"povms must be (K, 2, 2), (N, K, 2, 2) or (S, N, K, 2, 2) with N = {n}")
    S, K = int(m.shape[0]), int(m.shape[2])
    flat = torch.view_as_real(m.contiguous()).reshape(-1).tolist()
    return S, K, (ctypes.c_double * len(flat))(*flat)


def povm_probs_general(rho: torch.Tensor, povms, prec=None) -> torch.Tensor:
    """K^N probabilities of a product POVM with a K-element POVM per qubit
    (qst_povm_probs_general); povms (K, 2, 2) or (N, K, 2, 2)."""
    n, ld = _matrix(rho, "rho")
    p = _prec(rho.dtype, prec)
    S, K, arr = _general_povm_arg(povms, n)
    if S != 1:
        raise ValueError("povm_probs_general takes one setting")
    out = torch.empty(K ** n, dtype=real_dtype(p), device=rho.device)
    nb = int(_lib.lib().qst_workspace_bytes_general(n, p, K, QST_OP_POVM_PROBS))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=rho.device)
    _lib.check(_lib.lib().qst_povm_probs_general(n, p, rho.data_ptr(), ld, K, arr, out.data_ptr(), ws.data_ptr(), nb,
                                                 _stream(rho.device)), "qst_povm_probs_general")
    return out


def likelihood_forward_general(T: torch.Tensor, f: torch.Tensor, povms, prec=None, with_grad_matrix: bool = True):
    """qst_likelihood_general: L summed over the settings and G' for
    grad_product.  povms as in _general_povm_arg; f of shape (S, K^N) or
    (K^N,) for one setting.  Returns (out = [L, F], tau, G, bad)."""
    n, ld = _matrix(T, "T")
    pr = _prec(T.dtype, prec)
    S, K, arr = _general_povm_arg(povms, n)
    f2 = f.reshape(S, K ** n) if f.dim() == 1 else f
    if tuple(f2.shape) != (S, K ** n) or f2.dtype != real_dtype(pr) or not f2.is_contiguous():
        raise ValueError(f"f must be a contiguous {real_dtype(pr)} tensor of shape ({S}, {K ** n})")
    out = torch.empty(2, dtype=torch.float64, device=T.device)
    bad = torch.empty(2, dtype=torch.int64, device=T.device)
    tau = torch.empty((), dtype=torch.float64, device=T.device)
    G = torch.empty(T.shape, dtype=T.dtype, device=T.device) if with_grad_matrix else None
    nb = int(_lib.lib().qst_workspace_bytes_general(n, pr, K, QST_OP_LIKELIHOOD))
    ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=T.device)
    _lib.check(_lib.lib().qst_likelihood_general(n, pr, T.data_ptr(), ld, S, K, arr, f2.data_ptr(), tau.data_ptr(),
                                                 out.data_ptr(), bad.data_ptr(), _ptr(G),
                                                 0 if G is None else G.stride(0), ws.data_ptr(), nb,
                                                 _stream(T.device)), "qst_likelihood_general")
    return out, tau, G, bad


class GeneralLikelihoodFn(torch.autograd.Function):
    """L(T) summed over general product-POVM settings; forward =
    qst_likelihood_general (L and G'), backward = qst_grad_product."""

    @staticmethod
    def forward(ctx, T, f, povms, prec):
        ctx.prec = prec
        out, tau, G, _ = likelihood_forward_general(T, f, povms, prec, with_grad_matrix=ctx.needs_input_grad[0])
        ctx.save_for_backward(T, G, tau)
        return out[0].clone()

    @staticmethod
    def backward(ctx, g):
        T, G, tau = ctx.saved_tensors
        up = g.detach().to(torch.float64).reshape(1).contiguous()
        return grad_product(G, T, tau, ctx.prec, up), None, None, None


def likelihood_general(T: torch.Tensor, f: torch.Tensor, povms, prec=None):
    """Differentiable negative log-likelihood over general product-POVM
    settings (a K-element POVM per qubit, several settings)."""
    return GeneralLikelihoodFn.apply(T, f, povms, prec)


def likelihood(T: torch.Tensor, f: torch.Tensor, prec=None, recompute: bool | None = None, povm=None,
               mode: str | None = None, state_map: str = "plain", P: float = 2.0):
    """Differentiable negative log-likelihood (0-dim float64 tensor).

    mode: "fused" (default), "stored" or "recompute" (see LikelihoodFn).
    recompute=True / False select "recompute" / "stored" when mode is None.
    state_map: "plain" (rho from T), "hermitian" (Chol_H), "lower"
    (Chol_Delta) or "abs" (the P-order absolute projection of Eq. abs_P,
    order P): rho from the pre-mapped T (see STATE_MAPS)."""
    if mode is None:
        mode = "fused" if recompute is None else ("recompute" if recompute else "stored")
    if mode not in ("fused", "stored", "recompute"):
        raise ValueError(f"unknown mode {mode!r}")
    if state_map not in STATE_MAPS:
        raise ValueError(f"unknown state map {state_map!r}")
    if state_map == "abs":
        T = AbsMapFn.apply(T, P, prec, None)
    elif state_map != "plain":
        T = StatePremapFn.apply(T, state_map, prec)
    return LikelihoodFn.apply(T, f, prec, mode, povm)


class BatchPlan:
    """Many independent instances (1 <= N_i <= 8) in one persistent launch
    (qst_batch_* in include/qst.h).  Inputs and outputs are packed tensors:
    T_all / grad_all hold the d_i x d_i matrices back to back (complex), f_all
    the 4^N_i frequencies back to back (real); offsets() gives the starts."""

    def __init__(self, n_qubits, prec="f32", povm=None, tune_cache: str | None = None):
        self.n = [int(x) for x in n_qubits]
        self.prec = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        arr = (ctypes.c_int * len(self.n))(*self.n)
        handle = ctypes.c_void_p()
        cache = tune_cache.encode() if tune_cache else None
        self._handle = None
        _lib.check(_lib.lib().qst_batch_plan_create(arr, len(self.n), self.prec, _povm_arg(povm), cache,
                                                    ctypes.byref(handle)), "qst_batch_plan_create")
        self._handle = handle
        t_off = (ctypes.c_int64 * (len(self.n) + 1))()
        f_off = (ctypes.c_int64 * (len(self.n) + 1))()
        _lib.check(_lib.lib().qst_batch_offsets(self._handle, t_off, f_off), "qst_batch_offsets")
        self.t_off = list(t_off)
        self.f_off = list(f_off)

    def offsets(self):
        return self.t_off, self.f_off

    def pack(self, mats, vecs, device):
        """Pack per-instance T (d x d) and f (4^N) into the plan's layout."""
        cd, rd = complex_dtype(self.prec), real_dtype(self.prec)
        T_all = torch.empty(self.t_off[-1], dtype=cd, device=device)
        f_all = torch.empty(self.f_off[-1], dtype=rd, device=device)
        for i, (m, v) in enumerate(zip(mats, vecs)):
            T_all[self.t_off[i]:self.t_off[i + 1]] = torch.as_tensor(m).reshape(-1).to(cd)
            f_all[self.f_off[i]:self.f_off[i + 1]] = torch.as_tensor(v).reshape(-1).to(rd)
        return T_all, f_all

    def run(self, T_all: torch.Tensor, f_all: torch.Tensor, use_graph: bool = True, out=None):
        """Forward and adjoint of every instance: returns (nll [count, 2] with
        (L_i, F_i), grad_all packed like T_all, bad [count, 2])."""
        cd, rd = complex_dtype(self.prec), real_dtype(self.prec)
        if T_all.dtype != cd or f_all.dtype != rd or not T_all.is_cuda or not f_all.is_cuda:
            raise TypeError(f"T_all must be {cd} and f_all {rd}, on the GPU")
        if T_all.numel() != self.t_off[-1] or f_all.numel() != self.f_off[-1]:
            raise ValueError("packed sizes do not match the plan")
        if not (T_all.is_contiguous() and f_all.is_contiguous()):
            raise ValueError("packed buffers must be contiguous")
        if out is None:
            nll_out = torch.empty((len(self.n), 2), dtype=torch.float64, device=T_all.device)
            bad = torch.empty((len(self.n), 2), dtype=torch.int64, device=T_all.device)
            grad = torch.empty_like(T_all)
        else:
            nll_out, bad, grad = out
        stream = torch.cuda.current_stream(T_all.device)
        use_graph = bool(use_graph) and stream.cuda_stream != 0
        _lib.check(_lib.lib().qst_batch_run(self._handle, T_all.data_ptr(), f_all.data_ptr(), nll_out.data_ptr(),
                                            bad.data_ptr(), grad.data_ptr(), 1 if use_graph else 0,
                                            _stream(T_all.device)), "qst_batch_run")
        return nll_out, grad, bad

    def info(self):
        grid, so, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _lib.check(_lib.lib().qst_batch_info(self._handle, ctypes.byref(grid), ctypes.byref(so), ctypes.byref(ms)),
                   "qst_batch_info")
        th, rr = ctypes.c_int(), ctypes.c_int()
        _lib.check(_lib.lib().qst_batch_shape(self._handle, ctypes.byref(th), ctypes.byref(rr)), "qst_batch_shape")
        return {"grid": grid.value, "sorted_order": bool(so.value), "tuned_ms": ms.value, "threads": th.value,
                "register_round_passes": bool(rr.value)}

    def close(self):
        if self._handle is not None:
            _lib.lib().qst_batch_plan_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
