"""FP64 CPU oracle for the tomography likelihood path -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or call this module.  The product path (the HIP
library and its Python binding) never does; they share no code with it.

What it computes, written from the paper (Wang, Cheng, Li, Chen,
"Ultrafast quantum state tomography with feed-forward neural networks"):

* state map   rho = T T^dagger / Tr(T T^dagger)
              (Sec. 2.2.1 Eq. T_matrix; Sec. 3.2 Eq. unified_DP and Eq. abs_P
              at P = 2 -- see the reading of T^dagger T vs T T^dagger below)
* modes       the pre-maps of Chol_H (Hermitian part, Sec. 2.2.2 and
              Eq. unified_DP) and Chol_Delta (lower triangle, Eq. T_matrix),
              and the P-order absolute projection (Eq. abs_P) by eigh, with
              the absolute map A = Q |Lambda|^(P/2) Q^dagger and its adjoint
* network     the 3-layer FNN of Sec. 3.1 (4^N -> 2N -> 4^N) filling the
              Hermitian T, and its backward
* Born rule   p_k = Tr(M_k rho)                  (Sec. 2.1, Born rule)
* product POVM M_k = M^(1)_{k_1} (x) ... (x) M^(N)_{k_N}   (Sec. 3.3), any
              K-element POVM per qubit, and several such settings summed
              in the loss (Sec. 2.1: one POVM {M^i_k} per measurement i)
* tetrahedral single-qubit POVM M_a = (I + s_a . sigma)/4   (Sec. 4.1 setup)
* loss        L = -sum_k f_k log p_k              (Sec. 2.1 Eq. MLE; Sec. 3.1)
* gradient    dL/dT (PyTorch convention dL/dRe T + i dL/dIm T)
* fidelity    F_q (Sec. 2.3 Eq. F_QF) and F_c (Eq. F_CF)

Everything is numpy float64 / complex128.  Sums that define a scalar result
use ``math.fsum`` (correctly rounded).  Nothing is blocked, fused or
reordered beyond what the definitions state; the only library primitives are
``@`` (matrix product), ``np.kron`` and ``np.tensordot``.

Readings of the paper taken here (each also listed in the design notes):

1. The paper writes rho = T^dagger T / Tr(...).  This oracle maps rho = T T^dagger
   / Tr(T T^dagger); the two are the same map applied to T vs T^dagger, and
   coincide for the Hermitian T of the unified map (Eq. unified_DP).
2. Qubit 1 is the leftmost Kronecker factor, i.e. the most significant bit of
   the row index r and of the column index c of rho; the outcome index is
   k = sum_i k_i 4^(N-i); outcome a of one qubit is s_a in the paper's order.
3. Eq. PS pairs b_i with block B; the Born rule Tr(M rho) = sum_ab M_ab rho_ba
   pairs the (0,1) entry of M with the (1,0) block of rho.  The oracle follows
   the Born rule, not the printed pairing (which computes Tr(M^T rho)).
4. sigma = (X, Y, Z) with Y = [[0, -i], [i, 0]].
5. f is used as given (counts or frequencies); log is natural; terms with
   f_k = 0 contribute 0; a term with f_k > 0 and p_k <= 0 makes L = +inf.

Parity pins: every function here is checked in ``tests/test_oracle_pins.py``
against values that do not come from the oracle itself: brute force,
closed forms worked out by hand, invariants and library routines.  Each
pin is chosen so that a plausible slip (a dropped term or square, a wrong
sign, index or operand order) fails it; F_c, for instance, is fixed by
hand-computed values and by its factorisation over product states.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

# ----------------------------------------------------------------------------
# Single-qubit POVM (Sec. 4.1, experimental setups)
# ----------------------------------------------------------------------------

_T3 = 1.0 / math.sqrt(3.0)

#: Bloch vectors s_0..s_3 of the tetrahedral POVM, in the paper's order.
TETRA_S = np.array(
    [
        [_T3, _T3, _T3],
        [-_T3, -_T3, _T3],
        [-_T3, _T3, -_T3],
        [_T3, -_T3, -_T3],
    ],
    dtype=np.float64,
)

PAULI = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)


def povm_from_bloch(s: np.ndarray) -> np.ndarray:
    """M_a = (I + s_a . sigma)/4 for each row s_a of ``s``; shape (K, 2, 2)."""
    s = np.asarray(s, dtype=np.float64)
    out = np.empty((s.shape[0], 2, 2), dtype=np.complex128)
    for a in range(s.shape[0]):
        m = np.eye(2, dtype=np.complex128)
        for j in range(3):
            m = m + s[a, j] * PAULI[j]
        out[a] = m / 4.0
    return out


def tetrahedral_povm() -> np.ndarray:
    """The paper's single-qubit POVM {M_a}, a = 0..3; shape (4, 2, 2)."""
    return povm_from_bloch(TETRA_S)


# ----------------------------------------------------------------------------
# State map (Sec. 2.2.1 Eq. T_matrix; Sec. 3.2 Eq. unified_DP, Eq. abs_P)
# ----------------------------------------------------------------------------

def trace_tt(T: np.ndarray) -> float:
    """tau = Tr(T T^dagger) = sum_ij |T_ij|^2, correctly rounded."""
    a = np.asarray(T, dtype=np.complex128)
    return math.fsum((a.real.ravel() ** 2).tolist() + (a.imag.ravel() ** 2).tolist())


def state_map(T: np.ndarray) -> tuple[np.ndarray, float]:
    """rho = T T^dagger / tau and tau (Eq. T_matrix with reading 1).

    ``T`` may be d x r (a rank-r factor); rho is d x d.
    """
    a = np.asarray(T, dtype=np.complex128)
    tau = trace_tt(a)
    rho = (a @ a.conj().T) / tau
    return rho, tau


# State-map modes applied to the network output before the state map.
# Chol_Delta (Sec. 2.2.1 Eq. T_matrix): T lower triangular.  Chol_H (Sec. 3.2
# Eq. unified_DP, the paper's default): T Hermitian, made so by the Hermitian
# part (X + X^dagger)/2 (Sec. 2.2.2, the remark on non-Hermitian matrices).
# Both are orthogonal projections for the real inner product Re Tr(A^dagger
# B), hence self-adjoint: the same map sends dL/dT' back to dL/dT.
# ----------------------------------------------------------------------------

def hermitian_part(X: np.ndarray) -> np.ndarray:
    """(X + X^dagger) / 2."""
    a = np.asarray(X, dtype=np.complex128)
    return (a + a.conj().T) / 2.0


def lower_part(X: np.ndarray) -> np.ndarray:
    """Lower triangle of X (row >= column), strict upper part zero."""
    return np.tril(np.asarray(X, dtype=np.complex128))


def premap(X: np.ndarray, mode: str) -> np.ndarray:
    """The pre-map of a state-map mode: 'plain' (identity), 'hermitian'
    (Chol_H) or 'lower' (Chol_Delta)."""
    if mode == "plain":
        return np.asarray(X, dtype=np.complex128)
    if mode == "hermitian":
        return hermitian_part(X)
    if mode == "lower":
        return lower_part(X)
    raise ValueError(mode)


def abs_projection(H: np.ndarray, P: float) -> np.ndarray:
    """P-order absolute projection of a Hermitian H = Q Lambda Q^dagger
    (Sec. 3.2 Eq. abs_P): Q |Lambda|^P Q^dagger / Tr |Lambda|^P."""
    lam, Q = np.linalg.eigh(np.asarray(H, dtype=np.complex128))
    w = np.abs(lam) ** P
    return (Q * (w / math.fsum(w.tolist()))) @ Q.conj().T


def abs_map(T: np.ndarray, P: float):
    """P-order absolute map of Sec. 3.2: for the Hermitian part H = Q Lambda
    Q^dagger of T, A = Q |Lambda|^(P/2) Q^dagger.  A is Hermitian and
    positive semidefinite, so A A^dagger / Tr(A A^dagger) = Q |Lambda|^P
    Q^dagger / Tr |Lambda|^P: the P-order absolute projection (Eq. abs_P)
    computed by the library's state map.  Returns (A, Q, lam)."""
    lam, Q = np.linalg.eigh(hermitian_part(T))
    return (Q * np.abs(lam) ** (P / 2.0)) @ Q.conj().T, Q, lam


def abs_divided_differences(lam: np.ndarray, P: float) -> np.ndarray:
    """Gamma_ij = (g(l_i) - g(l_j)) / (l_i - l_j) for g(l) = |l|^(P/2), and
    g'(l_i) = (P/2) sign(l_i) |l_i|^(P/2 - 1) where l_i = l_j (0 at l = 0,
    the one-sided derivatives there being infinite or of opposite signs)."""
    lam = np.asarray(lam, dtype=np.float64)
    a = P / 2.0
    g = np.abs(lam) ** a
    with np.errstate(divide="ignore", invalid="ignore"):
        dg = np.where(lam == 0.0, 0.0, a * np.sign(lam) * np.abs(lam) ** (a - 1.0))
        num = g[:, None] - g[None, :]
        den = lam[:, None] - lam[None, :]
        gam = np.where(den == 0.0, 0.0, num / np.where(den == 0.0, 1.0, den))
    ties = den == 0.0
    gam[ties] = np.broadcast_to(dg[:, None], gam.shape)[ties]
    return gam


def abs_map_backward(Q: np.ndarray, lam: np.ndarray, P: float, GA: np.ndarray) -> np.ndarray:
    """dL/dT from dL/dA (both dL/dRe + i dL/dIm) through A = g(H), H the
    Hermitian part of T: the first-order change of a spectral function of a
    Hermitian matrix is Q (Gamma o (Q^dagger dH Q)) Q^dagger (Gamma the
    divided differences of g on the eigenvalues), which is self-adjoint, as
    is the Hermitian part; so dL/dT = Q (Gamma o (Q^dagger S Q)) Q^dagger
    with S = (GA + GA^dagger) / 2."""
    Q = np.asarray(Q, dtype=np.complex128)
    S = hermitian_part(GA)
    M = Q.conj().T @ S @ Q
    return Q @ (abs_divided_differences(lam, P) * M) @ Q.conj().T


def grad_T_abs(T: np.ndarray, f: np.ndarray, P: float, povm: np.ndarray | None = None):
    """Gradient of L(rho) with rho the P-order absolute projection of T:
    dL/dA at A = abs_map(T, P), then abs_map_backward.  Returns (grad, L)."""
    A, Q, lam = abs_map(T, P)
    gA, L = grad_T(A, f, povm)
    return abs_map_backward(Q, lam, P, gA), L


# ----------------------------------------------------------------------------
# The mapping network (Sec. 3.1): a 3-layer FNN from the measured
# distribution x (K^N = 4^N inputs) through 2N hidden units with a leaky
# ReLU to 4^N real outputs, which fill the Hermitian T of Chol_H.
# Readings: negative slope 0.01; outputs y as a real d x d matrix Y (row
# major) fill T with T_ij = Y_ij + i Y_ji below the diagonal, its conjugate
# above, T_ii = Y_ii (a bijection of R^(d^2) onto Hermitian matrices).
# ----------------------------------------------------------------------------

LEAKY_SLOPE = 0.01


def leaky_relu(v: np.ndarray) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    return np.where(v > 0, v, LEAKY_SLOPE * v)


def fnn_fill(y: np.ndarray, d: int) -> np.ndarray:
    """Hermitian T from the 4^N outputs (reading above)."""
    Y = np.asarray(y, dtype=np.float64).reshape(d, d)
    L = np.tril(Y, -1)
    U = np.triu(Y, 1)
    return (L + L.T) + 1j * (U.T - U) + np.diag(np.diag(Y))


def fnn_unfill(G: np.ndarray) -> np.ndarray:
    """Adjoint of fnn_fill for Re Tr(A^dagger B): dL/dy from dL/dT
    (PyTorch convention dL/dRe T + i dL/dIm T), as a flat 4^N vector."""
    G = np.asarray(G, dtype=np.complex128)
    S = G.real + G.real.T
    A = G.imag.T - G.imag
    return (np.tril(S, -1) + np.triu(A, 1) + np.diag(np.diag(G.real))).ravel()


def fnn_forward(W1, b1, W2, b2, x):
    """h_pre = W1 x + b1, h = leaky(h_pre), y = W2 h + b2, T = fill(y).
    W1 is 2N x 4^N, W2 is 4^N x 2N.  Returns (T, h_pre, y)."""
    h_pre = np.asarray(W1, dtype=np.float64) @ np.asarray(x, dtype=np.float64) + np.asarray(b1, dtype=np.float64)
    y = np.asarray(W2, dtype=np.float64) @ leaky_relu(h_pre) + np.asarray(b2, dtype=np.float64)
    d = int(round(math.sqrt(y.size)))
    return fnn_fill(y, d), h_pre, y


def fnn_backward(W2, x, h_pre, G):
    """Gradients of L(T(W1, b1, W2, b2)) from G = dL/dT: returns
    (dW1, db1, dW2, db2)."""
    gy = fnn_unfill(G)
    h = leaky_relu(h_pre)
    dh = np.asarray(W2, dtype=np.float64).T @ gy
    dh_pre = dh * np.where(np.asarray(h_pre) > 0, 1.0, LEAKY_SLOPE)
    return np.outer(dh_pre, np.asarray(x, dtype=np.float64)), dh_pre, np.outer(gy, h), gy


def rprop_step(w, g, prev, step, etas=(0.5, 1.2), step_sizes=(1e-6, 50.0)):
    """One Rprop step, the optimiser of the paper's setup (Sec. 4.1), in the
    iRprop- form: where g and the previous gradient agree in sign the step
    grows by eta+, where they disagree it shrinks by eta- and that entry is
    not moved (its stored gradient becomes 0); steps are kept within
    step_sizes; w moves by -sign(g) step.  Returns (w, prev, step)."""
    w, g = np.asarray(w, dtype=np.float64), np.asarray(g, dtype=np.float64)
    prev, step = np.asarray(prev, dtype=np.float64), np.asarray(step, dtype=np.float64)
    s = np.sign(g) * np.sign(prev)
    factor = np.where(s > 0, etas[1], np.where(s < 0, etas[0], 1.0))
    step = np.clip(step * factor, step_sizes[0], step_sizes[1])
    g = np.where(s < 0, 0.0, g)
    return w - np.sign(g) * step, g, step


# ----------------------------------------------------------------------------
# Product-structured POVM probabilities (Sec. 2.1 Born rule; Sec. 3.3)
# ----------------------------------------------------------------------------

def n_qubits_of(dim: int) -> int:
    n = dim.bit_length() - 1
    if dim != 1 << n or n < 1:
        raise ValueError(f"dimension {dim} is not 2^N with N >= 1")
    return n


def per_qubit(povm, n: int) -> list:
    """The single-qubit POVM of each qubit 1..N as a list of (K, 2, 2) arrays.

    ``povm`` is None (the tetrahedral POVM on every qubit), one (K, 2, 2)
    POVM shared by every qubit, or (N, K, 2, 2): qubit i measured with its
    own K-element POVM M^(i) (Sec. 3.3 with a POVM per qubit; K is the same
    on every qubit, so there are K^N outcomes)."""
    if povm is None:
        return [tetrahedral_povm()] * n
    a = np.asarray(povm, dtype=np.complex128)
    if a.ndim == 3:
        return [a] * n
    if a.ndim != 4 or a.shape[0] != n:
        raise ValueError("povm must be (K, 2, 2) or (N, K, 2, 2)")
    return [a[i] for i in range(n)]


def product_element(povm, ks) -> np.ndarray:
    """M_k = M^(1)_{k_1} (x) ... (x) M^(N)_{k_N}, qubit 1 leftmost (Sec. 3.3);
    ``povm`` as in :func:`per_qubit`."""
    mats = per_qubit(povm, len(ks))
    m = np.ones((1, 1), dtype=np.complex128)
    for i, a in enumerate(ks):
        m = np.kron(m, mats[i][a])
    return m


def outcome_tuples(n: int, K: int = 4):
    """All k = (k_1..k_N) in the order k = sum_i k_i K^(N-i)."""
    return itertools.product(range(K), repeat=n)


def probs_kron(rho: np.ndarray, povm: np.ndarray | None = None) -> np.ndarray:
    """Brute force: p_k = Tr(M_k rho) with explicit Kronecker products.

    Exponential cost; intended for N <= 5.  Returns the real part; the
    imaginary part (zero for Hermitian rho) is checked by the tests.
    """
    n = n_qubits_of(rho.shape[0])
    mats = per_qubit(povm, n)
    K = mats[0].shape[0]
    out = np.empty(K ** n, dtype=np.complex128)
    for idx, ks in enumerate(outcome_tuples(n, K)):
        out[idx] = np.trace(product_element(np.array(mats), ks) @ rho)
    return out


def _pair_tensor(mat: np.ndarray) -> np.ndarray:
    """View a d x d matrix as a tensor over per-qubit pair indices
    m_i = 2 r_i + c_i, axes ordered qubit 1..N."""
    n = n_qubits_of(mat.shape[0])
    t = mat.reshape((2,) * (2 * n))  # (r_1..r_N, c_1..c_N)
    order = [ax for i in range(n) for ax in (i, n + i)]  # (r_1, c_1, r_2, c_2, ...)
    return t.transpose(order).reshape((4,) * n)


def _from_pair_tensor(t: np.ndarray) -> np.ndarray:
    n = t.ndim
    d = 1 << n
    x = t.reshape((2,) * (2 * n))  # (r_1, c_1, r_2, c_2, ...)
    order = [2 * i for i in range(n)] + [2 * i + 1 for i in range(n)]
    return x.transpose(order).reshape(d, d)


def probs(rho: np.ndarray, povm: np.ndarray | None = None) -> np.ndarray:
    """p_k = Tr(M_k rho) via the product structure (Sec. 3.3): one 4 x 4
    contraction per qubit over its pair index m_i = 2 r_i + c_i, with
    W[a, 2r + c] = (M_a)_{c, r} so that sum_m W[a, m] rho_m = Tr(M_a rho)
    for one qubit (Born rule).  Complex result (imaginary part ~ 0)."""
    x = _pair_tensor(np.asarray(rho, dtype=np.complex128))
    n = x.ndim
    mats = per_qubit(povm, n)
    K = mats[0].shape[0]
    for i in range(n):
        W = np.transpose(mats[i], (0, 2, 1)).reshape(K, 4)  # W[a, 2r+c] = M^(i)_a[c, r]
        x = np.tensordot(W, x, axes=([1], [i]))  # new axis first
        x = np.moveaxis(x, 0, i)
    return x.reshape(K ** n)


def probs_real(rho: np.ndarray, povm: np.ndarray | None = None, check: bool = True) -> np.ndarray:
    """Real probabilities; asserts the imaginary part is at rounding level."""
    pc = probs(rho, povm)
    if check:
        scale = max(float(np.max(np.abs(pc.real))), 1e-300)
        if float(np.max(np.abs(pc.imag))) > 1e-12 * scale:
            raise AssertionError("probabilities have a non-negligible imaginary part; rho not Hermitian")
    return pc.real.copy()


def outcome_digits(k: int, n: int, K: int = 4) -> tuple:
    """(k_1..k_N) of the flat outcome index k = sum_i k_i K^(N-i)."""
    out = []
    for _ in range(n):
        out.append(k % K)
        k //= K
    return tuple(reversed(out))


def probs_at(W: np.ndarray, outcomes, povm: np.ndarray | None = None) -> np.ndarray:
    """p_k = Tr(M_k rho) for the listed outcomes only (each a tuple k_1..k_N),
    rho = W W^dagger / Tr(W W^dagger) with W a d x r factor (Born rule,
    Sec. 2.1; product POVM, Sec. 3.3).  Uses Tr(M_k W W^dagger) =
    Tr(W^dagger M_k W): M_k = M_{k_1} (x) ... (x) M_{k_N} is applied to the
    row index of W one qubit at a time (qubit 1 = the most significant row
    bit), O(N d r) work per outcome, so single outcomes of the largest states
    can be evaluated without forming rho or the full map."""
    povm = tetrahedral_povm() if povm is None else np.asarray(povm, dtype=np.complex128)
    a = np.asarray(W, dtype=np.complex128)
    if a.ndim == 1:
        a = a[:, None]
    d, r = a.shape
    n = n_qubits_of(d)
    tau = trace_tt(a)
    base = a.reshape((2,) * n + (r,))
    out = []
    for ks in outcomes:
        if len(ks) != n:
            raise ValueError("outcome tuple length differs from the qubit count")
        x = base
        for i, kq in enumerate(ks):
            x = np.moveaxis(np.tensordot(povm[kq], x, axes=([1], [i])), 0, i)
        out.append(np.vdot(base, x).real)  # sum conj(W) * (M_k W)
    return np.asarray(out, dtype=np.float64) / tau


# ----------------------------------------------------------------------------
# Adjoint of the POVM map: G = sum_k g_k M_k
# ----------------------------------------------------------------------------

def adjoint_kron(g: np.ndarray, n: int, povm: np.ndarray | None = None) -> np.ndarray:
    """Brute force G = sum_k g_k M_k (N <= 5)."""
    mats = np.array(per_qubit(povm, n))
    d = 1 << n
    G = np.zeros((d, d), dtype=np.complex128)
    for idx, ks in enumerate(outcome_tuples(n, mats.shape[1])):
        G += g[idx] * product_element(mats, ks)
    return G


def adjoint(g: np.ndarray, n: int, povm: np.ndarray | None = None) -> np.ndarray:
    """G = sum_k g_k M_k via per-qubit contractions: G[r, c] =
    sum_k g_k prod_i (M^(i)_{k_i})_{r_i, c_i}, i.e. V[2r + c, a] =
    (M^(i)_a)_{r, c} applied along each qubit axis i (``povm`` as in
    :func:`per_qubit`)."""
    mats = per_qubit(povm, n)
    K = mats[0].shape[0]
    x = np.asarray(g, dtype=np.complex128).reshape((K,) * n)
    for i in range(n):
        V = mats[i].reshape(K, 4).T  # V[2r+c, a] = M^(i)_a[r, c]
        x = np.tensordot(V, x, axes=([1], [i]))
        x = np.moveaxis(x, 0, i)
    return _from_pair_tensor(x)


# ----------------------------------------------------------------------------
# Negative log-likelihood (Sec. 2.1 Eq. MLE; Sec. 3.1 loss)
# ----------------------------------------------------------------------------

def nll(p: np.ndarray, f: np.ndarray) -> float:
    """L = -sum_{k: f_k > 0} f_k ln p_k; +inf if some f_k > 0 has p_k <= 0."""
    p = np.asarray(p, dtype=np.float64).ravel()
    f = np.asarray(f, dtype=np.float64).ravel()
    terms = []
    for fk, pk in zip(f.tolist(), p.tolist()):
        if fk == 0.0:
            continue
        if pk <= 0.0:
            return math.inf
        terms.append(-fk * math.log(pk))
    return math.fsum(terms)


def nll_vec(p: np.ndarray, f: np.ndarray) -> float:
    """Same value as :func:`nll` for large vectors (vectorised log, fsum)."""
    p = np.asarray(p, dtype=np.float64).ravel()
    f = np.asarray(f, dtype=np.float64).ravel()
    m = f != 0.0
    if np.any(p[m] <= 0.0):
        return math.inf
    return math.fsum((-f[m] * np.log(p[m])).tolist())


def likelihood(T: np.ndarray, f: np.ndarray, povm: np.ndarray | None = None):
    """Forward chain T -> (rho, tau) -> p -> L.  Returns (L, p, rho, tau)."""
    rho, tau = state_map(T)
    n = n_qubits_of(rho.shape[0])
    p = probs_real(rho, povm) if n > 5 else probs_kron(rho, povm).real.copy()
    return nll_vec(p, f), p, rho, tau


# ----------------------------------------------------------------------------
# Gradient of L with respect to T
# ----------------------------------------------------------------------------

def cotangent(p: np.ndarray, f: np.ndarray) -> np.ndarray:
    """g'_k = F - f_k / p_k with F = sum_k f_k (g'_k = F where f_k = 0).

    From dL = (1/tau) Tr(G' dS), S = T T^dagger, with G' = sum_k g'_k M_k:
    the -f_k/p_k part is dL/dp_k, and F I = sum_k F M_k is the derivative of
    the trace normalisation (sum_k M_k = I, Eq. MLE constraint)."""
    p = np.asarray(p, dtype=np.float64).ravel()
    f = np.asarray(f, dtype=np.float64).ravel()
    F = math.fsum(f.tolist())
    g = np.full(p.shape, F)
    m = f != 0.0
    g[m] = F - f[m] / p[m]
    return g


def grad_T(T: np.ndarray, f: np.ndarray, povm: np.ndarray | None = None):
    """dL/dRe T + i dL/dIm T = (2/tau) G' T.  Returns (grad, L)."""
    L, p, rho, tau = likelihood(T, f, povm)
    n = n_qubits_of(rho.shape[0])
    g = cotangent(p, f)
    G = adjoint(g, n, povm) if n > 5 else adjoint_kron(g, n, povm)
    return (2.0 / tau) * (G @ np.asarray(T, dtype=np.complex128)), L


def loss_of_T(T: np.ndarray, f: np.ndarray, povm: np.ndarray | None = None) -> float:
    return likelihood(T, f, povm)[0]


def grad_T_mode(T: np.ndarray, f: np.ndarray, mode: str, povm: np.ndarray | None = None):
    """Gradient through a state-map mode: L(premap(T)); the pre-map is
    self-adjoint, so dL/dT = premap(dL/dT' at T' = premap(T)).
    Returns (grad, L)."""
    g, L = grad_T(premap(T, mode), f, povm)
    return premap(g, mode), L


def likelihood_settings(T: np.ndarray, fs, settings):
    """Several measurement settings (Sec. 2.1: each measurement i is a POVM
    {M^i_k} with its own frequencies): setting s is a product POVM (one
    K-element POVM per qubit, ``settings[s]`` as in :func:`per_qubit`) with
    frequencies fs[s] over its K^N outcomes, and the loss is the sum of the
    settings' negative log-likelihoods, L = -sum_s sum_k f^s_k ln p^s_k.
    Returns (L, [p_s], rho, tau)."""
    rho, tau = state_map(T)
    n = n_qubits_of(rho.shape[0])
    ps, Ls = [], []
    for f, povm in zip(fs, settings):
        p = probs_real(rho, povm) if n > 4 else probs_kron(rho, povm).real.copy()
        ps.append(p)
        Ls.append(nll_vec(p, f))
    return math.fsum(Ls), ps, rho, tau


def grad_T_settings(T: np.ndarray, fs, settings):
    """dL/dRe T + i dL/dIm T of :func:`likelihood_settings`: (2/tau) G' T with
    G' = sum_s sum_k (F_s - f^s_k / p^s_k) M^s_k, F_s = sum_k f^s_k.  Each
    setting's POVM sums to I, so the trace normalisation contributes
    (sum_s F_s) I = sum_s sum_k F_s M^s_k.  Returns (grad, L)."""
    L, ps, rho, tau = likelihood_settings(T, fs, settings)
    n = n_qubits_of(rho.shape[0])
    G = np.zeros_like(rho)
    for f, p, povm in zip(fs, ps, settings):
        g = cotangent(p, f)
        G += adjoint(g, n, povm) if n > 4 else adjoint_kron(g, n, povm)
    return (2.0 / tau) * (G @ np.asarray(T, dtype=np.complex128)), L


# ----------------------------------------------------------------------------
# Fidelities (Sec. 2.3)
# ----------------------------------------------------------------------------

def _psd_sqrt(a: np.ndarray) -> np.ndarray:
    w, v = np.linalg.eigh((a + a.conj().T) / 2.0)
    w = np.clip(w, 0.0, None)
    return (v * np.sqrt(w)) @ v.conj().T


def fidelity_q(rho_hat: np.ndarray, rho: np.ndarray) -> float:
    """F_q = (Tr sqrt(sqrt(rho_hat) rho sqrt(rho_hat)))^2 (Eq. F_QF)."""
    s = _psd_sqrt(rho_hat)
    m = s @ rho @ s
    w = np.clip(np.linalg.eigvalsh((m + m.conj().T) / 2.0), 0.0, None)
    return float(math.fsum(np.sqrt(w).tolist()) ** 2)


def fidelity_q_lowrank(rho_hat: np.ndarray, W: np.ndarray) -> float:
    """F_q(rho_hat, rho) for a target rho = W W^dagger / Tr(W W^dagger) of low
    rank r: sqrt(rho_hat) rho sqrt(rho_hat) and W^dagger rho_hat W / Tr share
    their nonzero eigenvalues, so F_q = (sum sqrt(eig(W^dagger rho_hat W)/Tr))^2
    needs only an r x r eigensolve."""
    W = np.asarray(W, dtype=np.complex128)
    tw = trace_tt(W)
    m = W.conj().T @ rho_hat @ W / tw
    w = np.clip(np.linalg.eigvalsh((m + m.conj().T) / 2.0), 0.0, None)
    return float(math.fsum(np.sqrt(w).tolist()) ** 2)


def fidelity_c(p_hat: np.ndarray, p: np.ndarray) -> float:
    """F_c = (sum_k sqrt(p_hat_k p_k))^2 (Eq. F_CF)."""
    a = np.clip(np.asarray(p_hat, dtype=np.float64), 0.0, None)
    b = np.clip(np.asarray(p, dtype=np.float64), 0.0, None)
    return math.fsum(np.sqrt(a * b).tolist()) ** 2


# ----------------------------------------------------------------------------
# Reference optimiser loop (training-shape workload): Adam on T directly
# ----------------------------------------------------------------------------

def adam_train(T0: np.ndarray, f: np.ndarray, steps: int, lr: float, betas=(0.9, 0.999),
               eps: float = 1e-12, povm: np.ndarray | None = None):
    """Plain Adam on the complex parameter T (real and imaginary parts as two
    real parameters, the torch convention), minimising L(T).  Returns
    (T_final, losses)."""
    b1, b2 = betas
    T = np.asarray(T0, dtype=np.complex128).copy()
    m = np.zeros_like(T)
    v = np.zeros(T.shape, dtype=np.float64)
    vi = np.zeros(T.shape, dtype=np.float64)
    losses = []
    for t in range(1, steps + 1):
        g, L = grad_T(T, f, povm)
        losses.append(L)
        m = b1 * m + (1 - b1) * g
        v = b2 * v + (1 - b2) * g.real ** 2
        vi = b2 * vi + (1 - b2) * g.imag ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        vih = vi / (1 - b2 ** t)
        T = T - lr * (mh.real / (np.sqrt(vh) + eps) + 1j * mh.imag / (np.sqrt(vih) + eps))
    return T, losses
