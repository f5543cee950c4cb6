"""Seeded synthetic inputs for the tomography likelihood path.

This module is the only code shared by the FP64 oracle side (tests) and the
GPU side (tests, bench).  It draws random numbers and builds target states;
it holds none of the likelihood arithmetic itself (no state map T -> rho, no
POVM probabilities, no log-likelihood, no gradient).  Where an input needs a
target's exact outcome probabilities (multinomial sampling), the caller passes
them in.

The paper's workloads are synthetic target states (Sec. 4, target-state list:
white-noise / depolarised pure states, product / GHZi / W states, random mixed
states) measured with the per-qubit tetrahedral POVM and sampled by a
multinomial distribution (Sec. 4.4.1).  These generators stand in for them.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    """The one RNG used everywhere: numpy PCG64 seeded with ``seed``."""
    return np.random.default_rng(seed)


def ginibre(g: np.random.Generator, rows: int, cols: int | None = None) -> np.ndarray:
    """Complex Ginibre matrix, iid N(0,1) real and imaginary parts.

    The real part is drawn first (row-major), then the imaginary part.
    Returned as complex128; callers cast to complex64 for the FP32 paths.
    """
    cols = rows if cols is None else cols
    re = g.standard_normal((rows, cols))
    im = g.standard_normal((rows, cols))
    return re + 1j * im


def haar_vector(g: np.random.Generator, d: int) -> np.ndarray:
    """Haar-random pure state: a normalised complex Gaussian vector."""
    v = g.standard_normal(d) + 1j * g.standard_normal(d)
    return v / np.linalg.norm(v)


def depolarised_pure(psi: np.ndarray, q: float) -> np.ndarray:
    """Target (1-q)|psi><psi| + q I/d (Sec. 4: white-noise and depolarising
    channel targets; q plays the role of 1-p there, lambda in the channel)."""
    d = psi.shape[0]
    return (1.0 - q) * np.outer(psi, psi.conj()) + (q / d) * np.eye(d, dtype=np.complex128)


def product_plus(n: int) -> np.ndarray:
    """|+>^{(x)N} (Sec. 4, product target)."""
    d = 1 << n
    return np.full(d, 1.0 / np.sqrt(d), dtype=np.complex128)


def ghzi(n: int) -> np.ndarray:
    """(|0...0> + i|1...1>)/sqrt(2) (Sec. 4, GHZi target)."""
    d = 1 << n
    v = np.zeros(d, dtype=np.complex128)
    v[0] = 1.0 / np.sqrt(2.0)
    v[d - 1] = 1j / np.sqrt(2.0)
    return v


def w_state(n: int) -> np.ndarray:
    """Equal superposition of the N one-excitation basis states (Sec. 4, W)."""
    d = 1 << n
    v = np.zeros(d, dtype=np.complex128)
    for i in range(n):
        v[1 << i] = 1.0 / np.sqrt(n)
    return v


def multinomial_freqs(g: np.random.Generator, shots: int, p0: np.ndarray) -> np.ndarray:
    """Frequencies counts/shots from ``shots`` multinomial draws of ``p0``
    (Sec. 4.4.1).  ``p0`` is clipped at 0 and renormalised first so that
    rounding noise in a computed distribution cannot make numpy reject it."""
    p = np.clip(np.asarray(p0, dtype=np.float64), 0.0, None)
    p = p / p.sum()
    counts = g.multinomial(shots, p)
    return counts.astype(np.float64) / float(shots)


def porter_thomas_probs(g: np.random.Generator, n_outcomes: int, q: float) -> np.ndarray:
    """Stand-in outcome distribution with the statistics of a depolarised
    random pure state: exponentially distributed weights (Porter-Thomas),
    mixed with the uniform distribution at weight q.  Used where a workload
    needs realistic frequencies but not the exact law of a named target."""
    w = g.exponential(size=n_outcomes)
    return (1.0 - q) * (w / w.sum()) + q / n_outcomes


def thin_factor_square(g: np.random.Generator, d: int, r: int) -> tuple[np.ndarray, np.ndarray]:
    """(T, W): W a d x r Ginibre factor and T = W Q^dagger, d x d, with Q a
    d x r matrix of orthonormal columns (QR of a Ginibre matrix), so that
    T T^dagger = W W^dagger exactly in exact arithmetic.  Every entry of T is
    generic (no zero rows or columns), while single outcome probabilities of
    T T^dagger / Tr can be evaluated from the thin W."""
    W = ginibre(g, d, r)
    Q, _ = np.linalg.qr(ginibre(g, d, r))
    return W @ Q.conj().T, W


def unit_directions(g: np.random.Generator, d: int, count: int) -> list[np.ndarray]:
    """``count`` complex Ginibre d x d directions with unit Frobenius norm."""
    out = []
    for _ in range(count):
        e = ginibre(g, d)
        out.append(e / np.linalg.norm(e))
    return out


def batch_qubit_counts(g: np.random.Generator, count: int, lo: int = 3, hi: int = 8) -> np.ndarray:
    """Qubit counts drawn uniformly from {lo, ..., hi} for batched instances."""
    return g.integers(lo, hi + 1, size=count)


def random_povm(g: np.random.Generator, K: int) -> np.ndarray:
    """A random K-element single-qubit POVM, shape (K, 2, 2): A_k = B_k B_k^dagger
    (B_k complex Gaussian 2 x 2), made to sum to I as S^(-1/2) A_k S^(-1/2)
    with S = sum_k A_k.  Every element is full rank."""
    A = []
    for _ in range(K):
        B = g.standard_normal((2, 2)) + 1j * g.standard_normal((2, 2))
        A.append(B @ B.conj().T)
    w, v = np.linalg.eigh(sum(A))
    s = (v / np.sqrt(w)) @ v.conj().T
    return np.array([s @ a @ s for a in A])
