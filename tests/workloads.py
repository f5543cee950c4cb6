"""Seeded inputs of the paper-shaped workloads, with exact target
probabilities from the FP64 oracle (test-side only).

Recipes (numpy PCG64 streams; the Ginibre real part is drawn before the
imaginary part):
  N=4 FP64 (seed 1): T 16x16 Ginibre; target (1-q)|psi><psi| + q I/16,
      psi Haar, q ~ U(0,1); 10^4 shots.
  N=8 FP32 (seeds 2..5 for r = 1, 4, 16, 256): T 256x256 Ginibre; target a
      rank-r Ginibre state W W^dagger / Tr (W 256 x r); 10^6 shots.
  N=11 (seeds 6, 7, 8 for q = 0, 0.05, 0.1): T 2048x2048 Ginibre; target a
      depolarised Haar pure state; 10^7 shots.
These stand in for the paper's synthetic targets (Sec. 4 target list) and
its multinomial sampling (Sec. 4.4.1); the paper uses no public dataset.
"""
from __future__ import annotations

import numpy as np

import oracle as O
import synth as S


def depolarised_case(n: int, seed: int, q: float | None, shots: int):
    g = S.rng(seed)
    d = 1 << n
    T = S.ginibre(g, d)
    psi = S.haar_vector(g, d)
    if q is None:
        q = float(g.uniform())
    rho0 = S.depolarised_pure(psi, q)
    f = S.multinomial_freqs(g, shots, O.probs_real(rho0))
    return T, f, rho0


def rank_r_case(n: int, seed: int, r: int, shots: int):
    g = S.rng(seed)
    d = 1 << n
    T = S.ginibre(g, d)
    W = S.ginibre(g, d, r)
    rho0, _ = O.state_map(W)
    f = S.multinomial_freqs(g, shots, O.probs_real(rho0))
    return T, f, W


def config1():
    return depolarised_case(4, 1, None, 10_000)


def config2(r: int):
    seed = {1: 2, 4: 3, 16: 4, 256: 5}[r]
    return rank_r_case(8, seed, r, 1_000_000)


def config3(q: float):
    seed = {0.0: 6, 0.05: 7, 0.1: 8}[q]
    return depolarised_case(11, seed, q, 10_000_000)


def rel_max(a, b) -> float:
    """max|a - b| / max|b|."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def rel_fro(a, b) -> float:
    """||a - b||_F / ||b||_F."""
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))
