"""General product POVMs through the C ABI (qst_povm_probs_general,
qst_likelihood_general + qst_grad_product): K outcomes per qubit, a
random K-element POVM of its own on every qubit, several settings summed
in the loss (Sec. 3.3; Sec. 2.1), against the oracle's probs /
grad_T_settings (pinned by brute-force Kronecker products and the
product-state, Pauli-6, trine and basis closed forms).

Tolerances (relative): FP64 1e-12, FP32 1e-5, BF16 2e-3 (BF16: the T T^dagger
product on bf16 operands, everything after it in FP32).
  p: max|dp| / max p;  L: |dL| / |L|;  G' and grad: ||d||_F / ||.||_F
"""
import math

import numpy as np
import pytest

import oracle as O
import synth as S
from workloads import rel_fro, rel_max

torch = pytest.importorskip("torch")
qst = pytest.importorskip("paper_2207_05341_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-3, "f32x6": 1e-5}


def say(*a):
    print(*a, flush=True)


def ctype(prec):
    return np.complex128 if prec == "f64" else np.complex64


def rtype(prec):
    return np.float64 if prec == "f64" else np.float32


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,K", [(1, 2), (2, 3), (3, 6), (5, 2), (6, 3), (7, 6), (8, 3), (10, 2), (10, 3)])
def test_povm_probs_general_against_oracle(n, K, prec):
    """K^N probabilities of a distinct random POVM per qubit from a random
    state (1..3 POVM passes for the Pauli coordinates, N real passes);
    padded leading dimension of rho; only its lower triangle is read."""
    say(f"general POVM probs N={n} K={K} {prec}")
    g = S.rng(9500 + 16 * n + K)
    d = 1 << n
    rho, _ = O.state_map(S.ginibre(g, d))
    povms = np.array([S.random_povm(g, K) for _ in range(n)])
    r = rho.astype(ctype(prec))
    buf = np.zeros((d, d + 3), dtype=ctype(prec))
    buf[:, :d] = np.tril(r) + np.triu(np.full((d, d), 7.0 + 5.0j), 1)  # junk above the diagonal
    rg = dev(buf)[:, :d]
    p = qst.povm_probs_general(rg, povms, prec)
    p2 = qst.povm_probs_general(rg, povms, prec)
    torch.cuda.synchronize()
    want = O.probs_real(r.astype(np.complex128), povms)
    e = rel_max(p.cpu().numpy(), want)
    say(f"  max|dp|/max p = {e:.2e}")
    assert e <= TOL[prec]
    assert torch.equal(p, p2)
    assert abs(float(p.double().sum()) - 1.0) <= (1e-12 if prec == "f64" else 1e-5)


def run_general(T, fs, settings, prec, upstream=None):
    Tg = dev(T.astype(ctype(prec)))
    f = dev(np.stack(fs).astype(rtype(prec)))
    out, tau, G, bad = qst.likelihood_forward_general(Tg, f, np.stack(settings), prec)
    up = None if upstream is None else torch.tensor([upstream], dtype=torch.float64, device=DEV)
    grad = qst.grad_product(G, Tg, tau, prec, up)
    torch.cuda.synchronize()
    return float(out[0].item()), float(out[1].item()), G.cpu().numpy(), grad.cpu().numpy(), bad.cpu().numpy()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f32x6"])
@pytest.mark.parametrize("n,K,nset", [(1, 2, 1), (3, 3, 3), (4, 6, 2), (6, 2, 3), (7, 3, 3), (9, 2, 3), (10, 3, 2)])
def test_likelihood_general_against_oracle(n, K, nset, prec):
    """L summed over settings, G' and dL/dT against the oracle's
    grad_T_settings; frequencies from multinomial sampling of a depolarised
    random pure state under each setting."""
    say(f"general likelihood N={n} K={K} settings={nset} {prec}")
    g = S.rng(9600 + 16 * n + K)
    d = 1 << n
    T = S.ginibre(g, d)
    settings = [np.array([S.random_povm(g, K) for _ in range(n)]) for _ in range(nset)]
    target = S.depolarised_pure(S.haar_vector(g, d), 0.1)
    fs = [S.multinomial_freqs(g, 20 * K ** n, O.probs_real(target, pv)) for pv in settings]
    L, F, G, grad, bad = run_general(T, fs, settings, prec)
    Tq = T.astype(ctype(prec)).astype(np.complex128)
    fq = [f.astype(rtype(prec)).astype(np.float64) for f in fs]
    wgrad, wL = O.grad_T_settings(Tq, fq, settings)
    _, ps, _, _ = O.likelihood_settings(Tq, fq, settings)
    wG = sum(O.adjoint(O.cotangent(p, f), n, pv) for p, f, pv in zip(ps, fq, settings))
    errs = {"L": abs(L - wL) / abs(wL), "G": rel_fro(G, wG), "grad": rel_fro(grad, wgrad)}
    say(f"  errors {errs}")
    for k, v in errs.items():
        assert v <= TOL[prec], (k, v)
    assert abs(F - math.fsum(np.concatenate(fq).tolist())) <= 1e-12 * F
    assert bad.tolist() == [0, 0]


def test_general_k4_tetrahedral_equals_fast_path():
    """The tetrahedral POVM on every qubit through the general route (Pauli
    coordinates and real factors) against the specialised fused call: L
    and G' to rounding, FP64, N = 8."""
    g = S.rng(9700)
    n, d = 8, 256
    T = S.ginibre(g, d)
    f = S.multinomial_freqs(g, 10 ** 6, O.probs_real(S.depolarised_pure(S.haar_vector(g, d), 0.1)))
    tet = np.array([O.tetrahedral_povm()] * n)
    L, _, G, _, _ = run_general(T, [f], [tet], "f64")
    out, tau, G0, _ = qst.likelihood_forward(dev(T), dev(f), "f64")
    torch.cuda.synchronize()
    assert abs(L - float(out[0].item())) <= 1e-13 * abs(L)
    assert rel_fro(G, G0.cpu().numpy()) <= 1e-13


def test_general_autograd_and_zero_frequencies():
    """likelihood_general through autograd (upstream scale 2.5) against the
    oracle, with zero frequencies (the f_k = 0 branch of the cotangent)."""
    g = S.rng(9800)
    n, K, d = 5, 3, 32
    T = S.ginibre(g, d)
    settings = [np.array([S.random_povm(g, K) for _ in range(n)]) for _ in range(2)]
    fs = [S.multinomial_freqs(g, 200, O.probs_real(S.depolarised_pure(S.haar_vector(g, d), 0.0), pv))
          for pv in settings]
    assert min(float(np.mean(f == 0)) for f in fs) > 0.2
    Tg = dev(T).requires_grad_(True)
    L = qst.likelihood_general(Tg, dev(np.stack(fs)), np.stack(settings))
    (2.5 * L).backward()
    wgrad, wL = O.grad_T_settings(T, fs, settings)
    assert abs(float(L.item()) - wL) <= 1e-12 * abs(wL)
    assert rel_fro(Tg.grad.cpu().numpy(), 2.5 * wgrad) <= 1e-12


def test_general_value_only_and_bad_entries():
    """G = NULL (value alone) gives the same L; f > 0 where a POVM element
    has p = 0 (a projective K = 2 basis on a basis state) makes L = +inf and
    is counted."""
    n, d = 3, 8
    basis = np.array([np.diag([1.0, 0.0]), np.diag([0.0, 1.0])]).astype(complex)
    T = np.zeros((d, d), dtype=complex)
    T[0, 0] = 1.0  # rho = |000><000|: p = e_0
    f = np.zeros(2 ** n)
    f[0], f[5] = 0.5, 0.5
    out, _, G, bad = qst.likelihood_forward_general(dev(T), dev(f), np.array([basis] * n), "f64",
                                                    with_grad_matrix=False)
    torch.cuda.synchronize()
    assert G is None
    assert math.isinf(float(out[0].item())) and bad.cpu().tolist() == [1, 0]
