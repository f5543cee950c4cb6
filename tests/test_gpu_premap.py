"""State-map modes through the C ABI (qst_state_premap) and through the
differentiable likelihood: Chol_H, the Hermitian part (X + X^dagger)/2
(Sec. 3.2 Eq. unified_DP; Sec. 2.2.2), and Chol_Delta, the lower triangle
(Sec. 2.2.1 Eq. T_matrix).

* The pre-map against the oracle on every entry: FP64 bitwise (the same two
  IEEE operations per entry), FP32 to one rounding of the exact value;
  several tile counts, d below one tile, padded leading dimensions, in
  place == out of place, the Hermitian part exactly Hermitian.
* L and dL/dT through each mode against the oracle's grad_T_mode (the
  gradient of L(P(T)), P self-adjoint), in the fused and recompute modes.

Tolerances as in the other parity tests: FP64 1e-12, FP32 1e-5.
"""
import numpy as np
import pytest

import oracle as O
import synth as S
from workloads import rel_fro

torch = pytest.importorskip("torch")
qst = pytest.importorskip("paper_2207_05341_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {"f64": 1e-12, "f32": 1e-5}


def say(*a):
    print(*a, flush=True)


def ctype(prec):
    return np.complex128 if prec == "f64" else np.complex64


def padded(X, pad):
    """X on the GPU inside a wider buffer (row stride d + pad)."""
    d = X.shape[0]
    buf = torch.zeros((d, d + pad), dtype=torch.complex128 if X.dtype == np.complex128 else torch.complex64,
                      device=DEV)
    buf[:, :d] = torch.from_numpy(X)
    return buf[:, :d]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 2, 4, 5, 6, 9, 11])
def test_premap_against_oracle(prec, n):
    say(f"pre-maps N={n} {prec}")
    g = S.rng(7000 + n)
    d = 1 << n
    X = S.ginibre(g, d).astype(ctype(prec))
    Xg = padded(X, 8 if n % 2 else 0)
    for mode, ref in (("hermitian", O.hermitian_part), ("lower", O.lower_part)):
        want = ref(X.astype(np.complex128))
        Y = qst.state_premap(Xg, mode, prec).cpu().numpy()
        if prec == "f64":
            assert np.array_equal(Y, want), mode
        else:
            # one rounding of the exact value to float32
            assert np.array_equal(Y, want.astype(np.complex64)), mode
        if mode == "hermitian":
            assert np.array_equal(Y, Y.conj().T)
        else:
            assert not np.any(np.triu(Y, 1))
        # in place (same buffer, same row stride)
        Z = padded(X, 8 if n % 2 else 0)
        qst.state_premap(Z, mode, prec, out=Z)
        torch.cuda.synchronize()
        assert np.array_equal(Z.cpu().numpy(), Y), mode
    assert np.array_equal(Xg.cpu().numpy(), X)  # the input is untouched


@pytest.mark.parametrize("prec,n", [("f64", 4), ("f64", 10), ("f32", 8), ("f32", 11)])
@pytest.mark.parametrize("state_map", ["hermitian", "lower"])
def test_likelihood_through_modes(prec, n, state_map):
    say(f"likelihood through {state_map}, N={n} {prec}")
    g = S.rng(7100 + n)
    d = 1 << n
    T = S.ginibre(g, d).astype(ctype(prec))
    psi = S.haar_vector(g, d)
    f = S.multinomial_freqs(g, 100_000, O.probs_real(S.depolarised_pure(psi, 0.1)))
    f = f.astype(np.float64 if prec == "f64" else np.float32)
    want_g, want_L = O.grad_T_mode(T.astype(np.complex128), f.astype(np.float64), state_map)
    for mode in ("fused", "recompute"):
        Tg = torch.from_numpy(T).to(DEV).requires_grad_(True)
        fg = torch.from_numpy(f).to(DEV)
        L = qst.likelihood(Tg, fg, prec, mode=mode, state_map=state_map)
        L.backward()
        torch.cuda.synchronize()
        eL = abs(float(L.item()) - want_L) / abs(want_L)
        eg = rel_fro(Tg.grad.cpu().numpy(), want_g)
        say(f"  {mode}: L rel {eL:.2e}, grad rel {eg:.2e}")
        assert eL <= TOL[prec] and eg <= TOL[prec], (mode, eL, eg)
        G = Tg.grad.cpu().numpy()
        if state_map == "hermitian":
            assert np.array_equal(G, G.conj().T)
        else:
            assert not np.any(np.triu(G, 1))
