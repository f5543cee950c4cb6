"""Fidelities through the C ABI (Sec. 2.3): qst_fidelity_lowrank (Eq. F_QF
against a target W W^dagger / Tr of rank r, r = 1 a pure state) and
qst_fidelity_classical (Eq. F_CF), against the oracle's fidelity_q_lowrank
(pinned against the full square-root route and scipy's sqrtm) and
fidelity_c.

Cases: N = 1 .. 11, ranks 1, 4 and the largest accepted (32, or d when
smaller), both precisions, padded leading dimensions; exact values F = 1
(target = the state itself) and the pure-state form |psi^dagger T|^2 /
(tau |psi|^2); bitwise reproducible repeats.  Tolerances: FP64 1e-12,
FP32 1e-5 (relative).
"""
import numpy as np
import pytest

import oracle as O
import synth as S

torch = pytest.importorskip("torch")
qst = pytest.importorskip("paper_2207_05341_amd")

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TOL = {"f64": 1e-12, "f32": 1e-5}


def say(*a):
    print(*a, flush=True)


def ctype(prec):
    return np.complex128 if prec == "f64" else np.complex64


def dev_matrix(X, pad=0):
    rows, cols = X.shape
    tdt = torch.complex128 if X.dtype == np.complex128 else torch.complex64
    buf = torch.zeros((rows, cols + pad), dtype=tdt, device=DEV)
    buf[:, :cols] = torch.from_numpy(X)
    return buf[:, :cols]


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 3, 6, 8, 11])
def test_fidelity_lowrank_against_oracle(prec, n):
    d = 1 << n
    g = S.rng(7200 + n)
    T = S.ginibre(g, d).astype(ctype(prec))
    rho_hat = O.state_map(T.astype(np.complex128))[0]
    Tg = dev_matrix(T, pad=4 if n % 2 else 0)
    for r in sorted({1, min(4, d), min(qst.QST_FIDELITY_MAX_RANK, d)}):
        W = S.ginibre(g, d, r).astype(ctype(prec))
        want = O.fidelity_q_lowrank(rho_hat, W.astype(np.complex128))
        F = qst.fidelity_lowrank(Tg, dev_matrix(W, pad=3), prec)
        F2 = qst.fidelity_lowrank(Tg, dev_matrix(W), prec)
        got = float(F.item())
        say(f"N={n} {prec} r={r}: F_q {got:.12f} oracle {want:.12f}")
        assert abs(got - want) <= TOL[prec] * want, (r, got, want)
        assert float(F2.item()) == got  # bitwise reproducible, any row stride of W


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fidelity_exact_values(prec):
    """F_q(rho, rho) = 1 for a rank-r state given by its own factor, and the
    pure-state closed form |psi^dagger T|^2 / (tau |psi|^2)."""
    g = S.rng(7300)
    n, d, r = 7, 128, 5
    Wf = S.ginibre(g, d, r).astype(ctype(prec))
    T = np.zeros((d, d), dtype=ctype(prec))
    T[:, :r] = Wf  # rho_hat = Wf Wf^dagger / Tr
    F = float(qst.fidelity_lowrank(dev_matrix(T), dev_matrix(Wf), prec).item())
    assert abs(F - 1.0) <= TOL[prec], F
    Tr = S.ginibre(g, d).astype(ctype(prec))
    psi = S.haar_vector(g, d).astype(ctype(prec))
    t64, p64 = Tr.astype(np.complex128), psi.astype(np.complex128)
    want = abs(np.vdot(p64, t64 @ t64.conj().T @ p64)) / (O.trace_tt(t64) * np.vdot(p64, p64).real)
    F = float(qst.fidelity_lowrank(dev_matrix(Tr), dev_matrix(psi.reshape(d, 1)), prec).item())
    assert abs(F - want) <= TOL[prec] * want, (F, want)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 5, 11])
def test_fidelity_classical_against_oracle(prec, n):
    g = S.rng(7400 + n)
    rt = np.float64 if prec == "f64" else np.float32
    ph = S.porter_thomas_probs(g, 4 ** n, 0.1).astype(rt)
    p = S.multinomial_freqs(g, 10_000, S.porter_thomas_probs(g, 4 ** n, 0.2)).astype(rt)
    p[: min(3, p.size)] = -p[: min(3, p.size)]  # negative entries read as 0
    want = O.fidelity_c(ph, p)
    F = qst.fidelity_classical(torch.from_numpy(ph).to(DEV), torch.from_numpy(p).to(DEV), prec)
    got = float(F.item())
    say(f"N={n} {prec}: F_c {got:.12f} oracle {want:.12f}")
    assert abs(got - want) <= TOL[prec] * want
    assert float(qst.fidelity_classical(torch.from_numpy(ph).to(DEV), torch.from_numpy(p).to(DEV), prec).item()) == got


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 3, 6, 8])
def test_fidelity_general_against_oracle(prec, n):
    """qst_fidelity_general (one eigensolve of T^dagger rho T, Eq. fq_decom)
    against the oracle's F_q by two square roots (Eq. F_QF) for full-rank
    targets: a Ginibre mixed state and the depolarised pure state of the
    paper's noise model; F = 1 for rho = rho_hat."""
    d = 1 << n
    g = S.rng(7250 + n)
    T = S.ginibre(g, d).astype(ctype(prec))
    T64 = T.astype(np.complex128)
    rho_hat = O.state_map(T64)[0]
    Tg = dev_matrix(T, pad=2)
    X = S.ginibre(g, d)
    targets = {"ginibre": (X @ X.conj().T) / np.trace(X @ X.conj().T).real,
               "depolarised": S.depolarised_pure(S.haar_vector(g, d), 0.3), "self": rho_hat}
    for name, rho in targets.items():
        r = rho.astype(ctype(prec))
        want = O.fidelity_q(rho_hat, r.astype(np.complex128))
        F, sweeps = qst.fidelity_general(Tg, dev_matrix(r), prec)
        got = float(F.item())
        say(f"N={n} {prec} {name}: F_q {got:.12f} oracle {want:.12f} ({sweeps} sweeps)")
        tol = TOL[prec] if name != "self" else max(TOL[prec], 1e-9 * d)
        assert abs(got - want) <= tol * want, (name, got, want)
    F1, _ = qst.fidelity_general(Tg, dev_matrix(rho_hat.astype(ctype(prec))), prec)
    assert abs(float(F1.item()) - 1.0) <= max(TOL[prec], 1e-9 * d)
