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


@pytest.mark.parametrize("prec,n", [("f64", 10), ("f32", 10), ("f32", 11)])
def test_fidelity_general_large_against_oracle(prec, n):
    """qst_fidelity_general at N = 10 and 11 (its FP64 products on the
    stream-K tiles) against the oracle's two-square-root F_q, for the
    depolarised pure state of the paper's noise model (q = 0.1)."""
    d = 1 << n
    g = S.rng(7280 + n)
    T = S.ginibre(g, d).astype(ctype(prec))
    rho_hat = O.state_map(T.astype(np.complex128))[0]
    rho = S.depolarised_pure(S.haar_vector(g, d), 0.1).astype(ctype(prec))
    want = O.fidelity_q(rho_hat, rho.astype(np.complex128))
    F, sweeps = qst.fidelity_general(dev_matrix(T), dev_matrix(rho), prec)
    got = float(F.item())
    say(f"N={n} {prec} depolarised q=0.1: F_q {got:.12f} oracle {want:.12f} ({sweeps} sweeps)")
    assert abs(got - want) <= TOL[prec] * want, (got, want)


@pytest.mark.parametrize("n,r", [(6, 1), (8, 4), (10, 1)])
def test_fidelity_general_low_rank_targets(n, r):
    """A pure (r = 1) or rank-r target through the general route (FP64),
    against the exact value of the rank-r route (oracle fidelity_q_lowrank)
    and against the library's rank-r call.

    The general route takes square roots of every eigenvalue of
    T^dagger rho T / tau, d - r of which are zero in exact arithmetic.  The
    eigensolver leaves each of them an absolute error of at most about its
    stopping threshold, 1e-14 of the Frobenius norm (about F_q here), so each
    adds at most sqrt(1e-14 F) to sum sqrt(lambda) = sqrt(F): the relative
    error of F_q is bounded by 2 (d - r) 1e-7.  The rank-r route has no such
    term and meets 1e-12."""
    d = 1 << n
    g = S.rng(7290 + n)
    T = S.ginibre(g, d)
    rho_hat = O.state_map(T)[0]
    W = S.ginibre(g, d, r)
    rho, _ = O.state_map(W)
    exact = O.fidelity_q_lowrank(rho_hat, W)
    F, sweeps = qst.fidelity_general(dev_matrix(T), dev_matrix(rho), "f64")
    got = float(F.item())
    low = float(qst.fidelity_lowrank(dev_matrix(T), dev_matrix(W), "f64").item())
    bound = 2.0 * (d - r) * 1e-7
    say(f"N={n} r={r}: general {got:.12f}, rank-r {low:.12f}, exact {exact:.12f}; "
        f"rel err {abs(got - exact) / exact:.2e} (bound {bound:.1e}), {sweeps} sweeps")
    assert abs(low - exact) <= 1e-12 * exact
    assert abs(got - exact) <= bound * exact


@pytest.mark.parametrize("prec,n,rot", [("f64", 4, False), ("f64", 7, False), ("f32", 7, True), ("f32", 8, False),
                                        ("f64", 8, True)])
def test_likelihood_fc_against_oracle(prec, n, rot):
    """qst_likelihood_fc: F_c (Eq. F_CF) of the model's distribution against
    a target distribution, formed in the fused last pass (N >= 7; N = 4 from
    the stored p), against the oracle's fidelity_c of the oracle's p; L, F
    and the rest of qst_likelihood's outputs as stated in the header.  rot: a rotated tetrahedral POVM
    (the general-POVM form of the fused pass)."""
    d = 1 << n
    g = S.rng(7460 + n)
    povm = None
    if rot:
        U, _ = np.linalg.qr(S.ginibre(g, 2))
        povm = np.array([U @ m @ U.conj().T for m in O.tetrahedral_povm()])
    T = S.ginibre(g, d).astype(ctype(prec))
    rt = np.float64 if prec == "f64" else np.float32
    psi = S.haar_vector(g, d)
    f = S.multinomial_freqs(g, 100_000, O.probs_real(S.depolarised_pure(psi, 0.2), povm)).astype(rt)
    pt = O.probs_real(S.depolarised_pure(psi, 0.1), povm).astype(rt)
    pt[:5] = 0.0
    p_hat = O.probs_real(O.state_map(T.astype(np.complex128))[0], povm)
    want = O.fidelity_c(p_hat, pt.astype(np.float64))
    Tg = torch.from_numpy(T).to(DEV)
    fg, ptg = torch.from_numpy(f).to(DEV), torch.from_numpy(pt).to(DEV)
    out, tau, G, bad, fc = qst.likelihood_forward_fc(Tg, fg, ptg, prec, povm)
    out0, tau0, G0, bad0 = qst.likelihood_forward(Tg, fg, prec, povm)
    torch.cuda.synchronize()
    got = float(fc.item())
    say(f"N={n} {prec} rot={rot}: F_c {got:.12f} oracle {want:.12f}")
    assert abs(got - want) <= TOL[prec] * want
    # a separate kernel instance: the same sums, contracted into FMAs as its
    # own code generation decides, so equal to rounding
    assert torch.equal(tau, tau0) and torch.equal(bad, bad0) and float(out[1]) == float(out0[1])
    # FP32: p itself may round differently (1 ulp), moving L by about 1e-11
    assert abs(float(out[0]) - float(out0[0])) <= (1e-14 if prec == "f64" else 1e-9) * abs(float(out0[0]))
    assert rel_fro(G.cpu().numpy(), G0.cpu().numpy()) <= (1e-14 if prec == "f64" else 1e-6)


def test_likelihood_fc_n11_equals_two_calls():
    """N = 11, FP32: F_c from the fused pass against the library's route
    with p stored (qst_povm_probs of qst_state_map, then
    qst_fidelity_classical)."""
    n, d = 11, 2048
    g = S.rng(7470)
    T = torch.from_numpy(S.ginibre(g, d).astype(np.complex64)).to(DEV)
    f = torch.from_numpy(S.multinomial_freqs(g, 10_000_000, S.porter_thomas_probs(g, 4 ** n, 0.1))
                         .astype(np.float32)).to(DEV)
    pt = torch.from_numpy(S.porter_thomas_probs(g, 4 ** n, 0.2).astype(np.float32)).to(DEV)
    _, _, _, _, fc = qst.likelihood_forward_fc(T, f, pt, "f32")
    rho, _ = qst.state_map(T, "f32")
    p = qst.povm_probs(rho, "f32")
    F2 = qst.fidelity_classical(p, pt, "f32")
    a, b = float(fc.item()), float(F2.item())
    say(f"N=11 f32: F_c fused {a:.10f}, two calls {b:.10f}")
    assert abs(a - b) <= 1e-5 * b
