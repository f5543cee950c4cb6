"""Pins of the FP64 oracle against facts that do not come from the oracle:
values the paper prints, closed forms, invariants, brute force on tiny
inputs, and library routines for the special cases that reduce to them.

Each test names the passage of the paper it rests on.  Tolerances are
stated in the tests; all arithmetic is float64.
"""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

import oracle as O
import synth as S
from conftest import read_table

T3 = 1.0 / math.sqrt(3.0)


def bloch_state(r):
    """(I + r . sigma)/2 written out entrywise (no Pauli table reuse)."""
    x, y, z = r
    return 0.5 * np.array([[1 + z, x - 1j * y], [x + 1j * y, 1 - z]], dtype=np.complex128)


def kron_all(mats):
    out = np.ones((1, 1), dtype=np.complex128)
    for m in mats:
        out = np.kron(out, m)
    return out


# --------------------------------------------------------------------------
# POVM constants (Sec. 4.1)
# --------------------------------------------------------------------------

def test_tetrahedral_constants_match_paper():
    rows = read_table("tetrahedral_bloch.txt")
    want = np.array([[float(v) * T3 for v in r[1:]] for r in rows])
    assert [int(r[0]) for r in rows] == [0, 1, 2, 3]
    np.testing.assert_allclose(O.TETRA_S, want, rtol=0, atol=1e-16)


def test_tetrahedral_povm_is_a_povm():
    M = O.tetrahedral_povm()
    # entrywise form of (I + s.sigma)/4 written out independently
    for a in range(4):
        sx, sy, sz = O.TETRA_S[a]
        want = 0.25 * np.array([[1 + sz, sx - 1j * sy], [sx + 1j * sy, 1 - sz]])
        np.testing.assert_allclose(M[a], want, atol=1e-16)
        w = np.linalg.eigvalsh(M[a])
        np.testing.assert_allclose(w, [0.0, 0.5], atol=1e-15)  # rank 1, PSD
        np.testing.assert_allclose(M[a], M[a].conj().T, atol=0)
    np.testing.assert_allclose(M.sum(axis=0), np.eye(2), atol=1e-15)  # sum M = I (Eq. MLE)


# --------------------------------------------------------------------------
# Born rule and product structure (Sec. 2.1, Sec. 3.3)
# --------------------------------------------------------------------------

def test_single_qubit_born_rule_by_hand():
    """N = 1: p_a = Tr(M_a rho) = sum_{x,y} (M_a)_{xy} rho_{yx}, summed by hand."""
    g = S.rng(11)
    M = O.tetrahedral_povm()
    for _ in range(5):
        rho, _ = O.state_map(S.ginibre(g, 2))
        want = [sum(M[a][x, y] * rho[y, x] for x in range(2) for y in range(2)) for a in range(4)]
        np.testing.assert_allclose(O.probs(rho), want, atol=1e-16)
        np.testing.assert_allclose(O.probs_kron(rho), want, atol=1e-16)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_contraction_equals_kronecker(n):
    """The per-qubit contraction is an exact refactoring of the Kronecker
    sum (Sec. 3.3); checked also on non-Hermitian input, where both sides
    are complex-valued linear maps."""
    g = S.rng(100 + n)
    d = 1 << n
    rho, _ = O.state_map(S.ginibre(g, d))
    X = S.ginibre(g, d)
    for A in (rho, X):
        pk = O.probs_kron(A)
        pt = O.probs(A)
        assert np.max(np.abs(pk - pt)) <= 1e-15 * max(1.0, np.max(np.abs(pk)))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8])
def test_product_state_closed_form(n):
    """rho = (x)_i (I + r_i.sigma)/2 gives p_k = prod_i (1 + s_{k_i}.r_i)/4.
    Distinct Bloch vectors per qubit with r_y != 0 fail under a wrong qubit
    order, a wrong outcome order, or the transposed pairing of Eq. PS."""
    g = S.rng(200 + n)
    r = g.standard_normal((n, 3))
    r = 0.95 * r / np.linalg.norm(r, axis=1, keepdims=True)
    assert np.all(np.abs(r[:, 1]) > 1e-3)
    rho = kron_all([bloch_state(ri) for ri in r])
    want = np.array([np.prod([(1.0 + O.TETRA_S[ks[i]] @ r[i]) / 4.0 for i in range(n)])
                     for ks in itertools.product(range(4), repeat=n)])
    p = O.probs_real(rho)
    assert np.max(np.abs(p - want)) <= 1e-15
    if n <= 5:
        assert np.max(np.abs(O.probs_kron(rho).real - want)) <= 1e-15


def pure_qubit(r):
    """Ket with Bloch vector r (|r| = 1): (cos(t/2), e^{i f} sin(t/2))."""
    t = math.acos(max(-1.0, min(1.0, r[2])))
    f = math.atan2(r[1], r[0])
    return np.array([math.cos(t / 2), complex(math.cos(f), math.sin(f)) * math.sin(t / 2)])


@pytest.mark.parametrize("n", [1, 3, 13])
def test_probs_at_product_state_closed_form(n):
    """Single outcomes from a rank-1 factor: W = (x)_i |psi_i>, pure qubits
    with distinct Bloch vectors (r_y != 0), gives p_k = prod_i (1 + s_{k_i}.r_i)/4
    at any N, N = 13 (8192 rows) included."""
    g = S.rng(250 + n)
    r = g.standard_normal((n, 3))
    r = r / np.linalg.norm(r, axis=1, keepdims=True)
    assert np.all(np.abs(r[:, 1]) > 1e-3)
    W = np.ones(1, dtype=np.complex128)
    for ri in r:
        W = np.kron(W, pure_qubit(ri))
    D = 4 ** n
    ks = list(range(D)) if D <= 64 else [0, D - 1] + [int(k) for k in g.integers(0, D, 62)]
    outs = [O.outcome_digits(k, n) for k in ks]
    want = np.array([np.prod([(1.0 + O.TETRA_S[o[i]] @ r[i]) / 4.0 for i in range(n)]) for o in outs])
    got = O.probs_at(W, outs)
    assert np.max(np.abs(got - want)) <= 1e-14 * np.max(want)


@pytest.mark.parametrize("n", [1, 3, 5])
@pytest.mark.parametrize("rank", [1, 3, None])
def test_probs_at_equals_full_map(n, rank):
    """probs_at(W) = the full product map of rho = W W^dagger / Tr at every
    outcome, for thin and square factors, tetrahedral and rotated POVMs;
    the outcome digits follow k = sum_i k_i 4^(N-i)."""
    g = S.rng(260 + 10 * n + (rank or 0))
    d = 1 << n
    W = S.ginibre(g, d, rank or d)
    rho, _ = O.state_map(W)
    U, _ = np.linalg.qr(S.ginibre(g, 2))
    rot = np.array([U @ m @ U.conj().T for m in O.tetrahedral_povm()])
    for povm in (None, rot):
        full = O.probs_real(rho, povm)
        outs = [O.outcome_digits(k, n) for k in range(4 ** n)]
        got = O.probs_at(W, outs, povm)
        assert np.max(np.abs(got - full)) <= 1e-14 * np.max(full)
    assert O.outcome_digits(4 ** n - 1, n) == (3,) * n
    assert O.outcome_digits(1, n)[-1] == 1 and O.outcome_digits(4 ** (n - 1), n)[0] == 1


def test_eq_ps_literal_pairing_is_transposed():
    """Reading of Eq. PS: pairing b_i (the (0,1) entry of M_i) with the
    (0,1) block B computes Tr(M^T rho), which flips s_y.  The Born rule pairs
    it with the (1,0) block.  On a state with r_y != 0 the two differ."""
    M = O.tetrahedral_povm()
    rho = bloch_state([0.1, 0.8, 0.2])
    born = np.array([np.trace(M[a] @ rho) for a in range(4)]).real
    literal = np.array([M[a][0, 0] * rho[0, 0] + M[a][0, 1] * rho[0, 1]
                        + M[a][1, 0] * rho[1, 0] + M[a][1, 1] * rho[1, 1] for a in range(4)]).real
    np.testing.assert_allclose(O.probs_real(rho), born, atol=1e-16)
    assert np.max(np.abs(born - literal)) > 0.05


@pytest.mark.parametrize("n", [1, 2, 3, 6, 10])
def test_ghzi_closed_form(n):
    """GHZi target (Sec. 4): rho has four nonzero entries, so
    p_k = 1/2 [prod (M_{k_i})_00 + prod (M_{k_i})_11] - Im prod (M_{k_i})_01."""
    M = O.tetrahedral_povm()
    psi = S.ghzi(n)
    rho = np.outer(psi, psi.conj())
    want = []
    for ks in itertools.product(range(4), repeat=n):
        a00 = np.prod([M[k][0, 0] for k in ks])
        a11 = np.prod([M[k][1, 1] for k in ks])
        a01 = np.prod([M[k][0, 1] for k in ks])
        want.append((0.5 * (a00 + a11)).real - a01.imag)
    assert np.max(np.abs(O.probs_real(rho) - np.array(want))) <= 1e-15


@pytest.mark.parametrize("n", [1, 4, 9])
def test_maximally_mixed_and_basis_state(n):
    d = 1 << n
    p = O.probs_real(np.eye(d, dtype=np.complex128) / d)
    np.testing.assert_allclose(p, np.full(4 ** n, 4.0 ** -n), rtol=1e-14, atol=0)
    e0 = np.zeros((d, d), dtype=np.complex128)
    e0[0, 0] = 1.0
    want = np.array([np.prod([(1.0 + O.TETRA_S[k][2]) / 4.0 for k in ks])
                     for ks in itertools.product(range(4), repeat=n)])
    np.testing.assert_allclose(O.probs_real(e0), want, rtol=0, atol=1e-16)


@pytest.mark.parametrize("n", [1, 3, 6, 8])
def test_probability_invariants(n):
    """sum_k p_k = Tr rho = 1 (sum M_k = I) and p_k >= 0 (M_k, rho PSD)."""
    g = S.rng(300 + n)
    rho, _ = O.state_map(S.ginibre(g, 1 << n))
    p = O.probs_real(rho)
    assert abs(math.fsum(p.tolist()) - 1.0) <= 1e-13
    assert p.min() >= 0.0


@pytest.mark.parametrize("n", [1, 2, 3])
def test_dual_frame_round_trip(n):
    """The tetrahedral POVM is informationally complete: with dual frame
    D_a = (I + 3 s_a.sigma)/2, rho = sum_k p_k (x)_i D_{k_i}.  The dual frame
    is built here entrywise, independent of the oracle's POVM table."""
    g = S.rng(400 + n)
    D = [bloch_state(3.0 * O.TETRA_S[a]) for a in range(4)]
    rho, _ = O.state_map(S.ginibre(g, 1 << n))
    p = O.probs_real(rho)
    rec = sum(p[idx] * kron_all([D[a] for a in ks])
              for idx, ks in enumerate(itertools.product(range(4), repeat=n)))
    assert np.max(np.abs(rec - rho)) <= 1e-14


# --------------------------------------------------------------------------
# State map (Sec. 2.2.1 Eq. T_matrix; Sec. 3.2 Eq. unified_DP / abs_P)
# --------------------------------------------------------------------------

def test_state_map_by_loops():
    g = S.rng(500)
    d = 4
    T = S.ginibre(g, d)
    tau_loop = 0.0
    for i in range(d):
        for j in range(d):
            tau_loop += T[i, j].real ** 2 + T[i, j].imag ** 2
    Sm = np.zeros((d, d), dtype=np.complex128)
    for i in range(d):
        for j in range(d):
            for k in range(d):
                Sm[i, j] += T[i, k] * np.conj(T[j, k])
    rho, tau = O.state_map(T)
    assert abs(tau - tau_loop) <= 1e-13 * tau
    assert abs(tau - np.linalg.norm(T) ** 2) <= 1e-13 * tau
    np.testing.assert_allclose(rho, Sm / tau_loop, atol=1e-15)


@pytest.mark.parametrize("n", [1, 3, 6])
def test_state_map_invariants(n):
    g = S.rng(600 + n)
    d = 1 << n
    T = S.ginibre(g, d)
    rho, _ = O.state_map(T)
    assert abs(np.trace(rho) - 1.0) <= 1e-14
    assert np.max(np.abs(rho - rho.conj().T)) <= 1e-16
    assert np.linalg.eigvalsh(rho).min() >= -1e-15
    # scale invariance and right-unitary invariance
    U, _ = np.linalg.qr(S.ginibre(g, d))
    np.testing.assert_allclose(O.state_map(3.7 * T)[0], rho, atol=1e-15)
    np.testing.assert_allclose(O.state_map(T @ U)[0], rho, atol=1e-14)
    np.testing.assert_allclose(O.state_map(np.eye(d))[0], np.eye(d) / d, atol=0)


def test_state_map_kron_and_hermitian_reading():
    """T = T1 (x) T2 gives rho1 (x) rho2; for Hermitian T (the unified map,
    Eq. unified_DP) T T^dagger = T^dagger T = T^2, so reading 1 is moot there;
    and at P = 2 the absolute map Q|L|^P Q^dagger/Tr|L|^P equals it
    (Eq. abs_P), checked with a library eigensolver."""
    g = S.rng(700)
    T1, T2 = S.ginibre(g, 2), S.ginibre(g, 4)
    np.testing.assert_allclose(O.state_map(np.kron(T1, T2))[0],
                               np.kron(O.state_map(T1)[0], O.state_map(T2)[0]), atol=1e-15)
    H = S.ginibre(g, 8)
    H = (H + H.conj().T) / 2
    rho, _ = O.state_map(H)
    w, Q = scipy.linalg.eigh(H)
    absP = (Q * np.abs(w) ** 2) @ Q.conj().T / np.sum(np.abs(w) ** 2)
    np.testing.assert_allclose(rho, absP, atol=1e-14)
    np.testing.assert_allclose(rho, (H.conj().T @ H) / np.trace(H.conj().T @ H).real, atol=1e-15)


# --------------------------------------------------------------------------
# Negative log-likelihood (Eq. MLE, Sec. 3.1 loss)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 4, 7])
def test_nll_maximally_mixed(n):
    """rho = I/d: every p_k = 4^-N, so L = N ln 4 * sum f."""
    g = S.rng(800 + n)
    f = g.integers(0, 5, size=4 ** n).astype(np.float64)
    p = O.probs_real(np.eye(1 << n, dtype=np.complex128) / (1 << n))
    want = n * math.log(4.0) * math.fsum(f.tolist())
    assert abs(O.nll(p, f) - want) <= 1e-13 * want
    assert abs(O.nll_vec(p, f) - want) <= 1e-13 * want


def test_nll_entropy_and_gibbs():
    """f = p(T) gives L = Shannon entropy H(p) (library routine); for any
    normalised f, L >= H(f) (Gibbs), with equality iff p = f."""
    g = S.rng(900)
    n = 4
    rho, _ = O.state_map(S.ginibre(g, 1 << n))
    p = O.probs_real(rho)
    assert abs(O.nll(p, p) - scipy.stats.entropy(p)) <= 1e-13
    f = S.multinomial_freqs(g, 1000, p)
    assert O.nll(p, f) >= scipy.stats.entropy(f) - 1e-14
    assert O.nll_vec(p, f) == O.nll(p, f)


def test_nll_zero_and_nonpositive_terms():
    p = np.array([0.5, 0.0, 0.25, 0.25])
    f = np.array([0.5, 0.0, 0.5, 0.0])
    assert O.nll(p, f) == pytest.approx(-(0.5 * math.log(0.5) + 0.5 * math.log(0.25)), rel=1e-15)
    f2 = np.array([0.5, 0.1, 0.4, 0.0])
    assert O.nll(p, f2) == math.inf and O.nll_vec(p, f2) == math.inf


# --------------------------------------------------------------------------
# Adjoint and gradient
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 4, 6])
def test_adjoint_dot_product(n):
    """<A(X), y> = Tr(X A^dagger(y)) for complex X and real y, where
    A(X)_k = Tr(M_k X): the adjoint is pinned to the (pinned) forward map."""
    g = S.rng(1000 + n)
    d = 1 << n
    X = S.ginibre(g, d)
    y = g.standard_normal(4 ** n)
    lhs = np.sum(O.probs(X) * y)
    rhs = np.trace(X @ O.adjoint(y, n))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))
    np.testing.assert_allclose(O.adjoint(np.ones(4 ** n), n), np.eye(d), atol=1e-14)
    if n <= 4:
        np.testing.assert_allclose(O.adjoint(y, n), O.adjoint_kron(y, n), atol=1e-14)


@pytest.mark.parametrize("n,seed", [(1, 1), (2, 2), (3, 3), (4, 4), (6, 5)])
def test_gradient_central_differences(n, seed):
    """Central finite differences of the forward loss on random complex
    directions E: (L(T+hE) - L(T-hE))/2h = Re<grad, E> (PyTorch convention)."""
    g = S.rng(1100 + seed)
    d = 1 << n
    T = S.ginibre(g, d)
    psi = S.haar_vector(g, d)
    f = S.multinomial_freqs(g, 5000, O.probs_real(S.depolarised_pure(psi, 0.3)))
    grad, _ = O.grad_T(T, f)
    h = 1e-5 * np.linalg.norm(T)
    for E in S.unit_directions(g, d, 6):
        fd = (O.loss_of_T(T + h * E, f) - O.loss_of_T(T - h * E, f)) / (2 * h)
        an = float(np.sum(grad.real * E.real + grad.imag * E.imag))
        assert abs(fd - an) <= 1e-6 * np.linalg.norm(grad) + 1e-12


@pytest.mark.parametrize("n", [2, 5])
def test_gradient_invariants(n):
    """L(T U) = L(T) for unitary U and L(cT) = L(T) make T^dagger grad
    Hermitian (skew part 0) and traceless; grad = 0 when f is proportional
    to p(T); G' = G + F I with G = sum_k (f_k/p_k) M_k."""
    g = S.rng(1200 + n)
    d = 1 << n
    T = S.ginibre(g, d)
    f = S.multinomial_freqs(g, 10000, O.probs_real(O.state_map(S.ginibre(g, d))[0]))
    grad, _ = O.grad_T(T, f)
    X = T.conj().T @ grad
    scale = np.max(np.abs(X))
    assert np.max(np.abs(X - X.conj().T)) <= 1e-13 * scale
    assert abs(np.trace(X)) <= 1e-13 * scale * d
    rho, tau = O.state_map(T)
    p = O.probs_real(rho)
    g0, _ = O.grad_T(T, 2.5 * p)
    assert np.max(np.abs(g0)) <= 1e-15 * np.max(np.abs(grad)) * 1e3
    F = math.fsum(f.tolist())
    Gp = O.adjoint(O.cotangent(p, f), n)
    G = O.adjoint(np.where(f != 0, f / p, 0.0), n)
    np.testing.assert_allclose(Gp, F * np.eye(d) - G, atol=1e-12)


# --------------------------------------------------------------------------
# Fidelities (Sec. 2.3) and the caption closed forms
# --------------------------------------------------------------------------

def test_caption_closed_forms():
    g = S.rng(1300)
    for kind, n, param, value in read_table("caption_closed_forms.txt"):
        n, param, value = int(n), float(param), float(value)
        psi = S.haar_vector(g, 1 << n)
        if kind == "purity":
            rho = S.depolarised_pure(psi, 1.0 - param)  # p|psi><psi| + (1-p) I/d
            assert abs(np.trace(rho @ rho).real - value) <= 1e-13
        else:
            rho = S.depolarised_pure(psi, param)
            pure = np.outer(psi, psi.conj())
            # the matrix-square-root route amplifies rounding in the d-1 zero
            # eigenvalues of the pure target (sqrt of ~1e-17 each), hence 1e-5
            assert abs(O.fidelity_q(rho, pure) - value) <= 1e-5
            assert abs(np.vdot(psi, rho @ psi).real - value) <= 1e-13


def test_fidelity_forms():
    g = S.rng(1400)
    d = 16
    rho, _ = O.state_map(S.ginibre(g, d))
    assert abs(O.fidelity_q(rho, rho) - 1.0) <= 1e-10
    W = S.ginibre(g, d, 3)
    target, _ = O.state_map(W)
    fq = O.fidelity_q(rho, target)
    # symmetric, low-rank shortcut, and the classical-fidelity upper bound
    # (Eq. F_CF).  The full square-root route loses ~1e-9 to the 13 zero
    # eigenvalues of the rank-3 target; the low-rank route has no such loss.
    assert abs(fq - O.fidelity_q(target, rho)) <= 1e-7
    assert abs(fq - O.fidelity_q_lowrank(rho, W)) <= 1e-7
    assert O.fidelity_c(O.probs_real(rho), O.probs_real(target)) >= fq - 1e-12
    # scipy's sqrtm as an independent route to Eq. F_QF
    s = scipy.linalg.sqrtm(rho)
    ref = np.trace(scipy.linalg.sqrtm(s @ target @ s)).real ** 2
    assert abs(fq - ref) <= 1e-8


def test_fidelity_c_closed_forms():
    """Eq. F_CF fixed by values worked out by hand, so that dropping the
    outer square, the square root, or the pairing of the two distributions
    fails at least one of them:

    * a point mass against the uniform distribution on 4 outcomes:
      (sqrt(1 * 1/4))^2 = 1/4 (without the square it would be 1/2);
    * disjoint supports give 0, equal normalised distributions give 1;
    * p_hat = (1/2, 1/2, 0, 0), p = (1/8, 1/8, 3/8, 3/8):
      (2 sqrt(1/16))^2 = 1/4;
    * product states under the product POVM (Sec. 3.3): the outcome
      distributions are products over qubits, so F_c is the product of the
      single-qubit values, each (sum_a sqrt(p_hat_a p_a))^2 with
      p_a = (1 + s_a . r)/4 (Sec. 4.1) -- an unsquared form gives the
      product of their square roots instead."""
    uni = np.full(4, 0.25)
    assert O.fidelity_c(np.array([1.0, 0.0, 0.0, 0.0]), uni) == pytest.approx(0.25, abs=1e-15)
    assert O.fidelity_c(np.array([0.5, 0.5, 0.0, 0.0]), np.array([0.0, 0.0, 0.5, 0.5])) == 0.0
    assert O.fidelity_c(uni, uni) == pytest.approx(1.0, abs=1e-15)
    assert O.fidelity_c(np.array([0.5, 0.5, 0.0, 0.0]),
                        np.array([0.125, 0.125, 0.375, 0.375])) == pytest.approx(0.25, abs=1e-15)

    g = S.rng(1410)
    n = 3
    ra = 0.9 * g.standard_normal((n, 3))
    rb = 0.9 * g.standard_normal((n, 3))
    ra /= np.maximum(1.0, np.linalg.norm(ra, axis=1, keepdims=True) / 0.9)
    rb /= np.maximum(1.0, np.linalg.norm(rb, axis=1, keepdims=True) / 0.9)
    per_qubit = []
    for i in range(n):
        pa = [(1.0 + O.TETRA_S[a] @ ra[i]) / 4.0 for a in range(4)]
        pb = [(1.0 + O.TETRA_S[a] @ rb[i]) / 4.0 for a in range(4)]
        per_qubit.append(sum(math.sqrt(x * y) for x, y in zip(pa, pb)) ** 2)
    want = math.prod(per_qubit)
    assert all(v < 0.999 for v in per_qubit)  # the square matters for every factor
    pa = O.probs_real(kron_all([bloch_state(r) for r in ra]))
    pb = O.probs_real(kron_all([bloch_state(r) for r in rb]))
    assert O.fidelity_c(pa, pb) == pytest.approx(want, rel=1e-13)
    assert abs(math.prod(math.sqrt(v) for v in per_qubit) - want) > 1e-3


def test_adam_matches_torch():
    """The oracle's Adam loop equals torch.optim.Adam (CPU, float64) driven by
    the oracle gradient, on a complex parameter."""
    import torch
    g = S.rng(1500)
    n = 2
    T0 = S.ginibre(g, 1 << n)
    f = S.multinomial_freqs(g, 1000, O.probs_real(S.depolarised_pure(S.haar_vector(g, 4), 0.2)))
    Tn, losses = O.adam_train(T0, f, steps=5, lr=1e-2)
    P = torch.nn.Parameter(torch.from_numpy(T0.copy()))
    opt = torch.optim.Adam([P], lr=1e-2, betas=(0.9, 0.999), eps=1e-12)
    for _ in range(5):
        opt.zero_grad()
        gr, _ = O.grad_T(P.detach().numpy(), f)
        P.grad = torch.from_numpy(gr)
        opt.step()
    np.testing.assert_allclose(P.detach().numpy(), Tn, atol=1e-13)
    assert losses[-1] < losses[0]


# --------------------------------------------------------------------------
# State-map modes (Sec. 2.2.1 Eq. T_matrix; Sec. 2.2.2; Sec. 3.2
# Eq. unified_DP, Eq. abs_P)
# --------------------------------------------------------------------------

def re_inner(A, B):
    """Re Tr(A^dagger B), written out entrywise."""
    return float(np.sum(A.real * B.real + A.imag * B.imag))


@pytest.mark.parametrize("n", [1, 3])
def test_premaps_are_orthogonal_projections(n):
    """Hermitian part and lower triangle: their images are Hermitian /
    lower-triangular matrices, they fix those, they are idempotent, and they
    are self-adjoint for Re Tr(A^dagger B) (so they also map dL/dT' back)."""
    g = S.rng(1300 + n)
    d = 1 << n
    X, Y = S.ginibre(g, d), S.ginibre(g, d)
    H = O.hermitian_part(X)
    for r in range(d):
        for c in range(d):
            # entrywise definition: (X_rc + conj(X_cr)) / 2
            want = (X[r, c] + np.conj(X[c, r])) / 2
            assert H[r, c] == want
    assert np.array_equal(H, H.conj().T)
    assert np.array_equal(O.hermitian_part(H), H)
    Lo = O.lower_part(X)
    for r in range(d):
        for c in range(d):
            assert Lo[r, c] == (X[r, c] if c <= r else 0)
    assert np.array_equal(O.lower_part(Lo), Lo)
    for mode in ("hermitian", "lower"):
        a = re_inner(O.premap(X, mode), Y)
        b = re_inner(X, O.premap(Y, mode))
        assert abs(a - b) <= 1e-13 * (abs(a) + 1.0)
    assert np.array_equal(O.premap(X, "plain"), X)


def test_abs_projection_closed_form_and_cholh():
    """Eq. abs_P on a diagonal H is diag(|lambda|^P) / sum |lambda|^P; for a
    Hermitian T, P = 2 is Eq. unified_DP: T T^dagger / Tr(T T^dagger)
    (the library eigensolver against a plain product)."""
    lam = np.array([2.0, -0.5, 0.0, -3.0])
    for P in (0.5, 1.0, 2.0, 3.5):
        w = np.abs(lam) ** P
        np.testing.assert_allclose(O.abs_projection(np.diag(lam), P), np.diag(w / w.sum()), atol=1e-15)
    g = S.rng(1310)
    for n in (2, 4):
        H = O.hermitian_part(S.ginibre(g, 1 << n))
        rho, _ = O.state_map(H)
        np.testing.assert_allclose(O.abs_projection(H, 2.0), rho, atol=1e-14)
        R = O.abs_projection(H, 1.3)
        assert abs(np.trace(R).real - 1.0) <= 1e-13
        assert np.min(np.linalg.eigvalsh(R)) >= -1e-14


def test_abs_map_closed_forms():
    """The absolute map A = Q |Lambda|^(P/2) Q^dagger of the Hermitian part H
    against forms that need no eigendecomposition: P = 0 gives I, P = 4
    gives H H, and A = (H H)^(P/4) by scipy's fractional matrix power
    (Schur-Pade) and its square root; A A^dagger / Tr is Eq. abs_P."""
    g = S.rng(1330)
    for n in (1, 3, 5):
        d = 1 << n
        T = S.ginibre(g, d)
        H = O.hermitian_part(T)
        HH = H @ H
        np.testing.assert_allclose(O.abs_map(T, 0.0)[0], np.eye(d), atol=1e-12)
        np.testing.assert_allclose(O.abs_map(T, 4.0)[0], HH, atol=1e-12 * np.abs(HH).max())
        np.testing.assert_allclose(O.abs_map(T, 2.0)[0], scipy.linalg.sqrtm(HH), atol=1e-10 * np.abs(H).max())
        for P in (0.5, 1.0, 1.5, 3.0):
            A, Q, lam = O.abs_map(T, P)
            want = scipy.linalg.fractional_matrix_power(HH, P / 4.0)
            assert np.abs(A - want).max() <= 1e-9 * np.abs(want).max(), P
            np.testing.assert_allclose(A, A.conj().T, atol=1e-13 * np.abs(A).max())
            rho = A @ A.conj().T / np.trace(A @ A.conj().T).real
            np.testing.assert_allclose(rho, O.abs_projection(H, P), atol=1e-13)
            np.testing.assert_allclose((Q * lam) @ Q.conj().T, H, atol=1e-13 * np.abs(H).max())


def test_abs_divided_differences():
    """Gamma for g = |l|^(P/2): P = 4 gives l_i + l_j (ties included), P = 2
    with the signs of l_i, l_j equal gives their common sign and with
    opposite signs (|l_i| - |l_j|)/(l_i - l_j); ties take g'."""
    lam = np.array([-2.0, -0.5, 0.25, 0.25, 3.0])
    np.testing.assert_allclose(O.abs_divided_differences(lam, 4.0), lam[:, None] + lam[None, :], atol=1e-15)
    G2 = O.abs_divided_differences(lam, 2.0)
    for i in range(5):
        for j in range(5):
            if np.sign(lam[i]) == np.sign(lam[j]):
                assert G2[i, j] == np.sign(lam[i])
            else:
                assert abs(G2[i, j] - (abs(lam[i]) - abs(lam[j])) / (lam[i] - lam[j])) <= 1e-15
    G1 = O.abs_divided_differences(lam, 1.0)
    assert abs(G1[2, 3] - 0.5 * 0.25 ** -0.5) <= 1e-15 and abs(G1[1, 1] + 0.5 * 0.5 ** -0.5) <= 1e-15


def test_abs_map_backward_p4_closed_form():
    """At P = 4, A = H H, so dL/dT = S H + H S (S the Hermitian part of
    dL/dA) with no eigendecomposition."""
    g = S.rng(1340)
    for n in (2, 4):
        d = 1 << n
        T, GA = S.ginibre(g, d), S.ginibre(g, d)
        A, Q, lam = O.abs_map(T, 4.0)
        H, Sg = O.hermitian_part(T), O.hermitian_part(GA)
        want = Sg @ H + H @ Sg
        np.testing.assert_allclose(O.abs_map_backward(Q, lam, 4.0, GA), want, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("P", [0.5, 1.0, 1.5, 2.0, 3.0])
def test_abs_map_backward_central_differences(P):
    """phi(T) = Re<W, A(T)> by central differences on random complex
    directions E against Re<abs_map_backward(W), E>."""
    g = S.rng(1350 + int(4 * P))
    d = 8
    T, W = S.ginibre(g, d), S.ginibre(g, d)
    A, Q, lam = O.abs_map(T, P)
    grad = O.abs_map_backward(Q, lam, P, W)
    h = 1e-6
    for _ in range(4):
        E = S.ginibre(g, d)
        fp = np.vdot(W, O.abs_map(T + h * E, P)[0]).real
        fm = np.vdot(W, O.abs_map(T - h * E, P)[0]).real
        fd, an = (fp - fm) / (2 * h), np.vdot(grad, E).real
        assert abs(fd - an) <= 1e-6 * (abs(an) + np.abs(grad).max()), (P, fd, an)


def test_abs_likelihood_gradient_central_differences():
    """L of the P-order absolute projection (P = 1.5) through the whole
    likelihood: grad_T_abs against central differences."""
    g = S.rng(1360)
    n, d, P = 3, 8, 1.5
    T = S.ginibre(g, d)
    psi = S.haar_vector(g, d)
    f = S.multinomial_freqs(g, 5000, O.probs_real(S.depolarised_pure(psi, 0.2)))
    grad, L = O.grad_T_abs(T, f, P)
    rho = O.abs_projection(O.hermitian_part(T), P)
    assert abs(L - O.nll(O.probs_real(rho), f)) <= 1e-12 * abs(L)
    h = 1e-6
    for _ in range(4):
        E = S.ginibre(g, d)
        Lp = O.loss_of_T(O.abs_map(T + h * E, P)[0], f)
        Lm = O.loss_of_T(O.abs_map(T - h * E, P)[0], f)
        fd, an = (Lp - Lm) / (2 * h), np.vdot(grad, E).real
        assert abs(fd - an) <= 1e-6 * (abs(an) + np.abs(grad).max())


@pytest.mark.parametrize("mode", ["hermitian", "lower"])
def test_mode_gradient_central_differences(mode):
    """L(premap(T)) by central differences on random complex directions
    against Re<grad_T_mode, E>; the gradient lies in the mode's image."""
    g = S.rng(1320 + len(mode))
    n, d = 3, 8
    T = S.ginibre(g, d)
    psi = S.haar_vector(g, d)
    f = S.multinomial_freqs(g, 5000, O.probs_real(S.depolarised_pure(psi, 0.2)))
    grad, L = O.grad_T_mode(T, f, mode)
    assert L == O.loss_of_T(O.premap(T, mode), f)
    h = 1e-5 * np.linalg.norm(T)
    for E in S.unit_directions(g, d, 6):
        fd = (O.loss_of_T(O.premap(T + h * E, mode), f) - O.loss_of_T(O.premap(T - h * E, mode), f)) / (2 * h)
        assert abs(fd - re_inner(grad, E)) <= 1e-6 * np.linalg.norm(grad) + 1e-12
    if mode == "hermitian":
        assert np.max(np.abs(grad - grad.conj().T)) <= 1e-15 * np.max(np.abs(grad)) * 10
    else:
        assert np.all(np.triu(grad, 1) == 0)


# --------------------------------------------------------------------------
# Mapping network (Sec. 3.1)
# --------------------------------------------------------------------------

def test_fnn_fill_definition_and_adjoint():
    """fill: entrywise T_ij = Y_ij + i Y_ji (i > j), conjugate above, Y_ii on
    the diagonal; Hermitian; a bijection (Y recovered from T); unfill is its
    adjoint for Re Tr(A^dagger B)."""
    g = S.rng(1400)
    d = 8
    y = g.standard_normal(d * d)
    Y = y.reshape(d, d)
    T = O.fnn_fill(y, d)
    for i in range(d):
        for j in range(d):
            if i > j:
                assert T[i, j] == Y[i, j] + 1j * Y[j, i]
            elif i < j:
                assert T[i, j] == Y[j, i] - 1j * Y[i, j]
            else:
                assert T[i, j] == Y[i, i]
    assert np.array_equal(T, T.conj().T)
    rec = np.tril(T.real) + np.triu(-T.imag, 1)  # Y from T
    assert np.array_equal(rec, Y)
    G = S.ginibre(g, d)
    a = float(np.sum(T.real * G.real + T.imag * G.imag))
    b = float(np.dot(y, O.fnn_unfill(G)))
    assert abs(a - b) <= 1e-13 * (abs(a) + 1.0)


def test_fnn_backward_central_differences():
    """L(fill(FNN(W1, b1, W2, b2; x))) by central differences along random
    directions in each parameter against the oracle's backward."""
    g = S.rng(1410)
    n, d = 2, 4
    D, H = 4 ** n, 2 * n
    x = S.porter_thomas_probs(g, D, 0.2)
    psi = S.haar_vector(g, d)
    f = S.multinomial_freqs(g, 4000, O.probs_real(S.depolarised_pure(psi, 0.2)))
    W1, b1 = g.standard_normal((H, D)), g.standard_normal(H)
    W2, b2 = g.standard_normal((D, H)) / 3, g.standard_normal(D) / 3
    params = [W1, b1, W2, b2]

    def loss(ps):
        T, _, _ = O.fnn_forward(*ps, x)
        return O.loss_of_T(T, f)

    T, h_pre, _ = O.fnn_forward(W1, b1, W2, b2, x)
    assert np.all(np.abs(h_pre) > 1e-3)  # away from the kink
    G, _ = O.grad_T(T, f)
    grads = O.fnn_backward(W2, x, h_pre, G)
    for k in range(4):
        for _ in range(3):
            E = g.standard_normal(params[k].shape)
            E /= np.linalg.norm(E)
            h = 1e-6
            plus = [p + (h * E if i == k else 0) for i, p in enumerate(params)]
            minus = [p - (h * E if i == k else 0) for i, p in enumerate(params)]
            fd = (loss(plus) - loss(minus)) / (2 * h)
            an = float(np.sum(grads[k] * E))
            assert abs(fd - an) <= 1e-6 * max(1.0, np.linalg.norm(grads[k])), (k, fd, an)
    assert np.array_equal(O.leaky_relu(np.array([-2.0, 0.0, 3.0])), np.array([-0.02, 0.0, 3.0]))


def test_rprop_step_matches_the_library_optimiser():
    """The oracle's Rprop against torch.optim.Rprop (CPU, float64) over a
    few steps with sign changes, and the rule's special cases by hand."""
    torch = pytest.importorskip("torch")
    g = S.rng(1500)
    w0 = g.standard_normal(50)
    p = torch.nn.Parameter(torch.from_numpy(w0.copy()))
    opt = torch.optim.Rprop([p], lr=1e-3)
    w, prev, step = w0.copy(), np.zeros(50), np.full(50, 1e-3)
    for k in range(6):
        grad = g.standard_normal(50) * (1 if k % 2 else -1)
        grad[:5] = 0.0
        p.grad = torch.from_numpy(grad.copy())
        opt.step()
        w, prev, step = O.rprop_step(w, grad, prev, step)
        np.testing.assert_allclose(p.detach().numpy(), w, rtol=0, atol=1e-15)
    # by hand: agreement grows the step, disagreement shrinks it and holds w
    w1, pr1, st1 = O.rprop_step(np.array([1.0, 1.0, 1.0]), np.array([2.0, -2.0, 3.0]),
                                np.array([1.0, 1.0, 0.0]), np.array([0.1, 0.1, 0.1]))
    np.testing.assert_allclose(st1, [0.12, 0.05, 0.1])
    np.testing.assert_allclose(w1, [0.88, 1.0, 0.9])
    np.testing.assert_allclose(pr1, [2.0, 0.0, 3.0])


# --------------------------------------------------------------------------
# General product POVMs: K outcomes per qubit, a POVM of its own on each
# qubit, several settings (Sec. 3.3; Sec. 2.1, one POVM per measurement;
# the multiple-POVM remark of the Sec. 4.1 setup)
# --------------------------------------------------------------------------

def random_povm(g, K):
    return S.random_povm(g, K)


def tr2(M, rho):
    """Tr(M rho) of 2 x 2 matrices, written out entry by entry."""
    return M[0, 0] * rho[0, 0] + M[0, 1] * rho[1, 0] + M[1, 0] * rho[0, 1] + M[1, 1] * rho[1, 1]


@pytest.mark.parametrize("n,K", [(1, 2), (2, 3), (3, 6), (4, 3), (3, 2)])
def test_general_povm_contraction_equals_kronecker(n, K):
    """Distinct random K-element POVMs per qubit: the per-qubit contraction
    (probs, adjoint) against explicit Kronecker products (probs_kron,
    adjoint_kron) on a random Hermitian matrix and a random real vector."""
    g = S.rng(9000 + 10 * n + K)
    povms = np.array([random_povm(g, K) for _ in range(n)])
    for M in povms:
        assert np.abs(M.sum(axis=0) - np.eye(2)).max() <= 1e-14
        assert min(np.linalg.eigvalsh(m).min() for m in M) > 0
    d = 1 << n
    X = S.ginibre(g, d)
    X = X + X.conj().T
    assert np.max(np.abs(O.probs(X, povms) - O.probs_kron(X, povms))) <= 1e-13
    y = g.standard_normal(K ** n)
    assert np.max(np.abs(O.adjoint(y, n, povms) - O.adjoint_kron(y, n, povms))) <= 1e-13


@pytest.mark.parametrize("n", [3, 5])
def test_general_povm_product_state_closed_form(n):
    """rho = (x)_i rho_i with distinct Bloch vectors (r_y != 0) and a distinct
    K = 3 POVM per qubit: p_k = prod_i Tr(M^(i)_{k_i} rho_i), each factor a
    2 x 2 trace written out.  A wrong qubit order, outcome order, pairing of
    M with rho, or one qubit's POVM applied to another fails it."""
    g = S.rng(9100 + n)
    K = 3
    povms = np.array([random_povm(g, K) for _ in range(n)])
    r = g.standard_normal((n, 3))
    r = 0.9 * r / np.linalg.norm(r, axis=1, keepdims=True)
    states = [bloch_state(ri) for ri in r]
    rho = kron_all(states)
    want = np.array([np.prod([tr2(povms[i][ks[i]], states[i]) for i in range(n)])
                     for ks in itertools.product(range(K), repeat=n)]).real
    p = O.probs_real(rho, povms)
    assert np.max(np.abs(p - want)) <= 1e-15
    assert abs(math.fsum(p.tolist()) - 1.0) <= 1e-14


def test_pauli6_trine_and_basis_closed_forms():
    """Textbook POVMs with known outcome laws:
    * Pauli-6 (K = 6), M_{+-j} = (I +- sigma_j)/6: p = prod_i (1 +- r_{i,j})/6;
    * trine (K = 3), M_k = (2/3)|psi_k><psi_k| with Bloch vectors
      (sin t_k, 0, cos t_k), t_k = 2 pi k / 3: p = prod_i (1 + n_k . r_i)/3;
    * computational basis (K = 2), M_b = |b><b|: p_k = rho_kk for any rho
      (k read as the binary row index, qubit 1 most significant)."""
    g = S.rng(9200)
    n = 3
    r = g.standard_normal((n, 3))
    r = 0.8 * r / np.linalg.norm(r, axis=1, keepdims=True)
    rho = kron_all([bloch_state(ri) for ri in r])
    X, Y, Z = (np.array([[0, 1], [1, 0]], dtype=complex), np.array([[0, -1j], [1j, 0]]),
               np.array([[1, 0], [0, -1]], dtype=complex))
    I2 = np.eye(2, dtype=complex)
    pauli6 = np.array([(I2 + X) / 6, (I2 - X) / 6, (I2 + Y) / 6, (I2 - Y) / 6, (I2 + Z) / 6, (I2 - Z) / 6])
    law6 = lambda k, ri: (1 + (1 - 2 * (k % 2)) * ri[k // 2]) / 6.0  # noqa: E731
    want = np.array([np.prod([law6(ks[i], r[i]) for i in range(n)]) for ks in itertools.product(range(6), repeat=n)])
    assert np.max(np.abs(O.probs_real(rho, pauli6) - want)) <= 1e-15
    ts = [2 * math.pi * k / 3 for k in range(3)]
    trine = np.array([(2.0 / 3.0) * np.outer(v, v) for v in
                      (np.array([math.cos(t / 2), math.sin(t / 2)], dtype=complex) for t in ts)])
    nk = [np.array([math.sin(t), 0.0, math.cos(t)]) for t in ts]
    want = np.array([np.prod([(1 + nk[ks[i]] @ r[i]) / 3.0 for i in range(n)])
                     for ks in itertools.product(range(3), repeat=n)])
    assert np.max(np.abs(O.probs_real(rho, trine) - want)) <= 1e-15
    basis = np.array([np.diag([1.0, 0.0]), np.diag([0.0, 1.0])]).astype(complex)
    m = 6
    R, _ = O.state_map(S.ginibre(g, 1 << m))
    assert np.max(np.abs(O.probs_real(R, basis) - np.diag(R).real)) <= 1e-15


def test_general_adjoint_dot_product():
    """<A(X), y> = Re Tr(X A^dagger(y)) for the per-qubit K = 6 map at N = 5
    (the adjoint is the transpose of the forward contraction)."""
    g = S.rng(9300)
    n, K = 5, 6
    povms = np.array([random_povm(g, K) for _ in range(n)])
    X = S.ginibre(g, 1 << n)
    X = X + X.conj().T
    y = g.standard_normal(K ** n)
    lhs = float(np.dot(O.probs(X, povms).real, y))
    rhs = float(np.trace(X @ O.adjoint(y, n, povms)).real)
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


@pytest.mark.parametrize("n", [3, 5])
def test_settings_gradient_central_differences(n):
    """Three settings (K = 2, 3, 6, a random POVM per qubit in each) summed in
    the loss: the gradient of grad_T_settings against central differences
    of likelihood_settings on random complex directions, and each setting's
    p against the single-setting route."""
    g = S.rng(9400 + n)
    d = 1 << n
    T = S.ginibre(g, d)
    settings = [np.array([random_povm(g, K) for _ in range(n)]) for K in (2, 3, 6)]
    target, _ = O.state_map(S.ginibre(g, d, 2))
    fs = [S.multinomial_freqs(g, 20_000, O.probs_real(target, pv)) for pv in settings]
    grad, L = O.grad_T_settings(T, fs, settings)
    assert L == pytest.approx(math.fsum(O.likelihood(T, f, pv)[0] for f, pv in zip(fs, settings)), rel=1e-14)
    h = 1e-6
    for _ in range(4):
        E = S.ginibre(g, d)
        E /= np.linalg.norm(E)
        fd = (O.likelihood_settings(T + h * E, fs, settings)[0]
              - O.likelihood_settings(T - h * E, fs, settings)[0]) / (2 * h)
        an = float(np.sum(grad.real * E.real + grad.imag * E.imag))
        assert abs(fd - an) <= 1e-7 * np.linalg.norm(grad)
