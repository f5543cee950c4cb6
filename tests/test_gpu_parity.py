"""GPU parity: the HIP path (through the C ABI, via the thin binding) against
the FP64 CPU oracle on identical seeded inputs.

Tolerances (relative): FP64 1e-12, FP32 1e-5, BF16 T T^dagger 2e-3, FP32 with
split-bf16 products (f32x6) 1e-5.
  p:    max|dp| / max|p|        L: |dL| / |L|       grad: ||dgrad||_F / ||grad||_F
  rho:  max|drho| / max|rho|
For FP32 / BF16 the oracle consumes the same complex64 / float32 values,
widened exactly to FP64.
"""
import math

import numpy as np
import pytest

import oracle as O
import synth as S
from workloads import config1, config2, config3, rel_fro, rel_max, depolarised_case

torch = pytest.importorskip("torch")
qst = pytest.importorskip("paper_2207_05341_amd")

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-3, "f32x6": 1e-5}
DEV = "cuda:0"


def ctype(prec):
    return np.complex128 if prec == "f64" else np.complex64


def rtype(prec):
    return np.float64 if prec == "f64" else np.float32


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)


def run_chain(T, f, prec, recompute=False, povm=None, f_from_forward=True):
    """Forward and backward through the C ABI; returns numpy (rho, tau, p, L, grad)."""
    Tg = to_dev(T.astype(ctype(prec)))
    fg = to_dev(f.astype(rtype(prec)))
    rho, tau = qst.state_map(Tg, prec)
    p = qst.povm_probs(rho, prec, povm)
    out, bad = qst.nll(p, fg, prec)
    grad = qst.nll_backward(Tg, fg, None if recompute else p, None if recompute else tau, prec, povm,
                            nll_out=out if f_from_forward else None)
    torch.cuda.synchronize()
    return host(rho), float(tau.item()), host(p).astype(np.float64), float(out[0].item()), host(grad), host(bad)


def oracle_chain(T, f, povm=None):
    rho, tau = O.state_map(T)
    n = O.n_qubits_of(T.shape[0])
    p = O.probs_real(rho, povm)
    L = O.nll_vec(p, f)
    G = O.adjoint(O.cotangent(p, f), n, povm)
    grad = (2.0 / tau) * (G @ T)
    return rho, tau, p, L, grad


def bf16_round(x):
    re = torch.from_numpy(np.ascontiguousarray(x.real.astype(np.float32))).to(torch.bfloat16).double().numpy()
    im = torch.from_numpy(np.ascontiguousarray(x.imag.astype(np.float32))).to(torch.bfloat16).double().numpy()
    return re + 1j * im


def bf16_split(x):
    """hi + lo with hi = bf16(x), lo = bf16(x - hi) (x given in fp32)."""
    x = x.astype(np.complex64).astype(np.complex128)
    hi = bf16_round(x)
    return hi + bf16_round((x - hi).astype(np.complex64).astype(np.complex128))


# ---------------------------------------------------------------------------
# Per-step parity at sizes the oracle finishes in seconds (several tiles,
# several passes, single-tile and small-matrix paths)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f32x6"])
@pytest.mark.parametrize("n", [1, 3, 5, 6, 7, 8, 9, 10])
def test_state_map(n, prec):
    say(f"state_map n={n} prec={prec}")
    g = S.rng(2000 + n)
    d = 1 << n
    T = S.ginibre(g, d).astype(ctype(prec)).astype(np.complex128)
    rho, tau = qst.state_map(to_dev(T.astype(ctype(prec))), prec)
    rho, tau = host(rho), float(tau.item())
    want_rho, want_tau = O.state_map(T)
    if prec == "bf16":
        # tau is the FP64 sum over the same represented T that the product
        # uses: bf16(T) for d >= 256, bf16 hi + lo below
        rep = bf16_round(T) if d >= 256 else bf16_split(T)
        assert abs(tau - O.trace_tt(rep)) <= 1e-12 * tau
    else:
        assert abs(tau - want_tau) <= 1e-12 * want_tau
    assert rel_max(rho, want_rho) <= TOL[prec]
    assert np.max(np.abs(rho - rho.conj().T)) <= TOL[prec] * np.max(np.abs(want_rho))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 2, 4, 6, 7, 8, 10])
def test_povm_probs(n, prec):
    """POVM map alone, fed the oracle's rho (upper triangle filled with junk
    to prove only the lower triangle is read)."""
    say(f"povm_probs n={n} prec={prec}")
    g = S.rng(2100 + n)
    d = 1 << n
    rho, _ = O.state_map(S.ginibre(g, d))
    rho_c = rho.astype(ctype(prec))
    junk = rho_c.copy()
    iu = np.triu_indices(d, 1)
    junk[iu] = 1e3 + 7j
    p = host(qst.povm_probs(to_dev(junk), prec)).astype(np.float64)
    want = O.probs_real(rho_c.astype(np.complex128))
    assert rel_max(p, want) <= TOL[prec]
    assert abs(math.fsum(p.tolist()) - 1.0) <= (1e-12 if prec == "f64" else 1e-4)


@pytest.mark.parametrize("n", [3, 7, 10, 12])
def test_povm_closed_forms(n):
    """Product state with distinct Bloch vectors (r_y != 0) and GHZi, FP64:
    p against the closed forms (no oracle involved)."""
    say(f"closed forms n={n}")
    g = S.rng(2200 + n)
    r = g.standard_normal((n, 3))
    r = 0.9 * r / np.linalg.norm(r, axis=1, keepdims=True)
    rho = np.ones((1, 1), dtype=np.complex128)
    for ri in r:
        x, y, z = ri
        rho = np.kron(rho, 0.5 * np.array([[1 + z, x - 1j * y], [x + 1j * y, 1 - z]]))
    p = host(qst.povm_probs(to_dev(rho), "f64"))
    # closed form prod_i (1 + s_{k_i} . r_i)/4 as an outer product over qubits
    factors = [(1.0 + O.TETRA_S @ ri) / 4.0 for ri in r]
    want = factors[0]
    for fct in factors[1:]:
        want = np.multiply.outer(want, fct).ravel()
    assert rel_max(p, want) <= 1e-12
    psi = S.ghzi(n)
    p = host(qst.povm_probs(to_dev(np.outer(psi, psi.conj())), "f64"))
    M = O.tetrahedral_povm()
    a00 = M[:, 0, 0].real
    a11 = M[:, 1, 1].real
    a01 = M[:, 0, 1]
    P00, P11, P01 = a00, a11, a01
    for _ in range(n - 1):
        P00 = np.multiply.outer(P00, a00).ravel()
        P11 = np.multiply.outer(P11, a11).ravel()
        P01 = np.multiply.outer(P01, a01).ravel()
    want = 0.5 * (P00 + P11) - P01.imag
    assert rel_max(p, want) <= 1e-12


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_nll_and_edge_cases(prec):
    say(f"nll prec={prec}")
    g = S.rng(2300)
    n = 6
    rho, _ = O.state_map(S.ginibre(g, 1 << n))
    p = O.probs_real(rho).astype(rtype(prec))
    f = S.multinomial_freqs(g, 3000, p.astype(np.float64)).astype(rtype(prec))
    out, bad = qst.nll(to_dev(p), to_dev(f), prec)
    want = O.nll_vec(p.astype(np.float64), f.astype(np.float64))
    # FP32 storage: each ln p_k is taken in FP32 (within 2 ulp), the sum in FP64
    assert abs(out[0].item() - want) <= (1e-13 if prec == "f64" else 3e-7) * abs(want)
    assert abs(out[1].item() - math.fsum(f.astype(np.float64).tolist())) <= 1e-13
    assert host(bad).tolist() == [0, 0]
    # f = 0 everywhere: L = 0, F = 0
    out, bad = qst.nll(to_dev(p), to_dev(np.zeros_like(f)), prec)
    assert out[0].item() == 0.0 and out[1].item() == 0.0
    # p <= 0 where f > 0: L = +inf and counted; f = 0 there: ignored
    p2 = p.copy()
    k = int(np.argmax(f))
    p2[k] = 0.0
    p2[k + 1] = -1e-3
    f2 = f.copy()
    f2[k + 1] = 0.0
    out, bad = qst.nll(to_dev(p2), to_dev(f2), prec)
    assert math.isinf(out[0].item()) and out[0].item() > 0
    assert host(bad).tolist() == [1, 0]
    p3 = p.copy()
    p3[3] = np.nan
    out, bad = qst.nll(to_dev(p3), to_dev(f), prec)
    assert math.isnan(out[0].item()) and host(bad)[1] == 1


# ---------------------------------------------------------------------------
# Whole chain, forward and adjoint
# ---------------------------------------------------------------------------

def check_chain(T, f, prec, povm=None, recompute=False):
    Tq = T.astype(ctype(prec)).astype(np.complex128)
    fq = f.astype(rtype(prec)).astype(np.float64)
    rho, tau, p, L, grad, bad = run_chain(T, f, prec, recompute, povm)
    w_rho, w_tau, w_p, w_L, w_grad = oracle_chain(Tq, fq, povm)
    errs = {"rho": rel_max(rho, w_rho), "p": rel_max(p, w_p), "L": abs(L - w_L) / abs(w_L),
            "grad": rel_fro(grad, w_grad)}
    say(f"  errors {errs} (grad max-entry {rel_max(grad, w_grad):.2e})")
    tol = TOL[prec]
    for k, v in errs.items():
        assert v <= tol, (k, v, tol)
    assert bad.tolist() == [0, 0]
    return errs


def test_config1_n4_f64():
    say("config 1: N=4 FP64")
    T, f, _ = config1()
    check_chain(T, f, "f64")


@pytest.mark.parametrize("r", [1, 4, 16, 256])
def test_config2_n8_f32(r):
    say(f"config 2: N=8 FP32 rank {r}")
    T, f, _ = config2(r)
    check_chain(T, f, "f32")


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f32x6"])
@pytest.mark.parametrize("n", [2, 5, 6, 7, 8, 9, 10])
def test_chain_sizes(n, prec):
    say(f"chain n={n} prec={prec}")
    T, f, _ = depolarised_case(n, 2400 + n, 0.1, 20 * 4 ** n)
    check_chain(T, f, prec)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [3, 8])
def test_general_povm(n, prec):
    """A non-tetrahedral POVM: the tetrahedron rotated by a random SU(2)
    element (still Hermitian PSD elements summing to I), generic kernels."""
    say(f"general povm n={n} prec={prec}")
    g = S.rng(2500 + n)
    U, _ = np.linalg.qr(S.ginibre(g, 2))
    M = np.array([U @ m @ U.conj().T for m in O.tetrahedral_povm()])
    T, f, _ = depolarised_case(n, 2510 + n, 0.2, 20 * 4 ** n)
    check_chain(T, f, prec, povm=M)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f32x6"])
def test_recompute_equals_stored_and_determinism(prec):
    say(f"recompute / determinism prec={prec}")
    T, f, _ = depolarised_case(9, 2600, 0.05, 10 ** 6)
    a = run_chain(T, f, prec, recompute=False)
    b = run_chain(T, f, prec, recompute=True)
    c = run_chain(T, f, prec, recompute=False)
    e = run_chain(T, f, prec, recompute=False, f_from_forward=False)
    assert np.array_equal(a[4], b[4])  # gradient bitwise identical
    assert np.array_equal(a[4], e[4])  # F from the forward NLL == F reduced in the backward
    for x, y in zip(a, c):
        if isinstance(x, np.ndarray):
            assert np.array_equal(x, y)
        else:
            assert x == y


def test_leading_dimension_and_upstream():
    """T stored with row stride > d, and an upstream gradient scale."""
    say("ld / upstream")
    n, d = 7, 128
    T, f, _ = depolarised_case(n, 2700, 0.1, 10 ** 5)
    big = np.zeros((d, d + 40), dtype=np.complex128)
    big[:, :d] = T
    Tg = to_dev(big)[:, :d]
    assert Tg.stride(0) == d + 40
    fg = to_dev(f)
    rho, tau = qst.state_map(Tg, "f64")
    p = qst.povm_probs(rho, "f64")
    up = torch.tensor([-2.5], dtype=torch.float64, device=DEV)
    grad = host(qst.nll_backward(Tg, fg, p, tau, "f64", None, up))
    w = oracle_chain(T, f)
    assert rel_max(host(rho), w[0]) <= 1e-12
    assert rel_fro(grad, -2.5 * w[4]) <= 1e-12


def test_autograd_function():
    say("autograd")
    T, f, _ = config1()
    Tg = to_dev(T).requires_grad_(True)
    L = qst.likelihood(Tg, to_dev(f))
    (3.0 * L).backward()
    w = oracle_chain(T, f)
    assert abs(L.item() - w[3]) <= 1e-12 * abs(w[3])
    assert rel_fro(host(Tg.grad), 3.0 * w[4]) <= 1e-12


def test_fd_directions_n8_f32():
    """Config 2: central finite differences of the FP64 oracle loss on 64
    random complex directions against the FP32 GPU directional derivative."""
    say("finite differences N=8 FP32, 64 directions")
    T, f, _ = config2(16)
    T32 = T.astype(np.complex64)
    f32 = f.astype(np.float32)
    Tq, fq = T32.astype(np.complex128), f32.astype(np.float64)
    grad = run_chain(T32, f32, "f32")[4].astype(np.complex128)
    g = S.rng(2800)
    h = 1e-6 * np.linalg.norm(Tq)
    gnorm = np.linalg.norm(grad)
    worst = 0.0
    for E in S.unit_directions(g, 256, 64):
        fd = (O.loss_of_T(Tq + h * E, fq) - O.loss_of_T(Tq - h * E, fq)) / (2 * h)
        an = float(np.sum(grad.real * E.real + grad.imag * E.imag))
        worst = max(worst, abs(fd - an) / gnorm)
    say(f"  worst |fd - <grad,E>| / ||grad|| = {worst:.3e}")
    assert worst <= 1e-5


# ---------------------------------------------------------------------------
# N = 11 (4,194,304 outcomes), the measured workload, all three precisions
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module", params=[0.0, 0.05, 0.1], ids=["q0", "q0.05", "q0.1"])
def n11(request):
    """Config 3 at each depolarising level: q = 0 is the pure target, with
    about 29% of the 4^11 frequencies zero (the f_k = 0 branch of the NLL and
    the cotangent at full size)."""
    say(f"building N=11 inputs (q = {request.param}) and FP64 oracle results")
    T, f, _ = config3(request.param)
    say(f"  zero frequencies: {float(np.mean(f == 0)):.3f}")
    return T, f, oracle_chain(T, f)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f32x6"])
def test_config3_n11(n11, prec):
    say(f"config 3: N=11 {prec}")
    T, f, w = n11
    if prec != "f64":
        Tq = T.astype(np.complex64).astype(np.complex128)
        fq = f.astype(np.float32).astype(np.float64)
        w = oracle_chain(Tq, fq)
    rho, tau, p, L, grad, bad = run_chain(T, f, prec)
    errs = {"rho": rel_max(rho, w[0]), "p": rel_max(p, w[2]), "L": abs(L - w[3]) / abs(w[3]),
            "grad": rel_fro(grad, w[4])}
    say(f"  errors {errs}")
    for k, v in errs.items():
        assert v <= TOL[prec], (k, v)
    assert bad.tolist() == [0, 0]
