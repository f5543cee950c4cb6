"""Parity at the largest sizes, through the C ABI.

* N = 12 (T 4096 x 4096, 16,777,216 outcomes; the training workload's size):
  every output of the separate-call path and of qst_likelihood /
  qst_grad_product against the full FP64 oracle, all three precisions.
* N = 13 (the largest N the library accepts: T 8192 x 8192, 67,108,864
  outcomes), where the full oracle is too slow for a test:
  - p_k on sampled outcomes, each evaluated one by one by the oracle from a
    thin factor W of T T^dagger (T = W Q^dagger, Q with orthonormal columns);
  - tau against Tr(W W^dagger);
  - the exact invariances of the gradient: L(c T) = L(T) for real c > 0 and
    L(e^{i phi} T) = L(T) give sum_ij conj(grad_ij) T_ij = 0 (real and
    imaginary parts), which holds only if G' is the adjoint of the forward
    map (sum_k (F - f_k/p_k) p_k = 0), up to the error of the computed p;
  - FP64: central differences of the library's own FP64 forward along
    random directions against <grad, E>;
  - the fused and separate-call paths agree.

Tolerances (relative) as in the other parity tests: FP64 1e-12, FP32 1e-5,
BF16 T T^dagger 2e-3.
"""
import numpy as np
import pytest

import oracle as O
import synth as S
from workloads import rel_fro, rel_max

torch = pytest.importorskip("torch")
qst = pytest.importorskip("paper_2207_05341_amd")

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5, "bf16": 2e-3, "f32x6": 1e-5}
DEV = "cuda:0"
RANK = 8


def say(*a):
    print(*a, flush=True)


def ctype(prec):
    return np.complex128 if prec == "f64" else np.complex64


def rtype(prec):
    return np.float64 if prec == "f64" else np.float32


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def inputs(n, seed):
    g = S.rng(seed)
    T, W = S.thin_factor_square(g, 1 << n, RANK)
    f = S.porter_thomas_probs(g, 4 ** n, 0.05)
    return g, T, W, f


# ---------------------------------------------------------------------------
# N = 12: full oracle
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def n12():
    say("building N=12 inputs")
    _, T, _, f = inputs(12, 4312)
    return T, f, {}


def oracle_full(T, f):
    rho, tau = O.state_map(T)
    p = O.probs_real(rho)
    L = O.nll_vec(p, f)
    G = O.adjoint(O.cotangent(p, f), 12)
    return rho, tau, p, L, G, (2.0 / tau) * (G @ T)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f32x6"])
def test_n12_against_full_oracle(n12, prec):
    T, f, cache = n12
    key = "f64" if prec == "f64" else "f32"
    if key not in cache:
        say(f"  FP64 oracle on the {key} inputs (N=12)")
        Tq = T.astype(ctype(key)).astype(np.complex128)
        fq = f.astype(rtype(key)).astype(np.float64)
        cache[key] = oracle_full(Tq, fq)
    w_rho, w_tau, w_p, w_L, w_G, w_grad = cache[key]
    say(f"N=12 {prec}: separate-call path")
    Tg, fg = to_dev(T.astype(ctype(prec))), to_dev(f.astype(rtype(prec)))
    rho, tau = qst.state_map(Tg, prec)
    e_rho = rel_max(host(rho), w_rho)
    p = qst.povm_probs(rho, prec)
    del rho
    out, bad = qst.nll(p, fg, prec)
    grad = qst.nll_backward(Tg, fg, p, tau, prec, nll_out=out)
    torch.cuda.synchronize()
    errs = {"rho": e_rho, "p": rel_max(host(p).astype(np.float64), w_p),
            "L": abs(float(out[0].item()) - w_L) / abs(w_L), "grad": rel_fro(host(grad), w_grad)}
    assert host(bad).tolist() == [0, 0]
    del p, grad
    say(f"N=12 {prec}: qst_likelihood + qst_grad_product")
    out2, tau2, G, bad2 = qst.likelihood_forward(Tg, fg, prec)
    grad2 = qst.grad_product(G, Tg, tau2, prec)
    torch.cuda.synchronize()
    errs.update({"L_fused": abs(float(out2[0].item()) - w_L) / abs(w_L), "G_fused": rel_fro(host(G), w_G),
                 "grad_fused": rel_fro(host(grad2), w_grad)})
    say(f"  errors {errs}")
    for k, v in errs.items():
        assert v <= TOL[prec], (k, v)
    if prec != "bf16":
        assert abs(float(tau.item()) - w_tau) <= 1e-12 * w_tau
    assert host(bad2).tolist() == [0, 0]


# ---------------------------------------------------------------------------
# N = 13: sampled outcomes, invariants, central differences
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def n13():
    say("building N=13 inputs and sampled oracle probabilities")
    n, D = 13, 4 ** 13
    g, T, W, f = inputs(n, 4313)
    ks = [0, D - 1, (D - 1) // 3, 2 * ((D - 1) // 3)]  # all digits 0, 3, 1, 2
    ks += [int(k) for k in g.integers(0, D, 252)]
    p_w = O.probs_at(W, [O.outcome_digits(k, n) for k in ks])
    return T, f, np.asarray(ks, dtype=np.int64), p_w, O.trace_tt(W)


def inner(a, b):
    """sum_ij conj(a_ij) b_ij in complex128 (test-side arithmetic)."""
    return complex(torch.sum(torch.conj(a.to(torch.complex128)) * b.to(torch.complex128)).item())


def fro(a):
    return float(torch.linalg.vector_norm(a.to(torch.complex128)).item())


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16", "f32x6"])
def test_n13_sampled_outcomes_and_invariants(n13, prec):
    T, f, ks, p_w, tau_w = n13
    say(f"N=13 {prec}: separate-call path, {len(ks)} sampled outcomes")
    Tg, fg = to_dev(T.astype(ctype(prec))), to_dev(f.astype(rtype(prec)))
    rho, tau = qst.state_map(Tg, prec)
    p = qst.povm_probs(rho, prec)
    del rho
    out, bad = qst.nll(p, fg, prec)
    grad_s = qst.nll_backward(Tg, fg, p, tau, prec, nll_out=out)
    p_s = host(p[torch.from_numpy(ks).to(DEV)]).astype(np.float64)
    torch.cuda.synchronize()
    del p
    e_p = float(np.max(np.abs(p_s - p_w)) / np.max(p_w))
    e_tau = abs(float(tau.item()) - tau_w) / tau_w
    say(f"  sampled p rel {e_p:.3e}  tau rel {e_tau:.3e}")
    assert e_p <= TOL[prec]
    # BF16: tau is the trace of the split operands the products use
    assert e_tau <= {"f64": 1e-12, "f32": 1e-6, "bf16": TOL["bf16"], "f32x6": 1e-6}[prec]
    assert host(bad).tolist() == [0, 0]

    say(f"N=13 {prec}: qst_likelihood + qst_grad_product")
    out2, tau2, G, bad2 = qst.likelihood_forward(Tg, fg, prec)
    grad = qst.grad_product(G, Tg, tau2, prec)
    G = None
    torch.cuda.synchronize()
    L_s, L_f = float(out[0].item()), float(out2[0].item())
    assert abs(L_f - L_s) <= TOL[prec] * abs(L_s)
    assert abs(float(out2[1].item()) - float(np.sum(f.astype(rtype(prec)).astype(np.float64)))) <= 1e-12
    assert host(bad2).tolist() == [0, 0]
    assert rel_fro(host(grad), host(grad_s)) <= TOL[prec]
    del grad_s
    # sum conj(grad) T = 2 sum_k (F - f_k/p_k) p_k^exact: a sum of terms whose
    # magnitudes add up to at most 2 (F sum p + sum f) = 4F, exactly 0 for
    # exact p; the computed p (relative error within TOL) leaves a residual
    # of order TOL * 4F.
    z = inner(grad, Tg)
    F = float(out2[1].item())
    say(f"  |sum conj(grad) T| / 4F = {abs(z) / (4 * F):.3e}"
        f"  (/ |grad||T|: {abs(z) / (fro(grad) * fro(Tg)):.3e})")
    assert abs(z) <= TOL[prec] * 4 * F

    if prec == "f64":
        gen = torch.Generator(device=DEV).manual_seed(4314)
        gn, tn = fro(grad), fro(Tg)
        h = 1e-4 * tn
        worst = 0.0
        for _ in range(3):
            E = torch.complex(torch.randn(Tg.shape, generator=gen, device=DEV, dtype=torch.float64),
                              torch.randn(Tg.shape, generator=gen, device=DEV, dtype=torch.float64))
            E /= fro(E)
            Lp = float(qst.likelihood_forward(Tg + h * E, fg, prec, with_grad_matrix=False)[0][0].item())
            Lm = float(qst.likelihood_forward(Tg - h * E, fg, prec, with_grad_matrix=False)[0][0].item())
            fd = (Lp - Lm) / (2 * h)
            an = inner(grad, E).real
            worst = max(worst, abs(fd - an) / gn)
            del E
        say(f"  central differences: worst |fd - <grad,E>| / |grad| = {worst:.3e}")
        assert worst <= 1e-5


def test_n13_one_call_f32x6(n13):
    """qst_likelihood_grad at N = 13 (plan 5, 4, 4: the gradient product's
    planes formed inside the call, pass 0 on 32 x 32 tiles) against the two
    calls: L, F and tau bitwise, the gradient to rounding."""
    T, f, ks, p_w, tau_w = n13
    say("N=13 f32x6: qst_likelihood_grad vs qst_likelihood + qst_grad_product")
    Tg, fg = to_dev(T.astype(np.complex64)), to_dev(f.astype(np.float32))
    out, tau, grad, bad = qst.likelihood_grad(Tg, fg, "f32x6")
    torch.cuda.synchronize()
    grad_h = host(grad)
    del grad
    out2, tau2, G, bad2 = qst.likelihood_forward(Tg, fg, "f32x6")
    grad2 = qst.grad_product(G, Tg, tau2, "f32x6")
    torch.cuda.synchronize()
    del G
    assert torch.equal(out, out2) and torch.equal(tau, tau2)
    e = rel_fro(grad_h, host(grad2))
    say(f"  grad rel {e:.2e}")
    assert e <= 1e-6
    assert host(bad).tolist() == [0, 0]
