"""The mapping network of Sec. 3.1 through the C ABI (qst_fnn_forward,
qst_fnn_backward) and through autograd, against the oracle's fnn_forward /
fnn_backward (pinned by the fill definition, its adjoint identity and
central differences through the whole loss).

* forward (T, h_pre) and backward (dW1, db1, dW2, db2 for a random dL/dT)
  at N = 1 .. 8 in both precisions; bitwise repeats;
* the whole NN-QST chain, network -> T -> likelihood, differentiated by
  autograd, against the oracle chain at N = 4 (FP64) and N = 8 (FP32);
* the Rprop step against the oracle and torch's Rprop; a short run lowers the
  loss; ten steps of the whole method against the oracle at N = 5.

Tolerances: FP64 1e-12, FP32 1e-5 (relative; Frobenius for matrices).
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


def params(g, n, rt):
    D, H = 4 ** n, 2 * n
    W1 = (g.uniform(-1, 1, (H, D)) / np.sqrt(D)).astype(rt)
    b1 = (g.uniform(-1, 1, H) / np.sqrt(D)).astype(rt)
    W2 = (g.uniform(-1, 1, (D, H)) / np.sqrt(H)).astype(rt)
    b2 = (g.uniform(-1, 1, D) / np.sqrt(H)).astype(rt)
    return W1, b1, W2, b2


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 2, 4, 6, 8])
def test_fnn_against_oracle(prec, n):
    say(f"network N={n} {prec}")
    rt = np.float64 if prec == "f64" else np.float32
    ct = np.complex128 if prec == "f64" else np.complex64
    g = S.rng(7500 + n)
    W1, b1, W2, b2 = params(g, n, rt)
    x = S.porter_thomas_probs(g, 4 ** n, 0.1).astype(rt)
    G = S.ginibre(g, 1 << n).astype(ct)
    T_w, hp_w, _ = O.fnn_forward(W1, b1, W2, b2, x)
    grads_w = O.fnn_backward(W2, x, hp_w, G.astype(np.complex128))
    Wg = [dev(a) for a in (W1, b1, W2, b2)]
    xg = dev(x)
    T, h_pre = qst.fnn_forward(*Wg, xg, prec)
    grads = qst.fnn_backward(Wg[2], xg, h_pre, dev(G), prec)
    T2, h_pre2 = qst.fnn_forward(*Wg, xg, prec)
    grads2 = qst.fnn_backward(Wg[2], xg, h_pre2, dev(G), prec)
    torch.cuda.synchronize()
    Tn = T.cpu().numpy()
    assert np.array_equal(Tn, Tn.conj().T)
    errs = {"T": rel_fro(Tn, T_w), "h_pre": rel_fro(h_pre.cpu().numpy(), hp_w)}
    for name, a, w in zip(("dW1", "db1", "dW2", "db2"), grads, grads_w):
        errs[name] = rel_fro(a.cpu().numpy(), w)
    say(f"  {errs}")
    for k, v in errs.items():
        assert v <= TOL[prec], (k, v)
    assert torch.equal(T, T2) and all(torch.equal(a, b) for a, b in zip(grads, grads2))


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_fnn_n11_against_oracle(prec):
    """The network at N = 11, the size the bench measures (4^11 inputs and
    outputs, 22 hidden units, 184.5M parameters): T, h_pre and all four
    parameter gradients against the oracle."""
    test_fnn_against_oracle(prec, 11)


@pytest.mark.parametrize("prec,n", [("f64", 4), ("f32", 8), ("f32", 11)])
def test_network_chain_through_autograd(prec, n):
    """MappingNetwork -> T -> likelihood: autograd's parameter gradients
    against the oracle's chain (grad_T at the network's T, then
    fnn_backward)."""
    say(f"network + likelihood N={n} {prec}")
    rt = torch.float64 if prec == "f64" else torch.float32
    gen = torch.Generator().manual_seed(7600 + n)
    net = qst.MappingNetwork(n, dtype=rt, device=DEV, generator=gen)
    g = S.rng(7610 + n)
    d = 1 << n
    psi = S.haar_vector(g, d)
    f = S.multinomial_freqs(g, 100_000, O.probs_real(S.depolarised_pure(psi, 0.1)))
    fr = f.astype(np.float64 if prec == "f64" else np.float32)
    x = (fr / fr.sum()).astype(fr.dtype)
    fg, xg = dev(fr), dev(x)
    T = net(xg, prec)
    L = qst.likelihood(T, fg, prec)
    L.backward()
    torch.cuda.synchronize()
    P = [p.detach().cpu().numpy().astype(np.float64) for p in (net.W1, net.b1, net.W2, net.b2)]
    xw, fw = x.astype(np.float64), fr.astype(np.float64)
    T_w, hp_w, _ = O.fnn_forward(*P, xw)
    G_w, L_w = O.grad_T(T_w, fw)
    grads_w = O.fnn_backward(P[2], xw, hp_w, G_w)
    eL = abs(float(L.item()) - L_w) / abs(L_w)
    errs = {"L": eL}
    for name, p, w in zip(("dW1", "db1", "dW2", "db2"), (net.W1, net.b1, net.W2, net.b2), grads_w):
        errs[name] = rel_fro(p.grad.cpu().numpy(), w)
    say(f"  {errs}")
    for k, v in errs.items():
        assert v <= TOL[prec], (k, v)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_rprop_step_against_oracle(prec):
    """qst_rprop_step over six steps (sign agreements, disagreements and
    zero gradients) against the oracle's rule, and the Rprop class against
    torch.optim.Rprop on the same parameters."""
    rt = np.float64 if prec == "f64" else np.float32
    g = S.rng(7800)
    count = 100_003  # not a multiple of the block
    w0 = g.standard_normal(count).astype(rt)
    p = torch.nn.Parameter(dev(w0.copy()))
    q = torch.nn.Parameter(dev(w0.copy()))
    ours, ref = qst.Rprop([p], lr=1e-3), torch.optim.Rprop([q], lr=1e-3)
    w, prev, step = w0.astype(np.float64), np.zeros(count), np.full(count, rt(1e-3), dtype=np.float64)
    for k in range(6):
        grad = (g.standard_normal(count) * (1 if k % 2 else -1)).astype(rt)
        grad[k::7] = 0
        p.grad, q.grad = dev(grad.copy()), dev(grad.copy())
        ours.step()
        ref.step()
        w, prev, step = O.rprop_step(w, grad.astype(np.float64), prev, step)
    torch.cuda.synchronize()
    got = p.detach().cpu().numpy()
    tol = 1e-14 if prec == "f64" else 1e-6
    assert np.max(np.abs(got - w)) <= tol * np.max(np.abs(w))
    assert np.max(np.abs(got - q.detach().cpu().numpy())) <= tol * np.max(np.abs(w))


def test_rprop_lowers_the_loss():
    """The paper's optimiser (Rprop, lr 1e-3) on the network at N = 4."""
    n, d = 4, 16
    gen = torch.Generator().manual_seed(7700)
    net = qst.MappingNetwork(n, dtype=torch.float64, device=DEV, generator=gen)
    g = S.rng(7701)
    psi = S.haar_vector(g, d)
    f = S.multinomial_freqs(g, 100_000, O.probs_real(S.depolarised_pure(psi, 0.1)))
    fg = dev(f)
    xg = dev(f / f.sum())
    opt = qst.Rprop(net.parameters(), lr=1e-3)
    losses = []
    for _ in range(30):
        opt.zero_grad(set_to_none=True)
        L = qst.likelihood(net(xg), fg, "f64")
        L.backward()
        opt.step()
        losses.append(float(L.item()))
    say(f"  Rprop losses {losses[0]:.6f} -> {losses[-1]:.6f}")
    assert losses[-1] < losses[0]


def test_nnqst_trajectory_against_oracle():
    """Ten steps of the whole method at N = 5 in FP64 -- network, likelihood,
    backward, Rprop -- against the same steps by the oracle from the same
    initial parameters: losses and final parameters."""
    n, d = 5, 32
    gen = torch.Generator().manual_seed(7900)
    net = qst.MappingNetwork(n, dtype=torch.float64, device=DEV, generator=gen)
    g = S.rng(7901)
    psi = S.haar_vector(g, d)
    f = S.multinomial_freqs(g, 100_000, O.probs_real(S.depolarised_pure(psi, 0.1)))
    x = f / f.sum()
    fg, xg = dev(f), dev(x)
    P = [p.detach().cpu().numpy().copy() for p in (net.W1, net.b1, net.W2, net.b2)]
    prev = [np.zeros_like(p) for p in P]
    step = [np.full_like(p, 1e-3) for p in P]
    opt = qst.Rprop(net.parameters(), lr=1e-3)
    worst = 0.0
    for _ in range(10):
        opt.zero_grad(set_to_none=True)
        L = qst.likelihood(net(xg), fg, "f64")
        L.backward()
        opt.step()
        T, h_pre, _ = O.fnn_forward(*P, x)
        G, L_w = O.grad_T(T, f)
        grads = O.fnn_backward(P[2], x, h_pre, G)
        for k in range(4):
            P[k], prev[k], step[k] = O.rprop_step(P[k], grads[k], prev[k], step[k])
        worst = max(worst, abs(float(L.item()) - L_w) / abs(L_w))
    torch.cuda.synchronize()
    say(f"  worst loss difference {worst:.2e}")
    assert worst <= 1e-12
    for p, w in zip((net.W1, net.b1, net.W2, net.b2), P):
        assert rel_fro(p.detach().cpu().numpy(), w) <= 1e-12
