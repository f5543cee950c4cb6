"""The P-order absolute map of Sec. 3.2 (Eq. abs_P) through the C ABI
(qst_abs_map, qst_abs_map_backward) and through autograd, against the
oracle's abs_map / abs_map_backward / grad_T_abs (pinned by closed forms at
P = 0 and P = 4, scipy's fractional matrix powers and central differences).

* A = Q |Lambda|^(P/2) Q^dagger of the Hermitian part at N = 1 .. 8 and 10
  for P in {0.5, 1, 1.5, 2, 3, 4} (the paper's orders), both precisions,
  padded leading dimensions; the eigenpairs: Q unitary, Q Lambda Q^dagger =
  H, the spectrum against numpy's; bitwise repeats;
* dL/dT from a random dL/dA against the oracle's adjoint (independent of
  the eigenvector phases and order, which differ between the two);
* closed forms: P = 0 gives I, P = 4 gives H H; P = 2 through the whole
  likelihood equals the library's Chol_H mode; a diagonal T returns its
  diagonal exactly;
* the direct solver (cold calls) and the warm-started Jacobi solver agree;
  degenerate spectra (the cluster treatment) against the oracle;
* the whole chain T -> A -> likelihood differentiated by autograd against
  the oracle's grad_T_abs.

Tolerances: FP64 1e-12, FP32 1e-5 (relative Frobenius; the eigensolver and
the products run in FP64 on both paths, FP32 only rounds the storage).
"""
import time

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
ORDERS = (0.5, 1.0, 1.5, 2.0, 3.0, 4.0)


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
@pytest.mark.parametrize("n", [1, 2, 3, 5, 6, 8])
def test_abs_map_against_oracle(prec, n):
    d = 1 << n
    g = S.rng(8100 + n)
    T = S.ginibre(g, d).astype(ctype(prec))
    T64 = T.astype(np.complex128)
    H = O.hermitian_part(T64)
    Tg = dev_matrix(T, pad=3 if n % 2 else 0)
    lam_w = np.linalg.eigvalsh(H)
    for P in ORDERS:
        t0 = time.perf_counter()
        A, Q, lam, sweeps = qst.abs_map(Tg, P, prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        A_w = O.abs_map(T64, P)[0]
        An, Qn, ln = A.cpu().numpy(), Q.cpu().numpy(), lam.cpu().numpy()
        e = rel_fro(An, A_w)
        say(f"N={n} {prec} P={P}: sweeps {sweeps}, {1e3 * dt:.1f} ms, A rel err {e:.2e}")
        assert e <= TOL[prec], (P, e)
        assert np.abs(Qn.conj().T @ Qn - np.eye(d)).max() <= 1e-13 * d
        assert sweeps == 0  # the direct solver
        assert rel_fro((Qn * ln) @ Qn.conj().T, H) <= (1e-13 if prec == "f64" else 1e-9)
        assert np.abs(np.sort(ln) - lam_w).max() <= 1e-13 * np.abs(lam_w).max()
    A2 = qst.abs_map(Tg, 1.5, prec)[0]
    A3 = qst.abs_map(Tg, 1.5, prec)[0]
    assert torch.equal(A2, A3)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n", [1, 3, 6, 8])
def test_abs_map_backward_against_oracle(prec, n):
    d = 1 << n
    g = S.rng(8200 + n)
    T = S.ginibre(g, d).astype(ctype(prec))
    GA = S.ginibre(g, d).astype(ctype(prec))
    T64, GA64 = T.astype(np.complex128), GA.astype(np.complex128)
    _, Qw, lw = O.abs_map(T64, 1.0)
    Tg, GAg = dev_matrix(T), dev_matrix(GA, pad=5)
    for P in ORDERS:
        _, Q, lam, _ = qst.abs_map(Tg, P, prec)
        GT = qst.abs_map_backward(Q, lam, P, GAg, prec)
        GT2 = qst.abs_map_backward(Q, lam, P, GAg, prec)
        torch.cuda.synchronize()
        want = O.abs_map_backward(Qw, lw, P, GA64)
        e = rel_fro(GT.cpu().numpy(), want)
        say(f"N={n} {prec} P={P}: dL/dT rel err {e:.2e}")
        assert e <= TOL[prec], (P, e)
        assert torch.equal(GT, GT2)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_abs_map_closed_forms(prec):
    """P = 0: A = I; P = 4: A = H H; a diagonal T: lam = its real diagonal
    exactly (every reflector is the identity)."""
    g = S.rng(8300)
    n, d = 7, 128
    T = S.ginibre(g, d).astype(ctype(prec))
    H = O.hermitian_part(T.astype(np.complex128))
    Tg = dev_matrix(T)
    A0 = qst.abs_map(Tg, 0.0, prec)[0].cpu().numpy()
    assert np.abs(A0 - np.eye(d)).max() <= 10 * TOL[prec]
    A4 = qst.abs_map(Tg, 4.0, prec)[0].cpu().numpy()
    assert rel_fro(A4, H @ H) <= TOL[prec]
    D = np.diag(g.standard_normal(d) + 1j * g.standard_normal(d)).astype(ctype(prec))
    A, Q, lam, sweeps = qst.abs_map(dev_matrix(D), 2.0, prec)
    assert sweeps == 0
    assert np.array_equal(lam.cpu().numpy(), np.diag(D).real.astype(np.float64))
    assert rel_fro(A.cpu().numpy(), np.diag(np.abs(np.diag(D).real)).astype(np.complex128)) <= TOL[prec]


@pytest.mark.parametrize("prec,n,P", [("f64", 4, 1.5), ("f64", 5, 0.5), ("f32", 7, 3.0), ("f32", 8, 1.0)])
def test_abs_likelihood_through_autograd(prec, n, P):
    """T -> A (AbsMapFn) -> likelihood: L and autograd's dL/dT against the
    oracle's grad_T_abs."""
    d = 1 << n
    g = S.rng(8400 + n)
    T = S.ginibre(g, d).astype(ctype(prec))
    psi = S.haar_vector(g, d)
    f = S.multinomial_freqs(g, 100_000, O.probs_real(S.depolarised_pure(psi, 0.1)))
    rt = torch.float64 if prec == "f64" else torch.float32
    Tg = torch.from_numpy(T).to(DEV).requires_grad_(True)
    fg = torch.from_numpy(f).to(DEV, rt)
    L = qst.likelihood(Tg, fg, prec, state_map="abs", P=P)
    L.backward()
    torch.cuda.synchronize()
    grad_w, L_w = O.grad_T_abs(T.astype(np.complex128), f, P)
    eL = abs(float(L.item()) - L_w) / abs(L_w)
    eg = rel_fro(Tg.grad.cpu().numpy(), grad_w)
    say(f"N={n} {prec} P={P}: L rel err {eL:.2e}, grad rel err {eg:.2e}")
    assert eL <= TOL[prec] and eg <= TOL[prec]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_abs_p2_equals_chol_h(prec):
    """Eq. abs_P at P = 2 is Chol_H: the library's two routes agree in L
    and dL/dT."""
    n, d = 6, 64
    g = S.rng(8500)
    T = S.ginibre(g, d).astype(ctype(prec))
    psi = S.haar_vector(g, d)
    f = S.multinomial_freqs(g, 100_000, O.probs_real(S.depolarised_pure(psi, 0.1)))
    rt = torch.float64 if prec == "f64" else torch.float32
    fg = torch.from_numpy(f).to(DEV, rt)
    out = {}
    for mode in ("abs", "hermitian"):
        Tg = torch.from_numpy(T).to(DEV).requires_grad_(True)
        L = qst.likelihood(Tg, fg, prec, state_map=mode, P=2.0)
        L.backward()
        out[mode] = (float(L.item()), Tg.grad.cpu().numpy())
    (La, ga), (Lh, gh) = out["abs"], out["hermitian"]
    assert abs(La - Lh) <= TOL[prec] * abs(Lh)
    assert rel_fro(ga, gh) <= (TOL[prec] if prec == "f64" else 1e-4)


def test_abs_map_n10_against_oracle():
    """N = 10 (the paper's size for the comparison of maps), FP32 storage,
    P = 1.5: A and dL/dT against the oracle (the products on MFMA tiles with
    the stream-K schedule)."""
    n, d, P = 10, 1024, 1.5
    g = S.rng(8600)
    T = S.ginibre(g, d).astype(np.complex64)
    GA = S.ginibre(g, d).astype(np.complex64)
    T64 = T.astype(np.complex128)
    t0 = time.perf_counter()
    A, Q, lam, sweeps = qst.abs_map(dev_matrix(T), P, "f32")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    A_w, Qw, lw = O.abs_map(T64, P)
    e = rel_fro(A.cpu().numpy(), A_w)
    GT = qst.abs_map_backward(Q, lam, P, dev_matrix(GA), "f32")
    eg = rel_fro(GT.cpu().numpy(), O.abs_map_backward(Qw, lw, P, GA.astype(np.complex128)))
    say(f"N=10 f32 P={P}: sweeps {sweeps}, {dt:.2f} s, A rel err {e:.2e}, dL/dT rel err {eg:.2e}")
    assert e <= 1e-5 and eg <= 1e-5


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_abs_map_n11_against_oracle(prec):
    """N = 11 (d = 2048), P = 1.5: A, the spectrum and dL/dT for a random
    dL/dA against the oracle, in both storage precisions."""
    n, d, P = 11, 2048, 1.5
    g = S.rng(8650)
    T = S.ginibre(g, d).astype(ctype(prec))
    GA = S.ginibre(g, d).astype(ctype(prec))
    T64 = T.astype(np.complex128)
    t0 = time.perf_counter()
    A, Q, lam, sweeps = qst.abs_map(dev_matrix(T), P, prec)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    A_w, Qw, lw = O.abs_map(T64, P)
    e = rel_fro(A.cpu().numpy(), A_w)
    GT = qst.abs_map_backward(Q, lam, P, dev_matrix(GA), prec)
    eg = rel_fro(GT.cpu().numpy(), O.abs_map_backward(Qw, lw, P, GA.astype(np.complex128)))
    el = float(np.abs(np.sort(lam.cpu().numpy()) - np.sort(lw)).max() / np.abs(lw).max())
    say(f"N=11 {prec} P={P}: sweeps {sweeps}, {dt:.2f} s, A rel err {e:.2e}, "
        f"dL/dT rel err {eg:.2e}, spectrum {el:.2e}")
    # FP64: the direct solver's errors at d = 2048 are about 1e-14
    tol = TOL[prec]
    assert e <= tol and eg <= tol
    assert el <= (1e-13 if prec == "f64" else 1e-9)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_abs_map_warm_start(prec):
    """Warm start (the Jacobi solver) from the eigenvectors of a nearby
    matrix: the same A and dL/dT as a cold start (the direct solver) to the
    tolerance, in a few sweeps; AbsProjection(warm=True) over a drifting T
    (a training loop's pattern) against cold-start calls."""
    n, d, P = 7, 128, 1.5
    g = S.rng(8700)
    T1 = S.ginibre(g, d)
    E = S.ginibre(g, d)
    T2 = (T1 + 1e-3 * E).astype(ctype(prec))
    _, Q1, _, _ = qst.abs_map(dev_matrix(T1.astype(ctype(prec))), P, prec)
    A_c, Q_c, lam_c, sw_c = qst.abs_map(dev_matrix(T2), P, prec)
    A_w, Q_w, lam_w, sw_w = qst.abs_map(dev_matrix(T2), P, prec, Q0=Q1)
    say(f"{prec}: cold {sw_c} sweeps (direct), warm {sw_w} sweeps")
    assert sw_c == 0 and 1 <= sw_w <= 4
    A_o = O.abs_map(T2.astype(np.complex128), P)[0]
    assert rel_fro(A_w.cpu().numpy(), A_o) <= TOL[prec]
    assert rel_fro(A_w.cpu().numpy(), A_c.cpu().numpy()) <= TOL[prec]
    GA = dev_matrix(S.ginibre(g, d).astype(ctype(prec)))
    G_c = qst.abs_map_backward(Q_c, lam_c, P, GA, prec).cpu().numpy()
    G_w = qst.abs_map_backward(Q_w, lam_w, P, GA, prec).cpu().numpy()
    assert rel_fro(G_w, G_c) <= TOL[prec]
    psi = S.haar_vector(g, d)
    f = S.multinomial_freqs(g, 100_000, O.probs_real(S.depolarised_pure(psi, 0.1)))
    rt = torch.float64 if prec == "f64" else torch.float32
    fg = torch.from_numpy(f).to(DEV, rt)
    proj = qst.AbsProjection(P, prec, warm=True)
    for k in range(4):
        Tk = (T1 + (1e-3 * k) * E).astype(ctype(prec))
        out = []
        for warm in (True, False):
            Tg = torch.from_numpy(Tk).to(DEV).requires_grad_(True)
            L = qst.likelihood(proj(Tg), fg, prec) if warm else qst.likelihood(Tg, fg, prec, state_map="abs", P=P)
            L.backward()
            out.append((float(L.item()), Tg.grad.cpu().numpy()))
        (Lw, gw), (Lc, gc) = out
        say(f"  step {k}: warm sweeps {proj.sweeps}, L {Lw:.12f} vs {Lc:.12f}")
        assert abs(Lw - Lc) <= TOL[prec] * abs(Lc) and rel_fro(gw, gc) <= 10 * TOL[prec]
        if k:
            assert 1 <= proj.sweeps <= 4


@pytest.mark.parametrize("case", ["4-fold", "two values", "cluster 1e-9", "identity + 1e-9 G", "rank 6"])
def test_abs_map_degenerate_spectra(case):
    """Repeated and nearly repeated eigenvalues (the direct solver's cluster
    treatment, and splitting of the tridiagonal): A and dL/dT against the
    oracle, Q unitary, Q Lambda Q^dagger = H."""
    n, d, P = 7, 128, 1.5
    g = S.rng(8750)
    U = np.linalg.qr(S.ginibre(g, d))[0]
    if case == "4-fold":
        lam = np.repeat(g.standard_normal(d // 4), 4)
    elif case == "two values":
        lam = np.repeat(g.standard_normal(2), d // 2)
    elif case == "cluster 1e-9":
        lam = np.sort(g.standard_normal(d))
        lam[d // 2:d // 2 + 5] = lam[d // 2] + 1e-9 * np.arange(5)
    elif case == "rank 6":
        lam = np.zeros(d)
        lam[:6] = g.standard_normal(6)
    else:
        lam = np.ones(d)
    H = (U * lam) @ U.conj().T
    if case == "identity + 1e-9 G":
        H = np.eye(d) + 1e-9 * O.hermitian_part(S.ginibre(g, d))
    H = O.hermitian_part(H)
    A, Q, lw, sweeps = qst.abs_map(dev_matrix(H), P, "f64")
    GA = S.ginibre(g, d)
    GT = qst.abs_map_backward(Q, lw, P, dev_matrix(GA), "f64")
    torch.cuda.synchronize()
    A_w, Qo, lo = O.abs_map(H, P)
    Qn, ln = Q.cpu().numpy(), lw.cpu().numpy()
    e = rel_fro(A.cpu().numpy(), A_w)
    uq = np.abs(Qn.conj().T @ Qn - np.eye(d)).max()
    res = rel_fro((Qn * ln) @ Qn.conj().T, H)
    say(f"{case}: A rel err {e:.2e}, |Q^H Q - I| {uq:.1e}, residual {res:.1e}")
    assert sweeps == 0
    assert uq <= 1e-13 * d and res <= 1e-13
    # rank 6: the d - 6 zero eigenvalues come out at the rounding level on
    # both sides, and |l|^(3/4) of them differs by about (1e-16)^(3/4)
    assert e <= (1e-10 if case == "rank 6" else TOL["f64"])
    if case in ("4-fold", "two values", "cluster 1e-9"):
        # the oracle's adjoint on the constructed spectrum (ascending, as
        # eigh orders its Q), so that ties are exact: its divided differences
        # are the plain quotient, which LAPACK's eigenvalues of a repeated
        # eigenvalue (apart by rounding) would turn into cancellation; near
        # ties 1e-9 apart still cost it about 1e-16 / 1e-9 relative
        want = O.abs_map_backward(Qo, np.sort(lam), P, GA)
        eg = rel_fro(GT.cpu().numpy(), want)
        say(f"  dL/dT rel err {eg:.2e}")
        assert eg <= (1e-6 if case == "cluster 1e-9" else 1e-12)


def test_abs_map_non_finite_input_is_an_error():
    """A NaN in T makes the tridiagonal matrix non-finite: qst_abs_map and
    qst_fidelity_general return QST_ERR_INVALID_ARG (raised as QstError)
    instead of a result; so does a warm-started call."""
    d = 16
    g = S.rng(8800)
    T = S.ginibre(g, d)
    T[3, 5] = np.nan
    Tg = torch.from_numpy(T).to(DEV)
    with pytest.raises(qst.QstError, match="did not converge"):
        qst.abs_map(Tg, 1.5, "f64")
    rho = torch.eye(d, dtype=torch.complex128, device=DEV) / d
    with pytest.raises(qst.QstError, match="did not converge"):
        qst.fidelity_general(Tg, rho, "f64")
    Q0 = torch.eye(d, dtype=torch.complex128, device=DEV)
    with pytest.raises(qst.QstError, match="did not converge"):
        qst.abs_map(Tg, 1.5, "f64", Q0=Q0)
    # the library stays usable
    T[3, 5] = 0.0
    A, _, _, sweeps = qst.abs_map(torch.from_numpy(T).to(DEV), 1.5, "f64")
    assert sweeps == 0 and rel_fro(A.cpu().numpy(), O.abs_map(T, 1.5)[0]) <= TOL["f64"]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_abs_map_async_equals_sync(prec):
    """qst_abs_map_async (nothing read back) against qst_abs_map: the same
    sweeps and bitwise the same A, Q, lam, for the direct solver and for a
    warm start (stopping rule on the device); too few warm sweeps report -1;
    qst_fidelity_general_async likewise."""
    n, d, P = 6, 64, 1.5
    g = S.rng(8900)
    T = dev_matrix(S.ginibre(g, d).astype(ctype(prec)))
    A, Q, lam, sw = qst.abs_map(T, P, prec)
    A2, Q2, lam2, sw2 = qst.abs_map_async(T, P, prec, max_sweeps=20)
    torch.cuda.synchronize()
    assert sw == 0 and int(sw2.item()) == sw
    assert torch.equal(A, A2) and torch.equal(Q, Q2) and torch.equal(lam, lam2)
    T2 = (T + 1e-3 * dev_matrix(S.ginibre(g, d).astype(ctype(prec)))).contiguous()
    A, Qw, lam, sw = qst.abs_map(T2, P, prec, Q0=Q)
    A2, Qw2, lam2, sw2 = qst.abs_map_async(T2, P, prec, max_sweeps=20, Q0=Q)
    torch.cuda.synchronize()
    assert sw >= 1 and int(sw2.item()) == sw
    assert torch.equal(A, A2) and torch.equal(Qw, Qw2) and torch.equal(lam, lam2)
    _, _, _, sw3 = qst.abs_map_async(T2, P, prec, max_sweeps=1, Q0=Q)
    assert int(sw3.item()) == -1
    rho = dev_matrix(S.depolarised_pure(S.haar_vector(g, d), 0.2).astype(ctype(prec)))
    F, fs = qst.fidelity_general(T, rho, prec)
    F2, fs2 = qst.fidelity_general_async(T, rho, prec, max_sweeps=20)
    torch.cuda.synchronize()
    assert int(fs2.item()) == fs and float(F2.item()) == float(F.item())


@pytest.mark.parametrize("warm", [True, False])
def test_abs_map_async_graph_replays(warm):
    """qst_abs_map_async captured in a HIP graph (outputs, workspace and the
    warm start preallocated), for the warm-started Jacobi solver and for the
    direct solver: three replays, with eager library work and
    synchronisations between them, each bitwise equal to the eager call."""
    n, d, P, prec = 7, 128, 1.0, "f32"
    g = S.rng(8910)
    T = dev_matrix(S.ginibre(g, d).astype(np.complex64))
    _, Q0, _, _ = qst.abs_map(T, P, prec)
    if not warm:
        Q0 = None
    T2 = (T + 1e-3 * dev_matrix(S.ginibre(g, d).astype(np.complex64))).contiguous()
    A_e, Q_e, lam_e, sw_e = qst.abs_map_async(T2, P, prec, max_sweeps=6, Q0=Q0)
    torch.cuda.synchronize()
    assert (0 < int(sw_e.item()) <= 6) if warm else int(sw_e.item()) == 0
    A = torch.empty_like(A_e)
    Q = torch.empty_like(Q_e)
    lam = torch.empty_like(lam_e)
    sw = torch.empty_like(sw_e)
    ws = torch.empty(qst.workspace_bytes(n, qst.QST_F32, qst._lib.QST_OP_ABS_MAP), dtype=torch.uint8, device=DEV)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        qst.abs_map_async(T2, P, prec, max_sweeps=6, Q0=Q0, out=A, Q=Q, lam=lam, sweeps=sw, ws=ws)  # warm-up
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        qst.abs_map_async(T2, P, prec, max_sweeps=6, Q0=Q0, out=A, Q=Q, lam=lam, sweeps=sw, ws=ws)
    for k in range(3):
        A.zero_()
        lam.zero_()
        sw.zero_()
        graph.replay()
        torch.cuda.synchronize()
        say(f"replay {k}: sweeps {int(sw.item())}")
        assert torch.equal(A, A_e) and torch.equal(Q, Q_e) and torch.equal(lam, lam_e)
        assert int(sw.item()) == int(sw_e.item())
        qst.abs_map(T, P, prec)  # eager work on the same stream between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("warm", [False, True])
def test_abs_projection_unsynchronised_warm_steps(warm):
    """AbsProjection(max_sweeps=...) runs its calls without synchronising
    (the direct solver, or warm-started Jacobi sweeps): the same losses and
    gradients as the synchronous projection over a drifting T."""
    n, d, P, prec = 7, 128, 1.5, "f64"
    g = S.rng(8920)
    T1, E = S.ginibre(g, d), S.ginibre(g, d)
    psi = S.haar_vector(g, d)
    f = torch.from_numpy(S.multinomial_freqs(g, 100_000, O.probs_real(S.depolarised_pure(psi, 0.1)))).to(DEV)
    sync_p = qst.AbsProjection(P, prec, warm=warm)
    async_p = qst.AbsProjection(P, prec, max_sweeps=6, warm=warm)
    for k in range(4):
        Tk = T1 + (1e-3 * k) * E
        out = []
        for proj in (sync_p, async_p):
            Tg = torch.from_numpy(Tk).to(DEV).requires_grad_(True)
            L = qst.likelihood(proj(Tg), f, prec)
            L.backward()
            out.append((float(L.item()), Tg.grad.cpu().numpy()))
        (Ls, gs), (La, ga) = out
        say(f"step {k}: sweeps sync {sync_p.sweeps} async {async_p.sweeps}")
        assert async_p.sweeps == sync_p.sweeps
        assert Ls == La and np.array_equal(gs, ga)
