"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/qst.h declares, sizes workspaces, and rejects invalid arguments on
the host before any HIP call (every call here fails validation, so no kernel
is ever launched)."""
import ctypes
import os
import re
import subprocess

import pytest

from conftest import ROOT

lib_mod = pytest.importorskip("paper_2207_05341_amd._lib")

HEADER = os.path.join(ROOT, "include", "qst.h")
FAKE = ctypes.c_void_p(0x10000)  # never dereferenced: validation fails first
FAKE2 = ctypes.c_void_p(0x20000)


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lib_mod.LIB_PATH):
        pytest.skip("libqst.so not built")
    return lib_mod.lib()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(qst_[a-z_]+)\s*\(", text))


def test_header_and_binding_agree():
    assert declared_symbols() == set(lib_mod.SIGNATURES)


def test_library_exports_every_declared_symbol(L):
    for name in declared_symbols():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", lib_mod.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (qst_\w+)", out))
    assert declared_symbols() <= exported


def test_status_strings(L):
    for code, name in enumerate(["QST_OK", "QST_ERR_INVALID_ARG", "QST_ERR_UNSUPPORTED", "QST_ERR_WORKSPACE",
                                 "QST_ERR_HIP"]):
        assert L.qst_status_string(code).decode() == name
    assert L.qst_version().decode().startswith("qst-mi355x")


def test_workspace_sizes(L):
    ws = lib_mod.workspace_bytes
    # invalid requests
    assert ws(0, 0, 0) == 0 and ws(14, 0, 0) == 0 and ws(5, 7, 0) == 0 and ws(5, 0, 10) == 0
    # single-pass POVM needs no workspace; N=11 needs one 4^N complex intermediate
    assert ws(6, 0, lib_mod.QST_OP_POVM_PROBS) == 0
    assert ws(11, lib_mod.QST_F64, lib_mod.QST_OP_POVM_PROBS) >= 16 * 4 ** 11
    assert ws(11, lib_mod.QST_F32, lib_mod.QST_OP_POVM_PROBS) >= 8 * 4 ** 11
    # backward (recompute bound): intermediate + G' + p
    assert ws(12, lib_mod.QST_F32, lib_mod.QST_OP_NLL_BACKWARD) >= 8 * 4 ** 12 * 2 + 4 * 4 ** 12
    for n in range(1, 14):
        for prec in (0, 1, 2):
            assert ws(n, prec, lib_mod.QST_OP_STATE_MAP) > 0
            assert ws(n, prec, lib_mod.QST_OP_NLL_BACKWARD) >= ws(n, prec, lib_mod.QST_OP_POVM_PROBS)
            # likelihood keeps rho and the POVM intermediates in the workspace
            cb = 16 if prec == 0 else 8
            assert ws(n, prec, lib_mod.QST_OP_LIKELIHOOD) >= cb * 4 ** n + ws(n, prec, lib_mod.QST_OP_POVM_PROBS)
            # the gradient product needs stream-K partials (N >= 10) and, on
            # the BF16 path, the split planes of G' and T^T (16 d^2 bytes)
            gp = ws(n, prec, lib_mod.QST_OP_GRAD_PRODUCT)
            assert (gp > 0) == (n >= 10)
            if prec == 2 and n >= 10:
                assert gp >= 16 * 4 ** n
            # BF16 state map from N = 8: bf16 planes of T (4 d^2 bytes)
            if prec == 2 and n >= 8:
                assert ws(n, prec, lib_mod.QST_OP_STATE_MAP) >= 4 * 4 ** n
            # the combined call: the likelihood's workspace plus G'
            assert ws(n, prec, lib_mod.QST_OP_LIKELIHOOD_GRAD) >= ws(n, prec, lib_mod.QST_OP_LIKELIHOOD) + cb * 4 ** n
        # QST_F32X6 from d = 128: the planes of G' T as well (36 d^2 bytes)
        if n >= 7:
            assert ws(n, lib_mod.QST_F32X6, lib_mod.QST_OP_LIKELIHOOD_GRAD) >= \
                ws(n, lib_mod.QST_F32X6, lib_mod.QST_OP_LIKELIHOOD) + (8 + 36) * 4 ** n
    assert ws(5, 0, 10) == 0
    # absolute map: three d x d complex FP64 buffers, any storage precision
    for n in (1, 6, 12):
        for prec in (0, 1, 2):
            assert ws(n, prec, lib_mod.QST_OP_ABS_MAP) >= 3 * 16 * 4 ** n
    # fidelity: the W^dagger T partials of 16 row blocks at the largest rank
    for n in (2, 6, 11):
        d = 1 << n
        assert ws(n, 0, lib_mod.QST_OP_FIDELITY) >= (16 if d >= 64 else 1) * lib_mod.QST_FIDELITY_MAX_RANK * d * 16


def _err(L):
    return L.qst_last_error().decode()


def test_state_map_validation(L):
    ok_ws = lib_mod.workspace_bytes(4, 0, 0)
    W = ctypes.c_void_p(0x30000)
    st = L.qst_state_map(0, 0, FAKE, 16, FAKE2, 16, FAKE, W, ok_ws, None)
    assert st == lib_mod.QST_ERR_INVALID_ARG and "n_qubits" in _err(L)
    st = L.qst_state_map(14, 0, FAKE, 1 << 14, FAKE2, 1 << 14, FAKE, W, ok_ws, None)
    assert st == lib_mod.QST_ERR_INVALID_ARG
    st = L.qst_state_map(4, 5, FAKE, 16, FAKE2, 16, FAKE, W, ok_ws, None)
    assert st == lib_mod.QST_ERR_INVALID_ARG and "precision" in _err(L)
    st = L.qst_state_map(4, 0, None, 16, FAKE2, 16, FAKE, W, ok_ws, None)
    assert st == lib_mod.QST_ERR_INVALID_ARG and "T is NULL" in _err(L)
    st = L.qst_state_map(4, 0, FAKE, 15, FAKE2, 16, FAKE, W, ok_ws, None)
    assert st == lib_mod.QST_ERR_INVALID_ARG and "leading dimension" in _err(L)
    st = L.qst_state_map(4, 0, FAKE, 16, FAKE2, 8, FAKE, W, ok_ws, None)
    assert st == lib_mod.QST_ERR_INVALID_ARG
    st = L.qst_state_map(4, 0, FAKE, 16, FAKE2, 16, None, W, ok_ws, None)
    assert st == lib_mod.QST_ERR_INVALID_ARG and "tau_dev" in _err(L)
    st = L.qst_state_map(4, 0, FAKE, 16, FAKE2, 16, FAKE, W, ok_ws - 1, None)
    assert st == lib_mod.QST_ERR_WORKSPACE and "workspace" in _err(L)
    st = L.qst_state_map(4, 0, FAKE, 16, FAKE2, 16, FAKE, None, ok_ws, None)
    assert st == lib_mod.QST_ERR_WORKSPACE
    st = L.qst_state_map(4, 0, FAKE, 16, FAKE, 16, FAKE2, W, ok_ws, None)
    assert st == lib_mod.QST_ERR_INVALID_ARG and "alias" in _err(L)


def _povm_array(vals):
    return (ctypes.c_double * 32)(*vals)


def _tetra_flat():
    import oracle as O
    M = O.tetrahedral_povm()
    flat = []
    for a in range(4):
        for x in range(2):
            for y in range(2):
                flat += [M[a][x, y].real, M[a][x, y].imag]
    return flat


def test_povm_validation(L):
    n = 8
    need = lib_mod.workspace_bytes(n, 0, lib_mod.QST_OP_POVM_PROBS)
    assert need > 0
    st = L.qst_povm_probs(n, 0, FAKE, 256, None, FAKE2, None, 0, None)
    assert st == lib_mod.QST_ERR_WORKSPACE
    st = L.qst_povm_probs(n, 0, FAKE, 256, None, None, FAKE, need, None)
    assert st == lib_mod.QST_ERR_INVALID_ARG and "p is NULL" in _err(L)
    flat = _tetra_flat()
    bad = list(flat)
    bad[8 * 1 + 2 * 1 + 1] += 0.1  # M_1[0][1] imaginary part: not Hermitian
    st = L.qst_povm_probs(n, 0, FAKE, 256, _povm_array(bad), FAKE2, FAKE, need, None)
    assert st == lib_mod.QST_ERR_INVALID_ARG and "Hermitian" in _err(L)
    bad = list(flat)
    bad[0] += 0.01  # M_0[0][0]: sum no longer the identity
    st = L.qst_povm_probs(n, 0, FAKE, 256, _povm_array(bad), FAKE2, FAKE, need, None)
    assert st == lib_mod.QST_ERR_INVALID_ARG and "identity" in _err(L)
    bad = list(flat)
    bad[5] = float("nan")
    st = L.qst_povm_probs(n, 0, FAKE, 256, _povm_array(bad), FAKE2, FAKE, need, None)
    assert st == lib_mod.QST_ERR_INVALID_ARG


def test_nll_validation(L):
    ws = lib_mod.workspace_bytes(5, 1, lib_mod.QST_OP_NLL)
    W = ctypes.c_void_p(0x30000)
    assert L.qst_nll(5, 1, None, FAKE, FAKE2, None, W, ws, None) == lib_mod.QST_ERR_INVALID_ARG
    assert L.qst_nll(5, 1, FAKE, None, FAKE2, None, W, ws, None) == lib_mod.QST_ERR_INVALID_ARG
    assert L.qst_nll(5, 1, FAKE, FAKE, None, None, W, ws, None) == lib_mod.QST_ERR_INVALID_ARG
    assert L.qst_nll(5, 1, FAKE, FAKE, FAKE2, None, W, 8, None) == lib_mod.QST_ERR_WORKSPACE


def test_backward_validation(L):
    n, d = 7, 128
    ws = lib_mod.workspace_bytes(n, 0, lib_mod.QST_OP_NLL_BACKWARD)
    W = ctypes.c_void_p(0x30000)
    args = dict(T=FAKE, ldT=d, f=FAKE2, p=FAKE2, tau=FAKE, povm=None, up=None, G=W, ldG=d)

    def call(**kw):
        a = dict(args, **kw)
        return L.qst_nll_backward(n, 0, a["T"], a["ldT"], a["f"], a["p"], a["tau"], None, a["povm"], a["up"],
                                  a["G"], a["ldG"], W, kw.get("ws", ws), None)

    assert call(T=None) == lib_mod.QST_ERR_INVALID_ARG
    assert call(f=None) == lib_mod.QST_ERR_INVALID_ARG
    assert call(G=None) == lib_mod.QST_ERR_INVALID_ARG
    assert call(ldT=d - 1) == lib_mod.QST_ERR_INVALID_ARG
    assert call(ldG=3) == lib_mod.QST_ERR_INVALID_ARG
    assert call(tau=None) == lib_mod.QST_ERR_INVALID_ARG and "tau_dev" in _err(L)
    assert call(G=FAKE) == lib_mod.QST_ERR_INVALID_ARG and "alias" in _err(L)
    assert call(ws=1024) == lib_mod.QST_ERR_WORKSPACE


def test_likelihood_validation(L):
    n, d = 8, 256
    ws = lib_mod.workspace_bytes(n, 1, lib_mod.QST_OP_LIKELIHOOD)
    W = ctypes.c_void_p(0x30000)
    G = ctypes.c_void_p(0x40000)
    args = dict(T=FAKE, ldT=d, f=FAKE2, povm=None, tau=FAKE, nll=FAKE2, bad=None, G=G, ldG=d, ws=ws)

    def call(**kw):
        a = dict(args, **kw)
        return L.qst_likelihood(n, 1, a["T"], a["ldT"], a["f"], a["povm"], a["tau"], a["nll"], a["bad"], a["G"],
                                a["ldG"], W, a["ws"], None)

    assert call(T=None) == lib_mod.QST_ERR_INVALID_ARG and "T is NULL" in _err(L)
    assert call(f=None) == lib_mod.QST_ERR_INVALID_ARG and "f is NULL" in _err(L)
    assert call(tau=None) == lib_mod.QST_ERR_INVALID_ARG and "tau_dev" in _err(L)
    assert call(nll=None) == lib_mod.QST_ERR_INVALID_ARG and "nll_dev" in _err(L)
    assert call(ldT=d - 1) == lib_mod.QST_ERR_INVALID_ARG
    assert call(ldG=d - 1) == lib_mod.QST_ERR_INVALID_ARG
    assert call(G=FAKE) == lib_mod.QST_ERR_INVALID_ARG and "alias" in _err(L)
    assert call(ws=ws - 1) == lib_mod.QST_ERR_WORKSPACE
    bad = _tetra_flat()
    bad[0] += 0.01
    assert call(povm=_povm_array(bad)) == lib_mod.QST_ERR_INVALID_ARG and "identity" in _err(L)


def test_likelihood_noalloc_limits(L):
    """The static-scratch variant rejects, before any device call, sizes
    whose workspace exceeds QST_STATIC_SCRATCH_BYTES (N >= 10) and invalid
    precisions or qubit counts; N <= 9 fits in every precision."""
    for prec in (0, 1, 2):
        assert lib_mod.workspace_bytes(9, prec, lib_mod.QST_OP_LIKELIHOOD) <= lib_mod.QST_STATIC_SCRATCH_BYTES
        assert lib_mod.workspace_bytes(10, prec, lib_mod.QST_OP_LIKELIHOOD) > lib_mod.QST_STATIC_SCRATCH_BYTES
        for n in (10, 11, 13):
            d = 1 << n
            st = L.qst_likelihood_noalloc(n, prec, FAKE, d, FAKE2, None, FAKE, FAKE2, None, None, 0, None)
            assert st == lib_mod.QST_ERR_WORKSPACE and "static scratch" in _err(L)
    assert L.qst_likelihood_noalloc(0, 1, FAKE, 1, FAKE2, None, FAKE, FAKE2, None, None, 0, None) \
        == lib_mod.QST_ERR_INVALID_ARG
    assert L.qst_likelihood_noalloc(4, 7, FAKE, 16, FAKE2, None, FAKE, FAKE2, None, None, 0, None) \
        == lib_mod.QST_ERR_INVALID_ARG


def test_general_povm_validation(L):
    """qst_povm_probs_general / qst_likelihood_general reject, before any
    device call: K outside [2, 8], settings outside [1, 64], K^N above 2^30,
    a NULL table, and per qubit a non-Hermitian or non-PSD element or
    elements that do not sum to I; the workspace sizes grow with K."""
    import numpy as np

    def table(mats):
        flat = np.ascontiguousarray(np.asarray(mats, dtype=np.complex128)).view(np.float64).ravel()
        return (ctypes.c_double * flat.size)(*flat.tolist())

    proj = np.array([np.diag([1.0, 0.0]), np.diag([0.0, 1.0])]).astype(complex)
    n, d = 3, 8
    ws = L.qst_workspace_bytes_general(n, 1, 2, lib_mod.QST_OP_LIKELIHOOD)
    assert ws > 0 and L.qst_workspace_bytes_general(n, 1, 6, lib_mod.QST_OP_LIKELIHOOD) > ws
    assert L.qst_workspace_bytes_general(n, 1, 9, lib_mod.QST_OP_LIKELIHOOD) == 0
    assert L.qst_workspace_bytes_general(n, 1, 2, lib_mod.QST_OP_NLL) == 0
    W = ctypes.c_void_p(0x30000)

    def lik(tab, K=2, S=1, nq=n):
        return L.qst_likelihood_general(nq, 1, FAKE, 1 << nq, S, K, tab, FAKE2, FAKE, FAKE2, None, None, 0, W, ws,
                                        None)

    good = table([proj] * n)
    assert lik(None) == lib_mod.QST_ERR_INVALID_ARG and "NULL" in _err(L)
    assert lik(good, K=1) == lib_mod.QST_ERR_INVALID_ARG and "K=1" in _err(L)
    assert lik(good, K=9) == lib_mod.QST_ERR_INVALID_ARG
    assert lik(good, S=0) == lib_mod.QST_ERR_INVALID_ARG and "settings" in _err(L)
    assert lik(good, S=65) == lib_mod.QST_ERR_INVALID_ARG
    assert lik(table([proj] * 13), K=8, nq=11) == lib_mod.QST_ERR_UNSUPPORTED and "2^30" in _err(L)
    nonherm = proj.copy()
    nonherm[0, 0, 1] = 0.1
    assert lik(table([proj, nonherm, proj])) == lib_mod.QST_ERR_INVALID_ARG and "qubit 2" in _err(L) \
        and "Hermitian" in _err(L)
    notpsd = np.array([np.diag([1.2, 0.0]), np.diag([-0.2, 1.0])]).astype(complex)
    assert lik(table([proj, proj, notpsd])) == lib_mod.QST_ERR_INVALID_ARG and "positive" in _err(L)
    short = np.array([np.diag([0.9, 0.0]), np.diag([0.0, 1.0])]).astype(complex)
    assert lik(table([short, proj, proj])) == lib_mod.QST_ERR_INVALID_ARG and "identity" in _err(L)
    wsp = L.qst_workspace_bytes_general(n, 1, 2, lib_mod.QST_OP_POVM_PROBS)
    assert L.qst_povm_probs_general(n, 1, FAKE, d, 2, good, FAKE2, W, wsp - 1, None) == lib_mod.QST_ERR_WORKSPACE


def test_grad_product_validation(L):
    n, d = 10, 1024
    ws = lib_mod.workspace_bytes(n, 0, lib_mod.QST_OP_GRAD_PRODUCT)
    W = ctypes.c_void_p(0x30000)
    out = ctypes.c_void_p(0x50000)

    def call(G=FAKE2, ldG=d, T=FAKE, ldT=d, tau=FAKE, grad=out, ldg=d, nb=ws):
        return L.qst_grad_product(n, 0, G, ldG, T, ldT, tau, None, grad, ldg, W, nb, None)

    assert call(G=None) == lib_mod.QST_ERR_INVALID_ARG
    assert call(T=None) == lib_mod.QST_ERR_INVALID_ARG
    assert call(grad=None) == lib_mod.QST_ERR_INVALID_ARG
    assert call(tau=None) == lib_mod.QST_ERR_INVALID_ARG and "tau_dev" in _err(L)
    assert call(ldg=5) == lib_mod.QST_ERR_INVALID_ARG
    assert call(grad=FAKE) == lib_mod.QST_ERR_INVALID_ARG and "alias" in _err(L)
    assert call(grad=FAKE2) == lib_mod.QST_ERR_INVALID_ARG
    assert call(nb=ws - 1) == lib_mod.QST_ERR_WORKSPACE


def test_likelihood_grad_validation(L):
    n, d = 10, 1024
    ws = lib_mod.workspace_bytes(n, 0, lib_mod.QST_OP_LIKELIHOOD_GRAD)
    W = ctypes.c_void_p(0x30000)
    out, tau, nll = ctypes.c_void_p(0x50000), ctypes.c_void_p(0x60000), ctypes.c_void_p(0x70000)

    def call(n=n, prec=0, T=FAKE, ldT=d, f=FAKE2, grad=out, ldg=d, tau=tau, nll=nll, nb=ws):
        return L.qst_likelihood_grad(n, prec, T, ldT, f, None, tau, nll, None, grad, ldg, W, nb, None)

    assert call(n=0) == lib_mod.QST_ERR_INVALID_ARG and "n_qubits" in _err(L)
    assert call(prec=9) == lib_mod.QST_ERR_INVALID_ARG and "precision" in _err(L)
    assert call(T=None) == lib_mod.QST_ERR_INVALID_ARG
    assert call(grad=None) == lib_mod.QST_ERR_INVALID_ARG
    assert call(ldg=5) == lib_mod.QST_ERR_INVALID_ARG
    assert call(grad=FAKE) == lib_mod.QST_ERR_INVALID_ARG and "alias" in _err(L)
    assert call(nb=ws - 1) == lib_mod.QST_ERR_WORKSPACE


def test_premap_validation(L):
    H, Lo = lib_mod.QST_PREMAP_HERMITIAN, lib_mod.QST_PREMAP_LOWER

    def call(n=4, prec=0, mode=H, X=FAKE, ldX=16, Y=FAKE2, ldY=16):
        return L.qst_state_premap(n, prec, mode, X, ldX, Y, ldY, None)

    assert call(n=0) == lib_mod.QST_ERR_INVALID_ARG and "n_qubits" in _err(L)
    assert call(prec=7) == lib_mod.QST_ERR_INVALID_ARG and "precision" in _err(L)
    assert call(mode=0) == lib_mod.QST_ERR_INVALID_ARG and "mode" in _err(L)
    assert call(mode=3) == lib_mod.QST_ERR_INVALID_ARG and "mode" in _err(L)
    assert call(mode=Lo, X=None) == lib_mod.QST_ERR_INVALID_ARG and "X is NULL" in _err(L)
    assert call(Y=None) == lib_mod.QST_ERR_INVALID_ARG and "Y is NULL" in _err(L)
    assert call(ldX=15) == lib_mod.QST_ERR_INVALID_ARG and "leading dimension" in _err(L)
    assert call(ldY=8) == lib_mod.QST_ERR_INVALID_ARG
    assert call(Y=FAKE, ldY=32) == lib_mod.QST_ERR_INVALID_ARG and "in place" in _err(L)


def test_abs_map_validation(L):
    n, d = 4, 16
    ws = lib_mod.workspace_bytes(n, 0, lib_mod.QST_OP_ABS_MAP)
    W = ctypes.c_void_p(0x30000)
    Q, lam = ctypes.c_void_p(0x40000), ctypes.c_void_p(0x50000)

    def fwd(n=n, prec=0, P=1.5, T=FAKE, ldT=d, Q0=None, A=FAKE2, ldA=d, Qp=Q, lp=lam, nb=ws):
        return L.qst_abs_map(n, prec, P, T, ldT, Q0, A, ldA, Qp, lp, None, W, nb, None)

    assert fwd(n=0) == lib_mod.QST_ERR_INVALID_ARG and "n_qubits" in _err(L)
    assert fwd(prec=9) == lib_mod.QST_ERR_INVALID_ARG and "precision" in _err(L)
    assert fwd(T=None) == lib_mod.QST_ERR_INVALID_ARG and "T is NULL" in _err(L)
    assert fwd(A=None) == lib_mod.QST_ERR_INVALID_ARG and "A is NULL" in _err(L)
    assert fwd(ldA=d - 1) == lib_mod.QST_ERR_INVALID_ARG and "leading dimension" in _err(L)
    assert fwd(Qp=None) == lib_mod.QST_ERR_INVALID_ARG and "Q is NULL" in _err(L)
    assert fwd(lp=None) == lib_mod.QST_ERR_INVALID_ARG and "lam is NULL" in _err(L)
    for bad in (-0.5, float("nan"), float("inf")):
        assert fwd(P=bad) == lib_mod.QST_ERR_INVALID_ARG and "order P" in _err(L)
    assert fwd(A=FAKE, ldA=d + 1) == lib_mod.QST_ERR_INVALID_ARG and "in place" in _err(L)
    assert fwd(Qp=FAKE2) == lib_mod.QST_ERR_INVALID_ARG and "alias" in _err(L)
    assert fwd(Q0=FAKE) == lib_mod.QST_ERR_INVALID_ARG and "Q0 must not alias" in _err(L)
    assert fwd(nb=ws - 1) == lib_mod.QST_ERR_WORKSPACE

    def bwd(P=1.5, Qp=Q, lp=lam, GA=FAKE, ldGA=d, GT=FAKE2, ldGT=d, nb=ws):
        return L.qst_abs_map_backward(n, 0, P, Qp, lp, GA, ldGA, GT, ldGT, W, nb, None)

    assert bwd(Qp=None) == lib_mod.QST_ERR_INVALID_ARG and "Q is NULL" in _err(L)
    assert bwd(lp=None) == lib_mod.QST_ERR_INVALID_ARG and "lam is NULL" in _err(L)
    assert bwd(GA=None) == lib_mod.QST_ERR_INVALID_ARG and "GA is NULL" in _err(L)
    assert bwd(ldGT=3) == lib_mod.QST_ERR_INVALID_ARG and "leading dimension" in _err(L)
    assert bwd(P=-1.0) == lib_mod.QST_ERR_INVALID_ARG and "order P" in _err(L)
    assert bwd(GT=FAKE, ldGT=d + 2) == lib_mod.QST_ERR_INVALID_ARG and "in place" in _err(L)
    assert bwd(GT=Q) == lib_mod.QST_ERR_INVALID_ARG and "alias" in _err(L)
    assert bwd(nb=0) == lib_mod.QST_ERR_WORKSPACE

    SW = ctypes.c_void_p(0x60000)

    def fwd_async(max_sweeps=8, sw=SW, T=FAKE, nb=ws):
        return L.qst_abs_map_async(n, 0, 1.5, T, d, None, FAKE2, d, Q, lam, max_sweeps, sw, W, nb, None)

    assert fwd_async(max_sweeps=0) == lib_mod.QST_ERR_INVALID_ARG and "max_sweeps" in _err(L)
    assert fwd_async(max_sweeps=41) == lib_mod.QST_ERR_INVALID_ARG and "max_sweeps" in _err(L)
    assert fwd_async(sw=None) == lib_mod.QST_ERR_INVALID_ARG and "sweeps_dev" in _err(L)
    assert fwd_async(T=None) == lib_mod.QST_ERR_INVALID_ARG and "T is NULL" in _err(L)
    assert fwd_async(nb=ws - 1) == lib_mod.QST_ERR_WORKSPACE
    assert L.qst_fidelity_general_async(n, 0, FAKE, d, FAKE2, d, W, 0, SW, W, ws, None) == lib_mod.QST_ERR_INVALID_ARG
    assert L.qst_fidelity_general_async(n, 0, FAKE, d, FAKE2, d, W, 8, None, W, ws, None) \
        == lib_mod.QST_ERR_INVALID_ARG and "sweeps_dev" in _err(L)


def test_likelihood_fc_validation(L):
    n, d = 7, 128
    ws = lib_mod.workspace_bytes(n, 1, lib_mod.QST_OP_LIKELIHOOD)
    W, F = ctypes.c_void_p(0x30000), ctypes.c_void_p(0x40000)

    def call(T=FAKE, f=FAKE2, pt=ctypes.c_void_p(0x50000), fc=ctypes.c_void_p(0x60000), nb=ws):
        return L.qst_likelihood_fc(n, 1, T, d, f, pt, None, F, F, fc, None, None, 0, W, nb, None)

    assert call(pt=None) == lib_mod.QST_ERR_INVALID_ARG and "p_target" in _err(L)
    assert call(fc=None) == lib_mod.QST_ERR_INVALID_ARG and "fc_dev" in _err(L)
    assert call(T=None) == lib_mod.QST_ERR_INVALID_ARG and "T is NULL" in _err(L)
    assert call(f=None) == lib_mod.QST_ERR_INVALID_ARG and "f is NULL" in _err(L)
    assert call(nb=ws - 1) == lib_mod.QST_ERR_WORKSPACE


def test_fidelity_general_validation(L):
    n, d = 5, 32
    ws = lib_mod.workspace_bytes(n, 0, lib_mod.QST_OP_ABS_MAP)
    W, F = ctypes.c_void_p(0x30000), ctypes.c_void_p(0x40000)

    def call(n=n, T=FAKE, ldT=d, R=FAKE2, ldR=d, Fd=F, nb=ws):
        return L.qst_fidelity_general(n, 0, T, ldT, R, ldR, Fd, None, W, nb, None)

    assert call(n=14) == lib_mod.QST_ERR_INVALID_ARG and "n_qubits" in _err(L)
    assert call(T=None) == lib_mod.QST_ERR_INVALID_ARG and "T is NULL" in _err(L)
    assert call(R=None) == lib_mod.QST_ERR_INVALID_ARG and "rho is NULL" in _err(L)
    assert call(ldR=d - 1) == lib_mod.QST_ERR_INVALID_ARG and "leading dimension" in _err(L)
    assert call(Fd=None) == lib_mod.QST_ERR_INVALID_ARG and "F_dev" in _err(L)
    assert call(nb=ws // 2) == lib_mod.QST_ERR_WORKSPACE


def test_fidelity_validation(L):
    n, d = 6, 64
    ws = lib_mod.workspace_bytes(n, 0, lib_mod.QST_OP_FIDELITY)
    W = ctypes.c_void_p(0x30000)
    F = ctypes.c_void_p(0x40000)

    def low(T=FAKE, ldT=d, Wt=FAKE2, ldW=4, r=4, Fd=F, nb=ws, n=n):
        return L.qst_fidelity_lowrank(n, 0, T, ldT, Wt, ldW, r, Fd, W, nb, None)

    assert low(n=0) == lib_mod.QST_ERR_INVALID_ARG
    assert low(T=None) == lib_mod.QST_ERR_INVALID_ARG and "T is NULL" in _err(L)
    assert low(ldT=d - 1) == lib_mod.QST_ERR_INVALID_ARG and "leading dimension" in _err(L)
    assert low(Wt=None) == lib_mod.QST_ERR_INVALID_ARG and "W is NULL" in _err(L)
    assert low(Fd=None) == lib_mod.QST_ERR_INVALID_ARG and "F_dev" in _err(L)
    assert low(r=0) == lib_mod.QST_ERR_INVALID_ARG and "rank" in _err(L)
    assert low(r=lib_mod.QST_FIDELITY_MAX_RANK + 1, ldW=64) == lib_mod.QST_ERR_INVALID_ARG and "rank" in _err(L)
    assert low(ldW=3) == lib_mod.QST_ERR_INVALID_ARG and "ldW" in _err(L)
    assert low(nb=ws - 1) == lib_mod.QST_ERR_WORKSPACE

    def cls(ph=FAKE, p=FAKE2, Fd=F, nb=ws):
        return L.qst_fidelity_classical(n, 0, ph, p, Fd, W, nb, None)

    assert cls(ph=None) == lib_mod.QST_ERR_INVALID_ARG and "p_hat" in _err(L)
    assert cls(p=None) == lib_mod.QST_ERR_INVALID_ARG
    assert cls(Fd=None) == lib_mod.QST_ERR_INVALID_ARG and "F_dev" in _err(L)
    assert cls(nb=0) == lib_mod.QST_ERR_WORKSPACE


def test_fnn_validation(L):
    n, d = 4, 16
    ws = lib_mod.workspace_bytes(n, 0, lib_mod.QST_OP_FNN)
    assert ws >= 1024 * 8 * 8 + 4 ** n * 8
    W = ctypes.c_void_p(0x30000)
    P = [ctypes.c_void_p(0x100000 * (i + 1)) for i in range(8)]

    def fwd(i=None, T=FAKE, ldT=d, nb=ws):
        a = [p if k != i else None for k, p in enumerate(P[:6])]
        return L.qst_fnn_forward(n, 0, *a, T, ldT, W, nb, None)

    for i, name in enumerate(["W1", "b1", "W2", "b2", "x", "h_pre"]):
        assert fwd(i) == lib_mod.QST_ERR_INVALID_ARG and f"{name} is NULL" in _err(L)
    assert fwd(T=None) == lib_mod.QST_ERR_INVALID_ARG and "T is NULL" in _err(L)
    assert fwd(ldT=d - 1) == lib_mod.QST_ERR_INVALID_ARG and "leading dimension" in _err(L)
    assert fwd(nb=ws - 1) == lib_mod.QST_ERR_WORKSPACE

    def bwd(i=None, G=FAKE, ldG=d, nb=ws):
        a = [p if k != i else None for k, p in enumerate(P[:7])]
        return L.qst_fnn_backward(n, 0, a[0], a[1], a[2], G, ldG, a[3], a[4], a[5], a[6], W, nb, None)

    for i, name in enumerate(["W2", "x", "h_pre", "dW1", "db1", "dW2", "db2"]):
        assert bwd(i) == lib_mod.QST_ERR_INVALID_ARG and f"{name} is NULL" in _err(L)
    assert bwd(G=None) == lib_mod.QST_ERR_INVALID_ARG and "G is NULL" in _err(L)
    assert bwd(ldG=3) == lib_mod.QST_ERR_INVALID_ARG
    assert bwd(nb=0) == lib_mod.QST_ERR_WORKSPACE


def test_rprop_validation(L):
    def call(count=8, prec=0, p=FAKE, g=FAKE2, pr=FAKE, st=FAKE2, em=0.5, ep=1.2, smin=1e-6, smax=50.0):
        return L.qst_rprop_step(count, prec, p, g, pr, st, em, ep, smin, smax, None)

    assert call(count=-1) == lib_mod.QST_ERR_INVALID_ARG and "negative" in _err(L)
    assert call(prec=9) == lib_mod.QST_ERR_INVALID_ARG and "precision" in _err(L)
    assert call(em=1.0) == lib_mod.QST_ERR_INVALID_ARG and "eta" in _err(L)
    assert call(ep=1.0) == lib_mod.QST_ERR_INVALID_ARG and "eta" in _err(L)
    assert call(smin=0.0) == lib_mod.QST_ERR_INVALID_ARG and "step" in _err(L)
    assert call(smin=2.0, smax=1.0) == lib_mod.QST_ERR_INVALID_ARG
    for k, name in enumerate(["param", "grad", "prev", "step"]):
        args = dict(p=FAKE, g=FAKE2, pr=FAKE, st=FAKE2)
        args[["p", "g", "pr", "st"][k]] = None
        assert call(**args) == lib_mod.QST_ERR_INVALID_ARG and f"{name} is NULL" in _err(L)
    assert call(count=0, p=None, g=None, pr=None, st=None) == lib_mod.QST_OK  # nothing to do


def test_plan_unit_builds_without_hip(tmp_path):
    """The validation / planning unit is HIP-free: it compiles with g++."""
    src = os.path.join(ROOT, "paper_2207_05341_amd", "csrc", "qst_plan.cpp")
    obj = tmp_path / "plan.o"
    res = subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-c", src, "-I",
                          os.path.join(ROOT, "include"), "-o", str(obj)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
