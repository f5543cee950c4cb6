#!/usr/bin/env python3
"""Likelihood forward + adjoint throughput at N = 11 on one MI355X.

One step = the whole hot path on one batch of synthetic input, inputs resident
in HBM before timing starts, as one call, qst_likelihood_grad:
    tau, T T^dagger, POVM map over 4^11 outcomes, NLL, cotangent, adjoint
    POVM map -> G' (the last POVM pass, the NLL terms, the cotangent and the
    first adjoint pass fused, p never stored), then 2/tau G' T.
The headline path is QST_F32X6 (FP32 storage and FP32-level accuracy; the
two complex products as six split-bf16 products per real product on the BF16
matrix cores, their operand planes formed inside the call); the FP64, FP32
(FP32 MFMA products) and BF16 paths, the same step as two calls
(qst_likelihood returning G', then qst_grad_product) and as four separate
calls with p stored (qst_state_map, qst_povm_probs, qst_nll,
qst_nll_backward) are reported alongside, each with its error against the
FP64 oracle.

Timing: each timed loop first runs untimed steps for --settle-ms (200 ms),
then --warmup steps, then exactly --steps timed steps between two device
synchronisations.  The settle phase is there because the GPU's clocks move
for some tens of milliseconds after a sustained load starts (a kernel trace
of 273 steps: the gradient product at 235 us for the first launches, 270 us
around launch 10, 228 us from launch 50 on), so a loop timed right after 5
warm-up steps would average over that transient instead of the steady state
a training loop runs in.

Workload (N = 11): T 2048 x 2048 complex Ginibre (seed 6); frequencies from
10^7 multinomial shots of a Porter-Thomas stand-in distribution of a
depolarised random pure state (q = 0.05).

Prints ONE JSON line with the throughput, the roofline of the dominant kernel
(durations from HIP events recorded by the library on its launch stream over
the timed region), accuracy against the FP64 oracle on the same inputs and
against the GPU FP64 path, the other precision paths, and the FP64 CPU oracle
timed on a bounded sample (all host threads, and one).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "likelihood fwd+bwd evals/sec at N=11 on 1 GPU; % HBM/MFMA peak; max|Δp| vs FP64"

PREC_NOTE = {
    "f64": "complex128 storage, FP64 MFMA products, FP64 POVM passes and NLL",
    "f32": "complex64 storage, FP32 MFMA products (3M form), FP32 POVM passes, tau and NLL sum in FP64",
    "bf16": "complex64 storage, T T^dagger on bf16-rounded T (BF16 MFMA, FP32 accumulate), G' T with split "
            "bf16 operands, FP32 POVM passes, tau and NLL sum in FP64",
    "f32x6": "complex64 storage; both complex products with every FP32 operand split exactly into three bf16 "
             "parts, six partial products per real product (3M form) on the BF16 MFMA, FP32 accumulation "
             "(FP32-accurate); FP32 POVM passes, tau and NLL sum in FP64",
}

# MI355X published peaks
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2500.0}
PEAK_HBM_GBS = 8000.0

# Memory traffic per launch of the dominant kernels: rocprofv3 FETCH_SIZE and
# WRITE_SIZE (separate runs, KiB per dispatch), each scaled by what the same
# counter reads for one plain 256 MiB device copy in the same run.  A figure
# holds only for the kernel sources it was measured on (SHA-256 over the
# record's source files, in order, the build script with its flags among
# them); otherwise the reported traffic is null.
TRAFFIC_F32_SOURCES = ["paper_2207_05341_amd/csrc/k_gemm.hip", "paper_2207_05341_amd/csrc/qst_gemm_tiles.h",
                       "paper_2207_05341_amd/csrc/qst_device.h", "paper_2207_05341_amd/build.py"]
TRAFFIC_X6_SOURCES = ["paper_2207_05341_amd/csrc/k_xgemm.hip", "paper_2207_05341_amd/csrc/qst_device.h",
                      "paper_2207_05341_amd/csrc/qst_plan.h", "paper_2207_05341_amd/build.py"]
TRAFFIC = {
    # N = 11, d = 2048: 173432.6 KiB fetched x 1.9998 + 32768.0 KiB written x 1.0000
    "hemm_f32": {"bytes": 388.72e6, "sources": TRAFFIC_F32_SOURCES,
                 "sources_sha256": "92d43825669e57af5b4f19e9eb0247c3d2ccf7bd79bec7799dba5a7c54c5f5ab"},
    # N = 11, d = 2048: 221292.0 KiB fetched x 1.9998 + 32768.0 KiB written x 1.0000
    "hemm_x6": {"bytes": 486.72e6, "sources": TRAFFIC_X6_SOURCES,
                "sources_sha256": "d07ab688a35ba92bf5fc8a9fcf87fd584398d052e065de90a6fb1023555d4950"},
}


def sources_sha256(paths):
    import hashlib

    h = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_of(kernel):
    rec = TRAFFIC.get(kernel)
    if not rec or rec["sources_sha256"] != sources_sha256(rec["sources"]):
        return None
    return rec["bytes"]


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--settle-ms", type=float, default=200.0,
                    help="untimed steps for this long before the warmup of every timed loop, so that the "
                         "timed steps see the GPU's steady clocks (0: none)")
    ap.add_argument("--prec", default="f32x6", choices=["f64", "f32", "bf16", "f32x6"],
                    help="precision path of the headline step (default f32x6: FP32 storage and accuracy, "
                         "complex products as six split-bf16 products on the BF16 MFMA)")
    ap.add_argument("--n", type=int, default=11)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-variants", action="store_true", help="skip the other precision paths")
    ap.add_argument("--no-long", action="store_true",
                    help="skip the records of the absolute projection and of the general POVMs")
    ap.add_argument("--nnqst-run", action="store_true",
                    help="also train a fresh network for 1000 Rprop steps at N=11 (an end-to-end use of the "
                         "library, not part of the headline measurement)")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-form measurement")
    ap.add_argument("--headline-only", action="store_true",
                    help="measure the headline step alone (no other paths, side records, batched form or CPU "
                         "leg), e.g. under a profiler whose per-kernel averages should cover only that step")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy (torch.neg) of this many MiB first, as the "
                         "reference dispatch for scaling memory-traffic counters")
    args = ap.parse_args()
    if args.headline_only:
        args.no_variants = args.no_long = args.no_batched = args.no_cpu_baseline = True
    return args


def make_inputs(n: int):
    import synth as S

    g = S.rng(6)
    d = 1 << n
    T = S.ginibre(g, d)
    f = S.multinomial_freqs(g, 10_000_000, S.porter_thomas_probs(g, 4 ** n, 0.05))
    return T, f


def to_prec(T, f, prec, dev):
    import numpy as np
    import torch

    ct = np.complex128 if prec == "f64" else np.complex64
    rt = np.float64 if prec == "f64" else np.float32
    return (torch.from_numpy(np.ascontiguousarray(T.astype(ct))).to(dev),
            torch.from_numpy(np.ascontiguousarray(f.astype(rt))).to(dev))


ROUTES = ("one_call", "two_calls", "separate")


def step(qst, T, f, prec, route="one_call"):
    """One pass of the whole path.  one_call: qst_likelihood_grad (L and dL/dT
    in one call; p and G' never leave the library's workspace); two_calls:
    qst_likelihood (tau, rho, p, L, F and G'; p never stored) then
    qst_grad_product; separate: the four separate calls with p stored
    between them."""
    if route == "one_call":
        out, _, grad, _ = qst.likelihood_grad(T, f, prec)
        return out, grad
    if route == "two_calls":
        out, tau, G, _ = qst.likelihood_forward(T, f, prec)
        grad = qst.grad_product(G, T, tau, prec)
        return out, grad
    rho, tau = qst.state_map(T, prec)
    p = qst.povm_probs(rho, prec)
    out, _ = qst.nll(p, f, prec)
    grad = qst.nll_backward(T, f, p, tau, prec, nll_out=out)
    return out, grad


def time_steps(qst, T, f, prec, steps, warmup, only=None, route="one_call", settle_s=0.0):
    """Run untimed steps for settle_s seconds (the GPU's clocks move for
    some tens of milliseconds after a load starts: measured in a kernel
    trace, G' T went 235 -> 270 -> 228 us over the first 50 steps), then
    warmup + steps; with `only`, the library times that kernel scope (HIP
    events on its launch stream) inside the same steps; `only=""` times
    every scope (each bracketing event costs queue time, so that loop is a
    breakdown, not the throughput figure)."""
    import torch

    from paper_2207_05341_amd import _lib

    t_end = time.perf_counter() + settle_s
    while time.perf_counter() < t_end:
        for _ in range(10):
            step(qst, T, f, prec, route)
        torch.cuda.synchronize()
    for _ in range(warmup):
        step(qst, T, f, prec, route)
    torch.cuda.synchronize()
    if only is not None:
        _lib.profile_report(reset=True)
        _lib.profile_enable(True, only or None)
    t0 = time.perf_counter()
    for _ in range(steps):
        step(qst, T, f, prec, route)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = {}
    if only is not None:
        _lib.profile_enable(False)
        kern = _lib.profile_report(reset=True)
    return (t1 - t0) / steps, kern


def batched(qst, prec, dev, reps=20, accuracy_sample=48):
    """Batched form: 1024 instances, N uniform on {3..8} (seed 9), Ginibre T,
    Porter-Thomas stand-in frequencies from 10^5 shots each.  One graph
    replay of the persistent launch vs 1024 separate single-instance call
    sequences (qst_likelihood + qst_grad_product) through the same C ABI;
    the tuned launch shape; the error of L and of the gradient against the
    FP64 oracle over a sample of instances (every N, the largest included)."""
    import numpy as np
    import torch

    import oracle as O
    import synth as S

    g = S.rng(9)
    ns = [int(x) for x in S.batch_qubit_counts(g, 1024, 3, 8)]
    ct = np.complex128 if prec == "f64" else np.complex64
    rt = np.float64 if prec == "f64" else np.float32
    Ts, fs = [], []
    for n in ns:
        d = 1 << n
        Ts.append(S.ginibre(g, d).astype(ct))
        fs.append(S.multinomial_freqs(g, 100_000, S.porter_thomas_probs(g, 4 ** n, 0.1)).astype(rt))
    plan = qst.BatchPlan(ns, prec)
    T_all, f_all = plan.pack(Ts, fs, dev)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        nll, grad, _ = plan.run(T_all, f_all, use_graph=True)  # tunes, captures
        side.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(side)
        for _ in range(reps):
            plan.run(T_all, f_all, use_graph=True)
        ev1.record(side)
    side.synchronize()
    graph_ms = ev0.elapsed_time(ev1) / reps
    # accuracy against the oracle (on the same rounded inputs)
    nll_h, grad_h = nll.cpu().numpy(), grad.cpu().numpy()
    sample = sorted(set(list(range(0, 1024, 1024 // accuracy_sample)) + [i for i in range(1024) if ns[i] == 8][:4]))
    worst_L = worst_g = 0.0
    for i in sample:
        T64, f64 = Ts[i].astype(np.complex128), fs[i].astype(np.float64)
        rho, tau = O.state_map(T64)
        p = O.probs_real(rho)
        L_ref = O.nll_vec(p, f64)
        g_ref = (2.0 / tau) * (O.adjoint(O.cotangent(p, f64), ns[i]) @ T64)
        d = 1 << ns[i]
        gi = grad_h[plan.t_off[i]:plan.t_off[i + 1]].reshape(d, d)
        worst_L = max(worst_L, abs(nll_h[i, 0] - L_ref) / abs(L_ref))
        worst_g = max(worst_g, float(np.linalg.norm(gi - g_ref) / np.linalg.norm(g_ref)))
    # separate launches
    Tg = [torch.from_numpy(T).to(dev) for T in Ts]
    fg = [torch.from_numpy(f).to(dev) for f in fs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for T, f in zip(Tg, fg):
        step(qst, T, f, prec)
    torch.cuda.synchronize()
    sep_ms = 1e3 * (time.perf_counter() - t0)
    info = plan.info()
    plan.close()
    flops = sum(4.0 * (1 << n) ** 2 * ((1 << n) + 1) + 8.0 * (1 << n) ** 3 for n in ns)
    return {"instances": len(ns), "n_range": [3, 8], "precision": prec,
            "graph_ms_per_batch": graph_ms, "instances_per_s": len(ns) / (graph_ms * 1e-3),
            "separate_launches_ms": sep_ms, "speedup_vs_separate": sep_ms / graph_ms,
            "tflops": flops / (graph_ms * 1e-3) / 1e12, "tuned": info,
            "vs_oracle": {"instances": len(sample), "max_rel_err_L": worst_L, "max_rel_err_grad": worst_g}}


def state_maps(qst, T, f, prec, reps=50):
    """The paper's two decomposition modes at the bench size: the pre-map
    kernels alone (achieved GB/s from algorithmic bytes: the Hermitian part
    reads and writes d^2 complex values, the lower triangle reads the lower
    d(d+1)/2 and writes d^2) and one fwd+bwd step through each mode (pre-map,
    qst_likelihood, qst_grad_product, pre-map of the gradient)."""
    import torch

    d = T.shape[0]
    cb = T.element_size()
    Y = torch.empty_like(T)
    out = {}
    for mode, nbytes in (("hermitian", 2 * d * d * cb), ("lower", (d * (d + 1) // 2 + d * d) * cb)):
        for _ in range(3):
            qst.state_premap(T, mode, prec, out=Y)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            qst.state_premap(T, mode, prec, out=Y)
        ev1.record()
        torch.cuda.synchronize()
        us = 1e3 * ev0.elapsed_time(ev1) / reps
        gbs = nbytes / (us * 1e-6) / 1e9
        out[mode + "_premap"] = {"us": round(us, 2), "GB_s": round(gbs, 1), "hbm_frac": round(gbs / 8000.0, 3)}

    def mode_step(mode):
        Tp = qst.state_premap(T, mode, prec)
        o, tau, G, _ = qst.likelihood_forward(Tp, f, prec)
        return o, qst.state_premap(qst.grad_product(G, Tp, tau, prec), mode, prec)

    for mode, key in (("hermitian", "chol_h"), ("lower", "chol_delta")):
        for _ in range(3):
            mode_step(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            mode_step(mode)
        torch.cuda.synchronize()
        out[key + "_evals_per_s"] = round(reps / (time.perf_counter() - t0), 1)
    return out


def fidelities(qst, T, prec, reps=20, f=None):
    """Fidelity calls at the bench size: F_q against a rank-8 target (as in
    the training workload; three launches, reading T once) and F_c between
    two 4^N probability vectors.  Achieved GB/s from algorithmic bytes.
    With f: the likelihood forward with F_c fused into its last pass
    (qst_likelihood_fc) against the plain forward (qst_likelihood)."""
    import numpy as np
    import torch

    import synth as S

    d = T.shape[0]
    g = S.rng(11)
    ct = np.complex128 if prec == "f64" else np.complex64
    W = torch.from_numpy(S.ginibre(g, d, 8).astype(ct)).to(T.device)
    rt = torch.float64 if prec == "f64" else torch.float32
    pa = torch.from_numpy(S.porter_thomas_probs(g, d * d, 0.1)).to(T.device, rt)
    pb = torch.from_numpy(S.porter_thomas_probs(g, d * d, 0.2)).to(T.device, rt)
    out = {}
    for key, fn, nbytes in (("lowrank_r8", lambda: qst.fidelity_lowrank(T, W, prec), (d * d + 8 * d) * T.element_size()),
                            ("classical", lambda: qst.fidelity_classical(pa, pb, prec), 2 * d * d * pa.element_size())):
        for _ in range(3):
            fn()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        us = 1e3 * ev0.elapsed_time(ev1) / reps
        gbs = nbytes / (us * 1e-6) / 1e9
        out[key] = {"us": round(us, 2), "GB_s": round(gbs, 1), "hbm_frac": round(gbs / 8000.0, 3)}
    if f is not None:
        # the fused last pass alone, timed by the library's HIP events on its
        # launch stream (a whole forward call is host-bound at this size)
        from paper_2207_05341_amd import _lib
        us = {}
        for key, fn in (("plain", lambda: qst.likelihood_forward(T, f, prec)),
                        ("with_fc", lambda: qst.likelihood_forward_fc(T, f, pb, prec))):
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            _lib.profile_report(reset=True)
            _lib.profile_enable(True, "povm_fused")
            for _ in range(reps):
                fn()
            torch.cuda.synchronize()
            _lib.profile_enable(False)
            c, t = _lib.profile_report(reset=True)["povm_fused"]
            us[key] = 1e3 * t / c
        out["classical_fused"] = {"fused_pass_us": round(us["plain"], 1), "fused_pass_with_fc_us": round(us["with_fc"], 1),
                                  "added_us": round(us["with_fc"] - us["plain"], 1)}
    return out


def abs_projection(qst, prec, dev, n=10, P=1.5, reps=5):
    """The P-order absolute projection (Eq. abs_P) at N = 10, the size at
    which the paper compares the state maps (P = 1.5, one of its orders):
    qst_abs_map cold (the direct FP64 eigensolver: Householder reduction,
    multisection, twisted factorizations, back-transformation; then
    A = Q |Lambda|^(P/2) Q^dagger), also at N = 11; qst_abs_map_backward;
    one whole step through the map (abs map, likelihood, gradient, adjoint
    of the map), synchronised and not; the warm-started Jacobi solver for
    comparison (sweeps, time per round and its achieved GB/s from
    algorithmic bytes: a round reads and writes every element of A and of
    V^T once, 64 d^2 bytes); the general fidelity (eigenvalues only)."""
    import numpy as np
    import torch

    import synth as S

    d = 1 << n
    g = S.rng(21)
    ct = np.complex128 if prec == "f64" else np.complex64
    rt = torch.float64 if prec == "f64" else torch.float32
    T = torch.from_numpy(S.ginibre(g, d).astype(ct)).to(dev)
    GA = torch.from_numpy(S.ginibre(g, d).astype(ct)).to(dev)
    f = torch.from_numpy(S.multinomial_freqs(g, 10_000_000, S.porter_thomas_probs(g, 4 ** n, 0.1))).to(dev, rt)

    def timed(fn, k=3):
        best = None
        for _ in range(k):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            best = dt if best is None else min(best, dt)
        return best, out

    qst.abs_map(T, P, prec)
    fwd_s, (A, Q, lam, sweeps) = timed(lambda: qst.abs_map(T, P, prec))
    qst.abs_map_backward(Q, lam, P, GA, prec)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        qst.abs_map_backward(Q, lam, P, GA, prec)
    ev1.record()
    torch.cuda.synchronize()
    bwd_ms = ev0.elapsed_time(ev1) / reps

    def step(Tin, proj=None):
        Tg = Tin.clone().requires_grad_(True)
        L = qst.likelihood(proj(Tg), f, prec) if proj else qst.likelihood(Tg, f, prec, state_map="abs", P=P)
        L.backward()
        return L

    step_s, _ = timed(lambda: step(T))
    # the same step with nothing synchronised inside it
    proj_a = qst.AbsProjection(P, prec, max_sweeps=6)
    step_a_s, _ = timed(lambda: step(T, proj_a))
    # a training loop's pattern with the Jacobi solver: T moved by 1e-3 of its
    # scale since the last step, warm-started from the last eigenvectors
    proj_w = qst.AbsProjection(P, prec, warm=True)
    proj_w(T)
    Tw = (T + 1e-3 * GA).contiguous()
    warm_s, _ = timed(lambda: step(Tw, proj_w), k=1)
    warm_sweeps = proj_w.sweeps
    jac_s, (_, _, _, jac_sweeps) = timed(lambda: qst.abs_map(Tw, P, prec, Q0=Q), k=1)
    rounds = max(jac_sweeps, 1) * (d - 1)
    round_us = 1e6 * jac_s / rounds
    gbs = 64.0 * d * d / (round_us * 1e-6) / 1e9
    # F_q against a full-rank target (a depolarised pure state): the
    # eigenvalues of T^dagger rho T
    rho = torch.from_numpy(S.depolarised_pure(S.haar_vector(g, d), 0.3).astype(ct)).to(dev)
    fq_s, _ = timed(lambda: qst.fidelity_general(T, rho, prec))
    del A, Q, lam, T, GA, Tw, proj_a, proj_w, rho
    # N = 11, cold
    T11 = torch.from_numpy(S.ginibre(g, 2 * d).astype(ct)).to(dev)
    fwd11_s, _ = timed(lambda: qst.abs_map(T11, P, prec), k=2)
    del T11
    return {"n_qubits": n, "P": P, "forward_ms": round(1e3 * fwd_s, 2), "sweeps": sweeps,
            "forward_n11_ms": round(1e3 * fwd11_s, 1), "backward_ms": round(bwd_ms, 3),
            "step_ms": round(1e3 * step_s, 1), "step_unsynchronised_ms": round(1e3 * step_a_s, 1),
            "warm_jacobi_step_ms": round(1e3 * warm_s, 1), "warm_jacobi_sweeps": warm_sweeps,
            "jacobi_round_us": round(round_us, 2), "jacobi_round_GB_s": round(gbs, 1),
            "jacobi_round_hbm_frac": round(gbs / 8000.0, 3),
            "fidelity_general_ms": round(1e3 * fq_s, 2),
            "note": "cold calls run the direct eigensolver (one synchronisation per call; none in the "
                    "unsynchronised step); the warm Jacobi step: T moved by 1e-3, sweeps started from the "
                    "previous eigenvectors; best of 3 wall times"}


def network(qst, f, prec, reps=10, long_run=True):
    """The mapping network of Sec. 3.1 at the bench size (4^N -> 2N -> 4^N,
    184.5M parameters at N = 11): forward and backward kernel time with
    achieved GB/s from algorithmic bytes (each weight matrix streamed once
    per pass; the backward also writes both weight gradients), and one whole
    NN-QST training step (network, fused likelihood, backward, the paper's
    Rprop at lr 1e-3 by qst_rprop_step) per second."""
    import torch

    d = 1 << ((f.numel().bit_length() - 1) // 2)
    n = d.bit_length() - 1
    D, H = d * d, 2 * n
    rt = torch.float64 if prec == "f64" else torch.float32
    rb = 8 if prec == "f64" else 4
    net = qst.MappingNetwork(n, dtype=rt, device=f.device, generator=torch.Generator().manual_seed(12))
    x = (f.double() / f.double().sum()).to(rt)
    P = (net.W1.detach(), net.b1.detach(), net.W2.detach(), net.b2.detach())
    T, h_pre = qst.fnn_forward(*P, x, prec)
    out, tau, G, _ = qst.likelihood_forward(T, f, prec)
    grad = qst.grad_product(G, T, tau, prec)

    def timed(fn):
        for _ in range(2):
            fn()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return 1e3 * ev0.elapsed_time(ev1) / reps

    fwd_us = timed(lambda: qst.fnn_forward(*P, x, prec))
    bwd_us = timed(lambda: qst.fnn_backward(P[2], x, h_pre, grad, prec))
    fwd_bytes = (2 * H * D + 2 * D) * rb + D * 2 * rb  # W1, W2, x, b2 read; T written
    bwd_bytes = (H * D + D) * rb + D * 2 * rb + (2 * H * D + D) * rb  # W2, x, G read; dW2, dW1, db2 written
    opt = qst.Rprop(net.parameters(), lr=1e-3)

    def train_step():
        opt.zero_grad(set_to_none=True)
        L = qst.likelihood(net(x, prec), f, prec)
        L.backward()
        opt.step()

    for _ in range(2):
        train_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        train_step()
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t0) / reps
    del net, opt, T, G, grad
    conv = convergence(qst, n, prec, f.device) if long_run else None
    return {"parameters": 2 * H * D + H + D,
            "forward_us": round(fwd_us, 1), "forward_GB_s": round(fwd_bytes / (fwd_us * 1e-6) / 1e9, 1),
            "forward_hbm_frac": round(fwd_bytes / (fwd_us * 1e-6) / 8e12, 3),
            "backward_us": round(bwd_us, 1), "backward_GB_s": round(bwd_bytes / (bwd_us * 1e-6) / 1e9, 1),
            "backward_hbm_frac": round(bwd_bytes / (bwd_us * 1e-6) / 8e12, 3),
            "nnqst_train_steps_per_s": round(1.0 / step_s, 1),
            "nnqst_1000_steps": conv,
            "note": "train step = network forward, qst_likelihood, qst_grad_product, network backward, "
                    "Rprop (lr 1e-3, qst_rprop_step) over all parameters"}


def convergence(qst, n, prec, dev, steps=1000):
    """NN-QST as the paper runs it: a fresh network trained by Rprop (lr
    1e-3) for 1000 steps on frequencies of 10^7 shots of a Haar-random pure
    state (p computed by the library from T0 = [psi 0 ... 0]); wall time,
    and F_q of the network's state against the target after the run."""
    import numpy as np
    import torch

    import synth as S

    d = 1 << n
    g = S.rng(13)
    psi = S.haar_vector(g, d)
    ct = np.complex128 if prec == "f64" else np.complex64
    T0 = np.zeros((d, d), dtype=ct)
    T0[:, 0] = psi
    rho0, _ = qst.state_map(torch.from_numpy(T0).to(dev), prec)
    p0 = qst.povm_probs(rho0, prec).double().cpu().numpy()
    del rho0
    p0 = np.clip(p0, 0.0, None)
    f_np = S.multinomial_freqs(g, 10_000_000, p0 / p0.sum())
    rt = torch.float64 if prec == "f64" else torch.float32
    f = torch.from_numpy(f_np).to(dev, rt)
    x = (f.double() / f.double().sum()).to(rt)
    net = qst.MappingNetwork(n, dtype=rt, device=dev, generator=torch.Generator().manual_seed(14))
    opt = qst.Rprop(net.parameters(), lr=1e-3)
    W = torch.from_numpy(psi.astype(ct).reshape(d, 1)).to(dev)
    with torch.no_grad():
        f_start = float(qst.fidelity_lowrank(net(x, prec).contiguous(), W, prec).item())
    trace = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(1, steps + 1):
        opt.zero_grad(set_to_none=True)
        L = qst.likelihood(net(x, prec), f, prec)
        L.backward()
        opt.step()
        if k % 100 == 0:
            with torch.no_grad():
                trace.append(qst.fidelity_lowrank(net(x, prec).contiguous(), W, prec))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    trace = [round(float(t.item()), 6) for t in trace]
    out = {"seconds": round(wall, 2), "loss_last": float(L.item()), "fidelity_start": round(f_start, 6),
           "fidelity_every_100_steps": trace,
           "target": "Haar-random pure state, 10^7 shots; F_q of the network's rho against it",
           "note": "wall time includes the ten fidelity evaluations"}
    del net, opt, f, x
    return out


def _oracle_eval(O, Tq, fq):
    """One full forward + adjoint evaluation by the oracle; returns p, L, grad."""
    n = O.n_qubits_of(Tq.shape[0])
    rho, tau = O.state_map(Tq)
    p = O.probs_real(rho)
    L = O.nll_vec(p, fq)
    G = O.adjoint(O.cotangent(p, fq), n)
    return p, L, (2.0 / tau) * (G @ Tq)


def general_povms(qst, prec, dev, reps=10):
    """General product POVMs (a K-element POVM per qubit, several settings):
    (a) the Pauli-6 POVM, M_(+-j) = (I +- sigma_j)/6, on every qubit at
    N = 10 (6^10 = 60,466,176 outcomes); (b) the three Pauli bases as three
    settings of K = 2 projectors at N = 11.  One step = qst_likelihood_general
    + qst_grad_product.  The real per-qubit factor passes are timed by the
    library's events (scope general_factor_pass) and their achieved GB/s is
    from algorithmic bytes: a pass over [A][m][B] reads A m_in B values and
    writes A m_out B (the first adjoint pass also reads f; the last one of
    each setting after the first reads its output to accumulate)."""
    import numpy as np
    import torch

    import synth as S
    from paper_2207_05341_amd import _lib

    I2 = np.eye(2, dtype=complex)
    X = np.array([[0, 1], [1, 0]], dtype=complex)
    Y = np.array([[0, -1j], [1j, 0]])
    Z = np.diag([1.0, -1.0]).astype(complex)
    pauli6 = np.array([(I2 + X) / 6, (I2 - X) / 6, (I2 + Y) / 6, (I2 - Y) / 6, (I2 + Z) / 6, (I2 - Z) / 6])
    bases = [np.array([(I2 + P) / 2, (I2 - P) / 2]) for P in (X, Y, Z)]
    ct = np.complex128 if prec == "f64" else np.complex64
    rt = np.float64 if prec == "f64" else np.float32
    rb = 8 if prec == "f64" else 4
    g = S.rng(31)
    out = {}
    for key, n, K, settings in (("pauli6_n10", 10, 6, [np.array([pauli6] * 10)]),
                                ("pauli_bases_3settings_n11", 11, 2, [np.array([b] * 11) for b in bases])):
        d, DK, Sn = 1 << n, K ** n, len(settings)
        T = torch.from_numpy(S.ginibre(g, d).astype(ct)).to(dev)
        fs = np.stack([S.multinomial_freqs(g, 10_000_000, S.porter_thomas_probs(g, DK, 0.1)) for _ in range(Sn)])
        f = torch.from_numpy(fs.astype(rt)).to(dev)
        povms = np.stack(settings)

        def stepg():
            o, tau, G, _ = qst.likelihood_forward_general(T, f, povms, prec)
            return qst.grad_product(G, T, tau, prec)

        for _ in range(2):
            stepg()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            stepg()
        torch.cuda.synchronize()
        step_s = (time.perf_counter() - t0) / reps
        _lib.profile_report(reset=True)
        _lib.profile_enable(True, "general_factor_pass")
        for _ in range(reps):
            stepg()
        torch.cuda.synchronize()
        _lib.profile_enable(False)
        calls, ms = _lib.profile_report(reset=True)["general_factor_pass"]
        fwd = sum(4 ** (j - 1) * K ** (n - j) * (4 + K) for j in range(1, n + 1))
        adj = fwd + DK + 4 ** n  # f read by the first adjoint pass; h read back by the last
        nbytes = rb * (Sn * (fwd + adj) - 4 ** n)  # the first setting writes h without reading it
        gbs = nbytes * reps / (ms * 1e-3) / 1e9
        out[key] = {"n_qubits": n, "K": K, "settings": Sn, "outcomes_per_setting": DK,
                    "step_ms": round(1e3 * step_s, 3), "factor_passes_ms_per_step": round(ms / reps, 3),
                    "factor_pass_launches_per_step": calls // reps,
                    "factor_passes_GB_s": round(gbs, 1), "factor_passes_hbm_frac": round(gbs / 8000.0, 3)}
        del T, f
    return out


def cpu_baseline(T, f, prec):
    """FP64 oracle timed on a bounded sample of the same N = 11 workload (the
    measured precision's T and f widened to FP64): full forward + adjoint
    evaluations, first with every BLAS thread of the host (up to 3 or
    20 s), then with one thread (up to 2 or 25 s).  Returns the record and
    the outputs of the first evaluation, which serve as the reference for
    the accuracy of the GPU paths on the same inputs."""
    import numpy as np

    import oracle as O

    try:
        from threadpoolctl import threadpool_info, threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_info = threadpool_limits = None
    ct = np.complex128 if prec == "f64" else np.complex64
    rt = np.float64 if prec == "f64" else np.float32
    Tq = T.astype(ct).astype(np.complex128)
    fq = f.astype(rt).astype(np.float64)

    def leg(max_evals, max_s):
        evals, ref = 0, None
        t0 = time.perf_counter()
        while True:
            out = _oracle_eval(O, Tq, fq)
            ref = ref or out
            evals += 1
            el = time.perf_counter() - t0
            if evals >= max_evals or el > max_s:
                return evals, el, ref

    threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1]) if threadpool_info else (os.cpu_count() or 1)
    evals, el, ref = leg(3, 20.0)
    single = None
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            e1, t1, _ = leg(2, 25.0)
        single = {"value": e1 / t1, "unit": "evals/s", "cores": 1, "kind": "oracle",
                  "sample": f"{e1} full forward+adjoint evaluations in FP64 numpy with one BLAS thread ({t1:.1f} s)"}
    rec = {"value": evals / el, "unit": "evals/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{evals} full forward+adjoint evaluations of the N=11 workload in FP64 numpy "
                     f"({el:.1f} s, {threads} BLAS threads)",
           "single_thread": single}
    return rec, ref


def note(msg):
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures the single-GPU likelihood path; this build uses exactly one GPU "
              "(--gpus 1).  Multi-GPU sharding is a design note only.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2207_05341_amd as qst

    dev = torch.device("cuda:0")
    n, d = args.n, 1 << args.n
    T_np, f_np = make_inputs(n)
    if args.calib_copy_mib > 0:
        src = torch.ones(args.calib_copy_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)
        torch.cuda.synchronize()
        del src, dst

    # the GPU FP64 path on the unrounded inputs, for max|dp| vs FP64
    T64, f64 = to_prec(T_np, f_np, "f64", dev)
    out64, g64 = step(qst, T64, f64, "f64")
    rho64, _ = qst.state_map(T64, "f64")
    p64 = qst.povm_probs(rho64, "f64")
    del rho64, T64, f64
    torch.cuda.synchronize()

    def measure(prec, steps, warmup, route="one_call"):
        """The path's outputs (for accuracy); a per-kernel breakdown (each
        scope timed alone, in warmed loops: the events bracketing a scope
        add their queue time to it only); then the timed loop, in which
        only the dominant kernel is bracketed by events."""
        T, f = to_prec(T_np, f_np, prec, dev)
        out, grad = step(qst, T, f, prec, route)
        rho, _ = qst.state_map(T, prec)
        p = qst.povm_probs(rho, prec)  # the forward map alone, for max|dp|
        del rho
        torch.cuda.synchronize()
        res = {"p": p.double().cpu().numpy(), "L": float(out[0].item()),
               "grad": grad.to(torch.complex128).cpu().numpy()}
        acc = {
            "max_dp_rel": float((p.double() - p64).abs().max() / p64.abs().max()),
            "L_rel": float(abs(out[0].item() - out64[0].item()) / abs(out64[0].item())),
            "grad_rel": float(torch.linalg.vector_norm(grad.to(torch.complex128) - g64)
                              / torch.linalg.vector_norm(g64)),
        }
        del p, out, grad
        # the scopes and the dominant one from a short loop that times them all
        _, names = time_steps(qst, T, f, prec, 3, 2, only="", route=route)
        dom = max(names, key=lambda k: names[k][1] / names[k][0])
        sec, kdom = time_steps(qst, T, f, prec, steps, warmup, only=dom, route=route, settle_s=args.settle_ms / 1e3)
        breakdown = {dom: kdom[dom]}
        for name in names:
            if name != dom:
                breakdown.update(time_steps(qst, T, f, prec, steps, 3, only=name, route=route)[1])
        return sec, breakdown, dom, kdom, acc, res

    sec, kern, dom, kdom, acc, res_main = measure(args.prec, args.steps, args.warmup)
    note(f"headline {args.prec}: {1e3 * sec:.4f} ms per step")
    kern_us = {k: 1e3 * ms / calls for k, (calls, ms) in kern.items()}

    # roofline of the dominant kernel (largest share of the step), its
    # duration from the events of the timed loop
    roofline = None
    if dom in kdom:
        avg_s = kdom[dom][1] * 1e-3 / kdom[dom][0]
        if dom.startswith("hemm") or dom.startswith("herk"):
            # Algorithmic flops of the algorithm each kernel runs: the fp32 /
            # fp64 products use the 3M form, three real products per complex
            # product (6 real flop per complex multiply-add): 3 d^2 (d+1) for
            # the Hermitian T T^dagger (lower triangle), 6 d^3 for G' T.  The
            # bf16 products use four real products per complex product (8 flop
            # per complex multiply-add), three split products for G' T
            # (24 d^3).  The conventional count, 8 flop per complex
            # multiply-add (4 d^2 (d+1) and 8 d^3), is reported beside it.
            herk = dom.startswith("herk")
            counted = 4.0 * d * d * (d + 1) if herk else 8.0 * d ** 3
            x6 = dom.endswith("x6")
            bf16 = dom.endswith(("bf16", "bf16x3"))
            peak_key = "bf16" if (bf16 or x6) else ("f64" if dom.endswith("f64") else "f32")
            if x6:
                # three real products per complex product, six bf16 products
                # per real product; T T^dagger on 128 x 128 lower tiles (the
                # diagonal tiles in full): 3 x 6 x 2 x 128^2 x d per tile
                t = d // 128
                executed = (36.0 * 128 * 128 * d * (t * (t + 1) // 2)) if herk else 36.0 * d ** 3
            else:
                executed = counted * (0.75 if not bf16 else (1.0 if herk else 3.0))
            ach = executed / avg_s / 1e12
            if x6:
                form = "36 x 128^2 d per lower 128-tile" if herk else "36 d^3"
            else:
                form = ("3 d^2(d+1)" if herk else "6 d^3") if not bf16 else ("4 d^2(d+1)" if herk else "24 d^3")
            roofline = {"kernel": dom, "bound": "mfma", "achieved": ach, "peak": PEAK_TFLOPS[peak_key],
                        "unit": "TFLOP/s", "frac": ach / PEAK_TFLOPS[peak_key], "traffic": traffic_of(dom),
                        "algorithmic_per_launch": f"{executed:.4g} flop ({form}, d={d}: "
                                                  + ("3M complex product, 3 real products, 6 bf16 products "
                                                     "each" if x6 else "3M complex product, 3 real products"
                                                     if not bf16 else "4 real products per complex product")
                                                  + ")",
                        "avg_launch_us": avg_s * 1e6, "launches": kdom[dom][0],
                        "counted_per_launch": f"{counted:.4g} flop ({'4d^2(d+1)' if herk else '8d^3'}, "
                                              "8 flop per complex multiply-add)",
                        "counted_tflops": counted / avg_s / 1e12}
    # POVM passes: achieved GB/s from algorithmic bytes.  N = 11 plan: pass 0
    # contracts qubits 6..11 of rho (lower triangle read) into X[(r, c)][kd]
    # with (r, c) the 528 lower pairs of the 5 remaining qubits and kd 4^6
    # digits; the fused pass reads X and f and writes the adjoint
    # intermediate in place; adjoint pass 0 writes G' in full.
    cb = 16 if args.prec == "f64" else 8
    rb = 8 if args.prec == "f64" else 4
    pairs, kd = 32 * 33 // 2, 4 ** 6
    tri = d * (d + 1) // 2
    povm_bytes = {
        "povm_fwd_p0": tri * cb + pairs * kd * cb,
        "povm_fused": 2 * pairs * kd * cb + 4 ** n * rb,
        "povm_adj_p0": pairs * kd * cb + d * d * cb,
    }
    povm_gbs = {k: v / (kern_us[k] * 1e-6) / 1e9 for k, v in povm_bytes.items() if k in kern_us} if n == 11 else {}

    paths, path_res = {}, {}
    if not args.no_variants:
        for prec in ("f64", "f32", "bf16", "f32x6"):
            if prec == args.prec:
                continue
            s2, k2, _, _, a2, path_res[prec] = measure(prec, max(10, args.steps // 2), 3)
            note(f"path {prec}: {1e3 * s2:.4f} ms per step")
            paths[prec] = {"evals_per_s": 1.0 / s2, "ms_per_step": 1e3 * s2, "accuracy_vs_f64": a2,
                           "kernels_us": {k: round(1e3 * ms / c, 2) for k, (c, ms) in k2.items()}}
        s2, k2, _, _, a2, _ = measure(args.prec, max(10, args.steps // 2), 3, route="two_calls")
        note(f"path {args.prec} two calls: {1e3 * s2:.4f} ms per step")
        paths[args.prec + "_two_calls"] = {
            "evals_per_s": 1.0 / s2, "ms_per_step": 1e3 * s2, "accuracy_vs_f64": a2,
            "kernels_us": {k: round(1e3 * ms / c, 2) for k, (c, ms) in k2.items()},
            "note": "qst_likelihood (G' returned) then qst_grad_product"}
        s2, k2, _, _, a2, _ = measure(args.prec, max(10, args.steps // 2), 3, route="separate")
        note(f"path {args.prec} separate calls: {1e3 * s2:.4f} ms per step")
        paths[args.prec + "_separate_calls"] = {
            "evals_per_s": 1.0 / s2, "ms_per_step": 1e3 * s2, "accuracy_vs_f64": a2,
            "kernels_us": {k: round(1e3 * ms / c, 2) for k, (c, ms) in k2.items()},
            "note": "qst_state_map, qst_povm_probs, qst_nll, qst_nll_backward with p stored"}
    del p64, g64

    Tm, fm = to_prec(T_np, f_np, args.prec, dev)
    modes = fids = net = None
    if not args.headline_only:
        modes = state_maps(qst, Tm, fm, args.prec)
        note("state maps done")
        fids = fidelities(qst, Tm, args.prec, f=fm)
        note("fidelities done")
        net = network(qst, fm, args.prec, long_run=args.nnqst_run)
        note("network done")
    absp = None if args.no_long else abs_projection(qst, args.prec, fm.device)
    genp = None if args.no_long else general_povms(qst, args.prec, dev)
    if not args.no_long:
        note("absolute projection and general POVMs done")
    del Tm, fm
    batch = None
    if not args.no_batched:
        batch = batched(qst, args.prec, dev)
        if args.prec != "f64":  # the FP64 path's batch, for its speed at its accuracy
            batch["f64"] = batched(qst, "f64", dev)
        note("batched form done")
    cpu, acc_oracle = None, None
    if not args.no_cpu_baseline:
        # the timed oracle leg also gives the reference outputs for the
        # measured precision's inputs; the FP64 path's reference (unrounded
        # inputs) is one more untimed evaluation when that path ran
        import oracle as O

        cpu, ref = cpu_baseline(T_np, f_np, args.prec)
        note("CPU oracle leg done")
        refs = {args.prec: ref}
        storage = {"f64": "f64", "f32": "f32", "bf16": "f32", "f32x6": "f32"}  # complex64 T except FP64
        for prec in path_res:
            if storage[prec] == storage[args.prec]:
                refs[prec] = ref
            elif storage[prec] == "f64":
                refs[prec] = _oracle_eval(O, T_np.astype(np.complex128), f_np.astype(np.float64))
            else:
                refs[prec] = _oracle_eval(O, T_np.astype(np.complex64).astype(np.complex128),
                                          f_np.astype(np.float32).astype(np.float64))

        def vs_oracle(res, r):
            pw, Lw, gw = r
            return {"max_dp_rel": float(np.max(np.abs(res["p"] - pw)) / np.max(np.abs(pw))),
                    "L_rel": abs(res["L"] - Lw) / abs(Lw),
                    "grad_rel": float(np.linalg.norm(res["grad"] - gw) / np.linalg.norm(gw))}

        acc_oracle = vs_oracle(res_main, refs[args.prec])
        for prec, res in path_res.items():
            paths[prec]["accuracy_vs_oracle"] = vs_oracle(res, refs[prec])
        del refs, ref

    line = {
        "metric": METRIC,
        "value": 1.0 / sec,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "settle_ms": args.settle_ms,
        "ms_per_step": 1e3 * sec,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": f"N={n} single state: T {d}x{d} complex Ginibre, {4 ** n} tetrahedral-POVM "
                               f"outcomes, f from 10^7 multinomial shots; forward+adjoint as one call, qst_likelihood_grad "
                               f"(p and G' not stored)",
                   "n_qubits": n, "precision": args.prec, "precision_note": PREC_NOTE[args.prec],
                   "parallelism": "none (1 GPU)"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "accuracy_vs_oracle": acc_oracle,
        "accuracy_vs_f64": acc,
        "kernels_us": {k: round(v, 2) for k, v in sorted(kern_us.items())},
        "kernels_sum_us": round(sum(kern_us.values()), 1),
        "povm_pass_gbs": {k: round(v, 1) for k, v in povm_gbs.items()},
        "paths": paths,
        "state_maps": modes,
        "abs_projection": absp,
        "general_povm": genp,
        "fidelity": fids,
        "network": net,
        "batched": batch,
        "device": torch.cuda.get_device_name(0),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
