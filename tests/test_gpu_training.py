"""Training-loop shape: Adam on T through the likelihood path, with rho and p
recomputed in the backward (nothing of length 4^N kept between passes).

* N = 6, FP64, 200 steps: the whole trajectory (losses, final T, fidelity)
  against the oracle's FP64 Adam loop from the same T0.
* N = 12, FP32 (T 4096 x 4096 complex64, 16,777,216 outcomes), target a
  rank-8 Ginibre state, 10^8-shot frequencies (seed 10), 200 Adam steps:
  steps/s, peak HBM, and fidelity against the target; the loss and fidelity
  after 2 steps against the oracle's FP64 Adam after 2 steps.

Adam: lr 1e-2, betas (0.9, 0.999), eps 1e-12 (gradient entries are small).
"""
import json
import math
import os
import time

import numpy as np
import pytest

import oracle as O
import synth as S

torch = pytest.importorskip("torch")
qst = pytest.importorskip("paper_2207_05341_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
LR, BETAS, EPS = 1e-2, (0.9, 0.999), 1e-12


def say(*a):
    print(*a, flush=True)


def gpu_fidelity_lowrank(T, W):
    """F_q(T T^dagger / tau, W W^dagger / tw) by the library
    (qst_fidelity_lowrank, checked against the oracle in
    test_gpu_fidelity.py)."""
    return float(qst.fidelity_lowrank(T.contiguous(), W).item())


def train_gpu(T0, f, steps, prec, mode="recompute"):
    T = torch.nn.Parameter(torch.from_numpy(T0).to(DEV))
    fg = torch.from_numpy(f).to(DEV)
    opt = torch.optim.Adam([T], lr=LR, betas=BETAS, eps=EPS)
    losses = []
    for _ in range(steps):
        opt.zero_grad(set_to_none=True)
        L = qst.likelihood(T, fg, prec, mode=mode)
        L.backward()
        opt.step()
        losses.append(L.detach())
    return T.detach(), [float(x) for x in torch.stack(losses).cpu()]


def test_training_trajectory_n6_f64():
    say("training N=6 FP64, 200 Adam steps, GPU vs oracle")
    g = S.rng(60)
    n, d = 6, 64
    T0 = S.ginibre(g, d)
    W = S.ginibre(g, d, 4)
    f = S.multinomial_freqs(g, 100_000, O.probs_real(O.state_map(W)[0]))
    Tg, losses = train_gpu(T0, f, 200, "f64", mode="recompute")
    To, lo = O.adam_train(T0, f, steps=200, lr=LR, betas=BETAS, eps=EPS)
    Tg = Tg.cpu().numpy()
    dl = max(abs(a - b) / abs(b) for a, b in zip(losses, lo))
    dT = np.linalg.norm(Tg - To) / np.linalg.norm(To)
    fg, fo = O.fidelity_q_lowrank(O.state_map(Tg)[0], W), O.fidelity_q_lowrank(O.state_map(To)[0], W)
    say(f"  max rel loss diff {dl:.2e}, rel T diff {dT:.2e}, fidelity gpu {fg:.10f} oracle {fo:.10f}")
    assert dl <= 1e-9 and dT <= 1e-7 and abs(fg - fo) <= 1e-8
    assert losses[-1] < losses[0]


def test_training_n12_f32():
    say("training N=12 FP32, 200 Adam steps, recompute and fused modes")
    g = S.rng(10)
    n, d = 12, 4096
    T0 = S.ginibre(g, d).astype(np.complex64)
    W = S.ginibre(g, d, 8)
    rho0, tw_unused = O.state_map(W)
    p0 = O.probs_real(rho0)
    del rho0
    f = S.multinomial_freqs(g, 100_000_000, p0).astype(np.float32)
    del p0
    Wg = torch.from_numpy(W.astype(np.complex64)).to(DEV)

    # 2 steps, compared with the oracle's FP64 Adam after 2 steps
    T2, l2 = train_gpu(T0, f, 2, "f32", mode="recompute")
    f2 = gpu_fidelity_lowrank(T2, Wg)
    T2b, l2b = train_gpu(T0, f, 2, "f32", mode="fused")
    f2b = gpu_fidelity_lowrank(T2b, Wg)
    say(f"  GPU after 2 steps: recompute losses {l2} fidelity {f2:.8f}; fused losses {l2b} fidelity {f2b:.8f}")
    t0 = time.perf_counter()
    To, lo = O.adam_train(T0.astype(np.complex128), f.astype(np.float64), steps=2, lr=LR, betas=BETAS, eps=EPS)
    fo = O.fidelity_q_lowrank(O.state_map(To)[0], W)
    say(f"  oracle after 2 steps ({time.perf_counter() - t0:.0f} s): losses {lo}, fidelity {fo:.8f}")
    for ls in (l2, l2b):
        for a, b in zip(ls, lo):
            assert abs(a - b) / abs(b) <= 1e-5
    assert abs(f2 - fo) <= 1e-5 and abs(f2b - fo) <= 1e-5

    # 200 steps, timed, in both modes: rho and p recomputed in the backward,
    # and the fused call (p never stored; G' kept between forward and backward)
    rec = {"config": "N=12 FP32 training, 200 Adam steps (lr 1e-2), target rank-8 Ginibre, 10^8 shots",
           "fidelity_after_2_gpu_recompute": f2, "fidelity_after_2_gpu_fused": f2b,
           "fidelity_after_2_oracle": fo,
           "fidelity_start": gpu_fidelity_lowrank(torch.from_numpy(T0).to(DEV), Wg)}
    for mode in ("recompute", "fused"):
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        t0 = time.perf_counter()
        T200, l200 = train_gpu(T0, f, 200, "f32", mode=mode)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        free1, total = torch.cuda.mem_get_info()
        rec[mode] = {"steps_per_s": 200 / dt, "ms_per_step": 1e3 * dt / 200,
                     "peak_torch_allocated_GiB": torch.cuda.max_memory_allocated() / 2 ** 30,
                     "device_used_GiB": (total - free1) / 2 ** 30,
                     "loss_first": l200[0], "loss_last": l200[-1],
                     "fidelity_final": gpu_fidelity_lowrank(T200, Wg)}
        assert all(math.isfinite(x) for x in l200)
        assert l200[-1] < l200[0] and rec[mode]["fidelity_final"] > rec["fidelity_start"]
        del T200
    say("  " + json.dumps(rec))
    if os.path.isdir("gpurun_out"):
        with open(os.path.join("gpurun_out", "config5_training.json"), "w") as fh:
            json.dump(rec, fh)
