"""Benchmark of the MOMFBD hot path on one MI355X.

Workload (full-field plain MOMFBD): 1024 x 1024 frames cut into 64 x 64
patches at stride 32 (961 patches), 12 frames, 2 objects (a wideband
channel and a +1 wave defocus phase-diversity channel sharing the modal
coefficients), 66 Zernike modes (Noll 2..67), D/r0 from 5 to 20 across the
field.  One step = one momfbd_loss_grad call: modal synthesis, pupil, PSF,
OTF, Wiener object, FP64 patch loss, adjoint and gradient contraction for
every (patch, channel, frame).  Inputs are resident in HBM before timing.

Prints ONE JSON line.  --gpus N > 1 is refused (one-GPU build).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3      # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0

N = 64
FFT_C2C = 5.0 * N * N * np.log2(N * N)       # FFTW convention, 245 760 flop
FFT_REAL = 0.5 * FFT_C2C                      # r2c or c2r, 122 880 flop
FLOP_PER_UNIT = 2 * FFT_C2C + 2 * FFT_REAL    # 737 280: 2 c2c + r2c + c2r
HALF_BYTES = N * (N // 2 + 1) * 8             # one data half spectrum, 16 896 B

# nominal FFT flops each kernel performs per unit (recomputation not counted)
KERNEL_FLOP_PER_UNIT = {"forward": FFT_C2C + FFT_REAL, "adjoint": FFT_C2C + FFT_REAL}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_inputs(dev):
    """Plan, data spectra D and an evaluation point alpha, all on the GPU.

    D = O_p S_pcj + N_pcj per patch: O_p the spectrum of the apodized patch of
    a k^-3 scene, S the OTFs of the true Kolmogorov coefficients (computed by
    the library's forward model), N the spectrum of apodized 1% noise."""
    import torch

    import synth
    from paper_2505_10639_amd import Plan

    g = synth.config1_geometry()
    pr = synth.make_problem(1, N=N, P=1, J=g["J"], M=g["M"], channels=g["channels"],
                            gamma=g["gamma"], border=g["border"], objects=np.zeros((1, 2, N, N)))
    P, C, J, M = g["P"], g["C"], g["J"], g["M"]
    plan = Plan(N, P, J, pr.channel_object, pr.pupil, pr.basis, pr.diversity, dev)
    win = torch.from_numpy(pr.window).to(dev)
    alpha_true = torch.from_numpy(synth.config1_alpha()).to(dev)
    scene = torch.from_numpy(synth.config1_object().astype(np.float32)).to(dev)
    # object spectra per patch through a 1-channel, 1-frame plan
    aux = Plan(N, P, 1, [0], pr.pupil[:1], pr.basis[:1, :1], None, dev)
    Ohat = aux.prepare_data(scene.reshape(1, 1, g["H"], g["W"]).contiguous(), g["stride"], win)
    aux.close()
    _, S = plan.forward(alpha_true, want_psf=False)
    gen = torch.Generator(device=dev)
    gen.manual_seed(synth.SEED_ROOT + 1)
    noise = 0.01 * torch.randn((C, J, g["H"], g["W"]), generator=gen, device=dev)
    Nhat = plan.prepare_data(noise, g["stride"], win)
    del noise
    D = (Ohat * S + Nhat).contiguous()
    del S, Nhat, Ohat
    rng = np.random.default_rng(synth.SEED_ROOT + 2)
    pert = torch.from_numpy((0.3 * rng.standard_normal((P, J, M))).astype(np.float32)).to(dev)
    alpha = (alpha_true + pert).contiguous()
    torch.cuda.synchronize()
    return plan, D, alpha, g


def cpu_baseline(D_host, alpha_host, g, budget_s=12.0):
    """The FP64 oracle on a bounded sample of the same workload (the first
    patches, until the time budget is used)."""
    import oracle
    import synth
    from threadpoolctl import threadpool_info

    pr = synth.make_problem(1, N=N, P=1, J=g["J"], M=g["M"], channels=g["channels"],
                            gamma=g["gamma"], border=g["border"], objects=np.zeros((1, 2, N, N)))
    t0 = time.perf_counter()
    n = 0
    while True:
        oracle.evaluate_patch(alpha_host[n], D_host[n], pr.basis, pr.diversity, pr.pupil,
                              pr.channel_object, pr.gamma)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= len(D_host):
            break
    threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    return {"value": n * g["J"] / el, "unit": "patch-frame loss+grad evals/s", "cores": threads,
            "kind": "oracle",
            "sample": f"first {n} of {g['P']} patches ({n * g['J']} patch-frames, "
                      f"{n * g['J'] * g['C']} units), {el:.1f} s, FP64 direct DFT"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy three times (for scaling "
                         "hardware byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the patches are "
              "independent, so a multi-GPU run would shard them by patch block with no "
              "exchange step.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2505_10639_amd import momfbd_profile_start, momfbd_profile_stop

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "copies": 3}), flush=True)
        return
    log("building inputs")
    plan, D, alpha, g = build_inputs(dev)
    P, C, J = g["P"], g["C"], g["J"]
    units = P * C * J
    loss = torch.empty(P, dtype=torch.float64, device=dev)
    grad = torch.empty_like(alpha)

    def step():
        plan.loss_grad(alpha, D, g["gamma"], None, True, loss, grad)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        step()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    assert torch.isfinite(loss).all(), "non-finite loss"

    # per-kernel durations: HIP events recorded by the library on the launch stream
    log("per-kernel timing")
    momfbd_profile_start(plan.handle, 8 * args.steps)
    for _ in range(args.steps):
        step()
    kern = momfbd_profile_stop(plan.handle)
    kern_avg = {k: v[0] / v[1] for k, v in kern.items()}
    dom = max(kern_avg, key=kern_avg.get)
    fl = KERNEL_FLOP_PER_UNIT.get(dom)
    if fl is not None:
        achieved = fl * units / (kern_avg[dom] * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": achieved,
                "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": None,
                "avg_ms": kern_avg[dom]}
    else:
        achieved = 2 * HALF_BYTES * units / (kern_avg[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                "avg_ms": kern_avg[dom]}

    step_tflops = FLOP_PER_UNIT * units / (ms * 1e-3) / 1e12
    out = {
        "metric": "patch-frame loss+grad evals/s",
        "value": P * J / (ms * 1e-3),
        "unit": "patch-frame evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "full-field plain MOMFBD: 1024x1024 frames, 961 patches of "
                               "64x64 at stride 32, 12 frames, 2 objects (wideband + "
                               "phase diversity), 66 Zernike modes, D/r0 5..20",
                   "patches": P, "frames": J, "channels": C, "objects": g["K"],
                   "modes": g["M"], "N": N, "units_per_step": units},
        "roofline": roof,
        "units_per_s": units / (ms * 1e-3),
        "step_nominal_fft_tflops": step_tflops,
        "step_frac_of_fp32_peak": step_tflops / PEAK_FP32_VECTOR_TFLOPS,
        "kernels_avg_ms": kern_avg,
    }
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        n_s = 512
        D_h = D[:n_s].cpu().numpy()
        a_h = alpha[:n_s].cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(D_h, a_h, g, args.cpu_budget)
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
