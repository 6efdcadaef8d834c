"""Benchmark of the MOMFBD hot path on one MI355X.

Headline workload (full-field plain MOMFBD): 1024 x 1024 frames cut into
64 x 64 patches at stride 32 (961 patches), 12 frames, 2 objects (a wideband
channel and a +1 wave defocus phase-diversity channel sharing the modal
coefficients), 66 Zernike modes (Noll 2..67), D/r0 from 5 to 20 across the
field.  One step = one momfbd_loss_grad call: modal synthesis, pupil, PSF,
OTF, Wiener object, FP64 patch loss, adjoint and gradient contraction for
every (patch, channel, frame).  Inputs are resident in HBM before timing.

A second block ("large_multi_object") times the same step on 2048 x 2048
frames in 128 x 128 patches at stride 64 (961 patches), 24 frames, four
objects at lambda/lambda_0 = 1.0/0.95/1.05/1.1, 150 modes, D/r0 = 15, with
the object smoothness prior as a per-frequency gamma.

Prints ONE JSON line.  --gpus N > 1 is refused (one-GPU build).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_VECTOR_TFLOPS = 157.3      # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0


def fft_flops(N):
    """Nominal FFT flops (FFTW convention): c2c, and r2c or c2r, of N x N."""
    c2c = 5.0 * N * N * np.log2(N * N)
    return c2c, 0.5 * c2c


def unit_flops(N):
    """Per (patch, channel, frame): 2 c2c + r2c + c2r for loss and gradient;
    forward and adjoint kernels each carry one c2c and one real transform."""
    c2c, real = fft_flops(N)
    return 2 * c2c + 2 * real, {"forward": c2c + real, "forward_object": c2c + real,
                                "adjoint": c2c + real}


# HBM traffic per launch of the transform and object kernels on the two
# timed workloads, from rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per
# dispatch), each scaled by the reading of the same counter for a plain
# 256 MiB device copy (FETCH_SIZE reads half the copied bytes: factor 2.0;
# WRITE_SIZE factor 1.0).  Valid only for the kernel sources they were taken
# on (a changed source hash reports null) and looked up by patch size and by
# the value of the launch-schedule knob that changes the kernel's traffic.
KERNEL_SOURCES = {
    ("adjoint", 64): ["kernels64.hip", "ops64.h", "fft_lane.h", "internal.h"],
    ("forward", 64): ["kernels64.hip", "ops64.h", "fft_lane.h", "internal.h"],
    ("object", 64): ["object.hip", "internal.h"],
    ("adjoint", 128): ["kernels128.hip", "ops128.h", "fft_lane.h", "internal.h"],
    ("forward", 128): ["kernels128.hip", "ops128.h", "fft_lane.h", "internal.h"],
    ("object", 128): ["object.hip", "internal.h"],
}
COPY_FETCH_SCALE = 1.9997991127905397   # 256 MiB copy: FETCH_SIZE read 131085.2 KiB
COPY_WRITE_SCALE = 1.0    # 256 MiB copy: WRITE_SIZE read 262144 KiB
# per (kernel, N): the knob and, per value of it, (HBM bytes read, written)
# per launch
COUNTED_TRAFFIC = {
    ("adjoint", 64): {"sources_sha1": "0a485a0ac71b", "knob": "xcd_adjoint",
                      "by_value": {1: (895264574, 94470144), 0: (1094290663, 94470144)}},
    ("forward", 64): {"sources_sha1": "0a485a0ac71b", "knob": "xcd_forward",
                      "by_value": {0: (94923414, 405011347), 1: (94926936, 401195873)}},
    ("object", 64): {"sources_sha1": "380df0fcb916", "knob": "object_pairs_per_thread",
                     "by_value": {1: (729207247, 32782494)}},
    ("adjoint", 128): {"sources_sha1": "64d2e7533f56", "knob": "xcd_adjoint",
                       "by_value": {1: (11984010648, 1511522304), 0: (13304748748, 1511522304)}},
    ("forward", 128): {"sources_sha1": "64d2e7533f56", "knob": "xcd_forward",
                       "by_value": {0: (3215663020, 8833985947), 1: (3230672758, 8745003407)}},
    ("object", 128): {"sources_sha1": "380df0fcb916", "knob": "object_pairs_per_thread",
                      "by_value": {1: (10901727308, 257959848)}},
}


def sources_sha(kernel, N=64):
    h = hashlib.sha1()
    for f in KERNEL_SOURCES.get((kernel, N), []):
        with open(os.path.join(ROOT, "paper_2505_10639_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def counted_traffic(kernel, schedule, N=64):
    rec = COUNTED_TRAFFIC.get((kernel, N))
    if rec is None or rec["sources_sha1"] != sources_sha(kernel, N):
        return None
    rw = rec["by_value"].get(schedule.get(rec["knob"]))
    return None if rw is None else rw[0] + rw[1]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def build_full_field(dev):
    """Plan, data spectra D and an evaluation point alpha of the headline
    workload, all on the GPU.

    D = O_p S_pcj + N_pcj per patch: O_p the spectrum of the apodized patch of
    a k^-3 scene, S the OTFs of the true Kolmogorov coefficients (computed by
    the library's forward model), N the spectrum of apodized 1% noise."""
    import torch

    import synth
    from paper_2505_10639_amd import Plan

    g = synth.config1_geometry()
    N = g["N"]
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
    # noise power of the apodized noise per frequency bin (for the
    # Loefdahl-Scharmer filter of the post-processing block)
    eta = 1e-4 * float(np.sum(pr.window.astype(np.float64) ** 2))
    g = dict(g, channel_object=[int(k) for k in pr.channel_object],
             support_frac=support_fraction(pr.pupil, pr.channel_object, N), noise_power=eta)
    return plan, D, alpha, g["gamma"], g


def postprocess_block(plan, D, alpha, gamma, g, reps=10):
    """Object post-processing of the restored full field: the Wiener objects
    of every patch at alpha through a Loefdahl-Scharmer filter (object 0, at
    the data's noise power) and top-hat filters (the other objects; 0.55-0.7
    of a diffraction limit at 0.45 N bins), the cosine-weighted mosaic of
    every object (border N/8), and the power spectrum of the first mosaic
    with its 30-degree sector means.  HIP events on the current stream around
    `reps` calls of each stage; ms per call."""
    import torch

    import synth
    from paper_2505_10639_amd import filter_spec, momfbd_power_spectrum

    N, K, stride = g["N"], g["K"], g["stride"]
    ny = (g["H"] - N) // stride + 1
    nx = (g["W"] - N) // stride + 1
    filters = [filter_spec("scharmer", noise_power=g["noise_power"])]
    filters += [filter_spec("tophat", 0.55, 0.7, 0.45 * N)] * (K - 1)
    L = (ny - 1) * stride + N
    win = torch.from_numpy(synth.hann_window(L, L // 16).astype(np.float32)).to(D.device)
    state = {}

    def filtered():
        state["obj"] = plan.object_filtered(alpha, D, filters, gamma)

    def mosaic():
        state["mos"] = plan.mosaic(state["obj"], ny, nx, stride, N // 8)

    def spectrum():
        state["spec"] = momfbd_power_spectrum(state["mos"][0].contiguous(), win)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    res = {"ms_filtered_objects": timed(filtered), "ms_mosaic": timed(mosaic),
           "ms_power_spectrum": timed(spectrum)}
    res["ms_restoration"] = sum(res.values())
    assert bool(torch.isfinite(state["mos"]).all()), "non-finite mosaic"
    res.update({"patches": g["P"], "objects": K, "mosaic": [K, L, L], "spectrum_side": L,
                "filters": ["loefdahl_scharmer"] + ["tophat"] * (K - 1), "reps": reps})
    return res


def build_large(dev):
    """The 128 x 128, four-object workload; gamma is the smoothness-prior
    table made by the library."""
    import torch

    import synth
    from paper_2505_10639_amd import Plan

    g = synth.config4_geometry()
    pr = synth.config4_template()
    N, P, C, J, M = g["N"], g["P"], g["C"], g["J"], g["M"]
    plan = Plan(N, P, J, pr.channel_object, pr.pupil, pr.basis, None, dev)
    win = torch.from_numpy(pr.window).to(dev)
    alpha_true = torch.from_numpy(synth.config4_alpha()).to(dev)
    scenes = torch.from_numpy(synth.config4_objects()).to(dev)
    aux = Plan(N, P, 1, list(range(C)), pr.pupil, pr.basis[:, :1], None, dev)
    Ohat = aux.prepare_data(scenes.reshape(C, 1, g["H"], g["W"]).contiguous(), g["stride"], win)
    aux.close()
    del scenes
    _, S = plan.forward(alpha_true, want_psf=False)
    gen = torch.Generator(device=dev)
    gen.manual_seed(synth.SEED_ROOT + 4)
    noise = 0.01 * torch.randn((C, J, g["H"], g["W"]), generator=gen, device=dev)
    Nhat = plan.prepare_data(noise, g["stride"], win)
    del noise
    D = (Ohat * S + Nhat).contiguous()
    del S, Nhat, Ohat
    rng = np.random.default_rng(synth.SEED_ROOT + 5)
    pert = torch.from_numpy((0.3 * rng.standard_normal((P, J, M))).astype(np.float32)).to(dev)
    alpha = (alpha_true + pert).contiguous()
    gamma = plan.smoothness_gamma([g["gamma"]] * g["K"], [g["smooth"]] * g["K"])
    torch.cuda.synchronize()
    g = dict(g, channel_object=[int(k) for k in pr.channel_object],
             support_frac=support_fraction(pr.pupil, pr.channel_object, N))
    return plan, D, alpha, gamma, g


KINDS = ("phase", "forward", "object", "forward_object", "adjoint", "grad")


def time_steps(plan, D, alpha, gamma, steps, warmup, tune=True, reps=10, schedule=None):
    """ms per loss+grad step (HIP events on the launch stream) and two sets
    of per-kernel average durations from the library's event pairs on the
    same stream: back to back (each launch of one kind issued `reps` times
    in a row inside one pair, as the kernels run inside a step, with no idle
    gap in front) and isolated (one pair around every launch).  The plan's
    launch schedules are first chosen by the library's autotuner on the
    same data (a setup step, outside the timed region), unless `schedule`
    (a momfbd_tuning dict) fixes them."""
    import torch

    if schedule:
        s = dict(plan.tuning(), **schedule)
        plan.set_tuning(s["xcd_forward"], s["xcd_adjoint"], s["object_pairs_per_thread"],
                        s["grad_waves"], s["grad_splits"], s["grad_row_tiles"],
                        s["phase_col_tiles"], s["phase_waves"], s["object_fused"])
    elif tune:
        plan.autotune(alpha, D, gamma, None, reps=3)

    from paper_2505_10639_amd import (momfbd_profile_repeat, momfbd_profile_start,
                                      momfbd_profile_stop)

    loss = torch.empty(plan.P, dtype=torch.float64, device=plan.device)
    grad = torch.empty_like(alpha)

    def step():
        plan.loss_grad(alpha, D, gamma, None, True, loss, grad)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream(plan.device)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    assert torch.isfinite(loss).all(), "non-finite loss"
    momfbd_profile_start(plan.handle, 8 * steps)
    for _ in range(steps):
        step()
    kern = momfbd_profile_stop(plan.handle)
    isolated = {k: v[0] / v[1] for k, v in kern.items()}
    b2b = {}
    for kind in (k for k in KINDS if k in isolated):
        momfbd_profile_start(plan.handle, 8)
        momfbd_profile_repeat(plan.handle, kind, reps)
        for _ in range(3):
            step()
        k = momfbd_profile_stop(plan.handle)[kind]
        b2b[kind] = k[0] / k[1]
    return ms, b2b, isolated, loss, grad


def support_fraction(pupils, channel_object, N):
    """Fraction of the half spectrum inside each object's spectral support,
    by the library's rule: the differences between the column spans of every
    pair of pupil rows; column kx keeps the largest |row difference| that
    reaches it."""
    K = int(max(channel_object)) + 1
    F = -np.ones((K, N // 2 + 1), dtype=np.int64)
    for c, A in enumerate(pupils):
        rows = [(y, np.flatnonzero(A[y])) for y in range(N) if np.any(A[y])]
        for y1, x1 in rows:
            for y2, x2 in rows:
                lo, hi = x2.min() - x1.max(), x2.max() - x1.min()
                dx = np.abs(np.arange(lo, hi + 1))
                dx = dx[dx <= N // 2]
                np.maximum.at(F[channel_object[c]], dx, abs(y2 - y1))
    ky = np.arange(N)
    aky = np.minimum(ky, N - ky)[:, None]
    return [float(np.mean(aky <= F[k][None, :])) for k in range(K)]


def kernel_io_bytes(N, P, J, channel_object, frac):
    """HBM bytes each kernel must read and write once per launch: the data
    and OTF half spectra and the object spectra within each object's
    spectral support (`frac`, the loads beyond it return zero without a
    memory access), the OTFs and objects written in full, and phi and
    dL/dphi on the (N/2)^2 pupil band (FP32)."""
    unit = N * (N // 2 + 1) * 8
    band = (N // 2) ** 2 * 4
    C = len(channel_object)
    K = int(max(channel_object)) + 1
    units = P * C * J
    spec_in = sum(P * J * unit * frac[channel_object[c]] for c in range(C))   # D or S
    obj_in = sum(P * unit * frac[k] for k in range(K))
    return {"adjoint": 2 * spec_in + obj_in + 2 * units * band,   # reads D, S, O, phi; writes dL/dphi
            "forward": units * band + units * unit,             # reads phi; writes S
            "object": units * unit + spec_in + P * K * unit,   # reads D, S; writes O
            # reads phi, D; writes S, O (its own OTFs come back from the caches)
            "forward_object": units * band + 2 * units * unit + P * K * unit}


def roofline(kern_avg, units, N, io_bytes, traffic_of):
    """Roofline object of the dominant (longest) kernel.  A transform kernel
    is priced by its nominal FFT flops against the FP32 vector peak (the path
    reads only D from HBM, 43.6 flop/B at N = 64, above the 19.7 flop/B
    ridge); hbm_view gives the bytes the same launch must read and write
    against the HBM peak.  The object kernel has no transform flops and is
    priced by its bytes against HBM."""
    _, per_kernel = unit_flops(N)
    dom = max(kern_avg, key=kern_avg.get)
    t = kern_avg[dom] * 1e-3
    fl = per_kernel.get(dom)
    nbytes = io_bytes[dom]
    gbs = nbytes / t / 1e9
    common = {"kernel": dom, "traffic": traffic_of(dom), "avg_ms": kern_avg[dom],
              "units_per_launch": units}
    if fl is None:
        return {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": gbs / PEAK_HBM_GBS, **common, "io_bytes": nbytes}
    tf = fl * units / t / 1e12
    return {"bound": "alu", "achieved": tf, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
            "frac": tf / PEAK_FP32_VECTOR_TFLOPS, **common, "flop_per_unit": fl,
            "hbm_view": {"io_bytes": nbytes, "achieved": gbs, "peak": PEAK_HBM_GBS,
                         "unit": "GB/s", "frac": gbs / PEAK_HBM_GBS}}


def warm_start_block(dev, steps, patches=961):
    """Learned warm start vs the plain zero start on single-object 64x64
    bursts (12 frames, 44 modes, D/r0 in 4..20, SNR 50..200): the network is
    trained on the GPU for `steps` Adam steps of 256 bursts made by the
    library's forward model.  Per-patch L-BFGS runs in solver rounds (one
    line-search trial per running patch per round, no host synchronisation
    within a chunk of 8 rounds): from zero until the summed loss changes by
    less than 1e-10 relative over 40 rounds (L_conv); then both starts are
    timed to sum L <= 1.001 L_conv (the warm start's time includes the
    network's inference)."""
    import torch

    import synth
    from paper_2505_10639_amd import Plan
    from paper_2505_10639_amd.warmstart import (BurstSource, WarmStartNet, mode_scale,
                                                solve_rounds_until)

    J, M = 12, 44
    tmpl = synth.make_problem(0, N=64, P=1, J=J, M=M)
    rng = np.random.default_rng(synth.SEED_ROOT + 3)
    scenes = [synth.object_field(rng, 768, 768) for _ in range(4)]
    src = BurstSource(tmpl.pupil, tmpl.basis, tmpl.window, J, 256, scenes, seed=1, device=dev)
    net = WarmStartNet(J, M, mode_scale(M), batch_max=256, device=dev)
    net.init(seed=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        D, a = src.next()
        loss = net.train_step(D, a, 1e-3 * 0.5 * (1 + np.cos(np.pi * it / steps)) + 2e-5)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    final_train = float(loss.cpu()[0])
    src.close()
    ev = BurstSource(tmpl.pupil, tmpl.basis, tmpl.window, J, patches,
                     [synth.object_field(np.random.default_rng(synth.SEED_ROOT + 6), 1024, 1024)],
                     seed=7, device=dev)
    D, a_true = ev.next()
    ev.close()
    plan = Plan(64, patches, J, [0], tmpl.pupil, tmpl.basis, None, dev)
    zero = torch.zeros_like(a_true)
    h_conv, t_conv, _, r_conv = solve_rounds_until(plan, zero, D, 1e-3, None, max_rounds=12000,
                                                   chunk=8, stall=5, rtol=1e-10)
    L_conv = h_conv[-1]
    target = 1.001 * L_conv
    hp, tp, _, rp = solve_rounds_until(plan, zero, D, 1e-3, target, max_rounds=12000, chunk=8)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    a0 = net.predict(D)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t1
    hw, tw, _, rw = solve_rounds_until(plan, a0, D, 1e-3, target, max_rounds=12000, chunk=8)
    L_true = float(plan.loss_grad(a_true, D, 1e-3)[0].sum())
    plan.close()
    net.close()
    return {
        "workload": f"{patches} bursts of 12 frames 64x64, 44 modes, D/r0 4..20, SNR 50..200",
        "train_steps": steps, "train_bursts_per_s": steps * 256 / t_train,
        "train_loss_final": final_train, "L_conv": L_conv, "L_conv_rounds": r_conv,
        "L_zero": hp[0], "L_cnn": hw[0], "L_true": L_true,
        "plain_s_to_1.001": tp, "plain_rounds": rp,
        "warm_s_to_1.001": tw + t_inf, "warm_rounds": rw, "inference_s": t_inf,
        "speedup": tp / (tw + t_inf),
    }


def warm_start_large_block(dev, steps, patches=128, batch=64, m_net=44):
    """Learned warm start vs the plain zero start on the large multi-object
    workload's shape: 128 x 128 patches, 24 frames, four objects at
    lambda/lambda0 = 1.0/0.95/1.05/1.1 sharing the wavefront, 150 Zernike
    modes, D/r0 = 15, smoothness prior; the first `patches` patches of the
    2048^2 field (one GPU's share when 961 patches are spread over eight).
    The network reads the wideband channel (lambda0) and predicts the lowest
    `m_net` modes of the 24 frames (the others start at zero); it is trained
    for `steps` Adam steps of `batch` single-channel bursts of the same
    pupil, 150-mode wavefronts with D/r0 uniform in 10..20 and SNR 50..200,
    made by the library's forward model and generator.  Plain and warm
    starts are then timed as in the 64 x 64 block: L-BFGS solver rounds to
    sum L <= 1.001 L_conv, inference included."""
    import torch

    import synth
    from paper_2505_10639_amd import Plan
    from paper_2505_10639_amd.warmstart import (BurstSource, WarmStartNet, mode_scale,
                                                solve_rounds_until)

    g = synth.config4_geometry()
    pr = synth.config4_template()
    N, C, J, M, K = g["N"], g["C"], g["J"], g["M"], g["K"]
    P = patches
    win = torch.from_numpy(pr.window).to(dev)
    # data: the first P patches of the large field (rows of the patch grid)
    rows = (P + g["nx"] - 1) // g["nx"]
    H = (rows - 1) * g["stride"] + N
    scenes = torch.from_numpy(np.ascontiguousarray(synth.config4_objects()[:, :H])).to(dev)
    P_rows = rows * g["nx"]
    aux = Plan(N, P_rows, 1, list(range(C)), pr.pupil, pr.basis[:, :1], None, dev)
    Ohat = aux.prepare_data(scenes.reshape(C, 1, H, g["W"]).contiguous(), g["stride"], win)[:P]
    aux.close()
    a_true = torch.from_numpy(np.ascontiguousarray(synth.config4_alpha()[:P])).to(dev)
    plan = Plan(N, P, J, pr.channel_object, pr.pupil, pr.basis, None, dev)
    _, S = plan.forward(a_true, want_psf=False)
    noise = torch.empty((P, C, J, N, N), dtype=torch.float32, device=dev)
    from paper_2505_10639_amd import _lib
    _lib.momfbd_random_normal(synth.SEED_ROOT + 44, 1, 0, noise)
    noise *= 0.01
    # noise spectra through the data preparation of a one-column field
    nplan = Plan(N, P, J, pr.channel_object, pr.pupil, pr.basis[:, :1], None, dev)
    Nhat = nplan.prepare_data(noise.permute(1, 2, 0, 3, 4).reshape(C, J, P * N, N).contiguous(),
                              N, win)
    nplan.close()
    D = (Ohat * S + Nhat).contiguous()
    del S, Nhat, Ohat, noise, scenes
    gamma = plan.smoothness_gamma([g["gamma"]] * K, [g["smooth"]] * K)
    # the network: single-channel bursts of the wideband pupil
    r0_range = (10.0, 20.0)
    scale = mode_scale(m_net, r0_range)
    rng = np.random.default_rng(synth.SEED_ROOT + 45)
    train_scenes = [synth.object_field(rng, 1024, 1024) for _ in range(4)]
    src = BurstSource(pr.pupil[:1], pr.basis[:1], pr.window, J, batch, train_scenes,
                      crop_stride=32, seed=11, r0_range=r0_range, device=dev)
    net = WarmStartNet(J, m_net, scale, batch_max=batch, device=dev, N=N)
    net.init(seed=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        Db, ab = src.next()
        loss = net.train_step(Db, ab[:, :, :m_net].contiguous(),
                              1e-3 * 0.5 * (1 + np.cos(np.pi * it / steps)) + 2e-5)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    final_train = float(loss.cpu()[0])
    src.close()
    zero = torch.zeros((P, J, M), dtype=torch.float32, device=dev)
    h_conv, t_conv, _, r_conv = solve_rounds_until(plan, zero, D, gamma, None, max_rounds=12000,
                                                   chunk=8, stall=5, rtol=1e-10)
    L_conv = h_conv[-1]
    target = 1.001 * L_conv
    hp, tp, _, rp = solve_rounds_until(plan, zero, D, gamma, target, max_rounds=12000, chunk=8)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    a0 = torch.zeros((P, J, M), dtype=torch.float32, device=dev)
    a0[:, :, :m_net] = net.predict(D)
    torch.cuda.synchronize()
    t_inf = time.perf_counter() - t1
    hw, tw, _, rw = solve_rounds_until(plan, a0, D, gamma, target, max_rounds=12000, chunk=8)
    L_true = float(plan.loss_grad(a_true, D, gamma)[0].sum())
    plan.close()
    net.close()
    return {
        "workload": f"{P} patches of the 2048^2 field: 128x128, 24 frames, 4 objects at "
                    "lambda/lambda0 1.0/0.95/1.05/1.1, 150 modes, D/r0 15, smoothness prior; "
                    f"network on the wideband channel, lowest {m_net} modes",
        "train_steps": steps, "train_batch": batch, "train_bursts_per_s": steps * batch / t_train,
        "train_s": t_train, "train_loss_final": final_train,
        "L_conv": L_conv, "L_conv_rounds": r_conv, "L_conv_s": t_conv,
        "L_zero": hp[0], "L_cnn": hw[0], "L_true": L_true,
        "plain_s_to_1.001": tp, "plain_rounds": rp,
        "warm_s_to_1.001": tw + t_inf, "warm_rounds": rw, "inference_s": t_inf,
        "speedup": tp / (tw + t_inf),
    }


def uneven_fields_block(dev, n_fields=64, fov=512, rounds=20):
    """Independent 512^2 fields with patch sizes 64, 96 or 128 (stride N/2),
    frame counts 6..24, 44..88 modes and 1..3 objects (one channel each),
    D/r0 5..20.  One round gives every patch of every field one line-search
    trial.  Timed three ways from fresh solver states: the fields of each
    patch size as one library group (one launch per stage for all of them,
    launch schedules autotuned), eagerly and replayed from one HIP graph;
    and, for comparison, every field issuing its own rounds as parallel
    branches of one HIP graph."""
    import torch

    import synth
    from paper_2505_10639_amd import Plan, _lib
    from paper_2505_10639_amd.batch import Field, FieldBatch

    rng = np.random.default_rng(synth.SEED_ROOT + 8)
    specs, units, pf = [], 0, 0
    for i in range(n_fields):
        N = int(rng.choice([64, 96, 128]))
        J = int(rng.integers(6, 25))
        M = int(rng.integers(44, 89))
        K = int(rng.integers(1, 4))
        stride = N // 2
        n = (fov - N) // stride + 1
        P = n * n
        ch = tuple((k, 0.0) for k in range(K))
        pr = synth.make_problem(1000 + i, N=N, P=1, J=J, M=M, channels=ch, gamma=1e-3,
                                border=N // 10, objects=np.zeros((1, K, N, N)))
        plan = Plan(N, P, J, pr.channel_object, pr.pupil, pr.basis, None, dev)
        win = torch.from_numpy(pr.window).to(dev)
        scene = torch.from_numpy(np.stack([synth.object_field(rng, fov, fov) for _ in range(K)])
                                 .astype(np.float32)).to(dev)
        aux = Plan(N, P, 1, list(range(K)), pr.pupil, pr.basis[:, :1], None, dev)
        Ohat = aux.prepare_data(scene.reshape(K, 1, fov, fov).contiguous(), stride, win)
        aux.close()
        d_r0 = rng.uniform(5.0, 20.0)
        a_true = synth.draw_kolmogorov(rng, P * J, M, d_r0).reshape(P, J, M).astype(np.float32)
        _, S = plan.forward(torch.from_numpy(a_true).to(dev), want_psf=False)
        noise = 0.01 * torch.randn((K, J, fov, fov), device=dev)
        D = (Ohat * S + plan.prepare_data(noise, stride, win)).contiguous()
        plan.close()
        specs.append((N, P, J, pr.channel_object, pr.pupil, pr.basis, D))
        units += P * K * J
        pf += P * J

    def fields():
        return [Field(N, P, J, co, pu, ba, None, D, 1e-3, device=dev)
                for (N, P, J, co, pu, ba, D) in specs]

    def timed(batch, graph):
        if graph:
            batch.capture()
        run = batch.launch if graph else batch.eager
        run()                                      # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(rounds):
            run()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / rounds

    out = {"workload": f"{n_fields} fields of {fov}^2: N in {{64,96,128}} at stride N/2, J 6..24, "
                       f"M 44..88, K 1..3, D/r0 5..20", "units": units, "patch_frames": pf,
           "fields_per_size": {str(n): sum(1 for s_ in specs if s_[0] == n) for n in (64, 96, 128)}}
    grouped = FieldBatch(fields(), mode="group")
    out["group_schedules"] = {str(g.N): g.autotune(2) for g in grouped.groups}
    out["ms_per_round_group_eager"] = 1e3 * timed(grouped, False)
    grouped.close()
    grouped = FieldBatch(fields(), mode="group")
    for g in grouped.groups:
        sch = out["group_schedules"][str(g.N)]
        _lib.momfbd_group_set_tuning(g.handle, sch["xcd_forward"], sch["xcd_adjoint"],
                                     sch["grad_splits"], sch["grad_row_tiles"])
    out["ms_per_round_group_graph"] = 1e3 * timed(grouped, True)
    grouped.close()
    grouped = FieldBatch(fields(), mode="group", parallel_sizes=False)
    for g in grouped.groups:
        sch = out["group_schedules"][str(g.N)]
        _lib.momfbd_group_set_tuning(g.handle, sch["xcd_forward"], sch["xcd_adjoint"],
                                     sch["grad_splits"], sch["grad_row_tiles"])
    out["ms_per_round_group_graph_one_stream"] = 1e3 * timed(grouped, True)
    grouped.close()
    branches = FieldBatch(fields(), mode="branches")
    out["ms_per_round_field_branches_graph"] = 1e3 * timed(branches, True)
    branches.close()
    out["patch_frame_evals_per_s_group_graph"] = pf / (1e-3 * out["ms_per_round_group_graph"])
    return out


def _host_cpu():
    """CPU model, logical CPUs of the host and CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    usable = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return model, os.cpu_count(), usable


def _oracle_problem(g):
    import synth
    N = g["N"]
    return synth.make_problem(1, N=N, P=1, J=g["J"], M=g["M"], channels=g["channels"],
                              gamma=g["gamma"], border=g["border"],
                              objects=np.zeros((1, 2, N, N)))


_WORKER_PROBLEM = {}


def _oracle_worker(job):
    """One patch of the oracle in a worker process with one BLAS thread."""
    from threadpoolctl import threadpool_limits

    import oracle
    g, D_p, a_p = job
    key = (g["N"], g["J"], g["M"])
    if key not in _WORKER_PROBLEM:
        _WORKER_PROBLEM[key] = _oracle_problem(g)
    pr = _WORKER_PROBLEM[key]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        oracle.evaluate_patch(a_p, D_p, pr.basis, pr.diversity, pr.pupil, pr.channel_object,
                              pr.gamma)
        return time.perf_counter() - t0


def cpu_baseline(D_host, alpha_host, g, budget_s):
    """The FP64 oracle on the same workload, timed three ways on the host:
    one process with one BLAS thread, one process with the BLAS library's
    default threads, and worker processes over patches (one BLAS thread
    each, as many workers as this process may use, at most 16).  Each leg
    runs patches from the start of the field until its share of the time
    budget is used; the process-parallel leg is the reported value."""
    import multiprocessing as mp

    from threadpoolctl import threadpool_info, threadpool_limits

    import oracle
    pr = _oracle_problem(g)
    model, logical, usable = _host_cpu()
    leg_s = budget_s / 3.0

    def serial(limit):
        ctx = threadpool_limits(limit) if limit else None
        try:
            if ctx is not None:
                ctx.__enter__()
            t0 = time.perf_counter()
            n = 0
            while n < len(D_host):
                oracle.evaluate_patch(alpha_host[n], D_host[n], pr.basis, pr.diversity,
                                      pr.pupil, pr.channel_object, pr.gamma)
                n += 1
                if time.perf_counter() - t0 >= leg_s:
                    break
            return n, time.perf_counter() - t0
        finally:
            if ctx is not None:
                ctx.__exit__(None, None, None)

    n1, t1 = serial(1)
    blas = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    nb, tb = serial(None)
    workers = max(1, min(16, usable))
    # patches for the parallel leg: what the workers finish in about leg_s at
    # the single-thread rate, a whole number of rounds
    per_patch = t1 / max(n1, 1)
    npar = int(min(len(D_host), max(workers, workers * int(leg_s / max(per_patch, 1e-6)))))
    jobs = [(g, D_host[p], alpha_host[p]) for p in range(npar)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_worker, jobs[:workers])          # start-up and imports
        t0 = time.perf_counter()
        pool.map(_oracle_worker, jobs, chunksize=1)
        tp = time.perf_counter() - t0
    J, C = g["J"], g["C"]
    return {"value": npar * J / tp, "unit": "patch-frame evals/s", "cores": workers,
            "kind": "oracle",
            "sample": f"patches 0..{npar - 1} of {g['P']} ({npar * J} patch-frames, "
                      f"{npar * J * C} units) in {tp:.1f} s over {workers} worker processes "
                      f"with one BLAS thread each; FP64 direct DFT",
            "host_cpu": model, "host_logical_cpus": logical, "usable_cpus": usable,
            "single_thread": {"value": n1 * J / t1, "unit": "patch-frame evals/s",
                              "cores": 1, "patches": n1, "seconds": t1},
            "blas_threads": {"value": nb * J / tb, "unit": "patch-frame evals/s",
                             "cores": blas, "patches": nb, "seconds": tb},
            "process_parallel": {"value": npar * J / tp, "unit": "patch-frame evals/s",
                                 "cores": workers, "patches": npar, "seconds": tp}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-large", action="store_true", help="skip the 128 x 128 workload")
    ap.add_argument("--no-post", action="store_true",
                    help="skip the object post-processing block (filters, mosaic, spectrum)")
    ap.add_argument("--no-tune", action="store_true",
                    help="keep the default launch schedules instead of autotuning them")
    ap.add_argument("--cpu-budget", type=float, default=24.0,
                    help="seconds of oracle time over the three CPU legs")
    ap.add_argument("--warm-steps", type=int, default=6000,
                    help="training steps of the warm-start network (0: skip that block)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy three times (for scaling "
                         "hardware byte counters) and exit")
    ap.add_argument("--schedule", type=json.loads, default=None,
                    help="fix launch-schedule fields (JSON, momfbd_tuning names) instead of "
                         "autotuning, e.g. for hardware-counter runs of one schedule")
    ap.add_argument("--warm-large-steps", type=int, default=2000,
                    help="training steps of the 128 x 128 warm-start network (0: skip)")
    ap.add_argument("--only", choices=["uneven", "warm", "large", "warm_large"],
                    help="run one secondary block alone and print its JSON (profiling runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the patches are "
              "independent, so a multi-GPU run would shard them by patch block with no "
              "exchange step.", file=sys.stderr)
        sys.exit(2)

    import torch

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

    if args.only:
        if args.only == "uneven":
            res = uneven_fields_block(dev)
        elif args.only == "warm":
            res = warm_start_block(dev, args.warm_steps)
        elif args.only == "warm_large":
            res = warm_start_large_block(dev, args.warm_large_steps)
        else:
            plan4, D4, alpha4, gamma4, g4 = build_large(dev)
            ms4, kern4, _, _, _ = time_steps(plan4, D4, alpha4, gamma4, max(2, args.steps // 2),
                                             min(args.warmup, 2), not args.no_tune,
                                             schedule=args.schedule)
            res = {"ms_per_step": ms4, "kernels_avg_ms": kern4, "launch_schedule": plan4.tuning()}
            plan4.close()
        print(json.dumps({args.only: res}), flush=True)
        return

    log("building full-field inputs")
    plan, D, alpha, gamma, g = build_full_field(dev)
    N, P, C, J = g["N"], g["P"], g["C"], g["J"]
    units = P * C * J
    log(f"timing {args.steps} steps after {args.warmup} warm-up")
    ms, kern_avg, kern_iso, _, _ = time_steps(plan, D, alpha, gamma, args.steps, args.warmup,
                                              not args.no_tune, schedule=args.schedule)
    sched = plan.tuning()
    roof = roofline(kern_avg, units, N, kernel_io_bytes(N, P, J, g["channel_object"],
                                                        g["support_frac"]),
                    lambda k: counted_traffic(k, sched, N))
    flop_unit, _ = unit_flops(N)
    step_tflops = flop_unit * units / (ms * 1e-3) / 1e12
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
                   "modes": g["M"], "N": N, "units_per_step": units,
                   "launch_schedule": plan.tuning()},
        "roofline": roof,
        "units_per_s": units / (ms * 1e-3),
        "step_nominal_fft_tflops": step_tflops,
        "step_frac_of_fp32_peak": step_tflops / PEAK_FP32_VECTOR_TFLOPS,
        "kernels_avg_ms": kern_avg,
        "kernels_avg_ms_isolated": kern_iso,
    }
    if not args.no_post:
        log("post-processing: filtered objects, mosaic, sector spectrum")
        out["postprocess"] = postprocess_block(plan, D, alpha, gamma, g)
    D_h = a_h = None
    if not args.no_cpu:
        D_h = D.cpu().numpy()
        a_h = alpha.cpu().numpy()
    plan.close()
    del D, alpha

    if not args.no_large:
        log("building 128x128 multi-object inputs")
        plan4, D4, alpha4, gamma4, g4 = build_large(dev)
        units4 = g4["P"] * g4["C"] * g4["J"]
        steps4 = max(2, args.steps // 2)
        log(f"timing {steps4} steps of the 128x128 workload")
        ms4, kern4, kern4_iso, _, _ = time_steps(plan4, D4, alpha4, gamma4, steps4,
                                                 min(args.warmup, 2), not args.no_tune)
        flop4, _ = unit_flops(g4["N"])
        t4 = flop4 * units4 / (ms4 * 1e-3) / 1e12
        out["large_multi_object"] = {
            "workload": "2048x2048 frames, 961 patches of 128x128 at stride 64, 24 frames, 4 "
                        "objects at lambda/lambda0 1.0/0.95/1.05/1.1, 150 Zernike modes, "
                        "D/r0 15, smoothness prior gamma(u)",
            "value": g4["P"] * g4["J"] / (ms4 * 1e-3), "unit": "patch-frame evals/s",
            "ms_per_step": ms4, "steps": steps4, "units_per_step": units4,
            "step_nominal_fft_tflops": t4, "step_frac_of_fp32_peak": t4 / PEAK_FP32_VECTOR_TFLOPS,
            "roofline": roofline(kern4, units4, g4["N"],
                                 kernel_io_bytes(g4["N"], g4["P"], g4["J"], g4["channel_object"],
                                                 g4["support_frac"]),
                                 lambda k: counted_traffic(k, plan4.tuning(), g4["N"])),
            "launch_schedule": plan4.tuning(),
            "kernels_avg_ms": kern4,
            "kernels_avg_ms_isolated": kern4_iso,
        }
        plan4.close()
        del D4, alpha4, gamma4

    if not args.no_large:
        log("uneven fields: groups per patch size, one launch per stage")
        out["uneven_fields"] = uneven_fields_block(dev)

    if args.warm_steps > 0:
        log(f"warm start: {args.warm_steps} training steps, then time to converged loss")
        out["warm_start"] = warm_start_block(dev, args.warm_steps)

    if args.warm_large_steps > 0 and not args.no_large:
        log(f"warm start at the large workload's shape: {args.warm_large_steps} training steps")
        out["warm_start_large"] = warm_start_large_block(dev, args.warm_large_steps)

    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(D_h, a_h, g, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
