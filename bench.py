#!/usr/bin/env python3
"""Benchmark: grouped-isochromat vs plain Bloch simulation on one MI355X.

Workload (timed step): one grouped simulation of the FSE sequence
(16 shots x ETL 16, 256 phase lines x 256 readout samples, 90/180 sinc RF of
3000 raster steps with Gz) on the 1024x1024x26 = 27,262,976-isochromat
six-class phantom; inputs resident in HBM, groups built before timing.
Throughput = K * (raster steps inside RF and ADC blocks) / time.

Also reported: the EPI workload (grouped), the plain per-isochromat method
on the same GPU (FSE: first shot of the sequence at full K; EPI: whole),
the grouped-vs-plain speedup, the roofline of the dominant kernel (the
fused grouped sweep k_sweep: algorithmic FP32 flops per launch over its
HIP-event-timed duration) and the FP64 CPU oracle timed on the host cores.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps 20] [--warmup 3]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, GB/s
FP32_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (published; counts packed FP32)
FP32_NONPACKED_TFLOPS = 78.6  # 256 CU x 64 lanes x 2 flop (FMA) x 2.4 GHz, no packed FP32
COUNTERS = os.path.join(ROOT, "profiles", "k_sweep_fse_27m_counters.json")
KERNEL_SRC = [os.path.join(ROOT, "paper_2508_03960_amd", "csrc", f)
              for f in ("k_grouped.hip", "device_math.hpp", "kernels.hpp")]


def kernel_source_sha():
    h = hashlib.sha256()
    for p in KERNEL_SRC:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed_runs(sim, gb, mode, steps, warmup, m_out, sig_out, flags=0):
    import torch
    for _ in range(warmup):
        sim.simulate(mode, m_out=m_out, sig_out=sig_out, flags=flags)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        _, _, st = sim.simulate(mode, m_out=m_out, sig_out=sig_out, flags=flags, stats=True)
        stats.append(st)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, stats


def traffic_per_launch():
    """HBM bytes per k_sweep launch from the committed rocprofv3 counter runs,
    scaled by the copy-kernel calibration; None if absent or stale."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
        if c.get("kernel_source_sha256") != kernel_source_sha():
            return None
        return float(c["hbm_bytes_per_launch"])
    except (OSError, ValueError, KeyError):
        return None


def cpu_baseline(ph, seq, target_s=15.0):
    """FP64 oracle on a seeded subset of isochromats, whole FSE sequence.
    Returns the timing record, the subset's indices and the oracle's M and
    signal of the subset as a phantom of its own."""
    import numpy as np

    import oracle
    import synth
    nt = oracle.max_threads()
    S = seq.stepped_count()
    idx0 = synth.random_subset_indices(ph.K, nt, seed=7)
    t = time.perf_counter()
    oracle.simulate(ph.subset(idx0), seq)
    t_one = time.perf_counter() - t
    n = int(max(nt, min(512 * nt, nt * round(target_s / max(t_one, 1e-3)))))
    idx = synth.random_subset_indices(ph.K, n, seed=7)
    sub = ph.subset(idx)
    t = time.perf_counter()
    M, sig = oracle.simulate(sub, seq)
    dt = time.perf_counter() - t
    return {"value": n * S / dt, "unit": "isochromat-steps/s", "cores": nt, "kind": "oracle",
            "sample": f"{n} seeded isochromats of the 27,262,976 x full FSE sequence "
                      f"({S} stepped raster steps each), FP64, {dt:.1f} s"}, idx, M, sig


def subset_errors(gb, ph, seq, M_full, idx, M_ref, sig_ref):
    """Errors of the grouped path against the oracle on a subset: max |dM| of
    the subset's rows of the full-phantom run, and the relative signal error
    of the subset simulated (grouped) as a phantom of its own."""
    import numpy as np
    import torch
    sim = gb.Simulator(0)
    try:
        sim.set_phantom(ph.subset(idx))
        sim.build_groups()
        sim.set_sequence(seq)
        _, s = sim.simulate(gb.GBS_GROUPED)
        torch.cuda.synchronize()
        s = s.cpu().numpy()
    finally:
        sim.close()
    return {"subset_isochromats": int(idx.size),
            "max_abs_dM": float(np.max(np.abs(M_full[:, idx] - M_ref))),
            "rel_signal": float(np.linalg.norm(s - sig_ref) / np.linalg.norm(sig_ref))}


# Algorithmic flops per isochromat and raster step of the plain and adjoint
# kernels, counted from their source (an FMA counts 2).  The rotation series
# are counted at the length a step under a quarter radian needs (q <= 1/16:
# six FP64 terms per series, five FP32 terms), the case of nearly every
# raster step; a step with a larger angle executes the longer series, which
# these figures do not count.
# k_plain (FP64): field 6, |B|^2 2, rotation series and coefficients 23, the
#   increment of the rotation 35 (cross products 9, B.M 5, three increments
#   18, adds 3), relaxation 7 -> 73 with B1; without B1 the rotation about z
#   costs 10 and |B|^2 1 -> 47.
PLAIN_FLOPS_B1, PLAIN_FLOPS_NO_B1 = 73, 47
# k_adj_forward (FP32), per raster op: w and |w|^2 14, series S, C, D3 24,
#   rotation increment 27, rotated state 3, relaxation increment 7, three
#   compensated adds 21 -> 96.  k_adj_backward per raster op: the op is
#   stepped twice (segment and sub-segment, 192), then its transpose: T1/T2
#   terms 14, D lambda 6, coefficients 38, RF gradient (parameter steps) 46,
#   rotation increment 27, compensated adds 21 -> 344.
ADJ_FWD_FLOPS, ADJ_BWD_FLOPS = 96, 344


def adjoint_raster_ops(seq, param_blocks):
    """Raster ops of the adjoint's flattened sequence: steps of parameter
    blocks and steps with B1 != 0 (runs without RF become closed-form ops)."""
    import numpy as np
    pb = set(int(b) for b in param_blocks)
    n = 0
    for b in range(seq.n_blocks):
        if seq.btype[b] == 3:
            continue
        o, k = int(seq.step_offset[b]), int(seq.n_steps[b])
        if b in pb:
            n += k
        else:
            n += int(np.count_nonzero((np.asarray(seq.rf_re[o:o + k]) != 0) | (np.asarray(seq.rf_im[o:o + k]) != 0)))
    return n


# FP64 flops of one raster step of the per-isochromat composition [A | b] <- D R [A | b]
# (k_cached, compose mode; FMA = 2): field and |B|^2 11, rotation coefficients 23
# (the six-term series, as for k_plain), rows of D R 32, the 3x3 by 3x4 product 60,
# T1 recovery 1.
COMPOSE_FLOPS_PER_ISO_STEP = 127
FP64_PEAK_TFLOPS = 78.6  # MI355X FP64 vector


def cached_leg(sim, gb, seq, m_out, sig, steps, ref_M=None, ref_sig=None):
    """The conventional accelerated method (per-isochromat transitions with
    dynamic caching, direct ADC evaluation) on a full-size workload: time,
    split by kernel kind, and agreement with the grouped result."""
    import numpy as np
    import torch
    sec, st = timed_runs(sim, gb, gb.GBS_CACHED, steps, 1, m_out, sig, flags=gb.GBS_PROFILE)
    last = st[-1]
    K = sim.K
    S = seq.stepped_count()
    # composed raster steps: the first occurrence of every distinct with-RF waveform
    comp_steps = 0
    seen = set()
    for b in range(seq.n_blocks):
        if int(seq.btype[b]) != 1:
            continue
        lo, n = int(seq.step_offset[b]), int(seq.n_steps[b])
        key = tuple(np.asarray(a[lo:lo + n], np.float32).tobytes() for a in
                    (seq.rf_re, seq.rf_im, seq.gx, seq.gy, seq.gz))
        if any(np.asarray(seq.rf_re[lo:lo + n]) != 0) or any(np.asarray(seq.rf_im[lo:lo + n]) != 0):
            if key not in seen:
                seen.add(key)
                comp_steps += n
    n_apply = last["n_rf_cached"] - last["n_distinct_rf"]
    ms_c, ms_a, ms_d = (float(np.mean([x[k] for x in st])) for k in ("ms_compose", "ms_apply", "ms_adc_direct"))
    flops_c = K * comp_steps * COMPOSE_FLOPS_PER_ISO_STEP
    # apply launches: FP64 state in and out (48 B), cached rows (48 B), M0 (4 B); the
    # closed-form pre map adds x, y, z, df, T1, T2 (24 B); map-only launches are counted alike
    n_samples = int(seq.total_samples)
    out = {"ms": sec * 1e3, "iso_steps_per_s": K * S / sec,
           "ms_compose": ms_c, "ms_apply": ms_a, "ms_adc_direct": ms_d,
           "n_rf_cached": last["n_rf_cached"], "n_distinct_rf": last["n_distinct_rf"],
           "n_adc_direct": last["n_adc_direct"], "cache_bytes": last["cache_bytes"],
           "compose_roofline": {"kernel": "k_cached<compose>", "bound": "alu",
                                "flops": flops_c, "achieved": flops_c / (ms_c * 1e-3) / 1e12 if ms_c else None,
                                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s (FP64)",
                                "flops_per_iso_step": COMPOSE_FLOPS_PER_ISO_STEP},
           "direct_adc_iso_samples_per_s": K * n_samples / (ms_d * 1e-3) if ms_d else None}
    if n_apply > 0 and ms_a > 0:
        n_map = 1  # the final map
        bytes_a = K * (n_apply * (48 + 48 + 4 + 24) + n_map * (24 + 12 + 4 + 24))
        out["apply_roofline"] = {"kernel": "k_cached<apply>", "bound": "hbm", "bytes": bytes_a,
                                 "achieved": bytes_a / (ms_a * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s"}
    if ref_M is not None:
        out["vs_grouped"] = {"max_abs_dM": float(np.max(np.abs(m_out.cpu().numpy() - ref_M))),
                             "rel_signal": float(np.linalg.norm(torch.view_as_complex(sig).cpu().numpy() - ref_sig)
                                                 / np.linalg.norm(ref_sig))}
    return out


MLP_MACS = 5 * 128 + 128 * 128 * 2 + 128 * 12  # multiply-adds per network evaluation
# per training sample: forward, hidden-layer data gradients (none for the inputs), weight gradients
TRAIN_FLOPS = 2 * (MLP_MACS + (MLP_MACS - 5 * 128) + MLP_MACS)
TRAIN_BATCH, TRAIN_LR = 1024, 3e-3
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix


def surrogate_leg(sim, gb, ph, fse, sig_exact, m_out, steps):
    """Learned RF-transition surrogate of the FSE 180-degree pulse: training on
    2M simulator-generated transitions, per-transition speed and accuracy over
    the whole phantom, then the FSE with the network in place of the exact
    composition: grouped (759 z-group transitions) and cached (one transition
    per isochromat, Eq. 7), each with the 1e-3 spot check on."""
    import numpy as np
    import torch

    import synth
    rf, gz, dt = synth.fse_refocusing_pulse()
    m = gb.Mlp(0, seed=7)
    m.set_pulse(rf, gz, dt)
    m.set_params(synth.mlp_init_params(seed=7))
    tup = torch.from_numpy(synth.surrogate_tuples(1 << 21, seed=36)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    T = m.exact(tup)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    epochs = 64
    t0 = time.perf_counter()
    hist = m.train(tup, T, epochs=epochs, batch=TRAIN_BATCH, lr_max=TRAIN_LR, lr_min=1e-6, seed=2)
    t_train = time.perf_counter() - t0
    del tup, T
    # per-isochromat transitions of the whole phantom (what a per-isochromat method needs)
    g_ref = float(np.max(np.abs(np.float32(gz))))
    pt = np.stack([synth.GAMMA_BAR * g_ref * ph.z, ph.df, ph.t1, ph.t2, np.ones(ph.K)], 1).astype(np.float32)
    pt = torch.from_numpy(pt).cuda()
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(2):  # second pass timed warm
        ev[0].record(st)
        Tm = m.infer(pt)
        ev[1].record(st)
        Te = m.exact(pt)
        ev[2].record(st)
        torch.cuda.synchronize()
    ms_inf, ms_ex = ev[0].elapsed_time(ev[1]), ev[1].elapsed_time(ev[2])
    err = (Tm.double() - Te).abs().max(dim=1).values
    err_q = torch.quantile(err[:: -(-ph.K // (1 << 24))].float(), torch.tensor([0.5, 0.99], device=err.device))
    res = {"training": {"samples": 1 << 21, "exact_data_s": t_data, "epochs": epochs, "batch": TRAIN_BATCH,
                        "lr_max": TRAIN_LR, "steps": int(hist.size), "train_s": t_train,
                        "us_per_step": t_train / hist.size * 1e6,
                        "samples_per_s": hist.size * TRAIN_BATCH / t_train,
                        "algorithmic_TFLOPs": TRAIN_FLOPS * hist.size * TRAIN_BATCH / t_train / 1e12,
                        "final_loss": float(hist[-1]),
                        "target": "8 (K - K_ref): residual over the pulse's own B1-scaled rotation table"},
           "per_isochromat_transitions": {
               "count": ph.K, "network_ms": ms_inf, "exact_fp64_ms": ms_ex, "speedup": ms_ex / ms_inf,
               "max_abs_err": float(err.max()), "median_abs_err": float(err_q[0]),
               "p99_abs_err": float(err_q[1]),
               "mfma_roofline": {"kernel": "k_mlp_infer", "bound": "mfma",
                                 "achieved": 2 * MLP_MACS * ph.K / (ms_inf * 1e-3) / 1e12,
                                 "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                                 "frac": 2 * MLP_MACS * ph.K / (ms_inf * 1e-3) / 1e12 / BF16_PEAK_TFLOPS,
                                 "issued_over_algorithmic": 2.0}}}
    del Tm, Te, pt, err
    sig = torch.empty_like(torch.view_as_real(sig_exact))
    ref = sig_exact.cpu().numpy()
    for name, tol in (("spot_checked_tol_1e-3", 1e-3), ("forced", 1e9)):
        gb.set_surrogate(sim, m, tol=tol, n_check=256, seed=11)
        sec, sts = timed_runs(sim, gb, gb.GBS_GROUPED, steps, 1, m_out, sig, flags=gb.GBS_SURROGATE)
        s_np = torch.view_as_complex(sig).cpu().numpy()
        res["fse_grouped_" + name] = {"ms": sec * 1e3, "fallback": bool(sts[-1]["n_surrogate_fallback"]),
                                      "spot_check_residual": sts[-1]["surrogate_residual"],
                                      "signal_rel_err_vs_grouped_exact": float(np.linalg.norm(s_np - ref) /
                                                                               np.linalg.norm(ref))}
    # GBS_CACHED: the network fills the 180-degree entry for every isochromat
    gb.set_surrogate(sim, m, tol=1e-3, n_check=256, seed=11)
    cached = {}
    for name, flags in (("exact", 0), ("network", gb.GBS_SURROGATE)):
        sec, sts = timed_runs(sim, gb, gb.GBS_CACHED, 1, 1, m_out, sig, flags=flags | gb.GBS_PROFILE)
        cached[name] = (sec, sts[-1], torch.view_as_complex(sig).cpu().numpy())
    (sec_x, st_x, s_x), (sec_n, st_n, s_n) = cached["exact"], cached["network"]
    res["fse_cached_spot_checked_tol_1e-3"] = {
        "ms": sec_n * 1e3, "exact_ms": sec_x * 1e3, "speedup": sec_x / sec_n,
        "compose_ms": st_n["ms_compose"], "exact_compose_ms": st_x["ms_compose"],
        "fallback": bool(st_n["n_surrogate_fallback"]), "spot_check_residual": st_n["surrogate_residual"],
        "n_check": 256,
        "signal_rel_err_vs_cached_exact": float(np.linalg.norm(s_n - s_x) / np.linalg.norm(s_x)),
        "signal_rel_err_vs_grouped_exact": float(np.linalg.norm(s_n - ref) / np.linalg.norm(ref))}
    gb.set_surrogate(sim, None)
    m.close()
    return res


def adjoint_leg(gb, steps):
    """Gradient of the GRE signal (3000 complex RF samples, 6 tissue T1/T2
    pairs) on the 256x256x16 phantom: forward with checkpoints every 256 ops,
    then the backward pass, FP32 state and FP64 sums."""
    import numpy as np
    import torch

    import synth
    ph, t1c, t2c, seq, rf, pb = synth.adjoint_workload()
    sim = gb.Simulator(0)
    sim.set_phantom(ph)
    sim.set_sequence(seq)
    adj = gb.Adjoint(sim, ph.labels, pb, every=256)
    rng = np.random.default_rng(12)
    w = rng.standard_normal(seq.total_samples) + 1j * rng.standard_normal(seq.total_samples)
    W = torch.tensor(np.stack([w.real, w.imag], 1), dtype=torch.float64, device="cuda")
    rft = torch.tensor(np.stack([rf.real, rf.imag], 1), dtype=torch.float32, device="cuda")
    t1 = torch.tensor(t1c, dtype=torch.float32, device="cuda")
    t2 = torch.tensor(t2c, dtype=torch.float32, device="cuda")
    fwd, bwd = [], []
    for i in range(steps + 1):  # first pass warms up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        adj.forward(rft, t1, t2)
        t_f = time.perf_counter() - t0
        t0 = time.perf_counter()
        adj.backward(W)
        t_b = time.perf_counter() - t0
        if i:
            fwd.append(t_f)
            bwd.append(t_b)
    S = seq.stepped_count()
    n_raster = adjoint_raster_ops(seq, pb)
    f, b = float(np.mean(fwd)), float(np.mean(bwd))
    sim.close()
    fl_f, fl_b = ADJ_FWD_FLOPS * n_raster * ph.K, ADJ_BWD_FLOPS * n_raster * ph.K
    rl = lambda kernel, fl, t: {"kernel": kernel, "bound": "alu", "flops": fl,
                                "achieved": fl / t / 1e12, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                                "frac": fl / t / 1e12 / FP32_PEAK_TFLOPS,
                                "frac_of_nonpacked_fp32": fl / t / 1e12 / FP32_NONPACKED_TFLOPS,
                                "time": "whole call (kernel dominated)"}
    return {"workload": f"GRE {ph.K} isochromats (256x256x16), {len(pb)} TRs of a 3000-sample complex sinc RF, "
                        f"{seq.total_samples} samples; gradient wrt 3000 complex RF samples + 6 (T1, T2) pairs",
            "forward_ms": f * 1e3, "backward_ms": b * 1e3, "backward_over_forward": b / f,
            "forward_iso_steps_per_s": ph.K * S / f, "backward_iso_steps_per_s": ph.K * S / b,
            "checkpoint_every": 256, "raster_ops": n_raster,
            "precision": "compensated FP32 state (hi + lo pairs), FP64 sums over isochromats",
            "roofline_forward": rl("k_adj_forward", fl_f, f),
            "roofline_backward": rl("k_adj_backward", fl_b, b)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-method runs")
    ap.add_argument("--no-epi", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned-surrogate leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the signal-gradient leg")
    ap.add_argument("--no-cached", action="store_true",
                    help="skip the conventional method with per-isochromat transition caching")
    ap.add_argument("--no-coils", action="store_true",
                    help="skip the multi-coil FSE (4 and 8 receive coils, grouped)")
    ap.add_argument("--no-oblique", action="store_true",
                    help="skip the oblique-slice FSE (two-axis groups vs per-isochromat stepping)")
    ap.add_argument("--no-nograds", action="store_true",
                    help="skip the fat-saturated FSE (no-grads groups vs x-groups)")
    ap.add_argument("--no-table2", action="store_true",
                    help="skip the four sequences of the paper's Table 2 (grouped vs cached) and the EPI read from a Pulseq file")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="accepted for older command lines: the 1 GiB device copies always run")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the simulator has no "
              "multi-GPU path; isochromats would shard by index with one signal reduce.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2508_03960_amd as gb

    dev = torch.device("cuda", 0)
    # measured device-copy bandwidth next to the 8 TB/s nominal: 1 GiB read and
    # 1 GiB written per copy (also the calibration kernel of the counter runs)
    a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(3):
        b.copy_(a)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 3 * 2 * (1 << 30) / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    del a, b
    log(f"device copy: {copy_gbs:.0f} GB/s (1 GiB read + 1 GiB written per copy)")

    t = time.perf_counter()
    ph = synth.brain_like_phantom()
    fse = synth.fse_sequence()
    epi = synth.epi_sequence()
    log(f"phantom K={ph.K} built in {time.perf_counter() - t:.1f} s")
    sim = gb.Simulator(0)
    sim.set_phantom(ph)
    torch.cuda.synchronize()
    t = time.perf_counter()
    sim.build_groups()
    torch.cuda.synchronize()
    t_groups = time.perf_counter() - t
    info = sim.info()
    log(f"groups {info['n_groups']} in {t_groups:.2f} s")
    K = ph.K
    m_out = torch.empty(3, K, device=dev, dtype=torch.float32)

    # ---- FSE grouped (the timed step) ------------------------------------------
    sim.set_sequence(fse)
    sig_fse = torch.empty(fse.total_samples, 2, device=dev, dtype=torch.float64)
    S_fse = fse.stepped_count()
    sec, stats = timed_runs(sim, gb, gb.GBS_GROUPED, args.steps, args.warmup, m_out, sig_fse,
                            flags=gb.GBS_PROFILE)
    value = K * S_fse / sec
    log(f"FSE grouped: {sec * 1e3:.2f} ms/step, {value:.3e} iso-steps/s; stats {stats[-1]}")
    n_sw = stats[-1]["n_sweeps"]
    sweep_ms = float(np.mean([s["pass_kernel_ms"] for s in stats])) / n_sw
    bytes_launch = stats[-1]["pass_bytes"] / n_sw
    flops_launch = stats[-1]["pass_flops"] / n_sw
    achieved = flops_launch / (sweep_ms * 1e-3) / 1e12
    M_fse = m_out.cpu().numpy()
    sig_fse_exact = torch.view_as_complex(sig_fse).clone()

    out = {
        "metric": "isochromat-steps/s grouped vs plain (same GPU); FSE/EPI sim time @27.3M isos",
        "value": value, "unit": "isochromat-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": sec * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "FSE grouped, 1024x1024x26 = 27,262,976 isochromats, 16 shots x ETL 16, "
                               "256x256 samples @4us, 90/180 sinc 3000 steps with Gz, TR 3 s",
                   "K": K, "stepped_steps": S_fse, "mode": "grouped", "n_groups_xyz": info["n_groups"]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_PEAK_TFLOPS, "traffic": traffic_per_launch(),
                     "kernel": "k_sweep", "flops_per_launch": flops_launch, "bytes_per_launch": bytes_launch,
                     "avg_launch_ms": sweep_ms, "launches_per_step": n_sw,
                     "hbm_GBs": bytes_launch / (sweep_ms * 1e-3) / 1e9,
                     "frac_of_nonpacked_fp32": achieved / FP32_NONPACKED_TFLOPS,
                     "grouped_ops_per_launch": stats[-1]["n_passes"] / n_sw,
                     "copy_GBs_measured": copy_gbs},
        "fse": {"grouped_ms": sec * 1e3, "phases_ms": {k: stats[-1][k] for k in
                                                      ("ms_prepare", "ms_passes", "ms_adc_eval")},
                "build_groups_s": t_groups},
    }

    # ---- EPI grouped --------------------------------------------------------------
    if not args.no_epi:
        sim.set_sequence(epi)
        sig_epi = torch.empty(epi.total_samples, 2, device=dev, dtype=torch.float64)
        S_epi = epi.stepped_count()
        sec_e, st_e = timed_runs(sim, gb, gb.GBS_GROUPED, args.steps, args.warmup, m_out, sig_epi)
        out["epi"] = {"grouped_ms": sec_e * 1e3, "grouped_iso_steps_per_s": K * S_epi / sec_e,
                      "stepped_steps": S_epi, "phases_ms": {k: st_e[-1][k] for k in
                                                            ("ms_prepare", "ms_passes", "ms_adc_eval")}}
        log(f"EPI grouped: {sec_e * 1e3:.2f} ms/step")
        M_epi = m_out.cpu().numpy()
        s_epi = sig_epi.cpu().numpy()
        if not args.no_plain:
            sec_p, _ = timed_runs(sim, gb, gb.GBS_PLAIN, 1, 0, m_out, sig_epi)
            s_pl = sig_epi.cpu().numpy()
            out["epi"].update({"plain_ms": sec_p * 1e3, "plain_iso_steps_per_s": K * S_epi / sec_p,
                               "speedup_grouped_fp32_vs_plain_fp64": sec_p / sec_e,
                               "grouped_vs_plain_fp64": {
                                   "max_abs_dM": float(np.max(np.abs(M_epi - m_out.cpu().numpy()))),
                                   "rel_signal": float(np.linalg.norm(s_epi - s_pl) / np.linalg.norm(s_pl))}})
            log(f"EPI plain: {sec_p * 1e3:.1f} ms; grouped vs plain {out['epi']['grouped_vs_plain_fp64']}")

    # ---- learned RF-transition surrogate (FSE 180-degree pulse) --------------------
    if not args.no_surrogate:
        sim.set_sequence(fse)
        out["surrogate"] = surrogate_leg(sim, gb, ph, fse, sig_fse_exact, m_out, args.steps)
        log(f"surrogate: {out['surrogate']}")

    # ---- gradient of the signal (adjoint) -------------------------------------------
    if not args.no_adjoint:
        out["adjoint"] = adjoint_leg(gb, max(1, min(args.steps, 3)))
        log(f"adjoint: {out['adjoint']}")

    # ---- conventional method with per-isochromat transition caching (Sec. 2.2) -------------
    if not args.no_cached:
        n_c = max(1, min(args.steps, 2))
        sim.set_sequence(fse)
        sig_c = torch.empty(fse.total_samples, 2, device=dev, dtype=torch.float64)
        out["cached"] = {"fse": cached_leg(sim, gb, fse, m_out, sig_c, n_c, M_fse,
                                           sig_fse_exact.cpu().numpy())}
        out["fse"]["speedup_grouped_vs_cached"] = out["cached"]["fse"]["ms"] / (sec * 1e3)
        log(f"FSE cached: {out['cached']['fse']}")
        if not args.no_epi:
            sim.set_sequence(epi)
            sig_c = torch.empty(epi.total_samples, 2, device=dev, dtype=torch.float64)
            out["cached"]["epi"] = cached_leg(sim, gb, epi, m_out, sig_c, n_c, M_epi, s_epi[:, 0] + 1j * s_epi[:, 1])
            out["epi"]["speedup_grouped_vs_cached"] = out["cached"]["epi"]["ms"] / out["epi"]["grouped_ms"]
            log(f"EPI cached: {out['cached']['epi']}")

    # ---- receive coils: the grouped FSE with 4 and 8 coil sensitivities ------------------
    if not args.no_coils:
        sim.set_sequence(fse)
        res = {"single_coil_ms": sec * 1e3}
        for P in (4, 8):
            sim.set_coils(synth.coil_maps(ph, P))
            sig_c = torch.empty(P * fse.total_samples, 2, device=dev, dtype=torch.float64)
            sec_c, _ = timed_runs(sim, gb, gb.GBS_GROUPED, max(1, min(args.steps, 3)), 1, m_out, sig_c)
            res[f"coils_{P}_ms"] = sec_c * 1e3
        sim.set_coils(None)
        # the sensitivities stream from HBM at every emission: 8 bytes per isochromat, coil and readout
        res["coil_bytes_per_step_P8"] = 8.0 * 8 * K * int((fse.btype == 2).sum())
        out["coils_fse"] = res
        log(f"coils: {res}")

    # ---- two-axis groups: the FSE with its slice tilted 20 degrees toward x -------------
    if not args.no_oblique:
        ob = synth.fse_sequence(tilt_deg=20.0)
        sim.set_sequence(ob)
        sig_ob = torch.empty(ob.total_samples, 2, device=dev, dtype=torch.float64)
        sec_o, st_o = timed_runs(sim, gb, gb.GBS_GROUPED, max(1, min(args.steps, 3)), 1, m_out, sig_ob)
        res = {"grouped_ms": sec_o * 1e3, "n_xz_groups": sim.info()["n_xz_groups"],
               "ms_prepare": float(np.mean([x["ms_prepare"] for x in st_o])),
               "ms_passes": float(np.mean([x["ms_passes"] for x in st_o])), "n_fallback": st_o[-1]["n_fallback"]}
        # without two-axis groups every oblique RF block is stepped per isochromat: time the
        # first one (the 90-degree pulse and the rephaser) and scale by the 272 RF blocks
        sim.build_groups(gb.GBS_AX_ALL & ~gb.GBS_AX_XZ)
        head = ob.head(2, name="oblique-rf1")
        sim.set_sequence(head)
        sec_h, st_h = timed_runs(sim, gb, gb.GBS_GROUPED, 1, 1, m_out, sig_ob)
        n_rf = int((ob.btype == 1).sum())
        res.update({"stepped_rf_block_ms": sec_h * 1e3, "stepped_fallback_s_extrapolated": sec_h * n_rf,
                    "speedup_vs_stepped_fallback": sec_h * n_rf / sec_o, "n_fallback_without": st_h[-1]["n_fallback"]})
        sim.build_groups()
        out["oblique_fse"] = res
        log(f"oblique FSE: {res}")

    # ---- no-grads groups: the FSE with a CHESS fat-saturation pulse per shot -------------
    if not args.no_nograds:
        fs = synth.fse_sequence(fat_sat=True)
        sim.set_sequence(fs)
        sig_fs = torch.empty(fs.total_samples, 2, device=dev, dtype=torch.float64)
        res, outs = {}, {}
        for label, axes in (("x_groups", gb.GBS_AX_X | gb.GBS_AX_Y | gb.GBS_AX_Z), ("tissue_groups", gb.GBS_AX_ALL)):
            sim.build_groups(axes)
            sec_f, st_f = timed_runs(sim, gb, gb.GBS_GROUPED, max(1, min(args.steps, 3)), 1, m_out, sig_fs)
            res[label] = {"ms": sec_f * 1e3, "ms_prepare": float(np.mean([x["ms_prepare"] for x in st_f])),
                          "n_distinct_rf": st_f[-1]["n_distinct_rf"]}
            outs[label] = (m_out.cpu().numpy(), torch.view_as_complex(sig_fs).cpu().numpy())
        res["n_tissue_groups"] = sim.info()["n_tissue_groups"]
        res["n_x_groups"] = sim.info()["n_groups"][0]
        (Mx_, sx_), (Mt_, st_) = outs["x_groups"], outs["tissue_groups"]
        res["tissue_vs_x"] = {"max_abs_dM": float(np.max(np.abs(Mt_ - Mx_))),
                              "rel_signal": float(np.linalg.norm(st_ - sx_) / np.linalg.norm(sx_))}
        out["fat_sat_fse"] = res
        log(f"fat-sat FSE: {res}")

    # ---- the paper's Table 2 sequences: grouped vs the cached conventional method ----------
    if not args.no_table2:
        out["table2"] = {}
        for name, seq in synth.table2_sequences().items():
            sim.set_sequence(seq)
            sig_t = torch.empty(seq.total_samples, 2, device=dev, dtype=torch.float64)
            sec_g, _ = timed_runs(sim, gb, gb.GBS_GROUPED, max(1, min(args.steps, 3)), 1, m_out, sig_t)
            M_g = m_out.cpu().numpy()
            s_g = torch.view_as_complex(sig_t).cpu().numpy()
            sec_c, _ = timed_runs(sim, gb, gb.GBS_CACHED, 1, 1, m_out, sig_t)
            s_c = torch.view_as_complex(sig_t).cpu().numpy()
            S_t = seq.stepped_count()
            out["table2"][name] = {
                "grouped_ms": sec_g * 1e3, "cached_ms": sec_c * 1e3, "speedup_grouped_vs_cached": sec_c / sec_g,
                "grouped_iso_steps_per_s": K * S_t / sec_g, "stepped_steps": S_t,
                "cached_vs_grouped": {"max_abs_dM": float(np.max(np.abs(m_out.cpu().numpy() - M_g))),
                                      "rel_signal": float(np.linalg.norm(s_c - s_g) / np.linalg.norm(s_g))}}
            log(f"table2 {name}: {out['table2'][name]}")

    # ---- the same EPI shape read from a Pulseq file: loader time and the grouped run -------
    if not args.no_table2:
        from synth.pulseq import epi_text
        txt = epi_text(n_lines=128, n_read=128, fov=0.256, dwell_us=4, ramp_us=44).encode()
        t0 = time.perf_counter()
        pseq = gb.load_pulseq(txt)
        t_load = time.perf_counter() - t0
        sim.set_sequence(pseq)
        sig_q = torch.empty(pseq.total_samples, 2, device=dev, dtype=torch.float64)
        sec_q, _ = timed_runs(sim, gb, gb.GBS_GROUPED, max(1, min(args.steps, 3)), 1, m_out, sig_q)
        S_q = int(pseq.n_steps[pseq.btype != gb.GBS_BLOCK_RELAX].sum())
        out["pulseq_epi"] = {"grouped_ms": sec_q * 1e3, "grouped_iso_steps_per_s": K * S_q / sec_q,
                             "stepped_steps": S_q, "load_ms": t_load * 1e3, "file_bytes": len(txt),
                             "blocks": pseq.n_blocks, "plan": gb.gbs_plan_summary(pseq)}
        log(f"Pulseq EPI: {out['pulseq_epi']}")

    # ---- plain FSE: first shot (1/16 of the sequence) at full K -------------------------
    if not args.no_plain:
        shot = fse.head(66, name="fse-shot1")
        sim.set_sequence(shot)
        sig_shot = torch.empty(shot.total_samples, 2, device=dev, dtype=torch.float64)
        sec_p, _ = timed_runs(sim, gb, gb.GBS_PLAIN, 1, 1, m_out, sig_shot)
        rate_p = K * shot.stepped_count() / sec_p
        rf_blocks = [b for b in range(shot.n_blocks) if shot.btype[b] != 3 and
                     np.any(np.asarray(shot.rf_re[shot.step_offset[b]:shot.step_offset[b] + shot.n_steps[b]]) != 0)]
        s_b1 = int(sum(int(shot.n_steps[b]) for b in rf_blocks))
        fl_p = K * (PLAIN_FLOPS_B1 * s_b1 + PLAIN_FLOPS_NO_B1 * (shot.stepped_count() - s_b1))
        out["plain"] = {"workload": "FSE first shot (17 RF + 16 ADC blocks, 67,384 stepped steps) at full K, FP64",
                        "ms": sec_p * 1e3, "iso_steps_per_s": rate_p,
                        "precision": "FP64 state and coefficients (the only plain stepper: FP32 stepping "
                                     "misses the 1e-5 bar by ~30x)",
                        "fse_full_s_extrapolated": K * S_fse / rate_p,
                        "roofline": {"kernel": "k_plain", "bound": "alu", "flops": fl_p,
                                     "achieved": fl_p / sec_p / 1e12, "peak": FP64_PEAK_TFLOPS,
                                     "unit": "TFLOP/s (FP64)", "frac": fl_p / sec_p / 1e12 / FP64_PEAK_TFLOPS,
                                     "time": "whole call (kernel dominated)"}}
        out["fse"]["speedup_grouped_fp32_vs_plain_fp64"] = value / rate_p
        log(f"FSE plain shot: {sec_p * 1e3:.1f} ms, {rate_p:.3e} iso-steps/s")

    # ---- FP64 oracle on the host cores, and the sampled error of the timed run -----------
    if not args.no_cpu:
        cb, idx, M_ref, s_ref = cpu_baseline(ph, fse)
        out["cpu_baseline"] = cb
        out["fse"]["vs_oracle"] = subset_errors(gb, ph, fse, M_fse, idx, M_ref, s_ref)
        log(f"cpu baseline {cb}; FSE vs oracle {out['fse']['vs_oracle']}")
        if not args.no_epi:  # the EPI run's error on a 16,384-isochromat subset as well
            import oracle
            import synth
            idx_e = synth.random_subset_indices(K, 1 << 14, seed=8)
            M_ref_e, s_ref_e = oracle.simulate(ph.subset(idx_e), epi)
            out["epi"]["vs_oracle"] = subset_errors(gb, ph, epi, M_epi, idx_e, M_ref_e, s_ref_e)
            log(f"EPI vs oracle {out['epi']['vs_oracle']}")
    print(json.dumps(out), flush=True)
    sim.close()


if __name__ == "__main__":
    main()
