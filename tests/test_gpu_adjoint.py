"""GPU parity of the adjoint (gradient of the signal) through the C ABI.

Workload: the GRE of the adjoint workload (3 ms sinc RF of 3000 complex
samples with Gz, 8 phase lines x 64 samples, TR 10 ms) on the 256x256x16
six-class phantom (1,048,576 isochromats).  Checks:

* against the FP64 oracle adjoint (oracle/bloch_adjoint.c) on a seeded
  4096-isochromat subset, for the 8-TR workload and for a sequence four
  times longer (32 TRs): the signal within the usual 1e-4 relative bar; the
  RF gradient within 1e-4 (relative L2) and every class T1 and T2 derivative
  within 5e-4 relative.  The kernels carry M and the adjoint state as
  compensated FP32 pairs, so that the small per-step increments are not
  rounded away the same way at every step; measured errors are 3e-6 to
  1e-4 and barely grow from 8 to 32 TRs;
* against central finite differences (relative step 1e-4) of the FP64 plain
  GPU path at full size, along seeded random directions of the pulse and for
  every class T1 and T2: 1e-4 for the pulse directions and 2e-4 norm-wise
  over the vector of the 12 T1/T2 derivatives (a class sum that cancels to a
  small value keeps only the absolute accuracy of its terms).  Differences
  of FP32 forward passes cannot serve: their rounding noise at this step is
  several per cent;
* the three branches of the rotation series (five terms, nine terms, sqrt
  and sincos) inside every wavefront, against the oracle adjoint;
* the torch.autograd.Function wrapper returns exactly the C ABI's gradient;
* the checkpoint interval (256, 16, 8) does not change the result.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_03960_amd as gb
    ph, t1c, t2c, seq, rf, pb = synth.adjoint_workload()
    rng = np.random.default_rng(12)
    w = rng.standard_normal(seq.total_samples) + 1j * rng.standard_normal(seq.total_samples)
    return gb, torch, ph, t1c, t2c, seq, rf, pb, w


def make(gb, torch, ph, seq, pb, every=256):
    sim = gb.Simulator(0)
    sim.set_phantom(ph)
    sim.set_sequence(seq)
    return sim, gb.Adjoint(sim, ph.labels, pb, every=every)


def tens(torch, rf, t1c, t2c):
    rft = torch.tensor(np.stack([rf.real, rf.imag], 1), dtype=torch.float32, device="cuda")
    return (rft, torch.tensor(t1c, dtype=torch.float32, device="cuda"),
            torch.tensor(t2c, dtype=torch.float32, device="cuda"))


def wt(torch, w):
    return torch.tensor(np.stack([w.real, w.imag], 1), dtype=torch.float64, device="cuda")


def run(adj, torch, rf, t1c, t2c, w):
    sig = adj.forward(*tens(torch, rf, t1c, t2c))
    grf, g1, g2 = adj.backward(wt(torch, w))
    torch.cuda.synchronize()
    s = sig.cpu().numpy()
    g = grf.cpu().numpy().astype(np.float64)
    return s[:, 0] + 1j * s[:, 1], g[:, 0] + 1j * g[:, 1], g1.cpu().numpy(), g2.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("n_lines", [8, 32])
def test_subset_vs_oracle_gradient(env, n_lines):
    """8 TRs (the workload) and 32 TRs (four times longer)."""
    gb, torch, ph, t1c, t2c, seq, rf, pb, w = env
    if n_lines != 8:
        ph, t1c, t2c, seq, rf, pb = synth.adjoint_workload(n_lines=n_lines)
        rng = np.random.default_rng(12)
        w = rng.standard_normal(seq.total_samples) + 1j * rng.standard_normal(seq.total_samples)
    sub = ph.subset(synth.random_subset_indices(ph.K, 4096, seed=7))
    say(f"[gpu] adjoint: 4096-isochromat subset, {n_lines} TRs, {seq.stepped_count()} stepped steps")
    sim, adj = make(gb, torch, sub, seq, pb)
    sig, g_rf, g1, g2 = run(adj, torch, rf, t1c, t2c, w)
    sim.close()
    rf32 = rf.real.astype(np.float32) + 1j * rf.imag.astype(np.float32)  # what the GPU played
    s_o, g_o, g1_o, g2_o = oracle.adjoint(sub, sub.labels, np.float32(t1c), np.float32(t2c), seq, rf32, pb, w)
    present = np.unique(sub.labels)
    r_sig, r_rf = rel(sig, s_o), rel(g_rf, g_o)
    r1 = float(np.max(np.abs(g1 - g1_o)[present] / np.abs(g1_o[present])))
    r2 = float(np.max(np.abs(g2 - g2_o)[present] / np.abs(g2_o[present])))
    say(f"[gpu] adjoint vs oracle: signal rel {r_sig:.2e}; dL/dB1 rel L2 {r_rf:.2e}; "
        f"dL/dT1 max rel {r1:.2e}; dL/dT2 max rel {r2:.2e}")
    assert r_sig <= 1e-4
    assert r_rf <= 1e-4 and r1 <= 5e-4 and r2 <= 5e-4


def test_adjoint_series_branches(env):
    """The adjoint's rotation coefficients switch per isochromat between a
    five-term series (q < 1/16), a nine-term series (q < 4) and sqrt plus
    sincos.  Each TR excites with the parameter pulse (no gradient), then plays
    a weak RF under a strong Gx with x the fastest phantom index, so that
    every wavefront has raster steps on all three branches: 0.1 rad per step
    at |x| = 4 mm up to 3.1 rad at the edge (MR raster steps rotate by far
    less).  A relaxation block rephases the Gx moment, so the echo and its
    gradients stay large.  Against the FP64 oracle adjoint: signal and RF
    gradient within 1e-4, T1 and T2 derivatives within 5e-4 (relative L2 over
    the classes)."""
    gb, torch = env[0], env[1]
    ph = synth.ellipse_phantom(32, 32, 2, (0.256, 0.256, 0.010), synth.SIX_T1, synth.SIX_T2, synth.SIX_PD,
                               df_range=50.0, df_levels=8, seed=77, name="adjoint-branches")
    dt, n_rf, n_g = 1e-5, 400, 200
    g = 0.1 / (2 * np.pi * synth.GAMMA_BAR * dt * 0.004)
    rf = synth.sinc_pulse(n_rf, dt, np.deg2rad(30.0), 4.0).astype(np.complex128) * np.exp(0.4j)
    weak = np.full(n_g, 2e-8 + 1e-8j)
    sb = synth.SeqBuilder(dt, name="adjoint-branches")
    for _ in range(2):
        sb.rf(rf)
        sb.rf(weak, g=(g, 0.0, 0.0))
        sb.relax(1e-3, moment=(-g * n_g * dt, 0.0, 0.0))
        sb.adc(64, (2e-3, 0.0, 0.0), np.arange(0, 64, 2))
        sb.relax(5e-3)
    seq = sb.build()
    pb = np.nonzero(np.asarray(seq.btype) == synth.BLOCK_RF)[0][::2].astype(np.int32)  # the excitations
    t1c, t2c = np.array(synth.SIX_T1), np.array(synth.SIX_T2)
    rng = np.random.default_rng(13)
    w = rng.standard_normal(seq.total_samples) + 1j * rng.standard_normal(seq.total_samples)
    say(f"[gpu] adjoint: series branches, K={ph.K}, {seq.stepped_count()} stepped steps")
    sim, adj = make(gb, torch, ph, seq, pb)
    sig, g_rf, g1, g2 = run(adj, torch, rf, t1c, t2c, w)
    sim.close()
    rf32 = rf.real.astype(np.float32) + 1j * rf.imag.astype(np.float32)
    s_o, g_o, g1_o, g2_o = oracle.adjoint(ph, ph.labels, np.float32(t1c), np.float32(t2c), seq, rf32, pb, w)
    r_sig, r_rf, r1, r2 = rel(sig, s_o), rel(g_rf, g_o), rel(g1, g1_o), rel(g2, g2_o)
    say(f"[gpu] adjoint, series branches: signal rel {r_sig:.2e}; dL/dB1 rel L2 {r_rf:.2e}; "
        f"dL/dT1 rel L2 {r1:.2e}; dL/dT2 rel L2 {r2:.2e}")
    assert r_sig <= 1e-4
    assert r_rf <= 1e-4 and r1 <= 5e-4 and r2 <= 5e-4


def _played(seq, rf, pb):
    """Sequence whose parameter blocks play rf (stored in float32 by the library)."""
    s = synth.Sequence(**{f: getattr(seq, f) for f in seq.__dataclass_fields__})
    s.rf_re, s.rf_im = np.array(seq.rf_re, np.float32), np.array(seq.rf_im, np.float32)
    for b in pb:
        o, n = int(seq.step_offset[b]), int(seq.n_steps[b])
        s.rf_re[o:o + n] = rf.real
        s.rf_im[o:o + n] = rf.imag
    return s


def test_fullsize_vs_finite_differences(env):
    """Central differences (relative step 1e-4) of L computed by the FP64 plain
    GPU path (an independent kernel whose FD noise is ~1e-12) at full size,
    against the FP32 adjoint; the perturbations are the float32 values the
    library actually plays, so input rounding does not enter."""
    gb, torch, ph, t1c, t2c, seq, rf, pb, w = env
    say(f"[gpu] adjoint: full size K={ph.K}, forward + backward")
    sim, adj = make(gb, torch, ph, seq, pb)
    t1c32, t2c32 = np.float32(t1c), np.float32(t2c)
    rf32 = (rf.real.astype(np.float32) + 1j * rf.imag.astype(np.float32)).astype(np.complex128)
    _, g_rf, g1, g2 = run(adj, torch, rf32, t1c32, t2c32, w)
    sim.close()
    plain = gb.Simulator(0)

    def L(rf_, t1_, t2_):
        p = synth.Phantom(ph.x, ph.y, ph.z, np.float32(t1_)[ph.labels], np.float32(t2_)[ph.labels], ph.df, ph.m0)
        plain.set_phantom(p)
        plain.set_sequence(_played(seq, rf_, pb))
        _, sig = plain.simulate(gb.GBS_PLAIN)
        sg = sig.cpu().numpy()
        return float(np.sum(w.real * sg.real + w.imag * sg.imag))

    rng = np.random.default_rng(21)
    scale = float(np.max(np.abs(rf)))
    worst_rf = 0.0
    for _ in range(2):
        d = rng.standard_normal(rf.size) + 1j * rng.standard_normal(rf.size)
        d *= 1e-4 * scale / np.sqrt(np.mean(np.abs(d) ** 2))
        rp = (rf32 + d).astype(np.complex64).astype(np.complex128)
        rm = (rf32 - d).astype(np.complex64).astype(np.complex128)
        fd = L(rp, t1c32, t2c32) - L(rm, t1c32, t2c32)
        an = float(np.sum(g_rf.real * (rp - rm).real + g_rf.imag * (rp - rm).imag))
        say(f"[gpu] adjoint FD (RF direction): dL fd {fd:.6e} adjoint {an:.6e}")
        worst_rf = max(worst_rf, abs(fd - an) / abs(an))
    v_fd, v_an = [], []
    for c in np.unique(ph.labels):
        for which, base, g in ((1, t1c32, g1), (2, t2c32, g2)):
            e = np.zeros(base.size, np.float64)
            e[c] = 1e-4 * base[c]
            hp, hm = np.float32(base + e), np.float32(base - e)
            dlt = float(hp[c]) - float(hm[c])
            if which == 1:
                fd = L(rf32, hp, t2c32) - L(rf32, hm, t2c32)
            else:
                fd = L(rf32, t1c32, hp) - L(rf32, t1c32, hm)
            say(f"[gpu] adjoint FD (T{which} class {c}): dL fd {fd:.6e} adjoint {g[c] * dlt:.6e}")
            v_fd.append(fd)
            v_an.append(g[c] * dlt)
    plain.close()
    v_fd, v_an = np.array(v_fd), np.array(v_an)
    r_t = rel(v_an, v_fd)
    r_inf = float(np.max(np.abs(v_an - v_fd)) / np.max(np.abs(v_fd)))
    say(f"[gpu] adjoint FD: RF directions worst rel {worst_rf:.2e}; T1/T2 vector rel L2 {r_t:.2e}, "
        f"max component error / largest component {r_inf:.2e}")
    # norm-wise bars: a class sum that cancels to a small value keeps only the
    # absolute accuracy of its terms
    assert worst_rf <= 1e-4 and r_t <= 2e-4 and r_inf <= 2e-4


def test_autograd_function_and_checkpoint_interval(env):
    gb, torch, ph, t1c, t2c, seq, rf, pb, w = env
    sub = ph.subset(synth.random_subset_indices(ph.K, 1000, seed=9))  # ragged: not a multiple of 256
    say("[gpu] adjoint: autograd wrapper and checkpoint interval, 1000 isochromats")
    sim, adj = make(gb, torch, sub, seq, pb, every=256)
    ref = run(adj, torch, rf, t1c, t2c, w)
    rft, t1t, t2t = (t.clone().requires_grad_(True) for t in tens(torch, rf, t1c, t2c))
    sig = gb.bloch_signal(adj, rft, t1t, t2t)
    (sig * wt(torch, w)).sum().backward()
    g = rft.grad.cpu().numpy().astype(np.float64)
    # two backward passes: the order of the workgroup's LDS atomics may differ
    assert rel(g[:, 0] + 1j * g[:, 1], ref[1]) <= 1e-6
    np.testing.assert_allclose(t1t.grad.cpu().numpy(), ref[2], rtol=1e-5)
    sim.close()
    for every in (16, 8):
        sim_e, adj_e = make(gb, torch, sub, seq, pb, every=every)
        r_e = run(adj_e, torch, rf, t1c, t2c, w)
        sim_e.close()
        say(f"[gpu] adjoint: every={every} vs 256: rf rel {rel(r_e[1], ref[1]):.2e}")
        assert np.array_equal(r_e[0], ref[0])
        assert rel(r_e[1], ref[1]) <= 1e-6 and np.allclose(r_e[2], ref[2], rtol=1e-6)


def test_no_parameter_blocks(env):
    """With no block listed as playing the parameter pulse, every RF block
    plays its own B1: the RF gradient is exactly zero and the T1/T2 gradients
    still match the oracle (512-isochromat subset, 2 TRs)."""
    gb, torch, ph, t1c, t2c, seq, rf, pb, w = env
    sub = ph.subset(synth.random_subset_indices(ph.K, 512, seed=11))
    ph2, _, _, seq2, _, _ = synth.adjoint_workload(8, 8, 2, n_lines=2, n_read=16, rf_steps=3000)
    w2 = w[:seq2.total_samples]
    none = np.zeros(0, np.int32)
    say("[gpu] adjoint: no parameter blocks, 512 isochromats, 2 TRs")
    sim, adj = make(gb, torch, sub, seq2, none)
    sig, g_rf, g1, g2 = run(adj, torch, rf, t1c, t2c, w2)
    sim.close()
    rf32 = rf.real.astype(np.float32) + 1j * rf.imag.astype(np.float32)
    s_o, _, g1_o, g2_o = oracle.adjoint(sub, sub.labels, np.float32(t1c), np.float32(t2c), seq2, rf32, none, w2)
    r1, r2 = rel(g1, g1_o), rel(g2, g2_o)  # norm-wise: some class sums nearly cancel
    say(f"[gpu] adjoint, no parameter blocks: signal rel {rel(sig, s_o):.2e}; T1 {r1:.2e}; T2 {r2:.2e}")
    assert not np.any(g_rf)
    assert rel(sig, s_o) <= 1e-4 and r1 <= 5e-4 and r2 <= 5e-4

