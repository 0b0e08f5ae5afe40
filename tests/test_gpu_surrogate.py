"""GPU parity of the learned RF-transition surrogate against its FP64 oracle
(oracle/surrogate.py), through the C ABI.

Bars:
* exact transitions (FP64 on both sides, different summation order over
  3000 steps): max |dT| <= 1e-9;
* network outputs: the GPU rounds weights to BF16 exactly as the oracle does;
  activations travel as BF16 hi + lo pairs (relative error <= 2^-17 each)
  with FP32 accumulation, so outputs of size O(1) agree to ~1e-5; the
  transition adds the reference K_ref (FP64 on both sides, from tables that
  agree to FP32 rounding) and 1/8 of the output; bar 1e-4;
* loss and gradient: relative 1e-4 (loss) and 1e-3 (gradient, L2), from the
  same per-operand error carried through the backward pass and the FP32
  sums over the batch;
* inside a simulation the usual parity bar (|dM| <= 1e-5, relative signal
  <= 1e-4) holds whenever the spot check falls back to the exact transition.
"""
import time

import numpy as np
import pytest

import oracle
import synth
from oracle import surrogate as so

pytestmark = pytest.mark.gpu

DM_TOL = 1e-5
SIG_TOL = 1e-4


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_03960_amd as gb
    pulse = synth.fse_refocusing_pulse()
    return gb, torch, pulse


@pytest.fixture(scope="module")
def table():
    return so.reference_table(synth.fse_refocusing_pulse())


def make_mlp(gb, pulse, seed=3):
    m = gb.Mlp(0)
    rf, gz, dt = pulse
    m.set_pulse(rf, gz, dt)
    m.set_params(synth.mlp_init_params(seed=seed))
    return m


def test_exact_transitions_vs_oracle(env):
    gb, torch, pulse = env
    m = make_mlp(gb, pulse)
    tup = synth.surrogate_tuples(13, seed=31)
    tup[0] = [0.0, 0.0, 1.0, 0.1, 1.0]
    say("[gpu] surrogate: exact transitions, 13 tuples")
    T = m.exact(torch.from_numpy(tup)).cpu().numpy()
    Tr = so.transition(pulse, tup)
    err = float(np.max(np.abs(T - Tr)))
    say(f"[gpu] surrogate: exact max|dT| = {err:.3e}")
    assert err <= 1e-9
    m.close()


def test_infer_vs_oracle_forward(env, table):
    gb, torch, pulse = env
    m = make_mlp(gb, pulse)
    tup = synth.surrogate_tuples(2021, seed=32)  # not a multiple of the 32-sample tile
    say("[gpu] surrogate: inference, 2021 tuples")
    T = m.infer(torch.from_numpy(tup)).cpu().numpy().astype(np.float64)
    Tr = so.mlp_transition(synth.mlp_init_params(seed=3), tup, pulse[2] * len(pulse[0]) / 2, table)
    err = float(np.max(np.abs(T - Tr)))
    say(f"[gpu] surrogate: inference max|dT| = {err:.3e} (outputs up to {np.max(np.abs(Tr)):.2f})")
    assert err <= 1e-4
    m.close()


def test_reference_vs_oracle(env, table):
    """A network whose last layer is zero outputs the reference transition
    alone: the library's table (built from its own exact transitions when the
    pulse is set) and interpolation against the oracle's."""
    gb, torch, pulse = env
    m = gb.Mlp(0)
    rf, gz, dt = pulse
    m.set_pulse(rf, gz, dt)
    parts = so.unpack(synth.mlp_init_params(seed=3))
    parts[6][:] = 0.0
    parts[7][:] = 0.0
    m.set_params(so.pack(parts).astype(np.float32))
    tup = synth.surrogate_tuples(3001, seed=41)
    tup[:5, 0] = [-1700.0, 1700.0, 0.0, 1599.9, -1600.0]  # clamped beyond the table, on and at its ends
    say("[gpu] surrogate: reference transition (zero last layer), 3001 tuples")
    T = m.infer(torch.from_numpy(tup)).cpu().numpy().astype(np.float64)
    half = dt * len(rf) / 2
    Tr = so.frame(so.reference(table, tup, half), tup, half, inverse=True)
    err = float(np.max(np.abs(T - Tr)))
    say(f"[gpu] surrogate: reference max|dT| = {err:.3e}")
    assert err <= 1e-5
    m.close()


def _targets(n, seed):
    tup = synth.surrogate_tuples(n, seed=seed)
    return tup, so.transition(synth.fse_refocusing_pulse(), tup)


@pytest.fixture(scope="module")
def batch512():
    return _targets(512, 33)


@pytest.mark.parametrize("n", [64, 192, 512])
def test_loss_grad_vs_oracle(env, batch512, table, n):
    """Loss and weight gradient against the FP64 oracle.  The gradient
    kernel splits the batch's 32-sample chunks over 8 wavefronts: 64 samples
    leave six of them empty, 192 split unevenly."""
    gb, torch, pulse = env
    m = make_mlp(gb, pulse)
    tup, T = batch512
    tup, T = tup[:n], T[:n]
    say(f"[gpu] surrogate: loss and gradient, {n} samples")
    loss, g = m.loss_grad(torch.from_numpy(tup), torch.from_numpy(T))
    g = g.cpu().numpy().astype(np.float64)
    half = pulse[2] * len(pulse[0]) / 2
    lr_, gr = so.loss_grad(synth.mlp_init_params(seed=3), so.features(tup), so.targets(T, tup, half, table))
    rel_l = abs(loss - lr_) / lr_
    rel_g = float(np.linalg.norm(g - gr) / np.linalg.norm(gr))
    say(f"[gpu] surrogate: loss {loss:.6e} vs {lr_:.6e} (rel {rel_l:.2e}); grad rel L2 {rel_g:.2e}")
    assert rel_l <= 1e-4
    assert rel_g <= 1e-3
    assert float(np.max(np.abs(g - gr))) <= 1e-3 * float(np.max(np.abs(gr)))
    m.close()


def test_adam_step_and_repack_vs_oracle(env, batch512, table):
    gb, torch, pulse = env
    m = make_mlp(gb, pulse)
    tup, T = batch512
    tup, T = tup[:256], T[:256]
    p0 = synth.mlp_init_params(seed=3).astype(np.float64)
    half = pulse[2] * len(pulse[0]) / 2
    _, gr = so.loss_grad(p0, so.features(tup), so.targets(T, tup, half, table))
    say("[gpu] surrogate: one Adam step, batch 256")
    m.train(torch.from_numpy(tup), torch.from_numpy(T), epochs=1, batch=256, lr_max=1e-3, lr_min=0.0)
    p1 = m.get_params().astype(np.float64)
    want, _, _ = so.adam(p0, np.zeros_like(p0), np.zeros_like(p0), gr, 1, 1e-3)
    sel = np.abs(gr) > 1e-3 * np.max(np.abs(gr))  # first Adam step is lr*sign(g): compare where g is clear
    err = float(np.max(np.abs(p1 - want)[sel]))
    say(f"[gpu] surrogate: Adam step max|dw| = {err:.3e} over {int(sel.sum())} parameters")
    assert err <= 1e-6
    assert float(np.max(np.abs(p1 - p0))) <= 1e-3 * (1 + 1e-5)
    # the BF16 fragments were repacked from the updated master weights
    probe = synth.surrogate_tuples(100, seed=34)
    Tm = m.infer(torch.from_numpy(probe)).cpu().numpy().astype(np.float64)
    err2 = float(np.max(np.abs(Tm - so.mlp_transition(p1, probe, half, table))))
    say(f"[gpu] surrogate: inference after the step max|dT| = {err2:.3e}")
    assert err2 <= 1e-4
    m.close()


def test_training_reduces_loss(env):
    gb, torch, pulse = env
    m = make_mlp(gb, pulse)
    n = 65536
    tup = torch.from_numpy(synth.surrogate_tuples(n, seed=35)).cuda()
    say("[gpu] surrogate: exact targets for 65536 tuples, then 24 epochs of batch 1024")
    T = m.exact(tup)
    hist = m.train(tup, T, epochs=24, batch=1024, lr_max=2e-3, lr_min=1e-4, seed=1)
    first, last = float(hist[:32].mean()), float(hist[-32:].mean())
    say(f"[gpu] surrogate: mean loss of the first and last 32 steps {first:.3e} -> {last:.3e} "
        f"over {hist.size} steps")
    assert np.all(np.isfinite(hist))
    assert last < first / 10
    m.close()


def _fse_small_run(gb, torch, m, tol, flags_extra):
    ph, seq = synth.workload("fse-small")
    sim = gb.Simulator(0)
    sim.set_phantom(ph)
    sim.set_sequence(seq)
    sim.build_groups()
    gb.set_surrogate(sim, m, tol=tol, n_check=16, seed=5)
    M, sig, st = sim.simulate(gb.GBS_GROUPED, flags=flags_extra, stats=True)
    torch.cuda.synchronize()
    out = M.cpu().numpy().astype(np.float64), sig.cpu().numpy().copy(), st
    sim.close()
    return out


def test_surrogate_in_grouped_fse_falls_back(env):
    gb, torch, pulse = env
    m = make_mlp(gb, pulse)  # untrained: its transitions are far from exact
    ph, seq = synth.workload("fse-small")
    Mr, sr = oracle.simulate(ph, seq)
    say("[gpu] surrogate: FSE-small grouped with an untrained network, tol 1e-3")
    M, sig, st = _fse_small_run(gb, torch, m, 1e-3, gb.GBS_SURROGATE)
    dm = float(np.max(np.abs(M - Mr)))
    rel = float(np.linalg.norm(sig - sr) / np.linalg.norm(sr))
    say(f"[gpu] surrogate: stats n={st['n_surrogate']} fallback={st['n_surrogate_fallback']} "
        f"residual={st['surrogate_residual']:.3e}; max|dM|={dm:.3e} rel_sig={rel:.3e}")
    assert st["n_surrogate"] == 1 and st["n_surrogate_fallback"] == 1
    assert st["surrogate_residual"] > 1e-3
    assert dm <= DM_TOL and rel <= SIG_TOL
    say("[gpu] surrogate: same with tol 1e9 (network accepted)")
    M2, sig2, st2 = _fse_small_run(gb, torch, m, 1e9, gb.GBS_SURROGATE)
    assert st2["n_surrogate_fallback"] == 0
    assert float(np.linalg.norm(sig2 - sr) / np.linalg.norm(sr)) > 1e-3  # the network's T was used
    m.close()


def test_surrogate_in_cached_fse_falls_back(env):
    """GBS_CACHED with the surrogate: an untrained network fails the spot
    check, the gated exact composition runs and the usual parity bar holds;
    with an infinite tolerance the network's transitions are used."""
    gb, torch, pulse = env
    m = make_mlp(gb, pulse)
    ph, seq = synth.workload("fse-small")
    Mr, sr = oracle.simulate(ph, seq)
    out = {}
    for tol in (1e-3, 1e9):
        sim = gb.Simulator(0)
        sim.set_phantom(ph)
        sim.set_sequence(seq)
        gb.set_surrogate(sim, m, tol=tol, n_check=16, seed=5)
        say(f"[gpu] surrogate: FSE-small cached with an untrained network, tol {tol:g}")
        M, sig, st = sim.simulate(gb.GBS_CACHED, flags=gb.GBS_SURROGATE, stats=True)
        torch.cuda.synchronize()
        out[tol] = M.cpu().numpy().astype(np.float64), sig.cpu().numpy().copy(), st
        sim.close()
    M, sig, st = out[1e-3]
    dm = float(np.max(np.abs(M - Mr)))
    rel = float(np.linalg.norm(sig - sr) / np.linalg.norm(sr))
    say(f"[gpu] surrogate: cached stats n={st['n_surrogate']} fallback={st['n_surrogate_fallback']} "
        f"residual={st['surrogate_residual']:.3e}; max|dM|={dm:.3e} rel_sig={rel:.3e}")
    assert st["n_surrogate"] == 1 and st["n_surrogate_fallback"] == 1
    assert st["surrogate_residual"] > 1e-3
    assert dm <= DM_TOL and rel <= SIG_TOL
    M2, sig2, st2 = out[1e9]
    assert st2["n_surrogate"] == 1 and st2["n_surrogate_fallback"] == 0
    assert float(np.linalg.norm(sig2 - sr) / np.linalg.norm(sr)) > 1e-3  # the network's T was used
    m.close()


def test_surrogate_without_matching_pulse(env):
    """A sequence none of whose RF waveforms is the network's pulse (EPI
    plays only a 90-degree excitation) keeps every exact transition: the
    surrogate flag changes nothing, bit for bit."""
    gb, torch, pulse = env
    m = make_mlp(gb, pulse)
    ph, seq = synth.workload("epi-small")
    out = []
    for flags in (0, gb.GBS_SURROGATE):
        sim = gb.Simulator(0)
        sim.set_phantom(ph)
        sim.set_sequence(seq)
        sim.build_groups()
        gb.set_surrogate(sim, m, tol=1e9, n_check=16, seed=5)
        M, sig, st = sim.simulate(gb.GBS_GROUPED, flags=flags, stats=True)
        torch.cuda.synchronize()
        out.append((M.cpu().numpy(), sig.cpu().numpy().copy(), st))
        sim.close()
    m.close()
    say(f"[gpu] surrogate: EPI-small with no matching pulse: n_surrogate={out[1][2]['n_surrogate']}")
    assert out[1][2]["n_surrogate"] == 0 and out[1][2]["n_surrogate_fallback"] == 0
    assert np.array_equal(out[0][0], out[1][0])
    assert np.allclose(out[0][1], out[1][1], rtol=0, atol=1e-12 * np.max(np.abs(out[0][1])))


def test_trained_surrogate_gain(env):
    """What the trained network buys, at the spec's residual of 1e-3.

    Trained on 2M transitions of the 180-degree pulse (64 epochs of batch
    1024).  Per transition, on 1M held-out tuples over the whole training
    domain: the network against the exact FP64 composition, in speed and
    error (p99 and median under 1e-3).  In a simulation: the FSE under
    GBS_CACHED on a 256x256x26 phantom (1,703,936 isochromats), where the
    network replaces the per-isochromat composition of Eq. 7: its spot check
    (256 seeded isochromats, tol 1e-3) passes, the run is faster than the
    same run without the network, and its signal is within 1e-3 of the
    exact cached run's."""
    gb, torch, pulse = env
    m = make_mlp(gb, pulse, seed=7)
    tup = torch.from_numpy(synth.surrogate_tuples(1 << 21, seed=36)).cuda()
    say("[gpu] surrogate gain: exact targets for 2,097,152 tuples, train 64 epochs of batch 1024")
    T = m.exact(tup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = m.train(tup, T, epochs=64, batch=1024, lr_max=3e-3, lr_min=1e-6, seed=2)
    t_train = time.perf_counter() - t0
    del tup, T
    test = torch.from_numpy(synth.surrogate_tuples(1 << 20, seed=37)).cuda()
    for _ in range(2):  # second pass timed warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Tm = m.infer(test)
        torch.cuda.synchronize()
        t_inf = time.perf_counter() - t0
        t0 = time.perf_counter()
        Te = m.exact(test)
        torch.cuda.synchronize()
        t_ex = time.perf_counter() - t0
    err = (Tm.double() - Te).abs().max(dim=1).values.cpu().numpy()
    say(f"[gpu] surrogate gain: {hist.size} Adam steps in {t_train:.2f} s, final loss {hist[-1]:.3e}; "
        f"1,048,576 transitions: network {t_inf * 1e3:.2f} ms, exact {t_ex * 1e3:.2f} ms (x{t_ex / t_inf:.1f}); "
        f"max|dT| {err.max():.3e}, p99 {np.quantile(err, 0.99):.3e}, median {np.median(err):.3e}, "
        f"within 1e-3: {np.mean(err <= 1e-3) * 100:.2f} %")
    assert t_inf * 5 < t_ex
    assert np.quantile(err, 0.99) <= 1e-3 and np.median(err) <= 1e-3
    del Tm, Te, test

    ph = synth.brain_like_phantom(nx=256, ny=256, nz=26)
    seq = synth.fse_sequence()
    sim = gb.Simulator(0)
    sim.set_phantom(ph)
    sim.set_sequence(seq)
    gb.set_surrogate(sim, m, tol=1e-3, n_check=256, seed=9)
    res = {}
    for name, flags in (("exact", 0), ("network", gb.GBS_SURROGATE)):
        best = None
        for _ in range(3):
            M, sig, st = sim.simulate(gb.GBS_CACHED, flags=flags | gb.GBS_PROFILE, stats=True)
            torch.cuda.synchronize()
            best = st if best is None or st["ms_total"] < best["ms_total"] else best
        res[name] = (sig.cpu().numpy().copy(), best)
    sim.close()
    m.close()
    s_ex, st_ex = res["exact"]
    s_nn, st_nn = res["network"]
    rel = float(np.linalg.norm(s_nn - s_ex) / np.linalg.norm(s_ex))
    say(f"[gpu] surrogate gain: cached FSE 1,703,936 isochromats: exact {st_ex['ms_total']:.1f} ms "
        f"(compose {st_ex['ms_compose']:.1f} ms), network {st_nn['ms_total']:.1f} ms "
        f"(compose {st_nn['ms_compose']:.1f} ms); spot check residual {st_nn['surrogate_residual']:.3e}, "
        f"fallback {st_nn['n_surrogate_fallback']}; signal rel err vs exact {rel:.3e}")
    assert st_nn["n_surrogate"] == 1 and st_nn["n_surrogate_fallback"] == 0
    assert st_nn["surrogate_residual"] <= 1e-3
    assert st_nn["ms_total"] < st_ex["ms_total"]
    assert rel <= 1e-3
