"""GPU parity at the benchmark's full size (1024x1024x26 = 27,262,976
isochromats), in the launch configuration bench.py times.

The FP64 oracle cannot run 27M isochromats through 1.08M raster steps, so:
* final M of seeded sampled isochromats is compared with the oracle run on
  just those isochromats (isochromats are independent);
* the full signal is compared with the FP64 plain GPU path (itself checked
  against the oracle on smaller workloads) where that path is affordable: the
  whole EPI and the first FSE shot;
* superposition (the signal is a sum over isochromats, Eq. 6) is checked for
  the whole FSE: phantom = A + B gives signal(A) + signal(B);
* the whole FSE and EPI are compared between the grouped update and the
  conventional method with per-isochromat transition caching.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

DM_TOL = 1e-5
SIG_TOL = 1e-4


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def big():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_03960_amd as gb
    ph = synth.brain_like_phantom()
    sim = gb.Simulator(0)
    sim.set_phantom(ph)
    sim.build_groups()
    yield gb, ph, sim
    sim.close()


def run(sim, gb, seq, mode):
    import torch
    sim.set_sequence(seq)
    M, sig = sim.simulate(mode)
    torch.cuda.synchronize()
    return M.cpu().numpy(), sig.cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def sampled_error(ph, seq, M, n=64, seed=11):
    idx = synth.random_subset_indices(ph.K, n, seed=seed)
    Mr, _ = oracle.simulate(ph.subset(idx), seq)
    return float(np.max(np.abs(M[:, idx].astype(np.float64) - Mr)))


def test_fse_fullsize_sampled_m(big):
    gb, ph, sim = big
    seq = synth.fse_sequence()
    say(f"[gpu] FSE full K={ph.K}: grouped")
    M, sig = run(sim, gb, seq, gb.GBS_GROUPED)
    assert np.all(np.isfinite(M)) and np.all(np.isfinite(sig))
    dm = sampled_error(ph, seq, M)
    say(f"[gpu] FSE full: sampled max|dM| = {dm:.3e}")
    assert dm <= DM_TOL


def test_epi_fullsize_vs_plain_fp64(big):
    gb, ph, sim = big
    seq = synth.epi_sequence()
    say("[gpu] EPI full: grouped")
    Mg, sg = run(sim, gb, seq, gb.GBS_GROUPED)
    say("[gpu] EPI full: plain FP64")
    Mp, sp = run(sim, gb, seq, gb.GBS_PLAIN)
    dm, r = float(np.max(np.abs(Mg - Mp))), rel(sg, sp)
    dmo = sampled_error(ph, seq, Mg)
    say(f"[gpu] EPI full: grouped vs plain max|dM|={dm:.3e} rel_sig={r:.3e}; sampled vs oracle {dmo:.3e}")
    assert dm <= DM_TOL and r <= SIG_TOL and dmo <= DM_TOL


def test_fse_first_shot_fullsize_vs_plain_fp64(big):
    gb, ph, sim = big
    shot = synth.fse_sequence().head(66, name="fse-shot1")
    say("[gpu] FSE shot 1 full: grouped")
    Mg, sg = run(sim, gb, shot, gb.GBS_GROUPED)
    say("[gpu] FSE shot 1 full: plain FP64")
    Mp, sp = run(sim, gb, shot, gb.GBS_PLAIN)
    dm, r = float(np.max(np.abs(Mg - Mp))), rel(sg, sp)
    say(f"[gpu] FSE shot 1 full: grouped vs plain max|dM|={dm:.3e} rel_sig={r:.3e}")
    assert dm <= DM_TOL and r <= SIG_TOL


@pytest.mark.parametrize("name", ["fse", "epi"])
def test_cached_fullsize_vs_grouped(big, name):
    """The conventional method with per-isochromat caching (GBS_CACHED) and the
    grouped update are independent algorithms for the same discrete model:
    at full size they must agree to the parity bar, and sampled isochromats of
    the cached result must match the oracle."""
    gb, ph, sim = big
    seq = synth.fse_sequence() if name == "fse" else synth.epi_sequence()
    say(f"[gpu] {name} full K={ph.K}: cached")
    Mc, sc = run(sim, gb, seq, gb.GBS_CACHED)
    say(f"[gpu] {name} full: grouped")
    Mg, sg = run(sim, gb, seq, gb.GBS_GROUPED)
    dm, r = float(np.max(np.abs(Mc - Mg))), rel(sc, sg)
    dmo = sampled_error(ph, seq, Mc, n=32, seed=13)
    say(f"[gpu] {name} full: cached vs grouped max|dM|={dm:.3e} rel_sig={r:.3e}; sampled vs oracle {dmo:.3e}")
    assert dm <= DM_TOL and r <= SIG_TOL and dmo <= DM_TOL


def test_coils_fullsize_grouped_vs_cached(big):
    """Four receive coils on the whole FSE: the grouped update (coil weights in
    every emission) against the cached conventional method (coil weights in
    every direct sample), per coil."""
    import torch
    gb, ph, sim = big
    seq = synth.fse_sequence()
    sim.set_sequence(seq)
    sim.set_coils(synth.coil_maps(ph, 4))
    say("[gpu] FSE full, 4 coils: grouped")
    Mg, sg = sim.simulate(gb.GBS_GROUPED)
    torch.cuda.synchronize()
    Mg, sg = Mg.cpu().numpy(), sg.cpu().numpy()
    say("[gpu] FSE full, 4 coils: cached")
    Mc, sc = sim.simulate(gb.GBS_CACHED)
    torch.cuda.synchronize()
    Mc, sc = Mc.cpu().numpy(), sc.cpu().numpy()
    sim.set_coils(None)
    dm = float(np.max(np.abs(Mg - Mc)))
    r = [rel(sg[p], sc[p]) for p in range(4)]
    say(f"[gpu] FSE full, 4 coils: max|dM|={dm:.3e} rel_sig per coil={r}")
    assert dm <= DM_TOL and max(r) <= SIG_TOL


@pytest.mark.parametrize("name", ["se-epi", "t2w-se", "oblique-fse", "fat-sat-fse"])
def test_workloads_fullsize_sampled(big, name):
    """The other full-size workloads the benchmark times (a Table 2 spin-echo
    EPI and T2W spin echo, the oblique-slice FSE with two-axis groups, the
    fat-saturated FSE with no-grads groups): sampled isochromats against the
    oracle, in the benchmark's configuration (all group axes built)."""
    gb, ph, sim = big
    seq = {"se-epi": lambda: synth.table2_sequences()["se-epi"],
           "t2w-se": lambda: synth.table2_sequences()["t2w-se"].head(40, name="t2w-se[:10 TR]"),
           "oblique-fse": lambda: synth.fse_sequence(tilt_deg=20.0),
           "fat-sat-fse": lambda: synth.fse_sequence(fat_sat=True)}[name]()
    say(f"[gpu] {name} full K={ph.K}: grouped")
    M, sig = run(sim, gb, seq, gb.GBS_GROUPED)
    assert np.all(np.isfinite(M)) and np.all(np.isfinite(sig))
    dm = sampled_error(ph, seq, M, n=32, seed=19)
    say(f"[gpu] {name} full: sampled max|dM| = {dm:.3e}")
    assert dm <= DM_TOL


def test_fse_fullsize_superposition(big):
    import torch
    gb, ph, sim = big
    seq = synth.fse_sequence()
    _, s_all = run(sim, gb, seq, gb.GBS_GROUPED)
    half = ph.K // 2 + 12345  # not a multiple of any tile
    parts = []
    for idx in (np.arange(half), np.arange(half, ph.K)):
        sub = gb.Simulator(0)
        sub.set_phantom(ph.subset(idx))
        sub.build_groups()
        sub.set_sequence(seq)
        _, s = sub.simulate(gb.GBS_GROUPED)
        torch.cuda.synchronize()
        parts.append(s.cpu().numpy())
        sub.close()
    r = rel(parts[0] + parts[1], s_all)
    say(f"[gpu] FSE full: superposition rel = {r:.3e}")
    assert r <= 1e-6


def test_pulseq_epi_fullsize(big):
    """The benchmark's EPI shape (128 lines of 128 samples, 4 us dwell) read
    from a Pulseq file, grouped at full size: sampled isochromats against the
    oracle, and the signal against the cached conventional method."""
    gb, ph, sim = big
    from synth.pulseq import epi_text
    seq = gb.load_pulseq(epi_text(n_lines=128, n_read=128, fov=0.256, dwell_us=4, ramp_us=44))
    say(f"[gpu] pulseq EPI full size: grouped, K={ph.K}, steps={seq.total_steps}")
    M, s = run(sim, gb, seq, gb.GBS_GROUPED)
    dm = sampled_error(ph, seq, M, n=256)
    say(f"[gpu] pulseq EPI full size: sampled max|dM| {dm:.3e}; cached")
    _, s_c = run(sim, gb, seq, gb.GBS_CACHED)
    r = rel(s, s_c)
    say(f"[gpu] pulseq EPI full size: grouped vs cached signal {r:.3e}")
    assert dm <= DM_TOL and r <= SIG_TOL
