"""GPU parity of multi-coil signals (Eq. 6 and Eq. 9 with P receive coils):
the grouped and the cached modes against the oracle's coil sums, built from
single-isochromat runs.  Same bar as the other parity tests, per coil."""
import numpy as np
import pytest

import oracle
import synth
from synth import SeqBuilder

pytestmark = pytest.mark.gpu

DM_TOL = 1e-5
SIG_TOL = 1e-4


@pytest.fixture(scope="module")
def gb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_03960_amd as gb
    return gb


def say(msg):
    print(msg, flush=True)


def run(gb, ph, seq, mode, sens, axes=None, m_init=None):
    import torch
    sim = gb.Simulator(0)
    sim.set_phantom(ph)
    sim.set_sequence(seq)
    if sens is not None:
        sim.set_coils(sens)
    if mode == gb.GBS_GROUPED:
        sim.build_groups(gb.GBS_AX_ALL if axes is None else axes)
    mi = None if m_init is None else torch.from_numpy(np.ascontiguousarray(m_init, np.float32))
    M, sig, st = sim.simulate(mode, m_init=mi, stats=True)
    torch.cuda.synchronize()
    out = M.cpu().numpy().astype(np.float64), sig.cpu().numpy().copy(), st, sim.info()
    sim.close()
    return out


def check(gb, name, ph, seq, sens, m_init=None, axes=None, plain=False):
    Mr, sr = oracle.simulate_coils(ph, seq, sens, m_init=m_init)
    modes = ((gb.GBS_GROUPED, "grouped"), (gb.GBS_CACHED, "cached")) + (((gb.GBS_PLAIN, "plain"),) if plain else ())
    for mode, label in modes:
        say(f"[gpu] coils {name}: {label} K={ph.K} P={sens.shape[0]}")
        M, sig, _, info = run(gb, ph, seq, mode, sens, axes=axes, m_init=m_init)
        sig = sig.reshape(sens.shape[0], -1)
        dm = float(np.max(np.abs(M - Mr)))
        rel = [float(np.linalg.norm(sig[p] - sr[p]) / np.linalg.norm(sr[p])) for p in range(sens.shape[0])]
        say(f"[gpu] coils {name}: {label} max|dM|={dm:.3e} rel_sig per coil={['%.2e' % r for r in rel]}")
        assert info["n_coils"] == sens.shape[0]
        assert dm <= DM_TOL and max(rel) <= SIG_TOL, (name, label, dm, rel)


def readouts_sequence():
    """Readouts along every axis and without gradients (x, y, z and no-grads
    emissions of the sweep), with an excitation and refocusing in between."""
    dt = 1e-6
    sb = SeqBuilder(dt, "coil-axes")
    sb.rf(synth.sinc_pulse(200, dt, np.pi / 2), (0, 0, 0.012))
    sb.relax(4e-4, (-2e-6, 1e-6, -1.2e-6))
    sb.adc(64, (0.01, 0, 0), 4 * np.arange(16) + 2)          # Gx readout
    sb.relax(2e-4, (0, -3e-6, 0))
    sb.adc(48, (0, 0.012, 0), 3 * np.arange(16) + 1)          # Gy readout
    sb.rf(synth.sinc_pulse(200, dt, np.pi, phase=np.pi / 2), (0, 0, 0.012))
    sb.relax(3e-4, (0, 0, 2e-6))
    sb.adc(40, (0, 0, 0.02), 5 * np.arange(8) + 2)            # Gz readout
    sb.adc(30, (0, 0, 0), 3 * np.arange(10))                  # no gradients
    return sb.build()


def test_coils_small_gre(gb):
    ph = synth.gre_phantom(8, 8, 2, seed=41)
    seq = synth.gre_sequence(n_lines=3, n_read=16, dwell_steps=4, rf_steps=400, te=2.5e-3, tr=6e-3)
    check(gb, "gre", ph, seq, synth.coil_maps(ph, 3), plain=True)


def test_coils_with_stepped_readouts(gb):
    """Readouts stepped per isochromat (RF during the ADC, a mixed-gradient
    readout) carry one weighted sum per coil in every mode; 8 coils cut the
    stepped launches to 32 samples, so a 100-sample readout takes four."""
    ph = synth.tiny_phantom(nx=7, ny=6, nz=3, n_classes=3, df_levels=3)
    sb = SeqBuilder(1e-6, "stepped-readouts")
    sb.rf(synth.sinc_pulse(200, 1e-6, np.pi / 2), (0, 0, 0.012))
    sb.relax(3e-4, (-1e-6, 2e-6, -1.2e-6))
    sb.adc(40, (0.01, 0, 0), [0, 5, 19, 39], b1=np.full(40, 1e-6 + 0j))      # RF during the readout
    sb.adc(200, (0.006, 0.004, 0), 2 * np.arange(100))                        # two gradients: stepped
    sb.adc(64, (0.01, 0, 0), 4 * np.arange(16) + 2)                           # grouped
    seq = sb.build()
    check(gb, "stepped/3", ph, seq, synth.coil_maps(ph, 3, radius=0.012, width=0.01), plain=True)
    check(gb, "stepped/8", ph, seq, synth.coil_maps(ph, 8, radius=0.012, width=0.01), plain=True)


def test_coils_every_emission_axis(gb):
    ph = synth.tiny_phantom(nx=7, ny=6, nz=3, n_classes=3, df_levels=3)
    seq = readouts_sequence()
    S = synth.coil_maps(ph, 4, radius=0.012, width=0.01)
    check(gb, "axes", ph, seq, S)
    check(gb, "axes/no tissue groups", ph, seq, S, axes=gb.GBS_AX_X | gb.GBS_AX_Y | gb.GBS_AX_Z)
    rng = np.random.default_rng(6)
    check(gb, "axes/m_init", ph, seq, S[:2], m_init=rng.uniform(-0.5, 0.5, (3, ph.K)))


@pytest.mark.parametrize("name", ["fse-small", "epi-small"])
def test_coils_fse_epi_small(gb, name):
    ph, seq = synth.workload(name)
    sub = synth.random_subset_indices(ph.K, 160, seed=9)  # the oracle runs every isochromat alone
    ph = ph.subset(sub)
    check(gb, name, ph, seq, synth.coil_maps(ph, 2, radius=0.03, width=0.03))


def test_coils_with_two_axis_and_emission_runs(gb):
    """Coils together with an oblique slice (transition rows per two-axis group
    in the coil sweep) and with an EPI readout train of more than 16
    emission-only operations (coil runs keep the coil sweep)."""
    ph = synth.tiny_phantom(nx=7, ny=6, nz=3, n_classes=3, df_levels=3)
    S = synth.coil_maps(ph, 3, radius=0.012, width=0.01)
    ob = synth.gre_sequence(n_lines=2, n_read=16, dwell_steps=4, rf_steps=300, te=2.5e-3, tr=6e-3, tilt_deg=25.0)
    check(gb, "oblique", ph, ob, S)
    _, _, st, info = run(gb, ph, ob, gb.GBS_GROUPED, S)
    assert st["n_fallback"] == 0 and info["n_xz_groups"] > 0, (st, info)
    epi = synth.epi_sequence(n_lines=20, n_read=16, rf_steps=400)
    check(gb, "epi20", ph, epi, S[:2])


def test_unit_sensitivity_equals_the_default(gb):
    """One coil of S = 1 through the coil path (general sweep) against the
    default single-coil run (fast sweep)."""
    ph, seq = synth.workload("fse-small")
    for mode in (gb.GBS_GROUPED, gb.GBS_CACHED):
        M0, s0, _, _ = run(gb, ph, seq, mode, None)
        M1, s1, _, info = run(gb, ph, seq, mode, np.ones((1, ph.K), np.complex128))
        assert info["n_coils"] == 1
        assert np.max(np.abs(M1 - M0)) <= 1e-6
        assert np.linalg.norm(s1.reshape(-1) - s0) <= 1e-6 * np.linalg.norm(s0)


def test_coil_errors(gb):
    import torch
    ph = synth.tiny_phantom(nx=5, ny=4, nz=2)
    seq = readouts_sequence()
    sim = gb.Simulator(0)
    sim.set_phantom(ph)
    sim.set_sequence(seq)
    sim.build_groups()
    S = synth.coil_maps(ph, 2)
    bad = S.copy()
    bad[1, 3] = np.nan
    codes = []
    for sens in (bad, np.ones((9, ph.K))):
        with pytest.raises(gb.GbsError) as e:
            sim.set_coils(sens)
        codes.append(e.value.code)
    assert codes == [gb.GBS_E_INVALID] * 2
    sim.set_coils(S)
    assert sim.info()["n_coils"] == 2
    sim.set_phantom(ph)  # back to one coil of unit sensitivity
    assert sim.info()["n_coils"] == 1
    sim.set_sequence(seq)
    sim.build_groups()
    M, sig = sim.simulate(gb.GBS_GROUPED)
    torch.cuda.synchronize()
    assert sig.shape == (seq.total_samples,)
    sim.close()
