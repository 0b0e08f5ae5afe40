"""GPU parity of GBS_CACHED, the conventional accelerated method (Sec. 2.2):
per-isochromat combined transitions (Eq. 7) composed at the first occurrence
of a with-RF waveform and reused from the cache, and with-ADC subsequences
evaluated at every sample from the block-start state (Eq. 4, 5, 6).

Same bar as the other modes against the FP64 oracle: max |dM| <= 1e-5 and
relative signal error <= 1e-4.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import SeqBuilder
from tests.test_gpu_parity import DM_TOL, SIG_TOL, check_case, errors, run_gpu, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_03960_amd as gb
    return gb


def test_cached_gre_4096(gb):
    ph, seq = synth.workload("gre")
    check_case(gb, "gre", ph, seq, modes=("cached",))
    _, _, st = run_gpu(gb, ph, seq, gb.GBS_CACHED)
    # 32 excitations of one waveform: composed once, read from the cache 31 times
    assert (st["n_rf_cached"], st["n_distinct_rf"], st["n_adc_direct"], st["n_fallback"]) == (32, 1, 32, 0), st
    assert st["cache_bytes"] == 48 * ph.K


def test_cached_fse_small(gb):
    ph, seq = synth.workload("fse-small")
    check_case(gb, "fse-small", ph, seq, modes=("cached",))


def test_cached_epi_small(gb):
    ph, seq = synth.workload("epi-small")
    check_case(gb, "epi-small", ph, seq, modes=("cached",))


def test_cached_ragged_k_and_initial_state(gb):
    ph = synth.gre_phantom(33, 31, 3, seed=21)  # K = 3069: not a multiple of a workgroup
    seq = synth.gre_sequence(n_lines=3, n_read=24, dwell_steps=4, rf_steps=600, te=2.5e-3, tr=7e-3)
    rng = np.random.default_rng(2)
    check_case(gb, "ragged+m_init", ph, seq, modes=("cached",), m_init=rng.uniform(-0.5, 0.5, (3, ph.K)))


def test_cached_classification_paths(gb):
    """Gx/Gy/no-grads and mixed-gradient RF (all cached per isochromat),
    Gy/Gz readouts with ramps (direct), ADC with RF (stepped)."""
    from tests.test_oracle_pins import _mini_sequences
    ph = synth.tiny_phantom(nx=9, ny=7, nz=3, n_classes=3, df_levels=3)
    for seq in _mini_sequences():
        check_case(gb, f"mini:{seq.name}", ph, seq, modes=("cached",))


def test_cached_edge_cases(gb):
    ph1 = synth.gre_phantom(1, 1, 1, seed=4)  # K = 1
    seq = synth.gre_sequence(n_lines=2, n_read=8, dwell_steps=2, rf_steps=200, te=1.5e-3, tr=4e-3)
    check_case(gb, "K=1", ph1, seq, modes=("cached",))
    ph = synth.tiny_phantom(nx=6, ny=5, nz=2)
    rng = np.random.default_rng(8)
    m_init = rng.uniform(-0.5, 0.5, (3, ph.K))
    sb = SeqBuilder(1e-6, "relax-only")
    sb.relax(2e-3, (1e-5, -2e-5, 3e-6))
    check_case(gb, "relax-only", ph, sb.build(), modes=("cached",), m_init=np.full((3, ph.K), 0.3))
    # a readout before any RF reads the initial state; 700 samples take three
    # launches; one sample per launch-chunk tail; a readout without samples
    sb = SeqBuilder(1e-6, "adc-first")
    sb.adc(800, (0.004, -0.002, 0.001), np.arange(0, 700))
    sb.relax(3e-4, (1e-6, 0, 0))
    sb.adc(30, (0.0, 0.0, 0.01), [])
    sb.rf(synth.sinc_pulse(80, 1e-6, 0.7), (0, 0, 0.01))
    sb.adc(40, (0.01, 0, 0), [3])
    check_case(gb, "adc-first", ph, sb.build(), modes=("cached",), m_init=m_init)
    sb = SeqBuilder(1e-6, "b1zero")
    sb.rf(np.zeros(50), (0, 0, 0.01))
    sb.rf(synth.sinc_pulse(80, 1e-6, 0.7), (0, 0, 0.01))
    sb.adc(16, (0.01, 0, 0), np.arange(0, 17, 4))
    check_case(gb, "b1zero", ph, sb.build(), modes=("cached",))
    check_case(gb, "empty", ph, SeqBuilder(1e-6, "empty").build(), modes=("cached",), m_init=m_init)


def test_cached_infinite_relaxation_times(gb):
    ph = synth.tiny_phantom(nx=5, ny=4, nz=2, n_classes=2)
    ph.t1[::3] = np.inf
    ph.t2[1::4] = np.inf
    seq = synth.gre_sequence(n_lines=2, n_read=8, dwell_steps=2, rf_steps=200, te=1.5e-3, tr=4e-3)
    check_case(gb, "T=inf", ph, seq, modes=("cached", "plain"))


def test_cached_reuse_matches_compose_and_repeats(gb):
    """Five occurrences of one waveform (composed once, applied four times from
    the FP32 cache) against the oracle; a second call on the same context
    recomposes and gives the same bits."""
    import torch
    ph = synth.tiny_phantom(nx=8, ny=6, nz=3, n_classes=3, df_levels=3)
    sb = SeqBuilder(1e-6, "reuse")
    b1 = synth.sinc_pulse(120, 1e-6, 0.9)
    for i in range(5):
        sb.rf(b1, (0, 0, 0.01))
        sb.relax(4e-4, (2e-6 * (i + 1), -1e-6, 0))
        sb.adc(24, (0.008, 0, 0), 3 * np.arange(8))
    seq = sb.build()
    check_case(gb, "reuse", ph, seq, modes=("cached",))
    sim = gb.Simulator(0)
    sim.set_phantom(ph)
    sim.set_sequence(seq)
    M1, s1, st = sim.simulate(gb.GBS_CACHED, stats=True, flags=gb.GBS_PROFILE)
    M1, s1 = M1.cpu().numpy().copy(), s1.cpu().numpy().copy()
    M2, s2 = sim.simulate(gb.GBS_CACHED)
    torch.cuda.synchronize()
    assert np.array_equal(M1, M2.cpu().numpy()) and np.array_equal(s1, s2.cpu().numpy())
    assert (st["n_rf_cached"], st["n_distinct_rf"], st["n_adc_direct"]) == (5, 1, 5), st
    assert st["ms_compose"] > 0 and st["ms_apply"] > 0 and st["ms_adc_direct"] > 0, st
    sim.close()


def test_cached_agrees_with_grouped_and_plain(gb):
    """Three implementations of the same discrete model on one mid-size case."""
    ph, seq = synth.workload("fse-small")
    Mc, sc, _ = run_gpu(gb, ph, seq, gb.GBS_CACHED)
    Mg, sg, _ = run_gpu(gb, ph, seq, gb.GBS_GROUPED)
    Mp, sp, _ = run_gpu(gb, ph, seq, gb.GBS_PLAIN)
    for name, M, s in (("grouped", Mg, sg), ("plain", Mp, sp)):
        dm, rel = errors(Mc, sc, M, s)
        say(f"[gpu] cached vs {name}: max|dM|={dm:.3e} rel_sig={rel:.3e}")
        assert dm <= DM_TOL and rel <= SIG_TOL
