"""The FP64 oracle against closed forms, library routines and invariants.

CPU only.  The checks themselves live in oracle_pins.py so that the mutation
test can run them against deliberately broken copies of the oracle.
"""
import numpy as np
import pytest

import synth
from synth import SeqBuilder
from tests import oracle_pins as pins


@pytest.mark.parametrize("check", pins.CHECKS, ids=lambda c: c.__name__)
def test_pin(check, oracle_lib):
    check(oracle_lib.simulate)


# ----------------------------------------------------------------- grouped == plain
def _mini_sequences(dt=1e-6):
    """Small sequences that exercise every subsequence type the grouped
    method distinguishes (Sec. 2.4, Sec. 3.1)."""
    G = synth.GAMMA_BAR
    seqs = []
    # GRE-like: Gz-only RF, Gx-only ADC, mixed relaxation
    sb = SeqBuilder(dt, "mini-gre")
    b1 = synth.sinc_pulse(120, dt, np.deg2rad(40))
    for line in range(3):
        sb.rf(b1, (0, 0, 0.02))
        sb.relax(3e-4, (-1e-5, (line - 1) * 2e-6, -1.2e-6))
        sb.adc(40, (0.012, 0, 0), 4 * np.arange(10) + 2)
        sb.relax(2e-3, (3e-5, -(line - 1) * 2e-6, 4e-5))
    seqs.append(sb.build())
    # FSE-like: 90x / 180y with Gz, two echoes
    sb = SeqBuilder(dt, "mini-fse")
    sb.rf(synth.sinc_pulse(90, dt, np.pi / 2), (0, 0, 0.015))
    sb.relax(5e-4, (8e-6, 0, -6e-7))
    for e in range(2):
        sb.rf(synth.sinc_pulse(90, dt, np.pi, phase=np.pi / 2), (0, 0, 0.015))
        sb.relax(4e-4, (-2e-6, (e - 0.5) * 3e-6, 1e-5))
        sb.adc(32, (0.01, 0, 0), 4 * np.arange(8) + 2)
        sb.relax(4e-4, (0, -(e - 0.5) * 3e-6, 1e-5))
    seqs.append(sb.build())
    # EPI-like: Gx-only ADC with alternating sign, Gy blips
    sb = SeqBuilder(dt, "mini-epi")
    sb.rf(synth.sinc_pulse(100, dt, np.pi / 2), (0, 0, 0.015))
    sb.relax(3e-4, (-5e-6, -3e-6, -7e-7))
    for line in range(4):
        s = 1 if line % 2 == 0 else -1
        sb.relax(2e-5, (s * 1e-7, 0, 0))
        sb.adc(24, (s * 0.01, 0, 0), 3 * np.arange(8) + 1)
        sb.relax(2e-5, (s * 1e-7, 0, 0))
        sb.relax(1e-5, (0, 1.5e-6, 0))
    seqs.append(sb.build())
    # other types: Gx-only RF, Gy-only ADC with a ramp, no-grads RF,
    # mixed-gradient RF (fallback), ADC with RF (fallback), samples at 0 and n
    sb = SeqBuilder(dt, "mini-misc")
    sb.rf(synth.sinc_pulse(60, dt, 0.6), (0.01, 0, 0))
    sb.adc(30, (0, np.linspace(0, 0.02, 30), 0), [0, 7, 7, 30])
    sb.rf(np.full(20, 2e-6 + 1e-6j), (0, 0, 0))
    sb.rf(synth.sinc_pulse(40, dt, 0.5), (0.004, 0, 0.01))
    sb.adc(20, (0.01, 0, 0), [0, 5, 19], b1=np.full(20, 1e-6 + 0j))
    sb.adc(16, (0, 0, 0.01), [3, 16])
    sb.relax(1e-3, (1e-6, 2e-6, 3e-6))
    seqs.append(sb.build())
    return seqs


@pytest.mark.parametrize("seq", _mini_sequences(), ids=lambda s: s.name)
def test_grouped_equals_plain(seq, oracle_lib):
    """The grouped method re-associates the plain product exactly (Sec. 2.3):
    brute-force grouped FP64 == plain FP64 to rounding."""
    from oracle.grouped import simulate_grouped
    ph = synth.tiny_phantom(nx=5, ny=4, nz=3, n_classes=2, df_levels=2)
    Mp, sp = oracle_lib.simulate(ph, seq)
    Mg, sg, st = simulate_grouped(ph, seq, return_stats=True)
    assert np.max(np.abs(Mp - Mg)) < 1e-11
    assert np.linalg.norm(sp - sg) <= 1e-11 * max(np.linalg.norm(sp), 1.0)
    assert st["grouped_rf"] + st["grouped_adc"] > 0
    if seq.name == "mini-misc":
        assert st["fallback"] == 2


def test_groups_are_fewer_than_isochromats():
    from oracle.grouped import build_groups, GX, GZ
    ph = synth.tiny_phantom(nx=5, ny=4, nz=3, n_classes=2, df_levels=2)
    g = build_groups(ph)
    assert len(g[GX][1]) < ph.K and len(g[GZ][1]) < ph.K


# ----------------------------------------------------------------- invariants
def _small_case():
    ph = synth.gre_phantom(8, 6, 2, seed=77)
    seq = synth.gre_sequence(n_lines=3, n_read=8, dwell_steps=3, rf_steps=300, te=2e-3, tr=6e-3)
    return ph, seq


def test_permutation_invariance(oracle_lib):
    ph, seq = _small_case()
    perm = np.random.default_rng(1).permutation(ph.K)
    M, s = oracle_lib.simulate(ph, seq)
    Mp, sp = oracle_lib.simulate(ph.subset(perm), seq)
    assert np.array_equal(Mp, M[:, perm])
    assert np.allclose(sp, s, rtol=0, atol=1e-12 * np.abs(s).max())


def test_superposition(oracle_lib):
    ph, seq = _small_case()
    idx = np.arange(ph.K)
    a, b = idx[: ph.K // 3], idx[ph.K // 3:]
    _, s = oracle_lib.simulate(ph, seq)
    _, sa = oracle_lib.simulate(ph.subset(a), seq)
    _, sb = oracle_lib.simulate(ph.subset(b), seq)
    assert np.allclose(sa + sb, s, rtol=0, atol=1e-12 * np.abs(s).max())


def test_linearity_in_m0(oracle_lib):
    ph, seq = _small_case()
    ph2 = ph.subset(np.arange(ph.K))
    ph2.m0 = (ph.m0 * 2).astype(np.float32)
    M, s = oracle_lib.simulate(ph, seq)
    M2, s2 = oracle_lib.simulate(ph2, seq)
    assert np.allclose(M2, 2 * M, rtol=0, atol=1e-13)
    assert np.allclose(s2, 2 * s, rtol=0, atol=1e-12 * np.abs(s).max())


def test_magnitude_bounded_when_t2_le_t1(oracle_lib):
    ph, seq = _small_case()
    assert np.all(ph.t2 <= ph.t1)
    M, _ = oracle_lib.simulate(ph, seq)
    assert np.all(np.linalg.norm(M, axis=0) <= ph.m0.astype(np.float64) * (1 + 1e-12))


def test_thread_count_only_changes_rounding(oracle_lib):
    ph, seq = _small_case()
    M1, s1 = oracle_lib.simulate(ph, seq, nthreads=1)
    M3, s3 = oracle_lib.simulate(ph, seq, nthreads=3)
    assert np.array_equal(M1, M3)
    assert np.allclose(s1, s3, rtol=0, atol=1e-13 * np.abs(s1).max())


# ----------------------------------------------------------------- input checks
def test_rejects_invalid_inputs(oracle_lib):
    ph, seq = _small_case()
    bad = ph.subset(np.arange(ph.K))
    bad.t2 = bad.t2.copy()
    bad.t2[3] = 0.0
    with pytest.raises(ValueError):
        oracle_lib.simulate(bad, seq)
    bad.t2[3] = np.nan
    with pytest.raises(ValueError):
        oracle_lib.simulate(bad, seq)
    sb = SeqBuilder(1e-6)
    sb.adc(10, (0.01, 0, 0), [4, 2])  # samples out of time order
    with pytest.raises(ValueError):
        oracle_lib.simulate(ph, sb.build())


def test_gre_workload_runs(oracle_lib):
    """The 4096-isochromat GRE workload: finite output, echo peak at k = 0
    (the 32-point grid aliases k = -32/FOV onto k = 0, so column 0 peaks too)."""
    ph, seq = synth.workload("gre")
    assert ph.K == 4096 and seq.stepped_count() == 84480
    M, s = oracle_lib.simulate(ph, seq)
    assert np.all(np.isfinite(M)) and np.all(np.isfinite(s))
    ks = np.abs(s.reshape(32, 64))
    assert ks[16, 32] >= 0.95 * ks.max()
