"""Pins of the oracle's multi-coil signal, Eq. (6) with P receive coils:
A(p, t_n) = sum_k S(k, p) Mxy(k, t_n).  The per-coil sums are built from
single-isochromat runs, so they are pinned against the oracle's own
all-isochromat sum (superposition) and against closed statements about S."""
import numpy as np
import pytest

import oracle
import synth


@pytest.fixture(scope="module")
def case():
    ph = synth.tiny_phantom(nx=5, ny=4, nz=2, n_classes=2, df_levels=2)
    seq = synth.gre_sequence(n_lines=2, n_read=8, dwell_steps=2, rf_steps=200, te=1.5e-3, tr=4e-3)
    return ph, seq, oracle.simulate(ph, seq)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_unit_sensitivity_is_the_single_coil_signal(case):
    ph, seq, (M, s) = case
    Mc, sc = oracle.simulate_coils(ph, seq, np.ones((1, ph.K)))
    assert np.max(np.abs(Mc - M)) <= 1e-12
    assert rel(sc[0], s) <= 1e-12


def test_indicator_coils_split_the_phantom(case):
    ph, seq, (_, s) = case
    inside = np.arange(ph.K) % 3 == 0
    S = np.stack([inside, ~inside]).astype(np.complex128)
    _, sc = oracle.simulate_coils(ph, seq, S)
    _, s_in = oracle.simulate(ph.subset(np.nonzero(inside)[0]), seq)
    assert rel(sc[0], s_in) <= 1e-12
    assert rel(sc[0] + sc[1], s) <= 1e-12


def test_constant_and_phase_sensitivities(case):
    ph, seq, (_, s) = case
    c = 0.7 * np.exp(1j * 0.9)
    _, sc = oracle.simulate_coils(ph, seq, np.full((1, ph.K), c))
    assert rel(sc[0], c * s) <= 1e-12


def test_linear_in_the_sensitivity(case):
    ph, seq, _ = case
    rng = np.random.default_rng(3)
    S1 = rng.normal(size=ph.K) + 1j * rng.normal(size=ph.K)
    S2 = rng.normal(size=ph.K) + 1j * rng.normal(size=ph.K)
    _, sc = oracle.simulate_coils(ph, seq, np.stack([S1, S2, S1 + 2 * S2]))
    assert rel(sc[2], sc[0] + 2 * sc[1]) <= 1e-12
