"""A sequence read from a Pulseq file runs through the HIP path: a 2D
gradient echo described by Pulseq events (sinc RF under a slice trapezoid,
prephasers, a trapezoid readout with ADC, an arbitrary-gradient spoiler) on
the 32x32x4 GRE phantom, every mode against the FP64 oracle
(|dM| <= 1e-5, relative signal error <= 1e-4)."""
import numpy as np
import pytest

import oracle
import synth
from synth.pulseq import epi_text, gre_text, rf_during_adc_text

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_03960_amd as gb
    return gb


@pytest.fixture(scope="module")
def case():
    gb = _gpu()
    seq = gb.load_pulseq(gre_text())
    ph = synth.gre_phantom()
    M_ref, s_ref = oracle.simulate(ph, seq)
    return gb, seq, ph, M_ref, s_ref


def test_loaded_gre_takes_the_grouped_path(case):
    gb, seq, *_ = case
    p = gb.gbs_plan_summary(seq)
    assert p["rf_grouped"] == 4 and p["adc_grouped"] == 4 and p["fallback"] == 0, p


@pytest.mark.parametrize("mode", ["grouped", "plain", "cached"])
def test_loaded_gre_matches_oracle(case, mode):
    gb, seq, ph, M_ref, s_ref = case
    import torch
    print(f"[gpu] pulseq GRE, mode {mode}, K={ph.K}, steps={seq.total_steps}", flush=True)
    sim = gb.Simulator(0)
    try:
        sim.set_phantom(ph)
        if mode == "grouped":
            sim.build_groups()
        sim.set_sequence(seq)
        M, s = sim.simulate({"grouped": gb.GBS_GROUPED, "plain": gb.GBS_PLAIN, "cached": gb.GBS_CACHED}[mode])
        torch.cuda.synchronize()
        M, s = M.cpu().numpy().astype(np.float64), s.cpu().numpy()
    finally:
        sim.close()
    dm = float(np.abs(M - M_ref).max())
    rel = float(np.linalg.norm(s - s_ref) / np.linalg.norm(s_ref))
    print(f"[gpu] pulseq GRE {mode}: max|dM| {dm:.2e}, rel signal {rel:.2e}", flush=True)
    assert dm <= 1e-5 and rel <= 1e-4


@pytest.mark.parametrize("which", ["epi", "rf_during_adc"])
@pytest.mark.parametrize("mode", ["grouped", "plain", "cached"])
def test_more_loaded_sequences_match_oracle(which, mode):
    """EPI from Pulseq events (ramped readouts of both polarities, blips as
    relaxation blocks) and RF during an ADC (stepped per isochromat in every
    mode), against the oracle."""
    gb = _gpu()
    import torch
    seq = gb.load_pulseq({"epi": epi_text, "rf_during_adc": rf_during_adc_text}[which]())
    ph = synth.gre_phantom()
    M_ref, s_ref = oracle.simulate(ph, seq)
    print(f"[gpu] pulseq {which}, mode {mode}, steps={seq.total_steps}", flush=True)
    sim = gb.Simulator(0)
    try:
        sim.set_phantom(ph)
        if mode == "grouped":
            sim.build_groups()
        sim.set_sequence(seq)
        M, s = sim.simulate({"grouped": gb.GBS_GROUPED, "plain": gb.GBS_PLAIN, "cached": gb.GBS_CACHED}[mode])
        torch.cuda.synchronize()
        M, s = M.cpu().numpy().astype(np.float64), s.cpu().numpy()
    finally:
        sim.close()
    dm = float(np.abs(M - M_ref).max())
    rel = float(np.linalg.norm(s - s_ref) / np.linalg.norm(s_ref))
    print(f"[gpu] pulseq {which} {mode}: max|dM| {dm:.2e}, rel signal {rel:.2e}", flush=True)
    assert dm <= 1e-5 and rel <= 1e-4
