"""Host-side checks of the C ABI: exported symbols, struct layouts, the
planner's classification, and input validation.  No GPU compute.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import synth
from synth import SeqBuilder

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gbloch.h")


@pytest.fixture(scope="module")
def gb():
    import paper_2508_03960_amd as gb
    return gb


def declared_functions():
    text = open(HEADER).read()
    return set(re.findall(r"^(?:int|const char \*|void)\s*\*?\s*(gbs_\w+)\s*\(", text, re.M))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("gbs_create", "gbs_destroy", "gbs_set_phantom", "gbs_set_sequence", "gbs_build_groups",
              "gbs_simulate"):
        assert f in names


def test_library_exports_every_declared_symbol(gb):
    out = subprocess.run(["nm", "-D", "--defined-only", gb.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT\s+(gbs_\w+)", out))
    missing = declared_functions() - exported
    assert not missing, missing
    assert set(gb.EXPORTED) == declared_functions()


def test_struct_layouts_match_c(gb, tmp_path):
    src = tmp_path / "sizes.c"
    src.write_text('#include "gbloch.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu\\n", sizeof(gbs_block), sizeof(gbs_info),'
                   ' sizeof(gbs_stats), offsetof(gbs_block, moment), offsetof(gbs_stats, pass_bytes));'
                   'return 0;}\n')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = list(map(int, subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()))
    assert got == [ctypes.sizeof(gb.gbs_block), ctypes.sizeof(gb.gbs_info), ctypes.sizeof(gb.gbs_stats),
                   gb.gbs_block.moment.offset, gb.gbs_stats.pass_bytes.offset]


def test_create_fails_cleanly_without_gpu(gb):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    assert gb.lib.gbs_create(ctypes.byref(h), 0, None) == gb.GBS_E_INVALID
    assert gb.lib.gbs_strerror(gb.GBS_E_STATE) == b"invalid call order or stale state"


# ------------------------------------------------------------ planner (Sec. 2.1, 2.4, 3.1)
def test_plan_fse(gb):
    s = gb.gbs_plan_summary(synth.fse_sequence())
    assert (s["rf_grouped"], s["adc_grouped"], s["fallback"], s["distinct_rf"]) == (272, 256, 0, 2)
    assert s["passes"] == 273 and s["emit_only"] == 0


def test_plan_epi(gb):
    s = gb.gbs_plan_summary(synth.epi_sequence())
    assert (s["rf_grouped"], s["adc_grouped"], s["fallback"], s["distinct_rf"]) == (1, 128, 0, 1)
    assert s["emit_only"] == 127 and s["passes"] == 129


def test_plan_gre(gb):
    s = gb.gbs_plan_summary(synth.gre_sequence())
    assert (s["rf_grouped"], s["adc_grouped"], s["distinct_rf"], s["passes"]) == (32, 32, 1, 33)


def _misc_seq(dt=1e-6):
    sb = SeqBuilder(dt, "misc")
    sb.rf(synth.sinc_pulse(60, dt, 0.6), (0.01, 0, 0))            # Gx-only RF
    sb.adc(30, (0, np.linspace(0, 0.02, 30), 0), [0, 7, 7, 30])   # Gy-only ADC
    sb.rf(np.full(20, 2e-6 + 1e-6j), (0, 0, 0))                   # no-grads RF
    sb.rf(synth.sinc_pulse(40, dt, 0.5), (0.004, 0, 0.01))         # mixed: fallback
    sb.adc(20, (0.01, 0, 0), [0, 5, 19], b1=np.full(20, 1e-6 + 0j))  # RF and ADC: fallback
    sb.rf(np.zeros(10), (0, 0, 0.01))                              # B1 = 0 RF block
    sb.relax(1e-3, (1e-6, 2e-6, 3e-6))
    return sb.build()


def test_plan_classification(gb):
    s = gb.gbs_plan_summary(_misc_seq(), axes=gb.GBS_AX_X | gb.GBS_AX_Y | gb.GBS_AX_Z)
    assert s["fallback"] == 2 and s["b1zero"] == 1
    assert s["rf_grouped"] == 2 and s["adc_grouped"] == 1
    # with two-axis groups the Gx+Gz RF block is grouped too; RF during ADC is still stepped
    s = gb.gbs_plan_summary(_misc_seq())
    assert s["fallback"] == 1 and s["rf_grouped"] == 3 and s["distinct_rf"] == 3
    # without y-groups the Gy-only readout is stepped per isochromat
    s = gb.gbs_plan_summary(_misc_seq(), axes=gb.GBS_AX_X | gb.GBS_AX_Z)
    assert s["fallback"] == 3 and s["adc_grouped"] == 0


def test_plan_no_grads_groups(gb):
    # GBS_AX_N changes where a no-grads transition is composed, not the counts
    a = gb.gbs_plan_summary(_misc_seq(), axes=gb.GBS_AX_X | gb.GBS_AX_Y | gb.GBS_AX_Z | gb.GBS_AX_N)
    b = gb.gbs_plan_summary(_misc_seq(), axes=gb.GBS_AX_X | gb.GBS_AX_Y | gb.GBS_AX_Z)
    assert a == b
    fs = synth.fse_sequence(n_shots=2, etl=2, n_read=16, fat_sat=True)
    s = gb.gbs_plan_summary(fs)
    assert (s["rf_grouped"], s["distinct_rf"], s["fallback"]) == (8, 3, 0)


def test_identical_rf_waveforms_share_one_transition(gb):
    sb = SeqBuilder(1e-6)
    b1 = synth.sinc_pulse(50, 1e-6, 1.0)
    for _ in range(5):
        sb.rf(b1, (0, 0, 0.01))
        sb.relax(1e-3)
    sb.rf(b1 * 0.5, (0, 0, 0.01))
    assert gb.gbs_plan_summary(sb.build())["distinct_rf"] == 2


# ------------------------------------------------ conventional method with caching (Sec. 2.2)
def test_cached_plan_fse(gb):
    # 16 x (90 + 16 x 180) RF blocks, two distinct waveforms composed once each;
    # 256 readouts of 256 samples, one direct-ADC launch each
    s = gb.gbs_plan_cached_summary(synth.fse_sequence())
    assert s == {"rf_cached": 272, "entries": 2, "adc_direct": 256, "adc_launches": 256, "fallback": 0,
                 "b1zero": 0}


def test_cached_plan_epi(gb):
    s = gb.gbs_plan_cached_summary(synth.epi_sequence())
    assert (s["rf_cached"], s["entries"], s["adc_direct"], s["fallback"]) == (1, 1, 128, 0)


def test_cached_plan_any_gradient(gb):
    # per-isochromat transitions need no grouping axis: the mixed-gradient RF
    # block is cached as well; only RF played during an ADC block is stepped
    s = gb.gbs_plan_cached_summary(_misc_seq())
    assert s == {"rf_cached": 3, "entries": 3, "adc_direct": 1, "adc_launches": 1, "fallback": 1, "b1zero": 1}


def test_cached_plan_splits_long_readouts(gb):
    sb = SeqBuilder(1e-6)
    sb.rf(synth.sinc_pulse(40, 1e-6, 0.5), (0, 0, 0.01))
    sb.adc(700, (0.01, 0, 0), np.arange(0, 700, 1))   # 700 samples: 3 launches
    sb.adc(10, (0.01, 0, 0), [])                      # no samples: no launch
    s = gb.gbs_plan_cached_summary(sb.build())
    assert (s["adc_direct"], s["adc_launches"]) == (2, 3)


def test_cached_plan_reuses_identical_waveforms(gb):
    sb = SeqBuilder(1e-6)
    b1 = synth.sinc_pulse(50, 1e-6, 1.0)
    for _ in range(5):
        sb.rf(b1, (0, 0, 0.01))
        sb.relax(1e-3)
    sb.rf(b1, (0, 0.01, 0))  # same B1, other gradient: its own entry
    s = gb.gbs_plan_cached_summary(sb.build())
    assert (s["rf_cached"], s["entries"]) == (6, 2)


@pytest.mark.parametrize("case", ["unsorted", "outside", "negative_tau", "rf_with_samples"])
def test_plan_rejects_bad_sequences(gb, case):
    sb = SeqBuilder(1e-6)
    sb.rf(np.full(4, 1e-6), (0, 0, 0))
    sb.adc(10, (0.01, 0, 0), [1, 2])
    seq = sb.build()
    if case == "unsorted":
        seq.adc_idx[:] = [5, 2]
    elif case == "outside":
        seq.adc_idx[1] = 11
    elif case == "negative_tau":
        seq.btype = np.append(seq.btype, 3).astype(np.int32)
        for f in ("step_offset", "n_steps", "sample_offset"):
            setattr(seq, f, np.append(getattr(seq, f), 0))
        seq.n_samples = np.append(seq.n_samples, 0).astype(np.int32)
        seq.tau = np.append(seq.tau, -1.0)
        seq.moment = np.vstack([seq.moment, [0, 0, 0]])
    elif case == "rf_with_samples":
        seq.n_samples[0] = 1
    with pytest.raises(gb.GbsError) as e:
        gb.gbs_plan_summary(seq)
    assert e.value.code == gb.GBS_E_INVALID
