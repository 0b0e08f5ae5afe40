"""Pulseq loader (gbs_pulseq_load): host logic, no GPU.

Expected rasters are worked out by hand from the event definitions of
Pulseq format 1.4 (each step holds the mean of the waveform over the step):
trapezoids, arbitrary gradients on the default timing, the compressed shape
form, ADC samples at the centres of their dwell intervals.  The loaded
sequences then go through the oracle for closed forms: the flip angle of a
block pulse and spin-echo refocusing of off-resonance (Sec. 2.1, Eq. 1-6).
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth
import paper_2508_03960_amd as gb
from synth.pulseq import SeqText, compress

GB = 42.577478518e6  # gamma / 2 pi (Hz/T), as the library states it

HEAD = """[VERSION]
major 1
minor 4
revision 1

[DEFINITIONS]
GradientRasterTime 1e-05
RadiofrequencyRasterTime 1e-06
AdcRasterTime 1e-07
BlockDurationRaster 1e-06
"""

# A: RF from a compressed shape; a trapezoid under an ADC; an arbitrary
# gradient in a relaxation block and under an ADC; a label-only block; RF
# during an ADC.
FIXTURE_A = HEAD + """
# NUM DUR RF GX GY GZ ADC EXT
[BLOCKS]
1 8 1 0 0 0 0 0
2 10 0 1 0 0 1 0
3 40 0 2 0 0 0 0
4 0 0 0 0 0 0 0
5 40 0 2 0 0 2 0
6 8 1 0 0 0 3 0

[RF]
1 1000 1 0 0 0 0 0

[TRAP]
1 1000 3 2 3 1

[GRADIENTS]
2 2000 0 0 2 0 0

[ADC]
1 2 4000 1 0 0
2 4 10000 0 0 0
3 1 2000 3 0 0

[SHAPES]

shape_id 1
num_samples 8
0
0.25
0.25
2
0
0
1

shape_id 2
num_samples 4
0
1
1
0
"""


def test_fixture_a_blocks_and_sizes():
    s = gb.load_pulseq(FIXTURE_A, dt=1e-6)
    assert s.n_blocks == 5  # the zero-duration block is dropped
    assert list(s.btype) == [gb.GBS_BLOCK_RF, gb.GBS_BLOCK_ADC, gb.GBS_BLOCK_RELAX, gb.GBS_BLOCK_ADC,
                             gb.GBS_BLOCK_ADC]
    assert list(s.n_steps) == [8, 10, 0, 40, 8]
    assert list(s.step_offset[[0, 1, 3, 4]]) == [0, 8, 18, 58]
    assert s.total_steps == 66 and s.total_samples == 7
    assert list(s.n_samples) == [0, 2, 0, 4, 1]
    assert list(s.sample_offset[[1, 3, 4]]) == [0, 2, 6]
    assert s.rasters == (1e-5, 1e-6, 1e-7, 1e-6)


def test_compressed_shape_decoding():
    # derivative 0, .25 x4, 0 x3 written as 0 | .25 .25 2 | 0 0 1; samples = running sum
    s = gb.load_pulseq(FIXTURE_A, dt=1e-6)
    np.testing.assert_allclose(s.rf_re[:8] * GB / 1000, [0, .25, .5, .75, 1, 1, 1, 1], rtol=0, atol=1e-6)
    assert not s.rf_im[:8].any()
    # RF during the ADC of block 6 keeps its waveform
    np.testing.assert_array_equal(s.rf_re[58:66], s.rf_re[:8])
    assert compress([0, .25, .5, .75, 1, 1, 1, 1]) == [0, .25, .25, 2, 0, 0, 1]


def test_trapezoid_step_means():
    # 1000 Hz/m, delay 1 us, rise 3, flat 2, fall 3 on a 1 us raster
    s = gb.load_pulseq(FIXTURE_A, dt=1e-6)
    want = np.array([0, 1 / 6, 1 / 2, 5 / 6, 1, 1, 5 / 6, 1 / 2, 1 / 6, 0])
    np.testing.assert_allclose(s.gx[8:18] * GB / 1000, want, rtol=0, atol=1e-6)
    assert not s.gy[8:18].any() and not s.gz[8:18].any()


def test_arbitrary_gradient_default_timing():
    # samples 0, 1, 1, 0 at 5, 15, 25, 35 us, first = last = 0 at 0 and 40 us
    s = gb.load_pulseq(FIXTURE_A, dt=1e-6)
    g = s.gx[18:58] * GB / 2000
    np.testing.assert_allclose(g[[4, 5, 10, 14, 15, 24, 25, 34, 35]],
                               [0, 0.05, 0.55, 0.95, 1, 1, 0.95, 0.05, 0], rtol=0, atol=1e-6)
    # relaxation block: tau = 40 us, moment = 2000 Hz/m * 20 us / gamma_bar
    assert s.tau[2] == pytest.approx(40e-6, rel=1e-12)
    np.testing.assert_allclose(s.moment[2], [2000 * 20e-6 / GB, 0, 0], rtol=1e-12)
    # the stepped copy carries the same moment
    assert g.sum() * 1e-6 == pytest.approx(20e-6, rel=1e-6)


def test_adc_sample_boundaries():
    s = gb.load_pulseq(FIXTURE_A, dt=1e-6)
    assert list(s.adc_idx) == [3, 7, 5, 15, 25, 35, 4]
    # dt = 2 us: the sample at 3 us lies inside a raster step
    with pytest.raises(gb.GbsError, match="raster boundary"):
        gb.load_pulseq(FIXTURE_A, dt=2e-6)


def test_adc_receiver_phase():
    t = SeqText(block_raster=1e-6)
    a = t.adc(3, 2000, 0, freq=100.0, phase=0.5)
    t.block(6, adc=a)
    s = gb.load_pulseq(t.text(), dt=1e-6)
    tj = (np.arange(3) + 0.5) * 2e-6
    np.testing.assert_allclose(s.adc_phase, 0.5 + 2 * np.pi * 100.0 * tj, rtol=1e-12)
    assert list(s.adc_idx) == [1, 3, 5]


def test_rf_phase_offset_and_phase_shape():
    t = SeqText(block_raster=1e-6)
    r1 = t.rf(500.0, [1, 1, 1, 1], phase_off=np.pi / 2)
    r2 = t.rf(500.0, [1, 1, 1, 1], phase=[0.5, 0.5, 0.5, 0.5])  # phase shape in cycles: pi
    r3 = t.rf(500.0, [1, 1], freq=1e5, delay_us=1)  # 100 kHz offset: 0.2 pi per 1 us sample
    t.block(4, rf=r1)
    t.block(4, rf=r2)
    t.block(4, rf=r3)
    s = gb.load_pulseq(t.text(), dt=1e-6)
    b = 500.0 / GB
    np.testing.assert_allclose(s.rf_im[:4], b, rtol=1e-6)
    np.testing.assert_allclose(s.rf_re[:4], 0, atol=1e-6 * b)
    np.testing.assert_allclose(s.rf_re[4:8], -b, rtol=1e-6)
    ph = 2 * np.pi * 1e5 * np.array([0.5e-6, 1.5e-6])
    np.testing.assert_allclose(s.rf_re[8:12], [0, b * np.cos(ph[0]), b * np.cos(ph[1]), 0], atol=1e-6 * b)
    np.testing.assert_allclose(s.rf_im[8:12], [0, b * np.sin(ph[0]), b * np.sin(ph[1]), 0], atol=1e-6 * b)


def test_coarse_raster_takes_exact_means():
    # a 10 us trapezoid sampled on dt = 5 us: means over [0, 5) and [5, 10)
    t = SeqText(block_raster=1e-6)
    g = t.trap(1000.0, 4, 2, 4)
    a = t.adc(1, 10000, 0)
    t.block(10, gx=g, adc=a)
    s = gb.load_pulseq(t.text(), dt=5e-6)
    # [0,4): area 2 us; [4,5): 1 us -> mean 3/5; symmetric second half
    np.testing.assert_allclose(s.gx * GB / 1000, [0.6, 0.6], rtol=1e-6)
    assert list(s.adc_idx) == [1]


def test_time_shaped_gradient():
    # extended trapezoid through (0, 0), (2 us, a), (6 us, a), (7 us, 0) on a 1 us gradient raster
    t = SeqText(grad_raster=1e-6, block_raster=1e-6)
    g = t.arb(1000.0, [0, 1, 1, 0], first=0, last=0, times=[0, 2, 6, 7])
    t.block(7, gz=g)
    a = t.adc(1, 6000, 0)
    t.block(7, gz=g, adc=a)
    s = gb.load_pulseq(t.text(), dt=1e-6)
    assert s.btype[0] == gb.GBS_BLOCK_RELAX
    np.testing.assert_allclose(s.moment[0], [0, 0, 1000 * 5.5e-6 / GB], rtol=1e-12)
    np.testing.assert_allclose(s.gz * GB / 1000, [0.25, 0.75, 1, 1, 1, 1, 0.5], atol=1e-6)


@pytest.mark.parametrize("bad,msg", [
    (FIXTURE_A.replace("minor 4", "minor 3"), "version"),
    (FIXTURE_A.replace("1 1000 1 0 0 0 0 0", "1 1000 7 0 0 0 0 0"), "missing shape"),
    (FIXTURE_A.replace("1 8 1 0 0 0 0 0", "1 6 1 0 0 0 0 0"), "RF outlasts"),
    (FIXTURE_A.replace("4 0 0 0 0 0 0 0", "4 0 0 1 0 0 0 0"), "zero duration"),
    (FIXTURE_A.replace("2 10 0 1 0 0 1 0", "2 8 0 1 0 0 1 0"), "outlasts the block"),
    (FIXTURE_A.replace("3 40 0 2 0 0 0 0", "3 40 0 2 0 0 0"), "columns"),
    (FIXTURE_A.replace("1 1000 1 0 0 0 0 0", "1 1000 1 0 3 0 0 0"), "time shape"),
    (FIXTURE_A.replace("num_samples 8", "num_samples 9"), "decodes to 8"),
    (FIXTURE_A.replace("0.25\n2\n", "0.25\nx\n"), "not a finite number"),
    (FIXTURE_A.replace("2 4 10000 0 0 0", "2 5 10000 0 0 0"), "outlast the block"),
])
def test_malformed_files_are_rejected(bad, msg):
    with pytest.raises(gb.GbsError, match=msg):
        gb.load_pulseq(bad, dt=1e-6)


def test_duration_off_the_raster():
    with pytest.raises(gb.GbsError, match="whole number of raster steps"):
        gb.load_pulseq(FIXTURE_A, dt=3e-6)


def test_fill_call_checks_capacity():
    text = FIXTURE_A.encode()
    sizes = (ctypes.c_int64 * 3)()
    err = ctypes.create_string_buffer(256)
    assert gb.lib.gbs_pulseq_load(text, len(text), 1e-6, sizes, *([None] * 9), err, 256) == gb.GBS_OK
    assert list(sizes) == [5, 66, 7]
    blocks = (gb.gbs_block * 5)()
    w = [np.zeros(66, np.float32) for _ in range(5)]
    adc = np.zeros(7, np.int32)
    sizes[1] = 65
    rc = gb.lib.gbs_pulseq_load(text, len(text), 1e-6, sizes, blocks, *(a.ctypes.data for a in w),
                                adc.ctypes.data, None, None, err, 256)
    assert rc == gb.GBS_E_INVALID and b"smaller" in err.value
    assert gb.lib.gbs_pulseq_load(None, 0, 1e-6, sizes, *([None] * 9), err, 256) == gb.GBS_E_INVALID


def test_default_dt_is_the_rf_raster():
    s = gb.load_pulseq(FIXTURE_A)
    assert s.dt == 1e-6 and s.total_steps == 66


def _one_spin(df=0.0, t2=1e9):
    one = np.ones(1, np.float32)
    z = np.zeros(1, np.float32)
    return synth.Phantom(x=z, y=z.copy(), z=z.copy(), t1=one * 1e9, t2=one * t2, df=z + df, m0=one)


@pytest.mark.parametrize("amp,mz", [(2500.0, 0.0), (5000.0, -1.0), (1250.0, np.cos(np.pi / 4))])
def test_block_pulse_flip_angle_through_the_oracle(amp, mz):
    # flip = 2 pi * amp * duration: 100 us at 2500 Hz is 90 degrees
    t = SeqText(block_raster=1e-6)
    r = t.rf(amp, np.ones(100))
    t.block(100, rf=r)
    s = gb.load_pulseq(t.text())
    assert len(t.shapes[0][1]) == 4  # 1 0 0 97: compressed
    M, _ = oracle.simulate(_one_spin(), s)
    assert M[2, 0] == pytest.approx(mz, abs=2e-6)
    assert np.hypot(M[0, 0], M[1, 0]) == pytest.approx(np.sqrt(1 - mz * mz), abs=2e-6)


def test_spin_echo_refocuses_off_resonance_through_the_oracle():
    """90x - TE/2 - 180y - TE/2: every off-resonance refocuses at TE, so the
    sample there is sum M0 exp(-TE/T2); samples 1 ms away are dephased."""
    t = SeqText(block_raster=1e-6)
    p90 = t.rf(25000.0, np.ones(10))
    p180 = t.rf(25000.0, np.ones(20), phase_off=np.pi / 2)
    te = 10e-3
    # centres: 90 at 5 us, 180 at 5 ms + 5 us (block 2 starts after 10 us + 4985 us)
    t.block(10, rf=p90)
    t.block(4985)
    t.block(20, rf=p180)
    # echo at 10.005 ms; ADC block starts at 5.015 ms: samples every 1 ms from 3.99 ms
    a = t.adc(3, 1e6, 3990 - 500)
    t.block(6000, adc=a)
    s = gb.load_pulseq(t.text())
    assert list(s.adc_idx) == [3990, 4990, 5990]
    df = np.linspace(-500.0, 500.0, 41)
    n = df.size
    ph = synth.Phantom(x=np.zeros(n, np.float32), y=np.zeros(n, np.float32), z=np.zeros(n, np.float32),
                       t1=np.full(n, 1e9, np.float32), t2=np.full(n, 0.08, np.float32),
                       df=df.astype(np.float32), m0=np.ones(n, np.float32))
    _, sig = oracle.simulate(ph, s)
    echo = abs(sig[1]) / n
    # the echo sample lies at 5.015 ms + 4.99 ms = 10.005 ms, the 90's centre plus TE
    assert echo == pytest.approx(np.exp(-te / 0.08), rel=2e-3)
    assert abs(sig[0]) / n < 0.2 and abs(sig[2]) / n < 0.2


@pytest.mark.parametrize("bad,msg", [
    (FIXTURE_A.replace("5 40 0 2 0 0 2 0", "5 300000000 0 2 0 0 2 0"), "longer than 2\\^28"),
    (FIXTURE_A.replace("2 4 10000 0 0 0", "2 2000000000 10000 0 0 0"), "outlast the block"),
    (FIXTURE_A.replace("0.25\n2\n", "0.25\n1000000000\n"), "more than num_samples"),
    (FIXTURE_A.replace("num_samples 8", "num_samples 99999999"), "outside \\[1, 2\\^26\\]"),
    (FIXTURE_A.replace("1 8 1 0 0 0 0 0", "1 99999999999 1 0 0 0 0 0"), "32-bit integer"),
    (FIXTURE_A.replace("1 1000 3 2 3 1", "1 1e300 3 2 3 1"), "float range"),
    (FIXTURE_A.replace("[RF]\n1 1000", "[RF]\n1 1e300"), "float range"),
])
def test_limits(bad, msg):
    with pytest.raises(gb.GbsError, match=msg):
        gb.load_pulseq(bad, dt=1e-6)


def test_mutated_files_fail_cleanly():
    """Seeded token, line and truncation mutations of valid files: every call
    returns a sequence or raises GbsError (the parser reads untrusted text)."""
    import random
    from synth.pulseq import gre_text
    rng = random.Random(11)
    bases = [FIXTURE_A, gre_text(n_lines=2, n_read=16)]
    vals = ["0", "-1", "1e300", "2147483648", "1e-300", "nan", "inf", "0.5", "3", "", "x", "[BLOCKS]",
            "shape_id", "num_samples", "268435457"]
    ok = 0
    for _ in range(400):
        lines = rng.choice(bases).split("\n")
        for _ in range(rng.randint(1, 5)):
            j, r = rng.randrange(len(lines)), rng.random()
            if r < 0.6:
                toks = lines[j].split(" ")
                toks[rng.randrange(len(toks))] = rng.choice(vals)
                lines[j] = " ".join(toks)
            elif r < 0.8:
                del lines[j]
            else:
                lines.insert(j, lines[rng.randrange(len(lines))])
        text = "\n".join(lines)
        if rng.random() < 0.1:
            text = text[:rng.randrange(len(text) + 1)]
        try:
            s = gb.load_pulseq(text.encode(), dt=rng.choice([None, 1e-6, 2e-6]))
            assert np.isfinite(s.rf_re).all() and np.isfinite(s.gx).all() and np.isfinite(s.moment).all()
            ok += 1
        except gb.GbsError:
            pass
    assert ok > 0


def test_relaxation_blocks_keep_their_exact_duration():
    # a 2000 s delay is no raster work; a 7.5 us one need not lie on the raster
    s = gb.load_pulseq(FIXTURE_A.replace("3 40 0 2 0 0 0 0", "3 2000000000 0 2 0 0 0 0"), dt=1e-6)
    assert s.tau[2] == pytest.approx(2000.0, rel=1e-15) and s.total_steps == 66
    t = SeqText(block_raster=0.5e-6)
    t.block(15)
    s = gb.load_pulseq(t.text(), dt=1e-6)
    assert s.n_blocks == 1 and s.tau[0] == pytest.approx(7.5e-6, rel=1e-12)


def test_paths_and_missing_version(tmp_path):
    f = tmp_path / "a.seq"
    f.write_text(FIXTURE_A)
    assert gb.load_pulseq(str(f)).total_steps == 66
    assert gb.load_pulseq(f).name == "a.seq"
    with pytest.raises(FileNotFoundError):
        gb.load_pulseq(str(tmp_path / "missing.seq"))
    with pytest.raises(gb.GbsError, match="no \\[VERSION\\]"):
        gb.load_pulseq(FIXTURE_A.replace("major 1\n", ""))
