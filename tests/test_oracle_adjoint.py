"""Pins of the FP64 adjoint oracle (oracle/bloch_adjoint.c): central finite
differences of the plain forward oracle, a closed-form derivative of a hard
pulse, and the forward signal of the adjoint equal to the plain oracle."""
import numpy as np
import pytest

import oracle
import synth

GAMMA_BAR = 42.577478518e6


def with_params(seq, rf_param, param_blocks):
    """Copy of seq whose parameter blocks play rf_param (FP64, no rounding)."""
    s = synth.Sequence(**{f: getattr(seq, f) for f in seq.__dataclass_fields__})
    s.rf_re = np.asarray(seq.rf_re, np.float64).copy()
    s.rf_im = np.asarray(seq.rf_im, np.float64).copy()
    s.gx, s.gy, s.gz = (np.asarray(a, np.float64) for a in (seq.gx, seq.gy, seq.gz))
    for b in param_blocks:
        o, n = int(seq.step_offset[b]), int(seq.n_steps[b])
        s.rf_re[o:o + n] = rf_param.real
        s.rf_im[o:o + n] = rf_param.imag
    return s


def objective(ph, t1c, t2c, seq, rf, pb, w):
    p = synth.Phantom(ph.x, ph.y, ph.z, t1c[ph.labels], t2c[ph.labels], ph.df, ph.m0)
    _, sig = oracle.simulate(p, with_params(seq, rf, pb))
    return float(np.sum(w.real * sig.real + w.imag * sig.imag)), sig


@pytest.fixture(scope="module")
def tiny():
    ph, t1c, t2c, seq, rf, pb = synth.adjoint_workload(6, 5, 2, n_lines=2, n_read=12, rf_steps=240)
    rng = np.random.default_rng(8)
    rf = rf * (1 + 0.3j * rng.standard_normal(rf.size))  # make the pulse genuinely complex
    w = rng.standard_normal(seq.total_samples) + 1j * rng.standard_normal(seq.total_samples)
    return ph, t1c, t2c, seq, rf, pb, w


def test_adjoint_forward_equals_plain_oracle(tiny):
    ph, t1c, t2c, seq, rf, pb, w = tiny
    sig, *_ = oracle.adjoint(ph, ph.labels, t1c, t2c, seq, rf, pb, w)
    _, ref = objective(ph, t1c, t2c, seq, rf, pb, w)
    assert np.max(np.abs(sig - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_adjoint_matches_central_differences(tiny):
    ph, t1c, t2c, seq, rf, pb, w = tiny
    _, g_rf, g1, g2 = oracle.adjoint(ph, ph.labels, t1c, t2c, seq, rf, pb, w)
    rng = np.random.default_rng(3)
    # RF: two random directions and three single samples (real and imaginary parts)
    scale = np.max(np.abs(rf))
    dirs = [rng.standard_normal(rf.size) + 1j * rng.standard_normal(rf.size) for _ in range(2)]
    for j in (0, rf.size // 2, rf.size - 1):
        for unit in (1.0, 1j):
            d = np.zeros(rf.size, complex)
            d[j] = unit
            dirs.append(d)
    for d in dirs:
        h = 1e-4 * scale
        fp, _ = objective(ph, t1c, t2c, seq, rf + h * d, pb, w)
        fm, _ = objective(ph, t1c, t2c, seq, rf - h * d, pb, w)
        fd = (fp - fm) / (2 * h)
        an = float(np.sum(g_rf.real * d.real + g_rf.imag * d.imag))
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * np.sum(np.abs(g_rf))), (fd, an)
    # T1 and T2 of every class present
    for c in np.unique(ph.labels):
        for arr, g in ((t1c, g1), (t2c, g2)):
            h = 1e-4 * arr[c]  # the FP64 forward carries ~1e-13 relative noise; 1e-4 balances it against O(h^2)
            e = np.zeros_like(arr)
            e[c] = h
            a1, a2 = (t1c + e, t2c) if arr is t1c else (t1c, t2c + e)
            b1, b2 = (t1c - e, t2c) if arr is t1c else (t1c, t2c - e)
            fd = (objective(ph, a1, a2, seq, rf, pb, w)[0] - objective(ph, b1, b2, seq, rf, pb, w)[0]) / (2 * h)
            assert abs(fd - g[c]) <= 1e-6 * max(abs(g[c]), 1e-6), (c, fd, g[c])


def test_hard_pulse_derivative_closed_form():
    """On resonance, no relaxation: after a hard pulse of total area a along x
    the sample is A = i M0 sin(2 pi gamma_bar a dt); dIm(A)/dB1x_j =
    M0 cos(.) 2 pi gamma_bar dt for every step j; dA/dB1y = 0 (first order)."""
    n, dt = 100, 1e-6
    b1 = np.full(n, 0.7 * np.pi / 2 / (2 * np.pi * GAMMA_BAR * n * dt)) + 0j
    sb = synth.SeqBuilder(dt, "hard")
    sb.rf(b1, (0.0, 0.0, 1e-3))
    sb.adc(1, (0.0, 0.0, 0.0), [0])
    seq = sb.build()
    ph = synth.Phantom(np.zeros(1), np.zeros(1), np.zeros(1), np.ones(1), np.ones(1), np.zeros(1),
                       np.full(1, 0.8), labels=np.zeros(1, np.int32))
    sig, g_rf, _, _ = oracle.adjoint(ph, ph.labels, np.array([1e12]), np.array([1e12]), seq, b1, [0],
                                     np.array([1j]))
    theta = 2 * np.pi * GAMMA_BAR * b1.real.sum() * dt
    assert abs(sig[0] - 0.8j * np.sin(theta)) <= 1e-12
    np.testing.assert_allclose(g_rf.real, 0.8 * np.cos(theta) * 2 * np.pi * GAMMA_BAR * dt, rtol=1e-9)
    assert np.max(np.abs(g_rf.imag)) <= 1e-9 * np.max(np.abs(g_rf.real))
