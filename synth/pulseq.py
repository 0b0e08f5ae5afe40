"""Writes the text of Pulseq 1.4 sequence files: deterministic workload
generators for the Pulseq loader (inputs only, none of the simulation's
arithmetic).

The sections and columns of format 1.4 ([VERSION],
[DEFINITIONS], [BLOCKS], [RF], [GRADIENTS], [TRAP], [ADC], [SHAPES]), and
shapes in the compressed form (the derivative, with a run of r >= 2 equal
values written as v, v, r - 2) or uncompressed.
"""
from __future__ import annotations


def compress(values):
    """Compressed form of a shape: run-length coded derivative."""
    d = [values[0]] + [values[i] - values[i - 1] for i in range(1, len(values))]
    out, i = [], 0
    while i < len(d):
        j = i
        while j + 1 < len(d) and d[j + 1] == d[i]:
            j += 1
        r = j - i + 1
        out += [d[i]] if r == 1 else [d[i], d[i], r - 2]
        i = j + 1
    return out


def _f(v):
    v = float(v)
    return str(int(v)) if v.is_integer() and abs(v) < 1e15 else repr(v)


class SeqText:
    def __init__(self, grad_raster=10e-6, rf_raster=1e-6, adc_raster=100e-9, block_raster=10e-6,
                 version=(1, 4, 1)):
        self.defs = dict(GradientRasterTime=grad_raster, RadiofrequencyRasterTime=rf_raster,
                         AdcRasterTime=adc_raster, BlockDurationRaster=block_raster)
        self.version = version
        self.blocks, self.rfs, self.grads, self.traps, self.adcs, self.shapes = [], [], [], [], [], []

    def shape(self, values, compressed=True):
        vals = [float(v) for v in values]
        c = compress(vals)
        # a list as long as num_samples is read as the samples themselves
        self.shapes.append((len(vals), c if compressed and len(c) < len(vals) else vals))
        return len(self.shapes)

    def rf(self, amp_hz, mag, phase=None, delay_us=0.0, freq=0.0, phase_off=0.0, time_id=0):
        m = self.shape(mag)
        p = self.shape(phase) if phase is not None else 0
        self.rfs.append((amp_hz, m, p, time_id, delay_us, freq, phase_off))
        return len(self.rfs)

    def trap(self, amp_hz_m, rise_us, flat_us, fall_us, delay_us=0.0):
        self.traps.append((amp_hz_m, rise_us, flat_us, fall_us, delay_us))
        return self._gid("t", len(self.traps))

    def arb(self, amp_hz_m, shape, first, last, delay_us=0.0, times=None):
        s = self.shape(shape)
        t = self.shape(times) if times is not None else 0
        self.grads.append((amp_hz_m, first, last, s, t, delay_us))
        return self._gid("g", len(self.grads))

    def adc(self, num, dwell_ns, delay_us, freq=0.0, phase=0.0):
        self.adcs.append((num, dwell_ns, delay_us, freq, phase))
        return len(self.adcs)

    def block(self, dur, rf=0, gx=0, gy=0, gz=0, adc=0):
        """dur in units of BlockDurationRaster; gradients are ids from trap()/arb()."""
        self.blocks.append((dur, rf, gx, gy, gz, adc))

    # gradient ids share one number space ([TRAP] and [GRADIENTS] rows)
    def _gid(self, kind, k):
        if not hasattr(self, "_ids"):
            self._ids = []
        self._ids.append((kind, k))
        return len(self._ids)

    def text(self):
        L = ["# Pulseq sequence file", "[VERSION]", f"major {self.version[0]}", f"minor {self.version[1]}",
             f"revision {self.version[2]}", "", "[DEFINITIONS]"]
        L += [f"{k} {_f(v)}" for k, v in self.defs.items()]
        L += ["", "# NUM DUR RF GX GY GZ ADC EXT", "[BLOCKS]"]
        L += [f"{i + 1} {d} {rf} {gx} {gy} {gz} {adc} 0" for i, (d, rf, gx, gy, gz, adc) in enumerate(self.blocks)]
        if self.rfs:
            L += ["", "# id amplitude mag_id phase_id time_shape_id delay freq phase", "[RF]"]
            L += [f"{i + 1} {_f(a)} {m} {p} {t} {_f(d)} {_f(f)} {_f(ph)}" for i, (a, m, p, t, d, f, ph) in enumerate(self.rfs)]
        ids = getattr(self, "_ids", [])
        g = [(n + 1, self.grads[k - 1]) for n, (kind, k) in enumerate(ids) if kind == "g"]
        t = [(n + 1, self.traps[k - 1]) for n, (kind, k) in enumerate(ids) if kind == "t"]
        if g:
            L += ["", "# id amplitude first last amp_shape_id time_shape_id delay", "[GRADIENTS]"]
            L += [f"{i} {_f(a)} {_f(fi)} {_f(la)} {s} {tt} {_f(d)}" for i, (a, fi, la, s, tt, d) in g]
        if t:
            L += ["", "# id amplitude rise flat fall delay", "[TRAP]"]
            L += [f"{i} {_f(a)} {_f(r)} {_f(fl)} {_f(fa)} {_f(d)}" for i, (a, r, fl, fa, d) in t]
        if self.adcs:
            L += ["", "# id num dwell delay freq phase", "[ADC]"]
            L += [f"{i + 1} {n} {_f(dw)} {_f(d)} {_f(f)} {_f(ph)}" for i, (n, dw, d, f, ph) in enumerate(self.adcs)]
        if self.shapes:
            L += ["", "[SHAPES]"]
            for i, (n, vals) in enumerate(self.shapes):
                L += ["", f"shape_id {i + 1}", f"num_samples {n}"] + [_f(v) for v in vals]
        return "\n".join(L) + "\n"


def gre_text(n_lines=4, n_read=32, flip_deg=30.0, thk=0.005, fov=0.2, te_fill=10, tr_fill=300):
    """A 2D gradient-echo sequence as Pulseq text: a Hamming-windowed sinc
    (time-bandwidth 4, 400 us) under a Gz trapezoid, prephasers and the phase
    encode in one block, a trapezoid readout with its ADC (10 us dwell), an
    arbitrary-gradient spoiler on z and a delay.  Block raster 10 us."""
    import numpy as np
    t = SeqText()
    n_rf = 400
    x = (np.arange(n_rf) + 0.5) / n_rf - 0.5
    env = np.sinc(4 * x) * (0.54 + 0.46 * np.cos(2 * np.pi * x))
    env = env / env.max()
    amp = np.deg2rad(flip_deg) / (2 * np.pi * env.sum() * 1e-6)
    rf = t.rf(amp, env, delay_us=100)
    gz_amp = (4 / 400e-6) / thk  # Hz/m: bandwidth / thickness
    gz = t.trap(gz_amp, 100, 400, 100)
    gz_reph = t.trap(-gz_amp * 250e-6 / 400e-6, 100, 300, 100)  # -(half flat + ramp) area over 400 us
    dk = 1.0 / fov
    gx_amp = n_read * dk / (n_read * 10e-6)  # Hz/m: one k-space step per dwell
    gx_read = t.trap(gx_amp, 100, n_read * 10, 100)
    gx_pre = t.trap(-gx_amp * (n_read * 10 / 2 + 55) / 400, 100, 300, 100)  # k = 0 at sample n/2
    spoil = t.arb(4e5, np.sin(np.linspace(0, np.pi, 30)) ** 2, 0, 0)
    adc = t.adc(n_read, 10000, 100)
    for line in range(n_lines):
        ky = (line - n_lines // 2) * dk
        gy = t.trap(ky / 400e-6, 100, 300, 100)
        t.block(60, rf=rf, gz=gz)
        t.block(50, gx=gx_pre, gy=gy, gz=gz_reph)
        t.block(te_fill)
        t.block(20 + n_read, gx=gx_read, adc=adc)
        t.block(30, gz=spoil)
        t.block(tr_fill)
    return t.text()


def epi_text(n_lines=8, n_read=32, fov=0.2, thk=0.005, dwell_us=10, ramp_us=50):
    """Single-shot EPI as Pulseq text: the sinc excitation under a slice
    trapezoid, prephasers, then n_lines readouts of alternating polarity
    (trapezoids with their ADC, one k-space step per dwell) separated by Gy
    blips.  A readout block lasts 2 ramp_us + n_read dwell_us, a whole number
    of 10 us block-raster units."""
    import numpy as np
    ro_us = 2 * ramp_us + n_read * dwell_us
    if ro_us % 10:
        raise ValueError("readout duration must be a multiple of the 10 us block raster")
    t = SeqText()
    n_rf = 400
    x = (np.arange(n_rf) + 0.5) / n_rf - 0.5
    env = np.sinc(4 * x) * (0.54 + 0.46 * np.cos(2 * np.pi * x))
    env = env / env.max()
    rf = t.rf(np.pi / 2 / (2 * np.pi * env.sum() * 1e-6), env, delay_us=100)
    gz_amp = (4 / 400e-6) / thk
    gz = t.trap(gz_amp, 100, 400, 100)
    gz_reph = t.trap(-gz_amp * 250e-6 / 400e-6, 100, 300, 100)
    dk = 1.0 / fov
    g_read = dk / (dwell_us * 1e-6)
    ro = [t.trap(s * g_read, ramp_us, n_read * dwell_us, ramp_us) for s in (1, -1)]
    # k = 0 at sample n_read / 2 of the first readout
    gx_pre = t.trap(-g_read * (n_read * dwell_us / 2 + ramp_us / 2 + dwell_us / 2) / 400, 100, 300, 100)
    gy_pre = t.trap(-(n_lines // 2) * dk / 400e-6, 100, 300, 100)
    blip = t.trap(dk / 20e-6, 10, 10, 10)
    adc = t.adc(n_read, dwell_us * 1000, ramp_us)
    t.block(60, rf=rf, gz=gz)
    t.block(50, gx=gx_pre, gy=gy_pre, gz=gz_reph)
    for line in range(n_lines):
        t.block(ro_us // 10, gx=ro[line % 2], adc=adc)
        if line + 1 < n_lines:
            t.block(3, gy=blip)
    t.block(100)
    return t.text()


def rf_during_adc_text(n=200):
    """A hard 30 degree pulse, then an ADC block that also plays weak RF
    (a constant 50 Hz B1) under a readout gradient: RF during ADC."""
    import numpy as np
    t = SeqText()
    p30 = t.rf(np.deg2rad(30) / (2 * np.pi * 100e-6), np.ones(100))
    weak = t.rf(50.0, np.ones(n * 10), phase_off=0.3)
    g = t.trap(2e5, 50, n * 10 - 100, 50)
    adc = t.adc(n, 10000, 0)
    t.block(10, rf=p30)
    t.block(n, rf=weak, gx=g, adc=adc)
    t.block(200)
    return t.text()
