"""Random tiny phantoms and block sequences for property tests (test helper).

Phantoms draw every key component from a few values, so isochromats collide
on the group keys (r_a, T1, T2, dB0) of every axis.  Sequences mix every
block kind the method distinguishes (Sec. 2.1, 2.4): with-RF blocks with Gx,
Gy or Gz only, without gradients, or with two gradients (stepped); with-ADC
blocks likewise, with RF during the ADC; relaxation blocks with moments.
Pure inputs: no arithmetic of the method.
"""
import numpy as np

import synth
from synth import SeqBuilder

KINDS = ("rf_x", "rf_y", "rf_z", "rf_none", "rf_xz", "adc_x", "adc_y", "adc_z", "adc_none", "adc_ramp",
         "adc_rf", "relax")


def phantom(rng, K):
    xs, ys, zs = rng.uniform(-0.01, 0.01, 3), rng.uniform(-0.01, 0.01, 3), rng.uniform(-0.002, 0.002, 2)
    t1s, t2s, dfs = np.array([0.4, 1.1]), np.array([0.03, 0.09]), np.array([-25.0, 0.0, 40.0])
    pick = lambda v: v[rng.integers(0, v.size, K)].astype(np.float32)
    return synth.Phantom(x=pick(xs), y=pick(ys), z=pick(zs), t1=pick(t1s), t2=pick(t2s), df=pick(dfs),
                         m0=rng.uniform(0.3, 1.0, K).astype(np.float32), name=f"random{K}")


def sequence(rng, kinds, dt=4e-6):
    sb = SeqBuilder(dt, "random")
    g = lambda: float(rng.uniform(-0.02, 0.02))
    for k in kinds:
        n = int(rng.integers(4, 40))
        b1 = synth.sinc_pulse(n, dt, float(rng.uniform(0.2, 2.5)), phase=float(rng.uniform(0, 6.28)))
        samples = np.sort(rng.integers(0, n + 1, int(rng.integers(0, 6))))
        if k == "rf_x":
            sb.rf(b1, (g(), 0, 0))
        elif k == "rf_y":
            sb.rf(b1, (0, g(), 0))
        elif k == "rf_z":
            sb.rf(b1, (0, 0, g()))
        elif k == "rf_none":
            sb.rf(b1)
        elif k == "rf_xz":
            sb.rf(b1, (g(), 0, g()))
        elif k == "adc_x":
            sb.adc(n, (g(), 0, 0), samples)
        elif k == "adc_y":
            sb.adc(n, (0, g(), 0), samples)
        elif k == "adc_z":
            sb.adc(n, (0, 0, g()), samples)
        elif k == "adc_none":
            sb.adc(n, (0, 0, 0), samples)
        elif k == "adc_ramp":
            sb.adc(n, (np.linspace(0, g(), n), 0, 0), samples)
        elif k == "adc_rf":
            sb.adc(n, (g(), 0, 0), samples, b1=b1 * 0.3)
        else:
            sb.relax(float(rng.uniform(0, 3e-3)), (g() * 1e-3, g() * 1e-3, g() * 1e-3))
    return sb.build()
