"""Pins of the surrogate oracle's reference transition, written as checks of a
module so that the mutant tests can run them against altered copies.

Each check compares the module against something other than itself: scipy's
Rotation, the exact transition of the plain C oracle in cases where the
reference is exact by construction (on resonance, no RF, a centred hard
pulse), and the interpolation error bound of the table.
"""
import numpy as np

import synth


def _fse(m):
    pulse = synth.fse_refocusing_pulse()
    return pulse, m.reference_table(pulse), pulse[2] * len(pulse[0]) / 2


def check_quaternion(m):
    """Quaternion extraction and its inverse against scipy's Rotation (an
    independent implementation), including angles at and near 180 degrees."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(8)
    axes = rng.normal(size=(20, 3))
    axes /= np.linalg.norm(axes, axis=1, keepdims=True)
    angles = np.r_[np.full(10, np.pi), np.pi - 1e-6 * np.arange(10)]
    rots = list(Rotation.random(40, random_state=2)) + [Rotation.from_rotvec(a * t) for a, t in zip(axes, angles)]
    for r in rots:
        q = m.quaternion(r.as_matrix())
        x, y, z, w = r.as_quat()
        qs = np.array([w, x, y, z])
        assert min(np.abs(q - qs).max(), np.abs(q + qs).max()) < 1e-12
        assert np.abs(m.rotation_of(q[None])[0] - r.as_matrix()).max() < 1e-12


def check_on_resonance(m):
    """On resonance (f_z + f_B0 = 0) a pulse of constant phase is a rotation
    about one fixed axis by an angle proportional to its amplitude: the
    reference (table angle times the B1 scale) is exact for every B1 scale."""
    pulse, table, half = _fse(m)
    b1 = np.array([0.8, 0.93, 1.0, 1.17, 1.2])
    t = np.stack([[0.0, 300.0, -20.0, 0.0, 55.0], [0.0, -300.0, 20.0, 0.0, -55.0], np.full(5, np.inf),
                  np.full(5, np.inf), b1], 1)
    K = m.frame(m.transition(pulse, t), t, half)
    assert np.abs(m.reference(table, t, half) - K).max() < 1e-10


def check_between_grid(m):
    """B1 scale 1 without relaxation: exact up to the error of linear
    interpolation on the 0.78 Hz grid (measured 7e-7)."""
    pulse, table, half = _fse(m)
    f = np.random.default_rng(3).uniform(-1500, 1500, 200)
    t = np.stack([0.9 * f, 0.1 * f, np.full(200, np.inf), np.full(200, np.inf), np.ones(200)], 1)
    K = m.frame(m.transition(pulse, t), t, half)
    assert np.abs(m.reference(table, t, half) - K).max() < 5e-6


def check_zero_rf(m):
    """B1 = 0: the frame leaves relaxation alone, which the symmetric split
    reproduces exactly (A = diag(E2, E2, E1) over tau, b = (1 - E1) e_z)."""
    n, dt = 300, 1e-6
    pulse = (np.zeros(n, complex), np.full(n, 2.0 ** -9), dt)
    table = m.reference_table(pulse)
    t = np.array([[700.0, -40.0, 0.9, 0.07, 1.0], [-250.0, 90.0, 1.7, 0.2, 1.1], [1300.0, 100.0, 0.3, 0.031, 0.8]])
    K = m.frame(m.transition(pulse, t), t, n * dt / 2)
    assert np.abs(m.reference(table, t, n * dt / 2) - K).max() < 1e-10


def check_centred_hard_pulse(m):
    """A 90-degree hard pulse in the single middle raster step, on resonance:
    the transition is relaxation over the first half, the rotation,
    relaxation over the second half, which is the reference's split up to
    the relaxation inside that one step (dt / T2 = 2e-5)."""
    n, dt = 301, 1e-6
    rf = np.zeros(n, complex)
    rf[n // 2] = 0.25 / (synth.GAMMA_BAR * dt)
    pulse = (rf, np.full(n, 2.0 ** -9), dt)
    table = m.reference_table(pulse)
    t = np.array([[0.0, 0.0, 0.3, 0.05, 1.0], [40.0, -40.0, 0.8, 0.09, 1.0]])
    K = m.frame(m.transition(pulse, t), t, n * dt / 2)
    assert np.abs(m.reference(table, t, n * dt / 2) - K).max() < 1e-4


def check_round_trip(m):
    """Training targets and inference are inverse to each other: a network
    whose last layer outputs exactly the targets of a tuple (W4 = 0, b4 =
    targets) gives back that tuple's exact transition."""
    pulse, table, half = _fse(m)
    t = synth.surrogate_tuples(6, seed=12)
    T = m.transition(pulse, t)
    Y = m.targets(T, t, half, table)
    for k in range(len(t)):
        parts = m.unpack(synth.mlp_init_params(seed=1))
        parts[6][:] = 0.0
        parts[7][:] = Y[k]
        got = m.mlp_transition(m.pack(parts), t[k:k + 1], half, table)
        assert np.abs(got[0] - T[k]).max() < 1e-12


CHECKS = [check_quaternion, check_on_resonance, check_between_grid, check_zero_rf, check_centred_hard_pulse,
          check_round_trip]
