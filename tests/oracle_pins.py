"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each ``check_*`` takes ``sim`` (a callable with the signature of
``oracle.simulate``) and raises AssertionError when the oracle disagrees with
an *independent* expectation: a library routine (scipy rotations, matrix
exponentials, numpy matrix powers and FFTs), a closed form of the paper
(Eq. 4, Eq. 5) or a textbook special case (hard pulses, spin echoes).  The
same checks run against the real oracle (test_oracle_pins.py) and against
deliberately broken copies of it (test_oracle_mutants.py), which shows that
plausible mistakes are caught.
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import expm
from scipy.spatial.transform import Rotation

from synth import Phantom, SeqBuilder

GB = 42.577478518e6  # Hz/T, the test's own copy of gamma/2pi
TWO_PI = 2 * np.pi


def f32(v):
    """Value as the single-precision input both sides actually read."""
    return np.float64(np.float32(v))


def phantom(n, x=0.0, y=0.0, z=0.0, t1=np.inf, t2=np.inf, df=0.0, m0=1.0):
    vals = [np.broadcast_to(np.asarray(v, dtype=np.float64), (n,)) for v in (x, y, z, t1, t2, df, m0)]
    return Phantom(*(np.ascontiguousarray(v, dtype=np.float32) for v in vals))


def extract_affine(sim, seq, **iso):
    """Return the 4x4 homogeneous transition one isochromat sees over `seq`.

    Columns of the 3x3 block come from unit initial states with M0 = 0; the
    translation column from M = 0 with M0 = 1 (Eq. 2)."""
    ph = phantom(4, m0=[0.0, 0.0, 0.0, 1.0], **iso)
    m_init = np.zeros((3, 4))
    m_init[0, 0] = m_init[1, 1] = m_init[2, 2] = 1.0
    M, _ = sim(ph, seq, m_init=m_init)
    U = np.eye(4)
    U[:3, :3] = M[:, :3]
    U[:3, 3] = M[:, 3]
    return U


def skew(b):
    return np.array([[0, -b[2], b[1]], [b[2], 0, -b[0]], [-b[1], b[0], 0.0]])


def hom(R3):
    U = np.eye(4)
    U[:3, :3] = R3
    return U


def relax_generator(t1, t2):
    """Generator of the relaxation part of Eq. (1), decaying toward M0."""
    G = np.zeros((4, 4))
    G[0, 0] = G[1, 1] = -1.0 / t2
    G[2, 2] = -1.0 / t1
    G[2, 3] = 1.0 / t1
    return G


def one_step_seq(b1, g, dt=1e-6, n=1):
    sb = SeqBuilder(dt)
    sb.rf(np.full(n, b1, dtype=np.complex128), g)
    return sb.build()


# ---------------------------------------------------------------- checks
def check_rotation_matches_scipy(sim):
    """One step with no relaxation is the rotation solving dM/dt = gamma M x B
    over dt: compare with scipy's rotation-vector map and with expm."""
    rng = np.random.default_rng(11)
    dt = 1e-6
    for _ in range(4):
        b1 = complex(*rng.uniform(-2e-5, 2e-5, 2))
        gz, z, df = rng.uniform(-0.02, 0.02), rng.uniform(-0.05, 0.05), rng.uniform(-80, 80)
        U = extract_affine(sim, one_step_seq(b1, (0, 0, gz), dt), z=z, df=df)
        B = np.array([f32(b1.real), f32(b1.imag), f32(gz) * f32(z) + f32(df) / GB])
        nb = np.linalg.norm(B)
        theta = -TWO_PI * GB * nb * dt
        R_scipy = Rotation.from_rotvec(theta * B / nb).as_matrix()
        R_expm = expm(-TWO_PI * GB * skew(B) * dt)
        assert np.allclose(U[:3, :3], R_scipy, atol=1e-12, rtol=0), "rotation != scipy"
        assert np.allclose(U[:3, :3], R_expm, atol=1e-12, rtol=0), "rotation != expm(Bloch)"
        assert np.allclose(U[:3, 3], 0, atol=1e-15)


def check_relaxation_matches_expm(sim):
    """B = 0: one step is the exact relaxation propagator (Eq. A1)."""
    for t1, t2 in ((0.8, 0.05), (0.3, 0.3), (2.0, 0.02)):
        dt = 1e-3
        U = extract_affine(sim, one_step_seq(0.0, (0, 0, 0), dt), t1=t1, t2=t2)
        E = expm(relax_generator(f32(t1), f32(t2)) * dt)
        assert np.allclose(U, E, atol=1e-13, rtol=0), "relaxation step != expm"


def check_splitting_order(sim):
    """U = D R (rotation first, then relaxation), not R D (Appendix A)."""
    dt = 1e-6
    b1 = 3e-3  # about 0.8 rad per step
    t1, t2 = 1.0, 2e-5
    U = extract_affine(sim, one_step_seq(b1, (0, 0, 0), dt), t1=t1, t2=t2)
    B = np.array([f32(b1), 0.0, 0.0])
    R = hom(Rotation.from_rotvec(-TWO_PI * GB * dt * B).as_matrix())
    D = expm(relax_generator(f32(t1), f32(t2)) * dt)
    assert np.allclose(U, D @ R, atol=1e-13, rtol=0), "step != D R"
    assert not np.allclose(D @ R, R @ D, atol=1e-6), "test cannot tell the orders apart"


def check_rectangular_pulse_power(sim):
    """N equal steps compose to the N-th power of one step (Eq. 3, Eq. 7)."""
    it = dict(z=0.004, t1=0.9, t2=0.07, df=35.0)
    U1 = extract_affine(sim, one_step_seq(4e-6 + 2e-6j, (0, 0, 0.01)), **it)
    UN = extract_affine(sim, one_step_seq(4e-6 + 2e-6j, (0, 0, 0.01), n=500), **it)
    assert np.allclose(UN, np.linalg.matrix_power(U1, 500), atol=1e-11, rtol=0), "U^N mismatch"
    it_free = dict(z=0.004, df=35.0)
    UN = extract_affine(sim, one_step_seq(4e-6 + 2e-6j, (0, 0, 0.01), n=500), **it_free)
    B = np.array([f32(4e-6), f32(2e-6), f32(0.01) * f32(0.004) + f32(35.0) / GB])
    R = Rotation.from_rotvec(-TWO_PI * GB * 500e-6 * B).as_matrix()
    assert np.allclose(UN[:3, :3], R, atol=1e-11, rtol=0), "U^N != R(u, N theta)"


def check_hard_90_tips_to_plus_y(sim):
    """B1 along +x rotates +z toward +y (dM/dt = gamma M x B)."""
    dt = 1e-6
    b1 = 0.25 / (GB * dt)
    M, _ = sim(phantom(1, m0=0.8), one_step_seq(b1, (0, 0, 0), dt))
    a = TWO_PI * GB * f32(b1) * dt
    exp_ = f32(0.8) * np.array([0.0, np.sin(a), np.cos(a)])
    assert np.allclose(M[:, 0], exp_, atol=1e-14), f"hard 90: {M[:, 0]} vs {exp_}"


def check_sinc_flip_area(sim):
    """On resonance a real RF of any envelope rotates about x by gamma*sum(B1)*dt."""
    from synth import sinc_pulse
    dt = 1e-6
    b1 = sinc_pulse(3000, dt, np.deg2rad(73.0)).real.astype(np.float32).astype(np.float64)
    sb = SeqBuilder(dt)
    sb.rf(b1, (0, 0, 0))
    M, _ = sim(phantom(1, m0=1.0), sb.build())
    a = TWO_PI * GB * dt * np.sum(b1)
    assert np.allclose(M[:, 0], [0, np.sin(a), np.cos(a)], atol=1e-12), "sinc flip area"


def check_free_precession_closed_form(sim):
    """B1 = 0 stepping equals Eq. (4), Eq. (5) with the stepped field integral."""
    rng = np.random.default_rng(3)
    dt, n = 2e-6, 700
    gx, gy, gz = (rng.uniform(-0.03, 0.03, n).astype(np.float32) for _ in range(3))
    sb = SeqBuilder(dt)
    sb.adc(n, (gx, gy, gz), [])
    seq = sb.build()
    r = (0.031, -0.017, 0.006)
    t1, t2, df = 0.7, 0.04, -42.0
    m0 = 0.9
    ph = phantom(1, *r, t1=t1, t2=t2, df=df, m0=m0)
    mi = np.array([[0.3], [-0.5], [0.2]])
    M, _ = sim(ph, seq, m_init=mi)
    X, Y, Z = (f32(v) for v in r)
    bz = gx.astype(np.float64) * X + gy.astype(np.float64) * Y + gz.astype(np.float64) * Z + f32(df) / GB
    phase = TWO_PI * GB * np.sum(bz) * dt
    tau = n * dt
    mxy = (0.3 - 0.5j) * np.exp(-tau / f32(t2)) * np.exp(-1j * phase)
    mz = f32(m0) + (0.2 - f32(m0)) * np.exp(-tau / f32(t1))
    assert np.allclose(M[:, 0], [mxy.real, mxy.imag, mz], atol=1e-12), "free precession"


def check_relax_block_equals_stepping(sim):
    """A relaxation block (tau, moment) equals stepping the same B1 = 0 raster."""
    rng = np.random.default_rng(4)
    dt, n = 1e-6, 400
    g = [rng.uniform(-0.02, 0.02, n).astype(np.float32) for _ in range(3)]
    sb1 = SeqBuilder(dt)
    sb1.rf(np.full(n, 1e-5), (0, 0, 0))  # put the state off the z axis first
    sb1.adc(n, g, [])
    sb2 = SeqBuilder(dt)
    sb2.rf(np.full(n, 1e-5), (0, 0, 0))
    sb2.relax(n * dt, tuple(float(np.sum(gi.astype(np.float64)) * dt) for gi in g))
    ph = phantom(5, x=np.linspace(-0.05, 0.05, 5), y=np.linspace(0.04, -0.03, 5),
                 z=np.linspace(-0.01, 0.02, 5), t1=0.5, t2=0.06, df=np.linspace(-30, 30, 5))
    M1, _ = sim(ph, sb1.build())
    M2, _ = sim(ph, sb2.build())
    assert np.allclose(M1, M2, atol=1e-12), "relax block != stepped B1=0 block"


def check_spin_echo(sim):
    """90x - tau - 180y - tau refocuses off-resonance: echo = i sum M0 e^{-2tau/T2}."""
    dt = 1e-8
    b90 = 0.25 / (GB * dt)
    b180 = 0.5 / (GB * dt)
    tau = 0.02
    t2 = np.array([0.05, 0.08, 0.11, 0.05, 0.2])
    dfv = np.array([-50.0, -12.0, 0.0, 23.0, 50.0])
    m0 = np.array([1.0, 0.7, 0.9, 0.5, 0.6])
    ph = phantom(5, x=np.linspace(-0.1, 0.1, 5), t1=1.0, t2=t2, df=dfv, m0=m0)
    sb = SeqBuilder(dt)
    sb.rf([b90], (0, 0, 0))
    sb.relax(tau, (0.003, 0, 0))
    sb.rf([1j * b180], (0, 0, 0))
    sb.relax(tau, (0.003, 0, 0))
    sb.adc(0, (0, 0, 0), [0])
    _, sig = sim(ph, sb.build())
    t2f, m0f = t2.astype(np.float32).astype(np.float64), m0.astype(np.float32).astype(np.float64)
    a90 = TWO_PI * GB * f32(b90) * dt
    a180 = TWO_PI * GB * f32(b180) * dt
    expect = 1j * np.sum(m0f * np.sin(a90) * np.sin(a180 / 2) ** 2 * np.exp(-(2 * tau + 2 * dt) / t2f))
    assert abs(sig[0] - expect) < 1e-5 * abs(expect), f"spin echo {sig[0]} vs {expect}"


def check_dft_readout(sim):
    """Hard 90x then a Gx readout samples the 1D Fourier transform of M0 (Eq. 6):
    A(n) = i sin(a) sum_k M0_k exp(-2 pi i k_n x_k), k_n = (n - N/2)/FOV."""
    N, fov, dt = 32, 0.064, 1e-6
    xs = (np.arange(N) + 0.5) * fov / N - fov / 2
    rng = np.random.default_rng(9)
    m0 = rng.uniform(0.2, 1.0, N)
    ph = phantom(N, x=xs, m0=m0)
    g = 1.0 / (GB * dt * fov)
    b90 = 0.25 / (GB * dt)
    sb = SeqBuilder(dt)
    sb.rf([b90], (0, 0, 0))
    sb.relax(1e-3, (-g * (N // 2) * dt, 0, 0))
    sb.adc(N, (g, 0, 0), np.arange(N))
    _, sig = sim(ph, sb.build())
    a = TWO_PI * GB * f32(b90) * dt
    m = np.arange(N) - N // 2
    m0f = m0.astype(np.float32).astype(np.float64)
    # sum_i M0_i exp(-2 pi i m (i - N/2 + 1/2)/N) = (-1)^m exp(-i pi m / N) FFT(M0)[m]
    expect = 1j * np.sin(a) * ((-1.0) ** m) * np.exp(-1j * np.pi * m / N) * np.fft.fft(m0f)[m % N]
    err = np.max(np.abs(sig - expect)) / np.max(np.abs(expect))
    assert err < 1e-5, f"DFT readout mismatch {err}"


CHECKS = [check_rotation_matches_scipy, check_relaxation_matches_expm, check_splitting_order,
          check_rectangular_pulse_power, check_hard_90_tips_to_plus_y, check_sinc_flip_area,
          check_free_precession_closed_form, check_relax_block_equals_stepping, check_spin_echo,
          check_dft_readout]
