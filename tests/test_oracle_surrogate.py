"""Pins of the surrogate oracle (oracle/surrogate.py) against things other than
itself: torch autograd and torch.optim.Adam (independent implementations),
central finite differences, closed forms of the frame and of simple pulses,
and the affine property of the exact transition."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import surrogate as so
from tests import surrogate_pins as spins


@pytest.fixture(scope="module")
def small():
    rng = np.random.default_rng(5)
    p = synth.mlp_init_params(seed=3).astype(np.float64)
    tuples = synth.surrogate_tuples(40, seed=9)
    U = so.features(tuples)
    K = rng.uniform(-1, 1, (40, 12))
    return p, U, K


def test_bf16_rounding_ties_to_even():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -2.5, 1 + 2 ** -7 + 2 ** -9], np.float32)
    assert list(so.bf16(x)) == [1.0, 1.0, 1 + 2 ** -6, -2.5, 1 + 2 ** -7]


def test_loss_grad_matches_torch_autograd(small):
    p, U, K = small
    loss, g = so.loss_grad(p, U, K, round_weights=False)
    P = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    parts, o = [], 0
    for s in so.SHAPES:
        n = int(np.prod(s))
        parts.append(P[o:o + n].reshape(s))
        o += n
    W1, b1, W2, b2, W3, b3, W4, b4 = parts
    x = torch.tensor(U)
    h = torch.nn.functional.silu(torch.nn.functional.linear(x, W1, b1))
    h = torch.nn.functional.silu(torch.nn.functional.linear(h, W2, b2))
    h = torch.nn.functional.silu(torch.nn.functional.linear(h, W3, b3))
    y = torch.nn.functional.linear(h, W4, b4)
    lt = torch.nn.functional.mse_loss(y, torch.tensor(K))
    lt.backward()
    assert abs(loss - lt.item()) <= 1e-14 * abs(lt.item())
    np.testing.assert_allclose(g, P.grad.numpy(), rtol=1e-10, atol=1e-15)


def test_loss_grad_matches_central_differences(small):
    p, U, K = small
    _, g = so.loss_grad(p, U, K, round_weights=False)
    rng = np.random.default_rng(1)
    # a few coordinates from every layer
    offs = np.cumsum([0] + [int(np.prod(s)) for s in so.SHAPES])
    idx = np.concatenate([rng.integers(offs[i], offs[i + 1], 3) for i in range(8)])
    h = 1e-6
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (so.loss_grad(p + e, U, K, False)[0] - so.loss_grad(p - e, U, K, False)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-7 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(2)
    w = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    wt = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.Adam([wt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.normal(size=50)
        w, m, v = so.adam(w, m, v, g, t, 1e-2)
        wt.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(w, wt.detach().numpy(), rtol=0, atol=1e-12)


def test_adam_first_step_is_a_sign_step():
    g = np.array([3.0, -1e-3, 0.5])
    w, _, _ = so.adam(np.zeros(3), np.zeros(3), np.zeros(3), g, 1, 0.01, eps=1e-12)
    np.testing.assert_allclose(w, -0.01 * np.sign(g), rtol=1e-8)


def test_frame_round_trip_and_free_precession():
    rng = np.random.default_rng(4)
    tuples = synth.surrogate_tuples(6, seed=1)
    T = rng.normal(size=(6, 12))
    np.testing.assert_allclose(so.frame(so.frame(T, tuples, 1.5e-3), tuples, 1.5e-3, inverse=True), T,
                               atol=1e-12)
    # a pulse with B1 = 0 is free precession + relaxation: K is the relaxation alone
    n, dt = 300, 1e-6
    gz = np.full(n, 2.0 ** -9)  # exact in float32, so f_z is exact
    pulse = (np.zeros(n, complex), gz, dt)
    tup = np.array([[700.0, -40.0, 0.9, 0.07, 1.0], [-250.0, 90.0, 1.7, 0.2, 1.1]])
    T = so.transition(pulse, tup)
    K = so.frame(T, tup, n * dt / 2)
    for k, (_, _, t1, t2, _) in enumerate(tup):
        e1, e2 = np.exp(-n * dt / t1), np.exp(-n * dt / t2)
        want = np.array([e2, 0, 0, 0, e2, 0, 0, 0, e1, 0, 0, 1 - e1])
        np.testing.assert_allclose(K[k], want, atol=1e-9)


def test_transition_hard_pulse_and_affinity():
    n, dt = 250, 1e-6
    flip = np.pi / 2
    b1 = np.full(n, flip / (2 * np.pi * so.GAMMA_BAR * n * dt))
    pulse = (b1.astype(complex), np.full(n, 1e-3), dt)
    tup = np.array([[0.0, 0.0, 1e9, 1e9, 1.0]])  # on resonance, no relaxation
    T = so.transition(pulse, tup)[0]
    A = T[:9].reshape(3, 3)
    # hard 90 along x: +z -> +y; the bar is the float32 rounding of B1 (~1e-7 rad of flip)
    np.testing.assert_allclose(A @ [0, 0, 1], [0, 1, 0], atol=2e-7)
    np.testing.assert_allclose(A @ [1, 0, 0], [1, 0, 0], atol=2e-7)
    # affine: T applied to (M, M0) equals the oracle run from that state
    tup = np.array([[310.0, 25.0, 0.8, 0.05, 0.93]])
    rf, gz, dt = synth.fse_refocusing_pulse(rf_steps=600)
    T = so.transition((rf, gz, dt), tup)[0]
    sb = synth.SeqBuilder(dt, "p")
    sb.rf(0.93 * rf, (np.zeros(600), np.zeros(600), gz))
    z = 310.0 / (so.GAMMA_BAR * gz[0])
    ph = synth.Phantom(np.zeros(1), np.zeros(1), np.full(1, z), np.full(1, 0.8), np.full(1, 0.05),
                       np.full(1, 25.0), np.full(1, 0.7))
    m = np.array([[0.3], [-0.2], [0.5]])
    M, _ = oracle.simulate(ph, sb.build(), m_init=m)
    np.testing.assert_allclose(T[:9].reshape(3, 3) @ m[:, 0] + T[9:] * 0.7, M[:, 0], atol=1e-12)



def test_quaternion_matches_scipy_at_every_angle():
    spins.check_quaternion(so)


def test_reference_on_resonance_scales_the_angle_exactly():
    spins.check_on_resonance(so)


def test_reference_between_grid_points():
    spins.check_between_grid(so)


def test_reference_is_exact_without_rf():
    spins.check_zero_rf(so)


def test_reference_split_for_a_centred_hard_pulse():
    spins.check_centred_hard_pulse(so)


def test_targets_and_mlp_transition_round_trip():
    spins.check_round_trip(so)
