"""FP64 oracle of the learned RF-transition surrogate.

TEST INFRASTRUCTURE ONLY (tests, the smoke check and the benchmark's CPU leg):
nothing here is shared with or imported by the GPU library.

* ``transition`` -- the exact 3x4 affine transition T (Eq. 7: the product of
  the per-step U = D R of Eq. A1, A2) of one with-RF subsequence, for any
  parameter tuple, obtained from the plain C oracle by running the pulse on
  the basis states: A[:, j] is the final M for M = e_j with M0 = 0, and b is
  the final M for M = 0 with M0 = 1.
* ``frame`` -- K = P(-a) A P(-a), k_b = P(-a) b with P the z rotation of
  Eq. A2 and a = -2 pi (f_z + f_B0) tau / 2 (the pulse's free precession over
  each half removed), and its inverse.
* ``reference_table`` / ``reference`` -- the reference transition K_ref that
  the network corrects.  The table holds the relaxation-free transition of
  the pulse at B1 scale 1 in the frame above (a rotation) on a uniform grid
  of f = f_z + f_B0, as rotation angle theta(f) and unit axis n(f) (from its
  unit quaternion, signs chosen continuous along f).  K_ref for a tuple
  interpolates theta and n linearly in f, scales the angle by the B1 scale
  (exact on resonance for a pulse of constant phase) and splits the
  relaxation over the pulse symmetrically around the rotation:
  A_ref = D R D, b_ref = (1 - E1) (D R e_z + e_z), D = diag(E2, E2, E1) with
  E = exp(-(tau/2)/T).  With B1 = 0, K_ref is the exact transition.
* ``targets`` -- what the network is trained to output:
  RESIDUAL_SCALE * (K - K_ref).
* ``forward`` / ``loss_grad`` -- the 5-128-128-128-12 SiLU network and the
  gradient of its mean squared error by backpropagation, written out in FP64
  with the weights rounded to BF16 as the matrix cores see them.
* ``mlp_transition`` -- T from the network: K = K_ref + Y / RESIDUAL_SCALE,
  mapped back by the frame.
* ``adam`` -- one Adam step (Kingma and Ba, Algorithm 1).
"""
from __future__ import annotations

import numpy as np

import oracle
import synth

GAMMA_BAR = 42.577478518e6

# flat parameter layout: W1[128][5] b1[128] W2[128][128] b2[128] W3[128][128] b3[128] W4[12][128] b4[12]
SHAPES = [(128, 5), (128,), (128, 128), (128,), (128, 128), (128,), (12, 128), (12,)]
N_PARAMS = sum(int(np.prod(s)) for s in SHAPES)

REF_GRID = 4097        # points of the reference-rotation table
REF_FMAX = 1600.0      # the table spans f = f_z + f_B0 in [-REF_FMAX, REF_FMAX] Hz
RESIDUAL_SCALE = 8.0   # the network outputs RESIDUAL_SCALE * (K - K_ref)


def unpack(p):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(p[o:o + n], np.float64).reshape(s))
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(a, np.float64).ravel() for a in parts])


def bf16(x):
    """Round float32 values to BF16 (nearest, ties to even); returns float64."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def default_norm():
    """(center, scale) of the five features over the training ranges."""
    r = synth.SURROGATE_RANGES
    lo = np.array([r["f_z"][0], r["f_b0"][0], np.log(r["t1"][0]), np.log(r["t2"][0]), r["b1"][0]])
    hi = np.array([r["f_z"][1], r["f_b0"][1], np.log(r["t1"][1]), np.log(r["t2"][1]), r["b1"][1]])
    return 0.5 * (lo + hi), 0.5 * (hi - lo)


def features(tuples, norm=None):
    c, s = default_norm() if norm is None else norm
    t = np.asarray(tuples, np.float64)
    v = np.stack([t[:, 0], t[:, 1], np.log(t[:, 2]), np.log(t[:, 3]), t[:, 4]], 1)
    return (v - c) / s


def transition(pulse, tuples, lib=None):
    """Exact transitions (n, 12) (A row-major, then b) of ``pulse`` =
    (complex B1 per step, Gz per step, dt) for tuples (n, 5), via the C oracle.
    Tuples with the same B1 scale run in one oracle call (four isochromats
    per tuple: the three basis states with M0 = 0 and the zero state with
    M0 = 1)."""
    rf, gz, dt = pulse
    # the library holds the pulse in float32: B1 = s * float32(B1), Gz = float32(Gz),
    # and f_z refers to the peak |Gz| of those values
    rf = np.asarray(rf)
    re32 = rf.real.astype(np.float32).astype(np.float64)
    im32 = rf.imag.astype(np.float32).astype(np.float64)
    gz32 = np.asarray(gz, np.float32).astype(np.float64)
    g_ref = float(np.max(np.abs(gz32)))
    t = np.asarray(tuples, np.float64).reshape(-1, 5)
    out = np.empty((len(t), 12))
    for s1 in np.unique(t[:, 4]):
        sel = np.flatnonzero(t[:, 4] == s1)
        n = len(sel)
        sb = synth.SeqBuilder(dt, "pulse")
        sb.rf(np.zeros(len(rf)), (np.zeros(len(rf)), np.zeros(len(rf)), np.zeros(len(rf))))
        seq = sb.build()
        seq.rf_re, seq.rf_im, seq.gz = s1 * re32, s1 * im32, gz32.copy()  # FP64, no further rounding
        rep = lambda v: np.repeat(v, 4)
        z = t[sel, 0] / (GAMMA_BAR * g_ref)
        ph = synth.Phantom(np.zeros(4 * n), np.zeros(4 * n), rep(z), rep(t[sel, 2]), rep(t[sel, 3]),
                           rep(t[sel, 1]), np.tile([0.0, 0.0, 0.0, 1.0], n))
        m_init = np.zeros((3, 4 * n))
        m_init[0, 0::4] = m_init[1, 1::4] = m_init[2, 2::4] = 1.0
        M, _ = oracle.simulate(ph, seq, m_init=m_init, lib=lib)
        M = M.reshape(3, n, 4)
        out[sel, :9] = M[:, :, :3].transpose(1, 0, 2).reshape(n, 9)  # row i, column j = component i of image of e_j
        out[sel, 9:] = M[:, :, 3].T
    return out


def _pz(a):
    c, s = np.cos(a), np.sin(a)
    P = np.zeros((len(a), 3, 3))
    P[:, 0, 0] = c
    P[:, 0, 1] = -s
    P[:, 1, 0] = s
    P[:, 1, 1] = c
    P[:, 2, 2] = 1.0
    return P


def frame(T, tuples, half, inverse=False):
    """K = P(-a) A P(-a), k_b = P(-a) b (inverse: T = P(a) K P(a), P(a) k_b)."""
    t = np.asarray(tuples, np.float64)
    a = -2 * np.pi * (t[:, 0] + t[:, 1]) * half
    P = _pz(a if inverse else -a)
    T = np.asarray(T, np.float64)
    A = T[:, :9].reshape(-1, 3, 3)
    b = T[:, 9:]
    out = np.empty_like(T)
    out[:, :9] = (P @ A @ P).reshape(-1, 9)
    out[:, 9:] = np.einsum("nij,nj->ni", P, b)
    return out


def quaternion(R):
    """Unit quaternion (w, x, y, z) of a 3x3 rotation matrix, from its
    largest diagonal combination (numerically safe at every angle)."""
    R = np.asarray(R, np.float64)
    tr = R[0, 0] + R[1, 1] + R[2, 2]
    k = int(np.argmax([tr, R[0, 0], R[1, 1], R[2, 2]]))
    if k == 0:
        w = 0.5 * np.sqrt(1.0 + tr)
        q = [w, (R[2, 1] - R[1, 2]) / (4 * w), (R[0, 2] - R[2, 0]) / (4 * w), (R[1, 0] - R[0, 1]) / (4 * w)]
    elif k == 1:
        x = 0.5 * np.sqrt(1.0 + R[0, 0] - R[1, 1] - R[2, 2])
        q = [(R[2, 1] - R[1, 2]) / (4 * x), x, (R[0, 1] + R[1, 0]) / (4 * x), (R[0, 2] + R[2, 0]) / (4 * x)]
    elif k == 2:
        y = 0.5 * np.sqrt(1.0 - R[0, 0] + R[1, 1] - R[2, 2])
        q = [(R[0, 2] - R[2, 0]) / (4 * y), (R[0, 1] + R[1, 0]) / (4 * y), y, (R[1, 2] + R[2, 1]) / (4 * y)]
    else:
        z = 0.5 * np.sqrt(1.0 - R[0, 0] - R[1, 1] + R[2, 2])
        q = [(R[1, 0] - R[0, 1]) / (4 * z), (R[0, 2] + R[2, 0]) / (4 * z), (R[1, 2] + R[2, 1]) / (4 * z), z]
    return np.array(q)


def rotation_of(q):
    """3x3 rotation matrix of unit quaternions q (n, 4) = (w, x, y, z)."""
    w, x, y, z = (np.asarray(q, np.float64)[:, i] for i in range(4))
    R = np.empty((len(w), 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def reference_table(pulse, lib=None):
    """(f grid, theta, axis) of the relaxation-free B1-scale-1 transition of
    ``pulse`` in the frame, on REF_GRID points over [-REF_FMAX, REF_FMAX] Hz."""
    rf, gz, dt = pulse
    half = dt * len(rf) / 2
    fg = np.linspace(-REF_FMAX, REF_FMAX, REF_GRID)
    tg = np.stack([fg, np.zeros(REF_GRID), np.full(REF_GRID, np.inf), np.full(REF_GRID, np.inf),
                   np.ones(REF_GRID)], 1)
    K = frame(transition(pulse, tg, lib=lib), tg, half)
    q = np.array([quaternion(k[:9].reshape(3, 3)) for k in K])
    for j in range(1, REF_GRID):  # q and -q are the same rotation: keep the path continuous
        if np.dot(q[j], q[j - 1]) < 0:
            q[j] = -q[j]
    if q[0, 0] < 0:
        q = -q
    v = np.linalg.norm(q[:, 1:], axis=1)
    theta = 2 * np.arctan2(v, q[:, 0])
    axis = np.where(v[:, None] > 1e-300, q[:, 1:] / np.maximum(v, 1e-300)[:, None], np.array([0.0, 0.0, 1.0]))
    return fg, theta, axis


def reference(table, tuples, half):
    """K_ref (n, 12) of tuples (n, 5): interpolated rotation with its angle
    scaled by the B1 scale, relaxation split around it (see the header)."""
    fg, theta, axis = table
    t = np.asarray(tuples, np.float64).reshape(-1, 5)
    u = (t[:, 0] + t[:, 1] - fg[0]) / (fg[1] - fg[0])
    i0 = np.clip(np.floor(u).astype(np.int64), 0, len(fg) - 2)
    w = np.clip(u - i0, 0.0, 1.0)
    th = (1 - w) * theta[i0] + w * theta[i0 + 1]
    n = (1 - w)[:, None] * axis[i0] + w[:, None] * axis[i0 + 1]
    nn = np.linalg.norm(n, axis=1)
    n = np.where(nn[:, None] > 0, n / np.maximum(nn, 1e-300)[:, None], np.array([0.0, 0.0, 1.0]))
    h = 0.5 * t[:, 4] * th
    R = rotation_of(np.concatenate([np.cos(h)[:, None], np.sin(h)[:, None] * n], 1))
    e1, e2 = np.exp(-half / t[:, 2]), np.exp(-half / t[:, 3])
    d = np.stack([e2, e2, e1], 1)
    A = d[:, :, None] * R * d[:, None, :]
    b = (1 - e1)[:, None] * (d * R[:, :, 2])
    b[:, 2] += 1 - e1
    return np.concatenate([A.reshape(-1, 9), b], 1)


def targets(T, tuples, half, table):
    """Training targets of exact transitions T: RESIDUAL_SCALE * (K - K_ref)."""
    return RESIDUAL_SCALE * (frame(T, tuples, half) - reference(table, tuples, half))


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(params, U, round_weights=True):
    """Network outputs (n, 12) for features U (n, 5); returns (Y, cache)."""
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(params)
    if round_weights:
        W1, W2, W3, W4 = (bf16(w) for w in (W1, W2, W3, W4))
    Z1 = U @ W1.T + b1
    H1 = Z1 * _sig(Z1)
    Z2 = H1 @ W2.T + b2
    H2 = Z2 * _sig(Z2)
    Z3 = H2 @ W3.T + b3
    H3 = Z3 * _sig(Z3)
    Y = H3 @ W4.T + b4
    return Y, (U, Z1, H1, Z2, H2, Z3, H3, W2, W3, W4)


def _dsilu(z):
    s = _sig(z)
    return s * (1.0 + z * (1.0 - s))


def loss_grad(params, U, Ktarget, round_weights=True):
    """Mean over samples and the 12 outputs of (Y - K)^2, and its gradient
    with respect to the flat parameter vector."""
    Y, (U, Z1, H1, Z2, H2, Z3, H3, W2, W3, W4) = forward(params, U, round_weights)
    n = U.shape[0]
    R = Y - Ktarget
    loss = float(np.mean(R * R))
    dY = 2.0 * R / (12.0 * n)
    gW4, gb4 = dY.T @ H3, dY.sum(0)
    dZ3 = (dY @ W4) * _dsilu(Z3)
    gW3, gb3 = dZ3.T @ H2, dZ3.sum(0)
    dZ2 = (dZ3 @ W3) * _dsilu(Z2)
    gW2, gb2 = dZ2.T @ H1, dZ2.sum(0)
    dZ1 = (dZ2 @ W2) * _dsilu(Z1)
    gW1, gb1 = dZ1.T @ U, dZ1.sum(0)
    return loss, pack([gW1, gb1, gW2, gb2, gW3, gb3, gW4, gb4])


def adam(w, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step at step count t (1-based); returns (w, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def mlp_transition(params, tuples, half, table, norm=None):
    """The surrogate's T (n, 12): K = K_ref + Y / RESIDUAL_SCALE, mapped back
    by the frame."""
    Y, _ = forward(params, features(tuples, norm))
    return frame(reference(table, tuples, half) + Y / RESIDUAL_SCALE, tuples, half, inverse=True)
