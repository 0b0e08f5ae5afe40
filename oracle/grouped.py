"""Brute-force FP64 transcription of the grouped-isochromat method.

TEST INFRASTRUCTURE ONLY, for tiny phantoms (Python loops over groups and
steps).  It shares nothing with the GPU library and is pinned against the
plain oracle (``oracle.simulate``): the paper's grouped method re-associates
the same per-step products (Sec. 2.3), so both must agree to rounding.

The steps follow the paper in its order:

1. split the sequence into with-RF, with-ADC and relaxation subsequences and
   give each with-RF / with-ADC subsequence a gradient type: Gx-only,
   Gy-only, Gz-only (exactly one gradient axis nonzero over the whole block),
   no-grads (all zero) or unclassified (Sec. 2.1, Sec. 2.4, Sec. 3.1);
2. group the isochromats once per type by the key (r_a, T1, T2, dB0), or by
   (T1, T2, dB0) for no-grads (Sec. 2.4, Fig. 2);
3. a with-RF subsequence of a known type: the combined transition
   T = U_{N-1} ... U_1 U_0 (Eq. 7) is computed once per group and applied to
   every member (Sec. 2.3);
4. a with-ADC subsequence of a known type with B1 = 0:
   (i)  A_block(g, t0) = sum over members of Mxy (Eq. 9, one coil, S = 1);
   (ii) every sample A(t) = sum over groups of Eq. (10) evolved from
        A_block(g, t0) (Eq. 8);
   (iii) every member is moved to the block end by Eq. (4) and Eq. (5);
5. relaxation subsequences: Eq. (4) and Eq. (5) per isochromat;
6. anything else falls back to conventional per-isochromat stepping (Sec. 3.1).
"""
from __future__ import annotations

import numpy as np

GAMMA_BAR = 42.577478518e6  # Hz/T (proton), this module's own copy
TWO_PI = 2.0 * np.pi

RF, ADC, RELAX = 1, 2, 3
GX, GY, GZ, NOGRADS, UNCLASSIFIED = 0, 1, 2, 3, 4


def step_matrix(bx, by, bz, dt, t1, t2):
    """U = D R of Appendix A for one raster step (4x4, FP64)."""
    nb = np.sqrt(bx * bx + by * by + bz * bz)
    R = np.eye(4)
    if nb > 0:
        ux, uy, uz = bx / nb, by / nb, bz / nb
        th = -TWO_PI * GAMMA_BAR * nb * dt
        c, s = np.cos(th), np.sin(th)
        v = 1.0 - c
        R[:3, :3] = [[c + ux * ux * v, -uz * s + ux * uy * v, uy * s + ux * uz * v],
                     [uz * s + ux * uy * v, c + uy * uy * v, -ux * s + uy * uz * v],
                     [-uy * s + ux * uz * v, ux * s + uy * uz * v, c + uz * uz * v]]
    e1, e2 = np.exp(-dt / t1), np.exp(-dt / t2)
    D = np.array([[e2, 0, 0, 0], [0, e2, 0, 0], [0, 0, e1, 1 - e1], [0, 0, 0, 1.0]])
    return D @ R


def gradient_type(gx, gy, gz):
    active = [a for a, g in enumerate((gx, gy, gz)) if np.any(g != 0)]
    if not active:
        return NOGRADS
    if len(active) == 1:
        return active[0]
    return UNCLASSIFIED


def build_groups(ph):
    """Group ids per type: key (r_a, T1, T2, dB0) for a = x, y, z; (T1, T2, dB0) for no-grads."""
    coords = (ph.x, ph.y, ph.z)
    out = {}
    for t in (GX, GY, GZ, NOGRADS):
        keys = {}
        gid = np.empty(ph.K, np.int64)
        for k in range(ph.K):
            tissue = (float(ph.t1[k]), float(ph.t2[k]), float(ph.df[k]))
            key = tissue if t == NOGRADS else (float(coords[t][k]),) + tissue
            gid[k] = keys.setdefault(key, len(keys))
        members = [np.nonzero(gid == g)[0] for g in range(len(keys))]
        out[t] = (gid, members)
    return out


def _relax_closed_form(M, tau, m, x, y, z, df, t1, t2, m0):
    """Eq. (4) and Eq. (5) for arrays of isochromats, in place."""
    cycles = GAMMA_BAR * (m[0] * x + m[1] * y + m[2] * z) + df * tau
    phase = TWO_PI * (cycles - np.rint(cycles))
    mxy = (M[:, 0] + 1j * M[:, 1]) * np.exp(-tau / t2) * np.exp(-1j * phase)
    M[:, 0], M[:, 1] = mxy.real, mxy.imag
    M[:, 2] = m0 + (M[:, 2] - m0) * np.exp(-tau / t1)


def simulate_grouped(ph, seq, m_init=None, return_stats=False):
    """Grouped FP64 simulation; returns (M (3, K), sig complex) like oracle.simulate."""
    K = ph.K
    f = lambda a: np.asarray(a, dtype=np.float64)
    x, y, z, t1, t2, df, m0 = (f(a) for a in ph.arrays())
    coords = (x, y, z)
    M = np.zeros((K, 4))
    if m_init is None:
        M[:, 2] = m0
    else:
        M[:, :3] = np.asarray(m_init, dtype=np.float64).reshape(3, K).T
    M[:, 3] = m0
    groups = build_groups(ph)
    sig = np.zeros(seq.total_samples, np.complex128)
    dt = float(seq.dt)
    wf = [f(a) for a in (seq.rf_re, seq.rf_im, seq.gx, seq.gy, seq.gz)]
    stats = {"grouped_rf": 0, "grouped_adc": 0, "fallback": 0, "relax": 0}

    for b in range(seq.n_blocks):
        bt = int(seq.btype[b])
        if bt == RELAX:
            _relax_closed_form(M, float(seq.tau[b]), seq.moment[b], x, y, z, df, t1, t2, m0)
            stats["relax"] += 1
            continue
        s0, n = int(seq.step_offset[b]), int(seq.n_steps[b])
        sl = slice(s0, s0 + n)
        b1r, b1i, gx, gy, gz = (w[sl] for w in wf)
        g = (gx, gy, gz)
        gtype = gradient_type(gx, gy, gz)
        has_b1 = bool(np.any(b1r != 0) or np.any(b1i != 0))
        so, nsamp = int(seq.sample_offset[b]), int(seq.n_samples[b])
        sidx = np.asarray(seq.adc_idx[so:so + nsamp], dtype=np.int64)

        if bt == RF and gtype != UNCLASSIFIED:
            stats["grouped_rf"] += 1
            gid, members = groups[gtype]
            ga = np.zeros(n) if gtype == NOGRADS else g[gtype]
            for mem in members:
                k0 = mem[0]
                coord = 0.0 if gtype == NOGRADS else coords[gtype][k0]
                T = np.eye(4)
                for j in range(n):  # Eq. (7): later steps multiply from the left
                    bz = ga[j] * coord + df[k0] / GAMMA_BAR
                    T = step_matrix(b1r[j], b1i[j], bz, dt, t1[k0], t2[k0]) @ T
                M[mem] = M[mem] @ T.T
            continue

        if bt == ADC and not has_b1 and gtype != UNCLASSIFIED:
            stats["grouped_adc"] += 1
            gid, members = groups[gtype]
            ga = np.zeros(n) if gtype == NOGRADS else g[gtype]
            # moment of the active gradient from t0 to each raster boundary
            mom = np.concatenate([[0.0], np.cumsum(ga * dt)])
            for mem in members:
                k0 = mem[0]
                coord = 0.0 if gtype == NOGRADS else coords[gtype][k0]
                a_block = np.sum(M[mem, 0] + 1j * M[mem, 1])  # (i) Eq. (9)
                tau_n = sidx * dt
                cyc = GAMMA_BAR * coord * mom[sidx] + df[k0] * tau_n
                ph_n = TWO_PI * (cyc - np.rint(cyc))
                sig[so:so + nsamp] += np.exp(-tau_n / t2[k0]) * np.exp(-1j * ph_n) * a_block  # (ii)
            # (iii) Eq. (4), Eq. (5) to the block end, any gradient type
            m_blk = (np.sum(gx) * dt, np.sum(gy) * dt, np.sum(gz) * dt)
            _relax_closed_form(M, n * dt, m_blk, x, y, z, df, t1, t2, m0)
            continue

        # conventional per-isochromat stepping (unclassified, or RF and ADC together)
        stats["fallback"] += 1
        for k in range(K):
            nxt = 0
            for j in range(n + 1):
                while nxt < nsamp and sidx[nxt] == j:
                    sig[so + nxt] += M[k, 0] + 1j * M[k, 1]
                    nxt += 1
                if j == n:
                    break
                bz = gx[j] * x[k] + gy[j] * y[k] + gz[j] * z[k] + df[k] / GAMMA_BAR
                M[k] = step_matrix(b1r[j], b1i[j], bz, dt, t1[k], t2[k]) @ M[k]
    out = M[:, :3].T.copy()
    return (out, sig, stats) if return_stats else (out, sig)
