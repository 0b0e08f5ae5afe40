"""Seeded synthetic phantoms and pulse sequences.

This module only *constructs inputs*: isochromat parameter maps and block
sequences (RF, ADC and relaxation subsequences, Sec. 2.1 and Fig. 1 of the
paper).  It holds none of the simulation arithmetic.  Both the FP64 CPU oracle
and the GPU library read the arrays built here, so every constant below only
has to be fixed and shared; none of them affects parity.

Layout conventions (shared interface, not arithmetic):

* phantom arrays are float32 SoA of length K, grid order z-major, then y, with
  x fastest: ``k = (iz*ny + iy)*nx + ix``;
* a sequence is a list of blocks over a uniform raster ``dt``; RF and ADC
  blocks carry per-step waveforms (B1 = rf_re + i rf_im in T, gradients in
  T/m); relaxation blocks carry only a duration and a gradient moment
  (integral of G dt, T*s/m);
* ADC sample n of a block is taken at a raster boundary ``adc_idx`` counted
  from the block start (0 = before the first step, n_steps = after the last).
  Generators place it at the centre of its dwell: ``dwell*n + dwell//2``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

# Proton gyromagnetic ratio / 2pi in Hz/T (CODATA 2018).  Used here only to
# calibrate flip angles and gradient strengths of the generated sequences.
GAMMA_BAR = 42.577478518e6

BLOCK_RF, BLOCK_ADC, BLOCK_RELAX = 1, 2, 3


# --------------------------------------------------------------------------
# phantoms
# --------------------------------------------------------------------------
@dataclass
class Phantom:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    t1: np.ndarray
    t2: np.ndarray
    df: np.ndarray  # off-resonance in Hz
    m0: np.ndarray
    shape: tuple | None = None  # (nz, ny, nx) for grid phantoms
    name: str = ""
    labels: np.ndarray | None = None  # tissue class per isochromat (int32), when known

    @property
    def K(self) -> int:
        return int(self.x.shape[0])

    def arrays(self):
        return (self.x, self.y, self.z, self.t1, self.t2, self.df, self.m0)

    def subset(self, idx: np.ndarray, name: str | None = None) -> "Phantom":
        idx = np.asarray(idx)
        return Phantom(*(a[idx].copy() for a in self.arrays()), shape=None,
                       name=name or (self.name + f"[{idx.size}]"),
                       labels=None if self.labels is None else self.labels[idx].copy())


def _grid(n, extent):
    return ((np.arange(n, dtype=np.float64) + 0.5) * extent / n - extent / 2)


def ellipse_phantom(nx, ny, nz, fov, t1s, t2s, pds, df_range, df_levels,
                    n_ellipses=12, seed=1000, name="ellipses"):
    """Tissue classes on seeded ellipses, replicated over z; quantized B0 map.

    ``fov`` = (fx, fy, fz) in metres (cell-centred grid).  Class 0 fills the
    background; each ellipse, drawn in turn, overwrites with a class in
    1..C-1.  The off-resonance map is a seeded low-order polynomial in the
    normalised coordinates, scaled to +-df_range Hz and snapped to the
    nearest of ``df_levels`` evenly spaced levels.
    """
    rng = np.random.default_rng(seed)
    fx, fy, fz = fov
    xs, ys, zs = _grid(nx, fx), _grid(ny, fy), _grid(nz, fz)
    C = len(t1s)
    X2, Y2 = np.meshgrid(xs, ys, indexing="xy")  # (ny, nx)
    cls = np.zeros((ny, nx), dtype=np.int32)
    for _ in range(n_ellipses):
        cx, cy = rng.uniform(-0.35, 0.35, 2) * np.array([fx, fy])
        ax, ay = rng.uniform(0.05, 0.30, 2) * np.array([fx, fy])
        ang = rng.uniform(0.0, np.pi)
        c = int(rng.integers(1, C)) if C > 1 else 0
        dx, dy = X2 - cx, Y2 - cy
        u = (dx * np.cos(ang) + dy * np.sin(ang)) / ax
        v = (-dx * np.sin(ang) + dy * np.cos(ang)) / ay
        cls[u * u + v * v <= 1.0] = c
    coef = rng.standard_normal(6)
    xh = X2 / (fx / 2)
    yh = Y2 / (fy / 2)
    base2d = coef[0] + coef[1] * xh + coef[2] * yh + coef[3] * xh * yh + coef[4] * (xh * xh - yh * yh)
    zh = zs / (fz / 2) if fz > 0 else np.zeros_like(zs)
    fieldmap = base2d[None, :, :] + coef[5] * zh[:, None, None]  # (nz, ny, nx)
    mx = np.abs(fieldmap).max()
    fieldmap = fieldmap * (df_range / mx if mx > 0 else 0.0)
    if df_levels > 1:
        step = 2.0 * df_range / (df_levels - 1)
        q = np.clip(np.rint((fieldmap + df_range) / step), 0, df_levels - 1)
        levels = np.linspace(-df_range, df_range, df_levels)
        df = levels[q.astype(np.int64)]
    else:
        df = np.zeros_like(fieldmap)
    t1 = np.asarray(t1s, dtype=np.float64)[cls]
    t2 = np.asarray(t2s, dtype=np.float64)[cls]
    pd = np.asarray(pds, dtype=np.float64)[cls]
    shp = (nz, ny, nx)
    Z = np.broadcast_to(zs[:, None, None], shp)
    Y = np.broadcast_to(ys[None, :, None], shp)
    X = np.broadcast_to(xs[None, None, :], shp)
    f32 = lambda a: np.ascontiguousarray(np.broadcast_to(a, shp), dtype=np.float32).ravel()
    labels = np.ascontiguousarray(np.broadcast_to(cls[None], shp), dtype=np.int32).ravel()
    return Phantom(f32(X), f32(Y), f32(Z), f32(t1[None]), f32(t2[None]), f32(df),
                   f32(pd[None]), shape=shp, name=name, labels=labels)


def gre_phantom(nx=32, ny=32, nz=4, seed=1000):
    """2D GRE oracle workload: 32x32x4 over 200x200x5 mm, 4 classes, 8 B0 levels in +-50 Hz."""
    return ellipse_phantom(nx, ny, nz, (0.200, 0.200, 0.005),
                           t1s=(0.300, 0.800, 1.200, 2.000),
                           t2s=(0.040, 0.080, 0.120, 0.250),
                           pds=(0.6, 0.8, 0.9, 1.0),
                           df_range=50.0, df_levels=8, seed=seed, name=f"gre{nx}x{ny}x{nz}")


SIX_T1 = tuple(np.geomspace(0.250, 2.500, 6))
SIX_T2 = tuple(np.geomspace(0.030, 0.300, 6))
SIX_PD = (0.70, 0.75, 0.80, 0.85, 0.90, 1.00)


def brain_like_phantom(nx=1024, ny=1024, nz=26, seed=1001):
    """FSE/EPI phantom: 6 classes (T1 250-2500 ms, T2 30-300 ms, log-spaced,
    paired), 16 B0 levels in +-100 Hz; FOV 256x256 mm in-plane, z over +-10 mm."""
    return ellipse_phantom(nx, ny, nz, (0.256, 0.256, 0.020), SIX_T1, SIX_T2, SIX_PD,
                           df_range=100.0, df_levels=16, seed=seed,
                           name=f"six-class {nx}x{ny}x{nz}")


def tiny_phantom(nx=4, ny=3, nz=2, n_classes=2, df_levels=2, seed=5, fov=(0.02, 0.02, 0.004)):
    """Small grid with many equal keys, for grouped-vs-plain brute force."""
    rng = np.random.default_rng(seed)
    t1s = tuple(rng.uniform(0.2, 1.5, n_classes))
    t2s = tuple(rng.uniform(0.02, 0.15, n_classes))
    pds = tuple(rng.uniform(0.5, 1.0, n_classes))
    return ellipse_phantom(nx, ny, nz, fov, t1s, t2s, pds, df_range=30.0,
                           df_levels=df_levels, n_ellipses=3, seed=seed, name="tiny")


def random_subset_indices(K, n, seed=7):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(K, size=n, replace=False)).astype(np.int64)


def coil_maps(ph: "Phantom", n_coils: int, radius=0.16, width=0.12, seed=31) -> np.ndarray:
    """Receive-coil sensitivities S(k, p), complex (n_coils, K): coils on a
    circle of `radius` (m) around the z axis, Gaussian magnitude of `width`
    (m) about each coil's centre and a seeded constant phase per coil."""
    rng = np.random.default_rng(seed)
    ang = 2 * np.pi * np.arange(n_coils) / n_coils
    phase = rng.uniform(-np.pi, np.pi, n_coils)
    x, y = ph.x.astype(np.float64), ph.y.astype(np.float64)
    d2 = (x[None, :] - radius * np.cos(ang)[:, None]) ** 2 + (y[None, :] - radius * np.sin(ang)[:, None]) ** 2
    return np.exp(-d2 / (2 * width ** 2)) * np.exp(1j * phase)[:, None]


# --------------------------------------------------------------------------
# sequences
# --------------------------------------------------------------------------
@dataclass
class Sequence:
    dt: float
    btype: np.ndarray
    step_offset: np.ndarray
    n_steps: np.ndarray
    n_samples: np.ndarray
    sample_offset: np.ndarray
    tau: np.ndarray
    moment: np.ndarray  # (nb, 3)
    rf_re: np.ndarray
    rf_im: np.ndarray
    gx: np.ndarray
    gy: np.ndarray
    gz: np.ndarray
    adc_idx: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_blocks(self):
        return int(self.btype.shape[0])

    @property
    def total_steps(self):
        return int(self.rf_re.shape[0])

    @property
    def total_samples(self):
        return int(self.adc_idx.shape[0])

    def stepped_count(self):
        """Raster steps inside RF and ADC blocks (relaxation blocks excluded)."""
        m = (self.btype == BLOCK_RF) | (self.btype == BLOCK_ADC)
        return int(self.n_steps[m].sum())

    def head(self, n_blocks: int, name: str | None = None) -> "Sequence":
        """The first n_blocks blocks as a sequence of their own."""
        nb = int(n_blocks)
        stepped = self.btype[:nb] != BLOCK_RELAX
        s_end = int((self.step_offset[:nb] + self.n_steps[:nb])[stepped].max()) if stepped.any() else 0
        q_end = int((self.sample_offset[:nb] + self.n_samples[:nb]).max()) if nb else 0
        return Sequence(dt=self.dt, btype=self.btype[:nb].copy(), step_offset=self.step_offset[:nb].copy(),
                        n_steps=self.n_steps[:nb].copy(), n_samples=self.n_samples[:nb].copy(),
                        sample_offset=self.sample_offset[:nb].copy(), tau=self.tau[:nb].copy(),
                        moment=self.moment[:nb].copy(), rf_re=self.rf_re[:s_end].copy(),
                        rf_im=self.rf_im[:s_end].copy(), gx=self.gx[:s_end].copy(), gy=self.gy[:s_end].copy(),
                        gz=self.gz[:s_end].copy(), adc_idx=self.adc_idx[:q_end].copy(),
                        name=name or f"{self.name}[:{nb}]", meta=dict(self.meta))


class SeqBuilder:
    def __init__(self, dt=1e-6, name=""):
        self.dt = float(dt)
        self.name = name
        self.blocks = []
        self.wave = []  # list of (rf complex, gx, gy, gz) per stepped block
        self.nsteps = 0
        self.sample_lists = []
        self.nsamp = 0

    @staticmethod
    def _arr(v, n):
        a = np.asarray(v, dtype=np.float64)
        return np.full(n, float(a)) if a.ndim == 0 else a.astype(np.float64)

    def _stepped(self, btype, rf, g, samples=()):
        n = len(rf)
        gx, gy, gz = (self._arr(gi, n) for gi in g)
        samples = np.asarray(samples, dtype=np.int64)
        if samples.size and (samples.min() < 0 or samples.max() > n):
            raise ValueError("ADC sample index outside its block")
        self.blocks.append(dict(type=btype, step_offset=self.nsteps, n_steps=n,
                                n_samples=int(samples.size), sample_offset=self.nsamp,
                                tau=0.0, moment=(0.0, 0.0, 0.0)))
        self.wave.append((np.asarray(rf, dtype=np.complex128), gx, gy, gz))
        self.nsteps += n
        if samples.size:
            self.sample_lists.append(samples)
            self.nsamp += int(samples.size)

    def rf(self, b1, g=(0.0, 0.0, 0.0)):
        self._stepped(BLOCK_RF, b1, g)

    def adc(self, n_steps, g, samples, b1=None):
        rf = np.zeros(n_steps, dtype=np.complex128) if b1 is None else b1
        self._stepped(BLOCK_ADC, rf, g, samples)

    def relax(self, tau, moment=(0.0, 0.0, 0.0)):
        if tau < 0:
            raise ValueError("negative relaxation duration")
        self.blocks.append(dict(type=BLOCK_RELAX, step_offset=self.nsteps, n_steps=0,
                                n_samples=0, sample_offset=self.nsamp, tau=float(tau),
                                moment=tuple(float(m) for m in moment)))

    def build(self, **meta) -> Sequence:
        nb = len(self.blocks)
        col = lambda k, dt: np.array([b[k] for b in self.blocks], dtype=dt)
        if self.wave:
            rf = np.concatenate([w[0] for w in self.wave])
            gx, gy, gz = (np.concatenate([w[i] for w in self.wave]) for i in (1, 2, 3))
        else:
            rf = np.zeros(0, np.complex128)
            gx = gy = gz = np.zeros(0)
        adc = np.concatenate(self.sample_lists) if self.sample_lists else np.zeros(0, np.int64)
        f32 = lambda a: np.ascontiguousarray(a, dtype=np.float32)
        return Sequence(
            dt=self.dt, btype=col("type", np.int32), step_offset=col("step_offset", np.int64),
            n_steps=col("n_steps", np.int64), n_samples=col("n_samples", np.int32),
            sample_offset=col("sample_offset", np.int64), tau=col("tau", np.float64),
            moment=np.array([b["moment"] for b in self.blocks], dtype=np.float64).reshape(nb, 3),
            rf_re=f32(rf.real), rf_im=f32(rf.imag), gx=f32(gx), gy=f32(gy), gz=f32(gz),
            adc_idx=np.ascontiguousarray(adc, dtype=np.int32), name=self.name, meta=meta)


def sinc_envelope(n_steps, tbw=4.0):
    """Hamming-windowed sinc with `tbw` zero-crossings across the pulse
    (tbw=4: a central lobe and one side lobe on each side), sampled at step
    midpoints."""
    T = float(n_steps)
    t = np.arange(n_steps, dtype=np.float64) + 0.5 - T / 2
    return np.sinc(tbw * t / T) * (0.54 + 0.46 * np.cos(2 * np.pi * t / T))


def sinc_pulse(n_steps, dt, flip_rad, tbw=4.0, phase=0.0):
    """Complex B1 (T) whose on-resonance rotation angle gamma*sum(B1)*dt is flip_rad."""
    env = sinc_envelope(n_steps, tbw)
    amp = flip_rad / (2 * np.pi * GAMMA_BAR * dt * env.sum())
    return amp * env * np.exp(1j * phase)


def chess_pulse(n_steps, dt, flip_rad, offset_hz, tbw=2.0):
    """Frequency-selective (CHESS) pulse without gradients: a sinc whose
    centre frequency is moved by offset_hz (fat saturation: about -440 Hz at 3 T)."""
    t = (np.arange(n_steps) + 0.5 - n_steps / 2) * dt
    return sinc_pulse(n_steps, dt, flip_rad, tbw) * np.exp(2j * np.pi * offset_hz * t)


def slice_gradient(n_steps, dt, thk, tbw=4.0):
    return tbw / (n_steps * dt * GAMMA_BAR * thk)


def readout_gradient(dwell, fov):
    return 1.0 / (GAMMA_BAR * dwell * fov)


def gre_sequence(n_lines=32, n_read=64, dwell_steps=10, fov=(0.200, 0.200), thk=0.005,
                 flip_deg=30.0, rf_steps=2000, te=5e-3, tr=20e-3, dt=1e-6, tbw=4.0, tilt_deg=0.0):
    """Spoiled 2D gradient echo: sinc RF with Gz, rephase + prephase + phase
    encode (relaxation), Gx readout (ADC), rewind + spoil to TR (relaxation).
    tilt_deg tilts the slice normal from z toward x (an oblique slice: the
    slice-select gradient and its rephaser gain an x component)."""
    sn, cs = np.sin(np.deg2rad(tilt_deg)), np.cos(np.deg2rad(tilt_deg))
    sb = SeqBuilder(dt, name=f"gre{n_lines}x{n_read}")
    b1 = sinc_pulse(rf_steps, dt, np.deg2rad(flip_deg), tbw)
    gz = slice_gradient(rf_steps, dt, thk, tbw)
    g_ro = readout_gradient(dwell_steps * dt, fov[0])
    ro_steps = n_read * dwell_steps
    samples = dwell_steps * np.arange(n_read) + dwell_steps // 2
    echo_step = int(samples[n_read // 2])
    tau_pre = te - rf_steps * dt / 2 - echo_step * dt
    tau_post = tr - rf_steps * dt - tau_pre - ro_steps * dt
    assert tau_pre > 0 and tau_post > 0
    spoil_z = 4.0 / (GAMMA_BAR * thk)
    for line in range(n_lines):
        my = (line - n_lines // 2) / (GAMMA_BAR * fov[1])
        sb.rf(b1, (sn * gz, 0.0, cs * gz))
        sb.relax(tau_pre, (-g_ro * echo_step * dt - sn * 0.5 * gz * rf_steps * dt, my, -cs * 0.5 * gz * rf_steps * dt))
        sb.adc(ro_steps, (g_ro, 0.0, 0.0), samples)
        sb.relax(tau_post, (2.0 * g_ro * ro_steps * dt, -my, spoil_z))
    return sb.build(kind="gre", n_lines=n_lines, n_read=n_read, fov=fov)


def fse_sequence(n_shots=16, etl=16, n_read=256, dwell_steps=4, fov=(0.256, 0.256), thk=0.010,
                 rf_steps=3000, esp=8e-3, tr=3.0, dt=1e-6, tbw=4.0, fat_sat=False, tilt_deg=0.0):
    """CPMG fast spin echo: 90x then `etl` 180y refocusing pulses (sinc with Gz),
    each echo read out with Gx; phase-encode line = etl_index*n_shots + shot.
    Crushers bracket every refocusing pulse; relaxation to TR ends each shot.
    fat_sat: every shot starts with a 2 ms CHESS 90-degree pulse at -440 Hz
    (a no-grads with-RF subsequence) and a 1 ms spoiler, taken from the end
    of the TR.  tilt_deg tilts the slice normal from z toward x (an oblique
    slice): slice selection, its rephaser and the crushers gain an x part."""
    sn, cs = np.sin(np.deg2rad(tilt_deg)), np.cos(np.deg2rad(tilt_deg))
    sb = SeqBuilder(dt, name=f"fse{n_shots}x{etl}x{n_read}" + ("fs" if fat_sat else ""))
    chess = chess_pulse(2000, dt, np.pi / 2, -440.0) if fat_sat else None
    fs_time = 3e-3 if fat_sat else 0.0
    b90 = sinc_pulse(rf_steps, dt, np.pi / 2, tbw, phase=0.0)
    b180 = sinc_pulse(rf_steps, dt, np.pi, tbw, phase=np.pi / 2)
    gz = slice_gradient(rf_steps, dt, thk, tbw)
    g_ro = readout_gradient(dwell_steps * dt, fov[0])
    ro_steps = n_read * dwell_steps
    samples = dwell_steps * np.arange(n_read) + dwell_steps // 2
    echo_step = int(samples[n_read // 2])
    a = g_ro * dt  # readout moment per raster step
    crush = 2.0 / (GAMMA_BAR * thk)
    half_rf = rf_steps * dt / 2
    n_lines = n_shots * etl
    tau_90_180 = esp / 2 - 2 * half_rf
    tau_pre = esp / 2 - half_rf - echo_step * dt
    tau_post = esp / 2 - (ro_steps - echo_step) * dt - half_rf
    assert min(tau_90_180, tau_pre, tau_post) > 0
    shot_len = 2 * half_rf + tau_90_180 + etl * (2 * half_rf + tau_pre + ro_steps * dt + tau_post)
    tau_end = tr - shot_len + tau_post - fs_time
    assert tau_end > 0
    # x-moments: prephaser P, pre-readout Q, post-readout R = 0 such that every
    # echo centre (sample n_read//2) sees zero net x-moment.
    P = (ro_steps - echo_step) * a
    Q = P - echo_step * a
    for shot in range(n_shots):
        if fat_sat:
            sb.rf(chess, (0.0, 0.0, 0.0))
            sb.relax(1e-3, (8.0 / (GAMMA_BAR * fov[0]), 8.0 / (GAMMA_BAR * fov[1]), 8.0 / (GAMMA_BAR * thk)))
        sb.rf(b90, (sn * gz, 0.0, cs * gz))
        s_m = -0.5 * gz * rf_steps * dt + crush  # slice rephaser and crusher
        sb.relax(tau_90_180, (P + sn * s_m, 0.0, cs * s_m))
        for e in range(etl):
            line = e * n_shots + shot
            my = (line - n_lines // 2) / (GAMMA_BAR * fov[1])
            sb.rf(b180, (sn * gz, 0.0, cs * gz))
            sb.relax(tau_pre, (Q + sn * crush, my, cs * crush))
            sb.adc(ro_steps, (g_ro, 0.0, 0.0), samples)
            if e + 1 < etl:
                sb.relax(tau_post, (sn * crush, -my, cs * crush))
            else:
                sb.relax(tau_end, (4.0 * g_ro * ro_steps * dt + sn * 4.0 * crush, -my, cs * 4.0 * crush))
    return sb.build(kind="fse", n_shots=n_shots, etl=etl, n_read=n_read, fov=fov)


def epi_sequence(n_lines=128, n_read=128, dwell_steps=4, fov=(0.256, 0.256), thk=0.010,
                 rf_steps=3000, ramp=120e-6, blip=100e-6, dt=1e-6, tbw=4.0, te_fill=2e-3):
    """Single-shot gradient-echo EPI: 90x sinc with Gz, then `n_lines` readouts
    with alternating Gx flat tops (ADC), trapezoid ramps and triangular Gy
    blips as relaxation blocks."""
    sb = SeqBuilder(dt, name=f"epi{n_lines}x{n_read}")
    b90 = sinc_pulse(rf_steps, dt, np.pi / 2, tbw)
    gz = slice_gradient(rf_steps, dt, thk, tbw)
    g_ro = readout_gradient(dwell_steps * dt, fov[0])
    ro_steps = n_read * dwell_steps
    samples = dwell_steps * np.arange(n_read) + dwell_steps // 2
    a = g_ro * dt
    ramp_m = 0.5 * g_ro * ramp
    blip_m = 1.0 / (GAMMA_BAR * fov[1])
    sb.rf(b90, (0.0, 0.0, gz))
    pre_x = -(ramp_m + samples[n_read // 2] * a)
    pre_y = -(n_lines // 2) * blip_m
    sb.relax(te_fill, (pre_x, pre_y, -0.5 * gz * rf_steps * dt))
    for line in range(n_lines):
        s = 1.0 if line % 2 == 0 else -1.0
        sb.relax(ramp, (s * ramp_m, 0.0, 0.0))
        sb.adc(ro_steps, (s * g_ro, 0.0, 0.0), samples)
        sb.relax(ramp, (s * ramp_m, 0.0, 0.0))
        if line + 1 < n_lines:
            sb.relax(blip, (0.0, blip_m, 0.0))
    return sb.build(kind="epi", n_lines=n_lines, n_read=n_read, fov=fov)


# ---- the four pulse sequences of the paper's Table 2 --------------------------
# Hamming-windowed sinc pulses of 4000 us at 1 us per sample (90 and 180
# degrees), FOV 256 mm x 256 mm, one 10 mm slice, 256 readout samples (128 for
# the EPI).  Timing the table leaves open (gaps, crushers, ramps) is ours.
def se_sequence(n_lines=256, n_read=256, dwell_steps=5, fov=(0.256, 0.256), thk=0.010, rf_steps=4000,
                te=10e-3, tr=500e-3, dt=1e-6, tbw=4.0):
    """2D spin echo: per TR a 90x and a 180y sinc with Gz, one Gx readout whose
    centre sample is at TE after the centre of the 90; readout prephaser and
    phase encode before the 180, crushers on both sides of it, spoiling to TR.
    Table 2: T1W is TE 10 ms, TR 500 ms, 5 us/sample; T2W is TE 100 ms,
    TR 4500 ms, 50 us/sample."""
    sb = SeqBuilder(dt, name=f"se{n_lines}x{n_read}")
    b90 = sinc_pulse(rf_steps, dt, np.pi / 2, tbw, phase=0.0)
    b180 = sinc_pulse(rf_steps, dt, np.pi, tbw, phase=np.pi / 2)
    gz = slice_gradient(rf_steps, dt, thk, tbw)
    g_ro = readout_gradient(dwell_steps * dt, fov[0])
    ro_steps = n_read * dwell_steps
    samples = dwell_steps * np.arange(n_read) + dwell_steps // 2
    echo_step = int(samples[n_read // 2])
    half_rf = rf_steps * dt / 2
    crush = 2.0 / (GAMMA_BAR * thk)
    tau_1 = te / 2 - 2 * half_rf                  # end of the 90 to the start of the 180
    tau_2 = te / 2 - half_rf - echo_step * dt     # end of the 180 to the start of the readout
    tau_end = tr - (4 * half_rf + tau_1 + tau_2 + ro_steps * dt)
    assert min(tau_1, tau_2, tau_end) > 0
    spoil_z = 4.0 / (GAMMA_BAR * thk)
    for line in range(n_lines):
        my = (line - n_lines // 2) / (GAMMA_BAR * fov[1])
        sb.rf(b90, (0.0, 0.0, gz))
        # the 180 negates the phase of everything before it, so the prephaser
        # has the readout's sign
        sb.relax(tau_1, (g_ro * echo_step * dt, my, -0.5 * gz * rf_steps * dt + crush))
        sb.rf(b180, (0.0, 0.0, gz))
        sb.relax(tau_2, (0.0, 0.0, crush))
        sb.adc(ro_steps, (g_ro, 0.0, 0.0), samples)
        sb.relax(tau_end, (2.0 * g_ro * ro_steps * dt, 0.0, spoil_z))
    return sb.build(kind="se", n_lines=n_lines, n_read=n_read, fov=fov, te=te, tr=tr)


def se_epi_sequence(n_lines=96, n_full=128, n_read=128, dwell_steps=3, fov=(0.256, 0.256), thk=0.010,
                    rf_steps=4000, te=70e-3, ramp=120e-6, blip=100e-6, dt=1e-6, tbw=4.0):
    """Single-shot spin-echo EPI with partial Fourier: 90x and 180y sinc with
    Gz, then n_lines of the n_full phase-encode lines (from
    n_full/2 - n_lines to n_full/2 - 1 about the centre), alternating Gx flat
    tops (ADC) with trapezoid ramps and Gy blips as relaxation blocks.  The
    centre sample of the centre line is at TE after the centre of the 90.
    Table 2: 96 of 128 lines, 128 samples at 3 us, TE 70 ms."""
    sb = SeqBuilder(dt, name=f"seepi{n_lines}of{n_full}x{n_read}")
    b90 = sinc_pulse(rf_steps, dt, np.pi / 2, tbw, phase=0.0)
    b180 = sinc_pulse(rf_steps, dt, np.pi, tbw, phase=np.pi / 2)
    gz = slice_gradient(rf_steps, dt, thk, tbw)
    g_ro = readout_gradient(dwell_steps * dt, fov[0])
    ro_steps = n_read * dwell_steps
    samples = dwell_steps * np.arange(n_read) + dwell_steps // 2
    echo_step = int(samples[n_read // 2])
    half_rf = rf_steps * dt / 2
    ramp_m = 0.5 * g_ro * ramp
    blip_m = 1.0 / (GAMMA_BAR * fov[1])
    crush = 2.0 / (GAMMA_BAR * thk)
    first = n_full // 2 - n_lines  # phase-encode index of the first line (centre = 0)
    c = -first                     # acquisition index of the centre line
    period = ro_steps * dt + 2 * ramp + blip
    tau_a = te / 2 - 2 * half_rf
    tau_b = te - (te / 2 + half_rf) - (c * period + ramp + echo_step * dt)
    assert n_lines <= n_full and first <= 0 and tau_a > 0 and tau_b > 0
    sb.rf(b90, (0.0, 0.0, gz))
    sb.relax(tau_a, (0.0, 0.0, -0.5 * gz * rf_steps * dt + crush))
    sb.rf(b180, (0.0, 0.0, gz))
    sb.relax(tau_b, (-(ramp_m + echo_step * g_ro * dt), first * blip_m, crush))
    for line in range(n_lines):
        s = 1.0 if line % 2 == 0 else -1.0
        sb.relax(ramp, (s * ramp_m, 0.0, 0.0))
        sb.adc(ro_steps, (s * g_ro, 0.0, 0.0), samples)
        sb.relax(ramp, (s * ramp_m, 0.0, 0.0))
        if line + 1 < n_lines:
            sb.relax(blip, (0.0, blip_m, 0.0))
    return sb.build(kind="se-epi", n_lines=n_lines, n_full=n_full, n_read=n_read, fov=fov, te=te)


def table2_sequences(small=False):
    """The four Table 2 sequences by name (full size, or a reduced version of
    the same structure for oracle-checked parity runs)."""
    if small:
        return {
            "t1w-se": se_sequence(n_lines=3, n_read=16, dwell_steps=5, rf_steps=400, te=10e-3, tr=30e-3),
            "t2w-se": se_sequence(n_lines=2, n_read=16, dwell_steps=50, rf_steps=400, te=100e-3, tr=0.3),
            "se-epi": se_epi_sequence(n_lines=12, n_full=16, n_read=16, rf_steps=400, te=20e-3),
            "fse-etl5": fse_sequence(n_shots=2, etl=5, n_read=16, dwell_steps=8, rf_steps=400, esp=12e-3,
                                     tr=0.2),
        }
    return {
        "t1w-se": se_sequence(te=10e-3, tr=500e-3, dwell_steps=5),
        "t2w-se": se_sequence(te=100e-3, tr=4500e-3, dwell_steps=50),
        "se-epi": se_epi_sequence(),
        "fse-etl5": fse_sequence(n_shots=52, etl=5, n_read=256, dwell_steps=8, rf_steps=4000, esp=12e-3, tr=1.5),
    }


# ---- learned RF-transition surrogate: the modelled pulse and its inputs ----
def fse_refocusing_pulse(rf_steps=3000, dt=1e-6, thk=0.010, tbw=4.0):
    """The FSE 180-degree refocusing pulse (about y) with its slice gradient:
    (complex B1 per step [T], Gz per step [T/m], dt)."""
    b180 = sinc_pulse(rf_steps, dt, np.pi, tbw, phase=np.pi / 2)
    gz = np.full(rf_steps, slice_gradient(rf_steps, dt, thk, tbw))
    return b180, gz, dt


SURROGATE_RANGES = {  # training domain of the surrogate inputs
    "f_z": (-1400.0, 1400.0),   # Hz, gamma_bar * Gz * z (slice +-10 mm covers +-1333 Hz)
    "f_b0": (-100.0, 100.0),    # Hz
    "t1": (0.25, 2.5),          # s, log-uniform
    "t2": (0.03, 0.3),          # s, log-uniform
    "b1": (0.8, 1.2),           # B1 scale
}


def surrogate_tuples(n, seed=2024):
    """Seeded random surrogate inputs, float32 (n, 5): f_z, f_B0, T1, T2, B1 scale."""
    r = SURROGATE_RANGES
    rng = np.random.default_rng(seed)
    out = np.empty((n, 5), np.float32)
    out[:, 0] = rng.uniform(*r["f_z"], n)
    out[:, 1] = rng.uniform(*r["f_b0"], n)
    out[:, 2] = np.exp(rng.uniform(np.log(r["t1"][0]), np.log(r["t1"][1]), n))
    out[:, 3] = np.exp(rng.uniform(np.log(r["t2"][0]), np.log(r["t2"][1]), n))
    out[:, 4] = rng.uniform(*r["b1"], n)
    return out


def mlp_init_params(seed=0):
    """Seeded parameters of the 5-128-128-128-12 network in the flat order
    W1 b1 W2 b2 W3 b3 W4 b4, each drawn from U(-1/sqrt(fan_in), 1/sqrt(fan_in))."""
    rng = np.random.default_rng(seed)
    shapes = [((128, 5), 5), ((128,), 5), ((128, 128), 128), ((128,), 128),
              ((128, 128), 128), ((128,), 128), ((12, 128), 128), ((12,), 128)]
    parts = [rng.uniform(-1, 1, int(np.prod(s))) / np.sqrt(f) for s, f in shapes]
    return np.concatenate(parts).astype(np.float32)


# ---- adjoint (gradient of the signal) workload ----------------------------
def adjoint_workload(nx=256, ny=256, nz=16, n_lines=8, n_read=64, rf_steps=3000, seed=1002):
    """GRE for the signal gradient: a (nx, ny, nz) six-class phantom over
    256x256x10 mm, 8 B0 levels in +-50 Hz; n_lines TRs of a 3 ms sinc 30-degree
    RF with Gz (5 mm slice), n_read samples at 10 us, TE 5 ms, TR 10 ms.

    Returns (phantom, class T1, class T2, sequence, rf_param, param_blocks):
    the RF blocks listed in param_blocks all play the complex pulse rf_param."""
    ph = ellipse_phantom(nx, ny, nz, (0.256, 0.256, 0.010), SIX_T1, SIX_T2, SIX_PD,
                         df_range=50.0, df_levels=8, seed=seed, name=f"adjoint {nx}x{ny}x{nz}")
    seq = gre_sequence(n_lines=n_lines, n_read=n_read, dwell_steps=10, fov=(0.256, 0.256), thk=0.005,
                       rf_steps=rf_steps, te=5e-3, tr=10e-3)
    rf = sinc_pulse(rf_steps, 1e-6, np.deg2rad(30.0), 4.0)
    blocks = np.nonzero(np.asarray(seq.btype) == BLOCK_RF)[0].astype(np.int32)
    return ph, np.array(SIX_T1), np.array(SIX_T2), seq, rf.astype(np.complex128), blocks


# Workload registry: the sizes used by the benchmark and the parity tests.
def workload(name: str):
    """Return (phantom, sequence) for a named workload."""
    if name == "gre":  # plain FP64 oracle workload, 4096 isochromats
        return gre_phantom(), gre_sequence()
    if name == "fse":  # 1024x1024x26 isochromats, 16 shots x ETL 16, 256 samples
        return brain_like_phantom(), fse_sequence()
    if name == "epi":  # same phantom, 128 lines x 128 samples
        return brain_like_phantom(), epi_sequence()
    if name == "fse-small":
        return brain_like_phantom(48, 40, 3), fse_sequence(n_shots=2, etl=3, n_read=32)
    if name == "epi-small":
        return brain_like_phantom(48, 40, 3), epi_sequence(n_lines=12, n_read=32, rf_steps=1000)
    raise KeyError(name)
