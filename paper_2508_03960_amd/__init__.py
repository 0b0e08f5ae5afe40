"""Python binding of libgbloch (include/gbloch.h): grouped-isochromat Bloch
simulation on gfx950.

Argument marshalling only: every step of the simulation runs in the HIP
kernels of ``libgbloch.so``.  PyTorch provides device memory and the stream.
The library must be built (``python paper_2508_03960_amd/build.py``); there is
no CPU fallback, and importing this package fails loudly without it.
"""
from __future__ import annotations

import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgbloch.so")

GBS_OK, GBS_E_INVALID, GBS_E_STATE, GBS_E_HIP, GBS_E_NOMEM, GBS_E_WORKSPACE = 0, -1, -2, -3, -4, -5
GBS_BLOCK_RF, GBS_BLOCK_ADC, GBS_BLOCK_RELAX = 1, 2, 3
GBS_AX_X, GBS_AX_Y, GBS_AX_Z, GBS_AX_N, GBS_AX_XZ = 1, 2, 4, 8, 16
GBS_AX_ALL = GBS_AX_X | GBS_AX_Y | GBS_AX_Z | GBS_AX_N | GBS_AX_XZ
GBS_PLAIN, GBS_GROUPED, GBS_CACHED = 0, 1, 2
GBS_ASYNC = 1
GBS_PROFILE = 4
GBS_SURROGATE = 8
GBS_MLP_PARAMS = 35340
GBS_STATIC_WORKSPACE_BYTES = 64 << 20

EXPORTED = ("gbs_create", "gbs_destroy", "gbs_set_phantom", "gbs_set_sequence", "gbs_build_groups",
            "gbs_simulate", "gbs_workspace_size", "gbs_simulate_static", "gbs_get_info", "gbs_last_error", "gbs_strerror", "gbs_plan_summary",
            "gbs_plan_cached_summary", "gbs_set_coils",
            "gbs_mlp_create", "gbs_mlp_destroy", "gbs_mlp_last_error", "gbs_mlp_set_pulse",
            "gbs_mlp_set_norm", "gbs_mlp_get_params", "gbs_mlp_set_params", "gbs_mlp_exact",
            "gbs_mlp_infer", "gbs_mlp_loss_grad", "gbs_mlp_train", "gbs_set_surrogate",
            "gbs_adj_forward", "gbs_adj_backward", "gbs_pulseq_load")


class gbs_block(ctypes.Structure):
    _fields_ = [("type", ctypes.c_int32), ("n_samples", ctypes.c_int32),
                ("step_offset", ctypes.c_int64), ("n_steps", ctypes.c_int64),
                ("sample_offset", ctypes.c_int64), ("tau", ctypes.c_double),
                ("moment", ctypes.c_double * 3)]


class gbs_info(ctypes.Structure):
    _fields_ = [("K", ctypes.c_int64), ("n_blocks", ctypes.c_int64), ("total_steps", ctypes.c_int64),
                ("total_samples", ctypes.c_int64), ("stepped_steps", ctypes.c_int64),
                ("n_groups", ctypes.c_int64 * 3), ("groups_valid", ctypes.c_int32),
                ("device", ctypes.c_int32), ("n_tissue_groups", ctypes.c_int64), ("n_coils", ctypes.c_int64),
                ("n_xz_groups", ctypes.c_int64)]


class gbs_stats(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("ms_prepare", ctypes.c_double),
                ("ms_passes", ctypes.c_double), ("ms_adc_eval", ctypes.c_double),
                ("ms_stepped", ctypes.c_double), ("n_passes", ctypes.c_int64),
                ("n_emit_only", ctypes.c_int64), ("n_rf_grouped", ctypes.c_int64),
                ("n_adc_grouped", ctypes.c_int64), ("n_fallback", ctypes.c_int64),
                ("n_distinct_rf", ctypes.c_int64), ("n_b1zero", ctypes.c_int64),
                ("pass_bytes", ctypes.c_double), ("pass_kernel_ms", ctypes.c_double),
                ("n_sweeps", ctypes.c_int64), ("pass_flops", ctypes.c_double),
                ("n_surrogate", ctypes.c_int64), ("n_surrogate_fallback", ctypes.c_int64),
                ("surrogate_residual", ctypes.c_double), ("n_rf_cached", ctypes.c_int64),
                ("n_adc_direct", ctypes.c_int64), ("cache_bytes", ctypes.c_double),
                ("ms_compose", ctypes.c_double), ("ms_apply", ctypes.c_double),
                ("ms_adc_direct", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class gbs_train_cfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr_max", ctypes.c_float),
                ("lr_min", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("seed", ctypes.c_uint64)]


def _load(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python paper_2508_03960_amd/build.py`")
    lib = ctypes.CDLL(path)
    P, I64, I32, U32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32, ctypes.c_double
    sig = {
        "gbs_create": ([ctypes.POINTER(P), ctypes.c_int, P], ctypes.c_int),
        "gbs_destroy": ([P], ctypes.c_int),
        "gbs_set_phantom": ([P, I64] + [P] * 7, ctypes.c_int),
        "gbs_set_coils": ([P, I32, P, P], ctypes.c_int),
        "gbs_set_sequence": ([P, P, I64, P, P, P, P, P, I64, P, I64, D], ctypes.c_int),
        "gbs_build_groups": ([P, U32], ctypes.c_int),
        "gbs_simulate": ([P, ctypes.c_int, U32, P, ctypes.c_size_t, P, P, P, P], ctypes.c_int),
        "gbs_workspace_size": ([P, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
        "gbs_simulate_static": ([P, ctypes.c_int, U32, P, P, P, P], ctypes.c_int),
        "gbs_get_info": ([P, P], ctypes.c_int),
        "gbs_last_error": ([P], ctypes.c_char_p),
        "gbs_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "gbs_plan_summary": ([P, I64, P, P, P, P, P, I64, P, I64, D, U32, P], ctypes.c_int),
        "gbs_plan_cached_summary": ([P, I64, P, P, P, P, P, I64, P, I64, D, P], ctypes.c_int),
        "gbs_mlp_create": ([ctypes.POINTER(P), ctypes.c_int, P, ctypes.c_uint64], ctypes.c_int),
        "gbs_mlp_destroy": ([P], ctypes.c_int),
        "gbs_mlp_last_error": ([P], ctypes.c_char_p),
        "gbs_mlp_set_pulse": ([P, P, P, P, P, P, I64, D], ctypes.c_int),
        "gbs_mlp_set_norm": ([P, P, P], ctypes.c_int),
        "gbs_mlp_get_params": ([P, P, I64], ctypes.c_int),
        "gbs_mlp_set_params": ([P, P, I64], ctypes.c_int),
        "gbs_mlp_exact": ([P, P, I64, P], ctypes.c_int),
        "gbs_mlp_infer": ([P, P, I64, P], ctypes.c_int),
        "gbs_mlp_loss_grad": ([P, P, P, I64, P, P], ctypes.c_int),
        "gbs_mlp_train": ([P, P, P, I64, P, P, I64], ctypes.c_int),
        "gbs_set_surrogate": ([P, P, ctypes.c_float, I32, ctypes.c_uint64], ctypes.c_int),
        "gbs_adj_forward": ([P, P, I32, P, P, P, I64, P, I32, I32, P], ctypes.c_int),
        "gbs_adj_backward": ([P, P, P, P, P], ctypes.c_int),
        "gbs_pulseq_load": ([ctypes.c_char_p, I64, D, P, P] + [P] * 9 + [I64], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


lib = _load()


class GbsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{lib.gbs_strerror(code).decode()} ({code}): {msg}")
        self.code = code


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _host(a, dtype):
    import numpy as np
    return np.ascontiguousarray(a, dtype=dtype)


def sequence_blocks(seq):
    """gbs_block array for a synth.Sequence-like object (host)."""
    nb = seq.n_blocks
    arr = (gbs_block * max(nb, 1))()
    for b in range(nb):
        k = arr[b]
        k.type = int(seq.btype[b])
        k.n_samples = int(seq.n_samples[b])
        k.step_offset = int(seq.step_offset[b])
        k.n_steps = int(seq.n_steps[b])
        k.sample_offset = int(seq.sample_offset[b])
        k.tau = float(seq.tau[b])
        for i in range(3):
            k.moment[i] = float(seq.moment[b][i])
    return arr


def gbs_plan_summary(seq, axes=GBS_AX_ALL):
    """Host-only classification counts (see gbloch.h)."""
    import numpy as np
    blocks = sequence_blocks(seq)
    w = [_host(a, np.float32) for a in (seq.rf_re, seq.rf_im, seq.gx, seq.gy, seq.gz)]
    adc = _host(seq.adc_idx, np.int32)
    out = (ctypes.c_int64 * 8)()
    rc = lib.gbs_plan_summary(blocks, seq.n_blocks, *(a.ctypes.data for a in w), seq.total_steps,
                              adc.ctypes.data, seq.total_samples, float(seq.dt), axes, out)
    if rc != GBS_OK:
        raise GbsError(rc, "gbs_plan_summary rejected the sequence")
    keys = ("rf_grouped", "adc_grouped", "fallback", "b1zero", "passes", "emit_only", "distinct_rf", "relax")
    return dict(zip(keys, list(out)))


def gbs_plan_cached_summary(seq):
    """Host-only counts of what GBS_CACHED runs (see gbloch.h)."""
    import numpy as np
    blocks = sequence_blocks(seq)
    w = [_host(a, np.float32) for a in (seq.rf_re, seq.rf_im, seq.gx, seq.gy, seq.gz)]
    adc = _host(seq.adc_idx, np.int32)
    out = (ctypes.c_int64 * 6)()
    rc = lib.gbs_plan_cached_summary(blocks, seq.n_blocks, *(a.ctypes.data for a in w), seq.total_steps,
                                     adc.ctypes.data, seq.total_samples, float(seq.dt), out)
    if rc != GBS_OK:
        raise GbsError(rc, "gbs_plan_cached_summary rejected the sequence")
    keys = ("rf_cached", "entries", "adc_direct", "adc_launches", "fallback", "b1zero")
    return dict(zip(keys, list(out)))


class PulseqSequence:
    """A sequence read from a Pulseq 1.4 file by gbs_pulseq_load: the block
    form gbs_set_sequence takes (the same fields as the seeded generators'
    sequences), plus ``adc_phase`` (receiver phase per sample, radians) and
    ``rasters`` (gradient, RF, ADC and block-duration raster times, s)."""

    def __init__(self, dt, blocks, rf_re, rf_im, gx, gy, gz, adc_idx, adc_phase, rasters, name=""):
        import numpy as np
        nb = len(blocks)
        self.dt = float(dt)
        self.btype = np.array([b.type for b in blocks], np.int32)
        self.step_offset = np.array([b.step_offset for b in blocks], np.int64)
        self.n_steps = np.array([b.n_steps for b in blocks], np.int64)
        self.n_samples = np.array([b.n_samples for b in blocks], np.int32)
        self.sample_offset = np.array([b.sample_offset for b in blocks], np.int64)
        self.tau = np.array([b.tau for b in blocks], np.float64)
        self.moment = np.array([list(b.moment) for b in blocks], np.float64).reshape(nb, 3)
        self.rf_re, self.rf_im, self.gx, self.gy, self.gz = rf_re, rf_im, gx, gy, gz
        self.adc_idx, self.adc_phase, self.rasters = adc_idx, adc_phase, rasters
        self.name = name
        self.meta = {"source": "pulseq"}

    @property
    def n_blocks(self):
        return int(self.btype.shape[0])

    @property
    def total_steps(self):
        return int(self.rf_re.shape[0])

    @property
    def total_samples(self):
        return int(self.adc_idx.shape[0])


def load_pulseq(source, dt=None, name=None):
    """Read a Pulseq 1.4 sequence (a path; or the file's text as bytes, or as
    a str of several lines) into a PulseqSequence on the raster ``dt`` (s; None = the file's RF
    raster time).  Raises GbsError with the parser's message on a bad file."""
    import numpy as np
    if isinstance(source, (bytes, bytearray)):
        text = bytes(source)
    elif isinstance(source, os.PathLike) or (isinstance(source, str) and "\n" not in source):
        with open(source, "rb") as fh:  # a path (one line); file text has several
            text = fh.read()
        name = name or os.path.basename(os.fspath(source))
    else:
        text = source.encode()
    err = ctypes.create_string_buffer(512)
    sizes = (ctypes.c_int64 * 3)()
    rasters = (ctypes.c_double * 4)()
    dtv = float(dt) if dt else 0.0
    rc = lib.gbs_pulseq_load(text, len(text), dtv, sizes, None, None, None, None, None, None, None, None,
                             rasters, err, len(err))
    if rc != GBS_OK:
        raise GbsError(rc, err.value.decode(errors="replace"))
    nb, ns, nq = list(sizes)
    blocks = (gbs_block * max(nb, 1))()
    w = [np.zeros(max(ns, 1), np.float32) for _ in range(5)]
    adc = np.zeros(max(nq, 1), np.int32)
    ph = np.zeros(max(nq, 1), np.float64)
    rc = lib.gbs_pulseq_load(text, len(text), dtv, sizes, blocks, *(a.ctypes.data for a in w), adc.ctypes.data,
                             ph.ctypes.data, rasters, err, len(err))
    if rc != GBS_OK:
        raise GbsError(rc, err.value.decode(errors="replace"))
    used_dt = dtv if dtv > 0 else rasters[1]
    return PulseqSequence(used_dt, list(blocks)[:nb], *(a[:ns] for a in w), adc[:nq], ph[:nq], tuple(rasters),
                          name=name or "pulseq")


class Simulator:
    """One gbs context on a CUDA (HIP) device; thin wrapper over the C ABI."""

    def __init__(self, device=0, stream=None):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = lib.gbs_create(ctypes.byref(h), self.device.index or 0, ctypes.c_void_p(stream.cuda_stream))
        if rc != GBS_OK:
            raise GbsError(rc, "gbs_create failed")
        self._h = h
        self._destroy = lib.gbs_destroy  # still reachable while the interpreter shuts down
        self._keep = ()
        self._coils = ()
        self._ws = None  # workspace tensor (uint8), grown on demand
        self.K = 0
        self.n_samples = 0
        self.n_coils = 1

    def _check(self, rc):
        if rc != GBS_OK:
            raise GbsError(rc, lib.gbs_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None

    __del__ = close

    def gbs_set_phantom(self, x, y, z, t1, t2, df_hz, m0):
        ts = [t.to(self.device, torch.float32).contiguous() for t in (x, y, z, t1, t2, df_hz, m0)]
        self._keep = ts  # the library keeps views of these tensors
        self._check(lib.gbs_set_phantom(self._h, ts[0].numel(), *(_ptr(t) for t in ts)))
        self.K = ts[0].numel()
        self._coils = ()
        self.n_coils = 1

    def set_phantom(self, ph):
        """From a synth.Phantom (host numpy arrays)."""
        self.gbs_set_phantom(*(torch.from_numpy(a) for a in ph.arrays()))

    def gbs_set_coils(self, sens):
        """Receive-coil sensitivities S(k, p): complex (P, K) array or tensor
        (None: one coil of unit sensitivity).  Signals then have P rows."""
        if sens is None:
            self._check(lib.gbs_set_coils(self._h, 1, None, None))
            self._coils, self.n_coils = (), 1
            return
        st = torch.as_tensor(sens)
        if st.dim() != 2 or st.shape[1] != self.K:
            raise ValueError(f"sensitivities must be (P, K={self.K}), got {tuple(st.shape)}")
        re = st.real.to(self.device, torch.float32).contiguous()
        im = (st.imag if st.is_complex() else torch.zeros_like(st.real)).to(self.device, torch.float32).contiguous()
        self._check(lib.gbs_set_coils(self._h, st.shape[0], _ptr(re), _ptr(im)))
        self._coils, self.n_coils = (re, im), st.shape[0]  # the library keeps views

    set_coils = gbs_set_coils

    def gbs_set_sequence(self, seq):
        import numpy as np
        blocks = sequence_blocks(seq)
        w = [_host(a, np.float32) for a in (seq.rf_re, seq.rf_im, seq.gx, seq.gy, seq.gz)]
        adc = _host(seq.adc_idx, np.int32)
        self._check(lib.gbs_set_sequence(self._h, blocks, seq.n_blocks, *(a.ctypes.data for a in w),
                                         seq.total_steps, adc.ctypes.data, seq.total_samples, float(seq.dt)))
        self.n_samples = seq.total_samples

    set_sequence = gbs_set_sequence

    def gbs_build_groups(self, axes=GBS_AX_ALL):
        self._check(lib.gbs_build_groups(self._h, axes))

    build_groups = gbs_build_groups

    def gbs_get_info(self):
        info = gbs_info()
        self._check(lib.gbs_get_info(self._h, ctypes.byref(info)))
        return {"K": info.K, "n_blocks": info.n_blocks, "total_steps": info.total_steps,
                "total_samples": info.total_samples, "stepped_steps": info.stepped_steps,
                "n_groups": list(info.n_groups), "groups_valid": bool(info.groups_valid),
                "n_tissue_groups": info.n_tissue_groups, "n_coils": info.n_coils,
                "n_xz_groups": info.n_xz_groups}

    info = gbs_get_info

    def gbs_workspace_size(self, mode=GBS_GROUPED):
        """Bytes of device workspace gbs_simulate needs in `mode`."""
        n = ctypes.c_size_t()
        self._check(lib.gbs_workspace_size(self._h, mode, ctypes.byref(n)))
        return int(n.value)

    workspace_size = gbs_workspace_size

    def workspace(self, mode=GBS_GROUPED):
        """A uint8 device tensor of at least the workspace size of `mode`,
        kept by this object and reused (torch's allocator owns the memory)."""
        n = self.gbs_workspace_size(mode)
        if self._ws is None or self._ws.numel() < n:
            self._ws = None
            self._ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        return self._ws

    def release_workspace(self):
        self._ws = None

    def gbs_simulate(self, mode=GBS_GROUPED, m_init=None, m_out=None, sig_out=None, flags=0,
                     stats=False, workspace=None):
        """Returns (M (3, K) float32 device tensor, signal complex128 device tensor[, stats]).
        The signal is (N,) for one coil and (P, N) after set_coils with P rows.
        workspace: a uint8 device tensor of at least gbs_workspace_size(mode)
        bytes; None uses (and grows) the one this object keeps."""
        ws = self.workspace(mode) if workspace is None else workspace
        if m_out is None:
            m_out = torch.empty(3, self.K, device=self.device, dtype=torch.float32)
        if sig_out is None:
            sig_out = torch.empty(max(self.n_coils * self.n_samples, 1), 2, device=self.device, dtype=torch.float64)
        mi = None if m_init is None else m_init.to(self.device, torch.float32).contiguous()
        st = gbs_stats() if stats else None
        self._check(lib.gbs_simulate(self._h, mode, flags, _ptr(ws), ws.numel() * ws.element_size(), _ptr(mi),
                                     _ptr(m_out), _ptr(sig_out), ctypes.byref(st) if st is not None else None))
        sig = torch.view_as_complex(sig_out)[: self.n_coils * self.n_samples]
        if self.n_coils > 1:
            sig = sig.view(self.n_coils, self.n_samples)
        return (m_out, sig, st.as_dict()) if stats else (m_out, sig)

    simulate = gbs_simulate


class Mlp:
    """A gbs_mlp network (learned RF-transition surrogate) on a HIP device."""

    def __init__(self, device=0, seed=0, stream=None):
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        rc = lib.gbs_mlp_create(ctypes.byref(h), self.device.index or 0, ctypes.c_void_p(stream.cuda_stream),
                                int(seed))
        if rc != GBS_OK:
            raise GbsError(rc, "gbs_mlp_create failed")
        self._h = h
        self._destroy = lib.gbs_mlp_destroy

    def _check(self, rc):
        if rc != GBS_OK:
            raise GbsError(rc, lib.gbs_mlp_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._destroy(self._h)
            self._h = None

    __del__ = close

    def set_pulse(self, rf, gz, dt, gx=None, gy=None):
        """rf: complex host array (T), gz: host array (T/m) of the same length."""
        import numpy as np
        rf = np.asarray(rf)
        n = rf.size
        w = [_host(a, np.float32) for a in (rf.real, rf.imag,
                                            np.zeros(n) if gx is None else gx,
                                            np.zeros(n) if gy is None else gy, gz)]
        self._check(lib.gbs_mlp_set_pulse(self._h, *(a.ctypes.data for a in w), n, float(dt)))

    def set_norm(self, center, scale):
        import numpy as np
        c, sc = _host(center, np.float32), _host(scale, np.float32)
        self._check(lib.gbs_mlp_set_norm(self._h, c.ctypes.data, sc.ctypes.data))

    def get_params(self):
        import numpy as np
        p = np.empty(GBS_MLP_PARAMS, np.float32)
        self._check(lib.gbs_mlp_get_params(self._h, p.ctypes.data, p.size))
        return p

    def set_params(self, p):
        import numpy as np
        p = _host(p, np.float32)
        self._check(lib.gbs_mlp_set_params(self._h, p.ctypes.data, p.size))

    def _tuples(self, tuples):
        return tuples.to(self.device, torch.float32).contiguous()

    def exact(self, tuples):
        """Exact FP64 transitions (n, 12) of the pulse for device/host tuples (n, 5)."""
        t = self._tuples(tuples)
        out = torch.empty(t.shape[0], 12, device=self.device, dtype=torch.float64)
        self._check(lib.gbs_mlp_exact(self._h, _ptr(t), t.shape[0], _ptr(out)))
        return out

    def infer(self, tuples):
        t = self._tuples(tuples)
        out = torch.empty(t.shape[0], 12, device=self.device, dtype=torch.float32)
        self._check(lib.gbs_mlp_infer(self._h, _ptr(t), t.shape[0], _ptr(out)))
        return out

    def loss_grad(self, tuples, T_exact):
        t = self._tuples(tuples)
        T = T_exact.to(self.device, torch.float64).contiguous()
        g = torch.empty(GBS_MLP_PARAMS, device=self.device, dtype=torch.float32)
        loss = ctypes.c_float()
        self._check(lib.gbs_mlp_loss_grad(self._h, _ptr(t), _ptr(T), t.shape[0], _ptr(g), ctypes.byref(loss)))
        return float(loss.value), g

    def train(self, tuples, T_exact, epochs=10, batch=4096, lr_max=2e-3, lr_min=1e-5, beta1=0.9,
              beta2=0.999, eps=1e-8, seed=0):
        """Adam on the GPU; returns the per-step batch losses (numpy)."""
        import numpy as np
        t = self._tuples(tuples)
        T = T_exact.to(self.device, torch.float64).contiguous()
        cfg = gbs_train_cfg(int(epochs), int(batch), float(lr_max), float(lr_min), float(beta1), float(beta2),
                            float(eps), int(seed))
        steps = int(epochs) * (t.shape[0] // int(batch))
        hist = np.zeros(max(steps, 1), np.float32)
        self._check(lib.gbs_mlp_train(self._h, _ptr(t), _ptr(T), t.shape[0], ctypes.byref(cfg),
                                      hist.ctypes.data, hist.size))
        return hist[:steps]


def set_surrogate(sim, mlp, tol=1e-3, n_check=32, seed=0):
    """Attach (or with mlp=None detach) a trained surrogate to a Simulator."""
    sim._mlp = mlp  # keep the network alive while attached
    sim._check(lib.gbs_set_surrogate(sim._h, None if mlp is None else mlp._h, float(tol), int(n_check),
                                     int(seed)))


class Adjoint:
    """Gradient of the signal of a Simulator's phantom and sequence with
    respect to a complex parameter pulse and per-class T1/T2 (gbs_adj_*)."""

    def __init__(self, sim, labels, param_blocks, every=256):
        import numpy as np
        self.sim = sim
        self.cls = torch.as_tensor(np.asarray(labels, np.int32)).to(sim.device).contiguous()
        self.param_blocks = np.ascontiguousarray(param_blocks, dtype=np.int32)
        self.every = int(every)
        self._held = None
        self.generation = 0

    def forward(self, rf, t1c, t2c):
        """rf: (n_rf, 2) float32 (re, im) in T; t1c, t2c: (C,) float32.  Returns
        the signal as a (N, 2) float64 device tensor."""
        dev = self.sim.device
        rf = rf.detach().to(dev, torch.float32).contiguous()
        t1c = t1c.detach().to(dev, torch.float32).contiguous()
        t2c = t2c.detach().to(dev, torch.float32).contiguous()
        sig = torch.empty(max(self.sim.n_samples, 1), 2, device=dev, dtype=torch.float64)
        self._held = (rf, t1c, t2c)  # the library reads these again in backward
        self.sim._check(lib.gbs_adj_forward(self.sim._h, _ptr(self.cls), t1c.numel(), _ptr(t1c), _ptr(t2c),
                                            _ptr(rf), rf.shape[0], self.param_blocks.ctypes.data,
                                            self.param_blocks.size, self.every, _ptr(sig)))
        self.generation += 1
        return sig[: self.sim.n_samples]

    def backward(self, grad_sig):
        """grad_sig: (N, 2) cotangent of the signal.  Returns (grad_rf (n_rf, 2)
        float32, grad_t1 (C,) float64, grad_t2 (C,) float64)."""
        if self._held is None:  # no forward pass yet: the library reports the call order
            self.sim._check(lib.gbs_adj_backward(self.sim._h, None, None, None, None))
        rf, t1c, _ = self._held
        dev = self.sim.device
        g = grad_sig.detach().to(dev, torch.float64).contiguous()
        grf = torch.empty_like(rf)
        g1 = torch.empty(t1c.numel(), device=dev, dtype=torch.float64)
        g2 = torch.empty_like(g1)
        self.sim._check(lib.gbs_adj_backward(self.sim._h, _ptr(g), _ptr(grf), _ptr(g1), _ptr(g2)))
        return grf, g1, g2


class BlochSignal(torch.autograd.Function):
    """signal = BlochSignal.apply(rf, t1c, t2c, adjoint): differentiable with
    respect to the parameter pulse rf (n_rf, 2) and the class T1/T2."""

    @staticmethod
    def forward(ctx, rf, t1c, t2c, adj):
        sig = adj.forward(rf, t1c, t2c)
        ctx.adj = adj
        ctx.generation = adj.generation
        ctx.dtypes = (rf.dtype, t1c.dtype, t2c.dtype)
        return sig

    @staticmethod
    def backward(ctx, grad_sig):
        adj = ctx.adj
        if adj.generation != ctx.generation:
            raise RuntimeError("the adjoint's checkpoints belong to a later forward pass")
        grf, g1, g2 = adj.backward(grad_sig)
        return grf.to(ctx.dtypes[0]), g1.to(ctx.dtypes[1]), g2.to(ctx.dtypes[2]), None


def bloch_signal(adj, rf, t1c, t2c):
    return BlochSignal.apply(rf, t1c, t2c, adj)
