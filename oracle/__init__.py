"""FP64 CPU oracle of the plain and grouped Bloch simulation.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here imports, links or shares
code with the GPU library; both sides only read the same seeded inputs from
``synth``.

* ``simulate`` wraps the plain per-isochromat C oracle (``bloch_oracle.c``):
  raster stepping with U = D*R (Eq. 2, Eq. A1, Eq. A2), closed-form
  relaxation blocks (Eq. 4, Eq. 5) and the k-space sum (Eq. 6).
* ``oracle.grouped.simulate_grouped`` is a brute-force FP64 transcription of
  the grouped method (Sec. 2.3 and 2.4) for tiny phantoms.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "bloch_oracle.c")

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc + OpenMP into oracle/liboracle.so."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               SRC_PATH, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def bind(path: str):
    """Load an oracle shared library built from ``bloch_oracle.c`` (or a
    deliberately altered copy of it, for the mutation tests)."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.oracle_simulate.restype = ctypes.c_int
    lib.oracle_simulate.argtypes = (
        [ctypes.c_int64] + [P] * 8 + [ctypes.c_int64] + [P] * 7 + [ctypes.c_int64] + [P] * 5
        + [ctypes.c_int64, P, ctypes.c_double, ctypes.c_int, P, P])
    lib.oracle_max_threads.restype = ctypes.c_int
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
            build()
        _lib = bind(LIB_PATH)
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def simulate(ph, seq, m_init=None, nthreads: int = 0, lib=None):
    """Plain FP64 simulation of phantom ``ph`` under sequence ``seq``.

    Returns ``(M, sig)``: M is float64 (3, K) = (Mx, My, Mz); sig is complex128
    of length ``seq.total_samples``.
    """
    lib = lib or _load()
    K = ph.K
    arrs = [_f64(a) for a in ph.arrays()]
    mi = None if m_init is None else _f64(np.asarray(m_init).reshape(3, K))
    rf_re, rf_im, gx, gy, gz = (_f64(a) for a in (seq.rf_re, seq.rf_im, seq.gx, seq.gy, seq.gz))
    bt = np.ascontiguousarray(seq.btype, np.int32)
    so = np.ascontiguousarray(seq.step_offset, np.int64)
    ns = np.ascontiguousarray(seq.n_steps, np.int64)
    nsm = np.ascontiguousarray(seq.n_samples, np.int32)
    sof = np.ascontiguousarray(seq.sample_offset, np.int64)
    tau = _f64(seq.tau)
    mom = _f64(seq.moment).reshape(-1)
    adc = np.ascontiguousarray(seq.adc_idx, np.int32)
    m_out = np.zeros((3, K), np.float64)
    sig = np.zeros(2 * max(seq.total_samples, 0), np.float64)
    p = lambda a: None if a is None else a.ctypes.data
    rc = lib.oracle_simulate(
        K, *(p(a) for a in arrs), p(mi),
        seq.n_blocks, p(bt), p(so), p(ns), p(nsm), p(sof), p(tau), p(mom),
        seq.total_steps, p(rf_re), p(rf_im), p(gx), p(gy), p(gz),
        seq.total_samples, p(adc), float(seq.dt), int(nthreads), p(m_out), p(sig))
    if rc != 0:
        raise ValueError(f"oracle_simulate rejected its inputs (code {rc})")
    return m_out, sig[0::2] + 1j * sig[1::2]
