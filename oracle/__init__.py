"""FP64 CPU oracle of the plain and grouped Bloch simulation.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  Nothing here imports, links or shares
code with the GPU library; both sides only read the same seeded inputs from
``synth``.

* ``simulate`` wraps the plain per-isochromat C oracle (``bloch_oracle.c``):
  raster stepping with U = D*R (Eq. 2, Eq. A1, Eq. A2), closed-form
  relaxation blocks (Eq. 4, Eq. 5) and the k-space sum (Eq. 6).
* ``simulate_coils`` gives the signal of P receive coils (Eq. 6 with
  S(k, p)): every isochromat is simulated on its own by ``simulate`` (its
  signal is its Mxy at the sample instants) and the coil signals are the
  S-weighted sums of those.  For tiny phantoms only.
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
ADJ_PATH = os.path.join(_HERE, "bloch_adjoint.c")

_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc + OpenMP into oracle/liboracle.so."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               SRC_PATH, ADJ_PATH, "-o", tmp, "-lm"]
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
    if hasattr(lib, "oracle_adjoint"):
        lib.oracle_adjoint.restype = ctypes.c_int
        lib.oracle_adjoint.argtypes = (
            [ctypes.c_int64] + [P] * 6 + [ctypes.c_int32, P, P, ctypes.c_int64] + [P] * 7
            + [ctypes.c_int64] + [P] * 5 + [ctypes.c_int64, P, ctypes.c_double, ctypes.c_int64, P,
                                             ctypes.c_int32, P, P, ctypes.c_int, P, P, P, P])
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < max(
                os.path.getmtime(SRC_PATH), os.path.getmtime(ADJ_PATH)):
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


def adjoint(ph, cls, t1c, t2c, seq, rf_param, param_blocks, w, nthreads: int = 0, lib=None):
    """FP64 signal and gradient of L = sum_n (w_re Re A_n + w_im Im A_n)
    (``bloch_adjoint.c``).

    ph: phantom (its t1/t2 are ignored: isochromat k has T1 = t1c[cls[k]],
    T2 = t2c[cls[k]]); rf_param: complex (n_rf,), the B1 of every block in
    ``param_blocks``; w: complex (total_samples,).  Returns
    (sig complex, g_rf complex (n_rf,) = dL/dRe + i dL/dIm, g_t1, g_t2)."""
    lib = lib or _load()
    K = ph.K
    x, y, z, _, _, df, m0 = (_f64(a) for a in ph.arrays())
    cls = np.ascontiguousarray(cls, dtype=np.int32)
    t1c, t2c = _f64(t1c), _f64(t2c)
    C = t1c.size
    rf_re, rf_im, gx, gy, gz = (_f64(a) for a in (seq.rf_re, seq.rf_im, seq.gx, seq.gy, seq.gz))
    btype = np.ascontiguousarray(seq.btype, dtype=np.int32)
    i64 = [np.ascontiguousarray(a, dtype=np.int64) for a in (seq.step_offset, seq.n_steps, seq.n_samples,
                                                            seq.sample_offset)]
    tau, mom = _f64(seq.tau), _f64(np.asarray(seq.moment).reshape(-1, 3))
    adc = np.ascontiguousarray(seq.adc_idx, dtype=np.int32)
    rp = np.asarray(rf_param, dtype=np.complex128)
    n_rf = rp.size
    rpi = _f64(np.stack([rp.real, rp.imag], 1).ravel())
    pb = np.ascontiguousarray(param_blocks, dtype=np.int32)
    wv = np.asarray(w, dtype=np.complex128)
    wi = _f64(np.stack([wv.real, wv.imag], 1).ravel())
    N = seq.total_samples
    sig = np.zeros(2 * max(N, 1))
    g_rf = np.zeros(2 * max(n_rf, 1))
    g1, g2 = np.zeros(C), np.zeros(C)
    d = lambda a: a.ctypes.data
    rc = lib.oracle_adjoint(K, d(x), d(y), d(z), d(df), d(m0), d(cls), C, d(t1c), d(t2c), seq.n_blocks,
                            d(btype), *(d(a) for a in i64), d(tau), d(mom), seq.total_steps,
                            d(rf_re), d(rf_im), d(gx), d(gy), d(gz), N, d(adc), float(seq.dt), n_rf,
                            d(pb), pb.size, d(rpi), d(wi), nthreads, d(sig), d(g_rf), d(g1), d(g2))
    if rc != 0:
        raise ValueError(f"oracle_adjoint rejected its input ({rc})")
    return (sig[0:2 * N:2] + 1j * sig[1:2 * N:2], g_rf[0:2 * n_rf:2] + 1j * g_rf[1:2 * n_rf:2], g1, g2)


def simulate_coils(ph, seq, sens, m_init=None):
    """Signals of P receive coils, Eq. (6): A(p, t_n) = sum_k S(k, p) Mxy(k, t_n).

    ``sens`` is complex (P, K).  Each isochromat k is simulated alone, which
    gives Mxy(k, t_n) at every sample; the coil signals weight and add those.
    Returns ``(M, sig)`` with M float64 (3, K) and sig complex128 (P, N).
    """
    sens = np.asarray(sens, np.complex128)
    K = ph.K
    assert sens.ndim == 2 and sens.shape[1] == K
    mi = None if m_init is None else np.asarray(m_init, np.float64).reshape(3, K)
    M = np.zeros((3, K))
    sig = np.zeros((sens.shape[0], seq.total_samples), np.complex128)
    for k in range(K):
        Mk, sk = simulate(ph.subset(np.array([k])), seq, m_init=None if mi is None else mi[:, k:k + 1], nthreads=1)
        M[:, k] = Mk[:, 0]
        sig += sens[:, k:k + 1] * sk[None, :]
    return M, sig
