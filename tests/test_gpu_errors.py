"""Error behaviour of the C ABI on the GPU (through the Python binding).

Each call below must be refused with the documented status code, leave no
work on the device, and leave the context usable: the test ends every case
with a valid simulation that still matches the FP64 oracle.  The invalid
inputs are all caught by the host or by the library's own validation kernels
(which only read the inputs and set a flag); none reaches a compute kernel.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_03960_amd as gb
    return gb


def say(msg):
    print(msg, flush=True)


def code_of(gb, fn):
    with pytest.raises(gb.GbsError) as e:
        fn()
    return e.value.code


def still_works(gb, sim, ph, seq):
    """A valid grouped run on the same context, against the oracle."""
    import torch
    sim.set_phantom(ph)
    sim.set_sequence(seq)
    sim.build_groups()
    M, sig = sim.simulate(gb.GBS_GROUPED)
    torch.cuda.synchronize()
    Mr, sr = oracle.simulate(ph, seq)
    dm = float(np.max(np.abs(M.cpu().numpy().astype(np.float64) - Mr)))
    rel = float(np.linalg.norm(sig.cpu().numpy() - sr) / np.linalg.norm(sr))
    assert dm <= 1e-5 and rel <= 1e-4, (dm, rel)


def small():
    ph = synth.tiny_phantom(nx=6, ny=5, nz=2)
    seq = synth.gre_sequence(n_lines=2, n_read=8, dwell_steps=2, rf_steps=200, te=1.5e-3, tr=4e-3)
    return ph, seq


def test_call_order(gb):
    ph, seq = small()
    sim = gb.Simulator(0)
    say("[gpu] errors: coils before a phantom")
    assert code_of(gb, lambda: sim.set_coils(None)) == gb.GBS_E_STATE
    say("[gpu] errors: simulate / build_groups before their inputs")
    assert code_of(gb, lambda: sim.simulate(gb.GBS_PLAIN)) == gb.GBS_E_STATE
    assert code_of(gb, lambda: sim.build_groups()) == gb.GBS_E_STATE
    sim.set_phantom(ph)
    assert code_of(gb, lambda: sim.simulate(gb.GBS_PLAIN)) == gb.GBS_E_STATE  # no sequence yet
    sim.set_sequence(seq)
    assert code_of(gb, lambda: sim.simulate(gb.GBS_GROUPED)) == gb.GBS_E_STATE  # no groups yet
    sim.build_groups()
    sim.set_phantom(ph)  # groups are stale now
    assert code_of(gb, lambda: sim.simulate(gb.GBS_GROUPED)) == gb.GBS_E_STATE
    assert code_of(gb, lambda: sim.simulate(7)) == gb.GBS_E_INVALID  # no such mode
    assert code_of(gb, lambda: sim.build_groups(gb.GBS_AX_Y)) == gb.GBS_E_INVALID  # x axis is required
    assert code_of(gb, lambda: sim.build_groups(gb.GBS_AX_X | gb.GBS_AX_XZ)) == gb.GBS_E_INVALID  # needs z
    assert code_of(gb, lambda: sim.build_groups(gb.GBS_AX_ALL | 32)) == gb.GBS_E_INVALID  # unknown bit
    # GBS_SURROGATE without a network, or with the plain mode; flag 2 (a removed FP32 plain
    # option) is unknown
    sim.build_groups()
    assert code_of(gb, lambda: sim.simulate(gb.GBS_GROUPED, flags=gb.GBS_SURROGATE)) == gb.GBS_E_INVALID
    assert code_of(gb, lambda: sim.simulate(gb.GBS_CACHED, flags=gb.GBS_SURROGATE)) == gb.GBS_E_INVALID
    assert code_of(gb, lambda: sim.simulate(gb.GBS_PLAIN, flags=gb.GBS_SURROGATE)) == gb.GBS_E_INVALID
    assert code_of(gb, lambda: sim.simulate(gb.GBS_PLAIN, flags=2)) == gb.GBS_E_INVALID
    still_works(gb, sim, ph, seq)
    sim.close()


def test_invalid_phantom_and_sequence(gb):
    ph, seq = small()
    sim = gb.Simulator(0)
    for what, field, value in (("NaN x", "x", np.nan), ("T1 = 0", "t1", 0.0), ("T2 < 0", "t2", -1.0),
                               ("inf df", "df", np.inf)):
        bad = synth.Phantom(ph.x.copy(), ph.y.copy(), ph.z.copy(), ph.t1.copy(), ph.t2.copy(), ph.df.copy(),
                            ph.m0.copy())
        getattr(bad, field)[3] = value
        say(f"[gpu] errors: phantom with {what}")
        assert code_of(gb, lambda: sim.set_phantom(bad)) == gb.GBS_E_INVALID
    bad_seq = synth.Sequence(**{f: getattr(seq, f) for f in seq.__dataclass_fields__})
    bad_seq.gz = np.array(seq.gz, np.float32)
    bad_seq.gz[5] = np.nan
    say("[gpu] errors: sequence with a NaN gradient sample")
    assert code_of(gb, lambda: sim.set_sequence(bad_seq)) == gb.GBS_E_INVALID
    still_works(gb, sim, ph, seq)
    sim.close()


def test_adjoint_limits(gb):
    import torch
    ph, t1c, t2c, seq, rf, pb = synth.adjoint_workload(8, 8, 2, n_lines=2, n_read=16, rf_steps=400)
    sim = gb.Simulator(0)
    sim.set_phantom(ph)
    sim.set_sequence(seq)
    rft = torch.tensor(np.stack([rf.real, rf.imag], 1), dtype=torch.float32, device="cuda")
    t1 = torch.tensor(t1c, dtype=torch.float32, device="cuda")
    t2 = torch.tensor(t2c, dtype=torch.float32, device="cuda")
    w = torch.zeros(seq.total_samples, 2, dtype=torch.float64, device="cuda")

    say("[gpu] errors: adjoint backward before forward")
    adj = gb.Adjoint(sim, ph.labels, pb, every=64)
    assert code_of(gb, lambda: adj.backward(w)) == gb.GBS_E_STATE
    say("[gpu] errors: adjoint checkpoint interval, pulse length, class index, T <= 0, blocks")
    for every in (12, 0, 512):
        a = gb.Adjoint(sim, ph.labels, pb, every=every)
        assert code_of(gb, lambda: a.forward(rft, t1, t2)) == gb.GBS_E_INVALID
    long_rf = torch.zeros(4000, 2, dtype=torch.float32, device="cuda")
    assert code_of(gb, lambda: adj.forward(long_rf, t1, t2)) == gb.GBS_E_INVALID
    bad_labels = ph.labels.copy()
    bad_labels[0] = t1c.size  # one past the last class
    a = gb.Adjoint(sim, bad_labels, pb, every=64)
    assert code_of(gb, lambda: a.forward(rft, t1, t2)) == gb.GBS_E_INVALID
    t1_bad = t1.clone()
    t1_bad[1] = 0.0
    assert code_of(gb, lambda: adj.forward(rft, t1_bad, t2)) == gb.GBS_E_INVALID
    relax_block = np.nonzero(np.asarray(seq.btype) != synth.BLOCK_RF)[0][:1].astype(np.int32)
    a = gb.Adjoint(sim, ph.labels, relax_block, every=64)
    assert code_of(gb, lambda: a.forward(rft, t1, t2)) == gb.GBS_E_INVALID
    # the context still computes a correct gradient afterwards
    sig = adj.forward(rft, t1, t2)
    grf, g1, _ = adj.backward(torch.ones(seq.total_samples, 2, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    rf32 = rf.real.astype(np.float32) + 1j * rf.imag.astype(np.float32)
    wv = np.ones(seq.total_samples) * (1 + 1j)
    s_o, g_o, g1_o, _ = oracle.adjoint(ph, ph.labels, np.float32(t1c), np.float32(t2c), seq, rf32, pb, wv)
    s = sig.cpu().numpy()
    g = grf.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(s[:, 0] + 1j * s[:, 1] - s_o) <= 1e-4 * np.linalg.norm(s_o)
    assert np.linalg.norm(g[:, 0] + 1j * g[:, 1] - g_o) <= 2e-3 * np.linalg.norm(g_o)
    sim.close()


def test_workspace_contract(gb):
    """gbs_simulate takes its scratch from the caller: a workspace of
    gbs_workspace_size bytes (256-byte aligned) works in every mode, and its
    previous contents do not matter; a null, short or misaligned one is
    refused with GBS_E_WORKSPACE before any work."""
    import ctypes
    import torch
    ph, seq = small()
    Mr, sr = oracle.simulate(ph, seq)
    sim = gb.Simulator(0)
    say("[gpu] workspace: size before a sequence")
    sim.set_phantom(ph)
    assert code_of(gb, lambda: sim.workspace_size(gb.GBS_PLAIN)) == gb.GBS_E_STATE
    sim.set_sequence(seq)
    assert code_of(gb, lambda: sim.workspace_size(gb.GBS_GROUPED)) == gb.GBS_E_STATE  # no groups yet
    sim.build_groups()
    m_out = torch.empty(3, ph.K, device="cuda", dtype=torch.float32)
    sig = torch.empty(seq.total_samples, 2, device="cuda", dtype=torch.float64)
    for mode in (gb.GBS_PLAIN, gb.GBS_GROUPED, gb.GBS_CACHED):
        need = sim.workspace_size(mode)
        say(f"[gpu] workspace: mode {mode} needs {need} bytes for K={ph.K}")
        assert need > 0
        big = torch.empty(need + 512, dtype=torch.uint8, device="cuda")
        for fill in (0, 255):  # scratch: whatever it held before must not matter
            big.fill_(fill)
            ws = big[:need]
            M, s = sim.simulate(mode, workspace=ws, m_out=m_out, sig_out=sig)
            torch.cuda.synchronize()
            dm = float(np.max(np.abs(M.cpu().numpy().astype(np.float64) - Mr)))
            rel = float(np.linalg.norm(s.cpu().numpy() - sr) / np.linalg.norm(sr))
            assert dm <= 1e-5 and rel <= 1e-4, (mode, fill, dm, rel)
        say(f"[gpu] workspace: short, misaligned and null workspaces in mode {mode}")
        assert code_of(gb, lambda: sim.simulate(mode, workspace=big[:need - 1])) == gb.GBS_E_WORKSPACE
        assert code_of(gb, lambda: sim.simulate(mode, workspace=big[8:need + 8])) == gb.GBS_E_WORKSPACE
        rc = gb.lib.gbs_simulate(sim._h, mode, 0, None, 0, None, ctypes.c_void_p(m_out.data_ptr()),
                                 ctypes.c_void_p(sig.data_ptr()), None)
        assert rc == gb.GBS_E_WORKSPACE
        # straight through the C ABI with a workspace of its own
        rc = gb.lib.gbs_simulate(sim._h, mode, 0, ctypes.c_void_p(big.data_ptr()), need, None,
                                 ctypes.c_void_p(m_out.data_ptr()), ctypes.c_void_p(sig.data_ptr()), None)
        assert rc == gb.GBS_OK, gb.lib.gbs_last_error(sim._h)
        torch.cuda.synchronize()
        assert float(np.max(np.abs(m_out.cpu().numpy().astype(np.float64) - Mr))) <= 1e-5
    # a larger phantom needs more, and the same context still computes it right
    ph2 = synth.tiny_phantom(nx=12, ny=9, nz=3)
    sim.set_phantom(ph2)
    sim.build_groups()
    assert sim.workspace_size(gb.GBS_CACHED) > need
    still_works(gb, sim, ph2, seq)
    sim.close()
