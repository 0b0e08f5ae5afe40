"""gbs_simulate_static (the workspace is the library's static device array)
against gbs_simulate with a caller workspace, through the C ABI: every mode
on a phantom, then on a smaller one (the array keeps the first call's
contents, which must not matter), each also against the FP64 oracle; and a
call whose workspace would not fit the array is refused."""
import ctypes

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


def vp(t):
    return ctypes.c_void_p(t.data_ptr())


def run(gb, sim, mode, static):
    """One call through the C ABI; returns (M float64 (3, K), complex signal)."""
    import torch
    m_out = torch.full((3, sim.K), np.nan, device="cuda", dtype=torch.float32)
    sig = torch.full((max(sim.n_samples, 1), 2), np.nan, device="cuda", dtype=torch.float64)
    if static:
        rc = gb.lib.gbs_simulate_static(sim._h, mode, 0, None, vp(m_out), vp(sig), None)
    else:
        ws = torch.empty(sim.workspace_size(mode), dtype=torch.uint8, device="cuda")
        rc = gb.lib.gbs_simulate(sim._h, mode, 0, vp(ws), ws.numel(), None, vp(m_out), vp(sig), None)
    assert rc == gb.GBS_OK, (rc, gb.lib.gbs_last_error(sim._h))
    torch.cuda.synchronize()
    s = sig.cpu().numpy()[: sim.n_samples]
    return m_out.cpu().numpy().astype(np.float64), s[:, 0] + 1j * s[:, 1]


def errors(M, s, Mr, sr):
    return float(np.max(np.abs(M - Mr))), float(np.linalg.norm(s - sr) / np.linalg.norm(sr))


def test_static_workspace_matches_caller_workspace(gb):
    seq = synth.gre_sequence(n_lines=4, n_read=16, dwell_steps=4, rf_steps=400, te=2e-3, tr=8e-3)
    for ph in (synth.gre_phantom(40, 36, 3, seed=2), synth.gre_phantom(9, 7, 2, seed=3)):  # then smaller
        Mr, sr = oracle.simulate(ph, seq)
        sim = gb.Simulator(0)
        sim.set_phantom(ph)
        sim.set_sequence(seq)
        sim.build_groups()
        for mode in (gb.GBS_GROUPED, gb.GBS_CACHED, gb.GBS_PLAIN):
            say(f"[gpu] static scratch: K={ph.K} mode {mode}, workspace {sim.workspace_size(mode)} bytes")
            assert sim.workspace_size(mode) <= gb.GBS_STATIC_WORKSPACE_BYTES
            Ms, ss = run(gb, sim, mode, static=True)
            Mw, sw = run(gb, sim, mode, static=False)
            dm, rel = errors(Ms, ss, Mw, sw)
            dmo, relo = errors(Ms, ss, Mr, sr)
            say(f"[gpu] static vs caller workspace: max|dM|={dm:.2e} rel={rel:.2e}; vs oracle {dmo:.2e} {relo:.2e}")
            assert dm <= 1e-5 and rel <= 1e-4, (ph.K, mode, dm, rel)
            assert dmo <= 1e-5 and relo <= 1e-4, (ph.K, mode, dmo, relo)
        sim.close()


def test_static_workspace_refuses_what_does_not_fit(gb):
    import torch
    ph = synth.brain_like_phantom(512, 512, 10)  # grouped workspace: about 28 B x 2.7M slots > 64 MiB
    seq = synth.gre_sequence(n_lines=2, n_read=8, dwell_steps=2, rf_steps=200, te=1.5e-3, tr=4e-3)
    sim = gb.Simulator(0)
    sim.set_phantom(ph)
    sim.set_sequence(seq)
    sim.build_groups()
    need = sim.workspace_size(gb.GBS_GROUPED)
    say(f"[gpu] static scratch: K={ph.K} needs {need} bytes, the array holds {gb.GBS_STATIC_WORKSPACE_BYTES}")
    assert need > gb.GBS_STATIC_WORKSPACE_BYTES
    m_out = torch.empty(3, ph.K, device="cuda", dtype=torch.float32)
    sig = torch.empty(seq.total_samples, 2, device="cuda", dtype=torch.float64)
    rc = gb.lib.gbs_simulate_static(sim._h, gb.GBS_GROUPED, 0, None, vp(m_out), vp(sig), None)
    assert rc == gb.GBS_E_WORKSPACE
    assert str(need).encode() in gb.lib.gbs_last_error(sim._h)
    M, s = sim.simulate(gb.GBS_GROUPED)  # the context still runs with a caller workspace
    torch.cuda.synchronize()
    assert np.isfinite(M.cpu().numpy()).all()
    sim.close()
