"""GPU parity on the four pulse sequences of the paper's Table 2 (reduced in
lines and pulse length, same block structure): plain, grouped and cached
modes against the FP64 oracle, at the bar of the other parity tests."""
import pytest

import oracle
import synth
from tests.test_gpu_parity import check_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2508_03960_amd as gb
    return gb


@pytest.mark.parametrize("name", ["t1w-se", "t2w-se", "se-epi", "fse-etl5"])
def test_table2_sequence(gb, name):
    ph = synth.brain_like_phantom(48, 40, 3)
    seq = synth.table2_sequences(small=True)[name]
    ref = oracle.simulate(ph, seq)
    check_case(gb, f"table2:{name}", ph, seq, modes=("plain", "grouped", "cached"), ref=ref)
