"""Plant plausible mistakes in copies of the surrogate oracle's reference
transition and show that its pins (tests/surrogate_pins.py) catch each one.

CPU only.  Each mutant is oracle/surrogate.py with one textual change, loaded
as a separate module from a temporary directory; the real oracle is never
modified.
"""
import importlib.util
import os

import pytest

from oracle import surrogate as so
from tests import surrogate_pins as spins

MUTANTS = {
    "no_b1_scaling": ("h = 0.5 * t[:, 4] * th", "h = 0.5 * th"),
    "one_sided_relaxation": ("A = d[:, :, None] * R * d[:, None, :]", "A = d[:, :, None] * R"),
    "recovery_not_rotated": ("b = (1 - e1)[:, None] * (d * R[:, :, 2])", "b = (1 - e1)[:, None] * (d * R[:, 2, :])"),
    "quaternion_vector_sign": ("q = [w, (R[2, 1] - R[1, 2]) / (4 * w)", "q = [w, (R[1, 2] - R[2, 1]) / (4 * w)"),
    "axis_not_interpolated": ("n = (1 - w)[:, None] * axis[i0] + w[:, None] * axis[i0 + 1]", "n = axis[i0]"),
    "angle_not_halved": ("h = 0.5 * t[:, 4] * th", "h = t[:, 4] * th"),
    "residual_unscaled": ("Y / RESIDUAL_SCALE, tuples, half, inverse=True)", "Y, tuples, half, inverse=True)"),
}


@pytest.fixture(scope="module")
def source():
    with open(so.__file__) as f:
        return f.read()


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_surrogate_mutant_is_caught(name, source, tmp_path):
    old, new = MUTANTS[name]
    assert source.count(old) == 1, f"mutation anchor for {name} not unique"
    path = tmp_path / f"surrogate_{name}.py"
    path.write_text(source.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"surrogate_{name}", str(path))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    failed = []
    for check in spins.CHECKS:
        try:
            check(mod)
        except AssertionError:
            failed.append(check.__name__)
    assert failed, f"no pin detects mutant {name}"
    os.remove(path)
