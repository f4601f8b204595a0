"""CPU checks of the Python binding's argument validation: a tensor handed to
the library as a raw pointer must be complex128, on the solver's device, of
shape (rows, n_rhs) with n_rhs in range; anything else is refused before the
library reads memory through the pointer."""
import pytest

import paper_1808_04713_amd as hdp

torch = pytest.importorskip("torch")

DEV = torch.device("cpu")   # stands in for the solver's device (no GPU here)


def test_accepts_a_valid_operand():
    t = torch.zeros(7, 3, dtype=torch.complex128)
    assert hdp.check_operand(t, 7, 4, DEV, "v") is t


def test_makes_a_transposed_operand_contiguous():
    t = torch.zeros(3, 7, dtype=torch.complex128).T
    out = hdp.check_operand(t, 7, 4, DEV, "v")
    assert out.is_contiguous() and out.shape == (7, 3)


@pytest.mark.parametrize("bad", [
    torch.zeros(7, 3, dtype=torch.complex64),           # single precision
    torch.zeros(7, 3, dtype=torch.float64),             # real
    torch.zeros(21, dtype=torch.complex128),            # 1-D
    torch.zeros(6, 3, dtype=torch.complex128),          # too few rows
    torch.zeros(8, 3, dtype=torch.complex128),          # too many rows
    torch.zeros(7, 5, dtype=torch.complex128),          # more columns than the handle holds
    torch.zeros(7, 0, dtype=torch.complex128),          # no columns
])
def test_refuses_wrong_dtype_shape_or_columns(bad):
    with pytest.raises(ValueError):
        hdp.check_operand(bad, 7, 4, DEV, "v")


def test_refuses_another_device():
    t = torch.zeros(7, 3, dtype=torch.complex128)
    with pytest.raises(ValueError):
        hdp.check_operand(t, 7, 4, torch.device("cuda", 0), "v")


def test_refuses_non_tensors():
    import numpy as np
    with pytest.raises(TypeError):
        hdp.check_operand(np.zeros((7, 3), complex), 7, 4, DEV, "v")
