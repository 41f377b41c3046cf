"""Argument checks of the Python binding (no GPU): tensors the library would
read or write through a raw pointer must have the matrix's dtype and size,
be contiguous and live on the context's device; workspaces are uint8."""
import pytest
import torch

from paper_1501_03358_amd import krs


def test_check_vec_accepts_a_matching_vector():
    krs.check_vec(torch.zeros(12, dtype=torch.float64), 12, torch.float64, "cpu", "b")


@pytest.mark.parametrize("t,match", [
    (torch.zeros(12, dtype=torch.float32), "dtype"),
    (torch.zeros(11, dtype=torch.float64), "values"),
    (torch.zeros(24, dtype=torch.float64)[::2], "contiguous"),
])
def test_check_vec_rejects(t, match):
    with pytest.raises(ValueError, match=match):
        krs.check_vec(t, 12, torch.float64, "cpu", "b")


def test_check_vec_rejects_another_device_and_none():
    with pytest.raises(ValueError, match="is on"):
        krs.check_vec(torch.zeros(12, dtype=torch.float64), 12, torch.float64, "cuda:0", "x")
    with pytest.raises(ValueError, match="None"):
        krs.check_vec(None, 12, torch.float64, "cpu", "x")


def test_check_ws():
    krs.check_ws(torch.empty(64, dtype=torch.uint8), 64, "cpu")
    with pytest.raises(ValueError, match="uint8"):
        krs.check_ws(torch.empty(64, dtype=torch.float32), 1, "cpu")
    with pytest.raises(ValueError, match="bytes"):
        krs.check_ws(torch.empty(8, dtype=torch.uint8), 64, "cpu")
    with pytest.raises(ValueError, match="is on"):
        krs.check_ws(torch.empty(64, dtype=torch.uint8), 1, "cuda:0")
