"""The binding refuses tensors the C ABI would misread: it passes bare device
pointers and the library assumes contiguous float32 D [H, W] and uint8
M [V, H, W] on the context's device.  Checked here on host tensors (no GPU
needed): every rejection is raised before any pointer is handed over."""
import pytest

torch = pytest.importorskip("torch")

from paper_2408_14050_amd.occl import check_frame, check_tensor  # noqa: E402


def test_rejects_wrong_dimensions():
    with pytest.raises(ValueError, match="dimensions"):
        check_frame(torch.zeros(3, 4, 5), torch.zeros(1, 4, 5, dtype=torch.uint8), 1)


def test_rejects_wrong_dtype_of_D():
    with pytest.raises(ValueError, match="float32"):
        check_frame(torch.zeros(4, 5, dtype=torch.float64), torch.zeros(1, 4, 5, dtype=torch.uint8), 1)


def test_rejects_non_contiguous_D():
    D = torch.zeros(4, 10)[:, ::2]  # a column slice: row stride 10, not W = 5
    with pytest.raises(ValueError, match="contiguous"):
        check_frame(D, torch.zeros(1, 4, 5, dtype=torch.uint8), 1)


def test_rejects_host_tensor():
    with pytest.raises(ValueError, match="device tensor"):
        check_frame(torch.zeros(4, 5), torch.zeros(1, 4, 5, dtype=torch.uint8), 1)


def test_rejects_wrong_mask_dtype():
    D = torch.zeros(4, 5)
    with pytest.raises(ValueError, match="uint8"):
        check_tensor(torch.zeros(1, 4, 5, dtype=torch.int32), "M", torch.uint8, shape=(1, 4, 5))
    with pytest.raises(ValueError):
        check_frame(D, torch.zeros(1, 4, 5, dtype=torch.int32), 1)


def test_rejects_short_mask():
    # the D check fails first on a host tensor, so check M's shape alone
    with pytest.raises(ValueError, match="shape"):
        check_tensor(torch.zeros(1, 4, 5, dtype=torch.uint8), "M", torch.uint8, shape=(8, 4, 5))
    with pytest.raises(ValueError, match="shape"):
        check_tensor(torch.zeros(8, 4, 4, dtype=torch.uint8), "M", torch.uint8, shape=(8, 4, 5))


def test_rejects_non_contiguous_mask():
    M = torch.zeros(2, 4, 5, dtype=torch.uint8).transpose(1, 2).contiguous().transpose(1, 2)
    assert tuple(M.shape) == (2, 4, 5) and not M.is_contiguous()
    with pytest.raises(ValueError, match="contiguous"):
        check_tensor(M, "M", torch.uint8, shape=(2, 4, 5))


def test_rejects_none():
    with pytest.raises(ValueError, match="None"):
        check_tensor(None, "D", torch.float32)
