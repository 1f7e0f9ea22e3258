"""CPU checks of the binding's tensor validation (no GPU needed): every
tensor whose address goes to the library is checked for type, dtype, size,
device and layout first."""
import pytest

torch = pytest.importorskip("torch")


def _check():
    from paper_1502_02294_amd import check_tensor
    return check_tensor


def test_accepts_and_copies_noncontiguous():
    ct = _check()
    t = torch.zeros(8, 8, 8, dtype=torch.float32)
    assert ct(t, "g", dtypes=(torch.float32,), numel=512, device=torch.device("cpu")) is t
    nc = torch.zeros(8, 16, 8)[:, ::2, :]
    assert not nc.is_contiguous()
    out = ct(nc, "g", dtypes=(torch.float32,), numel=512, device=torch.device("cpu"))
    assert out.is_contiguous() and out.shape == nc.shape
    with pytest.raises(ValueError, match="contiguous"):
        ct(nc, "out", dtypes=(torch.float32,), numel=512, device=torch.device("cpu"), copy_ok=False)


@pytest.mark.parametrize("bad,exc,msg", [
    (torch.zeros(512, dtype=torch.float16), TypeError, "dtype"),
    (torch.zeros(511, dtype=torch.float32), ValueError, "elements"),
    ([0.0] * 512, TypeError, "torch.Tensor"),
    (torch.zeros(512, dtype=torch.int32), TypeError, "dtype"),
])
def test_rejects_wrong_type_dtype_size(bad, exc, msg):
    ct = _check()
    with pytest.raises(exc, match=msg):
        ct(bad, "grid", dtypes=(torch.float32, torch.float64), numel=512, device=torch.device("cpu"))


def test_rejects_host_tensor_for_device_only_argument():
    ct = _check()
    t = torch.zeros(512, dtype=torch.float32)
    dev = torch.device("cuda", 0)
    with pytest.raises(ValueError, match="host memory"):
        ct(t, "step source", dtypes=(torch.float32,), numel=512, device=dev)
    assert ct(t, "pushed grid", dtypes=(torch.float32,), numel=512, device=dev, allow_host=True) is t
