"""The binding checks every device buffer before its address reaches the
library, which writes through raw addresses: a CPU, mistyped, strided or
short tensor raises ValueError in Python and never reaches a kernel.  Runs
on the host with a stand-in context (no device call is made)."""
import types

import pytest

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def qbe():
    import paper_2004_10892_amd as q
    return q


def fake_ctx():
    return types.SimpleNamespace(device=0, handle=None)


def test_contract_async_rejects_host_buffers(qbe):
    ws = torch.empty(16, dtype=torch.uint8)
    out = torch.zeros(2, dtype=torch.float64)
    with pytest.raises(ValueError, match="cuda:0"):
        qbe.qbe_contract_async(fake_ctx(), None, ws, out)


def test_dev_buffer_rejects_wrong_dtype_short_and_strided(qbe):
    meta = torch.empty(4, dtype=torch.float32, device="meta")
    # the device check comes first; a tensor on another device type fails it
    with pytest.raises(ValueError, match="must live on"):
        qbe._dev_buffer(fake_ctx(), meta, "d_out", torch.float64, 2)
    with pytest.raises(ValueError, match="torch tensor"):
        qbe._dev_buffer(fake_ctx(), [0.0, 0.0], "d_out", torch.float64, 2)


def test_batch_contract_async_rejects_host_amplitudes(qbe):
    batch = qbe.Batch.__new__(qbe.Batch)
    batch.ctx = fake_ctx()
    batch.plans = [None, None]
    batch.handle = None
    with pytest.raises(ValueError):
        batch.contract_async(torch.empty(8, dtype=torch.uint8), torch.zeros(4, dtype=torch.float64))


def test_permute_rejects_host_tensors(qbe):
    x = torch.zeros(16, dtype=torch.complex64)
    with pytest.raises(ValueError, match="cuda:0"):
        qbe.qbe_permute(fake_ctx(), x, x.clone(), 4, [0, 1, 2, 3])


def test_checks_on_device_like_tensors(qbe, monkeypatch):
    """dtype, contiguity and length checks, with the device check satisfied
    by a stand-in that reports cuda:0 (no memory is touched)."""
    class T:
        def __init__(self, dtype, n, contiguous=True):
            self.device = torch.device("cuda", 0)
            self.dtype = dtype
            self._n = n
            self._c = contiguous

        def is_contiguous(self):
            return self._c

        def numel(self):
            return self._n

        def data_ptr(self):
            return 4096

    monkeypatch.setattr(torch, "Tensor", T)
    ctx = fake_ctx()
    assert qbe._dev_buffer(ctx, T(torch.float64, 2), "d_out", torch.float64, 2).value == 4096
    with pytest.raises(ValueError, match="float64"):
        qbe._dev_buffer(ctx, T(torch.float32, 4), "d_out", torch.float64, 2)
    with pytest.raises(ValueError, match="at least 2"):
        qbe._dev_buffer(ctx, T(torch.float64, 1), "d_out", torch.float64, 2)
    with pytest.raises(ValueError, match="contiguous"):
        qbe._dev_buffer(ctx, T(torch.float64, 2, contiguous=False), "d_out", torch.float64, 2)
    other = T(torch.float64, 2)
    other.device = torch.device("cuda", 1)
    with pytest.raises(ValueError, match="cuda:0"):
        qbe._dev_buffer(ctx, other, "d_out", torch.float64, 2)
