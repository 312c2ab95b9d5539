"""mlp_forward_static, the network's inference entry point for callers that
cannot allocate device memory: through the C ABI, its outputs equal those of
mlp_forward bit for bit, on two calls in a row (the second smaller, over the
array the first call left behind), and it refuses batches beyond its array."""
import numpy as np
import pytest

from paper_0705_0497_amd import binding as B

pytestmark = pytest.mark.gpu


def test_static_forward_equals_forward_on_two_calls():
    import torch
    torch.cuda.set_device(0)
    rng = np.random.default_rng(77)
    params = (rng.standard_normal(B.MLP_NPARAM) * 0.05).astype(np.float32)
    net = B.Network(max_batch=B.MLP_STATIC_MAX_BATCH, params=params)
    stream = net.stream
    for batch in (B.MLP_STATIC_MAX_BATCH, 777):
        print(f"mlp_forward_static batch {batch}", flush=True)
        x = torch.tensor(rng.uniform(-1.0, 1.0, (batch, 3)).astype(np.float32), device="cuda")
        y_ref = torch.full((batch, 6), float("nan"), dtype=torch.float32, device="cuda")
        y_st = torch.full((batch, 6), float("nan"), dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        with torch.cuda.stream(stream):
            B.mlp_forward(net.h, batch, x.data_ptr(), y_ref.data_ptr())
            B.mlp_forward_static(net.h, batch, x.data_ptr(), y_st.data_ptr())
        stream.synchronize()
        a, b = y_ref.cpu().numpy(), y_st.cpu().numpy()
        assert np.all(np.isfinite(a)) and np.all(np.isfinite(b))
        np.testing.assert_array_equal(a, b)
    with pytest.raises(B.PicError) as e:
        B.mlp_forward_static(net.h, B.MLP_STATIC_MAX_BATCH + 1, x.data_ptr(), y_st.data_ptr())
    assert e.value.code == B.PIC_EINVAL
    net.close()
