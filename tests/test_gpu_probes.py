"""The measurement probes (stream copy, dependent gathers) on the GPU: the
gather buffer holds one cycle over all its elements, rates are positive,
and bad arguments are refused before any launch."""
import numpy as np
import pytest
import torch

import paper_1806_07300_amd as fp

pytestmark = pytest.mark.gpu


def test_stream_probe():
    a = torch.ones(1 << 24, dtype=torch.int32, device="cuda")
    b = torch.zeros_like(a)
    gbps = fp.fp_probe_stream(a, b)
    torch.cuda.synchronize()
    assert gbps > 50.0
    assert torch.equal(a, b)


@pytest.mark.parametrize("n", [4096, 256])  # 256 x 64 B: the L1-resident ceiling's working set
@pytest.mark.parametrize("fetch_bytes", [16, 48, 64])
def test_gather_buffer_is_one_cycle(fetch_bytes, n):
    buf = torch.zeros(n * fetch_bytes // 4 + 7, dtype=torch.int32, device="cuda")
    rate = fp.fp_probe_gather(buf, fetch_bytes, chains=2, steps=16)
    assert rate > 0
    words = buf.cpu().numpy().view(np.uint32)[:n * fetch_bytes // 4].reshape(n, fetch_bytes // 4)
    nxt = words[:, 0].astype(np.int64)
    assert ((0 <= nxt) & (nxt < n)).all()
    seen = np.zeros(n, bool)
    i = 0
    for _ in range(n):
        assert not seen[i]
        seen[i] = True
        i = nxt[i]
    assert i == 0 and seen.all()


def test_probe_arguments_refused():
    buf = torch.zeros(1 << 16, dtype=torch.int32, device="cuda")
    for kw in ({"fetch_bytes": 32}, {"chains": 3}, {"steps": 0}):
        with pytest.raises(fp.FPError) as e:
            fp.fp_probe_gather(buf, **{"fetch_bytes": 16, "chains": 1, "steps": 4, **kw})
        assert e.value.code == fp.FP_EINVAL
    with pytest.raises(fp.FPError):
        fp.fp_probe_gather(torch.zeros(100, dtype=torch.int32, device="cuda"), 16, 1, 4)  # fewer than 64 elements
