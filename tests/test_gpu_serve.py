"""Serving on the GPU: requests that overlap on the device (continuous
batching over per-slot streams) give the same result as each request run
alone (bitwise: same plan, fixed tiles and reduction orders)."""
import numpy as np
import pytest

from paper_2406_19920_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_mixed_equals_alone():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2406_19920_amd import serve
    print("case serve mixed vs alone", flush=True)
    reqs = synth.serving_requests(rate=3000, count=24, seed=11, nmin=32, nmax=96)
    ex = serve.GpuExecutor(slots=4)
    srv = serve.Server(ex, 8 << 30, slots=4, keep_outputs=True)
    res = srv.run(reqs)
    s = res.summary()
    print("summary", s, flush=True)
    assert res.completed == len(reqs)
    assert res.max_inflight >= 2
    for r in reqs:
        alone = srv.run_alone(r)
        mixed = res.outputs[r["rid"]]
        for a, m in zip(alone, mixed):
            np.testing.assert_array_equal(a.numpy(), m.numpy(), err_msg=f"request {r['rid']}")
    srv.close()
