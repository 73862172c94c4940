"""The benchmark step run as three concurrent chains (HIP streams driven by
host threads) gives bit-identical outputs to the same ops in sequence on
one stream: every kernel of the step is deterministic, so any missing
cross-stream dependency would show up as a difference."""
import concurrent.futures as cf

import pytest
import torch

import bench

pytestmark = pytest.mark.gpu


def test_concurrent_step_equals_serial():
    d = bench.Device(bench.make_inputs(32, 8))
    d.plan_fwd = d.plan_bwd = None
    d.spmv_bwd_mode = "fused"
    d.streams = tuple(torch.cuda.Stream() for _ in range(3))
    d.pool = cf.ThreadPoolExecutor(2)
    ref = {}
    bench.run_step(d, bench.Marks(False), ref)
    torch.cuda.synchronize()
    assert len(ref) == 19
    for _ in range(3):  # later steps reuse memory the earlier ones freed
        got = {}
        bench.run_step_streams(d, [bench.Marks(False) for _ in range(3)], got)
        torch.cuda.synchronize()
        assert sorted(got) == sorted(ref)
        for k in ref:
            assert torch.equal(got[k], ref[k]), k
    d.pool.shutdown()
