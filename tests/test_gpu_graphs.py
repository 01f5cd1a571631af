"""The batched entry points are graph-capturable: a uniform batch and a
variable-size batch (device-side planning, persistent tile queues) captured
together in one HIP graph (through torch.cuda.graph) and replayed three
times, with other eager work and synchronisation between the replays, give
the eager result bit for bit every time."""
import pytest
import torch

import bench
from paper_2203_09353_amd import bgemm, workloads

pytestmark = pytest.mark.gpu


def test_uniform_and_variable_batches_replay_from_a_graph():
    h = bgemm.Handle()
    try:
        u = workloads.build("u64", scale=0.00025)[0]        # 50 x 64^3, beta 1
        v = workloads.build("vb", scale=0.003)[0]           # 300 mixed sizes, beta 0.5
        u.pointers()                                        # pointer arrays made before capture
        cu0, cv0 = u.C.clone(), v.slabs[2].clone()
        torch.cuda.synchronize()
        # eager reference
        bench.part_launch(h, u)
        bench.part_launch(h, v)
        torch.cuda.synchronize()
        eu, ev = u.C.clone(), v.slabs[2].clone()
        # warm-up on a side stream, then capture
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            bench.part_launch(h, u)
            bench.part_launch(h, v)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            bench.part_launch(h, u)
            bench.part_launch(h, v)
        torch.cuda.synchronize()
        other = workloads.build("u64", scale=0.0001)[0]
        for rep in range(3):
            u.C.copy_(cu0)
            v.slabs[2].copy_(cv0)
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(u.C.view(torch.int64), eu.view(torch.int64)), rep
            assert torch.equal(v.slabs[2].view(torch.int64), ev.view(torch.int64)), rep
            assert int(torch.count_nonzero(v.info)) == 0
            bench.part_launch(h, other)                     # unrelated eager work
            torch.cuda.synchronize()
        del g
    finally:
        h.close()
