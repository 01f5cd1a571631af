"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times: every part of the measured step (200,000 x 64^3, 20,000 x
256^3, 5,000 x 512^3 symmetric, 100,000 variable sizes with and without
padded leading dimensions) and the precision batch (20,000 x 256^3 with
entries spread over 2^+-20, int8-digit emulation), built one part at a time.
Sampled instances are compared with the CPU oracle one by one: <= 1e-13
relative Frobenius for binary64, bit for bit for the emulated mode; the
variable-size info array must be all zero."""
import gc

import numpy as np
import pytest
import torch

import bench
from oracle import precision as P
from paper_2203_09353_amd import bgemm, inputs, workloads
from paper_2203_09353_amd.workloads import host_instance

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    hd = bgemm.Handle()
    yield hd
    hd.close()


def _free(parts):
    parts.clear()
    gc.collect()
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name", ["u64", "u256", "s512", "vb", "vb8"])
def test_full_size_part_sampled_against_oracle(h, name):
    parts = workloads.build(name)
    try:
        worst = bench.sampled_parity(h, parts, 6, seed=23)
        assert worst[name] <= 1e-13, worst
        if name.startswith("vb"):
            assert int(torch.count_nonzero(parts[0].info)) == 0
    finally:
        _free(parts)


def test_full_size_int8_emulation_bit_exact(h):
    parts = workloads.build("config4")
    try:
        p = parts[0]
        picks = inputs.permutation(29, 4, p.batch)[:3].tolist()
        before = {i: host_instance(p, i) for i in picks}
        bench.mode_launch(h, p, (4, 7))
        torch.cuda.synchronize()
        for i in picks:
            A, B, C0 = before[i]
            Am = np.ascontiguousarray(A[:, :p.m].T)
            Bm = np.ascontiguousarray(B[:, :p.k].T)
            ref = P.int8_emulated_gemm(Am, Bm, 7, p.alpha, p.beta, np.ascontiguousarray(C0[:, :p.m].T))
            got = np.ascontiguousarray(host_instance(p, i)[2][:, :p.m].T)
            assert np.array_equal(got.view(np.int64), ref.view(np.int64)), i
    finally:
        _free(parts)
