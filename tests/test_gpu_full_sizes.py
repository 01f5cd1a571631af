"""GPU parity at the benchmark's full sizes, in the launch configuration the
benchmark times: every part of the measured step (200,000 x 64^3, 20,000 x
256^3, 5,000 x 512^3 symmetric, 100,000 variable sizes with and without
padded leading dimensions), built one part at a time and run once; then
EVERY instance is compared with the CPU oracle (<= 1e-13 relative Frobenius
and the componentwise rounding bound; ld padding untouched; variable-size
info all zero), copying to the host in chunks.  On the symmetric part, the
instances whose A and B share their orthogonal basis are also checked
against the spectral closed forms (trace and Frobenius norm of A B).  The
precision batch (20,000 x 256^3 with entries spread over 2^+-20) is checked
bit for bit against the int8-digit emulation oracle on sampled instances."""
import gc

import numpy as np
import pytest
import torch

import bench
from oracle import precision as P
from paper_2203_09353_amd import bgemm, inputs, workloads
from paper_2203_09353_amd.workloads import host_instance
from tests import fullparity

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
def test_full_size_part_every_instance(h, name):
    parts = workloads.build(name)
    try:
        p = parts[0]
        launch = lambda: bench.part_launch(h, p)
        print("[full-size parity] %s: %d instances" % (name, p.batch), flush=True)
        if name.startswith("vb"):
            worst = fullparity.every_instance_vb(launch, p)
        else:
            sym = [i for i in range(p.batch) if i % 100 == 0] if name == "s512" else []
            C0 = {i: p.C[i].cpu().numpy() for i in sym}
            worst = fullparity.every_instance_uniform(launch, p)
            if sym:
                assert fullparity.symmetric_identities(p, C0) == len(sym) == 50
        print("[full-size parity] %s: worst rel Frobenius %.3e" % (name, worst), flush=True)
        assert worst <= 1e-13
    finally:
        _free(parts)


def test_full_size_int8_emulation_bit_exact(h):
    parts = workloads.build("config4")
    try:
        p = parts[0]
        picks = inputs.permutation(29, 4, p.batch)[:8].tolist()
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
