"""The seeded input generator: determinism, counter independence from layout
and chunking, range and moments, and the size distribution."""
import numpy as np
import torch

from paper_2203_09353_amd import inputs


def test_fmix32_known_values():
    # MurmurHash3 fmix32 reference values (fmix32(0) = 0 is a fixed point)
    assert inputs._fmix32_int(0) == 0
    t = torch.tensor([0, 1, 0xFFFFFFFF, 0x12345678], dtype=torch.int64)
    got = inputs._fmix32(t).tolist()
    assert got == [inputs._fmix32_int(int(x)) for x in t.tolist()]
    assert inputs._fmix32_int(1) == 0x514E28B7


def test_uniform_deterministic_and_chunk_independent():
    a = inputs.uniform_flat(3, 1, 1000, 5000)
    b = inputs.uniform_flat(3, 1, 1000, 5000, chunk=777)
    c = inputs.uniform_flat(3, 1, 3000, 100)
    assert torch.equal(a, b)
    assert torch.equal(a[2000:2100], c)
    assert not torch.equal(a, inputs.uniform_flat(4, 1, 1000, 5000))
    assert not torch.equal(a, inputs.uniform_flat(3, 2, 1000, 5000))


def test_uniform_range_and_moments():
    x = inputs.uniform_flat(0, 0, 0, 1 << 20).numpy()
    assert x.min() >= -1.0 and x.max() < 1.0
    assert abs(x.mean()) < 3e-3
    assert abs(x.var() - 1.0 / 3.0) < 3e-3
    # counters above 2**32 work and differ from the low ones
    y = inputs.uniform_flat(0, 0, (1 << 32) + 5, 1000)
    assert not torch.equal(y, inputs.uniform_flat(0, 0, 5, 1000))


def test_batch_layout_and_instance_regeneration():
    full = inputs.uniform_batch(9, 2, 6, 5, 4, ld=8)
    assert full.shape == (6, 4, 8)
    assert torch.isnan(full[:, :, 5:]).all()
    some = inputs.uniform_batch(9, 2, 6, 5, 4, ld=8, instances=[4, 1])
    assert torch.equal(some[0, :, :5], full[4, :, :5])
    assert torch.equal(some[1, :, :5], full[1, :, :5])
    tight = inputs.uniform_batch(9, 2, 6, 5, 4)
    assert torch.equal(tight, full[:, :, :5])


def test_ragged_regeneration():
    rows, cols = [3, 7, 1, 9], [2, 5, 4, 1]
    allm = inputs.uniform_ragged(1, 0, rows, cols, lds=[4, 8, 1, 16])
    one = inputs.uniform_ragged(1, 0, rows, cols, lds=[4, 8, 1, 16], instances=[2])
    assert torch.equal(one[0], allm[2])
    assert torch.isnan(allm[3][:, 9:]).all()


def test_log_uniform_sizes_support():
    s = inputs.log_uniform_sizes(11, 0, 200000).numpy()
    support = sorted({2 ** j + d for j in range(3, 10) for d in (-1, 0, 1)})
    vals, counts = np.unique(s, return_counts=True)
    assert list(vals) == support
    p = counts / counts.sum()
    assert np.all(np.abs(p - 1.0 / 21) < 0.004)


def test_haar_orthogonal():
    q = inputs.haar_orthogonal(2, 0, 3, 16)
    eye = torch.eye(16, dtype=torch.float64)
    for i in range(3):
        assert torch.allclose(q[i] @ q[i].T, eye, atol=1e-13)


def test_wide_values_support_and_exponents():
    x = inputs.wide_flat(9, 2, 0, 200_000, emax=20)
    m, e = torch.frexp(x)
    assert torch.all((e - 1 >= -20) & (e - 1 <= 20))
    assert set((e - 1).unique().tolist()) == set(range(-20, 21))
    assert torch.all((m.abs() >= 0.5) & (m.abs() < 1.0))
    frac_neg = (x < 0).double().mean().item()
    assert abs(frac_neg - 0.5) < 0.01
    # significand 2|m| - 1 uniform on [0, 1)
    sig = 2 * m.abs() - 1
    assert abs(sig.mean().item() - 0.5) < 0.01
    assert torch.equal(inputs.wide_flat(9, 2, 1000, 10), x[1000:1010])
