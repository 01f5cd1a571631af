"""Seeded synthetic inputs for batched GEMM workloads.

This module is shared by the GPU path's callers (benchmark, tests) and by the
CPU oracle's callers; it holds no GEMM arithmetic of its own.  Values come from
a counter-based generator, so the value of element ``e`` of stream ``s`` under
seed ``x`` is a pure function of ``(x, s, e)``: a device can fill a slab of many
gigabytes while the host regenerates any single instance bit-for-bit.

Generator: the MurmurHash3 32-bit finaliser (``fmix32``, Austin Appleby,
public domain) applied to the element counter, two independent 32-bit words
per element, joined into a 53-bit integer ``u`` and mapped to
``u * 2**-52 - 1`` in [-1, 1) (exact in binary64).  All integer work is done in
int64 on values below 2**49, so it is exact and identical on every device.

Matrix layout: a batch of column-major matrices with ``rows x cols`` and
leading dimension ``ld >= rows`` is a tensor of shape ``(batch, cols, ld)``;
element (r, c) of instance b is ``t[b, c, r]``.  The generator's counter runs
over the ``rows x cols`` payload only, ``((b * cols) + c) * rows + r``, so the
padding rows ``r >= rows`` draw nothing; they are filled with NaN, which a
correct GEMM never reads or writes.
"""
from __future__ import annotations

import math

import torch

M32 = 0xFFFFFFFF


def _fmix32_int(h: int) -> int:
    h &= M32
    h ^= h >> 16
    h = (h * 0x85EBCA6B) & M32
    h ^= h >> 13
    h = (h * 0xC2B2AE35) & M32
    h ^= h >> 16
    return h


def _mul32(h: torch.Tensor, c: int) -> torch.Tensor:
    """(h * c) mod 2**32 for int64 h in [0, 2**32) without int64 overflow."""
    lo, hi = c & 0xFFFF, c >> 16
    return (h * lo + (((h * hi) & 0xFFFF) << 16)) & M32


def _fmix32(h: torch.Tensor) -> torch.Tensor:
    h = h ^ (h >> 16)
    h = _mul32(h, 0x85EBCA6B)
    h = h ^ (h >> 13)
    h = _mul32(h, 0xC2B2AE35)
    return h ^ (h >> 16)


def _keys(seed: int, stream: int) -> tuple[int, int, int, int]:
    base = _fmix32_int((seed & M32) ^ _fmix32_int((seed >> 32) ^ 0x9E3779B9))
    return tuple(_fmix32_int(base ^ (((stream * 4 + j + 1) * 0x632BE5AB) & M32))
                 for j in range(4))


def uniform_flat(seed: int, stream: int, start: int, count: int,
                 device="cpu", chunk: int = 1 << 26) -> torch.Tensor:
    """Values U(seed, stream, e) for e in [start, start + count), float64."""
    k0, k1, k2, k3 = _keys(seed, stream)
    out = torch.empty(count, dtype=torch.float64, device=device)
    scale = 2.0 ** -52
    for off in range(0, count, chunk):
        n = min(chunk, count - off)
        e = torch.arange(start + off, start + off + n, dtype=torch.int64,
                         device=device)
        lo = e & M32
        hi = e >> 32
        hm1 = _fmix32(hi ^ k0)
        hm2 = _fmix32(hi ^ k3)
        w1 = _fmix32(_fmix32(lo ^ k1) ^ hm1)
        w2 = _fmix32(_fmix32(lo ^ k2) ^ hm2)
        u = (w1 << 21) | (w2 >> 11)
        out[off:off + n] = u.to(torch.float64) * scale - 1.0
        del e, lo, hi, hm1, hm2, w1, w2, u
    return out


def uniform_batch(seed: int, stream: int, batch: int, rows: int, cols: int,
                  ld: int | None = None, device="cpu",
                  instances=None) -> torch.Tensor:
    """Uniform[-1, 1) column-major batch, shape (len, cols, ld), NaN padding.

    ``instances`` (a list of instance numbers) regenerates only those
    instances of the full batch; ``None`` generates instances 0..batch-1.
    """
    ld = rows if ld is None else ld
    assert ld >= rows
    per = rows * cols
    if instances is None:
        flat = uniform_flat(seed, stream, 0, batch * per, device)
        payload = flat.view(batch, cols, rows)
        nb = batch
    else:
        parts = [uniform_flat(seed, stream, int(i) * per, per, device)
                 for i in instances]
        nb = len(parts)
        payload = (torch.stack(parts) if parts else
                   torch.empty(0, dtype=torch.float64, device=device)
                   ).view(nb, cols, rows)
    if ld == rows:
        return payload.contiguous()
    out = torch.full((nb, cols, ld), float("nan"), dtype=torch.float64,
                     device=device)
    out[:, :, :rows] = payload
    return out


def uniform_ragged(seed: int, stream: int, rows, cols, lds=None, device="cpu",
                   instances=None):
    """Per-instance sizes: list of (cols_i, ld_i) tensors, NaN padding.

    The counter of instance i starts at sum_{j<i} rows_j * cols_j.
    """
    n = len(rows)
    lds = list(rows) if lds is None else list(lds)
    offs = [0] * (n + 1)
    for i in range(n):
        offs[i + 1] = offs[i] + int(rows[i]) * int(cols[i])
    sel = range(n) if instances is None else instances
    out = []
    for i in sel:
        r, c, ld = int(rows[i]), int(cols[i]), int(lds[i])
        vals = uniform_flat(seed, stream, offs[i], r * c, device).view(c, r)
        m = torch.full((c, ld), float("nan"), dtype=torch.float64, device=device)
        m[:, :r] = vals
        out.append(m)
    return out


def gaussian_flat(seed: int, stream: int, start: int, count: int,
                  device="cpu") -> torch.Tensor:
    """Standard normal values by the Box-Muller transform of two streams."""
    u1 = (uniform_flat(seed, 2 * stream, start, count, device) + 1.0) * 0.5
    u2 = (uniform_flat(seed, 2 * stream + 1, start, count, device) + 1.0) * 0.5
    u1 = 1.0 - u1  # (0, 1]
    return torch.sqrt(-2.0 * torch.log(u1)) * torch.cos(2.0 * math.pi * u2)


def haar_orthogonal(seed: int, stream: int, count: int, size: int):
    """``count`` Haar-distributed orthogonal matrices (Mezzadri's recipe:
    QR of a Gaussian matrix, then column signs from diag(R)); CPU float64,
    shape (count, size, size)."""
    g = gaussian_flat(seed, stream, 0, count * size * size).view(count, size, size)
    q, r = torch.linalg.qr(g)
    d = torch.sign(torch.diagonal(r, dim1=-2, dim2=-1))
    d[d == 0] = 1.0
    return q * d.unsqueeze(-2)


def log_uniform_sizes(seed: int, stream: int, count: int, jmin=3, jmax=9):
    """Sizes 2**j + delta with j uniform in [jmin, jmax] and delta uniform in
    {-1, 0, +1}; int64 tensor of length ``count``."""
    u = uniform_flat(seed, stream, 0, 2 * count)
    nj = jmax - jmin + 1
    j = torch.clamp(((u[:count] + 1.0) * 0.5 * nj).floor().to(torch.int64), 0, nj - 1) + jmin
    dlt = torch.clamp(((u[count:] + 1.0) * 0.5 * 3).floor().to(torch.int64), 0, 2) - 1
    return (2 ** j) + dlt


def wide_flat(seed: int, stream: int, start: int, count: int, emax: int = 20,
              device="cpu") -> torch.Tensor:
    """Values s * m * 2**e with m uniform in [1, 2), s = +-1 equiprobable and
    e uniform on the integers -emax..emax (two streams: 2 * stream gives s
    and m, 2 * stream + 1 gives e)."""
    v = uniform_flat(seed, 2 * stream, start, count, device)
    w = uniform_flat(seed, 2 * stream + 1, start, count, device)
    e = torch.clamp(((w + 1.0) * 0.5 * (2 * emax + 1)).floor(), 0, 2 * emax) - emax
    mag = 1.0 + torch.abs(v)
    return torch.where(v < 0, -mag, mag) * torch.exp2(e)


def permutation(seed: int, stream: int, count: int) -> torch.Tensor:
    """A seeded permutation of range(count) (argsort of uniform keys)."""
    return torch.argsort(uniform_flat(seed, stream, 0, count), stable=True)


def round_up(x: int, q: int) -> int:
    return (x + q - 1) // q * q
