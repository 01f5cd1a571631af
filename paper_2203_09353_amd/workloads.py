"""Device-resident synthetic workloads shaped like the paper's batched GEMMs.

Each workload part is built on the device from the seeded counter-based
generator (``inputs``); a few instances can be copied back to the host for
the oracle.  No GEMM of the method is computed here: the one matrix product
(Q diag(d) Q^T for the symmetric operands) is input synthesis done by torch.

Parts (all FP64, column-major, pointer arrays in a seeded shuffled order so
kernels cannot rely on contiguity):
  u32  : 1000 x 32^3, alpha 1, beta 0, A, B uniform[-1, 1) seed 0 (C = NaN)
  u64  : 200,000 x 64^3, alpha = beta = 1, A, B, C uniform[-1, 1) seed 1
  u256 : 20,000 x 256^3, alpha = beta = 1, seed 2
  s512 : 5,000 x 512^3, alpha = beta = 1, A_i = Qa diag(da) Qa^T and
         B_i = Qb diag(db) Qb^T (Q from a pool of Haar orthogonal matrices,
         d uniform[-1, 1)), C uniform, seed 3
  w256 : 20,000 x 256^3, alpha 1, beta 0, entries s m 2^e (m uniform in
         [1, 2), e uniform in -20..20, s = +-1), C = NaN, seed 5 -- the
         input of the precision modes
  vb   : 100,000 variable sizes, m, n, k independently 2^j + delta with j
         uniform in 3..9 and delta uniform in {-1, 0, 1}; alpha 1, beta 0.5;
         ld = rows (``vb``) or rows rounded up to a multiple of 8 (``vb8``);
         seed 4
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import inputs

DEFAULT_POOL = 32


@dataclass
class UniformPart:
    name: str
    m: int
    n: int
    k: int
    batch: int
    alpha: float
    beta: float
    A: torch.Tensor          # (batch, k, m) storage, i.e. A_i is m x k, lda = m
    B: torch.Tensor          # (batch, n, k)
    C: torch.Tensor          # (batch, n, m)
    perm: torch.Tensor       # order in which instances are handed to the library
    pA: torch.Tensor = None
    pB: torch.Tensor = None
    pC: torch.Tensor = None
    C0_host: dict = field(default_factory=dict)

    @property
    def flops(self) -> float:
        return 2.0 * self.m * self.n * self.k * self.batch

    @property
    def bytes(self) -> float:
        """Algorithmic HBM bytes: A, B read once, C written once and read
        when beta != 0, plus the three 8-byte pointers per instance."""
        c_rw = 2 if self.beta != 0 else 1
        per = 8 * (self.m * self.k + self.k * self.n + c_rw * self.m * self.n) + 24
        return float(per) * self.batch

    def pointers(self):
        if self.pA is None:
            mk = lambda X: (torch.arange(self.batch, device=X.device, dtype=torch.int64)
                            * (X.stride(0) * 8) + X.data_ptr())[self.perm]
            self.pA, self.pB, self.pC = mk(self.A), mk(self.B), mk(self.C)
        return self.pA, self.pB, self.pC


@dataclass
class VbPart:
    name: str
    batch: int
    alpha: float
    beta: float
    m: torch.Tensor          # device int32, in library order
    n: torch.Tensor
    k: torch.Tensor
    lda: torch.Tensor
    ldb: torch.Tensor
    ldc: torch.Tensor
    pA: torch.Tensor
    pB: torch.Tensor
    pC: torch.Tensor
    slabs: tuple             # (A, B, C) flat device tensors holding the data
    offs: tuple              # host int64 element offsets per instance (A, B, C), natural order
    perm: torch.Tensor
    sizes_host: tuple        # (m, n, k, lda, ldb, ldc) host int64, natural order
    info: torch.Tensor = None

    @property
    def flops(self) -> float:
        m, n, k = (x.to(torch.float64) for x in self.sizes_host[:3])
        return float((2.0 * m * n * k).sum())

    @property
    def bytes(self) -> float:
        m, n, k = (x.to(torch.float64) for x in self.sizes_host[:3])
        c_rw = 2 if self.beta != 0 else 1
        return float((8 * (m * k + k * n + c_rw * m * n)).sum() + 48 * self.batch)

    def per_instance_roofline_s(self, peak_flops: float, peak_bw: float) -> float:
        """Sum over instances of max(flops_i / peak, bytes_i / bandwidth)."""
        m, n, k = (x.to(torch.float64) for x in self.sizes_host[:3])
        c_rw = 2 if self.beta != 0 else 1
        f = 2.0 * m * n * k
        b = 8 * (m * k + k * n + c_rw * m * n) + 48
        return float(torch.maximum(f / peak_flops, b / peak_bw).sum())


def _fill_uniform(t: torch.Tensor, seed: int, stream: int, chunk: int = 1 << 26):
    flat = t.view(-1)
    for off in range(0, flat.numel(), chunk):
        n = min(chunk, flat.numel() - off)
        flat[off:off + n] = inputs.uniform_flat(seed, stream, off, n, device=t.device)


def _fill_wide(t: torch.Tensor, seed: int, stream: int, chunk: int = 1 << 25):
    flat = t.view(-1)
    for off in range(0, flat.numel(), chunk):
        n = min(chunk, flat.numel() - off)
        flat[off:off + n] = inputs.wide_flat(seed, stream, off, n, device=t.device)


def uniform_part(name, batch, m, n, k, alpha, beta, seed, device="cuda", c_nan=False,
                 wide=False):
    A = torch.empty(batch, k, m, dtype=torch.float64, device=device)
    B = torch.empty(batch, n, k, dtype=torch.float64, device=device)
    C = torch.empty(batch, n, m, dtype=torch.float64, device=device)
    fill = _fill_wide if wide else _fill_uniform
    fill(A, seed, 0)
    fill(B, seed, 1)
    if c_nan:
        C.fill_(float("nan"))
    else:
        _fill_uniform(C, seed, 2)
    perm = inputs.permutation(seed, 9, batch).to(device)
    return UniformPart(name, m, n, k, batch, alpha, beta, A, B, C, perm)


def symmetric_part(name, batch, size, alpha, beta, seed, device="cuda", pool=DEFAULT_POOL,
                   chunk=256):
    """A_i = Qa diag(da) Qa^T, B_i = Qb diag(db) Qb^T with Qa, Qb drawn from a
    pool of Haar orthogonal matrices; instance i uses pool entries
    (i mod pool) and ((7 i + 3) mod pool), except every 100th instance, which
    uses the same Q for both (its product is Q diag(da db) Q^T)."""
    Q = inputs.haar_orthogonal(seed, 5, pool, size).to(device)
    QT = Q.transpose(1, 2).contiguous()
    A = torch.empty(batch, size, size, dtype=torch.float64, device=device)
    B = torch.empty(batch, size, size, dtype=torch.float64, device=device)
    C = torch.empty(batch, size, size, dtype=torch.float64, device=device)
    idx = torch.arange(batch, device=device)
    qa = idx % pool
    qb = (7 * idx + 3) % pool
    qb = torch.where(idx % 100 == 0, qa, qb)
    for s in range(0, batch, chunk):
        e = min(batch, s + chunk)
        da = inputs.uniform_flat(seed, 0, s * size, (e - s) * size, device).view(e - s, 1, size)
        db = inputs.uniform_flat(seed, 1, s * size, (e - s) * size, device).view(e - s, 1, size)
        # column-major storage of a symmetric matrix equals its row-major one
        X = torch.matmul((Q[qa[s:e]] * da).contiguous(), QT[qa[s:e]])
        A[s:e] = 0.5 * (X + X.transpose(1, 2))  # exactly symmetric
        X = torch.matmul((Q[qb[s:e]] * db).contiguous(), QT[qb[s:e]])
        B[s:e] = 0.5 * (X + X.transpose(1, 2))
        del X
    _fill_uniform(C, seed, 2)
    perm = inputs.permutation(seed, 9, batch).to(device)
    part = UniformPart(name, size, size, size, batch, alpha, beta, A, B, C, perm)
    part.sym = (qa.cpu(), qb.cpu())
    return part


def vb_part(name, batch, alpha, beta, seed, pad8=False, device="cuda", group=4096):
    ms = inputs.log_uniform_sizes(seed, 0, batch)
    ns = inputs.log_uniform_sizes(seed, 1, batch)
    ks = inputs.log_uniform_sizes(seed, 2, batch)
    rnd = (lambda x: (x + 7) // 8 * 8) if pad8 else (lambda x: x)
    lda, ldb, ldc = rnd(ms), rnd(ks), rnd(ms)
    na, nb, nc = lda * ks, ldb * ns, ldc * ns
    offs = []
    slabs = []
    for cnt, (rows, cols, ld, stream) in zip((na, nb, nc), ((ms, ks, lda, 0), (ks, ns, ldb, 1),
                                                            (ms, ns, ldc, 2))):
        o = torch.zeros(batch + 1, dtype=torch.int64)
        o[1:] = torch.cumsum(cnt, 0)
        offs.append(o)
        slab = torch.empty(int(o[-1]), dtype=torch.float64, device=device)
        if pad8:
            slab.fill_(float("nan"))
            # payload counters run over rows * cols per instance, as in
            # inputs.uniform_ragged; padding keeps NaN
            _fill_padded(slab, o, rows, cols, ld, seed, stream, device, group)
        else:
            _fill_uniform(slab, seed, stream)
        slabs.append(slab)
    perm = inputs.permutation(seed, 9, batch)
    dev_i32 = lambda x: x[perm].to(torch.int32).to(device)
    ptr = lambda slab, o: (slab.data_ptr() + 8 * o[:-1])[perm].to(device)
    part = VbPart(name, batch, alpha, beta, dev_i32(ms), dev_i32(ns), dev_i32(ks), dev_i32(lda),
                  dev_i32(ldb), dev_i32(ldc), ptr(slabs[0], offs[0]), ptr(slabs[1], offs[1]),
                  ptr(slabs[2], offs[2]), tuple(slabs), tuple(offs), perm.to(device),
                  (ms, ns, ks, lda, ldb, ldc))
    part.info = torch.empty(batch, dtype=torch.int32, device=device)
    return part


def _fill_padded(slab, o, rows, cols, ld, seed, stream, device, group=4096):
    """Writes the payload of each instance into its padded column-major
    block; instances are processed in groups to bound temporaries."""
    batch = rows.numel()
    pay = rows * cols
    poff = torch.zeros(batch + 1, dtype=torch.int64)
    poff[1:] = torch.cumsum(pay, 0)
    for s in range(0, batch, group):
        e = min(batch, s + group)
        vals = inputs.uniform_flat(seed, stream, int(poff[s]), int(poff[e] - poff[s]), device)
        # destination index of each payload element
        r_all, c_all, l_all, b_all = (x[s:e].to(device) for x in (rows, cols, ld, o[:-1]))
        cnt = (r_all * c_all)
        inst = torch.repeat_interleave(torch.arange(e - s, device=device), cnt)
        local = torch.arange(vals.numel(), device=device) - torch.repeat_interleave(
            poff[s:e].to(device) - int(poff[s]), cnt)
        r = local % r_all[inst]
        c = local // r_all[inst]
        slab[b_all[inst] + c * l_all[inst] + r] = vals


def host_instance(part, i):
    """Host copies (A, B, C) of instance i (natural order) of a part as
    (cols, ld) float64 numpy arrays -- the oracle's inputs."""
    if isinstance(part, UniformPart):
        return (part.A[i].cpu().numpy(), part.B[i].cpu().numpy(), part.C[i].cpu().numpy())
    ms, ns, ks, lda, ldb, ldc = (int(x[i]) for x in part.sizes_host)
    out = []
    for slab, o, rows, cols, ld in zip(part.slabs, part.offs, (ms, ks, ms), (ks, ns, ns),
                                       (lda, ldb, ldc)):
        a = int(o[i])
        out.append(slab[a:a + cols * ld].view(cols, ld).cpu().numpy())
    return tuple(out)


PARTS = {
    "u32": lambda d, b: uniform_part("u32", b(1000), 32, 32, 32, 1.0, 0.0, 0, d, c_nan=True),
    "u64": lambda d, b: uniform_part("u64", b(200_000), 64, 64, 64, 1.0, 1.0, 1, d),
    "u256": lambda d, b: uniform_part("u256", b(20_000), 256, 256, 256, 1.0, 1.0, 2, d),
    "s512": lambda d, b: symmetric_part("s512", b(5_000), 512, 1.0, 1.0, 3, d),
    "w256": lambda d, b: uniform_part("w256", b(20_000), 256, 256, 256, 1.0, 0.0, 5, d,
                                      c_nan=True, wide=True),
    "vb": lambda d, b: vb_part("vb", b(100_000), 1.0, 0.5, 4, False, d),
    "vb8": lambda d, b: vb_part("vb8", b(100_000), 1.0, 0.5, 4, True, d),
}
ALIASES = {"config1": "u32", "config2": "u64+u256+s512", "config3": "vb",
           "config2+vb": "u64+u256+s512+vb", "config4": "w256"}


def build(name: str, device="cuda", scale: float = 1.0):
    """The parts of a workload: a '+'-joined list of part names (or an alias
    such as config2+vb).  ``scale`` < 1 shrinks every batch (at least one
    instance) while keeping the shapes, for tests."""
    b = lambda n: max(1, int(round(n * scale)))
    names = ALIASES.get(name, name).split("+")
    for n in names:
        if n not in PARTS:
            raise ValueError("unknown workload part " + n)
    return [PARTS[n](device, b) for n in names]


NAMES = tuple(PARTS) + tuple(ALIASES)
