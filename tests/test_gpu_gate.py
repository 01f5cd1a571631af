"""GPU parity of the two-spin gate (bg_zgate2_batched) against the gate
oracle, through the C ABI: every site of small states, a 2^21-amplitude
state, unitary invariants, invalid sites and 8-byte-aligned states."""
import numpy as np
import pytest
import torch

from oracle import gates as G
from paper_2203_09353_amd import bgemm, inputs

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


@pytest.fixture(scope="module")
def h():
    hd = bgemm.Handle()
    yield hd
    hd.close()


def _states(seed, batch, S):
    re = inputs.uniform_flat(seed, 0, 0, batch << S).view(batch, 1 << S)
    im = inputs.uniform_flat(seed, 1, 0, batch << S).view(batch, 1 << S)
    return torch.complex(re, im)


def _gates(seed, batch, unitary=False):
    g = inputs.gaussian_flat(seed, 2, 0, batch * 32).view(batch, 32).numpy()
    if unitary:
        return np.stack([G.haar_unitary(g[i, :16], g[i, 16:]) for i in range(batch)])
    return (g[:, :16] + 1j * g[:, 16:]).reshape(batch, 4, 4)


def _check(got, ref, U, psi):
    # |error| <= 8 u sum_q' |U[q, q']| |v_q'| per amplitude (both sides)
    for i in range(got.shape[0]):
        assert np.allclose(got[i], ref[i], rtol=0, atol=8 * U64 * 4 * np.abs(U[i]).max() *
                           np.abs(psi[i]).max() * 4)


@pytest.mark.parametrize("S", [2, 3, 7, 12])
def test_every_site(h, S):
    for s in range(S - 1):
        batch = 3
        psi = _states(S + s, batch, S)
        U = _gates(S + 10 * s, batch)
        sites = torch.tensor([s, max(0, s - 1), S - 2], dtype=torch.int32)
        d = psi.cuda()
        info = h.zgate2(S, sites.cuda(), torch.tensor(U).cuda(), d)
        torch.cuda.synchronize()
        assert info.cpu().tolist() == [0, 0, 0]
        got = d.cpu().numpy()
        ref = np.stack([G.apply_gate(psi.numpy()[i], S, int(sites[i]), U[i])
                        for i in range(batch)])
        _check(got, ref, U, psi.numpy())


def test_large_state_and_unitary_invariants(h):
    S = 21
    psi = _states(5, 2, S)
    psi = psi / torch.linalg.norm(psi, dim=1, keepdim=True)
    U = _gates(6, 2, unitary=True)
    d = psi.cuda()
    sites = torch.tensor([0, 13], dtype=torch.int32).cuda()
    h.zgate2(S, sites, torch.tensor(U).cuda(), d)
    torch.cuda.synchronize()
    got = d.cpu().numpy()
    for i, s in enumerate((0, 13)):
        ref = G.apply_gate(psi.numpy()[i], S, s, U[i])
        _check(got[i:i + 1], ref[None], U[i:i + 1], psi.numpy()[i:i + 1])
        assert abs(np.linalg.norm(got[i]) - 1.0) < 1e-12
    # U^H undoes U
    Uh = np.conj(np.transpose(U, (0, 2, 1))).copy()
    h.zgate2(S, sites, torch.tensor(Uh).cuda(), d)
    torch.cuda.synchronize()
    assert np.allclose(d.cpu().numpy(), psi.numpy(), rtol=0, atol=1e-13)


def test_invalid_site_and_unaligned_state(h):
    S = 9
    psi = _states(8, 2, S)
    U = _gates(9, 2)
    d = psi.cuda()
    info = h.zgate2(S, torch.tensor([S - 1, -1], dtype=torch.int32).cuda(),
                    torch.tensor(U).cuda(), d)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [-3, -3]
    assert torch.equal(d.cpu().view(torch.float64), psi.view(torch.float64))
    # a state starting 8 bytes past a 16-byte boundary
    flat = torch.zeros(1 + 2 * (1 << S), dtype=torch.float64, device="cuda")
    flat[1:] = torch.view_as_real(psi[0]).reshape(-1).cuda()
    L = bgemm.lib()
    Ucm = torch.tensor(U[:1]).transpose(1, 2).contiguous().cuda()
    pU = torch.tensor([Ucm.data_ptr()], dtype=torch.int64, device="cuda")
    pP = torch.tensor([flat.data_ptr() + 8], dtype=torch.int64, device="cuda")
    st_ = torch.tensor([4], dtype=torch.int32, device="cuda")
    h._sync_stream()
    assert L.bg_zgate2_batched(h._h, S, st_.data_ptr(), pU.data_ptr(), pP.data_ptr(), 1, None) == 0
    torch.cuda.synchronize()
    got = torch.view_as_complex(flat[1:].cpu().view(-1, 2)).numpy()
    ref = G.apply_gate(psi.numpy()[0], S, 4, U[0])
    _check(got[None], ref[None], U[:1], psi.numpy()[:1])


def test_gate_argument_errors(h):
    L = bgemm.lib()
    assert L.bg_zgate2_batched(h._h, 1, None, None, None, 0, None) == 1
    assert h.last_invalid_arg() == 2
    assert L.bg_zgate2_batched(h._h, 5, None, None, None, 2, None) == 1
    assert h.last_invalid_arg() == 3
    assert L.bg_zgate2_batched(h._h, 5, None, None, None, 0, None) == 0
