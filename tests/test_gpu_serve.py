"""GPU tests of the request loop (include/bgserve.h) through the C ABI: the
device generator against the Philox oracle bit for bit, final client states
against the CPU replay, results identical alone and in the mix, the timing
outputs and the memory budget."""
import numpy as np
import pytest
import torch

from oracle import philox, serving
from paper_2203_09353_amd import bgemm, serve

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    hd = bgemm.Handle()
    yield hd
    hd.close()


@pytest.mark.parametrize("n,client,j", [(1, 0, 0), (5, 3, 7), (32, 63, 2 ** 40 + 3), (33, 1, 12),
                                        (128, 2, 0), (257, 9, 1)])
def test_generator_matches_oracle(h, n, client, j):
    out = torch.full((n * n,), float("nan"), dtype=torch.float64, device="cuda")
    serve.fill_factor(77, client, j, n, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().reshape(n, n).T             # column-major storage
    ref = philox.factor(77, client, j, n, serving.scale(n))
    assert np.array_equal(got.view(np.int64), ref.view(np.int64))


SIZES = [32, 64, 33, 128, 32, 7]


def _schedule():
    a, c, l = serve.requests(9, len(SIZES), 4000.0, 0.01)
    return a, c, np.minimum(l, 6)       # short chains keep the CPU replay quick


def test_final_states_match_replay_and_timing(h):
    a, c, l = _schedule()
    srv = serve.Server(h, SIZES, seed=123)
    try:
        st, fi, ticks = srv.run(a, c, l)
        assert np.all(st >= a) and np.all(fi > st)
        assert ticks >= l.max() and ticks <= l.sum()
        prods = serving.products_per_client(len(SIZES), c, l)
        for cl, n in enumerate(SIZES):
            S, p = srv.state(cl)
            assert p == prods[cl]
            ref = serving.final_state(123, cl, n, int(p))
            err = np.linalg.norm(S - ref) / np.linalg.norm(ref)
            assert err <= 1e-13 * max(1, int(p)), (cl, n, p, err)
    finally:
        srv.close()


def test_results_identical_alone_and_in_the_mix(h):
    a, c, l = _schedule()
    srv = serve.Server(h, SIZES, seed=5)
    try:
        srv.run(a, c, l)
        mixed = {cl: srv.state(cl)[0] for cl in range(len(SIZES))}
        for cl in (0, 3):
            srv.reset()
            sel = c == cl
            srv.run(a[sel], c[sel], l[sel])
            alone, _ = srv.state(cl)
            assert np.array_equal(alone.view(np.int64), mixed[cl].view(np.int64)), cl
        # reset really restores the identity
        srv.reset()
        S, p = srv.state(2)
        assert p == 0 and np.array_equal(S, np.eye(SIZES[2]))
    finally:
        srv.close()


def test_budget_and_argument_errors(h):
    need = serve.bytes_needed(SIZES)
    with pytest.raises(bgemm.BgemmError) as e:
        serve.Server(h, SIZES, seed=1, budget=need - 1)
    assert e.value.status == 4
    with pytest.raises(bgemm.BgemmError) as e:
        serve.Server(h, [32, 0], seed=1)
    assert e.value.status == 1
    srv = serve.Server(h, SIZES, seed=1, budget=need)
    try:
        with pytest.raises(bgemm.BgemmError) as e:
            srv.run([0.0, 0.0], [0, 9], [1, 1])
        assert e.value.status == 1
        st, fi, ticks = srv.run([], [], [])
        assert ticks == 0
    finally:
        srv.close()
