"""Host-side tests of the request loop: the scheduler's rules on a virtual
clock (bs_simulate, no device), argument checks, the request workload, and
pins for the CPU replay of the final states (oracle/serving.py)."""
import math

import numpy as np
import pytest

from oracle import philox, serving
from paper_2203_09353_amd import bgemm, serve


def _check_schedule(nc, a, c, l, st, fi, tick):
    eps = 1e-9
    assert np.all(st >= a - eps)
    # each request lasts exactly its chain length in ticks
    assert np.allclose(fi - st, l * tick, rtol=0, atol=1e-6 * tick + 1e-12 * l.max())
    for cl in range(nc):
        idx = np.nonzero(c == cl)[0]
        prev_finish = 0.0
        for r in idx:                     # arrival order = FIFO order
            assert st[r] >= prev_finish - eps
            # work conserving: started within one tick of becoming startable
            ready = max(a[r], prev_finish)
            assert st[r] - ready <= tick + eps
            prev_finish = fi[r]


@pytest.mark.parametrize("rate,tick", [(500.0, 1e-4), (20000.0, 2e-4), (3000.0, 5e-3)])
def test_scheduler_rules_on_a_virtual_clock(rate, tick):
    nc = 16
    a, c, l = serve.requests(3, nc, rate, 0.2)
    st, fi, ticks = serve.simulate(nc, a, c, l, tick)
    _check_schedule(nc, a, c, l, st, fi, tick)
    # every tick serves at least one request; products = sum of lengths
    assert ticks <= l.sum()
    assert ticks >= l.max()


def test_one_client_is_served_alone_in_order():
    a = np.array([0.0, 0.0, 0.0])
    c = np.array([0, 0, 0])
    l = np.array([2, 1, 3])
    st, fi, ticks = serve.simulate(1, a, c, l, 1.0)
    assert ticks == 6
    assert list(st) == [0.0, 2.0, 3.0]
    assert list(fi) == [2.0, 3.0, 6.0]


def test_clients_share_ticks():
    # two clients arriving together run in the same ticks
    a = np.array([0.0, 0.0])
    st, fi, ticks = serve.simulate(2, a, np.array([0, 1]), np.array([4, 4]), 1.0)
    assert ticks == 4 and list(fi) == [4.0, 4.0]


def test_idle_gaps_jump_to_the_next_arrival():
    st, fi, ticks = serve.simulate(2, np.array([0.0, 10.0]), np.array([0, 1]), np.array([1, 1]),
                                   0.5)
    assert list(st) == [0.0, 10.0] and list(fi) == [0.5, 10.5] and ticks == 2


@pytest.mark.parametrize("a,c,l", [
    ([1.0, 0.5], [0, 0], [1, 1]),      # arrivals not ascending
    ([0.0], [3], [1]),                  # client out of range
    ([0.0], [0], [0]),                  # empty chain
    ([-1.0], [0], [1]),                 # negative arrival
])
def test_schedule_argument_errors(a, c, l):
    with pytest.raises(bgemm.BgemmError) as e:
        serve.simulate(2, a, c, l, 1e-3)
    assert e.value.status == 1


def test_workload_recipe():
    sizes = serve.client_sizes(5, 64)
    assert set(sizes.tolist()) <= {32, 64, 128, 256, 512}
    assert len(set(sizes.tolist())) == 5
    a, c, l = serve.requests(5, 64, 20000.0, 1.0)
    assert abs(len(a) - 20000) < 4 * math.sqrt(20000)
    assert np.all(np.diff(a) >= 0) and a[-1] < 1.0
    assert l.min() == 1 and l.max() == 16 and abs(l.mean() - 8.5) < 0.2
    assert c.min() == 0 and c.max() == 63
    gaps = np.diff(a)
    assert abs(gaps.mean() * 20000 - 1) < 0.05 and abs(gaps.std() / gaps.mean() - 1) < 0.05


def test_bytes_needed():
    # three n x n binary64 buffers per client, plus two sets (two ticks in
    # flight) of a 32-byte job and three 8-byte pointers
    assert serve.bytes_needed([32, 64]) == 3 * 8 * (32 * 32 + 64 * 64) + 2 * 2 * (32 + 24)


def test_replay_pins():
    n = 9
    F0 = philox.factor(21, 2, 0, n, serving.scale(n))
    F1 = philox.factor(21, 2, 1, n, serving.scale(n))
    assert np.array_equal(serving.final_state(21, 2, n, 0), np.eye(n))
    # identity start: the first product is exactly the first factor
    assert np.array_equal(serving.final_state(21, 2, n, 1), F0)
    S2 = serving.final_state(21, 2, n, 2)
    ref = F1 @ F0
    assert np.linalg.norm(S2 - ref) <= 1e-14 * np.linalg.norm(ref)
    assert list(serving.products_per_client(3, [0, 2, 0], [4, 1, 2])) == [6, 0, 1]


def test_serial_baseline_runs_one_request_at_a_time():
    nc = 8
    a, c, l = serve.requests(4, nc, 3000.0, 0.05)
    tick = 1e-4
    st, fi, ticks = serve.simulate(nc, a, c, l, tick, max_active=1)
    order = np.argsort(st, kind="stable")
    assert np.array_equal(order, np.arange(len(a)))        # started in arrival order
    assert ticks == l.sum()                                 # one product per tick
    assert np.all(st[1:] >= fi[:-1] - 1e-12)                # never two at once
    prev = 0.0
    for r in range(len(a)):                                 # work conserving
        assert st[r] - max(a[r], prev) <= tick + 1e-12
        prev = fi[r]
    # with no limit the same schedule needs fewer ticks and finishes sooner
    st2, fi2, ticks2 = serve.simulate(nc, a, c, l, tick)
    assert ticks2 < ticks and fi2.max() < fi.max()


def test_limited_active_requests():
    nc = 8
    a, c, l = serve.requests(6, nc, 20000.0, 0.02)
    st, fi, ticks = serve.simulate(nc, a, c, l, 1e-4, max_active=3)
    # at every tick start at most three requests are in flight
    for t in np.unique(st):
        assert np.sum((st <= t) & (fi > t)) <= 3
    with pytest.raises(bgemm.BgemmError):
        serve.simulate(nc, a, c, l, 1e-4, max_active=-1)
