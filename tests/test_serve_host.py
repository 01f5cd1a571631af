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
    # two resident n x n binary64 states per client, a factor pool holding
    # every client's factor (256-byte aligned), plus two sets (two ticks in
    # flight) of a 32-byte job, three 8-byte pointers and six 4-byte sizes
    assert serve.bytes_needed([32, 64]) == 3 * 8 * (32 * 32 + 64 * 64) + 2 * 2 * (32 + 24 + 24)
    assert serve.bytes_needed([7]) == 2 * 8 * 49 + 512 + 2 * (32 + 24 + 24)


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


def _overlap(st, fi, i, j):
    return st[i] < fi[j] and st[j] < fi[i]


@pytest.mark.parametrize("rate", [2000.0, 30000.0])
def test_lockstep_rounds(rate):
    """Lock step: requests start only at round boundaries, when no request is
    active; requests that overlap in time started together; each round lasts
    its longest chain; requests of one client still run in arrival order."""
    nc, tick = 16, 1e-4
    a, c, l = serve.requests(7, nc, rate, 0.05)
    st, fi, ticks = serve.simulate(nc, a, c, l, tick, policy=serve.POLICY_LOCKSTEP)
    starts = np.unique(st)
    for t in starts:
        rnd = np.nonzero(st == t)[0]
        # the round ends with its longest chain; nothing else starts before
        end = t + l[rnd].max() * tick
        assert np.allclose(fi[rnd], t + l[rnd] * tick)
        later = st > t
        assert np.all(st[later] >= end - 1e-9)
    for i in range(len(a)):
        assert st[i] >= a[i] - 1e-12
    for cl in range(nc):
        idx = np.nonzero(c == cl)[0]
        assert np.all(np.diff(st[idx]) > 0)
    # the same arrivals under continuous batching finish no later, on average
    st2, fi2, ticks2 = serve.simulate(nc, a, c, l, tick)
    assert (fi2 - a).mean() <= (fi - a).mean()
    assert ticks2 <= ticks or rate < 5000


def test_pool_admission_holds_the_budget():
    """A factor pool smaller than every client's factor at once: the bytes
    held by active requests never exceed it, requests wait (counted), every
    request still completes, and a pool holding every factor gives the same
    schedule as no pool at all."""
    sizes = np.array([32, 64, 128, 256, 512, 256, 128, 64], dtype=np.int32)
    need = sizes.astype(np.int64) ** 2 * 8
    nc, tick = len(sizes), 1e-4
    a, c, l = serve.requests(8, nc, 40000.0, 0.02)
    pool = int(need.max() + need[3])                  # the largest plus one 256^2
    st, fi, ticks, waits = serve.simulate(nc, a, c, l, tick, sizes=sizes, pool_bytes=pool,
                                          with_waits=True)
    assert waits > 0 and np.all(fi > st)
    for t in np.unique(st):
        held = (st <= t) & (fi > t)
        assert need[c[held]].sum() <= pool
    # no limit from the pool: identical to the unlimited schedule
    st0, fi0, ticks0 = serve.simulate(nc, a, c, l, tick)
    st1, fi1, ticks1, w1 = serve.simulate(nc, a, c, l, tick, sizes=sizes,
                                          pool_bytes=int(need.sum()), with_waits=True)
    assert w1 == 0 and ticks1 == ticks0
    assert np.array_equal(st1, st0) and np.array_equal(fi1, fi0)
    # the tight pool costs time
    assert fi.max() > fi0.max()


def test_pool_oldest_request_is_not_overtaken():
    # one client of 512 (2 MiB factor) and one of 32; a pool of one 512 factor:
    # while the first 512 request runs, a 32 request that arrived after a
    # waiting 512 request must not start before it
    sizes = [512, 32, 512]
    need = [512 * 512 * 8, 32 * 32 * 8, 512 * 512 * 8]
    a = np.array([0.0, 0.0, 0.0])
    c = np.array([0, 2, 1])
    l = np.array([3, 1, 1])
    st, fi, ticks, waits = serve.simulate(3, a, c, l, 1.0, sizes=sizes, pool_bytes=need[0],
                                          with_waits=True)
    assert list(st) == [0.0, 3.0, 4.0] and list(fi) == [3.0, 4.0, 5.0] and waits > 0


def test_pool_and_policy_argument_errors():
    a, c, l = np.array([0.0]), np.array([0]), np.array([1])
    with pytest.raises(bgemm.BgemmError) as e:
        serve.simulate(1, a, c, l, 1.0, sizes=[64], pool_bytes=64 * 64 * 8 - 1)
    assert e.value.status == 4
    with pytest.raises(bgemm.BgemmError) as e:
        serve.simulate(1, a, c, l, 1.0, policy=2)
    assert e.value.status == 1
    with pytest.raises(bgemm.BgemmError) as e:
        serve.simulate(1, a, c, l, 1.0, pool_bytes=1 << 20)     # a pool needs sizes
    assert e.value.status == 1
