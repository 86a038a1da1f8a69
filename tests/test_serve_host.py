"""Host logic of the server: the HBM pool allocator, slot layout and the
per-generation selection seeds (no GPU)."""
import numpy as np

from paper_2504_06067_amd import serve
from paper_2504_06067_amd import workloads as wl


def test_pool_first_fit_and_coalescing():
    p = serve.Pool(4096, "cpu")
    a = p.alloc(1000)   # -> 1024 bytes
    b = p.alloc(256)
    c = p.alloc(2000)   # -> 2048
    assert (a, b, c) == (0, 1024, 1280)
    assert p.alloc(1024) is None            # only 768 left
    p.release(b, 256)
    assert p.alloc(800) is None             # hole of 256 and tail of 768 are apart
    assert p.alloc(200) == 1024             # first fit takes the hole
    p.release(1024, 200)
    p.release(a, 1000)
    p.release(c, 2000)
    assert p.free == [(0, 4096)] and p.used() == 0


def test_pool_views_are_disjoint():
    p = serve.Pool(1 << 16, "cpu")
    lay, nb = serve.slot_layout(1000, 5, 495, 12, False)
    o1 = p.alloc(nb) if nb <= p.size else None
    assert o1 is None or o1 == 0
    spans = sorted(lay.values())
    for (o, n), (o2, _) in zip(spans, spans[1:]):
        assert o + n <= o2 and o % 256 == 0


def test_slot_layout_plain_holds_header():
    lay_b, nb_b = serve.slot_layout(2000, 3, 861, 12, False)
    lay_p, nb_p = serve.slot_layout(2000, 3, 861, 12, True)
    assert lay_p["ws"][1] > lay_b["ws"][1]
    assert nb_p >= nb_b


def test_selection_seeds_differ_per_generation_and_run():
    s = {serve.selection_seed(seed, g) for seed in range(20) for g in range(1, 51)}
    assert len(s) == 1000


def test_served_trace_shape():
    tr = wl.served_trace(0, 50, qps=10.0)
    assert [q["rid"] for q in tr] == list(range(50))
    arr = np.array([q["arrival"] for q in tr])
    assert arr[0] == 0 and np.all(np.diff(arr) > 0)
    for q in tr:
        assert 1000 <= q["M"] <= 100000 and q["M"] % 2 == 0 and q["N"] == q["M"] // 2
        assert q["m"] in (3, 5, 10, 15) and q["Z"].shape[1] == q["m"]
        assert q["A"].shape == (q["m"], q["d"] - 1)
    H = {q["m"]: len(q["Z"]) for q in tr}
    assert H == {3: 861, 5: 495, 10: 220, 15: 135}


def _admission(arrivals, sizes, capacity, max_bypass):
    """Drive admit_arrived over a fake pool of `capacity` units where nothing
    is released; returns the admission order."""
    import collections

    queue = collections.deque(dict(rid=i, arrival=a, size=s)
                              for i, (a, s) in enumerate(zip(arrivals, sizes)))
    used = [0]
    order = []

    def try_admit(q):
        if q["size"] > capacity:
            return None
        if used[0] + q["size"] > capacity:
            return False
        used[0] += q["size"]
        order.append(q["rid"])
        return True

    passed = {}
    n = serve.admit_arrived(queue, 10.0, try_admit, passed, max_bypass)
    return order, n, passed, [q["rid"] for q in queue]


def test_admission_lets_fitting_requests_pass_a_blocked_one():
    # request 1 (size 8) does not fit after request 0 (size 5) of capacity 10;
    # the small requests behind it pass it
    order, n, passed, left = _admission([0, 1, 2, 3], [5, 8, 1, 2], 10, max_bypass=8)
    assert order == [0, 2, 3] and left == [1]
    assert n == 2 and passed == {1: 2}


def test_admission_bypass_is_bounded():
    # after two requests passed it, the blocked request holds the queue
    order, n, passed, left = _admission([0, 1, 2, 3, 4], [5, 8, 1, 1, 1], 10, max_bypass=2)
    assert order == [0, 2, 3] and left == [1, 4] and passed == {1: 2}
    # strict FIFO with no bypass at all
    order, _, _, left = _admission([0, 1, 2], [5, 8, 1], 10, max_bypass=0)
    assert order == [0] and left == [1, 2]


def test_admission_drops_what_can_never_fit_and_waits_for_arrivals():
    order, _, _, left = _admission([0, 1, 20], [1, 50, 1], 10, max_bypass=8)
    assert order == [0] and left == [2]
