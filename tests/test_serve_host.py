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
