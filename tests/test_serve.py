"""Serving scheduler on the CPU (virtual clock, simulated service times):
every request is served once, per-stream FIFO admission, the HBM budget is
never exceeded, small budgets defer and evict instead of deadlocking,
oversized streams are rejected, and the plain reference never overlaps.
The slot arena: first-fit placement, coalescing on release, and a scheduler
that evicts further when the free bytes are there but not in one piece."""
import numpy as np

from paper_2106_07927_amd import serve
from paper_2106_07927_amd.serve import FakeBackend, Server, StreamSpec


def specs():
    return [StreamSpec(640, 512, 128, 1), StreamSpec(1242, 375, 128, 2),
            StreamSpec(1920, 1080, 256, 3), StreamSpec(640, 512, 256, 4)]


def run(budget, hip_streams=8, duration=2.0, rate=30.0, mdes=1e5):
    sp = specs()
    trace = serve.make_trace(sp, rate, duration, 4, seed=5)
    be = FakeBackend(sp, mdes_per_s=mdes)
    srv = Server(sp, be, budget_bytes=budget, hip_streams=hip_streams)
    return sp, trace, be, srv, srv.run(trace, release=False)


def test_every_request_served_once_and_fifo_per_stream():
    sp, trace, be, srv, st = run(budget=64 << 30)
    assert st.served == len(trace) and st.rejected == 0
    seen = {(r.request.stream, r.request.seq) for r in st.results}
    assert len(seen) == len(trace)
    for s in range(len(sp)):
        seqs = [req.seq for (_, req) in be.submitted if req.stream == s]
        assert seqs == sorted(seqs)
    lat = st.latencies_ms()
    service = {s: sp[s].width * sp[s].height * sp[s].ndisp / 1e11 * 1e3 for s in range(len(sp))}
    for r, l in zip(st.results, lat):
        assert l >= service[r.request.stream] - 1e-9
    assert st.peak_bytes <= 64 << 30


def test_budget_is_respected_with_waits_and_evictions():
    sizes = [serve.slot_bytes(s, 8, 120) for s in specs()]
    budget = max(sizes) + min(sizes)               # room for about two slots
    sp, trace, be, srv, st = run(budget=budget, mdes=2e4)
    assert st.served == len(trace)
    assert st.peak_bytes <= budget
    assert st.deferred > 0 and st.evictions > 0
    assert srv.used_bytes <= budget
    live = sum(srv.sizes[s] for s, lst in srv.slots.items() for _ in lst)
    assert live == srv.used_bytes and be.allocs - be.frees == sum(len(v) for v in srv.slots.values())


def test_oversized_stream_is_rejected():
    sizes = [serve.slot_bytes(s, 8, 120) for s in specs()]
    budget = sorted(sizes)[-2]                      # the largest stream never fits
    sp, trace, be, srv, st = run(budget=budget)
    big = int(np.argmax(sizes))
    assert st.rejected == sum(1 for r in trace if r.stream == big)
    assert st.served == len(trace) - st.rejected


def test_plain_reference_serves_one_at_a_time():
    sp = specs()
    trace = serve.make_trace(sp, 30.0, 1.0, 4, seed=9)
    st = serve.serve_plain(trace, sp, FakeBackend(sp, mdes_per_s=5e4))
    spans = sorted((r.start, r.done) for r in st.results)
    for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
        assert b0 >= a1 - 1e-12
    assert st.served == len(trace)


def test_continuous_batching_beats_fifo_on_latency():
    sp = specs()
    trace = serve.make_trace(sp, 30.0, 2.0, 4, seed=11)
    mix = Server(sp, FakeBackend(sp, mdes_per_s=3e4), budget_bytes=1 << 40).run(trace)
    fifo = serve.serve_plain(trace, sp, FakeBackend(sp, mdes_per_s=3e4))
    assert np.percentile(mix.latencies_ms(), 99) <= np.percentile(fifo.latencies_ms(), 99)


def test_slot_bytes_match_the_library_workspace():
    """The scheduler's slot size uses the library's workspace formula."""
    import os
    from paper_2106_07927_amd import sgm
    if not os.path.exists(sgm.LIB_PATH):
        import pytest
        pytest.skip("libsgm.so not built")
    lib = sgm.load_library()
    a = serve.Arena.round
    for sp in specs() + [StreamSpec(320, 240, 100, 5), StreamSpec(64, 48, 7, 6)]:
        for npaths in (4, 8):
            for p2 in (86, 120, 127, 128, 200, 300):
                n = sp.width * sp.height
                fixed = 2 * a(n) + 2 * a(8 * n) + a(n * sp.ndisp) + 2 * a(2 * n)
                work = lib.sgm_aggregate_select_work_bytes(sp.width, sp.height, sp.ndisp, npaths, p2)
                assert serve.slot_bytes(sp, npaths, p2) == fixed + a(work), (sp, npaths, p2)


def test_arena_first_fit_and_coalescing():
    ar = serve.Arena(10 * 256 + 17)
    assert ar.capacity == 10 * 256
    a = ar.alloc(300)            # 2 units
    b = ar.alloc(256)            # 1 unit
    c = ar.alloc(1000)           # 4 units
    assert (a, b, c) == (0, 512, 768)
    assert ar.alloc(4 * 256) is None          # 3 units left
    ar.release(b, 256)
    assert ar.largest_free() == 3 * 256
    ar.release(a, 300)                        # merges with b's range
    assert ar.free[0] == (0, 3 * 256)
    ar.release(c, 1000)                       # everything merges back
    assert ar.free == [(0, 10 * 256)] and ar.used == 0


def test_arena_fragmentation_forces_extra_evictions():
    """Budget bytes that are free but split: the scheduler releases more
    idle slots until one range fits, and never exceeds the arena."""
    sp = specs()
    sizes = [serve.slot_bytes(s, 8, 120) for s in sp]
    budget = serve.Arena.round(max(sizes) + min(sizes) + 2 * sorted(sizes)[1])
    trace = serve.make_trace(sp, 30.0, 2.0, 4, seed=21)
    be = FakeBackend(sp, mdes_per_s=2e4, arena_bytes=budget)
    srv = Server(sp, be, budget_bytes=budget, hip_streams=8)
    st = srv.run(trace, release=False)
    assert st.served == len(trace) and st.rejected == 0
    assert st.evictions > 0 and st.deferred > 0
    assert be.arena.used == sum(serve.Arena.round(srv.sizes[t]) for t, lst in srv.slots.items()
                                for _ in lst)
    assert be.arena.used <= be.arena.capacity


def test_servers_in_turn_share_one_arena():
    """A run hands its slots back to the backend, so a second server on the
    same arena can place its own (it used to wait forever for memory that
    the first server still held)."""
    sp = specs()
    sizes = [serve.slot_bytes(s, 8, 120) for s in sp]
    cap = serve.Arena.round(sum(serve.Arena.round(b) for b in sizes))
    be = FakeBackend(sp, mdes_per_s=5e4, arena_bytes=cap)
    trace = serve.make_trace(sp, 30.0, 1.0, 4, seed=31)
    for _ in range(3):
        st = Server(sp, be, budget_bytes=cap, hip_streams=4).run(trace)
        assert st.served == len(trace) and st.rejected == 0
        assert be.arena.used == 0 and be.arena.free == [(0, be.arena.capacity)]
    assert be.allocs == be.frees


def test_memory_held_elsewhere_rejects_instead_of_hanging():
    """When the backend's arena is taken by someone else, frames that can
    never get a slot are rejected; the run still ends."""
    sp = specs()
    sizes = [serve.slot_bytes(s, 8, 120) for s in sp]
    cap = serve.Arena.round(sum(serve.Arena.round(b) for b in sizes))
    be = FakeBackend(sp, mdes_per_s=5e4, arena_bytes=cap)
    held = be.arena.alloc(cap - serve.Arena.round(min(sizes)))   # room for the smallest only
    trace = serve.make_trace(sp, 30.0, 1.0, 4, seed=32)
    st = Server(sp, be, budget_bytes=cap, hip_streams=4).run(trace)
    small = int(np.argmin(sizes))
    assert st.served == sum(1 for r in trace if r.stream == small)
    assert st.rejected == len(trace) - st.served
    be.arena.release(held, cap - serve.Arena.round(min(sizes)))
    assert be.arena.used == 0
