"""Host logic of the serving loop (no GPU): admission by footprint with pooled
handles counted against the budget, FIFO order, least-recently-used freeing of
idle handles, rejection of requests larger than the budget, and the request
stream."""
from paper_2405_14903_amd.serving import Admission, Request, make_stream, episode_bytes


class _Handle:
    live = set()

    def __init__(self, n):
        self.n = n
        _Handle.live.add(id(self))
        self.closed = False

    def close(self):
        assert not self.closed
        self.closed = True
        _Handle.live.discard(id(self))


def _req(i, n, ep=10):
    r = Request(i, float(i), n, 8, "fwd", i)
    r._ep = ep
    return r


def _adm(budget, max_active=8):
    return Admission(budget, max_active, handle_bytes=lambda n: n, episode_bytes=lambda r: r._ep, make=_Handle)


def test_admission_counts_handles_and_episodes_fifo():
    adm = _adm(200, max_active=3)
    for i, n in enumerate([40, 50, 30, 20, 191]):
        assert adm.offer(_req(i, n)) == (n + 10 <= 200)
    got = adm.admit()
    assert [r.rid for r, h in got] == [0, 1, 2]           # 50 + 60 + 40 = 150; the slot limit stops the rest
    assert adm.used == 150
    assert adm.admit() == []
    r0, h0 = got[0]
    adm.release(r0, h0)
    assert adm.used == 140                                # the idle handle (40) stays counted
    got2 = adm.admit()
    assert [r.rid for r, h in got2] == [3]                # 20 + 10 fits next to the idle handle
    assert adm.used == 170 and len(adm.active) == 3


def test_idle_handle_reused_and_lru_freed():
    adm = _adm(100)
    adm.offer(_req(0, 40))
    (r0, h0), = adm.admit()
    adm.release(r0, h0)                                   # idle 40
    adm.offer(_req(1, 30))
    (r1, h1), = adm.admit()
    adm.release(r1, h1)                                   # idle 40, 30 (40 least recently used)
    assert adm.used == 70
    adm.offer(_req(2, 40))                                # reuses the idle 40: only its episode bytes
    (r2, h2), = adm.admit()
    assert h2 is h0 and adm.used == 80
    adm.offer(_req(3, 25))                                # needs 35: the idle 30 must go
    (r3, h3), = adm.admit()
    assert h1.closed and not h0.closed and adm.used == 40 + 10 + 25 + 10
    adm.release(r2, h2)
    adm.release(r3, h3)
    adm.close()
    assert adm.used == 0 and h0.closed and h3.closed


def test_head_of_queue_waits_for_room():
    adm = _adm(100)
    adm.offer(_req(0, 60))
    (r0, h0), = adm.admit()
    adm.offer(_req(1, 50))                                # 60 + 10 used, 60 more do not fit
    adm.offer(_req(2, 5))
    assert adm.admit() == []                              # FIFO: the small one waits behind the head
    adm.release(r0, h0)                                   # idle 60 is freed for the head
    got = adm.admit()
    assert [r.rid for r, h in got] == [1, 2] and h0.closed


def test_stream_is_seeded_and_shaped():
    a = make_stream(400, rate=50.0, seed=3)
    b = make_stream(400, rate=50.0, seed=3)
    assert [(r.arrival, r.n, r.steps, r.mode) for r in a] == [(r.arrival, r.n, r.steps, r.mode) for r in b]
    assert all(a[i].arrival < a[i + 1].arrival for i in range(399))
    assert {r.n for r in a} <= {32, 48, 64, 96, 128, 192}
    assert all(8 <= r.steps <= 64 for r in a)
    modes = [r.mode for r in a]
    assert set(modes) == {"fwd", "fwd+adj", "poisson"}
    assert 10 <= modes.count("poisson") <= 80
    mean_gap = a[-1].arrival / 400
    assert 0.01 < mean_gap < 0.03                  # rate 50 req/s
    assert episode_bytes(64, 32, "fwd+adj") > episode_bytes(64, 32, "fwd")
