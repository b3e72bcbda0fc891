"""Host logic of the serving loop (no GPU): admission by footprint, FIFO order,
rejection of requests larger than the budget, and the request stream."""
from paper_2405_14903_amd.serving import Admission, Request, make_stream, episode_bytes


def _req(i, n):
    return Request(i, float(i), n, 8, "fwd", i)


def test_admission_respects_budget_and_order():
    adm = Admission(budget_bytes=100, max_active=3, footprint=lambda r: r.n)
    for i, n in enumerate([40, 50, 30, 20, 101]):
        ok = adm.offer(_req(i, n))
        assert ok == (n <= 100)
    got = adm.admit()
    assert [r.rid for r in got] == [0, 1]          # 40 + 50 fit, 30 would exceed
    assert adm.used == 90
    assert adm.admit() == []
    adm.release(got[0])
    got2 = adm.admit()
    assert [r.rid for r in got2] == [2, 3]         # FIFO: 30 then 20
    assert adm.used == 100 and len(adm.active) == 3
    adm.release(got[1])
    adm.release(got2[0])
    adm.release(got2[1])
    assert adm.used == 0 and not adm.active


def test_slot_limit():
    adm = Admission(budget_bytes=10 ** 9, max_active=2, footprint=lambda r: 1)
    for i in range(5):
        adm.offer(_req(i, 1))
    assert len(adm.admit()) == 2
    assert len(adm.admit()) == 0


def test_stream_is_seeded_and_shaped():
    a = make_stream(200, rate=50.0, seed=3)
    b = make_stream(200, rate=50.0, seed=3)
    assert [(r.arrival, r.n, r.steps, r.mode) for r in a] == [(r.arrival, r.n, r.steps, r.mode) for r in b]
    assert all(a[i].arrival < a[i + 1].arrival for i in range(199))
    assert {r.n for r in a} <= {32, 48, 64, 96, 128, 192}
    assert all(8 <= r.steps <= 64 for r in a)
    assert {r.mode for r in a} == {"fwd", "fwd+adj"}
    mean_gap = a[-1].arrival / 200
    assert 0.01 < mean_gap < 0.03                  # rate 50 req/s
    assert episode_bytes(64, 32, "fwd+adj") > episode_bytes(64, 32, "fwd")
