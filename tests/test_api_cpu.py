"""Host logic of the tensor helpers (CPU): the plan cache is keyed by stream
and thread and bounded (least recently used plans are dropped)."""
import threading
import types

import pytest

from paper_1507_02525_amd import api


class _FakePlan:
    made = 0

    def __init__(self, m=0, batch=1, dtype="c64", device=None, **kw):
        _FakePlan.made += 1
        self.key = (m, batch, dtype, str(device))


@pytest.fixture
def fake(monkeypatch):
    cur = {"s": 11}
    monkeypatch.setattr(api, "Plan", _FakePlan)
    monkeypatch.setattr(api.torch.cuda, "current_stream",
                        lambda device=None: types.SimpleNamespace(cuda_stream=cur["s"]))
    api.clear_plan_cache()
    _FakePlan.made = 0
    yield cur
    api.clear_plan_cache()


def test_same_key_same_plan(fake):
    a = api.get_plan(10, 2, "c64", "cuda:0")
    b = api.get_plan(10, 2, "c64", "cuda:0")
    assert a is b and _FakePlan.made == 1


def test_other_stream_other_plan(fake):
    a = api.get_plan(10, 2, "c64", "cuda:0")
    fake["s"] = 12                                   # a call queued on another stream
    b = api.get_plan(10, 2, "c64", "cuda:0")
    assert a is not b and _FakePlan.made == 2


def test_other_thread_other_plan(fake):
    a = api.get_plan(10, 2, "c64", "cuda:0")
    got = []
    t = threading.Thread(target=lambda: got.append(api.get_plan(10, 2, "c64", "cuda:0")))
    t.start()
    t.join()
    assert got[0] is not a


def test_cache_is_bounded_lru(fake):
    first = api.get_plan(1, 1, "c64", "cuda:0")
    for m in range(2, 2 + api.CACHE_SIZE - 1):
        api.get_plan(m, 1, "c64", "cuda:0")
    assert api.get_plan(1, 1, "c64", "cuda:0") is first          # touched: most recent now
    api.get_plan(100, 1, "c64", "cuda:0")                       # evicts the least recent (m = 2)
    assert len(api._cache) == api.CACHE_SIZE
    assert api.get_plan(1, 1, "c64", "cuda:0") is first
    n = _FakePlan.made
    api.get_plan(2, 1, "c64", "cuda:0")                         # was evicted: made again
    assert _FakePlan.made == n + 1
