"""The serving loop's scheduling on the CPU with a fake executor: grouping
by (index, k) in arrival order, the batch limit, admission against the
memory budget (back-pressure, never failure), and every request answered
once."""
import numpy as np

from paper_1603_08390_amd import serving


class FakeExecutor:
    def __init__(self, bytes_per_query=100, polls=3):
        self.bytes_per_query = bytes_per_query
        self.polls = polls
        self.launched = []
        self.live = 0
        self.max_live = 0

    def free_memory(self):
        return 10 ** 9

    def need_bytes(self, group):
        return self.bytes_per_query * len(group)

    def launch(self, slot, group):
        self.launched.append((slot, [q.rid for q in group], group[0].target, group[0].k))
        self.live += 1
        self.max_live = max(self.max_live, self.live)
        return {"left": self.polls, "group": group}

    def done(self, h):
        h["left"] -= 1
        if h["left"] <= 0:
            self.live -= 1
            return True
        return False

    def fetch(self, h):
        g = h["group"]
        ids = np.array([[q.rid] * q.k for q in g], dtype=np.uint32)
        return ids, ids.copy()


def _reqs(n, rng):
    out = []
    for i in range(n):
        out.append(serving.Request(i, "a" if i % 3 else "b", int(rng.choice([1, 2])), 0.0,
                                   items=np.zeros((1, 3), np.uint32)))
    return out


def test_every_request_answered_once_and_grouped():
    ex = FakeExecutor()
    srv = serving.Server(slots=3, max_batch=5, hbm_budget=10 ** 6, executor=ex)
    reqs = _reqs(40, np.random.default_rng(0))
    res = srv.run(reqs)
    assert sorted(r.rid for r in res) == list(range(40))
    for r in res:
        assert r.ids[0] == r.rid
    by_id = {q.rid: q for q in reqs}
    for slot, rids, target, k in ex.launched:
        assert len(rids) <= 5
        assert all(by_id[r].target == target and by_id[r].k == k for r in rids)
    assert ex.max_live <= 3
    assert srv.in_use == 0


def test_memory_budget_queues_instead_of_failing():
    ex = FakeExecutor(bytes_per_query=100)
    srv = serving.Server(slots=4, max_batch=8, hbm_budget=250, executor=ex)
    res = srv.run(_reqs(30, np.random.default_rng(1)))
    assert len(res) == 30
    assert srv.waited_for_memory > 0
    for _, rids, _, _ in ex.launched:
        assert len(rids) * 100 <= 250


def test_arrival_order_is_respected():
    ex = FakeExecutor(polls=1)
    srv = serving.Server(slots=1, max_batch=1, hbm_budget=10 ** 6, executor=ex)
    reqs = [serving.Request(i, "a", 1, 0.001 * (9 - i), items=np.zeros((1, 3), np.uint32))
            for i in range(10)]
    srv.run(reqs)
    assert [rids[0] for _, rids, _, _ in ex.launched] == list(range(9, -1, -1))


def test_groups_keep_arrival_order_within_a_key_under_memory_pressure():
    ex = FakeExecutor(bytes_per_query=100, polls=2)
    srv = serving.Server(slots=2, max_batch=6, hbm_budget=300, executor=ex)
    rng = np.random.default_rng(2)
    reqs = [serving.Request(i, "a" if rng.random() < 0.5 else "b", 1, 0.0,
                            items=np.zeros((1, 3), np.uint32)) for i in range(50)]
    res = srv.run(reqs)
    assert sorted(r.rid for r in res) == list(range(50))
    for target in ("a", "b"):
        order = [r for _, rids, t, _ in ex.launched if t == target for r in rids]
        assert order == sorted(order)


class HoldingExecutor(FakeExecutor):
    """Like a graph executor: the first group of each (slot, index, k) makes a
    plan of fixed size that stays; groups themselves need nothing more."""

    def __init__(self, plan_bytes):
        super().__init__(bytes_per_query=0, polls=2)
        self.plan_bytes = plan_bytes
        self.plans = set()

    def need_bytes(self, group):
        return 0

    def new_held_bytes(self, slot, group):
        return 0 if (slot, group[0].target, group[0].k) in self.plans else self.plan_bytes

    def held_bytes(self):
        return self.plan_bytes * len(self.plans)

    def release_held(self):
        assert self.live == 0
        self.plans.clear()

    def launch(self, slot, group):
        self.plans.add((slot, group[0].target, group[0].k))
        assert self.held_bytes() <= self.budget
        return super().launch(slot, group)


def test_memory_held_between_groups_counts_against_the_budget():
    # room for three plans: the kinds that would need a fourth plan run on
    # slots that already hold theirs, and every request is still answered
    ex = HoldingExecutor(plan_bytes=100)
    ex.budget = 350
    srv = serving.Server(slots=4, max_batch=4, hbm_budget=350, executor=ex)
    res = srv.run(_reqs(60, np.random.default_rng(3)))
    assert sorted(r.rid for r in res) == list(range(60))
    assert len(ex.plans) <= 3
    assert srv.released > 0
    assert srv.in_use == 0


def test_request_that_can_never_fit_raises():
    import pytest
    ex = FakeExecutor(bytes_per_query=1000)
    srv = serving.Server(slots=2, max_batch=4, hbm_budget=500, executor=ex)
    with pytest.raises(MemoryError):
        srv.run(_reqs(3, np.random.default_rng(4)))
