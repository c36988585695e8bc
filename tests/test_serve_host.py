"""Host logic of the serving loop (no GPU): admission of requests into a
launch and the latency statistics."""
import numpy as np

from paper_1805_08331_amd.serve import ASSIGN, DIST, Request, completed, latency_summary, nearest_centroid, plan_batch


def _reqs(kinds):
    pts = np.zeros((3, 2), np.float32)
    out = []
    for i, k in enumerate(kinds):
        r = Request(k, 100, [pts, pts] if k == DIST else [pts])
        r.rid = i
        out.append(r)
    return out


def test_plan_batch_pair_cap_in_arrival_order():
    """k = 4: a distance is one pair, an assignment four.  The cap of 6 pairs
    admits D, A (5 pairs); the next D would make 6 and fits; the A after it
    does not, and nothing behind it overtakes."""
    w = _reqs([DIST, ASSIGN, DIST, ASSIGN, DIST])
    b = plan_batch(w, 4, 6, 1 << 40, lambda r: 0, lambda nd, na: 0)
    assert [r.rid for r in b] == [0, 1, 2]


def test_plan_batch_memory_budget_counts_workspaces():
    """Each request costs 10 bytes, each workspace 100 per distance and 1000 per
    assignment: a budget of 1240 admits D, D, A (30 + 200 + 1000 = 1230)."""
    w = _reqs([DIST, DIST, ASSIGN, DIST])
    b = plan_batch(w, 2, 100, 1240, lambda r: 10, lambda nd, na: 100 * nd + 1000 * na)
    assert [r.rid for r in b] == [0, 1, 2]
    assert plan_batch(w, 2, 100, 1229, lambda r: 10, lambda nd, na: 100 * nd + 1000 * na) == w[:2]


def test_plan_batch_empty_when_first_request_does_not_fit():
    w = _reqs([ASSIGN, DIST])
    assert plan_batch(w, 8, 4, 1 << 40, lambda r: 0, lambda nd, na: 0) == []
    assert plan_batch([], 8, 4, 1 << 40, lambda r: 0, lambda nd, na: 0) == []


def test_latency_summary_nearest_rank():
    lat = np.arange(1, 201) * 1e-3          # 1 .. 200 ms
    s = latency_summary(lat)
    assert s["p50_ms"] == 100.0 and s["p99_ms"] == 198.0 and s["max_ms"] == 200.0 and s["n"] == 200
    assert latency_summary([])["n"] == 0
    assert latency_summary([0.005])["p99_ms"] == 5.0


def test_autotune_pick_fastest_median_and_ties():
    """The tuner keeps the candidate with the smallest median time; on a tie
    the larger switch point wins."""
    from paper_1805_08331_amd.autotune import pick_fastest
    assert pick_fastest({5e-4: [3.0, 9.0, 3.1], 8e-4: [2.9, 3.0, 30.0], 1e-3: [3.2, 3.2, 3.2]}) == 8e-4
    assert pick_fastest({5e-4: [2.0], 8e-4: [2.0]}) == 8e-4


def test_failed_launch_puts_requests_back_in_order():
    """A launch that raises leaves its requests at the head of the queue, in
    arrival order (exercised with a stand-in server: no GPU)."""
    from collections import deque
    from paper_1805_08331_amd import serve

    class _G:
        def __init__(self, reqs):
            self.waiting = deque(reqs)
            self.ws_cache = {}

    srv = serve.Server.__new__(serve.Server)
    w = _reqs([DIST, DIST, DIST])
    g = _G(w)
    srv.grids = {100: g}
    srv.streams = [None]
    srv.busy = [None]
    srv.k, srv.max_pairs, srv.mem_budget = 1, 2, 1 << 40
    srv.in_flight_bytes = srv.peak_bytes = srv.n_launches = 0
    srv.done = []
    srv._req_bytes = lambda g, r: 0
    srv._ws_bytes = lambda g, nd, na: 0

    def boom(g, stream, batch):
        raise RuntimeError("launch failed")

    srv._launch = boom
    try:
        srv.poll()
    except RuntimeError:
        pass
    else:
        raise AssertionError("the launch error was swallowed")
    assert [r.rid for r in g.waiting] == [0, 1, 2] and srv.in_flight_bytes == 0


def test_submit_rejects_points_the_discretisation_would_drop():
    """Points outside [0, 1]^2, non-finite, or with birth > death are refused at
    submission (the library would drop them silently); valid diagrams are
    stored as float32 [n, 2]."""
    from paper_1805_08331_amd import serve

    class _G:
        centroids = object()

        def __init__(self):
            from collections import deque
            self.waiting = deque()

    srv = serve.Server.__new__(serve.Server)
    srv.grids = {100: _G()}
    srv.clock = lambda: 1.0
    srv._next_id = 0
    srv.mem_budget = 1 << 40
    srv._launch_bytes = lambda g, reqs: 0
    ok = srv.submit(serve.Request(ASSIGN, 100, [[0.1, 0.5, 0.0, 1.0]]))
    assert ok.diagrams[0].dtype == np.float32 and ok.diagrams[0].shape == (2, 2) and ok.rid == 0
    for bad in ([[0.5, 0.4]], [[0.1, 1.5]], [[-0.1, 0.2]], [[np.nan, 0.3]], [[0.1, 0.2, 0.3]]):
        try:
            srv.submit(serve.Request(ASSIGN, 100, [np.asarray(bad, np.float64)]))
        except ValueError:
            pass
        else:
            raise AssertionError(bad)
    assert len(srv.grids[100].waiting) == 1


def test_submit_rejects_request_beyond_memory_budget():
    """A request that alone needs more device memory than the budget could
    never be admitted; it is refused at submission instead of blocking the
    head of its grid's queue."""
    from paper_1805_08331_amd import serve

    class _G:
        centroids = object()

        def __init__(self):
            from collections import deque
            self.waiting = deque()

    srv = serve.Server.__new__(serve.Server)
    srv.grids = {100: _G()}
    srv.clock = lambda: 1.0
    srv._next_id = 0
    srv.mem_budget = 1000
    srv._launch_bytes = lambda g, reqs: 500 * sum(len(r.diagrams[0]) for r in reqs)
    srv.submit(serve.Request(ASSIGN, 100, [[0.1, 0.5, 0.2, 0.6]]))
    try:
        srv.submit(serve.Request(ASSIGN, 100, [[0.1, 0.5, 0.2, 0.6, 0.3, 0.7]]))
    except ValueError:
        pass
    else:
        raise AssertionError("oversized request accepted")
    assert len(srv.grids[100].waiting) == 1 and srv._next_id == 1


def test_completed_requests_from_posted_records():
    """Requests own runs of records (one pair for a distance, k for an
    assignment); a request is complete when every record of its run carries
    the launch's tag.  Records of an earlier launch (another tag) do not
    count, and requests already handed out are not returned again."""
    starts = np.array([0, 1, 4, 5, 8])          # D, A(3), D, A(3)
    tags = np.array([7, 7, 7, 0, 7, 7, 7, 7], np.uint32)
    open_ = np.ones(4, bool)
    assert list(completed(tags, 7, starts, open_)) == [0, 2, 3]
    open_[[0, 2, 3]] = False
    assert list(completed(tags, 7, starts, open_)) == []
    tags[3] = 6                                 # a stale record from a previous launch
    assert list(completed(tags, 7, starts, open_)) == []
    tags[3] = 7
    assert list(completed(tags, 7, starts, open_)) == [1]
    assert list(completed(np.zeros(0, np.uint32), 1, np.array([0]), np.zeros(0, bool))) == []


def test_nearest_centroid_rule():
    """The library's assignment rule: smallest cost, ties to the lowest index,
    NaN never wins, 0 when no cost is finite."""
    assert nearest_centroid([3.0, 1.0, 2.0]) == 1
    assert nearest_centroid([2.0, 1.0, 1.0]) == 1
    assert nearest_centroid([np.nan, 5.0, 4.0]) == 2
    assert nearest_centroid([np.nan, np.nan]) == 0
    assert nearest_centroid([np.inf, np.inf, 3.0]) == 2
