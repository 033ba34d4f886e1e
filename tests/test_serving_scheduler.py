"""The serving loop's scheduling rules on the CPU (no device): admission by
memory budget, per-stream order, in-flight limits, continuous batching."""
import random

import pytest

from paper_2505_07158_amd.serving import Request, Scheduler


class FakeHandle:
    def __init__(self):
        self.finished = False

    def query(self):
        return self.finished


class FakeBackend:
    def __init__(self):
        self.launched = []   # (kind, [(stream, seq)], handle)

    def launch(self, kind, reqs):
        h = FakeHandle()
        self.launched.append((kind, [(r.stream, r.seq) for r in reqs], h))
        return h

    def finish_all(self):
        for _, _, h in self.launched:
            h.finished = True


def req(stream, seq, kind="enc", nbytes=10, arrival=0.0):
    return Request(stream=stream, seq=seq, kind=kind, frame=None, out=None, nbytes=nbytes, arrival=arrival)


def test_frames_of_a_stream_launch_in_order():
    be = FakeBackend()
    s = Scheduler(be.launch, hbm_budget=1000)
    s.submit(req(0, 1))          # frame 1 arrives before frame 0
    s.submit(req(1, 0))
    s.pump()
    assert be.launched[0][1] == [(1, 0)]          # stream 0 waits for its frame 0
    s.submit(req(0, 0))
    be.finish_all()
    s.pump()
    assert be.launched[1][1] == [(0, 0), (0, 1)]  # then both, in sequence order
    be.finish_all()
    s.pump()
    assert s.idle() and len(s.completed) == 3


def test_budget_limits_in_flight_bytes():
    be = FakeBackend()
    s = Scheduler(be.launch, hbm_budget=100, max_inflight=4)
    for k in range(10):
        s.submit(req(k, 0, nbytes=30))
    s.pump()
    # 3 requests fit in the first batch; nothing else fits while it is in flight
    assert [len(b) for _, b, _ in be.launched] == [3]
    assert s.inflight_bytes == 90
    be.finish_all()
    s.pump()
    assert [len(b) for _, b, _ in be.launched] == [3, 3]


def test_oversized_request_runs_alone():
    be = FakeBackend()
    s = Scheduler(be.launch, hbm_budget=100)
    s.submit(req(0, 0, nbytes=500))
    s.submit(req(1, 0, nbytes=10))
    s.pump()
    assert be.launched[0][1] == [(0, 0)]
    assert len(be.launched) == 1     # the small one waits: the big one holds more than the budget
    be.finish_all()
    s.pump()
    assert be.launched[1][1] == [(1, 0)]


def test_inflight_limit_and_continuous_admission():
    be = FakeBackend()
    s = Scheduler(be.launch, hbm_budget=10**9, max_inflight=2)
    s.submit(req(0, 0))
    s.pump()
    s.submit(req(1, 0))
    s.pump()
    s.submit(req(2, 0))
    s.pump()
    assert len(be.launched) == 2                   # two batches in flight, the third request waits
    be.launched[0][2].finished = True
    s.pump()                                       # a slot frees: the waiting request is admitted
    assert len(be.launched) == 3 and be.launched[2][1] == [(2, 0)]


def test_encrypt_and_decrypt_are_independent_kinds():
    be = FakeBackend()
    s = Scheduler(be.launch, hbm_budget=10**9, max_inflight=1)
    s.submit(req(0, 0, "enc"))
    s.submit(req(0, 0, "dec"))     # same stream id, other context: its own sequence
    s.pump()
    assert sorted(k for k, _, _ in be.launched) == ["dec", "enc"]


@pytest.mark.parametrize("seed", range(5))
def test_random_arrivals_all_complete_in_order(seed):
    rng = random.Random(seed)
    be = FakeBackend()
    s = Scheduler(be.launch, hbm_budget=200, max_inflight=2, max_batch=7)
    reqs = [req(st, q, rng.choice(["enc", "dec"]) if st % 2 else "enc", nbytes=rng.randint(1, 60))
            for st in range(6) for q in range(12)]
    # per stream (and kind) sequence numbers must be dense: renumber per (kind, stream)
    nxt = {}
    for r in reqs:
        r.seq = nxt.get((r.kind, r.stream), 0)
        nxt[(r.kind, r.stream)] = r.seq + 1
    order = list(reqs)
    rng.shuffle(order)
    for r in order:
        s.submit(r)
        s.pump()
        if rng.random() < 0.5:
            for _, _, h in be.launched:
                if rng.random() < 0.5:
                    h.finished = True
        assert s.inflight_bytes <= 200 or len(s.inflight) == 1
    while not s.idle():
        be.finish_all()
        s.pump()
    assert len(s.completed) == len(reqs)
    launched_seq = {}
    for kind, items, _ in be.launched:
        for st, q in items:
            assert q == launched_seq.get((kind, st), 0)
            launched_seq[(kind, st)] = q + 1


def test_batch_class_keeps_batches_homogeneous():
    be = FakeBackend()
    cls = {0: "small", 1: "big", 2: "small", 3: "big"}
    s = Scheduler(be.launch, hbm_budget=10**9, max_inflight=8, batch_class=lambda r: cls[r.stream])
    for q in range(3):
        for st in range(4):
            s.submit(req(st, q))
    s.pump()
    assert len(be.launched) == 2
    for _, items, _ in be.launched:
        assert len({cls[st] for st, _ in items}) == 1
    assert sorted(len(items) for _, items, _ in be.launched) == [6, 6]


def test_per_stream_inflight_limit():
    be = FakeBackend()
    s = Scheduler(be.launch, hbm_budget=10**9, max_inflight=8, max_stream_inflight=2)
    for q in range(5):
        s.submit(req(0, q))
    s.pump()
    assert [items for _, items, _ in be.launched] == [[(0, 0), (0, 1)]]
    be.finish_all()
    s.pump()
    assert be.launched[1][1] == [(0, 2), (0, 3)]


def test_hash_first_hashes_beside_the_ordered_stage():
    be = FakeBackend()
    s = Scheduler(be.launch, hbm_budget=10**9, max_inflight=4, hash_first=True)
    s.submit(req(0, 1))                  # frame 1 arrives first: admission waits for frame 0
    s.pump()
    assert be.launched == []
    s.submit(req(0, 0))
    s.pump()
    assert be.launched[0][0] == "hash" and be.launched[0][1] == [(0, 0), (0, 1)]
    s.submit(req(0, 2))
    s.pump()                             # frame 2 hashes while 0 and 1 are still hashing
    assert be.launched[1][0] == "hash" and be.launched[1][1] == [(0, 2)]
    be.launched[1][2].finished = True    # frame 2 hashed first: it waits for 0 and 1
    s.pump()
    assert [k for k, _, _ in be.launched] == ["hash", "hash"]
    be.launched[0][2].finished = True
    s.pump()
    assert be.launched[2][0] == "enc" and be.launched[2][1] == [(0, 0), (0, 1), (0, 2)]
    be.finish_all()
    s.pump()
    assert s.idle() and len(s.completed) == 3 and all(r.hashed for r in s.completed)


def test_hash_first_charges_the_budget_once():
    be = FakeBackend()
    s = Scheduler(be.launch, hbm_budget=100, max_inflight=4, hash_first=True)
    for k in range(5):
        s.submit(req(k, 0, nbytes=30))
    s.pump()
    assert [len(b) for _, b, _ in be.launched] == [3] and s.inflight_bytes == 90
    be.launched[0][2].finished = True
    s.pump()                             # hashed: on to the ordered stage, still holding 90 bytes
    assert [k for k, _, _ in be.launched] == ["hash", "enc"] and s.inflight_bytes == 90
    be.finish_all()
    s.pump()                             # done: the other two are admitted
    assert s.inflight_bytes == 60 and be.launched[-1][0] == "hash"


@pytest.mark.parametrize("seed", range(4))
def test_hash_first_random_arrivals(seed):
    rng = random.Random(100 + seed)
    be = FakeBackend()
    s = Scheduler(be.launch, hbm_budget=150, max_inflight=2, max_batch=5, hash_first=True, max_stream_inflight=3)
    reqs = [req(st, q, "dec" if st == 5 else "enc", nbytes=rng.randint(1, 50)) for st in range(6) for q in range(10)]
    order = list(reqs)
    rng.shuffle(order)
    for r in order:
        s.submit(r)
        s.pump()
        for _, _, h in be.launched:
            if rng.random() < 0.4:
                h.finished = True
        assert s.inflight_bytes <= 150 or len(s.inflight) == 1
        assert all(v <= 3 for v in s.stream_inflight.values())
    while not s.idle():
        be.finish_all()
        s.pump()
    assert len(s.completed) == len(reqs)
    hashed = {(st, q) for k, items, _ in be.launched if k == "hash" for st, q in items}
    assert hashed == {(r.stream, r.seq) for r in reqs if r.kind == "enc"}
    nxt = {}
    for kind, items, _ in be.launched:
        if kind == "hash":
            continue
        for st, q in items:
            assert q == nxt.get((kind, st), 0)
            nxt[(kind, st)] = q + 1


def test_failed_launch_completes_its_requests_and_breaks_only_their_streams():
    """A batch whose launch fails completes its requests with the failure's
    status and releases their budget; later frames of those streams complete
    with VC_EORDER without launching (the library's chain never advanced
    past the failed frame); other streams go on."""
    from paper_2505_07158_amd import vcipher as V
    be = FakeBackend()
    fail_streams = {1}

    def launch(kind, reqs):
        if any(r.stream in fail_streams for r in reqs):
            raise RuntimeError("launch failed")
        return be.launch(kind, reqs)

    s = Scheduler(launch, hbm_budget=1000, max_batch=1, max_inflight=4)
    s.submit(req(1, 0))
    with pytest.raises(RuntimeError):
        s.pump()
    failed = [r for r in s.completed if r.stream == 1]
    assert [(r.seq, r.status) for r in failed] == [(0, V.VC_EDEVICE)]
    assert s.inflight_bytes == 0
    fail_streams.clear()     # the backend recovers; stream 1 stays broken
    for q in range(3):
        s.submit(req(0, q))
        s.submit(req(1, q + 1))
    while not s.idle():
        s.pump()
        be.finish_all()
    by = {(r.stream, r.seq): r.status for r in s.completed}
    assert all(by[(0, q)] == 0 for q in range(3))
    assert all(by[(1, q)] == V.VC_EORDER for q in range(1, 4))
    assert all(all(st != 1 for st, _ in b) for _, b, _ in be.launched)   # stream 1 never launched again
    assert s.inflight_bytes == 0 and s.inflight == []


def test_hash_batches_have_their_own_inflight_limit():
    """max_inflight_hash: hash batches (latency-bound, few SIMDs) may run
    several at once per class while the ordered stage keeps max_inflight."""
    be = FakeBackend()
    s = Scheduler(be.launch, hbm_budget=10**9, max_inflight=1, max_batch=1, hash_first=True, max_inflight_hash=3)
    for k in range(5):
        s.submit(req(k, 0))
    s.pump()
    assert [kind for kind, _, _ in be.launched] == ["hash"] * 3     # three hash batches, not one
    assert len(s.inflight) == 3
    be.finish_all()
    s.pump()
    kinds = [kind for kind, _, _ in be.launched[3:]]
    assert kinds.count("enc") == 1 and kinds.count("hash") == 2   # one ordered batch; the last two hashes
    while not s.idle():
        be.finish_all()
        s.pump()
    assert len(s.completed) == 5 and all(r.hashed for r in s.completed)


class CheckingBackend:
    """A fake backend that checks, at every launch, the scheduler's limits:
    batches of one kind and class in flight, batch size, one class per
    batch."""

    def __init__(self, limits, max_batch, cls_of):
        self.limits, self.max_batch, self.cls_of = limits, max_batch, cls_of
        self.launched = []   # (kind, [Request], handle)

    def launch(self, kind, reqs):
        assert 1 <= len(reqs) <= self.max_batch
        cls = {self.cls_of(r) for r in reqs}
        assert len(cls) == 1
        busy = sum(1 for k, rs, h in self.launched if k == kind and self.cls_of(rs[0]) in cls and not h.finished)
        assert busy < self.limits[kind], (kind, busy)
        h = FakeHandle()
        self.launched.append((kind, list(reqs), h))
        return h


hyp = pytest.importorskip("hypothesis")
st = hyp.strategies


@hyp.settings(max_examples=60, deadline=None)
@hyp.given(budget=st.integers(20, 300), max_inflight=st.integers(1, 3), max_inflight_hash=st.integers(0, 3),
           max_batch=st.integers(1, 8), hash_first=st.booleans(), max_stream_inflight=st.integers(0, 4),
           streams=st.integers(1, 5), frames=st.integers(1, 6), classes=st.integers(1, 3),
           seed=st.integers(0, 10 ** 6))
def test_scheduler_invariants_over_random_configurations(budget, max_inflight, max_inflight_hash, max_batch,
                                                         hash_first, max_stream_inflight, streams, frames, classes,
                                                         seed):
    """Over random configurations and arrival orders, after every pump: the
    in-flight bytes are the footprints of the admitted, unfinished requests
    and stay within the budget unless one request holds them alone; per
    stream at most max_stream_inflight frames are admitted; at every launch
    the in-flight batches of that kind and class stay under their limit and
    a batch holds one class and at most max_batch requests; every request
    completes exactly once, after its last batch has finished; ordered
    batches keep each stream's frames in sequence."""
    rng = random.Random(seed)
    kinds = {st_: rng.choice(["enc", "dec"]) for st_ in range(streams)}
    cls_of = lambda r: r.stream % classes
    limits = {"enc": max_inflight, "dec": max_inflight, "hash": max_inflight_hash or max_inflight}
    be = CheckingBackend(limits, max_batch, cls_of)
    s = Scheduler(be.launch, hbm_budget=budget, max_inflight=max_inflight, max_batch=max_batch,
                  batch_class=cls_of, max_stream_inflight=max_stream_inflight, hash_first=hash_first,
                  max_inflight_hash=max_inflight_hash)
    reqs = [req(st_, q, kinds[st_], nbytes=rng.choice([1, 5, 20, 60, budget + 10]))
            for st_ in range(streams) for q in range(frames)]
    order = list(reqs)
    rng.shuffle(order)

    def last_batch(r):
        return [h for _, rs, h in be.launched if any(x is r for x in rs)][-1]

    seen = [0]

    def check():
        # requests completed by this pump: their last batch had finished
        for r in s.completed[seen[0]:]:
            assert last_batch(r).finished
        seen[0] = len(s.completed)
        admitted = [r for r in reqs if r.launched == r.launched and r.done != r.done]
        assert s.inflight_bytes == sum(r.nbytes for r in admitted)
        assert s.inflight_bytes <= budget or len(admitted) == 1
        if max_stream_inflight:
            per = {}
            for r in admitted:
                per[(r.kind, r.stream)] = per.get((r.kind, r.stream), 0) + 1
            assert all(v <= max_stream_inflight for v in per.values())

    for r in order:
        s.submit(r)
        s.pump()
        check()
        for _, _, h in be.launched:
            if rng.random() < 0.5:
                h.finished = True
    for _ in range(10 * len(reqs) + 10):
        if s.idle():
            break
        for _, _, h in be.launched:
            h.finished = True
        s.pump()
        check()
    assert s.idle()
    assert sorted(id(r) for r in s.completed) == sorted(id(r) for r in reqs)
    assert all(r.status == 0 for r in reqs)
    nxt = {}
    for kind, rs, _ in be.launched:
        if kind == "hash":
            continue
        for r in rs:
            assert r.seq == nxt.get((kind, r.stream), 0)
            nxt[(kind, r.stream)] = r.seq + 1
    hashed = {(r.stream, r.seq) for k, rs, _ in be.launched if k == "hash" for r in rs}
    assert hashed == ({(r.stream, r.seq) for r in reqs if r.kind == "enc"} if hash_first else set())
