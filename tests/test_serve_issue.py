"""Host logic of the serving loop's chunk issue (no GPU): a batch steps every
graph in its slots, so a graph whose cost class changed (its last stage was
just chosen) must leave its old batch before that batch steps again;
otherwise it is stepped twice in one pass of the loop and its layout depends on when
the other class had room for a chunk."""
from collections import deque
from types import SimpleNamespace

from paper_2303_03964_amd import serve


class _Event:
    def __init__(self, complete=True):
        self.complete = complete

    def record(self, stream):
        pass

    def query(self):
        return self.complete


_FAKE_TORCH = SimpleNamespace(cuda=SimpleNamespace(Event=lambda **kw: _Event()))


class _Batch:
    def __init__(self, name, log):
        self.name, self.log, self.members = name, log, set()

    def add(self, lay):
        self.members.add(lay.tag)
        self.log.append(("add", self.name, lay.tag))

    def remove(self, lay):
        self.members.discard(lay.tag)
        self.log.append(("remove", self.name, lay.tag))

    def step(self, iters, stream):
        self.log.append(("step", self.name, tuple(sorted(self.members))))


def _run(tag, n, k_mode, group, done=0, iters=200):
    lay = SimpleNamespace(tag=tag, params=SimpleNamespace(k_mode=k_mode))
    g = serve._Graph(key=tag, graph=SimpleNamespace(n=n, nnz=10 * n), lay=lay)
    run = serve._Run(g, SimpleNamespace(), iters)
    run.tuned = True  # past the final-stage choice: no box reads in this test
    run.done = done
    run.group = group
    return run


def _server(log, light=None):
    srv = object.__new__(serve.Server)
    srv.torch = _FAKE_TORCH
    srv.plain = False
    srv.chunk = 10
    srv.light_iteration = light
    srv.streams = ["s0", "s1"] if light is None else ["s0", "s1", "s2"]
    srv.batches = [_Batch(i, log) for i in range(len(srv.streams))]
    srv.max_inflight = [2] * len(srv.streams)
    return srv


def test_class_change_leaves_old_batch_before_it_steps():
    log = []
    srv = _server(log)
    small = _run("small", 2_000, -1, group=0)
    # a large graph whose last stage is now the exact method: its iterations
    # are long, so it belongs to the expensive class, but it is still a
    # member of the batch of the cheap class
    big = _run("big", 150_000, 0, group=0, done=190)
    srv.batches[0].members = {"small", "big"}
    finished, issued = srv._issue({1: small, 2: big}, [deque(), deque()])
    assert issued
    steps = [e for e in log if e[0] == "step"]
    assert ("step", 0, ("small",)) in steps
    assert ("step", 1, ("big",)) in steps
    # the move happens before the first batch steps
    assert log.index(("remove", 0, "big")) < log.index(("step", 0, ("small",)))
    assert big.group == 1 and small.group == 0


def test_class_change_while_new_class_is_full():
    # the expensive class has two chunks in flight: the moved graph waits in
    # its new batch and is not stepped by the old one
    log = []
    srv = _server(log)
    small = _run("small", 2_000, -1, group=0)
    big = _run("big", 150_000, 0, group=0, done=190)
    srv.batches[0].members = {"small", "big"}
    srv._issue({1: small, 2: big}, [deque(), deque([_Event(False), _Event(False)])])
    steps = [e for e in log if e[0] == "step"]
    assert steps == [("step", 0, ("small",))]
    assert big.done == 190 and srv.batches[1].members == {"big"}
