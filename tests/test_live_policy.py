"""Host logic of the live pipelining policy (Sec. 6: the newest image is the
target, frames that arrive while one is processed are skipped, not
queued): the one-frame mailbox between camera and correlator.  CPU only."""
import random
import threading

import numpy as np

from paper_1905_06228_amd import LatestFrame


def test_take_returns_newest_and_counts_skips():
    box = LatestFrame()
    assert box.take() == (None, -1)
    assert box.put("a") == 0
    assert box.take() == ("a", 0)
    assert box.take() == (None, -1)
    box.put("b")
    box.put("c")
    box.put("d")
    assert box.take() == ("d", 3)
    assert (box.received, box.skipped) == (4, 2)
    box.put(None)                       # a frame may be any object, even None
    assert box.take() == (None, 4)
    assert box.take() == (None, -1)


def test_threaded_producer_consumer_invariants():
    """A fast camera and a slow correlator: every frame is either taken once
    or skipped, taken frames come in increasing order, and the last one put
    is always delivered."""
    box = LatestFrame()
    n = 5000
    taken = []
    done = threading.Event()

    def camera():
        rng = random.Random(3)
        for k in range(n):
            assert box.put(np.int64(k)) == k
            if rng.random() < 0.01:
                threading.Event().wait(0.0005)
        done.set()

    def correlator():
        rng = random.Random(4)
        while True:
            finished = done.is_set()
            f, seq = box.take()
            if f is not None:
                assert int(f) == seq
                taken.append(seq)
            elif finished:
                return
            if rng.random() < 0.05:
                threading.Event().wait(0.0002)

    t1 = threading.Thread(target=camera)
    t2 = threading.Thread(target=correlator)
    t2.start()
    t1.start()
    t1.join()
    t2.join()
    assert box.received == n
    assert len(taken) + box.skipped == n
    assert all(a < b for a, b in zip(taken, taken[1:]))
    assert taken[-1] == n - 1
