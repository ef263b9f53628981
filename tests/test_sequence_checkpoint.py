"""Host logic of the sequence checkpoint (no GPU): files, latest pair,
whole-file writes, mismatches refused, resume without a directory refused,
and the status histogram."""
import os

import numpy as np
import pytest

import paper_1905_06228_amd as dic


def state(n, k):
    rng = np.random.default_rng(k)
    return (rng.integers(-5, 5, (n, 2)).astype(np.int32), rng.standard_normal((n, 6)),
            rng.standard_normal((n, 6)), rng.integers(0, 7, n).astype(np.int32))


def test_save_load_latest(tmp_path):
    ck = dic.SequenceCheckpoint(str(tmp_path / "ck"))
    assert ck.frames() == []
    with pytest.raises(dic.DicError):
        ck.load()
    saved = {}
    for k in (1, 2, 3, 10):
        saved[k] = state(7, k)
        ck.save(k, "previous", *saved[k])
    assert ck.frames() == [1, 2, 3, 10]
    assert not [f for f in os.listdir(tmp_path / "ck") if f.endswith(".tmp")]
    k, st = ck.load()
    assert k == 10
    for k in (2, 10):
        _, st = ck.load(k)
        seed, p_seed, p, status = saved[k]
        np.testing.assert_array_equal(st["seed"], seed)
        np.testing.assert_array_equal(st["p_seed"], p_seed)
        np.testing.assert_array_equal(st["p"], p)
        np.testing.assert_array_equal(st["status"], status)
        assert str(st["reference"]) == "previous" and int(st["n"]) == 7
    with pytest.raises(dic.DicError):
        ck.load(4)


def test_resume_needs_directory():
    with pytest.raises(dic.DicError):
        dic.correlate_sequence([np.zeros((8, 8), np.float32)] * 2, None, 2, 1, resume=True)


def test_status_histogram():
    st = np.array([0, 0, 1, 2, 0, 6, 9], np.int32)
    h = dic.status_histogram(st)
    assert h == {"OK": 3, "NOT_CONVERGED": 1, "OUT_OF_BOUNDS": 1, "NAN_INPUT": 1, "UNKNOWN_9": 1}
    assert sum(h.values()) == len(st)
