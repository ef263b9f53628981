"""Pins of the oracle's frame-sequence policies (Sec. 3: the reference is
updated after every evaluation, so each pair is two consecutive images;
Sec. 6: the newest frame is correlated against the previously used one):
against translations whose per-frame and accumulated displacements are known
in closed form, and against the exact increments of a heterogeneous field
between the frames actually used.  CPU only."""
import numpy as np
import pytest

import dicgen
from oracle import dic_oracle as O

D = (2.6, -1.7)          # per-frame translation (px)


@pytest.fixture(scope="module")
def translation_frames():
    b = dicgen.make_blobs(dicgen.rng_for(91, 0, 0), 900, 112, 112)
    frames = [dicgen.render_image(b, None if k == 0 else dicgen.rigid(k * D[0], k * D[1]),
                                  112, 112) for k in range(4)]
    M, S = 7, 3
    pois = np.array([(x, y) for x in (30, 56, 82) for y in (30, 56, 82)], dtype=np.int32)
    return frames, pois, M, S


def test_previous_reference_gives_the_per_frame_translation(translation_frames):
    frames, pois, M, S = translation_frames
    res = O.correlate_sequence(frames, pois, M, S, reference="previous")
    assert len(res) == 3
    for r in res:
        assert np.all(r["status"] == O.OK)
        np.testing.assert_allclose(r["p"][:, 0], D[0], atol=0.02)
        np.testing.assert_allclose(r["p"][:, 3], D[1], atol=0.02)


def test_first_reference_accumulates_and_needs_the_seed(translation_frames):
    """Frame k against frame 0 moves k D: beyond the +-3 window from frame 2
    on, so only a window centred on the previous result finds it."""
    frames, pois, M, S = translation_frames
    res = O.correlate_sequence(frames, pois, M, S, reference="first")
    for k, r in enumerate(res, start=1):
        assert np.all(r["status"] == O.OK)
        np.testing.assert_allclose(r["p"][:, 0], k * D[0], atol=0.02)
        np.testing.assert_allclose(r["p"][:, 3], k * D[1], atol=0.02)
    unseeded = O.correlate(frames[0], frames[3], pois, M, S)
    assert not np.allclose(unseeded["p"][:, 0], 3 * D[0], atol=0.5)
    # the increments of the other policy add up to the same total
    inc = O.correlate_sequence(frames, pois, M, S, reference="previous")
    total = sum(r["p"][:, [0, 3]] for r in inc)
    np.testing.assert_allclose(total, res[-1]["p"][:, [0, 3]], atol=0.05)


@pytest.mark.parametrize("used", [[0, 1, 2, 3, 4], [0, 2, 3, 5]])
def test_increments_of_a_heterogeneous_field(used):
    """Frames under u = 0.002 k X (1 + 0.5 sin(2 pi Y / 1500)),
    v = -0.0006 k Y, noise-free; the frames ``used`` (a live run that skipped
    some) against their predecessors: each result is the exact increment of
    the field between the two frames at the POIs of the earlier one."""
    all_frames = dicgen.sequence_frames(max(used) + 1, 200, 260, 2400, noise=0.0, tag=53,
                                        pad=48.0)
    frames = [all_frames[k] for k in used]
    M, S = 10, 6
    pois = dicgen.poi_grid(260, 200, M, S, 19)
    res = O.correlate_sequence(frames, pois, M, S, reference="previous")
    for (a, b), r in zip(zip(used[:-1], used[1:]), res):
        ok = r["status"] == O.OK
        assert ok.mean() > 0.95
        truth = dicgen.true_increment(None if a == 0 else dicgen.heterogeneous_strain(a),
                                      dicgen.heterogeneous_strain(b), pois[ok])
        err = np.abs(r["p"][ok][:, [0, 3]] - truth)
        assert err.mean() < 0.01 and err.max() < 0.05, (a, b, err.mean(), err.max())
        if a > 0:
            # an increment, not the displacement from frame 0
            total = dicgen.true_displacement(dicgen.heterogeneous_strain(b),
                                             pois[ok].astype(np.float64))
            assert np.abs(total - truth).max() > 0.3


def test_unknown_policy_rejected(translation_frames):
    frames, pois, M, S = translation_frames
    with pytest.raises(ValueError):
        O.correlate_sequence(frames, pois, M, S, reference="last")
