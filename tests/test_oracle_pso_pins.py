"""Pins of the oracle's particle swarm searches (Sec. 2.1, Eqs. 2-4; Sec. 5.2)
against facts outside their own code: the paper's evaluation bounds, the
closed-form flight of a swarm without attraction (Eq. 3 with the Eq. 4
weights), a greedy ascent on the brute-force score map for the star step,
the brute-force maximum on an exact shift, Eq. (1) at the reported position,
and the status rules.  CPU only."""
import json
import os

import numpy as np
import pytest

import dicgen
from oracle import dic_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "pso_evaluation_bounds.json")


@pytest.fixture(scope="module")
def pair():
    return dicgen.affine_pair_1024(size=256, tag=2)


def test_weight_schedule_eq4():
    assert O.pso_weight(0, 5) == 0.9
    assert abs(O.pso_weight(5, 5) - 0.4) < 1e-15
    assert abs(O.pso_weight(2, 5) - 0.7) < 1e-15


def test_evaluations_within_paper_bounds(pair):
    """Sec. 5.2: 50 particles over at most 5 generations evaluate at most 250
    coefficients, the modified form (particle and four neighbours) at most
    1250."""
    g = json.load(open(GOLDEN))
    pois = pair.pois[::61]
    R = dicgen.swarm_random(len(pois), 3)
    for i, (x0, y0) in enumerate(pois):
        a = O.pso_search(pair.ref, pair.defm, int(x0), int(y0), pair.M, pair.S, R[i])
        m = O.pso_search(pair.ref, pair.defm, int(x0), int(y0), pair.M, pair.S, R[i], modified=True)
        assert a.evaluations <= g["pso_max_evaluations"]
        assert m.evaluations <= g["modified_pso_max_evaluations"]
        assert a.generations <= g["max_generations"] and m.generations <= g["max_generations"]


def test_flight_without_attraction_closed_form(pair):
    """c1 = c2 = 0: v_t = w(t-1) v_(t-1), q_t = q_(t-1) + v_t (Eqs. 2-4 with no
    attraction); small initial velocities never reach the clip."""
    P, G, S = 6, 5, pair.S
    rng = np.random.default_rng(12)
    rand = rng.random((G, P, 4), dtype=np.float32)
    rand[0, :, 0:2] = 0.5 + 0.2 * (rand[0, :, 0:2] - 0.5)      # start near the centre
    rand[0, :, 2:4] = 0.5 + 0.05 * (rand[0, :, 2:4] - 0.5)     # |v0| <= 0.05 S
    r = O.pso_search(pair.ref, pair.defm, 120, 120, pair.M, S, rand, c1=0.0, c2=0.0,
                     stop_cc=2.0, keep_trace=True)
    q = 2.0 * S * rand[0, :, 0:2].astype(np.float64) - S
    v = 2.0 * S * rand[0, :, 2:4].astype(np.float64) - S
    assert r.generations == G
    for t, (ks, _) in enumerate(r.trace):
        np.testing.assert_array_equal(ks, np.rint(q).astype(np.int64))
        v = (0.9 - t / (2.0 * G)) * v
        q = q + v


def test_star_step_is_greedy_ascent(pair):
    """One particle, no attraction, no velocity: the modified form climbs the
    brute-force score map one four-neighbour step per generation."""
    x0, y0 = 100, 140
    S = pair.S
    scores = O.integer_search(pair.ref, pair.defm, x0, y0, pair.M, S, keep_scores=True).scores
    rand = np.full((5, 1, 4), 0.5, np.float32)
    rand[0, 0, 0] = (S - 5) / (2 * S)     # start at window offset (-5, 3)
    rand[0, 0, 1] = (S + 3) / (2 * S)
    r = O.pso_search(pair.ref, pair.defm, x0, y0, pair.M, S, rand, modified=True, c1=0.0,
                     c2=0.0, stop_cc=2.0, keep_trace=True)
    k = np.array([-5, 3])
    side = 2 * S + 1
    for t in range(5):
        np.testing.assert_array_equal(r.trace[t][0][0], k)
        best = (scores[k[1] + S, k[0] + S], (k[1] + S) * side + k[0] + S, k.copy())
        for sx, sy in O.STAR_STEPS:
            n = k + (sx, sy)
            if np.all(np.abs(n) <= S):
                c = scores[n[1] + S, n[0] + S]
                idx = (n[1] + S) * side + n[0] + S
                if c > best[0] + 1e-12 or (c >= best[0] - 1e-12 and idx < best[1]):
                    best = (c, idx, n)
        k = best[2]


@pytest.mark.parametrize("modified", [False, True])
def test_reported_coefficient_is_eq1_and_swarm_maximum(pair, modified):
    pois = pair.pois[::97]
    R = dicgen.swarm_random(len(pois), 9)
    for i, (x0, y0) in enumerate(pois):
        r = O.pso_search(pair.ref, pair.defm, int(x0), int(y0), pair.M, pair.S, R[i],
                         modified=modified, keep_trace=True)
        assert r.status == O.OK
        fs = O.subset(pair.ref, int(x0), int(y0), pair.M)
        gs = O.subset(pair.defm, int(x0) + r.du, int(y0) + r.dv, pair.M)
        assert abs(r.zncc - np.corrcoef(fs.ravel(), gs.ravel())[0, 1]) < 1e-12
        seen = {(int(a), int(b)) for ks, _ in r.trace for a, b in ks}
        for kx, ky in seen:
            gs2 = O.subset(pair.defm, int(x0) + kx, int(y0) + ky, pair.M)
            assert np.corrcoef(fs.ravel(), gs2.ravel())[0, 1] <= r.zncc + 1e-12


def test_exact_shift_found_and_early_stop():
    """g is f shifted by whole pixels: the modified swarm reaches coefficient
    1 and stops in the generation that found it (the 0.995 rule)."""
    b = dicgen.make_blobs(dicgen.rng_for(904, 1, 0), 1500, 150, 150)
    f = dicgen.render_image(b, None, 150, 150)
    g = np.roll(np.roll(f, -2, axis=0), 3, axis=1)
    R = dicgen.swarm_random(1, 21)[0]
    r = O.pso_search(f, g, 75, 75, 10, 8, R, modified=True, keep_trace=True)
    assert (r.du, r.dv, r.status) == (3, -2, O.OK)
    assert abs(r.zncc - 1.0) < 1e-12
    assert r.generations == len(r.trace) and r.generations < O.PSO_GENERATIONS


def test_memo_changes_nothing(pair):
    R = dicgen.swarm_random(3, 4)
    for i, (x0, y0) in enumerate(pair.pois[[5, 200, 400]]):
        for mod in (False, True):
            a = O.pso_search(pair.ref, pair.defm, int(x0), int(y0), pair.M, pair.S, R[i], modified=mod)
            b = O.pso_search(pair.ref, pair.defm, int(x0), int(y0), pair.M, pair.S, R[i], modified=mod,
                             memo=False)
            assert (a.du, a.dv, a.zncc, a.generations) == (b.du, b.dv, b.zncc, b.generations)


def test_statuses_and_radius_zero(pair):
    f, g, M = pair.ref, pair.defm, pair.M
    R = dicgen.swarm_random(1, 2)[0]
    assert O.pso_search(f, g, 5, 120, M, 4, R).status == O.OUT_OF_BOUNDS
    fn = f.copy()
    fn[121, 123] = np.nan
    assert O.pso_search(fn, g, 120, 120, M, 4, R).status == O.NAN_INPUT
    assert O.pso_search(np.full_like(f, 50.0), g, 120, 120, M, 4, R).status == O.ZERO_VARIANCE
    # every window position leaves the image
    r = O.pso_search(f, g, 120, 120, M, 4, R, cu=200)
    assert r.status == O.NO_VALID_CANDIDATE
    # radius 0: the seed itself, Eq. (1) there
    r = O.pso_search(f, g, 120, 120, M, 0, R, cu=3, cv=-3)
    assert (r.du, r.dv, r.evaluations) == (3, -3, 1)
    assert abs(r.zncc - O.zncc(O.subset(f, 120, 120, M), O.subset(g, 123, 117, M))) < 1e-15
