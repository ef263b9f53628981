"""GPU parity of the reference-update policies against the oracle: frame k
against frame k - 1 (Sec. 3: the reference updated after every evaluation)
and the live policy (Sec. 6: the newest frame against the previously used
one, frames arriving meanwhile skipped).  Integer results and statuses
bit-exact, sub-pixel displacements within 1e-3 px, coefficients within
1e-5, for every pair."""
import numpy as np
import pytest
import torch

import dicgen
import paper_1905_06228_amd as dic
from oracle import dic_oracle as O
from tests._parity import compare, to_dev

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

M, S = 10, 6


@pytest.fixture(scope="module")
def frames():
    return dicgen.sequence_frames(7, 200, 260, 2400, noise=3.0, tag=54, pad=48.0)


def host(o):
    return {k: v.cpu().numpy() for k, v in o.items() if isinstance(v, torch.Tensor)}


@pytest.mark.parametrize("name,prec", [("fp32", dic.FP32_BATCHED), ("fp64", dic.FP64_PLAIN)])
def test_previous_reference_matches_oracle(frames, name, prec):
    fr = frames[:5]
    pois = dicgen.poi_grid(260, 200, M, S, 13)
    print(f"case sequence previous {name} frames={len(fr)} N={len(pois)}", flush=True)
    ref = O.correlate_sequence(fr, pois, M, S, reference="previous")
    got = dic.correlate_sequence([torch.from_numpy(f) for f in fr], to_dev(pois), M, S,
                                 precision=prec, reference="previous")
    assert len(got) == len(ref)
    for k, (g, r) in enumerate(zip(got, ref), start=1):
        compare(host(g), r, M, label=f"sequence previous {k}/{name}")
    # from device frames, in place: the same bits
    dev = dic.correlate_sequence([to_dev(f) for f in fr], to_dev(pois), M, S, precision=prec,
                                 reference="previous")
    for a, b in zip(got, dev):
        for key in a:
            np.testing.assert_array_equal(a[key].cpu().numpy(), b[key].cpu().numpy(), err_msg=key)


def test_previous_reference_with_graph_replay(frames):
    """Three rotating frame buffers give three captured graphs; the replays
    match the eager driver."""
    fr = frames[:6]
    pois = dicgen.poi_grid(260, 200, M, S, 17)
    print(f"case sequence previous graph N={len(pois)}", flush=True)
    eager = dic.correlate_sequence([torch.from_numpy(f) for f in fr], to_dev(pois), M, S,
                                   reference="previous")
    graph = dic.correlate_sequence([torch.from_numpy(f) for f in fr], to_dev(pois), M, S,
                                   reference="previous", flags=dic.FLAG_USE_GRAPH)
    for a, b in zip(eager, graph):
        for key in a:
            np.testing.assert_array_equal(a[key].cpu().numpy(), b[key].cpu().numpy(), err_msg=key)


def test_live_policy_skips_and_matches_oracle(frames):
    pois = dicgen.poi_grid(260, 200, M, S, 13)
    Q = to_dev(pois)
    live = dic.LiveCorrelator(200, 260, Q, M, S)
    print(f"case live N={len(pois)}", flush=True)
    outs = []
    assert live.step() is None                      # nothing arrived
    live.put(frames[0])
    assert live.step() is None                      # first frame: the reference
    live.put(frames[1])
    live.put(frames[2])                             # frame 1 skipped
    outs.append(live.step())
    live.put(to_dev(frames[3]))                     # a device frame (copied)
    outs.append(live.step())
    assert live.step() is None
    live.put(frames[4])
    live.put(frames[5])
    live.put(frames[6])                             # frames 4, 5 skipped
    outs.append(live.step())
    torch.cuda.synchronize()
    assert [(o["frame"], o["reference"]) for o in outs] == [(2, 0), (3, 2), (6, 3)]
    assert (live.mailbox.received, live.mailbox.skipped, live.pairs) == (7, 3, 3)
    used = [frames[k] for k in (0, 2, 3, 6)]
    ref = O.correlate_sequence(used, pois, M, S, reference="previous")
    for k, (o, r) in enumerate(zip(outs, ref)):
        compare(host(o), r, M, label=f"live pair {k}")
    # the same pairs through the sequence driver: the same bits
    seq = dic.correlate_sequence([torch.from_numpy(f) for f in used], Q, M, S,
                                 reference="previous")
    for a, b in zip(outs, seq):
        for key in b:
            np.testing.assert_array_equal(a[key].cpu().numpy(), b[key].cpu().numpy(), err_msg=key)


def test_camera_scale_pair_sampled():
    """One pair of the 4096 x 3000 camera sequence (frames 1 and 2, ~600k
    blobs, noise 3; 239,932 POIs, subset 29 x 29, search +-24, so the
    matrix-core form with 2 x 2 tiles) in the launch configuration of the
    sequence benchmark; 24 seeded POIs checked against the oracle one by one,
    the increment against the generating field at every POI."""
    H, W, M, S, step = 3000, 4096, 14, 24, 7
    fr = dicgen.sequence_frames_torch(3, H, W, 600_000, noise=3.0, tag=5, pad=96.0,
                                      device=torch.device("cuda", 0))
    pois = dicgen.poi_grid(W, H, M, S, step)
    Q = to_dev(pois)
    print(f"case camera pair N={len(pois)}", flush=True)
    got = dic.correlate_sequence([fr[1], fr[2]], Q, M, S, reference="previous")[0]
    torch.cuda.synchronize()
    h = host(got)
    f1, f2 = fr[1].cpu().numpy(), fr[2].cpu().numpy()
    idx = np.sort(np.random.default_rng(19).choice(len(pois), 24, replace=False))
    ref = O.correlate(f1, f2, pois[idx], M, S)
    compare(h, ref, M, idx=idx, label="camera pair sampled")
    ok = h["status"] == O.OK
    assert ok.mean() > 0.99
    truth = dicgen.true_increment(dicgen.heterogeneous_strain(1), dicgen.heterogeneous_strain(2),
                                  pois[ok])
    err = np.abs(h["p"][ok][:, [0, 3]] - truth)
    print(f"[camera pair] ok={ok.mean():.4f} mean err={err.mean():.4f} px", flush=True)
    assert err.mean() < 0.02


@pytest.mark.parametrize("flag", [0, dic.FLAG_INTERP_BSPLINE, dic.FLAG_BICUBIC_LUT])
def test_first_reference_with_reused_slots_matches_fresh_plans(frames, flag):
    """Host frames against frame 0: the deformed frames take turns in two
    device slots, so a pointer comes back with new pixels (frames 1, 3 and
    2, 4).  Every pair must equal a fresh, uncached plan's result for the
    same frames and seeds, bit for bit: nothing of an earlier frame (box
    sums, interpolation table) may be reused."""
    fr = frames[:5]
    pois = dicgen.poi_grid(260, 200, M, S, 13)
    Q = to_dev(pois)
    N = len(pois)
    print(f"case sequence first reused slots flag={flag} N={N}", flush=True)
    got = dic.correlate_sequence([torch.from_numpy(f) for f in fr], Q, M, S, flags=flag)
    plan = dic.single_pair_plan(260, 200, M, S, N, flags=flag)
    seed = torch.zeros((N, 2), dtype=torch.int32, device="cuda")
    p_seed = torch.zeros((N, 6), dtype=torch.float64, device="cuda")
    F0 = to_dev(fr[0])
    for k in range(1, len(fr)):
        o = plan.correlate(F0, to_dev(fr[k]), Q, seed, p_seed)
        plan.seed_update(o["p"], o["status"], seed, p_seed)
        torch.cuda.synchronize()
        ref = host(o)
        g = host(got[k - 1])
        for key in ref:
            np.testing.assert_array_equal(ref[key], g[key], err_msg=f"frame {k} {key}")


@pytest.mark.parametrize("reference", ["first", "previous"])
def test_sequence_resume_from_checkpoint(frames, tmp_path, reference):
    """A sequence checkpointed after every pair and resumed after pair 2 (its
    reference prepared again, the seeds read back) gives the pairs after 2
    bit-identical to the uninterrupted run."""
    fr = [torch.from_numpy(f) for f in frames[:6]]
    pois = to_dev(dicgen.poi_grid(260, 200, M, S, 15))
    print(f"case sequence resume {reference} N={len(pois)}", flush=True)
    whole = dic.correlate_sequence(fr, pois, M, S, reference=reference,
                                   checkpoint=str(tmp_path))
    assert dic.SequenceCheckpoint(str(tmp_path)).frames() == [1, 2, 3, 4, 5]
    part = dic.correlate_sequence(fr, pois, M, S, reference=reference,
                                  checkpoint=str(tmp_path / "again"), resume=False)
    resumed = dic.correlate_sequence(fr, pois, M, S, reference=reference,
                                     checkpoint=str(tmp_path), resume=2)
    assert len(resumed) == 3
    for a, b in zip(whole[2:], resumed):
        for key in a:
            np.testing.assert_array_equal(a[key].cpu().numpy(), b[key].cpu().numpy(), err_msg=key)
    for a, b in zip(whole, part):
        np.testing.assert_array_equal(a["p"].cpu().numpy(), b["p"].cpu().numpy())
    # the saved warp of a pair is that pair's result
    _, st = dic.SequenceCheckpoint(str(tmp_path)).load(4)
    np.testing.assert_array_equal(st["p"], whole[3]["p"].cpu().numpy())
    np.testing.assert_array_equal(st["status"], whole[3]["status"].cpu().numpy())
