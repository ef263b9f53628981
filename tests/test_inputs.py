"""The seeded input generators: the torch renderer used for camera-scale
frames reproduces the NumPy renderer (same blobs, fields and noise streams),
including under the strongest shear of the frame sequence.  CPU only."""
import numpy as np

import dicgen


def test_torch_frames_match_numpy_frames():
    a = dicgen.sequence_frames(3, 150, 220, 1200, noise=3.0, tag=61, pad=30.0)
    b = dicgen.sequence_frames_torch(3, 150, 220, 1200, noise=3.0, tag=61, pad=30.0, device="cpu")
    for k in range(3):
        np.testing.assert_allclose(b[k].numpy(), a[k], rtol=0, atol=1e-4, err_msg=f"frame {k}")


def test_torch_render_under_late_frame_shear():
    H, W = 120, 900
    blobs = dicgen.make_blobs(dicgen.rng_for(62, 0, 0), 3000, H, W, pad=96.0)
    k = 31
    a = dicgen.render_image(blobs, dicgen.heterogeneous_strain(k), H, W)
    b = dicgen.render_image_torch(blobs, dicgen.heterogeneous_strain_torch(k), H, W,
                                  dicgen.heterogeneous_strain_lipschitz(k, W + 96.0),
                                  device="cpu").numpy()
    np.testing.assert_allclose(b, a, rtol=0, atol=1e-4)


def test_torch_sinusoidal_batch_matches_numpy():
    a = dicgen.sinusoidal_batch(n_pairs=2, size=96, first=5)
    b = dicgen.sinusoidal_batch_torch(n_pairs=2, size=96, first=5, device="cpu")
    for pa, pb in zip(a, b):
        assert (pa.M, pa.S) == (pb.M, pb.S) and np.array_equal(pa.pois, pb.pois)
        np.testing.assert_allclose(pb.ref.numpy(), pa.ref, rtol=0, atol=1e-4)
        np.testing.assert_allclose(pb.defm.numpy(), pa.defm, rtol=0, atol=1e-4)


def test_batch_pair_params_are_the_pairs():
    """The helper the oracle baseline extrapolates with gives each batched
    pair's amplitude, wavelength and subset size, and the subset sizes cover
    all four in the first eight pairs."""
    pairs = dicgen.sinusoidal_batch(n_pairs=3, size=64, first=2)
    for k, p in zip(range(2, 5), pairs):
        A, lam, sub = dicgen.batch_pair_params(k)
        assert (p.meta["A"], p.meta["lam"], 2 * p.M + 1) == (A, lam, sub)
    assert {dicgen.batch_pair_params(k)[2] for k in range(8)} == set(dicgen.BATCH_SUBSETS)
