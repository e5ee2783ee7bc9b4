"""The seeded generators: the device assembly of the long synthetic video draws
the same scene as the host generator (checked on the CPU device)."""
import numpy as np

from paper_1702_02241_amd import synth


def test_video_device_assembly_matches_host_scene():
    X0, L0, S0 = synth.video_frames(n_frames=40, width=64, height=48, seed=11, noise=0.0)
    Xd = synth.video_frames_device(40, 64, 48, seed=11, noise=0.0, device="cpu").numpy()
    assert Xd.shape == (40, 64 * 48)
    assert np.abs(Xd - X0.T).max() <= 1e-6
    # with noise: the same frames plus N(0, 0.01^2) noise from the device generator
    Xn = synth.video_frames_device(40, 64, 48, seed=11, noise=0.01, device="cpu").numpy()
    r = (Xn - X0.T).ravel()
    assert abs(r.mean()) < 1e-3 and abs(r.std() - 0.01) < 1e-3
