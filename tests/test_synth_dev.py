"""The device-side input generators reproduce synth.py (checked on the CPU)."""
import numpy as np

from paper_2605_27534_amd import synth, synth_dev


def test_vof_ball_matches_host_generator():
    n = (24, 20, 28)
    h = 1.0 / 24
    for centre, period in (((0.5, 0.4, 0.6), None), ((0.45, 0.5, 0.1), 28 * h)):
        ref = synth.vof_ball(n, h, centre, 0.27, 3, period_z=period)
        got = synth_dev.vof_ball(n, h, centre, 0.27, period_z=period).numpy()
        assert np.array_equal(got, ref)


def test_hadamard_faces_match_host_generator():
    n = (20, 18, 22)
    h = 1.0 / 20
    c = (0.5, 0.45, 0.3)
    ref = synth.u_hadamard(n, h, c, 0.2, -0.5, 0.01, frame_shift=0.5, period_z=22 * h)
    got = synth_dev.u_hadamard(n, h, c, 0.2, -0.5, 0.01, frame_shift=0.5, period_z=22 * h)
    for a, b in zip(got, ref):
        a = a.numpy()
        assert a.shape == b.shape
        assert np.max(np.abs(a - b)) <= 1e-14 * np.max(np.abs(b))
