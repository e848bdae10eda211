"""The seeded input generator: determinism, shapes, geometry and power bookkeeping."""
import numpy as np

import synth


def test_geometry():
    p = synth.ring_array60()
    assert p.shape == (60, 3)
    r = np.hypot(p[:, 0], p[:, 1])
    assert np.allclose(np.sort(np.unique(np.round(r, 9))), [0.10, 0.15, 0.20, 0.25])
    assert np.allclose(np.sort(np.unique(np.round(p[:, 2], 9))), [0.0, 0.1, 0.2, 0.3])
    c = synth.circle_array(8, 0.1)
    assert np.allclose(np.hypot(c[:, 0], c[:, 1]), 0.1) and np.all(c[:, 2] == 0)


def test_grid_and_steering():
    g = synth.DirectionGrid(72, 19)
    az, el = g.angles_deg()
    assert g.D == 1368 and az[73] == 5.0 and el[73] == 5.0
    u = g.unit_vectors()
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0)
    H = synth.steering_table(synth.ring_array60(), g, synth.bin_freqs(5, 16000, 512))
    assert H.dtype == np.complex64 and H.shape == (5, 1368, 60)
    assert np.allclose(np.abs(H), 1.0, atol=1e-6)
    assert np.all(H[0] == 1.0)                       # DC bin has no phase


def test_blocks_are_seeded_and_distinct():
    w = synth.workload_small(n_blocks=4)
    X0, d0, s0 = w.block(0)
    X0b, d0b, _ = w.block(0)
    X1, d1, _ = w.block(1)
    assert X0.dtype == np.complex64 and X0.shape == (257, 50, 8)
    assert np.array_equal(X0, X0b) and d0 == d0b
    assert not np.array_equal(X0, X1)
    assert s0 == 10.0
    Xn = w.noise_frames()
    assert Xn.shape == (257, 50, 8)
    assert np.array_equal(Xn, w.noise_frames())


def test_paper_workload_powers():
    w = synth.workload_paper(n_blocks=8)
    assert (w.M, w.F, w.T, w.Ns, w.D, w.n_noise_frames) == (60, 257, 50, 2, 1368, 240)
    az, el = w.grid.angles_deg()
    for b in range(8):
        X, dirs, snr = w.block(b)
        assert -5.0 <= snr <= 10.0 and len(set(dirs)) == 2
        assert all(el[d] <= 80.0 for d in dirs)
        # empirical per-channel power ~ p_s * Ns + noise total (3 units)
        p_s = 3.0 * 10 ** (snr / 10)
        pw = np.mean(np.abs(X.astype(np.complex128)) ** 2)
        assert abs(pw - (2 * p_s + 3.0)) / (2 * p_s + 3.0) < 0.1
