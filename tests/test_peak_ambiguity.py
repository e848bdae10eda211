"""Host logic of the near-tie rule used by the GPU parity tests (tests/gpu_util.py): only
decisions that can change the returned peaks are flagged (peak rule: last paragraph of Sec. III-A)."""
import numpy as np

from gpu_util import peak_ambiguity, peaks_ambiguous


def grid(n_el, n_az, fill=1.0):
    return np.full(n_el * n_az, fill)


def test_clear_peaks_are_not_ambiguous():
    v = grid(5, 12)
    v[2 * 12 + 3] = 10.0
    v[1 * 12 + 9] = 5.0
    assert peak_ambiguity(v, 5, 12, 2, 1e-4) == []


def test_rank_near_tie_at_the_cut_and_inside():
    v = grid(5, 12)
    v[2 * 12 + 3] = 10.0
    v[1 * 12 + 9] = 5.0
    v[4 * 12 + 0] = 5.0001          # within 2 rtol of the second peak: the cut may flip
    assert ("rank", 1) in peak_ambiguity(v, 5, 12, 2, 1e-4)
    v[2 * 12 + 3] = 5.0002          # the first two are now near-equal too
    assert ("rank", 0) in peak_ambiguity(v, 5, 12, 2, 1e-4)
    assert not peaks_ambiguous(v, 5, 12, 2, 1e-6)


def test_flank_of_a_returned_peak():
    v = grid(5, 12)
    d = 2 * 12 + 3
    v[d] = 10.0
    v[d + 1] = 9.9995               # a neighbour within 2 rtol: the maximum may move
    assert ("flank", d) in peak_ambiguity(v, 5, 12, 1, 1e-4)


def test_flank_across_the_azimuth_wrap():
    v = grid(3, 8)
    v[1 * 8 + 0] = 10.0
    v[1 * 8 + 7] = 9.9999
    assert ("flank", 8) in peak_ambiguity(v, 3, 8, 1, 1e-4)


def test_rise_of_a_non_maximum_near_the_cut():
    v = grid(5, 12)
    v[2 * 12 + 3] = 10.0
    v[0 * 12 + 8] = 6.0
    v[0 * 12 + 9] = 5.9998          # beaten only by a near-equal neighbour, above the 2nd peak?
    v[4 * 12 + 5] = 3.0             # second returned peak well below
    assert ("rise", 9) in peak_ambiguity(v, 5, 12, 2, 1e-4)


def test_lobe_flank_beaten_by_a_clear_maximum_is_ignored():
    """A point on a peak's flank that has a near-equal neighbour but is beaten by a clearly larger
    one can never become a peak: not flagged (the case that made the old rule flag every
    60-channel block)."""
    v = grid(5, 12)
    v[2 * 12 + 4] = 10.0            # the peak
    v[2 * 12 + 3] = 7.0             # two flank points of it, side by side ...
    v[1 * 12 + 3] = 6.9999          # ... near-equal, both beaten by the peak
    v[1 * 12 + 9] = 4.0
    assert peak_ambiguity(v, 5, 12, 2, 1e-4) == []


def test_fewer_maxima_than_requested():
    v = np.arange(12, dtype=float)   # one row: one maximum at the end
    assert peak_ambiguity(v, 1, 12, 3, 1e-4) == []
