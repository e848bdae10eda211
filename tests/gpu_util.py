"""Helpers shared by the GPU tests: device tensors, oracle comparisons, tolerances."""
from __future__ import annotations

import numpy as np

U32 = 2.0 ** -24     # FP32 unit roundoff


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


def to_host(t) -> np.ndarray:
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def projector(E):
    return E @ E.conj().T


def corr_bound(X: np.ndarray) -> np.ndarray:
    """Elementwise forward-error bound of an FP32 correlation of T frames: each entry is a sum of
    2T real products, so |dR| <= (2T + 2) u (1/T) sum_t |x_ti| |x_tj| (plus the final scale)."""
    T = X.shape[1]
    Xa = np.abs(X.astype(np.complex128))
    return (2 * T + 4) * U32 * np.einsum("fti,ftj->fij", Xa, Xa) / T


def _neighbours(d: int, n_el: int, n_az: int):
    """The 8-neighbourhood of flat index d (azimuth circular, elevation clamped), as the peak rule
    of the last paragraph of Sec. III-A is read here; duplicates removed (tiny grids)."""
    el, az = divmod(d, n_az)
    out = []
    for de in (-1, 0, 1):
        e = el + de
        if e < 0 or e >= n_el:
            continue
        for da in (-1, 0, 1):
            nb = e * n_az + (az + da) % n_az
            if nb != d and nb not in out:
                out.append(nb)
    return out


def peak_ambiguity(Pbar: np.ndarray, n_el: int, n_az: int, Ns: int, rtol: float) -> list:
    """Decisions of the peak search on the reference Pbar that a relative perturbation of at most
    rtol per value could change, i.e. the only places where two correct evaluations may return
    different peaks.  Returns a list of (kind, index) reasons, empty when the returned peaks
    (indices and order) are fixed by the values:
      ("flank", d)   a returned peak d has a neighbour within 2 rtol, so either may be the maximum;
      ("rank", k)    the k-th and (k+1)-th largest local maxima are within 2 rtol (k < Ns), so the
                     order of the returned peaks, or which one makes the cut, may flip;
      ("rise", d)    a point that is not a local maximum could become one (every neighbour that
                     beats it is within 2 rtol) and is not clearly below the Ns-th returned peak.
    Points that are beaten by a clearly larger neighbour can never become peaks and are ignored."""
    v = np.asarray(Pbar, dtype=np.float64)
    D = n_el * n_az
    close = lambda a, b: abs(a - b) <= 2 * rtol * max(abs(a), abs(b))
    beats = lambda nb, d: v[nb] > v[d] or (v[nb] == v[d] and nb < d)
    nbrs = [_neighbours(d, n_el, n_az) for d in range(D)]
    ismax = [all(not beats(nb, d) for nb in nbrs[d]) for d in range(D)]
    maxima = sorted((d for d in range(D) if ismax[d]), key=lambda d: (-v[d], d))
    top = maxima[:Ns]
    reasons = []
    for d in top:
        if any(close(v[d], v[nb]) for nb in nbrs[d]):
            reasons.append(("flank", d))
    for k in range(min(Ns, len(maxima) - 1)):
        if close(v[maxima[k]], v[maxima[k + 1]]):
            reasons.append(("rank", k))
    floor = v[top[-1]] * (1 - 2 * rtol) if len(top) == Ns else -np.inf
    for d in range(D):
        if ismax[d] or v[d] < floor:
            continue
        if all(close(v[d], v[nb]) for nb in nbrs[d] if beats(nb, d)):
            reasons.append(("rise", d))
    return reasons


def peaks_ambiguous(Pbar: np.ndarray, n_el: int, n_az: int, Ns: int, rtol: float) -> bool:
    """True when a relative perturbation of rtol could change the returned peaks."""
    return bool(peak_ambiguity(Pbar, n_el, n_az, Ns, rtol))
