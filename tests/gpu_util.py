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


def peaks_ambiguous(Pbar: np.ndarray, n_el: int, n_az: int, Ns: int, rtol: float) -> bool:
    """True when the peak decision on Pbar could flip under a relative perturbation of rtol:
    a local-maximum test or the ranking at the Ns cut involves values within 2 rtol."""
    D = n_el * n_az
    v = Pbar
    close = lambda a, b: abs(a - b) <= 2 * rtol * max(abs(a), abs(b))
    cands = []
    for d in range(D):
        el, az = divmod(d, n_az)
        ismax, amb = True, False
        for de in (-1, 0, 1):
            e = el + de
            if e < 0 or e >= n_el:
                continue
            for da in (-1, 0, 1):
                if de == 0 and da == 0:
                    continue
                nb = e * n_az + (az + da) % n_az
                if nb == d:
                    continue
                if close(v[d], v[nb]):
                    amb = True
                if v[nb] > v[d] or (v[nb] == v[d] and nb < d):
                    ismax = False
        if ismax or amb:
            cands.append((v[d], d, ismax, amb))
    cands.sort(key=lambda c: (-c[0], c[1]))
    # any ambiguous local-max test among values that could reach the top Ns + 1
    top = [c for c in cands if c[2]][:Ns + 1]
    floor = top[-1][0] if top else -np.inf
    for val, d, ismax, amb in cands:
        if amb and val >= floor * (1 - 2 * rtol):
            return True
    real = [c for c in cands if c[2]]
    for k in range(min(Ns, len(real) - 1)):
        if close(real[k][0], real[k + 1][0]):
            return True
    return False
