"""FP64 CPU oracle for the GSVD-MUSIC localization path -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
this package.  It wraps ``ssl_oracle.c`` (plain C, FP64, explicit loops) with
numpy marshalling; it imports nothing from the HIP library's package and the
HIP library imports nothing from here.

Each wrapper names the passage of arXiv 2504.03373 that it follows; the C
source carries the full derivation.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ssl_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libssl_oracle.so")

OK, NOT_PD, NO_CONV, NONFINITE = 0, 1, 2, 3

# Jacobi stopping rule of the oracle: |b_i^H b_j| <= M * 2^-53 * |b_i| |b_j|, at most 60 sweeps.
def default_tol(M: int) -> float:
    return M * 2.0 ** -53


DEFAULT_MAX_SWEEPS = 60


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP over bins).  Always recompiles when force=True."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
               "-Wall", "-Wextra", "-Wno-unused-parameter", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_double
        L.orc_corr.argtypes = [P, i32, i32, i32, i64, i64, f64, P]
        L.orc_hann.argtypes = [i32, P]
        L.orc_stft.argtypes = [P, i32, i32, i32, P, i32, P]
        L.orc_cholesky.argtypes = [P, i32, P]
        L.orc_cholesky.restype = i32
        L.orc_chol_solve.argtypes = [P, P, i32, P]
        L.orc_chol_solve.restype = i32
        L.orc_jacobi_svd.argtypes = [P, i32, f64, i32, P, P, P, P]
        L.orc_jacobi_svd.restype = i32
        L.orc_sort_desc.argtypes = [i32, P, P, P, P]
        L.orc_gsvd.argtypes = [P, P, i32, i32, i32, f64, i32, i32, P, P, P, P]
        L.orc_spectrum.argtypes = [P, P, P, i32, i32, i32, i32, i32, i32, P, P]
        L.orc_is_local_max.argtypes = [P, i32, i32, i32]
        L.orc_is_local_max.restype = i32
        L.orc_peaks.argtypes = [P, i32, i32, i32, P, P]
        L.orc_peaks.restype = i32
        L.orc_localize.argtypes = [P, i32, i32, i32, i64, i64, P, P, i32, i32, i32, i32,
                                   f64, i32, i32, P, P, P, P, P]
        L.orc_localize_m.argtypes = [P, i32, i32, i32, i64, i64, P, P, i32, i32, i32, i32,
                                     f64, i32, i32, i32, P, P, P, P, P]
        L.orc_inv_sqrt.argtypes = [P, i32, f64, i32, P]
        L.orc_inv_sqrt.restype = i32
        L.orc_gevd.argtypes = [P, P, i32, i32, i32, f64, i32, i32, P, P, P]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


# ----------------------------------------------------------------------------
def hann(N: int) -> np.ndarray:
    """Periodic Hann window 1/2 - 1/2 cos(2 pi n / N) (the default STFT window)."""
    w = np.empty(N, np.float64)
    lib().orc_hann(N, _ptr(w))
    return w


def stft(pcm: np.ndarray, nfft: int, hop: int, T: int, window=None) -> np.ndarray:
    """eq.1: X [nfft/2 + 1][T][M] complex128 of pcm [n_samples][M] float32, frames t*hop .. t*hop +
    nfft - 1 (t < T), window (float, [nfft]) or the periodic Hann window."""
    pcm = np.ascontiguousarray(pcm, dtype=np.float32)
    n, M = pcm.shape
    if (T - 1) * hop + nfft > n:
        raise ValueError("not enough samples for T frames")
    win = hann(nfft) if window is None else np.ascontiguousarray(window, dtype=np.float64)
    X = np.empty((nfft // 2 + 1, T, M), np.complex128)
    lib().orc_stft(_ptr(pcm), M, nfft, hop, _ptr(win), T, _ptr(X))
    return X


def corr(X: np.ndarray, scale: float | None = None) -> np.ndarray:
    """eq.2-3: R[f] = scale * sum_t X[f,t,:] X[f,t,:]^H for X [F][T][M] complex64 (any strides
    along F and T with M contiguous).  scale defaults to 1/T."""
    if X.dtype != np.complex64:
        raise TypeError("X must be complex64")
    if X.strides[2] != 8:
        X = np.ascontiguousarray(X)
    F, T, M = X.shape
    R = np.empty((F, M, M), np.complex128)
    lib().orc_corr(_ptr(X), F, T, M, X.strides[0] // 8, X.strides[1] // 8,
                   (1.0 / T) if scale is None else float(scale), _ptr(R))
    return R


def cholesky(K: np.ndarray):
    """K = L L^H (one bin).  Returns (status, L)."""
    K = _c128(K)
    M = K.shape[0]
    L = np.zeros((M, M), np.complex128)
    st = lib().orc_cholesky(_ptr(K), M, _ptr(L))
    return st, L


def solve(K: np.ndarray, R: np.ndarray):
    """Sec. III-B: A = K^{-1} R for one bin.  Returns (status, A)."""
    K, R = _c128(K), _c128(R)
    M = K.shape[0]
    A = np.zeros((M, M), np.complex128)
    st = lib().orc_chol_solve(_ptr(K), _ptr(R), M, _ptr(A))
    return st, A


def jacobi_svd(A: np.ndarray, tol: float | None = None, max_sweeps: int = DEFAULT_MAX_SWEEPS,
               sort: bool = True):
    """eq.4: one-sided Jacobi SVD A = U diag(sigma) V^H (V = W / sigma).
    Returns (status, U, sigma, W, sweeps) with sigma descending when sort=True."""
    A = _c128(A)
    M = A.shape[0]
    U = np.zeros((M, M), np.complex128)
    W = np.zeros((M, M), np.complex128)
    s = np.zeros(M, np.float64)
    sw = ctypes.c_int(0)
    st = lib().orc_jacobi_svd(_ptr(A), M, default_tol(M) if tol is None else tol, max_sweeps,
                              _ptr(U), _ptr(W), _ptr(s), ctypes.byref(sw))
    if sort:
        lib().orc_sort_desc(M, _ptr(s), _ptr(U), _ptr(W), None)
    return st, U, s, W, sw.value


def sort_desc(sigma: np.ndarray):
    """Returns the permutation the oracle's stable descending sort applies."""
    s = np.ascontiguousarray(sigma, dtype=np.float64).copy()
    M = s.shape[0]
    perm = np.zeros(M, np.int32)
    lib().orc_sort_desc(M, _ptr(s), None, None, _ptr(perm))
    return s, perm


def gsvd(K: np.ndarray, R: np.ndarray, Ns: int, tol: float | None = None,
         max_sweeps: int = DEFAULT_MAX_SWEEPS, nthreads: int = 1):
    """eq.4 per bin: returns (En [F][M-Ns][M], sigma [F][M], status [F], sweeps [F])."""
    K, R = _c128(K), _c128(R)
    F, M, _ = R.shape
    En = np.zeros((F, M - Ns, M), np.complex128)
    sig = np.zeros((F, M), np.float64)
    st = np.zeros(F, np.int32)
    sw = np.zeros(F, np.int32)
    lib().orc_gsvd(_ptr(K), _ptr(R), F, M, Ns, default_tol(M) if tol is None else tol,
                   max_sweeps, nthreads, _ptr(En), _ptr(sig), _ptr(st), _ptr(sw))
    return En, sig, st, sw


def spectrum(H: np.ndarray, En: np.ndarray, Ns: int, p: int = 2, status=None, nthreads: int = 1):
    """eq.5-6: returns (P [F][D], Pbar [D]) in FP64."""
    H = np.ascontiguousarray(H, dtype=np.complex64)
    En = _c128(En)
    F, D, M = H.shape
    P = np.zeros((F, D), np.float64)
    Pbar = np.zeros(D, np.float64)
    stp = None
    if status is not None:
        status = np.ascontiguousarray(status, dtype=np.int32)
        stp = _ptr(status)
    lib().orc_spectrum(_ptr(H), _ptr(En), stp, F, D, M, Ns, p, nthreads, _ptr(P), _ptr(Pbar))
    return P, Pbar


def is_local_max(Pbar: np.ndarray, n_el: int, n_az: int, d: int) -> bool:
    Pbar = np.ascontiguousarray(Pbar, dtype=np.float64)
    return bool(lib().orc_is_local_max(_ptr(Pbar), n_el, n_az, d))


def peaks(Pbar: np.ndarray, n_el: int, n_az: int, Ns: int):
    """Peak search of Sec. III-A on the n_el x n_az grid.  Returns (peaks int32[Ns], vals)."""
    Pbar = np.ascontiguousarray(Pbar, dtype=np.float64)
    pk = np.full(Ns, -1, np.int32)
    vals = np.zeros(Ns, np.float64)
    lib().orc_peaks(_ptr(Pbar), n_el, n_az, Ns, _ptr(pk), _ptr(vals))
    return pk, vals


def inv_sqrt(K: np.ndarray, tol: float | None = None, max_sweeps: int = DEFAULT_MAX_SWEEPS):
    """K^{-1/2} (Hermitian inverse square root) of one bin's K.  Returns (status, W)."""
    K = _c128(K)
    M = K.shape[0]
    W = np.zeros((M, M), np.complex128)
    st = lib().orc_inv_sqrt(_ptr(K), M, default_tol(M) if tol is None else tol, max_sweeps, _ptr(W))
    return st, W


def gevd(K: np.ndarray, R: np.ndarray, Ns: int, tol: float | None = None,
         max_sweeps: int = DEFAULT_MAX_SWEEPS, nthreads: int = 1):
    """GEVD-MUSIC per bin: the generalized eigenvectors R e = lambda K e of the M - Ns smallest
    lambda (K-orthonormal), via K^{-1/2} R K^{-1/2}; returns (En [F][M-Ns][M], sigma = the
    generalized eigenvalues descending, status)."""
    K, R = _c128(K), _c128(R)
    F, M, _ = R.shape
    En = np.zeros((F, M - Ns, M), np.complex128)
    sig = np.zeros((F, M), np.float64)
    st = np.zeros(F, np.int32)
    lib().orc_gevd(_ptr(K), _ptr(R), F, M, Ns, default_tol(M) if tol is None else tol, max_sweeps,
                   nthreads, _ptr(En), _ptr(sig), _ptr(st))
    return En, sig, st


def localize(X: np.ndarray, K: np.ndarray, H: np.ndarray, n_az: int, n_el: int, Ns: int,
             p: int = 2, tol: float | None = None, max_sweeps: int = DEFAULT_MAX_SWEEPS,
             nthreads: int = 1, want_P: bool = False, gevd: bool = False):
    """One block end to end (GSVD-MUSIC, or GEVD-MUSIC with gevd=True).  Returns dict(peaks,
    peak_val, Pbar, status[, P])."""
    if X.dtype != np.complex64:
        raise TypeError("X must be complex64")
    if X.strides[2] != 8:
        X = np.ascontiguousarray(X)
    F, T, M = X.shape
    K = _c128(K)
    H = np.ascontiguousarray(H, dtype=np.complex64)
    D = n_az * n_el
    pk = np.full(Ns, -1, np.int32)
    pv = np.zeros(Ns, np.float64)
    Pbar = np.zeros(D, np.float64)
    st = np.zeros(F, np.int32)
    P = np.zeros((F, D), np.float64) if want_P else None
    lib().orc_localize_m(_ptr(X), F, T, M, X.strides[0] // 8, X.strides[1] // 8, _ptr(K),
                         _ptr(H), n_az, n_el, Ns, p, default_tol(M) if tol is None else tol,
                         max_sweeps, nthreads, int(bool(gevd)), _ptr(pk), _ptr(pv), _ptr(Pbar),
                         _ptr(st), _ptr(P) if want_P else None)
    out = dict(peaks=pk, peak_val=pv, Pbar=Pbar, status=st)
    if want_P:
        out["P"] = P
    return out


def sliding_corr(X: np.ndarray, T: int, f: int) -> np.ndarray:
    """eq.3 as printed: R(w, f) = (1/T) sum_{i = -T+1}^{0} x(w, f + i) x(w, f + i)^H, the
    correlation of the T frames ending at frame f of a frame sequence X [F][n_frames][M]
    (complex64); needs T - 1 <= f < n_frames."""
    if f < T - 1 or f >= X.shape[1]:
        raise ValueError("frame f has fewer than T frames before it, or is past the sequence")
    return corr(X[:, f - T + 1:f + 1, :], 1.0 / T)


def localize_frame(X: np.ndarray, T: int, f: int, K, H: np.ndarray, n_az: int, n_el: int,
                   Ns: int, p: int = 2, nthreads: int = 1):
    """The localization of frame f of a frame sequence: eq.3's window of the T frames ending at f,
    then the whole method on it (K None: SEVD-MUSIC, K = I)."""
    if f < T - 1 or f >= X.shape[1]:
        raise ValueError("frame f has fewer than T frames before it, or is past the sequence")
    W = X[:, f - T + 1:f + 1, :]
    if K is None:
        K = np.broadcast_to(np.eye(X.shape[2], dtype=np.complex128), (X.shape[0],) + (X.shape[2],) * 2)
    return localize(W, K, H, n_az, n_el, Ns, p=p, nthreads=nthreads)


def noise_corr(Xn: np.ndarray) -> np.ndarray:
    """K estimated from noise-only frames with the eq.2-3 definition (scale 1/N)."""
    return corr(Xn)
