"""MI355X (gfx950) GSVD-MUSIC sound-source localization -- Python binding of the C ABI.

Thin ctypes layer over ``libssl_mi355x.so`` (include/ssl.h).  Functions carry the C names and
only marshal arguments: tensors become device pointers, the current torch stream becomes the
hipStream_t, errors become :class:`SSLError`.  Every step of the method runs in the library's
HIP kernels; there is no other implementation behind these calls, and importing or calling them
without the built library raises immediately.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libssl_mi355x.so")

# ssl_status
SSL_OK, SSL_ERR_ARG, SSL_ERR_NOMEM, SSL_ERR_BUDGET, SSL_ERR_HIP, SSL_ERR_STATE = 0, -1, -2, -3, -4, -5
# ssl_bin_status
SSL_BIN_OK, SSL_BIN_NOT_PD, SSL_BIN_NO_CONV, SSL_BIN_NONFINITE = 0, 1, 2, 3
# ssl_prec
SSL_FP32, SSL_BF16, SSL_FP16, SSL_FP64 = 0, 1, 2, 3
# ssl_svd
SSL_SVD_JACOBI, SSL_SVD_BIDIAG_QR = 0, 1
# ssl_subspace
SSL_SUBSPACE_GSVD, SSL_SUBSPACE_GEVD = 0, 1
# ssl_stop
SSL_STOP_NEVER, SSL_STOP_BATCH, SSL_STOP_LOCALIZE, SSL_STOP_ALSO_GSVD = 0, 1, 2, 3
# ssl_projection
SSL_PROJ_NOISE, SSL_PROJ_SIGNAL = 0, 1
# fixed scratch of ssl_localize_noalloc (bytes, per device)
SSL_NOALLOC_SCRATCH_BYTES = 64 << 20

EXPORTED = [
    "ssl_ctx_create", "ssl_ctx_destroy", "ssl_ctx_workspace_bytes", "ssl_last_error", "ssl_version",
    "ssl_corr_accum", "ssl_noise_create", "ssl_noise_set", "ssl_noise_update", "ssl_noise_get",
    "ssl_noise_destroy", "ssl_gsvd", "ssl_music_spectrum", "ssl_peaks", "ssl_localize",
    "ssl_ctx_timing", "ssl_ctx_timing_read", "ssl_localize_batch", "ssl_ctx_use_graphs",
    "ssl_ctx_set_jacobi_lanes", "ssl_ctx_get_jacobi_lanes", "ssl_autotune_jacobi",
    "ssl_ctx_set_steer_waves", "ssl_ctx_get_steer_waves", "ssl_autotune_steer",
    "ssl_noise_update_frames",
    "ssl_noise_update_frames_from",
    "ssl_localize_noalloc", "ssl_localize_noalloc_bytes", "ssl_stft",
    "ssl_tf_write", "ssl_tf_info_read", "ssl_tf_load", "ssl_steering_convert",
    "ssl_sliding_create", "ssl_sliding_destroy", "ssl_sliding_push", "ssl_sliding_frames",
    "ssl_sliding_corr", "ssl_sliding_localize", "ssl_ctx_set_svd", "ssl_ctx_get_svd",
    "ssl_ctx_set_subspace", "ssl_ctx_get_subspace", "ssl_noise_enable_gevd",
    "ssl_ctx_set_stop", "ssl_ctx_get_stop", "ssl_ctx_set_projection", "ssl_ctx_get_projection",
]


class BlockDesc(ctypes.Structure):
    """ssl_block_desc."""
    _fields_ = [("X", ctypes.c_void_p), ("strideF", ctypes.c_int64), ("strideT", ctypes.c_int64),
                ("F", ctypes.c_int), ("T", ctypes.c_int), ("M", ctypes.c_int), ("Ns", ctypes.c_int),
                ("K", ctypes.c_void_p), ("H", ctypes.c_void_p), ("n_az", ctypes.c_int),
                ("n_el", ctypes.c_int), ("peaks", ctypes.c_void_p), ("peak_val", ctypes.c_void_p),
                ("Pbar", ctypes.c_void_p), ("bin_status", ctypes.c_void_p),
                ("conv", ctypes.c_void_p)]
KERNELS = ["corr", "noise", "whiten", "jacobi", "steer", "binsum"]


class TfInfo(ctypes.Structure):
    """ssl_tf_info."""
    _fields_ = [("M", ctypes.c_int), ("F", ctypes.c_int), ("n_az", ctypes.c_int),
                ("n_el", ctypes.c_int), ("nfft", ctypes.c_int), ("fs", ctypes.c_float),
                ("az0_deg", ctypes.c_float), ("az_step_deg", ctypes.c_float),
                ("el0_deg", ctypes.c_float), ("el_step_deg", ctypes.c_float)]


class SSLError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed with status {code}: {msg}")
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Loads the built HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2504_03373_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    P, I, I64, D, SZ = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_size_t
    sig = {
        "ssl_ctx_create": (I, [ctypes.POINTER(P), I, SZ]),
        "ssl_ctx_destroy": (None, [P]),
        "ssl_ctx_workspace_bytes": (SZ, [P]),
        "ssl_last_error": (ctypes.c_char_p, []),
        "ssl_version": (I, []),
        "ssl_ctx_timing": (I, [P, I]),
        "ssl_ctx_timing_read": (I, [P, P, P, I]),
        "ssl_corr_accum": (I, [P, P, I, I, I, I64, I64, D, I, I, P, P]),
        "ssl_noise_create": (I, [P, I, I, ctypes.POINTER(P)]),
        "ssl_noise_set": (I, [P, P, I, P, P]),
        "ssl_noise_update": (I, [P, P, I, D, P, P]),
        "ssl_noise_get": (I, [P, P, P]),
        "ssl_noise_destroy": (None, [P]),
        "ssl_gsvd": (I, [P, P, P, I, I, I, P, P, P, P, I, P]),
        "ssl_music_spectrum": (I, [P, P, I, P, I, I, I, I, I, P, P, P, P]),
        "ssl_peaks": (I, [P, P, I, I, I, P, P, P]),
        "ssl_localize": (I, [P, P, I, I, I, I64, I64, P, P, I, I, I, I, I, P, P, P, P, P]),
        "ssl_localize_noalloc": (I, [P, P, I, I, I, I64, I64, P, P, I, I, I, I, I, P, P, P, P, P]),
        "ssl_stft": (I, [P, P, I64, I, I, I, I, P, P, P]),
        "ssl_ctx_set_svd": (I, [P, I]),
        "ssl_ctx_get_svd": (I, [P]),
        "ssl_ctx_set_subspace": (I, [P, I]),
        "ssl_ctx_get_subspace": (I, [P]),
        "ssl_noise_enable_gevd": (I, [P, P]),
        "ssl_ctx_set_stop": (I, [P, I]),
        "ssl_ctx_get_stop": (I, [P]),
        "ssl_ctx_set_projection": (I, [P, I]),
        "ssl_ctx_get_projection": (I, [P]),
        "ssl_sliding_create": (I, [P, I, I, I, ctypes.POINTER(P)]),
        "ssl_sliding_destroy": (None, [P]),
        "ssl_sliding_push": (I, [P, P, I, I64, I64, P]),
        "ssl_sliding_frames": (I64, [P]),
        "ssl_sliding_corr": (I, [P, P, P]),
        "ssl_sliding_localize": (I, [P, P, P, I, I, I, I, I, I, P, P, P, P, P, P]),
        "ssl_tf_write": (I, [ctypes.c_char_p, ctypes.POINTER(TfInfo), P, P]),
        "ssl_tf_info_read": (I, [ctypes.c_char_p, ctypes.POINTER(TfInfo), P]),
        "ssl_tf_load": (I, [P, ctypes.c_char_p, I, P, P]),
        "ssl_steering_convert": (I, [P, P, I, I, I, I, P, P]),
        "ssl_localize_noalloc_bytes": (ctypes.c_size_t, [I, I, I, I]),
        "ssl_localize_batch": (I, [P, ctypes.POINTER(BlockDesc), I, I, I, P]),
        "ssl_ctx_use_graphs": (I, [P, I]),
        "ssl_ctx_set_jacobi_lanes": (I, [P, I, I]),
        "ssl_ctx_get_jacobi_lanes": (I, [P, I]),
        "ssl_autotune_jacobi": (I, [P, P, P, I, I, I, I, I, ctypes.POINTER(I),
                                    ctypes.POINTER(ctypes.c_double), P]),
        "ssl_ctx_set_steer_waves": (I, [P, I, I, I, I]),
        "ssl_noise_update_frames": (I, [P, I, ctypes.POINTER(P), ctypes.POINTER(P),
                                        ctypes.POINTER(I), ctypes.c_double, P]),
        "ssl_noise_update_frames_from": (I, [P, I, ctypes.POINTER(P), ctypes.POINTER(P),
                                             ctypes.POINTER(P), ctypes.POINTER(I),
                                             ctypes.c_double, P]),
        "ssl_ctx_get_steer_waves": (I, [P, I, I, I]),
        "ssl_autotune_steer": (I, [P, P, I, P, I, I, I, I, I, I, I, ctypes.POINTER(I),
                                   ctypes.POINTER(ctypes.c_double), P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda:
        raise ValueError("array arguments must be device tensors")
    return t.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(fn: str, code: int):
    if code != SSL_OK:
        raise SSLError(fn, code, lib().ssl_last_error().decode())


# ------------------------------------------------------------------------------------------------
def ssl_version() -> int:
    return lib().ssl_version()


def ssl_ctx_timing(ctx: int, enable: bool) -> None:
    _check("ssl_ctx_timing", lib().ssl_ctx_timing(ctx, int(bool(enable))))


def ssl_ctx_timing_read(ctx: int, reset: bool = True) -> dict:
    """{kernel: (launches, total device ms)} since the last reset (waits for recorded events)."""
    n = (ctypes.c_int64 * len(KERNELS))()
    ms = (ctypes.c_double * len(KERNELS))()
    _check("ssl_ctx_timing_read", lib().ssl_ctx_timing_read(ctx, n, ms, int(bool(reset))))
    return {k: (int(n[i]), float(ms[i])) for i, k in enumerate(KERNELS)}


def ssl_last_error() -> str:
    return lib().ssl_last_error().decode()


def ssl_ctx_create(device: int = 0, hbm_budget_bytes: int = 0) -> int:
    out = ctypes.c_void_p()
    _check("ssl_ctx_create", lib().ssl_ctx_create(ctypes.byref(out), device, hbm_budget_bytes))
    return out.value


def ssl_ctx_destroy(ctx: int) -> None:
    lib().ssl_ctx_destroy(ctx)


def ssl_ctx_workspace_bytes(ctx: int) -> int:
    return lib().ssl_ctx_workspace_bytes(ctx)


def ssl_tf_write(path, info: "TfInfo", pos, H) -> None:
    """Host: writes a table file.  pos: float64 numpy [M][3]; H: complex64 numpy [F][D][M]."""
    import numpy as np
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    H = np.ascontiguousarray(H, dtype=np.complex64)
    if pos.shape != (info.M, 3) or H.shape != (info.F, info.n_az * info.n_el, info.M):
        raise ValueError("pos / H shapes do not match info")
    _check("ssl_tf_write", lib().ssl_tf_write(os.fsencode(path), ctypes.byref(info),
                                              pos.ctypes.data_as(ctypes.c_void_p),
                                              H.ctypes.data_as(ctypes.c_void_p)))


def ssl_tf_info_read(path):
    """Host: returns (TfInfo, pos float64 numpy [M][3])."""
    import numpy as np
    info = TfInfo()
    _check("ssl_tf_info_read", lib().ssl_tf_info_read(os.fsencode(path), ctypes.byref(info), None))
    pos = np.zeros((info.M, 3), np.float64)
    _check("ssl_tf_info_read", lib().ssl_tf_info_read(os.fsencode(path), ctypes.byref(info),
                                                      pos.ctypes.data_as(ctypes.c_void_p)))
    return info, pos


def ssl_tf_load(ctx, path, prec, H, stream=None):
    """Loads a table file into the device tensor H ([F][D][M] complex64 for SSL_FP32, [F][D][2M]
    bfloat16 / float16 otherwise)."""
    _check("ssl_tf_load", lib().ssl_tf_load(ctx, os.fsencode(path), prec, _ptr(H), _stream(stream)))


def ssl_steering_convert(ctx, H, prec, Hout, stream=None):
    F, D, M = H.shape
    _check("ssl_steering_convert", lib().ssl_steering_convert(ctx, _ptr(H), F, D, M, prec, _ptr(Hout),
                                                              _stream(stream)))


def ssl_ctx_set_svd(ctx, method: int) -> None:
    _check("ssl_ctx_set_svd", lib().ssl_ctx_set_svd(ctx, method))


def ssl_ctx_get_svd(ctx) -> int:
    return int(lib().ssl_ctx_get_svd(ctx))


def ssl_ctx_set_subspace(ctx, method: int) -> None:
    _check("ssl_ctx_set_subspace", lib().ssl_ctx_set_subspace(ctx, method))


def ssl_ctx_get_subspace(ctx) -> int:
    return int(lib().ssl_ctx_get_subspace(ctx))


def ssl_ctx_set_stop(ctx, mode: int) -> None:
    _check("ssl_ctx_set_stop", lib().ssl_ctx_set_stop(ctx, mode))


def ssl_ctx_get_stop(ctx) -> int:
    return int(lib().ssl_ctx_get_stop(ctx))


def ssl_ctx_set_projection(ctx, mode: int) -> None:
    _check("ssl_ctx_set_projection", lib().ssl_ctx_set_projection(ctx, mode))


def ssl_ctx_get_projection(ctx) -> int:
    return int(lib().ssl_ctx_get_projection(ctx))


def ssl_noise_enable_gevd(noise, stream=None) -> None:
    _check("ssl_noise_enable_gevd", lib().ssl_noise_enable_gevd(noise, _stream(stream)))


def ssl_sliding_create(ctx, F: int, M: int, T: int) -> int:
    out = ctypes.c_void_p()
    _check("ssl_sliding_create", lib().ssl_sliding_create(ctx, F, M, T, ctypes.byref(out)))
    return out.value


def ssl_sliding_destroy(s) -> None:
    lib().ssl_sliding_destroy(s)


def ssl_sliding_push(s, X, stream=None):
    """Appends the frames of X: complex64 device tensor [F][n][M] (M contiguous)."""
    F, n, M = X.shape
    sF, sT, sM = X.stride()
    if sM != 1:
        raise ValueError("X must be contiguous along M")
    _check("ssl_sliding_push", lib().ssl_sliding_push(s, _ptr(X), n, sF, sT, _stream(stream)))


def ssl_sliding_frames(s) -> int:
    return int(lib().ssl_sliding_frames(s))


def ssl_sliding_corr(s, R, stream=None):
    _check("ssl_sliding_corr", lib().ssl_sliding_corr(s, _ptr(R), _stream(stream)))


def ssl_sliding_localize(s, noise, H, prec, n_az, n_el, Ns, p, warm, peaks, peak_val, Pbar=None,
                         bin_status=None, conv=None, stream=None):
    _check("ssl_sliding_localize",
           lib().ssl_sliding_localize(s, noise, _ptr(H), prec, n_az, n_el, Ns, p, int(warm),
                                      _ptr(peaks), _ptr(peak_val), _ptr(Pbar), _ptr(bin_status),
                                      _ptr(conv), _stream(stream)))


def ssl_stft(ctx, pcm, nfft, hop, T, X, window=None, stream=None):
    """eq.1.  pcm: float32 device tensor [n_samples][M] (contiguous); X: complex64 device tensor
    [nfft/2 + 1][T][M]; window: float32 device tensor [nfft] or None (periodic Hann)."""
    if pcm.dim() != 2 or not pcm.is_contiguous():
        raise ValueError("pcm must be a contiguous [n_samples][M] tensor")
    n, M = pcm.shape
    if tuple(X.shape) != (nfft // 2 + 1, T, M) or not X.is_contiguous():
        raise ValueError(f"X must be a contiguous [{nfft // 2 + 1}][{T}][{M}] tensor")
    _check("ssl_stft", lib().ssl_stft(ctx, _ptr(pcm), n, M, nfft, hop, T, _ptr(window), _ptr(X),
                                      _stream(stream)))


def ssl_corr_accum(ctx, X, scale, accumulate, prec, R, stream=None, F=None, T=None, M=None):
    """eq.2-3.  X: complex64 device tensor [F][T][M] (M contiguous, any F/T strides)."""
    F_, T_, M_ = X.shape
    sF, sT, sM = X.stride()
    if sM != 1:
        raise ValueError("X must be contiguous along M")
    _check("ssl_corr_accum", lib().ssl_corr_accum(ctx, _ptr(X), F_, T_, M_, sF, sT, float(scale),
                                                  int(accumulate), prec, _ptr(R), _stream(stream)))


def ssl_noise_create(ctx, F: int, M: int) -> int:
    out = ctypes.c_void_p()
    _check("ssl_noise_create", lib().ssl_noise_create(ctx, F, M, ctypes.byref(out)))
    return out.value


def ssl_noise_set(noise, K, kprec, bin_status=None, stream=None):
    _check("ssl_noise_set", lib().ssl_noise_set(noise, _ptr(K), kprec, _ptr(bin_status), _stream(stream)))


def ssl_noise_update(noise, Khat, kprec, alpha, bin_status=None, stream=None):
    _check("ssl_noise_update", lib().ssl_noise_update(noise, _ptr(Khat), kprec, float(alpha),
                                                      _ptr(bin_status), _stream(stream)))


def _frames_args(Xns, n):
    if len(Xns) != n:
        raise ValueError("one frame tensor per noise handle")
    for X in Xns:
        if not X.is_contiguous():
            raise ValueError("noise frames must be contiguous")
    xs = (ctypes.c_void_p * max(n, 1))(*[X.data_ptr() for X in Xns])
    ts = (ctypes.c_int * max(n, 1))(*[int(X.shape[1]) for X in Xns])
    return xs, ts


def ssl_noise_update_frames(ctx, noises, Xns, alpha, stream=None):
    """Serving EMA update of many handles from their noise-only frames (each [F][T][M] complex64,
    contiguous, on the device), one library call."""
    n = len(noises)
    xs, ts = _frames_args(Xns, n)
    hs = (ctypes.c_void_p * max(n, 1))(*noises)
    _check("ssl_noise_update_frames", lib().ssl_noise_update_frames(ctx, n, hs, xs, ts, float(alpha),
                                                                    _stream(stream)))


def ssl_noise_update_frames_from(ctx, dst, src, Xns, alpha, stream=None):
    """As ssl_noise_update_frames, blending from src[i]'s K into dst[i]."""
    n = len(dst)
    if len(src) != n:
        raise ValueError("one source handle per destination")
    xs, ts = _frames_args(Xns, n)
    hd = (ctypes.c_void_p * max(n, 1))(*dst)
    hs = (ctypes.c_void_p * max(n, 1))(*src)
    _check("ssl_noise_update_frames_from",
           lib().ssl_noise_update_frames_from(ctx, n, hd, hs, xs, ts, float(alpha), _stream(stream)))


def ssl_noise_get(noise, K_out, stream=None):
    _check("ssl_noise_get", lib().ssl_noise_get(noise, _ptr(K_out), _stream(stream)))


def ssl_noise_destroy(noise) -> None:
    lib().ssl_noise_destroy(noise)


def ssl_gsvd(ctx, R, noise, Ns, En, sigma=None, bin_status=None, conv=None, max_sweeps=0,
             stream=None):
    F, M, _ = R.shape
    _check("ssl_gsvd", lib().ssl_gsvd(ctx, _ptr(R), noise, F, M, Ns, _ptr(En), _ptr(sigma),
                                      _ptr(bin_status), _ptr(conv), max_sweeps, _stream(stream)))


def ssl_music_spectrum(ctx, H, hprec, En, Ns, p, P=None, Pbar=None, bin_status=None, stream=None,
                       F=None, D=None, M=None):
    """eq.5-6.  H: [F][D][M] complex64 (SSL_FP32) or [F][D][2M] bf16/fp16 pairs."""
    F_ = H.shape[0] if F is None else F
    D_ = H.shape[1] if D is None else D
    M_ = En.shape[2] if M is None else M
    _check("ssl_music_spectrum", lib().ssl_music_spectrum(ctx, _ptr(H), hprec, _ptr(En), F_, D_, M_,
                                                          Ns, p, _ptr(P), _ptr(Pbar),
                                                          _ptr(bin_status), _stream(stream)))


def ssl_peaks(ctx, Pbar, n_az, n_el, Ns, peaks, peak_val, stream=None):
    _check("ssl_peaks", lib().ssl_peaks(ctx, _ptr(Pbar), n_az, n_el, Ns, _ptr(peaks), _ptr(peak_val),
                                        _stream(stream)))


def ssl_localize(ctx, X, noise, H, prec, n_az, n_el, Ns, p, peaks, peak_val, Pbar=None,
                 bin_status=None, stream=None):
    F, T, M = X.shape
    sF, sT, sM = X.stride()
    if sM != 1:
        raise ValueError("X must be contiguous along M")
    _check("ssl_localize", lib().ssl_localize(ctx, _ptr(X), F, T, M, sF, sT, noise, _ptr(H), prec,
                                              n_az, n_el, Ns, p, _ptr(peaks), _ptr(peak_val),
                                              _ptr(Pbar), _ptr(bin_status), _stream(stream)))


def ssl_localize_noalloc(ctx, X, noise, H, prec, n_az, n_el, Ns, p, peaks, peak_val, Pbar=None,
                         bin_status=None, stream=None):
    F, T, M = X.shape
    sF, sT, sM = X.stride()
    if sM != 1:
        raise ValueError("X must be contiguous along M")
    _check("ssl_localize_noalloc",
           lib().ssl_localize_noalloc(ctx, _ptr(X), F, T, M, sF, sT, noise, _ptr(H), prec, n_az,
                                      n_el, Ns, p, _ptr(peaks), _ptr(peak_val), _ptr(Pbar),
                                      _ptr(bin_status), _stream(stream)))


def ssl_localize_noalloc_bytes(F, M, Ns, D):
    return int(lib().ssl_localize_noalloc_bytes(F, M, Ns, D))


def block_desc(X, noise, H, n_az, n_el, Ns, peaks, peak_val, Pbar=None, bin_status=None,
               conv=None):
    """One ssl_block_desc for ssl_localize_batch (X: complex64 device tensor [F][T][M]; conv:
    optional int32 [F][3] device tensor for the Jacobi statistics)."""
    F, T, M = X.shape
    sF, sT, sM = X.stride()
    if sM != 1:
        raise ValueError("X must be contiguous along M")
    return BlockDesc(_ptr(X), sF, sT, F, T, M, Ns, noise, _ptr(H), n_az, n_el, _ptr(peaks),
                     _ptr(peak_val), _ptr(Pbar), _ptr(bin_status), _ptr(conv))


def ssl_localize_batch(ctx, descs, prec, p, stream=None):
    """Whole path for a list of BlockDesc (see block_desc) in one set of launches."""
    arr = (BlockDesc * len(descs))(*descs)
    _check("ssl_localize_batch", lib().ssl_localize_batch(ctx, arr, len(descs), prec, p,
                                                          _stream(stream)))


def ssl_ctx_use_graphs(ctx, enable: bool) -> None:
    _check("ssl_ctx_use_graphs", lib().ssl_ctx_use_graphs(ctx, int(bool(enable))))


def ssl_ctx_set_jacobi_lanes(ctx, M: int, lanes: int) -> None:
    _check("ssl_ctx_set_jacobi_lanes", lib().ssl_ctx_set_jacobi_lanes(ctx, M, lanes))


def ssl_ctx_get_jacobi_lanes(ctx, M: int) -> int:
    return lib().ssl_ctx_get_jacobi_lanes(ctx, M)


def ssl_autotune_jacobi(ctx, R, noise, Ns: int, nblocks: int = 1, reps: int = 3, stream=None):
    """Times the Jacobi variants of R's channel class, one block per launch (nblocks = 1) or the
    persistent batched kernel over nblocks blocks; returns (best lanes, {lanes: ms})."""
    F, M, _ = R.shape
    best = ctypes.c_int(0)
    ms = (ctypes.c_double * 3)()
    _check("ssl_autotune_jacobi", lib().ssl_autotune_jacobi(ctx, _ptr(R), noise, F, M, Ns, nblocks, reps,
                                                            ctypes.byref(best), ms, _stream(stream)))
    return best.value, {l: ms[i] for i, l in enumerate((4, 8, 16)) if ms[i] >= 0}


def ssl_ctx_set_steer_waves(ctx, M: int, Ns: int, hprec: int, waves: int) -> None:
    _check("ssl_ctx_set_steer_waves", lib().ssl_ctx_set_steer_waves(ctx, M, Ns, hprec, waves))


def ssl_ctx_get_steer_waves(ctx, M: int, Ns: int, hprec: int) -> int:
    return lib().ssl_ctx_get_steer_waves(ctx, M, Ns, hprec)


def ssl_autotune_steer(ctx, H, hprec, En, Ns: int, p: int = 2, nblocks: int = 1, reps: int = 3,
                       stream=None):
    """Times the projection tile shapes on (H, En), single-block (nblocks = 1) or batched over
    nblocks blocks sharing H; returns (best waves, {waves: ms})."""
    F, D = H.shape[0], H.shape[1]
    M = En.shape[2]                                  # En: [F][M - Ns][M], a noise vector per row
    best = ctypes.c_int(0)
    ms = (ctypes.c_double * 3)()
    _check("ssl_autotune_steer", lib().ssl_autotune_steer(ctx, _ptr(H), hprec, _ptr(En), F, D, M,
                                                          Ns, p, nblocks, reps, ctypes.byref(best), ms,
                                                          _stream(stream)))
    return best.value, {w: ms[i] for i, w in enumerate((4, 8, 16))}
