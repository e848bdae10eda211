"""Seeded synthetic inputs for GSVD-MUSIC sound-source localization.

This module only *builds inputs*: microphone-array geometries, free-field
transfer-function tables H(theta, omega) (the quantity in eq.5 that the paper
measures for its 60-channel array, Sec. V-C), STFT-domain multichannel blocks
X(omega, f) (eq.1) and noise-only frames from which the preset noise
correlation K is estimated (Sec. III-A, the text after eq.4).  It contains
none of the method's arithmetic (no correlation, no solve, no SVD, no
spectrum, no peak search): both the HIP path and the CPU oracle consume the
exact complex64 bytes produced here.

Conventions (the paper does not fix them; they are stated once here):
  * far-field free-field steering H_m(theta, omega) = exp(+j 2 pi f_omega (u . p_m) / c),
    f_omega = omega * fs / nfft, c = 343 m/s, u = (cos el cos az, cos el sin az, sin el);
  * direction grid: az = az_step * k (k < n_az), el = el_step * l (l < n_el),
    flat index d = l * n_az + k;
  * STFT-domain synthesis X = sum_s h(theta_s) s + sum_j h(theta_j) n_j + w with
    s, n_j, w i.i.d. circular complex Gaussian over (bin, frame).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Sequence

import numpy as np

C_SOUND = 343.0


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
def circle_array(M: int, radius: float = 0.1) -> np.ndarray:
    """Uniform circular array in the xy-plane, p_m = r (cos 2 pi m/M, sin 2 pi m/M, 0)."""
    m = np.arange(M, dtype=np.float64)
    ang = 2.0 * np.pi * m / M
    return np.stack([radius * np.cos(ang), radius * np.sin(ang), np.zeros(M)], axis=1)


def ring_array60() -> np.ndarray:
    """60 microphones in 4 horizontal rings of 15.

    Ring q = 0..3 has radius 0.10 + 0.05 q m, height 0.10 q m and the ring is
    rotated by q * 2 pi / 60 so that no two rings share azimuths.
    """
    pos = []
    for q in range(4):
        r = 0.10 + 0.05 * q
        z = 0.10 * q
        for k in range(15):
            phi = 2.0 * np.pi * k / 15.0 + q * 2.0 * np.pi / 60.0
            pos.append((r * np.cos(phi), r * np.sin(phi), z))
    return np.asarray(pos, dtype=np.float64)


def array_for(M: int) -> np.ndarray:
    """Geometry used for an M-channel stream: 60 -> rings, otherwise a circle of r = 0.1 m."""
    return ring_array60() if M == 60 else circle_array(M, 0.1)


@dataclasses.dataclass(frozen=True)
class DirectionGrid:
    n_az: int
    n_el: int
    az_step_deg: float = 5.0
    el_step_deg: float = 5.0

    @property
    def D(self) -> int:
        return self.n_az * self.n_el

    def angles_deg(self):
        """(az, el) in degrees for every flat index d = l * n_az + k."""
        k = np.arange(self.n_az)
        l = np.arange(self.n_el)
        az = np.tile(k * self.az_step_deg, self.n_el)
        el = np.repeat(l * self.el_step_deg, self.n_az)
        return az.astype(np.float64), el.astype(np.float64)

    def unit_vectors(self) -> np.ndarray:
        az, el = self.angles_deg()
        return unit_vector(az, el)


def unit_vector(az_deg, el_deg) -> np.ndarray:
    az = np.deg2rad(np.asarray(az_deg, dtype=np.float64))
    el = np.deg2rad(np.asarray(el_deg, dtype=np.float64))
    return np.stack([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)], axis=-1)


def bin_freqs(F: int, fs: float = 16000.0, nfft: Optional[int] = None) -> np.ndarray:
    """Centre frequency of bin omega = 0..F-1 of an nfft-point STFT (nfft = 2 (F - 1) by default)."""
    if nfft is None:
        nfft = 2 * (F - 1)
    return np.arange(F, dtype=np.float64) * fs / nfft


def steering(pos: np.ndarray, u: np.ndarray, freqs: np.ndarray) -> np.ndarray:
    """Free-field far-field transfer functions, complex128 of shape [F][D][M]."""
    delay = (u @ pos.T) / C_SOUND                       # [D][M] seconds
    phase = 2.0 * np.pi * freqs[:, None, None] * delay[None, :, :]
    return np.exp(1j * phase)


def steering_table(pos: np.ndarray, grid: DirectionGrid, freqs: np.ndarray) -> np.ndarray:
    """The [F][D][M] complex64 table H(theta, omega) handed to both paths."""
    return np.ascontiguousarray(steering(pos, grid.unit_vectors(), freqs).astype(np.complex64))


def angular_distance_deg(u1: np.ndarray, u2: np.ndarray) -> float:
    c = float(np.clip(np.dot(u1, u2), -1.0, 1.0))
    return math.degrees(math.acos(c))


# ----------------------------------------------------------------------------
# signals
# ----------------------------------------------------------------------------
def cn(rng: np.random.Generator, shape, power: float) -> np.ndarray:
    """Circular complex Gaussian CN(0, power)."""
    s = math.sqrt(power / 2.0)
    return s * rng.standard_normal(shape) + 1j * (s * rng.standard_normal(shape))


def mix(rng: np.random.Generator, pos, freqs, n_frames: int,
        src_u: Sequence[np.ndarray], p_src: Sequence[float],
        noise_u: Sequence[np.ndarray], p_noise: Sequence[float],
        sigma_d2: float) -> np.ndarray:
    """X[F][n_frames][M] complex64 = sum of plane-wave sources + directional noises + white noise."""
    F = freqs.shape[0]
    M = pos.shape[0]
    X = cn(rng, (F, n_frames, M), sigma_d2) if sigma_d2 > 0 else np.zeros((F, n_frames, M), np.complex128)
    for u, p in list(zip(src_u, p_src)) + list(zip(noise_u, p_noise)):
        h = steering(pos, np.asarray(u)[None, :], freqs)[:, 0, :]      # [F][M]
        s = cn(rng, (F, n_frames), p)                                    # [F][T]
        X += s[:, :, None] * h[:, None, :]
    return np.ascontiguousarray(X.astype(np.complex64))


def pcm_scene(rng: np.random.Generator, pos, fs: float, n_samples: int,
              src_u: Sequence[np.ndarray], p_src: Sequence[float],
              noise_u: Sequence[np.ndarray], p_noise: Sequence[float],
              sigma_d2: float) -> np.ndarray:
    """Time-domain multichannel PCM [n_samples][M] float32 (channel-interleaved): plane-wave
    sources and directional noises, each a white Gaussian signal of power p reaching microphone m
    (u . p_m) / c seconds early -- applied as a phase exp(+j 2 pi f (u . p_m) / c) on its
    circular spectrum, the free-field convention of the steering table -- plus white noise of
    power sigma_d2 per channel."""
    M = pos.shape[0]
    freqs = np.fft.rfftfreq(n_samples, 1.0 / fs)
    x = math.sqrt(sigma_d2) * rng.standard_normal((n_samples, M)) if sigma_d2 > 0 \
        else np.zeros((n_samples, M))
    for u, p in list(zip(src_u, p_src)) + list(zip(noise_u, p_noise)):
        sig = math.sqrt(p) * rng.standard_normal(n_samples)
        S = np.fft.rfft(sig)
        adv = (np.asarray(u) @ pos.T) / C_SOUND                          # [M] seconds early
        Sm = S[:, None] * np.exp(2j * np.pi * freqs[:, None] * adv[None, :])
        x += np.fft.irfft(Sm, n=n_samples, axis=0)
    return np.ascontiguousarray(x.astype(np.float32))


def pcm_workload(M: int = 8, seed: int = 1006, nfft: int = 512, hop: int = 160, T: int = 50,
                 n_blocks: int = 4):
    """Time-domain version of the 8-mic (M = 8) or 60-mic workload for the STFT front end:
    blocks of T frames of nfft samples at hop `hop` (16 kHz), sources on the direction grid.
    Returns (workload, pcm_block(b) -> (pcm, dirs), noise_pcm) where noise_pcm holds 4M frames of
    the noise field alone (for K)."""
    w = workload_small(n_blocks=n_blocks, seed=seed) if M == 8 else \
        workload_paper(n_blocks=n_blocks, seed=seed, M=M)
    fs = 16000.0
    n = (T - 1) * hop + nfft
    n_noise = (max(4 * M, 50) - 1) * hop + nfft

    def pcm_block(b: int):
        rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(3)[2].spawn(b + 1)[b])
        dirs = w._source_dirs(rng)
        ref = w.sigma_d2 if w.white_ref else w.sigma_d2 + sum(w.p_noise)
        p_s = ref * 10.0 ** (float(rng.uniform(*w.snr_db_range)) / 10.0)
        az, el = w.grid.angles_deg()
        src_u = [unit_vector(az[d], el[d]) for d in dirs]
        return pcm_scene(rng, w.pos, fs, n, src_u, [p_s] * w.Ns, w.noise_u, w.p_noise,
                         w.sigma_d2), dirs

    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(3)[0])
    noise = pcm_scene(rng, w.pos, fs, n_noise, [], [], w.noise_u, w.p_noise, w.sigma_d2)
    return w, pcm_block, noise


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    """One localization workload: geometry, grid, powers and the seeded draws."""
    name: str
    M: int
    F: int
    T: int
    Ns: int
    grid: DirectionGrid
    n_blocks: int
    n_noise_frames: int
    pos: np.ndarray
    freqs: np.ndarray
    noise_u: list
    p_noise: list
    sigma_d2: float
    snr_db_range: tuple
    white_ref: bool          # True: SNR is taken against the white noise only
    max_src_el: float
    seed: int

    @property
    def D(self) -> int:
        return self.grid.D

    def steering_table(self) -> np.ndarray:
        return steering_table(self.pos, self.grid, self.freqs)

    def noise_frames(self) -> np.ndarray:
        """Noise-only frames [F][N_K][M] from which K is estimated (same noise field as the blocks)."""
        rng = np.random.default_rng(np.random.SeedSequence(self.seed).spawn(1)[0].spawn(1)[0])
        return mix(rng, self.pos, self.freqs, self.n_noise_frames, [], [],
                   self.noise_u, self.p_noise, self.sigma_d2)

    def _source_dirs(self, rng):
        """Ns distinct grid directions, el <= max_src_el, >= 20 deg from the noises and each other."""
        az, el = self.grid.angles_deg()
        ok = np.nonzero(el <= self.max_src_el + 1e-9)[0]
        chosen = []
        for _ in range(10000):
            d = int(rng.choice(ok))
            u = unit_vector(az[d], el[d])
            if any(angular_distance_deg(u, v) < 20.0 for v in self.noise_u):
                continue
            if any(angular_distance_deg(u, unit_vector(az[c], el[c])) < 20.0 for c in chosen):
                continue
            chosen.append(d)
            if len(chosen) == self.Ns:
                return chosen
        raise RuntimeError("could not place sources")

    def block(self, b: int):
        """Block b: returns (X [F][T][M] complex64, list of source flat indices, snr_db)."""
        ss = np.random.SeedSequence(self.seed).spawn(2)[1].spawn(self.n_blocks if b < self.n_blocks else b + 1)[b]
        rng = np.random.default_rng(ss)
        dirs = self._source_dirs(rng)
        snr_db = float(rng.uniform(*self.snr_db_range)) if self.snr_db_range[0] != self.snr_db_range[1] \
            else float(self.snr_db_range[0])
        ref = self.sigma_d2 if self.white_ref else self.sigma_d2 + sum(self.p_noise)
        p_s = ref * 10.0 ** (snr_db / 10.0)
        az, el = self.grid.angles_deg()
        src_u = [unit_vector(az[d], el[d]) for d in dirs]
        X = mix(rng, self.pos, self.freqs, self.T, src_u, [p_s] * self.Ns,
                self.noise_u, self.p_noise, self.sigma_d2)
        return X, dirs, snr_db


def workload_small(n_blocks: int = 10, seed: int = 1001) -> Workload:
    """8-mic circle (r = 0.1 m), 257 bins of a 512-point STFT at 16 kHz, T = 50, Ns = 1 on a
    72-direction azimuth grid; white noise 10 dB below the source, one directional noise at
    the source power; K from 50 noise-only frames."""
    grid = DirectionGrid(72, 1)
    F = 257
    return Workload(name="gsvd-music-8ch-257bin-72dir", M=8, F=F, T=50, Ns=1, grid=grid,
                    n_blocks=n_blocks, n_noise_frames=50, pos=circle_array(8, 0.1),
                    freqs=bin_freqs(F, 16000.0, 512), noise_u=[unit_vector(200.0, 0.0)],
                    p_noise=[1.0], sigma_d2=0.1, snr_db_range=(10.0, 10.0), white_ref=True,
                    max_src_el=0.0, seed=seed)


def workload_paper(n_blocks: int = 1000, seed: int = 1002, M: int = 60, F: int = 257,
                   Ns: int = 2) -> Workload:
    """60-mic 4-ring array, 257 bins, T = 50, Ns = 2 at random grid directions (el <= 80 deg),
    SNR ~ U[-5, 10] dB against white + 2 directional noises of equal power; K from 4M frames;
    72 x 19 = 1368 directions (upper hemisphere, 5 degree steps).  Other M use a circle of
    r = 0.1 m, other F the matching STFT length."""
    grid = DirectionGrid(72, 19)
    nfft = 2 * (F - 1)
    return Workload(name=f"gsvd-music-{M}ch-{F}bin-1368dir", M=M, F=F, T=50, Ns=Ns, grid=grid,
                    n_blocks=n_blocks, n_noise_frames=4 * M, pos=array_for(M),
                    freqs=bin_freqs(F, 16000.0, nfft),
                    noise_u=[unit_vector(135.0, 10.0), unit_vector(290.0, 30.0)],
                    p_noise=[1.0, 1.0], sigma_d2=1.0, snr_db_range=(-5.0, 10.0), white_ref=False,
                    max_src_el=80.0, seed=seed)


@dataclasses.dataclass
class ArrayStream:
    """One simulated array stream for the serving workload: fixed geometry and noise field,
    sources whose azimuths random-walk by +-2 degrees per block (off-grid), el fixed per source."""
    sid: int
    M: int
    F: int
    T: int
    Ns: int
    grid: DirectionGrid
    pos: np.ndarray
    freqs: np.ndarray
    noise_u: list
    p_noise: list
    sigma_d2: float
    snr_db: float
    src_az0: list
    src_el: list
    seed: int

    @property
    def D(self) -> int:
        return self.grid.D

    def source_azimuths(self, seq: int) -> list:
        """Azimuths (degrees) of the sources in block `seq` (random walk from the start angles)."""
        rng = np.random.default_rng(np.random.SeedSequence(self.seed).spawn(3)[2])
        steps = rng.choice([-2.0, 2.0], size=(seq + 1, self.Ns))
        steps[0] = 0.0
        return list((np.asarray(self.src_az0) + np.cumsum(steps, axis=0)[seq]) % 360.0)

    def block(self, seq: int):
        """(X [F][T][M], noise-only frames [F][T][M]) of block `seq`, both complex64."""
        rng = np.random.default_rng(np.random.SeedSequence(self.seed).spawn(2)[1].spawn(seq + 1)[seq])
        az = self.source_azimuths(seq)
        src_u = [unit_vector(a, e) for a, e in zip(az, self.src_el)]
        p_s = (self.sigma_d2 + sum(self.p_noise)) * 10.0 ** (self.snr_db / 10.0)
        X = mix(rng, self.pos, self.freqs, self.T, src_u, [p_s] * self.Ns, self.noise_u,
                self.p_noise, self.sigma_d2)
        Xn = mix(rng, self.pos, self.freqs, self.T, [], [], self.noise_u, self.p_noise, self.sigma_d2)
        return X, Xn

    def initial_noise_frames(self) -> np.ndarray:
        """4M noise-only frames for the stream's first K."""
        rng = np.random.default_rng(np.random.SeedSequence(self.seed).spawn(1)[0])
        return mix(rng, self.pos, self.freqs, 4 * self.M, [], [], self.noise_u, self.p_noise,
                   self.sigma_d2)


def serving_streams(n_streams: int = 64, seed: int = 1005, Ms=(8, 16, 60)):
    """Array streams of the serving workload: M drawn uniformly from Ms (Ns = 2 for 60 mics,
    1 otherwise), 257 bins, T = 50, 1368-direction grid, two directional noises + white noise,
    SNR ~ U[0, 10] dB, sources starting at random azimuths (el 0-40 degrees)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    out = []
    for s in range(n_streams):
        M = int(rng.choice(list(Ms)))
        Ns = 2 if M == 60 else 1
        out.append(ArrayStream(sid=s, M=M, F=257, T=50, Ns=Ns, grid=DirectionGrid(72, 19),
                               pos=array_for(M), freqs=bin_freqs(257, 16000.0, 512),
                               noise_u=[unit_vector(135.0, 10.0), unit_vector(290.0, 30.0)],
                               p_noise=[1.0, 1.0], sigma_d2=1.0,
                               snr_db=float(rng.uniform(0.0, 10.0)),
                               src_az0=list(rng.uniform(0.0, 360.0, size=Ns)),
                               src_el=list(rng.choice([0.0, 20.0, 40.0], size=Ns)),
                               seed=seed * 1000 + s))
    return out


def poisson_arrivals(n_streams: int, duration_s: float, mean_period_s: float = 0.010,
                     seed: int = 1006):
    """(emit time, stream, seq) of every block emitted in [0, duration): per stream, exponential
    inter-arrival times with the given mean (a Poisson process), sorted by time."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    ev = []
    for s in range(n_streams):
        t = float(rng.uniform(0.0, mean_period_s))
        seq = 0
        while t < duration_s:
            ev.append((t, s, seq))
            seq += 1
            t += float(rng.exponential(mean_period_s))
    ev.sort()
    return ev


def uneven_shapes(n_blocks: int, seed: int = 1004):
    """Shapes of an uneven batch: M in {8, 16, 32, 60}, 512- or 1024-point STFT (F = 257 / 513) and
    Ns in {1, 2, 3}, each uniform; returns a list of (M, F, Ns) tuples."""
    rng = np.random.default_rng(np.random.SeedSequence(seed))
    Ms = rng.choice([8, 16, 32, 60], size=n_blocks)
    Fs = rng.choice([257, 513], size=n_blocks)
    Nss = rng.integers(1, 4, size=n_blocks)
    return [(int(m), int(f), int(n)) for m, f, n in zip(Ms, Fs, Nss)]


def analytic_noise_corr(pos, freqs, noise_u, sigma_d2: float, rho: float) -> np.ndarray:
    """K = sigma_d^2 I + rho sum_j d_j d_j^H (complex128 [F][M][M]); one directional term gives
    cond(K) = 1 + M rho / sigma_d^2 exactly (|d_m| = 1)."""
    F = freqs.shape[0]
    M = pos.shape[0]
    K = np.zeros((F, M, M), np.complex128)
    K += sigma_d2 * np.eye(M)[None]
    for u in noise_u:
        d = steering(pos, np.asarray(u)[None, :], freqs)[:, 0, :]
        K += rho * d[:, :, None] * d[:, None, :].conj()
    return K
