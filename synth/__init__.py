"""Seeded synthetic visibilities for the online RFI screen.

Input generator shared by the oracle's checks, the GPU parity tests and the
benchmark.  It models what a correlator hands to the screen (Section 2,
eq. V): for every baseline (p, q) of N dual-polarised stations, every channel
and every time sample, the instantaneous 2x2 correlation matrix
V_pq = e_p e_q^H of the stations' complex voltage 2-vectors e.

The voltages follow the simulation recipe of Section 4.2 (receiver noise and
sky noise drawn as circular complex Gaussians, RFI added with a random
polarisation state), re-parameterised for per-channel streams:

* e_p = sqrt(1 - rho) n_p + sqrt(rho) s, with n_p, s ~ CN(0, I_2) i.i.d. and
  the sky signal s common to all stations (rho = "sky correlation").  The sky
  may be partially polarised: s = L z with L L^H = I + f (q s3 + u s1 + v s2).
* RFI is injected at the voltage level, e_p += A g(t) exp(i(2 pi f0 t + phi_p)) j,
  with a Jones vector j(theta, chi) of unit norm, a 0/1 time envelope g, a tone
  frequency f0 and a per-station phase phi_p.  The tone phase cancels in the
  conjugate product, so within a pulse the RFI part of V_pq is the constant,
  fully polarised matrix A^2 exp(i(phi_p - phi_q)) j j^H.
* The interference-to-noise ratio is defined in-pulse, per affected channel and
  per station voltage: INR = A^2 |j|^2 / E|e_p|^2 = A^2 / 2.

Nothing here computes any part of the screen (Stokes parameters, moments,
statistics, flags or averages).  Random numbers come from NumPy's PCG64, seeded
per call, so every array is reproducible from its seed.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "baseline_pairs", "n_baselines", "jones", "inr_to_amplitude", "Rfi",
    "Scene", "make_voltages", "correlate", "correlate_torch", "to_cf16",
    "scene_plain", "scene_fp32_baseline", "scene_mixed", "scene_null",
    "scene_serving_array", "rfi_truth", "device_voltages", "serving_mix", "PostRfi",
    "correlate_scene",
]


# --------------------------------------------------------------------------- geometry

def n_baselines(n_stations: int) -> int:
    """N stations give N(N+1)/2 correlation streams, autocorrelations included (Section 2)."""
    return n_stations * (n_stations + 1) // 2


def baseline_pairs(n_stations: int):
    """Station pairs (p, q), p <= q, in row-major upper-triangle order (autos included)."""
    p, q = np.triu_indices(n_stations)
    return p.astype(np.int64), q.astype(np.int64)


# --------------------------------------------------------------------------- RFI sources

def jones(theta: float, chi: float) -> np.ndarray:
    """Unit Jones vector of an elliptically polarised wave: orientation theta, ellipticity chi."""
    return np.array([np.cos(theta) * np.cos(chi) - 1j * np.sin(theta) * np.sin(chi),
                     np.sin(theta) * np.cos(chi) + 1j * np.cos(theta) * np.sin(chi)],
                    dtype=np.complex128)


def inr_to_amplitude(inr_db: float) -> float:
    """Voltage amplitude A for an in-pulse INR (dB): INR = A^2 / 2 for unit-variance noise per pol."""
    return float(np.sqrt(2.0 * 10.0 ** (inr_db / 10.0)))


@dataclass
class PostRfi:
    """RFI added after correlation with a fixed coherency (the simulation model of Section 4.2):
    V_pq += A^2 g(t) exp(i (phi_p - phi_q)) C,  C = pol_frac j j^H + (1 - pol_frac) I / 2,
    so its degree of polarisation is pol_frac and tr C = 1 (INR = A^2 / 2 as for Rfi)."""
    channels: Sequence[int]
    inr_db: float
    theta: float = 0.0
    chi: float = 0.0
    envelope: Optional[np.ndarray] = None
    pol_frac: float = 1.0


@dataclass
class Rfi:
    """One RFI source injected at voltage level.

    channels  : channel indices it occupies
    inr_db    : in-pulse interference-to-noise ratio
    theta,chi : polarisation state (Jones vector j(theta, chi)); ignored if ``unpolarized``
    envelope  : 0/1 time envelope of length T (None = always on)
    f0        : tone frequency in cycles per sample
    unpolarized : a constant-modulus wave whose polarisation is a random unit 2-vector drawn
                  independently per sample (no preferred direction)
    pol_frac  : fraction of the RFI power in the fixed state j; the rest is unpolarised as above
    """
    channels: Sequence[int]
    inr_db: float
    theta: float = 0.0
    chi: float = 0.0
    envelope: Optional[np.ndarray] = None
    f0: float = 0.05
    unpolarized: bool = False
    pol_frac: float = 1.0


def pulse_train(T: int, period: int, on: int, phase: int) -> np.ndarray:
    t = np.arange(T)
    return (((t + phase) % period) < on).astype(np.float32)


def burst_envelope(T: int, starts: Sequence[int], lengths: Sequence[int]) -> np.ndarray:
    g = np.zeros(T, np.float32)
    for s, n in zip(starts, lengths):
        g[s:s + n] = 1.0
    return g


# --------------------------------------------------------------------------- scenes

@dataclass
class Scene:
    """A fully specified synthetic integration: stations, channels, samples and sources."""
    n_stations: int
    n_channels: int
    n_samples: int
    seed: int
    rho: float = 0.1
    sky_pol_frac: float = 0.0
    rfi: List[Rfi] = field(default_factory=list)
    noise_scale: float = 1.0
    noise_free: bool = False       # RFI only (for closed-form checks)
    post_rfi: List[PostRfi] = field(default_factory=list)

    @property
    def n_baselines(self) -> int:
        return n_baselines(self.n_stations)


def _cn(rng, shape) -> np.ndarray:
    """Circular complex Gaussian CN(0, 1) in complex64 (real and imaginary variance 1/2)."""
    x = rng.standard_normal(size=shape + (2,), dtype=np.float32)
    x *= np.float32(np.sqrt(0.5))
    return x.view(np.complex64)[..., 0]


def make_voltages(scene: Scene) -> np.ndarray:
    """Station voltages e[N][C][T][2] (complex64) for a scene; deterministic in ``scene.seed``."""
    rng = np.random.default_rng(scene.seed)
    N, C, T = scene.n_stations, scene.n_channels, scene.n_samples
    e = _cn(rng, (N, C, T, 2))
    s = _cn(rng, (C, T, 2))
    if scene.sky_pol_frac > 0.0:
        # s -> L s with L L^H = I + f (q s3 + u s1 + v s2), (q, u, v) a random unit vector
        d = rng.standard_normal(3)
        d /= np.linalg.norm(d)
        f = scene.sky_pol_frac
        coh = np.array([[1 + f * d[0], f * (d[1] - 1j * d[2])],
                        [f * (d[1] + 1j * d[2]), 1 - f * d[0]]])
        L = np.linalg.cholesky(coh).astype(np.complex64)
        s = s @ L.T
    a = np.float32(np.sqrt(1.0 - scene.rho))
    b = np.float32(np.sqrt(scene.rho))
    e *= a
    e += b * s[None]
    if scene.noise_scale != 1.0:
        e *= np.float32(scene.noise_scale)
    if scene.noise_free:
        e[...] = 0
    t = np.arange(T)
    for src in scene.rfi:
        A = inr_to_amplitude(src.inr_db) * scene.noise_scale
        g = np.ones(T, np.float32) if src.envelope is None else src.envelope.astype(np.float32)
        phi = rng.uniform(0.0, 2 * np.pi, size=N)
        tone = np.exp(1j * (2 * np.pi * src.f0 * t))                        # [T]
        rot = np.exp(1j * phi)[:, None, None]                                # [N, 1, 1]
        for c in src.channels:
            p = 0.0 if src.unpolarized else src.pol_frac
            jv = np.sqrt(p) * jones(src.theta, src.chi)[None, :] * np.ones((T, 1))
            if p < 1.0:
                u = _cn(rng, (T, 2)).astype(np.complex128)
                u /= np.linalg.norm(u, axis=1, keepdims=True)                # random unit 2-vector
                jv = jv + np.sqrt(1.0 - p) * u
            sig = A * (g * tone)[:, None] * jv                               # [T, 2]
            e[:, c] += (rot * sig[None]).astype(np.complex64)
    return e


def rfi_truth(scene: Scene) -> np.ndarray:
    """Boolean [C][T]: True where any RFI source is on (ground truth for detection studies)."""
    truth = np.zeros((scene.n_channels, scene.n_samples), bool)
    for src in list(scene.rfi) + list(scene.post_rfi):
        g = np.ones(scene.n_samples, bool) if src.envelope is None else src.envelope > 0
        for c in src.channels:
            truth[c] |= g
    return truth


def correlate(e: np.ndarray, baselines=None) -> np.ndarray:
    """Visibilities vis[B][C][T][4] complex64 from voltages e[N][C][T][2].

    Polarisation order (xx, xy, yx, yy): V_pq = e_p e_q^H, so xy = x_p conj(y_q).
    ``baselines`` optionally restricts the output to a subset of baseline indices.
    """
    p, q = baseline_pairs(e.shape[0])
    if baselines is not None:
        p, q = p[baselines], q[baselines]
    ep = e[p]                                   # [B, C, T, 2]
    eq = np.conj(e[q])
    out = ep[..., :, None] * eq[..., None, :]   # [B, C, T, 2, 2]
    out = out.reshape(out.shape[:-2] + (4,)).astype(np.complex64)
    _hermitian_autos(out, p == q)
    return out


def _hermitian_autos(out, is_auto):
    """Autocorrelations are Hermitian: xx, yy real and yx = conj(xy), exactly, as a
    correlator writes them (a plain complex product can differ by one rounding)."""
    if not np.any(is_auto):
        return
    a = out[is_auto]
    a[..., 0] = a[..., 0].real
    a[..., 3] = a[..., 3].real
    a[..., 2] = np.conj(a[..., 1])
    out[is_auto] = a


def correlate_scene(scene: Scene, e: np.ndarray) -> np.ndarray:
    """Visibilities of a scene: voltage products, then its post-correlation RFI sources."""
    vis = correlate(e)
    if not scene.post_rfi:
        return vis
    rng = np.random.default_rng(scene.seed + 7_000_003)
    p, q = baseline_pairs(scene.n_stations)
    for src in scene.post_rfi:
        A2 = inr_to_amplitude(src.inr_db) ** 2
        j = jones(src.theta, src.chi)
        coh = src.pol_frac * np.outer(j, j.conj()) + (1.0 - src.pol_frac) * 0.5 * np.eye(2)
        coh = np.array([[coh[0, 0].real, coh[0, 1]], [np.conj(coh[0, 1]), coh[1, 1].real]])  # exactly Hermitian
        phi = rng.uniform(0.0, 2 * np.pi, size=scene.n_stations)
        g = np.ones(scene.n_samples) if src.envelope is None else src.envelope
        ph = np.exp(1j * (phi[p] - phi[q]))                                  # [B]
        add = (A2 * ph[:, None, None] * g[None, :, None] * coh.reshape(4)[None, None, :])
        for c in src.channels:
            vis[:, c] += add.astype(np.complex64)
    return vis


def correlate_torch(e_dev, out_dev, fmt: str = "cf32", chunk: int = 64):
    """Same correlation on a torch device, written into a preallocated buffer.

    e_dev  : complex64 tensor [N][C][T][2] on the device
    out_dev: float32 [B][C][T][4][2] (cf32) or float16 [B][C][T][4][2] (cf16) tensor
    The CF16 form is the round-to-nearest-even conversion of the complex64 product.
    """
    import torch
    N = e_dev.shape[0]
    p, q = baseline_pairs(N)
    pt = torch.as_tensor(p, device=e_dev.device)
    qt = torch.as_tensor(q, device=e_dev.device)
    B = p.size
    for b0 in range(0, B, chunk):
        b1 = min(B, b0 + chunk)
        prod = e_dev[pt[b0:b1]].unsqueeze(-1) * e_dev[qt[b0:b1]].conj().unsqueeze(-2)
        prod = prod.reshape(prod.shape[:-2] + (4,))
        auto = torch.as_tensor(p[b0:b1] == q[b0:b1], device=e_dev.device)
        if bool(auto.any()):
            a = prod[auto]
            a[..., 0] = a[..., 0].real.to(a.dtype)
            a[..., 3] = a[..., 3].real.to(a.dtype)
            a[..., 2] = a[..., 1].conj()
            prod[auto] = a
        prod = torch.view_as_real(prod)
        if fmt == "cf16":
            out_dev[b0:b1].copy_(prod.to(torch.float16))
        else:
            out_dev[b0:b1].copy_(prod)
    return out_dev


def device_voltages(scene: Scene, device, seed_offset: int = 0):
    """Station voltages e[N][C][T][2] (complex64) drawn directly on a torch device.

    Same model as ``make_voltages`` (receiver noise, common sky, voltage-level RFI)
    but with torch's device generator seeded from the scene, for arrays too large to
    draw on the host quickly.  Not bit-identical to ``make_voltages``.
    """
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(scene.seed) * 7919 + seed_offset)
    N, C, T = scene.n_stations, scene.n_channels, scene.n_samples
    std = float(np.sqrt(0.5))
    e = torch.complex(torch.randn((N, C, T, 2), generator=g, device=device) * std,
                      torch.randn((N, C, T, 2), generator=g, device=device) * std)
    s = torch.complex(torch.randn((C, T, 2), generator=g, device=device) * std,
                      torch.randn((C, T, 2), generator=g, device=device) * std)
    e.mul_(float(np.sqrt(1.0 - scene.rho))).add_(s.unsqueeze(0), alpha=float(np.sqrt(scene.rho)))
    rng = np.random.default_rng(scene.seed + seed_offset)
    t = np.arange(T)
    for src in scene.rfi:
        A = inr_to_amplitude(src.inr_db)
        env = np.ones(T) if src.envelope is None else src.envelope
        sig = A * (env * np.exp(2j * np.pi * src.f0 * t))[:, None] * jones(src.theta, src.chi)[None, :]
        rot = np.exp(1j * rng.uniform(0.0, 2 * np.pi, size=N))[:, None, None]
        add = torch.from_numpy((rot * sig[None]).astype(np.complex64)).to(device)   # [N, T, 2]
        for c in src.channels:
            e[:, c] += add
    return e


def to_cf16(vis: np.ndarray) -> np.ndarray:
    """complex64 [..., 4] -> float16 [..., 4, 2] (re, im), round to nearest even."""
    return np.ascontiguousarray(vis).view(np.float32).reshape(vis.shape + (2,)).astype(np.float16)


# --------------------------------------------------------------------------- named workloads

def scene_plain(seed: int = 0) -> Scene:
    """Plain CPU-sized case: 4 stations (10 baselines), 16 channels, 256 samples.

    A fully polarised pulsed sinusoid in channels 3 and 11: period 80 samples with
    8 on (10 % duty), random phase, in-pulse INR 10 dB, random polarisation.
    """
    rng = np.random.default_rng(seed + 1_000_003)
    T = 256
    theta = rng.uniform(0, np.pi)
    chi = rng.uniform(-np.pi / 4, np.pi / 4)
    env = pulse_train(T, 80, 8, int(rng.integers(0, 80)))
    return Scene(4, 16, T, seed, rho=0.1,
                 rfi=[Rfi([3, 11], 10.0, theta, chi, env, f0=0.05)])


def scene_fp32_baseline(seed: int = 1, n_stations: int = 48, n_channels: int = 64,
                        n_samples: int = 3072) -> Scene:
    """One 1 s integration of a 48-station array: 64 channels x 3072 samples.

    RFI in round(5 %) of the channels, one source each: random polarisation
    (theta ~ U[0, pi), chi ~ U[-pi/4, pi/4]), one pulse train with duty cycle
    U[1, 20] %, in-pulse INR U[0, 20] dB.
    """
    rng = np.random.default_rng(seed + 2_000_003)
    T = n_samples
    n_rfi = max(1, int(round(0.05 * n_channels)))
    chans = rng.choice(n_channels, size=n_rfi, replace=False)
    srcs = []
    for c in chans:
        duty = rng.uniform(0.01, 0.20)
        period = int(rng.integers(50, 500))
        on = max(1, int(round(duty * period)))
        env = pulse_train(T, period, on, int(rng.integers(0, period)))
        srcs.append(Rfi([int(c)], float(rng.uniform(0, 20)), float(rng.uniform(0, np.pi)),
                        float(rng.uniform(-np.pi / 4, np.pi / 4)), env,
                        f0=float(rng.uniform(-0.5, 0.5))))
    return Scene(n_stations, n_channels, T, seed, rho=0.1, rfi=srcs)


def scene_mixed(seed: int = 3, n_stations: int = 64, n_channels: int = 256,
                n_samples: int = 3072) -> Scene:
    """Larger mixed-RFI case: continuous CW, 1 %-duty radar pulse trains,
    broadband impulsive bursts, and a 20 %-polarised Gaussian sky."""
    rng = np.random.default_rng(seed + 3_000_003)
    T, C = n_samples, n_channels
    srcs = []
    n_cw = max(1, int(round(0.02 * C)))
    n_radar = max(1, int(round(0.02 * C)))
    chans = rng.choice(C, size=n_cw + n_radar, replace=False)
    for c in chans[:n_cw]:                                   # continuous narrowband CW
        srcs.append(Rfi([int(c)], float(rng.uniform(0, 20)), float(rng.uniform(0, np.pi)),
                        float(rng.uniform(-np.pi / 4, np.pi / 4)), None,
                        f0=float(rng.uniform(-0.5, 0.5))))
    for c in chans[n_cw:]:                                   # radar: 3 on / 297 off
        env = pulse_train(T, 300, 3, int(rng.integers(0, 300)))
        srcs.append(Rfi([int(c)], float(rng.uniform(10, 20)), float(rng.uniform(0, np.pi)),
                        float(rng.uniform(-np.pi / 4, np.pi / 4)), env,
                        f0=float(rng.uniform(-0.5, 0.5))))
    n_burst = 3                                              # broadband bursts, 1-4 samples
    starts = rng.integers(0, T - 4, size=n_burst)
    lens = rng.integers(1, 5, size=n_burst)
    srcs.append(Rfi(list(range(C)), 10.0, float(rng.uniform(0, np.pi)),
                    float(rng.uniform(-np.pi / 4, np.pi / 4)),
                    burst_envelope(T, starts, lens), f0=0.0))
    return Scene(n_stations, C, T, seed, rho=0.1, sky_pol_frac=0.2, rfi=srcs)


def scene_null(n_stations: int, n_channels: int, n_samples: int, seed: int,
               rho: float = 0.1) -> Scene:
    """RFI-free realisation (used to calibrate d and the thresholds)."""
    return Scene(n_stations, n_channels, n_samples, seed, rho=rho)


def scene_serving_array(n_stations: int, n_channels: int, seed: int,
                        n_samples: int = 3072) -> Scene:
    """One array of the serving mix: like the FP32 baseline scene at another size."""
    return scene_fp32_baseline(seed, n_stations, n_channels, n_samples)


def serving_mix(seed: int = 4, n_arrays: int = 16, max_total_bytes: float = 96e9,
                n_samples: int = 3072):
    """The serving workload: arrays of 12, 24, 48 or 64 stations with 16-256 channels,
    drawn per seed; redrawn (deterministically) until their complex-half inputs fit
    ``max_total_bytes`` together.  Returns a list of scenes."""
    rng = np.random.default_rng(seed + 5_000_003)
    while True:
        Ns = rng.choice([12, 24, 48, 64], size=n_arrays)
        Cs = rng.choice([16, 32, 64, 128, 256], size=n_arrays)
        total = sum(n_baselines(int(n)) * int(c) * n_samples * 16 for n, c in zip(Ns, Cs))
        if total <= max_total_bytes:
            break
    return [scene_serving_array(int(n), int(c), seed * 100 + i, n_samples) for i, (n, c) in enumerate(zip(Ns, Cs))]
