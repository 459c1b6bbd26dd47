"""Seeded synthetic inputs shaped like the paper's workloads.

This module draws inputs only: k-space trajectories, sample times, coil
sensitivity maps, off-resonance maps, complex phantoms, dynamic frame series,
unit complex Gaussian noise and serving-request traces.  It holds none of the
reconstruction arithmetic: it never forms an encoding matrix, never applies the
forward model and never scales noise to a signal level.  Both the FP64 oracle
and the device path consume what it returns.

Conventions (paper Sec. 2, Eq. 2 and Sec. 3.3):
  * k is in cycles per field of view, inside [-n/2, n/2) per axis.
  * voxel centre r_v = ((ix - nx/2)/nx, (iy - ny/2)/ny) in FOV units.
  * voxel index v = iy*nx + ix; unknown index n = s*V + v (species-major).
  * data row index m = c*K + i (coil-major).
  * sample time t_i = i*dwell (seconds), time origin at the first sample.

Seeds follow numpy.random.default_rng(1000*wid + j), where wid numbers the
workload (1 radial 32x32, 2 spiral 64x64 with 8 coils, 3 spiral 96x96 with 16
coils, 4 five-species 32x32, 5 serving trace, 6 spiral 128x128 with 8 coils)
and j = 1 phantom, 2 coils, 3 B0, 4 noise, 5 dynamics, 6 serving trace.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

GOLDEN_ANGLE = math.pi * (math.sqrt(5.0) - 1.0) / 2.0  # ~111.246 degrees

SEED_PHANTOM, SEED_COILS, SEED_B0, SEED_NOISE, SEED_DYN, SEED_TRACE = 1, 2, 3, 4, 5, 6


def rng_for(wid: int, j: int) -> np.random.Generator:
    return np.random.default_rng(1000 * wid + j)


@dataclasses.dataclass
class Encoding:
    """Everything that defines one encoding matrix (no matrix is formed here).

    k          [K, 2] float64, cycles/FOV
    t          [K] float64 seconds, or None (only needed with species or B0)
    coil       [C, V] complex128 sensitivities, or None (single unit coil)
    b0_hz      [V] float64 off-resonance in Hz, or None
    species_hz [S] float64 species frequencies in Hz, or None (=> one species at 0 Hz)
    voxels     [V] int32 ascending grid indices iy*nx + ix of the unknown voxels (a
               mask), or None (every grid voxel is an unknown); coil and b0_hz
               still cover the whole grid
    """

    nx: int
    ny: int
    k: np.ndarray
    t: Optional[np.ndarray] = None
    coil: Optional[np.ndarray] = None
    b0_hz: Optional[np.ndarray] = None
    species_hz: Optional[np.ndarray] = None
    voxels: Optional[np.ndarray] = None

    @property
    def V(self) -> int:
        return self.nx * self.ny if self.voxels is None else int(len(self.voxels))

    @property
    def S(self) -> int:
        return 1 if self.species_hz is None else int(len(self.species_hz))

    @property
    def N(self) -> int:
        return self.S * self.V

    @property
    def K(self) -> int:
        return int(self.k.shape[0])

    @property
    def C(self) -> int:
        return 1 if self.coil is None else int(self.coil.shape[0])

    @property
    def M(self) -> int:
        return self.C * self.K

    def __post_init__(self):
        self.k = np.ascontiguousarray(self.k, dtype=np.float64)
        assert self.k.ndim == 2 and self.k.shape[1] == 2
        if self.t is not None:
            self.t = np.ascontiguousarray(self.t, dtype=np.float64)
            assert self.t.shape == (self.K,)
        if self.coil is not None:
            self.coil = np.ascontiguousarray(self.coil, dtype=np.complex128)
            assert self.coil.shape[1] == self.nx * self.ny
        if self.b0_hz is not None:
            self.b0_hz = np.ascontiguousarray(self.b0_hz, dtype=np.float64)
            assert self.b0_hz.shape == (self.nx * self.ny,)
        if self.voxels is not None:
            self.voxels = np.ascontiguousarray(self.voxels, dtype=np.int32)
            assert self.voxels.ndim == 1 and len(self.voxels) >= 1
            assert np.all(np.diff(self.voxels) > 0)
            assert self.voxels[0] >= 0 and self.voxels[-1] < self.nx * self.ny
        if self.species_hz is not None:
            self.species_hz = np.ascontiguousarray(self.species_hz, dtype=np.float64)
        if (self.S > 1 or self.b0_hz is not None) and self.t is None:
            raise ValueError("sample times are required with several species or a B0 map")


# ----------------------------------------------------------------------------
# grids and trajectories
# ----------------------------------------------------------------------------

def voxel_centres(nx: int, ny: int):
    """Voxel centres in FOV units, each [V], v = iy*nx + ix."""
    ix = np.arange(nx, dtype=np.float64)
    iy = np.arange(ny, dtype=np.float64)
    x = (ix - nx / 2.0) / nx
    y = (iy - ny / 2.0) / ny
    X, Y = np.meshgrid(x, y)  # [ny, nx]
    return X.ravel(), Y.ravel()


def cartesian_full(nx: int, ny: int) -> np.ndarray:
    """Fully sampled Cartesian grid: integer k in [-n/2, n/2), ky-major order."""
    kx = np.arange(nx, dtype=np.float64) - nx // 2
    ky = np.arange(ny, dtype=np.float64) - ny // 2
    KX, KY = np.meshgrid(kx, ky)
    return np.stack([KX.ravel(), KY.ravel()], axis=1)


def golden_radial(n: int, spokes: int, samples: int) -> np.ndarray:
    """Golden-angle radial spokes; spoke j at angle j*pi*(sqrt5-1)/2, samples
    k = (-n/2 + n*s/samples)*(cos, sin), s = 0..samples-1."""
    j = np.arange(spokes, dtype=np.float64)
    th = j * GOLDEN_ANGLE
    s = np.arange(samples, dtype=np.float64)
    rho = -n / 2.0 + n * s / samples
    kx = rho[None, :] * np.cos(th)[:, None]
    ky = rho[None, :] * np.sin(th)[:, None]
    return np.stack([kx.ravel(), ky.ravel()], axis=1)


def vd_spiral(n: int, K: int, turns: Optional[float] = None) -> np.ndarray:
    """Single-interleave variable-density spiral: u=(i+0.5)/K, rho=kmax*u^1.5,
    theta = 2*pi*turns*u with kmax = n/2 and turns = n/4 by default."""
    if turns is None:
        turns = n / 4.0
    u = (np.arange(K, dtype=np.float64) + 0.5) / K
    rho = (n / 2.0) * u ** 1.5
    th = 2.0 * math.pi * turns * u
    return np.stack([rho * np.cos(th), rho * np.sin(th)], axis=1)


def sample_times(K: int, dwell: float = 4e-6) -> np.ndarray:
    return np.arange(K, dtype=np.float64) * dwell


# ----------------------------------------------------------------------------
# voxel masks
# ----------------------------------------------------------------------------

def circular_mask(nx: int, ny: int, diameter: float = 1.0) -> np.ndarray:
    """Grid indices iy*nx + ix of the voxels whose centres lie inside a circle
    of `diameter` (in FOV units, 1 = the side of the image) centred on the
    field of view; ascending int32."""
    X, Y = voxel_centres(nx, ny)
    return np.flatnonzero(X ** 2 + Y ** 2 <= (diameter / 2.0) ** 2).astype(np.int32)


def threshold_mask(image: np.ndarray, fraction: float) -> np.ndarray:
    """Grid indices of the voxels whose magnitude is at least `fraction` of the
    image's maximum magnitude; ascending int32."""
    a = np.abs(np.asarray(image).ravel())
    return np.flatnonzero(a >= fraction * a.max()).astype(np.int32)


# ----------------------------------------------------------------------------
# maps and phantoms
# ----------------------------------------------------------------------------

def coil_maps(nx: int, ny: int, C: int, rng: np.random.Generator) -> np.ndarray:
    """C smooth Gaussian-magnitude bumps around a circle of radius 0.45 FOV,
    each with a constant phase and a linear phase ramp (|g| <= 0.5 cyc/FOV)."""
    X, Y = voxel_centres(nx, ny)
    out = np.empty((C, nx * ny), dtype=np.complex128)
    for c in range(C):
        ang = 2.0 * math.pi * c / C + rng.uniform(-0.1, 0.1)
        cx, cy = 0.45 * math.cos(ang), 0.45 * math.sin(ang)
        w = rng.uniform(0.25, 0.4)
        phi = rng.uniform(-math.pi, math.pi)
        gmag = rng.uniform(0.0, 0.5)
        gang = rng.uniform(0.0, 2.0 * math.pi)
        gx, gy = gmag * math.cos(gang), gmag * math.sin(gang)
        mag = np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2.0 * w * w))
        out[c] = mag * np.exp(1j * (phi + 2.0 * math.pi * (gx * X + gy * Y)))
    return out


def b0_map(nx: int, ny: int, rng: np.random.Generator, max_hz: float = 30.0) -> np.ndarray:
    """Four seeded Gaussian bumps plus a linear term, rescaled so max|B0| = max_hz."""
    X, Y = voxel_centres(nx, ny)
    f = rng.uniform(-1, 1) * X + rng.uniform(-1, 1) * Y
    for _ in range(4):
        cx, cy = rng.uniform(-0.35, 0.35, size=2)
        w = rng.uniform(0.08, 0.25)
        a = rng.uniform(-1, 1)
        f = f + a * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (2 * w * w))
    f = f * (max_hz / np.max(np.abs(f)))
    return f


def ellipse_phantom(nx: int, ny: int, rng: np.random.Generator, count: int = 10) -> np.ndarray:
    """Sum of `count` random ellipses with complex amplitudes; [V] complex128."""
    X, Y = voxel_centres(nx, ny)
    img = np.zeros(nx * ny, dtype=np.complex128)
    for _ in range(count):
        cx, cy = rng.uniform(-0.3, 0.3, size=2)
        a, b = rng.uniform(0.05, 0.35, size=2)
        th = rng.uniform(0.0, math.pi)
        amp = rng.uniform(0.2, 1.0) * np.exp(1j * rng.uniform(-math.pi, math.pi))
        dx, dy = X - cx, Y - cy
        u = dx * math.cos(th) + dy * math.sin(th)
        w = -dx * math.sin(th) + dy * math.cos(th)
        img[(u / a) ** 2 + (w / b) ** 2 <= 1.0] += amp
    return img


def dynamic_frames(x: np.ndarray, F: int, rng: np.random.Generator) -> np.ndarray:
    """x_f(v) = x(v)*(1 + 0.05*sin(2*pi*nu_v*f/F + phi_v)), nu_v in {1..5}; [F, V]."""
    V = x.shape[0]
    nu = rng.integers(1, 6, size=V).astype(np.float64)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=V)
    f = np.arange(F, dtype=np.float64)[:, None]
    return x[None, :] * (1.0 + 0.05 * np.sin(2.0 * math.pi * nu[None, :] * f / F + phi[None, :]))


def unit_complex_noise(shape, rng: np.random.Generator) -> np.ndarray:
    """Complex Gaussian with E|n|^2 = 1 (independent real/imag parts of variance 1/2)."""
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) * math.sqrt(0.5)


def random_frames(shape, rng: np.random.Generator) -> np.ndarray:
    """Seeded complex Gaussian frames (value-independent timing work)."""
    return unit_complex_noise(shape, rng)


# ----------------------------------------------------------------------------
# the workloads
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Workload:
    name: str
    enc: Encoding
    rel_lambda: float
    images: np.ndarray          # [F, N] complex128 ground truth
    noise: np.ndarray           # [F, M] unit complex Gaussian (scaled by the user)
    snr_db: float = 30.0


def radial_32x32_c1(F: int = 1) -> Workload:
    """32x32 single coil, 16 golden-angle spokes x 128 samples (M=2048), FP64."""
    wid = 1
    k = golden_radial(32, 16, 128)
    enc = Encoding(32, 32, k)
    x = ellipse_phantom(32, 32, rng_for(wid, SEED_PHANTOM))
    imgs = np.repeat(x[None, :], F, axis=0) if F > 1 else x[None, :]
    noise = unit_complex_noise((F, enc.M), rng_for(wid, SEED_NOISE))
    return Workload("fp64_32x32_radial16x128_c1", enc, 1e-3, imgs, noise)


def _spiral_multicoil(wid: int, n: int, C: int, K: int, F: int, name: str,
                      rel: float = 1e-3) -> Workload:
    k = vd_spiral(n, K)
    coil = coil_maps(n, n, C, rng_for(wid, SEED_COILS))
    enc = Encoding(n, n, k, coil=coil)
    x = ellipse_phantom(n, n, rng_for(wid, SEED_PHANTOM))
    imgs = dynamic_frames(x, F, rng_for(wid, SEED_DYN))
    noise = unit_complex_noise((F, enc.M), rng_for(wid, SEED_NOISE))
    return Workload(name, enc, rel, imgs, noise)


def spiral_64x64_c8(F: int = 1000) -> Workload:
    """64x64 (N=4096), 8 coils, 4096-sample VD spiral per coil (M=32768), F frames."""
    return _spiral_multicoil(2, 64, 8, 4096, F, "64x64_c8_spiral4096_f1000")


def spiral_96x96_c16(F: int = 500, rel: float = 1e-3) -> Workload:
    """96x96 (N=9216), 16 coils, 8192-sample spiral per coil (M=131072), F frames."""
    return _spiral_multicoil(3, 96, 16, 8192, F, "96x96_c16_spiral8192_f500", rel)


def spiral_128x128_c8(F: int = 1000) -> Workload:
    """128x128 (N=16384), 8 coils, VD spiral of 2N = 32768 samples per coil
    (M=262144), F frames: the largest shape of the serving mix (2N samples per
    coil) at its middle coil count.  Frame noise is left to the caller (F x M
    is 4 GB in complex128); `noise` here is empty."""
    wid, n, C, K = 6, 128, 8, 2 * 128 * 128
    k = vd_spiral(n, K)
    coil = coil_maps(n, n, C, rng_for(wid, SEED_COILS))
    enc = Encoding(n, n, k, coil=coil)
    x = ellipse_phantom(n, n, rng_for(wid, SEED_PHANTOM))
    imgs = dynamic_frames(x, F, rng_for(wid, SEED_DYN))
    return Workload(f"128x128_c8_spiral{K}_f{F}", enc, 1e-3, imgs, np.zeros((0, enc.M), np.complex128))


def species5_32x32_c8(F: int = 200) -> Workload:
    """5 species {0,120,260,390,520} Hz x 32x32 (N=5120), 8 coils, 6144-sample
    single-shot spiral at 4 us dwell (M=49152), B0 within +-30 Hz, F frames."""
    wid, n, C, K = 4, 32, 8, 6144
    k = vd_spiral(n, K, turns=8.0)
    t = sample_times(K, 4e-6)
    coil = coil_maps(n, n, C, rng_for(wid, SEED_COILS))
    b0 = b0_map(n, n, rng_for(wid, SEED_B0))
    species = np.array([0.0, 120.0, 260.0, 390.0, 520.0])
    enc = Encoding(n, n, k, t=t, coil=coil, b0_hz=b0, species_hz=species)
    rp = rng_for(wid, SEED_PHANTOM)
    maps = [ellipse_phantom(n, n, rp) for _ in range(len(species))]
    rd = rng_for(wid, SEED_DYN)
    kappa = rd.uniform(0.005, 0.03, size=len(species))
    f = np.arange(F, dtype=np.float64)
    imgs = np.concatenate([np.exp(-kappa[s] * f)[:, None] * maps[s][None, :]
                           for s in range(len(species))], axis=1)
    noise = unit_complex_noise((F, enc.M), rng_for(wid, SEED_NOISE))
    return Workload("species5_32x32_c8_spiral6144_b0_f200", enc, 1e-3, imgs, noise)


def small_case(seed: int, nx: int, ny: int, C: int, K: int, F: int, species=None,
               b0: bool = False, traj: str = "spiral") -> Workload:
    """Reduced-size case of the same structure, for parity at oracle-friendly sizes."""
    rng = np.random.default_rng(seed)
    n = max(nx, ny)
    if traj == "spiral":
        k = vd_spiral(n, K)
    elif traj == "radial":
        spokes = max(1, K // (2 * n))
        k = golden_radial(n, spokes, K // spokes)[:K]
        if k.shape[0] < K:
            k = np.concatenate([k, vd_spiral(n, K - k.shape[0])], axis=0)
    else:
        raise ValueError(traj)
    need_t = b0 or (species is not None and len(species) > 1)
    t = sample_times(K, 4e-6) if need_t else None
    coil = coil_maps(nx, ny, C, rng) if C > 1 else None
    b0map = b0_map(nx, ny, rng) if b0 else None
    sp = None if species is None else np.asarray(species, dtype=np.float64)
    enc = Encoding(nx, ny, k, t=t, coil=coil, b0_hz=b0map, species_hz=sp)
    S = enc.S
    base = np.concatenate([ellipse_phantom(nx, ny, rng) for _ in range(S)])
    imgs = dynamic_frames(base, F, rng)
    noise = unit_complex_noise((F, enc.M), rng)
    return Workload(f"small_{nx}x{ny}_c{C}_k{K}_s{S}_b0{int(b0)}_f{F}", enc, 1e-3, imgs, noise)


# ----------------------------------------------------------------------------
# serving trace
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Request:
    rid: int
    arrival_s: float
    n: int              # image side; N = n*n
    coils: int
    enc_id: int         # which encoding this request reconstructs with
    new_build: bool     # True if this enc_id is issued for the first time here
    frames: int


def serving_trace(rate_per_s: float = 4.0, duration_s: float = 120.0, wid: int = 5,
                  sides=(32, 64, 96, 128), probs=(0.4, 0.3, 0.2, 0.1),
                  coil_choices=(1, 8, 16), reuse: float = 0.7,
                  frames_range=(50, 2000)) -> List[Request]:
    """Poisson arrivals; each request draws an image side and coil count for a
    new encoding (30%) or reuses one issued earlier (70%)."""
    rng = rng_for(wid, SEED_TRACE)
    t = 0.0
    out: List[Request] = []
    encs: List[tuple] = []
    rid = 0
    while True:
        t += rng.exponential(1.0 / rate_per_s)
        if t > duration_s:
            break
        frames = int(rng.integers(frames_range[0], frames_range[1] + 1))
        if encs and rng.uniform() < reuse:
            eid = int(rng.integers(0, len(encs)))
            n, c = encs[eid]
            out.append(Request(rid, t, n, c, eid, False, frames))
        else:
            n = int(rng.choice(sides, p=probs))
            c = int(rng.choice(coil_choices))
            encs.append((n, c))
            out.append(Request(rid, t, n, c, len(encs) - 1, True, frames))
        rid += 1
    return out


def serving_encoding(n: int, coils: int, enc_id: int, wid: int = 5) -> Encoding:
    """Encoding of a serving request: n x n grid, spiral of 2*n*n samples per coil."""
    K = 2 * n * n
    k = vd_spiral(n, K)
    rng = np.random.default_rng(1000 * wid + 100 + enc_id)
    coil = coil_maps(n, n, coils, rng) if coils > 1 else None
    return Encoding(n, n, k, coil=coil)
