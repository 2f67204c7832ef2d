"""Seeded synthetic inputs shared by the oracle and the GPU path.

This module holds only input generation: workload shapes, random scatterer
profiles, their rasterisation to a pixel grid, antenna placement, and the raw
random draws (noise samples, angle jitter).  It contains none of the inversion
method's arithmetic, so either side may import it without sharing solver code.

The paper evaluates on the "Austria" profile and on the Fresnel "FoamDielExt" /
"FoamDielInt" measurements (Sec. 4 and Sec. 5); neither is available, so random
disc / ellipse / ring profiles with the paper's grid, array and contrast ranges
stand in for them.

Every draw uses ``numpy.random.Generator(PCG64(seed))``; the three independent
streams of one seed (profile, noise, jitter) come from ``SeedSequence(seed).spawn``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

C0 = 299_792_458.0  # speed of light in vacuum, m/s


@dataclasses.dataclass(frozen=True)
class Workload:
    """Shape of one reconstruction problem.

    Lengths are in wavelengths of the base frequency; ``freq_hz`` is the base
    frequency (the paper uses 400 MHz over a 1.5 m = 2 wavelength domain).
    """
    name: str
    M: int                    # inversion grid side (pixels)
    side_wl: float            # domain side, wavelengths
    n_tx: int
    n_rx: int
    radius_wl: float          # antenna circle radius, wavelengths
    K: int                    # Fourier truncation per axis (odd: centred set)
    M_fine: int               # grid used to synthesise the measured fields
    noise: float              # relative complex AWGN level (nu)
    jitter_deg: float         # uniform antenna-angle jitter half width
    n_iter: int               # Adam iterations of a reconstruction
    freq_hz: float = 400e6
    freq_mult: tuple = (1.0,)
    precision: str = "fp32"
    profile: str = "cfg2"     # recipe name for draw_profile

    @property
    def wavelength(self) -> float:
        return C0 / self.freq_hz

    @property
    def side(self) -> float:
        return self.side_wl * self.wavelength

    @property
    def radius(self) -> float:
        return self.radius_wl * self.wavelength


WORKLOADS = {
    # 32x32 over 2 lambda, 16 Tx / 32 Rx on a 3 lambda circle, K = 9, FP64,
    # two discs eps_r in [1.5, 2.5], data from a 64x64 MoM plus 5 % noise.
    "cfg1": Workload("cfg1", 32, 2.0, 16, 32, 3.0, 9, 64, 0.05, 0.0, 100,
                     precision="fp64", profile="cfg1"),
    # 64x64 over 2 lambda, 32 / 32 on a 3 lambda circle, K = 15, FP32,
    # 1-3 discs / ellipses eps_r in [2, 4], data from a 128x128 MoM plus 10 %
    # noise and +-2 degree antenna-angle jitter.
    "cfg2": Workload("cfg2", 64, 2.0, 32, 32, 3.0, 15, 128, 0.10, 2.0, 1000,
                     precision="fp32", profile="cfg2"),
    # Paper-shaped context run: 64x64, 36 / 36 antennas on a 20 lambda circle.
    "paper": Workload("paper", 64, 2.0, 36, 36, 20.0, 15, 128, 0.0, 0.0, 1000,
                      precision="fp32", profile="cfg2"),
    # Large multi-frequency: 256x256 over 8 lambda, 64 / 64 on a 10 lambda
    # circle, four frequencies, K = 41.
    "cfg5": Workload("cfg5", 256, 8.0, 64, 64, 10.0, 41, 512, 0.05, 0.0, 500,
                     freq_mult=(1.0, 1.5, 2.0, 2.5), precision="fp32",
                     profile="cfg5"),
}


@dataclasses.dataclass(frozen=True)
class Shape:
    kind: str        # "ellipse" (a disc when a == b) or "ring"
    cx: float        # centre, metres
    cy: float
    a: float         # semi-axis along the rotated x axis (ring: outer radius)
    b: float         # semi-axis along the rotated y axis (ring: inner radius)
    theta: float     # rotation, radians
    eps_r: complex

    @property
    def bound_radius(self) -> float:
        return max(self.a, self.b) if self.kind == "ellipse" else self.a

    def contains(self, x: np.ndarray, y: np.ndarray) -> np.ndarray:
        dx = x - self.cx
        dy = y - self.cy
        if self.kind == "ring":
            r2 = dx * dx + dy * dy
            return (r2 <= self.a * self.a) & (r2 >= self.b * self.b)
        c, s = math.cos(self.theta), math.sin(self.theta)
        u = c * dx + s * dy
        v = -s * dx + c * dy
        return (u / self.a) ** 2 + (v / self.b) ** 2 <= 1.0


def streams(seed: int):
    """Three independent PCG64 generators (profile, noise, jitter) of a seed."""
    ss = np.random.SeedSequence(int(seed))
    return [np.random.Generator(np.random.PCG64(s)) for s in ss.spawn(3)]


def _place(rng, side: float, radius: float, placed: List[Shape],
           margin: float) -> Optional[tuple]:
    half = side / 2.0 - radius - margin
    if half <= 0:
        return None
    for _ in range(1000):
        cx, cy = rng.uniform(-half, half, size=2)
        ok = all(math.hypot(cx - s.cx, cy - s.cy) > radius + s.bound_radius + margin
                 for s in placed)
        if ok:
            return float(cx), float(cy)
    return None


def draw_profile(workload: Workload, seed: int) -> List[Shape]:
    """Random non-overlapping scatterers fully inside the domain.

    cfg1: two discs, radius U[0.2, 0.4] lambda, eps_r U[1.5, 2.5].
    cfg2: 1-3 objects, disc or ellipse with probability 1/2, semi-axes
          U[0.2, 0.4] lambda, orientation U[0, pi), eps_r U[2, 4].
    cfg5: 5-10 discs or rings (outer U[0.2, 0.6] lambda, width >= 0.1 lambda),
          eps_r U[1.5, 3.5].
    Non-overlap and containment use each shape's bounding circle.
    """
    rng = streams(seed)[0]
    lam = workload.wavelength
    side = workload.side
    margin = 0.02 * lam
    recipe = workload.profile
    for _attempt in range(100):
        shapes: List[Shape] = []
        if recipe == "cfg1":
            n_obj = 2
        elif recipe == "cfg2":
            n_obj = int(rng.integers(1, 4))
        elif recipe == "cfg5":
            n_obj = int(rng.integers(5, 11))
        else:
            raise ValueError(recipe)
        failed = False
        for _ in range(n_obj):
            if recipe == "cfg1":
                r = rng.uniform(0.2, 0.4) * lam
                eps = rng.uniform(1.5, 2.5)
                shp = ("ellipse", r, r, 0.0, eps)
            elif recipe == "cfg2":
                is_ellipse = rng.uniform() < 0.5
                a = rng.uniform(0.2, 0.4) * lam
                b = rng.uniform(0.2, 0.4) * lam if is_ellipse else a
                th = rng.uniform(0.0, math.pi) if is_ellipse else 0.0
                eps = rng.uniform(2.0, 4.0)
                shp = ("ellipse", a, b, th, eps)
            else:
                eps = rng.uniform(1.5, 3.5)
                if rng.uniform() < 0.5:
                    r = rng.uniform(0.2, 0.6) * lam
                    shp = ("ellipse", r, r, 0.0, eps)
                else:
                    ro = rng.uniform(0.3, 0.6) * lam
                    ri = rng.uniform(0.2 * lam, ro - 0.1 * lam)
                    shp = ("ring", ro, ri, 0.0, eps)
            kind, a, b, th, eps = shp
            bound = max(a, b) if kind == "ellipse" else a
            pos = _place(rng, side, bound, shapes, margin)
            if pos is None:
                failed = True
                break
            shapes.append(Shape(kind, pos[0], pos[1], a, b, th, complex(eps)))
        if not failed:
            return shapes
    raise RuntimeError("could not place scatterers")


def rasterize(shapes: Sequence[Shape], M: int, side: float, cx: float = 0.0,
              cy: float = 0.0, sub: int = 8) -> np.ndarray:
    """Relative permittivity on an M x M grid by area fraction.

    Each pixel is sampled at sub x sub interior points; eps = 1 + sum over
    shapes of (eps_s - 1) * covered fraction.  Row i runs along y, column j
    along x, pixel centres at -side/2 + (index + 1/2) h.
    """
    h = side / M
    off = (np.arange(sub) + 0.5) / sub * h
    base = -side / 2.0 + np.arange(M) * h
    xs = (cx + base[:, None] + off[None, :]).reshape(-1)   # M*sub
    ys = (cy + base[:, None] + off[None, :]).reshape(-1)
    eps = np.ones((M, M), dtype=np.complex128)
    for s in shapes:
        # only the pixels of the shape's bounding square (plus one) can hold a sample inside it
        r = s.bound_radius
        j0 = max(0, int(math.floor((s.cx - r - cx + side / 2.0) / h)) - 1)
        j1 = min(M, int(math.ceil((s.cx + r - cx + side / 2.0) / h)) + 1)
        i0 = max(0, int(math.floor((s.cy - r - cy + side / 2.0) / h)) - 1)
        i1 = min(M, int(math.ceil((s.cy + r - cy + side / 2.0) / h)) + 1)
        if i0 >= i1 or j0 >= j1:
            continue
        X, Y = np.meshgrid(xs[j0 * sub:j1 * sub], ys[i0 * sub:i1 * sub])
        inside = s.contains(X, Y).astype(np.float64)
        frac = inside.reshape(i1 - i0, sub, j1 - j0, sub).mean(axis=(1, 3))
        eps[i0:i1, j0:j1] += (s.eps_r - 1.0) * frac
    return eps


def uneven_shapes(n: int, seed: int, grids=(32, 48, 64, 96, 128), antennas=(16, 24, 32, 48, 64),
                  truncations=(7, 9, 11, 13, 15, 17, 19, 21)):
    """Per-instance (M, N_i = N_s, K) of an uneven batch, drawn uniformly from the given sets
    (K <= M is kept by redrawing K)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(n):
        M = int(rng.choice(grids))
        a = int(rng.choice(antennas))
        K = int(rng.choice(truncations))
        while K > M:
            K = int(rng.choice(truncations))
        out.append((M, a, K))
    return out


def antenna_positions(n: int, radius: float, cx: float = 0.0, cy: float = 0.0,
                      angle_offsets: Optional[np.ndarray] = None) -> np.ndarray:
    """n antennas equally spaced on a circle, the first at angle 0; [n, 2] (x, y)."""
    ang = 2.0 * math.pi * np.arange(n) / n
    if angle_offsets is not None:
        ang = ang + np.asarray(angle_offsets, dtype=np.float64)
    return np.stack([cx + radius * np.cos(ang), cy + radius * np.sin(ang)], axis=1)


def draw_jitter(seed: int, n_tx: int, n_rx: int, deg: float):
    """Independent U[-deg, deg] angle offsets (radians) for every Tx and Rx."""
    rng = streams(seed)[2]
    d = math.radians(deg)
    return rng.uniform(-d, d, size=n_tx), rng.uniform(-d, d, size=n_rx)


def draw_noise(seed: int, shape) -> tuple:
    """Two independent standard-normal arrays (real and imaginary draws)."""
    rng = streams(seed)[1]
    return rng.standard_normal(shape), rng.standard_normal(shape)


def truth_eps(workload: Workload, seed: int, M: Optional[int] = None) -> np.ndarray:
    """True relative permittivity of a seed's profile on an M x M grid."""
    return rasterize(draw_profile(workload, seed), M or workload.M, workload.side)


def add_noise(esca: np.ndarray, nu: float, n1: np.ndarray, n2: np.ndarray) -> np.ndarray:
    """Complex AWGN of relative level nu (Sec. 4.2 adds AWGN at a stated SNR):
    e + nu * (||e||_F / sqrt(size)) * (n1 + i n2) / sqrt(2), with n1, n2 the
    standard-normal draws of draw_noise, so that ||noise|| is about nu ||e||.
    An SNR in dB maps to nu = 10^(-SNR/20)."""
    scale = nu * np.linalg.norm(esca) / np.sqrt(esca.size)
    return esca + scale * (n1 + 1j * n2) / np.sqrt(2.0)


def fcnn_theta(seed: int, B: int, K: int, H: int, out_scale: float = 0.0) -> np.ndarray:
    """Start weights of the coefficient network (three dense layers 2K^2 -> H -> H -> 2K^2,
    each a block of (in + 1) x out numbers, the last row the bias) for B reconstructions:
    U[-1/sqrt(in), 1/sqrt(in)] for every weight and bias, the output block multiplied by
    out_scale (0: the network starts at alpha_hat = alpha_0).  [B][n_params] float64."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 0x4643])))
    D = 2 * K * K
    shapes = [(D, H), (H, H), (H, D)]
    out = np.empty((B, sum((i + 1) * o for i, o in shapes)))
    for b in range(B):
        parts = []
        for li, (i, o) in enumerate(shapes):
            s = (out_scale if li == 2 else 1.0) / math.sqrt(i)
            parts.append(rng.uniform(-s, s, size=(i + 1) * o))
        out[b] = np.concatenate(parts)
    return out


def draw_position_errors(seed: int, n_tx: int, n_rx: int, sigma_m: float):
    """Antenna position errors: independent N(0, sigma_m^2) offsets of x and y for every Tx
    and Rx (metres), as [n][2] arrays."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), 0x504F53])))
    return rng.normal(0.0, sigma_m, size=(n_tx, 2)), rng.normal(0.0, sigma_m, size=(n_rx, 2))
