"""Seeded synthetic stand-ins for the paper's workloads.

The paper analyses SKA1-Low stations: 256 identical log-periodic elements in a
pseudo-random layout with a minimum spacing of about 1.35 m (Section I, station
layout figure), frequencies 50-350 MHz (Section I), and arrays up to 1500
elements of the same density (Section IV).  Neither the element mesh nor the
layouts survive in the paper, so everything below is synthetic:

* an element is a set of N_m macro basis functions (MBFs), each a cloud of N_s
  point-dipole samples at uniform positions in a 0.5 x 0.5 x 2 m box, oriented
  along x or z with probability 1/2, with circular complex normal amplitudes
  (real and imaginary parts each N(0, 1/2));
* a layout is random sequential addition in a disk (radius R sqrt(u), angle
  2 pi v), rejecting points closer than s_min to an accepted one;
* pattern directions are uniform on the upper hemisphere (theta = acos U,
  phi = 2 pi U).

Only numpy's PCG64 generator is used; no part of the method is computed here.
The sample record layout (8 float64 per sample: x, y, z, ux, uy, uz, a_re, a_im)
is the one the C-ABI documents for elements.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Speed of light in vacuum, m/s.  Used only to choose the harmonic order P of a
# configuration (a recipe parameter), never for any arithmetic of the method.
_C0 = 299_792_458.0

SAMPLE_FIELDS = 8  # x, y, z, ux, uy, uz, a_re, a_im

CONFIG_NAMES = ("small16", "station_sweep", "batched_layouts", "station_110mhz", "large1024")


@dataclass
class Element:
    """One element: n_mbf MBFs of n_samp point-dipole samples each.

    samples has shape (n_mbf, n_samp, 8), float64, C-contiguous:
    position (m) relative to the element reference point, unit orientation,
    complex moment (A m) as (re, im).
    """

    samples: np.ndarray
    wire_radius: float = 0.02

    @property
    def n_mbf(self) -> int:
        return int(self.samples.shape[0])

    @property
    def n_samp(self) -> int:
        return int(self.samples.shape[1])

    def amplitudes(self) -> np.ndarray:
        return self.samples[..., 6] + 1j * self.samples[..., 7]


@dataclass
class Workload:
    name: str
    x: np.ndarray                 # antenna reference points, m
    y: np.ndarray
    elem: Element
    freqs: np.ndarray             # Hz
    P: list                       # harmonic order per frequency
    Q: int                        # polynomial order
    r_min: float                  # model's inner radius (layout minimum spacing)
    ri: float = 0.0               # radius of influence; <= 0 means none
    extra: dict = field(default_factory=dict)

    @property
    def n_ant(self) -> int:
        return int(self.x.shape[0])

    @property
    def n(self) -> int:
        return self.n_ant * self.elem.n_mbf


def element(n_mbf: int, n_samp: int, seed: int, wire_radius: float = 0.02) -> Element:
    """Random MBF set: positions in [-0.25, 0.25]^2 x [0, 2] m, x/z orientation,
    circular CN(0, 1) moments.  Draw order: positions, orientations, Re, Im."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(size=(n_mbf, n_samp, 3))
    pos[..., 0] = pos[..., 0] * 0.5 - 0.25
    pos[..., 1] = pos[..., 1] * 0.5 - 0.25
    pos[..., 2] = pos[..., 2] * 2.0
    zdir = rng.integers(0, 2, size=(n_mbf, n_samp)).astype(bool)
    are = rng.standard_normal((n_mbf, n_samp)) * math.sqrt(0.5)
    aim = rng.standard_normal((n_mbf, n_samp)) * math.sqrt(0.5)
    s = np.zeros((n_mbf, n_samp, SAMPLE_FIELDS), dtype=np.float64)
    s[..., 0:3] = pos
    s[..., 3] = np.where(zdir, 0.0, 1.0)
    s[..., 5] = np.where(zdir, 1.0, 0.0)
    s[..., 6] = are
    s[..., 7] = aim
    return Element(np.ascontiguousarray(s), wire_radius)


def layout_disk(n_ant: int, radius: float, s_min: float, seed: int,
                max_tries: int = 2_000_000) -> tuple[np.ndarray, np.ndarray]:
    """Random sequential addition of n_ant points in a disk with minimum
    spacing s_min (pseudo-random station layouts)."""
    rng = np.random.default_rng(seed)
    xs = np.empty(n_ant)
    ys = np.empty(n_ant)
    cnt = 0
    tries = 0
    s2 = s_min * s_min
    while cnt < n_ant:
        if tries >= max_tries:
            raise RuntimeError(f"layout_disk: could not place {n_ant} points "
                               f"in R={radius} with s_min={s_min}")
        tries += 1
        u, v = rng.uniform(size=2)
        rho = radius * math.sqrt(u)
        th = 2.0 * math.pi * v
        px, py = rho * math.cos(th), rho * math.sin(th)
        if cnt:
            d2 = (xs[:cnt] - px) ** 2 + (ys[:cnt] - py) ** 2
            if d2.min() < s2:
                continue
        xs[cnt] = px
        ys[cnt] = py
        cnt += 1
    return xs, ys


def directions(n_dir: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """theta = acos(U), phi = 2 pi U: uniform over the upper hemisphere."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(size=(n_dir, 2))
    return np.arccos(u[:, 0]), 2.0 * math.pi * u[:, 1]


def harp_orders(freq_hz: float, q: int = 6, half_diag: float = 0.5 * math.sqrt(2.0)):
    """Recipe for the model orders: P = max(6, ceil(k D_h) + 6), Q = 6."""
    kd = 2.0 * math.pi * freq_hz / _C0 * half_diag
    return max(6, int(math.ceil(kd)) + 6), q


CFG2_FREQS = np.array([50e6 + 20e6 * i for i in range(16)])


def workload(name: str, n_freq: int | None = None) -> Workload:
    """The five synthetic configurations (plain small system, station sweep,
    batched layouts, adjoint station, large array with a radius of influence).

    n_freq truncates a frequency sweep (used for fast test variants)."""
    if name == "small16":
        x, y = layout_disk(16, 6.0, 1.5, seed=101)
        el = element(4, 32, seed=201)
        freqs = np.array([100e6])
        return Workload(name, x, y, el, freqs, [6], 6, 1.5)
    if name == "station_sweep":
        x, y = layout_disk(256, 19.0, 1.5, seed=102)
        el = element(8, 64, seed=202)
        freqs = CFG2_FREQS.copy()
        if n_freq is not None:
            idx = np.linspace(0, len(freqs) - 1, n_freq).round().astype(int)
            freqs = freqs[idx]
        return Workload(name, x, y, el, freqs, [harp_orders(f)[0] for f in freqs], 6, 1.5)
    if name == "station_110mhz":
        x, y = layout_disk(256, 19.0, 1.5, seed=102)
        el = element(8, 64, seed=202)
        th, ph = directions(1024, seed=304)
        f = 110e6
        return Workload(name, x, y, el, np.array([f]), [harp_orders(f)[0]], 6, 1.5,
                        extra={"theta": th, "phi": ph, "fd_step": 1e-4})
    if name == "large1024":
        x, y = layout_disk(1024, 38.0, 1.5, seed=105)
        el = element(8, 64, seed=202)
        f = 200e6
        return Workload(name, x, y, el, np.array([f]), [harp_orders(f)[0]], 6, 1.5, ri=12.0)
    if name == "batched_layouts":
        raise ValueError("batched_layouts is a batch of layouts: use batched_layouts()")
    raise KeyError(name)


def batched_layouts(n_layouts: int = 48, seed0: int = 103):
    """Batched station layouts: N_a uniform in {64..512}, R = 19 sqrt(N_a/256),
    8 frequencies per layout drawn without replacement from the 16-point sweep.

    Returns a list of (x, y, freq_indices)."""
    out = []
    for l in range(n_layouts):
        rng = np.random.default_rng(seed0 + l)
        na = int(rng.integers(64, 513))
        fidx = np.sort(rng.choice(len(CFG2_FREQS), size=8, replace=False))
        x, y = layout_disk(na, 19.0 * math.sqrt(na / 256.0), 1.5, seed=seed0 + l + 10_000)
        out.append((x, y, fidx))
    return out
