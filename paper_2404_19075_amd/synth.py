"""Seeded synthetic inputs for the DINR training step and its queries.

This module is the one source of inputs shared by the GPU path, the FP64
oracle and the benchmark.  It holds plain data descriptions (geometry, network
shape, sampling), seeded generators for the frozen Fourier matrix B and the
initial weights, a moving/deforming ellipsoid phantom, and an analytic X-ray
simulator that produces the measured projections for a ray batch.

The simulator is the "scanner", not the method: it integrates the phantom's
attenuation exactly along each detector ray (closed-form ray/ellipsoid chords),
which is what a real measurement p_i = -log(lambda_i / lambda0_i) is in the
noise-free case (Sec. II).  It carries its own ray construction, written
separately from both the oracle and the HIP path; the three agree on the
detector convention only because all three implement the same stated
convention:

  parallel beam: at theta = 0 rays travel along +x, detector u along +y and
  v along +z; pixel centre (u, v) = ((col - (cols-1)/2) pitch_u + off_u,
  (row - (rows-1)/2) pitch_v + off_v); projection index i = m N + row cols + col.
  cone beam: source at (-SOD, 0, 0), flat detector at x = SDD - SOD.
  view m rotates origin and direction by R_z(-theta_m) (Sec. II: rotating the
  object by theta equals rotating the source-detector pair by -theta).

Nothing here evaluates the network, the Fourier encoding or the quadrature.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# --------------------------------------------------------------------- specs


@dataclasses.dataclass
class Geometry:
    kind: int = 0                    # 0 parallel, 1 cone
    rows: int = 32
    cols: int = 32
    n_views: int = 90
    fov_kind: int = 0                # 0 box, 1 cylinder
    sod: float = 0.0
    sdd: float = 0.0
    pitch_u: float = 3.0 / 32
    pitch_v: float = 3.0 / 32
    off_u: float = 0.0
    off_v: float = 0.0
    fov: tuple = (-1.0, 1.0, -1.0, 1.0, -1.0, 1.0)
    t0: float = 0.0
    t1: float = 1.0
    theta: np.ndarray = None         # [n_views] float64 radians
    time: np.ndarray = None          # [n_views] float64

    @property
    def n_pixels(self) -> int:
        return self.rows * self.cols

    @property
    def n_proj(self) -> int:
        return self.rows * self.cols * self.n_views


@dataclasses.dataclass
class MLPSpec:
    n_freq: int = 64                 # C; the encoding has 2C features
    width: int = 64                  # H
    depth: int = 3                   # L hidden layers
    act: int = 0                     # 0 ReLU, 1 Swish
    out_act: int = 1                 # 0 identity, 1 softplus
    mu0: float = 1.0
    sigma_t: float = 4.0
    sigma_s: float = 4.0

    @property
    def n_params(self) -> int:
        c2, h, l = 2 * self.n_freq, self.width, self.depth
        return h * c2 + h + (l - 1) * (h * h + h) + h + 1

    def layer_shapes(self):
        """(fan_out, fan_in) of each hidden layer, then the output layer."""
        c2, h = 2 * self.n_freq, self.width
        shapes = [(h, c2)] + [(h, h)] * (self.depth - 1)
        return shapes + [(1, h)]

    def flops_per_point(self) -> int:
        """Algorithmic FLOP per ray sample for forward + backward: 2 fan_in
        fan_out per layer forward, the same again for the weight gradient, and
        the input gradient of every layer but the first."""
        shapes = self.layer_shapes()
        fwd = sum(2 * o * i for o, i in shapes)
        dx = sum(2 * o * i for o, i in shapes[1:])
        return 2 * fwd + dx

    def fwd_flops_per_point(self) -> int:
        return sum(2 * o * i for o, i in self.layer_shapes())


@dataclasses.dataclass
class Sampling:
    mode: int = 0                    # 0 fixed n, 1 n = clamp(ceil(l/h), n_min, n_max)
    n: int = 64
    h: float = 1.0 / 256
    n_min: int = 32
    n_max: int = 512
    sub: int = 1                     # D: D x D rays per projection (Appendix A)
    jitter: int = 0                  # 1: stratified random sample positions (Sec. IV)
    seed: int = 0                    # key words of the position generator
    epoch: int = 0


@dataclasses.dataclass
class Phantom:
    """Ellipsoids: centre c + v t, semi-axes s (1 + kappa t), orientation R,
    attenuation a (additive where they overlap)."""
    c: np.ndarray       # [E,3]
    v: np.ndarray       # [E,3]
    s: np.ndarray       # [E,3]
    kappa: np.ndarray   # [E]
    a: np.ndarray       # [E]
    R: np.ndarray       # [E,3,3]

    def packed(self) -> np.ndarray:
        """[E,20] = c, v, s, kappa, a, R (row-major), the oracle's layout."""
        e = len(self.a)
        out = np.zeros((e, 20))
        out[:, 0:3] = self.c
        out[:, 3:6] = self.v
        out[:, 6:9] = self.s
        out[:, 9] = self.kappa
        out[:, 10] = self.a
        out[:, 11:20] = self.R.reshape(e, 9)
        return out


@dataclasses.dataclass
class Workload:
    name: str
    geom: Geometry
    mlp: MLPSpec
    sampling: Sampling
    n_rays: int
    n_ellipsoids: int
    centre_range: float
    max_speed: float
    axes_range: tuple
    kappa_range: float
    rotate: bool
    noise: float                     # Gaussian sigma as a fraction of max projection
    precision: str                   # "fp32" or "bf16"
    recompute: bool = False
    seed: int = 0


# ------------------------------------------------------------------ presets

def _views(n_views: int, span: float) -> tuple:
    v = np.arange(n_views, dtype=np.float64)
    return v * span / n_views, v / n_views


def workload(name: str) -> Workload:
    """The workloads: c0 tiny parity case, c1 FP32 parallel beam, c2 the same
    in BF16, c3 ragged cone beam, c4 serving (weights as c2), "paper", the
    paper's own Swish network on the c2 geometry, and "paper_cyl", the same in
    a cylindrical field of view."""
    if name == "c0":
        th, tt = _views(90, math.pi)
        g = Geometry(kind=0, rows=32, cols=32, n_views=90, pitch_u=3.0 / 32, pitch_v=3.0 / 32,
                     theta=th, time=tt)
        return Workload("c0", g, MLPSpec(n_freq=64, width=64, depth=3, act=0, out_act=1,
                                         sigma_t=4.0, sigma_s=4.0),
                        Sampling(mode=0, n=64), n_rays=1024, n_ellipsoids=3,
                        centre_range=0.3, max_speed=0.2, axes_range=(0.2, 0.5), kappa_range=0.0,
                        rotate=True, noise=0.0, precision="fp32", seed=1000)
    if name in ("c1", "c2", "c4"):
        th, tt = _views(720, 2 * math.pi)
        g = Geometry(kind=0, rows=256, cols=256, n_views=720, pitch_u=3.0 / 256,
                     pitch_v=3.0 / 256, theta=th, time=tt)
        return Workload(name, g, MLPSpec(n_freq=128, width=256, depth=6, act=0, out_act=1,
                                         sigma_t=4.0, sigma_s=4.0),
                        Sampling(mode=0, n=256), n_rays=65536, n_ellipsoids=20,
                        centre_range=0.4, max_speed=0.2, axes_range=(0.05, 0.3),
                        kappa_range=0.3, rotate=True, noise=0.01,
                        precision="fp32" if name == "c1" else "bf16", seed=1001)
    if name == "c3":
        th, tt = _views(1800, 2 * math.pi)
        g = Geometry(kind=1, rows=512, cols=512, n_views=1800, sod=500.0, sdd=1000.0,
                     pitch_u=3.0 / 256, pitch_v=3.0 / 256, theta=th, time=tt)
        return Workload("c3", g, MLPSpec(n_freq=128, width=256, depth=8, act=0, out_act=1,
                                         sigma_t=4.0, sigma_s=4.0),
                        Sampling(mode=1, h=1.0 / 256, n_min=32, n_max=512), n_rays=131072,
                        n_ellipsoids=20, centre_range=0.4, max_speed=0.2,
                        axes_range=(0.05, 0.3), kappa_range=0.3, rotate=True, noise=0.01,
                        precision="bf16", recompute=True, seed=1003)
    if name == "paper":
        # the network of Appendix B (Swish hidden layers, linear output,
        # 2C = H = 256, five hidden layers, sigma_s = 0.5, sigma_t = 0.1) on the
        # c2 geometry and batch
        w = workload("c2")
        return dataclasses.replace(
            w, name="paper", mlp=MLPSpec(n_freq=128, width=256, depth=5, act=1, out_act=0,
                                         sigma_t=0.1, sigma_s=0.5), seed=1005)
    if name == "paper_cyl":
        # the paper's network in the paper's kind of field of view (Sec. II: the
        # object lies in a cylinder; App. B item 1 normalises coordinates by
        # its bounds): radius 1, z in [-1, 1], on the c2 geometry and batch
        w = workload("paper")
        g = dataclasses.replace(w.geom, fov_kind=1, fov=(1.0, -1.0, 1.0, 0.0, 0.0, 0.0))
        return dataclasses.replace(w, name="paper_cyl", geom=g, seed=1006)
    raise KeyError(name)


# ------------------------------------------------------- weights and encoding

def make_B(spec: MLPSpec, seed: int) -> np.ndarray:
    """Frozen GRFF matrix B [C,4] (Appendix B item 2): column 0 (time) drawn
    from N(0, sigma_t^2), columns 1..3 (z, y, x) from N(0, sigma_s^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    B = rng.standard_normal((spec.n_freq, 4))
    B[:, 0] *= spec.sigma_t
    B[:, 1:] *= spec.sigma_s
    return B.astype(np.float32)


def make_params(spec: MLPSpec, seed: int) -> np.ndarray:
    """Flat FP32 parameters: for each hidden layer W [H, fan_in] row-major then
    b [H]; then w_o [H], b_o.  Each entry ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for fo, fi in spec.layer_shapes():
        k = 1.0 / math.sqrt(fi)
        parts.append(rng.uniform(-k, k, size=fo * fi))
        parts.append(rng.uniform(-k, k, size=fo))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == spec.n_params
    return p


# -------------------------------------------------------------------- phantom

def _rotations(rng, n: int) -> np.ndarray:
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def make_phantom(w: Workload, seed: Optional[int] = None) -> Phantom:
    rng = np.random.Generator(np.random.PCG64(w.seed + 17 if seed is None else seed))
    e = w.n_ellipsoids
    c = rng.uniform(-w.centre_range, w.centre_range, size=(e, 3))
    d = rng.standard_normal((e, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    v = d * rng.uniform(0.0, w.max_speed, size=(e, 1))
    s = rng.uniform(w.axes_range[0], w.axes_range[1], size=(e, 3))
    kappa = rng.uniform(-w.kappa_range, w.kappa_range, size=e) if w.kappa_range > 0 \
        else np.zeros(e)
    a = rng.uniform(0.5, 1.0, size=e)
    R = _rotations(rng, e) if w.rotate else np.tile(np.eye(3), (e, 1, 1))
    return Phantom(c, v, s, kappa, a, R)


# -------------------------------------------------------------- the scanner

def scanner_rays(g: Geometry, idx: np.ndarray):
    """Origins, unit directions and times of detector rays (scanner side)."""
    idx = np.asarray(idx, dtype=np.int64)
    npix = g.rows * g.cols
    m = idx // npix
    pix = idx % npix
    row = pix // g.cols
    col = pix % g.cols
    u = (col - 0.5 * (g.cols - 1)) * g.pitch_u + g.off_u
    v = (row - 0.5 * (g.rows - 1)) * g.pitch_v + g.off_v
    th = np.asarray(g.theta)[m]
    ct, st = np.cos(th), np.sin(th)
    n = idx.shape[0]
    if g.kind == 0:
        o0 = np.stack([np.zeros(n), u, v], axis=1)
        d0 = np.tile(np.array([1.0, 0.0, 0.0]), (n, 1))
    else:
        o0 = np.tile(np.array([-g.sod, 0.0, 0.0]), (n, 1))
        d0 = np.stack([np.full(n, g.sdd), u, v], axis=1)
        d0 /= np.linalg.norm(d0, axis=1, keepdims=True)
    def rot(p):
        return np.stack([ct * p[:, 0] + st * p[:, 1], -st * p[:, 0] + ct * p[:, 1], p[:, 2]],
                        axis=1)
    return rot(o0), rot(d0), np.asarray(g.time)[m]


def scanner_fov_chord(g: Geometry, o: np.ndarray, d: np.ndarray):
    """Entry parameter and length of each ray inside the FOV (0 for a miss)."""
    n = o.shape[0]
    lo = np.full(n, -np.inf)
    hi = np.full(n, np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        if g.fov_kind == 0:
            for a in range(3):
                b0, b1 = g.fov[2 * a], g.fov[2 * a + 1]
                par = d[:, a] == 0
                ta = (b0 - o[:, a]) / d[:, a]
                tb = (b1 - o[:, a]) / d[:, a]
                t_lo = np.where(par, np.where((o[:, a] >= b0) & (o[:, a] <= b1), -np.inf, np.inf),
                                np.minimum(ta, tb))
                t_hi = np.where(par, np.where((o[:, a] >= b0) & (o[:, a] <= b1), np.inf, -np.inf),
                                np.maximum(ta, tb))
                lo = np.maximum(lo, t_lo)
                hi = np.minimum(hi, t_hi)
        else:
            R, z0, z1 = g.fov[0], g.fov[1], g.fov[2]
            qa = d[:, 0] ** 2 + d[:, 1] ** 2
            qb = 2 * (o[:, 0] * d[:, 0] + o[:, 1] * d[:, 1])
            qc = o[:, 0] ** 2 + o[:, 1] ** 2 - R * R
            disc = qb * qb - 4 * qa * qc
            sq = np.sqrt(np.maximum(disc, 0))
            lo = np.where(disc > 0, (-qb - sq) / (2 * qa), np.inf)
            hi = np.where(disc > 0, (-qb + sq) / (2 * qa), -np.inf)
            ta = (z0 - o[:, 2]) / d[:, 2]
            tb = (z1 - o[:, 2]) / d[:, 2]
            par = d[:, 2] == 0
            inside = (o[:, 2] >= z0) & (o[:, 2] <= z1)
            lo = np.maximum(lo, np.where(par, np.where(inside, -np.inf, np.inf),
                                         np.minimum(ta, tb)))
            hi = np.minimum(hi, np.where(par, np.where(inside, np.inf, -np.inf),
                                         np.maximum(ta, tb)))
    ln = np.where(hi > lo, hi - lo, 0.0)
    return np.where(hi > lo, lo, 0.0), ln


def ellipsoid_chords(ph: Phantom, o: np.ndarray, d: np.ndarray, t: np.ndarray) -> np.ndarray:
    """[n_rays, E] exact chord length of each ray through each ellipsoid at the
    ray's time."""
    n, e = o.shape[0], len(ph.a)
    out = np.zeros((n, e))
    for k in range(e):
        c = ph.c[k][None, :] + ph.v[k][None, :] * t[:, None]
        s = ph.s[k][None, :] * (1.0 + ph.kappa[k] * t[:, None])
        # body-frame coordinates q(s) = diag(1/s) R^T (o + s d - c)
        RT = ph.R[k].T
        po = (o - c) @ RT.T / s
        pd = d @ RT.T / s
        A = np.sum(pd * pd, axis=1)
        B = 2 * np.sum(po * pd, axis=1)
        C = np.sum(po * po, axis=1) - 1.0
        disc = B * B - 4 * A * C
        out[:, k] = np.where(disc > 0, np.sqrt(np.maximum(disc, 0)) / A, 0.0)
    return out


def project_phantom(g: Geometry, ph: Phantom, idx: np.ndarray) -> np.ndarray:
    """Noise-free line integrals sum_e a_e chord_e(t) for projection indices."""
    o, d, t = scanner_rays(g, idx)
    return ellipsoid_chords(ph, o, d, t) @ ph.a


def _splitmix(x: np.ndarray) -> np.ndarray:
    x = (x + np.uint64(0x9E3779B97F4A7C15)) & np.uint64(0xFFFFFFFFFFFFFFFF)
    z = x
    z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & np.uint64(0xFFFFFFFFFFFFFFFF)
    z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & np.uint64(0xFFFFFFFFFFFFFFFF)
    return z ^ (z >> np.uint64(31))


def index_normal(seed: int, idx: np.ndarray) -> np.ndarray:
    """Standard normal keyed by (seed, projection index): the same pixel gets
    the same noise in whatever batch it is drawn (Box-Muller on two
    splitmix64 draws)."""
    with np.errstate(over="ignore"):
        k = np.asarray(idx, dtype=np.uint64) * np.uint64(2) + np.uint64(seed) * np.uint64(0x632BE59BD9B4E019)
        a = _splitmix(k)
        b = _splitmix(k + np.uint64(1))
    u1 = ((a >> np.uint64(11)).astype(np.float64) + 0.5) / 2.0 ** 53
    u2 = (b >> np.uint64(11)).astype(np.float64) / 2.0 ** 53
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2 * np.pi * u2)


def draw_rays(g: Geometry, n_rays: int, seed: int) -> np.ndarray:
    """n_rays distinct projection indices, uniform among pixels whose ray
    crosses the FOV (the sparse batch Omega_k of Sec. II)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    chosen: List[np.ndarray] = []
    seen = set()
    total = 0
    while total < n_rays:
        cand = rng.integers(0, g.n_proj, size=max(2 * (n_rays - total), 1024), dtype=np.int64)
        o, d, _ = scanner_rays(g, cand)
        _, ln = scanner_fov_chord(g, o, d)
        cand = cand[ln > 0]
        keep = []
        for c in cand.tolist():
            if c not in seen:
                seen.add(c)
                keep.append(c)
                if total + len(keep) == n_rays:
                    break
        chosen.append(np.asarray(keep, dtype=np.int64))
        total += len(keep)
    return np.concatenate(chosen)[:n_rays]


def noise_scale(w: Workload, ph: Phantom, n_probe: int = 1 << 18) -> float:
    """sigma = noise * max noise-free projection, the maximum taken over a fixed
    seeded subsample of pixels."""
    if w.noise <= 0:
        return 0.0
    rng = np.random.Generator(np.random.PCG64(w.seed + 99))
    probe = rng.integers(0, w.geom.n_proj, size=n_probe, dtype=np.int64)
    return float(w.noise * project_phantom(w.geom, ph, probe).max())


def measurements(w: Workload, ph: Phantom, idx: np.ndarray, sigma: float) -> np.ndarray:
    p = project_phantom(w.geom, ph, idx)
    if sigma > 0:
        p = p + sigma * index_normal(w.seed + 7, idx)
    return p.astype(np.float32)


@dataclasses.dataclass
class Batch:
    workload: Workload
    B: np.ndarray          # [C,4] float32
    params: np.ndarray     # [n_params] float32
    idx: np.ndarray        # [R] int64
    meas: np.ndarray       # [R] float32
    phantom: Phantom


def make_batch(name_or_w, n_rays: Optional[int] = None, seed_offset: int = 0) -> Batch:
    w = workload(name_or_w) if isinstance(name_or_w, str) else name_or_w
    R = w.n_rays if n_rays is None else n_rays
    ph = make_phantom(w)
    B = make_B(w.mlp, w.seed + 1)
    P = make_params(w.mlp, w.seed + 2)
    idx = draw_rays(w.geom, R, w.seed + 3 + seed_offset)
    sigma = noise_scale(w, ph)
    meas = measurements(w, ph, idx, sigma)
    return Batch(w, B, P, idx, meas, ph)
