"""Seeded synthetic MUSER-shaped imaging workloads.

This module is the input generator shared by the GPU path, the FP64 oracle and the
benchmark.  It models the instrument and the sky only (antenna layout, baseline
coordinates, analytic visibilities of a solar-disk-like sky); it contains none of the
imaging arithmetic (no gridding, transform or deconvolution).

What it follows in the paper:
  * MUSER-I: 40 antennas, 0.4-2.0 GHz in 64 x 25 MHz channels; MUSER-II: 60 antennas,
    2-15 GHz in 520 channels; baselines from a few metres to about 3 km (Table 1).
  * Observatory latitude 42.211833 deg (Sec. 3.2.2, UVW calculation).
  * A solar disk centred in the field of view; the image is 2-D (w ignored), as in the
    snapshot reduction of Sec. 2.
The MUSER observations themselves are not available, so everything here is synthetic:
a three-arm log-spiral array, the textbook hour-angle/declination rotation to (u, v, w),
and a sky of a uniform disk (radius 16 arcmin) plus three Gaussian sources plus noise,
with analytic visibilities evaluated in FP64 and stored as complex64.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
from scipy import special

C_LIGHT = 299792458.0
LATITUDE_DEG = 42.211833333          # Mingantu station latitude (Sec. 3.2.2)
ARCMIN = math.pi / (180.0 * 60.0)
FOV_RAD = math.radians(1.2)          # field of view used for every workload


# ----------------------------------------------------------------------------------
# array and (u, v, w)
# ----------------------------------------------------------------------------------
def spiral_array(k_per_arm: int, r_min: float, r_max: float, centre: bool, seed: int) -> np.ndarray:
    """East/North antenna positions (metres) on three log-spiral arms (pitch 60 deg)."""
    rng = np.random.default_rng(seed)
    phi0 = rng.uniform(0.0, 2.0 * math.pi)
    pos = []
    if centre:
        pos.append((0.0, 0.0))
    for a in range(3):
        theta_a = phi0 + 2.0 * math.pi * a / 3.0
        for k in range(k_per_arm):
            r = r_min * (r_max / r_min) ** (k / (k_per_arm - 1))
            th = theta_a + math.log(r / r_min) / math.tan(math.radians(60.0))
            r_j = r * (1.0 + 0.05 * rng.standard_normal())
            th_j = th + 0.02 * rng.standard_normal()
            pos.append((r_j * math.cos(th_j), r_j * math.sin(th_j)))
    return np.asarray(pos, dtype=np.float64)


def muser1_array() -> np.ndarray:
    """40 antennas: one centre antenna + 13 per arm, 8 m .. 1.5 km (780 baselines)."""
    return spiral_array(13, 8.0, 1500.0, True, seed=1)


def muser2_array() -> np.ndarray:
    """60 antennas: 20 per arm, 4 m .. 3 km (1770 baselines)."""
    return spiral_array(20, 4.0, 3000.0, False, seed=2)


def baselines(pos: np.ndarray) -> np.ndarray:
    i, j = np.triu_indices(len(pos), k=1)
    return pos[j] - pos[i]                       # (n_bl, 2) east, north in metres


def uvw_metres(bl_en: np.ndarray, ha_rad: float, dec_rad: float,
               lat_rad: float = math.radians(LATITUDE_DEG)) -> np.ndarray:
    """(u, v, w) in metres for a flat array (up = 0) at hour angle H and declination d."""
    e, n = bl_en[:, 0], bl_en[:, 1]
    x = -math.sin(lat_rad) * n
    y = e
    z = math.cos(lat_rad) * n
    sh, ch = math.sin(ha_rad), math.cos(ha_rad)
    sd, cd = math.sin(dec_rad), math.cos(dec_rad)
    u = sh * x + ch * y
    v = -sd * ch * x + sd * sh * y + cd * z
    w = cd * ch * x - cd * sh * y + sd * z
    return np.stack([u, v, w], axis=1)


# ----------------------------------------------------------------------------------
# sky model (analytic visibilities, convention V(u,v) = sum I(l,m) exp(-2 pi i (ul+vm)))
# ----------------------------------------------------------------------------------
@dataclasses.dataclass
class Sky:
    radius: float                    # disk radius (rad); total disk flux is 1
    gauss: np.ndarray                # (3, 4): peak brightness, sigma (rad), l0, m0
    limb: float = 0.0                # limb-brightening coefficient a in B(1 + a rho^2/R^2)
    centre: tuple = (0.0, 0.0)       # (l, m) of the disk centre (rad): the whole sky is displaced

    @property
    def b_disk(self) -> float:
        return 1.0 / (math.pi * self.radius ** 2)


def make_sky(seed: int, radius: float = 16.0 * ARCMIN, limb: float = 0.0) -> Sky:
    rng = np.random.default_rng(seed)
    b_disk = 1.0 / (math.pi * radius ** 2)
    g = np.zeros((3, 4))
    for s in range(3):
        sigma = rng.uniform(1.0, 3.0) * ARCMIN
        peak = rng.uniform(5.0, 50.0) * b_disk
        rr = 0.8 * radius * math.sqrt(rng.uniform())
        ang = rng.uniform(0.0, 2.0 * math.pi)
        g[s] = (peak, sigma, rr * math.cos(ang), rr * math.sin(ang))
    return Sky(radius=radius, gauss=g, limb=limb)


def disk_vis(q: np.ndarray, radius: float) -> np.ndarray:
    """Uniform disk of unit total flux: 2 J1(2 pi q R) / (2 pi q R)."""
    x = 2.0 * math.pi * q * radius
    out = np.ones_like(x)
    nz = x > 1e-12
    out[nz] = 2.0 * special.j1(x[nz]) / x[nz]
    return out


def limb_vis(q: np.ndarray, radius: float, a: float, b_disk: float) -> np.ndarray:
    """Transform of a * b_disk * (rho/R)^2 inside the disk (limb-brightening excess)."""
    k = 2.0 * math.pi * q
    out = np.full_like(k, 2.0 * math.pi * a * b_disk / radius ** 2 * radius ** 4 / 4.0)
    nz = k * radius > 1e-6
    kk = k[nz]
    integral = radius ** 3 * special.j1(kk * radius) / kk - 2.0 * radius ** 2 * special.jv(2, kk * radius) / kk ** 2
    out[nz] = 2.0 * math.pi * a * b_disk / radius ** 2 * integral
    return out


def gauss_vis(u: np.ndarray, v: np.ndarray, peak: float, sigma: float, l0: float, m0: float) -> np.ndarray:
    q2 = u * u + v * v
    amp = peak * 2.0 * math.pi * sigma ** 2 * np.exp(-2.0 * math.pi ** 2 * sigma ** 2 * q2)
    return amp * np.exp(-2j * math.pi * (u * l0 + v * m0))


def sky_vis(sky: Sky, u: np.ndarray, v: np.ndarray) -> np.ndarray:
    q = np.hypot(u, v)
    vis = disk_vis(q, sky.radius).astype(np.complex128)
    if sky.limb != 0.0:
        vis = vis + limb_vis(q, sky.radius, sky.limb, sky.b_disk)
    for peak, sigma, l0, m0 in sky.gauss:
        vis = vis + gauss_vis(u, v, peak, sigma, l0, m0)
    lc, mc = sky.centre
    if lc != 0.0 or mc != 0.0:                   # the sky displaced as a whole
        vis = vis * np.exp(-2j * math.pi * (u * lc + v * mc))
    return vis


def limb_coefficient(freq_hz: float) -> float:
    """a(nu) = 0.3 + 0.4 (nu - 2 GHz) / 13 GHz (a proposal; the paper is silent)."""
    return 0.3 + 0.4 * (freq_hz - 2.0e9) / 13.0e9


# ----------------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    vis: np.ndarray            # complex64 [M]
    uv: np.ndarray             # float32 [M, 2], wavelengths
    w: np.ndarray              # float32 [M], input weights (0 = flagged)
    vis_offset: np.ndarray     # int64 [n+1]
    n_img: np.ndarray          # int32 [n]
    cell_rad: np.ndarray       # float64 [n]
    weight_mode: np.ndarray    # int8 [n] (0 natural, 1 uniform)
    niter: np.ndarray          # int32 [n]
    freq_hz: np.ndarray        # float64 [n]
    gain: float = 0.1
    sky_centre: Optional[np.ndarray] = None   # float64 [n, 2]: true (l, m) of the disk centre (rad)
    w_lambda: Optional[np.ndarray] = None     # float32 [M]: w coordinate (wavelengths), when the
                                              # visibilities carry the w-term

    @property
    def n_inst(self) -> int:
        return len(self.n_img)

    def instance(self, i: int):
        a, b = int(self.vis_offset[i]), int(self.vis_offset[i + 1])
        return self.vis[a:b], self.uv[a:b], self.w[a:b]

    def instance_w(self, i: int):
        a, b = int(self.vis_offset[i]), int(self.vis_offset[i + 1])
        return self.w_lambda[a:b]

    def subset(self, idx) -> "Workload":
        idx = list(idx)
        parts = [self.instance(i) for i in idx]
        counts = [len(p[0]) for p in parts]
        off = np.zeros(len(idx) + 1, np.int64)
        off[1:] = np.cumsum(counts)
        cat = lambda k, dt: (np.concatenate([p[k] for p in parts]) if parts else np.zeros(0, dt))
        return Workload(
            name=f"{self.name}[{len(idx)}]",
            vis=cat(0, np.complex64).astype(np.complex64),
            uv=(np.concatenate([p[1] for p in parts]) if parts else np.zeros((0, 2), np.float32)).astype(np.float32),
            w=cat(2, np.float32).astype(np.float32),
            vis_offset=off, n_img=self.n_img[idx].copy(), cell_rad=self.cell_rad[idx].copy(),
            weight_mode=self.weight_mode[idx].copy(), niter=self.niter[idx].copy(),
            freq_hz=self.freq_hz[idx].copy(), gain=self.gain,
            sky_centre=None if self.sky_centre is None else self.sky_centre[idx].copy(),
            w_lambda=None if self.w_lambda is None else
            (np.concatenate([self.instance_w(i) for i in idx]) if idx else np.zeros(0, np.float32)))


def _instance_vis(bl_en, freq_hz, ha_rad, sky, noise_seed, dec_rad=math.radians(20.0)):
    uvw = uvw_metres(bl_en, ha_rad, dec_rad) * (freq_hz / C_LIGHT)
    u, v = uvw[:, 0], uvw[:, 1]
    vis = sky_vis(sky, u, v)
    rng = np.random.default_rng(noise_seed)
    sig = 0.01 * np.max(np.abs(vis))
    vis = vis + sig * (rng.standard_normal(len(u)) + 1j * rng.standard_normal(len(u)))
    return vis.astype(np.complex64), np.stack([u, v], 1).astype(np.float32)


def _assemble(name, items, gain=0.1) -> Workload:
    vis = np.concatenate([it["vis"] for it in items]) if items else np.zeros(0, np.complex64)
    uv = np.concatenate([it["uv"] for it in items]) if items else np.zeros((0, 2), np.float32)
    w = np.concatenate([it["w"] for it in items]) if items else np.zeros(0, np.float32)
    off = np.zeros(len(items) + 1, np.int64)
    off[1:] = np.cumsum([len(it["vis"]) for it in items])
    return Workload(
        name=name, vis=vis.astype(np.complex64), uv=uv.astype(np.float32), w=w.astype(np.float32),
        vis_offset=off,
        n_img=np.array([it["N"] for it in items], np.int32),
        cell_rad=np.array([FOV_RAD / it["N"] for it in items], np.float64),
        weight_mode=np.array([it["mode"] for it in items], np.int8),
        niter=np.array([it["niter"] for it in items], np.int32),
        freq_hz=np.array([it["freq"] for it in items], np.float64), gain=gain)


def c1_snapshot() -> Workload:
    """Single snapshot: 780 baselines at 1.7 GHz, 256^2, natural weighting, 500 iterations."""
    bl = baselines(muser1_array())
    sky = make_sky(3)
    vis, uv = _instance_vis(bl, 1.7e9, 0.0, sky, 1000)
    return _assemble("c1_snapshot_256", [dict(vis=vis, uv=uv, w=np.ones(len(vis), np.float32),
                                               N=256, mode=0, niter=500, freq=1.7e9)])


def c2_muser1_batch(n_chan: int = 64, n_snap: int = 20) -> Workload:
    """MUSER-I-like batch: 64 channels x 20 snapshots, 512^2, uniform weighting, 2000 iterations."""
    bl = baselines(muser1_array())
    sky = make_sky(3)
    items = []
    inst = 0
    for s in range(n_snap):
        ha = (-1.0 + 2.0 * s / 19.0) * math.pi / 12.0
        for c in range(n_chan):
            f = (0.4125 + 0.025 * c) * 1e9
            vis, uv = _instance_vis(bl, f, ha, sky, 1000 + inst)
            items.append(dict(vis=vis, uv=uv, w=np.ones(len(vis), np.float32), N=512, mode=1, niter=2000, freq=f))
            inst += 1
    return _assemble(f"c2_muser1_{n_chan}x{n_snap}_512", items)


def c3_muser2(n_chan: int = 520, chans: Optional[List[int]] = None, N: int = 1024, niter: int = 5000) -> Workload:
    """MUSER-II-like: 1770 baselines, 2.0125..14.9875 GHz, 1024^2, limb-brightened disk, natural weighting."""
    bl = baselines(muser2_array())
    chans = list(range(n_chan)) if chans is None else list(chans)
    items = []
    for inst, c in enumerate(chans):
        f = (2.0125 + 0.025 * c) * 1e9
        sky = make_sky(3, limb=limb_coefficient(f))
        vis, uv = _instance_vis(bl, f, 0.0, sky, 1000 + c)
        items.append(dict(vis=vis, uv=uv, w=np.ones(len(vis), np.float32), N=N, mode=0, niter=niter, freq=f))
    return _assemble(f"c3_muser2_{len(chans)}ch_{N}", items)


def c3_w_lambda(n_chan: int = 520, chans: Optional[List[int]] = None) -> np.ndarray:
    """w coordinates (wavelengths, float32, same order as c3_muser2's visibilities) of the
    MUSER-II-like array at the C3 pointing (hour angle 0, declination +20 deg)."""
    bl = baselines(muser2_array())
    chans = list(range(n_chan)) if chans is None else list(chans)
    w_m = uvw_metres(bl, 0.0, math.radians(20.0))[:, 2]
    return np.concatenate([w_m * ((2.0125 + 0.025 * c) * 1e9 / C_LIGHT) for c in chans]).astype(np.float32)


def c4_uneven(n: int = 256) -> Workload:
    """Uneven serving-style batch: 200..1770 baselines, N in {256,512,1024}, niter 500..5000."""
    pos = muser2_array()
    bl_all = baselines(pos)
    rng = np.random.default_rng(5)
    flag_rng = np.random.default_rng(4)
    items = []
    for inst in range(n):
        n_bl = int(rng.integers(200, 1771))
        N = int(rng.choice([256, 512, 1024]))
        c = int(rng.integers(0, 520))
        niter = int(rng.integers(500, 5001))
        mode = int(rng.integers(0, 2))
        f = (2.0125 + 0.025 * c) * 1e9
        keep = np.sort(flag_rng.choice(len(bl_all), size=n_bl, replace=False))
        sky = make_sky(3, limb=limb_coefficient(f))
        vis, uv = _instance_vis(bl_all[keep], f, 0.0, sky, 1000 + inst)
        w = np.ones(n_bl, np.float32)
        w[flag_rng.uniform(size=n_bl) < 0.05] = 0.0
        items.append(dict(vis=vis, uv=uv, w=w, N=N, mode=mode, niter=niter, freq=f))
    return _assemble(f"c4_uneven_{n}", items)


def c5_differentiable(n_chan: int = 32, N: int = 1024) -> Workload:
    """60 antennas, 32 channels evenly spaced in 2-15 GHz, natural weighting."""
    bl = baselines(muser2_array())
    sky = make_sky(3)
    items = []
    for c, f in enumerate(np.linspace(2.0e9, 15.0e9, n_chan)):
        vis, uv = _instance_vis(bl, float(f), 0.0, sky, 1000 + c)
        items.append(dict(vis=vis, uv=uv, w=np.ones(len(vis), np.float32), N=N, mode=0, niter=0, freq=float(f)))
    return _assemble(f"c5_diff_{n_chan}ch_{N}", items)


def fd_subset() -> Workload:
    """The 16 innermost MUSER-II antennas (120 baselines) at 2.0125 GHz on a 64^2 grid."""
    pos = muser2_array()
    order = np.argsort(np.hypot(pos[:, 0], pos[:, 1]))[:16]
    bl = baselines(pos[np.sort(order)])
    sky = make_sky(6)
    f = 2.0125e9
    vis, uv = _instance_vis(bl, f, 0.0, sky, 1006)
    # small grid: widen the field so the inner baselines fit (cell 1/(N dl) with dl = FOV/N)
    return _assemble("fd_subset_64", [dict(vis=vis, uv=uv, w=np.ones(len(vis), np.float32),
                                           N=64, mode=0, niter=0, freq=f)])


def offset_disk(seed: int = 7, n: int = 6, sizes=(256, 512), max_offset_px: float = 24.0,
                niter: int = 3000) -> Workload:
    """Displaced-disk instances for the disk-centering step: MUSER-II-like array, channels
    over 2-15 GHz, the whole sky (disk, limb, sources) shifted by a random offset of up to
    `max_offset_px` pixels in each axis (a phase / pointing error); natural weighting."""
    rng = np.random.default_rng(seed)
    bl = baselines(muser2_array())
    items, centres = [], []
    for k in range(n):
        N = int(sizes[k % len(sizes)])
        c = int(rng.integers(0, 520))
        f = (2.0125 + 0.025 * c) * 1e9
        cell = FOV_RAD / N
        off = rng.uniform(-max_offset_px, max_offset_px, 2) * cell
        sky = dataclasses.replace(make_sky(3, limb=limb_coefficient(f)), centre=(float(off[0]), float(off[1])))
        vis, uv = _instance_vis(bl, f, 0.0, sky, 2000 + k)
        items.append(dict(vis=vis, uv=uv, w=np.ones(len(vis), np.float32), N=N, mode=0, niter=niter, freq=f))
        centres.append(off)
    wl = _assemble(f"offset_disk_{n}", items)
    wl.sky_centre = np.array(centres, np.float64)
    return wl


def wterm_points(seed: int = 9, n: int = 4, sizes=(256, 512), freq_hz: float = 1.7e9, n_src: int = 4,
                 dec_deg: float = -23.4, ha_hours=(-4.0, -2.0, 2.0, 4.0)) -> Workload:
    """Point sources seen with the w-term (the measurement equation with w, closed form):
    MUSER-II-like array, winter declination and hour angles away from transit (low
    elevation, so |w| reaches a large fraction of the baseline), sources anywhere within
    0.4 of the field from the centre, 1 % noise; natural weighting.  w_lambda holds w."""
    rng = np.random.default_rng(seed)
    bl = baselines(muser2_array())
    items, ws = [], []
    for k in range(n):
        N = int(sizes[k % len(sizes)])
        ha = ha_hours[k % len(ha_hours)] * math.pi / 12.0
        uvw = uvw_metres(bl, ha, math.radians(dec_deg)) * (freq_hz / C_LIGHT)
        u, v, w = uvw[:, 0], uvw[:, 1], uvw[:, 2]
        vis = np.zeros(len(u), np.complex128)
        for _ in range(n_src):
            l0, m0 = rng.uniform(-0.4, 0.4, 2) * FOV_RAD
            n0 = math.sqrt(1.0 - l0 * l0 - m0 * m0)
            vis += rng.uniform(0.5, 2.0) * np.exp(-2j * math.pi * (u * l0 + v * m0 + w * (n0 - 1.0)))
        sig = 0.01 * np.max(np.abs(vis))
        vis += sig * (rng.standard_normal(len(u)) + 1j * rng.standard_normal(len(u)))
        items.append(dict(vis=vis.astype(np.complex64), uv=np.stack([u, v], 1).astype(np.float32),
                          w=np.ones(len(u), np.float32), N=N, mode=0, niter=500, freq=freq_hz))
        ws.append(w.astype(np.float32))
    wl = _assemble(f"wterm_points_{n}", items)
    wl.w_lambda = np.concatenate(ws).astype(np.float32)
    return wl


def random_instances(seed: int, sizes, m_range=(1, 300), uniform_frac=0.5, fill=0.8) -> Workload:
    """Small random instances (uniformly scattered uv inside the keepable band) for parity tests."""
    rng = np.random.default_rng(seed)
    items = []
    for N in sizes:
        m = int(rng.integers(m_range[0], m_range[1] + 1))
        lim = (N / 2 - 4) * fill
        cell = FOV_RAD / N
        du = 1.0 / (N * cell)
        u = rng.uniform(-lim, lim, size=m) * du
        v = rng.uniform(-lim, lim, size=m) * du
        vis = (rng.standard_normal(m) + 1j * rng.standard_normal(m)).astype(np.complex64)
        w = rng.uniform(0.5, 2.0, size=m).astype(np.float32)
        w[rng.uniform(size=m) < 0.05] = 0.0
        mode = int(rng.uniform() < uniform_frac)
        items.append(dict(vis=vis, uv=np.stack([u, v], 1).astype(np.float32), w=w, N=int(N), mode=mode,
                          niter=int(rng.integers(1, 60)), freq=1.0e9))
    return _assemble(f"random_{seed}", items)


CONFIGS = {
    "c1": c1_snapshot,
    "c2": c2_muser1_batch,
    "c3": c3_muser2,
    "c4": c4_uneven,
    "c5": c5_differentiable,
}
