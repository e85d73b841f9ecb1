"""Seeded synthetic Pb-Pb-shaped TPC input generator.

Input side only: it produces zero-suppressed (ZS) ADC samples and the
generator truth that goes with them.  Both the CPU oracle and the GPU library
consume its arrays; it holds none of the reconstruction arithmetic
(clusterization, neighbour finding, seeding, fitting).

The paper (Hardware and data flow; Software) says the TPC data of complete
collisions is zero-suppressed on the readout FPGA and reconstructed on the
EPN GPUs, but specifies no detector model or event shapes.  The model used
here (geometry, drift, charge, noise, kinematics) is stated in
``tpcsynth/csrc/synth.c``.

Layout of a generated ZS input (all numpy, host memory)::

    pad, time, adc : uint16[n_samples]   sorted by (unit, row, time, pad)
    row_start      : uint32[n_units*152 + 1]
    n_units        : int (unit u is sector u % 36 of its chunk)
    n_time_bins    : int
"""
from __future__ import annotations

import ctypes
import dataclasses
import math
import os
from typing import List, Optional

import numpy as np

NROW = 152
NPAD_MAX = 138
BZ_B = 0.299792458e-3 * 5.0  # curvature per (GeV/c)^-1 per cm at Bz = 0.5 T

_here = os.path.dirname(os.path.abspath(__file__))
_lib = None


def library_path() -> str:
    return os.path.join(_here, "libtpcsynth.so")


def build() -> str:
    """Compile the native generator core with gcc (OpenMP)."""
    import subprocess

    out = library_path()
    src = os.path.join(_here, "csrc", "synth.c")
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                           "-o", out + ".tmp", src, "-lm"])
    os.replace(out + ".tmp", out)
    return out


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        build()
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.synth_geometry.argtypes = [P, P, P]
    lib.synth_crossings.argtypes = [ctypes.c_int64] + [P] * 7 + [ctypes.c_int32, ctypes.c_int32] + [P] * 12
    lib.synth_crossings.restype = None
    lib.synth_digitize.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, P, ctypes.c_double,
                                   ctypes.c_double, P, ctypes.c_uint64, P]
    lib.synth_digitize.restype = ctypes.c_int64
    lib.synth_digitize_fetch.argtypes = [P, P, P]
    lib.synth_pack_pages.argtypes = [ctypes.c_int32, P, P, P, P, P]
    lib.synth_pack_pages.restype = ctypes.c_int64
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def geometry():
    """Generator-side detector geometry: (x_r [cm], pitch_r [cm], n_pads_r)."""
    lib = _load()
    x = np.zeros(NROW)
    pitch = np.zeros(NROW)
    npads = np.zeros(NROW, dtype=np.int32)
    lib.synth_geometry(_ptr(x), _ptr(pitch), _ptr(npads))
    return x, pitch, npads


# --------------------------------------------------------------- configs
@dataclasses.dataclass
class Collision:
    t0: float
    n_prim: int
    n_sec: int


@dataclasses.dataclass
class EventConfig:
    name: str
    n_time_bins: int
    collisions: List[Collision]
    sector_mode: int = 0            # 0: 36 sectors, 1: sector 0 only (entry-azimuth rule)
    eta_min: float = -0.9
    eta_max: float = 0.9
    pt_min: float = 0.1
    pt_max: float = 10.0
    low_pt_frac: float = 0.0        # fraction of tracks with pT ~ U(0.05, 0.2)
    sigma_noise: float = 1.0
    dead_frac: float = 0.0
    sec_decay_cm: float = 5.0

    @property
    def n_units(self) -> int:
        return 1 if self.sector_mode == 1 else 36


@dataclasses.dataclass
class Event:
    config: EventConfig
    pad: np.ndarray
    time: np.ndarray
    adc: np.ndarray
    row_start: np.ndarray
    n_units: int
    n_time_bins: int
    tracks: dict
    deposits: dict
    dead: Optional[np.ndarray]

    @property
    def n_samples(self) -> int:
        return int(self.pad.shape[0])


def config_c1() -> EventConfig:
    """One sector, 200 tracks from the origin, 500 time bins."""
    return EventConfig("C1", 500, [Collision(0.0, 200, 0)], sector_mode=1, eta_min=0.0)


def config_c2() -> EventConfig:
    """One central-like collision: 3000 primaries + 600 displaced secondaries."""
    return EventConfig("C2", 500, [Collision(0.0, 3000, 600)])


def glauber_like_multiplicity(rng: np.random.Generator, n: int) -> np.ndarray:
    """dN/deta = 20 + 1580 (1-c)^2 with c = b^2/b_max^2 ~ U(0,1)."""
    c = rng.random(n)
    return 20.0 + 1580.0 * (1.0 - c) ** 2


def _collisions(rng: np.random.Generator, n_coll: int, t0_span: float) -> List[Collision]:
    t0 = rng.random(n_coll) * t0_span
    dndeta = glauber_like_multiplicity(rng, n_coll)
    nprim = rng.poisson(1.8 * dndeta)
    return [Collision(float(t0[i]), int(nprim[i]), int(round(0.2 * nprim[i])))
            for i in range(n_coll)]


def config_c3(seed: int = 303, n_coll: int = 100) -> EventConfig:
    """2 ms slice at 50 kHz: 100 minimum-bias collisions over 10,500 bins."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, 3]))
    return EventConfig("C3", 10000 + 500, _collisions(rng, n_coll, 10000.0))


def config_chunk(seed: int, index: int, stress: bool = False,
                 n_coll: Optional[int] = None) -> EventConfig:
    """Serving-stream chunk: n ~ U{10..200} collisions, 100 n + 500 bins.

    ``stress`` gives the precision-stress variant: 30% of tracks at
    pT ~ U(0.05, 0.2), noise sigma 2 ADC and 10% dead pads.
    """
    ss = np.random.SeedSequence(seed).spawn(index + 1)[index]
    rng = np.random.default_rng(ss.spawn(1)[0])
    n = int(rng.integers(10, 201)) if n_coll is None else int(n_coll)
    cfg = EventConfig(("C5" if stress else "C4") + f"[{index}]", 100 * n + 500,
                      _collisions(rng, n, 100.0 * n))
    if stress:
        cfg.low_pt_frac = 0.3
        cfg.sigma_noise = 2.0
        cfg.dead_frac = 0.1
    return cfg


def config_small(n_tracks: int, n_time_bins: int = 500, sector_mode: int = 1,
                 n_sec: int = 0, sigma_noise: float = 1.0, t0: float = 0.0) -> EventConfig:
    """Small events for tests: n_tracks primaries (entry-azimuth rule if sector_mode 1)."""
    return EventConfig(f"small{n_tracks}", n_time_bins, [Collision(t0, n_tracks, n_sec)],
                       sector_mode=sector_mode, eta_min=0.0 if sector_mode == 1 else -0.9,
                       sigma_noise=sigma_noise)


# ------------------------------------------------------------ kinematics
def sample_pt_powerlaw(rng: np.random.Generator, n: int, a: float = 0.1, b: float = 10.0) -> np.ndarray:
    """pT with pdf ~ pT^-3 on [a, b], by inverse CDF."""
    u = rng.random(n)
    return (a ** -2 - u * (a ** -2 - b ** -2)) ** -0.5


def _tracks(cfg: EventConfig, rng: np.random.Generator) -> dict:
    cols = []
    for ic, col in enumerate(cfg.collisions):
        n = col.n_prim + col.n_sec
        if n == 0:
            continue
        pt = sample_pt_powerlaw(rng, n, cfg.pt_min, cfg.pt_max)
        if cfg.low_pt_frac > 0:
            low = rng.random(n) < cfg.low_pt_frac
            pt = np.where(low, rng.uniform(0.05, 0.2, n), pt)
        eta = rng.uniform(cfg.eta_min, cfg.eta_max, n)
        phi = rng.uniform(0.0, 2.0 * math.pi, n)
        q = np.where(rng.random(n) < 0.5, -1.0, 1.0)
        curv = -q * BZ_B / pt
        prim = np.arange(n) < col.n_prim
        vx = np.zeros(n)
        vy = np.zeros(n)
        vz = np.zeros(n)
        if col.n_sec:
            ns = col.n_sec
            d = rng.exponential(cfg.sec_decay_cm, ns)
            veta = rng.uniform(cfg.eta_min, cfg.eta_max, ns)
            vphi = rng.uniform(0.0, 2.0 * math.pi, ns)
            th = 2.0 * np.arctan(np.exp(-veta))
            vx[col.n_prim:] = d * np.sin(th) * np.cos(vphi)
            vy[col.n_prim:] = d * np.sin(th) * np.sin(vphi)
            vz[col.n_prim:] = d * np.cos(th)
        if cfg.sector_mode == 1:
            # azimuth where the track crosses rho = 85 cm is uniform in sector 0
            phi85 = rng.uniform(0.0, math.radians(20.0), n)
            phi = phi85 - np.sign(curv) * np.arcsin(np.minimum(85.0 * np.abs(curv) / 2.0, 1.0))
        cols.append(dict(pt=pt, eta=eta, phi0=phi, q=q, curv=curv, tgl=np.sinh(eta),
                         vx=vx, vy=vy, vz=vz, primary=prim,
                         collision=np.full(n, ic, dtype=np.int32),
                         t0=np.full(n, col.t0)))
    if not cols:
        keys = ["pt", "eta", "phi0", "q", "curv", "tgl", "vx", "vy", "vz", "t0"]
        out = {k: np.zeros(0) for k in keys}
        out["primary"] = np.zeros(0, dtype=bool)
        out["collision"] = np.zeros(0, dtype=np.int32)
        return out
    return {k: np.concatenate([c[k] for c in cols]) for k in cols[0]}


def crossings(tr: dict, sector_mode: int, n_time_bins: int) -> dict:
    """Exact helix / row-plane crossings of every track (track-major, by arc)."""
    lib = _load()
    n = len(tr["curv"])
    counts = np.zeros(n, dtype=np.int64)
    args = [np.ascontiguousarray(tr[k], dtype=np.float64)
            for k in ("vx", "vy", "vz", "phi0", "curv", "tgl", "t0")]
    nul = [None] * 10
    lib.synth_crossings(n, *[_ptr(a) for a in args], sector_mode, n_time_bins,
                        _ptr(counts), None, *nul)
    offsets = np.zeros(n, dtype=np.int64)
    if n:
        offsets[1:] = np.cumsum(counts)[:-1]
    m = int(counts.sum())
    out = dict(track=np.zeros(m, np.int32), unit=np.zeros(m, np.int32), row=np.zeros(m, np.int32),
               leg=np.zeros(m, np.int32), y=np.zeros(m), z=np.zeros(m), snp=np.zeros(m),
               mu_pad=np.zeros(m), mu_time=np.zeros(m), s=np.zeros(m))
    order = ["track", "unit", "row", "leg", "y", "z", "snp", "mu_pad", "mu_time", "s"]
    lib.synth_crossings(n, *[_ptr(a) for a in args], sector_mode, n_time_bins,
                        _ptr(counts), _ptr(offsets), *[_ptr(out[k]) for k in order])
    return out


def landau_charge(rng: np.random.Generator, n: int, mpv: float = 100.0, xi: float = 10.0,
                  qmax: float = 5000.0) -> np.ndarray:
    """Landau-distributed deposit charge (ADC units) with MPV 100 and width 10."""
    import scipy.stats as st

    if n == 0:
        return np.zeros(0)
    q = st.landau.rvs(loc=mpv + 0.22278 * xi, scale=xi, size=n, random_state=rng)
    return np.clip(q, 0.0, qmax)


def generate(cfg: EventConfig, seed: int) -> Event:
    """Generate one event (time frame / chunk) from a config and a seed."""
    lib = _load()
    ss = np.random.SeedSequence(seed)
    s_kin, s_q, s_dig, s_dead = ss.spawn(4)
    tr = _tracks(cfg, np.random.default_rng(s_kin))
    dep = crossings(tr, cfg.sector_mode, cfg.n_time_bins)
    ndep = len(dep["track"])
    dep["q"] = landau_charge(np.random.default_rng(s_q), ndep)
    dep["id"] = np.arange(ndep, dtype=np.int64)
    n_units = cfg.n_units
    # group deposits by (unit,row) for the digitizer (stable: keeps id order)
    ur = dep["unit"].astype(np.int64) * NROW + dep["row"]
    order = np.argsort(ur, kind="stable")
    dep_start = np.zeros(n_units * NROW + 1, dtype=np.int64)
    np.add.at(dep_start, ur + 1, 1)
    dep_start = np.cumsum(dep_start)
    dead = None
    if cfg.dead_frac > 0:
        dead = (np.random.default_rng(s_dead).random(n_units * NROW * NPAD_MAX)
                < cfg.dead_frac).astype(np.uint8)
    row_counts = np.zeros(n_units * NROW, dtype=np.int64)
    mu_pad = np.ascontiguousarray(dep["mu_pad"][order])
    mu_time = np.ascontiguousarray(dep["mu_time"][order])
    qq = np.ascontiguousarray(dep["q"][order])
    dig_seed = int(np.random.default_rng(s_dig).integers(0, 2 ** 63))
    total = lib.synth_digitize(n_units, cfg.n_time_bins, _ptr(dep_start), _ptr(mu_pad),
                               _ptr(mu_time), _ptr(qq), 0.8, cfg.sigma_noise, _ptr(dead),
                               dig_seed, _ptr(row_counts))
    pad = np.empty(total, np.uint16)
    time = np.empty(total, np.uint16)
    adc = np.empty(total, np.uint16)
    lib.synth_digitize_fetch(_ptr(pad), _ptr(time), _ptr(adc))
    row_start = np.zeros(n_units * NROW + 1, dtype=np.uint32)
    row_start[1:] = np.cumsum(row_counts)
    return Event(cfg, pad, time, adc, row_start, n_units, cfg.n_time_bins, tr, dep, dead)


def stack(events: List[Event]) -> Event:
    """Concatenate events unit-wise, so that many chunks form one batch.

    Units stay independent; the batch has sum(n_units) units and the largest
    time range of its members.
    """
    pad = np.concatenate([e.pad for e in events])
    time = np.concatenate([e.time for e in events])
    adc = np.concatenate([e.adc for e in events])
    rs = [np.zeros(1, np.uint64)]
    off = 0
    for e in events:
        rs.append(e.row_start[1:].astype(np.uint64) + off)
        off += e.n_samples
    row_start = np.concatenate(rs).astype(np.uint32)
    n_units = sum(e.n_units for e in events)
    T = max(e.n_time_bins for e in events)
    return Event(events[0].config, pad, time, adc, row_start, n_units, T, {}, {}, None)


def select_units(ev: Event, units: List[int]) -> Event:
    """The given units of an event, as an event of their own (same time range).

    Used to cut a bounded sample out of a large frame; units are independent,
    so every unit reconstructs the same alone as inside its frame.
    """
    rs = ev.row_start.astype(np.int64)
    parts, starts = [], [np.zeros(1, np.int64)]
    off = 0
    for u in units:
        a, b = int(rs[u * NROW]), int(rs[(u + 1) * NROW])
        parts.append((a, b))
        starts.append(rs[u * NROW + 1:(u + 1) * NROW + 1] - a + off)
        off += b - a
    idx = np.concatenate([np.arange(a, b) for a, b in parts]) if parts else np.zeros(0, np.int64)
    dep = {}
    if ev.deposits:
        # the deposits of the chosen units, renumbered to their new unit index
        newu = np.full(int(ev.n_units), -1, np.int64)
        newu[np.asarray(units, np.int64)] = np.arange(len(units))
        m = newu[ev.deposits["unit"].astype(np.int64)] >= 0
        dep = {k: v[m] for k, v in ev.deposits.items()}
        dep["unit"] = newu[ev.deposits["unit"][m].astype(np.int64)].astype(
            ev.deposits["unit"].dtype)
        if "id" in dep:  # ids are positions; renumbering keeps their order
            dep["id"] = np.arange(int(m.sum()), dtype=ev.deposits["id"].dtype)
    return Event(ev.config, ev.pad[idx], ev.time[idx], ev.adc[idx],
                 np.concatenate(starts).astype(np.uint32), len(units), ev.n_time_bins,
                 ev.tracks, dep, None)


PAGE_WORDS = 2048


def zs_pages(ev: Event) -> np.ndarray:
    """The event's samples packed into raw zero-suppressed pages (uint32
    [n_pages, 2048]): the input format of the library's page decoder, as a
    readout card would ship it.  One (unit, row) per page, runs of
    consecutive pads per time bin, 10-bit ADC fields."""
    lib = _load()
    rs = np.ascontiguousarray(ev.row_start, np.uint32)
    pad = np.ascontiguousarray(ev.pad, np.uint16)
    time = np.ascontiguousarray(ev.time, np.uint16)
    adc = np.ascontiguousarray(ev.adc, np.uint16)
    n = lib.synth_pack_pages(ev.n_units, _ptr(rs), _ptr(pad), _ptr(time), _ptr(adc), None)
    out = np.zeros((max(n, 0), PAGE_WORDS), np.uint32)
    if n > 0:
        lib.synth_pack_pages(ev.n_units, _ptr(rs), _ptr(pad), _ptr(time), _ptr(adc), _ptr(out))
    return out
