"""CPU oracle of the TPC reconstruction chain -- TEST INFRASTRUCTURE ONLY.

A plain, double-precision C implementation (``oracle/oracle.c``) of every
step of the reconstruction path, written from the paper's description of it
and the readings stated in ``oracle.c``'s header, plus this ctypes wrapper.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the GPU library
(``paper_2208_07412_amd``), and the GPU library never calls it.

Every function takes and returns host numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

NROW = 152
_here = os.path.dirname(os.path.abspath(__file__))
_lib = None


def library_path() -> str:
    return os.path.join(_here, "liboracle.so")


def build() -> str:
    """Compile the oracle with gcc (no fast-math: IEEE binary64 throughout)."""
    out = library_path()
    src = os.path.join(_here, "oracle.c")
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-Wall", "-Wextra",
                           "-Wno-unused-parameter", "-o", out + ".tmp", src, "-lm", "-lpthread"])
    os.replace(out + ".tmp", out)
    return out


class OParams(ctypes.Structure):
    _fields_ = [
        ("qmax_min", ctypes.c_int32), ("min_tracklet", ctypes.c_int32),
        ("max_miss", ctypes.c_int32), ("min_track_hits", ctypes.c_int32),
        ("win_y", ctypes.c_int64), ("win_z", ctypes.c_int64), ("s_max", ctypes.c_int64),
        ("chi2_max", ctypes.c_double), ("snp_max", ctypes.c_double), ("bz_b", ctypes.c_double),
        ("c0_snp", ctypes.c_double), ("c0_tgl", ctypes.c_double), ("c0_qpt", ctypes.c_double),
        ("qpt_clamp", ctypes.c_double), ("edge_margin", ctypes.c_double),
        ("lowpt_qpt", ctypes.c_double),
        ("c0r_y", ctypes.c_double), ("c0r_z", ctypes.c_double), ("c0r_snp", ctypes.c_double),
        ("c0r_tgl", ctypes.c_double), ("c0r_qpt", ctypes.c_double),
        ("refit_snp_max", ctypes.c_double),
        ("sigma_y", ctypes.c_double * NROW), ("sigma_z", ctypes.c_double * NROW),
        ("brute_force", ctypes.c_int32), ("n_threads", ctypes.c_int32),
    ]


class OClusters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in (
        "ppad", "ptime", "qtot", "qmax", "nsamp", "sp", "st", "spp", "stt", "flags",
        "pad", "time", "s2pad", "s2time", "y_fx", "z_fx", "sample_label", "crow_start")]


class OFit(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in (
        "hits", "near_tie", "follow_ok", "pb_state", "cluster_owner", "kept", "par", "cov",
        "chi2", "row", "nhits", "flags", "par_cond")]


def default_params(noise_sigma: float = 1.0) -> dict:
    """Reconstruction constants (all readings; the paper gives none).

    The peak threshold scales with the noise: round(5 * sigma_noise).
    """
    return dict(
        qmax_min=int(round(5 * noise_sigma)), min_tracklet=5, max_miss=6, min_track_hits=15,
        win_y=163840, win_z=163840, s_max=1 << 32,
        chi2_max=16.0, snp_max=0.95, bz_b=0.299792458e-3 * 5.0,
        c0_snp=0.1, c0_tgl=0.1, c0_qpt=10.0, qpt_clamp=20.0, edge_margin=1.0, lowpt_qpt=5.0,
        c0r_y=5.0, c0r_z=5.0, c0r_snp=0.5, c0r_tgl=0.5, c0r_qpt=10.0, refit_snp_max=0.999,
        sigma_y=[0.06] * NROW, sigma_z=[0.05] * NROW,
    )


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(library_path()):
        build()
    lib = ctypes.CDLL(library_path())
    P = ctypes.c_void_p
    lib.oracle_geometry.argtypes = [P, P, P]
    lib.oracle_cluster.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, P, P, ctypes.c_int64, P]
    lib.oracle_cluster.restype = ctypes.c_int64
    lib.oracle_find_neighbours.argtypes = [P, ctypes.c_int32, P, P, P, P, P, P]
    lib.oracle_build_tracklets.argtypes = [P, ctypes.c_int64, P, P, P, P, ctypes.c_int64, P, P]
    lib.oracle_build_tracklets.restype = ctypes.c_int64
    lib.oracle_fit_tracks.argtypes = [P, ctypes.c_int32, P, P, P, P, P, ctypes.c_int64, P, P, P]
    lib.oracle_helix_propagate.argtypes = [P, P, ctypes.c_double, ctypes.c_double, P]
    lib.oracle_helix_propagate.restype = ctypes.c_int
    lib.oracle_kalman_fit.argtypes = [P, ctypes.c_int, P, P, P, P, P, P, P, P]
    lib.oracle_kalman_fit.restype = ctypes.c_int
    lib.oracle_seed.argtypes = [P, P, P, ctypes.c_int, ctypes.c_int, P]
    lib.oracle_seed.restype = ctypes.c_int
    lib.oracle_is_pd.argtypes = [P]
    lib.oracle_is_pd.restype = ctypes.c_int
    lib.oracle_decode_zs_pages.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, P, P, P, P, ctypes.c_int64, P]
    lib.oracle_decode_zs_pages.restype = ctypes.c_int
    lib.oracle_compress.argtypes = [P, ctypes.c_int32] + [P] * 6 + [ctypes.c_int64] + [P] * 6 + \
        [P, ctypes.c_int64, P, P]
    lib.oracle_compress.restype = ctypes.c_int
    lib.oracle_decompress.argtypes = [P, P, ctypes.c_int64, ctypes.c_int64] + [P] * 8
    lib.oracle_decompress.restype = ctypes.c_int64
    lib.oracle_track_model.argtypes = [P, P, ctypes.c_int32, ctypes.c_int, ctypes.c_int, P, P, P,
                                       P]
    lib.oracle_track_model.restype = None
    lib.oracle_merge_tracks.argtypes = [P, ctypes.c_int32, P, P, P, ctypes.c_int64, P, P, P, P,
                                        P, P, P]
    lib.oracle_merge_tracks.restype = None
    _lib = lib
    return lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def make_params(params: Optional[dict] = None, brute_force: bool = False,
                n_threads: int = 1) -> OParams:
    d = default_params()
    d.update(params or {})  # a partial dict overrides the defaults
    op = OParams()
    for k, v in d.items():
        if k in ("sigma_y", "sigma_z"):
            arr = getattr(op, k)
            for i in range(NROW):
                arr[i] = float(v[i])
        else:
            setattr(op, k, v)
    op.brute_force = 1 if brute_force else 0
    op.n_threads = int(n_threads)
    return op


def geometry():
    """Oracle geometry: (n_pads[152], X_fx[152], P_fx[152]) in 2^-16 cm."""
    lib = _load()
    npads = np.zeros(NROW, np.int32)
    xfx = np.zeros(NROW, np.int64)
    pfx = np.zeros(NROW, np.int64)
    lib.oracle_geometry(_p(npads), _p(xfx), _p(pfx))
    return npads, xfx, pfx


def cluster(pad, time, adc, row_start, n_units: int, n_time_bins: int,
            params: Optional[dict] = None, labels: bool = False, n_threads: int = 1,
            capacity: Optional[int] = None) -> dict:
    """Clusterize zero-suppressed samples sorted by (unit, row, time, pad)."""
    lib = _load()
    op = make_params(params, n_threads=n_threads)
    pad = np.ascontiguousarray(pad, np.uint16)
    time = np.ascontiguousarray(time, np.uint16)
    adc = np.ascontiguousarray(adc, np.uint16)
    row_start = np.ascontiguousarray(row_start, np.uint32)
    ns = len(pad)
    cap = ns if capacity is None else capacity
    out = dict(
        ppad=np.zeros(cap, np.uint16), ptime=np.zeros(cap, np.uint16),
        qtot=np.zeros(cap, np.uint16), qmax=np.zeros(cap, np.uint16),
        nsamp=np.zeros(cap, np.uint16), sp=np.zeros(cap, np.int32), st=np.zeros(cap, np.int32),
        spp=np.zeros(cap, np.int32), stt=np.zeros(cap, np.int32), flags=np.zeros(cap, np.uint8),
        pad=np.zeros(cap), time=np.zeros(cap), s2pad=np.zeros(cap), s2time=np.zeros(cap),
        y_fx=np.zeros(cap, np.int32), z_fx=np.zeros(cap, np.int32),
    )
    label = np.zeros(max(ns, 1), np.int32) if labels else None
    crow = np.zeros(n_units * NROW + 1, np.uint32)
    oc = OClusters(**{k: _p(v) for k, v in out.items()}, sample_label=_p(label),
                   crow_start=_p(crow))
    n = lib.oracle_cluster(ctypes.byref(op), n_units, n_time_bins, _p(pad), _p(time), _p(adc),
                           _p(row_start), cap, ctypes.byref(oc))
    if n < 0:
        raise ValueError("oracle_cluster: input not sorted by (time, pad) per row or out of range")
    if n > cap:
        raise ValueError(f"oracle_cluster: {n} clusters exceed capacity {cap}")
    res = {k: v[:n].copy() for k, v in out.items()}
    res["crow_start"] = crow
    res["n_units"] = n_units
    if labels:
        res["sample_label"] = label[:ns].copy()
    return res


def find_neighbours(cl: dict, params: Optional[dict] = None, brute_force: bool = False,
                    n_threads: int = 1):
    """Raw CA links (down[], up[]) of every cluster."""
    lib = _load()
    op = make_params(params, brute_force=brute_force, n_threads=n_threads)
    n = len(cl["y_fx"])
    down = np.full(max(n, 1), -1, np.int32)
    up = np.full(max(n, 1), -1, np.int32)
    y = np.ascontiguousarray(cl["y_fx"], np.int32)
    z = np.ascontiguousarray(cl["z_fx"], np.int32)
    pt = np.ascontiguousarray(cl["ptime"], np.uint16)
    crow = np.ascontiguousarray(cl["crow_start"], np.uint32)
    lib.oracle_find_neighbours(ctypes.byref(op), cl["n_units"], _p(y), _p(z), _p(pt), _p(crow),
                               _p(down), _p(up))
    return down[:n].copy(), up[:n].copy()


def build_tracklets(down, up, params: Optional[dict] = None) -> dict:
    lib = _load()
    op = make_params(params)
    n = len(down)
    down = np.ascontiguousarray(down, np.int32)
    up = np.ascontiguousarray(up, np.int32)
    downc = np.full(max(n, 1), -1, np.int32)
    upc = np.full(max(n, 1), -1, np.int32)
    cap = max(n // 2, 1)
    tl_start = np.zeros(cap, np.uint32)
    tl_len = np.zeros(cap, np.uint16)
    nt = lib.oracle_build_tracklets(ctypes.byref(op), n, _p(down), _p(up), _p(downc), _p(upc),
                                    cap, _p(tl_start), _p(tl_len))
    assert nt <= cap
    return dict(downc=downc[:n].copy(), upc=upc[:n].copy(), tl_start=tl_start[:nt].copy(),
                tl_len=tl_len[:nt].copy())


def fit_tracks(cl: dict, tl: dict, params: Optional[dict] = None, brute_force: bool = False,
               n_threads: int = 1, cond: bool = False) -> dict:
    """Following (pass A/B), conflict resolution and refit of all tracklets.

    cond: also return par_cond, the refit from a start scaled by 1 + 2^-24
    (one binary32 rounding unit): how far the FP64 result itself moves under a
    perturbation of that size (NaN where that refit fails)."""
    lib = _load()
    op = make_params(params, brute_force=brute_force, n_threads=n_threads)
    nt = len(tl["tl_start"])
    nc = len(cl["y_fx"])
    m = max(nt, 1)
    out = dict(hits=np.full(m * NROW, -1, np.int32), near_tie=np.zeros(m, np.int32),
               follow_ok=np.zeros(m, np.int32), pb_state=np.zeros(m * 6),
               cluster_owner=np.full(max(nc, 1), -1, np.int32), kept=np.zeros(m, np.int32),
               par=np.zeros(m * 5), cov=np.zeros(m * 15), chi2=np.zeros(m),
               row=np.full(m, -1, np.int32), nhits=np.zeros(m, np.int32),
               flags=np.zeros(m, np.int32))
    if cond:
        out["par_cond"] = np.zeros(m * 5)
    of = OFit(**{k: _p(v) for k, v in out.items()})
    y = np.ascontiguousarray(cl["y_fx"], np.int32)
    z = np.ascontiguousarray(cl["z_fx"], np.int32)
    pt = np.ascontiguousarray(cl["ptime"], np.uint16)
    crow = np.ascontiguousarray(cl["crow_start"], np.uint32)
    upc = np.ascontiguousarray(tl["upc"], np.int32)
    ts = np.ascontiguousarray(tl["tl_start"], np.uint32)
    tln = np.ascontiguousarray(tl["tl_len"], np.uint16)
    lib.oracle_fit_tracks(ctypes.byref(op), cl["n_units"], _p(y), _p(z), _p(pt), _p(crow),
                          _p(upc), nt, _p(ts), _p(tln), ctypes.byref(of))
    res = {k: v for k, v in out.items()}
    res["hits"] = out["hits"][: nt * NROW].reshape(nt, NROW)
    res["pb_state"] = out["pb_state"][: nt * 6].reshape(nt, 6)
    res["par"] = out["par"][: nt * 5].reshape(nt, 5)
    res["cov"] = out["cov"][: nt * 15].reshape(nt, 15)
    if cond:
        res["par_cond"] = out["par_cond"][: nt * 5].reshape(nt, 5)
    for k in ("near_tie", "follow_ok", "kept", "chi2", "row", "nhits", "flags"):
        res[k] = out[k][:nt]
    res["cluster_owner"] = out["cluster_owner"][:nc]
    return res


def process(pad, time, adc, row_start, n_units: int, n_time_bins: int,
            params: Optional[dict] = None, n_threads: int = 1, labels: bool = False,
            cond: bool = False) -> dict:
    """The whole chain: clusters, links, tracklets, tracks (cond: see fit_tracks)."""
    cl = cluster(pad, time, adc, row_start, n_units, n_time_bins, params, labels=labels,
                 n_threads=n_threads)
    down, up = find_neighbours(cl, params, n_threads=n_threads)
    tl = build_tracklets(down, up, params)
    fit = fit_tracks(cl, tl, params, n_threads=n_threads, cond=cond)
    return dict(clusters=cl, down=down, up=up, tracklets=tl, fit=fit)


# -------------------------------------------------------------- primitives
def helix_propagate(p, x1: float, x2: float, params: Optional[dict] = None, jacobian=False):
    lib = _load()
    op = make_params(params)
    p = np.array(p, dtype=np.float64)
    J = np.zeros(25) if jacobian else None
    rc = lib.oracle_helix_propagate(ctypes.byref(op), _p(p), x1, x2, _p(J))
    if jacobian:
        return rc, p, J.reshape(5, 5)
    return rc, p


def kalman_fit(rows, my, mz, vy, vz, p0, C0, params: Optional[dict] = None):
    lib = _load()
    op = make_params(params)
    n = len(rows)
    rows = np.ascontiguousarray(rows, np.int32)
    arrs = [np.ascontiguousarray(a, np.float64) for a in (my, mz, vy, vz)]
    p = np.array(p0, dtype=np.float64)
    C = np.array(C0, dtype=np.float64).reshape(25).copy()
    chi2 = np.zeros(1)
    rc = lib.oracle_kalman_fit(ctypes.byref(op), n, _p(rows), *[_p(a) for a in arrs], _p(p),
                               _p(C), _p(chi2))
    return rc, p, C.reshape(5, 5), float(chi2[0])


def seed(y_fx, z_fx, r1: int, params: Optional[dict] = None):
    lib = _load()
    op = make_params(params)
    y = np.ascontiguousarray(y_fx, np.int32)
    z = np.ascontiguousarray(z_fx, np.int32)
    p = np.zeros(5)
    rc = lib.oracle_seed(ctypes.byref(op), _p(y), _p(z), r1, len(y), _p(p))
    return rc, p


def is_pd(C) -> bool:
    lib = _load()
    c = np.ascontiguousarray(np.asarray(C, np.float64).reshape(25))
    return bool(lib.oracle_is_pd(_p(c)))


# ---------------------------------------------------------------- QC
QC_QTOT, QC_QMAX, QC_NHITS, QC_ATTACH, QC_BINS = 0, 256, 512, 665, 667


def qc_histograms(qtot, qmax, cluster_track, hit_start) -> np.ndarray:
    """Quality-control histograms of a reconstruction's outputs.  The paper
    (section "Software") says the synchronous processing validates the
    detector data in real time but names no quantities; these are chosen
    here: clusters by total charge (bin min(qtot >> 3, 255)), by peak charge
    (bin min(qmax >> 2, 255)), tracks by hit count (hit_start[j+1] -
    hit_start[j], 0..152) and clusters off / on a track (cluster_track -1 /
    >= 0), at the bin offsets QC_QTOT, QC_QMAX, QC_NHITS, QC_ATTACH."""
    qtot = np.asarray(qtot, np.int64)
    qmax = np.asarray(qmax, np.int64)
    ct = np.asarray(cluster_track, np.int64)
    hs = np.asarray(hit_start, np.int64)
    h = np.zeros(QC_BINS, np.int64)
    h[QC_QTOT:QC_QTOT + 256] = np.bincount(np.minimum(qtot >> 3, 255), minlength=256)
    h[QC_QMAX:QC_QMAX + 256] = np.bincount(np.minimum(qmax >> 2, 255), minlength=256)
    h[QC_NHITS:QC_NHITS + NROW + 1] = np.bincount(np.minimum(np.diff(hs), NROW),
                                                  minlength=NROW + 1)
    h[QC_ATTACH:QC_ATTACH + 2] = np.bincount((ct >= 0).astype(np.int64), minlength=2)
    return h


ZS_PAGE_WORDS = 2048


def decode_zs_pages(pages, n_units: int, n_time_bins: int, validate: bool = False,
                    capacity: Optional[int] = None) -> dict:
    """Raw zero-suppressed pages (uint32, n_pages x 2048 words) -> samples in
    the clusterizer's input layout: pad, time, adc, row_start, and the status
    (0; -3 malformed input; -2 more samples than `capacity`)."""
    lib = _load()
    pg = np.ascontiguousarray(pages, np.uint32).reshape(-1, ZS_PAGE_WORDS)
    n_pages = pg.shape[0]
    cap = int(n_pages * ZS_PAGE_WORDS * 32 // 10) if capacity is None else int(capacity)
    pad = np.zeros(max(cap, 1), np.uint16)
    time = np.zeros(max(cap, 1), np.uint16)
    adc = np.zeros(max(cap, 1), np.uint16)
    rs = np.zeros(n_units * NROW + 1, np.uint32)
    n = ctypes.c_int64(0)
    st = lib.oracle_decode_zs_pages(_p(pg), n_pages, n_units, n_time_bins, 1 if validate else 0,
                                    _p(pad), _p(time), _p(adc), _p(rs), cap, ctypes.byref(n))
    m = min(n.value, cap)
    return dict(status=st, n_samples=n.value, pad=pad[:m].copy(), time=time[:m].copy(),
                adc=adc[:m].copy(), row_start=rs)


def tracks_from_fit(res: dict) -> dict:
    """The oracle's kept tracks in the library's output layout: ascending
    tracklet order, parameters rounded to float32, kept hits in ascending
    row, z anchor (drift z of the tracklet start), and the cluster -> track
    map."""
    fit = res["fit"]
    cl = res["clusters"]
    ts = res["tracklets"]["tl_start"]
    owner = fit["cluster_owner"]
    kept = np.nonzero(fit["kept"])[0]
    hs, hits = [0], []
    for t in kept:
        h = fit["hits"][t]
        h = h[h >= 0]  # one per row, ascending row
        h = h[owner[h] == t]
        hits.append(h)
        hs.append(hs[-1] + len(h))
    idx = np.full(len(fit["kept"]), -1, np.int64)
    idx[kept] = np.arange(len(kept))
    ct = np.where(owner >= 0, idx[np.maximum(owner, 0)], -1).astype(np.int32)
    return dict(tracklet=kept.astype(np.uint32), par=fit["par"][kept].astype(np.float32),
                row=fit["row"][kept].astype(np.uint8),
                z_anchor=cl["z_fx"][ts[kept]].astype(np.int32),
                hit_start=np.array(hs, np.uint32),
                hits=(np.concatenate(hits) if hits else np.zeros(0)).astype(np.uint32),
                cluster_track=ct)


def compress(clusters: dict, tracks: dict, n_units: int, params: Optional[dict] = None,
             capacity_words: Optional[int] = None) -> dict:
    """Track-model compression of a frame's clusters: the stream (uint32
    words), its status (0; -2 capacity; -3 input the format cannot hold) and
    the residual histograms (bins [0,128) y, [128,256) z)."""
    lib = _load()
    op = make_params(params)
    crow = np.ascontiguousarray(clusters["crow_start"], np.uint32)
    y = np.ascontiguousarray(clusters["y_fx"], np.int32)
    z = np.ascontiguousarray(clusters["z_fx"], np.int32)
    qt = np.ascontiguousarray(clusters["qtot"], np.uint16)
    qm = np.ascontiguousarray(clusters["qmax"], np.uint16)
    fl = np.ascontiguousarray(clusters["flags"], np.uint8)
    n_tr = len(tracks["hit_start"]) - 1
    par = np.ascontiguousarray(tracks["par"], np.float32).reshape(-1)
    za = np.ascontiguousarray(tracks["z_anchor"], np.int32)
    row = np.ascontiguousarray(tracks["row"], np.uint8)
    hs = np.ascontiguousarray(tracks["hit_start"], np.uint32)
    hits = np.ascontiguousarray(tracks["hits"], np.uint32)
    ct = np.ascontiguousarray(tracks["cluster_track"], np.int32)
    nc = len(y)
    cap = capacity_words if capacity_words is not None else \
        64 + (n_tr + 1) + n_units * NROW + 1 + (nc * 200 + n_tr * 200) // 32
    out = np.zeros(max(cap, 1), np.uint32)
    hist = np.zeros(256, np.int64)
    nw = ctypes.c_int64(0)
    st = lib.oracle_compress(ctypes.byref(op), n_units, _p(crow), _p(y), _p(z), _p(qt), _p(qm),
                             _p(fl), n_tr, _p(par), _p(za), _p(row), _p(hs), _p(hits), _p(ct),
                             _p(out), cap, ctypes.byref(nw), _p(hist))
    return dict(status=st, words=out[:nw.value].copy() if st == 0 else None,
                n_words=nw.value, hist=hist)


def decompress(words, params: Optional[dict] = None, capacity: Optional[int] = None) -> dict:
    """Decoded clusters in stream order (unit, row, quantised y_fx and z_fx,
    qtot, qmax, flags, track index or -1); status = count, or -2 / -3."""
    lib = _load()
    op = make_params(params)
    w = np.ascontiguousarray(words, np.uint32)
    nc = int(w[4]) if len(w) > 4 else 0
    cap = nc if capacity is None else capacity
    m = max(cap, 1)
    out = dict(unit=np.zeros(m, np.uint16), row=np.zeros(m, np.uint8),
               y_fx=np.zeros(m, np.int32), z_fx=np.zeros(m, np.int32),
               qtot=np.zeros(m, np.uint16), qmax=np.zeros(m, np.uint16),
               flags=np.zeros(m, np.uint8), track=np.zeros(m, np.int32))
    n = lib.oracle_decompress(ctypes.byref(op), _p(w), len(w), cap,
                              *[_p(out[k]) for k in ("unit", "row", "y_fx", "z_fx", "qtot",
                                                      "qmax", "flags", "track")])
    res = {k: v[:max(n, 0)].copy() for k, v in out.items()}
    res["status"] = int(n) if n < 0 else 0
    return res


def track_model(par, z_anchor: int, row0: int, rows, params: Optional[dict] = None):
    """The codec's integer helix at the given rows (ascending): y, z in
    2^-16 cm and whether the model had stopped (|sin phi| near 1)."""
    lib = _load()
    op = make_params(params)
    p = np.ascontiguousarray(par, np.float32)
    rows = np.ascontiguousarray(rows, np.int32)
    n = len(rows)
    y = np.zeros(n, np.int64)
    z = np.zeros(n, np.int64)
    fr = np.zeros(n, np.int32)
    lib.oracle_track_model(ctypes.byref(op), _p(p), int(z_anchor), int(row0), n, _p(rows), _p(y),
                           _p(z), _p(fr))
    return y, z, fr


MERGE_FIT_FIELDS = ("n_segments", "n_hits", "xc", "yc", "radius", "dzdpsi", "zd_axis", "t0",
                    "tgl", "flags", "turn")


def merge_tracks(clusters: dict, tracks: dict, n_units: int,
                 params: Optional[dict] = None) -> dict:
    """Segments joined into tracks (cross-sector, looper legs), with the
    merged helix fit and T0: label per segment (the component's smallest
    segment index), near_tie per segment, and per component (at its label)
    the fields of MERGE_FIT_FIELDS."""
    lib = _load()
    op = make_params(params)
    crow = np.ascontiguousarray(clusters["crow_start"], np.uint32)
    y = np.ascontiguousarray(clusters["y_fx"], np.int32)
    z = np.ascontiguousarray(clusters["z_fx"], np.int32)
    n = len(tracks["hit_start"]) - 1
    par = np.ascontiguousarray(tracks["par"], np.float32).reshape(-1)
    row = np.ascontiguousarray(tracks["row"], np.uint8)
    hs = np.ascontiguousarray(tracks["hit_start"], np.uint32)
    hits = np.ascontiguousarray(tracks["hits"], np.uint32)
    label = np.zeros(max(n, 1), np.int64)
    tie = np.zeros(max(n, 1), np.int32)
    fit = np.zeros(max(n, 1) * 12)
    lib.oracle_merge_tracks(ctypes.byref(op), n_units, _p(crow), _p(y), _p(z), n, _p(par), _p(row),
                            _p(hs), _p(hits), _p(label), _p(tie), _p(fit))
    f = fit[:n * 12].reshape(n, 12)
    out = dict(label=label[:n].copy(), near_tie=tie[:n].astype(bool))
    for i, k in enumerate(MERGE_FIT_FIELDS):
        out[k] = f[:, i].copy()
    return out
