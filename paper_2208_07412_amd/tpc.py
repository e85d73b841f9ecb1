"""Python binding of libtpcreco (include/tpc.h): argument marshalling only.

Device memory comes from torch tensors on the GPU, the stream is torch's
current stream; every step of the reconstruction runs in the library's HIP
kernels.  There is no CPU fallback: if the library is missing, loading it
raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np

NROW = 152
_here = os.path.dirname(os.path.abspath(__file__))
_lib = None

P = ctypes.c_void_p
U32 = ctypes.c_uint32
I32 = ctypes.c_int32


class TpcParams(ctypes.Structure):
    _fields_ = [
        ("qmax_min", I32), ("min_tracklet", I32), ("max_miss", I32), ("min_track_hits", I32),
        ("win_y", ctypes.c_int64), ("win_z", ctypes.c_int64), ("s_max", ctypes.c_int64),
        ("chi2_max", ctypes.c_double), ("snp_max", ctypes.c_double), ("bz_b", ctypes.c_double),
        ("c0_snp", ctypes.c_double), ("c0_tgl", ctypes.c_double), ("c0_qpt", ctypes.c_double),
        ("qpt_clamp", ctypes.c_double), ("edge_margin", ctypes.c_double),
        ("lowpt_qpt", ctypes.c_double),
        ("c0r_y", ctypes.c_double), ("c0r_z", ctypes.c_double), ("c0r_snp", ctypes.c_double),
        ("c0r_tgl", ctypes.c_double), ("c0r_qpt", ctypes.c_double),
        ("refit_snp_max", ctypes.c_double),
        ("sigma_y", ctypes.c_double * NROW), ("sigma_z", ctypes.c_double * NROW),
        ("validate", I32), ("force_fallback", I32),
    ]


class TpcSizes(ctypes.Structure):
    _fields_ = [("max_units", U32), ("max_time_bins", U32), ("max_clusters", U32),
                ("max_tracklets", U32), ("max_samples", U32)]


class TpcZsInput(ctypes.Structure):
    _fields_ = [("pad", P), ("time", P), ("adc", P), ("row_start", P), ("n_samples", U32),
                ("n_units", U32), ("n_time_bins", U32)]


class TpcZsSoa(ctypes.Structure):
    _fields_ = [("capacity", U32), ("n_units", U32), ("n_time_bins", U32), ("n_samples", P),
                ("pad", P), ("time", P), ("adc", P), ("row_start", P)]


class TpcCompressed(ctypes.Structure):
    _fields_ = [("capacity", U32), ("stream", P), ("n_words", P), ("res_hist", P)]


class TpcDecoded(ctypes.Structure):
    _fields_ = [("capacity", U32), ("n_clusters", P), ("unit", P), ("row", P), ("y_fx", P),
                ("z_fx", P), ("qtot", P), ("qmax", P), ("flags", P), ("track", P)]


class TpcMerged(ctypes.Structure):
    _fields_ = [("capacity", U32), ("n_merged", P), ("label", P), ("near_tie", P), ("fit", P)]


class TpcClusters(ctypes.Structure):
    _fields_ = [("capacity", U32), ("n_units", U32), ("n_time_bins", U32), ("n_clusters", P),
                ("crow_start", P), ("y_fx", P), ("z_fx", P), ("dpad", P), ("dtime", P),
                ("s2pad", P), ("s2time", P), ("qtot", P), ("qmax", P), ("ppad", P), ("ptime", P),
                ("flags", P), ("sp", P), ("st", P), ("spp", P), ("stt", P), ("nsamp", P),
                ("sample_label", P)]


class TpcLinks(ctypes.Structure):
    _fields_ = [("capacity", U32), ("down", P), ("up", P), ("downc", P), ("upc", P)]


class TpcTracklets(ctypes.Structure):
    _fields_ = [("capacity", U32), ("n_tracklets", P), ("start", P), ("len", P)]


class TpcTracks(ctypes.Structure):
    _fields_ = [("capacity", U32), ("hit_capacity", U32), ("n_tracks", P), ("n_hits", P),
                ("tracklet", P), ("par", P), ("cov", P), ("chi2", P), ("ndf", P), ("row", P),
                ("flags", P), ("z_anchor", P), ("hit_start", P), ("hits", P),
                ("cluster_track", P), ("follow_hits", P)]


# capacities named by tpc_counts.overflow (bit k) and required_by[k]
OVERFLOW_KINDS = ("clusters", "tracklets", "tracks", "hits")


class TpcCounts(ctypes.Structure):
    _fields_ = [("status", I32), ("required", U32), ("n_samples", U32), ("n_clusters", U32),
                ("n_tracklets", U32), ("n_tracks", U32), ("n_hits", U32), ("n_fallback", U32),
                ("n_fallback_fail", U32), ("n_not_pd", U32), ("n_refit_fail", U32),
                ("overflow", U32), ("required_by", U32 * 4), ("follow_steps", ctypes.c_uint64),
                ("follow_candidates", ctypes.c_uint64), ("follow_updates", ctypes.c_uint64),
                ("follow_lane_slots", ctypes.c_uint64)]


class TpcTuning(ctypes.Structure):
    _fields_ = [("cl_window", I32), ("cl_chunk", I32), ("follow_block", I32), ("follow_mode", I32),
                ("refit_waves", I32), ("cl_mode", I32)]


EXPORTS = ["tpc_params_default", "tpc_geometry", "tpc_workspace_size", "tpc_create",
           "tpc_destroy", "tpc_cluster", "tpc_find_neighbours", "tpc_build_tracklets",
           "tpc_fit_tracks", "tpc_process_timeframe", "tpc_sync", "tpc_stream",
           "tpc_status_string", "tpc_profile_enable", "tpc_profile_read",
           "tpc_profile_stage_name", "tpc_tuning_default", "tpc_set_tuning", "tpc_get_tuning",
           "tpc_qc_histograms", "tpc_qc_histograms_noalloc", "tpc_decode_zs_pages",
           "tpc_compress", "tpc_decompress", "tpc_merge_tracks"]
PROF_STAGES = 16
# quality-control histogram layout (bin offsets; see tpc_qc_histograms)
QC_QTOT, QC_QMAX, QC_NHITS, QC_ATTACH, QC_BINS = 0, 256, 512, 665, 667


def library_path() -> str:
    return os.path.join(_here, "libtpcreco.so")


def load():
    """Load libtpcreco.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} not built: run __graft_entry__.build() "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    lib.tpc_params_default.argtypes = [P, ctypes.c_double]
    lib.tpc_geometry.argtypes = [P, P, P]
    lib.tpc_workspace_size.argtypes = [P, P]
    lib.tpc_create.argtypes = [P, P, P, P]
    lib.tpc_destroy.argtypes = [P]
    lib.tpc_cluster.argtypes = [P, P, P]
    lib.tpc_find_neighbours.argtypes = [P, P, P]
    lib.tpc_build_tracklets.argtypes = [P, P, P, P]
    lib.tpc_fit_tracks.argtypes = [P, P, P, P, P]
    lib.tpc_process_timeframe.argtypes = [P, P, P, P, P, P]
    lib.tpc_qc_histograms.argtypes = [P, P, P, P]
    lib.tpc_qc_histograms_noalloc.argtypes = [P, P, P, P]
    lib.tpc_decode_zs_pages.argtypes = [P, P, U32, P]
    lib.tpc_compress.argtypes = [P, P, P, P]
    lib.tpc_decompress.argtypes = [P, P, U32, P]
    lib.tpc_merge_tracks.argtypes = [P, P, P, P]
    lib.tpc_sync.argtypes = [P, P]
    lib.tpc_stream.argtypes = [P]
    lib.tpc_stream.restype = P
    lib.tpc_status_string.argtypes = [ctypes.c_int]
    lib.tpc_status_string.restype = ctypes.c_char_p
    lib.tpc_profile_enable.argtypes = [P, ctypes.c_int]
    lib.tpc_profile_read.argtypes = [P, P, P]
    lib.tpc_profile_stage_name.argtypes = [ctypes.c_int]
    lib.tpc_profile_stage_name.restype = ctypes.c_char_p
    lib.tpc_tuning_default.argtypes = [P]
    lib.tpc_set_tuning.argtypes = [P, P]
    lib.tpc_get_tuning.argtypes = [P, P]
    _lib = lib
    return lib


class TpcError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        msg = load().tpc_status_string(code).decode()
        super().__init__(f"{what}: {msg} ({code})" if what else f"{msg} ({code})")
        self.code = code


def _check(rc: int, what: str):
    if rc != 0:
        raise TpcError(rc, what)


def params(overrides: Optional[dict] = None, noise_sigma: float = 1.0) -> TpcParams:
    """Library defaults, optionally overridden by a dict of field values."""
    p = TpcParams()
    _check(load().tpc_params_default(ctypes.byref(p), noise_sigma), "tpc_params_default")
    for k, v in (overrides or {}).items():
        if k in ("sigma_y", "sigma_z"):
            arr = getattr(p, k)
            for i in range(NROW):
                arr[i] = float(v[i])
        else:
            setattr(p, k, v)
    return p


def geometry():
    npads = np.zeros(NROW, np.int32)
    xfx = np.zeros(NROW, np.int32)
    pfx = np.zeros(NROW, np.int32)
    load().tpc_geometry(npads.ctypes.data, xfx.ctypes.data, pfx.ctypes.data)
    return npads, xfx, pfx


def workspace_size(max_units: int, max_time_bins: int, max_clusters: int, max_tracklets: int,
                   max_samples: Optional[int] = None) -> int:
    s = TpcSizes(max_units, max_time_bins, max_clusters, max_tracklets,
                 max_clusters if max_samples is None else max_samples)
    out = ctypes.c_size_t(0)
    _check(load().tpc_workspace_size(ctypes.byref(s), ctypes.byref(out)), "tpc_workspace_size")
    return out.value


def _torch():
    import torch

    return torch


def _dptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def to_device_zs(pad, time, adc, row_start, n_units: int, n_time_bins: int, device="cuda") -> dict:
    """Copy a host ZS input (numpy) to device tensors (unsigned as signed views)."""
    torch = _torch()
    t = lambda a, dt, vt: torch.from_numpy(np.ascontiguousarray(a, dt).view(vt)).to(device)
    return dict(pad=t(pad, np.uint16, np.int16), time=t(time, np.uint16, np.int16),
                adc=t(adc, np.uint16, np.int16), row_start=t(row_start, np.uint32, np.int32),
                n_samples=int(len(pad)), n_units=int(n_units), n_time_bins=int(n_time_bins))


def zs_struct(zs: dict) -> TpcZsInput:
    return TpcZsInput(_dptr(zs["pad"]), _dptr(zs["time"]), _dptr(zs["adc"]), _dptr(zs["row_start"]),
                      zs["n_samples"], zs["n_units"], zs["n_time_bins"])


class Buffers:
    """Device tensors of one stage's outputs plus the matching C struct."""

    def __init__(self, tensors: Dict[str, object], struct):
        self.t = tensors
        self.s = struct

    def __getitem__(self, k):
        return self.t[k]


class Reco:
    """One library context bound to a torch stream on one GPU."""

    def __init__(self, max_units: int, max_time_bins: int, max_clusters: int,
                 max_tracklets: int, param_overrides: Optional[dict] = None,
                 noise_sigma: float = 1.0, device: str = "cuda", stream=None,
                 max_samples: Optional[int] = None):
        """max_samples bounds the samples of one call (default: max_clusters)."""
        torch = _torch()
        self.lib = load()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.params = params(param_overrides, noise_sigma)
        self.sizes = TpcSizes(max_units, max_time_bins, max_clusters, max_tracklets,
                              max_clusters if max_samples is None else max_samples)
        self.ctx = P()
        with torch.cuda.device(self.device):
            _check(self.lib.tpc_create(ctypes.byref(self.ctx), ctypes.byref(self.params),
                                       ctypes.byref(self.sizes), self.stream.cuda_stream),
                   "tpc_create")

    def close(self):
        if self.ctx:
            self.lib.tpc_destroy(self.ctx)
            self.ctx = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ buffers
    def alloc_clusters(self, n_units: int, n_time_bins: int, capacity: int, n_samples: int = 0,
                       moments: bool = False, labels: bool = False) -> Buffers:
        torch = _torch()
        d = self.device
        e = lambda n, dt: torch.empty(max(n, 1), dtype=dt, device=d)
        cap = int(capacity)
        t = dict(n_clusters=torch.zeros(1, dtype=torch.int32, device=d),
                 crow_start=e(n_units * NROW + 1, torch.int32),
                 y_fx=e(cap, torch.int32), z_fx=e(cap, torch.int32),
                 dpad=e(cap, torch.float32), dtime=e(cap, torch.float32),
                 s2pad=e(cap, torch.float32), s2time=e(cap, torch.float32),
                 qtot=e(cap, torch.int16), qmax=e(cap, torch.int16),
                 ppad=e(cap, torch.int16), ptime=e(cap, torch.int16), flags=e(cap, torch.uint8))
        if moments:
            for k in ("sp", "st", "spp", "stt"):
                t[k] = e(cap, torch.int32)
            t["nsamp"] = e(cap, torch.int16)
        if labels:
            t["sample_label"] = e(n_samples, torch.int32)
        s = TpcClusters(cap, n_units, n_time_bins, *[_dptr(t.get(k)) for k in (
            "n_clusters", "crow_start", "y_fx", "z_fx", "dpad", "dtime", "s2pad", "s2time", "qtot",
            "qmax", "ppad", "ptime", "flags", "sp", "st", "spp", "stt", "nsamp", "sample_label")])
        return Buffers(t, s)

    def clusters_from_host(self, cl: dict, n_units: int, n_time_bins: int) -> Buffers:
        """Device copy of a host cluster set (positions, peaks, row table)."""
        torch = _torch()
        n = len(cl["y_fx"])
        b = self.alloc_clusters(n_units, n_time_bins, max(n, 1))
        dev = lambda a, dt, vt: torch.from_numpy(np.ascontiguousarray(a, dt).view(vt)).to(self.device)
        b.t["n_clusters"].copy_(torch.tensor([n], dtype=torch.int32))
        b.t["crow_start"].copy_(dev(cl["crow_start"], np.uint32, np.int32))
        if n:
            b.t["y_fx"][:n].copy_(dev(cl["y_fx"], np.int32, np.int32))
            b.t["z_fx"][:n].copy_(dev(cl["z_fx"], np.int32, np.int32))
            for k in ("ptime", "ppad", "qtot", "qmax"):
                if k in cl:
                    b.t[k][:n].copy_(dev(cl[k], np.uint16, np.int16))
            if "flags" in cl:
                b.t["flags"][:n].copy_(dev(cl["flags"], np.uint8, np.uint8))
        return b

    def tracks_from_host(self, tr: dict, cluster_capacity: int) -> Buffers:
        """Device copy of a host track set (parameters, rows, anchors, hit
        lists, cluster -> track map), e.g. the oracle's tracks."""
        torch = _torch()
        n = len(tr["hit_start"]) - 1
        nh = int(tr["hit_start"][-1])
        b = self.alloc_tracks(max(n, 1), max(nh, 1), cluster_capacity)
        dev = lambda a, dt, vt: torch.from_numpy(np.ascontiguousarray(a, dt).view(vt)).to(self.device)
        b.t["n_tracks"].copy_(torch.tensor([n], dtype=torch.int32))
        b.t["n_hits"].copy_(torch.tensor([nh], dtype=torch.int32))
        b.t["hit_start"][:n + 1].copy_(dev(tr["hit_start"], np.uint32, np.int32))
        if "cluster_track" in tr and len(tr["cluster_track"]):
            nc = len(tr["cluster_track"])
            b.t["cluster_track"][:nc].copy_(dev(tr["cluster_track"], np.int32, np.int32))
        else:
            b.t["cluster_track"].fill_(-1)
        if n:
            b.t["par"][:n * 5].copy_(dev(np.asarray(tr["par"]).reshape(-1), np.float32, np.float32))
            b.t["row"][:n].copy_(dev(tr["row"], np.uint8, np.uint8))
            b.t["z_anchor"][:n].copy_(dev(tr["z_anchor"], np.int32, np.int32))
        if nh:
            b.t["hits"][:nh].copy_(dev(tr["hits"], np.uint32, np.int32))
        return b

    def alloc_compressed(self, capacity_words: int, hist: bool = True) -> Buffers:
        """Device buffer for a compressed stream (tpc_compressed)."""
        torch = _torch()
        d = self.device
        t = dict(stream=torch.empty(max(int(capacity_words), 1), dtype=torch.int32, device=d),
                 n_words=torch.zeros(1, dtype=torch.int32, device=d))
        if hist:
            t["res_hist"] = torch.zeros(256, dtype=torch.int32, device=d)
        s = TpcCompressed(int(capacity_words), _dptr(t["stream"]), _dptr(t["n_words"]),
                          _dptr(t.get("res_hist")))
        return Buffers(t, s)

    def alloc_merged(self, capacity: int) -> Buffers:
        """Device arrays for merged tracks (tpc_merged)."""
        torch = _torch()
        d = self.device
        cap = max(int(capacity), 1)
        t = dict(n_merged=torch.zeros(1, dtype=torch.int32, device=d),
                 label=torch.empty(cap, dtype=torch.int32, device=d),
                 near_tie=torch.empty(cap, dtype=torch.uint8, device=d),
                 fit=torch.empty(cap * MERGE_FIT, dtype=torch.float64, device=d))
        s = TpcMerged(cap, *[_dptr(t[k]) for k in ("n_merged", "label", "near_tie", "fit")])
        return Buffers(t, s)

    def alloc_decoded(self, capacity: int) -> Buffers:
        """Device arrays for decompressed clusters (tpc_decoded_clusters)."""
        torch = _torch()
        d = self.device
        e = lambda dt: torch.empty(max(int(capacity), 1), dtype=dt, device=d)
        t = dict(n_clusters=torch.zeros(1, dtype=torch.int32, device=d), unit=e(torch.int16),
                 row=e(torch.uint8), y_fx=e(torch.int32), z_fx=e(torch.int32),
                 qtot=e(torch.int16), qmax=e(torch.int16), flags=e(torch.uint8),
                 track=e(torch.int32))
        s = TpcDecoded(int(capacity), *[_dptr(t[k]) for k in (
            "n_clusters", "unit", "row", "y_fx", "z_fx", "qtot", "qmax", "flags", "track")])
        return Buffers(t, s)

    def alloc_links(self, capacity: int) -> Buffers:
        torch = _torch()
        cap = max(int(capacity), 1)
        t = {k: torch.empty(cap, dtype=torch.int32, device=self.device)
             for k in ("down", "up", "downc", "upc")}
        return Buffers(t, TpcLinks(cap, *[_dptr(t[k]) for k in ("down", "up", "downc", "upc")]))

    def alloc_tracklets(self, capacity: int) -> Buffers:
        torch = _torch()
        cap = max(int(capacity), 1)
        t = dict(n_tracklets=torch.zeros(1, dtype=torch.int32, device=self.device),
                 start=torch.empty(cap, dtype=torch.int32, device=self.device),
                 len=torch.empty(cap, dtype=torch.int16, device=self.device))
        return Buffers(t, TpcTracklets(cap, _dptr(t["n_tracklets"]), _dptr(t["start"]),
                                       _dptr(t["len"])))

    def alloc_tracks(self, capacity: int, hit_capacity: int, cluster_capacity: int,
                     follow_capacity: int = 0) -> Buffers:
        torch = _torch()
        d = self.device
        cap = max(int(capacity), 1)
        e = lambda n, dt: torch.empty(max(int(n), 1), dtype=dt, device=d)
        t = dict(n_tracks=torch.zeros(1, dtype=torch.int32, device=d),
                 n_hits=torch.zeros(1, dtype=torch.int32, device=d),
                 tracklet=e(cap, torch.int32), par=e(cap * 5, torch.float32),
                 cov=e(cap * 15, torch.float32), chi2=e(cap, torch.float32),
                 ndf=e(cap, torch.int16), row=e(cap, torch.uint8), flags=e(cap, torch.uint8),
                 z_anchor=e(cap, torch.int32), hit_start=e(cap + 1, torch.int32),
                 hits=e(hit_capacity, torch.int32), cluster_track=e(cluster_capacity, torch.int32))
        if follow_capacity:
            t["follow_hits"] = e(follow_capacity * NROW, torch.int32)
        s = TpcTracks(cap, max(int(hit_capacity), 1), *[_dptr(t.get(k)) for k in (
            "n_tracks", "n_hits", "tracklet", "par", "cov", "chi2", "ndf", "row", "flags",
            "z_anchor", "hit_start", "hits", "cluster_track", "follow_hits")])
        return Buffers(t, s)

    def alloc_zs_soa(self, n_units: int, n_time_bins: int, capacity: int) -> Buffers:
        """Device arrays for decoded raw pages (tpc_zs_soa)."""
        torch = _torch()
        d = self.device
        e = lambda n, dt: torch.empty(max(n, 1), dtype=dt, device=d)
        t = dict(n_samples=torch.zeros(1, dtype=torch.int32, device=d),
                 pad=e(capacity, torch.int16), time=e(capacity, torch.int16),
                 adc=e(capacity, torch.int16), row_start=e(n_units * NROW + 1, torch.int32))
        s = TpcZsSoa(int(capacity), n_units, n_time_bins,
                     *[_dptr(t[k]) for k in ("n_samples", "pad", "time", "adc", "row_start")])
        return Buffers(t, s)

    # ------------------------------------------------------------ calls
    def decode_zs_pages(self, pages, out: Buffers, n_pages: Optional[int] = None):
        """Raw zero-suppressed pages (device tensor of n_pages * 2048 32-bit
        words) -> out's sample arrays and row offsets (tpc_decode_zs_pages)."""
        if n_pages is None:
            n_pages = pages.numel() // ZS_PAGE_WORDS
        if pages.numel() < n_pages * ZS_PAGE_WORDS or pages.element_size() != 4 or not pages.is_cuda:
            raise ValueError("decode_zs_pages: pages must be a device tensor of 32-bit words")
        _check(self.lib.tpc_decode_zs_pages(self.ctx, ctypes.c_void_p(pages.data_ptr()),
                                            int(n_pages), ctypes.byref(out.s)),
               "tpc_decode_zs_pages")

    def compress(self, cl: Buffers, tr: Buffers, out: Buffers):
        """Track-model compression of a reconstruction's clusters (tpc_compress)."""
        _check(self.lib.tpc_compress(self.ctx, ctypes.byref(cl.s), ctypes.byref(tr.s),
                                     ctypes.byref(out.s)), "tpc_compress")

    def decompress(self, stream, out: Buffers, stream_words: Optional[int] = None):
        """Decode a stream (device tensor of 32-bit words) into out (tpc_decompress)."""
        n = stream.numel() if stream_words is None else int(stream_words)
        if stream.numel() < n or stream.element_size() != 4 or not stream.is_cuda:
            raise ValueError("decompress: stream must be a device tensor of 32-bit words")
        _check(self.lib.tpc_decompress(self.ctx, ctypes.c_void_p(stream.data_ptr()), n,
                                       ctypes.byref(out.s)), "tpc_decompress")

    def merge_tracks(self, cl: Buffers, tr: Buffers, out: Buffers):
        """Join segments into tracks and fit them, with T0 (tpc_merge_tracks)."""
        _check(self.lib.tpc_merge_tracks(self.ctx, ctypes.byref(cl.s), ctypes.byref(tr.s),
                                         ctypes.byref(out.s)), "tpc_merge_tracks")

    def cluster(self, zs: dict, out: Buffers):
        _check(self.lib.tpc_cluster(self.ctx, ctypes.byref(zs_struct(zs)), ctypes.byref(out.s)),
               "tpc_cluster")

    def find_neighbours(self, cl: Buffers, links: Buffers):
        _check(self.lib.tpc_find_neighbours(self.ctx, ctypes.byref(cl.s), ctypes.byref(links.s)),
               "tpc_find_neighbours")

    def build_tracklets(self, cl: Buffers, links: Buffers, tl: Buffers):
        _check(self.lib.tpc_build_tracklets(self.ctx, ctypes.byref(cl.s), ctypes.byref(links.s),
                                            ctypes.byref(tl.s)), "tpc_build_tracklets")

    def fit_tracks(self, cl: Buffers, links: Buffers, tl: Buffers, tr: Buffers):
        _check(self.lib.tpc_fit_tracks(self.ctx, ctypes.byref(cl.s), ctypes.byref(links.s),
                                       ctypes.byref(tl.s), ctypes.byref(tr.s)), "tpc_fit_tracks")

    def qc_histograms(self, cl: Buffers, tr: Buffers, out=None):
        """Quality-control histograms of a reconstruction's outputs (int32
        device tensor of QC_BINS counts, laid out as QC_QTOT, QC_QMAX,
        QC_NHITS, QC_ATTACH say), enqueued on the context's stream."""
        torch = _torch()
        if out is None:
            out = torch.empty(QC_BINS, dtype=torch.int32, device=self.device)
        if out.numel() < QC_BINS or out.dtype != torch.int32 or not out.is_cuda:
            raise ValueError("qc_histograms: out must be an int32 device tensor of QC_BINS")
        _check(self.lib.tpc_qc_histograms(self.ctx, ctypes.byref(cl.s), ctypes.byref(tr.s),
                                          ctypes.c_void_p(out.data_ptr())), "tpc_qc_histograms")
        return out

    def qc_histograms_noalloc(self, cl: Buffers, tr: Buffers, out, stream=None):
        """tpc_qc_histograms_noalloc on the same outputs: no context and no
        allocation inside the call (out: int32 device tensor of QC_BINS,
        caller-allocated).  Enqueued on `stream` (a torch stream; default:
        this context's stream)."""
        return qc_histograms_noalloc(cl, tr, out, stream if stream is not None else self.stream)

    def process(self, zs: dict, cl: Buffers, links: Buffers, tl: Buffers, tr: Buffers,
                zs_s: Optional[TpcZsInput] = None):
        s = zs_s if zs_s is not None else zs_struct(zs)
        _check(self.lib.tpc_process_timeframe(self.ctx, ctypes.byref(s), ctypes.byref(cl.s),
                                              ctypes.byref(links.s), ctypes.byref(tl.s),
                                              ctypes.byref(tr.s)), "tpc_process_timeframe")

    def tuning(self) -> dict:
        t = TpcTuning()
        _check(self.lib.tpc_get_tuning(self.ctx, ctypes.byref(t)), "tpc_get_tuning")
        return {k: getattr(t, k) for k, _ in TpcTuning._fields_}

    def set_tuning(self, **kw):
        """Change launch shapes (cl_window, cl_chunk, follow_block, follow_mode, refit_waves,
        cl_mode)."""
        t = TpcTuning()
        _check(self.lib.tpc_get_tuning(self.ctx, ctypes.byref(t)), "tpc_get_tuning")
        for k, v in kw.items():
            if k not in ("cl_window", "cl_chunk", "follow_block", "follow_mode", "refit_waves",
                         "cl_mode"):
                raise KeyError(k)
            setattr(t, k, int(v))
        _check(self.lib.tpc_set_tuning(self.ctx, ctypes.byref(t)), "tpc_set_tuning")

    def profile(self, on: bool = True, count_work: bool = False):
        """Stage timers on/off; count_work also counts the following's work."""
        _check(self.lib.tpc_profile_enable(self.ctx, (1 if on else 0) | (2 if count_work else 0)),
               "tpc_profile_enable")

    def profile_read(self) -> dict:
        """Summed milliseconds and launch counts per stage since the last read."""
        ms = np.zeros(PROF_STAGES, np.float64)
        n = np.zeros(PROF_STAGES, np.uint32)
        _check(self.lib.tpc_profile_read(self.ctx, ms.ctypes.data, n.ctypes.data),
               "tpc_profile_read")
        return {self.lib.tpc_profile_stage_name(i).decode(): (float(ms[i]), int(n[i]))
                for i in range(PROF_STAGES)}

    def sync(self, raise_on_error: bool = True) -> dict:
        c = TpcCounts()
        rc = self.lib.tpc_sync(self.ctx, ctypes.byref(c))
        out = {k: getattr(c, k) for k, _ in TpcCounts._fields_}
        out["required_by"] = {name: int(c.required_by[i])
                              for i, name in enumerate(OVERFLOW_KINDS) if c.overflow >> i & 1}
        if raise_on_error and rc != 0:
            raise TpcError(rc, f"tpc_sync (required {c.required})")
        return out


# ---------------------------------------------------------------- host views
ZS_PAGE_WORDS = 2048


def zs_from_soa(soa: Buffers) -> dict:
    """Decoded pages as a clusterizer input: the arrays hold up to
    `capacity` samples and the device row offsets bound every row."""
    t, s = soa.t, soa.s
    return dict(pad=t["pad"], time=t["time"], adc=t["adc"], row_start=t["row_start"],
                n_samples=int(s.capacity), n_units=int(s.n_units), n_time_bins=int(s.n_time_bins))


def pages_to_device(pages, device="cuda"):
    """Host pages (uint32 [n_pages, 2048]) as a device tensor of 32-bit words."""
    torch = _torch()
    a = np.ascontiguousarray(pages, np.uint32).reshape(-1)
    return torch.from_numpy(a.view(np.int32)).to(device)


def zs_soa_to_host(b: Buffers) -> dict:
    n = int(b["n_samples"].item())
    m = min(n, int(b.s.capacity))
    return dict(n_samples=n, pad=_u(b["pad"], m, np.uint16), time=_u(b["time"], m, np.uint16),
                adc=_u(b["adc"], m, np.uint16),
                row_start=_u(b["row_start"], int(b.s.n_units) * NROW + 1, np.uint32))


MERGE_FIT = 12
MERGE_FIT_FIELDS = ("n_segments", "n_hits", "xc", "yc", "radius", "dzdpsi", "zd_axis", "t0",
                    "tgl", "flags", "turn")


def merged_to_host(b: Buffers, n_tracks: int) -> dict:
    f = b["fit"][: n_tracks * MERGE_FIT].cpu().numpy().reshape(n_tracks, MERGE_FIT)
    out = dict(n_merged=int(b["n_merged"].item()), label=b["label"][:n_tracks].cpu().numpy(),
               near_tie=b["near_tie"][:n_tracks].cpu().numpy().astype(bool))
    for i, k in enumerate(MERGE_FIT_FIELDS):
        out[k] = f[:, i].copy()
    return out


def compressed_to_host(b: Buffers) -> dict:
    n = int(b["n_words"].item())
    m = min(n, int(b.s.capacity))
    out = dict(n_words=n, words=_u(b["stream"], m, np.uint32))
    if "res_hist" in b.t:
        out["hist"] = b["res_hist"].cpu().numpy().astype(np.int64)
    return out


def decoded_to_host(b: Buffers) -> dict:
    n = min(int(b["n_clusters"].item()), int(b.s.capacity))
    return dict(unit=_u(b["unit"], n, np.uint16), row=_u(b["row"], n, np.uint8),
                y_fx=_u(b["y_fx"], n, np.int32), z_fx=_u(b["z_fx"], n, np.int32),
                qtot=_u(b["qtot"], n, np.uint16), qmax=_u(b["qmax"], n, np.uint16),
                flags=_u(b["flags"], n, np.uint8), track=_u(b["track"], n, np.int32))


QC_NOALLOC_MAX = 1024 * 65536


def qc_histograms_noalloc(cl: Buffers, tr: Buffers, out, stream=None):
    """Quality-control histograms through tpc_qc_histograms_noalloc: the
    library's fixed per-GPU scratch, no context, nothing allocated.  `out` is
    an int32 device tensor of QC_BINS counts; `stream` a torch stream (None:
    torch's current stream)."""
    torch = _torch()
    lib = load()
    if out.numel() < QC_BINS or out.dtype != torch.int32 or not out.is_cuda:
        raise ValueError("qc_histograms_noalloc: out must be an int32 device tensor of QC_BINS")
    s = stream if stream is not None else torch.cuda.current_stream(out.device)
    _check(lib.tpc_qc_histograms_noalloc(ctypes.byref(cl.s), ctypes.byref(tr.s),
                                         ctypes.c_void_p(out.data_ptr()),
                                         ctypes.c_void_p(s.cuda_stream)),
           "tpc_qc_histograms_noalloc")
    return out


def _u(t, n, dt):
    a = t[:n].cpu().numpy()
    return a.view(dt) if a.dtype.itemsize == np.dtype(dt).itemsize else a.astype(dt)


def clusters_to_host(b: Buffers, n_units: int) -> dict:
    n = int(b["n_clusters"].item())
    out = dict(crow_start=b["crow_start"][: n_units * NROW + 1].cpu().numpy().view(np.uint32),
               n_units=n_units)
    for k, dt in (("y_fx", np.int32), ("z_fx", np.int32), ("dpad", np.float32),
                  ("dtime", np.float32), ("s2pad", np.float32), ("s2time", np.float32),
                  ("qtot", np.uint16), ("qmax", np.uint16), ("ppad", np.uint16),
                  ("ptime", np.uint16), ("flags", np.uint8), ("sp", np.int32), ("st", np.int32),
                  ("spp", np.int32), ("stt", np.int32), ("nsamp", np.uint16)):
        if k in b.t:
            out[k] = _u(b[k], n, dt)
    if "sample_label" in b.t:
        out["sample_label"] = b["sample_label"].cpu().numpy()
    return out


def links_to_host(b: Buffers, n: int) -> dict:
    return {k: b[k][:n].cpu().numpy() for k in ("down", "up", "downc", "upc")}


def tracklets_to_host(b: Buffers) -> dict:
    n = int(b["n_tracklets"].item())
    return dict(tl_start=_u(b["start"], n, np.uint32), tl_len=_u(b["len"], n, np.uint16))


def tracks_to_host(b: Buffers, n_clusters: int, n_tracklets: int = 0) -> dict:
    n = int(b["n_tracks"].item())
    nh = int(b["n_hits"].item())
    out = dict(tracklet=_u(b["tracklet"], n, np.uint32),
               par=b["par"][: n * 5].cpu().numpy().reshape(n, 5),
               cov=b["cov"][: n * 15].cpu().numpy().reshape(n, 15),
               chi2=b["chi2"][:n].cpu().numpy(), ndf=_u(b["ndf"], n, np.uint16),
               row=b["row"][:n].cpu().numpy(), flags=b["flags"][:n].cpu().numpy(),
               z_anchor=b["z_anchor"][:n].cpu().numpy(),
               hit_start=_u(b["hit_start"], n + 1, np.uint32), hits=_u(b["hits"], nh, np.uint32),
               cluster_track=b["cluster_track"][:n_clusters].cpu().numpy())
    if "follow_hits" in b.t and n_tracklets:
        out["follow_hits"] = b["follow_hits"][: n_tracklets * NROW].cpu().numpy().reshape(
            n_tracklets, NROW)
    return out
