"""Pins of the oracle's track-model cluster compression.

The paper (section "Hardware and data flow") says TPC data compression relies
on the tracking and gives no codec; the library defines its own (stated with
tpc_compress).  The oracle's encoder and decoder are pinned by
* a frame worked out bit by bit by hand (tests/golden/compress_example.txt):
  header, directory, every code of a straight-line track and of the clusters
  on no track, the decoded clusters and the residual histograms;
* round trips on generated events with the oracle's own tracks: decoding
  gives back every cluster's quantised position (within half a 2^-7 cm step
  of the original), its charges and flags, and its track;
* the integer helix model against the exact FP64 helix (circle in the
  bending plane, drift length summed over the row chords) for pT from 0.1 to
  10 GeV/c, both charges and both drift directions;
* a row of 150 clusters on no track read with an independent bit reader:
  its chunk offset fields, each chunk starting with its z coded whole, and a
  corrupted field rejected;
* the error rules (stream too large for its buffer, a hit below the model's
  row, malformed streams).
"""
import os

import numpy as np
import pytest

import oracle
import tpcsynth

HERE = os.path.dirname(os.path.abspath(__file__))
NROW = 152
B = 0.299792458e-3 * 5.0


def q(v):
    return np.floor_divide(np.asarray(v, np.int64) + 256, 512)


def load_example():
    cl, tr, bits, meta = [], None, [], {}
    for line in open(os.path.join(HERE, "golden", "compress_example.txt")):
        f = line.split("#", 1)[0].split()
        if not f:
            continue
        if f[0] == "cluster":
            cl.append([int(x) for x in f[1:]])
        elif f[0] == "track":
            tr = [float(x) for x in f[1:6]] + [int(f[6]), int(f[7])]
        elif f[0] == "bits":
            bits.append(f[1])
        elif f[0] == "repeat":
            bits.append(f[2] * int(f[1]))
        elif f[0] in ("header", "track_offsets", "row_offsets"):
            meta[f[0]] = f[1:]
    cl = np.array(cl, np.int64)
    rows = cl[:, 0]
    crow = np.searchsorted(rows, np.arange(NROW + 1), side="left").astype(np.uint32)
    clusters = dict(crow_start=crow, y_fx=cl[:, 1].astype(np.int32), z_fx=cl[:, 2].astype(np.int32),
                    qtot=cl[:, 3].astype(np.uint16), qmax=cl[:, 4].astype(np.uint16),
                    flags=cl[:, 5].astype(np.uint8))
    on = np.nonzero(cl[:, 6] >= 0)[0]
    tracks = dict(par=np.array([tr[:5]], np.float32), row=np.array([tr[5]], np.uint8),
                  z_anchor=np.array([tr[6]], np.int32),
                  hit_start=np.array([0, len(on)], np.uint32), hits=on.astype(np.uint32),
                  cluster_track=cl[:, 6].astype(np.int32))
    return clusters, tracks, "".join(bits), meta, cl


def test_hand_worked_example():
    clusters, tracks, bits, meta, cl = load_example()
    c = oracle.compress(clusters, tracks, 1)
    assert c["status"] == 0
    w = c["words"]
    hdr = [int(meta["header"][0], 16)] + [int(x) for x in meta["header"][1:]]
    assert w[:8].tolist() == hdr
    assert len(bits) == hdr[6] == 484
    assert w[8:10].tolist() == [int(x) for x in meta["track_offsets"]]
    ro = w[10:10 + NROW + 1].astype(np.int64)
    assert ro[0] == 254 and ro[1] == 255
    assert np.array_equal(ro[2:], 334 + np.arange(NROW - 1))
    payload = w[10 + NROW + 1:]
    assert len(payload) == (484 + 31) // 32
    got = "".join(str((int(payload[i // 32]) >> (i % 32)) & 1) for i in range(len(payload) * 32))
    assert got[:484] == bits and set(got[484:]) <= {"0"}
    # residual histograms: dy 2, -3 and dz 0, 2
    h = c["hist"]
    exp = np.zeros(256, np.int64)
    for d in (2, -3):
        exp[d + 64] += 1
    for d in (0, 2):
        exp[128 + d + 64] += 1
    assert np.array_equal(h, exp)
    d = oracle.decompress(w)
    assert d["status"] == 0
    order = [2, 3, 0, 1]  # the track's hits, then the clusters on no track
    assert np.array_equal(d["row"], cl[order, 0])
    assert np.array_equal(d["y_fx"], q(cl[order, 1]) * 512)
    assert np.array_equal(d["z_fx"], q(cl[order, 2]) * 512)
    assert np.array_equal(d["qtot"], cl[order, 3]) and np.array_equal(d["qmax"], cl[order, 4])
    assert np.array_equal(d["flags"], cl[order, 5]) and np.array_equal(d["track"], cl[order, 6])


def _expected(clusters, tracks, n_units):
    crow = clusters["crow_start"].astype(np.int64)
    ur_of = np.repeat(np.arange(n_units * NROW), np.diff(crow))
    hs = tracks["hit_start"].astype(np.int64)
    order, trk = [], []
    for j in range(len(hs) - 1):
        h = tracks["hits"][hs[j]:hs[j + 1]].astype(np.int64)
        order += h.tolist()
        trk += [j] * len(h)
    un = np.nonzero(tracks["cluster_track"] < 0)[0]  # canonical order = (unit,row) order
    order += un.tolist()
    trk += [-1] * len(un)
    o = np.array(order, np.int64)
    return dict(unit=ur_of[o] // NROW, row=ur_of[o] % NROW, y_fx=q(clusters["y_fx"][o]) * 512,
                z_fx=q(clusters["z_fx"][o]) * 512, qtot=clusters["qtot"][o],
                qmax=clusters["qmax"][o], flags=clusters["flags"][o], track=np.array(trk)), o


@pytest.mark.parametrize("which", ["c1", "small36", "pileup"])
def test_round_trip_generated(which):
    cfg, seed = {"c1": (tpcsynth.config_c1(), 101),
                 "small36": (tpcsynth.config_small(400, sector_mode=0, n_sec=80), 11),
                 "pileup": (tpcsynth.config_chunk(404, 1, n_coll=3), 4041)}[which]
    ev = tpcsynth.generate(cfg, seed)
    o = oracle.process(ev.pad, ev.time, ev.adc, ev.row_start, ev.n_units, ev.n_time_bins,
                       n_threads=8)
    tracks = oracle.tracks_from_fit(o)
    assert len(tracks["hit_start"]) > 10
    c = oracle.compress(o["clusters"], tracks, ev.n_units)
    assert c["status"] == 0
    d = oracle.decompress(c["words"])
    assert d["status"] == 0
    exp, idx = _expected(o["clusters"], tracks, ev.n_units)
    for k, v in exp.items():
        assert np.array_equal(d[k].astype(np.int64), np.asarray(v, np.int64)), k
    # within the stated quantisation of the originals
    assert np.abs(d["y_fx"] - o["clusters"]["y_fx"][idx].astype(np.int64)).max() <= 256
    assert np.abs(d["z_fx"] - o["clusters"]["z_fx"][idx].astype(np.int64)).max() <= 256
    nc = len(o["clusters"]["y_fx"])
    n_hits = int(tracks["hit_start"][-1])
    assert c["hist"][:128].sum() == n_hits == c["hist"][128:].sum()
    print(f"{which}: {nc} clusters ({n_hits} on tracks) in {4 * c['n_words']} bytes: "
          f"{4 * c['n_words'] / nc:.2f} B/cluster")


class _Bits:
    """Independent LSB-first reader of a stream's payload (for the pins)."""

    def __init__(self, words, pos):
        self.w, self.pos = [int(x) for x in words], pos

    def get(self, n):
        v = 0
        for i in range(n):
            v |= ((self.w[self.pos // 32] >> (self.pos % 32)) & 1) << i
            self.pos += 1
        return v

    def eg(self, k):
        n = 0
        while self.get(1) == 0:
            n += 1
        qv = (1 << n) | self.get(n)
        return ((qv - 1) << k) | self.get(k)


def _unzig(v):
    return v >> 1 if v % 2 == 0 else -((v + 1) >> 1)


def chunk_frame(n=150, r=7, seed=5):
    """One unit, n clusters on no track in row r (no tracks): a row of
    several chunks."""
    rng = np.random.default_rng(seed)
    t = np.sort(rng.integers(0, 200, n))
    crow = np.zeros(NROW + 1, np.uint32)
    crow[r + 1:] = n
    clusters = dict(crow_start=crow, y_fx=rng.integers(-2_000_000, 2_000_000, n).astype(np.int32),
                    z_fx=(t * 32768 + rng.integers(0, 32768, n)).astype(np.int32),
                    qtot=rng.integers(1, 3000, n).astype(np.uint16),
                    qmax=rng.integers(1, 1023, n).astype(np.uint16),
                    flags=rng.integers(0, 4, n).astype(np.uint8))
    tracks = dict(par=np.zeros((0, 5), np.float32), row=np.zeros(0, np.uint8),
                  z_anchor=np.zeros(0, np.int32), hit_start=np.zeros(1, np.uint32),
                  hits=np.zeros(0, np.uint32), cluster_track=np.full(n, -1, np.int32))
    return n, r, clusters, tracks


def test_row_chunks():
    # One row with 150 clusters on no track: the count, then two 32-bit
    # fields with the offsets of chunks 1 and 2 (clusters 64 and 128) from the
    # end of the fields, and every chunk starts with its z coded whole
    # (EG(12)), so each chunk decodes on its own.  Read with a reader of its
    # own, not the oracle's.
    n, r, clusters, tracks = chunk_frame()
    cl_y, cl_z = clusters["y_fx"], clusters["z_fx"]
    c = oracle.compress(clusters, tracks, 1)
    assert c["status"] == 0
    w = c["words"]
    assert w[1] == 2  # the format with row chunks
    dir0 = 8 + 1  # no tracks: one closing track offset
    payload = 8 + 1 + NROW + 1
    start = int(w[dir0 + r])
    b = _Bits(w[payload:], start)
    assert b.eg(0) == n
    offs = [b.get(32), b.get(32)]
    chunk0 = b.pos
    # sequential decode of the whole row
    seq = []
    zprev = 0
    for i in range(n):
        if i % 64 == 0:
            assert i == 0 or b.pos == chunk0 + offs[i // 64 - 1]
        yq = _unzig(b.eg(10))
        zq = _unzig(b.eg(12)) if i % 64 == 0 else zprev + _unzig(b.eg(6))
        zprev = zq
        seq.append((yq, zq, b.eg(6), b.eg(5), b.get(2)))
    assert b.pos == int(w[dir0 + r + 1])
    assert [s[0] for s in seq] == q(cl_y).tolist() and [s[1] for s in seq] == q(cl_z).tolist()
    assert [s[2] for s in seq] == clusters["qtot"].tolist()
    # each chunk on its own from its field
    for k in (1, 2):
        bk = _Bits(w[payload:], chunk0 + offs[k - 1])
        assert _unzig(bk.eg(10)) == q(cl_y[64 * k])
        assert _unzig(bk.eg(12)) == q(cl_z[64 * k])
    d = oracle.decompress(w)
    assert d["status"] == 0 and len(d["y_fx"]) == n
    assert np.array_equal(d["y_fx"], q(cl_y) * 512) and np.array_equal(d["z_fx"], q(cl_z) * 512)
    # a wrong offset field is a malformed stream
    bad = w.copy()
    pos = payload * 32 + start + 1 + 2 * 8 + 1  # inside the first field (EG(0) of 150 is 15 bits)
    bad[pos // 32] ^= 1 << (pos % 32)
    assert oracle.decompress(bad)["status"] == -3


def _exact_model(par, z_anchor, row0, rows, xr):
    """FP64 helix from the model's parameters: the float32 values as the
    codec holds them (y, z to 2^-16 cm, sin phi and tan lambda to 2^-30, q/pT
    to 2^-16 c/GeV, the field constant to 2^-30), the circle in the bending
    plane (sin phi linear in x), the drift length summed over row chords."""
    y = np.rint(float(par[0]) * 2 ** 16) / 2 ** 16
    z = np.rint(float(par[1]) * 2 ** 16) / 2 ** 16
    s = np.rint(float(par[2]) * 2 ** 30) / 2 ** 30
    tgl = np.rint(float(par[3]) * 2 ** 30) / 2 ** 30
    qpt = np.rint(float(par[4]) * 2 ** 16) / 2 ** 16
    C = -np.rint(B * 2 ** 30) / 2 ** 30 * qpt
    x = xr[row0]
    zz = z + z_anchor / 65536.0
    out_y, out_z, frozen = [], [], []
    r = row0
    stopped = False
    for rt in rows:
        while r < rt:
            x1 = xr[r + 1]
            s1 = s + C * (x1 - x)
            if stopped or abs(s1) >= 1 - 2 ** -10:
                stopped = True
                r += 1
                x = x1
                continue
            c0, c1 = np.sqrt(1 - s * s), np.sqrt(1 - s1 * s1)
            f = (s + s1) / (c0 + c1)
            y += (x1 - x) * f
            zz += tgl * (x1 - x) * np.sqrt(1 + f * f)
            s, x, r = s1, x1, r + 1
        out_y.append(y)
        out_z.append(zz)
        frozen.append(stopped)
    return np.array(out_y), np.array(out_z), np.array(frozen)


def test_model_against_exact_helix():
    npads, xfx, pfx = oracle.geometry()
    xr = xfx / 65536.0
    rng = np.random.default_rng(5)
    worst_y = worst_z = 0.0
    n_frozen = 0
    for i in range(400):
        pt = 0.1 * 100 ** rng.random()
        qsign = rng.choice([-1, 1])
        row0 = int(rng.integers(0, 100))
        par = np.array([rng.uniform(-20, 20), rng.uniform(-50, 50), rng.uniform(-0.8, 0.8),
                        rng.uniform(-1.0, 1.0), qsign / pt], np.float32)
        za = int(rng.integers(0, 1 << 29))
        rows = np.arange(row0, NROW)
        y, z, fr = oracle.track_model(par, za, row0, rows)
        ey, ez, efr = _exact_model(par, za, row0, rows, xr)
        ok = ~efr & (fr == 0)
        # the stop rule agrees except at a row where |sin phi| is within rounding of the limit
        assert (fr.astype(bool) != efr).sum() <= 1
        n_frozen += efr.any()
        worst_y = max(worst_y, np.abs(y[ok] / 65536.0 - ey[ok]).max(initial=0))
        worst_z = max(worst_z, np.abs(z[ok] / 65536.0 - ez[ok]).max(initial=0))
    print(f"integer helix vs FP64: worst |dy| {worst_y:.2e} cm, |dz| {worst_z:.2e} cm; "
          f"{n_frozen} of 400 tracks reach the |sin phi| limit")
    assert n_frozen > 10
    assert worst_y < 5e-4 and worst_z < 5e-4  # a 2^-7 cm step is 7.8e-3


def test_model_straight_line_and_sign():
    npads, xfx, pfx = oracle.geometry()
    # a straight line: y constant for sin phi = 0, z grows by floor(T D / 2^30) per row
    y, z, fr = oracle.track_model(np.array([1.5, 0.25, 0, 0.5, 0], np.float32), 200000, 10,
                                  [10, 11, 12])
    assert y.tolist() == [98304] * 3 and z.tolist() == [216384, 251105, 285826]
    # positive charge in +Bz bends clockwise: sin phi decreases outward, so y
    # falls below the tangent line
    rows = np.arange(0, 60)
    yp, _, _ = oracle.track_model(np.array([0, 0, 0, 0, 2.0], np.float32), 0, 0, rows)
    ym, _, _ = oracle.track_model(np.array([0, 0, 0, 0, -2.0], np.float32), 0, 0, rows)
    assert yp[-1] < 0 < ym[-1] and abs(yp[-1] + ym[-1]) <= 4


def test_errors():
    clusters, tracks, bits, meta, cl = load_example()
    c = oracle.compress(clusters, tracks, 1, capacity_words=100)
    assert c["status"] == -2 and c["n_words"] == 8 + 2 + 153 + 16
    bad = dict(tracks, row=np.array([11], np.uint8))  # first hit (row 10) below the model's row
    assert oracle.compress(clusters, bad, 1)["status"] == -3
    w = oracle.compress(clusters, tracks, 1)["words"]
    assert oracle.decompress(w)["status"] == 0
    w2 = w.copy()
    w2[0] ^= 1
    assert oracle.decompress(w2)["status"] == -3            # magic
    assert oracle.decompress(w[:-1])["status"] == -3        # truncated
    w3 = w.copy()
    w3[9] += 1                                              # directory disagrees with the record
    assert oracle.decompress(w3)["status"] == -3
    assert oracle.decompress(w, capacity=3)["status"] == -2
