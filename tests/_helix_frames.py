"""Frames built from exact helices, for the pins of the segment merging and
the T0 / z fit: every crossing of a helix from the origin with the pad-row
planes of all 36 sectors (one revolution, |z| <= 250 cm), grouped into the
per-sector segments a tracker would produce (one per sector and leg), with
cluster positions in fixed point and the track parameters of each segment's
outward fit at its innermost row.  Written from the detector and drift
definitions: local x of row r = 85 + 160 r / 151 cm, sector s centred at
((s mod 18) + 0.5) 20 deg, side A (s < 18) for z > 0, drift coordinate
z_d = T0 / 2 + 250 - |z| cm, curvature C = dphi/ds = -b q/pT."""
import numpy as np

NROW = 152
B = 0.299792458e-3 * 5.0


def row_x_fx(r):
    num = (85 * 151 + 160 * np.asarray(r, np.int64)) * 65536
    return (2 * num + 151) // (2 * 151)


def helix_segments(phi0, qpt, tgl, t0, frame=0):
    """Segments [(unit, leg, [(row, y, z_d, s), ...] ascending row), ...] of a
    helix from the origin, and its curvature."""
    C = -B * qpt
    cx, cy = -np.sin(phi0) / C, np.cos(phi0) / C
    xr = row_x_fx(np.arange(NROW)) / 65536.0
    segs = {}
    for a in range(18):
        al = (a + 0.5) * np.pi / 9
        ca, sa = np.cos(al), np.sin(al)
        nc, mc = ca * cx + sa * cy, -sa * cx + ca * cy
        for r in range(NROW):
            k = C * (xr[r] - nc)
            if abs(k) > 1:
                continue
            for br in (0, 1):
                rel = np.arcsin(k) if br == 0 else np.pi - np.arcsin(k)
                psi = al + rel
                turn = (psi - phi0) if C > 0 else (phi0 - psi)
                turn = np.mod(turn, 2 * np.pi)
                s = turn / abs(C)
                y = mc - np.cos(rel) / C
                if abs(y) > xr[r] * np.tan(np.pi / 18):
                    continue
                z = tgl * s
                if abs(z) > 250 or z == 0:
                    continue
                unit = frame * 36 + a + (18 if z < 0 else 0)
                leg = 1 if np.cos(rel) > 0 else -1
                zd = 0.5 * t0 + 250 - abs(z)
                segs.setdefault((unit, leg), []).append((r, y, zd, s, psi))
    out = []
    for (unit, leg), pts in sorted(segs.items()):
        pts.sort()
        out.append((unit, leg, pts))
    return out, C


def segment_track(unit, pts, C, tgl):
    """Parameters (y, z - anchor, sin phi, tan lambda, q/pT) of the outward
    fit at the innermost row, the anchor (drift z of that cluster, fixed
    point) and the row."""
    r, y, zd, s, psi = pts[0]
    al = ((unit % 36) % 18 + 0.5) * np.pi / 9
    # direction of motion psi (global); outward in the sector when cos > 0
    outward = np.cos(psi - al) > 0
    phi_fit = psi if outward else psi + np.pi
    c_fit = C if outward else -C
    dzd_ds = -abs(tgl) * (1 if outward else -1)
    anchor = int(np.rint(zd * 65536))
    par = np.array([y, zd - anchor / 65536.0, np.sin(phi_fit - al), dzd_ds, -c_fit / B],
                   np.float32)
    return par, anchor, r


def build_frame(helices, n_units):
    """Clusters (canonical order by unit and row) and tracks of the given
    segments: helices = [(segments, C, tgl), ...]; returns clusters, tracks
    and the helix index of every track."""
    items = []  # (unit, row, y_fx, z_fx, track)
    tracks = []
    for hi, (segs, C, tgl) in enumerate(helices):
        for unit, leg, pts in segs:
            if len(pts) < 3:
                continue
            par, anchor, row = segment_track(unit, pts, C, tgl)
            t = len(tracks)
            tracks.append((par, anchor, row, hi))
            for (r, y, zd, s, psi) in pts:
                items.append((unit, r, int(np.rint(y * 65536)), int(np.rint(zd * 65536)), t))
    items.sort(key=lambda v: (v[0], v[1], v[3], v[4]))
    n = len(items)
    ur = np.array([it[0] * NROW + it[1] for it in items], np.int64)
    crow = np.searchsorted(ur, np.arange(n_units * NROW + 1), side="left").astype(np.uint32)
    clusters = dict(crow_start=crow, y_fx=np.array([it[2] for it in items], np.int32),
                    z_fx=np.array([it[3] for it in items], np.int32))
    hits = [[] for _ in tracks]
    for c, it in enumerate(items):
        hits[it[4]].append(c)
    hs = np.concatenate([[0], np.cumsum([len(h) for h in hits])]).astype(np.uint32)
    trk = dict(par=np.array([t[0] for t in tracks], np.float32).reshape(-1, 5),
               z_anchor=np.array([t[1] for t in tracks], np.int32),
               row=np.array([t[2] for t in tracks], np.uint8), hit_start=hs,
               hits=np.concatenate([np.array(h, np.int64) for h in hits]).astype(np.uint32))
    return clusters, trk, np.array([t[3] for t in tracks])
