"""Pins of the oracle neighbour finder and CA tracklet builder.

* neighbours: brute force over all (j, k) pairs of whole neighbouring rows on
  tiny inputs; exact straight lines give score 0 and the expected links;
* tracklets: chain extraction by an explicit graph walk; reciprocity and
  disjointness of the cleaned links.
"""
import numpy as np
import pytest

import oracle

P = oracle.default_params()


def brute_links(y, z, crow, n_units, wy=P["win_y"], wz=P["win_z"], smax=P["s_max"]):
    n = len(y)
    down = np.full(n, -1, np.int64)
    up = np.full(n, -1, np.int64)
    for u in range(n_units):
        for r in range(1, 151):
            b = u * 152 + r
            for i in range(crow[b], crow[b + 1]):
                best = None
                for j in range(crow[b - 1], crow[b]):
                    if abs(int(y[j]) - int(y[i])) > wy or abs(int(z[j]) - int(z[i])) > wz:
                        continue
                    for k in range(crow[b + 1], crow[b + 2]):
                        if abs(int(y[k]) - int(y[i])) > wy or abs(int(z[k]) - int(z[i])) > wz:
                            continue
                        dy = 2 * int(y[i]) - int(y[j]) - int(y[k])
                        dz = 2 * int(z[i]) - int(z[j]) - int(z[k])
                        s = dy * dy + dz * dz
                        if s <= smax and (best is None or (s, j, k) < best):
                            best = (s, j, k)
                if best:
                    down[i], up[i] = best[1], best[2]
    return down, up


def random_clusters(rng, n_units=1, per_row=(0, 6), T=60, spread=4.0):
    """Random clusters per row sorted by (ptime, ppad), with y/z near a few lines."""
    y, z, pt = [], [], []
    crow = [0]
    for u in range(n_units):
        lines = [(rng.uniform(-20, 20), rng.uniform(-0.8, 0.8), rng.uniform(5, T - 5),
                  rng.uniform(-1, 1)) for _ in range(3)]
        for r in range(152):
            pts = []
            for (y0, sy, t0, st) in lines:
                if rng.random() < 0.85:
                    yy = y0 + sy * r * 1.06 + rng.normal(0, 0.05)
                    tt = t0 + st * r * 0.3 + rng.normal(0, 0.1)
                    pts.append((yy, tt))
            for _ in range(rng.integers(*per_row)):
                pts.append((rng.uniform(-30, 30), rng.uniform(0, T)))
            rec = []
            for yy, tt in pts:
                tt = abs(tt)
                ptime = int(round(tt))
                rec.append((ptime, int(round(yy * 65536)), int(round(tt * 32768))))
            rec.sort()
            for ptime, yf, zf in rec:
                pt.append(ptime)
                y.append(yf)
                z.append(zf)
            crow.append(len(y))
    return dict(y_fx=np.array(y, np.int32), z_fx=np.array(z, np.int32),
                ptime=np.array(pt, np.uint16), crow_start=np.array(crow, np.uint32),
                n_units=n_units)


@pytest.mark.parametrize("seed", range(6))
def test_neighbours_match_bruteforce(seed):
    rng = np.random.default_rng(100 + seed)
    cl = random_clusters(rng, n_units=1 + seed % 2)
    down, up = oracle.find_neighbours(cl)
    bd, bu = brute_links(cl["y_fx"], cl["z_fx"], cl["crow_start"], cl["n_units"])
    assert np.array_equal(down, bd) and np.array_equal(up, bu)
    # the whole-row scan of the oracle agrees with its time-window scan
    d2, u2 = oracle.find_neighbours(cl, brute_force=True)
    assert np.array_equal(down, d2) and np.array_equal(up, u2)


def test_straight_line_gives_exact_links():
    # one cluster per row on an exact straight line in y and z
    y = np.array([int(1000 + 7000 * r) for r in range(152)], np.int32)
    z = np.array([int(3_000_000 + 4096 * r) for r in range(152)], np.int32)
    pt = (z // 32768).astype(np.uint16)
    crow = np.arange(153, dtype=np.uint32)
    cl = dict(y_fx=y, z_fx=z, ptime=pt, crow_start=crow, n_units=1)
    down, up = oracle.find_neighbours(cl)
    assert down[0] == -1 and up[0] == -1 and down[151] == -1 and up[151] == -1
    assert np.array_equal(down[1:151], np.arange(0, 150))
    assert np.array_equal(up[1:151], np.arange(2, 152))
    tl = oracle.build_tracklets(down, up)
    # rows 1..150 form one chain; rows 0 and 151 only via following
    assert list(tl["tl_start"]) == [1] and list(tl["tl_len"]) == [150]


def test_window_and_score_cuts():
    # middle cluster off the line by exactly the score limit and just beyond
    y = np.array([0, 32768, 0], np.int32)      # 2y - y - y = 65536 -> s = 2^32
    z = np.array([0, 0, 0], np.int32)
    cl = dict(y_fx=y, z_fx=z, ptime=np.zeros(3, np.uint16),
              crow_start=np.array([0] * 10 + [1, 2, 3] + [3] * 140, np.uint32), n_units=1)
    down, up = oracle.find_neighbours(cl)
    assert (down[1], up[1]) == (0, 2)
    cl["y_fx"] = np.array([0, 32769, 0], np.int32)
    down, up = oracle.find_neighbours(cl)
    assert (down[1], up[1]) == (-1, -1)


def graph_walk_tracklets(down, up, min_len):
    n = len(down)
    upc = [up[i] if up[i] >= 0 and down[up[i]] == i else -1 for i in range(n)]
    downc = [down[i] if down[i] >= 0 and up[down[i]] == i else -1 for i in range(n)]
    out = []
    for i in range(n):
        if downc[i] == -1 and upc[i] != -1:
            chain = [i]
            while upc[chain[-1]] != -1:
                chain.append(upc[chain[-1]])
            if len(chain) >= min_len:
                out.append(chain)
    return upc, downc, out


@pytest.mark.parametrize("seed", range(5))
def test_tracklets_match_graph_walk(seed):
    rng = np.random.default_rng(200 + seed)
    cl = random_clusters(rng, n_units=2)
    down, up = oracle.find_neighbours(cl)
    tl = oracle.build_tracklets(down, up)
    upc, downc, chains = graph_walk_tracklets(down, up, 5)
    assert np.array_equal(tl["upc"], upc) and np.array_equal(tl["downc"], downc)
    assert [c[0] for c in chains] == list(tl["tl_start"])
    assert [len(c) for c in chains] == list(tl["tl_len"])
    # cleaned links are reciprocal and chains are disjoint
    for i, k in enumerate(tl["upc"]):
        if k >= 0:
            assert tl["downc"][k] == i
    used = np.concatenate([np.array(c) for c in chains]) if chains else np.zeros(0)
    assert len(np.unique(used)) == len(used)
