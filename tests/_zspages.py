"""Raw ZS page fixtures shared by the CPU pins and the GPU parity tests:
the hand-assembled example in tests/golden and helpers that build single
pages from (time, first pad, ADC list) runs."""
import os

import numpy as np

WORDS = 2048
HERE = os.path.dirname(os.path.abspath(__file__))


def load_example():
    """(pages [n, 2048] uint32, n_units, n_time_bins, expected dict)."""
    pages, samples, rows = [], [], []
    meta = {}
    for line in open(os.path.join(HERE, "golden", "zs_pages_example.txt")):
        line = line.split("#", 1)[0].split()
        if not line:
            continue
        if line[0] in ("units", "time_bins"):
            meta[line[0]] = int(line[1])
        elif line[0] == "page":
            pg = np.zeros(WORDS, np.uint32)
            w = [int(x, 16) for x in line[1:]]
            pg[:len(w)] = w
            pages.append(pg)
        elif line[0] == "sample":
            samples.append([int(x) for x in line[1:]])
        elif line[0] == "rows":
            rows.append([int(x) for x in line[1:]])
    n_ur = meta["units"] * 152
    rs = np.full(n_ur + 1, -1, np.int64)
    for a, b, v in rows:
        rs[a:b + 1] = v
    assert (rs >= 0).all()
    s = np.array(samples, np.int64).reshape(-1, 3)
    exp = dict(pad=s[:, 0].astype(np.uint16), time=s[:, 1].astype(np.uint16),
               adc=s[:, 2].astype(np.uint16), row_start=rs.astype(np.uint32))
    return np.array(pages), meta["units"], meta["time_bins"], exp


def page(unit, row, runs, header=None):
    """One page from runs [(time, first_pad, [adc, ...]), ...] (no checks:
    malformed pages are built on purpose by the tests)."""
    pg = np.zeros(WORDS, np.uint32)
    ns = sum(len(a) for _, _, a in runs)
    pg[0] = 0x5A53 | (1 << 16)
    pg[1] = unit | (row << 16)
    pg[2] = len(runs) | (ns << 16)
    bits = []
    for i, (t, p0, adcs) in enumerate(runs):
        pg[4 + i] = t | (p0 << 16) | ((len(adcs) - 1) << 24)
        bits += adcs
    st = 4 + len(runs)
    acc = 0
    for k, a in enumerate(bits):
        acc |= (int(a) & 0x3FF) << (10 * k)
    nw = (10 * len(bits) + 31) // 32
    for w in range(nw):
        pg[st + w] = (acc >> (32 * w)) & 0xFFFFFFFF
    if header:
        for i, v in header.items():
            pg[i] = v
    return pg
