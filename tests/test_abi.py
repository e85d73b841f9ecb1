"""C-ABI checks that need no GPU: the library loads, exports every function
include/tpc.h declares, and its host-side logic (defaults, geometry,
workspace sizing, argument validation) behaves as documented."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from paper_2208_07412_amd import tpc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tpc.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void\*|const char\*)\s+(tpc_\w+)\s*\(", src, re.M)))


def test_header_declares_the_five_calls():
    names = declared_functions()
    for f in ("tpc_cluster", "tpc_find_neighbours", "tpc_build_tracklets", "tpc_fit_tracks",
              "tpc_process_timeframe"):
        assert f in names
    assert sorted(tpc.EXPORTS) == names


def test_library_exports_every_declared_symbol():
    lib = tpc.load()
    out = subprocess.run(["nm", "-D", "--defined-only", tpc.library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT\s+(tpc_\w+)", out))
    for name in declared_functions():
        assert name in exported, name
        assert getattr(lib, name) is not None


def test_defaults_agree_with_oracle_readings():
    p = tpc.params()
    d = oracle.default_params()
    for k, v in d.items():
        if k in ("sigma_y", "sigma_z"):
            assert list(getattr(p, k)) == v
        else:
            assert getattr(p, k) == v, k
    p2 = tpc.params(noise_sigma=2.0)
    assert p2.qmax_min == oracle.default_params(2.0)["qmax_min"] == 10


def test_geometry_agrees_with_oracle():
    n1, x1, p1 = tpc.geometry()
    n2, x2, p2 = oracle.geometry()
    assert np.array_equal(n1, n2) and np.array_equal(x1, x2) and np.array_equal(p1, p2)


def test_workspace_size():
    a = tpc.workspace_size(36, 500, 600_000, 50_000)
    b = tpc.workspace_size(36, 10_500, 20_000_000, 1_500_000)
    assert 0 < a < b
    # the dominant term: per-tracklet row table of 152 int32
    assert b >= 1_500_000 * 152 * 4
    with pytest.raises(tpc.TpcError):
        tpc.workspace_size(0, 500, 10, 10)
    with pytest.raises(tpc.TpcError):
        tpc.workspace_size(1, 70_000, 10, 10)
    with pytest.raises(tpc.TpcError):  # tracklet ids must fit the 24-bit claim key
        tpc.workspace_size(1, 500, 10, (1 << 24) + 1)


def test_create_rejects_bad_arguments_before_touching_the_device():
    lib = tpc.load()
    ctx = ctypes.c_void_p()
    p = tpc.params()
    bad_sizes = tpc.TpcSizes(0, 500, 10, 10)
    assert lib.tpc_create(ctypes.byref(ctx), ctypes.byref(p), ctypes.byref(bad_sizes), None) == -1
    sizes = tpc.TpcSizes(1, 500, 10, 10)
    for field, val in (("min_tracklet", 1), ("snp_max", 1.5), ("chi2_max", 0.0)):
        q = tpc.params({field: val})
        assert lib.tpc_create(ctypes.byref(ctx), ctypes.byref(q), ctypes.byref(sizes), None) == -1
    q = tpc.params()
    q.sigma_y[3] = 0.0
    assert lib.tpc_create(ctypes.byref(ctx), ctypes.byref(q), ctypes.byref(sizes), None) == -1
    assert lib.tpc_cluster(None, None, None) == -1
    assert lib.tpc_sync(None, None) == -1


def test_status_strings():
    lib = tpc.load()
    assert lib.tpc_status_string(0) == b"ok"
    assert lib.tpc_status_string(-2) == b"capacity exceeded"
    assert lib.tpc_status_string(99) == b"unknown status"


def test_struct_layouts_match_header(tmp_path):
    # every field offset and struct size of the binding against the header,
    # as the C compiler lays them out
    structs = {"tpc_params": tpc.TpcParams, "tpc_sizes": tpc.TpcSizes,
               "tpc_zs_input": tpc.TpcZsInput, "tpc_zs_soa": tpc.TpcZsSoa,
               "tpc_compressed": tpc.TpcCompressed, "tpc_decoded_clusters": tpc.TpcDecoded,
               "tpc_merged": tpc.TpcMerged,
               "tpc_clusters": tpc.TpcClusters,
               "tpc_links": tpc.TpcLinks, "tpc_tracklets": tpc.TpcTracklets,
               "tpc_tracks": tpc.TpcTracks, "tpc_counts": tpc.TpcCounts,
               "tpc_tuning": tpc.TpcTuning}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "tpc.h"', "int main(void) {"]
    expect = []
    for cname, cls in structs.items():
        lines.append(f'  printf("%zu\\n", sizeof({cname}));')
        expect.append(ctypes.sizeof(cls))
        for fname, _ in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({cname}, {fname}));')
            expect.append(getattr(cls, fname).offset)
    lines.append("  return 0;\n}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src),
                           "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert got == expect


def test_tuning_defaults_and_validation():
    lib = tpc.load()
    t = tpc.TpcTuning()
    assert lib.tpc_tuning_default(ctypes.byref(t)) == 0
    assert (t.cl_window, t.cl_chunk, t.follow_block, t.follow_mode, t.refit_waves, t.cl_mode) == \
        (32, 8, 64, 2, 6, 2)
    assert lib.tpc_set_tuning(None, ctypes.byref(t)) == -1
    assert lib.tpc_get_tuning(None, ctypes.byref(t)) == -1
    assert lib.tpc_tuning_default(None) == -1
    assert ctypes.sizeof(tpc.TpcTuning) == 24
