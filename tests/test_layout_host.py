"""Host logic of the library's layout builder, compiled for the CPU: the vertex
order is a per-sheet permutation, aggregates are compact patches of the rest
shape, the workgroup/aggregate overlap maps are consistent, and the coarse
dimensions follow the aggregate cap."""

import ctypes
import os
import subprocess

import numpy as np
import pytest

from paper_2203_11938_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = [os.path.join(HERE, "host", "layout_check.cpp"),
       os.path.join(ROOT, "paper_2203_11938_amd", "csrc", "mesh_prep.cpp")]


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("layout") / "liblayout_check.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC",
                    "-I" + os.path.join(ROOT, "paper_2203_11938_amd", "csrc"), *SRC, "-o", out],
                   check=True)
    return ctypes.CDLL(out)


def run(lib, sheets, agg_size, max_aggs=128, rows=128):
    nv = np.array([s[0].shape[0] for s in sheets], np.int32)
    nt = np.array([s[1].shape[0] for s in sheets], np.int32)
    tris = np.ascontiguousarray(np.concatenate([s[1] for s in sheets]).astype(np.int32))
    rest = np.ascontiguousarray(np.concatenate([s[0] for s in sheets]).astype(np.float64))
    npins = np.array([len(s[2]) for s in sheets], np.int32)
    pins = np.ascontiguousarray(np.concatenate([np.asarray(s[2], np.int32) for s in sheets]))
    V = int(nv.sum())
    vold = np.zeros(V, np.int32)
    vagg = np.zeros(V, np.int32)
    counts = np.zeros(11, np.int32)
    err = ctypes.create_string_buffer(256)
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = lib.layout_check(len(sheets), P(nv), P(nt), P(tris), P(rest), P(npins), P(pins),
                          agg_size, max_aggs, rows, P(vold), P(vagg), P(counts), err, 256)
    assert rc == 0, err.value
    return vold, vagg, counts


def sheet(n, pins="top2"):
    rest, tris = W.grid_sheet(n)
    return rest, tris, W.pin_set(n, pins)


def test_order_is_a_permutation_and_aggregates_are_square_patches(lib):
    rest, tris, pins = sheet(64)
    vold, vagg, counts = run(lib, [(rest, tris, pins)], 64)
    assert np.array_equal(np.sort(vold), np.arange(64 * 64))
    assert counts[0] == 64 and counts[1] == 384   # 8x8 patches, 6 modes each
    assert counts[4] == 64 and counts[5] == 0 and counts[6] == 0
    assert counts[8] == 0                          # overlap maps cover every vertex
    assert counts[9] == 0                          # halo tables name the right vertices
    assert 0 < counts[10] < 128                    # 8x16 patches have a thin halo
    assert counts[7] == 13                         # blocks per row of the grid sheet
    # each aggregate is an 8x8 block of grid cells, each run of 16 (the middle level)
    # a 4x4 block
    ij = np.stack([vold % 64, vold // 64], 1)
    for a in range(64):
        m = ij[vagg == a]
        assert len(m) == 64
        assert np.ptp(m[:, 0]) == 7 and np.ptp(m[:, 1]) == 7
    for r in range(64 * 64 // 16):
        m = ij[16 * r:16 * r + 16]
        assert np.ptp(m[:, 0]) == 3 and np.ptp(m[:, 1]) == 3


def test_aggregate_cap_and_batches(lib):
    rest, tris, pins = sheet(200, "topedge")
    _, vagg, counts = run(lib, [(rest, tris, pins)], 64, max_aggs=128)
    assert counts[0] <= 128 and counts[1] == 6 * counts[0]
    sizes = np.bincount(vagg)
    # the cap's aggregate size, rounded up to whole runs of the middle level (16)
    assert sizes.max() == int(np.ceil(np.ceil(200 * 200 / 128) / 16) * 16)
    # a batch keeps every sheet's vertices in its own range
    sh = [sheet(n) for n in (16, 23, 40)]
    vold, vagg, counts = run(lib, sh, 64)
    off = np.cumsum([0] + [s[0].shape[0] for s in sh])
    for b in range(3):
        seg = vold[off[b]:off[b + 1]]
        assert np.array_equal(np.sort(seg), np.arange(off[b], off[b + 1]))
    assert counts[8] == 0 and counts[9] == 0


def test_pinned_only_aggregate_has_no_modes(lib):
    rest, tris, _ = sheet(16)
    pins = np.arange(16 * 16)[: 16 * 4]  # the first four rows pinned
    _, vagg, counts = run(lib, [(rest, tris, pins)], 16)
    # 16-vertex aggregates of a 16x16 sheet: 4x4 patches; the bottom row of patches
    # is all pinned
    assert counts[0] == 16 and counts[6] == 4 and counts[4] == 12


def test_no_coarse_space(lib):
    rest, tris, pins = sheet(32)
    vold, vagg, counts = run(lib, [(rest, tris, pins)], 0)
    assert counts[0] == 0 and counts[1] == 0 and counts[2] == 0
    assert np.array_equal(np.sort(vold), np.arange(32 * 32))
