"""The C-ABI library loads and exports every entry point include/glbm.h declares.

Host-side checks only (configuration validation and sizing): no kernel is
launched, so these run without a GPU.
"""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1905_04597_amd import glbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "glbm.h")

pytestmark = pytest.mark.skipif(not os.path.exists(glbm.LIB_PATH), reason="libglbm.so not built")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(glbm_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_binding_symbols():
    assert declared_functions() == sorted(glbm.SYMBOLS)


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", glbm.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r"\bT (glbm_\w+)", out.stdout))
    missing = [s for s in declared_functions() if s not in exported]
    assert not missing, missing
    lib = glbm.load()
    for s in declared_functions():
        assert hasattr(lib, s)


def test_population_bytes_layout():
    # one dimension: one padded row of nxp = 64 + nx + N columns rounded up to
    # a multiple of 64, times the element size, each plane rounded to 256 bytes
    def nxp(nx, N):
        return (64 + nx + N + 63) // 64 * 64
    c = glbm.make_config(1, 3, 0, 2000, 1, kn=0.01, bc_x="eq_ends")
    assert glbm.population_bytes(c) == ((7 * nxp(2000, 3) * 4 + 255) // 256) * 256
    c = glbm.make_config(1, 4, 0, 1000, 1, tau=0.7, storage="bf16_shifted")
    assert glbm.population_bytes(c) == 9 * ((nxp(1000, 4) * 2 + 255) // 256 * 256)
    # two dimensions: compact rows of nx columns, each plane rounded up to 256
    # bytes, whatever nx
    c = glbm.make_config(2, 5, 5, 4096, 1024, kn=0.1, bc_y="wall", storage="f32")
    assert glbm.population_bytes(c) == 121 * 1024 * 4096 * 4
    c = glbm.make_config(2, 5, 5, 4096, 1024, kn=0.1, bc_y="wall", storage="bf16_shifted_sr")
    assert glbm.population_bytes(c) == 121 * 1024 * 4096 * 2
    c = glbm.make_config(2, 3, 3, 4, 37, kn=0.1, bc_y="wall", storage="f32_shifted")
    assert glbm.population_bytes(c) == 49 * ((37 * 4 * 4 + 255) // 256 * 256)
    c = glbm.make_config(2, 6, 6, 63, 100, tau=0.8, storage="bf16_shifted_sr")
    assert glbm.population_bytes(c) == 169 * ((100 * 63 * 2 + 255) // 256 * 256)
    c = glbm.make_config(2, 6, 6, 70, 33, tau=0.8, storage="bf16_shifted_sr")
    assert glbm.population_bytes(c) == 169 * ((33 * 70 * 2 + 255) // 256 * 256)
    # G-D1Q(2N+2) axes: 2N+2 velocities, ghosts as deep as the fastest one (2N+1)
    c = glbm.make_config(1, 3, 0, 500, 1, kn=0.01, bc_x="eq_ends", even_x=True)
    assert glbm.population_bytes(c) == 8 * nxp(500, 7) * 4
    c = glbm.make_config(2, 1, 3, 4, 41, kn=0.1, bc_y="wall", even_y=True, storage="f32_shifted")
    assert glbm.population_bytes(c) == 3 * 8 * ((41 * 4 * 4 + 255) // 256 * 256)


@pytest.mark.parametrize("kwargs,needle", [
    (dict(dims=4, level_x=1), "dims"),
    (dict(dims=1, level_x=0, nx=10), "level_x"),
    (dict(dims=1, level_x=14, nx=10), "level_x"),
    (dict(dims=2, level_x=3, level_y=3, nx=4, ny=5, bc_y="wall"), "fastest y velocity"),
    (dict(dims=2, level_x=2, level_y=2, nx=4, ny=8, bc_x="eq_ends", bc_y="wall"), "combined"),
    (dict(dims=2, level_x=7, level_y=7, nx=8192, ny=4096, bc_y="wall"), "4 GiB"),
    # the even axis reaches 2N+1 rows: ny >= 2 (2N+1) with walls
    (dict(dims=2, level_x=1, level_y=3, nx=4, ny=13, bc_y="wall", even_y=True), "fastest y velocity"),
    (dict(dims=2, level_x=1, level_y=3, nx=4, ny=6, even_y=True), "periodic ny"),
])
def test_invalid_configs_are_rejected(kwargs, needle):
    c = glbm.make_config(**kwargs)
    assert glbm.load().glbm_population_bytes(ctypes.byref(c)) == 0
    assert needle in glbm.load().glbm_last_error().decode()


def test_required_bytes_counts_both_buffers_and_the_statistics():
    # two population buffers plus the FP64 statistics: one row of 13 partial
    # sums per block of 256 nodes (at most 2048 rows, the blocks stride over
    # larger lattices) and the 13 totals
    c = glbm.make_config(2, 5, 5, 4096, 1024, kn=0.1, bc_y="wall", storage="f32_shifted")
    assert glbm.required_bytes(c) == 2 * glbm.population_bytes(c) + 8 * 13 * (2048 + 1)
    c = glbm.make_config(1, 3, 0, 2000, 1, kn=0.01, bc_x="eq_ends")
    assert glbm.required_bytes(c) == 2 * glbm.population_bytes(c) + 8 * 13 * (8 + 1)
    # lattices whose step starts with a wall pre-pass (three dimensions, the
    # symmetric G-D1Q(2N+2) products at N = 6 and 7, with walls): plus a wall
    # factor per (x, z) column and wall
    c = glbm.make_config(2, 7, 7, 1024, 64, kn=0.1, bc_y="wall", even_x=True, even_y=True)
    assert glbm.required_bytes(c) == 2 * glbm.population_bytes(c) + 8 * 13 * (256 + 1) + 4 * 2 * 1024
    c = glbm.make_config(3, 1, 3, 256, 128, kn=0.1, bc_y="wall", level_z=1, nz=128)
    assert glbm.required_bytes(c) == 2 * glbm.population_bytes(c) + 8 * 13 * (2048 + 1) + 4 * 2 * 256 * 128
    c = glbm.make_config(3, 1, 3, 256, 128, tau=0.8, level_z=1, nz=128)
    assert glbm.required_bytes(c) == 2 * glbm.population_bytes(c) + 8 * 13 * (2048 + 1)
    bad = glbm.make_config(4, 1)
    assert glbm.load().glbm_required_bytes(ctypes.byref(bad)) == 0


@pytest.mark.parametrize("kwargs", [
    dict(dims=2, level_x=3, level_y=3, nx=8, ny=16, tau=0.8, bc_y="wall"),
    dict(dims=1, level_x=3, nx=100, tau=0.8, g=1e-5),
])
def test_round_to_nearest_bf16_is_refused_for_driven_flows(kwargs):
    c = glbm.make_config(**kwargs, storage="bf16_shifted")
    assert glbm.load().glbm_population_bytes(ctypes.byref(c)) == 0
    assert "stalls driven flows" in glbm.load().glbm_last_error().decode()
    # undriven lattices keep it
    c = glbm.make_config(1, 3, 0, 100, 1, tau=0.8, storage="bf16_shifted")
    assert glbm.population_bytes(c) > 0


def test_three_dimensional_layout_and_checks():
    # [q][z][y][x], compact rows, each plane rounded to 256 bytes
    c = glbm.make_config(3, 1, 1, 70, 9, tau=0.7, level_z=1, nz=6, storage="f32")
    assert glbm.population_bytes(c) == 27 * ((6 * 9 * 70 * 4 + 255) // 256 * 256)
    c = glbm.make_config(3, 1, 3, 4, 20, kn=0.1, bc_y="wall", level_z=1, nz=5, storage="f32_shifted")
    assert glbm.population_bytes(c) == 63 * ((5 * 20 * 4 * 4 + 255) // 256 * 256)
    lib = glbm.load()
    bad = glbm.make_config(3, 1, 1, 8, 4, tau=0.8, level_z=3, nz=2)
    assert lib.glbm_population_bytes(ctypes.byref(bad)) == 0
    assert "fastest z velocity" in lib.glbm_last_error().decode()
    bad = glbm.make_config(3, 1, 1, 8, 4, tau=0.8, level_z=1, nz=4, bc_x="eq_ends")
    assert lib.glbm_population_bytes(ctypes.byref(bad)) == 0
    assert "periodic in x" in lib.glbm_last_error().decode()


def test_axis_kind_is_validated():
    c = glbm.make_config(2, 2, 2, 8, 8, tau=0.8)
    c.kind_y = 5
    assert glbm.load().glbm_population_bytes(ctypes.byref(c)) == 0
    assert "axis kinds" in glbm.load().glbm_last_error().decode()


def test_create_rejects_missing_buffers_without_touching_the_gpu():
    lib = glbm.load()
    c = glbm.make_config(1, 2, 0, 16, 1, tau=0.7)
    h = ctypes.c_void_p()
    assert lib.glbm_create(ctypes.byref(c), None, None, None, ctypes.byref(h)) == -1
    assert "buffers" in lib.glbm_last_error().decode()
    assert lib.glbm_step(None, 1) == -1


def test_batch_entry_points_reject_bad_arguments_without_touching_the_gpu():
    lib = glbm.load()
    out = ctypes.c_void_p()
    opt = glbm.BatchOptions(96, 0, 0)
    assert lib.glbm_batch_create(None, 0, ctypes.byref(opt), None, ctypes.byref(out)) == -1
    assert "tile_nodes" in lib.glbm_last_error().decode()
    opt = glbm.BatchOptions(128, 7, 0)
    assert lib.glbm_batch_create(None, 0, ctypes.byref(opt), None, ctypes.byref(out)) == -1
    assert "order" in lib.glbm_last_error().decode()
    opt = glbm.BatchOptions(128, 1, -1)
    assert lib.glbm_batch_create(None, 0, ctypes.byref(opt), None, ctypes.byref(out)) == -1
    assert "graph_steps" in lib.glbm_last_error().decode()
    opt = glbm.BatchOptions(128, 1, 0, -5)
    assert lib.glbm_batch_create(None, 0, ctypes.byref(opt), None, ctypes.byref(out)) == -1
    assert "resident_nodes" in lib.glbm_last_error().decode()
    for streams in (9, -1):
        opt = glbm.BatchOptions(128, 1, 0, 0, streams)
        assert lib.glbm_batch_create(None, 0, ctypes.byref(opt), None, ctypes.byref(out)) == -1
        assert "streams" in lib.glbm_last_error().decode()
    assert lib.glbm_batch_create(None, 0, None, None, ctypes.byref(out)) == -1
    assert "at least one member" in lib.glbm_last_error().decode()
    assert lib.glbm_batch_create(None, 1, None, None, None) == -1
    assert lib.glbm_batch_step(None, 1) == -1
    assert lib.glbm_batch_destroy(None) == 0
    assert lib.glbm_batch_update(None, None, 0) == -1
