"""The rocprofv3 summary helpers on small synthetic result databases (CPU):
per-kernel medians of a memory counter, and the time during which at least
one batched step kernel ran (union of dispatch intervals, kernels of several
streams overlapping)."""
import sqlite3

import pytest

from paper_1905_04597_amd import profiling


def _db(tmp_path, name):
    path = str(tmp_path / name)
    db = sqlite3.connect(path)
    return path, db


def test_counter_medians_per_kernel_and_grid(tmp_path):
    path, db = _db(tmp_path, "pmc.db")
    db.execute("create table counters_collection (kernel_name text, counter_name text, value real, grid_size int)")
    rows = [("k", "FETCH_SIZE", v, 256) for v in (10.0, 30.0, 20.0)]
    rows += [("k", "FETCH_SIZE", 5.0, 512), ("k", "WRITE_SIZE", 99.0, 256), ("j", "FETCH_SIZE", 7.0, 256)]
    db.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    db.commit()
    got = profiling.counter(path, "FETCH_SIZE")
    assert got == {("k", 256): 20.0, ("k", 512): 5.0, ("j", 256): 7.0}


def test_batched_busy_is_the_union_of_intervals(tmp_path):
    path, db = _db(tmp_path, "kt.db")
    db.execute("create table kernels (name text, start int, end int)")
    a, b = "void glbm::batch_step_kernel<2, 2, 1>", "void glbm::batch_step_kernel<3, 3, 1>"
    rows = [
        (a, 0, 100), (b, 50, 160),          # overlapping: 0..160
        (a, 200, 300), (b, 300, 350),       # touching: 200..350
        (a, 400, 410), (b, 500, 520),       # apart: 10 + 20
        ("void glbm::step_kernel<5, 5, 1>", 0, 10000),  # not a batched kernel
    ]
    db.executemany("insert into kernels values (?, ?, ?)", rows)
    db.commit()
    busy_us, steps = profiling.batched_busy(path)
    assert busy_us == pytest.approx((160 + 150 + 10 + 20) / 1e3)
    assert steps == 3


def test_batched_busy_without_batched_kernels(tmp_path):
    path, db = _db(tmp_path, "kt0.db")
    db.execute("create table kernels (name text, start int, end int)")
    db.commit()
    assert profiling.batched_busy(path) == (0.0, 0)
