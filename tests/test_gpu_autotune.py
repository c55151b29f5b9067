"""The autotuner on the GPU: it writes a valid cache, reads it back without timing, ignores an
invalid one, and every launch choice it can make (radix order per transform length, splat
tile) gives the default solve's result within 1e-6 (relative L2): the choices change the time,
not the iteration."""

import json
import os

import numpy as np
import pytest

from oracle import epr_oracle as O
from synthetic import workload
from tests.helpers import api_objects, oracle_lines, rel_l2, requires_gpu, to_dev, to_np

pytestmark = [pytest.mark.gpu, requires_gpu]

N_ITER = 6


def fresh_ctx():
    # a handle of its own: tuned choices stay on it, not on the shared one of other tests
    from paper_2601_22793_amd import Context
    return Context(0)


def problem(shape, seed=0):
    w = workload("nonlocal-poly8-2048", shape=shape, n_iter=N_ITER)
    w.seed += seed
    obj = w.true_object()
    d = w.add_noise(O.forward(obj["phase"], obj["absorb"], oracle_lines(w), O.NONLOCAL))
    return w, d


def solve(c, w, d):
    geom, spec, mat = api_objects(w)
    return to_np(c.solve(to_dev(d), geom, spec, mat, "nonlocal", w.n_iter, w.relaxation))


def batch_entry(w, d):
    import torch
    geom, spec, mat = api_objects(w)
    return (to_dev(d), torch.zeros(w.shape, dtype=torch.float32, device="cuda"), geom, spec, mat)


def test_autotune_writes_and_reuses_its_cache(tmp_path):
    w, d = problem((1024, 1024))
    c = fresh_ctx()
    try:
        ref = solve(c, w, d)
        path = str(tmp_path / "tune.json")
        print("autotune 1024x1024, 8 lines", flush=True)
        got = c.autotune([batch_entry(w, d)], "nonlocal", relaxation=w.relaxation,
                         cache_json=path)
        assert set(got) >= {"splat_tx", "splat_ty", "row_512", "col_1024"}
        assert 0 <= got["row_512"] < 3 and 0 <= got["col_1024"] < 3
        assert got["splat_tx"] * got["splat_ty"] <= 4096
        tuned = solve(c, w, d)
        assert rel_l2(tuned, ref) <= 1e-6
        # a valid cache is taken as it is (nothing timed, file unchanged)
        before = open(path).read()
        c2 = fresh_ctx()
        try:
            c2.autotune([batch_entry(w, d)], "nonlocal", cache_json=path)
            assert open(path).read() == before
            assert rel_l2(solve(c2, w, d), tuned) <= 1e-6
        finally:
            c2.close()
    finally:
        c.close()


def test_invalid_cache_is_ignored_and_rewritten(tmp_path):
    w, d = problem((256, 320), 1)
    path = str(tmp_path / "bad.json")
    # 64 x 64 with 8 lines needs 8 * 66 * 66 * 4 = 139 KB of LDS: fits; 128 x 32 with 16 lines
    # would not, but these problems have 8 lines: use a tile over 4096 pixels instead
    with open(path, "w") as fh:
        json.dump({"splat_tx": 128, "splat_ty": 64}, fh)
    c = fresh_ctx()
    try:
        got = c.autotune([batch_entry(w, d)], "nonlocal", cache_json=path)
        assert got["splat_tx"] * got["splat_ty"] <= 4096
        with open(path, "w") as fh:
            json.dump({"splat_tx": 64, "splat_ty": 32, "col_1024": 7}, fh)   # out of range
        got = c.autotune([batch_entry(w, d)], "nonlocal", cache_json=path)
        assert got.get("col_1024", 0) < 3
    finally:
        c.close()


@pytest.mark.parametrize("key,nvar,shape", [("row_512", 3, (1024, 1024)),
                                            ("col_1024", 3, (1024, 1024)),
                                            ("row_1024", 3, (1024, 2048)),
                                            ("col_2048", 3, (2048, 1024)),
                                            ("row_1280", 3, (240, 2560)),
                                            ("col_2160", 3, (2160, 256))])
def test_every_radix_order_gives_the_default_solve(tmp_path, key, nvar, shape):
    w, d = problem(shape, 2)
    c = fresh_ctx()
    try:
        ref = solve(c, w, d)
        for v in range(1, nvar):
            path = str(tmp_path / f"{key}_{v}.json")
            with open(path, "w") as fh:
                json.dump({"splat_tx": 64, "splat_ty": 32, key: v}, fh)
            c.autotune([batch_entry(w, d)], "nonlocal", cache_json=path)
            err = rel_l2(solve(c, w, d), ref)
            print(f"{key} order {v} on {shape}: rel L2 vs order 0 {err:.2e}", flush=True)
            assert err <= 1e-6, (key, v)
    finally:
        c.close()


@pytest.mark.parametrize("tile", [(32, 32), (64, 16), (128, 32)])
def test_splat_tiles_give_the_default_solve(tmp_path, tile):
    w, d = problem((256, 320), 3)
    c = fresh_ctx()
    try:
        ref = solve(c, w, d)
        path = str(tmp_path / "tile.json")
        with open(path, "w") as fh:
            json.dump({"splat_tx": tile[0], "splat_ty": tile[1]}, fh)
        c.autotune([batch_entry(w, d)], "nonlocal", cache_json=path)
        assert rel_l2(solve(c, w, d), ref) <= 1e-6
    finally:
        c.close()


@pytest.mark.parametrize("lines", [2, 4])
def test_lines_per_row_workgroup_give_the_default_solve(tmp_path, lines):
    # the row pass with several lines per workgroup, transformed one after the other (shared
    # thickness stencil): single and batched solves, 1024^2 and 2048-wide rows (both row
    # lengths of the 512-thread class), 2560-wide rows (the 1024-thread class), and a line
    # count the group size does not divide (the last group is short)
    import torch
    c = fresh_ctx()
    try:
        path = str(tmp_path / "lines.json")
        with open(path, "w") as fh:
            json.dump({"splat_tx": 64, "splat_ty": 32, "row_lines": lines}, fh)
        default = str(tmp_path / "default.json")
        with open(default, "w") as fh:
            json.dump({"splat_tx": 64, "splat_ty": 32, "row_lines": 1}, fh)
        for shape, n_lines in [((1024, 1024), 8), ((256, 2048), 8), ((200, 320), 3),
                               ((120, 2560), 8)]:
            w = workload("nonlocal-poly8-2048" if n_lines == 8 else "nonlocal-mono-2048",
                         shape=shape, n_iter=N_ITER)
            if n_lines == 3:
                from synthetic import bremsstrahlung_bins
                w.energies_kev, w.weights = bremsstrahlung_bins(3, np.random.default_rng(9))
            obj = w.true_object()
            d = w.add_noise(O.forward(obj["phase"], obj["absorb"], oracle_lines(w), O.NONLOCAL))
            c.autotune([batch_entry(w, d)], "nonlocal", cache_json=default)
            ref = solve(c, w, d)
            c.autotune([batch_entry(w, d)], "nonlocal", cache_json=path)
            got = solve(c, w, d)
            print(f"{lines} lines per row workgroup {shape} x {n_lines}: rel L2 "
                  f"{rel_l2(got, ref):.2e}", flush=True)
            assert rel_l2(got, ref) <= 1e-6, shape
            e = batch_entry(w, d)
            c.solve_batched([e], "nonlocal", w.n_iter, w.relaxation)
            torch.cuda.synchronize()
            assert rel_l2(to_np(e[1]), ref) <= 1e-6, shape
    finally:
        c.close()


def test_invalid_row_lines_in_the_cache_are_ignored(tmp_path):
    w, d = problem((256, 320), 1)
    c = fresh_ctx()
    try:
        path = str(tmp_path / "bad.json")
        with open(path, "w") as fh:
            json.dump({"splat_tx": 64, "splat_ty": 32, "row_lines": 3}, fh)
        got = c.autotune([batch_entry(w, d)], "nonlocal", cache_json=path)
        assert got["row_lines"] in (1, 2, 4)
    finally:
        c.close()


@pytest.mark.parametrize("key,shape", [("row_512", (1024, 1024)), ("row_1024", (256, 2048))])
def test_grouped_row_pass_radix_orders_give_the_default_solve(tmp_path, key, shape):
    # every radix order of the row transforms gives the default solve with four lines per
    # row-pass workgroup too
    w, d = problem(shape, 2)
    c = fresh_ctx()
    try:
        ref = solve(c, w, d)
        for v in range(3):
            path = str(tmp_path / f"{key}_{v}.json")
            with open(path, "w") as fh:
                json.dump({"splat_tx": 64, "splat_ty": 32, "row_lines": 4, key: v}, fh)
            c.autotune([batch_entry(w, d)], "nonlocal", cache_json=path)
            err = rel_l2(solve(c, w, d), ref)
            print(f"grouped row pass, {key} order {v} on {shape}: rel L2 {err:.2e}", flush=True)
            assert err <= 1e-6, (key, v)
    finally:
        c.close()
