"""The autotuner and the launch-shape knobs it searches.

Every knob except chunk_paths changes speed only: where a wave leaves its
stepping loop (refill_lanes, max_quarters), how a windowed launch cuts its
work into jobs (job_split), and the window layout (window_kind,
window_margin) change neither the substeps of a path nor its random words
nor the fixed-order sums, so the results must be identical bit for bit.
The tuned shapes must survive a save / load round trip, and a batch must
still give each instance its solo result after batch tuning."""
import dataclasses
import os

import numpy as np
import pytest

from paper_1504_00084_amd import workloads as W
from gpu_helpers import say

pytestmark = pytest.mark.gpu

FIELDS = ("mean_x", "mean_y", "se_x", "se_y", "exit_frac")


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_00084_amd import mesh_sdd
    mesh_sdd.load()
    return mesh_sdd


def solve(M, ctx, h, inst, n_paths):
    m = M.mesh_sdd_num_interface_nodes(h)
    arrs, res = M.host_result(m)
    st = M.make_step(inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, paths_per_node=n_paths, mesh_step=inst.mesh_step)
    M.mesh_sdd_solve_interfaces(h, st, res)
    return M.result_dict(arrs, res, m)


def same(a, b, label):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), (label, k)
    assert a["executed_path_steps"] == b["executed_path_steps"], label


@pytest.mark.parametrize("which", ["front257", "rotbump129", "bump513"])
def test_speed_knobs_do_not_change_results(M, which):
    """front257: windowed kernel with three-field windows; rotbump129: the
    whole node tables in LDS; bump513: two-field windows over several
    blocks (kind and margin change the block layout)."""
    if which == "front257":
        inst = W.config3(n_paths=512)
    elif which == "rotbump129":
        inst = W.config2(n_paths=1024)
    else:
        inst = dataclasses.replace(max(W.config4(count=64), key=lambda it: it.n_xi * 1000 + it.sub_xi),
                                   n_paths=256)
    ctx = M.mesh_sdd_ctx_create(0)
    h = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP32))
    try:
        M.mesh_sdd_set_monitor(h, inst.rho)
        ref = solve(M, ctx, h, inst, inst.n_paths)
        shapes = [dict(refill_lanes=1, max_quarters=1), dict(refill_lanes=64, max_quarters=64),
                  dict(refill_lanes=40, max_quarters=3), dict(job_split=1), dict(job_split=4096),
                  dict(window_kind=1), dict(window_kind=2), dict(window_kind=1, window_margin=20),
                  dict(window_kind=1, window_margin=60), dict(window_kind=2, window_margin=10)]
        for kw in shapes:
            M.mesh_sdd_set_launch(ctx, M.make_launch(**kw))
            try:
                same(ref, solve(M, ctx, h, inst, inst.n_paths), "%s %s" % (which, kw))
            finally:
                M.mesh_sdd_set_launch(ctx, None)
        say("%s: %d launch shapes give the default shape's bits" % (which, len(shapes)))
    finally:
        M.mesh_sdd_destroy(h)
        M.mesh_sdd_ctx_destroy(ctx)


def test_autotune_save_load_round_trip(M, tmp_path):
    inst = W.config2(n_paths=20_000)
    ctx = M.mesh_sdd_ctx_create(0)
    h = M.mesh_sdd_create(ctx, M.desc_for(inst, M.FP32))
    try:
        M.mesh_sdd_set_monitor(h, inst.rho)
        st = M.make_step(inst.x, inst.y, inst.bnd_t0, inst.bnd_t1, paths_per_node=inst.n_paths)
        lo = M.mesh_sdd_autotune(h, st)
        say("tuned rotbump129: %s" % lo.as_dict())
        got = M.mesh_sdd_get_launch(h)
        for k in ("chunk_paths", "refill_lanes", "max_quarters"):
            assert getattr(got, k) == getattr(lo, k), k
        tuned = solve(M, ctx, h, inst, 4096)
        path = str(tmp_path / "tune.txt")
        M.mesh_sdd_tune_save(ctx, path)
        text = open(path).read()
        assert "bucket 129 129 0 0" in text
    finally:
        M.mesh_sdd_destroy(h)
        M.mesh_sdd_ctx_destroy(ctx)
    ctx2 = M.mesh_sdd_ctx_create(0)
    h2 = M.mesh_sdd_create(ctx2, M.desc_for(inst, M.FP32))
    try:
        M.mesh_sdd_tune_load(ctx2, path)
        got2 = M.mesh_sdd_get_launch(h2)
        for k in ("chunk_paths", "refill_lanes", "max_quarters"):
            assert getattr(got2, k) == getattr(lo, k), k
        M.mesh_sdd_set_monitor(h2, inst.rho)
        same(tuned, solve(M, ctx2, h2, inst, 4096), "after load")
        bad = str(tmp_path / "bad.txt")
        with open(bad, "w") as f:
            f.write("bucket 129 129 0 0 100 56 16 0 0 0\n")   # chunk 100 is not a multiple of 64
        with pytest.raises(M.MeshSddError) as e:
            M.mesh_sdd_tune_load(ctx2, bad)
        assert e.value.code == M.E_INVAL
    finally:
        M.mesh_sdd_destroy(h2)
        M.mesh_sdd_ctx_destroy(ctx2)


def test_autotune_batch_then_batch_equals_alone(M):
    """Batch tuning (each bucket, then the multi-instance knobs) on eight
    instances of the mix at reduced path counts; afterwards every
    instance's result inside the tuned batch equals its tuned solve alone."""
    insts = [dataclasses.replace(it, n_paths=max(256, it.n_paths // 200 // 64 * 64)) for it in W.config4(count=8)]
    ctx = M.mesh_sdd_ctx_create(0)
    hs = [M.mesh_sdd_create(ctx, M.desc_for(it, M.FP32)) for it in insts]
    try:
        steps = []
        for h, it in zip(hs, insts):
            M.mesh_sdd_set_monitor(h, it.rho)
            steps.append(M.make_step(it.x, it.y, it.bnd_t0, it.bnd_t1, paths_per_node=it.n_paths))
        lo = M.mesh_sdd_autotune_batch(hs, steps, scale_down=4)
        say("batch shape: %s" % lo.as_dict())
        alone = [solve(M, ctx, h, it, it.n_paths) for h, it in zip(hs, insts)]
        pairs = [M.host_result(M.mesh_sdd_num_interface_nodes(h)) for h in hs]
        M.mesh_sdd_solve_batch(hs, steps, [r for _, r in pairs])
        for q, (h, it) in enumerate(zip(hs, insts)):
            same(alone[q], M.result_dict(pairs[q][0], pairs[q][1], M.mesh_sdd_num_interface_nodes(h)), it.name)
        say("tuned batch of %d == alone (bitwise)" % len(insts))
    finally:
        for h in hs:
            M.mesh_sdd_destroy(h)
        M.mesh_sdd_ctx_destroy(ctx)
