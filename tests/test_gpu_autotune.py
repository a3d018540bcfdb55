"""Tile configurations (team shapes, grid sizes) and the autotuner: every
configuration gives bit-identical evaluations, and tuned choices are cached
and applied to new handles."""
import os

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

def _O():
    import paper_2303_07597_amd.otgs as O
    return O


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _handle(inst, mode):
    O = _O()
    return O.Handle([dict(labels=_dev(inst["labels"]), n_groups=inst["n_groups"], gamma=inst["gamma"],
                          mu=inst["mu"], x_src=_dev(inst["xs"]), x_tgt=_dev(inst["xt"]), cost_mode=mode,
                          cost_scale=0.0)])


def _evals(h, pts, O):
    out = []
    for mode in (O.OT_GS_DENSE, O.OT_GS_SNAPSHOT, O.OT_GS_SCREENED):
        for a, b in pts:
            ga, gb = torch.empty_like(a), torch.empty_like(b)
            obj = torch.empty(1, dtype=torch.float64, device="cuda")
            h.dual_grad(a, b, ga, gb, obj, mode=mode)
            out += [ga.cpu().numpy(), gb.cpu().numpy(), obj.cpu().numpy()]
    return out


def _instance(n_src=5000):
    # group sizes from 20 to over 1024 rows (5000 sources) or over 2048 rows
    # (12000): every bucket, split groups of either cost path too
    return synth.zipf_blobs(seed=51, n_src=n_src, n_tgt=2000, d=40, n_groups=40, gamma=0.05, mu=0.5)


@pytest.mark.parametrize("mode_name", ["OT_GS_COST_ONTHEFLY", "OT_GS_COST_MATERIALIZE"])
def test_every_tile_configuration_gives_the_same_result(mode_name):
    O = _O()
    inst = _instance(5000 if mode_name == "OT_GS_COST_ONTHEFLY" else 12000)
    h = _handle(inst, getattr(O, mode_name))
    a, b, _, _ = h.solve(max_iter=15, use_screen=0)
    a2 = (a + 0.001).contiguous()
    pts = [(a, b), (a2, b)]
    ref = _evals(h, pts, O)
    tried = 0
    NBUCKET = O.NBUCKET
    for bucket in range(NBUCKET + 1):
        cfg = h.get_tile_config(bucket)
        if cfg["n_tiles"] == 0:
            continue
        if mode_name == "OT_GS_COST_ONTHEFLY":
            nvar = 2 if 1 <= bucket <= 4 else 1
        else:
            # teams (or plain) / next tile in flight / LDS copy; bucket 0: teams
            # only; buckets past R = 32 (groups over 1024 rows): plain only
            nvar = 1 if bucket in (0, NBUCKET) else (3 if bucket <= 4 else 2 if bucket <= 8 else 1)
        for var in range(nvar):
            for gm in (1, 3):
                h.tile_config(bucket, var, gm)
                got = _evals(h, pts, O)
                for x, y in zip(ref, got):
                    np.testing.assert_array_equal(x, y)
                tried += 1
        h.tile_config(bucket, cfg["variant"], cfg["grid_mult"])
    assert tried >= 4


def test_autotune_caches_and_applies(tmp_path):
    O = _O()
    path = str(tmp_path / "tune.txt")
    os.environ["OTGS_AUTOTUNE_CACHE"] = path
    try:
        inst = _instance()
        h = _handle(inst, O.OT_GS_COST_ONTHEFLY)
        a, b, _, _ = h.solve(max_iter=10, use_screen=0)
        ref = _evals(h, [(a, b)], O)
        h.autotune(repeats=3)
        tuned = [h.get_tile_config(k) for k in range(O.NBUCKET + 1)]
        assert os.path.exists(path)
        lines = open(path).read().split("\n")
        assert sum(1 for x in lines if x.strip()) == sum(1 for t in tuned if t["n_tiles"] > 0)
        for x, y in zip(ref, _evals(h, [(a, b)], O)):
            np.testing.assert_array_equal(x, y)
        h2 = _handle(inst, O.OT_GS_COST_ONTHEFLY)
        assert [h2.get_tile_config(k) for k in range(O.NBUCKET + 1)] == tuned
    finally:
        del os.environ["OTGS_AUTOTUNE_CACHE"]


@pytest.mark.parametrize("mode_name", ["OT_GS_COST_ONTHEFLY", "OT_GS_COST_MATERIALIZE"])
def test_profile_tiles_times_and_leaves_results(mode_name):
    """The tile-launch timer (its launches recorded into a graph and
    replayed) returns a positive time, at the handle's own point and, for a
    materialised cost, at caller-order duals, and later evaluations give the
    same bits as before it ran."""
    O = _O()
    h = _handle(_instance(5000), getattr(O, mode_name))
    a, b, _, _ = h.solve(max_iter=10, use_screen=0)
    ref = _evals(h, [(a, b)], O)
    us = [h.profile_tiles(3)]
    if mode_name == "OT_GS_COST_MATERIALIZE":
        us.append(h.profile_tiles(3, alpha=a, beta=b))
    torch.cuda.synchronize()
    assert all(np.isfinite(u) and u > 0 for u in us), us
    for x, y in zip(_evals(h, [(a, b)], O), ref):
        np.testing.assert_array_equal(x, y)
