"""Batched ensembles (persistent launch + hipGraph + autotuner) against solo evaluations and
the FP64 oracle.  Inputs follow the uneven-ensemble recipe of workloads.batch_instances."""
import math
import os

import numpy as np
import pytest
import torch

from gpu_common import TOL, assert_field, modes_pair, to_np
from paper_2212_10961_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def grf():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2212_10961_amd.grf as g
    return g


def _instances(orc, grf, count, side_hi, n_modes, seed, dim=2):
    inst = wl.batch_instances(count, seed=seed, side_lo=20, side_hi=side_hi, n_modes=n_modes)
    out = []
    for p in inst:
        shape = p["shape"] if dim == 2 else (p["shape"][0], p["shape"][1], 3)
        ell = p["ell"] if dim == 2 else (p["ell"][0], p["ell"][1], 2.0)
        (zo, po), m = modes_pair(orc, grf, dim, p["cov"], n_modes, p["seed"], math.sqrt(p["sigma2"]), ell)
        out.append(dict(shape=shape, ell=ell, sigma=math.sqrt(p["sigma2"]), zo=zo, po=po, m=m,
                        y=torch.full((int(np.prod(shape)),), float("nan"), device="cuda")))
    return out


@pytest.mark.parametrize("meth", ["direct_f32", "sep_f16", "sep_bf16", "sep_f16_x3", "sep_bf16_x3"])
def test_batch_matches_solo_and_oracle(orc, grf, meth):
    print(f"case batch small {meth}", flush=True)
    inst = _instances(orc, grf, 24, 300, 192, 31)
    plan = grf.Plan(meth, graph=True, autotune=False)
    plan.run([(d["m"], d["shape"], d["y"]) for d in inst])
    info = plan.info()
    assert info["replayed"] == 0 and info["work_items"] > 0
    for i, d in enumerate(inst):
        y = to_np(d["y"])
        solo = to_np(grf.field_grid(d["m"], d["shape"], method=meth)["y"])
        if meth == "direct_f32":
            np.testing.assert_array_equal(y, solo)  # same tile kernel, same tables
        else:
            rel = np.sqrt(np.mean((y - solo) ** 2) / np.mean(solo ** 2))
            assert rel <= 2 * TOL[meth]["rel"], (i, rel)
            if meth.endswith("_x3"):
                # without tuning a slice of at least 192 x 192 takes 128x128 tiles (selector
                # 1), else 64x64 (selector 2): the same tile code and tables as the solo call
                tile = 1 if d["shape"][0] >= 192 and d["shape"][1] >= 192 else 2
                same = to_np(grf.field_grid(d["m"], d["shape"], method=meth, tile=tile)["y"])
                np.testing.assert_array_equal(y, same, err_msg=f"batch[{i}] {d['shape']} tile {tile}")
        if i % 6 == 0:
            cells = wl.sample_cells(y.size, 200, 500 + i)
            ref = orc.field_cells(d["zo"], d["po"], d["sigma"], d["ell"], d["shape"], cells)
            assert_field(y[cells], ref, d["sigma"], meth, f"batch[{i}] {d['shape']}")
    plan.close()


def test_batch_graph_replay_and_updates(orc, grf):
    """Replays of the captured graph, with eager work between them, equal eager evaluations;
    new mode values at the same addresses are picked up by the replay (tables rebuilt in-graph)."""
    print("case batch graph replay", flush=True)
    inst = _instances(orc, grf, 10, 260, 128, 32)
    items = [(d["m"], d["shape"], d["y"]) for d in inst]
    plan = grf.Plan("sep_f16", graph=True, autotune=False)
    plan.run(items)
    first = [to_np(d["y"]).copy() for d in inst]
    for rep in range(4):
        scratch = torch.randn(1 << 20, device="cuda")  # eager work between replays
        _ = (scratch * 2.0).sum().item()
        for d in inst:
            d["y"].fill_(float("nan"))
        plan.run(items)
        assert plan.info()["replayed"] == 1
        for d, f in zip(inst, first):
            np.testing.assert_array_equal(to_np(d["y"]), f)
    # change the phases in place: the replay must use the new values
    for d in inst:
        d["m"].phi.add_(0.37)
    plan.run(items)
    assert plan.info()["replayed"] == 1
    for d in inst[:4]:
        solo = to_np(grf.field_grid(d["m"], d["shape"], method="sep_f16")["y"])
        y = to_np(d["y"])
        assert np.sqrt(np.mean((y - solo) ** 2) / np.mean(solo ** 2)) <= 2 * TOL["sep_f16"]["rel"]
    # a different output pointer is a new signature: rebuilt, not replayed
    items[0] = (inst[0]["m"], inst[0]["shape"], torch.empty_like(inst[0]["y"]))
    plan.run(items)
    assert plan.info()["replayed"] == 0
    plan.close()


def test_batch_direct_3d_and_no_graph(orc, grf):
    print("case batch direct 3d", flush=True)
    inst = _instances(orc, grf, 6, 150, 100, 33, dim=3)
    plan = grf.Plan("direct_f32", graph=False, autotune=False)
    plan.run([(d["m"], d["shape"], d["y"]) for d in inst])
    for d in inst:
        np.testing.assert_array_equal(to_np(d["y"]), to_np(grf.field_grid(d["m"], d["shape"])["y"]))
    plan.close()


def test_batch_sep_3d(orc, grf):
    print("case batch sep 3d", flush=True)
    inst = _instances(orc, grf, 6, 150, 100, 34, dim=3)
    plan = grf.Plan("sep_f16_x3", graph=True, autotune=True)
    plan.run([(d["m"], d["shape"], d["y"]) for d in inst])
    for d in inst:
        ref = orc.field_grid(d["zo"], d["po"], d["sigma"], d["ell"], d["shape"])
        assert_field(to_np(d["y"]), ref, d["sigma"], "sep_f16_x3", f"batch3d {d['shape']}")
    plan.close()


def test_autotune_cache(orc, grf, tmp_path):
    print("case autotune cache", flush=True)
    cache = tmp_path / "tune.txt"
    inst = _instances(orc, grf, 12, 600, 256, 35)
    items = [(d["m"], d["shape"], d["y"]) for d in inst]
    plan = grf.Plan("sep_f16", graph=True, autotune=True, tune_cache=str(cache))
    plan.run(items)
    plan.close()
    lines = [l for l in cache.read_text().splitlines() if l.strip()]
    assert lines and all(l.startswith("sep ") and l.split()[-1] in ("0", "1") for l in lines)
    ys = [to_np(d["y"]).copy() for d in inst]
    plan2 = grf.Plan("sep_f16", graph=True, autotune=True, tune_cache=str(cache))
    plan2.run(items)  # classes come from the cache: nothing new is appended
    plan2.close()
    assert cache.read_text().splitlines() == lines
    for d, y in zip(inst, ys):
        np.testing.assert_array_equal(to_np(d["y"]), y)


@pytest.mark.parametrize("meth", ["sep_f16", "direct_f32"])
def test_batch512_full_sampled(orc, grf, meth):
    """The 512-instance uneven ensemble, sides 64..1024, N=2048, one persistent launch:
    1024 sampled cells of every instance against the oracle (and four whole instances)."""
    print(f"case batch512 full {meth}", flush=True)
    inst = wl.batch_instances()
    items = []
    for p in inst:
        z, phi = grf.make_modes(2, p["cov"], p["n_modes"], p["seed"])
        m = grf.modes_from_tables(z, phi, math.sqrt(p["sigma2"]), p["ell"])
        items.append((m, p["shape"], torch.full((p["shape"][0] * p["shape"][1],), float("nan"), device="cuda")))
    plan = grf.Plan(meth, graph=True, autotune=meth != "direct_f32")
    plan.run(items)
    torch.cuda.synchronize()
    ys, refs = [], []
    whole = set(int(v) for v in np.argsort([p["shape"][0] * p["shape"][1] for p in inst])[[0, 1, 255, 511]])
    for i, p in enumerate(inst):
        zo, po = orc.sample_modes(2, p["cov"], p["n_modes"], p["seed"])
        cells = wl.sample_cells(p["shape"][0] * p["shape"][1], 1024, 600 + i)
        if i in whole and p["shape"][0] * p["shape"][1] <= 300_000:
            cells = np.arange(p["shape"][0] * p["shape"][1], dtype=np.int64)
        y = to_np(items[i][2])[cells]
        ref = orc.field_cells(zo, po, math.sqrt(p["sigma2"]), p["ell"], p["shape"], cells)
        assert np.isfinite(y).all(), (i, p["shape"])
        sg = math.sqrt(p["sigma2"])
        assert np.max(np.abs(y - ref)) <= TOL[meth]["band"] * sg, (i, p["shape"])
        ys.append(y)
        refs.append(ref)
    assert_field(np.concatenate(ys), np.concatenate(refs), 1.0, meth, f"batch512 all instances")
    plan.close()


@pytest.mark.parametrize("meth", ["direct_f32", "sep_f16", "sep_f16_x3"])
def test_batch_epilogue(orc, grf, meth):
    """Per-instance epilogues in the persistent launch: K = exp(mu + Y) and facies indices
    with each instance's own mu and thresholds, equal to solo calls with the same epilogue
    (bitwise for the direct form and for hi+lo with the same tile) and to the oracle."""
    print(f"case batch epilogue {meth}", flush=True)
    inst = _instances(orc, grf, 12, 260, 160, 36)
    rng = np.random.default_rng(7)
    items = []
    for i, d in enumerate(inst):
        C = int(np.prod(d["shape"]))
        mu = float(rng.uniform(-1.0, 1.0))
        thr = np.sort(rng.normal(0.0, 0.7, size=1 + i % 3)).astype(np.float32)
        out = {"k": torch.full((C,), float("nan"), device="cuda"),
               "ind": torch.full((C,), 255, dtype=torch.uint8, device="cuda")}
        if i % 2 == 0:
            out["y"] = d["y"]
        d.update(mu=mu, thr=thr, out=out)
        items.append((d["m"], d["shape"], out, mu, thr))
    plan = grf.Plan(meth, graph=True, autotune=False)
    plan.run(items)
    for i, d in enumerate(inst):
        k, ind = to_np(d["out"]["k"]), to_np(d["out"]["ind"])
        solo = grf.field_grid(d["m"], d["shape"], method=meth, mu=d["mu"], thresholds=d["thr"], want_k=True,
                              want_ind=True, tile=(None if not meth.endswith("_x3") else
                                                   (1 if d["shape"][0] >= 192 and d["shape"][1] >= 192 else 2)))
        if meth != "sep_f16":
            np.testing.assert_array_equal(k, to_np(solo["k"]), err_msg=f"K batch[{i}]")
            np.testing.assert_array_equal(ind, to_np(solo["ind"]), err_msg=f"ind batch[{i}]")
            if "y" in d["out"]:
                np.testing.assert_array_equal(to_np(d["out"]["y"]), to_np(solo["y"]))
        ref = orc.field_grid(d["zo"], d["po"], d["sigma"], d["ell"], d["shape"])
        kref = orc.lognormal(ref, d["mu"])
        band = TOL[meth]["band"] * d["sigma"]
        assert np.max(np.abs(k - kref) / kref) <= 1.2 * band + 1e-6, (i, meth)
        want = (ref[:, None] > d["thr"][None, :].astype(np.float64)).sum(axis=1)
        near = np.any(np.abs(ref[:, None] - d["thr"][None, :]) <= band, axis=1)
        assert not np.any((ind != want) & ~near), (i, meth)
        if "y" in d["out"]:
            assert_field(to_np(d["out"]["y"]), ref, d["sigma"], meth, f"epi batch[{i}]")
    plan.close()


def test_batch_new_weights_rebuild(orc, grf):
    """A new per-mode weight tensor (same z, phi) is a new batch signature: the plan rebuilds
    its descriptors instead of replaying the ones that point at the old weights."""
    print("case batch new weights", flush=True)
    inst = _instances(orc, grf, 6, 200, 96, 37)
    rng = np.random.default_rng(11)
    for rnd in range(2):
        for d in inst:
            d["m"].w = torch.as_tensor(rng.uniform(0.2, 1.8, size=96), dtype=torch.float64, device="cuda")
        items = [(d["m"], d["shape"], d["y"]) for d in inst]
        if rnd == 0:
            plan = grf.Plan("direct_f32", graph=True, autotune=False)
        plan.run(items)
        assert plan.info()["replayed"] == 0
        for i, d in enumerate(inst):
            np.testing.assert_array_equal(to_np(d["y"]), to_np(grf.field_grid(d["m"], d["shape"])["y"]),
                                          err_msg=f"round {rnd} batch[{i}]")
        plan.run(items)   # same weights again: replayed, same values
        assert plan.info()["replayed"] == 1
    wo = to_np(inst[0]["m"].w)
    ref = orc.field_points_w(inst[0]["zo"], inst[0]["po"], wo, inst[0]["sigma"], inst[0]["ell"],
                             orc.grid_centres(inst[0]["shape"]))
    assert_field(to_np(inst[0]["y"]), ref, inst[0]["sigma"], "direct_f32", "weighted batch[0]")
    plan.close()
