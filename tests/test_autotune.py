"""Autotuner table format and candidate space (CPU), and one tuning run (GPU)."""
import json

import numpy as np
import pytest

from paper_2311_02811_amd import autotune


def test_candidates_cover_orders_and_geometries():
    for cls in range(3):
        c = autotune.candidates(cls)
        assert {x["order"] for x in c} == {2, 3, "full"}
        assert all(x["block"] in (256, 512, 1024) for x in c)
    assert all(x["block"] != 1024 for x in autotune.candidates(2))


def test_table_round_trip_and_validation():
    classes = [dict(order=2, block=512, edges_per_thread=1), dict(order="full", block=1024,
               edges_per_thread=2), dict(order=3, block=256, edges_per_thread=8)]
    text = autotune.to_json(classes, 4096, 100000, 1.5)
    d = autotune.from_json(text)
    assert d["classes"] == classes and d["lds_max_vertices"] == 4096
    bad = json.loads(text)
    bad["classes"][0]["block"] = 384
    with pytest.raises(ValueError):
        autotune.from_json(json.dumps(bad))
    bad["classes"] = bad["classes"][:2]
    with pytest.raises(ValueError):
        autotune.from_json(json.dumps(bad))


def test_committed_table_is_valid():
    import os
    path = os.path.join(os.path.dirname(autotune.__file__), "tuning_gfx950.json")
    if not os.path.exists(path):
        pytest.skip("no tuning table committed")
    autotune.from_json(open(path).read())


@pytest.mark.gpu
def test_tune_small_batch_gives_exact_plan(tmp_path):
    torch = pytest.importorskip("torch")
    import graphgen
    import oracle
    import paper_2311_02811_amd as contour
    b = graphgen.batch(300, 9, median=500, n_hi=200000)
    s = torch.from_numpy(b.src).cuda()
    d = torch.from_numpy(b.dst).cuda()
    out = tmp_path / "t.json"
    autotune.tune(b.edge_off, b.vertex_off, s, d, reps=1, orders=(2, "full"), lds_max_vertices=2000,
                  wg_max_edges=50000, out_path=str(out))
    tuning = autotune.load_tuning(str(out))
    plan = contour.BatchPlan(b.edge_off, b.vertex_off, s, d, tuning=tuning)
    plan.launch()
    torch.cuda.synchronize()
    exp = oracle.uf_batch(b.edge_off, b.vertex_off, b.src, b.dst)
    assert np.array_equal(plan.labels.cpu().numpy(), exp)
    plan.close()
