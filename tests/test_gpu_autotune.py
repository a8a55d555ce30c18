"""The autotuner returns tunables that keep results exact (single-root and batch)."""
import numpy as np
import pytest

import graphgen
import oracle
import paper_1604_02844_amd as bfs
from paper_1604_02844_amd import tune
from tests.gpu_helpers import check_root, load, torch_mod

pytestmark = pytest.mark.gpu


def test_autotune_single_and_batch(tmp_path, monkeypatch):
    torch = torch_mod()
    monkeypatch.setenv("BFS_TUNE_CACHE", str(tmp_path / "tune.json"))
    g = graphgen.rmat(14, 16, seed=51)
    dg = load(g)
    roots = graphgen.pick_roots(g, 8, seed=52)
    best = tune.tuned(dg, roots[:4], "rmat", mode=0)
    assert best["update_mode"] in (1, 2) and best["block_size"] in (256, 512, 1024)
    assert best == bfs.bfs_graph_get_tunables(dg)  # the winner is applied to the graph
    for r in roots[4:]:
        check_root(g, dg, int(r))
    again = tune.tuned(dg, roots[:4], "rmat", mode=0)  # cache hit
    assert again == bfs.bfs_graph_get_tunables(dg)
    best_b = bfs.bfs_autotune(dg, roots, 1)
    assert 1 <= best_b["batch_width"] <= 64
    lv = torch.empty((len(roots), g.n), dtype=torch.int32, device="cuda")
    pa = torch.empty((len(roots), g.n), dtype=torch.int32, device="cuda")
    bfs.bfs_run_batch(dg, roots, lv, pa)
    for i, r in enumerate(roots):
        ref, _, _ = oracle.bfs(g.offsets, g.cols, int(r))
        assert oracle.validate(g.offsets, g.cols, int(r), ref, lv[i].cpu().numpy(), pa[i].cpu().numpy())[0] == 0
