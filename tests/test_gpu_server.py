"""GPU tests of the continuous-batching server (bfs_server_* through the C ABI):
every response equals the oracle (levels exact, parents valid), the same request
gives the same levels alone and mixed with others, admission respects the memory
budget, and the error paths report the documented codes."""
import threading
import time

import numpy as np
import pytest

import graphgen
import oracle
import paper_1604_02844_amd as bfs
from tests.gpu_helpers import load, torch_mod

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def graphs():
    torch_mod()
    gs = [graphgen.rmat(12, 16, seed=41), graphgen.er(1 << 13, 8, seed=42),
          graphgen.disjoint(graphgen.path(300), graphgen.star(50)), graphgen.rmat(14, 16, seed=43)]
    return gs


def wait(srv, ticket, n, timeout=60.0):
    lv = np.empty(n, dtype=np.int32)
    pa = np.empty(n, dtype=np.int32)
    t0 = time.time()
    while True:
        st = bfs.bfs_server_poll(srv, ticket, lv, pa)
        if st is not None:
            return lv, pa, st
        if time.time() - t0 > timeout:
            raise TimeoutError(f"ticket {ticket} not done after {timeout}s")
        time.sleep(0.0005)


def check(g, root, lv, pa, st=None):
    ref, _, ost = oracle.bfs(g.offsets, g.cols, int(root))
    code, bad = oracle.validate(g.offsets, g.cols, int(root), ref, lv, pa)
    assert code == 0, f"{g.name} root {root}: {oracle.CHECK_NAMES[code]} at {bad}"
    if st is not None:
        assert st["reached"] == ost["reached"] and st["arcs_scanned"] == ost["arcs"], (st, ost)
        assert st["num_levels"] == ost["levels"], (st, ost)
        assert st["latency_ms"] >= st["queue_ms"] >= 0


WORKERS_OFF = ("single-root workers are refused (bfs_server_create returns BFS_E_INVALID_ARG for "
               "single_workers > 0): a serving run with them (8 resident graphs, Poisson arrivals) ended "
               "in a GPU memory fault whose cause is not found yet")
ROUTES = {
    "batched": {},                                        # every request in a multi-source instance
    "adaptive": pytest.param(dict(single_workers=2), marks=pytest.mark.skip(reason=WORKERS_OFF)),
    "single": pytest.param(dict(single_workers=4, batch_min_queue=1 << 20),
                           marks=pytest.mark.skip(reason=WORKERS_OFF)),
}


@pytest.mark.parametrize("cfg", [ROUTES[k] for k in sorted(ROUTES)], ids=sorted(ROUTES))
def test_server_many_requests_mixed_graphs(graphs, cfg):
    route = "single" if cfg.get("batch_min_queue") else ("batched" if not cfg else "adaptive")
    srv = bfs.bfs_server_create(**cfg)
    dgs = [load(g) for g in graphs]
    gids = [bfs.bfs_server_add_graph(srv, d) for d in dgs]
    rng = np.random.default_rng(5)
    reqs = []
    for _ in range(300):
        k = int(rng.integers(0, len(graphs)))
        root = int(rng.integers(0, graphs[k].n))
        reqs.append((k, root, bfs.bfs_server_submit(srv, gids[k], root)))
    print(f"[case] server ({route}): 300 requests over {len(graphs)} graphs", flush=True)
    paths = []
    for k, root, t in reqs:
        lv, pa, st = wait(srv, t, graphs[k].n)
        check(graphs[k], root, lv, pa, st)
        assert st["graph_id"] == gids[k]
        paths.append(st["batched"])
    bfs.bfs_server_destroy(srv)
    if route == "batched":
        assert all(b == 1 for b in paths)
    if route == "single":
        assert any(b == 0 for b in paths)


@pytest.mark.parametrize("cfg", [ROUTES[k] for k in sorted(ROUTES)], ids=sorted(ROUTES))
def test_alone_versus_in_the_mix(graphs, cfg):
    """The same request, alone and among others, has identical levels and valid
    parents, whichever path (single-root run or multi-source instance) serves it."""
    g = graphs[3]
    srv = bfs.bfs_server_create(**cfg)
    gid = bfs.bfs_server_add_graph(srv, load(g))
    other = [bfs.bfs_server_add_graph(srv, load(h)) for h in graphs[:3]]
    probe_roots = graphgen.pick_roots(g, 5, seed=44)
    alone = {}
    for r in probe_roots:
        lv, pa, st = wait(srv, bfs.bfs_server_submit(srv, gid, int(r)), g.n)
        check(g, r, lv, pa, st)
        alone[int(r)] = lv
    rng = np.random.default_rng(6)
    mixed = []
    for i in range(200):
        if i % 40 == 7:
            r = int(probe_roots[(i // 40) % len(probe_roots)])
            mixed.append(("probe", r, bfs.bfs_server_submit(srv, gid, r)))
        k = int(rng.integers(0, 3))
        root = int(rng.integers(0, graphs[k].n))
        mixed.append((k, root, bfs.bfs_server_submit(srv, other[k], root)))
        root = int(rng.integers(0, g.n))
        mixed.append(("g", root, bfs.bfs_server_submit(srv, gid, root)))
    for kind, root, t in mixed:
        if kind == "probe":
            lv, pa, st = wait(srv, t, g.n)
            check(g, root, lv, pa, st)
            assert np.array_equal(lv, alone[root]), "levels differ alone vs in the mix"
        elif kind == "g":
            lv, pa, st = wait(srv, t, g.n)
            check(g, root, lv, pa, st)
        else:
            h = graphs[kind]
            lv, pa, st = wait(srv, t, h.n)
            check(h, root, lv, pa, st)
    bfs.bfs_server_destroy(srv)


def test_continuous_arrivals_from_another_thread(graphs):
    g = graphs[0]
    srv = bfs.bfs_server_create(max_slots=16)
    gid = bfs.bfs_server_add_graph(srv, load(g))
    roots = graphgen.pick_roots(g, 120, seed=45)
    tickets = [None] * len(roots)

    def producer():
        for i, r in enumerate(roots):
            tickets[i] = bfs.bfs_server_submit(srv, gid, int(r))
            if i % 10 == 0:
                time.sleep(0.001)

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    for r, t in zip(roots, tickets):
        lv, pa, st = wait(srv, t, g.n)
        check(g, r, lv, pa, st)
    bfs.bfs_server_destroy(srv)


def test_memory_budget_admission(graphs):
    """With room for one instance and two result rows, requests still all finish:
    each poll returns its rows to the pool and the next request is admitted."""
    g = graphs[0]
    inst = ((g.n + 63) // 64 * 64) * 8 * 3 + 200_000
    budget = inst + 2 * g.n * 8
    srv = bfs.bfs_server_create(mem_budget_bytes=budget)
    gid = bfs.bfs_server_add_graph(srv, load(g))
    roots = graphgen.pick_roots(g, 12, seed=46)
    tickets = [bfs.bfs_server_submit(srv, gid, int(r)) for r in roots]
    for r, t in zip(roots, tickets):
        lv, pa, st = wait(srv, t, g.n)
        check(g, r, lv, pa, st)
    bfs.bfs_server_destroy(srv)


def test_device_output_and_many_instances(graphs):
    torch = torch_mod()
    g = graphs[1]
    srv = bfs.bfs_server_create(max_slots=8, max_instances_per_graph=3)
    gid = bfs.bfs_server_add_graph(srv, load(g))
    roots = graphgen.pick_roots(g, 60, seed=47)
    tickets = [bfs.bfs_server_submit(srv, gid, int(r)) for r in roots]
    lv = torch.empty(g.n, dtype=torch.int32, device="cuda")
    pa = torch.empty(g.n, dtype=torch.int32, device="cuda")
    for r, t in zip(roots, tickets):
        while bfs.bfs_server_poll(srv, t, lv, pa) is None:
            time.sleep(0.0005)
        check(g, r, lv.cpu().numpy(), pa.cpu().numpy())
    bfs.bfs_server_destroy(srv)


def test_server_errors(graphs):
    g = graphs[2]
    dg = load(g)
    srv = bfs.bfs_server_create()
    gid = bfs.bfs_server_add_graph(srv, dg)
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_server_submit(srv, gid + 5, 0)
    assert e.value.status == bfs.BFS_E_INVALID_ARG
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_server_submit(srv, gid, g.n)
    assert e.value.status == bfs.BFS_E_ROOT_RANGE
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_server_poll(srv, 987654321)
    assert e.value.status == bfs.BFS_E_UNKNOWN_TICKET
    t = bfs.bfs_server_submit(srv, gid, 0)
    wait(srv, t, g.n)
    with pytest.raises(bfs.BfsError) as e:  # a ticket is consumed by its first completed poll
        bfs.bfs_server_poll(srv, t)
    assert e.value.status == bfs.BFS_E_UNKNOWN_TICKET
    with pytest.raises(bfs.BfsError) as e:  # a registered graph cannot be freed
        bfs.bfs_graph_free(dg)
    assert e.value.status == bfs.BFS_E_BUSY
    for r in range(20):  # destroy with work still queued or running
        bfs.bfs_server_submit(srv, gid, r)
    bfs.bfs_server_destroy(srv)
    bfs.bfs_graph_free(dg)
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_server_create(max_slots=65)
    assert e.value.status == bfs.BFS_E_INVALID_ARG


def test_tunables_locked_while_served(graphs):
    """A graph held by a server keeps its tunables: replacing them (directly or
    through the autotuner) would rebuild tables and free workspaces that the
    server's instances use, so both calls report BFS_E_BUSY until the server is
    gone; the requests served meanwhile stay correct."""
    g = graphs[0]
    dg = load(g)
    before = bfs.bfs_graph_get_tunables(dg)
    srv = bfs.bfs_server_create()
    gid = bfs.bfs_server_add_graph(srv, dg)
    t = bfs.bfs_server_submit(srv, gid, 1)
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_graph_set_tunables(dg, wave_max_degree=1024)
    assert e.value.status == bfs.BFS_E_BUSY
    with pytest.raises(bfs.BfsError) as e:
        bfs.bfs_autotune(dg, [1, 2], mode=0)
    assert e.value.status == bfs.BFS_E_BUSY
    assert bfs.bfs_graph_get_tunables(dg) == before
    lv, pa, st = wait(srv, t, g.n)
    check(g, 1, lv, pa, st)
    bfs.bfs_server_destroy(srv)
    after = bfs.bfs_graph_set_tunables(dg, wave_max_degree=1024)
    assert after["wave_max_degree"] == 1024
    bfs.bfs_graph_free(dg)


@pytest.mark.slow
def test_serving_configured_graph_set():
    """The serving configuration's eight resident graphs (R-MAT scales 16, 18,
    20, 22, 24 at edgefactor 16; Erdos-Renyi 2^18 d8, 2^20 d16, 2^22 d32), six
    requests per graph submitted interleaved so that instances of every graph
    run at once. Every response is checked: against the oracle's levels up to
    2^22 vertices, by the V2-V5 certificate (exact at any size) above."""
    from concurrent.futures import ThreadPoolExecutor

    torch_mod()
    specs = [("rmat", dict(scale=16, edgefactor=16)), ("rmat", dict(scale=18, edgefactor=16)),
             ("rmat", dict(scale=20, edgefactor=16)), ("rmat", dict(scale=22, edgefactor=16)),
             ("rmat", dict(scale=24, edgefactor=16)), ("er", dict(n=1 << 18, avg_degree=8)),
             ("er", dict(n=1 << 20, avg_degree=16)), ("er", dict(n=1 << 22, avg_degree=32))]
    gs = []
    for kind, kw in specs:
        print(f"[case] generating {kind} {kw}", flush=True)
        gs.append(graphgen.cached(kind, seed=1, **kw))
    srv = bfs.bfs_server_create()
    dgs = [load(g) for g in gs]
    gids = [bfs.bfs_server_add_graph(srv, d) for d in dgs]
    reqs = []
    for k in range(6):
        for i, g in enumerate(gs):
            root = int(graphgen.pick_roots(g, 6, seed=70 + i)[k])
            reqs.append((i, root, bfs.bfs_server_submit(srv, gids[i], root)))
    print(f"[case] serving {len(reqs)} requests over the 8 configured graphs", flush=True)

    def judge(g, root, lv, pa, st):
        if g.n <= (1 << 22) and g.nnz < 200_000_000:
            check(g, root, lv, pa, st)
        else:
            code, bad = oracle.certify(g.offsets, g.cols, root, lv, pa)
            assert code == 0, f"{g.name} root {root}: {oracle.CHECK_NAMES[code]} at {bad}"
            assert st["reached"] == int((lv >= 0).sum())

    futs = []
    with ThreadPoolExecutor(max_workers=8) as ex:
        for i, root, t in reqs:
            lv, pa, st = wait(srv, t, gs[i].n, timeout=300.0)
            assert st["graph_id"] == gids[i]
            futs.append(ex.submit(judge, gs[i], root, lv, pa, st))
        for f in futs:
            f.result()
    bfs.bfs_server_destroy(srv)
