"""Served mode through the C ABI: sessions in one HBM arena, lanes with their
own streams, HIP graph replay.

The gate is bitwise identity with a plain apply on the same geometry (the
same kernels in the same order), for every apply of every session, alone or in
the mix, with and without graph replay; plain applies run between the replays.
Admission, budget, timeout and failure paths are forced from the host.
"""
import threading
import time

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch

    import paper_2506_20809_amd as sbie

    assert torch.cuda.is_available()
    c = sbie.Context(0)
    yield c
    c.close()


def _mix():
    """(geometry, p, op, precision) of a mixed request set: prolate/oblate
    suspensions of 5 to 30 particles, orders 4 to 12, S, D and Stokes, FP64 and
    mixed."""
    out = []
    specs = [(5, 8, 0, 0), (9, 4, 1, 0), (17, 12, 0, 1), (30, 8, 1, 1), (12, 6, 2, 0), (7, 12, 1, 0),
             (20, 8, 2, 1), (3, 16, 0, 0)]
    for k, (M, p, op, prec) in enumerate(specs):
        out.append((workloads.rsa_pack(M, 0.15, 0.05, 900 + k), p, op, prec))
    return out


def _densities(n, nrhs, N, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((nrhs, N)) if nrhs > 1 else rng.standard_normal(N) for _ in range(n)]


def _plain(ctx, geom, p, op, prec, dens):
    import torch

    import paper_2506_20809_amd as sbie

    g = sbie.Geometry(ctx, geom, p)
    out = []
    for d in dens:
        u = g.apply(op, torch.tensor(d, device="cuda"), precision=prec)
        g.sync()
        out.append(u.cpu().numpy())
    g.close()
    return out


@pytest.mark.parametrize("graphs", [True, False])
def test_served_mix_bitwise_equals_plain(ctx, graphs):
    import torch

    import paper_2506_20809_amd as sbie

    mix = _mix()
    napply = 3
    srv = sbie.Server(ctx, max_sessions=4, budget_bytes=512 << 20, graphs=graphs)
    results = [None] * len(mix)
    errors = []
    inputs = []
    for k, (geom, p, op, prec) in enumerate(mix):
        N = len(geom["A"]) * (p + 1) * (2 * p + 2)
        inputs.append(_densities(napply, 3 if op == 2 else 1, N, 40 + k))

    def client(k):
        try:
            geom, p, op, prec = mix[k]
            s = srv.open(geom, p, op, prec)
            outs = []
            for d in inputs[k]:
                dd = torch.tensor(d, device="cuda")
                u, st = s.apply(dd)
                assert st.status == 0 and st.end_us >= st.start_us >= st.submit_us >= st.open_us
                outs.append(u.cpu().numpy())
            s.close()
            results[k] = outs
        except Exception as e:  # reported below
            errors.append((k, repr(e)))

    threads = [threading.Thread(target=client, args=(k,)) for k in range(len(mix))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=300)
    assert not errors, errors
    info = srv.info()
    assert info.applies == napply * len(mix) and info.admitted == len(mix)
    assert info.graphs == (1 if graphs else 0)
    srv.close()
    for k, (geom, p, op, prec) in enumerate(mix):
        ref = _plain(ctx, geom, p, op, prec, inputs[k])
        for r in range(napply):
            assert np.array_equal(results[k][r], ref[r]), (k, r, np.max(np.abs(results[k][r] - ref[r])))


def test_served_graph_replays_between_plain_applies(ctx):
    """Replays of one session's graph, with plain applies on another geometry and
    synchronisations between them, each equal to the plain result."""
    import torch

    import paper_2506_20809_amd as sbie

    geom = workloads.rsa_pack(11, 0.15, 0.05, 77)
    other = workloads.rsa_pack(6, 0.15, 0.05, 78)
    p = 8
    N = 11 * (p + 1) * (2 * p + 2)
    dens = _densities(5, 1, N, 5)
    ref = _plain(ctx, geom, p, 1, 0, dens)
    g2 = sbie.Geometry(ctx, other, p)
    d2 = torch.ones(g2.N, dtype=torch.float64, device="cuda")
    v0 = g2.apply(1, d2)
    g2.sync()
    srv = sbie.Server(ctx, max_sessions=1, budget_bytes=256 << 20, graphs=True)
    s = srv.open(geom, p, 1, 0)
    for r, d in enumerate(dens):
        u, _ = s.apply(torch.tensor(d, device="cuda"))
        assert np.array_equal(u.cpu().numpy(), ref[r]), r
        v = g2.apply(1, d2)  # eager work on the device between replays
        g2.sync()
        assert torch.equal(v, v0)
    s.close()
    srv.close()
    g2.close()


def test_served_host_pointers(ctx):
    import paper_2506_20809_amd as sbie

    geom = workloads.rsa_pack(6, 0.15, 0.05, 79)
    p = 8
    N = 6 * (p + 1) * (2 * p + 2)
    dens = _densities(2, 3, N, 6)
    ref = _plain(ctx, geom, p, 2, 0, dens)
    srv = sbie.Server(ctx, max_sessions=2, budget_bytes=128 << 20)
    s = srv.open(geom, p, 2, 0)
    for r, d in enumerate(dens):
        u, _ = s.apply(np.ascontiguousarray(d))
        assert np.array_equal(u, ref[r])
    s.close()
    srv.close()


def test_served_budget_forces_admission_waits(ctx):
    """An arena that holds one session at a time: every session still runs,
    the arena's peak stays within the budget and later sessions wait."""
    import torch

    import paper_2506_20809_amd as sbie

    p = 8
    geoms = [workloads.rsa_pack(12, 0.15, 0.05, 120 + k) for k in range(5)]
    need = max(sbie.session_bytes(12, p, 0) for _ in geoms)
    budget = need + need // 2
    srv = sbie.Server(ctx, max_sessions=4, budget_bytes=budget)
    sessions = [srv.open(g, p, 0) for g in geoms]
    N = 12 * (p + 1) * (2 * p + 2)
    dens = _densities(1, 1, N, 9)[0]
    tickets, outs = [], []
    for s in sessions:
        o = torch.empty(N, dtype=torch.float64, device="cuda")
        d = torch.tensor(dens, device="cuda")
        tickets.append(s.submit(d, o))
        outs.append((d, o))
        s.close()
    stats = [srv.wait(t) for t in tickets]
    # the last session returns its bytes once its lane has torn it down
    for _ in range(200):
        info = srv.info()
        if info.in_use_bytes == 0:
            break
        time.sleep(0.01)
    assert info.peak_bytes <= info.budget_bytes
    assert info.waited >= 1 and info.admitted == 5 and info.in_use_bytes == 0 and info.active == 0
    # one at a time: the admissions do not overlap
    spans = sorted((st.admit_us, st.end_us) for st in stats)
    for a, b in zip(spans, spans[1:]):
        assert b[0] >= a[1]
    srv.close()
    for g, (d, o) in zip(geoms, outs):
        ref = _plain(ctx, g, p, 0, 0, [dens])[0]
        assert np.array_equal(o.cpu().numpy(), ref)


def test_served_smaller_session_passes_waiting_one(ctx):
    """A holds the arena; B (as large) waits; C (small) passes B; after A
    closes, B runs."""
    import torch

    import paper_2506_20809_amd as sbie

    p = 8
    big = [workloads.rsa_pack(24, 0.15, 0.05, 130 + k) for k in range(2)]
    small = workloads.rsa_pack(3, 0.15, 0.05, 132)
    nb, ns = sbie.session_bytes(24, p, 0), sbie.session_bytes(3, 4, 0)
    assert ns <= nb // 2
    srv = sbie.Server(ctx, max_sessions=3, budget_bytes=nb + nb // 2)
    A = srv.open(big[0], p, 0)
    dA = torch.zeros(A.N, dtype=torch.float64, device="cuda")
    A.apply(dA)  # A is admitted and stays open
    B = srv.open(big[1], p, 0)
    C = srv.open(small, 4, 0)
    dC = torch.ones(C.N, dtype=torch.float64, device="cuda")
    _, stC = C.apply(dC)
    dB = torch.ones(B.N, dtype=torch.float64, device="cuda")
    oB = torch.empty_like(dB)
    tB = B.submit(dB, oB)
    with pytest.raises(sbie.SbieError) as e:
        srv.wait(tB, timeout_us=20000)
    assert e.value.status == -7
    info = srv.info()
    assert info.passed >= 1 and info.pending == 1
    A.close()
    stB = srv.wait(tB)
    assert stB.admit_us > stC.admit_us
    C.close()
    B.close()
    srv.close()


def test_served_errors(ctx):
    import torch

    import paper_2506_20809_amd as sbie

    srv = sbie.Server(ctx, max_sessions=2, budget_bytes=8 << 20)
    with pytest.raises(sbie.SbieError) as e:
        srv.open(workloads.geometry("c2"), 16, 0)
    assert e.value.status == -5
    qz = [1.0, 0.0, 0.0, 0.0]
    over = {"centers": np.array([[0, 0, 0], [0.3, 0, 0]], float), "quats": np.array([qz, qz]),
            "A": np.array([0.5, 0.5]), "C": np.array([1.0, 1.0])}
    s = srv.open(over, 4, 0)
    d = torch.zeros(s.N, dtype=torch.float64, device="cuda")
    with pytest.raises(sbie.SbieError) as e:
        s.apply(d)
    assert e.value.status == -3
    s.close()
    ok = srv.open(workloads.geometry("c1"), 8, 1)
    u, st = ok.apply(torch.ones(ok.N, dtype=torch.float64, device="cuda"))
    assert st.status == 0 and torch.max(torch.abs(u + 0.5)).item() < 1e-9
    ok.close()
    with pytest.raises(sbie.SbieError) as e:
        srv.wait(123456789)
    assert e.value.status == -1
    srv.close()


def test_served_many_concurrent_clients(ctx):
    """Forty small sessions from sixteen client threads at once (the ticket table
    grows while clients wait on it); every result equals its plain apply."""
    import torch

    import paper_2506_20809_amd as sbie

    p = 4
    geoms = [workloads.rsa_pack(2 + k % 3, 0.15, 0.05, 200 + k) for k in range(40)]
    dens = [_densities(5, 1, len(g["A"]) * (p + 1) * (2 * p + 2), 300 + k) for k, g in enumerate(geoms)]
    results = [None] * len(geoms)
    errors = []
    srv = sbie.Server(ctx, max_sessions=8, budget_bytes=256 << 20, graphs=True)

    def client(ks):
        try:
            for k in ks:
                s = srv.open(geoms[k], p, k % 2)
                outs = []
                for d in dens[k]:
                    u, _ = s.apply(torch.tensor(d, device="cuda"))
                    outs.append(u.cpu().numpy())
                s.close()
                results[k] = outs
        except Exception as e:  # reported below
            errors.append(repr(e))

    threads = [threading.Thread(target=client, args=(list(range(t, 40, 16)),)) for t in range(16)]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=100)
    # the server is destroyed only once no client can still call into it
    assert not any(t.is_alive() for t in threads), "a client thread did not finish"
    assert not errors, errors
    srv.close()
    for k, g in enumerate(geoms):
        ref = _plain(ctx, g, p, k % 2, 0, dens[k])
        for r in range(5):
            assert np.array_equal(results[k][r], ref[r]), (k, r)


@pytest.mark.parametrize("op,prec", [(0, 0), (1, 1)])
def test_served_batched_bitwise_equals_plain(ctx, op, prec):
    """Batching lanes: four sessions of one kind (operator, precision, order 8)
    share a lane and run their applies in batched launches, a Stokes session
    (which never batches) takes the other lane; every result equals its plain
    apply bitwise."""
    import paper_2506_20809_amd as sbie

    p, napply = 8, 4
    kinds = [(5, op), (12, 2), (9, op), (17, op), (30, op)]
    geoms = [workloads.rsa_pack(M, 0.15, 0.05, 500 + k) for k, (M, _) in enumerate(kinds)]
    precs = [prec if o != 2 else 0 for _, o in kinds]
    nrhs = [3 if o == 2 else 1 for _, o in kinds]
    dens = [_densities(napply, nrhs[k], len(g["A"]) * (p + 1) * (2 * p + 2), 700 + k) for k, g in enumerate(geoms)]
    srv = sbie.Server(ctx, max_sessions=2, budget_bytes=1 << 30, graphs=True, batch=True)
    sess = [srv.open(g, p, o, pr) for g, (_, o), pr in zip(geoms, kinds, precs)]
    results = [[None] * napply for _ in sess]
    for r in range(napply):
        outs = [np.zeros_like(dens[k][r]) for k in range(len(sess))]
        tickets = [s.submit(np.ascontiguousarray(dens[k][r]), outs[k]) for k, s in enumerate(sess)]
        for t in tickets:
            assert srv.wait(t).status == 0
        for k in range(len(sess)):
            results[k][r] = outs[k]
    for s in sess:
        s.close()
    info = srv.info()
    srv.close()
    assert info.applies == napply * len(sess) and info.admitted == len(sess)
    assert info.batched > 0, "no apply ran in a batch"
    for k, (g, (_, o)) in enumerate(zip(geoms, kinds)):
        ref = _plain(ctx, g, p, o, precs[k], dens[k])
        for r in range(napply):
            assert np.array_equal(results[k][r], ref[r]), (k, r, np.max(np.abs(results[k][r] - ref[r])))


def test_served_tree_sessions_equal_plain_tree_applies(ctx):
    """SBIE_SERVER_TREE: S and D sessions of at least 64 particles build the
    tree far field (theta 0.6, order 10, leaf 2) in the arena and their applies
    equal a plain geometry's applies through the same tree, bitwise; a smaller
    session keeps the direct far field.  With an arena too small for the tree
    a large session keeps the direct far field too."""
    import paper_2506_20809_amd as sbie

    p = 8
    specs = [(80, 0, 0), (70, 1, 1), (20, 0, 0)]
    geoms = [workloads.rsa_pack(M, 0.15, 0.05, 610 + k) for k, (M, _, _) in enumerate(specs)]
    dens = [_densities(2, 1, len(g["A"]) * (p + 1) * (2 * p + 2), 620 + k) for k, g in enumerate(geoms)]

    def plain(geom, op, prec, ds, tree):
        g = sbie.Geometry(ctx, geom, p)
        if tree:
            g.far_tree(0.6, 10, 2)
        out = [g.apply(op, d, precision=prec, tree=tree) for d in ds]
        g.close()
        return out

    srv = sbie.Server(ctx, max_sessions=3, budget_bytes=1 << 30, graphs=True, tree=True)
    sess = [srv.open(g, p, op, prec) for g, (_, op, prec) in zip(geoms, specs)]
    results = [[s.apply(d)[0] for d in dens[k]] for k, s in enumerate(sess)]
    for s in sess:
        s.close()
    info = srv.info()
    srv.close()
    assert info.tree_sessions == 2 and info.applies == 6
    for k, (geom, (M, op, prec)) in enumerate(zip(geoms, specs)):
        ref = plain(geom, op, prec, dens[k], M >= 64)
        for r in range(2):
            assert np.array_equal(results[k][r], ref[r]), (k, r)
    # an arena with room for the session but not for its tree
    nb = sbie.session_bytes(80, p, 0)
    srv = sbie.Server(ctx, max_sessions=1, budget_bytes=nb + (1 << 20), graphs=True, tree=True)
    s = srv.open(geoms[0], p, 0, 0)
    out = s.apply(dens[0][0])[0]
    s.close()
    info = srv.info()
    srv.close()
    assert info.tree_sessions == 0
    assert np.array_equal(out, plain(geoms[0], 0, 0, dens[0][:1], False)[0])
