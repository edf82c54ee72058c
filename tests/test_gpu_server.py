"""GPU tests of the request server (pbc_jk_server_*).

Cells of the serving stream (8-60 atoms of H/C/O, mixed precision) are built
alone, each on a fresh handle, and then all together through the server,
where up to four builds overlap on the device.  Each result must be the same
in the mix as alone: the two differ only by the order of floating-point
atomic additions, far below the stated tolerances (1e-7 per matrix element,
1e-6 Eh/atom), which are asserted at 1e-10.  Admission, eviction, cache
reuse, cancellation and per-request failure are checked on the same cells.
"""
import numpy as np
import pytest

from paper_2410_22278_amd import inputs

pytestmark = pytest.mark.gpu

REQ_IDS = list(range(13))          # 8-60 atoms, nbf 45-304


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2410_22278_amd import pbcjk
    pbcjk.load()
    return pbcjk


@pytest.fixture(scope="module")
def alone(lib):
    """Each request alone on its own handle."""
    out = {}
    for i in REQ_IDS:
        s = inputs.serving_request(i)
        with lib.Handle(s) as h:
            J, K, EJ, EK = h.build(s.D)
        out[i] = (s, J, K, EJ, EK)
        print(f"alone req{i}: natom={s.natom} nbf={s.nbf} E_J={EJ:.10f} E_K={EK:.10f}", flush=True)
    return out


def _same(tag, r, ref):
    s, J, K, EJ, EK = ref
    assert r["status"] == 0, f"{tag}: status {r['status']} {r['error']}"
    dJ = np.abs(r["J"] - J).max()
    dK = np.abs(r["K"] - K).max()
    dEJ = abs(r["E_J"] - EJ) / s.natom
    dEK = abs(r["E_K"] - EK) / s.natom
    print(f"{tag}: max|dJ|={dJ:.2e} max|dK|={dK:.2e} dE_J/atom={dEJ:.2e} dE_K/atom={dEK:.2e} "
          f"queue={r['queue_ms']:.1f} setup={r['setup_ms']:.1f} build={r['build_ms']:.1f} ms "
          f"hit={r['cache_hit']} retries={r['retries']}", flush=True)
    assert dJ < 1e-10 and dK < 1e-10 and dEJ < 1e-10 and dEK < 1e-10, tag


def test_alone_vs_mix(lib, alone):
    with lib.Server(slots=4, cache_cells=False) as srv:
        tickets = {i: srv.submit(alone[i][0]) for i in REQ_IDS}
        res = {i: srv.wait(t) for i, t in tickets.items()}
        st = srv.stats()
    print("server stats:", st, flush=True)
    for i in REQ_IDS:
        _same(f"mix req{i}", res[i], alone[i])
    assert st["completed"] == len(REQ_IDS) and st["failed"] == 0
    assert st["peak_running"] > 1          # builds did overlap
    assert st["in_use"] == 0               # every cell released


def test_admission_under_a_tight_budget(lib, alone):
    """Budget of 1.5x the largest single footprint: requests must queue for
    memory, and every result is still the same as alone."""
    with lib.Server(slots=4, cache_cells=False) as srv:
        r = srv.wait(srv.submit(alone[1][0]))       # the largest cell (nbf 304)
        big = r["device_bytes"]
    budget = int(1.5 * big)
    with lib.Server(hbm_budget=budget, slots=4, cache_cells=False) as srv:
        tickets = {i: srv.submit(alone[i][0]) for i in REQ_IDS}
        res = {i: srv.wait(t) for i, t in tickets.items()}
        st = srv.stats()
    print(f"budget {budget} B: stats {st}", flush=True)
    for i in REQ_IDS:
        _same(f"tight req{i}", res[i], alone[i])
    assert st["peak_in_use"] <= st["budget"]


def test_oversize_request_fails_alone(lib, alone):
    """A cell larger than the whole budget fails with ENOMEM; the others run."""
    small = [4, 5, 7]
    with lib.Server(slots=2, cache_cells=False) as srv:
        foot = max(srv.wait(srv.submit(alone[i][0]))["device_bytes"] for i in small)
    with lib.Server(hbm_budget=int(1.2 * foot), slots=2, cache_cells=False) as srv:
        t_big = srv.submit(alone[1][0])
        ts = {i: srv.submit(alone[i][0]) for i in small}
        rb = srv.wait(t_big)
        res = {i: srv.wait(t) for i, t in ts.items()}
    print(f"oversize: status {rb['status']} '{rb['error']}'", flush=True)
    assert rb["status"] == lib.PBC_JK_ENOMEM
    for i in small:
        _same(f"beside oversize req{i}", res[i], alone[i])


def test_cache_reuse_and_eviction(lib, alone):
    """Repeated builds of one cell reuse its resident setup; a budget that
    holds one cell at a time forces least-recently-used eviction."""
    a, b = alone[2], alone[3]
    with lib.Server(slots=1, cache_cells=True) as srv:
        r1 = srv.wait(srv.submit(a[0]))
        r2 = srv.wait(srv.submit(a[0]))
        fa = r1["device_bytes"]
        fb = srv.wait(srv.submit(b[0]))["device_bytes"]
    assert r1["cache_hit"] == 0 and r2["cache_hit"] == 1
    _same("cache first", r1, a)
    _same("cache second", r2, a)
    with lib.Server(hbm_budget=int(1.1 * max(fa, fb)), slots=1, cache_cells=True) as srv:
        seq = [a, b, a, b]
        out = [srv.wait(srv.submit(x[0])) for x in seq]
        st = srv.stats()
    for k, (x, r) in enumerate(zip(seq, out)):
        _same(f"evict step {k}", r, x)
    assert st["evictions"] >= 3 and st["cache_hits"] == 0


def test_cancel_and_bad_request_isolation(lib, alone):
    s_ok = alone[4][0]
    bad_D = s_ok.D.copy()
    bad_D[0, 0] = np.nan
    with lib.Server(slots=1, cache_cells=False) as srv:
        t1 = srv.submit(alone[0][0])              # occupies the only slot
        t2 = srv.submit(alone[5][0])
        rc = srv.cancel(t2)
        t3 = srv.submit(s_ok, D=bad_D)
        t4 = srv.submit(s_ok)
        r1, r2, r3, r4 = (srv.wait(t) for t in (t1, t2, t3, t4))
        st = srv.stats()
    print(f"cancel rc={rc} -> {r2['status']}; bad D -> {r3['status']} '{r3['error']}'", flush=True)
    _same("before cancel", r1, alone[0])
    if rc == 0:
        assert r2["status"] == lib.PBC_JK_ECANCELED
    else:
        assert rc == lib.PBC_JK_EBUSY
    assert r3["status"] == lib.PBC_JK_EINVAL
    _same("after bad request", r4, alone[4])
    assert st["failed"] == 1


@pytest.mark.parametrize("cache", [False, True], ids=["no_cache", "cache"])
def test_cancel_second_request_of_same_cell(lib, alone, cache):
    """Two requests for the same cell (the second with another density) on a
    one-slot server, the second cancelled while the first is queued or its
    cell is being created: the first keeps its cell and completes with the
    alone result, and a third request for the cell still runs."""
    s = alone[2][0]
    D2 = 0.5 * s.D
    with lib.Server(slots=1, cache_cells=cache) as srv:
        t1 = srv.submit(s)
        t2 = srv.submit(s, D=D2)
        rc = srv.cancel(t2)
        r1 = srv.wait(t1)
        r2 = srv.wait(t2)
        r3 = srv.wait(srv.submit(s))
        st = srv.stats()
    print(f"same-cell cancel (cache={cache}): rc={rc} -> {r2['status']}; stats {st}", flush=True)
    _same("same cell, first", r1, alone[2])
    _same("same cell, after the cancel", r3, alone[2])
    if rc == 0:
        assert r2["status"] == lib.PBC_JK_ECANCELED
    else:
        assert rc == lib.PBC_JK_EBUSY and r2["status"] == 0
    assert st["failed"] == 0
    if not cache:
        assert st["in_use"] == 0


@pytest.mark.parametrize("policy", ["arrival", "deadline"])
def test_queue_policy(lib, alone, policy):
    """One slot, a running build, then a large and a small request queued
    behind it: in arrival order the large one runs first; with the deadline
    order (submission time plus c nbf^2) the small one passes it.  Both
    results stay those of the builds alone."""
    blocker, big, small = 12, 1, 4
    with lib.Server(slots=1, cache_cells=False, policy=policy) as srv:
        tb = srv.submit(alone[blocker][0])
        tl = srv.submit(alone[big][0])
        ts = srv.submit(alone[small][0])
        rb, rl, rs = srv.wait(tb), srv.wait(tl), srv.wait(ts)
    for r in (rb, rl, rs):
        assert r["status"] == 0, r.get("error")
    print(f"policy {policy}: large queue {rl['queue_ms']:.1f} ms, small queue {rs['queue_ms']:.1f} ms", flush=True)
    if policy == "arrival":
        assert rs["queue_ms"] > rl["queue_ms"]
    else:
        assert rs["queue_ms"] < rl["queue_ms"]
    for i, r in ((big, rl), (small, rs)):
        _, J, K, _, _ = alone[i]
        assert np.abs(r["J"] - J).max() < 1e-10 and np.abs(r["K"] - K).max() < 1e-10
