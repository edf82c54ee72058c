"""Graph mode of the host-memory build (pbc_jk_set_graph): the first build
captures the device work into a HIP graph, later builds replay it.  Every
replay, with other eager GPU work and synchronisations between the replays
and densities of different rank (so the device decides the exchange form
afresh), must give the eager build's J, K and energies; the request server
replays graphs for repeated builds of a resident cell."""
import numpy as np
import pytest

from paper_2410_22278_amd import inputs

pytestmark = pytest.mark.gpu

CELL = dict(seed=41, natom=36, a_ang=7.0, recipe=((0, 0), (1, 0)), delta=1e-10, g_cut=2.0, r_cut=8.0)
CELL_D = dict(seed=21, natom=2, recipe=((0, 0), (1, 0), (2, 1)), a_ang=3.2, lo=0.3, hi=4.0)


@pytest.fixture(scope="module")
def lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2410_22278_amd import pbcjk
    pbcjk.load()
    return pbcjk


def _densities(s, rng):
    n = s.nbf
    C1 = rng.standard_normal((n, n // 3)) / np.sqrt(n)
    C2 = rng.standard_normal((n, n // 5)) / np.sqrt(n)
    X = rng.standard_normal((n, n)) / n
    return [s.D, C1 @ C1.T, C2 @ C2.T, X + X.T, s.D]   # low rank, other ranks, indefinite (dense form)


def _close(tag, a, b, natom):
    dJ = np.abs(a[0] - b[0]).max()
    dK = np.abs(a[1] - b[1]).max()
    dE = max(abs(a[2] - b[2]), abs(a[3] - b[3])) / natom
    print(f"{tag}: max|dJ|={dJ:.2e} max|dK|={dK:.2e} max dE/atom={dE:.2e}", flush=True)
    assert dJ < 1e-10 and dK < 1e-10 and dE < 1e-10, tag


@pytest.mark.parametrize("case", [CELL, CELL_D], ids=["sp144", "spd"])
def test_graph_replays_match_eager(lib, case):
    import torch
    s = inputs.small_cell(**case)
    Ds = _densities(s, np.random.default_rng(3))
    with lib.Handle(s) as eager:
        ref = [eager.build(D) for D in Ds]
    other = inputs.small_cell(seed=5, natom=3, recipe=((0, 0), (0, 0), (1, 0)), skew=0.15, omega=0.35)
    with lib.Handle(s) as h, lib.Handle(other) as h2:
        h.build(Ds[0])                       # eager first build
        h.set_graph(True)
        for rep in range(2):
            for k, D in enumerate(Ds):
                got = h.build(D)
                _close(f"graph replay {rep}.{k}", got, ref[k], s.natom)
                # eager work of the program between replays
                h2.build(other.D)
                torch.cuda.synchronize()
        h.set_graph(False)
        _close("eager again", h.build(Ds[1]), ref[1], s.natom)


def test_server_graphs_for_resident_cells(lib):
    s = inputs.serving_request(3)
    rng = np.random.default_rng(9)
    n = s.nbf
    Ds = [s.D]
    for _ in range(3):
        C = rng.standard_normal((n, max(1, n // 4))) / np.sqrt(n)
        Ds.append(C @ C.T)
    with lib.Handle(s) as h:
        ref = [h.build(D) for D in Ds]
    with lib.Server(slots=1, cache_cells=True, use_graphs=True) as srv:
        res = [srv.wait(srv.submit(s, D=D)) for D in Ds + Ds]
        st = srv.stats()
    for k, r in enumerate(res):
        assert r["status"] == 0, r["error"]
        _close(f"server build {k} (cache hit {r['cache_hit']})", (r["J"], r["K"], r["E_J"], r["E_K"]),
               ref[k % len(Ds)], s.natom)
    assert st["cache_hits"] == len(res) - 1
