"""Serving loop on the GPU: continuous batching must not change any result.

Each request's energies and iteration count in the mix are compared bit for bit with the
same request solved alone through pb_solve (with the tile layout the serving loop uses,
32-plane x-chunks); admission honours the memory budget; requests are not admitted before
their arrival time."""
import time
from dataclasses import replace

import numpy as np
import pytest

from oracle import oracle as O
from paper_2502_09323_amd import binding as B
from paper_2502_09323_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctxs():
    import torch

    B.load()
    main = B.Context(0)
    side = B.Context(0, stream=torch.cuda.Stream(0))
    yield main, side
    main.close()
    side.close()


def small_stream(n=10, seed=7):
    rng = np.random.default_rng(seed)
    reqs = []
    for k in range(n):
        na = int(rng.integers(20, 400))
        R = 3.0 + 4.0 * (na / 400) ** (1 / 3)
        h = float(rng.choice([0.4, 0.5, 0.6]))
        nn = int(2 * (R + 3.0) / h) + 5
        mol = I.random_molecule(na, R, 1000 + k)
        grid = I.cubic_grid(nn, h, precision=I.MIXED, rtol=1e-8, inner_rtol=1e-2)
        reqs.append((mol, grid))
    return reqs


def run_server(srv, reqs, arrivals=None, timeout_s=60.0):
    for i, (mol, grid) in enumerate(reqs):
        srv.submit(mol, grid, i, None if arrivals is None else arrivals[i])
    out = {}
    t0 = time.time()
    while len(out) < len(reqs):
        srv.step()
        for r in srv.poll():
            out[r["id"]] = r
        assert time.time() - t0 < timeout_s, "serving loop did not finish"
    return out


def test_mix_equals_alone_bitwise(ctxs):
    main, side = ctxs
    reqs = small_stream()
    srv = B.Server(main, side, max_resident=4)
    served = run_server(srv, reqs)
    srv.close()
    for i, (mol, grid) in enumerate(reqs):
        r = served[i]
        assert r["code"] == 0
        alone = B.solve(mol, replace(grid, tile_planes=32), main)
        for k in ("e_pol", "e_ion", "e_coul", "q_pol_total", "area_total"):
            assert r[k] == alone[k], (i, k, r[k], alone[k])
        assert r["iters"] == alone["iters"] and r["outer_iters"] == alone["outer_iters"]


def test_multigrid_requests_in_the_mix_equal_alone_bitwise(ctxs):
    """Requests with the multigrid preconditioner run their own launches between the batched
    chunks; each result equals the same request solved alone, bit for bit."""
    main, side = ctxs
    reqs = small_stream(n=8, seed=11)
    reqs = [(mol, replace(grid, precond=I.MG) if i % 2 == 0 else grid) for i, (mol, grid) in enumerate(reqs)]
    # one request on a grid with n - 1 even, so that its V-cycle has several levels
    mol = I.random_molecule(150, 5.0, 77)
    reqs.append((mol, I.cubic_grid(41, 0.5, precision=I.MIXED, rtol=1e-8, inner_rtol=1e-2, precond=I.MG)))
    srv = B.Server(main, side, max_resident=4)
    served = run_server(srv, reqs)
    srv.close()
    for i, (mol, grid) in enumerate(reqs):
        r = served[i]
        assert r["code"] == 0
        alone = B.solve(mol, replace(grid, tile_planes=32), main)
        for k in ("e_pol", "e_ion", "e_coul", "q_pol_total", "area_total"):
            assert r[k] == alone[k], (i, k, r[k], alone[k])
        assert r["iters"] == alone["iters"] and r["outer_iters"] == alone["outer_iters"]
    # the 41^3 request has four levels (41, 21, 11, 6); the others' n - 1 is mostly odd, where
    # the preconditioner is red-black symmetric Gauss-Seidel alone
    assert served[len(reqs) - 1]["iters"] < 30


def test_served_energies_match_fp64_oracle(ctxs):
    main, side = ctxs
    reqs = small_stream(n=4, seed=11)
    srv = B.Server(main, side, max_resident=8)
    served = run_server(srv, reqs)
    srv.close()
    for i, (mol, grid) in enumerate(reqs):
        ref = O.run(mol, grid, rtol=1e-12).energy
        for k in ("e_pol", "e_ion"):
            assert abs(served[i][k] - ref[k]) <= 1e-6 * abs(ref[k]), (i, k)


def test_budget_admission_and_rejection(ctxs):
    import torch

    main_tight = B.Context(0, hbm_budget_bytes=60 << 20)
    side = B.Context(0, stream=torch.cuda.Stream(0))
    reqs = small_stream(n=4, seed=3)
    big = (I.random_molecule(50, 4.0, 9), I.cubic_grid(161, 0.25, precision=I.MIXED, rtol=1e-6))
    srv = B.Server(main_tight, side, max_resident=8)
    served = run_server(srv, reqs + [big])
    srv.close()
    assert all(served[i]["code"] == 0 for i in range(4))
    assert served[4]["code"] == B.PB_ENOMEM
    main_tight.close()
    side.close()


def test_future_arrivals_wait(ctxs):
    main, side = ctxs
    reqs = small_stream(n=3, seed=5)
    srv = B.Server(main, side, max_resident=4)
    t = srv.now()
    arrivals = [t, t + 0.3, t + 0.6]
    served = run_server(srv, reqs, arrivals)
    srv.close()
    for i in range(3):
        assert served[i]["code"] == 0
        assert served[i]["done_s"] >= arrivals[i]


def test_long_stream_holds_the_budget_and_returns_it(ctxs):
    """A stream eight times longer than the resident limit under a budget of a few requests:
    the accounted memory never exceeds the budget, comes back to zero when the stream is done,
    and waiting for memory changes no result."""
    import torch

    budget = 48 << 20
    main_b = B.Context(0, hbm_budget_bytes=budget)
    side = B.Context(0, stream=torch.cuda.Stream(0))
    reqs = small_stream(n=24, seed=13)
    srv = B.Server(main_b, side, max_resident=3)
    served = run_server(srv, reqs, timeout_s=120.0)
    mem = srv.memory()
    srv.close()
    print("serving memory:", mem, flush=True)
    assert all(served[i]["code"] == 0 for i in range(len(reqs)))
    assert 0 < mem["peak"] <= budget
    assert mem["in_use"] == 0 and mem["over_budget"] == 0
    for i in (0, 11, 23):
        mol, grid = reqs[i]
        alone = B.solve(mol, replace(grid, tile_planes=32), ctxs[0])
        assert served[i]["e_pol"] == alone["e_pol"] and served[i]["e_ion"] == alone["e_ion"]
    main_b.close()
    side.close()


def test_cancel_and_time_limit(ctxs):
    main, side = ctxs
    reqs = small_stream(n=6, seed=17)
    srv = B.Server(main, side, max_resident=2)
    for i, (mol, grid) in enumerate(reqs):
        srv.submit(mol, grid, i)
    srv.step()                      # admits requests 0 and 1 (builds start)
    srv.cancel(0)                   # being built
    srv.cancel(5)                   # still queued
    for _ in range(3):
        srv.step()
    srv.cancel(1)                   # being built, resident or read back
    with pytest.raises(B.PbError) as e:
        srv.cancel(1)               # already cancelled
    assert e.value.code == B.PB_EINVAL
    with pytest.raises(B.PbError):
        srv.cancel(99)              # unknown
    out = {}
    t0 = time.time()
    while len(out) < len(reqs):
        srv.step()
        for r in srv.poll():
            out[r["id"]] = r
        assert time.time() - t0 < 60, "serving loop did not finish"
    mem = srv.memory()
    srv.close()
    assert [out[i]["code"] for i in range(6)] == [B.PB_ECANCELED, B.PB_ECANCELED, 0, 0, 0, B.PB_ECANCELED]
    assert mem["in_use"] == 0
    mol, grid = reqs[3]
    alone = B.solve(mol, replace(grid, tile_planes=32), main)
    assert out[3]["e_pol"] == alone["e_pol"] and out[3]["iters"] == alone["iters"]
    # a time limit: requests that arrived a second ago and requests already admitted expire
    srv = B.Server(main, side, max_resident=2)
    t = srv.now()
    for i, (mol, grid) in enumerate(reqs[:4]):
        srv.submit(mol, grid, i, t if i < 2 else t - 1.0)
    srv.set_timeout(30.0)
    srv.step()                      # admits requests 0 and 1
    srv.set_timeout(1e-6)
    out = {}
    t0 = time.time()
    while len(out) < 4:
        srv.step()
        for r in srv.poll():
            out[r["id"]] = r
        assert time.time() - t0 < 60, "serving loop did not finish"
    mem = srv.memory()
    srv.close()
    assert all(out[i]["code"] == B.PB_ETIMEDOUT for i in range(4))
    assert mem["in_use"] == 0
    with pytest.raises(B.PbError):
        srv2 = B.Server(main, side, max_resident=2)
        try:
            srv2.set_timeout(-1.0)
        finally:
            srv2.close()
