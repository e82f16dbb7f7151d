"""GPU tests of the served form: the batched small-solve engine and the
continuous-batching request loop.  Each result must be the same alone and in
the mix (bitwise: every reduction is confined to one workgroup or one stream
in a fixed order), match the FP64 oracle, and admission must respect the HBM
budget."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1806_08020_amd import workloads as W

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(np.asarray(x)).to("cuda")


def lap_closed(nx, ny):
    i = np.arange(1, nx + 1)[:, None]
    j = np.arange(1, ny + 1)[None, :]
    return np.sort((4 - 2 * np.cos(i * np.pi / (nx + 1)) - 2 * np.cos(j * np.pi / (ny + 1))).ravel())


def make_req(csr, seed, d, m, k, nev):
    b, v0 = W.start_vectors(csr.n, seed)
    return dict(csr=csr, b=b, v0=v0, d=d, m=m, k=k, nev=nev)


def submit(lib, B, rq, max_cycles=40):
    c = rq["csr"]
    return B.submit(dev(c.rowptr), dev(c.colind), dev(c.vals), rq["d"], rq["m"], rq["k"], rq["nev"],
                    dev(rq["b"]), dev(rq["v0"]), rtol=1e-8, max_cycles=max_cycles)


def run_alone(lib, rq):
    B = lib.Batch(4)
    s = submit(lib, B, rq)
    while True:
        fin, _ = B.step()
        if s in fin:
            return B.result(s)


REQS = [
    make_req(W.laplacian_2d(30, 31), 1, 8, 20, 10, 5),
    make_req(W.convdiff_2d(40, 0.3), 2, 12, 30, 12, 7),
    make_req(W.convdiff_2d(24, 0.7), 3, 20, 30, 10, 5),
    make_req(W.laplacian_2d(64), 4, 16, 40, 17, 12),
    make_req(W.convdiff_2d(50, 0.1), 5, 30, 30, 15, 10),
]


def test_batch_engine_matches_oracle_and_closed_form(lib):
    rq = REQS[0]
    r = run_alone(lib, rq)
    assert r.converged and r.nconv == 5
    lam = lap_closed(30, 31)
    assert np.allclose(r.mu.real, lam[:5], rtol=1e-10, atol=0)
    assert np.all(np.abs(r.mu.imag) < 1e-12)
    ores, _ = O.pp_eigs(rq["csr"], rq["b"], rq["v0"], m=20, k=10, nev=5, d=8, rtol=1e-8, max_cycles=40)
    assert np.allclose(r.mu.real, ores.mu.real, rtol=1e-10, atol=0)
    assert r.cycles == ores.cycles
    assert np.all(r.resid <= 1e-8 * O.infnorm(rq["csr"]))


def test_batch_alone_equals_mix(lib):
    """Staggered admission into one engine: every result is bitwise the one
    computed alone."""
    alone = [run_alone(lib, rq) for rq in REQS]
    B = lib.Batch(8)
    slots = {}
    for i in (0, 2):
        slots[submit(lib, B, REQS[i])] = i
    got = {}
    steps = 0
    while len(got) < len(REQS):
        fin, _ = B.step()
        steps += 1
        for s in fin:
            got[slots.pop(s)] = B.result(s)
        if steps == 2:
            slots[submit(lib, B, REQS[1])] = 1
        if steps == 4:
            slots[submit(lib, B, REQS[3])] = 3
            slots[submit(lib, B, REQS[4])] = 4
        assert steps < 2000
    for i, a in enumerate(alone):
        g = got[i]
        assert np.array_equal(a.mu, g.mu) and np.array_equal(a.resid, g.resid), i
        assert (a.cycles, a.mvps, a.dots, a.nconv) == (g.cycles, g.mvps, g.dots, g.nconv)
        # and each one agrees with the oracle's converged eigenvalues
        rq = REQS[i]
        ores, _ = O.pp_eigs(rq["csr"], rq["b"], rq["v0"], m=rq["m"], k=rq["k"], nev=rq["nev"],
                            d=rq["d"], rtol=1e-8, max_cycles=40)
        if ores.converged and a.converged:
            anorm = O.infnorm(rq["csr"])
            assert np.all(a.resid <= 1e-8 * anorm)


def test_batch_full_engine_reports_busy(lib):
    B = lib.Batch(1)
    assert submit(lib, B, REQS[0]) is not None
    assert submit(lib, B, REQS[1]) is None


def test_server_budget_and_identity(lib):
    """A tight HBM budget forces queueing; every request finishes, memory in
    use never exceeds the budget, and the results equal the alone runs of
    the same paths."""
    from paper_1806_08020_amd import serve as S
    reqs = []
    for i, rq in enumerate(REQS):
        reqs.append(S.Request(i, rq["csr"], rq["d"], rq["m"], rq["k"], rq["nev"], rq["b"], rq["v0"],
                              1e-8, 40, arrival=0.002 * i))
    big = W.convdiff_2d(200, 0.2)   # n = 40000 > small_n: stream path
    b, v0 = W.start_vectors(big.n, 77)
    reqs.append(S.Request(len(reqs), big, 20, 30, 12, 6, b, v0, 1e-8, 20, arrival=0.0))
    fps = [S.batch_footprint(r) if r.csr.n <= 16384 else S.stream_footprint(r) for r in reqs]
    budget = max(fps) + min(fps)
    srv = S.Server(hbm_budget=budget, max_slots=4, small_n=16384, stream_workers=2)
    try:
        done = srv.run(reqs)
    finally:
        srv.close()
    assert len(done) == len(reqs) and all(c.error is None for c in done)
    assert srv.stats["max_used_bytes"] <= budget
    alone = [run_alone(lib, rq) for rq in REQS]
    for c in done[: len(REQS)]:
        assert c.path == "batch"
        a = alone[c.rid]
        assert np.array_equal(a.mu, c.result.mu) and np.array_equal(a.resid, c.result.resid)
    cbig = done[-1]
    assert cbig.path == "stream"
    A = lib.Matrix(big)
    r2 = lib.eigs(A, lib.Poly.build(A, 20, dev(b)), dev(v0), 30, 12, 6, rtol=1e-8, max_cycles=20)
    assert np.array_equal(r2.mu, cbig.result.mu)


def test_server_rejects_request_above_budget(lib):
    from paper_1806_08020_amd import serve as S
    rq = REQS[0]
    r = S.Request(0, rq["csr"], rq["d"], rq["m"], rq["k"], rq["nev"], rq["b"], rq["v0"])
    srv = S.Server(hbm_budget=1000, max_slots=2, stream_workers=1)
    try:
        with pytest.raises(ValueError):
            srv.run([r])
    finally:
        srv.close()
