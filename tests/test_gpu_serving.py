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


def convdiff_closed(N, bh):
    """Eigenvalues of the h^2-scaled 2-D operator -u_xx - u_yy + beta u_x on
    an N x N grid, lambda_ij = 4 - 2 sqrt(1 - b^2) cos(i pi/(N+1)) - 2 cos(j pi/(N+1))
    with b = beta h / 2, and the condition number of each: the x factor is
    D S D^-1 with S symmetric and D = diag(rho^k), rho = sqrt((1+b)/(1-b)),
    so its eigenvectors are D q_i (right) and D^-1 q_i (left) with q_i the
    sine vectors, kappa_i = ||D q_i|| ||D^-1 q_i|| / ||q_i||^2; the y factor
    is symmetric."""
    b = 0.5 * bh
    k = np.arange(1, N + 1)
    th = k * np.pi / (N + 1)
    rho = np.sqrt((1 + b) / (1 - b))
    D = rho ** k
    kap = np.empty(N)
    for i in range(1, N + 1):
        q = np.sin(i * th)
        kap[i - 1] = np.linalg.norm(D * q) * np.linalg.norm(q / D) / (q @ q)
    lam = 4 - 2 * np.sqrt(1 - b * b) * np.cos(th)[:, None] - 2 * np.cos(th)[None, :]
    kk = np.repeat(kap[:, None], N, axis=1)
    o = np.argsort(lam.ravel())
    return lam.ravel()[o], kk.ravel()[o]


# eigenvalues and condition numbers of each request's operator
CLOSED = {}


def closed_for(i):
    if i not in CLOSED:
        if i == 0:
            lam = lap_closed(30, 31)
            CLOSED[i] = (lam, np.ones_like(lam), True)
        elif i == 3:
            lam = lap_closed(64, 64)
            CLOSED[i] = (lam, np.ones_like(lam), True)
        else:
            N, bh = {1: (40, 0.3), 2: (24, 0.7), 4: (50, 0.1)}[i]
            lam, kap = convdiff_closed(N, bh)
            CLOSED[i] = (lam, kap, False)
    return CLOSED[i]


def check_eigenvalues(i, res, anorm):
    """Each returned eigenvalue lies within its certified distance of a
    closed-form eigenvalue, and no simple eigenvalue is claimed twice.  A unit
    vector with residual r is within r^2 / gap of an eigenvalue of a
    symmetric matrix (gap: distance to the next distinct eigenvalue), and
    within kappa * r of a nonsymmetric one to first order (asserted with a
    factor 2), up to the rounding of y* A y and of the closed form, a few
    units of eps * ||A|| (1e-14 ||A|| allowed)."""
    lam, kap, sym = closed_for(i)
    claimed = {}
    for mu, r in zip(res.mu, res.resid):
        assert r <= 1e-8 * anorm
        t = int(np.argmin(np.abs(lam - mu.real)))
        if sym:
            distinct = np.unique(np.round(lam, 12))
            u = int(np.argmin(np.abs(distinct - lam[t])))
            gap = np.min(np.abs(np.delete(distinct, u) - distinct[u]))
            bound = r * r / gap + 1e-14 * anorm
            mult = int(np.sum(np.abs(lam - lam[t]) <= 1e-12))
        else:
            bound = 2.0 * kap[t] * r + 1e-14 * anorm
            mult = 1
        assert abs(mu - lam[t]) <= bound, (i, mu, lam[t], bound)
        key = round(float(lam[t]), 12)
        claimed[key] = claimed.get(key, 0) + 1
        assert claimed[key] <= mult, (i, key)


def make_req(csr, seed, d, m, k, nev):
    b, v0 = W.start_vectors(csr.n, seed)
    return dict(csr=csr, b=b, v0=v0, d=d, m=m, k=k, nev=nev)


def submit(lib, B, rq, max_cycles=40, precision="f64"):
    c = rq["csr"]
    return B.submit(dev(c.rowptr), dev(c.colind), dev(c.vals), rq["d"], rq["m"], rq["k"], rq["nev"],
                    dev(rq["b"]), dev(rq["v0"]), rtol=1e-8, max_cycles=max_cycles, precision=precision)


def run_alone(lib, rq, precision="f64"):
    B = lib.Batch(4)
    s = submit(lib, B, rq, precision=precision)
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
        # every eigenvalue within its certified distance of the closed form,
        # and of the oracle's: both runs converge to rtol, so the two lie
        # within the sum of their bounds of the same eigenvalue
        rq = REQS[i]
        anorm = O.infnorm(rq["csr"])
        assert a.converged, i
        check_eigenvalues(i, a, anorm)
        ores, _ = O.pp_eigs(rq["csr"], rq["b"], rq["v0"], m=rq["m"], k=rq["k"], nev=rq["nev"],
                            d=rq["d"], rtol=1e-8, max_cycles=40)
        assert ores.converged, i
        check_eigenvalues(i, ores, anorm)
        lam, kap, sym = closed_for(i)
        for mu, r in zip(a.mu, a.resid):
            t = int(np.argmin(np.abs(ores.mu - mu)))
            tl = int(np.argmin(np.abs(lam - mu.real)))
            tol = (2e-10 * abs(mu) if sym else 2.0 * kap[tl] * (r + ores.resid[t])) + 2e-14 * anorm
            assert abs(mu - ores.mu[t]) <= tol, (i, mu, ores.mu[t], tol)


def test_batch_mixed_precision_eigenvalues(lib):
    """Mixed precision in the batched engine (FP32 pi(A)v, FP64 elsewhere,
    the closing FP64 Rayleigh-Ritz pass): every request converges to rtol on
    A in FP64 after at least one FP32 cycle, every eigenvalue lies within its
    certified distance of the closed form, and within the sum of both runs'
    bounds of the FP64 oracle's."""
    for i, rq in enumerate(REQS):
        r = run_alone(lib, rq, "mixed")
        anorm = O.infnorm(rq["csr"])
        print(f"request {i}: cycles {r.cycles}, fp32 cycles {r.fp32_cycles}, mvps {r.mvps}, "
              f"fp32 passes {r.spmv_passes_f32}, max resid {r.max_resid / anorm:.2e}", flush=True)
        assert r.converged and r.nconv == rq["nev"], i
        assert r.fp32_cycles >= 1 and 0 < r.spmv_passes_f32 < r.spmv_passes, i
        check_eigenvalues(i, r, anorm)
        # a closing Rayleigh-Ritz pass that misses rtol hands over to FP64
        # cycles from v0: the FP64 request's cycles and bits follow
        rf = run_alone(lib, rq)
        if r.cycles > r.fp32_cycles:
            assert r.cycles == r.fp32_cycles + rf.cycles, i
            assert np.array_equal(r.mu, rf.mu) and np.array_equal(r.resid, rf.resid), i
        ores, _ = O.pp_eigs(rq["csr"], rq["b"], rq["v0"], m=rq["m"], k=rq["k"], nev=rq["nev"],
                            d=rq["d"], rtol=1e-8, max_cycles=40)
        lam, kap, sym = closed_for(i)
        for mu, res in zip(r.mu, r.resid):
            t = int(np.argmin(np.abs(ores.mu - mu)))
            tl = int(np.argmin(np.abs(lam - mu.real)))
            tol = (2e-10 * abs(mu) if sym else 2.0 * kap[tl] * (res + ores.resid[t])) + 2e-14 * anorm
            assert abs(mu - ores.mu[t]) <= tol, (i, mu, ores.mu[t], tol)


def test_batch_mixed_alone_equals_mix(lib):
    """Mixed and FP64 solves share one engine: each result is bitwise the one
    computed alone in its own precision."""
    prec = ["mixed", "f64", "mixed", "mixed", "f64"]
    alone = [run_alone(lib, rq, p) for rq, p in zip(REQS, prec)]
    B = lib.Batch(8)
    slots = {}
    for i in (0, 1):
        slots[submit(lib, B, REQS[i], precision=prec[i])] = i
    got = {}
    steps = 0
    while len(got) < len(REQS):
        fin, _ = B.step()
        steps += 1
        for s in fin:
            got[slots.pop(s)] = B.result(s)
        if steps == 3:
            for i in (2, 3, 4):
                slots[submit(lib, B, REQS[i], precision=prec[i])] = i
        assert steps < 2000
    for i, a in enumerate(alone):
        g = got[i]
        assert np.array_equal(a.mu, g.mu) and np.array_equal(a.resid, g.resid), i
        assert (a.cycles, a.fp32_cycles, a.mvps, a.dots, a.spmv_passes_f32) == \
            (g.cycles, g.fp32_cycles, g.mvps, g.dots, g.spmv_passes_f32), i


@pytest.mark.parametrize("cap", [1, 2, 3])
def test_batch_mixed_cycle_cap(lib, cap):
    """A mixed-precision request under a tight cycle cap ends cleanly at the
    cap: cycles <= cap, FP32 cycles <= cycles, every returned residual
    recomputable (finite), and the status says whether it converged."""
    rq = REQS[4]
    B = lib.Batch(2)
    s = submit(lib, B, rq, max_cycles=cap, precision="mixed")
    steps = 0
    while True:
        fin, _ = B.step()
        steps += 1
        assert steps < 500
        if s in fin:
            r = B.result(s)
            break
    assert 1 <= r.cycles <= cap and 1 <= r.fp32_cycles <= r.cycles
    anorm = O.infnorm(rq["csr"])
    fin = np.isfinite(r.resid)
    assert fin.any() and np.array_equal(fin, np.isfinite(r.mu))
    assert r.nconv == int(np.sum(r.resid[fin] <= 1e-8 * anorm))
    if r.converged:
        assert fin.all() and r.nconv == rq["nev"]


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_batch_largest_small_request(lib, precision):
    """A request at the engine's size limit (n = 16384, the 128 x 128
    Laplacian): converged, every eigenvalue within r^2 / gap of the closed
    form, multiplicities (2 for i != j) respected."""
    N = 128
    rq = make_req(W.laplacian_2d(N), 9, 20, 40, 15, 10)
    r = run_alone(lib, rq, precision)
    assert r.converged and r.nconv == 10
    if precision == "mixed":
        assert r.fp32_cycles >= 1
    lam = lap_closed(N, N)
    distinct = np.unique(np.round(lam, 13))
    claimed = {}
    anorm = O.infnorm(rq["csr"])
    for mu, res in zip(r.mu, r.resid):
        assert res <= 1e-8 * anorm and abs(mu.imag) <= 1e-14 * anorm
        u = int(np.argmin(np.abs(distinct - mu.real)))
        gap = np.min(np.abs(np.delete(distinct, u) - distinct[u]))
        assert abs(mu.real - distinct[u]) <= res * res / gap + 1e-14 * anorm
        claimed[u] = claimed.get(u, 0) + 1
        assert claimed[u] <= int(np.sum(np.abs(lam - distinct[u]) <= 1e-12))


def test_batch_mixed_workspace_and_precision_checks(lib):
    """The mixed workspace adds the FP32 values and four FP32 vectors; an
    unknown precision is refused."""
    from paper_1806_08020_amd import ppa
    c = REQS[1]["csr"]
    f64 = ppa.batch_workspace_bytes(c.n, 12, 30, 7)
    mixed = ppa.batch_workspace_bytes(c.n, 12, 30, 7, c.nnz, "mixed")
    assert mixed >= f64 + 4 * c.nnz + 16 * c.n
    B = lib.Batch(2)
    with pytest.raises(ValueError):
        submit(lib, B, REQS[1], precision="f32")
    # a workspace sized for FP64 is too small for a mixed request
    rq = REQS[1]
    ws = torch.empty(f64, dtype=torch.uint8, device="cuda")
    with pytest.raises(ppa.PPAError):
        B.submit(dev(c.rowptr), dev(c.colind), dev(c.vals), rq["d"], rq["m"], rq["k"], rq["nev"],
                 dev(rq["b"]), dev(rq["v0"]), ws=ws, precision="mixed")


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


def test_server_mixed_both_paths(lib):
    """Mixed-precision requests through the server: the small ones run in the
    batched engine with FP32 cycles and equal their alone runs bitwise, the
    large one runs on a worker stream and equals the single-solve path."""
    from paper_1806_08020_amd import serve as S
    reqs = [S.Request(i, rq["csr"], rq["d"], rq["m"], rq["k"], rq["nev"], rq["b"], rq["v0"],
                      1e-8, 40, arrival=0.0, precision="mixed") for i, rq in enumerate(REQS[:3])]
    big = W.convdiff_2d(200, 0.2)
    b, v0 = W.start_vectors(big.n, 77)
    reqs.append(S.Request(3, big, 20, 30, 12, 6, b, v0, 1e-8, 20, arrival=0.0, precision="mixed"))
    srv = S.Server(hbm_budget=8 << 30, max_slots=4, small_n=16384, stream_workers=1)
    try:
        done = srv.run(reqs)
    finally:
        srv.close()
    assert all(c.error is None for c in done)
    for c in done[:3]:
        assert c.path == "batch" and c.result.fp32_cycles >= 1
        a = run_alone(lib, REQS[c.rid], "mixed")
        assert np.array_equal(a.mu, c.result.mu) and np.array_equal(a.resid, c.result.resid)
    cbig = done[3]
    assert cbig.path == "stream" and cbig.result.fp32_cycles >= 1
    A = lib.Matrix(big, want_f32=True)
    r2 = lib.eigs(A, lib.Poly.build(A, 20, dev(b)), dev(v0), 30, 12, 6, rtol=1e-8, max_cycles=20,
                  precision="mixed")
    assert np.array_equal(r2.mu, cbig.result.mu)
    summ = S.summarize(done, 1.0)
    assert summ["by_path"]["batch"]["fp32_cycles"] >= 3


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
