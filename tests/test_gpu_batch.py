"""Batched and served solves on the GPU: many systems of different sizes in
one launch per CG kernel. Each system's share of a launch depends only on the
system, so its result must be bit for bit its single-system result, alone or
in any mix; and each must match the FP64 oracle to the single-solve bar."""
import sys
import time

import numpy as np
import pytest

import oracle
from paper_2510_27517_amd import inputs
from paper_2510_27517_amd.inputs import CSR

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu]", *a, flush=True)
    sys.stdout.flush()


def _mix(seed, count, tol=1e-8):
    """Systems of mixed kinds and sizes (2D/3D lognormal Poisson, RGG)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(count):
        kind = k % 3
        if kind == 0:
            A = inputs.poisson(2, int(rng.integers(4, 60)), 0.5, seed * 100 + k)
        elif kind == 1:
            A = inputs.poisson(3, int(rng.integers(3, 20)), 0.5, seed * 100 + k)
        else:
            A = inputs.rgg_laplacian(int(rng.integers(50, 5000)), seed * 100 + k)
        out.append(dict(A=A, b=inputs.rhs(A.n, seed * 100 + k), tol=tol, maxit=3000))
    return out


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_batch_equals_single_bitwise(gpu_lib, dt):
    pcg = gpu_lib
    systems = _mix(1, 12, tol=1e-8 if dt == "f64" else 1e-6)  # FP32 cannot certify 1e-8
    kw = dict(vec_dtype=dt, a_dtype=dt, g_dtype=dt)
    say("batch vs single", dt, [s["A"].n for s in systems])
    with pcg.Solver(pcg.default_config(**kw)) as s:
        batch = s.solve_batch(systems, iters_per_step=7)
    with pcg.Solver(pcg.default_config(**kw)) as s:
        for sd, (xb, rb) in zip(systems, batch):
            s.set_matrix(sd["A"])
            s.build_precond(pcg.G_FSAI)
            single = s.solve(sd["b"], tol=sd["tol"], maxit=sd["maxit"])
            # plain FP32 x cannot always certify the tolerance (the attainable
            # residual is about u32 ||A|| ||x||): equality is what is required
            assert rb["status"] == single.status
            if dt == "f64":
                assert rb["status"] == pcg.OK
            assert rb["iters"] == single.iters
            assert np.array_equal(xb, single.x)


@pytest.mark.parametrize("gdt", ["bf16", "f32"])
def test_refined_batch_equals_single_and_oracle(gpu_lib, gdt):
    """FP32 vectors and A, G in gdt, FP64 refinement to 1e-8 for every system
    of the batch: bit-identical to the single refined solve, and within the
    single-solve bar of the FP64 oracle."""
    pcg = gpu_lib
    systems = _mix(5, 9, tol=1e-8)
    kw = dict(vec_dtype="f32", a_dtype="f32", g_dtype=gdt, refine=1)
    say("refined batch", gdt, [s["A"].n for s in systems])
    with pcg.Solver(pcg.default_config(**kw)) as s:
        batch = s.solve_batch(systems, iters_per_step=6)
    with pcg.Solver(pcg.default_config(**kw)) as s:
        for sd, (xb, rb) in zip(systems, batch):
            s.set_matrix(sd["A"])
            s.build_precond(pcg.G_FSAI)
            single = s.solve(sd["b"], tol=1e-8, maxit=3000)
            assert rb["status"] == single.status == pcg.OK
            assert rb["iters"] == single.iters and rb["outer_iters"] == single.outer_iters
            assert np.array_equal(xb, single.x)
            r64 = np.linalg.norm(sd["b"] - oracle.spmv(sd["A"], xb)) / np.linalg.norm(sd["b"])
            assert r64 <= 1.0001e-8 and rb["relres_true"] <= 1e-8
            ref = oracle.pcg(sd["A"], oracle.fsai_g(sd["A"]), sd["b"], tol=1e-12, maxit=20000, delta_form=1)
            kappa_bound = 1e-8 * np.linalg.cond(sd["A"].to_dense()) if sd["A"].n <= 1500 else None
            err = np.linalg.norm(xb - ref.x) / np.linalg.norm(ref.x)
            say(f"  n={sd['A'].n} outer={rb['outer_iters']} inner={rb['iters']} relres64={r64:.2e} err={err:.2e}")
            if kappa_bound is not None:
                assert err <= kappa_bound


def test_batch_matches_oracle(gpu_lib):
    """Batched systems given the oracle's FSAI G (the library's own FSAI
    agrees with it to 1e-13 only): each equals the oracle's solve."""
    pcg = gpu_lib
    systems = _mix(2, 9)
    for sd in systems:
        sd["G"] = oracle.fsai_g(sd["A"])
    with pcg.Solver(pcg.default_config()) as s:
        batch = s.solve_batch(systems)
    for sd, (x, r) in zip(systems, batch):
        ref = oracle.pcg(sd["A"], sd["G"], sd["b"], tol=1e-8, maxit=3000, delta_form=1)
        # exact inner products on both sides: the oracle's trajectory bit for bit
        assert r["status"] == ref.status == pcg.OK and r["iters"] == ref.iters
        assert np.array_equal(x, ref.x)


def test_served_alone_equals_mixed(gpu_lib):
    """Continuous batching: requests arrive while others run (admitted between
    steps). A request's result is bit-identical to the same request alone."""
    pcg = gpu_lib
    systems = _mix(3, 15, tol=1e-8)
    cfg = pcg.default_config(vec_dtype="f32", a_dtype="f32", g_dtype="bf16", refine=1)
    alone = []
    with pcg.Solver(cfg) as s:
        for sd in systems:
            alone.append(s.solve_batch([sd])[0])
    say("served mix")
    with pcg.Solver(cfg) as s:
        tickets = []
        waves = [systems[0:5], systems[5:9], systems[9:15]]
        got = {}
        for w in waves:
            tickets += s.submit(w)
            for _ in range(3):
                s.progress(5)
                for t in tickets:
                    if t not in got:
                        r = s.poll(t)
                        if r is not None:
                            got[t] = r
        while len(got) < len(tickets):
            s.progress(10)
            for t in tickets:
                if t not in got:
                    r = s.poll(t)
                    if r is not None:
                        got[t] = r
        assert s.pool_info()[1] == 0  # everything retired and freed
    for sd, t, (xa, ra) in zip(systems, tickets, alone):
        xm, rm = got[t]
        say(f"  n={sd['A'].n} alone {ra['status']} {ra['iters']}/{ra['outer_iters']} {ra['relres_true']:.2e} "
            f"mixed {rm['status']} {rm['iters']}/{rm['outer_iters']} {rm['relres_true']:.2e} "
            f"latency {rm['t_latency_ms']:.1f} ms queue {rm['t_queue_ms']:.1f} ms")
    for t, (xa, ra) in zip(tickets, alone):
        xm, rm = got[t]
        assert rm["status"] == ra["status"] == pcg.OK and rm["relres_true"] <= 1e-8
        assert rm["iters"] == ra["iters"] and np.array_equal(xm, xa)
        assert rm["t_latency_ms"] >= rm["t_queue_ms"] >= 0


def test_batch_mixed_outcomes(gpu_lib):
    """Zero right-hand side, iteration limit and breakdown in one batch with a
    normal system: each system gets its own status, the normal one is
    unaffected."""
    pcg = gpu_lib
    A = inputs.poisson(2, 20, 0.5, 4)
    b = inputs.rhs(A.n, 4)
    neg = CSR(A.rowptr, A.col, -A.val)
    G = oracle.fsai_g(A)
    systems = [dict(A=A, b=b, G=G, tol=1e-8, maxit=3000), dict(A=A, b=np.zeros(A.n), x0=np.ones(A.n)),
               dict(A=A, b=b, G=G, tol=1e-8, maxit=5),
               dict(A=neg, b=b, G=oracle.identity(A.n), tol=1e-8, maxit=100)]
    with pcg.Solver(pcg.default_config()) as s:
        res = s.solve_batch(systems, iters_per_step=4)
    (x0, r0), (x1, r1), (x2, r2), (x3, r3) = res
    ref = oracle.pcg(A, G, b, tol=1e-8, maxit=3000, delta_form=1)
    assert r0["status"] == pcg.OK and np.array_equal(x0, ref.x)
    assert r1["status"] == pcg.OK and r1["iters"] == 0 and np.all(x1 == 0)
    assert r2["status"] == pcg.NOT_CONVERGED and r2["iters"] == 5
    ref5 = oracle.pcg(A, G, b, maxit=5, delta_form=1)
    assert np.array_equal(x2, ref5.x)
    assert r3["status"] == pcg.EBREAKDOWN


def test_admission_by_memory_budget(gpu_lib):
    """A 4 MiB pool: a system larger than the pool is refused with ENOMEM;
    the others are admitted as room frees up and all complete."""
    pcg = gpu_lib
    small = [dict(A=inputs.poisson(2, 30, 0.5, k), b=inputs.rhs(900, k), tol=1e-8, maxit=2000) for k in range(6)]
    big = inputs.poisson(3, 60, 0.5, 9)
    systems = small[:3] + [dict(A=big, b=inputs.rhs(big.n, 9), tol=1e-8, maxit=100)] + small[3:]
    with pcg.Solver(pcg.default_config(mem_budget_mb=4)) as s:
        res = s.solve_batch(systems, iters_per_step=10)
        cap, used = s.pool_info()
    assert cap == 4 << 20 and used == 0
    assert res[3][1]["status"] == pcg.ENOMEM
    for k, (x, r) in enumerate(res):
        if k != 3:
            assert r["status"] == pcg.OK and r["relres_true"] <= 1e-8


@pytest.mark.parametrize("refine", [0, 1])
def test_batch_with_blocked_systems_equals_single(gpu_lib, refine):
    """Elasticity systems (A in the 3x3-block layout) batched with Poisson and
    RGG systems (sliced ELL, CSR): each equals its single solve bit for bit,
    plain FP64 and FP32 with FP64 refinement (whose FP64 view of A keeps the
    block layout)."""
    pcg = gpu_lib
    systems = []
    for k, A in enumerate([inputs.elasticity(5, 1.0, 0.3, 1), inputs.poisson(3, 12, 0.5, 2),
                           inputs.elasticity(7, 1.0, 0.3, 3), inputs.rgg_laplacian(3000, 4)]):
        systems.append(dict(A=A, b=inputs.rhs(A.n, k), tol=1e-9, maxit=4000))
    kw = dict(vec_dtype="f32", a_dtype="f32", g_dtype="bf16", refine=1) if refine else {}
    say("blocked batch", refine, [s["A"].n for s in systems])
    with pcg.Solver(pcg.default_config(**kw)) as s:
        batch = s.solve_batch(systems, iters_per_step=9)
    with pcg.Solver(pcg.default_config(**kw)) as s:
        for sd, (xb, rb) in zip(systems, batch):
            s.set_matrix(sd["A"])
            s.build_precond(pcg.G_FSAI)
            single = s.solve(sd["b"], tol=sd["tol"], maxit=sd["maxit"])
            assert rb["status"] == single.status == pcg.OK
            assert rb["iters"] == single.iters and np.array_equal(xb, single.x)
            r64 = np.linalg.norm(sd["b"] - oracle.spmv(sd["A"], xb)) / np.linalg.norm(sd["b"])
            assert r64 <= 1.0001e-9


def test_wait_and_timeout(gpu_lib):
    """pcg_wait: a zero time limit returns pending with nothing collected;
    without a limit it drives the scheduler until every ticket is done and
    the results equal those of a batch solve; a collected ticket is refused;
    a ticket listed twice gets its result twice."""
    pcg = gpu_lib
    systems = _mix(6, 5)
    with pcg.Solver(pcg.default_config()) as s:
        ref = s.solve_batch(systems)
    with pcg.Solver(pcg.default_config()) as s:
        tickets = s.submit(systems)
        assert s.wait(tickets, timeout_s=0.0) is None
        got = s.wait(tickets)
        assert s.pool_info()[1] == 0
        st = s._lib.pcg_wait(s._h, 1, (pcg.ctypes.c_uint64 * 1)(tickets[0]), None, -1.0)
        assert st == pcg.EINVAL
        t2 = s.submit(systems[:2])
        dup = s.wait([t2[0], t2[1], t2[0]])
        assert s.pool_info()[1] == 0 and len(dup) == 3
        assert dup[0][1] == dup[2][1] and np.array_equal(dup[0][0], ref[0][0])
        assert np.array_equal(dup[1][0], ref[1][0])
    for (xr, rr), (xw, rw) in zip(ref, got):
        assert rw["status"] == rr["status"] == pcg.OK and rw["iters"] == rr["iters"]
        assert np.array_equal(xw, xr)


@pytest.mark.parametrize("refine", [0, 1])
def test_estimate_bytes_covers_admitted_storage(gpu_lib, refine):
    """The host-only estimate is an upper bound of what admission takes from
    the pool, for A in CSR, sliced diagonals and 3x3 blocks (it knows only n
    and the nonzero counts, so it cannot tell that a stencil needs no column
    indices in the sliced-diagonal layout: up to about 1.7x there)."""
    pcg = gpu_lib
    kw = dict(vec_dtype="f32", a_dtype="f32", g_dtype="bf16", refine=1) if refine else {}
    cfg = pcg.default_config(**kw)
    for A in [inputs.poisson(3, 24, 0.5, 1), inputs.elasticity(8, 1.0, 0.3, 2), inputs.rgg_laplacian(6000, 3)]:
        nnz_g = (A.nnz + A.n) // 2
        est = pcg.estimate_bytes(cfg, A.n, A.nnz, nnz_g)
        with pcg.Solver(cfg) as s:
            t = s.submit([dict(A=A, b=inputs.rhs(A.n, 1), tol=1e-10, maxit=5000)])
            used = 0
            for _ in range(2000):
                act, _q = s.progress(1)
                if act:
                    used = s.pool_info()[1]
                    break
                time.sleep(0.002)
            s.wait(t)
        say(f"estimate n={A.n} nnz={A.nnz} refine={refine}: used {used} estimate {est}")
        assert 0 < used <= est <= 1.8 * used + (512 << 10)


@pytest.mark.parametrize("mixed", [0, 1])
def test_device_fsai_at_admission_equals_host_fsai(gpu_lib, mixed):
    """g_device = 1 in a batch: the FSAI of each admitted system is factored
    on the device (the host lays out only the patterns); its values equal the
    host builder's bit for bit, so every result equals the host-FSAI batch.
    A system whose tril rows exceed the device builder's limit falls back to
    the host builder in the same batch."""
    pcg = gpu_lib
    systems = _mix(8, 7, tol=1e-8)
    big = _random_spd_long(900, 3)
    systems.append(dict(A=big, b=inputs.rhs(big.n, 3), tol=1e-8, maxit=3000))
    kw = dict(vec_dtype="f32", a_dtype="f32", g_dtype="bf16", refine=1) if mixed else {}
    with pcg.Solver(pcg.default_config(**kw)) as s:
        ref = s.solve_batch(systems, iters_per_step=8)
    with pcg.Solver(pcg.default_config(g_device=1, **kw)) as s:
        got = s.solve_batch(systems, iters_per_step=8)
    for sd, (xr, rr), (xg, rg) in zip(systems, ref, got):
        assert rg["status"] == rr["status"] == pcg.OK, (sd["A"].n, rg["status"])
        assert rg["iters"] == rr["iters"] and np.array_equal(xg, xr)


def _random_spd_long(n, seed):
    """Diagonally dominant SPD matrix with one row of n - 1 entries (its tril
    row exceeds the device FSAI's 80-entry limit)."""
    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    m = sp.random(n, n, density=4.0 / n, random_state=seed, data_rvs=lambda k: rng.uniform(-1, 1, k)).tolil()
    m[n - 1, : n - 1] = rng.uniform(-1, 1, n - 1) / n
    m = m.tocsr()
    m = m + m.T
    m.setdiag(0)
    m.eliminate_zeros()
    m = m + sp.diags(np.asarray(abs(m).sum(axis=1)).ravel() + 1.0)
    return CSR.from_scipy(m)


def test_submit_rejects_bad_systems(gpu_lib):
    """pcg_submit_batch checks every system before queueing any: a column out
    of range, or G arrays that disagree with nnz_g, give PCG_EINVAL with a
    message from the submission, nothing is queued, and the context then
    solves a good system."""
    pcg = gpu_lib
    A = inputs.poisson(2, 8, 0.5, 0)
    good = dict(A=A, b=inputs.rhs(A.n, 0), tol=1e-8, maxit=500)
    col = A.col.copy()
    col[-1] = A.n
    bad_a = dict(good, A=inputs.CSR(A.rowptr, col, A.val))
    bad_g = dict(good, G=inputs.CSR(A.rowptr, A.col[:-1].copy(), A.val[:-1].copy()))
    with pcg.Solver(pcg.default_config(mem_budget_mb=64)) as s:
        for bad in (bad_a, bad_g):
            with pytest.raises(pcg.PCGError) as e:
                s.submit([good, bad])
            say("rejected:", e.value)
            assert e.value.status == pcg.EINVAL and "pcg_submit_batch" in str(e.value)
            assert s.progress(1) == (0, 0)
        (x, r), = s.solve_batch([good])
    assert r["status"] == pcg.OK and r["relres_true"] <= 1e-8


def test_batched_restart_equals_single(gpu_lib):
    """The restart on a failed true-residual check (no replacement, tolerance
    near the attainable floor) in batched systems: each one restarts as its
    single solve does and as the oracle does, and ends bit for bit equal to
    both."""
    pcg = gpu_lib
    systems, refs = [], []
    for dim, N, sigma, seed in [(3, 16, 2.0, 1), (2, 48, 2.0, 2), (3, 12, 0.5, 3)]:
        A = inputs.poisson(dim, N, sigma, seed)
        b = inputs.rhs(A.n, seed)
        G = oracle.fsai_g(A)
        systems.append(dict(A=A, b=b, G=G, tol=1e-13, maxit=5000))
        refs.append(oracle.pcg(A, G, b, tol=1e-13, maxit=5000, rr_period=0, delta_form=1))
    with pcg.Solver(pcg.default_config(rr_period=0)) as s:
        batch = s.solve_batch(systems, iters_per_step=10)
    with pcg.Solver(pcg.default_config(rr_period=0)) as s:
        for sd, ref, (xb, rb) in zip(systems, refs, batch):
            s.set_matrix(sd["A"])
            s.set_precond(sd["G"])
            single = s.solve(sd["b"], tol=sd["tol"], maxit=sd["maxit"])
            say(f"batched restart n={sd['A'].n}: batch {rb['iters']} it {rb['restarts']} restarts, single "
                f"{single.iters} it {single.restarts}, oracle {ref.iters} it {ref.restarts}")
            assert rb["status"] == single.status == pcg.OK
            assert rb["restarts"] == single.restarts == ref.restarts
            assert rb["iters"] == single.iters == ref.iters
            assert np.array_equal(xb, single.x) and np.array_equal(xb, ref.x)
    assert sum(r.restarts for r in refs) >= 2


def test_block_fsai_in_a_batch_equals_single(gpu_lib):
    """Systems with the block FSAI built by the library at admission (host
    worker) solve bit for bit as alone, next to scalar-FSAI systems."""
    pcg = gpu_lib
    systems = []
    for k, N in enumerate((4, 7, 5)):
        A = inputs.elasticity(N, 1.0, 0.3, 30 + k)
        systems.append(dict(A=A, b=inputs.rhs(A.n, 30 + k), g_kind=pcg.G_BFSAI, tol=1e-9, maxit=4000))
    A = inputs.poisson(3, 12, 0.5, 33)
    systems.append(dict(A=A, b=inputs.rhs(A.n, 33), tol=1e-9, maxit=4000))
    with pcg.Solver(pcg.default_config()) as s:
        batch = s.solve_batch(systems, iters_per_step=5)
    with pcg.Solver(pcg.default_config()) as s:
        for sd, (xb, rb) in zip(systems, batch):
            s.set_matrix(sd["A"])
            s.build_precond(sd.get("g_kind", pcg.G_FSAI))
            single = s.solve(sd["b"], tol=sd["tol"], maxit=sd["maxit"])
            assert rb["status"] == single.status == pcg.OK
            assert rb["iters"] == single.iters and np.array_equal(xb, single.x)


def test_one_workgroup_systems_in_a_batch(gpu_lib):
    """Batched systems below the one-workgroup limit are solved whole, one
    workgroup each, in one launch per admission step beside the iterations of
    the larger ones: every result equals its single solve and the oracle's
    bit for bit, with the limit on or off."""
    pcg = gpu_lib
    systems = []
    for k, (dim, N) in enumerate([(2, 20), (3, 9), (2, 100), (3, 24), (2, 45), (3, 6)]):
        A = inputs.poisson(dim, N, 1.0, 40 + k)
        systems.append(dict(A=A, b=inputs.rhs(A.n, 40 + k), G=oracle.fsai_g(A), tol=1e-9, maxit=4000))
    out = {}
    for wg in (-1, 5000):
        with pcg.Solver(pcg.default_config(wg_max_n_batch=wg)) as s:
            out[wg] = s.solve_batch(systems, iters_per_step=7)
    for sd, (x1, r1), (x2, r2) in zip(systems, out[-1], out[5000]):
        ref = oracle.pcg(sd["A"], sd["G"], sd["b"], tol=1e-9, maxit=4000, delta_form=1)
        say(f"batch n={sd['A'].n}: three-kernel {r1['iters']} it, one-workgroup {r2['iters']} it, oracle {ref.iters}")
        assert r1["status"] == r2["status"] == ref.status == pcg.OK
        assert r1["iters"] == r2["iters"] == ref.iters
        assert np.array_equal(x1, x2) and np.array_equal(x2, ref.x)


def _banded(n, seed):
    """Symmetric banded SPD matrix (offsets 1, 2, 7; uniform off-diagonal
    values in (-1, -0.05); a dominant diagonal)."""
    import scipy.sparse as sp

    rng = np.random.default_rng(seed)
    rows, cols, vals = [], [], []
    for o in (o for o in (1, 2, 7) if o < n):
        i = np.arange(0, n - o)
        v = -rng.uniform(0.05, 1.0, n - o)
        rows += [i, i + o]
        cols += [i + o, i]
        vals += [v, v]
    rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    d = np.asarray(abs(m).sum(axis=1)).ravel() + 0.5
    return CSR.from_scipy((m + sp.diags(d)).tocsr())


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_one_workgroup_lds_bound_in_a_batch(gpu_lib, dt):
    """In a batch the one-workgroup solver keeps a system's seven iteration
    vectors in LDS up to 28,672 bytes (512 FP64 rows, 1024 FP32 rows) and in
    global memory above that, both in the same launch. Systems on both sides
    of the bound (and far from it) give their single solves' results bit for
    bit, and in FP64 the oracle's."""
    pcg = gpu_lib
    ns = (300, 511, 512, 513, 1024, 1025, 3000)
    kw = {} if dt == "f64" else dict(vec_dtype="f32", a_dtype="f32", g_dtype="f32")
    tol = 1e-9 if dt == "f64" else 1e-5
    systems = []
    for k, n in enumerate(ns):
        A = _banded(n, 70 + k)
        systems.append(dict(A=A, b=inputs.rhs(n, 70 + k), G=oracle.fsai_g(A), tol=tol, maxit=2000))
    with pcg.Solver(pcg.default_config(wg_max_n_batch=5000, **kw)) as s:
        batch = s.solve_batch(systems, iters_per_step=5)
    with pcg.Solver(pcg.default_config(wg_max_n=5000, **kw)) as s:
        for sd, (xb, rb) in zip(systems, batch):
            s.set_matrix(sd["A"])
            s.set_precond(sd["G"])
            single = s.solve(sd["b"], tol=sd["tol"], maxit=sd["maxit"])
            say(f"lds bound {dt} n={sd['A'].n}: batch {rb['iters']} it, single {single.iters} it")
            assert rb["status"] == single.status == pcg.OK
            assert rb["iters"] == single.iters and np.array_equal(xb, single.x)
            if dt == "f64":
                ref = oracle.pcg(sd["A"], sd["G"], sd["b"], tol=tol, maxit=2000, delta_form=1)
                assert ref.iters == single.iters and np.array_equal(ref.x, single.x)


def test_batch_stats_device_time_and_bytes(gpu_lib):
    """pcg_batch_stats_get: the scheduler's iteration steps are timed on the
    device and their bytes are each system's iterations times its bytes per
    iteration, so over a whole batch they add up to the results' own
    iterations x bytes_per_iter (split between the steps and the
    one-workgroup launches when small systems take those); a reset zeroes
    the counters."""
    pcg = gpu_lib
    systems = _mix(3, 9)
    for wgb in (-1, 0):
        with pcg.Solver(pcg.default_config(wg_max_n_batch=wgb)) as s:
            res = s.solve_batch(systems, iters_per_step=10)
            st = s.batch_stats(reset=True)
            st2 = s.batch_stats()
        want = sum(r["iters"] * r["bytes_per_iter"] for _, r in res)
        say("batch stats", wgb, st, want)
        assert all(r["status"] == pcg.OK for _, r in res)
        got = st["step_bytes"] + st["wg_bytes"]
        assert abs(got - want) <= 1e-9 * want
        if wgb == -1:
            assert st["wg_launches"] == 0 and st["steps"] > 0 and st["step_ms"] > 0
        else:
            assert st["wg_launches"] >= 1 and st["wg_ms"] > 0
        assert st2["steps"] == 0 and st2["step_bytes"] == 0 and st2["wg_launches"] == 0
