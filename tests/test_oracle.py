"""Pins for the FP64 oracle, against facts that do not come from the oracle
itself: dense brute force, exact rational arithmetic, closed forms, textbook
special cases (scipy's CG), and invariants of CG and FSAI."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from paper_2510_27517_amd import inputs
from paper_2510_27517_amd.inputs import CSR


def _random_csr(n, m, density, seed, empty_rows=()):
    rng = np.random.default_rng(seed)
    d = np.where(rng.random((n, m)) < density, rng.standard_normal((n, m)), 0.0)
    for r in empty_rows:
        d[r, :] = 0.0
    rp, cols, vals = [0], [], []
    for i in range(n):
        for j in range(m):
            if d[i, j] != 0.0:
                cols.append(j)
                vals.append(d[i, j])
        rp.append(len(cols))
    return CSR(np.array(rp, np.int32), np.array(cols, np.int32), np.array(vals)), d


def _dense_spd(n, seed, cond=50.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.geomspace(1.0, cond, n)
    return (Q * lam) @ Q.T


# ------------------------------------------------------------------ SpMV (P1, P2)

@pytest.mark.parametrize("n,density,seed", [(1, 1.0, 0), (17, 0.3, 1), (64, 0.1, 2), (200, 0.03, 3)])
def test_spmv_matches_dense(n, density, seed):
    A, d = _random_csr(n, n, density, seed, empty_rows=(0,) if n > 1 else ())
    x = np.random.default_rng(seed + 100).standard_normal(n)
    y = oracle.spmv(A, x)
    bound = (np.diff(A.rowptr).max(initial=0) + 1) * 2.0 ** -53 * (np.abs(d) @ np.abs(x))
    assert np.all(np.abs(y - d @ x) <= bound + 1e-300)
    if n > 1:
        assert y[0] == 0.0


def test_spmv_exact_on_integers():
    A, d = _random_csr(50, 50, 0.2, 9)
    A.val[:] = np.round(A.val * 8)
    d = A.to_dense()
    x = np.arange(50, dtype=np.float64) - 20
    assert np.array_equal(oracle.spmv(A, x), d @ x)


@pytest.mark.parametrize("n,seed", [(1, 0), (33, 4), (150, 5)])
def test_spmv_t_dense_and_adjoint(n, seed):
    G, d = _random_csr(n, n, 0.15 if n > 1 else 1.0, seed)
    rng = np.random.default_rng(seed)
    r, y = rng.standard_normal(n), rng.standard_normal(n)
    gt = oracle.spmv_t(G, r)
    assert np.allclose(gt, d.T @ r, rtol=0, atol=1e-13 * (np.abs(d.T) @ np.abs(r) + 1))
    assert abs(gt @ y - r @ oracle.spmv(G, y)) <= 1e-12 * (np.abs(gt) @ np.abs(y) + 1)


def test_transpose_dense_and_involution():
    G, d = _random_csr(40, 40, 0.2, 6, empty_rows=(3, 7))
    T = oracle.transpose(G)
    assert np.array_equal(CSR(T.rowptr, T.col, T.val).to_dense(), d.T)
    TT = oracle.transpose(T)
    assert np.array_equal(TT.rowptr, G.rowptr) and np.array_equal(TT.col, G.col) and np.array_equal(TT.val, G.val)
    for i in range(40):
        assert np.all(np.diff(T.col[T.rowptr[i]:T.rowptr[i + 1]]) > 0)


# --------------------------------------------------------- apply, locality (P3)

@pytest.mark.parametrize("eps", [0.0, 0.37])
def test_apply_matches_locality_formula(eps):
    """Eq. "spai-locality": s_j = eps r_j + sum_l G_jl sum_k G_kl r_k, with
    G on A's pattern, evaluated as the literal double sum over the graph."""
    A = inputs.poisson(2, 5, sigma=0.5, seed=1)
    rng = np.random.default_rng(2)
    G = CSR(A.rowptr.copy(), A.col.copy(), rng.standard_normal(A.nnz))
    r = rng.standard_normal(A.n)
    Gd = G.to_dense()
    n = A.n
    s_ref = np.empty(n)
    for j in range(n):
        acc = eps * r[j]
        for l in range(n):
            if Gd[j, l] == 0.0:
                continue
            inner = sum(Gd[k, l] * r[k] for k in range(n) if Gd[k, l] != 0.0)
            acc += Gd[j, l] * inner
        s_ref[j] = acc
    s = oracle.apply_precond(G, r, eps)
    assert np.allclose(s, s_ref, rtol=1e-13, atol=1e-13)


# ------------------------------------------------------------------ PCG (P4-P8)

def _exact_pcg(Ad, Gd, b, eps, steps):
    """CG of Algorithm 1 in exact rational arithmetic (no replacement needed)."""
    n = len(b)
    A = [[Fraction(v) for v in row] for row in Ad]
    G = [[Fraction(v) for v in row] for row in Gd]
    e = Fraction(eps)
    Minv = [[sum(G[i][k] * G[j][k] for k in range(n)) + (e if i == j else 0) for j in range(n)] for i in range(n)]
    mv = lambda M, v: [sum(M[i][j] * v[j] for j in range(n)) for i in range(n)]
    dotf = lambda a, c: sum(ai * ci for ai, ci in zip(a, c))
    x = [Fraction(0)] * n
    r = [Fraction(v) for v in b]
    d = mv(Minv, r)
    delta = dotf(r, d)
    xs, rs = [list(x)], [dotf(r, r)]
    for _ in range(steps):
        if delta == 0:
            break
        q = mv(A, d)
        alpha = delta / dotf(d, q)
        x = [xi + alpha * di for xi, di in zip(x, d)]
        r = [ri - alpha * qi for ri, qi in zip(r, q)]
        s = mv(Minv, r)
        dnew = dotf(r, s)
        beta = dnew / delta
        delta = dnew
        d = [si + beta * di for si, di in zip(s, d)]
        xs.append(list(x))
        rs.append(dotf(r, r))
    return xs, rs


@pytest.mark.parametrize("gkind,eps", [("identity", 0.0), ("diag", 0.0), ("lower", 0.25)])
def test_pcg_matches_exact_rational_cg(gkind, eps):
    Ad = np.array([[6, -1, 0, 2, 0], [-1, 5, -2, 0, 0], [0, -2, 7, -1, 1], [2, 0, -1, 4, 0], [0, 0, 1, 0, 3]], float)
    b = np.array([1.0, -2.0, 0.5, 3.0, -1.0])
    if gkind == "identity":
        Gd = np.eye(5)
    elif gkind == "diag":
        Gd = np.diag([0.5, 0.25, 1.0, 0.5, 0.5])
    else:
        Gd = np.tril(np.array([[1, 0, 0, 0, 0], [-0.25, 0.5, 0, 0, 0], [0, 0.125, 1, 0, 0],
                               [0.5, 0, -0.25, 1, 0], [0, 0, 0.25, 0, 0.5]], float))
    xs, rs = _exact_pcg(Ad, Gd, b, eps, 5)
    assert rs[-1] == 0  # exact CG terminates in n steps
    res = oracle.pcg(CSR.from_dense(Ad), CSR.from_dense(Gd), b, eps=eps, tol=1e-13, maxit=20,
                     history=True, x_history=True)
    assert res.status == oracle.OK
    for k in range(len(xs) - 1):
        xk = np.array([float(v) for v in xs[k]])
        assert np.allclose(res.xhist[k], xk, rtol=1e-12, atol=1e-13)
        assert abs(res.rhist[k] - np.sqrt(float(rs[k]))) <= 1e-12 * np.sqrt(float(rs[0]))
    xstar = np.linalg.solve(Ad, b)
    assert np.allclose(res.x, xstar, rtol=1e-12, atol=1e-13)
    assert res.iters <= 6


@pytest.mark.parametrize("n,seed", [(12, 0), (30, 1)])
def test_finite_termination(n, seed):
    Ad = _dense_spd(n, seed, cond=30.0)
    b = np.random.default_rng(seed).standard_normal(n)
    res = oracle.pcg(CSR.from_dense(Ad), oracle.identity(n), b, tol=1e-12, maxit=10 * n)
    # exact CG stops after n steps (pinned exactly by the rational test); in
    # FP64 the Krylov basis loses orthogonality, so allow a few extra steps
    assert res.status == oracle.OK and res.iters <= n + n // 4 + 2
    assert np.allclose(res.x, np.linalg.solve(Ad, b), rtol=1e-10)


def test_distinct_eigenvalues_terminate_early():
    n, m = 40, 5
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.repeat([1.0, 2.0, 3.5, 5.0, 9.0], n // m)
    Ad = (Q * lam) @ Q.T
    Ad = (Ad + Ad.T) / 2
    res = oracle.pcg(CSR.from_dense(Ad), oracle.identity(n), rng.standard_normal(n), tol=1e-10, maxit=100)
    assert res.status == oracle.OK and res.iters <= m + 1


def test_exact_inverse_preconditioner_one_iteration():
    """G = L^-T for A = L L^T gives M^-1 = A^-1: one iteration. The other
    orientation, G = L^-1 (G G^T != A^-1), must not."""
    n = 12
    Ad = _dense_spd(n, 4, cond=1e3)
    L = np.linalg.cholesky(Ad)
    Linv = np.linalg.inv(L)
    b = np.random.default_rng(4).standard_normal(n)
    A = CSR.from_dense(Ad)
    good = oracle.pcg(A, CSR.from_dense(Linv.T), b, tol=1e-8, maxit=50)
    assert good.status == oracle.OK and good.iters == 1
    bad = oracle.pcg(A, CSR.from_dense(Linv), b, tol=1e-8, maxit=50)
    assert bad.iters > 3


def test_monotone_energy_error():
    A = inputs.poisson(2, 12, sigma=1.0, seed=2)
    b = inputs.rhs(A.n, 1)
    Ad = A.to_dense()
    xstar = np.linalg.solve(Ad, b)
    for G in (oracle.fsai_g(A), oracle.identity(A.n)):
        res = oracle.pcg(A, G, b, tol=1e-10, maxit=500, x_history=True)
        e = res.xhist - xstar
        en = np.sqrt(np.einsum("ki,ij,kj->k", e, Ad, e))
        assert np.all(np.diff(en) <= 1e-12 * en[0])
        assert en[-1] < 1e-6 * en[0]


@pytest.mark.parametrize("gkind", ["identity", "jacobi"])
def test_matches_scipy_cg(gkind):
    A = inputs.poisson(2, 20, sigma=0.5, seed=7)
    b = inputs.rhs(A.n, 3)
    G = oracle.identity(A.n) if gkind == "identity" else oracle.diag_inv_sqrt(A)
    Gs = CSR(G.rowptr, G.col, G.val).to_scipy()
    M = spla.aslinearoperator(Gs @ Gs.T)
    count = [0]

    def cb(_):
        count[0] += 1

    xs, info = spla.cg(A.to_scipy(), b, rtol=1e-8, atol=0.0, maxiter=2000, M=M, callback=cb)
    assert info == 0
    res = oracle.pcg(A, G, b, tol=1e-8, maxit=2000, rr_period=0)
    assert res.status == oracle.OK
    assert abs(res.iters - count[0]) <= 1
    assert np.linalg.norm(res.x - xs) <= 1e-6 * np.linalg.norm(xs)


def test_power_of_two_scale_invariance_bitwise():
    """CG is invariant to the scale of A (Sec. 3.3): A -> 4A, G -> G/2 leaves
    every step's rounding unchanged, so x scales by exactly 1/4."""
    A = inputs.poisson(3, 6, sigma=1.0, seed=8)
    b = inputs.rhs(A.n, 8)
    G = oracle.fsai_g(A)
    r1 = oracle.pcg(A, G, b, tol=1e-10, maxit=500)
    A4 = CSR(A.rowptr, A.col, A.val * 4.0)
    G2 = oracle.Mat(G.rowptr, G.col, G.val * 0.5)
    r2 = oracle.pcg(A4, G2, b, tol=1e-10, maxit=500)
    assert r1.iters == r2.iters
    assert np.array_equal(r2.x * 4.0, r1.x)


def test_delta_forms_agree():
    A = inputs.poisson(3, 8, sigma=1.0, seed=9)
    b = inputs.rhs(A.n, 9)
    G = oracle.fsai_g(A)
    for eps in (0.0, 1e-3):
        a = oracle.pcg(A, G, b, eps=eps, delta_form=0)
        c = oracle.pcg(A, G, b, eps=eps, delta_form=1)
        assert a.status == c.status == oracle.OK
        assert abs(a.iters - c.iters) <= 1
        assert np.linalg.norm(a.x - c.x) <= 1e-9 * np.linalg.norm(a.x)


def test_cg_iteration_bound_closed_form():
    """Constant 2D Poisson, N=64: lambda_jk = 4 - 2cos(j pi/65) - 2cos(k pi/65).
    The classical CG bound ||r_k||/||b|| <= sqrt(kappa) 2 rho^k caps the
    iteration count of plain CG."""
    N = 64
    A = inputs.poisson(2, N)
    b = inputs.rhs(A.n, 0)
    th = np.arange(1, N + 1) * np.pi / (N + 1)
    lam = (2 - 2 * np.cos(th))[:, None] + (2 - 2 * np.cos(th))[None, :]
    kappa = lam.max() / lam.min()
    assert abs(kappa - 1711.6) < 0.5
    rho = (np.sqrt(kappa) - 1) / (np.sqrt(kappa) + 1)
    bound = np.log(2 * np.sqrt(kappa) / 1e-8) / -np.log(rho)
    res = oracle.pcg(A, oracle.identity(A.n), b, tol=1e-8)
    assert res.status == oracle.OK and res.iters <= bound
    g1 = oracle.pcg(A, oracle.g_cfg1(A), b, tol=1e-8)
    assert g1.status == oracle.OK and g1.iters < res.iters


def test_edge_cases():
    A = inputs.poisson(2, 4)
    G = oracle.identity(A.n)
    z = oracle.pcg(A, G, np.zeros(A.n), x0=np.ones(A.n))
    assert z.status == oracle.OK and z.iters == 0 and np.all(z.x == 0)
    b = inputs.rhs(A.n)
    x0 = np.full(A.n, 0.5)
    m0 = oracle.pcg(A, G, b, x0=x0, maxit=0)
    assert m0.status == oracle.NOT_CONVERGED and m0.iters == 0 and np.array_equal(m0.x, x0)
    one = oracle.pcg(CSR(np.array([0, 1], np.int32), np.array([0], np.int32), np.array([4.0])),
                     oracle.identity(1), np.array([2.0]))
    assert one.status == oracle.OK and one.iters == 1 and one.x[0] == 0.5
    neg = CSR(A.rowptr, A.col, -A.val)
    br = oracle.pcg(neg, G, b)
    assert br.status == oracle.EBREAKDOWN
    nanb = b.copy()
    nanb[3] = np.nan
    assert oracle.pcg(A, G, nanb).status != oracle.OK


def test_restart_on_drifted_recurrence_terminates():
    A = inputs.poisson(2, 32, sigma=1.0, seed=4)
    b = inputs.rhs(A.n, 4)
    res = oracle.pcg(A, oracle.identity(A.n), b, tol=1e-15, maxit=600, rr_period=0)
    assert res.iters <= 600
    if res.status == oracle.OK:
        assert res.relres_true <= 1e-15
    else:
        assert res.status == oracle.NOT_CONVERGED


# ------------------------------------------------------------------ FSAI (P9)

def test_fsai_invariants_on_tril_pattern():
    A = inputs.poisson(3, 6, sigma=1.0, seed=5)
    GL = oracle.fsai_lower(A)
    Ld = CSR(GL.rowptr, GL.col, GL.val).to_dense()
    Ad = A.to_dense()
    assert np.array_equal(Ld != 0, np.tril(Ad) != 0)
    P = Ld @ Ad @ Ld.T
    assert np.allclose(np.diag(P), 1.0, atol=1e-13)
    GA = Ld @ Ad
    for i in range(A.n):
        for j in GL.col[GL.rowptr[i]:GL.rowptr[i + 1]]:
            if j != i:
                assert abs(GA[i, j]) < 1e-13 * np.abs(Ad).max()

    def kaporin(M):
        ev = np.linalg.eigvalsh(M)
        return ev.mean() / np.exp(np.log(ev).mean())

    dinv = 1 / np.sqrt(np.diag(Ad))
    assert kaporin(P) <= kaporin(Ad * dinv[:, None] * dinv[None, :]) + 1e-12


def test_fsai_full_pattern_is_inverse_cholesky():
    n = 12
    Ad = _dense_spd(n, 7, cond=1e3)
    GL = oracle.fsai_lower(CSR.from_dense(Ad))
    Ld = CSR(GL.rowptr, GL.col, GL.val).to_dense()
    assert np.allclose(Ld, np.linalg.inv(np.linalg.cholesky(Ad)), atol=1e-10)


def test_fsai_orientation_beats_flipped_on_variable_coefficients():
    A = inputs.poisson(3, 16, sigma=1.0, seed=0)
    b = inputs.rhs(A.n, 0)
    good = oracle.pcg(A, oracle.fsai_g(A), b)
    flipped = oracle.pcg(A, oracle.fsai_lower(A), b)
    jac = oracle.pcg(A, oracle.diag_inv_sqrt(A), b)
    assert good.status == flipped.status == jac.status == oracle.OK
    assert good.iters < flipped.iters and good.iters < jac.iters


def test_cfg1_g_closed_form_values():
    A = inputs.poisson(2, 8)
    G = oracle.g_cfg1(A)
    for i in range(A.n):
        for k in range(G.rowptr[i], G.rowptr[i + 1]):
            j = G.col[k]
            assert j <= i
            assert G.val[k] == (0.5 if j == i else 0.0625)
    assert G.nnz == (A.nnz + A.n) // 2


@pytest.mark.parametrize("period", [1, 5])
def test_residual_replacement_schedule(period):
    """Algorithm 1 recomputes r = b - A x when the iteration index i is a
    positive multiple of the period (read: i > 0). After such an iteration the
    recurrence residual is bit-identical to b - A x formed from the stored
    iterate; after the others it is the updated r - alpha q."""
    A = inputs.poisson(2, 16, sigma=1.0, seed=3)
    b = inputs.rhs(A.n, 3)
    res = oracle.pcg(A, oracle.fsai_g(A), b, tol=1e-12, maxit=40, rr_period=period, history=True,
                     x_history=True)
    assert res.iters >= 12
    replaced, updated = 0, 0
    for k in range(1, 12):
        i = k - 1
        rt = b - oracle.spmv(A, res.xhist[k])
        tn = np.sqrt(oracle.dot(rt, rt))
        if i > 0 and i % period == 0:
            assert res.rhist[k] == tn
            replaced += 1
        else:
            updated += res.rhist[k] != tn  # the update r - alpha q rounds differently
            if i == 0:
                assert res.rhist[k] != tn  # no replacement at i = 0
    assert replaced >= 2
    if period > 1:
        assert updated >= 3


# ------------------------------------------------------- seeded full-pattern G

def _u_from_definition(seed, i, j, n):
    """2U - 1 for draw index i*n + j of the preconditioner stream, computed
    here from the SplitMix64 definition (not through the input module)."""
    MASK, GAMMA = (1 << 64) - 1, 0x9E3779B97F4A7C15

    def mix(z):
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)

    key = mix((mix((seed + GAMMA) & MASK) + 4 * GAMMA) & MASK)  # stream 3
    v = mix((key + (int(i) * int(n) + int(j) + 1) * GAMMA) & MASK)
    return 2.0 * (((v >> 11) + 1) * 2.0 ** -53) - 1.0


def test_seeded_g_definition():
    """Full pattern of A; G_ii = 1/sqrt(A_ii) exactly; G_ij equals
    0.25 u_ij |A_ij| / sqrt(A_ii A_jj) with u_ij from the generator's
    definition at index i*n + j; a different seed changes every off-diagonal
    entry; the draws are spread over (-1, 1]."""
    assert inputs.STREAM_G == 3
    A = inputs.poisson(2, 12, 1.0, 5)
    G = oracle.seeded_g(A, 42)
    assert np.array_equal(G.rowptr, A.rowptr) and np.array_equal(G.col, A.col)
    d = A.to_dense().diagonal()
    us = []
    for i in range(A.n):
        for k in range(A.rowptr[i], A.rowptr[i + 1]):
            j = A.col[k]
            if j == i:
                assert G.val[k] == 1.0 / np.sqrt(d[i])
            else:
                u = _u_from_definition(42, i, j, A.n)
                assert -1.0 < u <= 1.0
                assert G.val[k] == pytest.approx(0.25 * u * abs(A.val[k]) / np.sqrt(d[i] * d[j]), rel=1e-15)
                us.append(u)
    us = np.array(us)
    assert abs(us.mean()) < 0.1 and abs(us.var() - 1 / 3) < 0.05
    G2 = oracle.seeded_g(A, 43)
    off = A.col != np.repeat(np.arange(A.n), np.diff(A.rowptr))
    assert np.all(G2.val[off] != G.val[off]) and np.array_equal(G2.val[~off], G.val[~off])


def test_seeded_g_with_shift_solves_to_dense_solution():
    """With the shift eps = 1e-4 / mean|A_ij|, M^-1 = G G^T + eps I is SPD and
    PCG reaches the dense solution; the shift helper is that ratio."""
    A = inputs.rgg_laplacian(400, 8)
    b = inputs.rhs(A.n, 8)
    eps = oracle.eps_shift(A)
    assert eps == 1e-4 / np.mean(np.abs(A.val))
    G = oracle.seeded_g(A, 1)
    Gd = np.zeros((A.n, A.n))
    for i in range(A.n):
        Gd[i, G.col[G.rowptr[i]:G.rowptr[i + 1]]] = G.val[G.rowptr[i]:G.rowptr[i + 1]]
    Minv = Gd @ Gd.T + eps * np.eye(A.n)
    assert np.linalg.eigvalsh(Minv).min() > 0
    res = oracle.pcg(A, G, b, eps=eps, tol=1e-12, maxit=5000)
    xs = np.linalg.solve(A.to_dense(), b)
    assert res.status == oracle.OK
    assert np.linalg.norm(res.x - xs) <= 1e-9 * np.linalg.norm(xs)


# ------------------------------------------------------------ SAI loss (Sec. 3.3)

def _dense_g(G, n):
    D = np.zeros((n, n))
    for i in range(n):
        D[i, G.col[G.rowptr[i]:G.rowptr[i + 1]]] = G.val[G.rowptr[i]:G.rowptr[i + 1]]
    return D


@pytest.mark.parametrize("eps", [0.0, 0.02])
def test_sai_loss_unit_probes_give_the_frobenius_norm(eps):
    """With the n unit vectors as probes the sums are exact:
    sum_p sai = ||A M^-1 / ||A|| - I||_F^2 and sum_p l2 = ||A M^-1 - I||_F^2,
    formed here with dense matrices."""
    A = inputs.poisson(2, 5, 1.0, 3)
    G = oracle.fsai_g(A)
    n = A.n
    Ad = A.to_dense()
    Minv = _dense_g(G, n) @ _dense_g(G, n).T + eps * np.eye(n)
    na = np.mean(np.abs(A.val))
    out = oracle.sai_losses(A, G, np.eye(n), eps)
    E = Ad @ Minv / na - np.eye(n)
    F = Ad @ Minv - np.eye(n)
    assert out["sai"].sum() == pytest.approx(np.sum(E * E), rel=1e-12)
    assert out["l2"].sum() == pytest.approx(np.sum(F * F), rel=1e-12)
    for p in range(n):
        col = (Ad @ Minv)[:, p]
        assert out["cs"][p] == pytest.approx(col[p] / np.linalg.norm(col), rel=1e-12)


def test_sai_loss_exact_inverse_closed_form():
    """G = L^-T (A = L L^T) makes M^-1 = A^-1: y = w, so sai = (1/||A|| - 1)^2
    ||w||^2, l2 = 0 and cs = 1."""
    Ad = _dense_spd(12, 4)
    A = CSR.from_dense(Ad)
    L = np.linalg.cholesky(Ad)
    G = CSR.from_dense(np.linalg.inv(L).T)
    W = inputs.normal(1, inputs.STREAM_PROBE, 12 * 3).reshape(12, 3)
    out = oracle.sai_losses(A, G, W)
    na = np.mean(np.abs(A.val))
    for p in range(3):
        w = W[:, p]
        assert out["sai"][p] == pytest.approx((1 / na - 1) ** 2 * np.dot(w, w), rel=1e-10)
        assert out["l2"][p] <= 1e-20 * np.dot(w, w)
        assert out["cs"][p] == pytest.approx(1.0, abs=1e-12)


def test_sai_loss_scale_invariant_bitwise():
    """||A|| scales with A, so for a power-of-two factor the SAI loss is the
    same bit for bit (Sec. 3.3); the L2 loss is not scale invariant."""
    A = inputs.poisson(3, 6, 1.0, 2)
    G = oracle.fsai_g(A)
    W = inputs.normal(2, inputs.STREAM_PROBE, A.n * 4).reshape(A.n, 4)
    a = oracle.sai_losses(A, G, W)
    b = oracle.sai_losses(CSR(A.rowptr, A.col, A.val * 8.0), G, W)
    assert np.array_equal(a["sai"], b["sai"]) and np.array_equal(a["cs"], b["cs"])
    assert not np.allclose(a["l2"], b["l2"])


def test_hutchinson_mean_approaches_the_frobenius_norm():
    """E_w ||B w||^2 = ||B||_F^2 for w ~ N(0, I) (Eq. "loss-initial"): the mean
    over 4000 probes is within 10% (its relative spread is below 3%)."""
    A = inputs.poisson(2, 4, 1.0, 5)
    G = oracle.diag_inv_sqrt(A)
    n = A.n
    W = inputs.normal(3, inputs.STREAM_PROBE, n * 4000).reshape(n, 4000)
    out = oracle.sai_losses(A, G, W)
    exact = oracle.sai_losses(A, G, np.eye(n))["sai"].sum()
    assert abs(out["sai"].mean() - exact) <= 0.1 * exact


# ---------------------------------------------- mixed precision (emulation)

def test_round_storage_matches_numpy_binary32_and_binary16():
    """Once-rounded RNE onto binary32 and binary16 equals numpy's direct
    double-to-float conversions, normals, subnormals, ties and overflow."""
    rng = np.random.default_rng(40)
    x = rng.standard_normal(20000) * 10.0 ** rng.integers(-46, 40, 20000)
    x = np.concatenate([x, [0.0, -0.0, 3.4e38, 3.5e38, -1e39, 1e-45, 7e-46, 65504.0, 65519.9, 65520.0, 6e-8,
                            2.0 ** -25, 3 * 2.0 ** -26, 1.0 + 2.0 ** -24, 1.0 + 3 * 2.0 ** -24]])
    with np.errstate(over="ignore"):
        assert np.array_equal(oracle.round_storage(x, "f32"), x.astype(np.float32).astype(np.float64))
        assert np.array_equal(oracle.round_storage(x, "f16"), x.astype(np.float16).astype(np.float64))
    assert np.array_equal(oracle.round_storage(x, "f64"), x)


def test_round_storage_bfloat16_brute_force():
    """bfloat16: nearest of all finite values (the binary32 patterns with the
    low 16 bits clear), ties to the even pattern, including exact midpoints."""
    k = np.arange(0, 0x7F80, dtype=np.uint32)
    vals = (k << 16).view(np.float32).astype(np.float64)  # all finite non-negative bf16, ascending
    rng = np.random.default_rng(41)
    x = np.abs(rng.standard_normal(5000)) * 10.0 ** rng.integers(-40, 38, 5000)
    mids = (vals[1:] + vals[:-1]) / 2  # exact in FP64 (9 significant bits)
    x = np.concatenate([x, mids[rng.integers(0, mids.shape[0], 2000)], [0.0, vals[-1]]])
    i = np.clip(np.searchsorted(vals, x), 1, vals.shape[0] - 1)
    lo, hi = vals[i - 1], vals[i]
    pick_hi = (x - lo > hi - x) | ((x - lo == hi - x) & (k[i] % 2 == 0))
    want = np.where(x >= vals[-1], vals[-1], np.where(pick_hi, hi, lo))
    want = np.where(x == 0, 0.0, want)
    got = oracle.round_storage(x, "bf16")
    assert np.array_equal(got, want)
    assert np.array_equal(oracle.round_storage(-x, "bf16"), -want)


def test_g_storage_scale_places_max_in_binade():
    G = CSR(np.array([0, 1, 3], np.int32), np.array([0, 0, 1], np.int32), np.array([3e-7, -1.5e-9, 2.4e-7]))
    sc = oracle.g_storage_scale(G, "f16")
    assert 2.0 ** 13 <= np.abs(G.val).max() * sc < 2.0 ** 14 and np.log2(sc) == int(np.log2(sc))
    assert oracle.g_storage_scale(G, "bf16") == 1.0


def test_recurrence_only_stop_equals_confirmed_stop_without_drift():
    """stop_rule 2 (no true-residual confirmation) takes the same iterates as
    stop_rule 0 when the confirmation never fails."""
    A = inputs.poisson(2, 20, 0.5, 3)
    b = inputs.rhs(A.n, 3)
    G = oracle.fsai_g(A)
    r0 = oracle.pcg(A, G, b, tol=1e-6, rr_period=0, delta_form=1, stop_rule=0)
    r2 = oracle.pcg(A, G, b, tol=1e-6, rr_period=0, delta_form=1, stop_rule=2)
    assert r0.restarts == 0 and r0.status == r2.status == oracle.OK
    assert r0.iters == r2.iters and np.array_equal(r0.x, r2.x)
    assert r2.relres_rec <= 1e-6


def test_ir_exact_storage_one_step():
    """Unrounded storage and a tight inner tolerance: one outer step reaches
    tol and x is the dense solution to the residual bound."""
    A = inputs.poisson(2, 16, 0.5, 4)
    b = inputs.rhs(A.n, 4)
    res = oracle.pcg_ir(A, oracle.fsai_g(A), b, tol=1e-8, a_dtype="f64", g_dtype="f64", vec_dtype="f64",
                        inner_tol=1e-12)
    Ad = A.to_dense()
    xs = np.linalg.solve(Ad, b)
    assert res.status == oracle.OK and res.outer == 1 and res.relres_true <= 1e-8
    assert np.linalg.norm(res.x - xs) <= np.linalg.cond(Ad) * 1e-8 * np.linalg.norm(xs)


def test_inner_tolerance_schedule():
    """Steps run to inner_tol, or to a quarter of the remaining reduction when
    that is looser (never looser than 1/2); after the first step also when it
    is down to inner_tol / 10 (the finishing step)."""
    it = oracle.inner_tolerance
    assert it(1e-6, 1e-8, 1.0, 1.0, 0) == 1e-6           # 2.5e-9 needed: not the last step
    assert it(1e-6, 1e-8, 1.0, 1e-4, 1) == 0.25 * 1e-8 / 1e-4  # 2.5e-5: finish now
    assert it(1e-6, 1e-8, 1.0, 2e-2, 1) == 0.25 * 1e-8 / 2e-2  # 1.25e-7 >= inner_tol / 10: finish
    assert it(1e-6, 1e-8, 1.0, 2e-2, 0) == 1e-6          # the first step stays at inner_tol
    assert it(1e-6, 1e-6, 1.0, 1.0, 0) == 1e-6           # 2.5e-7: first step, not looser
    assert it(1e-6, 1e-8, 1.0, 2.6e-2, 1) == 1e-6        # 9.6e-8 < inner_tol / 10
    assert it(1e-6, 1e-4, 1.0, 1.0, 0) == 0.25 * 1e-4    # looser than inner_tol: any step
    assert it(1e-4, 1e-8, 1.0, 2e-9, 3) == 0.5           # capped


def test_ir_each_step_contracts_by_the_inner_tolerance():
    """Exact storage: the inner solve is CG on A c = r/||r|| itself, so the
    FP64 residual after x += ||r|| c is ||r|| times the inner relative
    residual, at most the inner tolerance of that step."""
    A = inputs.poisson(3, 8, 0.5, 5)
    b = inputs.rhs(A.n, 5)
    res = oracle.pcg_ir(A, oracle.fsai_g(A), b, tol=1e-13, a_dtype="f64", g_dtype="f64", vec_dtype="f64",
                        inner_tol=1e-3)
    h = res.rhist
    assert res.status == oracle.OK and res.outer == h.shape[0] - 1 >= 3
    for k in range(res.outer):
        eta = oracle.inner_tolerance(1e-3, 1e-13, 1.0, h[k], k)
        assert h[k + 1] <= eta * h[k] * (1 + 1e-6) + 1e-15, (k, h)


@pytest.mark.parametrize("gdt", ["bf16", "f16", "f32"])
def test_ir_rounded_storage_reaches_tolerance(gdt):
    """A in FP32, G in gdt, vectors rounded to FP32: the FP64 outer residual
    still reaches 1e-10 (the inner operator differs from A by about
    2^-24 |A|, far inside the contraction), decreasing at every step."""
    A = inputs.poisson(3, 10, 1.0, 6)
    b = inputs.rhs(A.n, 6)
    res = oracle.pcg_ir(A, oracle.fsai_g(A), b, tol=1e-10, a_dtype="f32", g_dtype=gdt)
    assert res.status == oracle.OK and res.relres_true <= 1e-10 and 2 <= res.outer <= 5
    assert np.all(np.diff(res.rhist) < 0)
    r = b - oracle.spmv(A, res.x)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b)


def test_ir_edge_cases():
    A = inputs.poisson(2, 12, 0.5, 7)
    b = inputs.rhs(A.n, 7)
    G = oracle.fsai_g(A)
    z = oracle.pcg_ir(A, G, np.zeros(A.n))
    assert z.status == oracle.OK and z.outer == 0 and np.all(z.x == 0)
    one = oracle.pcg_ir(A, G, b, tol=1e-14, max_outer=1)
    assert one.status == oracle.NOT_CONVERGED and one.outer == 1 and one.relres_true <= 1e-3
    neg = CSR(A.rowptr, A.col, -A.val)
    bd = oracle.pcg_ir(neg, oracle.identity(A.n), b)
    assert bd.status == oracle.EBREAKDOWN and bd.outer == 0
    # one plain CG step per inner solve gains less and less: the loop stops
    # at the first outer step that fails to gain 10 %
    L = inputs.poisson(2, 30, 0.5, 8)
    st = oracle.pcg_ir(L, oracle.identity(L.n), inputs.rhs(L.n, 8), tol=1e-12, a_dtype="f64", g_dtype="f64",
                       vec_dtype="f64", maxit=1, max_outer=50)
    assert st.status == oracle.NOT_CONVERGED and 1 < st.outer < 50
    assert st.rhist[-1] > 0.9 * st.rhist[-2] and np.all(st.rhist[1:-1] <= 0.9 * st.rhist[:-2])
    # high-contrast coefficients stored in bfloat16 lose definiteness: the
    # inner solve breaks down instead of returning a wrong answer
    H = inputs.poisson(2, 40, 2.0, 8)
    hb = oracle.pcg_ir(H, oracle.fsai_g(H), inputs.rhs(H.n, 8), tol=1e-12, a_dtype="bf16")
    assert hb.status == oracle.EBREAKDOWN and np.all(hb.x == 0)


# -------------------------------------------- FP32 products (mixed-precision path)

def _f32_rows_brute(d32, x32, reverse=False, wide=False):
    """y_i = sum over the stored columns j of row i of f32(d_ij * x_j), added
    one at a time from 0 in float32 (numpy float32 scalars: every product and
    sum rounded to binary32), columns ascending (descending with reverse);
    wide: products exact and sums in float64, rounded to float32 once (a
    wrong accumulator the pins must reject)."""
    n, m = d32.shape
    y = np.zeros(n, np.float32)
    for i in range(n):
        cols = [j for j in range(m) if d32[i, j] != 0]
        if reverse:
            cols = cols[::-1]
        if wide:
            y[i] = np.float32(sum(float(d32[i, j]) * float(x32[j]) for j in cols))
            continue
        s = np.float32(0.0)
        for j in cols:
            s = np.float32(s + np.float32(d32[i, j] * x32[j]))
        y[i] = s
    return y


def _mixed_scale_csr(n, density, seed):
    """Random pattern with values spread over many binades, so that float32
    sums depend on the order and the accumulator width."""
    A, d = _random_csr(n, n, density, seed)
    rng = np.random.default_rng(seed + 7)
    scale = np.exp2(rng.integers(-12, 13, A.nnz))
    A.val[:] = A.val * scale
    return A


@pytest.mark.parametrize("n,density,seed", [(1, 1.0, 0), (40, 0.3, 1), (120, 0.15, 2)])
def test_spmv_f32_matches_float32_brute_force(n, density, seed):
    A = _mixed_scale_csr(n, density, seed)
    v32 = A.val.astype(np.float32)
    d32 = CSR(A.rowptr, A.col, v32.astype(np.float64)).to_dense().astype(np.float32)
    x32 = (np.random.default_rng(seed + 50).standard_normal(n) * 3.0).astype(np.float32)
    got = oracle.spmv_f32(A.rowptr, A.col, v32, x32)
    assert got.dtype == np.float32
    ref = _f32_rows_brute(d32, x32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    if n > 1:  # the data tells the wrong orders and accumulators apart
        assert not np.array_equal(ref, _f32_rows_brute(d32, x32, reverse=True))
        assert not np.array_equal(ref, _f32_rows_brute(d32, x32, wide=True))


@pytest.mark.parametrize("n,density,seed", [(1, 1.0, 3), (40, 0.3, 4), (120, 0.15, 5)])
def test_spmv_t_f32_matches_float32_brute_force(n, density, seed):
    """(G^T x)_j = sum over i ascending of f32(G_ij x_i), in float32: the order
    in which scattering the rows of G delivers the terms of column j."""
    G = _mixed_scale_csr(n, density, seed)
    v32 = G.val.astype(np.float32)
    d32 = CSR(G.rowptr, G.col, v32.astype(np.float64)).to_dense().astype(np.float32)
    x32 = (np.random.default_rng(seed + 60).standard_normal(n) * 3.0).astype(np.float32)
    got = oracle.spmv_t_f32(G.rowptr, G.col, v32, x32)
    assert got.dtype == np.float32
    ref = _f32_rows_brute(np.ascontiguousarray(d32.T), x32)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    if n > 1:
        assert not np.array_equal(ref, _f32_rows_brute(np.ascontiguousarray(d32.T), x32, reverse=True))
        assert not np.array_equal(ref, _f32_rows_brute(np.ascontiguousarray(d32.T), x32, wide=True))


def test_spmv_f32_exact_on_small_integers():
    """Small integers: every product and partial sum is below 2^24, so float32
    arithmetic is exact in any order and equals the integer product."""
    A, _ = _random_csr(60, 60, 0.25, 11)
    A.val[:] = np.round(A.val * 50)
    d = A.to_dense()
    x = np.arange(60, dtype=np.float64) - 25
    v32, x32 = A.val.astype(np.float32), x.astype(np.float32)
    assert np.array_equal(oracle.spmv_f32(A.rowptr, A.col, v32, x32).astype(np.float64), d @ x)
    assert np.array_equal(oracle.spmv_t_f32(A.rowptr, A.col, v32, x32).astype(np.float64), d.T @ x)


def test_spmv_f32_rounds_each_operation_to_binary32():
    """One row [2^24, 1, 1] times ones: float32 adds lose each 1 (2^24 + 1 is a
    tie rounded to even), so the sum stays 2^24; an FP64 accumulator gives
    2^24 + 2. The reversed order gives 1 + 1 + 2^24 = 2^24 + 2 exactly."""
    rp, ci = np.array([0, 3], np.int32), np.array([0, 1, 2], np.int32)
    v = np.array([2.0 ** 24, 1.0, 1.0], np.float32)
    y = oracle.spmv_f32(rp, ci, v, np.ones(3, np.float32))
    assert float(y[0]) == 2.0 ** 24
    # transpose: column 0 of [[1],[1],[2^24]] (rows 0, 1, 2 scattered in order)
    rp3, ci3 = np.array([0, 1, 2, 3], np.int32), np.zeros(3, np.int32)
    vt = np.array([1.0, 1.0, 2.0 ** 24], np.float32)
    yt = oracle.spmv_t_f32(rp3, ci3, vt, np.ones(3, np.float32))
    assert float(yt[0]) == 2.0 ** 24 + 2.0
    vt2 = np.array([2.0 ** 24, 1.0, 1.0], np.float32)
    assert float(oracle.spmv_t_f32(rp3, ci3, vt2, np.ones(3, np.float32))[0]) == 2.0 ** 24


# ------------------------------------------------------- Jacobi factor D^-1/2

def test_diag_inv_sqrt_closed_form_constant_poisson():
    """Constant 2D Poisson has A_ii = 4, so G = D^-1/2 = I / 2 exactly."""
    A = inputs.poisson(2, 9)
    G = oracle.diag_inv_sqrt(A)
    assert np.array_equal(G.rowptr, np.arange(A.n + 1)) and np.array_equal(G.col, np.arange(A.n))
    assert np.all(G.val == 0.5)


def test_diag_inv_sqrt_matches_dense_diagonal():
    """Variable coefficients: G = diag(1 / sqrt(A_ii)) of the dense matrix, and
    G A G has a unit diagonal."""
    A = inputs.poisson(3, 5, sigma=1.0, seed=4)
    Ad = A.to_dense()
    G = oracle.diag_inv_sqrt(A)
    Gd = CSR(G.rowptr, G.col, G.val).to_dense()
    assert np.array_equal(np.diag(Gd), 1.0 / np.sqrt(np.diag(Ad)))
    assert np.count_nonzero(Gd - np.diag(np.diag(Gd))) == 0
    assert np.allclose(np.diag(Gd @ Ad @ Gd), 1.0, rtol=4e-16, atol=0)


# ------------------------------------------- exact inner products (reading)

def _exact_dot(a, b):
    """The exact sum of products in rational arithmetic, rounded once to the
    nearest double with ties to even (Python's int / int true division)."""
    return float(sum((Fraction(float(x)) * Fraction(float(y)) for x, y in zip(a, b)), Fraction(0)))


def _same_bits(x, y):
    return np.array([x]).view(np.uint64)[0] == np.array([y]).view(np.uint64)[0]


@pytest.mark.parametrize("kind", ["normal", "cancel", "binades", "tiny", "huge"])
def test_dot_is_the_exact_value_rounded_once(kind):
    rng = np.random.default_rng({"normal": 1, "cancel": 2, "binades": 3, "tiny": 4, "huge": 5}[kind])
    for n in (1, 2, 3, 17, 200):
        a, b = rng.standard_normal(n), rng.standard_normal(n)
        if kind == "cancel":  # pairs that cancel up to a small remainder
            a = np.concatenate([a, -a * (1 + 2.0 ** -40 * rng.standard_normal(n))])
            b = np.concatenate([b, b])
        elif kind == "binades":
            a = a * np.exp2(rng.integers(-300, 300, n))
        elif kind == "tiny":  # products in the subnormal range and below
            a = a * 2.0 ** -540
            b = b * 2.0 ** -530
        elif kind == "huge":  # products beyond the largest double that cancel
            a = np.concatenate([a * 2.0 ** 600, -a * 2.0 ** 600])
            b = np.concatenate([b * 2.0 ** 500, b * 2.0 ** 500 + 2.0 ** 380])
        got = oracle.dot(a, b)
        assert _same_bits(got, _exact_dot(a, b)), (n, got, _exact_dot(a, b))


def test_dot_ties_round_to_even_and_order_does_not_matter():
    u = 2.0 ** -53
    # 1 + u lies halfway between 1 and 1 + 2u: the even neighbour is 1
    assert oracle.dot([1.0, u], [1.0, 1.0]) == 1.0
    # (1 + 2u) + u lies halfway between 1 + 2u and 1 + 4u: the even one is 1 + 4u
    assert oracle.dot([1.0 + 2 * u, u], [1.0, 1.0]) == 1.0 + 4 * u
    # a tie broken by a far smaller term (sticky bit): rounds up
    assert oracle.dot([1.0, u, 2.0 ** -200], [1.0, 1.0, 1.0]) == 1.0 + 2 * u
    # a subnormal result is rounded once at the subnormal quantum: 2^-1074
    # (1.5 - 2^-60) gives 2^-1074 (rounding first to 53 bits would make it
    # the tie 1.5 2^-1074 and then round it to even, 2^-1073)
    t = 2.0 ** -537
    assert oracle.dot([t, t, -(2.0 ** -600)], [t, 2.0 ** -538, 2.0 ** -534]) == 2.0 ** -1074
    assert _exact_dot([t, t, -(2.0 ** -600)], [t, 2.0 ** -538, 2.0 ** -534]) == 2.0 ** -1074
    # cancellation a plain left-to-right sum gets wrong
    a, b = [1e16, 1.0, -1e16], [1.0, 1.0, 1.0]
    assert float(np.float64(1e16) + 1.0 - 1e16) != 1.0 and oracle.dot(a, b) == 1.0
    rng = np.random.default_rng(9)
    x = rng.standard_normal(5000) * np.exp2(rng.integers(-60, 60, 5000))
    y = rng.standard_normal(5000)
    ref = oracle.dot(x, y)
    for perm in (rng.permutation(5000), np.arange(5000)[::-1]):
        assert _same_bits(oracle.dot(x[perm], y[perm]), ref)
    for th in (2, 3, 16):
        assert _same_bits(oracle.dot(x, y, threads=th), ref)
    assert _same_bits(ref, _exact_dot(x, y))


def test_dot_overflow_and_non_finite():
    big = 2.0 ** 1000
    assert oracle.dot([big, big], [2.0 ** 23, 2.0 ** 23]) == np.inf
    assert oracle.dot([-big, -big], [2.0 ** 23, 2.0 ** 23]) == -np.inf
    assert oracle.dot([np.inf, 1.0], [1.0, 2.0]) == np.inf
    assert np.isnan(oracle.dot([np.inf, -np.inf], [1.0, 1.0]))
    assert np.isnan(oracle.dot([np.nan, 1.0], [1.0, 1.0]))
    assert np.isnan(oracle.dot([np.inf], [0.0]))
    assert oracle.dot([0.0, -0.0], [1.0, 1.0]) == 0.0


def test_pcg_is_independent_of_the_thread_count():
    """With exact inner products the whole iteration is independent of how
    the dot products are split: x, iterations and residuals bit for bit."""
    A = inputs.poisson(3, 14, sigma=1.0, seed=3)
    b = inputs.rhs(A.n, 3)
    G = oracle.fsai_g(A)
    r1 = oracle.pcg(A, G, b, tol=1e-10, maxit=500, delta_form=1, threads=1)
    for th in (3, 8):
        rt = oracle.pcg(A, G, b, tol=1e-10, maxit=500, delta_form=1, threads=th)
        assert rt.iters == r1.iters and np.array_equal(rt.x, r1.x)


# ------------------------------------------------------------- block FSAI

def _kaporin_log(B):
    n = B.shape[0]
    sign, logdet = np.linalg.slogdet(B)
    assert sign > 0
    return n * np.log(np.trace(B) / n) - logdet


def test_block_fsai_with_b1_is_the_scalar_fsai():
    for A in (inputs.poisson(2, 9, 1.0, 2), inputs.poisson(3, 5, 1.0, 3)):
        G1, B1 = oracle.fsai_lower(A), oracle.fsai_block_lower(A, b=1)
        assert np.array_equal(G1.rowptr, B1.rowptr) and np.array_equal(G1.col, B1.col)
        assert np.array_equal(G1.val, B1.val)


def test_block_fsai_invariants_on_elasticity():
    """Blocked 3-dof system: G_L is block lower with full 3x3 blocks on the
    block pattern of tril(A); each diagonal block of G_L A G_L^T is I_3; and
    (G_L A)_IJ = 0 for every other block J of row I's pattern."""
    A = inputs.elasticity(3, 1.0, 0.3, 1)
    GL = oracle.fsai_block_lower(A)
    Gd, Ad = CSR(GL.rowptr, GL.col, GL.val).to_dense(), A.to_dense()
    n = A.n
    assert np.count_nonzero(np.triu(Gd[:, :], 3)) == 0  # no block above the diagonal block
    P = Gd @ Ad @ Gd.T
    GA = Gd @ Ad
    for I in range(n // 3):
        assert np.allclose(P[3 * I:3 * I + 3, 3 * I:3 * I + 3], np.eye(3), rtol=0, atol=1e-13)
        blocks = sorted({int(c) // 3 for c in GL.col[GL.rowptr[3 * I]:GL.rowptr[3 * I + 1]]})
        assert blocks[-1] == I and all(np.sum(np.abs(Ad[3 * I:3 * I + 3, 3 * J:3 * J + 3])) > 0 for J in blocks)
        for J in blocks[:-1]:
            scale = np.abs(Gd[3 * I:3 * I + 3]).sum() * np.abs(Ad).max()
            assert np.abs(GA[3 * I:3 * I + 3, 3 * J:3 * J + 3]).max() <= 1e-13 * scale
    assert GL.nnz == 9 * sum(1 for I in range(n // 3) for J in range(I + 1)
                             if np.any(Ad[3 * I:3 * I + 3, 3 * J:3 * J + 3]))


def test_block_fsai_full_pattern_is_the_inverse():
    """All blocks of A nonzero: the block FSAI reproduces A^-1 = G_L^T G_L, and
    PCG with G = G_L^T converges in one iteration."""
    n = 12
    Ad = _dense_spd(n, 21, cond=200.0)
    A = CSR.from_dense(Ad)
    GL = oracle.fsai_block_lower(A)
    Gd = CSR(GL.rowptr, GL.col, GL.val).to_dense()
    assert np.allclose(Gd.T @ Gd, np.linalg.inv(Ad), rtol=0, atol=1e-11 * np.abs(np.linalg.inv(Ad)).max())
    b = np.random.default_rng(3).standard_normal(n)
    res = oracle.pcg(A, oracle.transpose(GL), b, tol=1e-10, maxit=10)
    assert res.status == oracle.OK and res.iters == 1


def test_block_fsai_kaporin_no_worse_than_block_jacobi():
    """The block FSAI minimises the Kaporin number of G_L A G_L^T over its
    pattern; block Jacobi (the block FSAI of A's block diagonal) has a pattern
    inside it, so its Kaporin number cannot be smaller."""
    A = inputs.elasticity(3, 1.0, 0.3, 4)
    Ad = A.to_dense()
    n = A.n
    Bd = np.zeros_like(Ad)
    for I in range(n // 3):
        Bd[3 * I:3 * I + 3, 3 * I:3 * I + 3] = Ad[3 * I:3 * I + 3, 3 * I:3 * I + 3]
    rp, ci, vals = [0], [], []
    for r in range(n):
        I = r // 3
        for c in range(3 * I, 3 * I + 3):
            ci.append(c)
            vals.append(Bd[r, c])
        rp.append(len(ci))
    B = CSR(np.array(rp, np.int32), np.array(ci, np.int32), np.array(vals))
    GJ = oracle.fsai_block_lower(B)
    GL = oracle.fsai_block_lower(A)
    kj = _kaporin_log(CSR(GJ.rowptr, GJ.col, GJ.val).to_dense() @ Ad @ CSR(GJ.rowptr, GJ.col, GJ.val).to_dense().T)
    kl = _kaporin_log(CSR(GL.rowptr, GL.col, GL.val).to_dense() @ Ad @ CSR(GL.rowptr, GL.col, GL.val).to_dense().T)
    assert kl < kj


def test_block_fsai_equals_scalar_fsai_as_a_preconditioner():
    """On an exactly blocked matrix the scalar tril pattern of each row of a
    block row is a prefix of the block row's column set, and row k of the
    inverse Cholesky factor of A[J,J] is the FSAI row of the leading k x k
    part: the block FSAI and the scalar FSAI give the same M^-1 = G_L^T G_L
    (they differ in the basis within each block row and in the explicit
    zeros of the diagonal blocks)."""
    A = inputs.elasticity(3, 1.0, 0.3, 6)
    B, S = oracle.fsai_block_lower(A), oracle.fsai_lower(A)
    Bd, Sd = CSR(B.rowptr, B.col, B.val).to_dense(), CSR(S.rowptr, S.col, S.val).to_dense()
    MB, MS = Bd.T @ Bd, Sd.T @ Sd
    assert np.abs(MB - MS).max() <= 1e-14 * np.abs(MS).max()
    assert B.nnz == S.nnz + A.n  # the three entries above the diagonal of each diagonal block


def test_block_fsai_rejects_unblocked_patterns():
    with pytest.raises(ValueError):
        oracle.fsai_block_lower(inputs.poisson(2, 5, 0.0, 0), b=3)  # n = 25, not a multiple of 3
    with pytest.raises(ValueError):
        oracle.fsai_block_lower(inputs.poisson(2, 6, 0.0, 0), b=3)  # n = 36, rows not in complete triples
