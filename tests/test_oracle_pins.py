"""Pins for the CPU oracle: it is checked against facts fixed by the paper and
by mathematics, never against itself.

* hand-derived 1D eigenvalues and a hand-solved n=1 control problem
  (tests/golden/fd_hand_values.txt);
* the closed-form constant-coefficient eigenpairs 4/h^2 sin^2(k pi h/2) and
  the DST-I vectors (Section 3.4);
* dense n^3 x n^3 brute force with distinct coefficients per mode (catches a
  transposed mode, a wrong Kronecker order, a dropped term of f);
* the alpha = 1 sparse identity (no eigensolver involved);
* alpha = 0 (both fractional powers become the identity, Section 4 remark);
* an eigenvector-triple design function (rank-1 exact solution);
* symmetry, positivity and linearity of the solution operator;
* the canonical-format definitions (Appendix 1) against full-grid evaluation;
* the slab-streamed error evaluator against a full-grid evaluation;
* the state and the cost functional: hand-solved n = 1 values, the dense
  matrix function, and the optimality of the exact control (J is stationary
  there, its second variation is the quadratic form of the problem, and
  J* = 1/2 <y_Omega, y_Omega - y*>);
* preconditioner case (A): the sine matrix against SciPy's DST-I, the sine
  diagonalisation of the finite-difference Laplacian, hand-solved n = 1
  values, the dense n^3 x n^3 matrix function of the anisotropic Laplacian,
  and exactness for constant coefficients (P F(A) = I).
"""
import os

import numpy as np
import pytest

import workloads as wl
from oracle import brute, fd, precond, solve, tensor

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fd_hand_values.txt")


def _golden_lines(kind):
    with open(GOLDEN) as fh:
        for line in fh:
            line = line.strip()
            if line.startswith(kind + " "):
                yield line[len(kind) + 1:]


def test_golden_fd_eigenvalues():
    seen = 0
    for rest in _golden_lines("eig"):
        lhs, rhs = rest.split(":")
        parts = lhs.split()
        n = int(parts[1])
        a = np.array([float(v) for v in parts[2:]])
        assert a.shape[0] == n + 1
        want = np.array([float(v) for v in rhs.split()])
        lam, V = fd.eig1d(a)
        np.testing.assert_allclose(lam, want, rtol=1e-13)
        seen += 1
    assert seen >= 4


def test_golden_control_n1():
    seen = 0
    for rest in _golden_lines("control"):
        lhs, rhs = rest.split(":")
        head, m2, m3 = lhs.split("|")
        h = head.split()
        alpha, beta, gamma = float(h[0]), float(h[1]), float(h[2])
        a = [np.array([float(v) for v in h[3:]]), np.array([float(v) for v in m2.split()]),
             np.array([float(v) for v in m3.split()])]
        one = np.ones((1, 1), order="F")
        prob = wl.Problem("golden", 1, a, alpha, beta, gamma, 1e-6, np.ones(1), [one, one, one])
        u = solve.solve_full(prob)
        np.testing.assert_allclose(u.reshape(-1), [float(rhs)], rtol=1e-14)
        seen += 1
    assert seen >= 2


def test_paper_literal_boundary_rows():
    # Section 3.2 prints diagonal entries 2 a_{3/2} and 2 a_{n-1/2} in the first
    # and last rows (times 1/h^2); the literal-sample reading reproduces them.
    a = np.array([0.7, 1.3, 2.1, 0.9, 1.6])
    n = 4
    d, e = fd.stiffness_tridiag(fd.paper_literal_samples(a))
    h2 = 1.0 / (n + 1) ** 2
    assert d[0] == pytest.approx(2 * a[1] / h2, rel=1e-15)
    assert d[-1] == pytest.approx(2 * a[-2] / h2, rel=1e-15)
    assert d[1] == pytest.approx((a[1] + a[2]) / h2, rel=1e-15)
    np.testing.assert_allclose(e, -a[1:-1] / h2, rtol=1e-15)


@pytest.mark.parametrize("n,c", [(7, 1.0), (50, 1.7), (257, 0.3)])
def test_closed_form_constant_coefficient(n, c):
    lam, V = fd.eig1d(np.full(n + 1, c))
    lam_cf, V_cf = fd.laplacian_closed_form(n, c)
    # backward-stable eigensolver: absolute error of order n * eps * ||A||
    np.testing.assert_allclose(lam, lam_cf, rtol=1e-12, atol=64 * 2.2e-16 * lam_cf.max())
    # eigenvectors agree up to sign
    M = np.abs(V.T @ V_cf)
    np.testing.assert_allclose(M, np.eye(n), atol=1e-10)


@pytest.mark.parametrize("seed", [0, 1])
def test_eigen_invariants(seed):
    rng = np.random.default_rng(seed)
    n = 300
    a = 0.1 + 1.8 * rng.random(n + 1)
    lam, V = fd.eig1d(a)
    A = fd.stiffness_dense(a)
    assert np.all(np.diff(lam) > 0)
    assert lam[0] > 0
    assert np.linalg.norm(V.T @ V - np.eye(n)) <= 1e-12
    assert np.linalg.norm(A @ V - V * lam[None, :]) <= 1e-12 * np.linalg.norm(A)


def _tiny_problem(n, alpha, beta=0.7, gamma=1.3, rank=2, seed=11):
    rng = np.random.default_rng(seed)
    xm = wl.midpoints(n)
    a = [1.0 + 0.5 * np.sin(2 * np.pi * xm), 0.3 + xm ** 2, 2.0 - np.cos(3 * xm)]
    w = rng.uniform(0.5, 1.5, rank)
    Y = [np.asfortranarray(rng.standard_normal((n, rank))) for _ in range(3)]
    return wl.Problem("tiny", n, a, alpha, beta, gamma, 1e-6, w, Y)


@pytest.mark.parametrize("alpha", [0.25, 0.5, 0.9, 1.0])
def test_dense_brute_force(alpha):
    prob = _tiny_problem(7, alpha)
    u = solve.solve_full(prob)
    ub = brute.dense_solve(prob)
    assert np.linalg.norm(u - ub) <= 1e-11 * np.linalg.norm(ub)
    # and the residual of the oracle's answer under the dense operator
    r = brute.dense_operator_apply(prob, u) - tensor.cp_full(prob.w, prob.Y)
    assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(tensor.cp_full(prob.w, prob.Y))


def test_dense_brute_force_mode_order():
    # Transposing two modes of the solution must break agreement: the three
    # coefficients differ, so the test is sensitive to the mode order.
    prob = _tiny_problem(6, 0.5)
    u = solve.solve_full(prob)
    ub = brute.dense_solve(prob)
    assert np.linalg.norm(u - ub) <= 1e-11 * np.linalg.norm(ub)
    assert np.linalg.norm(u.transpose(1, 0, 2) - ub) > 1e-3 * np.linalg.norm(ub)


@pytest.mark.parametrize("n", [12, 20])
def test_alpha1_sparse_identity(n):
    prob = _tiny_problem(n, 1.0, beta=1e-2, gamma=1.0)
    u = solve.solve_full(prob)
    us = brute.sparse_alpha1_solve(prob)
    assert np.linalg.norm(u - us) <= 1e-9 * np.linalg.norm(us)


def test_alpha0_is_scaled_identity():
    prob = _tiny_problem(9, 0.0, beta=0.4, gamma=2.0)
    u = solve.solve_full(prob)
    y = tensor.cp_full(prob.w, prob.Y)
    np.testing.assert_allclose(u, y / (0.4 + 2.0 / 0.4), rtol=1e-12, atol=1e-14)


def test_eigenvector_triple_rhs():
    base = wl.workload_sine(n=40, seed=3, rank=1)
    sp = solve.Spectral(base)
    p, q, r = 3, 17, 30
    prob = wl.eigvec_rhs_problem(base, [sp.V[0][:, p], sp.V[1][:, q], sp.V[2][:, r]])
    u = solve.solve_full(prob)
    fval = solve.f_control(sp.lam[0][p] + sp.lam[1][q] + sp.lam[2][r], prob.alpha, prob.beta,
                           prob.gamma)
    y = tensor.cp_full(prob.w, prob.Y)
    np.testing.assert_allclose(u, y / fval, rtol=1e-9, atol=1e-13 * np.abs(y).max() / fval)


def test_symmetry_positivity_linearity():
    p1 = _tiny_problem(10, 0.6, seed=1)
    p2 = _tiny_problem(10, 0.6, seed=2)
    u1, u2 = solve.solve_full(p1), solve.solve_full(p2)
    y1, y2 = tensor.cp_full(p1.w, p1.Y), tensor.cp_full(p2.w, p2.Y)
    s12, s21 = float(np.sum(y1 * u2)), float(np.sum(y2 * u1))
    assert abs(s12 - s21) <= 1e-12 * max(abs(s12), 1e-300) + 1e-14
    assert float(np.sum(y1 * u1)) > 0 and float(np.sum(y2 * u2)) > 0
    p3 = wl.Problem("lin", 10, p1.a, 0.6, p1.beta, p1.gamma, 1e-6,
                    np.concatenate([2.0 * p1.w, -3.0 * p2.w]),
                    [np.hstack([p1.Y[l], p2.Y[l]]) for l in range(3)])
    u3 = solve.solve_full(p3)
    np.testing.assert_allclose(u3, 2.0 * u1 - 3.0 * u2, rtol=1e-10, atol=1e-12 * np.abs(u3).max())


def test_canonical_definitions_against_full_grid():
    rng = np.random.default_rng(5)
    n = (6, 7, 8)
    A = [rng.standard_normal((n[l], 3)) for l in range(3)]
    B = [rng.standard_normal((n[l], 4)) for l in range(3)]
    wa, wb = rng.standard_normal(3), rng.standard_normal(4)
    TA, TB = tensor.cp_full(wa, A), tensor.cp_full(wb, B)
    assert tensor.cp_inner(wa, A, wb, B) == pytest.approx(float(np.sum(TA * TB)), rel=1e-12)
    wh, H = tensor.cp_hadamard(wa, A, wb, B)
    np.testing.assert_allclose(tensor.cp_full(wh, H), TA * TB, rtol=1e-12, atol=1e-12)
    assert len(wh) == 12 and wh[1 * 4 + 2] == pytest.approx(wa[1] * wb[2])


def test_hosvd_orthonormal_closed_form():
    # Orthonormal factors in every mode: the unfolding spectra are the |xi|,
    # so truncation drops the smallest terms and nothing else.
    rng = np.random.default_rng(3)
    n, r = 12, 6
    Q = [np.linalg.qr(rng.standard_normal((n, r)))[0] for _ in range(3)]
    xi = np.array([1.0, 0.5, 0.1, 1e-3, 1e-5, 1e-8])
    T = tensor.cp_full(xi, Q)
    # per-mode budget tol^2 ||T||^2 / 3 = 1e-8: drops 1e-5 and 1e-8, keeps 1e-3
    tol = 1e-4 * np.sqrt(3.0) / np.linalg.norm(xi)
    Tt, ranks, _ = tensor.hosvd_truncate(T, tol)
    assert ranks == (4, 4, 4)
    np.testing.assert_allclose(Tt, tensor.cp_full(xi[:4], [q[:, :4] for q in Q]), atol=1e-12)


def test_hosvd_recovers_tucker_rank():
    rng = np.random.default_rng(4)
    n, r = (14, 12, 10), (3, 4, 2)
    Z = [np.linalg.qr(rng.standard_normal((n[l], r[l])))[0] for l in range(3)]
    core = rng.standard_normal(r)
    T = tensor.tucker_full(core, Z)
    Tt, ranks, _ = tensor.hosvd_truncate(T, 1e-10)
    assert ranks == r
    assert np.linalg.norm(Tt - T) <= 1e-12 * np.linalg.norm(T)


def test_error_evaluator_matches_full_grid():
    prob = _tiny_problem(11, 0.5, rank=3)
    sp = solve.Spectral(prob)
    u = solve.solve_full(prob, sp)
    rng = np.random.default_rng(9)
    # a canonical candidate: perturbation of the exact solution is not low rank,
    # so test with an arbitrary rank-4 tensor plus a consistency check.
    F = [rng.standard_normal((11, 4)) for _ in range(3)]
    w = rng.standard_normal(4)
    Tc = tensor.cp_full(w, F)
    rep = solve.rel_error(prob, w, F, sp)
    want = np.linalg.norm(Tc - u) / np.linalg.norm(u)
    assert rep["rel_l2"] == pytest.approx(want, rel=1e-10)
    y = tensor.cp_full(prob.w, prob.Y)
    Fu = brute.dense_operator_apply(prob, Tc)
    assert rep["rel_residual"] == pytest.approx(np.linalg.norm(y - Fu) / np.linalg.norm(y), rel=1e-8)
    # sampled slabs: numerator and denominator over the same slabs
    rep_s = solve.rel_error(prob, w, F, sp, slabs=[0, 3, 4, 10])
    idx = [0, 3, 4, 10]
    want_s = np.linalg.norm(Tc[idx] - u[idx]) if False else None
    Uh = solve.mode_products(Tc, [V.T for V in sp.V])
    Ex = solve.mode_products(u, [V.T for V in sp.V])
    want_s = np.linalg.norm(Uh[idx] - Ex[idx]) / np.linalg.norm(Ex[idx])
    assert rep_s["rel_l2"] == pytest.approx(want_s, rel=1e-10)
    assert rep_s["slabs"] == 4


def test_slab_rows_and_threaded_evaluator():
    """The per-slab BLAS form of the canonical full tensor equals the
    definition sum_s w_s F1 o F2 o F3 (built elementwise here), and the
    threaded error evaluation equals the single-threaded one over several
    slab groups and a ragged last group."""
    rng = np.random.default_rng(21)
    F = [rng.standard_normal((n, 5)) for n in (13, 7, 9)]
    w = rng.standard_normal(5)
    full = np.einsum("s,is,js,ks->ijk", w, F[0], F[1], F[2])
    np.testing.assert_allclose(solve.slab_rows(w, F, 0, 13), full, rtol=0, atol=1e-13)
    np.testing.assert_allclose(solve.slab_rows(w, F, 4, 9), full[4:9], rtol=0, atol=1e-13)
    prob = _tiny_problem(19, 0.4, rank=2)
    sp = solve.Spectral(prob)
    G = [rng.standard_normal((19, 3)) for _ in range(3)]
    wg = rng.standard_normal(3)
    one = solve.rel_error(prob, wg, G, sp, block=4, workers=1)
    many = solve.rel_error(prob, wg, G, sp, block=4, workers=4)
    assert one["rel_l2"] == many["rel_l2"] and one["rel_residual"] == many["rel_residual"]
    Tc = tensor.cp_full(wg, G)
    u = solve.solve_full(prob, sp)
    assert many["rel_l2"] == pytest.approx(np.linalg.norm(Tc - u) / np.linalg.norm(u), rel=1e-10)


def test_state_recovery_dense():
    prob = _tiny_problem(6, 0.5)
    u = solve.solve_full(prob)
    y = solve.state_full(prob, u)
    A = brute.kron_sum_dense(prob)
    mu, Q = np.linalg.eigh(A)
    S = (Q * (prob.beta * mu ** (-prob.alpha))[None, :]) @ Q.T
    np.testing.assert_allclose(y.reshape(-1), S @ u.reshape(-1), rtol=1e-10,
                               atol=1e-12 * np.abs(y).max())


def test_workload_shapes_and_determinism():
    p = wl.workload_sine(n=64, seed=3)
    q = wl.workload_sine(n=64, seed=3)
    assert p.rank == 10 and all(Y.shape == (64, 10) for Y in p.Y)
    assert all(np.array_equal(p.Y[l], q.Y[l]) for l in range(3))
    assert all(len(a) == 65 and np.all(a > 0) for a in p.a)
    b = wl.workload_batched(count=8)
    assert len(b) == 8 and all(1 <= x.rank <= 10 and 0.2 <= x.alpha <= 0.8 for x in b)
    s = wl.workload_small()
    assert s.n == 32 and s.rank == 1


def test_golden_state_and_cost_n1():
    seen = 0
    for rest in _golden_lines("state"):
        lhs, rhs = rest.split(":")
        head, m2, m3 = lhs.split("|")
        h = head.split()
        alpha, beta, gamma = float(h[0]), float(h[1]), float(h[2])
        a = [np.array([float(v) for v in h[3:]]), np.array([float(v) for v in m2.split()]),
             np.array([float(v) for v in m3.split()])]
        one = np.ones((1, 1), order="F")
        prob = wl.Problem("golden", 1, a, alpha, beta, gamma, 1e-6, np.ones(1), [one, one, one])
        u = solve.solve_full(prob)
        y = solve.state_full(prob, u)
        want_y, want_J = (float(v) for v in rhs.split())
        np.testing.assert_allclose(y.reshape(-1), [want_y], rtol=1e-14)
        assert solve.cost_full(prob, u, y) == pytest.approx(want_J, rel=1e-14)
        assert solve.optimal_cost(prob) == pytest.approx(want_J, rel=1e-14)
        seen += 1
    assert seen >= 2


@pytest.mark.parametrize("alpha", [0.3, 1.0])
def test_cost_is_minimal_at_the_exact_control(alpha):
    """Second variation from the dense matrix function (no 1D eigenbases):
    J(u* + t w) - J(u*) = t^2/2 (||beta A^-alpha w||^2 + gamma ||w||^2) exactly,
    which holds only if the oracle's u* is stationary."""
    prob = _tiny_problem(5, alpha)
    u = solve.solve_full(prob)
    y = solve.state_full(prob, u)
    J0 = solve.cost_full(prob, u, y)
    A = brute.kron_sum_dense(prob)
    mu, Q = np.linalg.eigh(A)
    S = (Q * (prob.beta * mu ** (-prob.alpha))[None, :]) @ Q.T
    rng = np.random.default_rng(4)
    for t in (1e-2, 1e-1, 1.0):
        w = rng.standard_normal(u.shape)
        uw = u + t * w
        yw = (S @ uw.reshape(-1)).reshape(u.shape)
        Sw = S @ w.reshape(-1)
        quad = 0.5 * t * t * (float(Sw @ Sw) + prob.gamma * float(np.sum(w * w)))
        assert solve.cost_full(prob, uw, yw) - J0 == pytest.approx(quad, rel=1e-8, abs=1e-13)
    yom = tensor.cp_full(prob.w, prob.Y)
    assert J0 == pytest.approx(0.5 * float(np.sum(yom * (yom - y))), rel=1e-11)


def test_cost_and_state_evaluators_against_full_grid():
    prob = wl.workload_quadratic(n=12, alpha=0.6, rank=3)
    u = solve.solve_full(prob)
    y = solve.state_full(prob, u)
    # canonical-factor cost on a perturbed canonical pair
    rng = np.random.default_rng(8)
    Fu = [rng.standard_normal((12, 4)) for _ in range(3)]
    wu = rng.standard_normal(4)
    Fy = [rng.standard_normal((12, 5)) for _ in range(3)]
    wy = rng.standard_normal(5)
    uf = tensor.cp_full(wu, Fu)
    yf = tensor.cp_full(wy, Fy)
    assert solve.cost_from_factors(prob, wu, Fu, wy, Fy) == pytest.approx(
        solve.cost_full(prob, uf, yf), rel=1e-12)
    assert solve.optimal_cost(prob) == pytest.approx(solve.cost_full(prob, u, y), rel=1e-12)
    # state evaluator: a candidate with known full-grid error, all slabs and sampled
    cand = y + 1e-3 * yf / np.linalg.norm(yf) * np.linalg.norm(y)
    sp = solve.Spectral(prob)
    # the candidate written exactly as a canonical tensor: its core in a full
    # orthonormal basis, one term per core entry
    Qc = [np.linalg.qr(rng.standard_normal((12, 12)))[0] for _ in range(3)]
    core = solve.mode_products(cand, [q.T for q in Qc])
    idx = np.array(np.unravel_index(np.arange(12 ** 3), (12, 12, 12)))
    wc = core.reshape(-1)
    Fc = [Qc[l][:, idx[l]] for l in range(3)]
    rep = solve.state_rel_error(prob, wc, Fc, sp=sp)
    want = np.linalg.norm(cand - y) / np.linalg.norm(y)
    assert rep["rel_l2"] == pytest.approx(want, rel=1e-8)



# ---- preconditioner case (A), Section 3.5 ----------------------------------

@pytest.mark.parametrize("n", [1, 2, 7, 64, 1000])
def test_dst1_matrix_matches_library_dst(n):
    """S x equals SciPy's orthonormal DST-I; S is symmetric and its own inverse."""
    import scipy.fft
    S = precond.dst1_matrix(n)
    rng = np.random.default_rng(n)
    X = rng.standard_normal((n, 3))
    want = scipy.fft.dst(X, type=1, norm="ortho", axis=0)
    np.testing.assert_allclose(S @ X, want, rtol=0, atol=1e-13 * np.abs(want).max())
    np.testing.assert_allclose(S, S.T, rtol=0, atol=0)
    np.testing.assert_allclose(S @ S, np.eye(n), rtol=0, atol=1e-13 * max(1, n) ** 0.5)


@pytest.mark.parametrize("n", [2, 7, 50])
def test_sine_basis_diagonalises_the_fd_laplacian(n):
    """S Delta S = diag(mu) with Delta the finite-difference matrix of a = 1
    (Section 3.2) and mu ascending (eqn DiagLaplace)."""
    S = precond.dst1_matrix(n)
    Delta = fd.stiffness_dense(np.ones(n + 1))
    mu = precond.laplace_eigenvalues(n)
    D = S @ Delta @ S
    np.testing.assert_allclose(D, np.diag(mu), rtol=0, atol=1e-12 * mu.max())
    assert np.all(np.diff(mu) > 0)


def test_golden_case_a_n1():
    seen = 0
    for rest in _golden_lines("precond"):
        lhs, rhs = rest.split(":")
        v = [float(x) for x in lhs.split()]
        alpha, beta, gamma, b0 = v[0], v[1], v[2], v[3:6]
        one = np.ones((1, 1), order="F")
        prob = wl.Problem("golden", 1, [np.ones(2)] * 3, alpha, beta, gamma, 1e-6, np.ones(1),
                          [one, one, one])
        z = precond.apply_full(prob, np.ones((1, 1, 1)), b0)
        np.testing.assert_allclose(z.reshape(-1), [float(rhs)], rtol=1e-14)
        seen += 1
    assert seen >= 2


def test_b0_midrange():
    """eqn modcoeff: the mid-range of the samples; positive overrides win."""
    prob = _tiny_problem(3, 0.5)
    prob.a = [np.array([0.1, 2.0, 0.5, 1.0]), np.array([3.0, 3.0, 3.0, 3.0]),
              np.array([1.0, 5.0, 2.0, 4.0])]
    np.testing.assert_allclose(precond.b0_for(prob), [1.05, 3.0, 3.0])
    np.testing.assert_allclose(precond.b0_for(prob, [0.0, 1.0, -1.0]), [1.05, 1.0, 3.0])


@pytest.mark.parametrize("alpha", [0.1, 0.5, 1.0])
def test_case_a_dense_brute_force(alpha):
    """P r against the dense n^3 x n^3 matrix function: B = Kronecker sum of
    b0_l Delta assembled densely, B0 = beta B^-alpha + (gamma/beta) B^alpha
    from its dense eigendecomposition, z = B0^-1 r by a dense solve."""
    n = 4
    b0 = [1.7, 0.4, 2.3]
    prob = _tiny_problem(n, alpha)
    prob.beta, prob.gamma = 1.3, 0.6
    I = np.eye(n)
    Delta = fd.stiffness_dense(np.ones(n + 1))
    B = (np.kron(np.kron(b0[0] * Delta, I), I) + np.kron(np.kron(I, b0[1] * Delta), I)
         + np.kron(np.kron(I, I), b0[2] * Delta))
    mu, Q = np.linalg.eigh(B)
    B0 = (Q * (prob.beta * mu ** (-alpha) + prob.gamma / prob.beta * mu ** alpha)[None, :]) @ Q.T
    rng = np.random.default_rng(4)
    r = rng.standard_normal((n, n, n))
    want = np.linalg.solve(B0, r.reshape(-1)).reshape(n, n, n)
    got = precond.apply_full(prob, r, b0)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("alpha", [0.25, 1.0])
def test_case_a_is_exact_for_constant_coefficients(alpha):
    """With a_l = c_l constant, A = B for b0_l = c_l (the default mid-range),
    so P F(A) x = x: F(A) x from the oracle's eigen-path (LAPACK eigenpairs of
    the finite-difference matrices), P from the sine path."""
    n = 9
    c = [0.7, 1.9, 3.1]
    prob = _tiny_problem(n, alpha)
    prob.a = [np.full(n + 1, cl) for cl in c]
    b0 = precond.b0_for(prob)
    np.testing.assert_allclose(b0, c)
    rng = np.random.default_rng(5)
    x = rng.standard_normal((n, n, n))
    Fx = brute.dense_operator_apply(prob, x)
    np.testing.assert_allclose(precond.apply_full(prob, Fx, b0), x, rtol=0, atol=1e-11)
    sp = solve.Spectral(prob)
    xh = solve.mode_products(x, [V.T for V in sp.V])
    Fxh = solve.mode_products(Fx, [V.T for V in sp.V])
    np.testing.assert_allclose(precond.apply_eig(prob, sp, Fxh, b0), xh, rtol=0, atol=1e-11)


def test_case_a_spectral_bound_for_variable_coefficients():
    """Section 3.5 (the condition bound of case (A)): c1 B <= A <= c2 B in the
    Loewner order with c1 = min_l min a_l/b0_l, c2 = max_l max a_l/b0_l (the
    finite-difference matrix is monotone in its coefficient), so by the
    Loewner-Heinz inequality the spectrum of P F(A) lies in
    [min(c1^alpha, c2^-alpha), max(c1^-alpha, c2^alpha)].  Checked densely at
    n = 4 with the paper's coefficients."""
    n = 4
    prob = wl.workload_paper_shaped(n, 0.5)
    b0 = precond.b0_for(prob)
    Fx = np.stack([brute.dense_operator_apply(prob, e.reshape(n, n, n)).reshape(-1)
                   for e in np.eye(n ** 3)], axis=1)
    Pm = np.stack([precond.apply_full(prob, e.reshape(n, n, n), b0).reshape(-1)
                   for e in np.eye(n ** 3)], axis=1)
    ev = np.linalg.eigvals(Pm @ Fx)
    assert np.abs(ev.imag).max() < 1e-9
    ev = ev.real
    lo = min(float(np.min(a)) / b for a, b in zip(prob.a, b0))
    hi = max(float(np.max(a)) / b for a, b in zip(prob.a, b0))
    # f(t s)/f(s) lies in [min(t^-alpha, t^alpha), max(t^-alpha, t^alpha)]
    k = max(lo ** -prob.alpha, hi ** prob.alpha, lo ** prob.alpha, hi ** -prob.alpha)
    assert ev.min() > 1.0 / k - 1e-9 and ev.max() < k + 1e-9


# ---- the d = 2 variant -------------------------------------------------------

from oracle import solve2d  # noqa: E402


def _tiny_problem_2d(n, alpha, beta=0.7, gamma=1.3, rank=2, seed=13):
    rng = np.random.default_rng(seed)
    xm = wl.midpoints(n)
    a = [1.0 + 0.5 * np.sin(2 * np.pi * xm), 0.3 + xm ** 2]
    w = rng.uniform(0.5, 1.5, rank)
    Y = [np.asfortranarray(rng.standard_normal((n, rank))) for _ in range(2)]
    return wl.Problem("tiny2d", n, a, alpha, beta, gamma, 1e-6, w, Y)


def test_golden_control_2d_n1():
    seen = 0
    for rest in _golden_lines("control2d"):
        lhs, rhs = rest.split(":")
        head, m2 = lhs.split("|")
        h = head.split()
        alpha, beta, gamma = float(h[0]), float(h[1]), float(h[2])
        a = [np.array([float(v) for v in h[3:]]), np.array([float(v) for v in m2.split()])]
        one = np.ones((1, 1), order="F")
        prob = wl.Problem("golden2d", 1, a, alpha, beta, gamma, 1e-6, np.ones(1), [one, one])
        u = solve2d.solve_full_2d(prob)
        np.testing.assert_allclose(u.reshape(-1), [float(rhs)], rtol=1e-14)
        seen += 1
    assert seen >= 2


@pytest.mark.parametrize("alpha", [0.25, 0.5, 1.0])
def test_dense_brute_force_2d(alpha):
    """The n^2 x n^2 Kronecker sum eigendecomposed densely (distinct
    coefficients per mode catch a transposed mode)."""
    prob = _tiny_problem_2d(9, alpha)
    np.testing.assert_allclose(solve2d.solve_full_2d(prob), brute.dense_solve_2d(prob),
                               rtol=0, atol=1e-11)


@pytest.mark.parametrize("n", [20, 60])
def test_alpha1_sparse_identity_2d(n):
    prob = _tiny_problem_2d(n, 1.0)
    u = solve2d.solve_full_2d(prob)
    np.testing.assert_allclose(u, brute.sparse_alpha1_solve_2d(prob), rtol=0,
                               atol=1e-10 * np.abs(u).max())


def test_constant_coefficients_2d_by_sine_transform():
    """a_l = c_l: the eigenbasis is the sine basis with eigenvalues
    c_l (4/h^2) sin^2(k pi h/2), so the solution is also the sine transform,
    divide, sine transform back."""
    n = 33
    prob = _tiny_problem_2d(n, 0.5)
    prob.a = [np.full(n + 1, 0.8), np.full(n + 1, 2.2)]
    S = precond.dst1_matrix(n)
    mu = precond.laplace_eigenvalues(n)
    s = 0.8 * mu[:, None] + 2.2 * mu[None, :]
    y = solve2d.cp_full_2d(prob.w, prob.Y)
    u = S @ ((S @ y @ S) / solve.f_control(s, prob.alpha, prob.beta, prob.gamma)) @ S
    np.testing.assert_allclose(solve2d.solve_full_2d(prob), u, rtol=0, atol=1e-12 * np.abs(u).max())


def test_error_evaluator_2d():
    prob = _tiny_problem_2d(12, 0.5)
    u = solve2d.solve_full_2d(prob)
    # an exact rank-n factorisation of u has zero error; a perturbed one its own
    U, s, Vt = np.linalg.svd(u)
    rep = solve2d.rel_error_2d(prob, s, [U, Vt.T])
    assert rep["rel_l2"] < 1e-13 and rep["rel_residual"] < 1e-12
    rep2 = solve2d.rel_error_2d(prob, s * (1 + 1e-3), [U, Vt.T])
    assert rep2["rel_l2"] == pytest.approx(1e-3, rel=1e-6)
