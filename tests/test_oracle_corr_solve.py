"""Pins for the oracle's correlation (eq.2-3) and whitening solve (Sec. III-B, A = K^{-1} R).

Every check here is independent of the oracle's own arithmetic: numpy/LAPACK
routines the oracle never calls, exact rational arithmetic (sympy), closed-form
invariants (Hermitian, PSD, trace, rank) and backward-error bounds.
"""
import numpy as np
import pytest

from conftest import crandn, random_pd

EPS = 2.0 ** -53


def test_corr_matches_library_and_is_hermitian(orc):
    rng = np.random.default_rng(1)
    F, T, M = 5, 7, 6
    X = crandn(rng, F, T, M).astype(np.complex64)
    R = orc.corr(X)
    Xd = X.astype(np.complex128)
    ref = np.einsum("fti,ftj->fij", Xd, Xd.conj()) / T
    assert np.max(np.abs(R - ref)) <= 1e-14 * np.max(np.abs(ref))
    # exactly Hermitian: R_ij = conj(R_ji) to the bit
    assert np.array_equal(R, np.conj(np.swapaxes(R, 1, 2)))


def test_corr_not_transposed(orc):
    """x x^H, not x x^T and not x^* x^T: the (0,1) entry is x_0 conj(x_1)."""
    X = np.zeros((1, 1, 2), np.complex64)
    X[0, 0, 0] = 1 + 2j
    X[0, 0, 1] = 3 - 1j
    R = orc.corr(X, scale=1.0)
    assert R[0, 0, 1] == (1 + 2j) * np.conj(3 - 1j)
    assert R[0, 1, 0] == (3 - 1j) * np.conj(1 + 2j)
    assert R[0, 0, 0] == 5.0 and R[0, 1, 1] == 10.0


def test_corr_psd_trace_rank(orc):
    rng = np.random.default_rng(2)
    F, T, M = 3, 3, 8                # T < M: rank <= T
    X = crandn(rng, F, T, M).astype(np.complex64)
    R = orc.corr(X)
    Xd = X.astype(np.complex128)
    for f in range(F):
        ev = np.linalg.eigvalsh(R[f])
        nrm = np.abs(ev).max()
        assert ev.min() >= -1e-14 * nrm                          # PSD
        assert np.sum(ev > 1e-12 * nrm) <= T                     # rank <= T
        tr = np.sum(np.abs(Xd[f]) ** 2) / T
        assert abs(np.trace(R[f]).real - tr) <= 1e-14 * tr       # trace = (1/T) sum |x_t|^2
        assert abs(np.trace(R[f]).imag) == 0.0


def test_corr_strided_input(orc):
    rng = np.random.default_rng(3)
    F, T, M = 4, 6, 5
    big = crandn(rng, F, T + 2, M + 3).astype(np.complex64)
    view = big[:, 1:T + 1, :M]                 # strideT = M + 3, strideF = (T + 2)(M + 3)
    assert view.strides[2] == 8 and view.strides[1] != M * 8
    R1 = orc.corr(view)
    R2 = orc.corr(np.ascontiguousarray(view))
    assert np.array_equal(R1, R2)


def test_solve_backward_error(orc):
    rng = np.random.default_rng(4)
    for M, cond in [(2, 3.0), (8, 1e3), (33, 1e6), (60, 1e8)]:
        K = random_pd(rng, M, cond)
        Rm = crandn(rng, M, M)
        R = Rm @ Rm.conj().T
        st, A = orc.solve(K, R)
        assert st == orc.OK
        be = np.linalg.norm(K @ A - R, 2) / (np.linalg.norm(K, 2) * np.linalg.norm(A, 2))
        assert be <= 10 * M * EPS, (M, be)
        # forward error against LAPACK's solve (independent routine), within cond * eps
        ref = np.linalg.solve(K, R)
        assert np.linalg.norm(A - ref) / np.linalg.norm(ref) <= 50 * M * cond * EPS


def test_solve_identity_is_exact(orc):
    rng = np.random.default_rng(5)
    M = 9
    R = crandn(rng, M, M)
    st, A = orc.solve(np.eye(M), R)
    assert st == orc.OK and np.array_equal(A, R)


def test_solve_exact_gaussian_integers(orc):
    """K, R with Gaussian-integer entries; K^{-1} R computed exactly in rationals."""
    sympy = pytest.importorskip("sympy")
    rng = np.random.default_rng(6)
    M = 4
    G = rng.integers(-3, 4, (M, M)) + 1j * rng.integers(-3, 4, (M, M))
    K = G @ G.conj().T + 5 * np.eye(M)
    Rr = rng.integers(-4, 5, (M, M)) + 1j * rng.integers(-4, 5, (M, M))
    Ks = sympy.Matrix(M, M, lambda i, j: sympy.Integer(int(K[i, j].real)) + sympy.I * int(K[i, j].imag))
    Rs = sympy.Matrix(M, M, lambda i, j: sympy.Integer(int(Rr[i, j].real)) + sympy.I * int(Rr[i, j].imag))
    As = Ks.LUsolve(Rs)
    exact = np.array([[complex(sympy.N(As[i, j], 30)) for j in range(M)] for i in range(M)])
    st, A = orc.solve(K, Rr)
    assert st == orc.OK
    assert np.max(np.abs(A - exact)) <= 1e-13 * np.max(np.abs(exact))


def test_cholesky_factor(orc):
    rng = np.random.default_rng(7)
    M = 12
    K = random_pd(rng, M, 100.0)
    st, L = orc.cholesky(K)
    assert st == orc.OK
    assert np.allclose(np.triu(L, 1), 0)
    assert np.all(np.diag(L).real > 0) and np.all(np.diag(L).imag == 0)
    assert np.linalg.norm(L @ L.conj().T - K) <= 10 * M * EPS * np.linalg.norm(K)
    ref = np.linalg.cholesky(K)                     # LAPACK, independent
    assert np.max(np.abs(L - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_not_pd_detection(orc):
    rng = np.random.default_rng(8)
    M = 10
    # an eigenvalue below zero
    K = random_pd(rng, M, 10.0)
    w, V = np.linalg.eigh(K)
    w[3] = -0.5
    st, _ = orc.solve((V * w) @ V.conj().T, np.eye(M))
    assert st == orc.NOT_PD
    # rank-deficient sample correlation: fewer noise frames than channels
    Xn = crandn(rng, 1, M - 3, M).astype(np.complex64)
    Kd = orc.corr(Xn)[0]
    st, A = orc.solve(Kd, np.eye(M))
    assert st == orc.NOT_PD and np.all(A == 0)
    # zero and NaN matrices
    assert orc.solve(np.zeros((M, M)), np.eye(M))[0] == orc.NOT_PD
    Kn = np.eye(M, dtype=np.complex128)
    Kn[2, 2] = np.nan
    assert orc.solve(Kn, np.eye(M))[0] == orc.NOT_PD


def test_sliding_corr_definition_and_rank2_recurrence(orc):
    """eq.3's window: the direct sum over the T frames ending at f (einsum), and, on Gaussian-integer
    frames where FP64 is exact, R(f + 1) - R(f) = (x_{f+1} x_{f+1}^H - x_{f-T+1} x_{f-T+1}^H) / T
    exactly -- the rank-2 update a streaming implementation applies per frame."""
    rng = np.random.default_rng(41)
    F, N, M, T = 3, 20, 5, 8
    X = (rng.integers(-3, 4, (F, N, M)) + 1j * rng.integers(-3, 4, (F, N, M))).astype(np.complex64)
    x = X.astype(np.complex128)
    for f in range(T - 1, N):
        R = orc.sliding_corr(X, T, f)
        W = x[:, f - T + 1:f + 1]
        assert np.allclose(R, np.einsum("fti,ftj->fij", W, W.conj()) / T, rtol=0, atol=1e-13)
    for f in range(T - 1, N - 1):
        d = (orc.sliding_corr(X, T, f + 1) - orc.sliding_corr(X, T, f)) * T
        new, old = x[:, f + 1], x[:, f - T + 1]
        want = np.einsum("fi,fj->fij", new, new.conj()) - np.einsum("fi,fj->fij", old, old.conj())
        assert np.array_equal(np.round(d, 9), want)
    with pytest.raises(ValueError):
        orc.sliding_corr(X, T, T - 2)
