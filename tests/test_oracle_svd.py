"""Pins for the oracle's one-sided Jacobi SVD and the noise subspace (eq.4 and the E_n definition).

Independent anchors: LAPACK (numpy.linalg.svd / eigh, never called by the
oracle), the M = 2 closed form, an M = 4 case solved in exact rationals with
50-digit roots (sympy + mpmath), and structural facts (unitarity,
reconstruction, ordering).
"""
import numpy as np
import pytest

from conftest import crandn, projector, random_unitary


@pytest.mark.parametrize("M", [1, 2, 3, 7, 8, 16, 31, 60, 64])
def test_reconstruction_and_unitarity(orc, M):
    rng = np.random.default_rng(100 + M)
    A = crandn(rng, M, M)
    st, U, s, W, sw = orc.jacobi_svd(A)
    assert st == orc.OK
    assert np.linalg.norm(A - U @ W.conj().T) / np.linalg.norm(A) < 1e-12
    assert np.linalg.norm(U.conj().T @ U - np.eye(M), 2) < 1e-13 * M
    # columns of W are orthogonal with norms sigma
    G = W.conj().T @ W
    assert np.linalg.norm(G - np.diag(s ** 2)) < 1e-12 * s[0] ** 2
    assert np.all(np.diff(s) <= 0)
    ref = np.linalg.svd(A, compute_uv=False)
    assert np.max(np.abs(s - ref) / ref[0]) < 1e-12


def test_left_vectors_match_lapack_projectors(orc):
    rng = np.random.default_rng(11)
    M = 12
    A = crandn(rng, M, M)
    st, U, s, W, _ = orc.jacobi_svd(A)
    Ul, sl, Vh = np.linalg.svd(A)
    for k in (1, 2, 5):
        relgap = (sl[k - 1] - sl[k]) / sl[0]
        err = np.linalg.norm(projector(U[:, k:]) - projector(Ul[:, k:]), 2)
        assert err <= 1e-12 / relgap
        # and *left* (not right) vectors: the right-vector projector differs
        assert np.linalg.norm(projector(U[:, k:]) - projector(Vh.conj().T[:, k:]), 2) > 1e-3


def test_m2_closed_form(orc):
    rng = np.random.default_rng(12)
    for _ in range(5):
        A = crandn(rng, 2, 2)
        fro2 = np.sum(np.abs(A) ** 2)
        det = A[0, 0] * A[1, 1] - A[0, 1] * A[1, 0]
        disc = np.sqrt(fro2 ** 2 - 4 * abs(det) ** 2)
        s1, s2 = np.sqrt((fro2 + disc) / 2), np.sqrt((fro2 - disc) / 2)
        st, U, s, W, _ = orc.jacobi_svd(A)
        assert abs(s[0] - s1) < 1e-14 * s1 and abs(s[1] - s2) < 1e-13 * s1
        # noise projector for Ns = 1: (A A^H - s1^2 I) / (s2^2 - s1^2)
        Pn = (A @ A.conj().T - s1 ** 2 * np.eye(2)) / (s2 ** 2 - s1 ** 2)
        assert np.linalg.norm(projector(U[:, 1:]) - Pn) < 1e-13


def test_m4_exact_rational_projector(orc):
    """A = K^{-1} R with Gaussian-integer K, R.  C = A A^H in exact rationals, its characteristic
    polynomial's roots at 50 digits, noise projector as the sum of Frobenius covariants
    prod_{j != i} (C - l_j I) / (l_i - l_j) over the M - Ns smallest eigenvalues."""
    sympy = pytest.importorskip("sympy")
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    rng = np.random.default_rng(13)
    M, Ns = 4, 1
    G = rng.integers(-3, 4, (M, 3)) + 1j * rng.integers(-3, 4, (M, 3))
    R = G @ G.conj().T
    Hk = rng.integers(-2, 3, (M, M)) + 1j * rng.integers(-2, 3, (M, M))
    K = Hk @ Hk.conj().T + 3 * np.eye(M)
    toS = lambda Z: sympy.Matrix(M, M, lambda i, j: sympy.Integer(int(Z[i, j].real)) + sympy.I * int(Z[i, j].imag))
    Ks, Rs = toS(K), toS(R)
    As = Ks.inv() * Rs
    Cs = sympy.simplify(As * As.H)
    lam = sympy.Symbol("lam")
    poly = sympy.Poly(sympy.expand((Cs - lam * sympy.eye(M)).det()), lam)
    coeffs = [sympy.re(sympy.nsimplify(c)) for c in poly.all_coeffs()]
    roots = sorted([mpmath.re(r) for r in mpmath.polyroots([mpmath.mpf(sympy.Rational(c).p) / sympy.Rational(c).q
                                                              for c in coeffs], maxsteps=200, extraprec=200)])
    Cm = mpmath.matrix([[mpmath.mpc(str(sympy.N(sympy.re(Cs[i, j]), 60)), str(sympy.N(sympy.im(Cs[i, j]), 60)))
                         for j in range(M)] for i in range(M)])
    I = mpmath.eye(M)
    Pn = mpmath.zeros(M, M)
    for i in range(M - Ns):                   # the M - Ns smallest eigenvalues = noise subspace
        Pi = mpmath.eye(M)
        for j in range(M):
            if j != i:
                Pi = Pi * (Cm - roots[j] * I) / (roots[i] - roots[j])
        Pn += Pi
    Pn_np = np.array([[complex(Pn[i, j]) for j in range(M)] for i in range(M)])
    st, A = orc.solve(K, R)
    assert st == orc.OK
    st, U, s, W, _ = orc.jacobi_svd(A)
    assert st == orc.OK
    assert np.max(np.abs(projector(U[:, Ns:]) - Pn_np)) <= 1e-13
    # singular values squared are the roots
    assert np.max(np.abs(np.sort(s ** 2) - np.array([float(r) for r in roots]))) <= 1e-12 * s[0] ** 2


def test_sort_is_stable_descending(orc):
    s, perm = orc.sort_desc(np.array([1.0, 3.0, 2.0, 3.0, 1.0, 5.0]))
    assert list(perm) == [5, 1, 3, 2, 0, 4]
    assert list(s) == [5.0, 3.0, 3.0, 2.0, 1.0, 1.0]


def test_degenerate_inputs(orc):
    M = 6
    # zero matrix: U = I, sigma = 0, converged in one sweep
    st, U, s, W, sw = orc.jacobi_svd(np.zeros((M, M)))
    assert st == orc.OK and np.array_equal(U, np.eye(M)) and np.all(s == 0) and sw == 1
    # diagonal with repeated values: exact, ties keep index order
    D = np.diag([2.0, 5.0, 2.0, 1.0, 5.0, 0.0]).astype(np.complex128)
    st, U, s, W, sw = orc.jacobi_svd(D)
    assert list(s) == [5.0, 5.0, 2.0, 2.0, 1.0, 0.0]
    assert np.array_equal(np.abs(U), np.eye(M)[:, [1, 4, 0, 2, 3, 5]])
    # rank-deficient: U still unitary
    rng = np.random.default_rng(14)
    A = crandn(rng, M, 2) @ crandn(rng, 2, M)
    st, U, s, W, _ = orc.jacobi_svd(A)
    assert st == orc.OK
    assert np.linalg.norm(U.conj().T @ U - np.eye(M)) < 1e-13 * M
    assert np.all(s[2:] < 1e-13 * s[0])


def test_no_convergence_reported(orc):
    rng = np.random.default_rng(15)
    A = crandn(rng, 16, 16)
    st, *_ = orc.jacobi_svd(A, max_sweeps=1)
    assert st == orc.NO_CONV


def test_unitary_invariance(orc):
    """Left singular subspaces transform covariantly: SVD(Q A) has U' = Q U (as projectors)."""
    rng = np.random.default_rng(16)
    M = 10
    A = crandn(rng, M, M)
    Q = random_unitary(rng, M)
    _, U1, s1, _, _ = orc.jacobi_svd(A)
    _, U2, s2, _, _ = orc.jacobi_svd(Q @ A)
    assert np.max(np.abs(s1 - s2)) < 1e-12 * s1[0]
    assert np.linalg.norm(projector(U2[:, 3:]) - Q @ projector(U1[:, 3:]) @ Q.conj().T) < 1e-11
