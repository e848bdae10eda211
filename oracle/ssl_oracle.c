/*
 * ssl_oracle.c -- plain FP64 CPU oracle for the GSVD-MUSIC localization path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code, no
 * header and no constants with the HIP library: it is an independent
 * restatement of the method written for a reader who checks it against the
 * paper (arXiv 2504.03373) by eye.  Everything is double precision, explicit
 * loops, no BLAS; bins are independent so an OpenMP loop over bins is the only
 * parallelism.
 *
 * Steps and the passages they follow:
 *   orc_stft         eq.1: the frequency-domain input X(w, f) of every channel,
 *                    X_m(w, f) = sum_n win[n] x_m[f*hop + n] e^{-2 pi i w n / N}
 *                    (the direct DFT sum; orc_hann gives the default window)
 *   orc_corr         eq.2 and eq.3 (AddCorrelation + NormalizeCorrelation):
 *                    R = scale * sum_t x_t x_t^H
 *   orc_chol_solve   Sec. III-B: A = K^{-1} R.  K = L L^H (Cholesky, also the
 *                    positive-definiteness test), then L Y = R and L^H A = Y.
 *   orc_jacobi_svd   eq.4 / Sec. III-B category 1: one-sided (Hestenes) Jacobi
 *                    on B = A^H with cyclic-by-rows pair order; U = accumulated
 *                    rotations, so A = U Sigma W^H with W = B J.
 *   orc_sort_desc    Sec. III-B: singular values in descending order and the
 *                    singular vectors reordered with them (ties: lower index first).
 *   orc_gsvd         eq.4 + the definition of E_n after eq.4: E_n = columns
 *                    Ns..M-1 of the sorted left singular vectors of K^{-1} R.
 *   orc_inv_sqrt,    GEVD-MUSIC, the generalized-eigenvalue alternative (Sec. II): the noise
 *   orc_gevd         vectors are the generalized eigenvectors R e = lambda K e of the M - Ns
 *                    smallest lambda, computed as e = K^{-1/2} y from the eigenvectors y of
 *                    K^{-1/2} R K^{-1/2} (K^{-1/2} the Hermitian inverse square root of K, from
 *                    K = U diag(s) U^H by the Jacobi SVD of K, which for a Hermitian positive
 *                    definite K is its eigen-decomposition); the e are K-orthonormal.
 *   orc_spectrum     eq.5 (CalcAveragePower) and eq.6 (sum over bins).
 *   orc_peaks        Sec. III-A, last paragraph: the preset number of peaks of
 *                    P-bar over the direction grid.
 *
 * Readings where the paper is silent or garbled (listed with reasons in the
 * design notes): eq.2 is the outer product x x^H; the eq.5 denominator is
 * sum_i |H^H e_i|^p with p = 2 by default (p = 1 literal form available);
 * P = |H|^2 / max(den, DBL_MIN); a bin whose K is not positive definite or
 * whose Jacobi does not converge contributes 0 to P-bar; a peak is a grid point
 * that is >= all 8 neighbours (azimuth circular, elevation clamped) where an
 * equal neighbour with a lower flat index wins, ranked by value then index.
 *
 * Layouts (all row-major, complex numbers interleaved re, im):
 *   X  [F][T][M] complex64 with element strides strideF, strideT (M contiguous)
 *   R, K, A  [F][M][M] complex128, element (i, j) at i*M + j
 *   En [F][M-Ns][M] complex128, column c of bin f at (f*(M-Ns) + c)*M
 *   sigma [F][M] descending;  H [F][D][M] complex64;  P [F][D];  Pbar [D]
 */
#include <complex.h>
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static const double kPi = 3.14159265358979323846;

enum { ORC_OK = 0, ORC_NOT_PD = 1, ORC_NO_CONV = 2, ORC_NONFINITE = 3 };

/* ------------------------------------------------------------------------ */
/* eq.1: short-time Fourier transform                                         */
/* ------------------------------------------------------------------------ */
/* Periodic Hann window of length N (the reading taken for the unspecified window):
 * win[n] = 1/2 - 1/2 cos(2 pi n / N). */
void orc_hann(int N, double *win)
{
    for (int n = 0; n < N; ++n) win[n] = 0.5 - 0.5 * cos(2.0 * kPi * (double)n / (double)N);
}

/* pcm [n_samples][M] float (channel-interleaved); frame f covers samples f*hop .. f*hop + N - 1.
 * X [N/2 + 1][T][M] complex128: X[w][f][m] = sum_{n<N} win[n] pcm[f*hop + n][m] e^{-2 pi i w n/N},
 * summed over n in ascending order; the phase w*n/N is reduced modulo 1 exactly in integers and
 * e^{-2 pi i k / N} taken from a table of the N values (OpenMP over bins). */
void orc_stft(const float *pcm, int M, int N, int hop, const double *win, int T, cplx *X)
{
    const int F = N / 2 + 1;
    cplx *tw = malloc(sizeof(cplx) * (size_t)N);
    for (int k = 0; k < N; ++k) {
        const double ph = -2.0 * kPi * (double)k / (double)N;
        tw[k] = cos(ph) + I * sin(ph);
    }
#pragma omp parallel for schedule(dynamic)
    for (int w = 0; w < F; ++w)
        for (int f = 0; f < T; ++f)
            for (int m = 0; m < M; ++m) {
                cplx acc = 0.0;
                for (int n = 0; n < N; ++n) {
                    const double x = win[n] * (double)pcm[((size_t)f * hop + n) * M + m];
                    acc += x * tw[((long long)w * n) % N];
                }
                X[((size_t)w * T + f) * M + m] = acc;
            }
    free(tw);
}

/* ------------------------------------------------------------------------ */
/* eq.2 + eq.3                                                               */
/* ------------------------------------------------------------------------ */
void orc_corr(const float complex *X, int F, int T, int M, int64_t strideF, int64_t strideT,
              double scale, cplx *R)
{
    for (int f = 0; f < F; ++f) {
        cplx *Rf = R + (size_t)f * M * M;
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                cplx s = 0;
                for (int t = 0; t < T; ++t) {
                    const float complex *x = X + (size_t)f * strideF + (size_t)t * strideT;
                    cplx xi = (cplx)x[i];
                    cplx xj = (cplx)x[j];
                    s += xi * conj(xj);                    /* (x x^H)_{ij} */
                }
                Rf[i * M + j] = scale * s;
            }
    }
}

/* ------------------------------------------------------------------------ */
/* positive-definiteness rule shared by the whole path (a reading): a pivot  */
/* d_k of the Cholesky factorisation is rejected when it is not finite or    */
/* d_k <= 2^-40 * max_i Re K_ii.                                              */
/* ------------------------------------------------------------------------ */
static const double PD_REL = 9.094947017729282e-13;   /* 2^-40 */

/* K = L L^H, L lower triangular with real positive diagonal; returns ORC_OK or ORC_NOT_PD */
int orc_cholesky(const cplx *K, int M, cplx *L)
{
    double dmax = 0.0;
    for (int i = 0; i < M; ++i)
        if (creal(K[i * M + i]) > dmax) dmax = creal(K[i * M + i]);
    if (!(dmax > 0.0) || !isfinite(dmax)) return ORC_NOT_PD;
    memset(L, 0, sizeof(cplx) * M * M);
    for (int j = 0; j < M; ++j) {
        double d = creal(K[j * M + j]);
        for (int k = 0; k < j; ++k) d -= creal(L[j * M + k] * conj(L[j * M + k]));
        if (!isfinite(d) || d <= PD_REL * dmax) return ORC_NOT_PD;
        double ljj = sqrt(d);
        L[j * M + j] = ljj;
        for (int i = j + 1; i < M; ++i) {
            cplx s = K[i * M + j];
            for (int k = 0; k < j; ++k) s -= L[i * M + k] * conj(L[j * M + k]);
            L[i * M + j] = s / ljj;
        }
    }
    return ORC_OK;
}

/* A = K^{-1} R for one bin: Cholesky, then forward (L Y = R) and back (L^H A = Y) substitution */
int orc_chol_solve(const cplx *K, const cplx *R, int M, cplx *A)
{
    cplx *L = malloc(sizeof(cplx) * M * M);
    int st = orc_cholesky(K, M, L);
    if (st != ORC_OK) {
        memset(A, 0, sizeof(cplx) * M * M);
        free(L);
        return st;
    }
    for (int c = 0; c < M; ++c) {                         /* each right-hand side column */
        for (int i = 0; i < M; ++i) {                     /* forward: L y = r */
            cplx s = R[i * M + c];
            for (int k = 0; k < i; ++k) s -= L[i * M + k] * A[k * M + c];
            A[i * M + c] = s / L[i * M + i];
        }
        for (int i = M - 1; i >= 0; --i) {                /* back: L^H a = y, (L^H)_{ik} = conj(L_{ki}) */
            cplx s = A[i * M + c];
            for (int k = i + 1; k < M; ++k) s -= conj(L[k * M + i]) * A[k * M + c];
            A[i * M + c] = s / L[i * M + i];
        }
    }
    free(L);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* one-sided Jacobi SVD (Hestenes) on B = A^H                                */
/* ------------------------------------------------------------------------ */
/* Columns of B and J are stored contiguously: Bc[j*M + r] = B(r, j). */
int orc_jacobi_svd(const cplx *A, int M, double tol, int max_sweeps,
                   cplx *U, cplx *W, double *sigma, int *sweeps_out)
{
    cplx *B = malloc(sizeof(cplx) * M * M);
    cplx *J = malloc(sizeof(cplx) * M * M);
    for (int j = 0; j < M; ++j)
        for (int r = 0; r < M; ++r) {
            B[j * M + r] = conj(A[j * M + r]);             /* B(r, j) = conj(A(j, r)) */
            J[j * M + r] = (r == j) ? 1.0 : 0.0;
        }
    int converged = 0, sweep = 0;
    for (sweep = 0; sweep < max_sweeps && !converged; ++sweep) {
        int rotated = 0;
        for (int i = 0; i < M - 1; ++i)
            for (int j = i + 1; j < M; ++j) {
                cplx *bi = B + (size_t)i * M, *bj = B + (size_t)j * M;
                cplx *ji = J + (size_t)i * M, *jj = J + (size_t)j * M;
                double alpha = 0.0, beta = 0.0;
                cplx gamma = 0;
                for (int r = 0; r < M; ++r) {
                    alpha += creal(bi[r] * conj(bi[r]));
                    beta += creal(bj[r] * conj(bj[r]));
                    gamma += conj(bi[r]) * bj[r];          /* b_i^H b_j */
                }
                double g = cabs(gamma);
                if (!(g > tol * sqrt(alpha * beta))) continue;
                rotated = 1;
                /* make the pair's inner product real: scale column j by e^{-i arg gamma} */
                cplx ph = conj(gamma) / g;
                for (int r = 0; r < M; ++r) { bj[r] *= ph; jj[r] *= ph; }
                /* real symmetric 2x2 Jacobi on [[alpha, g], [g, beta]] */
                double zeta = (beta - alpha) / (2.0 * g);
                double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = c * t;
                for (int r = 0; r < M; ++r) {
                    cplx x = bi[r], y = bj[r];
                    bi[r] = c * x - s * y;
                    bj[r] = s * x + c * y;
                    x = ji[r]; y = jj[r];
                    ji[r] = c * x - s * y;
                    jj[r] = s * x + c * y;
                }
            }
        if (!rotated) converged = 1;
    }
    for (int j = 0; j < M; ++j) {
        double n = 0.0;
        for (int r = 0; r < M; ++r) n += creal(B[j * M + r] * conj(B[j * M + r]));
        sigma[j] = sqrt(n);
    }
    /* U(r, j) = J(r, j);  W(r, j) = B(r, j); both returned row-major */
    for (int r = 0; r < M; ++r)
        for (int j = 0; j < M; ++j) {
            U[r * M + j] = J[j * M + r];
            if (W) W[r * M + j] = B[j * M + r];
        }
    free(B);
    free(J);
    if (sweeps_out) *sweeps_out = sweep;
    return converged ? ORC_OK : ORC_NO_CONV;
}

/* Sort sigma descending (stable: equal values keep the lower original index first) and
 * permute the columns of U (and W if given) accordingly.  perm_out[k] = original column. */
void orc_sort_desc(int M, double *sigma, cplx *U, cplx *W, int *perm_out)
{
    int *perm = malloc(sizeof(int) * M);
    for (int k = 0; k < M; ++k) perm[k] = k;
    for (int k = 1; k < M; ++k) {                          /* insertion sort: stable */
        int p = perm[k];
        int q = k - 1;
        while (q >= 0 && sigma[perm[q]] < sigma[p]) { perm[q + 1] = perm[q]; --q; }
        perm[q + 1] = p;
    }
    double *s2 = malloc(sizeof(double) * M);
    cplx *tmp = malloc(sizeof(cplx) * M * M);
    for (int k = 0; k < M; ++k) s2[k] = sigma[perm[k]];
    memcpy(sigma, s2, sizeof(double) * M);
    for (int pass = 0; pass < 2; ++pass) {
        cplx *X = pass == 0 ? U : W;
        if (!X) continue;
        for (int r = 0; r < M; ++r)
            for (int k = 0; k < M; ++k) tmp[r * M + k] = X[r * M + perm[k]];
        memcpy(X, tmp, sizeof(cplx) * M * M);
    }
    if (perm_out) memcpy(perm_out, perm, sizeof(int) * M);
    free(perm);
    free(s2);
    free(tmp);
}

static int all_finite(const cplx *Z, size_t n)
{
    for (size_t k = 0; k < n; ++k)
        if (!isfinite(creal(Z[k])) || !isfinite(cimag(Z[k]))) return 0;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* eq.4: per-bin GSVD and the noise subspace                                 */
/* ------------------------------------------------------------------------ */
void orc_gsvd(const cplx *K, const cplx *R, int F, int M, int Ns, double tol, int max_sweeps,
              int nthreads, cplx *En, double *sigma, int *status, int *sweeps)
{
    const int Nn = M - Ns;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int f = 0; f < F; ++f) {
        const cplx *Kf = K + (size_t)f * M * M;
        const cplx *Rf = R + (size_t)f * M * M;
        cplx *A = malloc(sizeof(cplx) * M * M);
        cplx *U = malloc(sizeof(cplx) * M * M);
        double *sg = malloc(sizeof(double) * M);
        int st, sw = 0;
        if (!all_finite(Rf, (size_t)M * M) || !all_finite(Kf, (size_t)M * M)) {
            st = ORC_NONFINITE;
        } else {
            st = orc_chol_solve(Kf, Rf, M, A);
            if (st == ORC_OK) {
                st = orc_jacobi_svd(A, M, tol, max_sweeps, U, NULL, sg, &sw);
                if (st == ORC_OK) orc_sort_desc(M, sg, U, NULL, NULL);
            }
        }
        cplx *Enf = En + (size_t)f * Nn * M;
        for (int c = 0; c < Nn; ++c)
            for (int r = 0; r < M; ++r)
                Enf[c * M + r] = (st == ORC_OK) ? U[r * M + (Ns + c)] : 0.0;
        if (sigma)
            for (int k = 0; k < M; ++k) sigma[(size_t)f * M + k] = (st == ORC_OK) ? sg[k] : 0.0;
        status[f] = st;
        if (sweeps) sweeps[f] = sw;
        free(A);
        free(U);
        free(sg);
    }
}

/* W = K^{-1/2} = U diag(s^{-1/2}) U^H for Hermitian positive definite K (the Cholesky test decides
 * positive definiteness, as for the GSVD path).  Returns ORC_OK, ORC_NOT_PD or ORC_NO_CONV. */
int orc_inv_sqrt(const cplx *K, int M, double tol, int max_sweeps, cplx *W)
{
    cplx *L = malloc(sizeof(cplx) * M * M);
    int st = orc_cholesky(K, M, L);
    free(L);
    if (st != ORC_OK) return st;
    cplx *U = malloc(sizeof(cplx) * M * M);
    double *sg = malloc(sizeof(double) * M);
    int sw = 0;
    st = orc_jacobi_svd(K, M, tol, max_sweeps, U, NULL, sg, &sw);
    if (st == ORC_OK)
        for (int i = 0; i < M; ++i)
            for (int j = 0; j < M; ++j) {
                cplx acc = 0.0;
                for (int k = 0; k < M; ++k)
                    acc += U[i * M + k] * (1.0 / sqrt(sg[k])) * conj(U[j * M + k]);
                W[i * M + j] = acc;
            }
    free(U);
    free(sg);
    return st;
}

/* GEVD-MUSIC noise vectors per bin: C = W R W (W = K^{-1/2}), its singular vectors Y (C is
 * Hermitian positive semi-definite: its eigenvectors) sorted descending, E_n = W Y[:, Ns..M-1]:
 * the generalized eigenvectors of (R, K) of the M - Ns smallest generalized eigenvalues. */
void orc_gevd(const cplx *K, const cplx *R, int F, int M, int Ns, double tol, int max_sweeps,
              int nthreads, cplx *En, double *sigma, int *status)
{
    const int Nn = M - Ns;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (int f = 0; f < F; ++f) {
        const cplx *Kf = K + (size_t)f * M * M;
        const cplx *Rf = R + (size_t)f * M * M;
        cplx *W = malloc(sizeof(cplx) * M * M);
        cplx *T = malloc(sizeof(cplx) * M * M);
        cplx *C = malloc(sizeof(cplx) * M * M);
        cplx *U = malloc(sizeof(cplx) * M * M);
        double *sg = malloc(sizeof(double) * M);
        int st, sw = 0;
        if (!all_finite(Rf, (size_t)M * M) || !all_finite(Kf, (size_t)M * M)) {
            st = ORC_NONFINITE;
        } else {
            st = orc_inv_sqrt(Kf, M, tol, max_sweeps, W);
            if (st == ORC_OK) {
                for (int i = 0; i < M; ++i)               /* T = W R */
                    for (int j = 0; j < M; ++j) {
                        cplx acc = 0.0;
                        for (int k = 0; k < M; ++k) acc += W[i * M + k] * Rf[k * M + j];
                        T[i * M + j] = acc;
                    }
                for (int i = 0; i < M; ++i)               /* C = T W */
                    for (int j = 0; j < M; ++j) {
                        cplx acc = 0.0;
                        for (int k = 0; k < M; ++k) acc += T[i * M + k] * W[k * M + j];
                        C[i * M + j] = acc;
                    }
                st = orc_jacobi_svd(C, M, tol, max_sweeps, U, NULL, sg, &sw);
                if (st == ORC_OK) orc_sort_desc(M, sg, U, NULL, NULL);
            }
        }
        cplx *Enf = En + (size_t)f * Nn * M;
        for (int c = 0; c < Nn; ++c)
            for (int r = 0; r < M; ++r) {
                cplx acc = 0.0;
                if (st == ORC_OK)
                    for (int k = 0; k < M; ++k) acc += W[r * M + k] * U[k * M + (Ns + c)];
                Enf[c * M + r] = acc;
            }
        if (sigma)
            for (int k = 0; k < M; ++k) sigma[(size_t)f * M + k] = (st == ORC_OK) ? sg[k] : 0.0;
        status[f] = st;
        free(W);
        free(T);
        free(C);
        free(U);
        free(sg);
    }
}

/* ------------------------------------------------------------------------ */
/* eq.5 and eq.6                                                             */
/* ------------------------------------------------------------------------ */
void orc_spectrum(const float complex *H, const cplx *En, const int *status, int F, int D, int M,
                  int Ns, int p, int nthreads, double *P, double *Pbar)
{
    const int Nn = M - Ns;
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
    for (int f = 0; f < F; ++f) {
        const cplx *Enf = En + (size_t)f * Nn * M;
        for (int d = 0; d < D; ++d) {
            const float complex *h = H + ((size_t)f * D + d) * M;
            double val = 0.0;
            if (!status || status[f] == ORC_OK) {
                double num = 0.0;                          /* |H^H H| */
                for (int m = 0; m < M; ++m) num += creal((cplx)h[m] * conj((cplx)h[m]));
                double den = 0.0;
                for (int c = 0; c < Nn; ++c) {             /* sum_i |H^H e_i|^p */
                    cplx g = 0;
                    for (int m = 0; m < M; ++m) g += conj((cplx)h[m]) * Enf[c * M + m];
                    den += (p == 1) ? cabs(g) : creal(g * conj(g));
                }
                val = num / (den > DBL_MIN ? den : DBL_MIN);
            }
            if (P) P[(size_t)f * D + d] = val;
        }
    }
    for (int d = 0; d < D; ++d) {                          /* eq.6, ascending bin order */
        double s = 0.0;
        for (int f = 0; f < F; ++f) s += P[(size_t)f * D + d];
        Pbar[d] = s;
    }
}

/* ------------------------------------------------------------------------ */
/* peak search on the n_el x n_az grid, d = el * n_az + az                    */
/* ------------------------------------------------------------------------ */
/* a beats b: larger value, or equal value and lower flat index */
static int beats(const double *v, int a, int b)
{
    return v[a] > v[b] || (v[a] == v[b] && a < b);
}

int orc_is_local_max(const double *Pbar, int n_el, int n_az, int d)
{
    if (!isfinite(Pbar[d])) return 0;
    int el = d / n_az, az = d % n_az;
    for (int de = -1; de <= 1; ++de) {
        int e = el + de;
        if (e < 0 || e >= n_el) continue;                   /* elevation is clamped */
        for (int da = -1; da <= 1; ++da) {
            if (de == 0 && da == 0) continue;
            int a = ((az + da) % n_az + n_az) % n_az;       /* azimuth is circular */
            int nb = e * n_az + a;
            if (nb == d) continue;
            if (!isfinite(Pbar[nb])) continue;
            if (!beats(Pbar, d, nb)) return 0;
        }
    }
    return 1;
}

/* returns the number of peaks found; peaks[k] = -1 and vals[k] = 0 beyond it */
int orc_peaks(const double *Pbar, int n_el, int n_az, int Ns, int *peaks, double *vals)
{
    const int D = n_el * n_az;
    int *cand = malloc(sizeof(int) * (D > 0 ? D : 1));
    int nc = 0;
    for (int d = 0; d < D; ++d)
        if (orc_is_local_max(Pbar, n_el, n_az, d)) cand[nc++] = d;
    int found = 0;
    for (int k = 0; k < Ns; ++k) {
        int best = -1, bi = -1;
        for (int q = 0; q < nc; ++q) {
            if (cand[q] < 0) continue;
            if (best < 0 || beats(Pbar, cand[q], best)) { best = cand[q]; bi = q; }
        }
        if (best >= 0) {
            cand[bi] = -1;
            peaks[k] = best;
            vals[k] = Pbar[best];
            ++found;
        } else {
            peaks[k] = -1;
            vals[k] = 0.0;
        }
    }
    free(cand);
    return found;
}

/* ------------------------------------------------------------------------ */
/* one block end to end: R from X, A = K^{-1}R, SVD, E_n, spectrum, peaks     */
/* ------------------------------------------------------------------------ */
void orc_localize_m(const float complex *X, int F, int T, int M, int64_t strideF,
                    int64_t strideT, const cplx *K, const float complex *H, int n_az, int n_el,
                    int Ns, int p, double tol, int max_sweeps, int nthreads, int gevd,
                    int *peaks, double *peak_val, double *Pbar, int *status, double *P_out);

void orc_localize(const float complex *X, int F, int T, int M, int64_t strideF, int64_t strideT,
                  const cplx *K, const float complex *H, int n_az, int n_el, int Ns, int p,
                  double tol, int max_sweeps, int nthreads,
                  int *peaks, double *peak_val, double *Pbar, int *status, double *P_out)
{
    orc_localize_m(X, F, T, M, strideF, strideT, K, H, n_az, n_el, Ns, p, tol, max_sweeps,
                   nthreads, 0, peaks, peak_val, Pbar, status, P_out);
}

/* as orc_localize; gevd != 0 takes the noise subspace from orc_gevd instead of orc_gsvd */
void orc_localize_m(const float complex *X, int F, int T, int M, int64_t strideF,
                    int64_t strideT, const cplx *K, const float complex *H, int n_az, int n_el,
                    int Ns, int p, double tol, int max_sweeps, int nthreads, int gevd,
                    int *peaks, double *peak_val, double *Pbar, int *status, double *P_out)
{
    const int D = n_az * n_el;
    cplx *R = malloc(sizeof(cplx) * (size_t)F * M * M);
    cplx *En = malloc(sizeof(cplx) * (size_t)F * (M - Ns) * M);
    double *P = P_out ? P_out : malloc(sizeof(double) * (size_t)F * D);
    orc_corr(X, F, T, M, strideF, strideT, 1.0 / T, R);
    if (gevd)
        orc_gevd(K, R, F, M, Ns, tol, max_sweeps, nthreads, En, NULL, status);
    else
        orc_gsvd(K, R, F, M, Ns, tol, max_sweeps, nthreads, En, NULL, status, NULL);
    orc_spectrum(H, En, status, F, D, M, Ns, p, nthreads, P, Pbar);
    orc_peaks(Pbar, n_el, n_az, Ns, peaks, peak_val);
    if (!P_out) free(P);
    free(En);
    free(R);
}
