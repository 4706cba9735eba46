/*
 * Test infrastructure (oracle): cyclic Jacobi eigenvalue method for a dense
 * real symmetric matrix.  Used only by the CPU oracle to compute the
 * eigendecomposition of the symmetrised one-dimensional operator
 * T~ = D^{1/2} T D^{-1/2} (§2.2.1, Eq. reverse-similarity-transform), in place
 * of the LAPACK routines the paper uses at initialization (§3).
 *
 * Method: Jacobi rotations J(p,q,theta) chosen to annihilate A[p][q]
 * (Golub & Van Loan, "Matrix Computations", 4th ed., §8.5.2, symmetric 2x2
 * Schur decomposition), swept over all off-diagonal pairs in the round-robin
 * ("parallel") ordering of §8.5.5: each of the n'-1 rounds of a sweep applies
 * n'/2 disjoint rotations, which commute, so a round is one orthogonal
 * similarity A <- J^T A J, V <- V J.  Sweeps repeat until one sweep finds
 * every off-diagonal entry negligible (|a_pq| <= tol sqrt(|a_pp a_qq|), the
 * relative criterion of Demmel & Veselic, or |a_pq| <= tol max|a|).
 *
 * Plain C, no BLAS/LAPACK.  OpenMP only splits the independent row/column
 * updates of a round across threads.
 *
 * Precision: the rotations are accumulated in 80-bit extended precision
 * (C long double, 64-bit significand) and rounded to double at the end.  A
 * double-precision eigensolver determines an eigenvector only to about
 * eps ||T|| / gap; on a stretched grid with N ~ 10^2-10^3 that is 10^-12 to
 * 10^-11 for the smooth low modes that carry the solution of a Poisson
 * problem, which would make the oracle itself miss a 10^-12 comparison.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef long double real;

/* Round-robin schedule: m players (m even), round r in [0, m-1).  Player m-1
 * is fixed; the others rotate.  Fills pairs[2*i], pairs[2*i+1]. */
static void round_pairs(int m, int r, int *pairs)
{
    pairs[0] = m - 1;
    pairs[1] = r;
    for (int i = 1; i < m / 2; ++i) {
        pairs[2 * i] = (r + i) % (m - 1);
        pairs[2 * i + 1] = (r - i + (m - 1)) % (m - 1);
    }
}

/*
 * Ad: n*n row-major symmetric, overwritten (ends nearly diagonal).
 * Vd: n*n row-major output, columns are the eigenvectors.
 * w: n output eigenvalues (unsorted, w[i] belongs to column i of V).
 * Returns the number of sweeps used, or -1 if max_sweeps was reached.
 */
int oracle_jacobi(int n, double *Ad, double *Vd, double *w, double tol, int max_sweeps)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) Vd[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    if (n == 1) { w[0] = Ad[0]; return 0; }
    real *A = (real *)malloc(sizeof(real) * (size_t)n * n);
    real *V = (real *)malloc(sizeof(real) * (size_t)n * n);
    for (size_t e = 0; e < (size_t)n * n; ++e) { A[e] = Ad[e]; V[e] = Vd[e]; }
    int m = (n % 2) ? n + 1 : n;
    int *pairs = (int *)malloc(sizeof(int) * m);
    real *cs = (real *)malloc(sizeof(real) * m);   /* c, s per pair */
    int *pq = (int *)malloc(sizeof(int) * m);           /* active p, q per pair */
    /* A rotation is skipped (and a_pq treated as zero) when
     * |a_pq| <= tol * sqrt(|a_pp a_qq|) or |a_pq| <= tol * max|a_ij|; the
     * iteration stops after a sweep with no rotation.  The absolute floor
     * matters for (near-)zero eigenvalues, whose couplings cannot fall below
     * the rounding level of the whole matrix. */
    real amax = 0.0L;
    for (size_t e = 0; e < (size_t)n * n; ++e) amax = fmaxl(amax, fabsl(A[e]));
    const real rtol = (real)tol, atol = (real)tol * amax;
    int sweeps = -1;
    for (int sweep = 0; sweep <= max_sweeps; ++sweep) {
        int rotations = 0;
        for (int r = 0; r < m - 1; ++r) {
            round_pairs(m, r, pairs);
            int np = 0;
            for (int i = 0; i < m / 2; ++i) {
                int p = pairs[2 * i], q = pairs[2 * i + 1];
                if (p >= n || q >= n) continue;        /* dummy player for odd n */
                if (p > q) { int t = p; p = q; q = t; }
                real apq = A[(size_t)p * n + q];
                real app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                if (fabsl(apq) <= rtol * sqrtl(fabsl(app * aqq)) || fabsl(apq) <= atol) continue;
                real tau = (aqq - app) / (2.0L * apq);
                real t = (tau >= 0.0L) ? 1.0L / (tau + sqrtl(1.0L + tau * tau))
                                       : -1.0L / (-tau + sqrtl(1.0L + tau * tau));
                real c = 1.0L / sqrtl(1.0L + t * t);
                pq[2 * np] = p; pq[2 * np + 1] = q;
                cs[2 * np] = c; cs[2 * np + 1] = t * c;
                ++np;
            }
            rotations += np;
            if (np == 0) continue;
            /* rows: A <- J^T A  (row p <- c row_p - s row_q, row q <- s row_p + c row_q) */
            #pragma omp parallel for schedule(static)
            for (int k = 0; k < np; ++k) {
                int p = pq[2 * k], q = pq[2 * k + 1];
                real c = cs[2 * k], s = cs[2 * k + 1];
                real *rp = A + (size_t)p * n, *rq = A + (size_t)q * n;
                for (int j = 0; j < n; ++j) {
                    real x = rp[j], y = rq[j];
                    rp[j] = c * x - s * y;
                    rq[j] = s * x + c * y;
                }
            }
            /* columns: A <- A J and V <- V J (col p <- c col_p - s col_q, col q <- s col_p + c col_q) */
            #pragma omp parallel for schedule(static)
            for (int i = 0; i < n; ++i) {
                real *ra = A + (size_t)i * n, *rv = V + (size_t)i * n;
                for (int k = 0; k < np; ++k) {
                    int p = pq[2 * k], q = pq[2 * k + 1];
                    real c = cs[2 * k], s = cs[2 * k + 1];
                    real x = ra[p], y = ra[q];
                    ra[p] = c * x - s * y;
                    ra[q] = s * x + c * y;
                    x = rv[p]; y = rv[q];
                    rv[p] = c * x - s * y;
                    rv[q] = s * x + c * y;
                }
            }
        }
        if (rotations == 0) { sweeps = sweep; break; }
    }
    for (int i = 0; i < n; ++i) w[i] = (double)A[(size_t)i * n + i];
    for (size_t e = 0; e < (size_t)n * n; ++e) { Ad[e] = (double)A[e]; Vd[e] = (double)V[e]; }
    free(pairs); free(cs); free(pq); free(A); free(V);
    return sweeps;
}
