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
 * similarity A <- J^T A J, V <- V J.  Sweeps repeat until the off-diagonal
 * Frobenius norm is below tol * ||A||_F.
 *
 * Plain C, no BLAS/LAPACK.  OpenMP only splits the independent row/column
 * updates of a round across threads.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

static double off_norm2(int n, const double *A, double *fro2)
{
    double off = 0.0, all = 0.0;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            double v = A[(size_t)i * n + j];
            all += v * v;
            if (i != j) off += v * v;
        }
    *fro2 = all;
    return off;
}

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
 * A: n*n row-major symmetric, overwritten (ends nearly diagonal).
 * V: n*n row-major output, columns are the eigenvectors.
 * w: n output eigenvalues (unsorted, w[i] belongs to column i of V).
 * Returns the number of sweeps used, or -1 if max_sweeps was reached.
 */
int oracle_jacobi(int n, double *A, double *V, double *w, double tol, int max_sweeps)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    if (n == 1) { w[0] = A[0]; return 0; }
    int m = (n % 2) ? n + 1 : n;
    int *pairs = (int *)malloc(sizeof(int) * m);
    double *cs = (double *)malloc(sizeof(double) * m);   /* c, s per pair */
    int *pq = (int *)malloc(sizeof(int) * m);           /* active p, q per pair */
    int sweeps = -1;
    for (int sweep = 0; sweep <= max_sweeps; ++sweep) {
        double fro2;
        double off2 = off_norm2(n, A, &fro2);
        if (off2 <= tol * tol * fro2) { sweeps = sweep; break; }
        if (sweep == max_sweeps) break;
        for (int r = 0; r < m - 1; ++r) {
            round_pairs(m, r, pairs);
            int np = 0;
            for (int i = 0; i < m / 2; ++i) {
                int p = pairs[2 * i], q = pairs[2 * i + 1];
                if (p >= n || q >= n) continue;        /* dummy player for odd n */
                if (p > q) { int t = p; p = q; q = t; }
                double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0.0) ? 1.0 / (tau + sqrt(1.0 + tau * tau))
                                        : -1.0 / (-tau + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t);
                pq[2 * np] = p; pq[2 * np + 1] = q;
                cs[2 * np] = c; cs[2 * np + 1] = t * c;
                ++np;
            }
            if (np == 0) continue;
            /* rows: A <- J^T A  (row p <- c row_p - s row_q, row q <- s row_p + c row_q) */
            #pragma omp parallel for schedule(static)
            for (int k = 0; k < np; ++k) {
                int p = pq[2 * k], q = pq[2 * k + 1];
                double c = cs[2 * k], s = cs[2 * k + 1];
                double *rp = A + (size_t)p * n, *rq = A + (size_t)q * n;
                for (int j = 0; j < n; ++j) {
                    double x = rp[j], y = rq[j];
                    rp[j] = c * x - s * y;
                    rq[j] = s * x + c * y;
                }
            }
            /* columns: A <- A J and V <- V J (col p <- c col_p - s col_q, col q <- s col_p + c col_q) */
            #pragma omp parallel for schedule(static)
            for (int i = 0; i < n; ++i) {
                double *ra = A + (size_t)i * n, *rv = V + (size_t)i * n;
                for (int k = 0; k < np; ++k) {
                    int p = pq[2 * k], q = pq[2 * k + 1];
                    double c = cs[2 * k], s = cs[2 * k + 1];
                    double x = ra[p], y = ra[q];
                    ra[p] = c * x - s * y;
                    ra[q] = s * x + c * y;
                    x = rv[p]; y = rv[q];
                    rv[p] = c * x - s * y;
                    rv[q] = s * x + c * y;
                }
            }
        }
    }
    for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i];
    free(pairs); free(cs); free(pq);
    return sweeps;
}
