// 1-D operators and their eigendecomposition (host side of a plan).
//
// §2.2.1, Eq. poisson-fd2 / tridiagonal-coefficients: a_i = 1/(dx_i dx_{i-1/2}),
// c_i = 1/(dx_i dx_{i+1/2}), b_i = -(a_i + c_i), dx_i the control volume of
// unknown i and dx_{i+1/2} the distance to the next unknown.  Boundary rows
// (the paper leaves them unspecified) come from ghost values: a Neumann wall
// drops the wall coupling and keeps only the interior flux; a Dirichlet wall
// at a cell-centred direction mirrors the ghost (u_0 = -u_1 at distance dx_1),
// i.e. b_1 = -c_1 - 2/dx_1^2; face-located unknowns between Dirichlet walls
// are the interior faces with zero wall values; periodic directions close
// with the cyclic corners.  D T is symmetric (dx_i c_i = dx_{i+1} a_{i+1}), so
// T~ = D^{1/2} T D^{-1/2} is symmetric (Eq. reverse-similarity-transform).
#include "host_ops.h"

#include <algorithm>
#include <cmath>
#include <limits>
#include <numeric>

namespace tpt {

typedef long double real;

static bool nearly_equal(double x, double y, double tol) { return std::fabs(x - y) <= tol * std::fabs(y); }

std::string build_op1d(int ncells, const double* faces, int bc_lo, int bc_hi, int loc, Op1D& op) {
    if (ncells < 2) return "need at least 2 cells per direction";
    if (!faces) return "faces pointer is NULL";
    for (int i = 0; i < ncells; ++i)
        if (!(faces[i + 1] > faces[i])) return "faces must be strictly increasing";
    const bool per = bc_lo == BC_P;
    if (per != (bc_hi == BC_P)) return "periodic boundaries must be set on both sides";
    auto okbc = [](int b) { return b == BC_P || b == BC_N || b == BC_D; };
    if (!okbc(bc_lo) || !okbc(bc_hi)) return "unknown boundary condition";
    if (loc != LOC_C && loc != LOC_F) return "unknown location";
    std::vector<double> w(ncells);
    for (int i = 0; i < ncells; ++i) w[i] = faces[i + 1] - faces[i];
    op = Op1D();
    op.periodic = per;
    op.bc_lo = bc_lo;
    op.bc_hi = bc_hi;
    op.loc = loc;
    // dist_lo[i] = distance to unknown i-1, dist_hi[i] = distance to unknown i+1
    std::vector<double> vol, dlo, dhi;
    if (loc == LOC_C) {
        const int n = ncells;
        vol = w;
        dlo.resize(n);
        dhi.resize(n);
        for (int i = 0; i + 1 < n; ++i) {
            double d = 0.5 * (w[i] + w[i + 1]);  // centre-to-centre
            dhi[i] = d;
            dlo[i + 1] = d;
        }
        if (per) {
            dlo[0] = dhi[n - 1] = 0.5 * (w[0] + w[n - 1]);
        } else {
            dlo[0] = w[0];       // mirrored ghost at distance of one cell width
            dhi[n - 1] = w[n - 1];
        }
    } else {
        if (per) {
            const int n = ncells;  // unknown m on face x_{m+1} (x_n == x_0)
            vol.resize(n);
            dlo.resize(n);
            dhi.resize(n);
            for (int m = 0; m < n; ++m) {
                double wa = w[(m + 1) % n];
                vol[m] = 0.5 * (w[m] + wa);
                dlo[m] = w[m];
                dhi[m] = wa;
            }
        } else if (bc_lo == BC_D && bc_hi == BC_D) {
            const int n = ncells - 1;  // interior faces
            vol.resize(n);
            dlo.resize(n);
            dhi.resize(n);
            for (int m = 0; m < n; ++m) {
                vol[m] = 0.5 * (w[m] + w[m + 1]);
                dlo[m] = w[m];
                dhi[m] = w[m + 1];
            }
        } else {
            return "face-located unknowns need periodic or Dirichlet-Dirichlet walls";
        }
    }
    const int n = (int)vol.size();
    op.n = n;
    op.vol = vol;
    op.a.resize(n);
    op.b.resize(n);
    op.c.resize(n);
    for (int i = 0; i < n; ++i) {
        op.a[i] = 1.0 / (vol[i] * dlo[i]);
        op.c[i] = 1.0 / (vol[i] * dhi[i]);
        op.b[i] = -(op.a[i] + op.c[i]);
    }
    if (!per) {
        if (loc == LOC_C) {
            // lower wall
            if (bc_lo == BC_N) op.b[0] += op.a[0];
            else op.b[0] -= op.a[0];
            if (bc_hi == BC_N) op.b[n - 1] += op.c[n - 1];
            else op.b[n - 1] -= op.c[n - 1];
        }
        op.a[0] = 0.0;
        op.c[n - 1] = 0.0;
    }
    op.null_mode = per || (loc == LOC_C && bc_lo == BC_N && bc_hi == BC_N);
    // uniform: equal control volumes and equal neighbour distances
    bool uni = true;
    for (int i = 0; i < n && uni; ++i) {
        uni = nearly_equal(vol[i], vol[0], 1e-12) && nearly_equal(dlo[i], vol[0], 1e-12) &&
              nearly_equal(dhi[i], vol[0], 1e-12);
    }
    // a Dirichlet mirrored ghost at a cell-centred wall sits at distance dx_1: still uniform
    op.uniform = uni;
    return "";
}

// ---------------------------------------------------------------------------
// Analytic orthonormal eigenbases of the uniform operators (Fourier,
// cosine and sine bases; the modified wavenumbers are -(4/h^2) sin^2(theta)).
// ---------------------------------------------------------------------------
static bool analytic_basis(const Op1D& op, Eig1D& e) {
    if (!op.uniform) return false;
    const int n = op.n;
    const real h = op.vol[0];
    const real s4 = 4.0L / (h * h);
    e.n = n;
    e.lam.assign(n, 0.0);
    e.Qt.assign((size_t)n * n, 0.0);
    auto Q = [&](int i, int p) -> double& { return e.Qt[(size_t)i * n + p]; };
    const real pi = 3.14159265358979323846264338327950288L;
    if (op.periodic) {
        // real Fourier basis: p = 0 constant; pairs (cos, sin) of wavenumber m;
        // for even n the alternating vector.
        int p = 0;
        for (int i = 0; i < n; ++i) Q(i, 0) = (double)(1.0L / std::sqrt((real)n));
        e.lam[0] = 0.0;
        p = 1;
        for (int m = 1; 2 * m < n; ++m) {
            real th = pi * m / n;
            real lam = -s4 * std::sin(th) * std::sin(th);
            real nc = std::sqrt(2.0L / n);
            for (int i = 0; i < n; ++i) {
                real ang = 2.0L * pi * (real)(((long long)m * i) % n) / (real)n;
                Q(i, p) = (double)(nc * std::cos(ang));
                Q(i, p + 1) = (double)(nc * std::sin(ang));
            }
            e.lam[p] = e.lam[p + 1] = (double)lam;
            p += 2;
        }
        if (n % 2 == 0) {
            for (int i = 0; i < n; ++i) Q(i, p) = (double)(((i % 2) ? -1.0L : 1.0L) / std::sqrt((real)n));
            e.lam[p] = (double)(-s4);
            ++p;
        }
        e.null_index = 0;
        e.analytic = true;
        return true;
    }
    if (op.loc == LOC_C && op.bc_lo == BC_N && op.bc_hi == BC_N) {
        // cosine basis cos(pi k (i + 1/2) / n)
        for (int k = 0; k < n; ++k) {
            real nc = (k == 0) ? std::sqrt(1.0L / n) : std::sqrt(2.0L / n);
            // angle pi k (2i+1) / (2n), reduced exactly modulo 2 pi first
            for (int i = 0; i < n; ++i)
                Q(i, k) = (double)(nc * std::cos(pi * (real)(((long long)k * (2 * i + 1)) % (4LL * n)) / (2.0L * n)));
            real th = pi * k / (2.0L * n);
            e.lam[k] = (double)(-s4 * std::sin(th) * std::sin(th));
        }
        e.lam[0] = 0.0;
        e.null_index = 0;
        e.analytic = true;
        return true;
    }
    if (op.loc == LOC_C && op.bc_lo == BC_D && op.bc_hi == BC_D) {
        // sine basis sin(pi k (i + 1/2) / n), k = 1..n
        for (int k = 1; k <= n; ++k) {
            real nc = (k == n) ? std::sqrt(1.0L / n) : std::sqrt(2.0L / n);
            for (int i = 0; i < n; ++i)
                Q(i, k - 1) =
                    (double)(nc * std::sin(pi * (real)(((long long)k * (2 * i + 1)) % (4LL * n)) / (2.0L * n)));
            real th = pi * k / (2.0L * n);
            e.lam[k - 1] = (double)(-s4 * std::sin(th) * std::sin(th));
        }
        e.null_index = -1;
        e.analytic = true;
        return true;
    }
    if (op.loc == LOC_F && op.bc_lo == BC_D) {
        // interior faces of n+1 cells: sin(pi k (i + 1) / (n + 1)), k = 1..n
        const int m = n + 1;
        for (int k = 1; k <= n; ++k) {
            real nc = std::sqrt(2.0L / m);
            for (int i = 0; i < n; ++i)
                Q(i, k - 1) = (double)(nc * std::sin(pi * (real)(((long long)k * (i + 1)) % (2LL * m)) / m));
            real th = pi * k / (2.0L * m);
            e.lam[k - 1] = (double)(-s4 * std::sin(th) * std::sin(th));
        }
        e.null_index = -1;
        e.analytic = true;
        return true;
    }
    return false;  // mixed Neumann/Dirichlet: numerical
}

// ---------------------------------------------------------------------------
// Implicit QL for a symmetric tridiagonal matrix (Golub & Van Loan §8.3:
// implicit symmetric QR step with Wilkinson shift, run bottom-up).  The
// eigenvector matrix is kept column-major (one contiguous row per vector) so
// that each Givens rotation updates two contiguous arrays.
//
// The numerical eigensolvers run in 80-bit extended precision (long double)
// and round to double at the end: a double-precision eigensolver fixes an
// eigenvector only to about eps ||T|| / gap, i.e. 1e-12..1e-11 for the smooth
// low modes of a stretched operator with N ~ 10^2..10^3, and those modes carry
// the solution of a Poisson problem.
// ---------------------------------------------------------------------------
static bool tridiag_ql(int n, std::vector<real>& d, std::vector<real>& e, std::vector<real>& Zt) {
    if (n <= 1) return true;
    e.resize(n);
    e[n - 1] = 0.0L;
    const real eps = std::numeric_limits<real>::epsilon();
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            // find the first negligible off-diagonal at or below l
            int m = l;
            for (; m < n - 1; ++m) {
                real dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd) break;
            }
            if (m == l) break;
            if (++iter > 60) return false;
            // shift from the leading 2x2 block of the unreduced part (d[l], e[l], d[l+1])
            real g = (d[l + 1] - d[l]) / (2.0L * e[l]);
            real r = std::hypot(g, (real)1.0L);
            g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
            real s = 1.0L, c = 1.0L, p = 0.0L;
            int i = m - 1;
            bool underflow = false;
            for (; i >= l; --i) {
                real f = s * e[i];
                real b = c * e[i];
                r = std::hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0L) {  // deflation by underflow
                    d[i + 1] -= p;
                    e[m] = 0.0L;
                    underflow = true;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0L * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                // rotate eigenvector columns i and i+1
                real* zi = &Zt[(size_t)i * n];
                real* zj = &Zt[(size_t)(i + 1) * n];
                for (int k = 0; k < n; ++k) {
                    real t = zj[k];
                    zj[k] = s * zi[k] + c * t;
                    zi[k] = c * zi[k] - s * t;
                }
            }
            if (underflow) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0L;
        }
    }
    return true;
}

// Householder reduction to tridiagonal form (Golub & Van Loan §8.3.1):
// for k = 0..n-3 reflect A[k+1:, k] onto e_1, update the trailing block with
// the symmetric rank-2 form, accumulate Z = H_0 H_1 ... .  Zt is returned
// column-major (Zt[p*n + i] = Z[i][p]).
static void householder_tridiag(int n, std::vector<real> A, std::vector<real>& d, std::vector<real>& e,
                                std::vector<real>& Zt) {
    auto a = [&](int i, int j) -> real& { return A[(size_t)i * n + j]; };
    std::vector<real> Z((size_t)n * n, 0.0L);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0L;
    std::vector<real> v(n), pv(n), wv(n);
    for (int k = 0; k + 2 < n; ++k) {
        const int m = n - k - 1;  // length of x = A[k+1:, k]
        real alpha = 0.0L;
        for (int i = 0; i < m; ++i) alpha += a(k + 1 + i, k) * a(k + 1 + i, k);
        alpha = std::sqrt(alpha);
        if (alpha == 0.0L) continue;
        real x0 = a(k + 1, k);
        real sgn = x0 >= 0 ? 1.0L : -1.0L;
        // v = x + sgn*alpha*e1, H = I - beta v v^T, beta = 2 / v^T v
        for (int i = 0; i < m; ++i) v[i] = a(k + 1 + i, k);
        v[0] += sgn * alpha;
        real vtv = 0.0L;
        for (int i = 0; i < m; ++i) vtv += v[i] * v[i];
        if (vtv == 0.0L) continue;
        real beta = 2.0L / vtv;
        // p = beta * A22 v
        for (int i = 0; i < m; ++i) {
            real sum = 0.0L;
            const real* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
            for (int j = 0; j < m; ++j) sum += row[j] * v[j];
            pv[i] = beta * sum;
        }
        real ptv = 0.0L;
        for (int i = 0; i < m; ++i) ptv += pv[i] * v[i];
        real kk = 0.5L * beta * ptv;
        for (int i = 0; i < m; ++i) wv[i] = pv[i] - kk * v[i];
        // A22 -= v w^T + w v^T
        for (int i = 0; i < m; ++i) {
            real* row = &A[(size_t)(k + 1 + i) * n + (k + 1)];
            for (int j = 0; j < m; ++j) row[j] -= v[i] * wv[j] + wv[i] * v[j];
        }
        // column k / row k below the diagonal become (-sgn*alpha, 0, ...)
        a(k + 1, k) = -sgn * alpha;
        a(k, k + 1) = -sgn * alpha;
        for (int i = 1; i < m; ++i) {
            a(k + 1 + i, k) = 0.0L;
            a(k, k + 1 + i) = 0.0L;
        }
        // Z <- Z H  (columns k+1..n-1)
        for (int r = 0; r < n; ++r) {
            real* zr = &Z[(size_t)r * n + (k + 1)];
            real sum = 0.0L;
            for (int j = 0; j < m; ++j) sum += zr[j] * v[j];
            sum *= beta;
            for (int j = 0; j < m; ++j) zr[j] -= sum * v[j];
        }
    }
    d.assign(n, 0.0L);
    e.assign(n, 0.0L);
    for (int i = 0; i < n; ++i) d[i] = a(i, i);
    for (int i = 0; i + 1 < n; ++i) e[i] = a(i + 1, i);
    Zt.assign((size_t)n * n, 0.0L);
    for (int i = 0; i < n; ++i)
        for (int p = 0; p < n; ++p) Zt[(size_t)p * n + i] = Z[(size_t)i * n + p];
}

std::string eig_op1d(const Op1D& op, Eig1D& e) {
    e = Eig1D();
    const int n = op.n;
    e.n = n;
    if (analytic_basis(op, e)) return "";
    std::vector<real> s(n);
    for (int i = 0; i < n; ++i) s[i] = std::sqrt((real)op.vol[i]);
    std::vector<real> d(n), off(n, 0.0L), Zt;
    for (int i = 0; i < n; ++i) d[i] = op.b[i];
    if (!op.periodic) {
        // symmetric tridiagonal T~: off-diagonal sqrt(c_i a_{i+1})
        for (int i = 0; i + 1 < n; ++i) off[i] = std::sqrt((real)op.c[i] * (real)op.a[i + 1]);
        Zt.assign((size_t)n * n, 0.0L);
        for (int i = 0; i < n; ++i) Zt[(size_t)i * n + i] = 1.0L;
    } else {
        // cyclic: dense T~ with corners, reduced by Householder first
        std::vector<real> A((size_t)n * n, 0.0L);
        auto put = [&](int i, int j, double v) { A[(size_t)i * n + j] += (real)v * s[i] / s[j]; };
        for (int i = 0; i < n; ++i) {
            put(i, i, op.b[i]);
            put(i, (i + n - 1) % n, op.a[i]);
            put(i, (i + 1) % n, op.c[i]);
        }
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                real m = 0.5L * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
                A[(size_t)i * n + j] = A[(size_t)j * n + i] = m;
            }
        householder_tridiag(n, A, d, off, Zt);
    }
    if (!tridiag_ql(n, d, off, Zt)) return "QL eigensolver did not converge";
    // order by eigenvalue, largest (0 for a null mode) first
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] > d[y]; });
    std::vector<real> lam(n), Q((size_t)n * n);
    for (int p = 0; p < n; ++p) {
        lam[p] = d[idx[p]];
        const real* z = &Zt[(size_t)idx[p] * n];
        for (int i = 0; i < n; ++i) Q[(size_t)i * n + p] = z[i];
    }
    if (op.null_mode) {
        // exact null vector D^{1/2} 1 / ||D^{1/2} 1||, eigenvalue exactly 0; the
        // other vectors are made orthogonal to it
        int k0 = 0;
        for (int p = 1; p < n; ++p)
            if (std::fabs(lam[p]) < std::fabs(lam[k0])) k0 = p;
        real nrm = 0.0L;
        for (int i = 0; i < n; ++i) nrm += (real)op.vol[i];
        nrm = std::sqrt(nrm);
        std::vector<real> v0(n);
        for (int i = 0; i < n; ++i) v0[i] = s[i] / nrm;
        lam[k0] = 0.0L;
        for (int i = 0; i < n; ++i) Q[(size_t)i * n + k0] = v0[i];
        for (int p = 0; p < n; ++p) {
            if (p == k0) continue;
            real dot = 0.0L;
            for (int i = 0; i < n; ++i) dot += v0[i] * Q[(size_t)i * n + p];
            real q2 = 0.0L;
            for (int i = 0; i < n; ++i) {
                real& q = Q[(size_t)i * n + p];
                q -= dot * v0[i];
                q2 += q * q;
            }
            real inv = 1.0L / std::sqrt(q2);
            for (int i = 0; i < n; ++i) Q[(size_t)i * n + p] *= inv;
        }
        e.null_index = k0;
    }
    e.lam.resize(n);
    e.Qt.resize((size_t)n * n);
    for (int p = 0; p < n; ++p) e.lam[p] = (double)lam[p];
    for (size_t k = 0; k < (size_t)n * n; ++k) e.Qt[k] = (double)Q[k];
    return "";
}

}  // namespace tpt
