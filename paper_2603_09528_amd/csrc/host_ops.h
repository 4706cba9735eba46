// Host-side building blocks of a plan: 1-D operators with boundary rows and
// the eigendecomposition of the symmetrised operator (§2.2.1).
#pragma once
#include <string>
#include <vector>

namespace tpt {

enum Bc { BC_P = 0, BC_N = 1, BC_D = 2 };
enum Loc { LOC_C = 0, LOC_F = 1 };

// One-dimensional operator T of one direction: row i is
// a[i] u[i-1] + b[i] u[i] + c[i] u[i+1]; for a periodic direction a[0] couples
// to u[N-1] and c[N-1] to u[0] (the cyclic corners).  vol = diagonal of D.
struct Op1D {
    int n = 0;             // unknowns
    bool periodic = false;
    bool null_mode = false;  // T 1 = 0 (periodic, or Neumann-Neumann at cell centres)
    bool uniform = false;    // all control volumes and neighbour distances equal
    int bc_lo = BC_N, bc_hi = BC_N, loc = LOC_C;
    std::vector<double> a, b, c, vol;
};

// Returns an empty string on success, else the reason.
std::string build_op1d(int ncells, const double* faces, int bc_lo, int bc_hi, int loc, Op1D& op);

// Eigendecomposition of T~ = D^{1/2} T D^{-1/2}: lam[p], Qt[i*n + p] (column p
// is eigenvector p), orthonormal.  null_index = column of the exact null
// vector (lam = 0) or -1.  analytic = closed-form basis was used.
struct Eig1D {
    int n = 0;
    std::vector<double> lam, Qt;
    int null_index = -1;
    bool analytic = false;
};

std::string eig_op1d(const Op1D& op, Eig1D& e);

}  // namespace tpt
