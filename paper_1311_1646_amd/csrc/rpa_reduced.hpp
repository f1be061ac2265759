// The reduced DMRG-RPA eigenproblem (Sec. III E, eq. reducedrpa) on the host.
//
// In the span of l trial vectors U (first-order wavefunctions) the RPA
// amplitudes are X = U a, Y = U b; with the l x l matrices
//   H_R = U^T H U,  S_R = U^T U,  W_R = W(U, U)  (symmetric)
// the problem [[A, W], [W, A]] (a, b) = omega [[S, 0], [0, -S]] (a, b),
// A = H_R - E0 S_R, is brought to an orthonormal basis of the span by
// canonical orthogonalization of S_R and solved through the symmetric form
// (A - W)^(1/2) (A + W) (A - W)^(1/2) z = omega^2 z of a stable reference
// (A +- W positive definite there).
#pragma once
#include <vector>

namespace dmrg {

struct RpaReduced {
  int r = 0;                 // rank of S_R kept (orthonormal directions)
  std::vector<double> T;     // l x r, column-major: U T is S-orthonormal
  std::vector<double> omega; // all r positive roots, ascending
  std::vector<double> x, y;  // r x r, column-major: X', Y' of each root in the basis U T,
                             // normalized to X'^T X' - Y'^T Y' = 1
};

// Returns 0, or -1 when A - W or A + W is not positive definite on the kept
// directions (an unstable reference: imaginary RPA frequencies).
int rpa_reduced_solve(int l, const double* HR, const double* SR, const double* WR, double e0, double rank_tol,
                      RpaReduced& out);

// Symmetric eigen-decomposition by cyclic Jacobi rotations: eigenvalues
// ascending in w, eigenvectors in the columns of V (n x n, column-major).
void jacobi_eigh(int n, std::vector<double> A, std::vector<double>& w, std::vector<double>& V);

}  // namespace dmrg
