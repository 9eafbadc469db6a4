// Host-side FP64 set-up mathematics of libvps (no GPU code).
//
// The 1D Q_k element (Gauss-Lobatto support points), its reference mass and
// stiffness matrices, the 1D patch matrices of a two-cell patch, the
// generalized symmetric eigenproblem behind the fast diagonalization of
// Appendix A.3 (eq:fdm:eigen), the 1D transfer matrices (coarse basis
// functions evaluated at fine nodes, Section 2) and a dense Cholesky inverse
// for the variable-coefficient coarse solver.
#pragma once

#include <vector>

namespace vps {

using Mat = std::vector<double>;  // row-major dense matrix

// Legendre polynomial P_n and its first two derivatives at x in [-1, 1].
void legendre(int n, double x, double* p, double* dp, double* d2p);

// k+1 Gauss-Lobatto-Legendre points on [0, 1] (end points and roots of P_k').
std::vector<double> gll_points(int k);

// n-point Gauss-Legendre rule on [0, 1].
void gauss_rule(int n, std::vector<double>* x, std::vector<double>* w);

// l_a(x) and l_a'(x) of the Lagrange basis on `nodes`.
double lagrange(const std::vector<double>& nodes, int a, double x);
double lagrange_deriv(const std::vector<double>& nodes, int a, double x);

// Reference (unit interval) mass and stiffness matrices, (k+1) x (k+1).
void reference_matrices(int k, Mat* M, Mat* K);

// Matrices of `ncell` consecutive cells of size h assembled on their
// k*ncell+1 nodes; if `cell_weight` is given, cell c is weighted by it.
void assemble_1d(int k, int ncell, double h, Mat* M, Mat* K, const double* cell_weight = nullptr);

// Generalized symmetric-definite eigenproblem K t = lambda M t (n x n):
// returns T (column m = eigenvector m, T^T M T = I) and ascending lambda.
// Cholesky of M, then cyclic Jacobi on L^{-1} K L^{-T}.
void gen_eig(int n, const Mat& M, const Mat& K, Mat* T, std::vector<double>* lambda);

// Split the eigenvectors of a reversal-symmetric 1D problem (q odd) into the
// symmetric ones (T[q-1-i][m] = T[i][m], (q+1)/2 of them) and the
// antisymmetric ones ((q-1)/2), each group in ascending eigenvalue order.
// Te: (q+1)/2 x (q+1)/2, rows i = 0..(q-1)/2; To: (q-1)/2 x (q-1)/2, rows
// i = 0..(q-3)/2.  order[j] = original mode of internal mode j (symmetric
// first).  Returns false if some eigenvector is neither (tolerance 1e-10).
bool fdm_even_odd(int q, const Mat& T, Mat* Te, Mat* To, std::vector<int>* order);

// In-place inverse of an SPD matrix (Cholesky, then L^{-T} L^{-1}).
// Returns false if the matrix is not numerically SPD.
bool spd_inverse(int n, Mat* A);

// 1D prolongation: value of coarse basis function i (coarse mesh of nc cells)
// at fine node f (mesh of 2*nc cells), (2k nc + 1) x (k nc + 1).
void prolongation_1d(int k, int nc, Mat* P);

}  // namespace vps
