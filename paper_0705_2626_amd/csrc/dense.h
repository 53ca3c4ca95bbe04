// Host FP64 dense kernels for LOBPCG's small matrices (at most 3m x 3m).
// All matrices are row-major.
#pragma once

namespace lobpcg {
bool chol_scaled(int n, const double *G, double *R);          // G = R^T R, R upper
bool triu_inverse(int n, const double *R, double *Ri);
bool sym_eig(int n, const double *S, double *w, double *V);   // ascending
bool rayleigh_ritz(int n, int m, const double *gramA, const double *gramB, double *theta, double *C);
}  // namespace lobpcg
