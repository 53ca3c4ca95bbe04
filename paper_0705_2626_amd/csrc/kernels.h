// Host-side launchers of the LOBPCG kernels (internal to liblobpcg.so).
// Blocks are point-major N x k arrays (element (p, j) at p*k + j).
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>

namespace lobpcg {

enum { DT_F64 = 0, DT_F32 = 1 };

struct Grid3 {
    int nx, ny, nz;
    long long n() const { return (long long)nx * ny * nz; }
};

// ---- stencils (k_stencil.hip)
// out = s * L7 u
hipError_t launch_laplace7(int dtype, const Grid3 &g, int k, const void *u, void *out, double s, hipStream_t st);
// out = x + omega/(6 s) (b - s L7 x)        (weighted Jacobi on s*L7)
hipError_t launch_jacobi(int dtype, const Grid3 &g, int k, const void *x, const void *b, void *out, double s,
                         double omega, hipStream_t st);
// out = b - s L7 x
hipError_t launch_resid7(int dtype, const Grid3 &g, int k, const void *x, const void *b, void *out, double s,
                         hipStream_t st);
// out = A u, A = -div(k grad u) with face coefficients
hipError_t launch_varcoef7(int dtype, const Grid3 &g, int k, const double *kx, const double *ky,
                           const double *kz, const void *u, void *out, hipStream_t st);

// ---- multigrid transfers (k_mg.hip)
// out = c * b (the first Jacobi sweep from a zero guess)
hipError_t launch_scale(int dtype, long long n, const void *b, void *out, double c, hipStream_t st);
// bc = R rf, R = P^T / 8 (full weighting)
hipError_t launch_restrict(int dtype, const Grid3 &f, const Grid3 &c, int k, const void *rf, void *bc,
                           hipStream_t st);
// xf += P ec (trilinear)
hipError_t launch_prolong_add(int dtype, const Grid3 &f, const Grid3 &c, int k, const void *ec, void *xf,
                              hipStream_t st);
// x = sweeps weighted-Jacobi sweeps on s*L7 from zero, whole grid in LDS;
// returns hipErrorInvalidValue if the grid is too large for one workgroup
hipError_t launch_coarse_solve(int dtype, const Grid3 &g, int k, int sweeps, double s, double omega,
                               const void *b, void *x, hipStream_t st);
bool coarse_solve_fits(int dtype, const Grid3 &g);

// ---- block kernels (k_block.hip)
struct CombineArgs {
    const void *in[3];
    int ld[3];          // row length (columns) of each input
    int k[3];           // columns used
    const int *cols[3]; // device column maps (k[i] entries) or nullptr = columns 0..k-1
    int nin;
    const void *C;      // device, element type of the blocks, (sum k) x kout row-major
    int kout;
    const void *add;    // optional N x kout added to out
    void *out;          // N x kout
    void *out2;         // optional: out2 = in[0] C_0 + out, and then out = sum_{i>=1} in_i C_i
    long long N;
};
hipError_t launch_combine(int dtype, const CombineArgs &a, hipStream_t st);

// Residual of step 7 with the norms of step 8.  Writes W (N x nJ packed, column
// jj = column jmap_inv... see kernel) and per-block partial sums.
struct ResidualArgs {
    const void *X, *AX;     // N x m
    const double *lambda;   // device [m]
    const int *jpos;        // device [m]: packed column of j in W, or -1
    void *W;                // N x nJ (may be nullptr)
    int m, nJ;
    long long N;
    double *partials;       // [nblocks][2m]: sum (AX - lambda X)^2, sum X^2
    double *out;            // [2m] reduced
};
int residual_blocks(long long N, int m);
hipError_t launch_residual(int dtype, const ResidualArgs &a, hipStream_t st);

hipError_t launch_cast(int from, int to, long long n, const void *src, void *dst, hipStream_t st);

// d lambda_i / d k_f accumulation over faces (FP64), w[i] = gbar_i / (x_i, x_i)
hipError_t launch_eig_grad(const Grid3 &g, int m, const double *X, const double *w, double *gkx, double *gky,
                           double *gkz, hipStream_t st);

// ---- Gram products (k_gram.hip)
struct GramArgs {
    const void *S[3], *AS[3];
    int w[3];
    int nblk;
    long long N;
    double *partials;   // scratch, gram_partials_bytes
    double *out;        // device [2][Kp][Kp]: S^T S, S^T AS (upper tiles)
};
int gram_kpad(int K);
size_t gram_partials_bytes(int dtype, long long N, int K);
hipError_t launch_gram(int dtype, const GramArgs &a, hipStream_t st);

}  // namespace lobpcg
