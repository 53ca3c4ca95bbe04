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
// out = two weighted-Jacobi sweeps on s*L7 from x = 0 with right-hand side b
hipError_t launch_jacobi2_zero(int dtype, const Grid3 &g, int k, const void *b, void *out, double s, double omega,
                               hipStream_t st);
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

// ---- block kernels (k_update.hip, k_block.hip)
// Multivector products on MFMA (k_update.hip), for one side or two sides
// (an X-side and an A-side with the same coefficients):
//   out[s]  = sum_{i in I} in[s][i][:, cols_i] C_i (+ add on side 0),
//             I = all inputs, or the inputs >= 1 when out2 is given;
//             written only in columns c with opos[c] >= 0, at position opos[c]
//   out2[s] = in[s][0] C_0 + (the full sum over inputs >= 1)
// With partials/sums (needs two sides and out2) it also forms the residual
// R = out2[1] - out2[0] diag(theta), writes its columns with wpos[c] >= 0 to
// Wout (N x nW) and sums[c] = sum_p R_pc^2, sums[kout + c] = sum_p out2[0]_pc^2.
struct MVArgs {
    const void *in[2][3];
    int ld[3], k[3];
    const int *cols[3];
    int nin, nside, kout;
    const void *C;          // device, element type of the blocks, (sum k) x kout
    const void *add;
    void *out[2];
    const int *opos;        // device [kout] or nullptr (identity, nout = kout)
    int nout;
    void *out2[2];
    const double *theta;    // device [kout]
    const int *wpos;        // device [kout]
    void *Wout;
    int nW;
    double *partials;       // [mv_blocks(N)][2 kout]
    double *sums;           // [2 kout]
    long long N;
    int variant;            // 0: by shape (narrow: one point per thread; else 16-byte fragment loads),
                            // 1: per-element fragment loads, 2: tiles staged through LDS
};
int mv_blocks(long long N);
hipError_t launch_mv(int dtype, const MVArgs &a, hipStream_t st);

// out[p][jj] = in[p][map[jj]] for jj < nout (in: N x ld)
hipError_t launch_gather_cols(int dtype, long long N, const void *in, int ld, const int *map, int nout, void *out,
                              hipStream_t st);

// Residual of step 7 with the norms of step 8: W[:, jpos[j]] = AX_j - lambda_j X_j
// for the columns with jpos[j] >= 0 (W: N x nJ), and per column the sums of
// (AX_j - lambda_j X_j)^2 and X_j^2 (per-block partials, then reduced).
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
// Tiles of S^T S (mat 0) and S^T AS (mat 1), S = [S_0 .. S_{nblk-1}] with
// K = sum w <= 96 columns; tile codes (mat << 16) | (a << 8) | b cover rows
// 16a..16a+15 and columns 16b..16b+15.
static const int GRAM_MAX_TILES = 48;
struct GramArgs {
    const void *S[3], *AS[3];   // AS[0] == nullptr: S^T S only
    int w[3];
    int nblk;
    int ntiles;
    int tiles[GRAM_MAX_TILES];
    long long N;
    double *partials;   // scratch, gram_partials_bytes
    double *out;        // device [2][Kp][Kp], Kp = K rounded up to 16
    int staged;         // 1: the LDS-staged kernel also for narrow single blocks
};
int gram_kpad(int K);
size_t gram_partials_bytes(int dtype, long long N, int K);
hipError_t launch_gram(int dtype, const GramArgs &a, hipStream_t st);

}  // namespace lobpcg
