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
// out = b0 u + b1 (sum of the six axis neighbours of u), zero beyond the grid
hipError_t launch_mass7(int dtype, const Grid3 &g, int k, double b0, double b1, const void *u, void *out,
                        hipStream_t st);
// out = x + omega/(6 s) (b - s L7 x)        (weighted Jacobi on s*L7)
hipError_t launch_jacobi(int dtype, const Grid3 &g, int k, const void *x, const void *b, void *out, double s,
                         double omega, hipStream_t st);
// out = two weighted-Jacobi sweeps on s*L7 from x = 0 with right-hand side b
hipError_t launch_jacobi2_zero(int dtype, const Grid3 &g, int k, const void *b, void *out, double s, double omega,
                               hipStream_t st);
// The first and last sweeps of a cycle (precision dtype, k columns per
// point) on a block stored differently: as FP64 around an FP32 cycle, or
// with kc < k columns (k rounded up to the cycle's vector width; the columns
// past kc are zero in the cycle).  The two sweeps from zero read the
// right-hand side bsrc (dt_in, kc columns) once, write x and the
// right-hand side's copy bcopy in the cycle's layout; the sweep of
// launch_jacobi writes its result to out (dt_out, kc columns).
hipError_t launch_jacobi2_zero_in(int dt_in, int dtype, const Grid3 &g, int kc, int k, const void *bsrc, void *x,
                                  void *bcopy, double s, double omega, hipStream_t st);
hipError_t launch_jacobi_out(int dtype, int dt_out, const Grid3 &g, int kc, int k, const void *x, const void *b,
                             void *out, double s, double omega, hipStream_t st);
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
// Inputs wider than 32 columns, or more than 3 inputs, go to a separate wide
// kernel: the caller splits each block into pieces of at most 32 columns
// (MV_MAX_IN pieces in all) and, with out2, gives the number n0 of leading
// pieces that form the X part in0 C_0.  Outputs wider than 32 columns are
// computed in chunks of columns by separate launches: ld2 is then the row
// stride of out2 and add (and the pointers are offset to the chunk), and
// sums_ld the offset of the second half of sums.
static const int MV_MAX_IN = 12;
struct MVArgs {
    const void *in[2][MV_MAX_IN];
    int ld[MV_MAX_IN], k[MV_MAX_IN];
    const int *cols[MV_MAX_IN];
    int coff[MV_MAX_IN] = {};   // first column of a piece within its stored rows (wide kernel only)
    int nin, nside, kout;
    int n0 = 1;             // leading pieces of the X part (with out2)
    int ld2 = 0;            // row stride of out2 and add (0: kout)
    int sums_ld = 0;        // sums[c] and sums[sums_ld + c] (0: kout)
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
    int frag_only = 0;      // 1: the FP32 update on mvf_kernel even where the LDS-pipelined kernel applies
    int mvl_fragment_stores = 0;  // 1: that kernel stores P, AP and W per MFMA fragment also for few columns
};
int mv_blocks(long long N);
hipError_t launch_mv(int dtype, const MVArgs &a, hipStream_t st);
// widest output chunk (32, 16, or 0 if none fits in LDS) of the wide kernel
// for input pieces of the given widths
int mv_wide_chunk(int dtype, int nin, const int *k);
static const int MV_PIECE = 32;     // columns per input piece (and the widest non-wide output)

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

// out[p][j] = d[p] in[p][j] for an N x k block (B = diag(d) applied to a block)
hipError_t launch_diag_scale(int dtype, long long N, int k, const double *d, const void *in, void *out,
                             hipStream_t st);

// d lambda_i / d k_f accumulation over faces (FP64), w[i] = gbar_i / (x_i, x_i)
hipError_t launch_eig_grad(const Grid3 &g, int m, const double *X, const double *w, double *gkx, double *gky,
                           double *gkz, hipStream_t st);

// ---- Gram products (k_gram.hip)
// Entries of Lm^T Rm for N x KL and N x KR matrices whose columns are
// columns of up to GX_MAX_ARR point-major arrays: column i of Lm is column
// lmap[i] & 255 of array lmap[i] >> 8 (likewise Rm).  The listed 16 x 16 tiles
// (rows 16 ta..16 ta+15 of Lm^T Rm, columns 16 tb..16 tb+15; sorted by ta)
// are written to out[t][e], e = r*64 + lane of the MFMA accumulator layout
// (row 16 ta + Mfma<T>::row(lane, r), column 16 tb + lane % 16).
static const int GX_MAX_ARR = 9;
static const int GX_MAX_L = 96;
static const int GX_MAX_R = 192;
static const int GX_MAX_TILES = 64;
static const int GX_MAXB = 4;        // tiles per wave (sharing one Lm block)
struct GramXArgs {
    const void *arr[GX_MAX_ARR];
    int ld[GX_MAX_ARR];
    int KL, KR;
    unsigned short lmap[GX_MAX_L], rmap[GX_MAX_R];
    int ntiles;
    int ta[GX_MAX_TILES], tb[GX_MAX_TILES];
    long long N;
    double *partials;   // scratch, gram_partials_bytes(N)
    double *out;        // device [ntiles][256]
    int max_nt;         // most tiles per wave for FP64 blocks (1, 2 or GX_MAXB)
    int max_nt32;       // the same for FP32 blocks
    int direct = 0;     // 1: the direct-load kernel even where the LDS-staged one fits
};
size_t gram_partials_bytes(long long N);
hipError_t launch_gramx(int dtype, const GramXArgs &a, hipStream_t st);
// S^T S (w x w, w <= 8) of one block, one grid row per thread: out[i*ldout + j], i <= j
hipError_t launch_gram_rows(int dtype, const void *S, int w, long long N, double *partials, double *out, int ldout,
                            hipStream_t st);

}  // namespace lobpcg
