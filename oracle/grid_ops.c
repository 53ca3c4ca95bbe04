/*
 * Oracle grid operators -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, obviously correct FP64 loops for the operators that the
 * LOBPCG oracle applies to whole blocks of grid vectors.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load this
 * code; the GPU library never does, and the two share no source.
 *
 * Layout (deliberately different from the GPU library's): a block of k grid
 * vectors is an N x k column-major array, column j stored contiguously at
 * offset j*N.  Grid point (x, y, z) is p = x + nx*(y + ny*z), 0-based.  Values
 * outside the grid are zero (homogeneous Dirichlet boundary).
 *
 * Built with gcc -O2 -fopenmp and without -ffast-math: the paper warns that
 * aggressive optimisation can break the scaling invariance LOBPCG relies on
 * (Section 2.2, discussion after the algorithm).
 */
#include <stddef.h>
#include <stdlib.h>
#include <math.h>

typedef ptrdiff_t idx;

static double val(const double *u, int nx, int ny, int nz, int x, int y, int z)
{
    if (x < 0 || y < 0 || z < 0 || x >= nx || y >= ny || z >= nz) return 0.0;
    return u[(idx)x + (idx)nx * ((idx)y + (idx)ny * z)];
}

/* 7-point finite-difference Laplacian (Section 4): diagonal 6, each of the six
 * axis neighbours -1.  Its eigenvalues are the closed form of Section 4.1. */
void or_laplace7(int nx, int ny, int nz, int k, const double *u, double *out)
{
    idx N = (idx)nx * ny * nz;
    for (int j = 0; j < k; j++) {
        const double *uj = u + j * N;
        double *oj = out + j * N;
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++) {
                    double s = 6.0 * val(uj, nx, ny, nz, x, y, z)
                             - val(uj, nx, ny, nz, x - 1, y, z) - val(uj, nx, ny, nz, x + 1, y, z)
                             - val(uj, nx, ny, nz, x, y - 1, z) - val(uj, nx, ny, nz, x, y + 1, z)
                             - val(uj, nx, ny, nz, x, y, z - 1) - val(uj, nx, ny, nz, x, y, z + 1);
                    oj[(idx)x + (idx)nx * ((idx)y + (idx)ny * z)] = s;
                }
    }
}

/* Face-coefficient arrays (z-major C order):
 *   kx[(z*ny + y)*(nx+1) + i]  face between x-indices i-1 and i, i = 0..nx
 *   ky[(z*(ny+1) + i)*nx + x]  face between y-indices i-1 and i, i = 0..ny
 *   kz[(i*ny + y)*nx + x]      face between z-indices i-1 and i, i = 0..nz
 * Faces i = 0 and i = n touch the boundary, where u is zero. */
static idx fx(int nx, int ny, int x, int y, int z) { return ((idx)z * ny + y) * (nx + 1) + x; }
static idx fy(int nx, int ny, int x, int y, int z) { return ((idx)z * (ny + 1) + y) * nx + x; }
static idx fz(int nx, int ny, int x, int y, int z) { return ((idx)z * ny + y) * nx + x; }

/* Variable-coefficient operator -div(k grad u), cell-centred finite
 * differences with one coefficient per face:
 *   (Au)_p = sum over the six faces f of p of k_f (u_p - u_q),
 * q the grid point across f (u_q = 0 beyond the boundary).  With k = 1 on
 * every face this is exactly the 7-point Laplacian above. */
void or_varcoef7(int nx, int ny, int nz, int k, const double *kx, const double *ky,
                 const double *kz, const double *u, double *out)
{
    idx N = (idx)nx * ny * nz;
    for (int j = 0; j < k; j++) {
        const double *uj = u + j * N;
        double *oj = out + j * N;
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int x = 0; x < nx; x++) {
                    double up = val(uj, nx, ny, nz, x, y, z);
                    double s = 0.0;
                    s += kx[fx(nx, ny, x, y, z)]     * (up - val(uj, nx, ny, nz, x - 1, y, z));
                    s += kx[fx(nx, ny, x + 1, y, z)] * (up - val(uj, nx, ny, nz, x + 1, y, z));
                    s += ky[fy(nx, ny, x, y, z)]     * (up - val(uj, nx, ny, nz, x, y - 1, z));
                    s += ky[fy(nx, ny, x, y + 1, z)] * (up - val(uj, nx, ny, nz, x, y + 1, z));
                    s += kz[fz(nx, ny, x, y, z)]     * (up - val(uj, nx, ny, nz, x, y, z - 1));
                    s += kz[fz(nx, ny, x, y, z + 1)] * (up - val(uj, nx, ny, nz, x, y, z + 1));
                    oj[(idx)x + (idx)nx * ((idx)y + (idx)ny * z)] = s;
                }
    }
}

/* One 1-D prolongation weight: the contribution of coarse index I to fine
 * index i.  Coarse node I sits on fine node 2I+1; an even fine node 2I lies
 * half way between coarse nodes I-1 and I (linear interpolation, zero beyond
 * the coarse grid). */
static double pw(int i, int I)
{
    if (i == 2 * I + 1) return 1.0;
    if (i == 2 * I || i == 2 * I + 2) return 0.5;
    return 0.0;
}

/* Full-weighting restriction, R = P^T / 8 with P the trilinear prolongation
 * below: each coarse value is the (1,2,1)^3/64-weighted mean of the 27 fine
 * values around fine node (2I+1, 2J+1, 2K+1). */
void or_restrict(int nxf, int nyf, int nzf, int nxc, int nyc, int nzc, int k,
                 const double *rf, double *bc)
{
    idx Nf = (idx)nxf * nyf * nzf, Nc = (idx)nxc * nyc * nzc;
    for (int j = 0; j < k; j++) {
        const double *r = rf + j * Nf;
        double *b = bc + j * Nc;
#pragma omp parallel for schedule(static)
        for (int Z = 0; Z < nzc; Z++)
            for (int Y = 0; Y < nyc; Y++)
                for (int X = 0; X < nxc; X++) {
                    double s = 0.0;
                    for (int c = 2 * Z; c <= 2 * Z + 2; c++)
                        for (int b2 = 2 * Y; b2 <= 2 * Y + 2; b2++)
                            for (int a = 2 * X; a <= 2 * X + 2; a++)
                                s += pw(a, X) * pw(b2, Y) * pw(c, Z) * val(r, nxf, nyf, nzf, a, b2, c);
                    b[(idx)X + (idx)nxc * ((idx)Y + (idx)nyc * Z)] = s / 8.0;
                }
    }
}

/* Trilinear prolongation added onto a fine block: xf += P ec. */
void or_prolong_add(int nxf, int nyf, int nzf, int nxc, int nyc, int nzc, int k,
                    const double *ec, double *xf)
{
    idx Nf = (idx)nxf * nyf * nzf, Nc = (idx)nxc * nyc * nzc;
    for (int j = 0; j < k; j++) {
        const double *e = ec + j * Nc;
        double *x = xf + j * Nf;
#pragma omp parallel for schedule(static)
        for (int zf = 0; zf < nzf; zf++)
            for (int yf = 0; yf < nyf; yf++)
                for (int xf_ = 0; xf_ < nxf; xf_++) {
                    double s = 0.0;
                    /* coarse nodes with a nonzero weight on fine node i lie in
                     * [i/2 - 1, i/2]; pw() is zero for the others */
                    for (int Z = (zf - 2) / 2; Z <= zf / 2; Z++)
                        for (int Y = (yf - 2) / 2; Y <= yf / 2; Y++)
                            for (int X = (xf_ - 2) / 2; X <= xf_ / 2; X++) {
                                if (X < 0 || Y < 0 || Z < 0 || X >= nxc || Y >= nyc || Z >= nzc) continue;
                                s += pw(xf_, X) * pw(yf, Y) * pw(zf, Z) * e[(idx)X + (idx)nxc * ((idx)Y + (idx)nyc * Z)];
                            }
                    x[(idx)xf_ + (idx)nxf * ((idx)yf + (idx)nyf * zf)] += s;
                }
    }
}

/* One weighted-Jacobi sweep on level operator s*L7 (s = 4^-l):
 *   xout = x + omega / (6 s) * (b - s * L7 x).
 * x == NULL means x = 0 (the first sweep from a zero guess). */
void or_jacobi(int nx, int ny, int nz, int k, double s, double omega, const double *x,
               const double *b, double *xout)
{
    idx N = (idx)nx * ny * nz;
    for (int j = 0; j < k; j++) {
        const double *bj = b + j * N;
        const double *xj = x ? x + j * N : NULL;
        double *oj = xout + j * N;
#pragma omp parallel for schedule(static)
        for (int z = 0; z < nz; z++)
            for (int y = 0; y < ny; y++)
                for (int xx = 0; xx < nx; xx++) {
                    idx p = (idx)xx + (idx)nx * ((idx)y + (idx)ny * z);
                    double ax = 0.0, xp = 0.0;
                    if (xj) {
                        xp = xj[p];
                        ax = 6.0 * xp
                           - val(xj, nx, ny, nz, xx - 1, y, z) - val(xj, nx, ny, nz, xx + 1, y, z)
                           - val(xj, nx, ny, nz, xx, y - 1, z) - val(xj, nx, ny, nz, xx, y + 1, z)
                           - val(xj, nx, ny, nz, xx, y, z - 1) - val(xj, nx, ny, nz, xx, y, z + 1);
                    }
                    oj[p] = xp + omega / (6.0 * s) * (bj[p] - s * ax);
                }
    }
}

/* Hellmann-Feynman eigenvalue adjoint for -div(k grad u):
 * A = sum_f k_f (e_p - e_q)(e_p - e_q)^T, so for the Rayleigh quotient of x_i
 *   d lambda_i / d k_f = (x_i[p] - x_i[q])^2 / (x_i, x_i)
 * (x_i[q] = 0 beyond the boundary).  The vector-Jacobian product with the
 * cotangent gbar is g_f = sum_i gbar_i d lambda_i / d k_f. */
void or_eig_grad_faces(int nx, int ny, int nz, int m, const double *X, const double *gbar,
                       double *gkx, double *gky, double *gkz)
{
    idx N = (idx)nx * ny * nz;
    double *w = (double *)malloc(sizeof(double) * (m > 0 ? m : 1));
    for (int i = 0; i < m; i++) {
        double nn = 0.0;
        for (idx p = 0; p < N; p++) nn += X[i * N + p] * X[i * N + p];
        w[i] = gbar[i] / nn;
    }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int i = 0; i <= nx; i++) {
                double s = 0.0;
                for (int c = 0; c < m; c++) {
                    const double *x = X + c * N;
                    double d = val(x, nx, ny, nz, i - 1, y, z) - val(x, nx, ny, nz, i, y, z);
                    s += w[c] * d * d;
                }
                gkx[fx(nx, ny, i, y, z)] = s;
            }
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; z++)
        for (int i = 0; i <= ny; i++)
            for (int x0 = 0; x0 < nx; x0++) {
                double s = 0.0;
                for (int c = 0; c < m; c++) {
                    const double *x = X + c * N;
                    double d = val(x, nx, ny, nz, x0, i - 1, z) - val(x, nx, ny, nz, x0, i, z);
                    s += w[c] * d * d;
                }
                gky[fy(nx, ny, x0, i, z)] = s;
            }
#pragma omp parallel for schedule(static)
    for (int i = 0; i <= nz; i++)
        for (int y = 0; y < ny; y++)
            for (int x0 = 0; x0 < nx; x0++) {
                double s = 0.0;
                for (int c = 0; c < m; c++) {
                    const double *x = X + c * N;
                    double d = val(x, nx, ny, nz, x0, y, i - 1) - val(x, nx, ny, nz, x0, y, i);
                    s += w[c] * d * d;
                }
                gkz[fz(nx, ny, x0, y, i)] = s;
            }
    free(w);
}
