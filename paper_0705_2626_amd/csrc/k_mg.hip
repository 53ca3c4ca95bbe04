// Multigrid transfer and coarsest-level kernels for the V-cycle preconditioner
// (the preconditioner T of step 9, Section 2.2; Section 2.1.1 asks for T
// linear, symmetric and positive definite).
//
// Level l has floor(n/2^l) points per axis and coarse node I sits on fine node
// 2I+1.  Prolongation P is trilinear (fine 2I+1 <- coarse I; fine 2I <- half
// of coarse I-1 and I), restriction is R = P^T/8, i.e. the (1,2,1)^3/64 full
// weighting.  Blocks are point-major N x k; every thread owns V consecutive
// columns of one grid point.
#include "common.h"
#include "kernels.h"

namespace lobpcg {

template <typename T>
__global__ void __launch_bounds__(256) scale_kernel(i64 n, const T *__restrict__ b, T *__restrict__ out, T c)
{
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x)
        out[i] = c * b[i];
}

hipError_t launch_scale(int dtype, long long n, const void *b, void *out, double c, hipStream_t st)
{
    long long nb = (n + 255) / 256;
    unsigned blocks = (unsigned)(nb < 65536 ? nb : 65536);
    if (blocks == 0) return hipSuccess;
    if (dtype == DT_F32)
        hipLaunchKernelGGL(scale_kernel<float>, dim3(blocks), dim3(256), 0, st, (i64)n, (const float *)b,
                           (float *)out, (float)c);
    else
        hipLaunchKernelGGL(scale_kernel<double>, dim3(blocks), dim3(256), 0, st, (i64)n, (const double *)b,
                           (double *)out, c);
    return hipGetLastError();
}

// bc[P] = sum over the 27 fine neighbours of fine node (2X+1, 2Y+1, 2Z+1) of
// w(a) w(b) w(c) rf / 64, w = (1, 2, 1); fine nodes beyond the grid are zero.
template <typename T, int V>
__global__ void __launch_bounds__(256) restrict_kernel(int nxf, int nyf, int nzf, int nxc, int nyc, int nzc, int L,
                                                       const T *__restrict__ rf, T *__restrict__ bc)
{
    const i64 total = (i64)nxc * nyc * nzc * L;
    for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (i64)gridDim.x * blockDim.x) {
    const int c = (int)(t % L);
    const i64 P = t / L;
    const int X = (int)(P % nxc);
    const int Y = (int)((P / nxc) % nyc);
    const int Z = (int)(P / ((i64)nxc * nyc));
    T acc[V];
#pragma unroll
    for (int q = 0; q < V; q++) acc[q] = T(0);
    const T w[3] = {T(1), T(2), T(1)};
    for (int cz = 0; cz < 3; cz++) {
        const int zf = 2 * Z + cz;
        if (zf >= nzf) continue;
        for (int cy = 0; cy < 3; cy++) {
            const int yf = 2 * Y + cy;
            if (yf >= nyf) continue;
            for (int cx = 0; cx < 3; cx++) {
                const int xf = 2 * X + cx;
                if (xf >= nxf) continue;
                const T wt = w[cx] * w[cy] * w[cz];
                const i64 p = (i64)xf + (i64)nxf * ((i64)yf + (i64)nyf * zf);
                vec<T, V> r = vload<T, V>(rf + (p * L + c) * V);
#pragma unroll
                for (int q = 0; q < V; q++) acc[q] += wt * r.v[q];
            }
        }
    }
    vec<T, V> o;
#pragma unroll
    for (int q = 0; q < V; q++) o.v[q] = acc[q] * T(1.0 / 64.0);
    vstore<T, V>(bc + (P * L + c) * V, o);
    }
}

// Coarse indices and weights that reach fine index i along one axis.
__device__ __forceinline__ int prolong_1d(int i, int nc, int *I, float *w)
{
    if (i & 1) {
        I[0] = (i - 1) >> 1;
        w[0] = 1.f;
        return I[0] < nc ? 1 : 0;
    }
    int n = 0;
    const int a = (i >> 1) - 1, b = i >> 1;
    if (a >= 0 && a < nc) { I[n] = a; w[n] = 0.5f; n++; }
    if (b < nc) { I[n] = b; w[n] = 0.5f; n++; }
    return n;
}

template <typename T, int V>
__global__ void __launch_bounds__(256) prolong_add_kernel(int nxf, int nyf, int nzf, int nxc, int nyc, int nzc,
                                                          int L, const T *__restrict__ ec, T *__restrict__ xf)
{
    const i64 total = (i64)nxf * nyf * nzf * L;
    for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (i64)gridDim.x * blockDim.x) {
    const int c = (int)(t % L);
    const i64 p = t / L;
    const int x = (int)(p % nxf);
    const int y = (int)((p / nxf) % nyf);
    const int z = (int)(p / ((i64)nxf * nyf));
    int Ix[2], Iy[2], Iz[2];
    float wx[2], wy[2], wz[2];
    const int nx_ = prolong_1d(x, nxc, Ix, wx), ny_ = prolong_1d(y, nyc, Iy, wy), nz_ = prolong_1d(z, nzc, Iz, wz);
    T acc[V];
#pragma unroll
    for (int q = 0; q < V; q++) acc[q] = T(0);
    for (int a = 0; a < nz_; a++)
        for (int b2 = 0; b2 < ny_; b2++)
            for (int d = 0; d < nx_; d++) {
                const T wt = (T)(wx[d] * wy[b2] * wz[a]);
                const i64 P = (i64)Ix[d] + (i64)nxc * ((i64)Iy[b2] + (i64)nyc * Iz[a]);
                vec<T, V> e = vload<T, V>(ec + (P * L + c) * V);
#pragma unroll
                for (int q = 0; q < V; q++) acc[q] += wt * e.v[q];
            }
    T *dst = xf + (p * L + c) * V;
    vec<T, V> o = vload<T, V>(dst);
#pragma unroll
    for (int q = 0; q < V; q++) o.v[q] += acc[q];
    vstore<T, V>(dst, o);
    }
}

// Workgroups for a grid-stride loop over `total` items: enough to fill the
// chip many times over, capped so the grid stays small.
static unsigned stride_blocks(i64 total)
{
    i64 nb = (total + 255) / 256;
    return (unsigned)(nb < 65536 ? (nb > 0 ? nb : 1) : 65536);
}

template <typename T>
static int pick_vec(int k)
{
    const int maxv = 16 / (int)sizeof(T);
    for (int v = maxv; v > 1; v >>= 1)
        if (k % v == 0) return v;
    return 1;
}

template <typename T, int V>
static hipError_t run_restrict(const Grid3 &f, const Grid3 &c, int k, const void *rf, void *bc, hipStream_t st)
{
    const int L = k / V;
    const i64 total = c.n() * L;
    hipLaunchKernelGGL((restrict_kernel<T, V>), dim3(stride_blocks(total)), dim3(256), 0, st, f.nx,
                       f.ny, f.nz, c.nx, c.ny, c.nz, L, (const T *)rf, (T *)bc);
    return hipGetLastError();
}

template <typename T, int V>
static hipError_t run_prolong(const Grid3 &f, const Grid3 &c, int k, const void *ec, void *xf, hipStream_t st)
{
    const int L = k / V;
    const i64 total = f.n() * L;
    hipLaunchKernelGGL((prolong_add_kernel<T, V>), dim3(stride_blocks(total)), dim3(256), 0, st, f.nx,
                       f.ny, f.nz, c.nx, c.ny, c.nz, L, (const T *)ec, (T *)xf);
    return hipGetLastError();
}

hipError_t launch_restrict(int dtype, const Grid3 &f, const Grid3 &c, int k, const void *rf, void *bc,
                           hipStream_t st)
{
    if (c.n() == 0) return hipSuccess;
    if (dtype == DT_F32) {
        switch (pick_vec<float>(k)) {
        case 4: return run_restrict<float, 4>(f, c, k, rf, bc, st);
        case 2: return run_restrict<float, 2>(f, c, k, rf, bc, st);
        default: return run_restrict<float, 1>(f, c, k, rf, bc, st);
        }
    }
    if (pick_vec<double>(k) == 2) return run_restrict<double, 2>(f, c, k, rf, bc, st);
    return run_restrict<double, 1>(f, c, k, rf, bc, st);
}

hipError_t launch_prolong_add(int dtype, const Grid3 &f, const Grid3 &c, int k, const void *ec, void *xf,
                              hipStream_t st)
{
    if (dtype == DT_F32) {
        switch (pick_vec<float>(k)) {
        case 4: return run_prolong<float, 4>(f, c, k, ec, xf, st);
        case 2: return run_prolong<float, 2>(f, c, k, ec, xf, st);
        default: return run_prolong<float, 1>(f, c, k, ec, xf, st);
        }
    }
    if (pick_vec<double>(k) == 2) return run_prolong<double, 2>(f, c, k, ec, xf, st);
    return run_prolong<double, 1>(f, c, k, ec, xf, st);
}

// Coarsest level: `sweeps` weighted-Jacobi sweeps from x = 0 on s*L7, one
// workgroup per column with the whole grid in LDS.
static const int COARSE_MAX_POINTS = 2048;

bool coarse_solve_fits(int dtype, const Grid3 &g)
{
    (void)dtype;
    return g.n() <= COARSE_MAX_POINTS;
}

template <typename T>
__global__ void __launch_bounds__(256) coarse_solve_kernel(int nx, int ny, int nz, int k, int sweeps, T s, T c1,
                                                           const T *__restrict__ b, T *__restrict__ x)
{
    extern __shared__ unsigned char smem[];
    T *bl = reinterpret_cast<T *>(smem);
    const int n = nx * ny * nz;
    T *x0 = bl + n, *x1 = bl + 2 * n;
    const int col = blockIdx.x;
    for (int p = threadIdx.x; p < n; p += blockDim.x) {
        T bv = b[(i64)p * k + col];
        bl[p] = bv;
        x0[p] = sweeps > 0 ? c1 * bv : T(0);   // first sweep from the zero guess
    }
    __syncthreads();
    for (int it = 1; it < sweeps; it++) {
        for (int p = threadIdx.x; p < n; p += blockDim.x) {
            const int xx = p % nx, yy = (p / nx) % ny, zz = p / (nx * ny);
            T a = T(6) * x0[p];
            if (xx > 0) a -= x0[p - 1];
            if (xx + 1 < nx) a -= x0[p + 1];
            if (yy > 0) a -= x0[p - nx];
            if (yy + 1 < ny) a -= x0[p + nx];
            if (zz > 0) a -= x0[p - nx * ny];
            if (zz + 1 < nz) a -= x0[p + nx * ny];
            x1[p] = x0[p] + c1 * (bl[p] - s * a);
        }
        __syncthreads();
        T *tmp = x0;
        x0 = x1;
        x1 = tmp;
    }
    for (int p = threadIdx.x; p < n; p += blockDim.x) x[(i64)p * k + col] = x0[p];
}

hipError_t launch_coarse_solve(int dtype, const Grid3 &g, int k, int sweeps, double s, double omega,
                               const void *b, void *x, hipStream_t st)
{
    if (!coarse_solve_fits(dtype, g)) return hipErrorInvalidValue;
    const double c1 = omega / (6.0 * s);
    const size_t n = (size_t)g.n();
    if (dtype == DT_F32)
        hipLaunchKernelGGL(coarse_solve_kernel<float>, dim3(k), dim3(256), 3 * n * sizeof(float), st, g.nx, g.ny,
                           g.nz, k, sweeps, (float)s, (float)c1, (const float *)b, (float *)x);
    else
        hipLaunchKernelGGL(coarse_solve_kernel<double>, dim3(k), dim3(256), 3 * n * sizeof(double), st, g.nx, g.ny,
                           g.nz, k, sweeps, s, c1, (const double *)b, (double *)x);
    return hipGetLastError();
}

}  // namespace lobpcg
