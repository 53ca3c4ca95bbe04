// Multivector kernels of LOBPCG on point-major N x k blocks (gfx950):
//  - gather: packing a subset of a block's columns (the active set shrinks);
//  - residual: W_J = AX_J - X_J Lambda_J (step 7) with the column norms that
//    decide the active set (step 8), accumulated in FP64 in a fixed order;
//  - casts between FP32 and FP64 blocks;
//  - the Hellmann-Feynman face gradient of the eigenvalues.
#include "common.h"
#include "kernels.h"

namespace lobpcg {

template <typename T>
static int pick_vec(int k)
{
    const int maxv = 16 / (int)sizeof(T);
    for (int v = maxv; v > 1; v >>= 1)
        if (k % v == 0) return v;
    return 1;
}

static unsigned stride_blocks(i64 total, unsigned cap = 8192)
{
    i64 nb = (total + 255) / 256;
    if (nb < 1) nb = 1;
    return (unsigned)(nb < cap ? nb : cap);
}

// ---------------------------------------------------------------- column gather

static const int MV_MAX_GATHER = 256;   // widest gathered block (m <= 128 columns, twice for safety)

// one thread per output element; the column map in LDS, and 32-bit index
// arithmetic while the block has fewer than 2^31 elements (IDX = unsigned)
template <typename T, typename IDX>
__global__ void __launch_bounds__(256) gather_cols_kernel(i64 N, const T *__restrict__ in, int ld,
                                                          const int *__restrict__ map, int nout, T *__restrict__ out)
{
    __shared__ int smap[MV_MAX_GATHER];
    for (int j = threadIdx.x; j < nout; j += blockDim.x) smap[j] = map[j];
    __syncthreads();
    const IDX total = (IDX)(N * nout), step = (IDX)gridDim.x * blockDim.x;
    for (IDX t = (IDX)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += step) {
        const IDX p = t / (IDX)nout;
        const int j = (int)(t - p * (IDX)nout);
        out[t] = in[(i64)p * ld + smap[j]];
    }
}

hipError_t launch_gather_cols(int dtype, long long N, const void *in, int ld, const int *map, int nout, void *out,
                              hipStream_t st)
{
    const i64 total = (i64)N * nout;
    if (total == 0) return hipSuccess;
    if (nout > MV_MAX_GATHER) return hipErrorInvalidValue;
    const dim3 g(stride_blocks(total, 65536));
    const bool small = total < ((i64)1 << 31);
    if (dtype == DT_F32) {
        if (small)
            hipLaunchKernelGGL((gather_cols_kernel<float, unsigned>), g, dim3(256), 0, st, (i64)N, (const float *)in,
                               ld, map, nout, (float *)out);
        else
            hipLaunchKernelGGL((gather_cols_kernel<float, i64>), g, dim3(256), 0, st, (i64)N, (const float *)in, ld,
                               map, nout, (float *)out);
    } else {
        if (small)
            hipLaunchKernelGGL((gather_cols_kernel<double, unsigned>), g, dim3(256), 0, st, (i64)N,
                               (const double *)in, ld, map, nout, (double *)out);
        else
            hipLaunchKernelGGL((gather_cols_kernel<double, i64>), g, dim3(256), 0, st, (i64)N, (const double *)in,
                               ld, map, nout, (double *)out);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- residual + norms

static const int RES_MAX_BLOCKS = 1024;

int residual_blocks(long long N, int m)
{
    (void)m;
    long long nb = (N + 63) / 64;
    return (int)(nb < RES_MAX_BLOCKS ? (nb > 0 ? nb : 1) : RES_MAX_BLOCKS);
}

template <typename T, int V>
__global__ void __launch_bounds__(256) residual_kernel(const T *__restrict__ X, const T *__restrict__ AX,
                                                       const double *__restrict__ lambda, const int *__restrict__ jpos,
                                                       T *__restrict__ W, int m, int nJ, i64 N,
                                                       double *__restrict__ partials)
{
    extern __shared__ unsigned char smem[];
    double *red = reinterpret_cast<double *>(smem);           // [R][2m]
    const int L = m / V;
    const int R = blockDim.x / L;                             // points per block pass
    const int c = threadIdx.x % L, rs = threadIdx.x / L;
    double sr[V], sx[V];
#pragma unroll
    for (int q = 0; q < V; q++) sr[q] = sx[q] = 0.0;
    double lam[V];
    int jp[V];
#pragma unroll
    for (int q = 0; q < V; q++) {
        lam[q] = lambda[c * V + q];
        jp[q] = jpos[c * V + q];
    }
    if (rs < R) {
        for (i64 p = (i64)blockIdx.x * R + rs; p < N; p += (i64)gridDim.x * R) {
            vec<T, V> x = vload<T, V>(X + p * m + c * V);
            vec<T, V> ax = vload<T, V>(AX + p * m + c * V);
#pragma unroll
            for (int q = 0; q < V; q++) {
                const double xd = (double)x.v[q];
                const double r = (double)ax.v[q] - lam[q] * xd;
                sr[q] += r * r;
                sx[q] += xd * xd;
                if (W && jp[q] >= 0) W[p * nJ + jp[q]] = (T)r;
            }
        }
#pragma unroll
        for (int q = 0; q < V; q++) {
            red[rs * 2 * m + c * V + q] = sr[q];
            red[rs * 2 * m + m + c * V + q] = sx[q];
        }
    }
    __syncthreads();
    // fixed-order sum over the R point slots
    for (int e = threadIdx.x; e < 2 * m; e += blockDim.x) {
        double s = 0.0;
        for (int r = 0; r < R; r++) s += red[r * 2 * m + e];
        partials[(i64)blockIdx.x * 2 * m + e] = s;
    }
}

// out[e] = sum over blocks of partials[b][e]: one workgroup per entry,
// strided partial sums then a fixed-shape tree (a fixed order).
__global__ void __launch_bounds__(256) reduce_partials_kernel(const double *__restrict__ partials, int nb, int width,
                                                              double *__restrict__ out)
{
    __shared__ double red[256];
    const int e = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += partials[(i64)b * width + e];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[e] = red[0];
}

template <typename T, int V>
static hipError_t run_residual(const ResidualArgs &a, hipStream_t st)
{
    const int L = a.m / V;
    const int threads = 256;
    const int R = threads / L;
    const int nb = residual_blocks(a.N, a.m);
    const size_t shm = (size_t)R * 2 * a.m * sizeof(double);
    hipLaunchKernelGGL((residual_kernel<T, V>), dim3(nb), dim3(threads), shm, st, (const T *)a.X, (const T *)a.AX,
                       a.lambda, a.jpos, (T *)a.W, a.m, a.nJ, (i64)a.N, a.partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(reduce_partials_kernel, dim3(2 * a.m), dim3(256), 0, st, a.partials, nb, 2 * a.m, a.out);
    return hipGetLastError();
}

hipError_t launch_residual(int dtype, const ResidualArgs &a, hipStream_t st)
{
    // one thread per V columns; at most 256 column chunks per point
    if (dtype == DT_F32) {
        int v = pick_vec<float>(a.m);
        if (a.m / v > 256) return hipErrorInvalidValue;
        if (v == 4) return run_residual<float, 4>(a, st);
        if (v == 2) return run_residual<float, 2>(a, st);
        return run_residual<float, 1>(a, st);
    }
    int v = pick_vec<double>(a.m);
    if (a.m / v > 256) return hipErrorInvalidValue;
    if (v == 2) return run_residual<double, 2>(a, st);
    return run_residual<double, 1>(a, st);
}

// ---------------------------------------------------------------- casts

template <typename A, typename B>
__global__ void __launch_bounds__(256) cast_kernel(i64 n, const A *__restrict__ s, B *__restrict__ d)
{
    for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (i64)gridDim.x * blockDim.x) d[i] = (B)s[i];
}

hipError_t launch_cast(int from, int to, long long n, const void *src, void *dst, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const unsigned nb = stride_blocks(n, 65536);
    if (from == DT_F64 && to == DT_F32)
        hipLaunchKernelGGL((cast_kernel<double, float>), dim3(nb), dim3(256), 0, st, (i64)n, (const double *)src,
                           (float *)dst);
    else if (from == DT_F32 && to == DT_F64)
        hipLaunchKernelGGL((cast_kernel<float, double>), dim3(nb), dim3(256), 0, st, (i64)n, (const float *)src,
                           (double *)dst);
    else if (from == DT_F64)
        hipLaunchKernelGGL((cast_kernel<double, double>), dim3(nb), dim3(256), 0, st, (i64)n, (const double *)src,
                           (double *)dst);
    else
        hipLaunchKernelGGL((cast_kernel<float, float>), dim3(nb), dim3(256), 0, st, (i64)n, (const float *)src,
                           (float *)dst);
    return hipGetLastError();
}

// ---------------------------------------------------------------- diagonal B

// one thread per row: the row's k entries scaled by d[p]
template <typename T>
__global__ void __launch_bounds__(256) diag_scale_kernel(i64 N, int k, const double *__restrict__ d,
                                                         const T *__restrict__ in, T *__restrict__ out)
{
    for (i64 p = (i64)blockIdx.x * blockDim.x + threadIdx.x; p < N; p += (i64)gridDim.x * blockDim.x) {
        const double s = d[p];
        for (int j = 0; j < k; j++) out[p * k + j] = (T)(s * (double)in[p * k + j]);
    }
}

hipError_t launch_diag_scale(int dtype, long long N, int k, const double *d, const void *in, void *out,
                             hipStream_t st)
{
    if (N == 0) return hipSuccess;
    const unsigned nb = stride_blocks(N, 16384);
    if (dtype == DT_F32)
        hipLaunchKernelGGL(diag_scale_kernel<float>, dim3(nb), dim3(256), 0, st, (i64)N, k, d, (const float *)in,
                           (float *)out);
    else
        hipLaunchKernelGGL(diag_scale_kernel<double>, dim3(nb), dim3(256), 0, st, (i64)N, k, d, (const double *)in,
                           (double *)out);
    return hipGetLastError();
}

// ---------------------------------------------------------------- eigenvalue adjoint

// For each face f between grid points p and q (q beyond the boundary counts
// as zero): g_f = sum_i w_i (x_i[p] - x_i[q])^2, with w_i = gbar_i / (x_i, x_i)
// (the Hellmann-Feynman derivative of the Rayleigh quotient in k_f).
__global__ void __launch_bounds__(256) eig_grad_kernel(int nx, int ny, int nz, int m, const double *__restrict__ X,
                                                       const double *__restrict__ w, double *__restrict__ gkx,
                                                       double *__restrict__ gky, double *__restrict__ gkz)
{
    extern __shared__ unsigned char smem[];
    double *ws = reinterpret_cast<double *>(smem);
    for (int i = threadIdx.x; i < m; i += blockDim.x) ws[i] = w[i];
    __syncthreads();
    const i64 nfx = (i64)nz * ny * (nx + 1), nfy = (i64)nz * (ny + 1) * nx, nfz = (i64)(nz + 1) * ny * nx;
    const i64 total = nfx + nfy + nfz;
    for (i64 f = (i64)blockIdx.x * blockDim.x + threadIdx.x; f < total; f += (i64)gridDim.x * blockDim.x) {
        i64 pa = -1, pb = -1;   // grid points on the two sides (-1: beyond the boundary)
        double *dst;
        if (f < nfx) {
            const int i = (int)(f % (nx + 1));
            const i64 yz = f / (nx + 1);
            const i64 rowbase = yz * nx;  // point (0, y, z)
            if (i > 0) pa = rowbase + i - 1;
            if (i < nx) pb = rowbase + i;
            dst = gkx + f;
        } else if (f < nfx + nfy) {
            const i64 g = f - nfx;
            const int x = (int)(g % nx);
            const int i = (int)((g / nx) % (ny + 1));
            const i64 z = g / ((i64)nx * (ny + 1));
            if (i > 0) pa = x + (i64)nx * ((i - 1) + (i64)ny * z);
            if (i < ny) pb = x + (i64)nx * (i + (i64)ny * z);
            dst = gky + g;
        } else {
            const i64 g = f - nfx - nfy;
            const i64 xy = g % ((i64)nx * ny);
            const i64 i = g / ((i64)nx * ny);
            if (i > 0) pa = xy + (i - 1) * (i64)nx * ny;
            if (i < nz) pb = xy + i * (i64)nx * ny;
            dst = gkz + g;
        }
        double s = 0.0;
        for (int c = 0; c < m; c++) {
            const double va = pa >= 0 ? X[pa * m + c] : 0.0;
            const double vb = pb >= 0 ? X[pb * m + c] : 0.0;
            const double d = va - vb;
            s += ws[c] * d * d;
        }
        *dst = s;
    }
}

hipError_t launch_eig_grad(const Grid3 &g, int m, const double *X, const double *w, double *gkx, double *gky,
                           double *gkz, hipStream_t st)
{
    const i64 total = (i64)g.nz * g.ny * (g.nx + 1) + (i64)g.nz * (g.ny + 1) * g.nx + (i64)(g.nz + 1) * g.ny * g.nx;
    hipLaunchKernelGGL(eig_grad_kernel, dim3(stride_blocks(total, 65536)), dim3(256), m * sizeof(double), st, g.nx,
                       g.ny, g.nz, m, X, w, gkx, gky, gkz);
    return hipGetLastError();
}

}  // namespace lobpcg
