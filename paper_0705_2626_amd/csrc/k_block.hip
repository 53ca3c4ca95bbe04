// Multivector kernels of LOBPCG on point-major N x k blocks (gfx950):
//  - combine: out = sum_i in_i[:, cols_i] C_i, the "X*C" products of steps
//    3-4 (X R^-1, X Z), 11 and 14-15 (W R^-1, P_J R^-1) and the Ritz-vector
//    update of steps 27-28 / 31-32, fused so that P and X (or AP and AX) come
//    out of one pass over [X, W_J, P_J];
//  - residual: W_J = AX_J - X_J Lambda_J (step 7) with the column norms that
//    decide the active set (step 8), accumulated in FP64 in a fixed order;
//  - casts between FP32 and FP64 blocks;
//  - the Hellmann-Feynman face gradient of the eigenvalues.
#include "common.h"
#include "kernels.h"

namespace lobpcg {

template <typename T>
struct CombineDev {
    const T *in[3];
    int ld[3], k[3];
    const int *cols[3];
    int nin, kout, ksum;
    const T *C;
    const T *add;
    T *out, *out2;
    i64 N;
};

// One thread owns V consecutive output columns of one grid point.  The
// coefficients (and column maps) live in LDS; the input rows are read once per
// point by the kout/V threads that share it (L1 broadcast).
template <typename T, int V, bool OUT2>
__global__ void __launch_bounds__(256) combine_kernel(CombineDev<T> a)
{
    extern __shared__ unsigned char smem[];
    T *Cs = reinterpret_cast<T *>(smem);
    int *cmap = reinterpret_cast<int *>(Cs + a.ksum * a.kout);
    for (int i = threadIdx.x; i < a.ksum * a.kout; i += blockDim.x) Cs[i] = a.C[i];
    {
        int off = 0;
        for (int b = 0; b < a.nin; b++) {
            for (int r = threadIdx.x; r < a.k[b]; r += blockDim.x) cmap[off + r] = a.cols[b] ? a.cols[b][r] : r;
            off += a.k[b];
        }
    }
    __syncthreads();
    const int L = a.kout / V;
    const i64 total = a.N * L;
    for (i64 t = (i64)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (i64)gridDim.x * blockDim.x) {
        const int c = (int)(t % L);
        const i64 p = t / L;
        T acc[V], acc0[V];
        if (a.add) {
            vec<T, V> ad = vload<T, V>(a.add + p * a.kout + c * V);
#pragma unroll
            for (int q = 0; q < V; q++) acc[q] = ad.v[q];
        } else {
#pragma unroll
            for (int q = 0; q < V; q++) acc[q] = T(0);
        }
#pragma unroll
        for (int q = 0; q < V; q++) acc0[q] = T(0);
        int roff = 0;
        for (int b = 0; b < a.nin; b++) {
            const T *row = a.in[b] + p * a.ld[b];
            const int kb = a.k[b];
            for (int r = 0; r < kb; r++) {
                const T xv = row[cmap[roff + r]];
                const T *cr = Cs + (roff + r) * a.kout + c * V;
                if (OUT2 && b == 0) {
#pragma unroll
                    for (int q = 0; q < V; q++) acc0[q] += xv * cr[q];
                } else {
#pragma unroll
                    for (int q = 0; q < V; q++) acc[q] += xv * cr[q];
                }
            }
            roff += kb;
        }
        vec<T, V> o;
#pragma unroll
        for (int q = 0; q < V; q++) o.v[q] = acc[q];
        vstore<T, V>(a.out + p * a.kout + c * V, o);
        if (OUT2) {
#pragma unroll
            for (int q = 0; q < V; q++) o.v[q] = acc0[q] + acc[q];
            vstore<T, V>(a.out2 + p * a.kout + c * V, o);
        }
    }
}

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

template <typename T, int V>
static hipError_t run_combine(const CombineArgs &ha, hipStream_t st)
{
    CombineDev<T> a;
    a.ksum = 0;
    for (int i = 0; i < 3; i++) {
        a.in[i] = (const T *)ha.in[i];
        a.ld[i] = ha.ld[i];
        a.k[i] = ha.k[i];
        a.cols[i] = ha.cols[i];
        if (i < ha.nin) a.ksum += ha.k[i];
    }
    a.nin = ha.nin;
    a.kout = ha.kout;
    a.C = (const T *)ha.C;
    a.add = (const T *)ha.add;
    a.out = (T *)ha.out;
    a.out2 = (T *)ha.out2;
    a.N = ha.N;
    const size_t shm = (size_t)a.ksum * a.kout * sizeof(T) + (size_t)a.ksum * sizeof(int) + 16;
    const i64 total = a.N * (a.kout / V);
    if (ha.out2)
        hipLaunchKernelGGL((combine_kernel<T, V, true>), dim3(stride_blocks(total)), dim3(256), shm, st, a);
    else
        hipLaunchKernelGGL((combine_kernel<T, V, false>), dim3(stride_blocks(total)), dim3(256), shm, st, a);
    return hipGetLastError();
}

hipError_t launch_combine(int dtype, const CombineArgs &a, hipStream_t st)
{
    if (a.N == 0 || a.kout == 0) return hipSuccess;
    if (dtype == DT_F32) {
        switch (pick_vec<float>(a.kout)) {
        case 4: return run_combine<float, 4>(a, st);
        case 2: return run_combine<float, 2>(a, st);
        default: return run_combine<float, 1>(a, st);
        }
    }
    if (pick_vec<double>(a.kout) == 2) return run_combine<double, 2>(a, st);
    return run_combine<double, 1>(a, st);
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

__global__ void __launch_bounds__(256) reduce_partials_kernel(const double *__restrict__ partials, int nb, int width,
                                                              double *__restrict__ out)
{
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < width; e += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nb; b++) s += partials[(i64)b * width + e];
        out[e] = s;
    }
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
    hipLaunchKernelGGL(reduce_partials_kernel, dim3((2 * a.m + 255) / 256), dim3(256), 0, st, a.partials, nb,
                       2 * a.m, a.out);
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
