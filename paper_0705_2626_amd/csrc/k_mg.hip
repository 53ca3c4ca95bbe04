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

// Launch shape of the transfer kernels: one thread per (x, y) column of the
// output level and V-column chunk, marching in z over a chunk of planes; the
// planes are split into enough chunks to give about 2048 workgroups.
static void march_geometry(int nx, int ny, int nz, int L, dim3 &grid, int &zchunk)
{
    const i64 plane = (i64)nx * ny * L;
    const unsigned pb = (unsigned)((plane + 255) / 256);
    int zc = (int)((2048 + pb - 1) / pb);
    if (zc < 1) zc = 1;
    if (zc > nz) zc = nz;
    zchunk = (nz + zc - 1) / zc;
    grid = dim3(pb, (nz + zchunk - 1) / zchunk, 1);
}

// bc at coarse node (X, Y, Z) = sum over the 27 fine nodes (2X+a, 2Y+b, 2Z+c),
// a, b, c in {0, 1, 2}, of w_a w_b w_c rf / 64 with w = (1, 2, 1); fine
// nodes beyond the grid are zero.  The thread of coarse column (X, Y) forms
// the in-plane 3x3 sum of each fine plane once and combines three of them
// per coarse plane (the plane 2Z+2 is shared with Z+1).
template <typename T, int V>
__global__ void __launch_bounds__(256) restrict_kernel(int nxf, int nyf, int nzf, int nxc, int nyc, int nzc, int L,
                                                       int zchunk, const T *__restrict__ rf, T *__restrict__ bc)
{
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (unsigned)(nxc * nyc * L)) return;
    const int c = (int)(t % (unsigned)L);
    const unsigned pxy = t / (unsigned)L;
    const int X = (int)(pxy % (unsigned)nxc), Y = (int)(pxy / (unsigned)nxc);
    const int Z0 = blockIdx.y * zchunk, Z1 = min(nzc, Z0 + zchunk);
    const i64 k = (i64)L * V;
    const i64 fplane = (i64)nxf * nyf;
    auto plane_sum = [&](int zf) {
        vec<T, V> s = vzero<T, V>();
        if (zf >= nzf) return s;
#pragma unroll
        for (int b = 0; b < 3; b++) {
            const int yf = 2 * Y + b;
            if (yf >= nyf) continue;
            const T wb = b == 1 ? T(2) : T(1);
#pragma unroll
            for (int a = 0; a < 3; a++) {
                const int xf = 2 * X + a;
                if (xf >= nxf) continue;
                const T w = wb * (a == 1 ? T(2) : T(1));
                const vec<T, V> r = vload<T, V>(rf + ((i64)xf + (i64)nxf * yf + fplane * zf) * k + c * V);
#pragma unroll
                for (int q = 0; q < V; q++) s.v[q] += w * r.v[q];
            }
        }
        return s;
    };
    vec<T, V> s0 = plane_sum(2 * Z0);
    const i64 cplane = (i64)nxc * nyc;
    for (int Z = Z0; Z < Z1; Z++) {
        const vec<T, V> s1 = plane_sum(2 * Z + 1), s2 = plane_sum(2 * Z + 2);
        vec<T, V> o;
#pragma unroll
        for (int q = 0; q < V; q++) o.v[q] = (s0.v[q] + T(2) * s1.v[q] + s2.v[q]) * T(1.0 / 64.0);
        vstore<T, V>(bc + ((i64)X + (i64)nxc * Y + cplane * Z) * k + c * V, o);
        s0 = s2;
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

// xf += P ec.  The thread of fine column (x, y) forms the bilinear in-plane
// interpolation q(I) of each coarse plane I once; fine plane 2I+1 takes q(I),
// fine plane 2I takes (q(I-1) + q(I))/2 (q of a plane beyond the grid is 0).
template <typename T, int V>
__global__ void __launch_bounds__(256) prolong_add_kernel(int nxf, int nyf, int nzf, int nxc, int nyc, int nzc,
                                                          int L, int zchunk, const T *__restrict__ ec,
                                                          T *__restrict__ xf)
{
    const unsigned t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (unsigned)(nxf * nyf * L)) return;
    const int c = (int)(t % (unsigned)L);
    const unsigned pxy = t / (unsigned)L;
    const int x = (int)(pxy % (unsigned)nxf), y = (int)(pxy / (unsigned)nxf);
    const int z0 = blockIdx.y * zchunk, z1 = min(nzf, z0 + zchunk);
    const i64 k = (i64)L * V;
    int Ix[2], Iy[2];
    float wx[2], wy[2];
    const int nxt = prolong_1d(x, nxc, Ix, wx), nyt = prolong_1d(y, nyc, Iy, wy);
    const i64 cplane = (i64)nxc * nyc;
    auto q = [&](int I) {
        vec<T, V> s = vzero<T, V>();
        if (I < 0 || I >= nzc) return s;
        for (int b = 0; b < nyt; b++)
            for (int a = 0; a < nxt; a++) {
                const T w = (T)(wx[a] * wy[b]);
                const vec<T, V> e = vload<T, V>(ec + ((i64)Ix[a] + (i64)nxc * Iy[b] + cplane * I) * k + c * V);
#pragma unroll
                for (int r = 0; r < V; r++) s.v[r] += w * e.v[r];
            }
        return s;
    };
    int Ic = -2;          // coarse plane held in qc
    vec<T, V> qc = vzero<T, V>();
    const i64 fplane = (i64)nxf * nyf;
    for (int z = z0; z < z1; z++) {
        vec<T, V> val;
        if (z & 1) {
            const int I = (z - 1) >> 1;
            if (I != Ic) qc = q(I), Ic = I;
            val = qc;
        } else {
            const int I = z >> 1;
            const vec<T, V> qa = (Ic == I - 1) ? qc : q(I - 1);
            qc = q(I), Ic = I;
#pragma unroll
            for (int r = 0; r < V; r++) val.v[r] = T(0.5) * (qa.v[r] + qc.v[r]);
        }
        T *dst = xf + ((i64)x + (i64)nxf * y + fplane * z) * k + c * V;
        vec<T, V> o = vload<T, V>(dst);
#pragma unroll
        for (int r = 0; r < V; r++) o.v[r] += val.v[r];
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
    dim3 grid;
    int zchunk;
    march_geometry(c.nx, c.ny, c.nz, L, grid, zchunk);
    hipLaunchKernelGGL((restrict_kernel<T, V>), grid, dim3(256), 0, st, f.nx, f.ny, f.nz, c.nx, c.ny, c.nz, L,
                       zchunk, (const T *)rf, (T *)bc);
    return hipGetLastError();
}

template <typename T, int V>
static hipError_t run_prolong(const Grid3 &f, const Grid3 &c, int k, const void *ec, void *xf, hipStream_t st)
{
    const int L = k / V;
    dim3 grid;
    int zchunk;
    march_geometry(f.nx, f.ny, f.nz, L, grid, zchunk);
    hipLaunchKernelGGL((prolong_add_kernel<T, V>), grid, dim3(256), 0, st, f.nx, f.ny, f.nz, c.nx, c.ny, c.nz, L,
                       zchunk, (const T *)ec, (T *)xf);
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
    if (f.n() == 0) return hipSuccess;
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
