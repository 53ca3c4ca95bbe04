// Block stencil products on point-major N x k blocks (gfx950).
//
// A u for the 7-point Laplacian (Section 4) and for -div(k grad u), applied to
// all k columns of a block at once (the block product A*W of step 12).  The
// same kernel, with a different epilogue, gives the multigrid smoother and
// residual (weighted Jacobi on the level operator s*L7, s = 4^-l).
//
// Mapping: one thread owns V consecutive columns of R adjacent y-rows of one
// x position and marches in z, so the z-1 / z / z+1 values stay in registers
// and every element is fetched from HBM once; the y-neighbours between its
// rows come from registers too.  The x-1 / x+1 neighbours are the centre
// values of lanes -L / +L of the same wave and are exchanged by cross-lane
// shuffles (only lanes at a wave edge load them); the y-neighbours beyond the
// thread's rows are the centre values of threads of the same or a nearby
// workgroup, fetched through L1/L2.  Workgroups are remapped so that each XCD
// owns a contiguous range of (x, y) tiles.
#include "common.h"
#include "kernels.h"

namespace lobpcg {

enum { EPI_APPLY = 0, EPI_JACOBI = 1, EPI_RESID = 2, EPI_JACOBI2 = 3, EPI_MASS = 4 };

template <typename T, int V>
__device__ __forceinline__ vec<T, V> lap(const vec<T, V> &c, const vec<T, V> &zm, const vec<T, V> &zp,
                                         const vec<T, V> &xm, const vec<T, V> &xp, const vec<T, V> &ym,
                                         const vec<T, V> &yp)
{
    vec<T, V> r;
#pragma unroll
    for (int i = 0; i < V; i++)
        r.v[i] = T(6) * c.v[i] - zm.v[i] - zp.v[i] - xm.v[i] - xp.v[i] - ym.v[i] - yp.v[i];
    return r;
}

// x-1 / x+1 neighbours of the centre values cur (element offset i): lanes
// -L / +L of the wave hold them when they exist (consecutive lanes hold
// consecutive (point, chunk) items of one row); lanes at a wave edge load
// them, lanes at the grid's x faces take the Dirichlet zero.  Every lane of
// the wave must call this (the shuffles are wave-wide).
// V elements of type U at p, converted to T (a 16-byte load for U = T; two
// for an FP64 row read by FP32 arithmetic)
template <typename T, int V, typename U>
__device__ __forceinline__ vec<T, V> vload_as(const U *p)
{
    const vec<U, V> a = vload<U, V>(p);
    vec<T, V> r;
#pragma unroll
    for (int q = 0; q < V; q++) r.v[q] = (T)a.v[q];
    return r;
}

// The same at an address aligned to one element only (rows of a block whose
// column count is not a multiple of V)
template <typename U, int V>
struct uvec {
    typedef U type __attribute__((ext_vector_type(V), aligned(sizeof(U))));
};
template <typename T, int V, typename U>
__device__ __forceinline__ vec<T, V> vload_as_u(const U *p)
{
    const typename uvec<U, V>::type a = *reinterpret_cast<const typename uvec<U, V>::type *>(p);
    vec<T, V> r;
#pragma unroll
    for (int q = 0; q < V; q++) r.v[q] = (T)a[q];
    return r;
}
template <typename T, int V, typename U>
__device__ __forceinline__ void vstore_as_u(U *p, const vec<T, V> &x)
{
    typename uvec<U, V>::type a;
#pragma unroll
    for (int q = 0; q < V; q++) a[q] = (U)x.v[q];
    *reinterpret_cast<typename uvec<U, V>::type *>(p) = a;
}

template <typename T, int V, typename U>
__device__ __forceinline__ void vstore_nt_as(U *p, const vec<T, V> &x)
{
    vec<U, V> a;
#pragma unroll
    for (int q = 0; q < V; q++) a.v[q] = (U)x.v[q];
    vstore_nt<U, V>(p, a);
}

// The x-1 / x+1 neighbours of lane-edge items come from ldu(i -/+ sx): the
// loader of the kernel's input layout.
template <typename T, int V, typename LD>
__device__ __forceinline__ void x_neighbours(const vec<T, V> &cur, const LD &ldu, i64 i, i64 sx, int x, int nx,
                                             int L, bool row_ok, vec<T, V> &xm, vec<T, V> &xp)
{
    const int lane = threadIdx.x & 63;
    const bool in_m = lane >= L, in_p = lane + L < 64;
#pragma unroll
    for (int q = 0; q < V; q++) {
        xm.v[q] = __shfl(cur.v[q], in_m ? lane - L : lane, 64);
        xp.v[q] = __shfl(cur.v[q], in_p ? lane + L : lane, 64);
    }
    // a row outside the grid (only the last rows of a thread's row block)
    // has no neighbours to load: its results are not stored
    if (x == 0 || !row_ok) xm = vzero<T, V>();
    else if (!in_m) xm = ldu(i - sx);
    if (x + 1 == nx || !row_ok) xp = vzero<T, V>();
    else if (!in_p) xp = ldu(i + sx);
}

// EPI_APPLY : out = s * L7 u
// EPI_JACOBI: out = u + c1 * (b - s * L7 u)
// EPI_RESID : out = b - s * L7 u
// EPI_JACOBI2: two sweeps from zero with right-hand side u:
//             x1 = c1 u, out = x1 + c1 (u - s L7 x1)
// EPI_MASS  : out = c1 u + s (sum of the six neighbours), the 7-point
//             mass-type operator B with b0 = c1, b1 = s
// The arithmetic is in T.  u may be stored as TU and out as TO (FP64 blocks
// around an FP32 multigrid: the first sweep reads the FP64 right-hand side
// and, when ucopy is given, writes its FP32 copy for the later kernels of
// the cycle; the last sweep writes the FP64 result).  CIN / COUT: u / out
// are stored with kc <= L V columns per point (a block whose column count is
// not a multiple of V, run through a cycle on L V columns: the columns past
// kc read as zero and are not stored).
template <typename T, int V, int EPI, int R, typename TU = T, typename TO = T, bool CIN = false, bool COUT = false>
__global__ void __launch_bounds__(256) stencil7_kernel(int nx, int ny, int nz, int L, int zchunk,
                                                       const TU *__restrict__ u, TO *__restrict__ out,
                                                       const T *__restrict__ b, T s, T c1, T *__restrict__ ucopy,
                                                       int kc)
{
    const unsigned nbx = gridDim.x;
    const unsigned bx = xcd_remap(blockIdx.x, nbx);
    const int nyr = (ny + R - 1) / R;                  // row blocks of R rows
    const i64 plane = (i64)nx * nyr * L;               // threads per z-plane
    const i64 t0 = (i64)bx * blockDim.x + threadIdx.x;
    // lanes past the plane stay (on the plane's last item, without storing):
    // every lane of a wave takes part in the x-neighbour exchange
    const bool active = t0 < plane;
    const i64 t = active ? t0 : plane - 1;
    const int c = (int)(t % L);
    const i64 pxy = t / L;
    const int x = (int)(pxy % nx);
    const int y0 = (int)(pxy / nx) * R;
    const int z0 = blockIdx.y * zchunk;
    const int z1 = min(nz, z0 + zchunk);
    const i64 sx = (i64)L * V, sy = (i64)nx * L * V, sz = (i64)nx * ny * L * V;   // element strides
    const i64 base = (((i64)y0 * nx + x) * L + c) * V;                           // row y0
    const vec<T, V> zero = vzero<T, V>();
    // u's layout (kc columns per point with CIN) and its loader
    const i64 ku = CIN ? (i64)kc : sx;
    const i64 sxu = ku, syu = (i64)nx * ku, szu = (i64)nx * ny * ku;
    const i64 baseu = ((i64)y0 * nx + x) * ku + (i64)c * V;
    const bool whole = !(CIN || COUT) || c * V + V <= kc;   // this thread's chunk lies inside the stored row
    auto ldu = [&](i64 iu) -> vec<T, V> {
        if constexpr (CIN) {
            if (whole) return vload_as_u<T, V>(u + iu);
            vec<T, V> r;
#pragma unroll
            for (int q = 0; q < V; q++) r.v[q] = c * V + q < kc ? (T)u[iu + q] : T(0);
            return r;
        } else {
            return vload_as<T, V>(u + iu);
        }
    };
    // out's layout (kc columns per point with COUT)
    const i64 ko = COUT ? (i64)kc : sx;
    const i64 syo = (i64)nx * ko, szo = (i64)nx * ny * ko;
    const i64 baseo = ((i64)y0 * nx + x) * ko + (i64)c * V;
    auto sto = [&](i64 io, const vec<T, V> &o) {
        if constexpr (COUT) {
            if (whole) {
                vstore_as_u<T, V>(out + io, o);
            } else {
#pragma unroll
                for (int q = 0; q < V; q++)
                    if (c * V + q < kc) out[io + q] = (TO)o.v[q];
            }
        } else {
            vstore_nt_as<T, V>(out + io, o);
        }
    };
    // rows y0 .. y0+R-1 (those inside the grid) marched in z together: the
    // y-neighbours between them come from registers, only rows y0-1 and
    // y0+R are loaded
    bool rok[R];
    vec<T, V> prev[R], cur[R];
#pragma unroll
    for (int r = 0; r < R; r++) {
        rok[r] = y0 + r < ny;
        const i64 br = baseu + r * syu;
        prev[r] = (rok[r] && z0 > 0) ? ldu(br + (z0 - 1) * szu) : zero;
        cur[r] = rok[r] ? ldu(br + z0 * szu) : zero;
    }
    for (int z = z0; z < z1; z++) {
        const i64 i = base + z * sz, iu = baseu + z * szu, io = baseo + z * szo;
        vec<T, V> next[R];
#pragma unroll
        for (int r = 0; r < R; r++) next[r] = (rok[r] && z + 1 < nz) ? ldu(iu + r * syu + szu) : zero;
        const vec<T, V> ybelow = y0 > 0 ? ldu(iu - syu) : zero;
        const vec<T, V> yabove = (y0 + R < ny) ? ldu(iu + R * syu) : zero;
#pragma unroll
        for (int r = 0; r < R; r++) {
            const i64 ir = i + r * sy;
            vec<T, V> xm, xp;
            x_neighbours<T, V>(cur[r], ldu, iu + r * syu, sxu, x, nx, L, rok[r], xm, xp);
            if (ucopy && active && rok[r]) vstore<T, V>(ucopy + ir, cur[r]);
            const vec<T, V> ym = r == 0 ? ybelow : cur[r - 1];
            const vec<T, V> yp = r == R - 1 ? yabove : cur[r + 1];
            vec<T, V> o;
            if (EPI == EPI_MASS) {
#pragma unroll
                for (int q = 0; q < V; q++)
                    o.v[q] = c1 * cur[r].v[q] +
                             s * (prev[r].v[q] + next[r].v[q] + xm.v[q] + xp.v[q] + ym.v[q] + yp.v[q]);
                if (active && rok[r]) sto(io + r * syo, o);
                continue;
            }
            vec<T, V> au = lap<T, V>(cur[r], prev[r], next[r], xm, xp, ym, yp);
            if (EPI == EPI_APPLY) {
#pragma unroll
                for (int q = 0; q < V; q++) o.v[q] = s * au.v[q];
            } else if (EPI == EPI_JACOBI2) {
#pragma unroll
                for (int q = 0; q < V; q++) o.v[q] = c1 * cur[r].v[q] + c1 * (cur[r].v[q] - s * (c1 * au.v[q]));
            } else {
                vec<T, V> bb = rok[r] ? vload<T, V>(b + ir) : zero;
#pragma unroll
                for (int q = 0; q < V; q++) {
                    T rr = bb.v[q] - s * au.v[q];
                    o.v[q] = (EPI == EPI_JACOBI) ? cur[r].v[q] + c1 * rr : rr;
                }
            }
            if (active && rok[r]) sto(io + r * syo, o);
        }
#pragma unroll
        for (int r = 0; r < R; r++) {
            prev[r] = cur[r];
            cur[r] = next[r];
        }
    }
}

// Variable-coefficient operator: (A u)_p = sum_f k_f (u_p - u_q), face arrays
// kx (nz, ny, nx+1), ky (nz, ny+1, nx), kz (nz+1, ny, nx).
template <typename T, int V>
__global__ void __launch_bounds__(256) varcoef7_kernel(int nx, int ny, int nz, int L, int zchunk,
                                                       const double *__restrict__ kx,
                                                       const double *__restrict__ ky,
                                                       const double *__restrict__ kz,
                                                       const T *__restrict__ u, T *__restrict__ out)
{
    const unsigned bx = xcd_remap(blockIdx.x, gridDim.x);
    const i64 plane = (i64)nx * ny * L;
    const i64 t0 = (i64)bx * blockDim.x + threadIdx.x;
    const bool active = t0 < plane;   // idle lanes stay for the shuffles
    const i64 t = active ? t0 : plane - 1;
    const int c = (int)(t % L);
    const i64 pxy = t / L;
    const int x = (int)(pxy % nx);
    const int y = (int)(pxy / nx);
    const int z0 = blockIdx.y * zchunk;
    const int z1 = min(nz, z0 + zchunk);
    const i64 sx = (i64)L * V, sy = (i64)nx * L * V, sz = (i64)nx * ny * L * V;
    const i64 base = (pxy * L + c) * V;
    const vec<T, V> zero = vzero<T, V>();
    vec<T, V> prev = z0 > 0 ? vload<T, V>(u + base + (z0 - 1) * sz) : zero;
    vec<T, V> cur = vload<T, V>(u + base + z0 * sz);
    for (int z = z0; z < z1; z++) {
        const i64 i = base + z * sz;
        vec<T, V> next = (z + 1 < nz) ? vload<T, V>(u + i + sz) : zero;
        vec<T, V> xm, xp;
        x_neighbours<T, V>(cur, [&](i64 j) { return vload<T, V>(u + j); }, i, sx, x, nx, L, true, xm, xp);
        vec<T, V> ym = y > 0 ? vload<T, V>(u + i - sy) : zero;
        vec<T, V> yp = y + 1 < ny ? vload<T, V>(u + i + sy) : zero;
        const i64 fxi = ((i64)z * ny + y) * (nx + 1) + x;
        const i64 fyi = ((i64)z * (ny + 1) + y) * nx + x;
        const i64 fzi = ((i64)z * ny + y) * nx + x;
        const T kxm = (T)kx[fxi], kxp = (T)kx[fxi + 1];
        const T kym = (T)ky[fyi], kyp = (T)ky[fyi + nx];
        const T kzm = (T)kz[fzi], kzp = (T)kz[fzi + (i64)nx * ny];
        vec<T, V> o;
#pragma unroll
        for (int q = 0; q < V; q++) {
            T up = cur.v[q];
            o.v[q] = kxm * (up - xm.v[q]) + kxp * (up - xp.v[q]) + kym * (up - ym.v[q]) +
                     kyp * (up - yp.v[q]) + kzm * (up - prev.v[q]) + kzp * (up - next.v[q]);
        }
        if (active) vstore_nt<T, V>(out + i, o);
        prev = cur;
        cur = next;
    }
}

// Launch geometry: 256 threads over the (x, y, column-chunk) plane, z split
// into chunks until there are about zmin workgroups (a chunk re-reads the
// two planes at its ends; on small grids they come from the caches)
static void geometry(int nx, int ny, int nz, int L, dim3 &grid, int &zchunk, int zmin = 2048)
{
    const i64 plane = (i64)nx * ny * L;
    const unsigned pb = (unsigned)((plane + 255) / 256);
    int zc = (int)((zmin + pb - 1) / pb);
    if (zc > nz) zc = nz;
    if (zc < 1) zc = 1;
    zchunk = (nz + zc - 1) / zc;
    grid = dim3(pb, (nz + zchunk - 1) / zchunk, 1);
}

template <typename T>
static int pick_vec(int k)
{
    const int maxv = 16 / (int)sizeof(T);
    for (int v = maxv; v > 1; v >>= 1)
        if (k % v == 0) return v;
    return 1;
}

// y-rows per thread and workgroup target, measured on 256^3 blocks of 8-32
// columns: rows held in registers save the y-neighbour loads of the rows
// between them, but cost registers (waves in flight).  FP32 products: two
// rows (4.4 -> 5.0 TB/s at 32 columns); FP32 sweeps and residuals, which
// also stream b, are fastest with one row (5.1 TB/s); FP64: four rows
// (products 3.8 -> 4.8 TB/s, sweeps 4.1 -> 5.2 TB/s), two for narrow
// products.
template <typename T, int V, int EPI>
static hipError_t run_stencil(const Grid3 &g, int k, const void *u, void *out, const void *b, double s, double c1,
                              hipStream_t st)
{
    const int L = k / V;
    const bool product = EPI == EPI_APPLY || EPI == EPI_MASS;
    dim3 grid;
    int zchunk;
    auto launch = [&](auto Rc, int zmin) {
        constexpr int R = decltype(Rc)::value;
        geometry(g.nx, (g.ny + R - 1) / R, g.nz, L, grid, zchunk, zmin);
        hipLaunchKernelGGL((stencil7_kernel<T, V, EPI, R>), grid, dim3(256), 0, st, g.nx, g.ny, g.nz, L, zchunk,
                           (const T *)u, (T *)out, (const T *)b, (T)s, (T)c1, (T *)nullptr, 0);
    };
    if (sizeof(T) == 8) {
        if (product && k < 16) launch(std::integral_constant<int, 2>(), 8192);
        else launch(std::integral_constant<int, 4>(), product ? 4096 : 8192);
    } else {
        // the two sweeps from zero read one block, as a product does
        if (product || EPI == EPI_JACOBI2) launch(std::integral_constant<int, 2>(), 8192);
        else launch(std::integral_constant<int, 1>(), 2048);
    }
    return hipGetLastError();
}

template <typename T, int EPI>
static hipError_t dispatch_vec(const Grid3 &g, int k, const void *u, void *out, const void *b, double s,
                               double c1, hipStream_t st)
{
    switch (pick_vec<T>(k)) {
    case 4: return run_stencil<T, 4, EPI>(g, k, u, out, b, s, c1, st);
    case 2: return run_stencil<T, 2, EPI>(g, k, u, out, b, s, c1, st);
    default: return run_stencil<T, 1, EPI>(g, k, u, out, b, s, c1, st);
    }
}

template <typename T>
static hipError_t dispatch_epi(int epi, const Grid3 &g, int k, const void *u, void *out, const void *b,
                               double s, double c1, hipStream_t st)
{
    switch (epi) {
    case EPI_APPLY: return dispatch_vec<T, EPI_APPLY>(g, k, u, out, b, s, c1, st);
    case EPI_JACOBI: return dispatch_vec<T, EPI_JACOBI>(g, k, u, out, b, s, c1, st);
    case EPI_JACOBI2: return dispatch_vec<T, EPI_JACOBI2>(g, k, u, out, b, s, c1, st);
    case EPI_MASS: return dispatch_vec<T, EPI_MASS>(g, k, u, out, b, s, c1, st);
    default: return dispatch_vec<T, EPI_RESID>(g, k, u, out, b, s, c1, st);
    }
}

hipError_t launch_laplace7(int dtype, const Grid3 &g, int k, const void *u, void *out, double s, hipStream_t st)
{
    if (dtype == DT_F32) return dispatch_epi<float>(EPI_APPLY, g, k, u, out, nullptr, s, 0.0, st);
    return dispatch_epi<double>(EPI_APPLY, g, k, u, out, nullptr, s, 0.0, st);
}

hipError_t launch_mass7(int dtype, const Grid3 &g, int k, double b0, double b1, const void *u, void *out,
                        hipStream_t st)
{
    if (dtype == DT_F32) return dispatch_epi<float>(EPI_MASS, g, k, u, out, nullptr, b1, b0, st);
    return dispatch_epi<double>(EPI_MASS, g, k, u, out, nullptr, b1, b0, st);
}

hipError_t launch_jacobi(int dtype, const Grid3 &g, int k, const void *x, const void *b, void *out, double s,
                         double omega, hipStream_t st)
{
    const double c1 = omega / (6.0 * s);
    if (dtype == DT_F32) return dispatch_epi<float>(EPI_JACOBI, g, k, x, out, b, s, c1, st);
    return dispatch_epi<double>(EPI_JACOBI, g, k, x, out, b, s, c1, st);
}

hipError_t launch_jacobi2_zero(int dtype, const Grid3 &g, int k, const void *b, void *out, double s, double omega,
                               hipStream_t st)
{
    const double c1 = omega / (6.0 * s);
    if (dtype == DT_F32) return dispatch_epi<float>(EPI_JACOBI2, g, k, b, out, nullptr, s, c1, st);
    return dispatch_epi<double>(EPI_JACOBI2, g, k, b, out, nullptr, s, c1, st);
}

hipError_t launch_resid7(int dtype, const Grid3 &g, int k, const void *x, const void *b, void *out, double s,
                         hipStream_t st)
{
    if (dtype == DT_F32) return dispatch_epi<float>(EPI_RESID, g, k, x, out, b, s, 0.0, st);
    return dispatch_epi<double>(EPI_RESID, g, k, x, out, b, s, 0.0, st);
}

// The first and last sweeps of a cycle whose blocks differ from the cycle's
// (precision T, k = L V columns per point): the right-hand side u is read
// as stored (type TU, kc <= k columns) and its copy in the cycle's layout
// written to ucopy; the result is written as stored (type TO, kc columns).
// Shapes of the sweeps above: one row per thread for FP32 (two for the
// sweeps from zero, which read one block), four for FP64.
template <typename T, int V, int EPI, typename TU, typename TO, bool CIN, bool COUT>
static hipError_t run_edge_sweep(const Grid3 &g, int kc, int k, const void *u, void *out, const void *b, T *ucopy,
                                 double s, double c1, hipStream_t st)
{
    const int L = k / V;
    constexpr int R = sizeof(T) == 4 ? (EPI == EPI_JACOBI2 ? 2 : 1) : 4;
    dim3 grid;
    int zchunk;
    geometry(g.nx, (g.ny + R - 1) / R, g.nz, L, grid, zchunk, sizeof(T) == 4 && R == 1 ? 2048 : 8192);
    hipLaunchKernelGGL((stencil7_kernel<T, V, EPI, R, TU, TO, CIN, COUT>), grid, dim3(256), 0, st, g.nx, g.ny, g.nz,
                       L, zchunk, (const TU *)u, (TO *)out, (const T *)b, (T)s, (T)c1, ucopy, kc);
    return hipGetLastError();
}

// V for a cycle on k columns of T: the widest 16-byte vector that divides k
template <typename T, int EPI, typename TU, typename TO, bool CIN, bool COUT>
static hipError_t edge_sweep_v(const Grid3 &g, int kc, int k, const void *u, void *out, const void *b, T *ucopy,
                               double s, double c1, hipStream_t st)
{
    if constexpr (sizeof(T) == 4) {
        switch (pick_vec<T>(k)) {
        case 4: return run_edge_sweep<T, 4, EPI, TU, TO, CIN, COUT>(g, kc, k, u, out, b, ucopy, s, c1, st);
        case 2: return run_edge_sweep<T, 2, EPI, TU, TO, CIN, COUT>(g, kc, k, u, out, b, ucopy, s, c1, st);
        default: return run_edge_sweep<T, 1, EPI, TU, TO, CIN, COUT>(g, kc, k, u, out, b, ucopy, s, c1, st);
        }
    } else {
        if (pick_vec<T>(k) == 2) return run_edge_sweep<T, 2, EPI, TU, TO, CIN, COUT>(g, kc, k, u, out, b, ucopy, s, c1, st);
        return run_edge_sweep<T, 1, EPI, TU, TO, CIN, COUT>(g, kc, k, u, out, b, ucopy, s, c1, st);
    }
}

hipError_t launch_jacobi2_zero_in(int dt_in, int dtype, const Grid3 &g, int kc, int k, const void *bsrc, void *x,
                                  void *bcopy, double s, double omega, hipStream_t st)
{
    if (kc < 1 || kc > k) return hipErrorInvalidValue;
    const double c1 = omega / (6.0 * s);
    const bool cin = kc < k;
    if (dtype == DT_F32) {
        float *bc = (float *)bcopy;
        if (dt_in == DT_F64)
            return cin ? edge_sweep_v<float, EPI_JACOBI2, double, float, true, false>(g, kc, k, bsrc, x, nullptr, bc, s, c1, st)
                       : edge_sweep_v<float, EPI_JACOBI2, double, float, false, false>(g, kc, k, bsrc, x, nullptr, bc, s, c1, st);
        return cin ? edge_sweep_v<float, EPI_JACOBI2, float, float, true, false>(g, kc, k, bsrc, x, nullptr, bc, s, c1, st)
                   : edge_sweep_v<float, EPI_JACOBI2, float, float, false, false>(g, kc, k, bsrc, x, nullptr, bc, s, c1, st);
    }
    if (dt_in != DT_F64) return hipErrorInvalidValue;
    double *bc = (double *)bcopy;
    return cin ? edge_sweep_v<double, EPI_JACOBI2, double, double, true, false>(g, kc, k, bsrc, x, nullptr, bc, s, c1, st)
               : edge_sweep_v<double, EPI_JACOBI2, double, double, false, false>(g, kc, k, bsrc, x, nullptr, bc, s, c1, st);
}

hipError_t launch_jacobi_out(int dtype, int dt_out, const Grid3 &g, int kc, int k, const void *x, const void *b,
                             void *out, double s, double omega, hipStream_t st)
{
    if (kc < 1 || kc > k) return hipErrorInvalidValue;
    const double c1 = omega / (6.0 * s);
    const bool cout = kc < k;
    if (dtype == DT_F32) {
        if (dt_out == DT_F64)
            return cout ? edge_sweep_v<float, EPI_JACOBI, float, double, false, true>(g, kc, k, x, out, b, nullptr, s, c1, st)
                        : edge_sweep_v<float, EPI_JACOBI, float, double, false, false>(g, kc, k, x, out, b, nullptr, s, c1, st);
        return cout ? edge_sweep_v<float, EPI_JACOBI, float, float, false, true>(g, kc, k, x, out, b, nullptr, s, c1, st)
                    : edge_sweep_v<float, EPI_JACOBI, float, float, false, false>(g, kc, k, x, out, b, nullptr, s, c1, st);
    }
    if (dt_out != DT_F64) return hipErrorInvalidValue;
    return cout ? edge_sweep_v<double, EPI_JACOBI, double, double, false, true>(g, kc, k, x, out, b, nullptr, s, c1, st)
                : edge_sweep_v<double, EPI_JACOBI, double, double, false, false>(g, kc, k, x, out, b, nullptr, s, c1, st);
}

template <typename T, int V>
static hipError_t run_varcoef(const Grid3 &g, int k, const double *kx, const double *ky, const double *kz,
                              const void *u, void *out, hipStream_t st)
{
    const int L = k / V;
    dim3 grid;
    int zchunk;
    geometry(g.nx, g.ny, g.nz, L, grid, zchunk);
    hipLaunchKernelGGL((varcoef7_kernel<T, V>), grid, dim3(256), 0, st, g.nx, g.ny, g.nz, L, zchunk, kx, ky, kz,
                       (const T *)u, (T *)out);
    return hipGetLastError();
}

hipError_t launch_varcoef7(int dtype, const Grid3 &g, int k, const double *kx, const double *ky,
                           const double *kz, const void *u, void *out, hipStream_t st)
{
    if (dtype == DT_F32) {
        switch (pick_vec<float>(k)) {
        case 4: return run_varcoef<float, 4>(g, k, kx, ky, kz, u, out, st);
        case 2: return run_varcoef<float, 2>(g, k, kx, ky, kz, u, out, st);
        default: return run_varcoef<float, 1>(g, k, kx, ky, kz, u, out, st);
        }
    }
    switch (pick_vec<double>(k)) {
    case 2: return run_varcoef<double, 2>(g, k, kx, ky, kz, u, out, st);
    default: return run_varcoef<double, 1>(g, k, kx, ky, kz, u, out, st);
    }
}

}  // namespace lobpcg
