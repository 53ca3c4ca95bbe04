// Multivector products on MFMA: out = sum_i in_i[:, cols_i] C_i for point-major
// N x k blocks (gfx950).
//
// This is the "X*C" of LOBPCG: the Cholesky orthonormalisations X R^-1,
// W_J R^-1, P_J R^-1, AP_J R^-1 (steps 3, 11, 14-15), the initial Ritz rotation
// (step 4), and the Ritz-vector update of steps 25-33, which it fuses:
// one pass over [X, W_J, P_J] and [AX, AW_J, AP_J] writes
//   P = W_J C_W + P_J C_P,  X' = X C_X + P        (side 0)
//   AP = AW_J C_W + AP_J C_P, AX' = AX C_X + AP   (side 1)
// (P and AP only in the columns that stay active) and, from X' and AX' still
// in registers, the next residual W = AX' - X' Theta of step 7 with the FP64
// column sums of squares that decide the active set of step 8.
//
// A workgroup (4 waves) walks tiles of 64 grid points; every input block of a
// tile is staged in LDS with a coalesced pass and each wave multiplies its 16
// points by the coefficients (also in LDS) with 16x16x4 MFMA, NT 16-column
// output tiles at a time.  Per-workgroup partial sums of the norms are added in
// a fixed order by a second kernel.
#include "common.h"
#include "kernels.h"
#include "mfma.h"

namespace lobpcg {

static const int TP = 64;          // grid points per tile
static const int MAXW = 32;        // widest input row staged (stored columns)
static const int LDT = MAXW + 1;   // LDS row stride: odd, so the 16 rows of an A fragment hit 16 banks
static const int MV_MAX_BLOCKS = 4096;

template <typename T>
struct MVDev {
    const T *in[2][3];
    int ld[3], k[3];
    const int *cols[3];
    int nin, nside, kout, K, Kp;
    const T *C;
    const T *add;
    T *out[2];
    const int *opos;
    int nout;
    T *out2[2];
    const double *theta;
    const int *wpos;
    T *Wout;
    int nW;
    double *partials;
    i64 N;
};

// A tile of an input block: rows p0 .. p0+63 of an N x ld block, i.e. the
// contiguous run of 64*ld elements at src + p0*ld.  It is loaded into
// registers (16-byte vectors, at most NV per thread) one stage ahead of its
// use, so that the loads of the next stage are in flight while the current
// stage computes, and then written into tile[64][LDT].
template <typename T>
struct StageRegs {
    static const int VE = 16 / sizeof(T);
    static const int NV = TP * MAXW / VE / 256;
    vec<T, VE> v[NV];
};

template <typename T>
__device__ __forceinline__ void stage_load(StageRegs<T> &R, const T *__restrict__ src, int ld, i64 p0, i64 N)
{
    const int VE = StageRegs<T>::VE;
    const i64 rows = (N - p0) < TP ? (N - p0) : TP;
    const int nvec = TP * ld / VE, nvalid = (int)(rows * ld);
    const T *s = src + p0 * ld;
#pragma unroll
    for (int i = 0; i < StageRegs<T>::NV; i++) {
        const int vi = threadIdx.x + 256 * i;
        if (vi >= nvec) break;
        const int e0 = vi * VE;
        if (e0 + VE <= nvalid) {
            R.v[i] = vload<T, VE>(s + e0);
        } else {
#pragma unroll
            for (int q = 0; q < VE; q++) R.v[i].v[q] = (e0 + q < nvalid) ? s[e0 + q] : T(0);
        }
    }
}

template <typename T>
__device__ __forceinline__ void stage_store(T *tile, const StageRegs<T> &R, int ld)
{
    const int VE = StageRegs<T>::VE;
    const int nvec = TP * ld / VE;
    const float inv = 1.0f / (float)ld;
#pragma unroll
    for (int i = 0; i < StageRegs<T>::NV; i++) {
        const int vi = threadIdx.x + 256 * i;
        if (vi >= nvec) break;
#pragma unroll
        for (int q = 0; q < VE; q++) {
            const int e = vi * VE + q;
            // e < 64*32: the float quotient is within 2e-4 of e/ld, and
            // (e + 0.5)/ld is at least 0.5/32 away from an integer
            const int row = (int)(((float)e + 0.5f) * inv);
            tile[row * LDT + e - row * ld] = R.v[i].v[q];
        }
    }
}

template <typename T, int NT>
__device__ __forceinline__ void mma_input(typename Mfma<T>::acc *acc, const T *tile, const T *Cs, const int *cmap,
                                          int roff, int k, int wave, int lane)
{
    const int NC = NT * 16;
    const T *arow = tile + (16 * wave + (lane & 15)) * LDT;
    for (int k0 = 0; k0 < k; k0 += 4) {
        const int kr = k0 + (lane >> 4);
        const bool ok = kr < k;
        const T av = ok ? arow[cmap[roff + kr]] : T(0);
        const T *crow = Cs + (roff + kr) * NC + (lane & 15);
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            const T bv = ok ? crow[16 * nt] : T(0);
            acc[nt] = Mfma<T>::mma(av, bv, acc[nt]);
        }
    }
}

template <typename T, int NT>
__global__ void __launch_bounds__(256) mv_kernel(MVDev<T> a)
{
    typedef typename Mfma<T>::acc accT;
    const int NC = NT * 16;
    extern __shared__ unsigned char smem[];
    T *tile = reinterpret_cast<T *>(smem);
    T *Cs = tile + TP * LDT;
    double *theta = reinterpret_cast<double *>(Cs + (a.Kp + 4) * NC);
    double *red = theta + NC;                               // [16 slots][2][NC]
    int *cmap = reinterpret_cast<int *>(red + 16 * 2 * NC); // [K + 4]
    int *opos = cmap + a.K + 4;
    int *wpos = opos + NC;

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    for (int i = tid; i < (a.Kp + 4) * NC; i += blockDim.x) {
        const int r = i / NC, c = i % NC;
        Cs[i] = (r < a.K && c < a.kout) ? a.C[r * a.kout + c] : T(0);
    }
    {
        int roff = 0;
        for (int b = 0; b < a.nin; b++) {
            for (int r = tid; r < a.k[b]; r += blockDim.x) cmap[roff + r] = a.cols[b] ? a.cols[b][r] : r;
            roff += a.k[b];
        }
        for (int r = tid; r < 4; r += blockDim.x) cmap[a.K + r] = 0;
    }
    for (int c = tid; c < NC; c += blockDim.x) {
        opos[c] = c < a.kout ? (a.opos ? a.opos[c] : c) : -1;
        wpos[c] = (c < a.kout && a.wpos) ? a.wpos[c] : -1;
        theta[c] = (c < a.kout && a.theta) ? a.theta[c] : 0.0;
    }
    int roffs[3];
    roffs[0] = 0;
    roffs[1] = a.k[0];
    roffs[2] = a.k[0] + a.k[1];
    __syncthreads();

    const bool has2 = a.out2[0] != nullptr;
    const bool resid = a.partials != nullptr;
    double sr[NT], sx[NT];
#pragma unroll
    for (int nt = 0; nt < NT; nt++) sr[nt] = sx[nt] = 0.0;

    // the stages of one tile, in order: per side, inputs 1.. then 0 when a
    // second output is formed (input 0 is added on top for out2), else 0..
    int order[3];
    for (int q = 0; q < a.nin; q++) order[q] = has2 ? (q + 1) % a.nin : q;
    const int per_tile = a.nside * a.nin;
    const i64 ntiles = (a.N + TP - 1) / TP;
    i64 t = blockIdx.x;
    StageRegs<T> R;
    if (t < ntiles) stage_load<T>(R, a.in[0][order[0]], a.ld[order[0]], t * TP, a.N);
    accT acc[NT], acc2[NT], keepX[NT];
    int st = 0;   // stage index within the tile
    while (t < ntiles) {
        const i64 p0 = t * TP;
        const int s = st / a.nin, b = order[st % a.nin];
        if (st % a.nin == 0) {
#pragma unroll
            for (int nt = 0; nt < NT; nt++) acc[nt] = acc_zero<T>(), acc2[nt] = acc_zero<T>();
        }
        if (has2 && b == 0) {
#pragma unroll
            for (int nt = 0; nt < NT; nt++) acc2[nt] = acc[nt];
        }
        __syncthreads();
        stage_store<T>(tile, R, a.ld[b]);
        // prefetch the next stage (of this tile or the next one)
        {
            int ns = st + 1;
            i64 nt2 = t;
            if (ns == per_tile) ns = 0, nt2 = t + gridDim.x;
            if (nt2 < ntiles) {
                const int nb2 = order[ns % a.nin];
                stage_load<T>(R, a.in[ns / a.nin][nb2], a.ld[nb2], nt2 * TP, a.N);
            }
        }
        __syncthreads();
        mma_input<T, NT>((has2 && b == 0) ? acc2 : acc, tile, Cs, cmap, roffs[b], a.k[b], wave, lane);
        if (st % a.nin == a.nin - 1) {
            // outputs of side s
            T *out = a.out[s], *out2 = a.out2[s];
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const i64 p = p0 + 16 * wave + Mfma<T>::row(lane, r);
                if (p >= a.N) continue;
#pragma unroll
                for (int nt = 0; nt < NT; nt++) {
                    const int c = 16 * nt + (lane & 15);
                    if (c >= a.kout) continue;
                    T v = acc[nt][r];
                    if (a.add && s == 0) v += a.add[p * a.kout + c];
                    const int q = opos[c];
                    if (out && q >= 0) out[p * a.nout + q] = v;
                    if (has2) out2[p * a.kout + c] = acc2[nt][r];
                    if (resid && s == 1) {
                        const double x = (double)keepX[nt][r];
                        const double rv = (double)acc2[nt][r] - theta[c] * x;
                        sr[nt] += rv * rv;
                        sx[nt] += x * x;
                        const int w = wpos[c];
                        if (w >= 0) a.Wout[p * a.nW + w] = (T)rv;
                    }
                }
            }
            if (s == 0) {
#pragma unroll
                for (int nt = 0; nt < NT; nt++) keepX[nt] = acc2[nt];
            }
        }
        if (++st == per_tile) st = 0, t += gridDim.x;
    }
    if (resid) {
        // lanes l, l+16, l+32, l+48 of every wave share column l % 16 + 16 nt
        const int slot = wave * 4 + (lane >> 4);
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            const int c = 16 * nt + (lane & 15);
            red[(slot * 2 + 0) * NC + c] = sr[nt];
            red[(slot * 2 + 1) * NC + c] = sx[nt];
        }
        __syncthreads();
        for (int e = tid; e < 2 * a.kout; e += blockDim.x) {
            const int which = e / a.kout, c = e % a.kout;
            double s = 0.0;
            for (int sl = 0; sl < 16; sl++) s += red[(sl * 2 + which) * NC + c];
            a.partials[(i64)blockIdx.x * 2 * a.kout + e] = s;
        }
    }
}

// sums[e] = sum over workgroups of partials[b][e]: one workgroup per entry,
// strided partial sums then a fixed-shape tree, so the order never changes.
__global__ void __launch_bounds__(256) mv_reduce_kernel(const double *__restrict__ partials, int nb, int width,
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

int mv_blocks(long long N)
{
    long long nt = (N + TP - 1) / TP;
    return (int)(nt < MV_MAX_BLOCKS ? (nt > 0 ? nt : 1) : MV_MAX_BLOCKS);
}

template <typename T, int NT>
static hipError_t run_mv(const MVArgs &h, hipStream_t st)
{
    MVDev<T> a;
    a.K = 0;
    for (int b = 0; b < 3; b++) {
        for (int s = 0; s < 2; s++) a.in[s][b] = (const T *)h.in[s][b];
        a.ld[b] = h.ld[b];
        a.k[b] = b < h.nin ? h.k[b] : 0;
        a.cols[b] = h.cols[b];
        a.K += a.k[b];
    }
    a.nin = h.nin;
    a.nside = h.nside;
    a.kout = h.kout;
    a.Kp = (a.K + 3) / 4 * 4;
    a.C = (const T *)h.C;
    a.add = (const T *)h.add;
    for (int s = 0; s < 2; s++) {
        a.out[s] = (T *)h.out[s];
        a.out2[s] = (T *)h.out2[s];
    }
    a.opos = h.opos;
    a.nout = h.opos ? h.nout : h.kout;
    a.theta = h.theta;
    a.wpos = h.wpos;
    a.Wout = (T *)h.Wout;
    a.nW = h.nW;
    a.partials = h.partials;
    a.N = h.N;
    const int NC = NT * 16;
    size_t shm = (size_t)TP * LDT * sizeof(T) + (size_t)(a.Kp + 4) * NC * sizeof(T);
    shm = (shm + 7) / 8 * 8 + (size_t)NC * 8 + (size_t)16 * 2 * NC * 8 + (size_t)(a.K + 4 + 2 * NC) * sizeof(int);
    const int nb = mv_blocks(h.N);
    hipLaunchKernelGGL((mv_kernel<T, NT>), dim3(nb), dim3(256), shm, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !h.partials) return e;
    hipLaunchKernelGGL(mv_reduce_kernel, dim3(2 * h.kout), dim3(256), 0, st, h.partials, nb, 2 * h.kout, h.sums);
    return hipGetLastError();
}

hipError_t launch_mv(int dtype, const MVArgs &a, hipStream_t st)
{
    if (a.N == 0) return hipSuccess;
    for (int b = 0; b < a.nin; b++)
        if (a.ld[b] > MAXW || a.ld[b] < 1) return hipErrorInvalidValue;
    if (a.kout < 1 || a.kout > 32) return hipErrorInvalidValue;
    if (a.partials && (a.nside != 2 || !a.out2[0])) return hipErrorInvalidValue;
    const bool two = a.kout > 16;
    if (dtype == DT_F32) return two ? run_mv<float, 2>(a, st) : run_mv<float, 1>(a, st);
    return two ? run_mv<double, 2>(a, st) : run_mv<double, 1>(a, st);
}

}  // namespace lobpcg
