// Tall-skinny Gram products of LOBPCG on MFMA (gfx950).
//
// The Rayleigh-Ritz matrices of steps 17-23 and the Cholesky Gram matrices
// of steps 3, 11 and 14 are all entries of Lm^T Rm, where the columns of the
// N x KL matrix Lm and of the N x KR matrix Rm are columns of the blocks X,
// W_J, P_J, AX, AW_J, AP_J.  The host lists the columns of Lm and Rm (so that
// thin blocks can share one 16-column MFMA tile: Rm = [W P AW AP] in the
// paper's form) and the 16 x 16 tiles of Lm^T Rm that hold a needed entry.
//
// Each wave computes up to GX_MAXB tiles that share one 16-column block of
// Lm, with 16x16x4 MFMA whose operands are loaded straight from global
// memory: at k-step q lane l holds Lm[4q + l/16][16a + l%16] and
// Rm[4q + l/16][16b + l%16], 16 consecutive elements of a row for 16 lanes.
// There is no workgroup barrier in the main loop; waves of a workgroup walk
// the same rows, so operand blocks shared by several waves are served by the
// cache.  FP64 blocks accumulate in FP64 throughout; FP32 blocks use FP32
// MFMA within one 64-row chunk, then add the chunk into FP64 accumulators.
// Per-workgroup partial tiles are summed in a fixed order by a second
// kernel: results are reproducible bit for bit.
#include "common.h"
#include "kernels.h"
#include "mfma.h"

#include <algorithm>

namespace lobpcg {

static const int GX_WAVES = 4;
static const int GX_CH = 64;              // rows per chunk (16 k-steps)
static const int GX_BLOCKS = 1024;

template <typename T>
struct GXDev {
    const T *arr[GX_MAX_ARR];
    int ld[GX_MAX_ARR];
    int KL, KR;
    unsigned short lmap[GX_MAX_L], rmap[GX_MAX_R];   // (array << 8) | column
    int ngroups, ntiles;
    unsigned char ga[GX_MAX_TILES];                 // per group: Lm block
    unsigned char gtile[GX_MAX_TILES][GX_MAXB];     // per group: its tiles (255: an empty slot)
    unsigned char tb[GX_MAX_TILES];                 // per tile: Rm block
    i64 N;
    double *partials;   // [gridDim.x][ntiles][256]
};

template <typename T, int NT, int UNR>
__global__ void __launch_bounds__(256) gramx_kernel(GXDev<T> a)
{
    typedef typename Mfma<T>::acc accT;
    __shared__ double red[GX_WAVES][NT][256];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, kq = lane >> 4, lc = lane & 15;
    // workgroup -> (row slice, tile group), consecutive ids on one XCD: the
    // groups of one row slice read the same rows, so they share that L2
    const unsigned id = xcd_remap(blockIdx.x, gridDim.x);
    const int g = (int)(id % (unsigned)a.ngroups);
    const unsigned slice = id / (unsigned)a.ngroups, nslices = gridDim.x / (unsigned)a.ngroups;
    const int rsub = wave, nsub = GX_WAVES;   // the waves split the rows of a chunk

    // this lane's column of Lm and of the Rm blocks of the group's tiles
    const T *pl = a.arr[0];
    int ldl = 0;
    bool okl = false;
    {
        const int cl = 16 * a.ga[g] + lc;
        if (cl < a.KL) {
            const int code = a.lmap[cl];
            pl = a.arr[code >> 8] + (code & 255);
            ldl = a.ld[code >> 8];
            okl = true;
        }
    }
    const T *pr[NT];
    int ldr[NT];
    bool okr[NT];
#pragma unroll
    for (int j = 0; j < NT; j++) {
        pr[j] = a.arr[0], ldr[j] = 0, okr[j] = false;
        const int t = a.gtile[g][j];
        if (t != 255) {
            const int cr = 16 * a.tb[t] + lc;
            if (cr < a.KR) {
                const int code = a.rmap[cr];
                pr[j] = a.arr[code >> 8] + (code & 255);
                ldr[j] = a.ld[code >> 8];
                okr[j] = true;
            }
        }
    }

    // FP32 blocks: the FP64 running sums live in this lane's own entries of
    // red[wave] (registers are kept for the MFMA accumulators)
    accT acc[NT];
#pragma unroll
    for (int j = 0; j < NT; j++) {
        acc[j] = acc_zero<T>();
        if (sizeof(T) == 4)
#pragma unroll
            for (int r = 0; r < 4; r++) red[wave][j][r * 64 + lane] = 0.0;
    }
    // the wave's share of a chunk: k-steps s0 .. s0+ksteps-1 (4 rows each),
    // taken UNR at a time; the loads of the next UNR k-steps (of this chunk or
    // the next) are in flight while the current ones are multiplied
    const int ksteps = (GX_CH / 4) / nsub, s0 = rsub * ksteps;
    const int gpc = ksteps / UNR;                     // step groups per chunk
    const i64 nchunks = (a.N + GX_CH - 1) / GX_CH;
    const i64 mychunks = nchunks > (i64)slice ? (nchunks - 1 - slice) / nslices + 1 : 0;
    const i64 ngrp = mychunks * gpc;
    auto rowof = [&](i64 ch, int gi) { return ch * GX_CH + 4 * (s0 + gi * UNR) + kq; };
    auto load = [&](T(&av)[UNR], T(&bv)[UNR][NT], i64 row) {
        const T *ql = pl + row * ldl;
        const T *qr[NT];
#pragma unroll
        for (int j = 0; j < NT; j++) qr[j] = pr[j] + row * ldr[j];
        if (row + 4 * (UNR - 1) < a.N) {
            // every row present: plain loads (a lane without a column reads
            // element 0 of array 0 and drops it)
#pragma unroll
            for (int u = 0; u < UNR; u++) {
                av[u] = ql[4 * u * ldl];
#pragma unroll
                for (int j = 0; j < NT; j++) bv[u][j] = qr[j][4 * u * ldr[j]];
            }
        } else {
#pragma unroll
            for (int u = 0; u < UNR; u++) {
                const bool rok = row + 4 * u < a.N;
                av[u] = rok ? ql[4 * u * ldl] : T(0);
#pragma unroll
                for (int j = 0; j < NT; j++) bv[u][j] = rok ? qr[j][4 * u * ldr[j]] : T(0);
            }
        }
    };
    T av[UNR], bv[UNR][NT];
    i64 ch = slice;        // chunk and step group of the loads in flight
    int gi = 0;
    if (ngrp > 0) load(av, bv, rowof(ch, gi));
    for (i64 idx = 0; idx < ngrp; idx++) {
        T an[UNR], bn[UNR][NT];
        const bool more = idx + 1 < ngrp;
        const bool chunk_end = gi == gpc - 1;
        if (++gi == gpc) gi = 0, ch += nslices;
        if (more) load(an, bn, rowof(ch, gi));
#pragma unroll
        for (int u = 0; u < UNR; u++) {
            const T x = okl ? av[u] : T(0);
#pragma unroll
            for (int j = 0; j < NT; j++) acc[j] = Mfma<T>::mma(x, okr[j] ? bv[u][j] : T(0), acc[j]);
        }
        if (sizeof(T) == 4 && chunk_end) {
            // end of a chunk: FP32 partial sums into the FP64 accumulators
#pragma unroll
            for (int j = 0; j < NT; j++) {
#pragma unroll
                for (int r = 0; r < 4; r++) red[wave][j][r * 64 + lane] += (double)acc[j][r];
                acc[j] = acc_zero<T>();
            }
        }
        if (more) {
#pragma unroll
            for (int u = 0; u < UNR; u++) {
                av[u] = an[u];
#pragma unroll
                for (int j = 0; j < NT; j++) bv[u][j] = bn[u][j];
            }
        }
    }
    // the four waves' sums in a fixed order: one partial tile per row slice
#pragma unroll
    for (int j = 0; j < NT; j++)
#pragma unroll
        for (int r = 0; r < 4; r++)
            if (sizeof(T) == 8) red[wave][j][r * 64 + lane] = (double)acc[j][r];
    __syncthreads();
    for (int e = tid; e < NT * 256; e += blockDim.x) {
        const int j = e / 256, q = e % 256;
        const int t = a.gtile[g][j];
        if (t == 255) continue;
        const double s = (red[0][j][q] + red[1][j][q]) + (red[2][j][q] + red[3][j][q]);
        a.partials[((i64)slice * a.ntiles + t) * 256 + q] = s;
    }
}

// out[t][e] = sum over workgroups of partials[b][t][e]: 4 threads per entry
// in strided order, then a fixed combination.
__global__ void __launch_bounds__(256) gramx_reduce_kernel(const double *__restrict__ partials, int nb, int ntiles,
                                                           double *__restrict__ out)
{
    __shared__ double red[4][64];
    const i64 total = (i64)ntiles * 256;
    const int sub = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const i64 q = (i64)blockIdx.x * 64 + lane;
    double s = 0.0;
    if (q < total)
        for (int b = sub; b < nb; b += 4) s += partials[(i64)b * total + q];
    red[sub][lane] = s;
    __syncthreads();
    if (sub == 0 && q < total) out[q] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// A single narrow block (S^T S for W_J or P_J with at most 8 columns, the
// Cholesky Gram matrices of steps 11 and 14): one grid row per thread, the
// W(W+1)/2 products accumulated in FP64, then summed across each wave with a
// fixed xor-shuffle butterfly and across the waves in a fixed order.
static const int RBLOCKS = 1024;

template <typename T, int W>
__global__ void __launch_bounds__(256) gram_rows_kernel(const T *__restrict__ S, i64 N, double *__restrict__ partials)
{
    const int NP = W * (W + 1) / 2;
    __shared__ double red[4][NP];
    double acc[NP];
#pragma unroll
    for (int q = 0; q < NP; q++) acc[q] = 0.0;
    for (i64 r = (i64)blockIdx.x * blockDim.x + threadIdx.x; r < N; r += (i64)gridDim.x * blockDim.x) {
        double v[W];
#pragma unroll
        for (int c = 0; c < W; c++) v[c] = (double)S[r * W + c];
        int q = 0;
#pragma unroll
        for (int i = 0; i < W; i++)
#pragma unroll
            for (int j = i; j < W; j++, q++) acc[q] += v[i] * v[j];
    }
#pragma unroll
    for (int q = 0; q < NP; q++)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off, 64);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NP; q++) red[wave][q] = acc[q];
    __syncthreads();
    for (int q = threadIdx.x; q < NP; q += blockDim.x)
        partials[(i64)blockIdx.x * NP + q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
}

// out[i][j] (Kp x Kp) for i <= j from the per-workgroup pair sums: one
// workgroup per pair, strided sums then a fixed tree.
__global__ void __launch_bounds__(256) gram_rows_reduce_kernel(const double *__restrict__ partials, int nb, int W,
                                                               int Kp, double *__restrict__ out)
{
    __shared__ double red[256];
    const int q = blockIdx.x, NP = W * (W + 1) / 2;
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += 256) s += partials[(i64)b * NP + q];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int i = 0, rem = q;
        while (rem >= W - i) rem -= W - i, i++;
        out[(i64)i * Kp + i + rem] = red[0];
    }
}

template <typename T>
static hipError_t run_gram_rows(const T *S, int W, long long N, double *partials, double *out, int Kp, hipStream_t st)
{
    const i64 nb64 = (N + 255) / 256;
    const int nb = (int)(nb64 < RBLOCKS ? (nb64 > 0 ? nb64 : 1) : RBLOCKS);
    switch (W) {
    case 1: hipLaunchKernelGGL((gram_rows_kernel<T, 1>), dim3(nb), dim3(256), 0, st, S, (i64)N, partials); break;
    case 2: hipLaunchKernelGGL((gram_rows_kernel<T, 2>), dim3(nb), dim3(256), 0, st, S, (i64)N, partials); break;
    case 3: hipLaunchKernelGGL((gram_rows_kernel<T, 3>), dim3(nb), dim3(256), 0, st, S, (i64)N, partials); break;
    case 4: hipLaunchKernelGGL((gram_rows_kernel<T, 4>), dim3(nb), dim3(256), 0, st, S, (i64)N, partials); break;
    case 5: hipLaunchKernelGGL((gram_rows_kernel<T, 5>), dim3(nb), dim3(256), 0, st, S, (i64)N, partials); break;
    case 6: hipLaunchKernelGGL((gram_rows_kernel<T, 6>), dim3(nb), dim3(256), 0, st, S, (i64)N, partials); break;
    case 7: hipLaunchKernelGGL((gram_rows_kernel<T, 7>), dim3(nb), dim3(256), 0, st, S, (i64)N, partials); break;
    default: hipLaunchKernelGGL((gram_rows_kernel<T, 8>), dim3(nb), dim3(256), 0, st, S, (i64)N, partials);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gram_rows_reduce_kernel, dim3(W * (W + 1) / 2), dim3(256), 0, st, partials, nb, W, Kp, out);
    return hipGetLastError();
}

int gram_blocks(long long N)
{
    const long long nch = (N + GX_CH - 1) / GX_CH;
    return (int)(nch < GX_BLOCKS ? (nch > 0 ? nch : 1) : GX_BLOCKS);
}

size_t gram_partials_bytes(long long N)
{
    const size_t tiles = (size_t)gram_blocks(N) * GX_MAX_TILES * 256 * sizeof(double);
    const size_t rows = (size_t)RBLOCKS * 36 * sizeof(double);
    return tiles > rows ? tiles : rows;
}

template <typename T>
static hipError_t run_gramx(const GramXArgs &h, hipStream_t st)
{
    GXDev<T> a;
    for (int i = 0; i < GX_MAX_ARR; i++) {
        a.arr[i] = (const T *)h.arr[i];
        a.ld[i] = h.ld[i];
    }
    a.KL = h.KL;
    a.KR = h.KR;
    for (int i = 0; i < h.KL; i++) {
        const int ar = h.lmap[i] >> 8, col = h.lmap[i] & 255;
        if (ar >= GX_MAX_ARR || !h.arr[ar] || col >= h.ld[ar]) return hipErrorInvalidValue;
        a.lmap[i] = h.lmap[i];
    }
    for (int i = 0; i < h.KR; i++) {
        const int ar = h.rmap[i] >> 8, col = h.rmap[i] & 255;
        if (ar >= GX_MAX_ARR || !h.arr[ar] || col >= h.ld[ar]) return hipErrorInvalidValue;
        a.rmap[i] = h.rmap[i];
    }
    // tiles grouped by their Lm block, NT slots per group (the widest run of
    // one Lm block, at most GX_MAXB); empty slots compute nothing useful
    int NT = 1;
    for (int t = 0; t < h.ntiles;) {
        int n = 0;
        while (t + n < h.ntiles && h.ta[t + n] == h.ta[t]) n++;
        NT = std::max(NT, std::min(n, std::max(1, std::min(sizeof(T) == 4 ? h.max_nt32 : h.max_nt, GX_MAXB))));
        t += n;
    }
    if (NT == 3) NT = 4;
    a.ntiles = h.ntiles;
    a.ngroups = 0;
    for (int t = 0; t < h.ntiles;) {
        const int ta = h.ta[t];
        int n = 0;
        while (t + n < h.ntiles && h.ta[t + n] == ta && n < NT) n++;
        if (a.ngroups >= GX_MAX_TILES) return hipErrorInvalidValue;
        a.ga[a.ngroups] = (unsigned char)ta;
        for (int j = 0; j < GX_MAXB; j++) a.gtile[a.ngroups][j] = j < n ? (unsigned char)(t + j) : 255;
        a.ngroups++;
        t += n;
    }
    for (int t = 0; t < h.ntiles; t++) a.tb[t] = (unsigned char)h.tb[t];
    a.N = h.N;
    a.partials = h.partials;
    const int nb = gram_blocks(h.N);   // row slices
    const dim3 grid(nb * a.ngroups);
    if (NT == 1)
        hipLaunchKernelGGL((gramx_kernel<T, 1, 4>), grid, dim3(64 * GX_WAVES), 0, st, a);
    else if (NT == 2)
        hipLaunchKernelGGL((gramx_kernel<T, 2, 4>), grid, dim3(64 * GX_WAVES), 0, st, a);
    else
        hipLaunchKernelGGL((gramx_kernel<T, 4, 2>), grid, dim3(64 * GX_WAVES), 0, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const i64 total = (i64)h.ntiles * 256;
    hipLaunchKernelGGL(gramx_reduce_kernel, dim3((unsigned)((total + 63) / 64)), dim3(256), 0, st, h.partials, nb,
                       h.ntiles, h.out);
    return hipGetLastError();
}

hipError_t launch_gramx(int dtype, const GramXArgs &a, hipStream_t st)
{
    if (a.N < 1 || a.KL < 1 || a.KR < 1 || a.KL > GX_MAX_L || a.KR > GX_MAX_R || a.ntiles < 1 ||
        a.ntiles > GX_MAX_TILES)
        return hipErrorInvalidValue;
    for (int t = 0; t < a.ntiles; t++) {
        if (a.ta[t] < 0 || 16 * a.ta[t] >= a.KL || a.tb[t] < 0 || 16 * a.tb[t] >= a.KR) return hipErrorInvalidValue;
        if (t > 0 && a.ta[t] < a.ta[t - 1]) return hipErrorInvalidValue;   // sorted by Lm block
    }
    if (dtype == DT_F32) return run_gramx<float>(a, st);
    return run_gramx<double>(a, st);
}

hipError_t launch_gram_rows(int dtype, const void *S, int w, long long N, double *partials, double *out, int ldout,
                            hipStream_t st)
{
    if (w < 1 || w > 8 || N < 1) return hipErrorInvalidValue;
    if (dtype == DT_F32) return run_gram_rows<float>((const float *)S, w, N, partials, out, ldout, st);
    return run_gram_rows<double>((const double *)S, w, N, partials, out, ldout, st);
}

}  // namespace lobpcg
