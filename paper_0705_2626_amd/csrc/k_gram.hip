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

// The same products with each row chunk staged once through LDS.  The
// direct kernel above loads every 16-column operand block once per tile
// group that uses it (about five times over for the Rayleigh-Ritz products),
// and that traffic through the per-CU vector cache, not HBM, limits it.  Here
// a workgroup of GY_WAVES waves walks whole row chunks of the distinct
// 16-column panels of Lm and Rm (at most GY_MAX_P): every thread loads
// elements of two neighbouring panels of two rows (whole 128-byte lines when
// the panels are the two halves of a 32-column block), stores them into one
// of two LDS buffers, and after one barrier the waves multiply out their own
// tiles from LDS while the next chunk's loads are in flight.  Products with
// few panels stack several row sub-chunks into one LDS buffer, so that every
// chunk moves the same number of bytes.  Each wave takes a
// contiguous run of the tiles (sorted by Lm panel, so the Lm operands are
// mostly read once per chunk); its sums go to its own partial tiles, so the
// partials and their reduction are those of the direct kernel and results are
// reproducible bit for bit.
static const int GY_WAVES = 8;
static const int GY_MAX_P = 18;   // panels of the 9-slot shape
static const int GY_TPW = GX_MAX_TILES / GY_WAVES;   // most tiles per wave
static const int GY_BLOCKS = 512;

template <typename T>
struct GYDev {
    const T *arr[GX_MAX_ARR];
    int ld[GX_MAX_ARR];
    const T *safe;                        // a valid element: the address of every load that is not needed
    // slot-panel columns, (array << 8) | column, 0xFFFF: none (zeros).  Load
    // slot q (a pair of slot-panels 2q, 2q + 1) holds panel pair q % npairs
    // of row sub-chunk sub[q]; slots past nsub * npairs are unused.
    unsigned short pcode[GY_MAX_P][16];
    int sub[GY_MAX_P / 2];
    int npairs, nsub, ntiles;
    int wn[GY_WAVES];   // tiles of each wave
    // per wave: Lm panel | Rm panel << 8 | tile << 16 (panels of sub-chunk 0;
    // 32-bit entries keep the scalar loads of a wave's row dword-aligned)
    int wtile[GY_WAVES][GY_TPW];
    i64 N;
    double *partials;   // [gridDim.x][ntiles][256]
};

// Two shapes of the LDS buffers, NQ load slots of two panels each: 6 slots
// (up to 12 panels) of 48 FP32 / 16 FP64 rows, or 9 slots (up to 18 panels)
// of 32 FP32 / 16 FP64 rows; either way two workgroups' double buffers fit
// in one CU's 160 KB of LDS.  RC: rows per sub-chunk; PS: LDS panel stride (= 32 mod 64
// words for FP32, so that the four 16-lane groups of a store hit different
// banks); RPT: rows per thread and load slot.
template <typename T, int NQ>
struct GYShape {
    static const int RC = sizeof(T) == 4 ? (NQ == 6 ? 48 : 32) : 16;
    static const int PS = RC * 16 + (sizeof(T) == 8 && NQ == 9 ? 16 : 32);
    static const int RPT = RC / 16;
};

template <typename T, int TPW, int NQ>
__global__ void __launch_bounds__(64 * GY_WAVES) gramy_kernel(GYDev<T> a)
{
    typedef GYShape<T, NQ> S;
    typedef typename Mfma<T>::acc accT;
    typedef const __attribute__((address_space(1))) T *gptr;   // global loads, not flat ones
    const int NP = 2 * NQ;   // slot-panels
    const int BUF = NP * S::PS;
    __shared__ T lds[2 * BUF];
    __shared__ const T *tptr[NP * 16];
    __shared__ int tld[NP * 16];   // 0: a column of zeros (read from a.safe)
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (tid < NP * 16) {
        const int code = a.pcode[tid >> 4][tid & 15];
        const bool ok = code != 0xFFFF;
        tptr[tid] = ok ? a.arr[code >> 8] + (code & 255) : a.safe;
        tld[tid] = ok ? a.ld[code >> 8] : 0;
    }
    __syncthreads();
    const i64 N = a.N, rows_chunk = (i64)a.nsub * S::RC, nchunks = (N + rows_chunk - 1) / rows_chunk;
    // loads: lanes 0-31 take two rows of one panel, 32-63 the same rows of
    // the next panel (16 lanes per panel row)
    const int lc = lane & 15, lpan = lane >> 5, lrow = 2 * wave + ((lane >> 4) & 1);
    const int soff = lpan * S::PS + lrow * 16 + lc;
    // Every thread issues the same NQ * RPT loads per chunk, rows past N and
    // unused columns from valid addresses (zeroed when stored), so that the
    // loads in flight can be counted and waited for one chunk at a time.
    // Element offsets are 32-bit (the host checks N * ld < 2^32).
    typedef T Stage[NQ][S::RPT];
    const unsigned N32 = (unsigned)N;
    auto row0 = [&](i64 ch) { return (unsigned)(ch * rows_chunk) + (unsigned)lrow; };
    auto gload = [&](Stage &st, i64 ch) {
        const unsigned r0 = row0(ch);
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            const int e = (2 * q + lpan) * 16 + lc;
            const gptr base = (gptr)tptr[e];
            const unsigned ldv = (unsigned)tld[e], rq = r0 + (unsigned)(a.sub[q] * S::RC);
#pragma unroll
            for (int i = 0; i < S::RPT; i++) st[q][i] = base[min(rq + 16u * i, N32 - 1u) * ldv];
        }
    };
    auto lstore = [&](int buf, const Stage &st, i64 ch) {
        T *L = lds + buf * BUF + soff;
        const unsigned r0 = row0(ch);
#pragma unroll
        for (int q = 0; q < NQ; q++) {
            const bool okc = tld[(2 * q + lpan) * 16 + lc] > 0;
            const unsigned rq = r0 + (unsigned)(a.sub[q] * S::RC);
#pragma unroll
            for (int i = 0; i < S::RPT; i++) L[2 * q * S::PS + 256 * i] = (okc && rq + 16u * i < N32) ? st[q][i] : T(0);
        }
    };

    const int nt = a.wn[wave], nsub = a.nsub, subp = 2 * a.npairs * S::PS;
    int pa[TPW], pb[TPW];
#pragma unroll
    for (int j = 0; j < TPW; j++) pa[j] = (a.wtile[wave][j] & 255) * S::PS, pb[j] = ((a.wtile[wave][j] >> 8) & 255) * S::PS;
    accT acc[TPW];
    double sums[TPW][4];   // FP32 blocks: FP64 running sums of the sub-chunk products
#pragma unroll
    for (int j = 0; j < TPW; j++) {
        acc[j] = acc_zero<T>();
#pragma unroll
        for (int r = 0; r < 4; r++) sums[j][r] = 0.0;
    }
    // MFMA operands: lane l, k-step s reads row 4s + l/16, column l%16 of a
    // panel; a wave's consecutive tiles mostly share their Lm panel, whose
    // operands then stay in registers
    const int roff = (lane >> 4) * 16 + lc;
    auto compute = [&](int buf) {
        for (int sb = 0; sb < nsub; sb++) {
            const T *L = lds + buf * BUF + roff + sb * subp;
            T av[S::RC / 4];
#pragma unroll
            for (int j = 0; j < TPW; j++) {
                if (j < nt) {
                    if (j == 0 || pa[j] != pa[j - 1])
#pragma unroll
                        for (int s = 0; s < S::RC / 4; s++) av[s] = L[pa[j] + 64 * s];
#pragma unroll
                    for (int s = 0; s < S::RC / 4; s++) acc[j] = Mfma<T>::mma(av[s], L[pb[j] + 64 * s], acc[j]);
                    if (sizeof(T) == 4) {
#pragma unroll
                        for (int r = 0; r < 4; r++) sums[j][r] += (double)acc[j][r];
                        acc[j] = acc_zero<T>();
                    }
                }
            }
        }
    };
    // the loads of chunk c + G (G = gridDim.x) are in flight while chunk c is
    // multiplied out; the two LDS buffers alternate, and each was last read
    // before the previous barrier
    const i64 G = gridDim.x;
    Stage st;
    i64 ch = blockIdx.x;
    gload(st, ch);
    for (int buf = 0; ch < nchunks; ch += G, buf ^= 1) {
        lstore(buf, st, ch);
        __syncthreads();
        gload(st, ch + G);
        compute(buf);
    }
#pragma unroll
    for (int j = 0; j < TPW; j++)
        if (j < nt) {
            double *o = a.partials + ((i64)blockIdx.x * a.ntiles + (a.wtile[wave][j] >> 16)) * 256 + lane;
#pragma unroll
            for (int r = 0; r < 4; r++) o[r * 64] = sizeof(T) == 4 ? sums[j][r] : (double)acc[j][r];
        }
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

// The LDS-staged kernel when the tiles' operand blocks fit its panel table;
// false: they do not (nothing launched).  Column codes are checked by the caller.
template <typename T>
static bool run_gramy(const GramXArgs &h, hipStream_t st, hipError_t &err)
{
    GYDev<T> a;
    a.safe = nullptr;
    for (int i = 0; i < GX_MAX_ARR; i++) {
        a.arr[i] = (const T *)h.arr[i];
        a.ld[i] = h.ld[i];
    }
    // the distinct panels (16 column codes each) of the tiles' Lm and Rm blocks
    unsigned short pcode[GY_MAX_P][16];
    int np = 0;
    auto panel = [&](const unsigned short *map, int K, int blk) -> int {
        unsigned short code[16];
        for (int v = 0; v < 16; v++) code[v] = 16 * blk + v < K ? map[16 * blk + v] : 0xFFFF;
        for (int p = 0; p < np; p++)
            if (std::equal(code, code + 16, pcode[p])) return p;
        if (np == GY_MAX_P) return -1;
        std::copy(code, code + 16, pcode[np]);
        return np++;
    };
    int pl[GX_MAX_L / 16], pr[GX_MAX_R / 16];
    std::fill(pl, pl + GX_MAX_L / 16, -1);
    std::fill(pr, pr + GX_MAX_R / 16, -1);
    // tiles (sorted by Lm block) dealt in contiguous runs whose lengths
    // differ by at most one, longer runs first: waves w and w + 4 share a SIMD
    int nw[GY_WAVES] = {};
    for (int w = 0; w < GY_WAVES; w++) nw[w] = h.ntiles / GY_WAVES + (w < h.ntiles % GY_WAVES ? 1 : 0);
    for (int t = 0, w = 0, j = 0; t < h.ntiles; t++) {
        int &l = pl[h.ta[t]], &r = pr[h.tb[t]];
        if (l < 0 && (l = panel(h.lmap, h.KL, h.ta[t])) < 0) return false;
        if (r < 0 && (r = panel(h.rmap, h.KR, h.tb[t])) < 0) return false;
        while (j == nw[w]) w++, j = 0;
        a.wtile[w][j++] = l | r << 8 | t << 16;
    }
    int tpw = 0;
    for (int w = 0; w < GY_WAVES; w++) {
        a.wn[w] = nw[w];
        tpw = std::max(tpw, nw[w]);
        for (int j = nw[w]; j < GY_TPW; j++) a.wtile[w][j] = 0;
    }
    // load slots: panel pairs, repeated for as many row sub-chunks as fit
    const int NQ = np <= 12 ? 6 : 9;
    const int RC = NQ == 6 ? GYShape<T, 6>::RC : GYShape<T, 9>::RC;
    a.npairs = (np + 1) / 2;
    a.nsub = NQ / a.npairs;
    for (int q = 0; q < GY_MAX_P / 2; q++) {
        const bool used = q < a.nsub * a.npairs;
        a.sub[q] = used ? q / a.npairs : 0;
        for (int lp = 0; lp < 2; lp++) {
            const int p = 2 * (q % a.npairs) + lp;
            for (int v = 0; v < 16; v++) {
                const unsigned short c = used && p < np ? pcode[p][v] : 0xFFFF;
                a.pcode[2 * q + lp][v] = c;
                if (c != 0xFFFF && !a.safe) a.safe = a.arr[c >> 8] + (c & 255);
            }
        }
    }
    if (!a.safe) return false;
    // 32-bit element offsets: every row of every used array (and the rows a
    // prefetch past the end computes before clamping) must be addressable
    for (int p = 0; p < GY_MAX_P; p++)
        for (int v = 0; v < 16; v++)
            if (a.pcode[p][v] != 0xFFFF &&
                (unsigned long long)(h.N + 2 * GY_BLOCKS * 9 * RC) * (unsigned long long)h.ld[a.pcode[p][v] >> 8] >=
                    (1ull << 32))
                return false;
    a.ntiles = h.ntiles;
    a.N = h.N;
    a.partials = h.partials;
    const i64 rows = (i64)a.nsub * RC, nchunks = (h.N + rows - 1) / rows;
    const int nb = (int)std::min<i64>(std::min<i64>(nchunks, gram_blocks(h.N)), GY_BLOCKS);
    const dim3 grid(nb), block(64 * GY_WAVES);
#define GY_LAUNCH(TPW_, NQ_) hipLaunchKernelGGL((gramy_kernel<T, TPW_, NQ_>), grid, block, 0, st, a)
    const int tv = tpw <= 2 ? 2 : tpw <= 4 ? 4 : tpw <= 6 ? 6 : 8;
    if (NQ == 6) {
        if (tv == 2) GY_LAUNCH(2, 6);
        else if (tv == 4) GY_LAUNCH(4, 6);
        else if (tv == 6) GY_LAUNCH(6, 6);
        else GY_LAUNCH(8, 6);
    } else {
        if (tv == 2) GY_LAUNCH(2, 9);
        else if (tv == 4) GY_LAUNCH(4, 9);
        else if (tv == 6) GY_LAUNCH(6, 9);
        else GY_LAUNCH(8, 9);
    }
#undef GY_LAUNCH
    err = hipGetLastError();
    if (err != hipSuccess) return true;
    const i64 total = (i64)h.ntiles * 256;
    hipLaunchKernelGGL(gramx_reduce_kernel, dim3((unsigned)((total + 63) / 64)), dim3(256), 0, st, h.partials, nb,
                       h.ntiles, h.out);
    err = hipGetLastError();
    return true;
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
    if (!h.direct) {
        hipError_t e = hipSuccess;
        if (run_gramy<T>(h, st, e)) return e;
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
