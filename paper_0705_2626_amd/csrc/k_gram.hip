// Tall-skinny Gram products of LOBPCG on MFMA (gfx950).
//
// For S = [S_0 S_1 S_2] (the blocks X, W_J, P_J; N x K in total) and
// AS = [AS_0 AS_1 AS_2] it computes chosen 16x16 tiles of S^T S and S^T AS:
// the blocks of gramB and gramA that the Rayleigh-Ritz procedure of steps
// 17-23 needs, and the Cholesky Gram matrices of steps 3, 11 and 14 (one
// block, S^T S only).  The host lists the tiles, so blocks the paper's form
// takes as known (Lambda and I on the block diagonal) are not computed.
//
// Each workgroup (8 waves) stages a chunk of RC rows of S and AS in LDS
// (zero-padded to a multiple of 16 columns and past the end of the grid);
// each wave accumulates up to MAXT output tiles with
// v_mfma_f64_16x16x4f64 (FP64 blocks, accumulated in FP64 throughout) or
// v_mfma_f32_16x16x4f32 (FP32 blocks: FP32 only within one RC-row chunk,
// then added into FP64 accumulators).  Per-workgroup partial tiles are
// summed in a fixed order by a second kernel: results are reproducible bit
// for bit.
#include "common.h"
#include "kernels.h"
#include "mfma.h"

namespace lobpcg {

static const int WAVES = 8;
static const int MAXT = 6;                // tiles per wave per pass
static const int TILES_PER_GROUP = WAVES * MAXT;
static const int PAD = 16;                // LDS row padding (elements)
static const int GRAM_BLOCKS = 512;

template <typename T>
struct GramRC;
template <>
struct GramRC<float> {
    static const int v = 64;
};
template <>
struct GramRC<double> {
    static const int v = 32;
};

template <typename T>
struct GramDev {
    const T *S[3], *AS[3];
    int w[3], off[3];
    int nblk, K, Kp, ntiles, has_as;
    int tiles[GRAM_MAX_TILES];   // (mat << 16) | (a << 8) | b
    i64 N;
    double *partials;
};

template <typename T>
__global__ void __launch_bounds__(512) gram_kernel(GramDev<T> a)
{
    typedef typename Mfma<T>::acc accT;
    const int RC = GramRC<T>::v;
    extern __shared__ unsigned char smem[];
    const int ldl = a.Kp + PAD;
    T *Ss = reinterpret_cast<T *>(smem);
    T *As = Ss + RC * ldl;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int tbase = blockIdx.y * TILES_PER_GROUP + wave;

    int tmat[MAXT], ta[MAXT], tb[MAXT];
#pragma unroll
    for (int j = 0; j < MAXT; j++) {
        const int t = tbase + WAVES * j;
        if (t < a.ntiles) {
            const int code = a.tiles[t];
            tmat[j] = code >> 16;
            ta[j] = (code >> 8) & 255;
            tb[j] = code & 255;
        } else {
            tmat[j] = -1, ta[j] = tb[j] = 0;
        }
    }
    accT acc[MAXT];      // FP64: running sums; FP32: the current chunk
    double acc64[MAXT][4];
#pragma unroll
    for (int j = 0; j < MAXT; j++) {
        acc[j] = acc_zero<T>();
#pragma unroll
        for (int r = 0; r < 4; r++) acc64[j][r] = 0.0;
    }
    // zero the padding columns once; staging never writes them
    const int npad = a.Kp - a.K;
    for (int e = tid; e < RC * npad; e += blockDim.x) {
        const int row = e / npad, col = a.K + e % npad;
        Ss[row * ldl + col] = T(0);
        As[row * ldl + col] = T(0);
    }

    // Chunk ch of block b is the contiguous run of RC*w_b elements at
    // S_b + ch*RC*w_b; every thread moves at most one 16-byte vector of each
    // of S_b and AS_b per chunk.  The next chunk is loaded into registers
    // while the current one is multiplied.
    const int VE = 16 / sizeof(T);
    const i64 nchunks = (a.N + RC - 1) / RC;
    const int lrow = lane >> 4, lcol = lane & 15;
    vec<T, VE> rs[3], ra[3];
    auto load = [&](i64 ch) {
        const i64 r0 = ch * RC;
        const int nvalid = (int)(((a.N - r0) < RC ? (a.N - r0) : RC));
#pragma unroll
        for (int b = 0; b < 3; b++) {
            if (b >= a.nblk) break;
            const int wb = a.w[b];
            const int e0 = tid * VE;
            if (e0 >= RC * wb) continue;
            const T *sb = a.S[b] + r0 * wb;
            const T *ab = a.has_as ? a.AS[b] + r0 * wb : nullptr;
            if (e0 + VE <= nvalid * wb) {
                rs[b] = vload<T, VE>(sb + e0);
                if (ab) ra[b] = vload<T, VE>(ab + e0);
            } else {
#pragma unroll
                for (int q = 0; q < VE; q++) {
                    const bool ok = e0 + q < nvalid * wb;
                    rs[b].v[q] = ok ? sb[e0 + q] : T(0);
                    if (ab) ra[b].v[q] = ok ? ab[e0 + q] : T(0);
                }
            }
        }
    };
    if ((i64)blockIdx.x < nchunks) load(blockIdx.x);
    for (i64 ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        __syncthreads();
#pragma unroll
        for (int b = 0; b < 3; b++) {
            if (b >= a.nblk) break;
            const int wb = a.w[b];
            const int e0 = tid * VE;
            if (e0 >= RC * wb) continue;
            const float inv = 1.0f / (float)wb;
#pragma unroll
            for (int q = 0; q < VE; q++) {
                // e < 64*32: the float quotient is within 2e-4 of e/wb, and
                // (e + 0.5)/wb is at least 0.5/32 away from an integer
                const int e = e0 + q;
                const int row = (int)(((float)e + 0.5f) * inv);
                const int col = a.off[b] + e - row * wb;
                Ss[row * ldl + col] = rs[b].v[q];
                if (a.has_as) As[row * ldl + col] = ra[b].v[q];
            }
        }
        if (ch + gridDim.x < nchunks) load(ch + gridDim.x);
        __syncthreads();
#pragma unroll 2
        for (int kk = 0; kk < RC; kk += 4) {
            const T *srow = Ss + (kk + lrow) * ldl + lcol;
            const T *arow = As + (kk + lrow) * ldl + lcol;
#pragma unroll
            for (int j = 0; j < MAXT; j++) {
                if (tmat[j] < 0) continue;
                const T x = srow[16 * ta[j]];
                const T y = tmat[j] ? arow[16 * tb[j]] : srow[16 * tb[j]];
                acc[j] = Mfma<T>::mma(x, y, acc[j]);
            }
        }
        if (sizeof(T) == 4) {
#pragma unroll
            for (int j = 0; j < MAXT; j++) {
#pragma unroll
                for (int r = 0; r < 4; r++) acc64[j][r] += (double)acc[j][r];
                acc[j] = acc_zero<T>();
            }
        }
    }
    // partials[bx][tile][r*64 + lane]
    double *dst = a.partials + (i64)blockIdx.x * a.ntiles * 256;
#pragma unroll
    for (int j = 0; j < MAXT; j++) {
        const int t = tbase + WAVES * j;
        if (t >= a.ntiles) continue;
#pragma unroll
        for (int r = 0; r < 4; r++)
            dst[(i64)t * 256 + r * 64 + lane] = sizeof(T) == 4 ? acc64[j][r] : (double)acc[j][r];
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
static hipError_t run_gram_rows(const GramArgs &h, hipStream_t st)
{
    const int W = h.w[0], Kp = gram_kpad(W);
    const i64 nb64 = (h.N + 255) / 256;
    const int nb = (int)(nb64 < RBLOCKS ? (nb64 > 0 ? nb64 : 1) : RBLOCKS);
    const T *S = (const T *)h.S[0];
    switch (W) {
    case 1: hipLaunchKernelGGL((gram_rows_kernel<T, 1>), dim3(nb), dim3(256), 0, st, S, (i64)h.N, h.partials); break;
    case 2: hipLaunchKernelGGL((gram_rows_kernel<T, 2>), dim3(nb), dim3(256), 0, st, S, (i64)h.N, h.partials); break;
    case 3: hipLaunchKernelGGL((gram_rows_kernel<T, 3>), dim3(nb), dim3(256), 0, st, S, (i64)h.N, h.partials); break;
    case 4: hipLaunchKernelGGL((gram_rows_kernel<T, 4>), dim3(nb), dim3(256), 0, st, S, (i64)h.N, h.partials); break;
    case 5: hipLaunchKernelGGL((gram_rows_kernel<T, 5>), dim3(nb), dim3(256), 0, st, S, (i64)h.N, h.partials); break;
    case 6: hipLaunchKernelGGL((gram_rows_kernel<T, 6>), dim3(nb), dim3(256), 0, st, S, (i64)h.N, h.partials); break;
    case 7: hipLaunchKernelGGL((gram_rows_kernel<T, 7>), dim3(nb), dim3(256), 0, st, S, (i64)h.N, h.partials); break;
    default: hipLaunchKernelGGL((gram_rows_kernel<T, 8>), dim3(nb), dim3(256), 0, st, S, (i64)h.N, h.partials);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gram_rows_reduce_kernel, dim3(W * (W + 1) / 2), dim3(256), 0, st, h.partials, nb, W, Kp, h.out);
    return hipGetLastError();
}

// out[mat][i][j] (Kp x Kp each) = sum over workgroups: one workgroup per
// group of 64 tile entries, each entry summed by 4 threads in strided order
// and then combined in a fixed order, so the result never changes.
template <typename T>
__global__ void __launch_bounds__(256) gram_reduce_kernel(const double *__restrict__ partials, int nb, GramDev<T> a,
                                                          double *__restrict__ out)
{
    __shared__ double red[4][64];
    const i64 total = (i64)a.ntiles * 256;
    const int sub = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const i64 q = (i64)blockIdx.x * 64 + lane;
    double s = 0.0;
    if (q < total)
        for (int b = sub; b < nb; b += 4) s += partials[(i64)b * total + q];
    red[sub][lane] = s;
    __syncthreads();
    if (sub == 0 && q < total) {
        s = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
        const int t = (int)(q / 256), e = (int)(q % 256);
        const int r = e / 64, ln = e % 64;
        const int code = a.tiles[t];
        const int mat = code >> 16, ta = (code >> 8) & 255, tb = code & 255;
        const int i = 16 * ta + Mfma<T>::row(ln, r), j = 16 * tb + (ln & 15);
        out[(i64)mat * a.Kp * a.Kp + (i64)i * a.Kp + j] = s;
    }
}

int gram_kpad(int K) { return (K + 15) / 16 * 16; }

static int gram_blocks(long long N)
{
    const long long nch = (N + 31) / 32;
    return (int)(nch < GRAM_BLOCKS ? (nch > 0 ? nch : 1) : GRAM_BLOCKS);
}

size_t gram_partials_bytes(int dtype, long long N, int K)
{
    (void)dtype;
    const int TK = gram_kpad(K) / 16;
    const size_t ntiles = (size_t)TK * (TK + 1);
    const size_t staged = (size_t)gram_blocks(N) * ntiles * 256 * sizeof(double);
    const size_t rows = (size_t)RBLOCKS * 36 * sizeof(double);
    return staged > rows ? staged : rows;
}

template <typename T>
static hipError_t run_gram(const GramArgs &h, hipStream_t st)
{
    if (!h.staged && h.nblk == 1 && !h.AS[0] && h.w[0] >= 1 && h.w[0] <= 8) return run_gram_rows<T>(h, st);
    GramDev<T> a;
    int K = 0;
    for (int b = 0; b < 3; b++) {
        a.S[b] = (const T *)h.S[b];
        a.AS[b] = (const T *)h.AS[b];
        a.w[b] = b < h.nblk ? h.w[b] : 0;
        a.off[b] = K;
        if (b < h.nblk) K += h.w[b];
    }
    a.nblk = h.nblk;
    a.K = K;
    a.Kp = gram_kpad(K);
    a.has_as = h.AS[0] != nullptr;
    a.ntiles = h.ntiles;
    if (a.ntiles < 1 || a.ntiles > GRAM_MAX_TILES || K > 96) return hipErrorInvalidValue;
    // one 16-byte vector per thread and block covers a chunk: RC*w_b <= 512*VE
    for (int b = 0; b < a.nblk; b++)
        if (a.w[b] < 1 || (size_t)GramRC<T>::v * a.w[b] > 512 * (16 / sizeof(T))) return hipErrorInvalidValue;
    for (int t = 0; t < a.ntiles; t++) {
        const int code = h.tiles[t], mat = code >> 16, ta = (code >> 8) & 255, tb = code & 255;
        if (mat < 0 || mat > 1 || (mat == 1 && !a.has_as) || ta * 16 >= a.Kp || tb * 16 >= a.Kp)
            return hipErrorInvalidValue;
        a.tiles[t] = code;
    }
    a.N = h.N;
    a.partials = h.partials;
    int nb;
    nb = gram_blocks(h.N);
    const int ngroups = (a.ntiles + TILES_PER_GROUP - 1) / TILES_PER_GROUP;
    const size_t shm = (size_t)2 * GramRC<T>::v * (a.Kp + PAD) * sizeof(T);
    hipLaunchKernelGGL(gram_kernel<T>, dim3(nb, ngroups), dim3(64 * WAVES), shm, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const i64 total = (i64)a.ntiles * 256;
    hipLaunchKernelGGL(gram_reduce_kernel<T>, dim3((unsigned)((total + 63) / 64)), dim3(256), 0, st, h.partials, nb,
                       a, h.out);
    return hipGetLastError();
}

hipError_t launch_gram(int dtype, const GramArgs &a, hipStream_t st)
{
    if (dtype == DT_F32) return run_gram<float>(a, st);
    return run_gram<double>(a, st);
}

}  // namespace lobpcg
