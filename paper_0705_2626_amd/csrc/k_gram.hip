// Tall-skinny Gram products of LOBPCG on MFMA (gfx950).
//
// For S = [S_0 S_1 S_2] (the blocks X, W_J, P_J; N x K in total) and
// AS = [AS_0 AS_1 AS_2] it computes the upper 16x16 tiles of S^T S and S^T AS,
// which hold every block the Rayleigh-Ritz procedure of steps 17-23 needs
// (gramB and gramA), and the Cholesky Gram matrices of steps 3, 11 and 14
// when called with one block.
//
// Each workgroup stages a chunk of RC rows of S and AS in LDS (zero-padded to
// a multiple of 16 columns and to the end of the grid), and each of its four
// waves accumulates its share of the output tiles with
// v_mfma_{f64_16x16x4f64, f32_16x16x4f32}.  FP32 products are summed in FP32
// only within one RC-row chunk and then added to FP64 accumulators.  Per-
// workgroup partial tiles are summed in a fixed order by a second kernel, so
// results are bit-reproducible run to run.
#include "common.h"
#include "kernels.h"

namespace lobpcg {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

static const int RC = 32;         // rows per staged chunk
static const int MAXT = 12;       // output tiles per wave
static const int PAD = 16;        // LDS row padding (elements)
static const int GRAM_BLOCKS = 512;

template <typename T>
struct GramDev {
    const T *S[3], *AS[3];
    int w[3], off[3];
    int nblk, K, Kp, TK, ntiles;
    int has_as;     // 0: only S^T S is wanted
    i64 N;
    double *partials;
};

// Tile t in [0, ntiles): matrix mat (0: S^T S, 1: S^T AS), tile row a <= col b.
__device__ __forceinline__ void decode_tile(int t, int TK, int &mat, int &a, int &b)
{
    const int per = TK * (TK + 1) / 2;
    mat = t / per;
    int r = t % per;
    a = 0;
    while (r >= TK - a) {
        r -= TK - a;
        a++;
    }
    b = a + r;
}

template <typename T>
struct MfmaAcc;
template <>
struct MfmaAcc<float> {
    typedef floatx4 type;
    static __device__ __forceinline__ floatx4 mma(float x, float y, floatx4 c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
    }
};
template <>
struct MfmaAcc<double> {
    typedef doublex4 type;
    static __device__ __forceinline__ doublex4 mma(double x, double y, doublex4 c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
    }
};

template <typename T>
__global__ void __launch_bounds__(256) gram_kernel(GramDev<T> a)
{
    typedef typename MfmaAcc<T>::type accT;
    extern __shared__ unsigned char smem[];
    const int ldl = a.Kp + PAD;
    T *Ss = reinterpret_cast<T *>(smem);
    T *As = Ss + RC * ldl;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tbase = blockIdx.y * 4 * MAXT + wave;

    int tmat[MAXT], ta[MAXT], tb[MAXT];
#pragma unroll
    for (int j = 0; j < MAXT; j++) {
        const int t = tbase + 4 * j;
        if (t < a.ntiles) decode_tile(t, a.TK, tmat[j], ta[j], tb[j]);
        else tmat[j] = -1, ta[j] = tb[j] = 0;
    }
    double acc[MAXT][4];
#pragma unroll
    for (int j = 0; j < MAXT; j++)
#pragma unroll
        for (int r = 0; r < 4; r++) acc[j][r] = 0.0;

    const i64 nchunks = (a.N + RC - 1) / RC;
    const int lrow = lane >> 4, lcol = lane & 15;
    for (i64 ch = blockIdx.x; ch < nchunks; ch += gridDim.x) {
        const i64 r0 = ch * RC;
        const int rows = (int)((a.N - r0) < RC ? (a.N - r0) : RC);
        __syncthreads();
        // stage: block b's chunk is the contiguous run of rows*w_b elements at S_b + r0*w_b
        for (int b = 0; b < a.nblk; b++) {
            const int wb = a.w[b];
            const T *sb = a.S[b] + r0 * wb;
            const T *ab = a.AS[b] + r0 * wb;
            const int n = rows * wb;
            for (int e = threadIdx.x; e < n; e += blockDim.x) {
                const int row = e / wb, col = a.off[b] + e % wb;
                Ss[row * ldl + col] = sb[e];
                if (a.has_as) As[row * ldl + col] = ab[e];
            }
        }
        // zero the padding columns and the rows beyond the grid
        for (int e = threadIdx.x; e < RC * a.Kp; e += blockDim.x) {
            const int row = e / a.Kp, col = e % a.Kp;
            if (row >= rows || col >= a.K) {
                Ss[row * ldl + col] = T(0);
                As[row * ldl + col] = T(0);
            }
        }
        __syncthreads();
        accT part[MAXT];
#pragma unroll
        for (int j = 0; j < MAXT; j++)
#pragma unroll
            for (int r = 0; r < 4; r++) part[j][r] = T(0);
#pragma unroll 2
        for (int kk = 0; kk < RC; kk += 4) {
            const T *srow = Ss + (kk + lrow) * ldl + lcol;
            const T *arow = As + (kk + lrow) * ldl + lcol;
#pragma unroll
            for (int j = 0; j < MAXT; j++) {
                if (tmat[j] < 0) continue;
                const T x = srow[16 * ta[j]];
                const T y = tmat[j] ? arow[16 * tb[j]] : srow[16 * tb[j]];
                part[j] = MfmaAcc<T>::mma(x, y, part[j]);
            }
        }
#pragma unroll
        for (int j = 0; j < MAXT; j++)
#pragma unroll
            for (int r = 0; r < 4; r++) acc[j][r] += (double)part[j][r];
    }
    // partials[bx][tile][r*64 + lane]
    double *dst = a.partials + (i64)blockIdx.x * a.ntiles * 256;
#pragma unroll
    for (int j = 0; j < MAXT; j++) {
        const int t = tbase + 4 * j;
        if (t >= a.ntiles) continue;
#pragma unroll
        for (int r = 0; r < 4; r++) dst[(i64)t * 256 + r * 64 + lane] = acc[j][r];
    }
}

// out[mat][i][j] (Kp x Kp each) = sum over workgroups, fixed order.  MFMA
// 16x16 output layouts (lane l, accumulator register r, column l%16):
//   f32_16x16x4f32: row 4*(l/16) + r;   f64_16x16x4f64: row l/16 + 4*r.
__global__ void __launch_bounds__(256) gram_reduce_kernel(const double *__restrict__ partials, int nb, int ntiles,
                                                          int TK, int Kp, int f64_layout,
                                                          double *__restrict__ out)
{
    const i64 total = (i64)ntiles * 256;
    for (i64 q = (i64)blockIdx.x * blockDim.x + threadIdx.x; q < total; q += (i64)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int b = 0; b < nb; b++) s += partials[(i64)b * total + q];
        const int t = (int)(q / 256), e = (int)(q % 256);
        const int r = e / 64, lane = e % 64;
        int mat, ta, tb;
        decode_tile(t, TK, mat, ta, tb);
        const int row = f64_layout ? (lane >> 4) + 4 * r : 4 * (lane >> 4) + r;
        const int i = 16 * ta + row, j = 16 * tb + (lane & 15);
        out[(i64)mat * Kp * Kp + (i64)i * Kp + j] = s;
    }
}

int gram_kpad(int K) { return (K + 15) / 16 * 16; }

static int gram_blocks(long long N)
{
    long long nch = (N + RC - 1) / RC;
    return (int)(nch < GRAM_BLOCKS ? (nch > 0 ? nch : 1) : GRAM_BLOCKS);
}

size_t gram_partials_bytes(int dtype, long long N, int K)
{
    (void)dtype;
    const int TK = gram_kpad(K) / 16;
    const size_t ntiles = (size_t)TK * (TK + 1);
    return (size_t)gram_blocks(N) * ntiles * 256 * sizeof(double);
}

template <typename T>
static hipError_t run_gram(const GramArgs &h, hipStream_t st)
{
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
    a.TK = a.Kp / 16;
    a.has_as = h.AS[0] != nullptr;
    a.ntiles = (a.has_as ? 2 : 1) * a.TK * (a.TK + 1) / 2;
    a.N = h.N;
    a.partials = h.partials;
    const int nb = gram_blocks(h.N);
    const int ngroups = (a.ntiles + 4 * MAXT - 1) / (4 * MAXT);
    const size_t shm = (size_t)2 * RC * (a.Kp + PAD) * sizeof(T);
    hipLaunchKernelGGL(gram_kernel<T>, dim3(nb, ngroups), dim3(256), shm, st, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const i64 total = (i64)a.ntiles * 256;
    hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, h.partials, nb,
                       a.ntiles, a.TK, a.Kp, (int)(sizeof(T) == 8), h.out);
    return hipGetLastError();
}

hipError_t launch_gram(int dtype, const GramArgs &a, hipStream_t st)
{
    if (dtype == DT_F32) return run_gram<float>(a, st);
    return run_gram<double>(a, st);
}

}  // namespace lobpcg
