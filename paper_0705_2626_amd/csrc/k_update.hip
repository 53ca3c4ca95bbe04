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
// A workgroup (4 waves) walks tiles of 64 grid points; each wave multiplies
// its 16 points by the coefficients (kept in LDS) with 16x16x4 MFMA, NT
// 16-column output tiles at a time.  The MFMA A-fragment of a k-step is 16
// rows x 4 columns of an input.  Four kernels share this scheme:
//   mvf_kernel  (default) fragments loaded straight from global memory with
//               16-byte loads, the k-sum split in contiguous quarters;
//   mvn_kernel  at most 8 columns in and out: one point per thread, plain FMA;
//   mv_kernel / mvd_kernel  (kernel variants 2 / 1) wide inputs staged through
//               LDS one stage ahead / per-element fragment loads;
//   mvw_kernel  blocks wider than 32 columns: up to 12 input pieces of at most
//               32 columns, 16, 32 or 64 output columns per launch.
// Per-workgroup partial sums of the norms are added in a fixed order by a
// second kernel.
#include "common.h"
#include "kernels.h"
#include "mfma.h"

namespace lobpcg {

static const int TP = 64;          // grid points per tile (4 waves x 16)
static const int MAXW = 32;        // widest input (stored columns)
static const int NARROW = 8;       // inputs up to this width are not staged
static const int LDT = MAXW + 1;   // LDS row stride: odd, so the 16 rows of an A fragment hit 16 banks
static const int MV_MAX_BLOCKS = 4096;

template <typename T>
struct MVDev {
    const T *in[2][MV_MAX_IN];
    int ld[MV_MAX_IN], k[MV_MAX_IN];
    const int *cols[MV_MAX_IN];
    int coff[MV_MAX_IN];
    int nin, nside, kout, K, Kp;
    int n0, ld2;
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

// acc[nt] += A C[roff .. roff+k-1] with A-fragments from a staged LDS row
template <typename T, int NT>
__device__ __forceinline__ void mma_lds(typename Mfma<T>::acc (&acc)[NT], const T *arow, const T *Cs, const int *cmap,
                                        int roff, int k, int lane)
{
    const int NC = NT * 16;
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

// the same with A-fragments straight from global memory (row `src` of this
// lane, or zero past the grid); all loads of the input are issued first
template <typename T, int NT>
__device__ __forceinline__ void mma_global(typename Mfma<T>::acc (&acc)[NT], const T *__restrict__ src, bool pok,
                                           const T *Cs, const int *cmap, int roff, int k, int lane)
{
    const int NC = NT * 16, kq = lane >> 4, lc = lane & 15;
    T av[MAXW / 4];
#pragma unroll
    for (int i = 0; i < MAXW / 4; i++) {
        const int kr = 4 * i + kq;
        av[i] = (pok && kr < k) ? src[cmap[roff + kr]] : T(0);
    }
#pragma unroll
    for (int i = 0; i < MAXW / 4; i++) {
        if (4 * i >= k) break;
        const int kr = 4 * i + kq;
        const T *crow = Cs + (roff + kr) * NC + lc;
        const bool ok = kr < k;
#pragma unroll
        for (int nt = 0; nt < NT; nt++) acc[nt] = Mfma<T>::mma(av[i], ok ? crow[16 * nt] : T(0), acc[nt]);
    }
}

// Shared-memory layout of both kernels
template <typename T, int NT>
struct MVShared {
    T *tile, *Cs;
    double *theta, *red;
    int *cmap, *opos, *wpos;
    __device__ MVShared(unsigned char *smem, const MVDev<T> &a, bool staged)
    {
        const int NC = NT * 16;
        tile = reinterpret_cast<T *>(smem);
        Cs = tile + (staged ? TP * LDT : 0);
        theta = reinterpret_cast<double *>(Cs + (a.Kp + 4) * NC);
        red = theta + NC;                                    // [16 slots][2][NC]
        cmap = reinterpret_cast<int *>(red + 16 * 2 * NC);   // [K + 4]
        opos = cmap + a.K + 4;
        wpos = opos + NC;
    }
};

template <typename T, int NT>
__device__ __forceinline__ void mv_setup(const MVShared<T, NT> &sh, const MVDev<T> &a)
{
    const int NC = NT * 16, tid = threadIdx.x;
    for (int i = tid; i < (a.Kp + 4) * NC; i += blockDim.x) {
        const int r = i / NC, c = i % NC;
        sh.Cs[i] = (r < a.K && c < a.kout) ? a.C[r * a.kout + c] : T(0);
    }
    int roff = 0;
    for (int b = 0; b < a.nin; b++) {
        for (int r = tid; r < a.k[b]; r += blockDim.x) sh.cmap[roff + r] = a.cols[b] ? a.cols[b][r] : r;
        roff += a.k[b];
    }
    for (int r = tid; r < 4; r += blockDim.x) sh.cmap[a.K + r] = 0;
    for (int c = tid; c < NC; c += blockDim.x) {
        sh.opos[c] = c < a.kout ? (a.opos ? a.opos[c] : c) : -1;
        sh.wpos[c] = (c < a.kout && a.wpos) ? a.wpos[c] : -1;
        sh.theta[c] = (c < a.kout && a.theta) ? a.theta[c] : 0.0;
    }
}

// write the outputs of side s for the 16 points of this wave
// LDSACC: the residual sums of squares accumulate in this lane's own entries
// of sh.red (the slots mv_norms reduces) instead of in sr / sx
template <typename T, int NT, typename SH, bool SKIP2 = false, bool LDSACC = false>
__device__ __forceinline__ void mv_outputs(const MVDev<T> &a, const SH &sh, int s, i64 p0w,
                                           const typename Mfma<T>::acc (&acc)[NT],
                                           const typename Mfma<T>::acc (&acc2)[NT],
                                           const typename Mfma<T>::acc (&keepX)[NT], double (&sr)[NT],
                                           double (&sx)[NT], int lane)
{
    const bool has2 = a.out2[0] != nullptr, resid = a.partials != nullptr;
    T *out = a.out[s], *out2 = a.out2[s];
#pragma unroll
    for (int r = 0; r < 4; r++) {
        const i64 p = p0w + Mfma<T>::row(lane, r);
        if (p >= a.N) continue;
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            const int c = 16 * nt + (lane & 15);
            if (c >= a.kout) continue;
            T v = acc[nt][r];
            if (a.add && s == 0) v += a.add[p * a.ld2 + c];
            const int q = sh.opos[c];
            if (out && q >= 0) out[p * a.nout + q] = v;
            if (has2 && !SKIP2) out2[p * a.ld2 + c] = acc2[nt][r];
            if (resid && s == 1) {
                const double x = (double)keepX[nt][r];
                const double rv = (double)acc2[nt][r] - sh.theta[c] * x;
                if (LDSACC) {
                    const int slot = (threadIdx.x >> 6) * 4 + (lane >> 4);
                    sh.red[(slot * 2 + 0) * (NT * 16) + c] += rv * rv;
                    sh.red[(slot * 2 + 1) * (NT * 16) + c] += x * x;
                } else {
                    sr[nt] += rv * rv;
                    sx[nt] += x * x;
                }
                const int w = sh.wpos[c];
                if (w >= 0) a.Wout[p * a.nW + w] = (T)rv;
            }
        }
    }
}

// per-workgroup norm sums: lanes l, l+16, l+32, l+48 of every wave share a column
template <typename T, int NT, typename SH, bool LDSACC = false>
__device__ __forceinline__ void mv_norms(const MVDev<T> &a, const SH &sh, const double (&sr)[NT],
                                         const double (&sx)[NT], int wave, int lane)
{
    const int NC = NT * 16, tid = threadIdx.x;
    const int slot = wave * 4 + (lane >> 4);
    if (!LDSACC) {
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            const int c = 16 * nt + (lane & 15);
            sh.red[(slot * 2 + 0) * NC + c] = sr[nt];
            sh.red[(slot * 2 + 1) * NC + c] = sx[nt];
        }
    }
    __syncthreads();
    for (int e = tid; e < 2 * a.kout; e += blockDim.x) {
        const int which = e / a.kout, c = e % a.kout;
        double sum = 0.0;
        for (int sl = 0; sl < 16; sl++) sum += sh.red[(sl * 2 + which) * NC + c];
        a.partials[(i64)blockIdx.x * 2 * a.kout + e] = sum;
    }
}

// Staged kernel: wide inputs through LDS (prefetched one stage ahead), narrow
// inputs straight from global memory.
template <typename T, int NT>
__global__ void __launch_bounds__(256) mv_kernel(MVDev<T> a)
{
    typedef typename Mfma<T>::acc accT;
    extern __shared__ unsigned char smem[];
    MVShared<T, NT> sh(smem, a, true);
    mv_setup<T, NT>(sh, a);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int roffs[3] = {0, a.k[0], a.k[0] + a.k[1]};
    __syncthreads();

    const bool has2 = a.out2[0] != nullptr;
    // processing order within a side: with a second output, inputs 1.. first
    // (they form out), then input 0 on top (out2)
    int order[3];
    for (int q = 0; q < a.nin; q++) order[q] = has2 ? (q + 1) % a.nin : q;
    // the staged (wide) inputs of one tile, in order: stage k is (side, input)
    int st_s[6], st_b[6], nst = 0;
    for (int s = 0; s < a.nside; s++)
        for (int q = 0; q < a.nin; q++)
            if (a.ld[order[q]] > NARROW) st_s[nst] = s, st_b[nst] = order[q], nst++;

    double sr[NT], sx[NT];
#pragma unroll
    for (int nt = 0; nt < NT; nt++) sr[nt] = sx[nt] = 0.0;
    const T *arow = sh.tile + (16 * wave + (lane & 15)) * LDT;

    const i64 ntiles = (a.N + TP - 1) / TP;
    StageRegs<T> R;
    if ((i64)blockIdx.x < ntiles)
        stage_load<T>(R, a.in[st_s[0]][st_b[0]], a.ld[st_b[0]], (i64)blockIdx.x * TP, a.N);
    for (i64 t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const i64 p0 = t * TP, p0w = p0 + 16 * wave, prow = p0w + (lane & 15);
        const bool pok = prow < a.N;
        int k = 0;   // next stage of this tile
        accT keepX[NT];
        for (int s = 0; s < a.nside; s++) {
            accT acc[NT], acc2[NT];
#pragma unroll
            for (int nt = 0; nt < NT; nt++) acc[nt] = acc_zero<T>(), acc2[nt] = acc_zero<T>();
            // one input into a fixed accumulator array (a runtime choice of
            // array would force the accumulators out of registers)
            auto input = [&](accT(&tgt)[NT], int b) {
                if (a.ld[b] > NARROW) {
                    __syncthreads();
                    stage_store<T>(sh.tile, R, a.ld[b]);
                    // prefetch the next stage: of this tile, or the first of the next tile
                    const int kn = k + 1 < nst ? k + 1 : 0;
                    const i64 tn = k + 1 < nst ? t : t + gridDim.x;
                    if (tn < ntiles) stage_load<T>(R, a.in[st_s[kn]][st_b[kn]], a.ld[st_b[kn]], tn * TP, a.N);
                    k++;
                    __syncthreads();
                    mma_lds<T, NT>(tgt, arow, sh.Cs, sh.cmap, roffs[b], a.k[b], lane);
                } else {
                    mma_global<T, NT>(tgt, a.in[s][b] + prow * a.ld[b], pok, sh.Cs, sh.cmap, roffs[b], a.k[b],
                                      lane);
                }
            };
            for (int b = has2 ? 1 : 0; b < a.nin; b++) input(acc, b);
            if (has2) {
#pragma unroll
                for (int nt = 0; nt < NT; nt++) acc2[nt] = acc[nt];
                input(acc2, 0);
            }
            mv_outputs<T, NT>(a, sh, s, p0w, acc, acc2, keepX, sr, sx, lane);
            if (s == 0) {
#pragma unroll
                for (int nt = 0; nt < NT; nt++) keepX[nt] = acc2[nt];
            }
        }
    }
    if (a.partials) mv_norms<T, NT>(a, sh, sr, sx, wave, lane);
}

// All inputs straight from global memory: each wave owns groups of 16 grid
// points and runs without workgroup barriers.
template <typename T, int NT>
__global__ void __launch_bounds__(256) mvd_kernel(MVDev<T> a)
{
    typedef typename Mfma<T>::acc accT;
    extern __shared__ unsigned char smem[];
    MVShared<T, NT> sh(smem, a, false);
    mv_setup<T, NT>(sh, a);
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int roffs[3] = {0, a.k[0], a.k[0] + a.k[1]};
    __syncthreads();

    const bool has2 = a.out2[0] != nullptr;
    double sr[NT], sx[NT];
#pragma unroll
    for (int nt = 0; nt < NT; nt++) sr[nt] = sx[nt] = 0.0;

    const i64 ngroups = (a.N + 15) / 16;
    for (i64 g = (i64)blockIdx.x * 4 + wave; g < ngroups; g += (i64)gridDim.x * 4) {
        const i64 p0w = g * 16, prow = p0w + (lane & 15);
        const bool pok = prow < a.N;
        accT keepX[NT];
        for (int s = 0; s < a.nside; s++) {
            accT acc[NT], acc2[NT];
#pragma unroll
            for (int nt = 0; nt < NT; nt++) acc[nt] = acc_zero<T>(), acc2[nt] = acc_zero<T>();
            for (int b = has2 ? 1 : 0; b < a.nin; b++)
                mma_global<T, NT>(acc, a.in[s][b] + prow * a.ld[b], pok, sh.Cs, sh.cmap, roffs[b], a.k[b], lane);
            if (has2) {
#pragma unroll
                for (int nt = 0; nt < NT; nt++) acc2[nt] = acc[nt];
                mma_global<T, NT>(acc2, a.in[s][0] + prow * a.ld[0], pok, sh.Cs, sh.cmap, 0, a.k[0], lane);
            }
            mv_outputs<T, NT>(a, sh, s, p0w, acc, acc2, keepX, sr, sx, lane);
            if (s == 0) {
#pragma unroll
                for (int nt = 0; nt < NT; nt++) keepX[nt] = acc2[nt];
            }
        }
    }
    if (a.partials) mv_norms<T, NT>(a, sh, sr, sx, wave, lane);
}

// Fragment kernel: A-fragments loaded straight from global memory with
// 16-byte loads.  The k-sum of an input is split among the four lane groups
// of the MFMA's A operand by contiguous quarters instead of by residues mod 4:
// at k-step i lane l holds column (l/16)*k4 + i of its row (k4 = ceil(k/4)),
// so a lane's k4 values are consecutive in memory.  The coefficient operand
// follows the same permutation and is kept in LDS in fragment order
// (Cf[step][nt][lane]), so that its reads are conflict-free and need no index
// arithmetic.  Each wave owns groups of 16 grid points; no workgroup barrier
// after the set-up.
static const int KQ = MAXW / 4;    // most k-steps of one input

__host__ __device__ inline size_t mvf_stage_offset(int nsteps, int NT, int K, size_t esz);

// k-steps of one input in the fragment kernel: ceil(k/4), rounded up to whole
// 16-byte vectors per lane when the rows load as vectors (no column list,
// 16-byte aligned rows), so that each lane's quarter of a row is a run of
// vectors; the extra steps multiply zeros
__host__ __device__ inline int mvf_k4(int k, int ld, bool mapped, int esz)
{
    const int VE = 16 / esz;
    int k4 = (k + 3) / 4;
    if (!mapped && ld % VE == 0) k4 = (k4 + VE - 1) / VE * VE;
    return k4;
}

template <typename T, int NT>
struct MVFShared {
    T *Cf;                 // [sum k4][NT][64]
    double *theta, *red;
    int *cmap, *opos, *wpos;
    T *stage;              // [4 waves][16][NC + 4]: one output tile of each wave
    __device__ MVFShared(unsigned char *smem, const MVDev<T> &a, int nsteps)
    {
        const int NC = NT * 16;
        Cf = reinterpret_cast<T *>(smem);
        theta = reinterpret_cast<double *>(Cf + nsteps * NT * 64);
        red = theta + NC;
        cmap = reinterpret_cast<int *>(red + 16 * 2 * NC);
        opos = cmap + a.K + 4;
        wpos = opos + NC;
        stage = reinterpret_cast<T *>(reinterpret_cast<unsigned char *>(smem) +
                                      mvf_stage_offset(nsteps, NT, a.K, sizeof(T)));
    }
};

// the output staging area of MVFShared: after the other arrays, 16-byte aligned
__host__ __device__ inline size_t mvf_stage_offset(int nsteps, int NT, int K, size_t esz)
{
    const int NC = NT * 16;
    size_t off = (size_t)nsteps * NT * 64 * esz;
    off = (off + 7) / 8 * 8 + (size_t)NC * 8 + (size_t)16 * 2 * NC * 8 + (size_t)(K + 4 + 2 * NC) * sizeof(int);
    return (off + 15) / 16 * 16;
}
__host__ __device__ inline size_t mvf_stage_bytes(int NT, size_t esz) { return (size_t)4 * 16 * (NT * 16 + 4) * esz; }

// av[i] = column (l/16)*k4 + i of this lane's row (zero past k or the grid);
// rowlen: columns of the row from base on, aligned: base is 16-byte aligned
// for every row
// WHOLE: rowlen is a multiple of the vector length whenever the rows are
// aligned (whole stored rows), so a vector that starts before column k ends
// inside the row
template <typename T, bool WHOLE = false>
__device__ __forceinline__ void frag_load(T (&av)[KQ], const T *__restrict__ base, int rowlen, bool aligned, int k,
                                          int k4, const int *__restrict__ cmap, bool mapped, bool pok, int kq)
{
    const int VE = 16 / sizeof(T);
    const int j0 = kq * k4;
    if (!mapped && aligned && (k4 % VE) == 0) {
#pragma unroll
        for (int i = 0; i < KQ; i += VE) {
            if (i >= k4) break;
            const int col = j0 + i;
            vec<T, VE> v;
            if (WHOLE || col + VE <= rowlen) {
                v = (pok && col < k) ? vload<T, VE>(base + col) : vzero<T, VE>();
            } else {
                // a vector would run past the stored row: element by element
#pragma unroll
                for (int q = 0; q < VE; q++) v.v[q] = (pok && col + q < k) ? base[col + q] : T(0);
            }
#pragma unroll
            for (int q = 0; q < VE; q++) av[i + q] = (col + q < k) ? v.v[q] : T(0);
        }
    } else {
#pragma unroll
        for (int i = 0; i < KQ; i++) {
            if (i >= k4) break;
            const int j = j0 + i;
            av[i] = (pok && j < k) ? base[mapped ? cmap[j] : j] : T(0);
        }
    }
}

// Four waves per SIMD (at most 128 VGPRs, a few spilled): the kernel is bound
// by the load bytes in flight, and a fourth wave per SIMD raises them by a
// third (measured: 3.7 -> 4.2 TB/s for FP32 blocks, 4.6 -> 4.8 TB/s for FP64).
template <typename T, int NT>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8))) mvf_kernel(MVDev<T> a)
{
    typedef typename Mfma<T>::acc accT;
    extern __shared__ unsigned char smem[];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, kq = lane >> 4;
    const int NC = NT * 16;
    int k4[3], soff[3], roffs[3];
    int nsteps = 0, roff = 0;
    for (int b = 0; b < 3; b++) {
        k4[b] = b < a.nin ? mvf_k4(a.k[b], a.ld[b], a.cols[b] != nullptr, sizeof(T)) : 0;
        soff[b] = nsteps;
        roffs[b] = roff;
        nsteps += k4[b];
        roff += b < a.nin ? a.k[b] : 0;
    }
    MVFShared<T, NT> sh(smem, a, nsteps);
    // coefficients in fragment order
    for (int e = tid; e < nsteps * NT * 64; e += blockDim.x) {
        const int l = e & 63, nt = (e >> 6) % NT, st = (e >> 6) / NT;
        int b = 0;
        while (b + 1 < a.nin && st >= soff[b + 1]) b++;
        const int i = st - soff[b];
        const int j = (l >> 4) * k4[b] + i, c = 16 * nt + (l & 15);
        sh.Cf[e] = (j < a.k[b] && c < a.kout) ? a.C[(roffs[b] + j) * a.kout + c] : T(0);
    }
    for (int b = 0; b < a.nin; b++)
        for (int r = tid; r < a.k[b]; r += blockDim.x) sh.cmap[roffs[b] + r] = a.cols[b] ? a.cols[b][r] : r;
    for (int c = tid; c < NC; c += blockDim.x) {
        sh.opos[c] = c < a.kout ? (a.opos ? a.opos[c] : c) : -1;
        sh.wpos[c] = (c < a.kout && a.wpos) ? a.wpos[c] : -1;
        sh.theta[c] = (c < a.kout && a.theta) ? a.theta[c] : 0.0;
    }
    // the residual sums of squares accumulate in LDS (registers are kept for
    // the loads in flight); each lane owns its entries
    {
        const int slot = wave * 4 + (lane >> 4);
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            const int c = 16 * nt + (lane & 15);
            sh.red[(slot * 2 + 0) * NC + c] = 0.0;
            sh.red[(slot * 2 + 1) * NC + c] = 0.0;
        }
    }
    __syncthreads();

    const bool has2 = a.out2[0] != nullptr;
    double sr[NT], sx[NT];
#pragma unroll
    for (int nt = 0; nt < NT; nt++) sr[nt] = sx[nt] = 0.0;

    // the MFMAs of one input whose fragments are loaded, into a fixed
    // accumulator array (a runtime choice of array would force the
    // accumulators out of registers)
    auto mma_in = [&](accT(&tgt)[NT], const T(&av)[KQ], int b) {
        const T *cf = sh.Cf + soff[b] * NT * 64 + lane;
#pragma unroll
        for (int i = 0; i < KQ; i++) {
            if (i >= k4[b]) break;
#pragma unroll
            for (int nt = 0; nt < NT; nt++) tgt[nt] = Mfma<T>::mma(av[i], cf[(i * NT + nt) * 64], tgt[nt]);
        }
    };
    auto load_in = [&](T(&av)[KQ], int s, int b, i64 prow, bool pok) {
        frag_load<T, true>(av, a.in[s][b] + prow * a.ld[b], a.ld[b], (a.ld[b] % (16 / (int)sizeof(T))) == 0, a.k[b],
                     k4[b], sh.cmap + roffs[b], a.cols[b] != nullptr, pok, kq);
    };
    const i64 ngroups = (a.N + 15) / 16, gstride = (i64)gridDim.x * 4;
    i64 g = (i64)blockIdx.x * 4 + wave;
    if constexpr (sizeof(T) == 4) {
        const bool stage2 = has2 && (a.kout % 4) == 0 && (a.ld2 % 4) == 0;
        // FP32: input 0 (X, the widest block, or the only input) is loaded for
        // both sides one group ahead, so that its loads are in flight while the
        // current group is multiplied
        auto load0 = [&](T(&dst)[2][KQ], i64 gg) {
            const i64 prow = gg * 16 + (lane & 15);
#pragma unroll
            for (int s = 0; s < 2; s++)
                if (s < a.nside) load_in(dst[s], s, 0, prow, prow < a.N);
        };
        T x0[2][KQ];
        if (g < ngroups) load0(x0, g);
        for (; g < ngroups; g += gstride) {
            const i64 p0w = g * 16, prow = p0w + (lane & 15);
            const bool pok = prow < a.N;
            T xn[2][KQ];
            if (g + gstride < ngroups) load0(xn, g + gstride);
            accT keepX[NT];
#pragma unroll
            for (int s = 0; s < 2; s++) {
                if (s >= a.nside) break;
                accT acc[NT], acc2[NT];
#pragma unroll
                for (int nt = 0; nt < NT; nt++) acc[nt] = acc_zero<T>(), acc2[nt] = acc_zero<T>();
                if (!has2) mma_in(acc, x0[s], 0);
                for (int b = 1; b < a.nin; b++) {
                    T av[KQ];
                    load_in(av, s, b, prow, pok);
                    mma_in(acc, av, b);
                }
                if (has2) {
#pragma unroll
                    for (int nt = 0; nt < NT; nt++) acc2[nt] = acc[nt];
                    mma_in(acc2, x0[s], 0);
                }
                if (stage2) {
                    // out2 through LDS: the MFMA layout gives each lane one
                    // column of four rows; after the transpose each lane holds
                    // four consecutive columns of one row and stores 16 bytes.
                    // The tile is private to this wave and LDS operations of
                    // one wave complete in order.
                    mv_outputs<T, NT, MVFShared<T, NT>, true, true>(a, sh, s, p0w, acc, acc2, keepX, sr, sx, lane);
                    T *st = sh.stage + wave * 16 * (NC + 4);
#pragma unroll
                    for (int r = 0; r < 4; r++)
#pragma unroll
                        for (int nt = 0; nt < NT; nt++)
                            st[Mfma<T>::row(lane, r) * (NC + 4) + 16 * nt + (lane & 15)] = acc2[nt][r];
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    const int row = lane >> 2;
                    const i64 p = p0w + row;
#pragma unroll
                    for (int h = 0; h < NT * 4 / 4; h++) {
                        const int c0 = 4 * ((lane & 3) + 4 * h);
                        const vec<T, 4> v = *reinterpret_cast<const vec<T, 4> *>(st + row * (NC + 4) + c0);
                        if (p < a.N && c0 < a.kout) vstore<T, 4>(a.out2[s] + p * a.ld2 + c0, v);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                } else {
                    mv_outputs<T, NT, MVFShared<T, NT>, false, true>(a, sh, s, p0w, acc, acc2, keepX, sr, sx, lane);
                }
                if (s == 0) {
#pragma unroll
                    for (int nt = 0; nt < NT; nt++) keepX[nt] = acc2[nt];
                }
            }
#pragma unroll
            for (int s = 0; s < 2; s++)
#pragma unroll
                for (int i = 0; i < KQ; i++) x0[s][i] = xn[s][i];
        }
    } else {
        // FP64: each input loaded right before its products (the registers of
        // a second group would cost occupancy)
        auto input = [&](accT(&tgt)[NT], int s, int b, i64 prow, bool pok) {
            T av[KQ];
            load_in(av, s, b, prow, pok);
            mma_in(tgt, av, b);
        };
        for (; g < ngroups; g += gstride) {
            const i64 p0w = g * 16, prow = p0w + (lane & 15);
            const bool pok = prow < a.N;
            accT keepX[NT];
            for (int s = 0; s < a.nside; s++) {
                accT acc[NT], acc2[NT];
#pragma unroll
                for (int nt = 0; nt < NT; nt++) acc[nt] = acc_zero<T>(), acc2[nt] = acc_zero<T>();
                for (int b = has2 ? 1 : 0; b < a.nin; b++) input(acc, s, b, prow, pok);
                if (has2) {
#pragma unroll
                    for (int nt = 0; nt < NT; nt++) acc2[nt] = acc[nt];
                    input(acc2, s, 0, prow, pok);
                }
                mv_outputs<T, NT, MVFShared<T, NT>, false, true>(a, sh, s, p0w, acc, acc2, keepX, sr, sx, lane);
                if (s == 0) {
#pragma unroll
                    for (int nt = 0; nt < NT; nt++) keepX[nt] = acc2[nt];
                }
            }
        }
    }
    if (a.partials) mv_norms<T, NT, MVFShared<T, NT>, true>(a, sh, sr, sx, wave, lane);
}

// Wide kernel: blocks of more than MAXW columns, given as up to MV_MAX_IN
// pieces of at most MAXW columns each (a piece is a column range or a column
// list of one block).  The products are those of the fragment kernel's FP64
// branch, one piece after another; the per-piece tables live in LDS so that
// the piece loop can run over a runtime count without private arrays.  With
// out2 the first n0 pieces form the X part: acc = the sum over the pieces
// from n0 on, acc2 = acc + the X pieces.
template <typename T, int NT>
__global__ void __launch_bounds__(256) mvw_kernel(MVDev<T> a)
{
    typedef typename Mfma<T>::acc accT;
    extern __shared__ unsigned char smem[];
    __shared__ int tk4[MV_MAX_IN], tsoff[MV_MAX_IN], troff[MV_MAX_IN];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, kq = lane >> 4;
    const int NC = NT * 16;
    int nsteps = 0;
    for (int b = 0; b < a.nin; b++) nsteps += (a.k[b] + 3) / 4;
    if (tid == 0) {
        int st = 0, ro = 0;
        for (int b = 0; b < a.nin; b++) {
            tk4[b] = (a.k[b] + 3) / 4;
            tsoff[b] = st;
            troff[b] = ro;
            st += tk4[b];
            ro += a.k[b];
        }
    }
    __syncthreads();
    MVFShared<T, NT> sh(smem, a, nsteps);
    for (int e = tid; e < nsteps * NT * 64; e += blockDim.x) {
        const int l = e & 63, nt = (e >> 6) % NT, st = (e >> 6) / NT;
        int b = 0;
        while (b + 1 < a.nin && st >= tsoff[b + 1]) b++;
        const int i = st - tsoff[b];
        const int j = (l >> 4) * tk4[b] + i, c = 16 * nt + (l & 15);
        sh.Cf[e] = (j < a.k[b] && c < a.kout) ? a.C[(troff[b] + j) * a.kout + c] : T(0);
    }
    for (int b = 0; b < a.nin; b++)
        for (int r = tid; r < a.k[b]; r += blockDim.x) sh.cmap[troff[b] + r] = a.cols[b] ? a.cols[b][r] : r;
    for (int c = tid; c < NC; c += blockDim.x) {
        sh.opos[c] = c < a.kout ? (a.opos ? a.opos[c] : c) : -1;
        sh.wpos[c] = (c < a.kout && a.wpos) ? a.wpos[c] : -1;
        sh.theta[c] = (c < a.kout && a.theta) ? a.theta[c] : 0.0;
    }
    __syncthreads();

    const bool has2 = a.out2[0] != nullptr;
    double sr[NT], sx[NT];
#pragma unroll
    for (int nt = 0; nt < NT; nt++) sr[nt] = sx[nt] = 0.0;
    auto input = [&](accT(&tgt)[NT], int s, int b, i64 prow, bool pok) {
        const int k4 = tk4[b], ld = a.ld[b], co = a.coff[b];
        T av[KQ];
        frag_load<T>(av, a.in[s][b] + prow * ld + co, ld - co, ((ld | co) % (16 / (int)sizeof(T))) == 0, a.k[b], k4,
                     sh.cmap + troff[b], a.cols[b] != nullptr, pok, kq);
        const T *cf = sh.Cf + tsoff[b] * NT * 64 + lane;
#pragma unroll
        for (int i = 0; i < KQ; i++) {
            if (i >= k4) break;
#pragma unroll
            for (int nt = 0; nt < NT; nt++) tgt[nt] = Mfma<T>::mma(av[i], cf[(i * NT + nt) * 64], tgt[nt]);
        }
    };
    const i64 ngroups = (a.N + 15) / 16, gstride = (i64)gridDim.x * 4;
    for (i64 g = (i64)blockIdx.x * 4 + wave; g < ngroups; g += gstride) {
        const i64 p0w = g * 16, prow = p0w + (lane & 15);
        const bool pok = prow < a.N;
        accT keepX[NT];
        for (int s = 0; s < a.nside; s++) {
            accT acc[NT], acc2[NT];
#pragma unroll
            for (int nt = 0; nt < NT; nt++) acc[nt] = acc_zero<T>(), acc2[nt] = acc_zero<T>();
            for (int b = has2 ? a.n0 : 0; b < a.nin; b++) input(acc, s, b, prow, pok);
            if (has2) {
#pragma unroll
                for (int nt = 0; nt < NT; nt++) acc2[nt] = acc[nt];
                for (int b = 0; b < a.n0; b++) input(acc2, s, b, prow, pok);
            }
            mv_outputs<T, NT>(a, sh, s, p0w, acc, acc2, keepX, sr, sx, lane);
            if (s == 0) {
#pragma unroll
                for (int nt = 0; nt < NT; nt++) keepX[nt] = acc2[nt];
            }
        }
    }
    if (a.partials) mv_norms<T, NT>(a, sh, sr, sx, wave, lane);
}

// Narrow kernel (every input at most NARROW stored columns, at most NARROW
// outputs): one thread per grid point, plain FMA with the coefficients read
// from LDS (every lane reads the same word: a broadcast).  The k-sum runs in
// input order, columns ascending.
template <typename T>
__global__ void __launch_bounds__(256) mvn_kernel(MVDev<T> a)
{
    extern __shared__ unsigned char smem[];
    double *theta = reinterpret_cast<double *>(smem);       // [NARROW]
    double *red = theta + NARROW;                           // [256][2][NARROW] -> reused
    T *Cs = reinterpret_cast<T *>(red + 2 * NARROW * 256);  // [K][NARROW]
    int *cmap = reinterpret_cast<int *>(Cs + a.K * NARROW); // [K]
    int *opos = cmap + a.K, *wpos = opos + NARROW;
    const int tid = threadIdx.x;
    for (int e = tid; e < a.K * NARROW; e += blockDim.x) {
        const int r = e / NARROW, c = e % NARROW;
        Cs[e] = c < a.kout ? a.C[r * a.kout + c] : T(0);
    }
    int roffs[3], roff = 0;
    for (int b = 0; b < 3; b++) {
        roffs[b] = roff;
        if (b < a.nin) {
            for (int r = tid; r < a.k[b]; r += blockDim.x) cmap[roff + r] = a.cols[b] ? a.cols[b][r] : r;
            roff += a.k[b];
        }
    }
    for (int c = tid; c < NARROW; c += blockDim.x) {
        opos[c] = c < a.kout ? (a.opos ? a.opos[c] : c) : -1;
        wpos[c] = (c < a.kout && a.wpos) ? a.wpos[c] : -1;
        theta[c] = (c < a.kout && a.theta) ? a.theta[c] : 0.0;
    }
    __syncthreads();
    const bool has2 = a.out2[0] != nullptr, resid = a.partials != nullptr;
    double sr[NARROW], sx[NARROW];
#pragma unroll
    for (int c = 0; c < NARROW; c++) sr[c] = sx[c] = 0.0;

    for (i64 p = (i64)blockIdx.x * blockDim.x + tid; p < a.N; p += (i64)gridDim.x * blockDim.x) {
        T keepX[NARROW];
        for (int s = 0; s < a.nside; s++) {
            T acc[NARROW], acc2[NARROW];
#pragma unroll
            for (int c = 0; c < NARROW; c++) acc[c] = T(0);
            auto input = [&](T(&tgt)[NARROW], int b) {
                const T *row = a.in[s][b] + p * a.ld[b];
                const int *cm = cmap + roffs[b];
                const T *cr = Cs + roffs[b] * NARROW;
                T v[NARROW];
#pragma unroll
                for (int j = 0; j < NARROW; j++) v[j] = j < a.k[b] ? row[cm[j]] : T(0);
#pragma unroll
                for (int j = 0; j < NARROW; j++) {
                    if (j >= a.k[b]) break;
#pragma unroll
                    for (int c = 0; c < NARROW; c++) tgt[c] += v[j] * cr[j * NARROW + c];
                }
            };
            for (int b = has2 ? 1 : 0; b < a.nin; b++) input(acc, b);
            if (has2) {
#pragma unroll
                for (int c = 0; c < NARROW; c++) acc2[c] = acc[c];
                input(acc2, 0);
            }
            T *out = a.out[s], *out2 = a.out2[s];
#pragma unroll
            for (int c = 0; c < NARROW; c++) {
                if (c >= a.kout) break;
                T v = acc[c];
                if (a.add && s == 0) v += a.add[p * a.ld2 + c];
                if (out && opos[c] >= 0) out[p * a.nout + opos[c]] = v;
                if (has2) out2[p * a.ld2 + c] = acc2[c];
                if (resid && s == 1) {
                    const double x = (double)keepX[c];
                    const double rv = (double)acc2[c] - theta[c] * x;
                    sr[c] += rv * rv;
                    sx[c] += x * x;
                    if (wpos[c] >= 0) a.Wout[p * a.nW + wpos[c]] = (T)rv;
                }
            }
            if (s == 0 && has2) {
#pragma unroll
                for (int c = 0; c < NARROW; c++) keepX[c] = acc2[c];
            }
        }
    }
    if (resid) {
        // fixed-order workgroup sum: per thread slots, then a tree over threads
        __syncthreads();
#pragma unroll
        for (int c = 0; c < NARROW; c++) {
            red[(0 * NARROW + c) * 256 + tid] = sr[c];
            red[(1 * NARROW + c) * 256 + tid] = sx[c];
        }
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if (tid < h)
                for (int e = 0; e < 2 * NARROW; e++) red[e * 256 + tid] += red[e * 256 + tid + h];
            __syncthreads();
        }
        for (int e = tid; e < 2 * a.kout; e += blockDim.x) {
            const int which = e / a.kout, c = e % a.kout;
            a.partials[(i64)blockIdx.x * 2 * a.kout + e] = red[(which * NARROW + c) * 256];
        }
    }
}

// sums over workgroups of partials[b][e], e = which * kc + c, written to
// out[which * ld + c]: one workgroup per entry, strided partial sums then a
// fixed-shape tree, so the order never changes.
__global__ void __launch_bounds__(256) mv_reduce_kernel(const double *__restrict__ partials, int nb, int width,
                                                        int kc, int ld, double *__restrict__ out)
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
    if (threadIdx.x == 0) out[(e / kc) * ld + e % kc] = red[0];
}

// both kernels cover 64 grid points per workgroup pass (4 waves x 16 points)
int mv_blocks(long long N)
{
    long long nt = (N + TP - 1) / TP;
    return (int)(nt < MV_MAX_BLOCKS ? (nt > 0 ? nt : 1) : MV_MAX_BLOCKS);
}

// dynamic LDS of the wide kernel for pieces of widths k[0..nin)
static size_t mvw_lds(int NT, size_t esz, int nin, const int *k)
{
    int nsteps = 0, K = 0;
    for (int b = 0; b < nin; b++) nsteps += (k[b] + 3) / 4, K += k[b];
    return mvf_stage_offset(nsteps, NT, K, esz);
}
static const size_t MVW_MAX_LDS = 64 * 1024 - 256;   // with the kernel's static tables

int mv_wide_chunk(int dtype, int nin, const int *k)
{
    const size_t esz = dtype == DT_F32 ? 4 : 8;
    if (mvw_lds(4, esz, nin, k) <= MVW_MAX_LDS) return 64;
    if (mvw_lds(2, esz, nin, k) <= MVW_MAX_LDS) return 32;
    if (mvw_lds(1, esz, nin, k) <= MVW_MAX_LDS) return 16;
    return 0;
}

template <typename T>
static MVDev<T> make_dev(const MVArgs &h, bool &any_wide)
{
    MVDev<T> a;
    a.K = 0;
    any_wide = false;
    for (int b = 0; b < MV_MAX_IN; b++) {
        const bool used = b < h.nin;
        for (int s = 0; s < 2; s++) a.in[s][b] = used ? (const T *)h.in[s][b] : nullptr;
        a.ld[b] = used ? h.ld[b] : 1;
        a.k[b] = used ? h.k[b] : 0;
        a.cols[b] = used ? h.cols[b] : nullptr;
        a.coff[b] = used ? h.coff[b] : 0;
        a.K += a.k[b];
        if (used && h.ld[b] > NARROW) any_wide = true;
    }
    a.nin = h.nin;
    a.n0 = h.n0;
    a.ld2 = h.ld2 > 0 ? h.ld2 : h.kout;
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
    return a;
}

// the column sums of the residual, reduced in a fixed order
static hipError_t mv_reduce(const MVArgs &h, int nb, hipStream_t st)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !h.partials) return e;
    hipLaunchKernelGGL(mv_reduce_kernel, dim3(2 * h.kout), dim3(256), 0, st, h.partials, nb, 2 * h.kout, h.kout,
                       h.sums_ld > 0 ? h.sums_ld : h.kout, h.sums);
    return hipGetLastError();
}

// blocks wider than MAXW columns (pieces, chunked outputs): mvw_kernel
template <typename T, int NT>
static hipError_t run_mvw(const MVArgs &h, hipStream_t st)
{
    bool any_wide;
    MVDev<T> a = make_dev<T>(h, any_wide);
    const int nb = mv_blocks(h.N);
    int nsteps = 0;
    for (int b = 0; b < h.nin; b++) nsteps += (h.k[b] + 3) / 4;
    const size_t shm = mvf_stage_offset(nsteps, NT, a.K, sizeof(T));
    hipLaunchKernelGGL((mvw_kernel<T, NT>), dim3(nb), dim3(256), shm, st, a);
    return mv_reduce(h, nb, st);
}

template <typename T, int NT>
static hipError_t run_mv(const MVArgs &h, hipStream_t st)
{
    bool any_wide;
    MVDev<T> a = make_dev<T>(h, any_wide);
    const int NC = NT * 16;
    const int nb = mv_blocks(h.N);
    bool narrow = h.kout <= NARROW;
    for (int b = 0; b < h.nin; b++) narrow = narrow && h.ld[b] <= NARROW;
    const size_t tail = (size_t)NC * 8 + (size_t)16 * 2 * NC * 8 + (size_t)(a.K + 4 + 2 * NC) * sizeof(int);
    if (h.variant == 0 && narrow) {
        const size_t shm = (size_t)NARROW * 8 + (size_t)2 * NARROW * 256 * 8 + (size_t)a.K * NARROW * sizeof(T) +
                           (size_t)(a.K + 2 * NARROW) * sizeof(int);
        hipLaunchKernelGGL((mvn_kernel<T>), dim3(nb), dim3(256), shm, st, a);
    } else if (h.variant == 0) {
        int nsteps = 0;
        for (int b = 0; b < h.nin; b++) nsteps += mvf_k4(h.k[b], h.ld[b], h.cols[b] != nullptr, sizeof(T));
        const size_t shm = mvf_stage_offset(nsteps, NT, a.K, sizeof(T)) + mvf_stage_bytes(NT, sizeof(T));
        hipLaunchKernelGGL((mvf_kernel<T, NT>), dim3(nb), dim3(256), shm, st, a);
    } else {
        const bool staged = any_wide && h.variant == 2;
        size_t shm = (staged ? (size_t)TP * LDT * sizeof(T) : 0) + (size_t)(a.Kp + 4) * NC * sizeof(T);
        shm = (shm + 7) / 8 * 8 + tail;
        if (staged)
            hipLaunchKernelGGL((mv_kernel<T, NT>), dim3(nb), dim3(256), shm, st, a);
        else
            hipLaunchKernelGGL((mvd_kernel<T, NT>), dim3(nb), dim3(256), shm, st, a);
    }
    return mv_reduce(h, nb, st);
}

hipError_t launch_mv(int dtype, const MVArgs &a, hipStream_t st)
{
    if (a.N == 0) return hipSuccess;
    if (a.nin < 1 || a.nin > MV_MAX_IN || a.nside < 1 || a.nside > 2) return hipErrorInvalidValue;
    // the wide kernel takes more than 3 pieces, stored rows wider than MAXW
    // (pieces of a wider block), X parts of several pieces and chunked outputs
    bool wide = a.nin > 3 || a.n0 != 1 || (a.ld2 > 0 && a.ld2 != a.kout) || (a.sums_ld > 0 && a.sums_ld != a.kout);
    for (int b = 0; b < a.nin; b++) {
        if (a.ld[b] < 1 || a.k[b] < 1 || a.k[b] > MAXW || a.coff[b] < 0) return hipErrorInvalidValue;
        if (a.cols[b] ? a.coff[b] != 0 : a.coff[b] + a.k[b] > a.ld[b]) return hipErrorInvalidValue;
        if (a.ld[b] > MAXW || a.coff[b]) wide = true;
    }
    if (a.kout < 1 || a.kout > (wide ? 64 : 32)) return hipErrorInvalidValue;
    if (a.out2[0] && (a.n0 < 1 || a.n0 > a.nin)) return hipErrorInvalidValue;
    if (a.partials && (a.nside != 2 || !a.out2[0])) return hipErrorInvalidValue;
    if (wide) {
        // 16, 32 or 64 output columns per launch, as the coefficients fit LDS
        const int nt = a.kout > 32 ? 4 : a.kout > 16 ? 2 : 1;
        if (mv_wide_chunk(dtype, a.nin, a.k) < 16 * nt) return hipErrorInvalidValue;
        if (dtype == DT_F32)
            return nt == 4 ? run_mvw<float, 4>(a, st) : nt == 2 ? run_mvw<float, 2>(a, st) : run_mvw<float, 1>(a, st);
        return nt == 4 ? run_mvw<double, 4>(a, st) : nt == 2 ? run_mvw<double, 2>(a, st) : run_mvw<double, 1>(a, st);
    }
    const bool two = a.kout > 16;
    if (dtype == DT_F32) return two ? run_mv<float, 2>(a, st) : run_mv<float, 1>(a, st);
    return two ? run_mv<double, 2>(a, st) : run_mv<double, 1>(a, st);
}

}  // namespace lobpcg
