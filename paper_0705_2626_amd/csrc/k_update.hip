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
// rows x 4 columns of an input.  Three kernels share this scheme:
//   mvf_kernel  fragments loaded straight from global memory with 16-byte
//               loads, the k-sum split in contiguous quarters;
//   mvn_kernel  at most 8 columns in and out: one point per thread, plain FMA;
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
static const int NARROW = 8;       // blocks up to this width: one point per thread (mvn_kernel)
static const int MV_MAX_BLOCKS = 4096;

template <typename T>
struct MVDev {
    const T *in[2][MV_MAX_IN];
    int ld[MV_MAX_IN], k[MV_MAX_IN];
    const int *cols[MV_MAX_IN];
    int coff[MV_MAX_IN];
    int nin, nside, kout, K;
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

// ---------------------------------------------------------------- LDS-pipelined update (FP32)
//
// The fused update of steps 25-33 and 7 for FP32 blocks (mvf_kernel's case
// with X', AX', the residual and two or three inputs of at most 32 stored
// columns; an input given by a column list is loaded whole and its columns
// picked in LDS) with its inputs moved by the buffer loads' LDS path:
// global memory straight into LDS, no registers held while in flight.  Each
// wave walks its 16-point groups one side at a time (side 0: X, W, P; side
// 1: AX, AW, AP) and keeps the loads of the next two sides in flight in a
// two-slot ring while it multiplies the current one, so that the bytes in
// flight no longer depend on the registers (the FP32 fragment kernel holds
// half as many bytes per register as the FP64 one).  The loads and stores
// are inline assembly, so that the number of vector-memory operations issued
// between two sides is fixed and one vmcnt wait per side suffices; loads
// past N and stores of rows past N or of inactive columns use offsets past
// the buffer's range, which the hardware drops (loads return zero).
typedef int mvl_v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void mvl_lds_t;
static const unsigned MVL_OOB = 0x80000000u;   // a buffer offset past every range: the access is dropped

// buffer resource of `bytes` bytes from base (raw: no stride, no format)
__device__ __forceinline__ mvl_v4i mvl_rsrc(const void *base, unsigned bytes)
{
    const unsigned long long p = (unsigned long long)base;
    mvl_v4i r;
    r.x = __builtin_amdgcn_readfirstlane((int)(unsigned)p);
    r.y = __builtin_amdgcn_readfirstlane((int)((unsigned)(p >> 32) & 0xffffu));
    r.z = __builtin_amdgcn_readfirstlane((int)bytes);
    r.w = 0x00020000;
    return r;
}
// stores at byte offset off of buffer r (dropped when off is past its range)
__device__ __forceinline__ void mvl_st1(mvl_v4i r, unsigned off, float v)
{
    asm volatile("buffer_store_dword %0, %1, %2, 0 offen" ::"v"(v), "v"(off), "s"(r) : "memory");
}
__device__ __forceinline__ void mvl_st4(mvl_v4i r, unsigned off, floatx4 v)
{
    asm volatile("buffer_store_dwordx4 %0, %1, %2, 0 offen" ::"v"(v), "v"(off), "s"(r) : "memory");
}
// 16 bytes per lane from global memory (buffer r, byte offset voff) straight
// into LDS at byte address lds + 16 * lane.  Written as inline assembly, so
// that the compiler, which does not see these loads, adds no waits of its own
// before the LDS reads; the kernel waits for them itself (mvl_wait_vm).  The
// kernel uses m0 for nothing else.
__device__ __forceinline__ void mvl_dma16(mvl_v4i r, unsigned lds, unsigned voff)
{
    asm volatile("s_mov_b32 m0, %0\n\tbuffer_load_dwordx4 %1, %2, 0 offen lds" ::"s"(lds), "v"(voff), "s"(r)
                 : "memory");
}
// wait until at most N vector-memory operations of this wave are outstanding
// (they complete in issue order)
template <int N>
__device__ __forceinline__ void mvl_wait_vm()
{
    static_assert(N >= 0 && N < 64, "vmcnt");
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}
__device__ __forceinline__ void mvl_wait_lds() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

static const int MVL_SLOT = 16 * 32;   // floats of one input's 16 rows (at most 32 columns)
static const int MVL_CMAP = 128;       // column-list entries (3 inputs of at most 32 columns, 16-byte multiple)

// SW = 0: P, AP and W leave the MFMA accumulators directly, one 4-byte store
// per 4-row x 16-column fragment (8 per output).  SW = 1, 2 or 4: they have at
// most 4 SW stored columns and leave through the wave's LDS tile as compact
// rows, SW 4-byte stores per output (16 rows x 4 SW columns = 64 SW values):
// with few active columns the fragment stores are mostly dropped lanes, and
// their instructions, not their bytes, cost the time.
template <int NIN, int SW>
__global__ void __launch_bounds__(256) mvl_kernel(MVDev<float> a)
{
    // store instructions per side: P and X' (2), then AP, W and AX' (2)
    constexpr int SO = SW > 0 ? SW : 8;
    constexpr int MVL_ST0 = SO + 2, MVL_ST1 = 2 * SO + 2;
    typedef float T;
    typedef floatx4 accT;
    const int NT = 2, NC = 32;
    extern __shared__ unsigned char smem[];
    const int tid = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, kq = lane >> 4,
              lr = lane & 15;
    int k4[NIN], soff[NIN], roffs[NIN];
    int nsteps = 0, roff = 0;
#pragma unroll
    for (int b = 0; b < NIN; b++) {
        k4[b] = mvf_k4(a.k[b], a.ld[b], a.cols[b] != nullptr, 4);
        soff[b] = nsteps;
        roffs[b] = roff;
        nsteps += k4[b];
        roff += a.k[b];
    }
    T *Cf = reinterpret_cast<T *>(smem);
    double *theta = reinterpret_cast<double *>(Cf + nsteps * NT * 64);
    int *opos = reinterpret_cast<int *>(theta + NC), *wpos = opos + NC;
    int *cmap = wpos + NC;                                       // [MVL_CMAP]: the inputs' column lists
    T *stage = reinterpret_cast<T *>(cmap + MVL_CMAP);           // [4 waves][16][NC + 4]
    T *ring = stage + 4 * 16 * (NC + 4);                         // [4 waves][2][NIN][MVL_SLOT]
    for (int e = tid; e < nsteps * NT * 64; e += blockDim.x) {
        const int l = e & 63, nt = (e >> 6) % NT, st = (e >> 6) / NT;
        // the input of k-step st, without indexing the arrays by a runtime value
        int i = st, kb = a.k[0], k4b = k4[0], rb = 0;
#pragma unroll
        for (int b = 1; b < NIN; b++)
            if (st >= soff[b]) i = st - soff[b], kb = a.k[b], k4b = k4[b], rb = roffs[b];
        const int j = (l >> 4) * k4b + i, c = 16 * nt + (l & 15);
        Cf[e] = (j < kb && c < a.kout) ? a.C[(rb + j) * a.kout + c] : T(0);
    }
    for (int c = tid; c < NC; c += blockDim.x) {
        opos[c] = c < a.kout ? a.opos[c] : -1;
        wpos[c] = c < a.kout ? a.wpos[c] : -1;
        theta[c] = c < a.kout ? a.theta[c] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < NIN; b++)
        if (a.cols[b])
            for (int r = tid; r < a.k[b]; r += blockDim.x) cmap[roffs[b] + r] = a.cols[b][r];
    __syncthreads();

    // SW > 0: value e = 64 i + lane of a compact P / AP (W) row block of a
    // 16-point group, row e / nout and stored column q = e mod nout, comes
    // from the tile column c with opos[c] = q (wpos[c] = q); -1 where no
    // column is stored there (then nothing is written, as with SW = 0)
    int ptile[SW > 0 ? SW : 1], wtile[SW > 0 ? SW : 1];
    if constexpr (SW > 0) {
#pragma unroll
        for (int i = 0; i < SW; i++) {
            const int e = 64 * i + lane;
            ptile[i] = wtile[i] = -1;
            if (e < 16 * a.nout) {
                const int row = e / a.nout, q = e - row * a.nout;
                for (int c = 0; c < NC; c++)
                    if (opos[c] == q) ptile[i] = row * (NC + 4) + c;
            }
            if (e < 16 * a.nW) {
                const int row = e / a.nW, q = e - row * a.nW;
                for (int c = 0; c < NC; c++)
                    if (wpos[c] == q) wtile[i] = row * (NC + 4) + c;
            }
        }
    }

    // per input: the byte offset each lane fetches for DMA instruction j (two
    // per input, 64 lanes x 16 bytes each).  Rows of a multiple of 4 columns
    // go to LDS rotated by their row index, chunk c of row r at chunk
    // (c + r) mod cpr, so that the 16 rows of a fragment read hit distinct banks.
    unsigned voff[NIN][2];
    bool aligned[NIN];
#pragma unroll
    for (int b = 0; b < NIN; b++) {
        const int ld = a.ld[b];
        aligned[b] = (ld % 4) == 0 && !a.cols[b];   // rows rotated in LDS (read as 16-byte chunks)
#pragma unroll
        for (int j = 0; j < 2; j++) {
            const int P = 64 * j + lane;
            unsigned off = MVL_OOB;
            if (P < 4 * ld) {
                if (aligned[b]) {
                    const int cpr = ld / 4, r = P / cpr, cpos = P - r * cpr;
                    const int c = (cpos - r % cpr + cpr) % cpr;
                    off = (unsigned)((r * cpr + c) * 16);
                } else {
                    off = (unsigned)(P * 16);
                }
            }
            voff[b][j] = off;
        }
    }
    T *myring = ring + wave * 2 * NIN * MVL_SLOT;
    const unsigned ring_lds = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(uintptr_t)myring);
    const i64 ngroups = (a.N + 15) / 16, gstride = (i64)gridDim.x * 4, g0 = (i64)blockIdx.x * 4 + wave;
    const int G = g0 < ngroups ? (int)((ngroups - 1 - g0) / gstride + 1) : 0;
    const int Tn = 2 * G;
    auto issue = [&](int t) {
        const i64 p0 = (g0 + (i64)(t >> 1) * gstride) * 16;
        const int s = t & 1;
        const int nrows = (int)min((i64)16, a.N - p0);
#pragma unroll
        for (int b = 0; b < NIN; b++) {
            const mvl_v4i r = mvl_rsrc(a.in[s][b] + p0 * a.ld[b], (unsigned)(nrows * a.ld[b] * 4));
            const unsigned slot = ring_lds + (unsigned)(((t & 1) * NIN + b) * MVL_SLOT * 4);
#pragma unroll
            for (int j = 0; j < 2; j++) mvl_dma16(r, slot + 1024 * j, voff[b][j]);
        }
    };
    // fragments of input b from its LDS slot: av[i] = column kq*k4 + i of row lr
    auto frag = [&](T(&av)[KQ], const T *slot, int b) {
        const int k = a.k[b], ld = a.ld[b], j0 = kq * k4[b];
        if (aligned[b]) {
            const int cpr = ld / 4;
#pragma unroll
            for (int i = 0; i < KQ; i += 4) {
                if (i >= k4[b]) break;
                const int c = (j0 + i) >> 2;
                int cpos = c + lr % cpr;
                cpos = cpos >= cpr ? cpos - cpr : cpos;
                // always read (a chunk past the row is some other chunk of the
                // slot), then keep the columns below k
                const floatx4 v = *reinterpret_cast<const floatx4 *>(slot + ((lr * cpr + cpos) & (MVL_SLOT / 4 - 1)) * 4);
#pragma unroll
                for (int q = 0; q < 4; q++) av[i + q] = (4 * c + q < k) ? v[q] : T(0);
            }
        } else if (a.cols[b]) {
            // a column list (the active columns of a wider block)
            const int *cm = cmap + roffs[b];
#pragma unroll
            for (int i = 0; i < KQ; i++) {
                if (i >= k4[b]) break;
                const int j = j0 + i;
                const T v = slot[(lr * ld + cm[j < k ? j : 0]) & (MVL_SLOT - 1)];
                av[i] = j < k ? v : T(0);
            }
        } else {
#pragma unroll
            for (int i = 0; i < KQ; i++) {
                if (i >= k4[b]) break;
                const int j = j0 + i;
                const T v = slot[(lr * ld + j) & (MVL_SLOT - 1)];
                av[i] = j < k ? v : T(0);
            }
        }
    };
    auto mma_in = [&](accT(&tgt)[NT], const T(&av)[KQ], int b) {
        const T *cf = Cf + soff[b] * NT * 64 + lane;
#pragma unroll
        for (int i = 0; i < KQ; i++) {
            if (i >= k4[b]) break;
#pragma unroll
            for (int nt = 0; nt < NT; nt++) tgt[nt] = Mfma<T>::mma(av[i], cf[(i * NT + nt) * 64], tgt[nt]);
        }
    };
    double sr[NT], sx[NT];
#pragma unroll
    for (int nt = 0; nt < NT; nt++) sr[nt] = sx[nt] = 0.0;
    accT keepX[NT];
    T *st = stage + wave * 16 * (NC + 4);
    // an MFMA result into this wave's tile (row-major, NC + 4 floats a row)
    auto to_tile = [&](const accT(&v)[NT]) {
#pragma unroll
        for (int rr = 0; rr < 4; rr++)
#pragma unroll
            for (int nt = 0; nt < NT; nt++) st[Mfma<T>::row(lane, rr) * (NC + 4) + 16 * nt + lr] = v[nt][rr];
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    };
    // the compact rows from the tile: value 64 i + lane of the group's block
    // (rows past N fall outside the buffer's range and are dropped); the tile
    // is private to this wave and LDS operations of one wave complete in order
    auto compact_store = [&](mvl_v4i r, const int(&tl)[SW > 0 ? SW : 1]) {
#pragma unroll
        for (int i = 0; i < SW; i++) {
            const T v = st[tl[i] >= 0 ? tl[i] : 0];
            mvl_st1(r, tl[i] >= 0 ? (unsigned)((64 * i + lane) * 4) : MVL_OOB, v);
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    };
    if (Tn > 0) issue(0);
    if (Tn > 1) issue(1);
    for (int t = 0; t < Tn; t++) {
        // Stage t has arrived once no more than the operations issued after
        // its loads are outstanding: the loads of stage t+1 (2 NIN) and the
        // stores of stages t-2 and t-1 (MVL_ST0 on side 0, MVL_ST1 on side
        // 1); in the last stage, all of them
        if (t + 1 >= Tn) mvl_wait_vm<0>();
        else if (t == 0) mvl_wait_vm<2 * NIN>();
        else if (t == 1) mvl_wait_vm<2 * NIN + MVL_ST0>();
        else mvl_wait_vm<2 * NIN + MVL_ST0 + MVL_ST1>();
        const T *slots = myring + (t & 1) * NIN * MVL_SLOT;
        T av[NIN][KQ];
#pragma unroll
        for (int b = 0; b < NIN; b++) frag(av[b], slots + b * MVL_SLOT, b);
        mvl_wait_lds();   // the reads of slot t&1 are done before it is refilled
        if (t + 2 < Tn) issue(t + 2);
        const int s = t & 1;
        const i64 p0 = (g0 + (i64)(t >> 1) * gstride) * 16;
        const int nrows = (int)min((i64)16, a.N - p0);
        accT acc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; nt++) acc[nt] = acc_zero<T>();
#pragma unroll
        for (int b = 1; b < NIN; b++) mma_in(acc, av[b], b);
        // P (side 0) or AP (side 1) in the active columns
        {
            const mvl_v4i r = mvl_rsrc(a.out[s] + p0 * a.nout, (unsigned)(nrows * a.nout * 4));
            if constexpr (SW > 0) {
                to_tile(acc);
                compact_store(r, ptile);
            } else {
#pragma unroll
                for (int rr = 0; rr < 4; rr++)
#pragma unroll
                    for (int nt = 0; nt < NT; nt++) {
                        const int q = opos[16 * nt + lr];
                        const int row = Mfma<T>::row(lane, rr);
                        mvl_st1(r, q >= 0 ? (unsigned)((row * a.nout + q) * 4) : MVL_OOB, acc[nt][rr]);
                    }
            }
        }
        mma_in(acc, av[0], 0);
        // side 1: the residual W = AX' - X' Theta in the active columns and
        // the column sums of squares of step 8
        if (s == 1) {
            const mvl_v4i r = mvl_rsrc(a.Wout + p0 * a.nW, (unsigned)(nrows * a.nW * 4));
            accT wv[NT];
#pragma unroll
            for (int rr = 0; rr < 4; rr++)
#pragma unroll
                for (int nt = 0; nt < NT; nt++) {
                    const int c = 16 * nt + lr, row = Mfma<T>::row(lane, rr);
                    const double x = (double)keepX[nt][rr];
                    const double rv = (double)acc[nt][rr] - theta[c] * x;
                    if (row < nrows && c < a.kout) {
                        sr[nt] += rv * rv;
                        sx[nt] += x * x;
                    }
                    if constexpr (SW > 0) {
                        wv[nt][rr] = (T)rv;
                    } else {
                        const int w = wpos[c];
                        mvl_st1(r, w >= 0 ? (unsigned)((row * a.nW + w) * 4) : MVL_OOB, (T)rv);
                    }
                }
            if constexpr (SW > 0) {
                to_tile(wv);
                compact_store(r, wtile);
            }
        } else {
#pragma unroll
            for (int nt = 0; nt < NT; nt++) keepX[nt] = acc[nt];
        }
        // X' or AX' through this wave's LDS tile: after the transpose each
        // lane holds four consecutive columns of one row and stores 16 bytes
        {
#pragma unroll
            for (int rr = 0; rr < 4; rr++)
#pragma unroll
                for (int nt = 0; nt < NT; nt++) st[Mfma<T>::row(lane, rr) * (NC + 4) + 16 * nt + lr] = acc[nt][rr];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            const mvl_v4i r = mvl_rsrc(a.out2[s] + p0 * a.ld2, (unsigned)(nrows * a.ld2 * 4));
            const int row = lane >> 2;
#pragma unroll
            for (int h = 0; h < NT; h++) {
                const int c0 = 4 * ((lane & 3) + 4 * h);
                const floatx4 v = *reinterpret_cast<const floatx4 *>(st + row * (NC + 4) + c0);
                mvl_st4(r, c0 < a.kout ? (unsigned)((row * a.ld2 + c0) * 4) : MVL_OOB, v);
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        }
    }
    mvl_wait_vm<0>();
    // per-workgroup column sums, reduced over the 16 lane groups in LDS (the
    // ring is free now)
    __syncthreads();
    double *red = reinterpret_cast<double *>(ring);
    {
        const int slot = wave * 4 + kq;
#pragma unroll
        for (int nt = 0; nt < NT; nt++) {
            red[(slot * 2 + 0) * NC + 16 * nt + lr] = sr[nt];
            red[(slot * 2 + 1) * NC + 16 * nt + lr] = sx[nt];
        }
    }
    __syncthreads();
    for (int e = tid; e < 2 * a.kout; e += blockDim.x) {
        const int which = e / a.kout, c = e % a.kout;
        double sum = 0.0;
        for (int sl = 0; sl < 16; sl++) sum += red[(sl * 2 + which) * NC + c];
        a.partials[(i64)blockIdx.x * 2 * a.kout + e] = sum;
    }
}

// dynamic LDS of mvl_kernel: coefficients, theta, opos, wpos, the output
// tiles and the input rings
static size_t mvl_lds_bytes(int nin, int nsteps)
{
    return (size_t)nsteps * 2 * 64 * 4 + 32 * 8 + 2 * 32 * 4 + MVL_CMAP * 4 + 4 * 16 * 36 * 4 +
           (size_t)4 * 2 * nin * MVL_SLOT * 4;
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
static MVDev<T> make_dev(const MVArgs &h)
{
    MVDev<T> a;
    a.K = 0;
    for (int b = 0; b < MV_MAX_IN; b++) {
        const bool used = b < h.nin;
        for (int s = 0; s < 2; s++) a.in[s][b] = used ? (const T *)h.in[s][b] : nullptr;
        a.ld[b] = used ? h.ld[b] : 1;
        a.k[b] = used ? h.k[b] : 0;
        a.cols[b] = used ? h.cols[b] : nullptr;
        a.coff[b] = used ? h.coff[b] : 0;
        a.K += a.k[b];
    }
    a.nin = h.nin;
    a.n0 = h.n0;
    a.ld2 = h.ld2 > 0 ? h.ld2 : h.kout;
    a.nside = h.nside;
    a.kout = h.kout;
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
    MVDev<T> a = make_dev<T>(h);
    const int nb = mv_blocks(h.N);
    int nsteps = 0;
    for (int b = 0; b < h.nin; b++) nsteps += (h.k[b] + 3) / 4;
    const size_t shm = mvf_stage_offset(nsteps, NT, a.K, sizeof(T));
    hipLaunchKernelGGL((mvw_kernel<T, NT>), dim3(nb), dim3(256), shm, st, a);
    return mv_reduce(h, nb, st);
}

// the fused FP32 update that mvl_kernel takes
static bool mvl_fits(const MVArgs &h)
{
    if (h.nside != 2 || h.nin < 2 || h.nin > 3 || h.n0 != 1 || h.add || !h.partials || !h.theta || !h.opos ||
        !h.wpos || !h.Wout)
        return false;
    for (int s = 0; s < 2; s++)
        if (!h.out[s] || !h.out2[s]) return false;
    if (h.kout > MAXW || h.kout % 4 || (h.ld2 > 0 && h.ld2 != h.kout) || (h.sums_ld > 0 && h.sums_ld != h.kout))
        return false;
    bool narrow = h.kout <= NARROW;
    for (int b = 0; b < h.nin; b++) {
        if (h.coff[b] || h.ld[b] > MAXW || h.k[b] > h.ld[b]) return false;
        narrow = narrow && h.ld[b] <= NARROW;
    }
    return !narrow;
}

static hipError_t run_mvl(const MVArgs &h, hipStream_t st)
{
    MVDev<float> a = make_dev<float>(h);
    const int nb = mv_blocks(h.N);
    int nsteps = 0;
    for (int b = 0; b < h.nin; b++) nsteps += mvf_k4(h.k[b], h.ld[b], h.cols[b] != nullptr, 4);
    const size_t shm = mvl_lds_bytes(h.nin, nsteps);
    // P / AP and W with at most 16 stored columns: compact stores (SW of them)
    const int nst = h.nout > h.nW ? h.nout : h.nW;
    const int sw = h.mvl_fragment_stores ? 0 : nst <= 4 ? 1 : nst <= 8 ? 2 : nst <= 16 ? 4 : 0;
#define MVL_LAUNCH(NIN, SW) hipLaunchKernelGGL((mvl_kernel<NIN, SW>), dim3(nb), dim3(256), shm, st, a)
    if (h.nin == 3) {
        if (sw == 1) MVL_LAUNCH(3, 1);
        else if (sw == 2) MVL_LAUNCH(3, 2);
        else if (sw == 4) MVL_LAUNCH(3, 4);
        else MVL_LAUNCH(3, 0);
    } else {
        if (sw == 1) MVL_LAUNCH(2, 1);
        else if (sw == 2) MVL_LAUNCH(2, 2);
        else if (sw == 4) MVL_LAUNCH(2, 4);
        else MVL_LAUNCH(2, 0);
    }
#undef MVL_LAUNCH
    return mv_reduce(h, nb, st);
}

template <typename T, int NT>
static hipError_t run_mv(const MVArgs &h, hipStream_t st)
{
    MVDev<T> a = make_dev<T>(h);
    const int nb = mv_blocks(h.N);
    bool narrow = h.kout <= NARROW;
    for (int b = 0; b < h.nin; b++) narrow = narrow && h.ld[b] <= NARROW;
    if (narrow) {
        const size_t shm = (size_t)NARROW * 8 + (size_t)2 * NARROW * 256 * 8 + (size_t)a.K * NARROW * sizeof(T) +
                           (size_t)(a.K + 2 * NARROW) * sizeof(int);
        hipLaunchKernelGGL((mvn_kernel<T>), dim3(nb), dim3(256), shm, st, a);
    } else {
        int nsteps = 0;
        for (int b = 0; b < h.nin; b++) nsteps += mvf_k4(h.k[b], h.ld[b], h.cols[b] != nullptr, sizeof(T));
        const size_t shm = mvf_stage_offset(nsteps, NT, a.K, sizeof(T)) + mvf_stage_bytes(NT, sizeof(T));
        hipLaunchKernelGGL((mvf_kernel<T, NT>), dim3(nb), dim3(256), shm, st, a);
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
    if (dtype == DT_F32 && !a.frag_only && mvl_fits(a)) return run_mvl(a, st);
    if (dtype == DT_F32) return two ? run_mv<float, 2>(a, st) : run_mv<float, 1>(a, st);
    return two ? run_mv<double, 2>(a, st) : run_mv<double, 1>(a, st);
}

}  // namespace lobpcg
