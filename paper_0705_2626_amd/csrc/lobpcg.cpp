// liblobpcg.so: block LOBPCG (Section 2.2, steps 1-37, B = I, no constraints)
// with soft locking (Section 2.3) on one MI355X.  The host drives the
// iteration; every N-sized operation runs in the library's HIP kernels and
// only the small (<= 3m x 3m) FP64 matrices come back to the host for the
// Cholesky factorisations and the Rayleigh-Ritz eigenproblem, as in the
// paper's implementation (which calls LAPACK for them, Section 3).
#include "../../include/lobpcg.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "dense.h"
#include "kernels.h"

using namespace lobpcg;

namespace {

const size_t ALIGN = 256;
// The Gram kernel keeps 3m-column row chunks and the combine kernel its
// (3m x m) coefficients in LDS; this bounds m.
const int LOBPCG_MAX_M = 128;
const int COEF_SLOTS = 16;
// Entries of one coefficient ring slot: the (3m x m) update coefficients of
// steps 25-33, or the ((k + ny) x k) ones of a constraint projection (k <= m,
// ny <= LOBPCG_MAX_M).
size_t coef_slot_entries(int m) { return (size_t)std::max(3 * m, m + LOBPCG_MAX_M) * m; }

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }
size_t esize(int dt) { return dt == DT_F32 ? 4 : 8; }

// The eleven N x m blocks of one precision (steps 1-33 store 6m vectors for
// B = I; the extra ones are ping-pong and packed-active copies).
struct Blocks {
    void *X[2], *AX[2];   // current / next Ritz vectors and A X
    void *W, *AW;         // preconditioned residuals (packed |J| columns) and A W
    void *P, *AP;         // directions of all m columns, as produced by steps 27/31
    void *PJ, *APJ;       // orthonormalised active directions (packed)
    void *T0;             // multigrid fine-level scratch
    void *BX[2], *BW, *BP, *BPJ;   // B X, B W, B P and a spare, when B is not the identity
};

struct Layout {
    size_t blocks64, blocks32;          // offsets (or SIZE_MAX if absent)
    size_t blocksB;                     // the five FP64 B-blocks (or SIZE_MAX)
    size_t blocksB32;                   // the five FP32 B-blocks of the mixed solver (or SIZE_MAX)
    std::vector<size_t> mg;             // per level l >= 1: x, b, t (3 entries each)
    size_t lambda, jpos, cols, coef, gram_out, gram_part, res_part, mv_part, res_out, wvec;
    size_t total;
    int mg_dtype;
    std::vector<Grid3> levels;
};

bool op_ok(const lobpcg_op *A)
{
    if (!A) return false;
    if (A->nx < 1 || A->ny < 1 || A->nz < 1) return false;
    if (A->kind == LOBPCG_OP_LAPLACE7) return true;
    if (A->kind == LOBPCG_OP_VARCOEF7) return A->kx && A->ky && A->kz;
    return false;
}

// B of A's grid: a positive diagonal, or the 7-point mass-type operator
// b0 I + b1 (neighbour sum) with b0 > 6 |b1| (strictly diagonally dominant)
bool b_ok(const lobpcg_op *A, const lobpcg_op *B)
{
    if (B->nx != A->nx || B->ny != A->ny || B->nz != A->nz) return false;
    if (B->kind == LOBPCG_OP_DIAG) return B->diag != nullptr;
    if (B->kind == LOBPCG_OP_MASS7)
        return std::isfinite(B->b0) && std::isfinite(B->b1) && B->b0 > 6.0 * std::fabs(B->b1);
    return false;
}

int check_common(const lobpcg_op *A, const lobpcg_op *B, const lobpcg_precond *T, int m, int precision)
{
    if (!op_ok(A)) return LOBPCG_ERR_ARG;
    if (precision != LOBPCG_FP64 && precision != LOBPCG_MIXED) return LOBPCG_ERR_ARG;
    if (B && !b_ok(A, B)) return LOBPCG_ERR_ARG;
    const long long N = (long long)A->nx * A->ny * A->nz;
    if (m < 1 || m > LOBPCG_MAX_M || 3LL * m > N) return LOBPCG_ERR_ARG;
    if (T) {
        if (T->kind == LOBPCG_PC_GMG_V) {
            if (T->levels < 1 || T->levels > 30 || T->nu_pre < 0 || T->nu_post != T->nu_pre ||
                T->coarse_sweeps < 1 || !(T->omega > 0.0 && T->omega < 2.0))
                return LOBPCG_ERR_ARG;
            int nx = A->nx, ny = A->ny, nz = A->nz;
            for (int l = 1; l < T->levels; l++) {
                nx /= 2, ny /= 2, nz /= 2;
                if (nx < 1 || ny < 1 || nz < 1) return LOBPCG_ERR_ARG;
            }
        } else if (T->kind != LOBPCG_PC_NONE) {
            return LOBPCG_ERR_ARG;
        }
    }
    return LOBPCG_OK;
}

bool has_mg(const lobpcg_precond *T) { return T && T->kind == LOBPCG_PC_GMG_V; }

Layout make_layout(const lobpcg_op *A, const lobpcg_op *B, const lobpcg_precond *T, int m, int precision)
{
    Layout L;
    const long long N = (long long)A->nx * A->ny * A->nz;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = align_up(off);
        off = o + bytes;
        return o;
    };
    L.blocks64 = take(11 * (size_t)N * m * 8);
    L.blocks32 = precision == LOBPCG_MIXED ? take(11 * (size_t)N * m * 4) : (size_t)-1;
    L.blocksB = B ? take(5 * (size_t)N * m * 8) : (size_t)-1;
    L.blocksB32 = (B && precision == LOBPCG_MIXED) ? take(5 * (size_t)N * m * 4) : (size_t)-1;
    L.mg_dtype = precision == LOBPCG_MIXED ? DT_F32 : DT_F64;
    L.levels.push_back(Grid3{A->nx, A->ny, A->nz});
    if (has_mg(T)) {
        for (int l = 1; l < T->levels; l++) {
            Grid3 g = L.levels.back();
            L.levels.push_back(Grid3{g.nx / 2, g.ny / 2, g.nz / 2});
            for (int j = 0; j < 3; j++) L.mg.push_back(take((size_t)L.levels.back().n() * m * esize(L.mg_dtype)));
        }
    }
    L.lambda = take(sizeof(double) * m);
    L.jpos = take(sizeof(int) * m);
    L.cols = take(sizeof(int) * COEF_SLOTS * m);
    L.coef = take((size_t)COEF_SLOTS * coef_slot_entries(m) * 8);
    L.gram_out = take((size_t)GX_MAX_TILES * 256 * 8);
    L.gram_part = take(gram_partials_bytes(N));
    L.res_part = take((size_t)residual_blocks(N, m) * 2 * m * 8);
    L.mv_part = take((size_t)mv_blocks(N) * 2 * m * 8);
    L.res_out = take((size_t)2 * m * 8);
    L.wvec = take(sizeof(double) * m);
    L.total = align_up(off);
    return L;
}

double laplace7_norm(const Grid3 &g)
{
    // infinity norm: diagonal 6 plus one per axis neighbour that exists
    return 6.0 + std::min(2, g.nx - 1) + std::min(2, g.ny - 1) + std::min(2, g.nz - 1);
}

}  // namespace

struct lobpcg_ctx {
    Grid3 g;
    long long N;
    int m, precision;
    lobpcg_op A;
    lobpcg_precond T;
    bool mg;
    hipStream_t st;
    char *ws;
    Layout L;
    Blocks b64, b32;
    std::vector<void *> mgx, mgb, mgt;
    // small device areas
    double *d_lambda, *d_gram_out, *d_gram_part, *d_res_part, *d_mv_part, *d_res_out, *d_w;
    int *d_jpos, *d_cols;
    char *d_coef;
    // pinned host staging
    char *h_pin;
    size_t h_coef_off, h_cols_off, h_gram_off, h_res_off, h_small_off, h_pin_bytes;
    int coef_slot;
    // options
    double switch_tol;
    int stall_window;
    double stall_factor;
    bool profile, reactivate;
    double lock_gap;              // soft locking keeps a converged column active while an unconverged
                                  // one has a Ritz value within this relative distance (0: off)
    int nwant;                    // the run ends once the first nwant columns have converged (0: m)
    int mv_frag, mg_unpadded, gram_staged, gram_nt4, gram_nt32, gram_direct, mv_fragst;  // kernel variants (see LOBPCG_OPT_KERNELS)
    bool fp32_explicit;           // FP32 phase: Gram diagonal blocks computed, not assumed ...
    int fp32_explicit_above;      // ... while more columns than this are active (-1: m / 4)
    bool fp64_explicit;           // the same for FP64 iterations
    bool fold;                    // Cholesky-QR factors of W_J, P_J folded into Gram and coefficients
    bool hasB;                    // A x = lambda B x (B: Bop, a positive diagonal or the mass-type stencil)
    lobpcg_op Bop;
    const double *Y;              // constraints of the current solve (FP64, N x ny) or null
    int ny;
    std::vector<double> RY;       // Y^T Y = RY^T RY (upper, ny x ny)
    lobpcg_stats stats;
    // profiling: pending (step, start, end) event pairs
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> ev_step;
    int ev_used;
};

namespace {

#define HIPCHK(x)                                        \
    do {                                                 \
        if ((x) != hipSuccess) return LOBPCG_ERR_HIP;    \
    } while (0)

Blocks carve_blocks(char *base, long long N, int m, int dt)
{
    Blocks b;
    const size_t bs = (size_t)N * m * esize(dt);
    void **slots[11] = {&b.X[0], &b.X[1], &b.AX[0], &b.AX[1], &b.W, &b.AW, &b.P, &b.AP, &b.PJ, &b.APJ, &b.T0};
    for (int i = 0; i < 11; i++) *slots[i] = base + i * bs;
    b.BX[0] = b.BX[1] = b.BW = b.BP = b.BPJ = nullptr;
    return b;
}

// ---- profiling
void prof_begin(lobpcg_ctx *c, int step)
{
    if (!c->profile) return;
    if (c->ev_used + 2 > (int)c->ev_pool.size()) return;
    (void)hipEventRecord(c->ev_pool[c->ev_used], c->st);
    c->ev_step[c->ev_used / 2] = step;
    c->ev_used += 1;
}
void prof_end(lobpcg_ctx *c)
{
    if (!c->profile) return;
    if (c->ev_used % 2 == 0) return;
    (void)hipEventRecord(c->ev_pool[c->ev_used], c->st);
    c->ev_used += 1;
}
// algorithmic HBM bytes of a step's kernels (operands read once, results written once)
void add_bytes(lobpcg_ctx *c, int step, double bytes) { c->stats.step_bytes[step] += bytes; }

// called right after a stream synchronisation
void prof_collect(lobpcg_ctx *c)
{
    if (!c->profile) return;
    for (int i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev_pool[i], c->ev_pool[i + 1]) == hipSuccess) {
            c->stats.step_ms[c->ev_step[i / 2]] += ms;
            c->stats.step_calls[c->ev_step[i / 2]] += 1;
        }
    }
    c->ev_used = 0;
}

int sync(lobpcg_ctx *c)
{
    HIPCHK(hipStreamSynchronize(c->st));
    prof_collect(c);
    c->coef_slot = 0;
    return LOBPCG_OK;
}

// Upload small host data through a pinned ring slot; valid until the next sync.
int upload_coef(lobpcg_ctx *c, int dt, const double *C, int rows, int cols, const void **dptr)
{
    if (c->coef_slot >= COEF_SLOTS) {
        int s = sync(c);
        if (s) return s;
    }
    const size_t n = (size_t)rows * cols;
    if (rows < 0 || cols < 0 || n > coef_slot_entries(c->m)) return LOBPCG_ERR_ARG;
    const size_t slot_bytes = coef_slot_entries(c->m) * 8;
    char *h = c->h_pin + c->h_coef_off + c->coef_slot * slot_bytes;
    char *d = c->d_coef + c->coef_slot * slot_bytes;
    if (dt == DT_F32) {
        float *hf = (float *)h;
        for (size_t i = 0; i < n; i++) hf[i] = (float)C[i];
    } else {
        memcpy(h, C, n * 8);
    }
    HIPCHK(hipMemcpyAsync(d, h, n * esize(dt), hipMemcpyHostToDevice, c->st));
    *dptr = d;
    c->coef_slot++;
    return LOBPCG_OK;
}

int upload_cols(lobpcg_ctx *c, const std::vector<int> &cols, const int **dptr)
{
    // same ring index as the coefficients, separate area
    if (cols.size() > (size_t)c->m) return LOBPCG_ERR_ARG;
    if (c->coef_slot >= COEF_SLOTS) {
        int s = sync(c);
        if (s) return s;
    }
    int *h = (int *)(c->h_pin + c->h_cols_off) + c->coef_slot * c->m;
    int *d = c->d_cols + c->coef_slot * c->m;
    std::copy(cols.begin(), cols.end(), h);
    HIPCHK(hipMemcpyAsync(d, h, cols.size() * sizeof(int), hipMemcpyHostToDevice, c->st));
    *dptr = d;
    c->coef_slot++;
    return LOBPCG_OK;
}

// ---- kernel-level building blocks (asynchronous unless they return host data)

// B applied to an N x k block of precision dt (B = diag(d), or the 7-point
// mass-type operator)
int apply_B(lobpcg_ctx *c, int dt, const void *in, void *out, int k, int step)
{
    prof_begin(c, step);
    hipError_t e;
    if (c->Bop.kind == LOBPCG_OP_MASS7) {
        e = launch_mass7(dt, c->g, k, c->Bop.b0, c->Bop.b1, in, out, c->st);
        add_bytes(c, step, 2.0 * k * c->N * esize(dt));
    } else {
        e = launch_diag_scale(dt, c->N, k, c->Bop.diag, in, out, c->st);
        add_bytes(c, step, 2.0 * k * c->N * esize(dt) + 8.0 * c->N);
    }
    prof_end(c);
    return e == hipSuccess ? LOBPCG_OK : LOBPCG_ERR_HIP;
}

int apply_A(lobpcg_ctx *c, const lobpcg_op *A, int dt, const void *in, void *out, int k)
{
    prof_begin(c, LOBPCG_STEP_APPLY_A);
    hipError_t e;
    if (A->kind == LOBPCG_OP_VARCOEF7)
        e = launch_varcoef7(dt, c->g, k, A->kx, A->ky, A->kz, in, out, c->st);
    else
        e = launch_laplace7(dt, c->g, k, in, out, 1.0, c->st);
    prof_end(c);
    add_bytes(c, LOBPCG_STEP_APPLY_A, 2.0 * c->N * k * esize(dt) +
                                          (A->kind == LOBPCG_OP_VARCOEF7 ? 8.0 * (3.0 * c->N + c->g.nx * c->g.ny +
                                                                                  c->g.ny * c->g.nz + c->g.nz * c->g.nx)
                                                                         : 0.0));
    return e == hipSuccess ? LOBPCG_OK : LOBPCG_ERR_HIP;
}

// Gram products of S = [S_0 .. S_{n-1}] (widths w, K columns in all) and,
// when AS is given, AS = [AS_0 .. AS_{n-1}]; returns K x K host matrices
// (row-major, symmetric).  They are entries of Lm^T Rm with Lm = S and
//  - no AS: Rm = S (S^T S, the Cholesky Gram matrices of steps 3, 11, 14);
//  - AS, explicit form: Rm = [S_0 AS_0 S_1.. AS_1..], all of S^T S and S^T AS;
//  - AS, the paper's form (steps 17-23): Rm = [S_1.. AS_1..] (W, P, AW, AP)
//    and only the entries the paper does not take as known: gramB off the
//    block diagonal, gramA outside the X-X block (the caller fills Lambda
//    and the identities; other entries are zero).
// Entries (i, j) with i <= j are computed and mirrored.
int gram(lobpcg_ctx *c, int dt, int n, const void *const *S, const void *const *AS, const int *w,
         std::vector<double> &SS, std::vector<double> *SAS, int step, bool paper = false,
         const int *const *cols = nullptr, const int *ld = nullptr, bool diag_blocks = false,
         const void *const *BS = nullptr)
{
    int K = 0;
    std::vector<int> blk, col, off(n + 1, 0);
    bool plain = true;   // every block read whole
    for (int b = 0; b < n; b++) {
        const bool sel = cols && cols[b];
        for (int i = 0; i < w[b]; i++) blk.push_back(b), col.push_back(sel ? cols[b][i] : i);
        K += w[b];
        off[b + 1] = K;
        plain = plain && !sel && (!ld || ld[b] == w[b]);
    }
    double *h = (double *)(c->h_pin + c->h_gram_off);
    if (!AS && !BS && n == 1 && w[0] <= 8 && plain && !c->gram_staged) {
        // one narrow block: one grid row per thread
        prof_begin(c, step);
        hipError_t e = launch_gram_rows(dt, S[0], w[0], c->N, c->d_gram_part, c->d_gram_out, w[0], c->st);
        prof_end(c);
        if (e != hipSuccess) return LOBPCG_ERR_HIP;
        add_bytes(c, step, (double)w[0] * c->N * esize(dt));
        HIPCHK(hipMemcpyAsync(h, c->d_gram_out, (size_t)K * K * 8, hipMemcpyDeviceToHost, c->st));
        int s = sync(c);
        if (s) return s;
        SS.assign((size_t)K * K, 0.0);
        for (int i = 0; i < K; i++)
            for (int j = i; j < K; j++) SS[(size_t)i * K + j] = SS[(size_t)j * K + i] = h[(size_t)i * K + j];
        return LOBPCG_OK;
    }
    const bool pform = AS && paper && n > 1;
    GramXArgs a;
    for (int b = 0; b < GX_MAX_ARR; b++) a.arr[b] = nullptr, a.ld[b] = 1;
    for (int b = 0; b < n; b++) {
        const int l = ld ? ld[b] : w[b];
        a.arr[b] = S[b], a.ld[b] = l;
        if (AS) a.arr[3 + b] = AS[b], a.ld[3 + b] = l;
        if (BS) a.arr[6 + b] = BS[b], a.ld[6 + b] = l;
    }
    // with BS the "S^T S" products are S^T BS: Rm takes those columns from BS
    const int sb = BS ? 6 : 0;
    // Lm = S; Rm as above.  rs[j] / ra[j]: column of Rm holding S_j / AS_j (-1: none)
    std::vector<unsigned short> lmap(K), rmap;
    for (int i = 0; i < K; i++) lmap[i] = (unsigned short)((blk[i] << 8) | col[i]);
    std::vector<int> rs(K, -1), ra(K, -1);
    auto addr = [&](int arr, int i, std::vector<int> &pos) {
        pos[i] = (int)rmap.size();
        rmap.push_back((unsigned short)((arr << 8) | col[i]));
    };
    if (pform) {
        for (int i = w[0]; i < K; i++) addr(sb + blk[i], i, rs);
        for (int i = w[0]; i < K; i++) addr(3 + blk[i], i, ra);
    } else if (AS && n > 1) {
        // [S_0 AS_0 | S_1.. AS_1..]: the thin blocks share 16-column tiles
        for (int i = 0; i < w[0]; i++) addr(sb, i, rs);
        for (int i = 0; i < w[0]; i++) addr(3, i, ra);
        for (int i = w[0]; i < K; i++) addr(sb + blk[i], i, rs);
        for (int i = w[0]; i < K; i++) addr(3 + blk[i], i, ra);
    } else {
        for (int i = 0; i < K; i++) addr(sb + blk[i], i, rs);
        if (AS)
            for (int i = 0; i < K; i++) addr(3 + blk[i], i, ra);
    }
    const int KR = (int)rmap.size();
    // the entries wanted, as (row of Lm, column of Rm) pairs, and their tiles
    struct Want { int i, j, mat, r; };
    std::vector<Want> want;
    for (int i = 0; i < K; i++)
        for (int j = i; j < K; j++) {
            if (!pform || blk[i] < blk[j] || (diag_blocks && blk[i] == blk[j] && blk[i] > 0))
                want.push_back({i, j, 0, rs[j]});
            if (AS && (!pform || !(blk[i] == 0 && blk[j] == 0))) want.push_back({i, j, 1, ra[j]});
        }
    std::vector<int> tiles;   // (ta << 8) | tb, sorted
    for (const Want &q : want) tiles.push_back(((q.i / 16) << 8) | (q.r / 16));
    std::sort(tiles.begin(), tiles.end());
    tiles.erase(std::unique(tiles.begin(), tiles.end()), tiles.end());
    if (tiles.empty()) return LOBPCG_ERR_ARG;
    // Launches: the tiles in order, as many per launch as its argument
    // tables hold (one launch whenever the whole product fits)
    struct Launch { std::vector<int> la, lb; int t0, t1; };
    std::vector<Launch> launches;
    {
        Launch cur{{}, {}, 0, 0};
        for (int t = 0; t < (int)tiles.size(); t++) {
            const int ta = tiles[t] >> 8, tb = tiles[t] & 255;
            const bool newa = std::find(cur.la.begin(), cur.la.end(), ta) == cur.la.end();
            const bool newb = std::find(cur.lb.begin(), cur.lb.end(), tb) == cur.lb.end();
            if (cur.t1 > cur.t0 && (cur.t1 - cur.t0 >= GX_MAX_TILES || (newa && (int)cur.la.size() >= GX_MAX_L / 16) ||
                                    (newb && (int)cur.lb.size() >= GX_MAX_R / 16))) {
                launches.push_back(cur);
                cur = Launch{{}, {}, t, t};
            }
            if (std::find(cur.la.begin(), cur.la.end(), ta) == cur.la.end()) cur.la.push_back(ta);
            if (std::find(cur.lb.begin(), cur.lb.end(), tb) == cur.lb.end()) cur.lb.push_back(tb);
            cur.t1 = t + 1;
        }
        launches.push_back(cur);
    }
    const int KLp = (K + 15) / 16 * 16, KRp = (KR + 15) / 16 * 16;
    std::vector<double> M((size_t)KLp * KRp, 0.0);
    a.N = c->N;
    a.partials = c->d_gram_part;
    a.out = c->d_gram_out;
    a.max_nt = c->gram_nt4 ? GX_MAXB : 2;
    a.max_nt32 = c->gram_nt4 ? GX_MAXB : c->gram_nt32;
    a.direct = c->gram_direct;
    const bool single = launches.size() == 1 && K <= GX_MAX_L && KR <= GX_MAX_R;
    for (const Launch &L : launches) {
        // the launch's Lm / Rm: its 16-column blocks, in order; a partial last
        // block is padded with copies of its first column (results unused)
        std::vector<int> gta, gtb;   // global block of each local tile
        if (single) {
            a.KL = K;
            a.KR = KR;
            std::copy(lmap.begin(), lmap.end(), a.lmap);
            std::copy(rmap.begin(), rmap.end(), a.rmap);
        } else {
            a.KL = 16 * (int)L.la.size();
            a.KR = 16 * (int)L.lb.size();
            for (int u = 0; u < (int)L.la.size(); u++)
                for (int v = 0; v < 16; v++) {
                    const int i = 16 * L.la[u] + v;
                    a.lmap[16 * u + v] = lmap[i < K ? i : 16 * L.la[u]];
                }
            for (int u = 0; u < (int)L.lb.size(); u++)
                for (int v = 0; v < 16; v++) {
                    const int j = 16 * L.lb[u] + v;
                    a.rmap[16 * u + v] = rmap[j < KR ? j : 16 * L.lb[u]];
                }
        }
        a.ntiles = L.t1 - L.t0;
        for (int t = 0; t < a.ntiles; t++) {
            const int ta = tiles[L.t0 + t] >> 8, tb = tiles[L.t0 + t] & 255;
            gta.push_back(ta);
            gtb.push_back(tb);
            a.ta[t] = single ? ta : (int)(std::find(L.la.begin(), L.la.end(), ta) - L.la.begin());
            a.tb[t] = single ? tb : (int)(std::find(L.lb.begin(), L.lb.end(), tb) - L.lb.begin());
        }
        prof_begin(c, step);
        if (launch_gramx(dt, a, c->st) != hipSuccess) return LOBPCG_ERR_HIP;
        prof_end(c);
        if (single) {
            // the columns of each array that some tile reads, once
            std::vector<char> used(GX_MAX_ARR, 0);
            for (int t = 0; t < a.ntiles; t++) {
                for (int i = 16 * a.ta[t]; i < std::min(K, 16 * a.ta[t] + 16); i++) used[a.lmap[i] >> 8] = 1;
                for (int j = 16 * a.tb[t]; j < std::min(KR, 16 * a.tb[t] + 16); j++) used[a.rmap[j] >> 8] = 1;
            }
            double ncols = 0.0;
            for (int b = 0; b < GX_MAX_ARR; b++)
                if (used[b]) ncols += w[b % 3];
            add_bytes(c, step, ncols * c->N * esize(dt));
        } else {
            // the distinct columns this launch reads
            std::vector<unsigned short> cl(a.lmap, a.lmap + a.KL);
            cl.insert(cl.end(), a.rmap, a.rmap + a.KR);
            std::sort(cl.begin(), cl.end());
            cl.erase(std::unique(cl.begin(), cl.end()), cl.end());
            add_bytes(c, step, (double)cl.size() * c->N * esize(dt));
        }
        HIPCHK(hipMemcpyAsync(h, c->d_gram_out, (size_t)a.ntiles * 256 * 8, hipMemcpyDeviceToHost, c->st));
        int s = sync(c);
        if (s) return s;
        // tiles -> dense Lm^T Rm (entry e = r*64 + lane of the MFMA accumulator)
        for (int t = 0; t < a.ntiles; t++)
            for (int e = 0; e < 256; e++) {
                const int r = e / 64, lane = e % 64;
                const int row = dt == DT_F32 ? 4 * (lane / 16) + r : lane / 16 + 4 * r;
                M[(size_t)(16 * gta[t] + row) * KRp + 16 * gtb[t] + lane % 16] = h[(size_t)t * 256 + e];
            }
    }
    SS.assign((size_t)K * K, 0.0);
    if (SAS) SAS->assign((size_t)K * K, 0.0);
    for (const Want &q : want) {
        std::vector<double> &D = q.mat ? *SAS : SS;
        if (q.mat && !SAS) continue;
        D[(size_t)q.i * K + q.j] = D[(size_t)q.j * K + q.i] = M[(size_t)q.i * KRp + q.r];
    }
    return LOBPCG_OK;
}

// One multivector-product launch (see MVArgs); C is the host FP64
// coefficient matrix ((sum k_i) x kout, row-major), uploaded in the blocks'
// precision.
struct MV {
    int nside = 1, nin = 0, kout = 0;
    const void *in[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    int ld[3] = {0, 0, 0}, k[3] = {0, 0, 0};
    const int *cols[3] = {nullptr, nullptr, nullptr};
    const void *add = nullptr;
    void *out[2] = {nullptr, nullptr}, *out2[2] = {nullptr, nullptr};
    const int *opos = nullptr;
    int nout = 0;
    const double *theta = nullptr;
    const int *wpos = nullptr;
    void *Wout = nullptr;
    int nW = 0;
    bool resid = false;
    void input(int i, const void *x, const void *ax, int ldi, int ki, const int *cl = nullptr)
    {
        in[0][i] = x;
        in[1][i] = ax;
        ld[i] = ldi;
        k[i] = ki;
        cols[i] = cl;
        if (i + 1 > nin) nin = i + 1;
    }
};

int mv(lobpcg_ctx *c, int dt, const MV &q, const double *C, int step)
{
    int K = 0;
    bool wide = q.kout > MV_PIECE;
    for (int i = 0; i < q.nin; i++) {
        K += q.k[i];
        wide = wide || q.ld[i] > MV_PIECE || q.k[i] > MV_PIECE;
    }
    auto account = [&](int kout) {
        const int nout = q.opos ? std::min(q.nout, kout) : kout;
        double cols = (double)K * q.nside + (q.add ? kout : 0);
        cols += (double)q.nside * ((q.out[0] ? nout : 0) + (q.out2[0] ? kout : 0));
        if (q.resid && q.Wout) cols += std::min(q.nW, kout);
        add_bytes(c, step, cols * c->N * esize(dt));
    };
    MVArgs a;
    a.frag_only = c->mv_frag;
    a.mvl_fragment_stores = c->mv_fragst;
    a.nside = q.nside;
    a.N = c->N;
    a.partials = q.resid ? c->d_mv_part : nullptr;
    a.sums = q.resid ? c->d_res_out : nullptr;
    a.theta = q.theta;
    a.wpos = q.wpos;
    a.Wout = q.Wout;
    a.nW = q.nW;
    if (!wide) {
        for (int s2 = 0; s2 < 2; s2++)
            for (int i = 0; i < 3; i++) a.in[s2][i] = q.in[s2][i];
        for (int i = 0; i < 3; i++) {
            a.ld[i] = q.ld[i];
            a.k[i] = i < q.nin ? q.k[i] : 0;
            a.cols[i] = q.cols[i];
        }
        a.nin = q.nin;
        a.kout = q.kout;
        a.add = q.add;
        for (int s2 = 0; s2 < 2; s2++) {
            a.out[s2] = q.out[s2];
            a.out2[s2] = q.out2[s2];
        }
        a.opos = q.opos;
        a.nout = q.nout;
        int s = upload_coef(c, dt, C, K, q.kout, &a.C);
        if (s) return s;
        prof_begin(c, step);
        hipError_t e = launch_mv(dt, a, c->st);
        prof_end(c);
        account(q.kout);
        return e == hipSuccess ? LOBPCG_OK : LOBPCG_ERR_HIP;
    }
    // Wide blocks: each input split into pieces of at most MV_PIECE columns
    // (a column range, or a range of its column list), the outputs computed
    // MV_PIECE (or 16) columns per launch.  The pieces keep the row order of C.
    int np = 0, n0 = 0;
    for (int i = 0; i < q.nin; i++)
        for (int off = 0; off < q.k[i]; off += MV_PIECE) {
            if (np >= MV_MAX_IN) return LOBPCG_ERR_ARG;
            for (int s2 = 0; s2 < 2; s2++) a.in[s2][np] = q.in[s2][i];
            a.ld[np] = q.ld[i];
            a.k[np] = std::min(MV_PIECE, q.k[i] - off);
            a.cols[np] = q.cols[i] ? q.cols[i] + off : nullptr;
            a.coff[np] = q.cols[i] ? 0 : off;
            if (i == 0) n0++;
            np++;
        }
    a.nin = np;
    a.n0 = n0;
    const int chunk = mv_wide_chunk(dt, np, a.k);
    if (!chunk) return LOBPCG_ERR_ARG;
    // the output columns of out[] through a position list (identity if none)
    const int *opos = q.opos;
    int nout = q.nout;
    if (!opos && (q.out[0] || q.out[1])) {
        std::vector<int> id(q.kout);
        for (int j = 0; j < q.kout; j++) id[j] = j;
        int s2 = upload_cols(c, id, &opos);
        if (s2) return s2;
        nout = q.kout;
    }
    const size_t es = esize(dt);
    // the column chunks of C one after another (K x kc each), in one upload
    std::vector<double> Cs((size_t)K * q.kout);
    for (int c0 = 0; c0 < q.kout; c0 += chunk) {
        const int kc = std::min(chunk, q.kout - c0);
        for (int r = 0; r < K; r++)
            for (int j = 0; j < kc; j++) Cs[(size_t)K * c0 + (size_t)r * kc + j] = C[(size_t)r * q.kout + c0 + j];
    }
    const void *dC;
    int s = upload_coef(c, dt, Cs.data(), K, q.kout, &dC);
    if (s) return s;
    for (int c0 = 0; c0 < q.kout; c0 += chunk) {
        const int kc = std::min(chunk, q.kout - c0);
        a.C = (const char *)dC + (size_t)K * c0 * es;
        a.kout = kc;
        a.ld2 = q.kout;
        a.sums_ld = q.kout;
        a.add = q.add ? (const char *)q.add + c0 * es : nullptr;
        for (int s2 = 0; s2 < 2; s2++) {
            a.out[s2] = q.out[s2];
            a.out2[s2] = q.out2[s2] ? (char *)q.out2[s2] + c0 * es : nullptr;
        }
        a.opos = opos ? opos + c0 : nullptr;
        a.nout = nout;
        a.theta = q.theta ? q.theta + c0 : nullptr;
        a.wpos = q.wpos ? q.wpos + c0 : nullptr;
        a.sums = q.resid ? c->d_res_out + c0 : nullptr;
        prof_begin(c, step);
        hipError_t e = launch_mv(dt, a, c->st);
        prof_end(c);
        account(kc);
        if (e != hipSuccess) return LOBPCG_ERR_HIP;
    }
    return LOBPCG_OK;
}

int upload_doubles(lobpcg_ctx *c, const std::vector<double> &v, const double **dptr)
{
    const void *d;
    int s = upload_coef(c, DT_F64, v.data(), 1, (int)v.size(), &d);
    *dptr = (const double *)d;
    return s;
}

// Residual of step 7 over the m columns of (X, AX) with Ritz values lam;
// writes W for the columns listed in J (packed) when W is not null and
// returns the sums sum r_j^2, sum x_j^2 (both length m) on the host.
int residual(lobpcg_ctx *c, int dt, const void *X, const void *AX, const std::vector<double> &lam,
             const std::vector<int> &J, void *W, std::vector<double> &rr, std::vector<double> &xx)
{
    const int m = c->m;
    double *hs = (double *)(c->h_pin + c->h_small_off);
    int *hj = (int *)(hs + m);
    for (int j = 0; j < m; j++) hs[j] = lam[j], hj[j] = -1;
    for (size_t i = 0; i < J.size(); i++) hj[J[i]] = (int)i;
    HIPCHK(hipMemcpyAsync(c->d_lambda, hs, m * 8, hipMemcpyHostToDevice, c->st));
    HIPCHK(hipMemcpyAsync(c->d_jpos, hj, m * sizeof(int), hipMemcpyHostToDevice, c->st));
    ResidualArgs a;
    a.X = X;
    a.AX = AX;
    a.lambda = c->d_lambda;
    a.jpos = c->d_jpos;
    a.W = W;
    a.m = m;
    a.nJ = (int)J.size();
    a.N = c->N;
    a.partials = c->d_res_part;
    a.out = c->d_res_out;
    prof_begin(c, LOBPCG_STEP_RESIDUAL);
    if (launch_residual(dt, a, c->st) != hipSuccess) return LOBPCG_ERR_HIP;
    prof_end(c);
    add_bytes(c, LOBPCG_STEP_RESIDUAL, (2.0 * m + (W ? a.nJ : 0)) * c->N * esize(dt));
    double *h = (double *)(c->h_pin + c->h_res_off);
    HIPCHK(hipMemcpyAsync(h, c->d_res_out, 2 * m * 8, hipMemcpyDeviceToHost, c->st));
    int s = sync(c);
    if (s) return s;
    rr.assign(h, h + m);
    xx.assign(h + m, h + 2 * m);
    return LOBPCG_OK;
}

// The fine-level blocks of a V-cycle when they are stored differently from
// the cycle: FP64 blocks around an FP32 cycle (the FP64 phase of the mixed
// solver), or kc columns where the cycle runs on kc rounded up to its vector
// width (the extra columns are zero throughout and never stored).
struct CycleEdge {
    const void *src = nullptr;   // right-hand side as stored (type dt_src, kc columns)
    int dt_src = 0;
    void *dst = nullptr;         // T b as stored (type dt_dst, kc columns) ...
    bool dst_other = false;      // ... or in the fine-level buffer the last sweep does not read
    int dt_dst = 0;
    int kc = 0;
};

// V-cycle on N x k blocks of the multigrid precision.  b: right-hand side at
// level l; xa, xb: two buffers of that level; returns the buffer holding T b.
// With an edge, the fine level's first sweeps read the right-hand side from
// edge->src and write the cycle's copy of it into b (then used by the rest
// of the cycle), and the last sweep writes T b to the edge's destination
// (returned).
void *vcycle(lobpcg_ctx *c, int l, const void *b, void *xa, void *xb, int k, hipError_t &err,
             const CycleEdge *edge = nullptr)
{
    const int dt = c->L.mg_dtype;
    const Grid3 &g = c->L.levels[l];
    const double s = std::pow(4.0, -l), om = c->T.omega;
    const int Lv = (int)c->L.levels.size();
    auto chk = [&](hipError_t e) {
        if (e != hipSuccess && err == hipSuccess) err = e;
    };
    // algorithmic bytes: passes over level-l blocks of k columns
    const double lvl = (double)g.n() * k * esize(dt);
    auto passes = [&](double p) { add_bytes(c, LOBPCG_STEP_PRECOND, p * lvl); };
    if (l == Lv - 1) {
        if (coarse_solve_fits(dt, g)) {
            chk(launch_coarse_solve(dt, g, k, c->T.coarse_sweeps, s, om, b, xa, c->st));
            passes(2.0);
            return xa;
        }
        chk(launch_scale(dt, g.n() * k, b, xa, om / (6.0 * s), c->st));
        passes(2.0);
        void *cur = xa, *oth = xb;
        for (int i = 1; i < c->T.coarse_sweeps; i++) {
            chk(launch_jacobi(dt, g, k, cur, b, oth, s, om, c->st));
            passes(3.0);
            std::swap(cur, oth);
        }
        return cur;
    }
    void *cur = xa, *oth = xb;
    int pre = 1;
    const bool src = edge && edge->src;
    if (src && c->T.nu_pre >= 2) {
        // reads the right-hand side as stored once, writes x and the cycle's copy
        chk(launch_jacobi2_zero_in(edge->dt_src, dt, g, edge->kc, k, edge->src, cur, (void *)b, s, om, c->st));
        pre = 2;
        add_bytes(c, LOBPCG_STEP_PRECOND, (double)g.n() * (edge->kc * esize(edge->dt_src) + 2.0 * k * esize(dt)));
    } else {
        if (src) {
            // (edges with kc < k need the two sweeps above)
            chk(launch_cast(edge->dt_src, dt, g.n() * k, edge->src, (void *)b, c->st));
            passes(1.0 + (double)esize(edge->dt_src) / esize(dt));
        }
        if (c->T.nu_pre >= 2) {
            chk(launch_jacobi2_zero(dt, g, k, b, cur, s, om, c->st));
            pre = 2;
        } else {
            chk(launch_scale(dt, g.n() * k, b, cur, c->T.nu_pre > 0 ? om / (6.0 * s) : 0.0, c->st));
        }
        passes(2.0);
    }
    for (int i = pre; i < c->T.nu_pre; i++) {
        chk(launch_jacobi(dt, g, k, cur, b, oth, s, om, c->st));
        passes(3.0);
        std::swap(cur, oth);
    }
    chk(launch_resid7(dt, g, k, cur, b, oth, s, c->st));
    const Grid3 &gc = c->L.levels[l + 1];
    const double ratio = (double)gc.n() / (double)g.n();
    void *bc = c->mgb[l + 1], *xc = c->mgx[l + 1], *tc = c->mgt[l + 1];
    chk(launch_restrict(dt, g, gc, k, oth, bc, c->st));
    passes(3.0 + 1.0 + ratio);
    void *e = vcycle(c, l + 1, bc, xc, tc, k, err);
    chk(launch_prolong_add(dt, g, gc, k, e, cur, c->st));
    passes(2.0 + ratio);
    const bool dst = edge && (edge->dst || edge->dst_other);
    for (int i = 0; i < c->T.nu_post; i++) {
        if (dst && i + 1 == c->T.nu_post) {
            // the last sweep writes the result as stored
            void *to = edge->dst_other ? oth : edge->dst;
            chk(launch_jacobi_out(dt, edge->dt_dst, g, edge->kc, k, cur, b, to, s, om, c->st));
            add_bytes(c, LOBPCG_STEP_PRECOND, (double)g.n() * (2.0 * k * esize(dt) + edge->kc * esize(edge->dt_dst)));
            return to;
        }
        chk(launch_jacobi(dt, g, k, cur, b, oth, s, om, c->st));
        passes(3.0);
        std::swap(cur, oth);
    }
    if (dst) {
        // (edges with kc < k need a post-smoothing sweep)
        void *to = edge->dst_other ? oth : edge->dst;
        chk(launch_cast(dt, edge->dt_dst, g.n() * k, cur, to, c->st));
        passes(1.0 + (double)esize(edge->dt_dst) / esize(dt));
        return to;
    }
    return cur;
}

// T applied to the N x k block `in` (precision dt); result in one of the two
// fine-level buffers fa / fb of precision dt, returned.  In the FP64 phase of
// the mixed solver the FP32 multigrid runs on a down-cast copy.  An FP32
// cycle on k >= 3 columns, k not a multiple of 4, runs on k rounded up to a
// multiple of 4 (kp), so that every kernel moves 16-byte vectors: kernels on
// such counts move 4 or 8 bytes per lane and measured up to 1.25x slower
// per cycle at 256^3 (31 columns: 11.2 -> 9.4 ms rounded up, 13: 5.4 ->
// 4.5 ms); the extra columns are zero and cost kp/k of the traffic, which
// does not pay for 1 or 2 columns, nor for FP64 cycles (2 columns per 16
// bytes: no faster).  This needs the buffers to hold kp <= m columns, pre-
// and post-smoothing, and a free block `scratch` (N x m of precision dt)
// for the right-hand side's copy.
int apply_T(lobpcg_ctx *c, int dt, const void *in, void *fa, void *fb, int k, void **result, void *scratch)
{
    prof_begin(c, LOBPCG_STEP_PRECOND);
    hipError_t err = hipSuccess;
    const int mdt = c->L.mg_dtype;
    const int vw = 16 / (int)esize(mdt);
    const int kp = (k + vw - 1) / vw * vw;
    const bool multi = c->L.levels.size() > 1;
    const bool pad = kp != k && k >= 3 && mdt == DT_F32 && kp <= c->m && multi && c->T.nu_pre >= 2 &&
                     c->T.nu_post >= 1 && !c->mg_unpadded;
    if (dt == mdt) {
        if (pad && scratch) {
            CycleEdge e;
            e.src = in;
            e.dt_src = dt;
            e.dst_other = true;
            e.dt_dst = dt;
            e.kc = k;
            *result = vcycle(c, 0, scratch, fa, fb, kp, err, &e);
        } else {
            *result = vcycle(c, 0, in, fa, fb, k, err);
        }
    } else {
        // mixed solver, FP64 phase: b32 buffers are free; T in FP32 on FP64
        // blocks, the precision changes taken in the cycle's first and last
        // sweeps (a one-level cycle only: casts around it)
        const long long n = c->N * k;
        void *bin = c->b32.W, *xa = c->b32.AW, *xb = c->b32.T0;
        if (multi) {
            CycleEdge e;
            e.src = in;
            e.dt_src = dt;
            e.dst = fa;
            e.dt_dst = dt;
            e.kc = k;
            *result = vcycle(c, 0, bin, xa, xb, pad ? kp : k, err, &e);
        } else {
            if (launch_cast(dt, mdt, n, in, bin, c->st) != hipSuccess) err = hipErrorUnknown;
            void *r = vcycle(c, 0, bin, xa, xb, k, err);
            if (launch_cast(mdt, dt, n, r, fa, c->st) != hipSuccess) err = hipErrorUnknown;
            add_bytes(c, LOBPCG_STEP_PRECOND, 2.0 * n * (esize(dt) + esize(mdt)));
            *result = fa;
        }
    }
    prof_end(c);
    return err == hipSuccess ? LOBPCG_OK : LOBPCG_ERR_HIP;
}

// Cholesky orthonormalisation of a K x K Gram submatrix: returns R^-1.
bool chol_inv(int n, const std::vector<double> &G, std::vector<double> &Ri)
{
    std::vector<double> R((size_t)n * n);
    if (!chol_scaled(n, G.data(), R.data())) return false;
    Ri.resize((size_t)n * n);
    return triu_inverse(n, R.data(), Ri.data());
}

bool all_finite(const std::vector<double> &v)
{
    for (double x : v)
        if (!std::isfinite(x)) return false;
    return true;
}

double op_norm(lobpcg_ctx *c, const lobpcg_op *A)
{
    if (A->kind == LOBPCG_OP_LAPLACE7) return laplace7_norm(c->g);
    // infinity norm of -div(k grad u): diagonal = sum of the six face
    // coefficients, off-diagonal = the interior faces once more
    const int nx = c->g.nx, ny = c->g.ny, nz = c->g.nz;
    std::vector<double> kx((size_t)nz * ny * (nx + 1)), ky((size_t)nz * (ny + 1) * nx), kz((size_t)(nz + 1) * ny * nx);
    if (hipMemcpyAsync(kx.data(), A->kx, kx.size() * 8, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipMemcpyAsync(ky.data(), A->ky, ky.size() * 8, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipMemcpyAsync(kz.data(), A->kz, kz.size() * 8, hipMemcpyDeviceToHost, c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess)
        return -1.0;
    double best = 0.0;
    for (int z = 0; z < nz; z++)
        for (int y = 0; y < ny; y++)
            for (int x = 0; x < nx; x++) {
                const double a = kx[((size_t)z * ny + y) * (nx + 1) + x], b = kx[((size_t)z * ny + y) * (nx + 1) + x + 1];
                const double cc = ky[((size_t)z * (ny + 1) + y) * nx + x], d = ky[((size_t)z * (ny + 1) + y + 1) * nx + x];
                const double e = kz[((size_t)z * ny + y) * nx + x], f = kz[((size_t)(z + 1) * ny + y) * nx + x];
                double row = a + b + cc + d + e + f;
                row += (x > 0 ? a : 0) + (x + 1 < nx ? b : 0) + (y > 0 ? cc : 0) + (y + 1 < ny ? d : 0) +
                       (z > 0 ? e : 0) + (z + 1 < nz ? f : 0);
                best = std::max(best, row);
            }
    return best;
}

// ---- one LOBPCG phase (steps 6-33) in precision dt on blocks B.
struct PhaseState {
    int cur;                  // which X/AX buffer is current
    std::vector<double> lam;  // Ritz values
    std::vector<int> J;       // active set (step 8)
    std::vector<int> Pcols;   // the columns held (packed, in this order) by B.P / B.AP
    bool have_res;            // B.W holds W_J and d_res_out the norms for X[cur], AX[cur], lam
};

enum { PH_CONVERGED, PH_MAXIT, PH_SWITCH };

std::vector<int> positions(const std::vector<int> &sub, const std::vector<int> &in)
{
    std::vector<int> pos;
    for (int j : sub) {
        auto it = std::find(in.begin(), in.end(), j);
        pos.push_back(it == in.end() ? -1 : (int)(it - in.begin()));
    }
    return pos;
}

// Steps 2 and 10: dst = V - Y (Y^T B Y)^-1 (Y^T B V) for the N x k block V
// (FP64; B = I unless the context has B).  Y^T (B V) comes from the Gram
// kernel (Lm = Y, Rm = V or B V, the latter formed in the spare B-block BPJ,
// which holds nothing between two updates), the small solve runs on the
// host with the Cholesky factor of Y^T B Y, and the update is one
// multivector product [V Y] [I; -C].
int constrain64(lobpcg_ctx *c, const void *V, int k, void *dst, int step);

// Steps 2 and 10 on a block of precision dt.  An FP32 block (the FP32 phase
// of the mixed solver) is projected in FP64 against the FP64 constraints: it
// is up-cast into FP64 scratch blocks (unused during that phase), projected
// there and cast back into dst.
int constrain(lobpcg_ctx *c, int dt, const void *V, int k, void *dst, int step)
{
    if (dt == DT_F64) return constrain64(c, V, k, dst, step);
    const size_t n = (size_t)c->N * k;
    void *v64 = c->b64.W, *p64 = c->b64.T0;
    prof_begin(c, step);
    hipError_t e = launch_cast(DT_F32, DT_F64, (long long)n, V, v64, c->st);
    prof_end(c);
    add_bytes(c, step, 12.0 * n);
    if (e != hipSuccess) return LOBPCG_ERR_HIP;
    int s = constrain64(c, v64, k, p64, step);
    if (s) return s;
    prof_begin(c, step);
    e = launch_cast(DT_F64, DT_F32, (long long)n, p64, dst, c->st);
    prof_end(c);
    add_bytes(c, step, 12.0 * n);
    return e == hipSuccess ? LOBPCG_OK : LOBPCG_ERR_HIP;
}

// Y^T V (ny x k, row-major) for the N x k FP64 block V, in launches of at
// most GX_MAX_L rows of Y
int gram_Yt(lobpcg_ctx *c, const void *V, int k, std::vector<double> &G, int step)
{
    const int ny = c->ny;
    G.assign((size_t)ny * k, 0.0);
    for (int i0 = 0; i0 < ny; i0 += GX_MAX_L) {
        const int nr = std::min(GX_MAX_L, ny - i0);
        GramXArgs a;
        for (int b = 0; b < GX_MAX_ARR; b++) a.arr[b] = nullptr, a.ld[b] = 1;
        a.arr[0] = c->Y, a.ld[0] = ny;
        a.arr[1] = V, a.ld[1] = k;
        a.KL = nr;
        a.KR = k;
        for (int i = 0; i < nr; i++) a.lmap[i] = (unsigned short)(i0 + i);
        for (int j = 0; j < k; j++) a.rmap[j] = (unsigned short)((1 << 8) | j);
        const int TL = (nr + 15) / 16, TR = (k + 15) / 16;
        a.ntiles = TL * TR;
        if (k > GX_MAX_R || a.ntiles > GX_MAX_TILES) return LOBPCG_ERR_ARG;
        for (int t = 0; t < a.ntiles; t++) a.ta[t] = t / TR, a.tb[t] = t % TR;
        a.N = c->N;
        a.partials = c->d_gram_part;
        a.out = c->d_gram_out;
        a.max_nt = 2;
        a.max_nt32 = c->gram_nt32;
        a.direct = c->gram_direct;
        prof_begin(c, step);
        if (launch_gramx(DT_F64, a, c->st) != hipSuccess) return LOBPCG_ERR_HIP;
        prof_end(c);
        add_bytes(c, step, (double)(nr + k) * c->N * 8.0);
        double *h = (double *)(c->h_pin + c->h_gram_off);
        HIPCHK(hipMemcpyAsync(h, c->d_gram_out, (size_t)a.ntiles * 256 * 8, hipMemcpyDeviceToHost, c->st));
        int s = sync(c);
        if (s) return s;
        // FP64 accumulator layout: row l/16 + 4r
        for (int t = 0; t < a.ntiles; t++)
            for (int e = 0; e < 256; e++) {
                const int r = e / 64, lane = e % 64;
                const int i = 16 * a.ta[t] + lane / 16 + 4 * r, j = 16 * a.tb[t] + lane % 16;
                if (i < nr && j < k) G[(size_t)(i0 + i) * k + j] = h[(size_t)t * 256 + e];
            }
    }
    return all_finite(G) ? LOBPCG_OK : LOBPCG_ERR_NONFINITE;
}

int constrain64(lobpcg_ctx *c, const void *V, int k, void *dst, int step)
{
    const int ny = c->ny;
    const void *BV = V;
    if (c->hasB) {
        int s = apply_B(c, DT_F64, V, c->b64.BPJ, k, step);
        if (s) return s;
        BV = c->b64.BPJ;
    }
    std::vector<double> G;
    int s = gram_Yt(c, BV, k, G, step);
    if (s) return s;
    // C = (RY^T RY)^-1 G (RY^T RY = Y^T B Y): forward then back substitution,
    // column by column
    std::vector<double> C(G);
    for (int j = 0; j < k; j++) {
        for (int i = 0; i < ny; i++) {
            double v = C[(size_t)i * k + j];
            for (int l = 0; l < i; l++) v -= c->RY[(size_t)l * ny + i] * C[(size_t)l * k + j];
            C[(size_t)i * k + j] = v / c->RY[(size_t)i * ny + i];
        }
        for (int i = ny - 1; i >= 0; i--) {
            double v = C[(size_t)i * k + j];
            for (int l = i + 1; l < ny; l++) v -= c->RY[(size_t)i * ny + l] * C[(size_t)l * k + j];
            C[(size_t)i * k + j] = v / c->RY[(size_t)i * ny + i];
        }
    }
    // [V Y] [I; -C]
    std::vector<double> coef((size_t)(k + ny) * k, 0.0);
    for (int i = 0; i < k; i++) coef[(size_t)i * k + i] = 1.0;
    for (int i = 0; i < ny; i++)
        for (int j = 0; j < k; j++) coef[(size_t)(k + i) * k + j] = -C[(size_t)i * k + j];
    MV q;
    q.input(0, V, nullptr, k, k);
    q.input(1, c->Y, nullptr, ny, ny);
    q.kout = k;
    q.out[0] = dst;
    return mv(c, DT_F64, q, coef.data(), step);
}

// Steps 11-33 with the Cholesky-QR factors of W_J and P_J (steps 11 and 14-15)
// folded into the Gram matrices and the update coefficients instead of being
// applied to the blocks.  With W_J = Wn R_W and P_J = Pn R_P, the Gram blocks of
// the orthonormal Wn, Pn are R^-T (.) R^-1 of those of W_J, P_J, and
// Wn C_W = W_J (R_W^-1 C_W): the same algebra, with one pass over the blocks
// (the Gram products, which then include W_J^T W_J and P_J^T P_J) instead of
// three (Gram, R^-1 applied to W_J; Gram, R^-1 applied to P_J and AP_J).  A W_J
// is formed from the unnormalised W_J.  On entry W_J = T(residual) is in Wt.
// Sets `switched` when the FP32 phase of the mixed solver must end.
int folded_step(lobpcg_ctx *c, const lobpcg_op *A, int dt, Blocks &B, PhaseState &ps, void *Wt, int nJ,
                bool explicit_gram, bool allow_switch, bool &switched)
{
    const int m = c->m;
    int s;
    switched = false;
    if (Wt == B.AW)
        std::swap(B.W, B.AW);
    else if (Wt == B.T0)
        std::swap(B.W, B.T0);
    // step 12: A W_J (and B W_J)
    s = apply_A(c, A, dt, B.W, B.AW, nJ);
    if (s) return s;
    const bool hb = c->hasB;
    if (hb) {
        s = apply_B(c, dt, B.W, B.BW, nJ, LOBPCG_STEP_APPLY_A);
        if (s) return s;
    }
    // P_J: the active columns that have a direction, read in place from B.P
    std::vector<int> ppos;
    for (int j : ps.J) {
        auto it = std::find(ps.Pcols.begin(), ps.Pcols.end(), j);
        if (it != ps.Pcols.end()) ppos.push_back((int)(it - ps.Pcols.begin()));
    }
    int nP = (int)ppos.size();
    const int np = (int)ps.Pcols.size();
    // steps 17-23, with the Gram matrices of steps 11 and 14 in the same pass
    std::vector<double> SS, SAS;
    {
        const void *Sb[3] = {B.X[ps.cur], B.W, B.P};
        const void *ASb[3] = {B.AX[ps.cur], B.AW, B.AP};
        const void *BSb[3] = {B.BX[ps.cur], B.BW, B.BP};
        int wb[3] = {m, nJ, nP}, ldb[3] = {m, nJ, np};
        const int *cl[3] = {nullptr, nullptr, nP ? ppos.data() : nullptr};
        s = gram(c, dt, nP ? 3 : 2, Sb, ASb, wb, SS, &SAS, LOBPCG_STEP_GRAM, !explicit_gram, cl, ldb, true,
                 hb ? BSb : nullptr);
        if (s) return s;
        if (!all_finite(SS) || !all_finite(SAS)) return LOBPCG_ERR_NONFINITE;
    }
    const int K0 = m + nJ + nP;
    auto block = [&](int i0, int n0) {
        std::vector<double> G((size_t)n0 * n0);
        for (int i = 0; i < n0; i++)
            for (int j = 0; j < n0; j++) G[(size_t)i * n0 + j] = SS[(size_t)(i0 + i) * K0 + i0 + j];
        return G;
    };
    // step 11: R_W (failure: the error of step 11, or the end of the FP32 phase)
    std::vector<double> RiW, RiP;
    if (!chol_inv(nJ, block(m, nJ), RiW)) {
        if (allow_switch) {
            switched = true;
            return LOBPCG_OK;
        }
        return LOBPCG_ERR_CHOL;
    }
    // step 14: R_P (failure: this iteration runs without P)
    if (nP && !chol_inv(nP, block(m + nJ, nP), RiP)) {
        nP = 0;
        c->stats.restarts++;
    }
    const int nPr = nP;   // order of R_P^-1
    // (D^T M D) for D = diag(I, R_W^-1, R_P^-1) over the leading K x K part;
    // the R^-1 are upper triangular
    auto congruence = [&](const std::vector<double> &M, int K, int nPk) {
        auto dcol = [&](int j, int &b0, int &jj) {   // block start and index within the block
            if (j < m) { b0 = -1, jj = j; }
            else if (j < m + nJ) { b0 = m, jj = j - m; }
            else { b0 = m + nJ, jj = j - m - nJ; }
        };
        std::vector<double> T1((size_t)K * K), out((size_t)K * K);
        for (int i = 0; i < K; i++)
            for (int j = 0; j < K; j++) {
                int b0, jj;
                dcol(j, b0, jj);
                double v = 0.0;
                if (b0 < 0) v = M[(size_t)i * K0 + j];
                else if (b0 == m)
                    for (int l = 0; l <= jj; l++) v += M[(size_t)i * K0 + m + l] * RiW[(size_t)l * nJ + jj];
                else
                    for (int l = 0; l <= jj; l++) v += M[(size_t)i * K0 + m + nJ + l] * RiP[(size_t)l * nPk + jj];
                T1[(size_t)i * K + j] = v;
            }
        for (int i = 0; i < K; i++)
            for (int j = 0; j < K; j++) {
                int b0, ii;
                dcol(i, b0, ii);
                double v = 0.0;
                if (b0 < 0) v = T1[(size_t)i * K + j];
                else if (b0 == m)
                    for (int l = 0; l <= ii; l++) v += RiW[(size_t)l * nJ + ii] * T1[(size_t)(m + l) * K + j];
                else
                    for (int l = 0; l <= ii; l++) v += RiP[(size_t)l * nPk + ii] * T1[(size_t)(m + nJ + l) * K + j];
                out[(size_t)i * K + j] = v;
            }
        for (int i = 0; i < K; i++)
            for (int j = i + 1; j < K; j++) {
                const double v = 0.5 * (out[(size_t)i * K + j] + out[(size_t)j * K + i]);
                out[(size_t)i * K + j] = out[(size_t)j * K + i] = v;
            }
        return out;
    };
    // step 24 on the orthonormalised basis [X, Wn, Pn] (on failure with P,
    // retry without it)
    std::vector<double> theta(m), C;
    int Kused = 0;
    bool ok = false;
    for (int attempt = 0; attempt < 2 && !ok; attempt++) {
        if (attempt == 1) {
            if (!nP) break;
            nP = 0;
            c->stats.restarts++;
        }
        Kused = m + nJ + nP;
        std::vector<double> gA = congruence(SAS, Kused, nPr);
        std::vector<double> gB = congruence(SS, Kused, nPr);
        if (!explicit_gram) {
            // the paper's form: Lambda and identities on the block diagonal
            auto blk = [&](int i0, int n0, std::vector<double> &M, bool lam) {
                for (int i = 0; i < n0; i++)
                    for (int j = 0; j < n0; j++)
                        M[(size_t)(i0 + i) * Kused + i0 + j] = (i == j) ? (lam ? ps.lam[i] : 1.0) : 0.0;
            };
            blk(0, m, gA, true);
            blk(0, m, gB, false);
            blk(m, nJ, gB, false);
            if (nP) blk(m + nJ, nP, gB, false);
        }
        C.assign((size_t)Kused * m, 0.0);
        auto t0 = std::chrono::steady_clock::now();
        ok = rayleigh_ritz(Kused, m, gA.data(), gB.data(), theta.data(), C.data());
        auto t1 = std::chrono::steady_clock::now();
        c->stats.step_ms[LOBPCG_STEP_RR] += std::chrono::duration<double, std::milli>(t1 - t0).count();
        c->stats.step_calls[LOBPCG_STEP_RR] += 1;
    }
    if (!ok) {
        if (allow_switch) {
            switched = true;
            return LOBPCG_OK;
        }
        return LOBPCG_ERR_RR;
    }
    // coefficients for the unnormalised blocks: rows of W_J and P_J times R^-1
    {
        std::vector<double> Cd(C);
        for (int ii = 0; ii < nJ; ii++)
            for (int j = 0; j < m; j++) {
                double v = 0.0;
                for (int l = ii; l < nJ; l++) v += RiW[(size_t)ii * nJ + l] * C[(size_t)(m + l) * m + j];
                Cd[(size_t)(m + ii) * m + j] = v;
            }
        for (int ii = 0; ii < nP; ii++)
            for (int j = 0; j < m; j++) {
                double v = 0.0;
                for (int l = ii; l < nP; l++) v += RiP[(size_t)ii * nPr + l] * C[(size_t)(m + nJ + l) * m + j];
                Cd[(size_t)(m + nJ + ii) * m + j] = v;
            }
        C.swap(Cd);
    }
    // steps 25-33 fused with step 7 of the next iteration; the new P, AP go to
    // the spare pair of blocks (the old P_J is read in place)
    std::vector<int> jpos(m, -1);
    for (int i = 0; i < nJ; i++) jpos[ps.J[i]] = i;
    const int *djpos, *dppos = nullptr;
    const double *dtheta;
    s = upload_cols(c, jpos, &djpos);
    if (s) return s;
    // P_J is all of P, in order, whenever J has not changed since P was
    // written: then it is read whole (16-byte fragment loads) rather than
    // through a column list
    bool p_whole = nP == np;
    for (int i = 0; i < nP && p_whole; i++) p_whole = ppos[i] == i;
    if (nP && !p_whole) {
        s = upload_cols(c, ppos, &dppos);
        if (s) return s;
    }
    s = upload_doubles(c, theta, &dtheta);
    if (s) return s;
    MV q;
    q.nside = 2;
    if (hb) {
        // three sides: X alone, then B X and A X with the residual W = AX' - BX' Theta
        MV qx;
        qx.input(0, B.X[ps.cur], nullptr, m, m);
        qx.input(1, B.W, nullptr, nJ, nJ);
        if (nP) qx.input(2, B.P, nullptr, np, nP, dppos);
        qx.kout = m;
        qx.out[0] = B.PJ;
        qx.opos = djpos;
        qx.nout = nJ;
        qx.out2[0] = B.X[1 - ps.cur];
        s = mv(c, dt, qx, C.data(), LOBPCG_STEP_UPDATE);
        if (s) return s;
        q.input(0, B.BX[ps.cur], B.AX[ps.cur], m, m);
        q.input(1, B.BW, B.AW, nJ, nJ);
        if (nP) q.input(2, B.BP, B.AP, np, nP, dppos);
        q.out[0] = B.BPJ;
        q.out2[0] = B.BX[1 - ps.cur];
    } else {
        q.input(0, B.X[ps.cur], B.AX[ps.cur], m, m);
        q.input(1, B.W, B.AW, nJ, nJ);
        if (nP) q.input(2, B.P, B.AP, np, nP, dppos);
        q.out[0] = B.PJ;
        q.out2[0] = B.X[1 - ps.cur];
    }
    q.kout = m;
    q.out[1] = B.APJ;
    q.opos = djpos;
    q.nout = nJ;
    q.out2[1] = B.AX[1 - ps.cur];
    q.resid = true;
    q.theta = dtheta;
    q.wpos = djpos;
    q.Wout = B.T0;
    q.nW = nJ;
    s = mv(c, dt, q, C.data(), LOBPCG_STEP_UPDATE);
    if (s) return s;
    std::swap(B.P, B.PJ);
    std::swap(B.AP, B.APJ);
    if (hb) std::swap(B.BP, B.BPJ);
    std::swap(B.W, B.T0);
    ps.Pcols = ps.J;
    ps.cur = 1 - ps.cur;
    ps.lam = theta;
    ps.have_res = true;
    return LOBPCG_OK;
}

// An FP32 iteration with few active columns takes the paper's form of the
// Gram matrices even where the explicit one is chosen: X then changes little
// per iteration, and the Gram step reads neither AX nor the X-X tiles.
bool narrow_fp32(const lobpcg_ctx *c, int dt, int nJ)
{
    const int above = c->fp32_explicit_above >= 0 ? c->fp32_explicit_above : c->m / 4;
    return dt == DT_F32 && nJ <= above;
}

int run_phase(lobpcg_ctx *c, const lobpcg_op *A, int dt, Blocks &B, PhaseState &ps, double tol, double normA,
              int maxit, int &iters, double *h_hist, bool explicit_gram, bool allow_switch, int &outcome)
{
    const int m = c->m;
    const int nw = c->nwant > 0 ? c->nwant : m;   // wanted pairs; the others are guard columns
    std::vector<double> rr(m), xx(m), rho(m), SS, SAS, PP;
    std::vector<double> hist_max;
    outcome = PH_MAXIT;
    while (iters < maxit) {
        // steps 7-8: W_J and the residual norms of all m columns; after an
        // update they come from the fused update kernel
        int s;
        if (ps.have_res) {
            double *h = (double *)(c->h_pin + c->h_res_off);
            HIPCHK(hipMemcpyAsync(h, c->d_res_out, 2 * m * 8, hipMemcpyDeviceToHost, c->st));
            s = sync(c);
            if (s) return s;
            rr.assign(h, h + m);
            xx.assign(h + m, h + 2 * m);
        } else {
            s = residual(c, dt, c->hasB ? B.BX[ps.cur] : B.X[ps.cur], B.AX[ps.cur], ps.lam, ps.J, B.W, rr, xx);
            if (s) return s;
        }
        ps.have_res = false;
        double rmax = 0.0;   // over the wanted columns
        for (int j = 0; j < m; j++) {
            rho[j] = std::sqrt(rr[j]) / (normA * std::sqrt(xx[j]));
            if (!std::isfinite(rho[j])) return LOBPCG_ERR_NONFINITE;
            if (j < nw) rmax = std::max(rmax, rho[j]);
        }
        if (h_hist) std::copy(rho.begin(), rho.end(), h_hist + (size_t)iters * m);
        iters++;
        if (dt == DT_F32) c->stats.iters_fp32++;
        else c->stats.iters_fp64++;
        // a block wider than the wanted set (Section 2.1.3): done once the
        // first nw Ritz pairs have converged, whatever the guard columns do
        if (nw < m && rmax <= tol) {
            outcome = PH_CONVERGED;
            return LOBPCG_OK;
        }
        // step 8: drop converged columns; end only when every residual is small
        std::vector<int> Jn;
        for (int j : ps.J) {
            bool keep = rho[j] > tol;
            // a converged column of a cluster stays active while a column of
            // the same cluster is still unconverged
            for (size_t i = 0; i < ps.J.size() && !keep && c->lock_gap > 0.0; i++) {
                const int a = ps.J[i];
                keep = rho[a] > tol && std::fabs(ps.lam[a] - ps.lam[j]) <= c->lock_gap * std::fabs(ps.lam[a]);
            }
            if (keep) Jn.push_back(j);
        }
        if (Jn.empty() && c->reactivate)
            for (int j = 0; j < m; j++)
                if (rho[j] > tol) Jn.push_back(j);
        if (Jn.empty()) {
            outcome = PH_CONVERGED;
            return LOBPCG_OK;
        }
        if (allow_switch) {
            hist_max.push_back(rmax);
            const int wdw = c->stall_window;
            if ((int)hist_max.size() > wdw && rmax > c->stall_factor * hist_max[hist_max.size() - 1 - wdw]) {
                outcome = PH_SWITCH;
                return LOBPCG_OK;
            }
        }
        if (Jn != ps.J) {
            std::vector<int> pos = positions(Jn, ps.J);
            if (std::find(pos.begin(), pos.end(), -1) == pos.end()) {
                // the active set shrank: pack the surviving columns of W
                const int *dmap;
                s = upload_cols(c, pos, &dmap);
                if (s) return s;
                prof_begin(c, LOBPCG_STEP_RESIDUAL);
                hipError_t e = launch_gather_cols(dt, c->N, B.W, (int)ps.J.size(), dmap, (int)Jn.size(), B.T0, c->st);
                prof_end(c);
                add_bytes(c, LOBPCG_STEP_RESIDUAL, 2.0 * Jn.size() * c->N * esize(dt));
                if (e != hipSuccess) return LOBPCG_ERR_HIP;
                std::swap(B.W, B.T0);
                ps.J = Jn;
            } else {
                // columns made active again: form W for the new set
                ps.J = Jn;
                s = residual(c, dt, c->hasB ? B.BX[ps.cur] : B.X[ps.cur], B.AX[ps.cur], ps.lam, ps.J, B.W, rr, xx);
                if (s) return s;
            }
        }
        const int nJ = (int)ps.J.size();
        // step 9: W_J = T W_J
        void *Wt = B.W;
        if (c->mg) {
            s = apply_T(c, dt, B.W, B.AW, B.T0, nJ, &Wt, B.X[1 - ps.cur]);
            if (s) return s;
        }
        // step 10: W_J = W_J - Y (Y^T Y)^-1 (Y^T W_J)
        if (c->ny) {
            void *dst = (Wt == B.T0) ? B.AW : B.T0;
            s = constrain(c, dt, Wt, nJ, dst, LOBPCG_STEP_PRECOND);
            if (s) return s;
            Wt = dst;
        }
        if (c->fold) {
            bool switched;
            s = folded_step(c, A, dt, B, ps, Wt, nJ, explicit_gram && !narrow_fp32(c, dt, nJ), allow_switch,
                            switched);
            if (s) return s;
            if (switched) {
                outcome = PH_SWITCH;
                return LOBPCG_OK;
            }
            continue;
        }
        // step 11: W_J = W_J R^-1 with R = chol(W_J^T B W_J); the result goes
        // to whichever of W / T0 does not hold the input (with B, B W_J is
        // formed for the Gram matrix and again for the orthonormal W_J)
        const bool hb = c->hasB;
        {
            const void *Sb[1] = {Wt};
            const void *BSb[1] = {B.BW};
            int w1[1] = {nJ};
            if (hb) {
                s = apply_B(c, dt, Wt, B.BW, nJ, LOBPCG_STEP_ORTHO);
                if (s) return s;
            }
            s = gram(c, dt, 1, Sb, nullptr, w1, SS, nullptr, LOBPCG_STEP_ORTHO, false, nullptr, nullptr, false,
                     hb ? BSb : nullptr);
            if (s) return s;
            std::vector<double> Ri;
            if (!all_finite(SS)) return LOBPCG_ERR_NONFINITE;
            if (!chol_inv(nJ, SS, Ri)) {
                if (allow_switch) {
                    outcome = PH_SWITCH;
                    return LOBPCG_OK;
                }
                return LOBPCG_ERR_CHOL;
            }
            void *dst = (Wt == B.W) ? B.T0 : B.W;
            MV q;
            q.input(0, Wt, nullptr, nJ, nJ);
            q.kout = nJ;
            q.out[0] = dst;
            s = mv(c, dt, q, Ri.data(), LOBPCG_STEP_ORTHO);
            if (s) return s;
            if (dst == B.T0) std::swap(B.W, B.T0);
        }
        // step 12: AW_J = A W_J (and B W_J)
        s = apply_A(c, A, dt, B.W, B.AW, nJ);
        if (s) return s;
        if (hb) {
            s = apply_B(c, dt, B.W, B.BW, nJ, LOBPCG_STEP_ORTHO);
            if (s) return s;
        }
        // steps 13-16: orthonormalise the directions of the active columns
        // that have one (P holds the columns ps.Pcols)
        std::vector<int> Jp, ppos;
        for (int j : ps.J) {
            auto it = std::find(ps.Pcols.begin(), ps.Pcols.end(), j);
            if (it != ps.Pcols.end()) {
                Jp.push_back(j);
                ppos.push_back((int)(it - ps.Pcols.begin()));
            }
        }
        int nP = 0;
        if (!Jp.empty()) {
            const int np = (int)ps.Pcols.size();
            const void *Sb[1] = {B.P};
            const void *BSb[1] = {B.BP};
            int w1[1] = {np};
            s = gram(c, dt, 1, Sb, nullptr, w1, PP, nullptr, LOBPCG_STEP_ORTHO, false, nullptr, nullptr, false,
                     hb ? BSb : nullptr);
            if (s) return s;
            const int k = (int)Jp.size();
            std::vector<double> G((size_t)k * k), Ri;
            for (int i = 0; i < k; i++)
                for (int j = 0; j < k; j++) G[(size_t)i * k + j] = PP[(size_t)ppos[i] * np + ppos[j]];
            if (all_finite(G) && chol_inv(k, G, Ri)) {
                const int *dcols;
                s = upload_cols(c, ppos, &dcols);
                if (s) return s;
                MV q;
                q.nside = 2;
                q.input(0, B.P, B.AP, np, k, dcols);
                q.kout = k;
                q.out[0] = B.PJ;
                q.out[1] = B.APJ;
                s = mv(c, dt, q, Ri.data(), LOBPCG_STEP_ORTHO);
                if (s) return s;
                if (hb) {
                    MV qb;
                    qb.input(0, B.BP, nullptr, np, k, dcols);
                    qb.kout = k;
                    qb.out[0] = B.BPJ;
                    s = mv(c, dt, qb, Ri.data(), LOBPCG_STEP_ORTHO);
                    if (s) return s;
                }
                nP = k;
            } else {
                c->stats.restarts++;
            }
        }
        // steps 17-23: Gram matrices of the trial basis [X, W_J, P_J]
        const int nb = nP ? 3 : 2;
        const void *Sb[3] = {B.X[ps.cur], B.W, B.PJ};
        const void *ASb[3] = {B.AX[ps.cur], B.AW, B.APJ};
        int wb[3] = {m, nJ, nP};
        const bool eg = explicit_gram && !narrow_fp32(c, dt, nJ);
        const void *BSb[3] = {B.BX[ps.cur], B.BW, B.BPJ};
        s = gram(c, dt, nb, Sb, ASb, wb, SS, &SAS, LOBPCG_STEP_GRAM, !eg, nullptr, nullptr, false,
                 hb ? BSb : nullptr);
        if (s) return s;
        if (!all_finite(SS) || !all_finite(SAS)) return LOBPCG_ERR_NONFINITE;
        const int K = m + nJ + nP;
        std::vector<double> gA(SAS), gB(SS);
        if (!eg) {
            // the paper's form: Lambda and identities on the block diagonal
            auto blk = [&](int i0, int n0, std::vector<double> &M, bool lam) {
                for (int i = 0; i < n0; i++)
                    for (int j = 0; j < n0; j++)
                        M[(size_t)(i0 + i) * K + i0 + j] = (i == j) ? (lam ? ps.lam[i] : 1.0) : 0.0;
            };
            blk(0, m, gA, true);
            blk(0, m, gB, false);
            blk(m, nJ, gB, false);
            if (nP) blk(m + nJ, nP, gB, false);
        }
        // step 24 (on failure with P, retry on the leading [X, W_J] part)
        std::vector<double> theta(m), C;
        int Kused = K;
        bool ok = false;
        for (int attempt = 0; attempt < 2 && !ok; attempt++) {
            if (attempt == 1) {
                if (!nP) break;
                nP = 0;
                c->stats.restarts++;
                Kused = m + nJ;
            }
            std::vector<double> a2((size_t)Kused * Kused), b2((size_t)Kused * Kused);
            for (int i = 0; i < Kused; i++)
                for (int j = 0; j < Kused; j++) {
                    a2[(size_t)i * Kused + j] = gA[(size_t)i * K + j];
                    b2[(size_t)i * Kused + j] = gB[(size_t)i * K + j];
                }
            C.assign((size_t)Kused * m, 0.0);
            auto t0 = std::chrono::steady_clock::now();
            ok = rayleigh_ritz(Kused, m, a2.data(), b2.data(), theta.data(), C.data());
            auto t1 = std::chrono::steady_clock::now();
            c->stats.step_ms[LOBPCG_STEP_RR] += std::chrono::duration<double, std::milli>(t1 - t0).count();
            c->stats.step_calls[LOBPCG_STEP_RR] += 1;
        }
        if (!ok) {
            if (allow_switch) {
                outcome = PH_SWITCH;
                return LOBPCG_OK;
            }
            return LOBPCG_ERR_RR;
        }
        // steps 25-33 fused with step 7 of the next iteration:
        //   P = W_J C_W + P_J C_P, X' = X C_X + P (and AP, AX'); P and AP are
        //   stored for the active columns only; W = AX'_J - X'_J Theta_J
        std::vector<int> jpos(m, -1);
        for (int i = 0; i < nJ; i++) jpos[ps.J[i]] = i;
        const int *djpos;
        const double *dtheta;
        s = upload_cols(c, jpos, &djpos);
        if (s) return s;
        s = upload_doubles(c, theta, &dtheta);
        if (s) return s;
        MV q;
        q.nside = 2;
        if (hb) {
            // three sides, as in the folded step: X alone, then B X and A X
            // with the residual W = AX' - BX' Theta
            MV qx;
            qx.input(0, B.X[ps.cur], nullptr, m, m);
            qx.input(1, B.W, nullptr, nJ, nJ);
            if (nP) qx.input(2, B.PJ, nullptr, nP, nP);
            qx.kout = m;
            qx.out[0] = B.P;
            qx.opos = djpos;
            qx.nout = nJ;
            qx.out2[0] = B.X[1 - ps.cur];
            s = mv(c, dt, qx, C.data(), LOBPCG_STEP_UPDATE);
            if (s) return s;
            q.input(0, B.BX[ps.cur], B.AX[ps.cur], m, m);
            q.input(1, B.BW, B.AW, nJ, nJ);
            if (nP) q.input(2, B.BPJ, B.APJ, nP, nP);
            q.out[0] = B.BP;
            q.out2[0] = B.BX[1 - ps.cur];
        } else {
            q.input(0, B.X[ps.cur], B.AX[ps.cur], m, m);
            q.input(1, B.W, B.AW, nJ, nJ);
            if (nP) q.input(2, B.PJ, B.APJ, nP, nP);
            q.out[0] = B.P;
            q.out2[0] = B.X[1 - ps.cur];
        }
        q.kout = m;
        q.out[1] = B.AP;
        q.opos = djpos;
        q.nout = nJ;
        q.out2[1] = B.AX[1 - ps.cur];
        q.resid = true;
        q.theta = dtheta;
        q.wpos = djpos;
        q.Wout = B.T0;
        q.nW = nJ;
        s = mv(c, dt, q, C.data(), LOBPCG_STEP_UPDATE);
        if (s) return s;
        std::swap(B.W, B.T0);
        ps.Pcols = ps.J;
        ps.cur = 1 - ps.cur;
        ps.lam = theta;
        ps.have_res = true;
    }
    return LOBPCG_OK;
}

// Steps 3-4 (and the restart of the mixed solver in FP64): orthonormalise X
// if asked, A X, Rayleigh-Ritz on span(X).  On entry X is in B.X[ps.cur].
int init_phase(lobpcg_ctx *c, const lobpcg_op *A, int dt, Blocks &B, PhaseState &ps, bool ortho, bool explicit_gram)
{
    const int m = c->m;
    std::vector<double> SS, SAS;
    int s;
    const bool hb = c->hasB;
    if (ortho) {
        // step 3: R = chol(X^T B X), X = X R^-1 (and B X = B X R^-1)
        const void *Sb[1] = {B.X[ps.cur]};
        const void *BSb[1] = {hb ? B.BX[ps.cur] : nullptr};
        int w1[1] = {m};
        if (hb) {
            s = apply_B(c, dt, B.X[ps.cur], B.BX[ps.cur], m, LOBPCG_STEP_ORTHO);
            if (s) return s;
        }
        s = gram(c, dt, 1, Sb, nullptr, w1, SS, nullptr, LOBPCG_STEP_ORTHO, false, nullptr, nullptr, false,
                 hb ? BSb : nullptr);
        if (s) return s;
        if (!all_finite(SS)) return LOBPCG_ERR_NONFINITE;
        std::vector<double> Ri;
        if (!chol_inv(m, SS, Ri)) return LOBPCG_ERR_CHOL;
        MV q;
        if (hb) {
            q.nside = 2;
            q.input(0, B.X[ps.cur], B.BX[ps.cur], m, m);
            q.out[1] = B.BX[1 - ps.cur];
        } else {
            q.input(0, B.X[ps.cur], nullptr, m, m);
        }
        q.kout = m;
        q.out[0] = B.X[1 - ps.cur];
        s = mv(c, dt, q, Ri.data(), LOBPCG_STEP_ORTHO);
        if (s) return s;
        ps.cur = 1 - ps.cur;
    }
    if (hb && !ortho) {
        // B X of a start block that was not B-orthonormalised here (the
        // FP64 restart of the mixed solver)
        s = apply_B(c, dt, B.X[ps.cur], B.BX[ps.cur], m, LOBPCG_STEP_OTHER);
        if (s) return s;
    }
    s = apply_A(c, A, dt, B.X[ps.cur], B.AX[ps.cur], m);
    if (s) return s;
    const void *Sb[1] = {B.X[ps.cur]}, *ASb[1] = {B.AX[ps.cur]}, *BSb1[1] = {hb ? B.BX[ps.cur] : nullptr};
    int w1[1] = {m};
    // X^T B X (X^T X for B = I) and X^T A X
    s = gram(c, dt, 1, Sb, ASb, w1, SS, &SAS, LOBPCG_STEP_GRAM, false, nullptr, nullptr, false,
             hb ? BSb1 : nullptr);
    if (s) return s;
    if (!all_finite(SS) || !all_finite(SAS)) return LOBPCG_ERR_NONFINITE;
    if (!explicit_gram) {
        std::fill(SS.begin(), SS.end(), 0.0);
        for (int i = 0; i < m; i++) SS[(size_t)i * m + i] = 1.0;
    }
    std::vector<double> theta(m), Z((size_t)m * m);
    if (!rayleigh_ritz(m, m, SAS.data(), SS.data(), theta.data(), Z.data())) return LOBPCG_ERR_RR;
    MV q;
    q.nside = 2;
    q.input(0, B.X[ps.cur], B.AX[ps.cur], m, m);
    q.kout = m;
    q.out[0] = B.X[1 - ps.cur];
    q.out[1] = B.AX[1 - ps.cur];
    s = mv(c, dt, q, Z.data(), LOBPCG_STEP_OTHER);
    if (s) return s;
    if (hb) {
        MV qb;
        qb.input(0, B.BX[ps.cur], nullptr, m, m);
        qb.kout = m;
        qb.out[0] = B.BX[1 - ps.cur];
        s = mv(c, dt, qb, Z.data(), LOBPCG_STEP_OTHER);
        if (s) return s;
    }
    ps.cur = 1 - ps.cur;
    ps.lam = theta;
    ps.J.clear();
    for (int j = 0; j < m; j++) ps.J.push_back(j);
    ps.have_res = false;
    return LOBPCG_OK;
}

}  // namespace

// ============================================================================ ABI

extern "C" {

const char *lobpcg_status_string(int s)
{
    switch (s) {
    case LOBPCG_OK: return "converged";
    case LOBPCG_NOT_CONVERGED: return "not converged within maxit";
    case LOBPCG_ERR_ARG: return "invalid argument";
    case LOBPCG_ERR_UNSUPPORTED: return "unsupported combination of options";
    case LOBPCG_ERR_WORKSPACE: return "workspace too small or misaligned";
    case LOBPCG_ERR_CHOL: return "Cholesky factorisation failed";
    case LOBPCG_ERR_RR: return "Rayleigh-Ritz failed";
    case LOBPCG_ERR_NONFINITE: return "non-finite values";
    case LOBPCG_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
    }
}

int lobpcg_workspace_bytes(const lobpcg_op *A, const lobpcg_op *B, const lobpcg_precond *T, int m, int precision,
                           size_t *bytes)
{
    if (!bytes) return LOBPCG_ERR_ARG;
    int s = check_common(A, B, T, m, precision);
    if (s) return s;
    *bytes = make_layout(A, B, T, m, precision).total;
    return LOBPCG_OK;
}

int lobpcg_setup(lobpcg_ctx **out, const lobpcg_op *A, const lobpcg_op *B, const lobpcg_precond *T, int m,
                 int precision, void *d_workspace, size_t ws_bytes, void *stream)
{
    if (!out) return LOBPCG_ERR_ARG;
    *out = nullptr;
    int s = check_common(A, B, T, m, precision);
    if (s) return s;
    Layout L = make_layout(A, B, T, m, precision);
    if (!d_workspace || ws_bytes < L.total || ((uintptr_t)d_workspace % ALIGN)) return LOBPCG_ERR_WORKSPACE;
    lobpcg_ctx *c = new lobpcg_ctx();
    c->g = Grid3{A->nx, A->ny, A->nz};
    c->N = c->g.n();
    c->m = m;
    c->precision = precision;
    c->A = *A;
    c->mg = has_mg(T);
    if (T) c->T = *T;
    else memset(&c->T, 0, sizeof(c->T));
    c->st = (hipStream_t)stream;
    c->ws = (char *)d_workspace;
    c->L = L;
    c->b64 = carve_blocks(c->ws + L.blocks64, c->N, m, DT_F64);
    c->hasB = B != nullptr;
    if (B) {
        c->Bop = *B;
        const size_t bs = (size_t)c->N * m * 8;
        char *bb = c->ws + L.blocksB;
        c->b64.BX[0] = bb, c->b64.BX[1] = bb + bs, c->b64.BW = bb + 2 * bs, c->b64.BP = bb + 3 * bs;
        c->b64.BPJ = bb + 4 * bs;
    }
    if (precision == LOBPCG_MIXED) c->b32 = carve_blocks(c->ws + L.blocks32, c->N, m, DT_F32);
    else memset(&c->b32, 0, sizeof(c->b32));
    if (B && precision == LOBPCG_MIXED) {
        const size_t bs = (size_t)c->N * m * 4;
        char *bb = c->ws + L.blocksB32;
        c->b32.BX[0] = bb, c->b32.BX[1] = bb + bs, c->b32.BW = bb + 2 * bs, c->b32.BP = bb + 3 * bs;
        c->b32.BPJ = bb + 4 * bs;
    }
    c->mgx.assign(L.levels.size(), nullptr);
    c->mgb.assign(L.levels.size(), nullptr);
    c->mgt.assign(L.levels.size(), nullptr);
    for (size_t l = 1; l < L.levels.size(); l++) {
        c->mgx[l] = c->ws + L.mg[3 * (l - 1)];
        c->mgb[l] = c->ws + L.mg[3 * (l - 1) + 1];
        c->mgt[l] = c->ws + L.mg[3 * (l - 1) + 2];
    }
    c->d_lambda = (double *)(c->ws + L.lambda);
    c->d_jpos = (int *)(c->ws + L.jpos);
    c->d_cols = (int *)(c->ws + L.cols);
    c->d_coef = c->ws + L.coef;
    c->d_gram_out = (double *)(c->ws + L.gram_out);
    c->d_gram_part = (double *)(c->ws + L.gram_part);
    c->d_res_part = (double *)(c->ws + L.res_part);
    c->d_mv_part = (double *)(c->ws + L.mv_part);
    c->d_res_out = (double *)(c->ws + L.res_out);
    c->d_w = (double *)(c->ws + L.wvec);
    // pinned host staging
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = align_up(off);
        off = o + b;
        return o;
    };
    c->h_coef_off = take((size_t)COEF_SLOTS * coef_slot_entries(m) * 8);
    c->h_cols_off = take((size_t)COEF_SLOTS * m * sizeof(int));
    c->h_gram_off = take((size_t)GX_MAX_TILES * 256 * 8);
    c->h_res_off = take((size_t)2 * m * 8);
    c->h_small_off = take((size_t)m * 8 + (size_t)m * sizeof(int));
    c->h_pin_bytes = align_up(off);
    if (hipHostMalloc((void **)&c->h_pin, c->h_pin_bytes, hipHostMallocDefault) != hipSuccess) {
        delete c;
        return LOBPCG_ERR_HIP;
    }
    c->coef_slot = 0;
    c->switch_tol = 3e-7;
    c->stall_window = 10;
    c->stall_factor = 0.95;
    c->profile = false;
    c->reactivate = true;
    c->lock_gap = 0.0;
    c->nwant = 0;
    c->mv_frag = 0;
    c->mg_unpadded = 0;
    c->gram_staged = 0;
    c->gram_nt4 = 0;
    c->gram_nt32 = 2;
    c->gram_direct = 0;
    c->mv_fragst = 0;
    c->fp32_explicit = true;
    c->fp32_explicit_above = -1;
    c->fp64_explicit = false;
    c->fold = true;
    c->Y = nullptr;
    c->ny = 0;
    memset(&c->stats, 0, sizeof(c->stats));
    c->ev_used = 0;
    *out = c;
    return LOBPCG_OK;
}

void lobpcg_destroy(lobpcg_ctx *c)
{
    if (!c) return;
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    if (c->h_pin) (void)hipHostFree(c->h_pin);
    delete c;
}

int lobpcg_set_option(lobpcg_ctx *c, int key, double v)
{
    if (!c) return LOBPCG_ERR_ARG;
    switch (key) {
    case LOBPCG_OPT_SWITCH_TOL:
        if (!(v > 0)) return LOBPCG_ERR_ARG;
        c->switch_tol = v;
        return LOBPCG_OK;
    case LOBPCG_OPT_STALL_WINDOW:
        if (v < 1) return LOBPCG_ERR_ARG;
        c->stall_window = (int)v;
        return LOBPCG_OK;
    case LOBPCG_OPT_STALL_FACTOR:
        if (!(v > 0 && v <= 1)) return LOBPCG_ERR_ARG;
        c->stall_factor = v;
        return LOBPCG_OK;
    case LOBPCG_OPT_PROFILE:
        c->profile = v != 0;
        if (c->profile && c->ev_pool.empty()) {
            c->ev_pool.resize(512);
            c->ev_step.assign(256, 0);
            for (auto &e : c->ev_pool)
                if (hipEventCreate(&e) != hipSuccess) return LOBPCG_ERR_HIP;
        }
        return LOBPCG_OK;
    case LOBPCG_OPT_REACTIVATE: c->reactivate = v != 0; return LOBPCG_OK;
    case LOBPCG_OPT_NWANT:
        if (!(v >= 0.0 && v <= c->m) || v != std::floor(v)) return LOBPCG_ERR_ARG;
        c->nwant = (int)v;
        return LOBPCG_OK;
    case LOBPCG_OPT_LOCK_GAP:
        if (!(v >= 0.0 && v < 1.0)) return LOBPCG_ERR_ARG;
        c->lock_gap = v;
        return LOBPCG_OK;
    case LOBPCG_OPT_FP32_EXPLICIT_GRAM: c->fp32_explicit = v != 0; return LOBPCG_OK;
    case LOBPCG_OPT_FP32_EXPLICIT_ABOVE:
        if (!(v >= 0.0 && v <= c->m) || v != std::floor(v)) return LOBPCG_ERR_ARG;
        c->fp32_explicit_above = (int)v;
        return LOBPCG_OK;
    case LOBPCG_OPT_FOLD_CHOLQR: c->fold = v != 0; return LOBPCG_OK;
    case LOBPCG_OPT_FP64_EXPLICIT_GRAM: c->fp64_explicit = v != 0; return LOBPCG_OK;
    case LOBPCG_OPT_KERNELS:
        if (v < 0 || v > 127) return LOBPCG_ERR_ARG;
        c->mv_frag = ((int)v & 1) != 0;
        c->mg_unpadded = ((int)v & 2) != 0;
        c->gram_staged = ((int)v & 4) != 0;
        c->gram_nt4 = ((int)v & 8) != 0;
        c->gram_nt32 = ((int)v & 16) ? 4 : 2;
        c->gram_direct = ((int)v & 32) != 0;
        c->mv_fragst = ((int)v & 64) != 0;
        return LOBPCG_OK;
    default: return LOBPCG_ERR_ARG;
    }
}

int lobpcg_get_stats(const lobpcg_ctx *c, lobpcg_stats *st)
{
    if (!c || !st) return LOBPCG_ERR_ARG;
    *st = c->stats;
    return LOBPCG_OK;
}

static int same_op(const lobpcg_ctx *c, const lobpcg_op *A)
{
    return op_ok(A) && A->nx == c->g.nx && A->ny == c->g.ny && A->nz == c->g.nz && A->kind == c->A.kind;
}

static int same_precond(const lobpcg_ctx *c, const lobpcg_precond *T)
{
    if (!c->mg) return !T || T->kind == LOBPCG_PC_NONE;
    return T && T->kind == c->T.kind && T->levels == c->T.levels && T->nu_pre == c->T.nu_pre &&
           T->nu_post == c->T.nu_post && T->coarse_sweeps == c->T.coarse_sweeps && T->omega == c->T.omega;
}

static int solve_impl(lobpcg_ctx *c, const lobpcg_op *A, const lobpcg_op *B, const lobpcg_precond *T,
                      const double *d_Y, int ny, const double *d_X0, int m, double tol, int maxit, double *h_lambda,
                      double *d_X, double *h_hist, int *h_iters, double *h_final_resid)
{
    if (!c) return LOBPCG_ERR_ARG;
    if (!same_op(c, A) || !same_precond(c, T) || m != c->m || !d_X0 || !d_X || !h_lambda || !h_iters ||
        !(tol > 0) || maxit < 0)
        return LOBPCG_ERR_ARG;
    if ((B != nullptr) != c->hasB) return LOBPCG_ERR_ARG;
    if (B) {
        if (B->kind != c->Bop.kind || !b_ok(&c->A, B)) return LOBPCG_ERR_ARG;
        c->Bop = *B;
    }
    if (ny < 0 || ny > LOBPCG_MAX_M || (ny > 0 && !d_Y) || 3LL * m + ny > c->N) return LOBPCG_ERR_ARG;
    auto t0 = std::chrono::steady_clock::now();
    memset(&c->stats, 0, sizeof(c->stats));
    c->ev_used = 0;
    c->coef_slot = 0;
    *h_iters = 0;
    c->Y = ny ? d_Y : nullptr;
    c->ny = ny;
    if (ny) {
        // the Cholesky factor of Y^T B Y (Y must have full column rank)
        std::vector<double> G;
        if (c->hasB) {
            // B Y in pieces of at most m columns: the piece of Y copied into
            // the FP64 block W (free before the iterations), B applied into
            // T0, then Y^T (B Y_piece)
            G.assign((size_t)ny * ny, 0.0);
            for (int j0 = 0; j0 < ny; j0 += m) {
                const int kc = std::min(m, ny - j0);
                std::vector<double> E((size_t)ny * kc, 0.0);
                for (int j = 0; j < kc; j++) E[(size_t)(j0 + j) * kc + j] = 1.0;
                MV q;
                q.input(0, d_Y, nullptr, ny, ny);
                q.kout = kc;
                q.out[0] = c->b64.W;
                int s0 = mv(c, DT_F64, q, E.data(), LOBPCG_STEP_OTHER);
                if (s0) return s0;
                s0 = apply_B(c, DT_F64, c->b64.W, c->b64.T0, kc, LOBPCG_STEP_OTHER);
                if (s0) return s0;
                std::vector<double> Gp;
                s0 = gram_Yt(c, c->b64.T0, kc, Gp, LOBPCG_STEP_OTHER);
                if (s0) return s0;
                for (int i = 0; i < ny; i++)
                    for (int j = 0; j < kc; j++) G[(size_t)i * ny + j0 + j] = Gp[(size_t)i * kc + j];
            }
        } else {
            const void *Sb[1] = {d_Y};
            int w1[1] = {ny};
            int s0 = gram(c, DT_F64, 1, Sb, nullptr, w1, G, nullptr, LOBPCG_STEP_OTHER);
            if (s0) return s0;
            if (!all_finite(G)) return LOBPCG_ERR_NONFINITE;
        }
        c->RY.assign((size_t)ny * ny, 0.0);
        if (!chol_scaled(ny, G.data(), c->RY.data())) return LOBPCG_ERR_ARG;
    }
    const double normA = op_norm(c, A);
    if (!(normA > 0)) return LOBPCG_ERR_HIP;
    const size_t nm = (size_t)c->N * m;
    int iters = 0, s = LOBPCG_OK, outcome = PH_MAXIT;
    PhaseState ps;
    ps.cur = 0;
    ps.have_res = false;
    if (c->precision == LOBPCG_MIXED) {
        // FP32 phase (step 2 in FP64 first)
        const void *x0 = d_X0;
        if (ny) {
            s = constrain(c, DT_F64, d_X0, m, c->b64.X[0], LOBPCG_STEP_OTHER);
            if (s) return s;
            x0 = c->b64.X[0];
        }
        prof_begin(c, LOBPCG_STEP_OTHER);
        if (launch_cast(DT_F64, DT_F32, nm, x0, c->b32.X[0], c->st) != hipSuccess) return LOBPCG_ERR_HIP;
        prof_end(c);
        add_bytes(c, LOBPCG_STEP_OTHER, 12.0 * nm);
        s = init_phase(c, A, DT_F32, c->b32, ps, true, true);
        if (s == LOBPCG_OK) {
            s = run_phase(c, A, DT_F32, c->b32, ps, std::max(tol, c->switch_tol), normA, maxit, iters, h_hist,
                          c->fp32_explicit, true, outcome);
        }
        if (s == LOBPCG_OK) {
            // FP64 phase: up-cast X and the directions P, form A X and A P
            // explicitly in FP64, Rayleigh-Ritz on span(X); P is kept
            prof_begin(c, LOBPCG_STEP_OTHER);
            if (launch_cast(DT_F32, DT_F64, nm, c->b32.X[ps.cur], c->b64.X[0], c->st) != hipSuccess)
                return LOBPCG_ERR_HIP;
            const int np = (int)ps.Pcols.size();
            if (np && launch_cast(DT_F32, DT_F64, (size_t)c->N * np, c->b32.P, c->b64.P, c->st) != hipSuccess)
                return LOBPCG_ERR_HIP;
            prof_end(c);
            add_bytes(c, LOBPCG_STEP_OTHER, 12.0 * (nm + (double)c->N * np));
            ps.cur = 0;
            if (ny) {
                // FP32 rounding leaves components along span(Y) in X and P:
                // step 2 again, in FP64, on both; X is orthonormalised again
                s = constrain(c, DT_F64, c->b64.X[0], m, c->b64.X[1], LOBPCG_STEP_OTHER);
                if (s) return s;
                ps.cur = 1;
                if (np) {
                    s = constrain(c, DT_F64, c->b64.P, np, c->b64.PJ, LOBPCG_STEP_OTHER);
                    if (s) return s;
                    std::swap(c->b64.P, c->b64.PJ);
                }
            }
            if (np) {
                s = apply_A(c, A, DT_F64, c->b64.P, c->b64.AP, np);
                if (s) return s;
                if (c->hasB) {
                    s = apply_B(c, DT_F64, c->b64.P, c->b64.BP, np, LOBPCG_STEP_OTHER);
                    if (s) return s;
                }
            }
            s = init_phase(c, A, DT_F64, c->b64, ps, ny > 0, true);
            if (s == LOBPCG_OK)
                s = run_phase(c, A, DT_F64, c->b64, ps, tol, normA, maxit, iters, h_hist, c->fp64_explicit, false,
                              outcome);
        }
    } else {
        if (ny) {
            // step 2: X0 - Y (Y^T Y)^-1 (Y^T X0)
            s = constrain(c, DT_F64, d_X0, m, c->b64.X[0], LOBPCG_STEP_OTHER);
            if (s) return s;
        } else {
            HIPCHK(hipMemcpyAsync(c->b64.X[0], d_X0, nm * 8, hipMemcpyDeviceToDevice, c->st));
        }
        s = init_phase(c, A, DT_F64, c->b64, ps, true, false);
        if (s == LOBPCG_OK)
            s = run_phase(c, A, DT_F64, c->b64, ps, tol, normA, maxit, iters, h_hist, c->fp64_explicit, false,
                          outcome);
    }
    *h_iters = iters;
    c->stats.iters_total = iters;
    if (s != LOBPCG_OK) {
        c->stats.status = s;
        return s;
    }
    // outputs: X, Lambda, explicit residuals with a fresh A X
    HIPCHK(hipMemcpyAsync(d_X, c->b64.X[ps.cur], nm * 8, hipMemcpyDeviceToDevice, c->st));
    for (int j = 0; j < m; j++) h_lambda[j] = ps.lam[j];
    if (h_final_resid) {
        s = apply_A(c, A, DT_F64, c->b64.X[ps.cur], c->b64.AW, m);
        if (s) return s;
        const void *BXf = c->b64.X[ps.cur];
        if (c->hasB) {
            s = apply_B(c, DT_F64, c->b64.X[ps.cur], c->b64.BW, m, LOBPCG_STEP_OTHER);
            if (s) return s;
            BXf = c->b64.BW;
        }
        std::vector<double> rr, xx;
        std::vector<int> none;
        s = residual(c, DT_F64, BXf, c->b64.AW, ps.lam, none, nullptr, rr, xx);
        if (s) return s;
        for (int j = 0; j < m; j++) h_final_resid[j] = std::sqrt(rr[j]) / (normA * std::sqrt(xx[j]));
    }
    s = sync(c);
    if (s) return s;
    c->stats.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    c->stats.status = outcome == PH_CONVERGED ? LOBPCG_OK : LOBPCG_NOT_CONVERGED;
    return c->stats.status;
}

int lobpcg_solve(lobpcg_ctx *c, const lobpcg_op *A, const lobpcg_op *B, const lobpcg_precond *T, const double *d_X0,
                 int m, double tol, int maxit, double *h_lambda, double *d_X, double *h_hist, int *h_iters,
                 double *h_final_resid)
{
    return solve_impl(c, A, B, T, nullptr, 0, d_X0, m, tol, maxit, h_lambda, d_X, h_hist, h_iters, h_final_resid);
}

int lobpcg_solve_constrained(lobpcg_ctx *c, const lobpcg_op *A, const lobpcg_op *B, const lobpcg_precond *T,
                             const double *d_Y, int ny, const double *d_X0, int m, double tol, int maxit,
                             double *h_lambda, double *d_X, double *h_hist, int *h_iters, double *h_final_resid)
{
    if (ny < 1 || !d_Y) return LOBPCG_ERR_ARG;
    return solve_impl(c, A, B, T, d_Y, ny, d_X0, m, tol, maxit, h_lambda, d_X, h_hist, h_iters, h_final_resid);
}

int lobpcg_eig_grad_k(lobpcg_ctx *c, const double *d_X, const double *h_gbar, int m, double *gkx, double *gky,
                      double *gkz)
{
    if (!c || !d_X || !h_gbar || !gkx || !gky || !gkz || m < 1 || m > c->m) return LOBPCG_ERR_ARG;
    // column norms (x_i, x_i) through the residual kernel with AX = X and
    // lambda = 0, or (x_i, B x_i) from the Gram kernel with B X in the spare
    // B-block; both work on blocks of the context's width, so a narrower X
    // is first copied into zero-padded scratch
    std::vector<double> zero(c->m, 0.0), rr, xx;
    std::vector<int> none;
    const void *Xs = d_X;
    if (m != c->m) {
        void *t = c->b64.T0;
        HIPCHK(hipMemsetAsync(t, 0, (size_t)c->N * c->m * 8, c->st));
        HIPCHK(hipMemcpy2DAsync(t, (size_t)c->m * 8, d_X, (size_t)m * 8, (size_t)m * 8, (size_t)c->N,
                                hipMemcpyDeviceToDevice, c->st));
        Xs = t;
    }
    int s;
    if (c->hasB) {
        s = apply_B(c, DT_F64, Xs, c->b64.BPJ, c->m, LOBPCG_STEP_OTHER);
        if (s) return s;
        std::vector<double> G;
        const void *Sb[1] = {Xs}, *BSb[1] = {c->b64.BPJ};
        int w1[1] = {c->m};
        s = gram(c, DT_F64, 1, Sb, nullptr, w1, G, nullptr, LOBPCG_STEP_OTHER, false, nullptr, nullptr, false, BSb);
        if (s) return s;
        xx.assign(c->m, 0.0);
        for (int i = 0; i < c->m; i++) xx[i] = G[(size_t)i * c->m + i];
    } else {
        s = residual(c, DT_F64, Xs, Xs, zero, none, nullptr, rr, xx);
        if (s) return s;
    }
    std::vector<double> w(c->m, 0.0);
    for (int i = 0; i < m; i++) {
        if (!(xx[i] > 0)) return LOBPCG_ERR_ARG;
        w[i] = h_gbar[i] / xx[i];
    }
    double *hs = (double *)(c->h_pin + c->h_small_off);
    std::copy(w.begin(), w.end(), hs);
    HIPCHK(hipMemcpyAsync(c->d_w, hs, c->m * 8, hipMemcpyHostToDevice, c->st));
    if (launch_eig_grad(c->g, c->m, (const double *)Xs, c->d_w, gkx, gky, gkz, c->st) != hipSuccess)
        return LOBPCG_ERR_HIP;
    return sync(c);
}

// ---------------------------------------------------------------- the steps one by one

static int dtype_ok(const lobpcg_ctx *c, int dt)
{
    return dt == LOBPCG_F64 || (dt == LOBPCG_F32 && c->precision == LOBPCG_MIXED);
}

int lobpcg_apply_A(lobpcg_ctx *c, const lobpcg_op *A, int dt, const void *in, void *out, int k)
{
    if (!c || !same_op(c, A) || !dtype_ok(c, dt) || !in || !out || k < 1 || k > 3 * c->m) return LOBPCG_ERR_ARG;
    int s = apply_A(c, A, dt == LOBPCG_F32 ? DT_F32 : DT_F64, in, out, k);
    if (s) return s;
    return sync(c);
}

int lobpcg_apply_T(lobpcg_ctx *c, int dt, const void *in, void *out, int k)
{
    if (!c || !dtype_ok(c, dt) || !in || !out || k < 1 || k > c->m) return LOBPCG_ERR_ARG;
    const int d = dt == LOBPCG_F32 ? DT_F32 : DT_F64;
    const size_t bytes = (size_t)c->N * k * esize(d);
    if (!c->mg) {
        HIPCHK(hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, c->st));
        return sync(c);
    }
    Blocks &B = d == DT_F32 ? c->b32 : c->b64;
    void *r = nullptr;
    int s = apply_T(c, d, in, B.AW, B.T0, k, &r, B.X[1]);
    if (s) return s;
    HIPCHK(hipMemcpyAsync(out, r, bytes, hipMemcpyDeviceToDevice, c->st));
    return sync(c);
}

int lobpcg_gram(lobpcg_ctx *c, int dt, int n, const void *const *S, const void *const *AS, const int *w,
                int paper_form, double *h_SS, double *h_SAS)
{
    if (!c || !dtype_ok(c, dt) || n < 1 || n > 3 || !S || !w || !h_SS) return LOBPCG_ERR_ARG;
    if (paper_form != 0 && (paper_form != 1 || !AS || n < 2)) return LOBPCG_ERR_ARG;
    int K = 0;
    for (int i = 0; i < n; i++) {
        if (!S[i] || w[i] < 1 || (AS && !AS[i])) return LOBPCG_ERR_ARG;
        K += w[i];
    }
    if (K > 3 * c->m || (AS && !h_SAS)) return LOBPCG_ERR_ARG;
    std::vector<double> SS, SAS;
    int s = gram(c, dt == LOBPCG_F32 ? DT_F32 : DT_F64, n, S, AS, w, SS, AS ? &SAS : nullptr, LOBPCG_STEP_GRAM,
                 paper_form == 1);
    if (s) return s;
    std::copy(SS.begin(), SS.end(), h_SS);
    if (AS) std::copy(SAS.begin(), SAS.end(), h_SAS);
    return LOBPCG_OK;
}

int lobpcg_combine(lobpcg_ctx *c, int dt, int n, const void *const *in, const int *ld, const int *const *cols,
                   const int *k, const double *h_C, int kout, const void *d_add, void *d_out)
{
    if (!c || !dtype_ok(c, dt) || n < 1 || n > 3 || !in || !ld || !k || !h_C || !d_out || kout < 1 || kout > c->m)
        return LOBPCG_ERR_ARG;
    int ks = 0;
    MV q;
    for (int i = 0; i < n; i++) {
        if (!in[i] || ld[i] < 1 || ld[i] > LOBPCG_MAX_M || k[i] < 1 || in[i] == d_out) return LOBPCG_ERR_ARG;
        const int *dcol = nullptr;
        if (cols && cols[i]) {
            std::vector<int> cv(cols[i], cols[i] + k[i]);
            for (int x : cv)
                if (x < 0 || x >= ld[i]) return LOBPCG_ERR_ARG;
            if ((int)cv.size() > c->m) return LOBPCG_ERR_ARG;
            int s = upload_cols(c, cv, &dcol);
            if (s) return s;
        } else if (k[i] != ld[i]) {
            return LOBPCG_ERR_ARG;
        }
        q.input(i, in[i], nullptr, ld[i], k[i], dcol);
        ks += k[i];
    }
    if (ks > 3 * c->m) return LOBPCG_ERR_ARG;
    q.kout = kout;
    q.add = d_add;
    q.out[0] = d_out;
    int s = mv(c, dt == LOBPCG_F32 ? DT_F32 : DT_F64, q, h_C, LOBPCG_STEP_UPDATE);
    if (s) return s;
    return sync(c);
}

int lobpcg_update(lobpcg_ctx *c, int dt, const void *d_X, const void *d_AX, const void *d_W, const void *d_AW,
                  int nW, const void *d_P, const void *d_AP, int ldP, const int *h_Pcols, int nP, const double *h_C,
                  const double *h_theta, const int *h_J, int nJ, double norm_A, void *d_Xn, void *d_AXn,
                  void *d_Pn, void *d_APn, void *d_Wn, double *h_rho)
{
    if (!c || !dtype_ok(c, dt)) return LOBPCG_ERR_ARG;
    const int m = c->m;
    if (!d_X || !d_AX || !d_W || !d_AW || nW < 1 || nW > m || nP < 0 || nP > m || (nP && (!d_P || !d_AP)) ||
        !h_C || !h_theta || !h_J || nJ < 1 || nJ > m || !(norm_A > 0) || !d_Xn || !d_AXn || !d_Pn || !d_APn ||
        !d_Wn || !h_rho)
        return LOBPCG_ERR_ARG;
    if (nP && (h_Pcols ? ldP < 1 || ldP > m : ldP != nP)) return LOBPCG_ERR_ARG;
    const void *ins[6] = {d_X, d_AX, d_W, d_AW, d_P, d_AP};
    const void *outs[5] = {d_Xn, d_AXn, d_Pn, d_APn, d_Wn};
    for (const void *o : outs)
        for (const void *i : ins)
            if (o && o == i) return LOBPCG_ERR_ARG;
    std::vector<int> jpos(m, -1);
    for (int i = 0; i < nJ; i++) {
        const int j = h_J[i];
        if (j < 0 || j >= m || jpos[j] >= 0) return LOBPCG_ERR_ARG;
        jpos[j] = i;
    }
    const int *djpos, *dpcols = nullptr;
    const double *dtheta;
    int s = upload_cols(c, jpos, &djpos);
    if (s) return s;
    if (nP && h_Pcols) {
        std::vector<int> pc(h_Pcols, h_Pcols + nP);
        for (int x : pc)
            if (x < 0 || x >= ldP) return LOBPCG_ERR_ARG;
        s = upload_cols(c, pc, &dpcols);
        if (s) return s;
    }
    s = upload_doubles(c, std::vector<double>(h_theta, h_theta + m), &dtheta);
    if (s) return s;
    MV q;
    q.nside = 2;
    q.input(0, d_X, d_AX, m, m);
    q.input(1, d_W, d_AW, nW, nW);
    if (nP) q.input(2, d_P, d_AP, nP && h_Pcols ? ldP : nP, nP, dpcols);
    q.kout = m;
    q.out[0] = d_Pn;
    q.out[1] = d_APn;
    q.opos = djpos;
    q.nout = nJ;
    q.out2[0] = d_Xn;
    q.out2[1] = d_AXn;
    q.resid = true;
    q.theta = dtheta;
    q.wpos = djpos;
    q.Wout = d_Wn;
    q.nW = nJ;
    s = mv(c, dt == LOBPCG_F32 ? DT_F32 : DT_F64, q, h_C, LOBPCG_STEP_UPDATE);
    if (s) return s;
    double *h = (double *)(c->h_pin + c->h_res_off);
    HIPCHK(hipMemcpyAsync(h, c->d_res_out, 2 * m * 8, hipMemcpyDeviceToHost, c->st));
    s = sync(c);
    if (s) return s;
    for (int j = 0; j < m; j++) h_rho[j] = std::sqrt(h[j]) / (norm_A * std::sqrt(h[m + j]));
    return LOBPCG_OK;
}

int lobpcg_residual(lobpcg_ctx *c, int dt, const void *X, const void *AX, int m, const double *h_lambda,
                    const int *h_J, int nJ, double norm_A, void *d_W, double *h_rho)
{
    if (!c || !dtype_ok(c, dt) || !X || !AX || m != c->m || !h_lambda || nJ < 0 || nJ > m || (nJ > 0 && !h_J) ||
        !(norm_A > 0) || !h_rho || (nJ > 0 && !d_W))
        return LOBPCG_ERR_ARG;
    std::vector<double> lam(h_lambda, h_lambda + m), rr, xx;
    std::vector<int> J(h_J, h_J + nJ);
    std::vector<int> seen(m, 0);
    for (int j : J) {
        if (j < 0 || j >= m || seen[j]) return LOBPCG_ERR_ARG;
        seen[j] = 1;
    }
    int s = residual(c, dt == LOBPCG_F32 ? DT_F32 : DT_F64, X, AX, lam, J, nJ ? d_W : nullptr, rr, xx);
    if (s) return s;
    for (int j = 0; j < m; j++) h_rho[j] = std::sqrt(rr[j]) / (norm_A * std::sqrt(xx[j]));
    return LOBPCG_OK;
}

int lobpcg_dense_chol(int n, const double *G, double *R)
{
    if (n < 1 || !G || !R) return LOBPCG_ERR_ARG;
    return chol_scaled(n, G, R) ? LOBPCG_OK : LOBPCG_ERR_CHOL;
}

int lobpcg_dense_rr(int n, int m, const double *gramA, const double *gramB, double *theta, double *C)
{
    if (n < 1 || m < 1 || m > n || !gramA || !gramB || !theta || !C) return LOBPCG_ERR_ARG;
    return rayleigh_ritz(n, m, gramA, gramB, theta, C) ? LOBPCG_OK : LOBPCG_ERR_RR;
}

}  // extern "C"
