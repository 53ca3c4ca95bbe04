// lobpcg_residual_noalloc: the residual and norms of steps 7-8 for callers
// that cannot allocate (code under HIP graph capture, tight serving loops),
// with every input, output and the kernels' scratch in device memory and no
// host synchronisation.
//
// The scratch of the residual kernels -- one row of 2m partial sums per
// workgroup and the 2m reduced sums -- lives in the file-scope array
// `scratch` below instead of a context's workspace.  Host code never passes
// the array's name to a kernel: each device's address of it is looked up
// once with hipGetSymbolAddress (with that device current) and kept.
#include "../../include/lobpcg.h"

#include <mutex>

#include "common.h"
#include "kernels.h"

namespace lobpcg {

static const int NA_MAX_M = 128;                               // widest block
static const int NA_MAX_BLOCKS = 1024;                         // residual_blocks() never exceeds this
static const size_t NA_SUMS = (size_t)NA_MAX_BLOCKS * 2 * NA_MAX_M;   // partial sums (doubles)
static const size_t NA_DOUBLES = NA_SUMS + 2 * NA_MAX_M;            // + the reduced sums

// 2 MiB + 2 KiB per device, held until the process ends
static __device__ __align__(256) double scratch[NA_DOUBLES];

static std::mutex na_mutex;
static double *na_ptr[256];

// this device's address of `scratch` (looked up on the first call on it)
static int scratch_address(double **p)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 256) return LOBPCG_ERR_HIP;
    std::lock_guard<std::mutex> lock(na_mutex);
    if (!na_ptr[dev]) {
        void *q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return LOBPCG_ERR_HIP;
        na_ptr[dev] = static_cast<double *>(q);
    }
    *p = na_ptr[dev];
    return LOBPCG_OK;
}

// rho_j = sqrt(sum r_j^2) / (norm_A sqrt(sum x_j^2))
__global__ void __launch_bounds__(128) rho_kernel(const double *__restrict__ sums, int m, double norm_A,
                                                  double *__restrict__ rho)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m) rho[j] = sqrt(sums[j]) / (norm_A * sqrt(sums[m + j]));
}

}  // namespace lobpcg

using namespace lobpcg;

extern "C" int lobpcg_residual_noalloc(int dtype, long long N, const void *d_X, const void *d_AX, int m,
                                       const double *d_lambda, const int *d_jpos, int nJ, double norm_A, void *d_W,
                                       double *d_rho, void *stream)
{
    if ((dtype != LOBPCG_F64 && dtype != LOBPCG_F32) || N < 1 || !d_X || !d_AX || !d_lambda || !d_jpos || !d_rho ||
        nJ < 0 || nJ > m || (nJ > 0 && !d_W) || !(norm_A > 0.0))
        return LOBPCG_ERR_ARG;
    // the scratch holds one row of 2m sums per workgroup for m <= 128
    if (m < 1 || m > NA_MAX_M || (size_t)residual_blocks(N, m) * 2 * m > NA_SUMS) return LOBPCG_ERR_ARG;
    double *sc = nullptr;
    int s = scratch_address(&sc);
    if (s) return s;
    hipStream_t st = (hipStream_t)stream;
    ResidualArgs a;
    a.X = d_X;
    a.AX = d_AX;
    a.lambda = d_lambda;
    a.jpos = d_jpos;
    a.W = nJ > 0 ? d_W : nullptr;
    a.m = m;
    a.nJ = nJ;
    a.N = N;
    a.partials = sc;
    a.out = sc + NA_SUMS;
    if (launch_residual(dtype == LOBPCG_F32 ? DT_F32 : DT_F64, a, st) != hipSuccess) return LOBPCG_ERR_HIP;
    hipLaunchKernelGGL(rho_kernel, dim3((m + 127) / 128), dim3(128), 0, st, a.out, m, norm_A, d_rho);
    return hipGetLastError() == hipSuccess ? LOBPCG_OK : LOBPCG_ERR_HIP;
}
