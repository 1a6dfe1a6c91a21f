// Global flux balancing of the equilibrium-velocity boundary field on the
// device (Sec. 2.2 and 2.3): the net outward volume flux over the boundary
// cells, then the same normal-velocity shift for every cell, the
// least-squares smallest correction that zeroes the flux.
//
// Two launches, no host round trip: a fixed grid of FLUX_BLOCKS blocks writes
// one partial sum each (grid-stride over the cells, wavefront reductions);
// every block
// of the shift kernel sums the partials in the same fixed order, so all of
// them see the same Phi, and shifts its cells.  Deterministic run to run.
#include "lbm_launch.h"

namespace lbm {

namespace {

constexpr int FLUX_BLOCKS = 256;
constexpr int FLUX_THREADS = 256;

// outward normal of face F: axis F/2, sign - for the low face, + for the high
__device__ inline double flux_of(const double* __restrict__ uin, int slot, int F)
{
    const double v = uin[3 * (long long)slot + (F >> 1)];
    return (F & 1) ? v : -v;
}


__global__ void __launch_bounds__(FLUX_THREADS)
k_flux_partial(const int* __restrict__ slot, const int* __restrict__ face, long long n,
               const double* __restrict__ uin, double* __restrict__ partial)
{
    __shared__ double red[FLUX_THREADS / 64 + 1];
    double acc = 0.0;
    for (long long i = blockIdx.x * (long long)FLUX_THREADS + threadIdx.x; i < n;
         i += (long long)FLUX_THREADS * FLUX_BLOCKS)
        acc += flux_of(uin, slot[i], face[i]);
    const double s = block_sum_waves<FLUX_THREADS>(acc, red);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(FLUX_THREADS)
k_flux_shift(const int* __restrict__ slot, const int* __restrict__ face, long long n, double* __restrict__ uin,
             const double* __restrict__ partial, double* __restrict__ phi_out, int apply)
{
    __shared__ double red[FLUX_THREADS / 64 + 1];
    const double phi = block_sum_waves<FLUX_THREADS>(threadIdx.x < FLUX_BLOCKS ? partial[threadIdx.x] : 0.0, red);
    if (blockIdx.x == 0 && threadIdx.x == 0 && phi_out) phi_out[0] = phi;
    if (!apply) return;
    const double delta = phi / (double)n;
    for (long long i = blockIdx.x * (long long)FLUX_THREADS + threadIdx.x; i < n;
         i += (long long)FLUX_THREADS * FLUX_BLOCKS) {
        const int F = face[i];
        double* u = uin + 3 * (long long)slot[i] + (F >> 1);
        *u -= (F & 1) ? delta : -delta;   // U -= delta n_out
    }
}

static_assert(FLUX_BLOCKS <= FLUX_THREADS, "the shift kernel sums the partials with one block");

}  // namespace

hipError_t launch_flux_balance(const int* slot, const int* face, long long n, double* uin, double* partial,
                               double* phi_out, int apply, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flux_partial, dim3(FLUX_BLOCKS), dim3(FLUX_THREADS), 0, s, slot, face, n,
                       (const double*)uin, partial);
    hipLaunchKernelGGL(k_flux_shift, dim3(apply ? FLUX_BLOCKS : 1), dim3(FLUX_THREADS), 0, s, slot, face, n, uin,
                       (const double*)partial, phi_out, apply);
    return hipGetLastError();
}

int flux_partial_count() { return FLUX_BLOCKS; }

}  // namespace lbm
