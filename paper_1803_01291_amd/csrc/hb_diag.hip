// Diagnostics of one solve (FP64, deterministic): the integral of phi, the
// norms, max |Lap_h phi| (for the paper's P(t) = c max |Lap_h phi|, section 3),
// the discrete energy, and counts of non-finite and negative values.
#include <hip/hip_runtime.h>

#include "hb_internal.h"

namespace hb {
namespace {

// ---- diagnostics (FP64, deterministic) ----------------------------------------

constexpr int DIAG_THREADS = 256;

template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <bool COMP>
__device__ __forceinline__ double fld(const void* hi, const float* lo, long long o) {
    if constexpr (COMP) return (double)((gptr<const float>)hi)[o] + (double)((gptr<const float>)lo)[o];
    return ((gptr<const double>)hi)[o];
}

// One block per (y, z) row group; per-thread partial sums in a fixed order,
// then a fixed LDS tree.  Partials: DIAG_COUNT doubles per block.
template <bool COMP>
__global__ void __launch_bounds__(DIAG_THREADS)
diag_kernel(const SolveDesc* __restrict__ d, int par, double c, double* __restrict__ partials) {
    const int nx = d->nx, ny = d->ny, nz = d->nz;
    const long long sy = d->sy, sz = d->sz, cs = d->cs;  // cs elements per cell
    const void* P = d->y_phi[par];
    const void* S = d->y_psi[par];
    // FP32c low parts: in the whole-step state slot (phi hi, psi hi, phi lo,
    // psi lo) two elements after the high parts, else their own fields
    const float* LP = d->cs == 4 ? (const float*)P + 2 : d->lo_phi;
    const float* LS = d->cs == 4 ? (const float*)S + 2 : d->lo_psi;
    const double w0 = d->w0, mu2 = d->mu2, lam = d->lambda;
    // element offset of cell (x, y, z); periodic solves wrap it into the
    // interior, zero-halo solves read the halo
    const bool per = d->periodic != 0;
    auto off = [&](int x, int y, int z) -> long long {
        if (per) {
            x = ((x % nx) + nx) % nx;
            y = ((y % ny) + ny) % ny;
            z = ((z % nz) + nz) % nz;
        }
        return ((long long)z * sz + (long long)y * sy + x) * cs;
    };
    double acc[DIAG_COUNT];
    for (int k = 0; k < DIAG_COUNT; ++k) acc[k] = 0.0;
    const long long rows = (long long)ny * nz;
    for (long long row = blockIdx.x; row < rows; row += gridDim.x) {
        const int y = (int)(row % ny), z = (int)(row / ny);
        for (int x = threadIdx.x; x < nx; x += blockDim.x) {
            const long long o = off(x, y, z);
            const double p = fld<COMP>(P, LP, o);
            const double s = fld<COMP>(S, LS, o);
            double lap = w0 * p;
            for (int a = 0; a < 3; ++a) {
                const int ex = a == 0, ey = a == 1, ez = a == 2;
                lap += d->w1[a] * (fld<COMP>(P, LP, off(x - ex, y - ey, z - ez)) +
                                   fld<COMP>(P, LP, off(x + ex, y + ey, z + ez)));
                lap += d->w2[a] * (fld<COMP>(P, LP, off(x - 2 * ex, y - 2 * ey, z - 2 * ez)) +
                                   fld<COMP>(P, LP, off(x + 2 * ex, y + 2 * ey, z + 2 * ez)));
            }
            acc[DIAG_SUM_PHI] += p;
            acc[DIAG_SUM_PHI2] += p * p;
            acc[DIAG_SUM_PSI2] += s * s;
            acc[DIAG_MAX_PHI] = fmax(acc[DIAG_MAX_PHI], fabs(p));
            acc[DIAG_MAX_PSI] = fmax(acc[DIAG_MAX_PSI], fabs(s));
            acc[DIAG_MAX_LAP] = fmax(acc[DIAG_MAX_LAP], fabs(lap));
            acc[DIAG_ENERGY] += 0.5 * s * s + 0.5 * c * p * (-lap) - 0.5 * mu2 * p * p +
                                0.25 * lam * p * p * p * p;
            acc[DIAG_NONFINITE] += (isfinite(p) ? 0.0 : 1.0) + (isfinite(s) ? 0.0 : 1.0);
            acc[DIAG_NEGATIVE] += (p < 0.0) ? 1.0 : 0.0;
        }
    }
    __shared__ double red[DIAG_THREADS];
    for (int k = 0; k < DIAG_COUNT; ++k) {
        red[threadIdx.x] = acc[k];
        __syncthreads();
        for (int w = DIAG_THREADS / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                const double a = red[threadIdx.x], b = red[threadIdx.x + w];
                const bool is_max = (k == DIAG_MAX_PHI || k == DIAG_MAX_PSI || k == DIAG_MAX_LAP);
                red[threadIdx.x] = is_max ? fmax(a, b) : a + b;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) partials[(long long)blockIdx.x * DIAG_COUNT + k] = red[0];
        __syncthreads();
    }
}

// Final pass over the per-block partials, in an order fixed by nparts alone:
// thread t folds partials t, t + 256, t + 512, ... in increasing order, then
// a fixed LDS tree folds the 256 thread results.
__global__ void __launch_bounds__(DIAG_THREADS)
diag_final_kernel(const double* __restrict__ partials, int nparts, double* __restrict__ out) {
    __shared__ double red[DIAG_THREADS];
    for (int k = 0; k < DIAG_COUNT; ++k) {
        const bool is_max = (k == DIAG_MAX_PHI || k == DIAG_MAX_PSI || k == DIAG_MAX_LAP);
        double a = 0.0;
        for (int b = threadIdx.x; b < nparts; b += DIAG_THREADS) {
            const double v = partials[(long long)b * DIAG_COUNT + k];
            a = is_max ? fmax(a, v) : a + v;
        }
        red[threadIdx.x] = a;
        __syncthreads();
        for (int w = DIAG_THREADS / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                const double x = red[threadIdx.x], y = red[threadIdx.x + w];
                red[threadIdx.x] = is_max ? fmax(x, y) : x + y;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) out[k] = red[0];
        __syncthreads();
    }
}

}  // namespace

int diag_partials_needed(int nx, int ny, int nz) {
    const long long rows = (long long)ny * nz;
    return (int)(rows < 4096 ? rows : 4096);
}

int launch_diagnostics(int prec, const SolveDesc* desc, int parity, double c, double* partials,
                       int nparts, double* out, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    if (prec == PREC_F32C)
        hipLaunchKernelGGL((diag_kernel<true>), dim3(nparts), dim3(DIAG_THREADS), 0, s, desc, parity,
                           c, partials);
    else
        hipLaunchKernelGGL((diag_kernel<false>), dim3(nparts), dim3(DIAG_THREADS), 0, s, desc, parity,
                           c, partials);
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(DIAG_THREADS), 0, s, partials, nparts, out);
    return (int)hipGetLastError();
}

}  // namespace hb
