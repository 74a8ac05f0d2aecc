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

// ---- bubbles: connected sets of each sign ------------------------------------
//
// The paper's bubbles (section 1) are the maximal connected sets on which the
// solution has changed sign.  Nodes are classed as negative (phi < -eps),
// positive (phi > eps) or neither; two nodes of one class are connected
// when they are face neighbours (6-connectivity on the interior grid; with
// periodic boundaries the neighbour indices wrap).  Counted with a
// union-find over the interior nodes (linear index x + nx (y + ny z)):
// every classed node starts as its own root, each face-neighbour pair of
// one class is merged by hooking the larger root under the smaller one with
// a compare-and-swap (a parent index never exceeds its child's, so every
// chain ends at its set's smallest node), and the sets are the roots that
// remain.  The count is exact and does not depend on the order in which the
// merges land.  FP32c states are classed on hi + lo in FP64, the value
// hb_read returns.

namespace hb {
namespace {

constexpr int BUB_THREADS = 256;
constexpr unsigned BUB_NONE = 0xffffffffu;

// class of interior node (x, y, z): 1 negative, 2 positive, 0 neither
template <bool COMP>
__device__ __forceinline__ int bub_class(const SolveDesc* __restrict__ d, const void* P, const float* LP,
                                         int x, int y, int z, double eps) {
    const long long o = ((long long)z * d->sz + (long long)y * d->sy + x) * d->cs;
    const double p = fld<COMP>(P, LP, o);
    return p < -eps ? 1 : (p > eps ? 2 : 0);
}

__device__ __forceinline__ unsigned bub_load(unsigned* lab, unsigned i) {
    return __hip_atomic_load(lab + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// root of node i; shortens the chain behind it on the way (each link is
// replaced by a link to an ancestor, which keeps every set intact)
__device__ unsigned bub_find(unsigned* lab, unsigned i) {
    unsigned cur = bub_load(lab, i);
    if (cur == i) return i;
    unsigned prev = i, next;
    while (cur > (next = bub_load(lab, cur))) {
        __hip_atomic_store(lab + prev, next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        prev = cur;
        cur = next;
    }
    return cur;
}

// merge the sets of nodes a and b
__device__ void bub_union(unsigned* lab, unsigned a, unsigned b) {
    unsigned ra = bub_find(lab, a), rb = bub_find(lab, b);
    while (ra != rb) {
        if (ra > rb) {
            const unsigned t = ra;
            ra = rb;
            rb = t;
        }
        // hook root rb under ra; if rb stopped being a root meanwhile, the
        // returned parent is smaller and the walk continues from there
        const unsigned old = atomicCAS(lab + rb, rb, ra);
        if (old == rb) return;
        rb = bub_find(lab, old);
    }
}

template <bool COMP>
__global__ void __launch_bounds__(BUB_THREADS)
bub_init_kernel(const SolveDesc* __restrict__ d, int par, double eps, unsigned* __restrict__ lab) {
    const int nx = d->nx, ny = d->ny, nz = d->nz;
    const void* P = d->y_phi[par];
    const float* LP = d->cs == 4 ? (const float*)P + 2 : d->lo_phi;
    const long long total = (long long)nx * ny * nz;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int x = (int)(i % nx);
        const long long r = i / nx;
        const int y = (int)(r % ny), z = (int)(r / ny);
        lab[i] = bub_class<COMP>(d, P, LP, x, y, z, eps) ? (unsigned)i : BUB_NONE;
    }
}

// each node merges with its +x, +y and +z neighbours of the same class
template <bool COMP>
__global__ void __launch_bounds__(BUB_THREADS)
bub_union_kernel(const SolveDesc* __restrict__ d, int par, double eps, unsigned* lab) {
    const int nx = d->nx, ny = d->ny, nz = d->nz;
    const bool per = d->periodic != 0;
    const void* P = d->y_phi[par];
    const float* LP = d->cs == 4 ? (const float*)P + 2 : d->lo_phi;
    const long long total = (long long)nx * ny * nz;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        if (lab[i] == BUB_NONE) continue;  // set by the init kernel only
        const int x = (int)(i % nx);
        const long long r = i / nx;
        const int y = (int)(r % ny), z = (int)(r / ny);
        const int cls = bub_class<COMP>(d, P, LP, x, y, z, eps);
        for (int a = 0; a < 3; ++a) {
            int u = x + (a == 0), v = y + (a == 1), w = z + (a == 2);
            if (per) {
                u = u == nx ? 0 : u;
                v = v == ny ? 0 : v;
                w = w == nz ? 0 : w;
            } else if (u == nx || v == ny || w == nz) {
                continue;
            }
            if (bub_class<COMP>(d, P, LP, u, v, w, eps) != cls) continue;
            const unsigned j = (unsigned)(((long long)w * ny + v) * nx + u);
            bub_union(lab, (unsigned)i, j);
        }
    }
}

// counts[0] += roots of negative sets, counts[1] += roots of positive sets
template <bool COMP>
__global__ void __launch_bounds__(BUB_THREADS)
bub_count_kernel(const SolveDesc* __restrict__ d, int par, double eps, const unsigned* __restrict__ lab,
                 unsigned long long* __restrict__ counts) {
    const int nx = d->nx, ny = d->ny, nz = d->nz;
    const void* P = d->y_phi[par];
    const float* LP = d->cs == 4 ? (const float*)P + 2 : d->lo_phi;
    const long long total = (long long)nx * ny * nz;
    const long long stride = (long long)gridDim.x * blockDim.x;
    unsigned long long neg = 0, pos = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        if (lab[i] != (unsigned)i) continue;
        const int x = (int)(i % nx);
        const long long r = i / nx;
        const int y = (int)(r % ny), z = (int)(r / ny);
        if (bub_class<COMP>(d, P, LP, x, y, z, eps) == 1) ++neg;
        else ++pos;
    }
    __shared__ unsigned long long red[2][BUB_THREADS];
    red[0][threadIdx.x] = neg;
    red[1][threadIdx.x] = pos;
    __syncthreads();
    for (int w = BUB_THREADS / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (red[0][0]) atomicAdd(counts, red[0][0]);
        if (red[1][0]) atomicAdd(counts + 1, red[1][0]);
    }
}

__global__ void bub_zero_kernel(unsigned long long* counts) {
    if (threadIdx.x < 2) counts[threadIdx.x] = 0;
}

template <bool COMP>
int launch_bubbles_t(const SolveDesc* desc, int parity, double eps, long long points, unsigned* labels,
                     unsigned long long* counts, hipStream_t s) {
    const long long want = (points + BUB_THREADS - 1) / BUB_THREADS;
    const int blocks = (int)(want < 65536 ? want : 65536);
    hipLaunchKernelGGL(bub_zero_kernel, dim3(1), dim3(64), 0, s, counts);
    hipLaunchKernelGGL((bub_init_kernel<COMP>), dim3(blocks), dim3(BUB_THREADS), 0, s, desc, parity, eps,
                       labels);
    hipLaunchKernelGGL((bub_union_kernel<COMP>), dim3(blocks), dim3(BUB_THREADS), 0, s, desc, parity, eps,
                       labels);
    hipLaunchKernelGGL((bub_count_kernel<COMP>), dim3(blocks), dim3(BUB_THREADS), 0, s, desc, parity, eps,
                       labels, counts);
    return (int)hipGetLastError();
}

}  // namespace

int launch_bubbles(int prec, const SolveDesc* desc, int parity, double eps, long long points,
                   unsigned* labels, unsigned long long* counts, void* stream) {
    if (points <= 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    if (prec == PREC_F32C) return launch_bubbles_t<true>(desc, parity, eps, points, labels, counts, s);
    return launch_bubbles_t<false>(desc, parity, eps, points, labels, counts, s);
}

}  // namespace hb
