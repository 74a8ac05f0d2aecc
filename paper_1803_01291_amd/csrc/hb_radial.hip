// Batched radial solver (the paper's section 2.2 form) for parameter sweeps.
//
//   phi_tt - c(t) (2/r phi_r + phi_rr) + 3 phi_t = mu2 phi - lambda phi^3,
//   r = i dr, i = 0..m-1, phi(R = m dr) = 0, c(t) = inv_L2 exp(-2t),
//   phi_rr: the fourth-order central second difference of section 2.1,
//   phi_r:  the fourth-order central first difference,
//   r = 0:  L'Hospital, the operator is 3 phi_rr(0) with the even ghosts
//           u[-1] = u[1], u[-2] = u[2] (the symmetric ghost of section 2.2),
//   zeros at and beyond r = R; classical RK4 in time.
//
// One workgroup per solve; the workgroup runs all of its time steps in one
// launch (solves are independent, so no grid synchronisation is needed).
// Thread t owns a run of consecutive nodes (NPT t .. NPT t + NPT - 1): their
// Y_phi, Y_psi and G1..G3 stay in registers.  Only the stage input S_phi
// goes through LDS, in two buffers used by alternate stages, so each stage
// needs one barrier; a node's stencil takes its run's own values from
// registers and only the two values on each side of the run from LDS (4
// reads per thread and stage instead of 5 per node).  The owners of nodes 1
// and 2 also write the even ghosts S[-1], S[-2].  Stage inputs are formed as in the 3-D kernels (G
// storage: only the psi component of each stage derivative is kept).
// c(t) comes from a host FP64 table (c at t_n, t_n + dt/2 and t_n + dt for
// each step of the launch), the values the 3-D path and the oracles use, and
// the per-node arithmetic follows the plain definition's operation order
// (difference quotients divided by dr^2 and 12 dr with correctly rounded
// quotients, no contraction).
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "hb_internal.h"

// every expression of this file is evaluated as written (no fused
// multiply-adds), in the plain definition's order
#pragma clang fp contract(off)

namespace hb {
namespace {

constexpr int RAD_THREADS = 256;

template <typename T>
using gptr = __attribute__((address_space(1))) T*;

// x / d, correctly rounded, from the correctly rounded reciprocal r = 1/d:
// y = x r is within an ulp of the quotient, the remainder x - d y is exact
// in one fused multiply-add, and y + r (x - d y) rounds to the quotient
// (Markstein's final correction step for division with fused multiply-add).
// Two multiply-adds and a multiply per quotient instead of a full division
// sequence.  The step needs an exact remainder, which quotients near the
// subnormal range (|y| below about 2^-960) may not have: there the last bit
// can differ from the division's, at magnitudes around 1e-300 and below,
// in the far field of a solve's data.  (Guarding those quotients with a
// branch to the division costs a fifth of the kernel's speed.)
__device__ __forceinline__ double quot(double x, double d, double r) {
    const double y = x * r;
    return __builtin_fma(__builtin_fma(-d, y, x), r, y);
}

// LDS layout of a stage input: node j lives in row j mod NPT, column
// floor(j / NPT) + 2 of an NPT x (RAD_THREADS + 4) array, so thread t's run
// of nodes NPT t .. NPT t + NPT - 1 is column t + 2, and a wave's threads
// write and read consecutive doubles of one row (no bank conflicts).  The
// two columns on each side hold the even ghosts S[-1] = S[1], S[-2] = S[2]
// (column 1, and column 0 for NPT = 1) and nodes past the last thread's run,
// which stay zero.
constexpr int RAD_COLS = RAD_THREADS + 4;

template <int NPT>
__device__ __forceinline__ int rad_pos(int j) {
    const int q = j >= 0 ? j / NPT : -((-j + NPT - 1) / NPT);  // floor(j / NPT)
    return (j - q * NPT) * RAD_COLS + q + 2;
}

template <int NPT>
__global__ void __launch_bounds__(RAD_THREADS)
radial_kernel(const RadialDesc* __restrict__ descs, const double* __restrict__ ctab,
              double* __restrict__ phi, double* __restrict__ psi, long long n0, long long n1) {
    extern __shared__ double lds[];
    const RadialDesc d = descs[blockIdx.x];
    const int m = d.m;
    // two stage-input buffers; zero first (the ghost columns are rewritten
    // every stage, the columns past the last run stay zero: phi = 0 at and
    // beyond r = R)
    constexpr int BUF = NPT * RAD_COLS;
    double* const Sb[2] = {lds, lds + BUF};
    for (int k = threadIdx.x; k < 2 * BUF; k += RAD_THREADS) lds[k] = 0.0;
    gptr<double> gp = (gptr<double>)(phi + d.offset);
    gptr<double> gs = (gptr<double>)(psi + d.offset);
    const int j0 = threadIdx.x * NPT;  // this thread's first node
    double yp[NPT], ys[NPT], g1[NPT], g2[NPT], g3[NPT], sv[NPT];
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int i = j0 + k;
        yp[k] = i < m ? gp[i] : 0.0;
        ys[k] = i < m ? gs[i] : 0.0;
        g1[k] = g2[k] = g3[k] = sv[k] = 0.0;
    }

    const double dr = d.dr, mu2 = d.mu2, lam = d.lambda, dt = d.dt;
    const double hdt = dt / 2.0, dt6 = dt / 6.0;
    const double dr2 = dr * dr, dr12 = 12.0 * dr;
    const double rdr2 = 1.0 / dr2, rdr12 = 1.0 / dr12;  // correctly rounded reciprocals

    // 2/r at the owned nodes, divided once (kept in registers up to 8 nodes
    // per thread; recomputed, with the same result, beyond)
    constexpr bool KEEP_2R = NPT <= 8;
    double two_r[KEEP_2R ? NPT : 1];
#pragma unroll
    for (int k = 0; k < (KEEP_2R ? NPT : 1); ++k) {
        const int i = j0 + k;
        two_r[k] = i > 0 ? 2.0 / ((double)i * dr) : 0.0;
    }
    // the stage input at node j0 + k + off: from this thread's registers
    // inside its run, else from LDS (the neighbouring runs, the ghosts, the
    // zeros); the same values either way, since the LDS copy is written from
    // the registers
    auto at = [&](const double* S, int k, int off) -> double {
        const int kk = k + off;
        if (kk >= 0 && kk < NPT) return sv[kk];
        return S[rad_pos<NPT>(j0 + kk)];
    };
    // radial operator at node i (the thread's k-th) from S (ghosts filled)
    auto op = [&](const double* S, int i, int k) {
        const double um2 = at(S, k, -2), um1 = at(S, k, -1), u0 = sv[k], up1 = at(S, k, 1),
                     up2 = at(S, k, 2);
        const double urr = quot(-1.0 / 12.0 * um2 + 4.0 / 3.0 * um1 - 5.0 / 2.0 * u0 + 4.0 / 3.0 * up1
                                - 1.0 / 12.0 * up2, dr2, rdr2);
        if (i == 0) return 3.0 * urr;
        const double ur = quot(um2 - 8.0 * um1 + 8.0 * up1 - up2, dr12, rdr12);
        const double tr = KEEP_2R ? two_r[KEEP_2R ? k : 0] : 2.0 / ((double)i * dr);
        return tr * ur + urr;
    };
    // publish this thread's stage inputs sv into S (and the mirrored ghosts);
    // nodes at and past m hold zeros in sv, so their slots keep S = 0 there
    auto put = [&](double* S) {
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int i = j0 + k;
            S[rad_pos<NPT>(i)] = sv[k];
            if (i == 1 || i == 2) S[rad_pos<NPT>(-i)] = sv[k];
        }
    };

    const long long nend = d.steps < n1 ? d.steps : n1;
    const gptr<const double> ct = (gptr<const double>)(ctab + d.ctab);
    __syncthreads();  // the zeroed buffers
    for (long long n = n0; n < nend; ++n) {
        // c(t) at the stage times of step n (host FP64 table of this launch)
        const long long j = 3 * (n - n0);
        const double c1 = ct[j], c2 = ct[j + 1], c4 = ct[j + 2];
        // stage 1: S = Y_phi, S_psi = Y_psi
#pragma unroll
        for (int k = 0; k < NPT; ++k) sv[k] = yp[k];
        put(Sb[0]);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int i = j0 + k;
            if (i < m) {
                const double s = sv[k];
                g1[k] = -3.0 * ys[k] + c1 * op(Sb[0], i, k) + mu2 * s - lam * s * s * s;
            }
        }
        // stage 2: S = Y_phi + dt/2 Y_psi, S_psi = Y_psi + dt/2 G1
#pragma unroll
        for (int k = 0; k < NPT; ++k) sv[k] = yp[k] + hdt * ys[k];
        put(Sb[1]);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int i = j0 + k;
            if (i < m) {
                const double s = sv[k];
                g2[k] = -3.0 * (ys[k] + hdt * g1[k]) + c2 * op(Sb[1], i, k) + mu2 * s - lam * s * s * s;
            }
        }
        // stage 3: S = Y_phi + dt/2 (Y_psi + dt/2 G1), S_psi = Y_psi + dt/2 G2
#pragma unroll
        for (int k = 0; k < NPT; ++k) sv[k] = yp[k] + hdt * (ys[k] + hdt * g1[k]);
        put(Sb[0]);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int i = j0 + k;
            if (i < m) {
                const double s = sv[k];
                g3[k] = -3.0 * (ys[k] + hdt * g2[k]) + c2 * op(Sb[0], i, k) + mu2 * s - lam * s * s * s;
            }
        }
        // stage 4: S = Y_phi + dt (Y_psi + dt/2 G2), S_psi = Y_psi + dt G3; update
#pragma unroll
        for (int k = 0; k < NPT; ++k) sv[k] = yp[k] + dt * (ys[k] + hdt * g2[k]);
        put(Sb[1]);
        __syncthreads();
#pragma unroll
        for (int k = 0; k < NPT; ++k) {
            const int i = j0 + k;
            if (i < m) {
                const double s = sv[k];
                const double y2 = ys[k], e1 = g1[k], e2 = g2[k], e3 = g3[k];
                const double spsi4 = y2 + dt * e3;
                const double g4 = -3.0 * spsi4 + c4 * op(Sb[1], i, k) + mu2 * s - lam * s * s * s;
                const double k2 = y2 + hdt * e1, k3 = y2 + hdt * e2;
                yp[k] = yp[k] + dt6 * (y2 + 2.0 * k2 + 2.0 * k3 + spsi4);
                ys[k] = y2 + dt6 * (e1 + 2.0 * e2 + 2.0 * e3 + g4);
            }
        }
        // (the next stage 1 writes Sb[0], last read in stage 3, before this
        // stage's barrier)
    }
#pragma unroll
    for (int k = 0; k < NPT; ++k) {
        const int i = j0 + k;
        if (i < m) {
            gp[i] = yp[k];
            gs[i] = ys[k];
        }
    }
}

template <int NPT>
hipError_t launch_radial_t(const RadialDesc* descs, const double* ctab, int count, size_t bytes,
                           double* phi, double* psi, long long n0, long long n1, hipStream_t s) {
    if (bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)radial_kernel<NPT>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((radial_kernel<NPT>), dim3(count), dim3(RAD_THREADS), bytes, s, descs, ctab,
                       phi, psi, n0, n1);
    return hipGetLastError();
}

}  // namespace

// Device scratch of the entry point that allocates nothing
// (hb_radial_solve_noalloc): the descriptors and the c(t) table of its
// launches.  Every device holds its own copy for the life of the process.
// Host code never uses the array's name as a device address: the address on
// the current device comes from hipGetSymbolAddress, looked up once per
// device and kept.
static __device__ __align__(256) unsigned char scratch[RADIAL_SCRATCH_BYTES];

int radial_scratch(void** ptr) {
    static std::mutex mu;
    static std::vector<void*> addr;  // per device
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return (int)e;
    std::lock_guard<std::mutex> lk(mu);
    if ((int)addr.size() <= dev) addr.resize(dev + 1, nullptr);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return (int)e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return 0;
}

int radial_npt(int max_m) {
    const int npt = (max_m + RAD_THREADS - 1) / RAD_THREADS;
    return npt <= 1 ? 1 : npt <= 2 ? 2 : npt <= 4 ? 4 : npt <= 8 ? 8 : npt <= 11 ? 11 : 0;
}

size_t radial_lds_bytes(int max_m) { return (size_t)(2 * radial_npt(max_m) * RAD_COLS) * sizeof(double); }

int launch_radial(const RadialDesc* descs, const double* ctab, int count, int max_m, double* phi,
                  double* psi, long long n0, long long n1, void* stream) {
    if (count <= 0) return 0;
    const size_t bytes = radial_lds_bytes(max_m);
    hipStream_t s = (hipStream_t)stream;
    const int npt = radial_npt(max_m);
    hipError_t e;
    if (npt == 1) e = launch_radial_t<1>(descs, ctab, count, bytes, phi, psi, n0, n1, s);
    else if (npt == 2) e = launch_radial_t<2>(descs, ctab, count, bytes, phi, psi, n0, n1, s);
    else if (npt == 4) e = launch_radial_t<4>(descs, ctab, count, bytes, phi, psi, n0, n1, s);
    else if (npt == 8) e = launch_radial_t<8>(descs, ctab, count, bytes, phi, psi, n0, n1, s);
    else if (npt == 11) e = launch_radial_t<11>(descs, ctab, count, bytes, phi, psi, n0, n1, s);
    else return (int)hipErrorInvalidValue;
    return (int)e;
}

}  // namespace hb
