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
// One workgroup per solve; the whole state lives in LDS and the workgroup runs
// all of its time steps in one launch (solves are independent, so no grid
// synchronisation is needed).  Stage inputs are formed as in the 3-D kernels
// (G storage: only the psi component of each stage derivative is kept).
#include <hip/hip_runtime.h>

#include "hb_internal.h"

namespace hb {
namespace {

constexpr int RAD_THREADS = 256;

template <typename T>
using gptr = __attribute__((address_space(1))) T*;

__global__ void __launch_bounds__(RAD_THREADS)
radial_kernel(const RadialDesc* __restrict__ descs, double* __restrict__ phi,
              double* __restrict__ psi) {
    extern __shared__ double lds[];
    const RadialDesc d = descs[blockIdx.x];
    const int m = d.m;
    // LDS: S (stage input, with 2 leading ghost slots and 2 trailing zeros),
    // Y_phi, Y_psi, G1, G2, G3
    double* S = lds + 2;              // S[-2 .. m+1]
    double* Yp = lds + (m + 4);
    double* Ys = Yp + m;
    double* G1 = Ys + m;
    double* G2 = G1 + m;
    double* G3 = G2 + m;
    gptr<double> gp = (gptr<double>)(phi + d.offset);
    gptr<double> gs = (gptr<double>)(psi + d.offset);
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        Yp[i] = gp[i];
        Ys[i] = gs[i];
    }
    if (threadIdx.x < 2) S[m + threadIdx.x] = 0.0;  // phi(R) = 0 and beyond
    __syncthreads();

    const double dr = d.dr, mu2 = d.mu2, lam = d.lambda, dt = d.dt;
    const double hdt = dt / 2.0, dt6 = dt / 6.0;
    const double idr2 = 1.0 / (dr * dr), i12dr = 1.0 / (12.0 * dr);

    // radial operator at node i from S (ghosts filled)
    auto op = [&](int i) {
        const double um2 = S[i - 2], um1 = S[i - 1], u0 = S[i], up1 = S[i + 1], up2 = S[i + 2];
        const double urr = (-1.0 / 12.0 * um2 + 4.0 / 3.0 * um1 - 5.0 / 2.0 * u0 + 4.0 / 3.0 * up1
                            - 1.0 / 12.0 * up2) * idr2;
        if (i == 0) return 3.0 * urr;
        const double ur = (um2 - 8.0 * um1 + 8.0 * up1 - up2) * i12dr;
        return 2.0 / ((double)i * dr) * ur + urr;
    };
    auto ghosts = [&]() {
        if (threadIdx.x == 0) {
            S[-1] = m > 1 ? S[1] : 0.0;
            S[-2] = m > 2 ? S[2] : 0.0;
        }
    };

    for (long long n = 0; n < d.steps; ++n) {
        const double t = d.t0 + (double)n * dt;
        const double c1 = exp(-2.0 * t) * d.inv_L2;
        const double c2 = exp(-2.0 * (t + dt / 2.0)) * d.inv_L2;
        const double c4 = exp(-2.0 * (t + dt)) * d.inv_L2;
        // stage 1: S = Y_phi, S_psi = Y_psi
        for (int i = threadIdx.x; i < m; i += blockDim.x) S[i] = Yp[i];
        __syncthreads();
        ghosts();
        __syncthreads();
        for (int i = threadIdx.x; i < m; i += blockDim.x) {
            const double s = S[i];
            G1[i] = -3.0 * Ys[i] + c1 * op(i) + mu2 * s - lam * s * s * s;
        }
        __syncthreads();
        // stage 2: S = Y_phi + dt/2 Y_psi, S_psi = Y_psi + dt/2 G1
        for (int i = threadIdx.x; i < m; i += blockDim.x) S[i] = Yp[i] + hdt * Ys[i];
        __syncthreads();
        ghosts();
        __syncthreads();
        for (int i = threadIdx.x; i < m; i += blockDim.x) {
            const double s = S[i];
            G2[i] = -3.0 * (Ys[i] + hdt * G1[i]) + c2 * op(i) + mu2 * s - lam * s * s * s;
        }
        __syncthreads();
        // stage 3: S = Y_phi + dt/2 (Y_psi + dt/2 G1), S_psi = Y_psi + dt/2 G2
        for (int i = threadIdx.x; i < m; i += blockDim.x) S[i] = Yp[i] + hdt * (Ys[i] + hdt * G1[i]);
        __syncthreads();
        ghosts();
        __syncthreads();
        for (int i = threadIdx.x; i < m; i += blockDim.x) {
            const double s = S[i];
            G3[i] = -3.0 * (Ys[i] + hdt * G2[i]) + c2 * op(i) + mu2 * s - lam * s * s * s;
        }
        __syncthreads();
        // stage 4: S = Y_phi + dt (Y_psi + dt/2 G2), S_psi = Y_psi + dt G3; update
        for (int i = threadIdx.x; i < m; i += blockDim.x) S[i] = Yp[i] + dt * (Ys[i] + hdt * G2[i]);
        __syncthreads();
        ghosts();
        __syncthreads();
        for (int i = threadIdx.x; i < m; i += blockDim.x) {
            const double s = S[i];
            const double ys = Ys[i], e1 = G1[i], e2 = G2[i], e3 = G3[i];
            const double spsi4 = ys + dt * e3;
            const double g4 = -3.0 * spsi4 + c4 * op(i) + mu2 * s - lam * s * s * s;
            const double k2 = ys + hdt * e1, k3 = ys + hdt * e2;
            Yp[i] = Yp[i] + dt6 * (ys + 2.0 * k2 + 2.0 * k3 + spsi4);
            Ys[i] = ys + dt6 * (e1 + 2.0 * e2 + 2.0 * e3 + g4);
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < m; i += blockDim.x) {
        gp[i] = Yp[i];
        gs[i] = Ys[i];
    }
}

}  // namespace

size_t radial_lds_bytes(int max_m) { return (size_t)(6 * max_m + 4) * sizeof(double); }

int launch_radial(const RadialDesc* descs, int count, int max_m, double* phi, double* psi,
                  void* stream) {
    if (count <= 0) return 0;
    const size_t bytes = radial_lds_bytes(max_m);
    if (bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)radial_kernel,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return (int)e;
    }
    hipLaunchKernelGGL(radial_kernel, dim3(count), dim3(RAD_THREADS), radial_lds_bytes(max_m),
                       (hipStream_t)stream, descs, phi, psi);
    return (int)hipGetLastError();
}

}  // namespace hb
