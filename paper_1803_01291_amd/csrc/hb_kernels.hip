// HIP kernels for gfx950: one RK4 stage of the Higgs boson equation in de
// Sitter spacetime per launch (Balogh, Banda, Yagdjian, section 2.1).
//
// System (eq. (rhs)):  phi_t = psi,
//                      psi_t = -3 psi + c(t) Lap_h phi + mu2 phi - lambda phi^3,
// with the fourth-order 13-point Laplacian of section 2.1 and classical RK4.
//
// Storage scheme ("G storage", 19 field passes per step).  Only the psi
// component of each stage derivative needs storing, because the phi component
// of k_s is the psi component of the stage-s input:
//   G_s = g(t_s, S_phi,s, S_psi,s),  g(phi, psi) = -3 psi + c Lap phi + mu2 phi - lambda phi^3
//   S_phi,1 = Y_phi                          S_psi,1 = Y_psi
//   S_phi,2 = Y_phi + dt/2 Y_psi             S_psi,2 = Y_psi + dt/2 G1
//   S_phi,3 = Y_phi + dt/2 S_psi,2           S_psi,3 = Y_psi + dt/2 G2
//   S_phi,4 = Y_phi + dt   S_psi,3           S_psi,4 = Y_psi + dt   G3
//   phi' = Y_phi + dt/6 (Y_psi + 2 S_psi,2 + 2 S_psi,3 + S_psi,4)
//   psi' = Y_psi + dt/6 (G1 + 2 G2 + 2 G3 + G4)
// which is the classical RK4 update with each stage input formed in the same
// order as the textbook form.  Stage s reads, per point,
//   s=1: Y_phi (stencil), Y_psi                        -> writes G1
//   s=2: Y_phi, Y_psi (stencil), G1                     -> writes G2
//   s=3: Y_phi, Y_psi, G1 (stencil), G2                 -> writes G3
//   s=4: Y_phi, Y_psi, G2 (stencil), G1, G3             -> writes Y'_phi, Y'_psi
// The state ping-pongs by step parity (stage 4 stencil-reads Y while writing Y').
//
// Kernel shape.  A block owns a 64 x BY column tile (64-wide = one wavefront
// per row) and marches a z-range.  Each thread keeps its own column's stage
// input S_phi at planes z-2..z+2 in registers (the z part of the star), and
// the block stages plane z with a 2-cell x/y halo in LDS (the x and y parts).
// The raw fields of the thread's own column are loaded three planes ahead and
// those of the halo one plane ahead, so each plane's loads are in flight while
// the previous plane computes.  One __syncthreads per plane (double-buffered
// LDS).  No MFMA: the stencil is not a contraction and the path is bound by
// HBM bandwidth.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "hb_internal.h"

namespace hb {
namespace {

// Workgroups are dispatched round-robin over the 8 XCDs.  Give each XCD a
// contiguous range of the tile list, so tiles that share halo rows run on the
// same XCD and meet in its L2.  Bijective on [0, n).
__device__ __forceinline__ int xcd_remap(int b, int n) {
    const int q = n >> 3, r = n & 7;
    const int x = b & 7, l = b >> 3;
    return x * q + min(x, r) + l;
}

// Field pointers come from the descriptor, so the compiler cannot see that
// they address global memory and would emit flat accesses (which also count
// against the LDS wait counter and serialise prefetches with LDS traffic).
// All field accesses go through explicit global-address-space pointers.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ T ldg(const T* __restrict__ p, long long off, bool ok) {
    return ok ? ((gptr<const T>)p)[off] : T(0);
}

template <typename T>
__device__ __forceinline__ void stg(T* p, long long off, T v) {
    ((gptr<T>)p)[off] = v;
}

// Raw buffer access to one x-y plane of a field.  The resource's base is the
// plane's cell (-2, -2) and its size the plane's bytes.  Loads and stores go
// through buffer instructions with a per-lane 32-bit byte offset: a store
// whose offset lies past the plane is dropped by the hardware range check,
// which is how lanes without an output column skip a store without a branch.
// (Branch-free memory code keeps the number of memory operations between a
// load and its use the same on every path, so the wait before the use can
// leave the later prefetches in flight.)
constexpr int BUF_DWORD3 = 0x00020000;   // raw untyped buffer, gfx9 family
constexpr uint32_t BUF_SKIP = 0x80000000u;

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(unsigned long long base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, bytes, BUF_DWORD3);
}

template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, 0));
}

template <typename T>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t off, T v) {
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)off, 0, 0);
}

template <typename T, int STAGE, bool COMP>
struct OwnRec {
    T p, s, g1, g2, g3;
    float lp, ls;
};

template <typename T, int STAGE, int BY, bool COMP>
__global__ void __launch_bounds__(64 * BY)
stage_kernel(const SolveDesc* __restrict__ descs, const Tile* __restrict__ tiles, int ntiles,
             long long kstep) {
    constexpr int LX = TILE_X + 4;
    constexpr int LY = BY + 4;
    constexpr int NHALO = 4 * TILE_X + 4 * BY;
    static_assert(NHALO <= 64 * BY, "one halo column per thread at most");
    __shared__ T sm[2][LY][LX];

    const Tile tl = tiles[xcd_remap(blockIdx.x, ntiles)];
    const SolveDesc* __restrict__ d = descs + tl.solve;
    const long long n = d->nstep + kstep;
    if (n >= d->target) return;  // uniform over the block
    const int par = (int)(n & 1);

    const T* __restrict__ Yp = (const T*)d->y_phi[par];
    const T* __restrict__ Ys = (const T*)d->y_psi[par];
    const T* __restrict__ G1 = (const T*)d->g[0];
    const T* __restrict__ G2 = (const T*)d->g[1];
    const T* __restrict__ G3 = (const T*)d->g[2];
    const long long sy = d->sy, sz = d->sz;
    const int nx = d->nx, ny = d->ny;

    const T c = (T)ldg(d->ctab, 4 * n + (STAGE - 1), true);
    const T w0 = (T)d->w0;
    const T w1x = (T)d->w1[0], w1y = (T)d->w1[1], w1z = (T)d->w1[2];
    const T w2x = (T)d->w2[0], w2y = (T)d->w2[1], w2z = (T)d->w2[2];
    const T mu2 = (T)d->mu2, lam = (T)d->lambda;
    const T dtT = (T)d->dt, hdt = (T)d->hdt;

    const int tid = threadIdx.x;
    const int tx = tid & 63, ty = tid >> 6;
    const int x = tl.x0 + tx, y = tl.y0 + ty;
    const bool own_ld = (x < nx + 2) && (y < ny + 2);
    const bool own_st = (x < nx) && (y < ny);
    const long long own_off = (long long)y * sy + x;

    // this thread's halo column, if any: 4 rows of 64 above/below the tile,
    // then 2 columns left/right of each of the BY rows
    bool has_halo = false, halo_ld = false;
    int hlx = 0, hly = 0;
    long long halo_off = 0;
    if (tid < NHALO) {
        int hx, hy;
        if (tid < 4 * TILE_X) {
            const int r = tid >> 6;
            hy = (r < 2) ? tl.y0 - 2 + r : tl.y0 + BY + (r - 2);
            hx = tl.x0 + (tid & 63);
        } else {
            const int h = tid - 4 * TILE_X;
            const int k = h & 3;
            hy = tl.y0 + (h >> 2);
            hx = (k < 2) ? tl.x0 - 2 + k : tl.x0 + TILE_X + (k - 2);
        }
        has_halo = true;
        halo_ld = (hx >= -2) && (hx < nx + 2) && (hy >= -2) && (hy < ny + 2);
        hlx = hx - tl.x0 + 2;
        hly = hy - tl.y0 + 2;
        halo_off = (long long)hy * sy + hx;
    }

    using Rec = OwnRec<T, STAGE, COMP>;
    auto load_own = [&](int z) {
        Rec r;
        const long long o = (long long)z * sz + own_off;
        r.p = ldg(Yp, o, own_ld);
        r.s = ldg(Ys, o, own_ld);
        r.g1 = (STAGE >= 2) ? ldg(G1, o, own_ld) : T(0);
        r.g2 = (STAGE >= 3) ? ldg(G2, o, own_ld) : T(0);
        r.g3 = (STAGE == 4) ? ldg(G3, o, own_ld) : T(0);
        if constexpr (COMP && STAGE == 4) {
            r.lp = ldg(d->lo_phi, o, own_ld);
            r.ls = ldg(d->lo_psi, o, own_ld);
        } else {
            r.lp = 0.f;
            r.ls = 0.f;
        }
        return r;
    };
    // halo needs only the fields that make up the stencil input S_phi,s
    struct HaloRec { T p, s, g; };
    auto load_halo = [&](int z) {
        HaloRec r;
        const long long o = (long long)z * sz + halo_off;
        const bool ok = has_halo && halo_ld;
        r.p = ldg(Yp, o, ok);
        r.s = (STAGE >= 2) ? ldg(Ys, o, ok) : T(0);
        r.g = (STAGE == 3) ? ldg(G1, o, ok) : (STAGE == 4) ? ldg(G2, o, ok) : T(0);
        return r;
    };
    auto formS = [&](T p, T s, T g) -> T {
        if constexpr (STAGE == 1) return p;
        if constexpr (STAGE == 2) return p + hdt * s;
        if constexpr (STAGE == 3) return p + hdt * (s + hdt * g);
        return p + dtT * (s + hdt * g);
    };
    auto formS_own = [&](const Rec& r) -> T {
        return formS(r.p, r.s, (STAGE == 3) ? r.g1 : r.g2);
    };

    const int z0 = tl.z0, z1 = tl.z1;
    Rec rm2 = load_own(z0 - 2), rm1 = load_own(z0 - 1);
    Rec r0 = load_own(z0), r1 = load_own(z0 + 1), r2 = load_own(z0 + 2);
    HaloRec h0 = load_halo(z0);
    T q0 = formS_own(rm2), q1 = formS_own(rm1), q2 = formS_own(r0), q3 = formS_own(r1);
    int buf = 0;

    for (int z = z0; z < z1; ++z) {
        Rec rn{};
        HaloRec hn{};
        if (z + 3 <= z1 + 1) rn = load_own(z + 3);
        if (z + 1 < z1) hn = load_halo(z + 1);

        const T q4 = formS_own(r2);
        sm[buf][ty + 2][tx + 2] = q2;
        if (has_halo) sm[buf][hly][hlx] = formS(h0.p, h0.s, h0.g);
        __syncthreads();

        const T(*P)[LX] = sm[buf];
        const int lx = tx + 2, ly = ty + 2;
        T lap = w0 * q2;
        lap += w1x * (P[ly][lx - 1] + P[ly][lx + 1]);
        lap += w2x * (P[ly][lx - 2] + P[ly][lx + 2]);
        lap += w1y * (P[ly - 1][lx] + P[ly + 1][lx]);
        lap += w2y * (P[ly - 2][lx] + P[ly + 2][lx]);
        lap += w1z * (q1 + q3);
        lap += w2z * (q0 + q4);

        // centre: S_psi,s and the psi forcing g = -3 S_psi + c Lap + mu2 S - lambda S^3
        T spsi;
        if constexpr (STAGE == 1) spsi = r0.s;
        if constexpr (STAGE == 2) spsi = r0.s + hdt * r0.g1;
        if constexpr (STAGE == 3) spsi = r0.s + hdt * r0.g2;
        if constexpr (STAGE == 4) spsi = r0.s + dtT * r0.g3;
        const T S = q2;
        const T g = -T(3) * spsi + c * lap + mu2 * S - lam * S * S * S;

        const long long o = (long long)z * sz + own_off;
        if (own_st) {
            if constexpr (STAGE < 4) {
                stg((T*)d->g[STAGE - 1], o, g);
            } else if constexpr (!COMP) {
                const double dt6 = d->dt6;
                const T k2 = r0.s + hdt * r0.g1;
                const T k3 = r0.s + hdt * r0.g2;
                stg((T*)d->y_phi[par ^ 1], o, (T)(r0.p + dt6 * (r0.s + T(2) * k2 + T(2) * k3 + spsi)));
                stg((T*)d->y_psi[par ^ 1], o,
                    (T)(r0.s + dt6 * (r0.g1 + T(2) * r0.g2 + T(2) * r0.g3 + g)));
            } else {
                // compensated state: v = hi + lo carried in FP64 registers;
                // the stage derivatives come from the FP32 stage arithmetic
                const double hd = d->hdt, dd = d->dt, dt6 = d->dt6;
                const double p = (double)r0.p + (double)r0.lp;
                const double s = (double)r0.s + (double)r0.ls;
                const double a1 = r0.g1, a2 = r0.g2, a3 = r0.g3, a4 = g;
                const double k2 = s + hd * a1, k3 = s + hd * a2, k4 = s + dd * a3;
                const double np_ = p + dt6 * (s + 2.0 * k2 + 2.0 * k3 + k4);
                const double ns_ = s + dt6 * (a1 + 2.0 * a2 + 2.0 * a3 + a4);
                const float hp = (float)np_, hs = (float)ns_;
                stg((float*)d->y_phi[par ^ 1], o, hp);
                stg((float*)d->y_psi[par ^ 1], o, hs);
                stg(d->lo_phi, o, (float)(np_ - (double)hp));
                stg(d->lo_psi, o, (float)(ns_ - (double)hs));
            }
        }
        q0 = q1; q1 = q2; q2 = q3; q3 = q4;
        r0 = r1; r1 = r2; r2 = rn;
        h0 = hn;
        buf ^= 1;
    }
}

// Stage-pair kernels.  Because phi_t = psi, the stencil input of stage s is
// built from G_{s-2} at most (S_phi,2 from Y only, S_phi,4 from Y and G2), so
// stages 1+2 and stages 3+4 can each be evaluated in one pass over the grid:
//   PAIR 0: reads Y_phi, Y_psi (both stenciled)          -> writes G1, G2
//   PAIR 1: reads Y_phi, Y_psi, G1, G2 (all stenciled)   -> writes Y'_phi, Y'_psi
//           (G3 lives only in registers)
// 10 field passes per step instead of 19.  The per-point arithmetic and its
// order are those of the per-stage kernels above, so results are bitwise equal.
// Two stencil inputs per pass: two LDS planes and two register z-queues.
template <typename T, int PAIR, int BY, bool COMP>
__global__ void __launch_bounds__(64 * BY)
pair_kernel(const SolveDesc* __restrict__ descs, const Tile* __restrict__ tiles, int ntiles,
            long long kstep) {
    constexpr int LX = TILE_X + 4;
    constexpr int LY = BY + 4;
    constexpr int NHALO = 4 * TILE_X + 4 * BY;
    static_assert(NHALO <= 64 * BY, "one halo column per thread at most");
    __shared__ T sa[2][LY][LX];
    __shared__ T sb[2][LY][LX];

    const Tile tl = tiles[xcd_remap(blockIdx.x, ntiles)];
    const SolveDesc* __restrict__ d = descs + tl.solve;
    const long long n = d->nstep + kstep;
    if (n >= d->target) return;  // uniform over the block
    const int par = (int)(n & 1);

    const T* __restrict__ Yp = (const T*)d->y_phi[par];
    const T* __restrict__ Ys = (const T*)d->y_psi[par];
    const T* __restrict__ G1 = (const T*)d->g[0];
    const T* __restrict__ G2 = (const T*)d->g[1];
    const long long sy = d->sy, sz = d->sz;
    const int nx = d->nx, ny = d->ny;

    const T ca = (T)ldg(d->ctab, 4 * n + 2 * PAIR, true);
    const T cb = (T)ldg(d->ctab, 4 * n + 2 * PAIR + 1, true);
    const T w0 = (T)d->w0;
    const T w1x = (T)d->w1[0], w1y = (T)d->w1[1], w1z = (T)d->w1[2];
    const T w2x = (T)d->w2[0], w2y = (T)d->w2[1], w2z = (T)d->w2[2];
    const T mu2 = (T)d->mu2, lam = (T)d->lambda;
    const T dtT = (T)d->dt, hdt = (T)d->hdt;

    const int tid = threadIdx.x;
    const int tx = tid & 63, ty = tid >> 6;
    const int x = tl.x0 + tx, y = tl.y0 + ty;
    const bool own_ld = (x < nx + 2) && (y < ny + 2);
    const bool own_st = (x < nx) && (y < ny);
    const long long own_off = (long long)y * sy + x;

    bool has_halo = false, halo_ld = false;
    int hlx = 0, hly = 0;
    long long halo_off = 0;
    if (tid < NHALO) {
        int hx, hy;
        if (tid < 4 * TILE_X) {
            const int r = tid >> 6;
            hy = (r < 2) ? tl.y0 - 2 + r : tl.y0 + BY + (r - 2);
            hx = tl.x0 + (tid & 63);
        } else {
            const int h = tid - 4 * TILE_X;
            const int k = h & 3;
            hy = tl.y0 + (h >> 2);
            hx = (k < 2) ? tl.x0 - 2 + k : tl.x0 + TILE_X + (k - 2);
        }
        has_halo = true;
        halo_ld = (hx >= -2) && (hx < nx + 2) && (hy >= -2) && (hy < ny + 2);
        hlx = hx - tl.x0 + 2;
        hly = hy - tl.y0 + 2;
        halo_off = (long long)hy * sy + hx;
    }

    // raw fields of one point: PAIR 0 needs Y_phi, Y_psi; PAIR 1 also G1, G2
    struct Rec {
        T p, s, g1, g2;
    };
    auto load_at = [&](long long o, bool ok) {
        Rec r;
        r.p = ldg(Yp, o, ok);
        r.s = ldg(Ys, o, ok);
        r.g1 = (PAIR == 1) ? ldg(G1, o, ok) : T(0);
        r.g2 = (PAIR == 1) ? ldg(G2, o, ok) : T(0);
        return r;
    };
    auto load_own = [&](int z) { return load_at((long long)z * sz + own_off, own_ld); };
    auto load_halo = [&](int z) { return load_at((long long)z * sz + halo_off, has_halo && halo_ld); };
    // the two stencil inputs: PAIR 0: S_phi,1 and S_phi,2; PAIR 1: S_phi,3 and S_phi,4
    auto formA = [&](const Rec& r) -> T {
        if constexpr (PAIR == 0) return r.p;
        return r.p + hdt * (r.s + hdt * r.g1);
    };
    auto formB = [&](const Rec& r) -> T {
        if constexpr (PAIR == 0) return r.p + hdt * r.s;
        return r.p + dtT * (r.s + hdt * r.g2);
    };

    const int z0 = tl.z0, z1 = tl.z1;
    Rec rm2 = load_own(z0 - 2), rm1 = load_own(z0 - 1);
    Rec r0 = load_own(z0), r1 = load_own(z0 + 1), r2 = load_own(z0 + 2);
    Rec h0 = load_halo(z0);
    T a0 = formA(rm2), a1 = formA(rm1), a2 = formA(r0), a3 = formA(r1);
    T b0 = formB(rm2), b1 = formB(rm1), b2 = formB(r0), b3 = formB(r1);
    float lp = 0.f, ls = 0.f, lpn = 0.f, lsn = 0.f;
    if constexpr (COMP && PAIR == 1) {
        lp = ldg(d->lo_phi, (long long)z0 * sz + own_off, own_ld);
        ls = ldg(d->lo_psi, (long long)z0 * sz + own_off, own_ld);
    }
    int buf = 0;

    for (int z = z0; z < z1; ++z) {
        Rec rn{}, hn{};
        if (z + 3 <= z1 + 1) rn = load_own(z + 3);
        if (z + 1 < z1) hn = load_halo(z + 1);
        if constexpr (COMP && PAIR == 1) {
            if (z + 1 < z1) {
                lpn = ldg(d->lo_phi, (long long)(z + 1) * sz + own_off, own_ld);
                lsn = ldg(d->lo_psi, (long long)(z + 1) * sz + own_off, own_ld);
            }
        }

        const T a4 = formA(r2), b4 = formB(r2);
        sa[buf][ty + 2][tx + 2] = a2;
        sb[buf][ty + 2][tx + 2] = b2;
        if (has_halo) {
            sa[buf][hly][hlx] = formA(h0);
            sb[buf][hly][hlx] = formB(h0);
        }
        __syncthreads();

        const int lx = tx + 2, ly = ty + 2;
        const T(*PA)[LX] = sa[buf];
        const T(*PB)[LX] = sb[buf];
        T lapA = w0 * a2;
        lapA += w1x * (PA[ly][lx - 1] + PA[ly][lx + 1]);
        lapA += w2x * (PA[ly][lx - 2] + PA[ly][lx + 2]);
        lapA += w1y * (PA[ly - 1][lx] + PA[ly + 1][lx]);
        lapA += w2y * (PA[ly - 2][lx] + PA[ly + 2][lx]);
        lapA += w1z * (a1 + a3);
        lapA += w2z * (a0 + a4);
        T lapB = w0 * b2;
        lapB += w1x * (PB[ly][lx - 1] + PB[ly][lx + 1]);
        lapB += w2x * (PB[ly][lx - 2] + PB[ly][lx + 2]);
        lapB += w1y * (PB[ly - 1][lx] + PB[ly + 1][lx]);
        lapB += w2y * (PB[ly - 2][lx] + PB[ly + 2][lx]);
        lapB += w1z * (b1 + b3);
        lapB += w2z * (b0 + b4);

        const long long o = (long long)z * sz + own_off;
        if constexpr (PAIR == 0) {
            // stage 1: S_psi,1 = Y_psi;  stage 2: S_psi,2 = Y_psi + dt/2 G1
            const T SA = a2, SB = b2;
            const T g1 = -T(3) * r0.s + ca * lapA + mu2 * SA - lam * SA * SA * SA;
            const T spsi2 = r0.s + hdt * g1;
            const T g2 = -T(3) * spsi2 + cb * lapB + mu2 * SB - lam * SB * SB * SB;
            if (own_st) {
                stg((T*)d->g[0], o, g1);
                stg((T*)d->g[1], o, g2);
            }
        } else {
            // stage 3: S_psi,3 = Y_psi + dt/2 G2;  stage 4: S_psi,4 = Y_psi + dt G3
            const T SA = a2, SB = b2;
            const T spsi3 = r0.s + hdt * r0.g2;
            const T g3 = -T(3) * spsi3 + ca * lapA + mu2 * SA - lam * SA * SA * SA;
            const T spsi4 = r0.s + dtT * g3;
            const T g4 = -T(3) * spsi4 + cb * lapB + mu2 * SB - lam * SB * SB * SB;
            if (own_st) {
                if constexpr (!COMP) {
                    const double dt6 = d->dt6;
                    const T k2 = r0.s + hdt * r0.g1;
                    const T k3 = r0.s + hdt * r0.g2;
                    stg((T*)d->y_phi[par ^ 1], o,
                        (T)(r0.p + dt6 * (r0.s + T(2) * k2 + T(2) * k3 + spsi4)));
                    stg((T*)d->y_psi[par ^ 1], o,
                        (T)(r0.s + dt6 * (r0.g1 + T(2) * r0.g2 + T(2) * g3 + g4)));
                } else {
                    const double hd = d->hdt, dd = d->dt, dt6 = d->dt6;
                    const double p = (double)r0.p + (double)lp;
                    const double s = (double)r0.s + (double)ls;
                    const double e1 = r0.g1, e2 = r0.g2, e3 = g3, e4 = g4;
                    const double k2 = s + hd * e1, k3 = s + hd * e2, k4 = s + dd * e3;
                    const double np_ = p + dt6 * (s + 2.0 * k2 + 2.0 * k3 + k4);
                    const double ns_ = s + dt6 * (e1 + 2.0 * e2 + 2.0 * e3 + e4);
                    const float hp = (float)np_, hs = (float)ns_;
                    stg((float*)d->y_phi[par ^ 1], o, hp);
                    stg((float*)d->y_psi[par ^ 1], o, hs);
                    stg(d->lo_phi, o, (float)(np_ - (double)hp));
                    stg(d->lo_psi, o, (float)(ns_ - (double)hs));
                }
            }
        }
        a0 = a1; a1 = a2; a2 = a3; a3 = a4;
        b0 = b1; b1 = b2; b2 = b3; b3 = b4;
        r0 = r1; r1 = r2; r2 = rn;
        h0 = hn;
        lp = lpn; ls = lsn;
        buf ^= 1;
    }
}

// Whole-step kernel: all four stages of one RK4 step in one z-march.
// A block owns an interior tile of (RX-4) x 12 columns; its RX*16 threads own
// the RX x 16 columns of the tile plus a 2-cell ring (region R2).  RX = 64
// (1024 threads, one block per CU) or 32 (512 threads, two blocks per CU).
// Per plane zi:
//   stage 1+2 on R2: G1, G2 at plane zi from the stencils of Y_phi and S_phi,2
//     (x-y part from an LDS plane over the 4-cell ring R4, z part from each
//     thread's register queue of Y planes zi-2..zi+2); outside the grid
//     interior G1 = G2 = 0, exactly the zero halo the two-kernel scheme reads;
//   S_phi,3 and S_phi,4 at plane zi on R2 go to a 3-plane LDS ring (their
//     x-y stencil part) and to each thread's register queue (z part);
//   stage 3+4 and the update at plane z = zi - 2 on the tile, from the ring,
//     the queues and the thread's own Y and G1, G2 (2-plane delay).
// HBM traffic is Y in and Y' out (4 field passes per step); the ring columns'
// G1, G2 are recomputed by neighbouring blocks instead of stored.  The
// per-point arithmetic and its order are those of the stage-pair kernels, so
// results are bitwise equal to them.  One barrier per plane: the stage-1+2
// plane is double-buffered, and stages 3+4 read ring slots written two
// planes earlier.  All per-plane queues are rings indexed by the plane number
// modulo 6 and the loop is unrolled by 6, so queue shifts are register
// renaming rather than moves.
constexpr int SK_RY = 16;

// 32-wide blocks: two resident 8-wave blocks per CU = 4 waves per SIMD
// (the second launch-bounds argument is the minimum waves per SIMD)
template <typename T, bool COMP, int SK_RX>
__global__ void __launch_bounds__(SK_RX * SK_RY, SK_RX == 32 ? 4 : 1)
step_kernel(const SolveDesc* __restrict__ descs, const Tile* __restrict__ tiles, int ntiles,
            long long kstep) {
    constexpr int SK_QX = SK_RX + 4, SK_QY = SK_RY + 4;  // R4
    constexpr int SK_NOUTER = SK_QX * SK_QY - SK_RX * SK_RY;
    static_assert(SK_NOUTER <= SK_RX * SK_RY, "one outer-ring column per thread at most");
    __shared__ T pa[2][SK_QY][SK_QX];      // Y_phi at plane zi over R4 (double-buffered)
    __shared__ T pb[2][SK_QY][SK_QX];      // S_phi,2 at plane zi over R4
    __shared__ T r3[3][SK_RY][SK_RX];      // S_phi,3 at planes zi-2..zi over R2
    __shared__ T r4[3][SK_RY][SK_RX];      // S_phi,4

    const Tile tl = tiles[xcd_remap(blockIdx.x, ntiles)];
    const SolveDesc* __restrict__ d = descs + tl.solve;
    const long long n = d->nstep + kstep;
    if (n >= d->target) return;  // uniform over the block
    const int par = (int)(n & 1);

    const T* __restrict__ Yp = (const T*)d->y_phi[par];
    const T* __restrict__ Ys = (const T*)d->y_psi[par];
    T* __restrict__ Op = (T*)d->y_phi[par ^ 1];
    T* __restrict__ Os = (T*)d->y_psi[par ^ 1];
    const long long sy = d->sy, sz = d->sz;
    const int nx = d->nx, ny = d->ny, nz = d->nz;

    const T c1 = (T)ldg(d->ctab, 4 * n + 0, true), c2 = (T)ldg(d->ctab, 4 * n + 1, true);
    const T c3 = (T)ldg(d->ctab, 4 * n + 2, true), c4 = (T)ldg(d->ctab, 4 * n + 3, true);
    const T w0 = (T)d->w0;
    const T w1x = (T)d->w1[0], w1y = (T)d->w1[1], w1z = (T)d->w1[2];
    const T w2x = (T)d->w2[0], w2y = (T)d->w2[1], w2z = (T)d->w2[2];
    const T mu2 = (T)d->mu2, lam = (T)d->lambda;
    const T dtT = (T)d->dt, hdt = (T)d->hdt;
    const double dt6 = d->dt6, hdd = d->hdt, dtd = d->dt;

    const int tid = threadIdx.x;
    const int rx = tid % SK_RX, ry = tid / SK_RX;
    const int gx = tl.x0 - 2 + rx, gy = tl.y0 - 2 + ry;
    const bool col_int = (gx >= 0) && (gx < nx) && (gy >= 0) && (gy < ny);
    const bool core = (rx >= 2) && (rx < SK_RX - 2) && (ry >= 2) && (ry < SK_RY - 2);
    const bool own_st = core && col_int;

    // Loads are not predicated: a column or plane outside the stored range
    // [-2, n + 2) is clamped onto the nearest halo cell, which holds zero for
    // the life of the solve, so the loaded value is the zero the stencil
    // needs there.  A plane is addressed through a buffer resource (scalar
    // registers) and a thread's column by a 32-bit byte offset within the
    // plane, measured from the plane's cell (-2, -2); a plane is under 2 GiB.
    auto col_bytes = [&](int x, int y) -> uint32_t {
        const int cx = min(max(x, -2), nx + 1), cy = min(max(y, -2), ny + 1);
        return (uint32_t)(((long long)(cy + 2) * sy + (cx + 2)) * (long long)sizeof(T));
    };
    const uint32_t col_b = col_bytes(gx, gy);
    // plane p of a field starts (at its cell (-2, -2)) p * pbytes bytes past
    // the field's corner address; the products are 32 x 32 -> 64-bit scalar
    // multiplies and the bases scalar adds
    const int pbytes = (int)(sz * (long long)sizeof(T));
    const long long cb = (2 * sy + 2) * (long long)sizeof(T);
    const unsigned long long bYp = (unsigned long long)Yp - cb, bYs = (unsigned long long)Ys - cb;
    const unsigned long long bOp = (unsigned long long)Op - cb, bOs = (unsigned long long)Os - cb;
    const unsigned long long bLp = (unsigned long long)d->lo_phi - cb;
    const unsigned long long bLs = (unsigned long long)d->lo_psi - cb;
    auto poff = [&](int p) -> unsigned long long { return (unsigned long long)((long long)p * pbytes); };
    auto rs = [&](unsigned long long b, unsigned long long off) { return plane_rsrc(b + off, pbytes); };
    auto clampz = [&](int p) { return min(max(p, -2), nz + 1); };

    // outer ring (R4 minus R2): rows 0,1 and QY-2,QY-1 of R4, then columns
    // 0,1 and QX-2,QX-1 of the middle rows
    const bool has_outer = tid < SK_NOUTER;
    int ox = 0, oy = 0;
    if (has_outer) {
        if (tid < 4 * SK_QX) {
            const int r = tid / SK_QX;
            oy = (r < 2) ? r : SK_QY - 4 + r;
            ox = tid % SK_QX;
        } else {
            const int h = tid - 4 * SK_QX;
            const int k = h & 3;
            oy = 2 + (h >> 2);
            ox = (k < 2) ? k : SK_QX - 4 + k;
        }
    }
    // threads without an outer-ring column load the plane's corner cell (a
    // halo zero), so every thread issues the same loads
    const uint32_t outer_b = has_outer ? col_bytes(tl.x0 - 4 + ox, tl.y0 - 4 + oy) : 0u;
    const uint32_t lo_b = own_st ? col_b : 0u;           // FP32c low parts
    const uint32_t out_b = own_st ? col_b : BUF_SKIP;    // output column or none

    const int z0 = tl.z0, z1 = tl.z1;
    const int zbase = z0 - 2;           // first plane of stages 1+2
    const int niter = z1 - z0 + 4;      // planes zbase .. z1+1 carry work
    const int zlast = min(z1 + 3, nz + 1);  // highest plane a needed evaluation reads

    // rings indexed by (plane - zbase + 6) % 6 (+6: planes down to zbase-2)
    // Loads are issued at the end of a plane into the ring slot that plane
    // has just freed: own Y two planes beyond the current window, outer-ring
    // Y three planes ahead, so each load has about two planes of work to land.
    T qp[6], qs[6];        // Y_phi, Y_psi of the own column (window zi-2..zi+2 + zi+3)
    T a3q[6], a4q[6];      // own-column S_phi,3 and S_phi,4
    T g1r[6], g2r[6];      // own-column G1, G2
    T opr[3], osr[3];      // outer-ring Y, by plane mod 3
    float lpr[3], lsr[3];  // FP32c low parts, by output plane mod 3
    for (int k = 0; k < 6; ++k) {
        qp[k] = qs[k] = a3q[k] = a4q[k] = g1r[k] = g2r[k] = T(0);
    }
    for (int k = 0; k < 3; ++k) {
        opr[k] = osr[k] = T(0);
        lpr[k] = lsr[k] = 0.f;
    }
    // prologue: own Y at planes zbase-2 .. zbase+3, outer ring at planes
    // zbase .. zbase+2, issued in the order the march issues them (own plane
    // p, then outer plane p-1), so the waits in the march's first pass are
    // those of every later pass
    auto ld_own = [&](int k) {
        const int p = zbase - 2 + k;
        const unsigned long long o = poff(clampz(p));
        qp[(k + 4) % 6] = bload<T>(rs(bYp, o), col_b);
        qs[(k + 4) % 6] = bload<T>(rs(bYs, o), col_b);
    };
    auto ld_outer = [&](int k) {
        const int p = zbase + k;
        const unsigned long long o = poff(clampz(p));
        opr[k] = bload<T>(rs(bYp, o), outer_b);
        osr[k] = bload<T>(rs(bYs, o), outer_b);
    };
    ld_own(0);
    ld_own(1);
    ld_own(2);
    ld_own(3);
    ld_outer(0);
    ld_own(4);
    ld_outer(1);
    ld_own(5);
    ld_outer(2);
    // The first plane needs almost all of these.  Waiting for all of them
    // here also leaves no prologue load pending at the head of the march,
    // so the waits inside it are set by the march's own steady pattern.
    __builtin_amdgcn_s_waitcnt(0);

    // one plane; PH = (zi - zbase) % 6 is a compile-time constant
    auto plane = [&](auto ph, int it) {
        constexpr int PH = decltype(ph)::value;
        constexpr int B = PH & 1;                    // LDS double buffer
        constexpr int RS = PH % 3;                   // LDS ring slot of plane zi
        constexpr int RS2 = (PH + 1) % 3;            // ... of plane zi - 2
        constexpr int OS = PH % 3;                   // outer / low-part slot of plane zi
        constexpr int OS2 = (PH + 1) % 3;            // ... of plane zi - 2
        auto Q = [](int k) { return (PH + 6 + k) % 6; };  // ring slot of plane zi + k
        const int zi = zbase + it;

        // ---- stages 1 + 2 at plane zi over R2 ----
        const T yp0 = qp[Q(0)], ys0 = qs[Q(0)];
        pa[B][ry + 2][rx + 2] = yp0;
        pb[B][ry + 2][rx + 2] = yp0 + hdt * ys0;
        if (has_outer) {
            pa[B][oy][ox] = opr[OS];
            pb[B][oy][ox] = opr[OS] + hdt * osr[OS];
        }
        // the only barrier of the plane: it publishes this plane's stage-1+2
        // inputs and the ring slot written two planes ago (read below)
        __syncthreads();

        T g1 = T(0), g2 = T(0);
        if (col_int && zi >= 0 && zi < nz) {
            const int lx = rx + 2, ly = ry + 2;
            const T(*A)[SK_QX] = pa[B];
            const T(*Bp)[SK_QX] = pb[B];
            const T SA = yp0, SB = yp0 + hdt * ys0;
            T lapA = w0 * SA;
            lapA += w1x * (A[ly][lx - 1] + A[ly][lx + 1]);
            lapA += w2x * (A[ly][lx - 2] + A[ly][lx + 2]);
            lapA += w1y * (A[ly - 1][lx] + A[ly + 1][lx]);
            lapA += w2y * (A[ly - 2][lx] + A[ly + 2][lx]);
            lapA += w1z * (qp[Q(-1)] + qp[Q(1)]);
            lapA += w2z * (qp[Q(-2)] + qp[Q(2)]);
            T lapB = w0 * SB;
            lapB += w1x * (Bp[ly][lx - 1] + Bp[ly][lx + 1]);
            lapB += w2x * (Bp[ly][lx - 2] + Bp[ly][lx + 2]);
            lapB += w1y * (Bp[ly - 1][lx] + Bp[ly + 1][lx]);
            lapB += w2y * (Bp[ly - 2][lx] + Bp[ly + 2][lx]);
            lapB += w1z * ((qp[Q(-1)] + hdt * qs[Q(-1)]) + (qp[Q(1)] + hdt * qs[Q(1)]));
            lapB += w2z * ((qp[Q(-2)] + hdt * qs[Q(-2)]) + (qp[Q(2)] + hdt * qs[Q(2)]));
            g1 = -T(3) * ys0 + c1 * lapA + mu2 * SA - lam * SA * SA * SA;
            const T spsi2 = ys0 + hdt * g1;
            g2 = -T(3) * spsi2 + c2 * lapB + mu2 * SB - lam * SB * SB * SB;
        }
        // stage inputs of stages 3 and 4 at plane zi (zero outside the grid)
        const T s3 = yp0 + hdt * (ys0 + hdt * g1);
        const T s4 = yp0 + dtT * (ys0 + hdt * g2);
        a3q[Q(0)] = s3;
        a4q[Q(0)] = s4;
        g1r[Q(0)] = g1;
        g2r[Q(0)] = g2;
        r3[RS][ry][rx] = s3;
        r4[RS][ry][rx] = s4;

        // ---- stages 3 + 4 and the update at plane z = zi - 2 on the tile ----
        const int z = zi - 2;
        const bool zout = z >= z0 && z < z1;
        T op_ = T(0), os_ = T(0);
        float ol_p = 0.f, ol_s = 0.f;
        if (zout && own_st) {
            const T SA = a3q[Q(-2)], SB = a4q[Q(-2)];
            T lapA = w0 * SA;
            lapA += w1x * (r3[RS2][ry][rx - 1] + r3[RS2][ry][rx + 1]);
            lapA += w2x * (r3[RS2][ry][rx - 2] + r3[RS2][ry][rx + 2]);
            lapA += w1y * (r3[RS2][ry - 1][rx] + r3[RS2][ry + 1][rx]);
            lapA += w2y * (r3[RS2][ry - 2][rx] + r3[RS2][ry + 2][rx]);
            lapA += w1z * (a3q[Q(-3)] + a3q[Q(-1)]);
            lapA += w2z * (a3q[Q(-4)] + a3q[Q(0)]);
            T lapB = w0 * SB;
            lapB += w1x * (r4[RS2][ry][rx - 1] + r4[RS2][ry][rx + 1]);
            lapB += w2x * (r4[RS2][ry][rx - 2] + r4[RS2][ry][rx + 2]);
            lapB += w1y * (r4[RS2][ry - 1][rx] + r4[RS2][ry + 1][rx]);
            lapB += w2y * (r4[RS2][ry - 2][rx] + r4[RS2][ry + 2][rx]);
            lapB += w1z * (a4q[Q(-3)] + a4q[Q(-1)]);
            lapB += w2z * (a4q[Q(-4)] + a4q[Q(0)]);
            const T yp = qp[Q(-2)], ys = qs[Q(-2)], e1 = g1r[Q(-2)], e2 = g2r[Q(-2)];
            const T spsi3 = ys + hdt * e2;
            const T g3 = -T(3) * spsi3 + c3 * lapA + mu2 * SA - lam * SA * SA * SA;
            const T spsi4 = ys + dtT * g3;
            const T g4 = -T(3) * spsi4 + c4 * lapB + mu2 * SB - lam * SB * SB * SB;
            if constexpr (!COMP) {
                const T k2 = ys + hdt * e1;
                const T k3 = ys + hdt * e2;
                op_ = (T)(yp + dt6 * (ys + T(2) * k2 + T(2) * k3 + spsi4));
                os_ = (T)(ys + dt6 * (e1 + T(2) * e2 + T(2) * g3 + g4));
            } else {
                const double pp = (double)yp + (double)lpr[OS2];
                const double ss = (double)ys + (double)lsr[OS2];
                const double a1 = e1, a2 = e2, a3 = g3, a4 = g4;
                const double k2 = ss + hdd * a1, k3 = ss + hdd * a2, k4 = ss + dtd * a3;
                const double vp = pp + dt6 * (ss + 2.0 * k2 + 2.0 * k3 + k4);
                const double vs = ss + dt6 * (a1 + 2.0 * a2 + 2.0 * a3 + a4);
                const float hp = (float)vp, hs = (float)vs;
                op_ = hp;
                os_ = hs;
                ol_p = (float)(vp - (double)hp);
                ol_s = (float)(vs - (double)hs);
            }
        }
        // stores outside the branch: lanes and planes without output use an
        // offset past the plane, which the buffer range check drops
        {
            // (outside [z0, z1) no lane stores, so the base of plane z is
            // never dereferenced even where z is outside the field)
            const uint32_t ob = zout ? out_b : BUF_SKIP;
            const unsigned long long o = poff(z);
            bstore<T>(rs(bOp, o), ob, op_);
            bstore<T>(rs(bOs, o), ob, os_);
            if constexpr (COMP) {
                bstore<float>(rs(bLp, o), ob, ol_p);
                bstore<float>(rs(bLs, o), ob, ol_s);
            }
        }

        // ---- loads for later planes, into the slots this plane freed ----
        // (unconditional: past the planes a tile reads, the plane index is
        // clamped and the value is never used)
        // own plane zi+4 into the slot of plane zi-2 (last used just above);
        // zi+4 >= z0+2 >= 2, and planes past nz+1 are never needed
        const unsigned long long op4 = poff(min(zi + 4, zlast));
        qp[Q(4)] = bload<T>(rs(bYp, op4), col_b);
        qs[Q(4)] = bload<T>(rs(bYs, op4), col_b);
        // outer plane zi+3 into the slot of plane zi (used before the barrier)
        const unsigned long long oq3 = poff(min(zi + 3, z1 + 1));
        opr[OS] = bload<T>(rs(bYp, oq3), outer_b);
        osr[OS] = bload<T>(rs(bYs, oq3), outer_b);
        if constexpr (COMP) {
            // low parts of output plane zi (updated two planes from now);
            // the slot held output plane zi-3's, used one plane ago
            const unsigned long long ol = poff(min(zi, z1));
            lpr[OS] = bload<float>(rs(bLp, ol), lo_b);
            lsr[OS] = bload<float>(rs(bLs, ol), lo_b);
        }
    };

    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    using I4 = std::integral_constant<int, 4>;
    using I5 = std::integral_constant<int, 5>;
    // The march runs a multiple of 6 planes so that every pass of the loop
    // body is the same straight-line code (no per-plane exits); planes past
    // z1+1 compute values nothing reads and store nothing.  Every thread runs
    // the same sequence of barriers.
    const int nplanes = (niter + 5) / 6 * 6;
    for (int it = 0; it < nplanes; it += 6) {
        plane(I0{}, it);
        plane(I1{}, it + 1);
        plane(I2{}, it + 2);
        plane(I3{}, it + 3);
        plane(I4{}, it + 4);
        plane(I5{}, it + 5);
    }
}

__global__ void tick_kernel(SolveDesc* descs, int count, long long k) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) {
        const long long v = descs[i].nstep + k;
        descs[i].nstep = v < descs[i].target ? v : descs[i].target;
    }
}

__global__ void set_target_kernel(SolveDesc* descs, int i, long long target) {
    if (threadIdx.x == 0) descs[i].target = target;
}

__global__ void set_nstep_kernel(SolveDesc* descs, int i, long long nstep, long long target) {
    if (threadIdx.x == 0) {
        descs[i].nstep = nstep;
        descs[i].target = target;
    }
}

template <typename S, bool COMP>
__global__ void unpack_kernel(const S* __restrict__ src, int nx, int ny, int nz, long long sy,
                              long long sz, void* __restrict__ hi, float* __restrict__ lo) {
    const long long total = (long long)nx * ny * nz;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int x = (int)(i % nx);
        const long long r = i / nx;
        const int y = (int)(r % ny), z = (int)(r / ny);
        const long long o = (long long)z * sz + (long long)y * sy + x;
        const double v = src ? (double)src[i] : 0.0;
        if constexpr (COMP) {
            const float h = (float)v;
            ((float*)hi)[o] = h;
            lo[o] = (float)(v - (double)h);
        } else {
            ((double*)hi)[o] = v;
        }
    }
}

template <typename D, bool COMP>
__global__ void pack_kernel(D* __restrict__ dst, int nx, int ny, int nz, long long sy, long long sz,
                            const void* __restrict__ hi, const float* __restrict__ lo) {
    const long long total = (long long)nx * ny * nz;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int x = (int)(i % nx);
        const long long r = i / nx;
        const int y = (int)(r % ny), z = (int)(r / ny);
        const long long o = (long long)z * sz + (long long)y * sy + x;
        double v;
        if constexpr (COMP) v = (double)((const float*)hi)[o] + (double)lo[o];
        else v = ((const double*)hi)[o];
        dst[i] = (D)v;
    }
}

// ---- diagnostics (FP64, deterministic) ----------------------------------------

constexpr int DIAG_THREADS = 256;

template <bool COMP>
__device__ __forceinline__ double fld(const void* hi, const float* lo, long long o) {
    if constexpr (COMP) return (double)ldg((const float*)hi, o, true) + (double)ldg(lo, o, true);
    return ldg((const double*)hi, o, true);
}

// One block per (y, z) row group; per-thread partial sums in a fixed order,
// then a fixed LDS tree.  Partials: DIAG_COUNT doubles per block.
template <bool COMP>
__global__ void __launch_bounds__(DIAG_THREADS)
diag_kernel(const SolveDesc* __restrict__ d, int par, double c, double* __restrict__ partials) {
    const int nx = d->nx, ny = d->ny, nz = d->nz;
    const long long sy = d->sy, sz = d->sz;
    const void* P = d->y_phi[par];
    const void* S = d->y_psi[par];
    const float* LP = d->lo_phi;
    const float* LS = d->lo_psi;
    const double w0 = d->w0, mu2 = d->mu2, lam = d->lambda;
    double acc[DIAG_COUNT];
    for (int k = 0; k < DIAG_COUNT; ++k) acc[k] = 0.0;
    const long long rows = (long long)ny * nz;
    for (long long row = blockIdx.x; row < rows; row += gridDim.x) {
        const int y = (int)(row % ny), z = (int)(row / ny);
        for (int x = threadIdx.x; x < nx; x += blockDim.x) {
            const long long o = (long long)z * sz + (long long)y * sy + x;
            const double p = fld<COMP>(P, LP, o);
            const double s = fld<COMP>(S, LS, o);
            double lap = w0 * p;
            const long long st[3] = {1, sy, sz};
            for (int a = 0; a < 3; ++a) {
                lap += d->w1[a] * (fld<COMP>(P, LP, o - st[a]) + fld<COMP>(P, LP, o + st[a]));
                lap += d->w2[a] * (fld<COMP>(P, LP, o - 2 * st[a]) + fld<COMP>(P, LP, o + 2 * st[a]));
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

__global__ void diag_final_kernel(const double* __restrict__ partials, int nparts,
                                  double* __restrict__ out) {
    const int k = threadIdx.x;
    if (k >= DIAG_COUNT) return;
    const bool is_max = (k == DIAG_MAX_PHI || k == DIAG_MAX_PSI || k == DIAG_MAX_LAP);
    double a = 0.0;
    for (int b = 0; b < nparts; ++b) {
        const double v = partials[(long long)b * DIAG_COUNT + k];
        a = is_max ? fmax(a, v) : a + v;
    }
    out[k] = a;
}

// ---- bandwidth probe: R streamed reads and W streamed writes of 16-byte
// elements, grid-stride, no reuse (the measured HBM ceiling for kernels shaped
// like the stage kernels; also the plain copy used to calibrate byte counters)
template <int R, int W>
__global__ void __launch_bounds__(256)
probe_kernel(const double2* __restrict__ a0, const double2* __restrict__ a1,
             const double2* __restrict__ a2, const double2* __restrict__ a3,
             const double2* __restrict__ a4, double2* __restrict__ o0, double2* __restrict__ o1,
             long long n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        double2 v = a0[i];
        if constexpr (R > 1) { const double2 t = a1[i]; v.x += t.x; v.y += t.y; }
        if constexpr (R > 2) { const double2 t = a2[i]; v.x += t.x; v.y += t.y; }
        if constexpr (R > 3) { const double2 t = a3[i]; v.x += t.x; v.y += t.y; }
        if constexpr (R > 4) { const double2 t = a4[i]; v.x += t.x; v.y += t.y; }
        o0[i] = v;
        if constexpr (W > 1) o1[i] = make_double2(v.y, v.x);
    }
}

template <typename T, int STAGE, int BY, bool COMP>
hipError_t launch_one(const SolveDesc* descs, const Tile* tiles, int ntiles, long long kstep,
                      hipStream_t s) {
    hipLaunchKernelGGL((stage_kernel<T, STAGE, BY, COMP>), dim3(ntiles), dim3(64 * BY), 0, s, descs,
                       tiles, ntiles, kstep);
    return hipGetLastError();
}

template <typename T, int BY, bool COMP>
hipError_t launch_by_stage(int stage, const SolveDesc* descs, const Tile* tiles, int ntiles,
                           long long kstep, hipStream_t s) {
    switch (stage) {
        case 1: return launch_one<T, 1, BY, COMP>(descs, tiles, ntiles, kstep, s);
        case 2: return launch_one<T, 2, BY, COMP>(descs, tiles, ntiles, kstep, s);
        case 3: return launch_one<T, 3, BY, COMP>(descs, tiles, ntiles, kstep, s);
        case 4: return launch_one<T, 4, BY, COMP>(descs, tiles, ntiles, kstep, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, int BY, bool COMP>
hipError_t launch_pair_t(int pair, const SolveDesc* descs, const Tile* tiles, int ntiles,
                         long long kstep, hipStream_t s) {
    if (pair == 0)
        hipLaunchKernelGGL((pair_kernel<T, 0, BY, COMP>), dim3(ntiles), dim3(64 * BY), 0, s, descs,
                           tiles, ntiles, kstep);
    else
        hipLaunchKernelGGL((pair_kernel<T, 1, BY, COMP>), dim3(ntiles), dim3(64 * BY), 0, s, descs,
                           tiles, ntiles, kstep);
    return hipGetLastError();
}

template <typename T, bool COMP>
hipError_t launch_step_t(int width, const SolveDesc* descs, const Tile* tiles, int ntiles,
                         long long kstep, hipStream_t s) {
    if (width == 64)
        hipLaunchKernelGGL((step_kernel<T, COMP, 64>), dim3(ntiles), dim3(64 * SK_RY), 0, s, descs,
                           tiles, ntiles, kstep);
    else if (width == 32)
        hipLaunchKernelGGL((step_kernel<T, COMP, 32>), dim3(ntiles), dim3(32 * SK_RY), 0, s, descs,
                           tiles, ntiles, kstep);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace

int launch_stage(int prec, int stage, int by, const SolveDesc* descs, const Tile* tiles, int ntiles,
                 long long kstep, void* stream) {
    if (ntiles <= 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (prec == PREC_F64) {
        if (by == 8) e = launch_by_stage<double, 8, false>(stage, descs, tiles, ntiles, kstep, s);
        else if (by == 16) e = launch_by_stage<double, 16, false>(stage, descs, tiles, ntiles, kstep, s);
        else return (int)hipErrorInvalidValue;
    } else {
        if (by == 8) e = launch_by_stage<float, 8, true>(stage, descs, tiles, ntiles, kstep, s);
        else if (by == 16) e = launch_by_stage<float, 16, true>(stage, descs, tiles, ntiles, kstep, s);
        else return (int)hipErrorInvalidValue;
    }
    return (int)e;
}

int launch_pair(int prec, int pair, int by, const SolveDesc* descs, const Tile* tiles, int ntiles,
                long long kstep, void* stream) {
    if (ntiles <= 0) return 0;
    if (pair != 0 && pair != 1) return (int)hipErrorInvalidValue;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (prec == PREC_F64) {
        if (by == 8) e = launch_pair_t<double, 8, false>(pair, descs, tiles, ntiles, kstep, s);
        else if (by == 16) e = launch_pair_t<double, 16, false>(pair, descs, tiles, ntiles, kstep, s);
        else return (int)hipErrorInvalidValue;
    } else {
        if (by == 8) e = launch_pair_t<float, 8, true>(pair, descs, tiles, ntiles, kstep, s);
        else if (by == 16) e = launch_pair_t<float, 16, true>(pair, descs, tiles, ntiles, kstep, s);
        else return (int)hipErrorInvalidValue;
    }
    return (int)e;
}

int launch_step(int prec, int width, const SolveDesc* descs, const Tile* tiles, int ntiles,
                long long kstep, void* stream) {
    if (ntiles <= 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = prec == PREC_F64
                       ? launch_step_t<double, false>(width, descs, tiles, ntiles, kstep, s)
                       : launch_step_t<float, true>(width, descs, tiles, ntiles, kstep, s);
    return (int)e;
}

int launch_tick(SolveDesc* descs, int count, long long k, void* stream) {
    if (count <= 0) return 0;
    hipLaunchKernelGGL(tick_kernel, dim3((count + 63) / 64), dim3(64), 0, (hipStream_t)stream, descs,
                       count, k);
    return (int)hipGetLastError();
}

int launch_set_target(SolveDesc* descs, int index, long long target, void* stream) {
    hipLaunchKernelGGL(set_target_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, descs, index,
                       target);
    return (int)hipGetLastError();
}

int launch_set_nstep(SolveDesc* descs, int index, long long nstep, long long target, void* stream) {
    hipLaunchKernelGGL(set_nstep_kernel, dim3(1), dim3(64), 0, (hipStream_t)stream, descs, index,
                       nstep, target);
    return (int)hipGetLastError();
}

static unsigned grid_for(long long total) {
    long long blocks = (total + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    return (unsigned)(blocks < 1 ? 1 : blocks);
}

int launch_unpack(int prec, int src_dtype, const void* src, int nx, int ny, int nz, long long sy,
                  long long sz, void* hi, float* lo, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const unsigned g = grid_for((long long)nx * ny * nz);
    const bool comp = prec == PREC_F32C;
    if (src_dtype == 0) {
        if (comp) hipLaunchKernelGGL((unpack_kernel<double, true>), dim3(g), dim3(256), 0, s, (const double*)src, nx, ny, nz, sy, sz, hi, lo);
        else hipLaunchKernelGGL((unpack_kernel<double, false>), dim3(g), dim3(256), 0, s, (const double*)src, nx, ny, nz, sy, sz, hi, lo);
    } else {
        if (comp) hipLaunchKernelGGL((unpack_kernel<float, true>), dim3(g), dim3(256), 0, s, (const float*)src, nx, ny, nz, sy, sz, hi, lo);
        else hipLaunchKernelGGL((unpack_kernel<float, false>), dim3(g), dim3(256), 0, s, (const float*)src, nx, ny, nz, sy, sz, hi, lo);
    }
    return (int)hipGetLastError();
}

int launch_pack(int prec, int dst_dtype, void* dst, int nx, int ny, int nz, long long sy,
                long long sz, const void* hi, const float* lo, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const unsigned g = grid_for((long long)nx * ny * nz);
    const bool comp = prec == PREC_F32C;
    if (dst_dtype == 0) {
        if (comp) hipLaunchKernelGGL((pack_kernel<double, true>), dim3(g), dim3(256), 0, s, (double*)dst, nx, ny, nz, sy, sz, hi, lo);
        else hipLaunchKernelGGL((pack_kernel<double, false>), dim3(g), dim3(256), 0, s, (double*)dst, nx, ny, nz, sy, sz, hi, lo);
    } else {
        if (comp) hipLaunchKernelGGL((pack_kernel<float, true>), dim3(g), dim3(256), 0, s, (float*)dst, nx, ny, nz, sy, sz, hi, lo);
        else hipLaunchKernelGGL((pack_kernel<float, false>), dim3(g), dim3(256), 0, s, (float*)dst, nx, ny, nz, sy, sz, hi, lo);
    }
    return (int)hipGetLastError();
}

int launch_probe(int kind, void* const* in, void* const* out, long long n16, int blocks,
                 void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const double2* a[5];
    for (int k = 0; k < 5; ++k) a[k] = (const double2*)in[k];
    double2* o0 = (double2*)out[0];
    double2* o1 = (double2*)out[1];
    switch (kind) {
        case 0: hipLaunchKernelGGL((probe_kernel<1, 1>), dim3(blocks), dim3(256), 0, s, a[0], a[1], a[2], a[3], a[4], o0, o1, n16); break;
        case 1: hipLaunchKernelGGL((probe_kernel<2, 1>), dim3(blocks), dim3(256), 0, s, a[0], a[1], a[2], a[3], a[4], o0, o1, n16); break;
        case 2: hipLaunchKernelGGL((probe_kernel<5, 2>), dim3(blocks), dim3(256), 0, s, a[0], a[1], a[2], a[3], a[4], o0, o1, n16); break;
        default: return (int)hipErrorInvalidValue;
    }
    return (int)hipGetLastError();
}

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
    hipLaunchKernelGGL(diag_final_kernel, dim3(1), dim3(64), 0, s, partials, nparts, out);
    return (int)hipGetLastError();
}

}  // namespace hb
