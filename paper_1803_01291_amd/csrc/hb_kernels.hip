// HIP kernels for gfx950: the RK4 steps of the Higgs boson equation in de
// Sitter spacetime (Balogh, Banda, Yagdjian, section 2.1) on a 3-D grid.
//
// System (eq. (rhs)):  phi_t = psi,
//                      psi_t = -3 psi + c(t) Lap_h phi + mu2 phi - lambda phi^3,
// with the fourth-order 13-point Laplacian of section 2.1 and classical RK4.
//
// Storage scheme ("G storage").  Only the psi component of each stage
// derivative needs storing, because the phi component of k_s is the psi
// component of the stage-s input:
//   G_s = g(t_s, S_phi,s, S_psi,s),  g(phi, psi) = -3 psi + c Lap phi + mu2 phi - lambda phi^3
//   S_phi,1 = Y_phi                          S_psi,1 = Y_psi
//   S_phi,2 = Y_phi + dt/2 Y_psi             S_psi,2 = Y_psi + dt/2 G1
//   S_phi,3 = Y_phi + dt/2 S_psi,2           S_psi,3 = Y_psi + dt/2 G2
//   S_phi,4 = Y_phi + dt   S_psi,3           S_psi,4 = Y_psi + dt   G3
//   phi' = Y_phi + dt/6 (Y_psi + 2 S_psi,2 + 2 S_psi,3 + S_psi,4)
//   psi' = Y_psi + dt/6 (G1 + 2 G2 + 2 G3 + G4)
// which is the classical RK4 update.  One pass per stage would read, per point,
//   s=1: Y_phi (stencil), Y_psi                        -> write G1
//   s=2: Y_phi, Y_psi (stencil), G1                     -> write G2
//   s=3: Y_phi, Y_psi, G1 (stencil), G2                 -> write G3
//   s=4: Y_phi, Y_psi, G2 (stencil), G1, G3             -> write Y'_phi, Y'_psi
// (19 field passes).  The state ping-pongs by step parity.
//
// Three schemes, bitwise equal (they share the per-point arithmetic below):
//   stage_kernel  one launch per stage (19 passes per step);
//   pair_kernel   stages 1+2 and 3+4 per launch (10 passes);
//   step_kernel   the whole step per launch (4 passes: Y in, Y' out), the
//                 default.
// All march z with a register queue per column (the z part of the stencil)
// and stage each x-y plane with its halo in LDS (the x and y parts).  No
// MFMA: the stencil is not a contraction.
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

// A paired cell (phi, psi) in one access: 16 bytes (FP64) or 8 bytes (FP32).
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
template <typename T>
using pair_t = T __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ pair_t<T> bload2(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(pair_t<T>, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
    else
        return __builtin_bit_cast(pair_t<T>, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// i modulo n in [0, n) (periodic boundaries; i is at most a few cells outside)
__device__ __forceinline__ int wrap_index(int i, int n) {
    const int r = i % n;
    return r < 0 ? r + n : r;
}

// An FP32c cell (phi hi, psi hi, phi lo, psi lo) in one 16-byte access.
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 bload4(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}

__device__ __forceinline__ void bstore4(__amdgpu_buffer_rsrc_t r, uint32_t off, f32x4 v) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, (int)off, 0, 0);
}

template <typename T>
__device__ __forceinline__ void bstore2(__amdgpu_buffer_rsrc_t r, uint32_t off, T a, T b) {
    pair_t<T> v;
    v.x = a;
    v.y = b;
    if constexpr (sizeof(T) == 8)
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, v), r, (int)off, 0, 0);
    else
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off, 0, 0);
}

// ---- per-point arithmetic shared by every kernel ----
// Written as explicit operations (fused multiply-adds where named), with
// contraction off, in one fixed order, so the per-stage, stage-pair and
// whole-step kernels give bitwise-identical results.  The 13-point sum is one
// chain of fused multiply-adds over the six neighbour-pair sums (7 operations
// beside the pair sums; grouping it by axes costs two more, and the longer
// chain measured ~3% faster in FP64); in the psi forcing the stencil term is
// added last, to a part formed independently of the stencil.
__device__ __forceinline__ double fm(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fm(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
struct PointCoef {
    T w0, w1x, w1y, w1z, w2x, w2y, w2z, mu2, lam;
    T hdt, dt, m3h, m3d;  // dt/2, dt, -3 dt/2, -3 dt
};

template <typename T>
__device__ __forceinline__ PointCoef<T> point_coef(const SolveDesc* d) {
    PointCoef<T> k;
    k.w0 = (T)d->w0;
    k.w1x = (T)d->w1[0]; k.w1y = (T)d->w1[1]; k.w1z = (T)d->w1[2];
    k.w2x = (T)d->w2[0]; k.w2y = (T)d->w2[1]; k.w2z = (T)d->w2[2];
    k.mu2 = (T)d->mu2;
    k.lam = (T)d->lambda;
    k.hdt = (T)d->hdt;
    k.dt = (T)d->dt;
    k.m3h = T(-3) * k.hdt;
    k.m3d = T(-3) * k.dt;
    return k;
}

// x-y inputs of Lap_h at a point (eq. (lap)): centre value c and the
// neighbour pair sums x1 = S(x-1) + S(x+1), x2 = S(x-2) + S(x+2), y1, y2
// likewise
template <typename T>
struct LapXY {
    T c, x1, x2, y1, y2;
};
template <typename T>
__device__ __forceinline__ LapXY<T> lap_xy(const PointCoef<T>&, T c, T x1, T x2, T y1, T y2) {
    LapXY<T> v;
    v.c = c;
    v.x1 = x1;
    v.x2 = x2;
    v.y1 = y1;
    v.y2 = y2;
    return v;
}

// Lap_h from the x-y inputs and z1 = S(z-1) + S(z+1), z2 = S(z-2) + S(z+2):
// z terms, centre, x terms, y terms accumulated in that order
template <typename T>
__device__ __forceinline__ T lap_z(const PointCoef<T>& k, const LapXY<T>& v, T z1, T z2) {
#pragma clang fp contract(off)
    T t = fm(k.w2z, z2, k.w1z * z1);
    t = fm(k.w0, v.c, t);
    t = fm(k.w1x, v.x1, t);
    t = fm(k.w2x, v.x2, t);
    t = fm(k.w1y, v.y1, t);
    return fm(k.w2y, v.y2, t);
}

// psi forcing of eq. (rhs) without its stencil term, for S_psi = Y_psi + h G:
//   g = c Lap + S (mu2 - lambda S^2) - 3 Y_psi - 3 h G
// base = S (mu2 - lambda S^2) - 3 Y_psi
template <typename T>
__device__ __forceinline__ T force_base(const PointCoef<T>& k, T S, T ypsi) {
#pragma clang fp contract(off)
    const T m = fm(-k.lam, S * S, k.mu2);
    return fm(S, m, T(-3) * ypsi);
}

// S_phi of stages 2, 3, 4 from Y and the previous G (section 2.1, RK4 stages)
template <typename T>
__device__ __forceinline__ T s_phi2(const PointCoef<T>& k, T yp, T ys) {
    return fm(k.hdt, ys, yp);
}
template <typename T>
__device__ __forceinline__ T s_phi3(const PointCoef<T>& k, T yp, T ys, T g1) {
    return fm(k.hdt, fm(k.hdt, g1, ys), yp);
}
template <typename T>
__device__ __forceinline__ T s_phi4(const PointCoef<T>& k, T yp, T ys, T g2) {
    return fm(k.dt, fm(k.hdt, g2, ys), yp);
}

// classical RK4 update from the state (p, s) and the four psi derivatives:
//   phi' = p + dt/6 (s + 2 k2 + 2 k3 + k4),  k_j = s + c_j dt G_{j-1}
//   psi' = s + dt/6 (G1 + 2 G2 + 2 G3 + G4)
struct Upd {
    double p, s;
};
__device__ __forceinline__ Upd rk4_update(double p, double s, double e1, double e2, double e3,
                                         double e4, double hd, double dd, double dt6) {
#pragma clang fp contract(off)
    const double k2 = fm(hd, e1, s), k3 = fm(hd, e2, s), k4 = fm(dd, e3, s);
    Upd u;
    u.p = fm(dt6, fm(2.0, k2 + k3, s + k4), p);
    u.s = fm(dt6, fm(2.0, e2 + e3, e1 + e4), s);
    return u;
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
    const PointCoef<T> K = point_coef<T>(d);

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
        if constexpr (STAGE == 2) return s_phi2(K, p, s);
        if constexpr (STAGE == 3) return s_phi3(K, p, s, g);
        return s_phi4(K, p, s, g);
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
        const T lap = lap_z(K,
                            lap_xy(K, q2, P[ly][lx - 1] + P[ly][lx + 1], P[ly][lx - 2] + P[ly][lx + 2],
                                   P[ly - 1][lx] + P[ly + 1][lx], P[ly - 2][lx] + P[ly + 2][lx]),
                            q1 + q3, q0 + q4);

        // centre: G_s = c Lap + S (mu2 - lambda S^2) - 3 S_psi,s with
        // S_psi,s = Y_psi + h G_{s-1}
        const T base = force_base(K, q2, r0.s);
        T g;
        if constexpr (STAGE == 1) g = fm(c, lap, base);
        if constexpr (STAGE == 2) g = fm(c, lap, fm(K.m3h, r0.g1, base));
        if constexpr (STAGE == 3) g = fm(c, lap, fm(K.m3h, r0.g2, base));
        if constexpr (STAGE == 4) g = fm(c, lap, fm(K.m3d, r0.g3, base));

        const long long o = (long long)z * sz + own_off;
        if (own_st) {
            if constexpr (STAGE < 4) {
                stg((T*)d->g[STAGE - 1], o, g);
            } else if constexpr (!COMP) {
                const Upd u = rk4_update(r0.p, r0.s, r0.g1, r0.g2, r0.g3, g, d->hdt, d->dt, d->dt6);
                stg((T*)d->y_phi[par ^ 1], o, (T)u.p);
                stg((T*)d->y_psi[par ^ 1], o, (T)u.s);
            } else {
                // compensated state: v = hi + lo carried in FP64 registers;
                // the stage derivatives come from the FP32 stage arithmetic
                const double p = (double)r0.p + (double)r0.lp;
                const double s = (double)r0.s + (double)r0.ls;
                const Upd u = rk4_update(p, s, r0.g1, r0.g2, r0.g3, g, d->hdt, d->dt, d->dt6);
                const float hp = (float)u.p, hs = (float)u.s;
                stg((float*)d->y_phi[par ^ 1], o, hp);
                stg((float*)d->y_psi[par ^ 1], o, hs);
                stg(d->lo_phi, o, (float)(u.p - (double)hp));
                stg(d->lo_psi, o, (float)(u.s - (double)hs));
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
    const PointCoef<T> K = point_coef<T>(d);

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
        return s_phi3(K, r.p, r.s, r.g1);
    };
    auto formB = [&](const Rec& r) -> T {
        if constexpr (PAIR == 0) return s_phi2(K, r.p, r.s);
        return s_phi4(K, r.p, r.s, r.g2);
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
        const T lapA = lap_z(K,
                             lap_xy(K, a2, PA[ly][lx - 1] + PA[ly][lx + 1], PA[ly][lx - 2] + PA[ly][lx + 2],
                                    PA[ly - 1][lx] + PA[ly + 1][lx], PA[ly - 2][lx] + PA[ly + 2][lx]),
                             a1 + a3, a0 + a4);
        const T lapB = lap_z(K,
                             lap_xy(K, b2, PB[ly][lx - 1] + PB[ly][lx + 1], PB[ly][lx - 2] + PB[ly][lx + 2],
                                    PB[ly - 1][lx] + PB[ly + 1][lx], PB[ly - 2][lx] + PB[ly + 2][lx]),
                             b1 + b3, b0 + b4);

        const long long o = (long long)z * sz + own_off;
        if constexpr (PAIR == 0) {
            // stage 1: S_psi,1 = Y_psi;  stage 2: S_psi,2 = Y_psi + dt/2 G1
            const T g1 = fm(ca, lapA, force_base(K, a2, r0.s));
            const T g2 = fm(cb, lapB, fm(K.m3h, g1, force_base(K, b2, r0.s)));
            if (own_st) {
                stg((T*)d->g[0], o, g1);
                stg((T*)d->g[1], o, g2);
            }
        } else {
            // stage 3: S_psi,3 = Y_psi + dt/2 G2;  stage 4: S_psi,4 = Y_psi + dt G3
            const T g3 = fm(ca, lapA, fm(K.m3h, r0.g2, force_base(K, a2, r0.s)));
            const T g4 = fm(cb, lapB, fm(K.m3d, g3, force_base(K, b2, r0.s)));
            if (own_st) {
                if constexpr (!COMP) {
                    const Upd u = rk4_update(r0.p, r0.s, r0.g1, r0.g2, g3, g4, d->hdt, d->dt, d->dt6);
                    stg((T*)d->y_phi[par ^ 1], o, (T)u.p);
                    stg((T*)d->y_psi[par ^ 1], o, (T)u.s);
                } else {
                    const double p = (double)r0.p + (double)lp;
                    const double s = (double)r0.s + (double)ls;
                    const Upd u = rk4_update(p, s, r0.g1, r0.g2, g3, g4, d->hdt, d->dt, d->dt6);
                    const float hp = (float)u.p, hs = (float)u.s;
                    stg((float*)d->y_phi[par ^ 1], o, hp);
                    stg((float*)d->y_psi[par ^ 1], o, hs);
                    stg(d->lo_phi, o, (float)(u.p - (double)hp));
                    stg(d->lo_psi, o, (float)(u.s - (double)hs));
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
// A block's RX*RY threads own the RX x RY columns (region R2) of an interior
// tile of (RX-4) x (RY-4) columns plus a 2-cell ring; the shapes in use are
// listed with the launcher.  Per plane zi:
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
// per-point arithmetic is the shared one above, so results are bitwise equal
// to the other schemes.  One barrier per plane: the stage-1+2 plane is
// double-buffered, and stages 3+4 read ring slots written two planes
// earlier.  All per-plane queues are rings indexed by the plane number
// modulo 6 and the loop is unrolled by 6, so queue shifts are register
// renaming rather than moves.
//
// One block per CU (its LDS planes take most of the CU's 160 KB): the second
// launch-bounds argument, the block's waves per SIMD, is 4 for the 16-wave
// shapes (128 registers) and 3 for the 720-thread 36 x 20 shape.  PBC: the
// launch may hold periodic solves (each follows its own descriptor); without
// it the kernel is the zero-halo one alone.
template <typename T, bool COMP, int SK_RX, int SK_RY, bool PBC>
__global__ void __launch_bounds__(SK_RX * SK_RY, (SK_RX * SK_RY + 255) / 256)
step_kernel(const SolveDesc* __restrict__ descs, const Tile* __restrict__ tiles, int ntiles,
            long long kstep) {
    constexpr int SK_QX = SK_RX + 4, SK_QY = SK_RY + 4;  // R4
    constexpr int SK_NOUTER = SK_QX * SK_QY - SK_RX * SK_RY;
    // LDS row pitch of the R4 planes.  Where a region row is not one wave
    // (68 x 15, 36 x 28, 36 x 20), one wave holds pieces of two or three rows; a pitch
    // of the region width plus 256 bytes keeps those pieces in the bank order
    // of one contiguous run (with the natural pitch 9% (68 x 15) and 16%
    // (36 x 28) of the LDS cycles were bank conflicts; 2-7% of the step)
    constexpr int SK_PX = SK_RX != 64 ? SK_RX + 256 / (int)sizeof(T) : SK_QX;
    static_assert(SK_NOUTER <= SK_RX * SK_RY, "one outer-ring column per thread at most");
    __shared__ T pa[2][SK_QY][SK_PX];      // Y_phi at plane zi over R4 (double-buffered)
    __shared__ T pb[2][SK_QY][SK_PX];      // S_phi,2 at plane zi over R4
    __shared__ T r3[3][SK_RY][SK_RX];      // S_phi,3 at planes zi-2..zi over R2
    __shared__ T r4[3][SK_RY][SK_RX];      // S_phi,4

    const Tile tl = tiles[xcd_remap(blockIdx.x, ntiles)];
    const SolveDesc* __restrict__ d = descs + tl.solve;
    const long long n = d->nstep + kstep;
    if (n >= d->target) return;  // uniform over the block
    const int par = (int)(n & 1);

    // the state of a cell in one 16-byte slot: (phi, psi) in FP64, or
    // (phi hi, psi hi, phi lo, psi lo) in FP32c, ping-pong by step parity
    const T* __restrict__ Y = (const T*)d->y_phi[par];
    T* __restrict__ O = (T*)d->y_phi[par ^ 1];
    const long long sy = d->sy, sz = d->sz;
    const int nx = d->nx, ny = d->ny, nz = d->nz;
    constexpr int CB = 16;  // bytes per cell

    const T c1 = (T)ldg(d->ctab, 4 * n + 0, true), c2 = (T)ldg(d->ctab, 4 * n + 1, true);
    const T c3 = (T)ldg(d->ctab, 4 * n + 2, true), c4 = (T)ldg(d->ctab, 4 * n + 3, true);
    const PointCoef<T> K = point_coef<T>(d);
    const double dt6 = d->dt6, hdd = d->hdt, dtd = d->dt;

    const int tid = threadIdx.x;
    const int rx = tid % SK_RX, ry = tid / SK_RX;
    const int gx = tl.x0 - 2 + rx, gy = tl.y0 - 2 + ry;
    const bool col_int = (gx >= 0) && (gx < nx) && (gy >= 0) && (gy < ny);
    const bool core = (rx >= 2) && (rx < SK_RX - 2) && (ry >= 2) && (ry < SK_RY - 2);
    const bool own_st = core && col_int;
    // periodic boundaries: every region column and plane is a (wrapped) grid
    // point, so stages 1+2 run on all of them
    const bool per = PBC && d->periodic != 0;
    const bool col_work = per || col_int;

    // Loads are not predicated: a column or plane outside the stored range
    // [-2, n + 2) is clamped onto the nearest halo cell, which holds zero for
    // the life of the solve, so the loaded value is the zero the stencil
    // needs there (periodic solves: every index wraps into the interior).  A plane is addressed through a buffer resource (scalar
    // registers) and a thread's column by a 32-bit byte offset within the
    // plane, measured from the plane's cell (-2, -2); a plane is under 2 GiB.
    auto col_bytes = [&](int x, int y) -> uint32_t {
        const int cx = per ? wrap_index(x, nx) : min(max(x, -2), nx + 1);
        const int cy = per ? wrap_index(y, ny) : min(max(y, -2), ny + 1);
        return (uint32_t)(((long long)(cy + 2) * sy + (cx + 2)) * (long long)CB);
    };
    const uint32_t col_b = col_bytes(gx, gy);
    // plane p of a field starts (at its cell (-2, -2)) p * pbytes bytes past
    // the field's corner address; the products are 32 x 32 -> 64-bit scalar
    // multiplies and the bases scalar adds
    const int pbytes = (int)(sz * (long long)CB);
    const long long cb = (2 * sy + 2) * (long long)CB;
    const unsigned long long bY = (unsigned long long)Y - cb, bO = (unsigned long long)O - cb;
    auto poff = [&](int p) -> unsigned long long { return (unsigned long long)((long long)p * pbytes); };
    auto rs = [&](unsigned long long b, unsigned long long off) { return plane_rsrc(b + off, pbytes); };
    auto clampz = [&](int p) { return per ? wrap_index(p, nz) : min(max(p, -2), nz + 1); };
    auto zmap = [&](int p) { return per ? wrap_index(p, nz) : p; };

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
    const uint32_t out_b = own_st ? col_b : BUF_SKIP;    // output column or none

    const int z0 = tl.z0, z1 = tl.z1;
    const int zbase = z0 - 2;           // first plane of stages 1+2
    const int niter = z1 - z0 + 4;      // planes zbase .. z1+1 carry work
    const int zlast = per ? z1 + 3 : min(z1 + 3, nz + 1);  // highest plane a needed evaluation reads

    // rings indexed by (plane - zbase + 6) % 6 (+6: planes down to zbase-2)
    // Loads are issued at the end of a plane into the ring slot that plane
    // has just freed: own Y two planes beyond the current window, outer-ring
    // Y three planes ahead, so each load has about two planes of work to land.
    T qp[6], qs[6];        // Y_phi, Y_psi of the own column (window zi-2..zi+2 + zi+3)
    T a3q[6], a4q[6];      // own-column S_phi,3 and S_phi,4
    T g1r[6], g2r[6];      // own-column G1, G2
    T opr[3], osr[3];      // outer-ring Y, by plane mod 3
    float lqp[6], lqs[6];  // FP32c low parts of the own column, like qp, qs
    for (int k = 0; k < 6; ++k) {
        qp[k] = qs[k] = a3q[k] = a4q[k] = g1r[k] = g2r[k] = T(0);
        lqp[k] = lqs[k] = 0.f;
    }
    for (int k = 0; k < 3; ++k) opr[k] = osr[k] = T(0);
    // own column of plane p into ring slot k (FP32c: the low parts too)
    auto ld_own_slot = [&](int k, int p) {
        if constexpr (COMP) {
            const f32x4 v = bload4(rs(bY, poff(p)), col_b);
            qp[k] = v.x;
            qs[k] = v.y;
            lqp[k] = v.z;
            lqs[k] = v.w;
        } else {
            const pair_t<T> v = bload2<T>(rs(bY, poff(p)), col_b);
            qp[k] = v.x;
            qs[k] = v.y;
        }
    };
    // prologue: own Y at planes zbase-2 .. zbase+3, outer ring at planes
    // zbase .. zbase+2, issued in the order the march issues them (own plane
    // p, then outer plane p-1), so the waits in the march's first pass are
    // those of every later pass
    auto ld_own = [&](int k) { ld_own_slot((k + 4) % 6, clampz(zbase - 2 + k)); };
    auto ld_outer = [&](int k) {
        const int p = zbase + k;
        const pair_t<T> v = bload2<T>(rs(bY, poff(clampz(p))), outer_b);
        opr[k] = v.x;
        osr[k] = v.y;
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
        constexpr int OS = PH % 3;                   // outer-ring slot of plane zi
        auto Q = [](int k) { return (PH + 6 + k) % 6; };  // ring slot of plane zi + k
        const int zi = zbase + it;

        // ---- stages 1 + 2 at plane zi over R2 ----
        const T yp0 = qp[Q(0)], ys0 = qs[Q(0)];
        const T sb0 = s_phi2(K, yp0, ys0);
        pa[B][ry + 2][rx + 2] = yp0;
        pb[B][ry + 2][rx + 2] = sb0;
        if (has_outer) {
            pa[B][oy][ox] = opr[OS];
            pb[B][oy][ox] = s_phi2(K, opr[OS], osr[OS]);
        }
        // the only barrier of the plane: it publishes this plane's stage-1+2
        // inputs and the ring slot written two planes ago (read below)
        __syncthreads();

        T g1 = T(0), g2 = T(0);
        if (col_work && (per || (zi >= 0 && zi < nz))) {
            const int lx = rx + 2, ly = ry + 2;
            const T(*A)[SK_PX] = pa[B];
            const T(*Bp)[SK_PX] = pb[B];
            const T lapA = lap_z(K,
                                 lap_xy(K, yp0, A[ly][lx - 1] + A[ly][lx + 1], A[ly][lx - 2] + A[ly][lx + 2],
                                        A[ly - 1][lx] + A[ly + 1][lx], A[ly - 2][lx] + A[ly + 2][lx]),
                                 qp[Q(-1)] + qp[Q(1)], qp[Q(-2)] + qp[Q(2)]);
            const T lapB = lap_z(K,
                                 lap_xy(K, sb0, Bp[ly][lx - 1] + Bp[ly][lx + 1], Bp[ly][lx - 2] + Bp[ly][lx + 2],
                                        Bp[ly - 1][lx] + Bp[ly + 1][lx], Bp[ly - 2][lx] + Bp[ly + 2][lx]),
                                 s_phi2(K, qp[Q(-1)], qs[Q(-1)]) + s_phi2(K, qp[Q(1)], qs[Q(1)]),
                                 s_phi2(K, qp[Q(-2)], qs[Q(-2)]) + s_phi2(K, qp[Q(2)], qs[Q(2)]));
            g1 = fm(c1, lapA, force_base(K, yp0, ys0));
            g2 = fm(c2, lapB, fm(K.m3h, g1, force_base(K, sb0, ys0)));
        }
        // stage inputs of stages 3 and 4 at plane zi (zero outside the grid)
        const T s3 = s_phi3(K, yp0, ys0, g1);
        const T s4 = s_phi4(K, yp0, ys0, g2);
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
            const T(*R3)[SK_RX] = r3[RS2];
            const T(*R4)[SK_RX] = r4[RS2];
            const T lapA = lap_z(K,
                                 lap_xy(K, SA, R3[ry][rx - 1] + R3[ry][rx + 1], R3[ry][rx - 2] + R3[ry][rx + 2],
                                        R3[ry - 1][rx] + R3[ry + 1][rx], R3[ry - 2][rx] + R3[ry + 2][rx]),
                                 a3q[Q(-3)] + a3q[Q(-1)], a3q[Q(-4)] + a3q[Q(0)]);
            const T lapB = lap_z(K,
                                 lap_xy(K, SB, R4[ry][rx - 1] + R4[ry][rx + 1], R4[ry][rx - 2] + R4[ry][rx + 2],
                                        R4[ry - 1][rx] + R4[ry + 1][rx], R4[ry - 2][rx] + R4[ry + 2][rx]),
                                 a4q[Q(-3)] + a4q[Q(-1)], a4q[Q(-4)] + a4q[Q(0)]);
            const T yp = qp[Q(-2)], ys = qs[Q(-2)], e1 = g1r[Q(-2)], e2 = g2r[Q(-2)];
            const T g3 = fm(c3, lapA, fm(K.m3h, e2, force_base(K, SA, ys)));
            const T g4 = fm(c4, lapB, fm(K.m3d, g3, force_base(K, SB, ys)));
            if constexpr (!COMP) {
                const Upd u = rk4_update(yp, ys, e1, e2, g3, g4, hdd, dtd, dt6);
                op_ = (T)u.p;
                os_ = (T)u.s;
            } else {
                const double pp = (double)yp + (double)lqp[Q(-2)];
                const double ss = (double)ys + (double)lqs[Q(-2)];
                const Upd u = rk4_update(pp, ss, e1, e2, g3, g4, hdd, dtd, dt6);
                const float hp = (float)u.p, hs = (float)u.s;
                op_ = hp;
                os_ = hs;
                ol_p = (float)(u.p - (double)hp);
                ol_s = (float)(u.s - (double)hs);
            }
        }
        // stores outside the branch: lanes and planes without output use an
        // offset past the plane, which the buffer range check drops
        {
            // (outside [z0, z1) no lane stores, so the base of plane z is
            // never dereferenced even where z is outside the field)
            const uint32_t ob = zout ? out_b : BUF_SKIP;
            if constexpr (COMP) {
                f32x4 w;
                w.x = op_;
                w.y = os_;
                w.z = ol_p;
                w.w = ol_s;
                bstore4(rs(bO, poff(z)), ob, w);
            } else {
                bstore2<T>(rs(bO, poff(z)), ob, op_, os_);
            }
        }

        // ---- loads for later planes, into the slots this plane freed ----
        // (unconditional: past the planes a tile reads, the plane index is
        // clamped and the value is never used)
        // own plane zi+4 into the slot of plane zi-2 (last used just above);
        // zi+4 >= z0+2 >= 2, and planes past nz+1 are never needed
        ld_own_slot(Q(4), zmap(min(zi + 4, zlast)));
        // outer plane zi+3 into the slot of plane zi (used before the barrier);
        // the stencil needs only (phi, psi) (FP32c: the high parts)
        const pair_t<T> v3 = bload2<T>(rs(bY, poff(zmap(min(zi + 3, z1 + 1)))), outer_b);
        opr[OS] = v3.x;
        osr[OS] = v3.y;
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

// Debug layout check: every cell of a field that is neither interior nor in
// the 2-cell halo (row-pitch padding, the line-alignment prefix, the tail)
// gets quiet NaNs in all its elements, so a kernel that read one would carry
// NaN into its results.  `corner` is the cell index of (-2, -2, -2).
__global__ void poison_kernel(unsigned char* __restrict__ field, long long cells, int esz, int cs,
                              long long corner, long long sy, long long sz, int nx, int nz) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < cells; i += stride) {
        const long long r = i - corner;
        bool keep = false;
        if (r >= 0) {
            const long long zz = r / sz, xx = (r - zz * sz) % sy;  // rows of a plane are all kept
            keep = xx < nx + 4 && zz < nz + 4;
        }
        if (keep) continue;
        for (int e = 0; e < cs; ++e) {
            unsigned char* p = field + (i * cs + e) * esz;
            if (esz == 8)
                *(unsigned long long*)p = 0x7ff8000000000000ull;
            else
                *(unsigned int*)p = 0x7fc00000u;
        }
    }
}

template <typename S, bool COMP>
__global__ void unpack_kernel(const S* __restrict__ src, int nx, int ny, int nz, long long sy,
                              long long sz, int cs, void* __restrict__ hi, float* __restrict__ lo) {
    const long long total = (long long)nx * ny * nz;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int x = (int)(i % nx);
        const long long r = i / nx;
        const int y = (int)(r % ny), z = (int)(r / ny);
        const long long o = ((long long)z * sz + (long long)y * sy + x) * cs;
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
                            int cs, const void* __restrict__ hi, const float* __restrict__ lo) {
    const long long total = (long long)nx * ny * nz;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int x = (int)(i % nx);
        const long long r = i / nx;
        const int y = (int)(r % ny), z = (int)(r / ny);
        const long long o = ((long long)z * sz + (long long)y * sy + x) * cs;
        double v;
        if constexpr (COMP) v = (double)((const float*)hi)[o] + (double)lo[o];
        else v = ((const double*)hi)[o];
        dst[i] = (D)v;
    }
}

// ---- bandwidth probe: R streamed reads and W streamed writes of 16-byte
// elements, no reuse (the measured HBM streaming ceiling; also the plain copy
// used to calibrate byte counters).  Launched with one element per thread
// (a wave moves one contiguous 1 KiB run per array and exits), which measured
// faster than grid-stride loops of 8-64 blocks per CU, unrolled or not; the
// loop covers grids capped below one element per thread.
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

template <typename T, bool COMP, int RX, int RY>
hipError_t launch_step_shape(const SolveDesc* descs, const Tile* tiles, int ntiles, long long kstep,
                             bool pbc, hipStream_t s) {
    if (pbc)
        hipLaunchKernelGGL((step_kernel<T, COMP, RX, RY, true>), dim3(ntiles), dim3(RX * RY), 0, s,
                           descs, tiles, ntiles, kstep);
    else
        hipLaunchKernelGGL((step_kernel<T, COMP, RX, RY, false>), dim3(ntiles), dim3(RX * RY), 0, s,
                           descs, tiles, ntiles, kstep);
    return hipGetLastError();
}

// region shapes, indexed as STEP_SHAPES in hb_internal.h
template <typename T, bool COMP>
hipError_t launch_step_t(int shape, const SolveDesc* descs, const Tile* tiles, int ntiles,
                         long long kstep, bool pbc, hipStream_t s) {
    static_assert(STEP_SHAPES[0].rx == 36 && STEP_SHAPES[0].ry == 28, "shape table");
    static_assert(STEP_SHAPES[1].rx == 64 && STEP_SHAPES[1].ry == 16, "shape table");
    static_assert(STEP_SHAPES[2].rx == 68 && STEP_SHAPES[2].ry == 15, "shape table");
    static_assert(STEP_SHAPES[3].rx == 36 && STEP_SHAPES[3].ry == 20, "shape table");
    switch (shape) {
        case 0: return launch_step_shape<T, COMP, 36, 28>(descs, tiles, ntiles, kstep, pbc, s);
        case 1: return launch_step_shape<T, COMP, 64, 16>(descs, tiles, ntiles, kstep, pbc, s);
        case 2: return launch_step_shape<T, COMP, 68, 15>(descs, tiles, ntiles, kstep, pbc, s);
        case 3: return launch_step_shape<T, COMP, 36, 20>(descs, tiles, ntiles, kstep, pbc, s);
        default: return hipErrorInvalidValue;
    }
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

int launch_step(int prec, int shape, const SolveDesc* descs, const Tile* tiles, int ntiles,
                long long kstep, bool periodic, void* stream) {
    if (ntiles <= 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = prec == PREC_F64
                       ? launch_step_t<double, false>(shape, descs, tiles, ntiles, kstep, periodic, s)
                       : launch_step_t<float, true>(shape, descs, tiles, ntiles, kstep, periodic, s);
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

int launch_poison(void* field, long long cells, int esz, int cs, long long corner, long long sy,
                  long long sz, int nx, int nz, void* stream) {
    hipLaunchKernelGGL(poison_kernel, dim3(grid_for(cells)), dim3(256), 0, (hipStream_t)stream,
                       (unsigned char*)field, cells, esz, cs, corner, sy, sz, nx, nz);
    return (int)hipGetLastError();
}

int launch_unpack(int prec, int src_dtype, const void* src, int nx, int ny, int nz, long long sy,
                  long long sz, int cs, void* hi, float* lo, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const unsigned g = grid_for((long long)nx * ny * nz);
    const bool comp = prec == PREC_F32C;
    if (src_dtype == 0) {
        if (comp) hipLaunchKernelGGL((unpack_kernel<double, true>), dim3(g), dim3(256), 0, s, (const double*)src, nx, ny, nz, sy, sz, cs, hi, lo);
        else hipLaunchKernelGGL((unpack_kernel<double, false>), dim3(g), dim3(256), 0, s, (const double*)src, nx, ny, nz, sy, sz, cs, hi, lo);
    } else {
        if (comp) hipLaunchKernelGGL((unpack_kernel<float, true>), dim3(g), dim3(256), 0, s, (const float*)src, nx, ny, nz, sy, sz, cs, hi, lo);
        else hipLaunchKernelGGL((unpack_kernel<float, false>), dim3(g), dim3(256), 0, s, (const float*)src, nx, ny, nz, sy, sz, cs, hi, lo);
    }
    return (int)hipGetLastError();
}

int launch_pack(int prec, int dst_dtype, void* dst, int nx, int ny, int nz, long long sy,
                long long sz, int cs, const void* hi, const float* lo, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const unsigned g = grid_for((long long)nx * ny * nz);
    const bool comp = prec == PREC_F32C;
    if (dst_dtype == 0) {
        if (comp) hipLaunchKernelGGL((pack_kernel<double, true>), dim3(g), dim3(256), 0, s, (double*)dst, nx, ny, nz, sy, sz, cs, hi, lo);
        else hipLaunchKernelGGL((pack_kernel<double, false>), dim3(g), dim3(256), 0, s, (double*)dst, nx, ny, nz, sy, sz, cs, hi, lo);
    } else {
        if (comp) hipLaunchKernelGGL((pack_kernel<float, true>), dim3(g), dim3(256), 0, s, (float*)dst, nx, ny, nz, sy, sz, cs, hi, lo);
        else hipLaunchKernelGGL((pack_kernel<float, false>), dim3(g), dim3(256), 0, s, (float*)dst, nx, ny, nz, sy, sz, cs, hi, lo);
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

}  // namespace hb
