// Host runtime of libhb: layout planning, device allocation, coefficient
// tables, launch groups (one or many solves per launch), hipGraph step
// replay, the autotuner and the C ABI declared in include/hb.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/hb.h"
#include "hb_internal.h"

using namespace hb;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(HB_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));            \
    } while (0)

#define HB_TRY(expr)                                  \
    do {                                              \
        int r_ = (expr);                              \
        if (r_ != HB_OK) return r_;                   \
    } while (0)

int from_hip(int e, const char* what) {
    if (e == 0) return HB_OK;
    return fail(HB_E_HIP, "%s: %s", what, hipGetErrorString((hipError_t)e));
}

long long round_up(long long v, long long m) { return (v + m - 1) / m * m; }

// Step counts and indices are capped so that step arithmetic and the
// coefficient table's size cannot overflow (2^40 steps would already need a
// 35 TB table).
constexpr long long MAX_STEPS = 1LL << 40;

// ---- device memory: hipMalloc, or the caller's allocator (hb_set_allocator) ----

struct AllocHook {
    hb_alloc_fn alloc = nullptr;
    hb_free_fn release = nullptr;
    void* ctx = nullptr;
};
struct Hooked {
    AllocHook hook;  // the allocator that made it, and must free it
    size_t bytes;
    hipStream_t stream;  // the stream it was allocated for
};
std::mutex g_alloc_mu;
AllocHook g_hook;
std::unordered_map<void*, Hooked> g_hooked;

// device allocation of `bytes` for work on `stream`; a failure is HB_E_NOMEM
// and leaves no sticky HIP error
int dev_alloc(void** p, size_t bytes, const char* what, hipStream_t stream) {
    *p = nullptr;
    AllocHook h;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        h = g_hook;
    }
    if (h.alloc) {
        void* q = h.alloc(h.ctx, bytes, (void*)stream);
        if (!q) return fail(HB_E_NOMEM, "%s (%zu bytes): the installed allocator returned NULL", what, bytes);
        if ((uintptr_t)q % 256 != 0) {
            h.release(h.ctx, q, bytes);
            return fail(HB_E_NOMEM, "%s: the installed allocator returned memory not aligned to 256 bytes",
                        what);
        }
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        g_hooked[q] = Hooked{h, bytes, stream};
        *p = q;
        return HB_OK;
    }
    if (hipMalloc(p, bytes) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(HB_E_NOMEM, "%s (%zu bytes): device allocation failed", what, bytes);
    }
    return HB_OK;
}

// free what dev_alloc returned (NULL-safe) through the allocator that made
// it.  Memory from an installed allocator is handed back only once the stream
// it was allocated for has drained (hipFree waits for the device by itself).
void dev_free(void* p) {
    if (!p) return;
    Hooked rec{};
    bool hooked = false;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        auto it = g_hooked.find(p);
        if (it != g_hooked.end()) {
            rec = it->second;
            hooked = true;
            g_hooked.erase(it);
        }
    }
    if (hooked) {
        (void)hipStreamSynchronize(rec.stream);
        rec.hook.release(rec.hook.ctx, p, rec.bytes);
    } else {
        (void)hipFree(p);
    }
}

// ---- layout ------------------------------------------------------------------

// Schemes (one launch per RK4 step, per stage pair or per stage; bitwise-equal
// results).  The whole-step kernel keeps G1..G3 on chip, so its solves do not
// allocate them.
enum Scheme { SCHEME_STEP = 0, SCHEME_PAIRS = 1, SCHEME_STAGES = 2 };

int scheme_of(uint32_t flags) {
    if (flags & HB_STAGEWISE) return SCHEME_STAGES;
    if (flags & HB_PAIRWISE) return SCHEME_PAIRS;
    return SCHEME_STEP;
}

// Device state of a solve, as views (index into Solve::f): 0, 1 Y_phi
// (ping-pong by step parity), 2, 3 Y_psi, 4..6 G1..G3, 7, 8 the FP32 low
// parts of phi and psi (FP32c; see lo_view).
//  - whole-step solves keep a cell's state in one 16-byte slot, one field per
//    parity: (phi, psi) in FP64 (cs = 2), (phi hi, psi hi, phi lo, psi lo) in
//    FP32c (cs = 4); views 2, 3 are views 0, 1 plus one element, the low
//    parts views 0, 1 plus two and three elements; no G;
//  - stage-pair and per-stage solves keep one field per view (cs = 1),
//    G1..G3 included, and one low-part field per quantity (updated in place).
bool field_used(int k, int precision, int scheme) {
    if (k >= 4 && k <= 6) return scheme != SCHEME_STEP;
    if (k >= 7) return precision == HB_F32C;
    return true;
}

struct Layout {
    int nx, ny, nz;
    size_t esz;             // bytes per element
    int cs;                 // elements per cell (2 or 4: whole-step state slot, 1: separate fields)
    long long sy, sz;       // row / plane pitch (cells)
    long long origin_off;   // cells from field start to interior (0,0,0)
    long long field_cells;  // cells per field (a multiple of 256 bytes)
    int nfields;            // fields allocated: 2 whole-step, 7 or 9 separate
    size_t cell_bytes() const { return esz * (size_t)cs; }
};

Layout plan_layout(const hb_config& c, int scheme) {
    Layout L;
    L.nx = c.n[0];
    L.ny = c.n[1];
    L.nz = c.n[2];
    L.esz = c.precision == HB_F32C ? 4 : 8;
    L.cs = scheme == SCHEME_STEP ? (c.precision == HB_F32C ? 4 : 2) : 1;
    const long long line = 128 / (long long)L.cell_bytes();  // cells per 128-byte line
    L.sy = round_up((long long)L.nx + 4, line);
    L.sz = L.sy * ((long long)L.ny + 4);
    // cell (0, y, z) starts a 128-byte line, so rows of tiles that start on a
    // multiple of a line's cells are stored as whole lines (measured: FP32c
    // -4 to -6% at 512^3 against aligning cell (-2, y, z), FP64 -0.5 to -2%)
    L.origin_off = 2 * L.sz + 2 * L.sy + line;
    const long long last = L.origin_off + ((long long)L.nz + 1) * L.sz + ((long long)L.ny + 1) * L.sy +
                           L.nx + 2;
    L.field_cells = round_up(last, 256 / (long long)L.cell_bytes());
    if (L.cs > 1) {
        L.nfields = 2;
    } else {
        L.nfields = 0;
        for (int k = 0; k < 9; ++k) L.nfields += field_used(k, c.precision, scheme) ? 1 : 0;
    }
    return L;
}

size_t field_bytes(const Layout& L) { return (size_t)L.field_cells * L.cell_bytes(); }

int validate(const hb_config* c) {
    if (!c) return fail(HB_E_ARG, "config is NULL");
    for (int d = 0; d < 3; ++d) {
        if (c->n[d] < 1) return fail(HB_E_ARG, "n[%d] = %d must be >= 1", d, c->n[d]);
        if (!(c->hi[d] > c->lo[d]) || !std::isfinite(c->hi[d] - c->lo[d]))
            return fail(HB_E_ARG, "box axis %d must have hi > lo", d);
    }
    if ((long long)c->n[0] * c->n[1] * c->n[2] > (1LL << 40)) return fail(HB_E_ARG, "grid too large");
    if (!std::isfinite(c->mu2) || !std::isfinite(c->lambda) || !std::isfinite(c->inv_L2) ||
        !std::isfinite(c->t0))
        return fail(HB_E_ARG, "coefficients must be finite");
    if (!(c->dt > 0) || !std::isfinite(c->dt)) return fail(HB_E_ARG, "dt must be > 0");
    if (c->inv_L2 < 0) return fail(HB_E_ARG, "inv_L2 must be >= 0");
    if (c->precision != HB_F64 && c->precision != HB_F32C) return fail(HB_E_ARG, "bad precision");
    if ((c->flags & HB_BC_PERIODIC) && scheme_of(c->flags) != SCHEME_STEP)
        return fail(HB_E_ARG, "periodic boundaries need the whole-step scheme");
    if (scheme_of(c->flags) == SCHEME_STEP) {
        // the whole-step kernel addresses a plane with 32-bit byte offsets
        const Layout L = plan_layout(*c, SCHEME_STEP);
        if ((double)L.sz * (double)L.cell_bytes() >= 2147483648.0)
            return fail(HB_E_ARG, "an x-y plane (%lld x %lld padded cells of %zu bytes) must be under 2 GiB",
                        L.sy, (long long)c->n[1] + 4, L.cell_bytes());
    }
    if (!(c->flags & HB_ALLOW_UNSTABLE)) {
        // RK4 is stable on the imaginary axis up to |z| = 2 sqrt(2); -Lap_h has
        // spectral radius sum_d 16/(3 h_d^2) (symbol (1-cos)(7-cos)/3 <= 16/3)
        double rho = 0;
        for (int d = 0; d < 3; ++d) {
            const double h = (c->hi[d] - c->lo[d]) / c->n[d];
            rho += 16.0 / (3.0 * h * h);
        }
        const double c0 = c->inv_L2 * std::exp(-2.0 * c->t0);
        if (c->dt * std::sqrt(c0 * rho) > 2.0 * std::sqrt(2.0))
            return fail(HB_E_CFL, "dt = %g exceeds the RK4 stability limit %g", c->dt,
                        2.0 * std::sqrt(2.0) / std::sqrt(c0 * rho));
    }
    return HB_OK;
}

// ---- one solve -----------------------------------------------------------------

struct Solve {
    hb_config cfg{};
    Layout L{};
    char* mem = nullptr;          // all fields, one allocation
    void* f[9] = {};              // views: phi0, phi1, psi0, psi1, G1, G2, G3, lo_phi, lo_psi
                                  // (NULL where not allocated; lo_view gives the low parts)
    double* ctab = nullptr;       // device c(t) table, 4 per step
    long long ctab_steps = 0;
    long long nstep = 0;          // host mirror of the device counter
    long long target = 0;
    bool has_initial = false;
    double h[3]{};

    ~Solve() {
        dev_free(mem);
        dev_free(ctab);
    }
    int prec() const { return cfg.precision; }
    // FP32c low parts of phi (k = 0) or psi (k = 1) of the state at step
    // parity par: inside the whole-step state slot, else the in-place field
    float* lo_view(int k, int par) const {
        if (L.cs == 4) return (float*)f[par] + 2 + k;
        return (float*)f[7 + k];
    }
};

// steps the coefficient table holds when it must cover `need` steps
long long ctab_capacity(long long need, long long have) {
    long long cap = std::max<long long>(4096, have);
    while (cap < need) cap *= 2;
    return cap;
}

// device bytes of one solve whose coefficient table covers `steps` steps
size_t solve_footprint(const hb_config& c, int scheme, long long steps) {
    const Layout L = plan_layout(c, scheme);
    return field_bytes(L) * (size_t)L.nfields +
           (size_t)ctab_capacity(steps, 0) * 4 * sizeof(double);
}

// zero a solve's whole allocation on `stream` (the halo then stays zero for
// the life of the solve) and, with HB_DEBUG_POISON, fill every stored cell
// outside the interior and its halo with NaN
int solve_clear(Solve& s, hipStream_t stream) {
    const size_t fb = field_bytes(s.L);
    HIP_TRY(hipMemsetAsync(s.mem, 0, fb * (size_t)s.L.nfields, stream));
    if (s.cfg.flags & HB_DEBUG_POISON) {
        const long long corner = s.L.origin_off - 2 * s.L.sz - 2 * s.L.sy - 2;
        for (int k = 0; k < s.L.nfields; ++k)
            HB_TRY(from_hip(launch_poison(s.mem + fb * (size_t)k, s.L.field_cells, (int)s.L.esz, s.L.cs,
                                          corner, s.L.sy, s.L.sz, s.L.nx, s.L.nz, stream),
                            "poison"));
    }
    return HB_OK;
}

// configuration, layout and field views of a solve over its allocation
void solve_views(Solve& s, const hb_config& c, int scheme) {
    s.cfg = c;
    s.L = plan_layout(c, scheme);
    for (int d = 0; d < 3; ++d) s.h[d] = (c.hi[d] - c.lo[d]) / c.n[d];
    for (void*& v : s.f) v = nullptr;
    const size_t fb = field_bytes(s.L);
    const size_t org = (size_t)s.L.origin_off * s.L.cell_bytes();
    if (s.L.cs > 1) {
        for (int par = 0; par < 2; ++par) {
            s.f[par] = s.mem + fb * (size_t)par + org;
            s.f[2 + par] = (char*)s.f[par] + s.L.esz;
        }
    } else {
        int slot = 0;
        for (int k = 0; k < 9; ++k)
            if (field_used(k, c.precision, scheme)) s.f[k] = s.mem + fb * (size_t)slot++ + org;
    }
}

int solve_alloc(Solve& s, const hb_config& c, int scheme, hipStream_t stream) {
    const Layout L = plan_layout(c, scheme);
    HB_TRY(dev_alloc((void**)&s.mem, field_bytes(L) * (size_t)L.nfields, "solve state", stream));
    solve_views(s, c, scheme);
    return solve_clear(s, stream);
}

// c(t) = inv_L2 exp(-2 t) at the stage times t_n, t_n + dt/2, t_n + dt/2,
// t_n + dt with t_n = t0 + n dt (section 2.1 eq. (rhs) and the RK4 stages)
void fill_ctab(const hb_config& c, long long n0, long long n1, std::vector<double>& out) {
    out.resize((size_t)(n1 - n0) * 4);
    for (long long n = n0; n < n1; ++n) {
        const double t = c.t0 + (double)n * c.dt;
        double* o = &out[(size_t)(n - n0) * 4];
        o[0] = std::exp(-2.0 * t) * c.inv_L2;
        o[1] = std::exp(-2.0 * (t + c.dt / 2.0)) * c.inv_L2;
        o[2] = o[1];
        o[3] = std::exp(-2.0 * (t + c.dt)) * c.inv_L2;
    }
}

// make the device table cover steps [0, need); grows by doubling (synchronous)
int ensure_ctab(Solve& s, long long need, hipStream_t stream, bool* reallocated) {
    if (reallocated) *reallocated = false;
    if (need <= s.ctab_steps) return HB_OK;
    const long long cap = ctab_capacity(need, s.ctab_steps);
    // the table holds 4 doubles per step from step 0, so its size follows the
    // caller's step count: a count too large for host memory is HB_E_NOMEM
    std::vector<double> host;
    try {
        fill_ctab(s.cfg, 0, cap, host);
    } catch (const std::bad_alloc&) {
        return fail(HB_E_NOMEM, "coefficient table for %lld steps: host allocation failed", cap);
    }
    double* nt = nullptr;
    HB_TRY(dev_alloc((void**)&nt, host.size() * sizeof(double), "coefficient table", stream));
    hipError_t e = hipStreamSynchronize(stream);
    if (e == hipSuccess)
        e = hipMemcpy(nt, host.data(), host.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        dev_free(nt);
        return fail(HB_E_HIP, "coefficient table upload: %s", hipGetErrorString(e));
    }
    dev_free(s.ctab);
    s.ctab = nt;
    s.ctab_steps = cap;
    if (reallocated) *reallocated = true;
    return HB_OK;
}

SolveDesc make_desc(const Solve& s) {
    SolveDesc d;
    std::memset(&d, 0, sizeof d);
    d.y_phi[0] = s.f[0];
    d.y_phi[1] = s.f[1];
    d.y_psi[0] = s.f[2];
    d.y_psi[1] = s.f[3];
    d.g[0] = s.f[4];
    d.g[1] = s.f[5];
    d.g[2] = s.f[6];
    d.lo_phi = (float*)s.f[7];  // separate fields only (the whole-step slot holds its own)
    d.lo_psi = (float*)s.f[8];
    d.ctab = s.ctab;
    d.sy = s.L.sy;
    d.sz = s.L.sz;
    d.cs = s.L.cs;
    d.periodic = (s.cfg.flags & HB_BC_PERIODIC) ? 1 : 0;
    d.nx = s.L.nx;
    d.ny = s.L.ny;
    d.nz = s.L.nz;
    d.prec = s.cfg.precision;
    double sum = 0;
    for (int a = 0; a < 3; ++a) {
        const double ih2 = 1.0 / (s.h[a] * s.h[a]);
        sum += ih2;
        d.w1[a] = 4.0 / 3.0 * ih2;
        d.w2[a] = -1.0 / 12.0 * ih2;
    }
    d.w0 = -5.0 / 2.0 * sum;
    d.mu2 = s.cfg.mu2;
    d.lambda = s.cfg.lambda;
    d.dt = s.cfg.dt;
    d.hdt = s.cfg.dt / 2.0;
    d.dt6 = s.cfg.dt / 6.0;
    d.nstep = s.nstep;
    d.target = s.target;
    return d;
}

int upload_state(Solve& s, int slot_phi, int slot_psi, const void* phi, const void* psi, int mem,
                 int dtype, hipStream_t stream) {
    if (dtype != HB_DTYPE_F64 && dtype != HB_DTYPE_F32) return fail(HB_E_ARG, "bad dtype");
    if (mem != HB_HOST && mem != HB_DEVICE) return fail(HB_E_ARG, "bad memory kind");
    const long long cnt = (long long)s.L.nx * s.L.ny * s.L.nz;
    const size_t bytes = (size_t)cnt * (dtype == HB_DTYPE_F64 ? 8 : 4);
    const void* src[2] = {phi, psi};
    void* hi[2] = {s.f[slot_phi], s.f[slot_psi]};
    float* lo[2] = {s.lo_view(0, slot_phi & 1), s.lo_view(1, slot_phi & 1)};
    for (int k = 0; k < 2; ++k) {
        const void* dsrc = src[k];
        void* staged = nullptr;
        if (src[k] && mem == HB_HOST) {
            HB_TRY(dev_alloc(&staged, bytes, "staging buffer", stream));
            hipError_t e = hipMemcpyAsync(staged, src[k], bytes, hipMemcpyHostToDevice, stream);
            if (e != hipSuccess) {
                dev_free(staged);
                return fail(HB_E_HIP, "H2D copy failed: %s", hipGetErrorString(e));
            }
            dsrc = staged;
        }
        int r = launch_unpack(s.prec(), dtype, dsrc, s.L.nx, s.L.ny, s.L.nz, s.L.sy, s.L.sz, s.L.cs,
                              hi[k], lo[k], stream);
        if (staged) {
            // the host copy and the unpack must finish before the staging buffer goes
            hipError_t e = hipStreamSynchronize(stream);
            dev_free(staged);
            if (e != hipSuccess) return fail(HB_E_HIP, "sync failed: %s", hipGetErrorString(e));
        }
        HB_TRY(from_hip(r, "unpack"));
    }
    return HB_OK;
}

int download_state(Solve& s, void* phi, void* psi, int mem, int dtype, hipStream_t stream) {
    if (dtype != HB_DTYPE_F64 && dtype != HB_DTYPE_F32) return fail(HB_E_ARG, "bad dtype");
    if (mem != HB_HOST && mem != HB_DEVICE) return fail(HB_E_ARG, "bad memory kind");
    const int par = (int)(s.nstep & 1);
    const long long cnt = (long long)s.L.nx * s.L.ny * s.L.nz;
    const size_t bytes = (size_t)cnt * (dtype == HB_DTYPE_F64 ? 8 : 4);
    void* dst[2] = {phi, psi};
    const void* hi[2] = {s.f[0 + par], s.f[2 + par]};
    const float* lo[2] = {s.lo_view(0, par), s.lo_view(1, par)};
    for (int k = 0; k < 2; ++k) {
        if (!dst[k]) continue;
        if (mem == HB_DEVICE) {
            HB_TRY(from_hip(launch_pack(s.prec(), dtype, dst[k], s.L.nx, s.L.ny, s.L.nz, s.L.sy, s.L.sz,
                                        s.L.cs, hi[k], lo[k], stream),
                            "pack"));
        } else {
            void* staged = nullptr;
            HB_TRY(dev_alloc(&staged, bytes, "staging buffer", stream));
            int r = launch_pack(s.prec(), dtype, staged, s.L.nx, s.L.ny, s.L.nz, s.L.sy, s.L.sz,
                                s.L.cs, hi[k], lo[k], stream);
            hipError_t e = r ? (hipError_t)r : hipMemcpyAsync(dst[k], staged, bytes,
                                                              hipMemcpyDeviceToHost, stream);
            hipError_t e2 = hipStreamSynchronize(stream);
            dev_free(staged);
            if (e != hipSuccess) return fail(HB_E_HIP, "D2H failed: %s", hipGetErrorString(e));
            if (e2 != hipSuccess) return fail(HB_E_HIP, "sync failed: %s", hipGetErrorString(e2));
        }
    }
    HIP_TRY(hipStreamSynchronize(stream));
    return HB_OK;
}

// ---- launch group: all solves of one precision share each launch -----------

constexpr int DEFAULT_BY = 16;
// Whole-step groups of several solves (batches, the serving pool) default to
// 36 x 28 regions with 128-plane marches: the batch autotuner's choice on a
// 64-solve batch of 64^3-192^3 grids (FP64 1.10x, FP32c 1.05x over 64 x 16
// regions with 32-plane marches), and on the served stream of mixed
// requests 1.11x the completed solves per second of that older default.
constexpr int MULTI_BY = 8;

int default_zc(const Layout& L, int by) {
    // z-marches of 64 planes (4 warm-up planes = 6% extra stencil reads), cut
    // shorter only while one solve would give fewer than 256 tiles (one
    // 16-wave block per CU); measured best on 256^3 and 512^3 grids
    const long long xy = (long long)((L.nx + TILE_X - 1) / TILE_X) * ((L.ny + by - 1) / by);
    long long zc = std::min<long long>(L.nz, 64);
    while (zc > 8 && xy * ((L.nz + zc - 1) / zc) < 256) zc = (zc + 1) / 2;
    return (int)std::max<long long>(1, zc);
}

// Pinned host staging for asynchronous uploads: a buffer from hipHostMalloc
// (grown on demand) and an event recorded after the last copy that read or
// wrote it, so it is refilled only once that copy has finished (a wait on
// the copy alone, not on the stream's kernels).
struct Staging {
    void* buf = nullptr;
    size_t cap = 0;
    hipEvent_t used = nullptr;
    ~Staging() { release(); }
    void release() {
        if (used) (void)hipEventSynchronize(used);
        if (buf) (void)hipHostFree(buf);
        if (used) (void)hipEventDestroy(used);
        buf = nullptr;
        used = nullptr;
        cap = 0;
    }
    // a buffer of at least `bytes` bytes that no pending copy uses
    int get(size_t bytes, void** out) {
        if (used) HIP_TRY(hipEventSynchronize(used));
        if (bytes > cap) {
            if (buf) (void)hipHostFree(buf);
            buf = nullptr;
            cap = 0;
            const size_t want = std::max<size_t>(bytes, 1 << 16);
            if (hipHostMalloc(&buf, want, hipHostMallocDefault) != hipSuccess) {
                buf = nullptr;
                (void)hipGetLastError();
                return fail(HB_E_NOMEM, "pinned staging (%zu bytes): host allocation failed", want);
            }
            cap = want;
        }
        if (!used) HIP_TRY(hipEventCreateWithFlags(&used, hipEventDisableTiming));
        *out = buf;
        return HB_OK;
    }
    // mark the copies enqueued on `stream` so far as the buffer's last use
    int mark(hipStream_t stream) {
        HIP_TRY(hipEventRecord(used, stream));
        return HB_OK;
    }
};

struct Group {
    int prec = HB_F64;
    int scheme = SCHEME_STEP;  // 1 whole-step, 2 stage-pair or 4 per-stage launches per step
    int by = DEFAULT_BY;
    int zc = 0;  // 0 = default per solve
    std::vector<Solve*> members;
    SolveDesc* d_desc = nullptr;
    int desc_cap = 0;
    Tile* d_tiles = nullptr;
    int tile_cap = 0;
    int ntiles = 0;
    bool periodic = false;  // some member has periodic boundaries
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int graph_k = 0;
    Staging staging;  // descriptor and tile-table uploads

    ~Group() { release(); }
    void drop_graph() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
        graph_k = 0;
    }
    void release() {
        drop_graph();
        staging.release();
        dev_free(d_desc);
        dev_free(d_tiles);
        d_desc = nullptr;
        d_tiles = nullptr;
        desc_cap = tile_cap = 0;
    }
};

int device_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
    }
    return cus;
}

// whole-step kernel region shape (STEP_SHAPES): by = 8 selects 36 x 28
// regions (32 x 24 tiles), by = 16 selects 64 x 16 regions (60 x 12 tiles),
// by = 11 selects 68 x 15 regions (64 x 11 tiles) and by = 20 selects 36 x 20
// regions (32 x 16 tiles); the last two are whole-step shapes only.
int step_shape(int by) { return by == 16 ? 1 : by == 11 ? 2 : by == 20 ? 3 : 0; }
bool valid_by(int by, int scheme) {
    return by == 8 || by == 16 || ((by == 11 || by == 20) && scheme == SCHEME_STEP);
}

// z-march length for one solve.  Blocks run in rounds of (CUs x blocks per
// CU); a march of zc planes costs about zc + 4 planes (warm-up) rounded up to
// the unroll of 6, plus a fixed start-up.  Pick the zc that minimises
// rounds x cost per block, so the last round is not mostly empty and the
// warm-up planes stay a small share.  Groups of several solves use fixed
// marches (their many tiles already fill the rounds): 128 planes with the
// 36 x 28 regions they default to, else 32.
struct ZPlan {
    int zc;
    double cost;  // rounds x planes per block, in plane units
};
ZPlan plan_zc_step(const Layout& L, int by) {
    const StepShape sh = STEP_SHAPES[step_shape(by)];
    const long long tx = sh.rx - 4, ty = sh.ry - 4;
    const long long xy = ((L.nx + tx - 1) / tx) * ((L.ny + ty - 1) / ty);
    const long long slots = (long long)device_cus() * sh.blocks_per_cu;
    int best = std::min(L.nz, 32);
    double best_cost = 1e300;
    for (int zc = std::min(L.nz, 8); zc <= L.nz; ++zc) {
        const long long chunks = (L.nz + zc - 1) / zc;
        const long long rounds = (xy * chunks + slots - 1) / slots;
        const int planes = (zc + 4 + 5) / 6 * 6;
        const double cost = (double)rounds * (planes + 3);
        if (cost < best_cost - 1e-9) {
            best_cost = cost;
            best = zc;
        }
    }
    return {best, best_cost};
}

int default_zc_step(const Layout& L, int by, int nmembers) {
    if (nmembers > 1) return std::min(L.nz, by == MULTI_BY ? 128 : 32);
    return plan_zc_step(L, by).zc;
}

// Default region shape of a single solve.  First 36 x 20, where its march
// cost weighted by the work of one of its planes (stage-1+2 region plus
// tile), times a measured per-work penalty of its three-waves-per-SIMD blocks
// (1.16 FP64, 1.12 FP32c), is at least 2% below the weighted costs of
// 68 x 15 and 36 x 28: on grids whose x-y tiles and z-chunks fill whole
// rounds of the device in 32 x 16 tiles but not in the others, e.g. 96^3,
// 160^3 and 256^3 (FP64 -9%, -1.5%, -5%; FP32c -8%, -4%, -9.5% against the
// next best shape), and on none of 128^3, 192^3, 224^3, 288^3, 320^3,
// 384^3, 512^3 (where it loses 3-11%).  Else 64 x 16, or 68 x 15 where the
// march model gives it at least 3% (FP64) / 5% (FP32c) fewer block-planes,
// or 36 x 28 where the model gives that at least 8% (FP64) / 15% (FP32c)
// fewer block-planes than the better of the other two.  The model overstates
// the differences (a block's cost also depends on its shape), so the margins
// are set from measurements on eight grids (192^3 to 512^3, a 512 x 512 x 64
// slab; both precisions; two devices): the rule picks the fastest shape or
// one within 2% of it in 31 of the 32 cases (192^3 FP32c: 4%), e.g. 68 x 15
// on 512^3, 36 x 28 on 384^3 (FP64 -8% against 64 x 16).  A later sweep of
// the whole rule over 14 cubes (96^3 to 512^3, both precisions) found its
// pick the fastest shape or within 2.8% of it in all 28 cases.  Groups of
// several solves default to 36 x 28 regions instead (MULTI_BY).
int default_step_by(const Layout& L, int precision) {
    const double c16 = plan_zc_step(L, 16).cost, c11 = plan_zc_step(L, 11).cost;
    const double c8 = plan_zc_step(L, 8).cost, c20 = plan_zc_step(L, 20).cost;
    const bool f32c = precision == HB_F32C;
    auto work = [](int by, double cost) {
        const StepShape sh = STEP_SHAPES[step_shape(by)];
        return cost * (sh.rx * sh.ry + (sh.rx - 4) * (sh.ry - 4));
    };
    if (work(20, c20) * (f32c ? 1.12 : 1.16) <= 0.98 * std::min(work(11, c11), work(8, c8))) return 20;
    if (c8 <= (f32c ? 0.85 : 0.92) * std::min(c16, c11)) return 8;
    return c11 <= (f32c ? 0.95 : 0.97) * c16 ? 11 : 16;
}

void make_tiles(const Solve& s, int solve_index, int scheme, int by, int zc_req, int nmembers,
                std::vector<Tile>& out) {
    const Layout& L = s.L;
    const int tx = scheme == SCHEME_STEP ? STEP_SHAPES[step_shape(by)].rx - 4 : TILE_X;
    const int ty = scheme == SCHEME_STEP ? STEP_SHAPES[step_shape(by)].ry - 4 : by;
    const int zc = zc_req > 0 ? zc_req
                              : (scheme == SCHEME_STEP ? default_zc_step(L, by, nmembers)
                                                       : default_zc(L, by));
    // z-chunk major, then y, then x: consecutive tiles are spatial neighbours,
    // and the XCD remap hands each XCD a contiguous run of them
    for (int z0 = 0; z0 < L.nz; z0 += zc)
        for (int y0 = 0; y0 < L.ny; y0 += ty)
            for (int x0 = 0; x0 < L.nx; x0 += tx) {
                Tile t;
                std::memset(&t, 0, sizeof t);
                t.solve = solve_index;
                t.x0 = x0;
                t.y0 = y0;
                t.z0 = z0;
                t.z1 = std::min(L.nz, z0 + zc);
                out.push_back(t);
            }
}

// (re)upload descriptors and the tile table; invalidates any captured graph.
// The upload is ordered on `stream` after the work already enqueued there
// (which may still read the old tables) and does not wait for it: the host
// copies go through the group's pinned staging.  Device tables grow by
// doubling, so a growing group rarely replaces them (a replacement frees
// the old table, which waits for the device).
int group_rebuild(Group& g, hipStream_t stream) {
    g.drop_graph();
    std::vector<SolveDesc> descs;
    std::vector<Tile> tiles;
    for (size_t i = 0; i < g.members.size(); ++i) {
        descs.push_back(make_desc(*g.members[i]));
        make_tiles(*g.members[i], (int)i, g.scheme, g.by, g.zc, (int)g.members.size(), tiles);
    }
    if ((int)descs.size() > g.desc_cap) {
        const int old_cap = g.desc_cap;
        dev_free(g.d_desc);
        g.d_desc = nullptr;
        g.desc_cap = 0;
        const int cap = std::max<int>(std::max<int>(1, (int)descs.size()), 2 * old_cap);
        HB_TRY(dev_alloc((void**)&g.d_desc, cap * sizeof(SolveDesc), "descriptors", stream));
        g.desc_cap = cap;
    }
    if ((int)tiles.size() > g.tile_cap) {
        const int old_cap = g.tile_cap;
        dev_free(g.d_tiles);
        g.d_tiles = nullptr;
        g.tile_cap = 0;
        const int cap = std::max<int>(std::max<int>(1, (int)tiles.size()), 2 * old_cap);
        HB_TRY(dev_alloc((void**)&g.d_tiles, cap * sizeof(Tile), "tile table", stream));
        g.tile_cap = cap;
    }
    const size_t db = descs.size() * sizeof(SolveDesc), tb = tiles.size() * sizeof(Tile);
    const size_t toff = (size_t)round_up((long long)db, 256);
    if (db + tb > 0) {
        void* h = nullptr;
        HB_TRY(g.staging.get(toff + tb, &h));
        if (db) std::memcpy(h, descs.data(), db);
        if (tb) std::memcpy((char*)h + toff, tiles.data(), tb);
        if (db) HIP_TRY(hipMemcpyAsync(g.d_desc, h, db, hipMemcpyHostToDevice, stream));
        if (tb) HIP_TRY(hipMemcpyAsync(g.d_tiles, (char*)h + toff, tb, hipMemcpyHostToDevice, stream));
        HB_TRY(g.staging.mark(stream));
    }
    g.ntiles = (int)tiles.size();
    g.periodic = false;
    for (Solve* m : g.members) g.periodic = g.periodic || (m->cfg.flags & HB_BC_PERIODIC);
    return HB_OK;
}

int kernels_per_step(const Group& g) {
    return g.scheme == SCHEME_STAGES ? 4 : g.scheme == SCHEME_PAIRS ? 2 : 1;
}

// kernel i of one step (the whole step, stage pair i, or stage i+1)
int launch_step_kernel(const Group& g, int i, long long kstep, hipStream_t stream) {
    if (g.scheme == SCHEME_STEP)
        return from_hip(launch_step(g.prec, step_shape(g.by), g.d_desc, g.d_tiles, g.ntiles, kstep,
                                    g.periodic, stream),
                        "step launch");
    if (g.scheme == SCHEME_STAGES)
        return from_hip(launch_stage(g.prec, i + 1, g.by, g.d_desc, g.d_tiles, g.ntiles, kstep, stream),
                        "stage launch");
    return from_hip(launch_pair(g.prec, i, g.by, g.d_desc, g.d_tiles, g.ntiles, kstep, stream),
                    "stage-pair launch");
}

int enqueue_steps(Group& g, long long k, hipStream_t stream) {
    for (long long j = 0; j < k; ++j)
        for (int i = 0; i < kernels_per_step(g); ++i) HB_TRY(launch_step_kernel(g, i, j, stream));
    return from_hip(launch_tick(g.d_desc, (int)g.members.size(), k, stream), "tick");
}

constexpr int GRAPH_STEPS = 16;

int capture_graph(Group& g, hipStream_t stream) {
    g.drop_graph();
    HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    int r = enqueue_steps(g, GRAPH_STEPS, stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(stream, &graph);
    if (r != HB_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return r;
    }
    if (e != hipSuccess) return fail(HB_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&g.gexec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(HB_E_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    g.graph = graph;
    g.graph_k = GRAPH_STEPS;
    return HB_OK;
}

// Advance every member of g by up to k steps; member targets must be set.
int group_step(Group& g, long long k, bool use_graph, hipStream_t stream) {
    if (g.members.empty() || k <= 0) return HB_OK;
    long long done = 0;
    if (use_graph && k >= GRAPH_STEPS) {
        if (!g.gexec) HB_TRY(capture_graph(g, stream));
        while (k - done >= GRAPH_STEPS) {
            HIP_TRY(hipGraphLaunch(g.gexec, stream));
            done += GRAPH_STEPS;
        }
    }
    if (k > done) HB_TRY(enqueue_steps(g, k - done, stream));
    for (Solve* s : g.members) s->nstep = std::min(s->nstep + k, s->target);
    return HB_OK;
}

int group_step_timed(Group& g, long long k, hipStream_t stream, double* stage_ms) {
    hipEvent_t ev[5] = {};
    int rc = HB_OK;
    for (int i = 0; i < 5 && rc == HB_OK; ++i) rc = from_hip(hipEventCreate(&ev[i]), "event create");
    double acc[4] = {0, 0, 0, 0};
    const int nk = kernels_per_step(g);
    for (long long j = 0; j < k && rc == HB_OK; ++j) {
        rc = from_hip(hipEventRecord(ev[0], stream), "event record");
        for (int i = 0; i < nk && rc == HB_OK; ++i) {
            rc = launch_step_kernel(g, i, 0, stream);
            if (rc == HB_OK) rc = from_hip(hipEventRecord(ev[i + 1], stream), "event record");
        }
        if (rc == HB_OK) rc = from_hip(launch_tick(g.d_desc, (int)g.members.size(), 1, stream), "tick");
        if (rc == HB_OK && hipEventSynchronize(ev[nk]) != hipSuccess) rc = fail(HB_E_HIP, "event sync");
        for (int st = 0; st < nk && rc == HB_OK; ++st) {
            float ms = 0;
            rc = from_hip(hipEventElapsedTime(&ms, ev[st], ev[st + 1]), "event elapsed");
            acc[st] += ms;
        }
        if (rc == HB_OK)
            for (Solve* s : g.members) s->nstep = std::min(s->nstep + 1, s->target);
    }
    for (int i = 0; i < 5; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (stage_ms)
        for (int i = 0; i < 4; ++i) stage_ms[i] = acc[i];
    return rc;
}

int set_targets(Group& g, long long extra, hipStream_t stream, bool* tables_moved) {
    // every member gets target = nstep + extra; tables must cover the target
    bool moved = false;
    for (size_t i = 0; i < g.members.size(); ++i) {
        Solve* s = g.members[i];
        const long long target = s->nstep + extra;
        bool re = false;
        HB_TRY(ensure_ctab(*s, target, stream, &re));
        s->target = target;
        moved = moved || re;
    }
    if (tables_moved) *tables_moved = moved;
    return HB_OK;
}

}  // namespace

// ---- C ABI: single solve -------------------------------------------------------

struct hb_solver {
    std::unique_ptr<Solve> s;
    Group g;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool built = false;
    double* d_partials = nullptr;
    double* d_diag = nullptr;
    int nparts = 0;
    unsigned* d_labels = nullptr;            // bubble count: one label per interior point
    unsigned long long* d_counts = nullptr;  // ... and its two set counts
    ~hb_solver() {
        g.release();
        dev_free(d_partials);
        dev_free(d_diag);
        dev_free(d_labels);
        dev_free(d_counts);
        s.reset();
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

extern "C" {

const char* hb_last_error(void) { return g_last_error.c_str(); }

int hb_set_allocator(hb_alloc_fn alloc, hb_free_fn release, void* ctx) {
    if ((alloc == nullptr) != (release == nullptr))
        return fail(HB_E_ARG, "give both an allocation and a release function, or neither");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_hook = AllocHook{alloc, release, alloc ? ctx : nullptr};
    return HB_OK;
}

int hb_default_tiling(const hb_config* cfg, int* by, int* zc) {
    g_last_error.clear();
    if (!by || !zc) return fail(HB_E_ARG, "NULL argument");
    HB_TRY(validate(cfg));
    const int scheme = scheme_of(cfg->flags);
    const Layout L = plan_layout(*cfg, scheme);
    if (scheme == SCHEME_STEP) {
        *by = default_step_by(L, cfg->precision);
        *zc = default_zc_step(L, *by, 1);
    } else {
        *by = DEFAULT_BY;
        *zc = default_zc(L, DEFAULT_BY);
    }
    return HB_OK;
}

size_t hb_footprint(const hb_config* cfg) {
    if (!cfg) return 0;
    hb_config c = *cfg;
    c.flags |= HB_ALLOW_UNSTABLE;
    if (validate(&c) != HB_OK) return 0;
    return solve_footprint(c, scheme_of(c.flags), 4096);
}

int hb_create(const hb_config* cfg, hb_solver** out) {
    g_last_error.clear();
    if (!out) return fail(HB_E_ARG, "out is NULL");
    *out = nullptr;
    HB_TRY(validate(cfg));
    auto h = std::make_unique<hb_solver>();
    if (cfg->stream) {
        h->stream = (hipStream_t)cfg->stream;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
        h->own_stream = true;
    }
    h->s = std::make_unique<Solve>();
    HB_TRY(solve_alloc(*h->s, *cfg, scheme_of(cfg->flags), h->stream));
    HB_TRY(ensure_ctab(*h->s, 4096, h->stream, nullptr));
    h->g.prec = cfg->precision;
    h->g.scheme = scheme_of(cfg->flags);
    h->g.by = h->g.scheme == SCHEME_STEP ? default_step_by(h->s->L, cfg->precision) : DEFAULT_BY;
    h->g.members.push_back(h->s.get());
    HIP_TRY(hipStreamSynchronize(h->stream));
    *out = h.release();
    return HB_OK;
}

static int solver_rebuild(hb_solver* h) {
    HB_TRY(group_rebuild(h->g, h->stream));
    h->built = true;
    return HB_OK;
}

int hb_set_state(hb_solver* h, const void* phi, const void* psi, int64_t n, int mem, int dtype) {
    if (!h) return fail(HB_E_ARG, "solver is NULL");
    if (!phi) return fail(HB_E_ARG, "phi is NULL");
    if (n < 0 || n > MAX_STEPS) return fail(HB_E_ARG, "step index must be in [0, 2^40]");
    Solve& s = *h->s;
    const int par = (int)(n & 1);
    HB_TRY(upload_state(s, 0 + par, 2 + par, phi, psi, mem, dtype, h->stream));
    s.nstep = n;
    s.target = n;
    s.has_initial = true;
    HB_TRY(ensure_ctab(s, n + 1, h->stream, nullptr));
    HB_TRY(solver_rebuild(h));
    return HB_OK;
}

int hb_set_initial(hb_solver* h, const void* phi0, const void* phi1, int mem, int dtype) {
    return hb_set_state(h, phi0, phi1, 0, mem, dtype);
}

// HB_TRACE set (and not "0") in the environment: hb_step times every kernel
// launch with events, waits for it, and prints one line per step to stderr
static bool trace_enabled() {
    static const bool on = [] {
        const char* e = std::getenv("HB_TRACE");
        return e && *e && std::strcmp(e, "0") != 0;
    }();
    return on;
}

int hb_step(hb_solver* h, int64_t nsteps) {
    if (!h) return fail(HB_E_ARG, "solver is NULL");
    if (nsteps < 0 || nsteps > MAX_STEPS) return fail(HB_E_ARG, "nsteps must be in [0, 2^40]");
    if (!h->s->has_initial) return fail(HB_E_STATE, "no initial data");
    if (nsteps == 0) return HB_OK;
    bool moved = false;
    HB_TRY(set_targets(h->g, nsteps, h->stream, &moved));
    if (moved || !h->built) HB_TRY(solver_rebuild(h));
    HB_TRY(from_hip(launch_set_target(h->g.d_desc, 0, h->s->target, h->stream), "set target"));
    if (trace_enabled()) {
        const int nk = kernels_per_step(h->g);
        for (long long j = 0; j < nsteps; ++j) {
            double ms[4];
            HB_TRY(group_step_timed(h->g, 1, h->stream, ms));
            std::fprintf(stderr, "hb_trace solver %p step %lld:", (void*)h, h->s->nstep);
            for (int k = 0; k < nk; ++k) std::fprintf(stderr, " %.4f ms", ms[k]);
            std::fprintf(stderr, "\n");
        }
        return HB_OK;
    }
    return group_step(h->g, nsteps, (h->s->cfg.flags & HB_USE_GRAPH) != 0, h->stream);
}

int hb_step_timed(hb_solver* h, int64_t nsteps, double* stage_ms) {
    if (!h) return fail(HB_E_ARG, "solver is NULL");
    if (nsteps < 0 || nsteps > MAX_STEPS) return fail(HB_E_ARG, "nsteps must be in [0, 2^40]");
    if (!h->s->has_initial) return fail(HB_E_STATE, "no initial data");
    bool moved = false;
    HB_TRY(set_targets(h->g, nsteps, h->stream, &moved));
    if (moved || !h->built) HB_TRY(solver_rebuild(h));
    HB_TRY(from_hip(launch_set_target(h->g.d_desc, 0, h->s->target, h->stream), "set target"));
    return group_step_timed(h->g, nsteps, h->stream, stage_ms);
}

int hb_read(hb_solver* h, void* phi, void* phi_t, int mem, int dtype) {
    if (!h) return fail(HB_E_ARG, "solver is NULL");
    if (!h->s->has_initial) return fail(HB_E_STATE, "no initial data");
    return download_state(*h->s, phi, phi_t, mem, dtype, h->stream);
}

int hb_time(const hb_solver* h, double* t, int64_t* n) {
    if (!h) return fail(HB_E_ARG, "solver is NULL");
    const Solve& s = *h->s;
    if (t) *t = s.cfg.t0 + (double)s.nstep * s.cfg.dt;
    if (n) *n = s.nstep;
    return HB_OK;
}

int hb_sync(hb_solver* h) {
    if (!h) return fail(HB_E_ARG, "solver is NULL");
    HIP_TRY(hipStreamSynchronize(h->stream));
    return HB_OK;
}

int hb_diagnostics(hb_solver* h, hb_diag* out) {
    if (!h || !out) return fail(HB_E_ARG, "NULL argument");
    Solve& s = *h->s;
    if (!s.has_initial) return fail(HB_E_STATE, "no initial data");
    if (!h->built) HB_TRY(solver_rebuild(h));
    if (!h->d_partials || !h->d_diag) {  // both, or again after a failed allocation
        dev_free(h->d_partials);
        h->d_partials = nullptr;
        h->nparts = diag_partials_needed(s.L.nx, s.L.ny, s.L.nz);
        HB_TRY(dev_alloc((void**)&h->d_partials, (size_t)h->nparts * DIAG_COUNT * sizeof(double),
                         "diagnostics partials", h->stream));
        HB_TRY(dev_alloc((void**)&h->d_diag, DIAG_COUNT * sizeof(double), "diagnostics", h->stream));
    }
    const double t = s.cfg.t0 + (double)s.nstep * s.cfg.dt;
    const double c = std::exp(-2.0 * t) * s.cfg.inv_L2;
    HB_TRY(from_hip(launch_diagnostics(s.prec(), h->g.d_desc, (int)(s.nstep & 1), c, h->d_partials,
                                       h->nparts, h->d_diag, h->stream),
                    "diagnostics"));
    double v[DIAG_COUNT];
    HIP_TRY(hipMemcpyAsync(v, h->d_diag, sizeof v, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    const double vol = s.h[0] * s.h[1] * s.h[2];
    out->t = t;
    out->step = s.nstep;
    out->integral = vol * v[DIAG_SUM_PHI];
    out->l2_phi = std::sqrt(vol * v[DIAG_SUM_PHI2]);
    out->l2_psi = std::sqrt(vol * v[DIAG_SUM_PSI2]);
    out->linf_phi = v[DIAG_MAX_PHI];
    out->linf_psi = v[DIAG_MAX_PSI];
    out->lap_max = c * v[DIAG_MAX_LAP];
    out->energy = vol * v[DIAG_ENERGY];
    out->nonfinite = (int64_t)v[DIAG_NONFINITE];
    out->negative = (int64_t)v[DIAG_NEGATIVE];
    if (out->nonfinite > 0) return fail(HB_E_NONFINITE, "state holds %lld non-finite values",
                                        (long long)out->nonfinite);
    return HB_OK;
}

int hb_bubbles(hb_solver* h, double eps, int64_t* negative_sets, int64_t* positive_sets) {
    if (!h || !negative_sets || !positive_sets) return fail(HB_E_ARG, "NULL argument");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(HB_E_ARG, "eps must be finite and >= 0");
    Solve& s = *h->s;
    if (!s.has_initial) return fail(HB_E_STATE, "no initial data");
    const long long pts = (long long)s.L.nx * s.L.ny * s.L.nz;
    if (pts >= (long long)0xffffffffLL)
        return fail(HB_E_ARG, "bubble count: %lld interior points (at most 2^32 - 2)", pts);
    if (!h->built) HB_TRY(solver_rebuild(h));
    if (!h->d_labels) {
        HB_TRY(dev_alloc((void**)&h->d_labels, (size_t)pts * sizeof(unsigned), "bubble labels", h->stream));
    }
    if (!h->d_counts) {
        HB_TRY(dev_alloc((void**)&h->d_counts, 2 * sizeof(unsigned long long), "bubble counts", h->stream));
    }
    HB_TRY(from_hip(launch_bubbles(s.prec(), h->g.d_desc, (int)(s.nstep & 1), eps, pts, h->d_labels,
                                   h->d_counts, h->stream),
                    "bubbles"));
    unsigned long long v[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(v, h->d_counts, sizeof v, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    *negative_sets = (int64_t)v[0];
    *positive_sets = (int64_t)v[1];
    return HB_OK;
}

int hb_set_tiling(hb_solver* h, int by, int zc) {
    if (!h) return fail(HB_E_ARG, "solver is NULL");
    if (!valid_by(by, h->g.scheme)) return fail(HB_E_ARG, "by must be 8 or 16 (or 11 or 20, whole-step scheme)");
    if (zc < 0) return fail(HB_E_ARG, "zc must be >= 0");
    h->g.by = by;
    h->g.zc = zc;
    h->built = false;
    return HB_OK;
}

int hb_destroy(hb_solver* h) {
    if (!h) return HB_OK;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    delete h;
    return HB_OK;
}

}  // extern "C"

// ---- autotuner -------------------------------------------------------------------

namespace {

// Cache key of a launch group: device architecture, precision, scheme and
// the grids it holds.  One solve: its grid ("NXxNYxNZ|m1"); a batch: the
// member count and a 64-bit FNV-1a hash of the members' sorted grid list,
// so batches with the same mix of sizes share an entry and others do not.
std::string tune_key(const Group& g) {
    hipDeviceProp_t p;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::string name = "unknown";
    if (hipGetDeviceProperties(&p, dev) == hipSuccess) name = p.gcnArchName;
    const Solve& s = *g.members[0];
    std::ostringstream k;
    k << name << "|prec" << s.cfg.precision << "|scheme" << scheme_of(s.cfg.flags) << "|";
    if (g.members.size() == 1) {
        k << s.L.nx << "x" << s.L.ny << "x" << s.L.nz << "|m1";
    } else {
        std::vector<std::array<int, 3>> dims;
        for (const Solve* m : g.members) dims.push_back({m->L.nx, m->L.ny, m->L.nz});
        std::sort(dims.begin(), dims.end());
        unsigned long long hsh = 1469598103934665603ULL;
        for (const auto& d : dims)
            for (int v : d)
                for (int b = 0; b < 4; ++b) {
                    hsh ^= (unsigned long long)((unsigned)v >> (8 * b) & 0xffu);
                    hsh *= 1099511628211ULL;
                }
        char hex[17];
        snprintf(hex, sizeof hex, "%016llx", hsh);
        k << "batch" << hex << "|m" << g.members.size();
    }
    return k.str();
}

// flat "key by zc" lines: simple, robust to partial writes
bool cache_lookup(const std::string& key, int* by, int* zc) {
    const char* path = std::getenv("HB_TUNE_CACHE");
    if (!path || !*path) return false;
    std::ifstream f(path);
    std::string k;
    int b, z;
    bool found = false;
    while (f >> k >> b >> z)
        if (k == key) {
            *by = b;
            *zc = z;
            found = true;
        }
    return found;
}

void cache_store(const std::string& key, int by, int zc) {
    const char* path = std::getenv("HB_TUNE_CACHE");
    if (!path || !*path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << by << " " << zc << "\n";
}

// Snapshot of the state fields of every member (current parity + low parts).
struct Snapshot {
    std::vector<void*> bufs;
    ~Snapshot() {
        for (void* b : bufs) dev_free(b);
    }
};

// the allocated fields that hold the state of step parity `par` (paired:
// the state field and, FP32c, the low parts; separate: phi, psi and the low
// parts), as field start addresses
std::vector<char*> state_fields(const Solve& s, int par) {
    const size_t org = (size_t)s.L.origin_off * s.L.cell_bytes();
    std::vector<int> views = {par};
    if (s.L.cs == 1) {
        views.push_back(2 + par);
        if (s.prec() == HB_F32C) {
            views.push_back(7);
            views.push_back(8);
        }
    }
    std::vector<char*> out;
    for (int v : views) out.push_back((char*)s.f[v] - org);
    return out;
}

int snapshot_take(Group& g, Snapshot& snap, hipStream_t stream) {
    for (Solve* s : g.members) {
        const size_t fb = field_bytes(s->L);
        for (char* base : state_fields(*s, (int)(s->nstep & 1))) {
            void* b = nullptr;
            HB_TRY(dev_alloc(&b, fb, "autotune snapshot", stream));
            snap.bufs.push_back(b);
            HIP_TRY(hipMemcpyAsync(b, base, fb, hipMemcpyDeviceToDevice, stream));
        }
    }
    return HB_OK;
}

int snapshot_restore(Group& g, Snapshot& snap, const std::vector<long long>& nsteps, hipStream_t stream) {
    size_t i = 0;
    for (size_t m = 0; m < g.members.size(); ++m) {
        Solve* s = g.members[m];
        s->nstep = nsteps[m];
        s->target = nsteps[m];
        const size_t fb = field_bytes(s->L);
        for (char* base : state_fields(*s, (int)(s->nstep & 1)))
            HIP_TRY(hipMemcpyAsync(base, snap.bufs[i++], fb, hipMemcpyDeviceToDevice, stream));
    }
    HIP_TRY(hipStreamSynchronize(stream));
    return HB_OK;
}

int group_autotune(Group& g, int trial_steps, hipStream_t stream, int* best_by, int* best_zc) {
    if (g.members.empty()) return fail(HB_E_STATE, "nothing to tune");
    const std::string key = tune_key(g);
    int cb = 0, cz = 0;
    if (cache_lookup(key, &cb, &cz)) {
        g.by = cb;
        g.zc = cz;
        HB_TRY(group_rebuild(g, stream));
        *best_by = cb;
        *best_zc = cz;
        return HB_OK;
    }
    std::vector<long long> saved;
    for (Solve* s : g.members) saved.push_back(s->nstep);
    Snapshot snap;
    HB_TRY(snapshot_take(g, snap, stream));
    std::vector<std::pair<int, int>> cand;
    int maxz = 0;
    for (Solve* s : g.members) maxz = std::max(maxz, s->L.nz);
    if (g.scheme == SCHEME_STEP) {
        for (int by : {16, 11, 8, 20})
            for (int zc : {0, 16, 32, 64, 128, 256})
                if (zc <= maxz) cand.push_back({by, zc});
    } else {
        for (int by : {8, 16})
            for (int zc : {0, 16, 32, 64, 128})
                if (zc <= maxz) cand.push_back({by, zc});
    }
    double best = 1e300;
    int bb = DEFAULT_BY, bz = 0;
    for (auto [by, zc] : cand) {
        HB_TRY(snapshot_restore(g, snap, saved, stream));
        g.by = by;
        g.zc = zc;
        bool moved;
        HB_TRY(set_targets(g, trial_steps + 1, stream, &moved));
        HB_TRY(group_rebuild(g, stream));
        double ms[4];
        HB_TRY(group_step_timed(g, 1, stream, ms));  // warm-up
        HB_TRY(group_step_timed(g, trial_steps, stream, ms));
        const double tot = ms[0] + ms[1] + ms[2] + ms[3];
        if (tot < best) {
            best = tot;
            bb = by;
            bz = zc;
        }
    }
    HB_TRY(snapshot_restore(g, snap, saved, stream));
    g.by = bb;
    g.zc = bz;
    HB_TRY(group_rebuild(g, stream));
    cache_store(key, bb, bz);
    *best_by = bb;
    *best_zc = bz;
    return HB_OK;
}

}  // namespace

extern "C" int hb_autotune(hb_solver* h, int trial_steps, int* by, int* zc) {
    if (!h) return fail(HB_E_ARG, "solver is NULL");
    if (!h->s->has_initial) return fail(HB_E_STATE, "no initial data");
    if (trial_steps < 1) return fail(HB_E_ARG, "trial_steps must be >= 1");
    int b = 0, z = 0;
    HB_TRY(group_autotune(h->g, trial_steps, h->stream, &b, &z));
    h->built = true;
    if (by) *by = b;
    if (zc) *zc = z;
    return HB_OK;
}

// ---- C ABI: batched form ---------------------------------------------------------

struct hb_batch {
    std::vector<std::unique_ptr<Solve>> solves;
    Group groups[2];  // by precision
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool built = false;
    bool use_graph = false;
    ~hb_batch() {
        groups[0].release();
        groups[1].release();
        solves.clear();
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

extern "C" {

int hb_batch_create(int count, const hb_config* cfgs, void* stream, hb_batch** out) {
    g_last_error.clear();
    if (!out) return fail(HB_E_ARG, "out is NULL");
    *out = nullptr;
    if (count < 1 || !cfgs) return fail(HB_E_ARG, "need count >= 1 configs");
    for (int i = 0; i < count; ++i) {
        HB_TRY(validate(&cfgs[i]));
        if (scheme_of(cfgs[i].flags) != scheme_of(cfgs[0].flags))
            return fail(HB_E_ARG, "solve %d selects another scheme than solve 0", i);
    }
    auto b = std::make_unique<hb_batch>();
    if (stream) {
        b->stream = (hipStream_t)stream;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
        b->own_stream = true;
    }
    b->groups[0].prec = HB_F64;
    b->groups[1].prec = HB_F32C;
    for (int i = 0; i < count; ++i) {
        auto s = std::make_unique<Solve>();
        HB_TRY(solve_alloc(*s, cfgs[i], scheme_of(cfgs[0].flags), b->stream));
        HB_TRY(ensure_ctab(*s, 4096, b->stream, nullptr));
        b->groups[cfgs[i].precision].members.push_back(s.get());
        if (i == 0)
            for (Group& g : b->groups) {
                g.scheme = scheme_of(cfgs[i].flags);
                g.by = g.scheme == SCHEME_STEP ? MULTI_BY : DEFAULT_BY;
            }
        b->use_graph = b->use_graph || (cfgs[i].flags & HB_USE_GRAPH);
        b->solves.push_back(std::move(s));
    }
    HIP_TRY(hipStreamSynchronize(b->stream));
    *out = b.release();
    return HB_OK;
}

int hb_batch_set_initial(hb_batch* b, int i, const void* phi0, const void* phi1, int mem, int dtype) {
    if (!b || i < 0 || i >= (int)b->solves.size()) return fail(HB_E_ARG, "bad batch index");
    if (!phi0) return fail(HB_E_ARG, "phi0 is NULL");
    Solve& s = *b->solves[i];
    HB_TRY(upload_state(s, 0, 2, phi0, phi1, mem, dtype, b->stream));
    s.nstep = 0;
    s.target = 0;
    s.has_initial = true;
    b->built = false;
    return HB_OK;
}

int hb_batch_step(hb_batch* b, int64_t nsteps) {
    if (!b) return fail(HB_E_ARG, "batch is NULL");
    if (nsteps < 0 || nsteps > MAX_STEPS) return fail(HB_E_ARG, "nsteps must be in [0, 2^40]");
    for (auto& s : b->solves)
        if (!s->has_initial) return fail(HB_E_STATE, "a solve has no initial data");
    if (nsteps == 0) return HB_OK;
    for (Group& g : b->groups) {
        if (g.members.empty()) continue;
        bool moved = false;
        HB_TRY(set_targets(g, nsteps, b->stream, &moved));
        if (moved || !b->built) HB_TRY(group_rebuild(g, b->stream));
        for (size_t i = 0; i < g.members.size(); ++i)
            HB_TRY(from_hip(launch_set_target(g.d_desc, (int)i, g.members[i]->target, b->stream),
                            "set target"));
    }
    b->built = true;
    for (Group& g : b->groups) HB_TRY(group_step(g, nsteps, b->use_graph, b->stream));
    return HB_OK;
}

int hb_batch_read(hb_batch* b, int i, void* phi, void* phi_t, int mem, int dtype) {
    if (!b || i < 0 || i >= (int)b->solves.size()) return fail(HB_E_ARG, "bad batch index");
    if (!b->solves[i]->has_initial) return fail(HB_E_STATE, "no initial data");
    return download_state(*b->solves[i], phi, phi_t, mem, dtype, b->stream);
}

int hb_batch_sync(hb_batch* b) {
    if (!b) return fail(HB_E_ARG, "batch is NULL");
    HIP_TRY(hipStreamSynchronize(b->stream));
    return HB_OK;
}

int hb_batch_set_tiling(hb_batch* b, int by, int zc) {
    if (!b) return fail(HB_E_ARG, "batch is NULL");
    if (!valid_by(by, b->groups[0].scheme)) return fail(HB_E_ARG, "by must be 8 or 16 (or 11 or 20, whole-step scheme)");
    if (zc < 0) return fail(HB_E_ARG, "zc must be >= 0");
    for (Group& g : b->groups) {
        g.by = by;
        g.zc = zc;
    }
    b->built = false;
    return HB_OK;
}

int hb_batch_autotune(hb_batch* b, int trial_steps, int* by, int* zc) {
    if (!b) return fail(HB_E_ARG, "batch is NULL");
    if (trial_steps < 1) return fail(HB_E_ARG, "trial_steps must be >= 1");
    for (auto& s : b->solves)
        if (!s->has_initial) return fail(HB_E_STATE, "a solve has no initial data");
    for (int p = 0; p < 2; ++p) {
        Group& g = b->groups[p];
        int bb = -1, bz = -1;
        if (!g.members.empty()) HB_TRY(group_autotune(g, trial_steps, b->stream, &bb, &bz));
        if (by) by[p] = bb;
        if (zc) zc[p] = bz;
    }
    // each group was rebuilt with its choice; targets were restored, so the
    // next hb_batch_step sets them again
    b->built = true;
    return HB_OK;
}

int hb_batch_destroy(hb_batch* b) {
    if (!b) return HB_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    delete b;
    return HB_OK;
}

}  // extern "C"

// ---- C ABI: served form (continuous batching) -------------------------------------

struct hb_pool {
    struct Slot {
        std::unique_ptr<Solve> s;
        size_t bytes = 0;
        bool busy = false;
        bool done = false;
        bool reported = false;
        bool joined = false;           // the compute stream has waited for `ready`
        bool has_fin = false;
        hipEvent_t ready = nullptr;    // admission transfer complete (copy stream)
        hipEvent_t fin = nullptr;      // compute-stream point after its last step
    };
    // a released solve, kept for an admission whose fields and coefficient
    // table need exactly its allocations
    struct Spare {
        std::unique_ptr<Solve> s;
        size_t bytes = 0;              // its footprint (counted against the budget)
        size_t mem_bytes = 0;          // its field allocation
        hipEvent_t retired = nullptr;  // compute-stream point after which nothing touches it
    };
    std::vector<Slot> slots;
    std::vector<Spare> spares;
    size_t budget = 0, in_use = 0, spare_bytes = 0;
    Group groups[2];
    hipStream_t stream = nullptr;  // compute: the step launches
    hipStream_t xfer = nullptr;    // copies: admissions and reads of finished solves
    bool own_stream = false;
    bool dirty = true;
    Staging hst;                   // pinned host staging of the copy stream
    void* dstage = nullptr;        // device staging (used in copy-stream order)
    size_t dstage_cap = 0;
    ~hb_pool() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (xfer) (void)hipStreamSynchronize(xfer);
        groups[0].release();
        groups[1].release();
        for (auto& sl : slots) {
            if (sl.ready) (void)hipEventDestroy(sl.ready);
            if (sl.fin) (void)hipEventDestroy(sl.fin);
        }
        for (auto& sp : spares)
            if (sp.retired) (void)hipEventDestroy(sp.retired);
        slots.clear();
        spares.clear();
        hst.release();
        dev_free(dstage);
        if (xfer) (void)hipStreamDestroy(xfer);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
    // device staging of at least `bytes` (its previous contents are used only
    // by copy-stream work, which later copy-stream work follows)
    int device_staging(size_t bytes, void** out) {
        if (bytes > dstage_cap) {
            dev_free(dstage);  // waits for the copy stream's use of it
            dstage = nullptr;
            dstage_cap = 0;
            const size_t want = std::max<size_t>(bytes, 1 << 20);
            HB_TRY(dev_alloc(&dstage, want, "pool staging", xfer));
            dstage_cap = want;
        }
        *out = dstage;
        return HB_OK;
    }
};

namespace {

int ensure_event(hipEvent_t* e) {
    if (!*e) HIP_TRY(hipEventCreateWithFlags(e, hipEventDisableTiming));
    return HB_OK;
}

// Admission transfer of one solve on the copy stream: zero its allocation,
// upload its coefficient table and its initial state (host inputs through
// the pinned staging).  Nothing here waits for the compute stream.
int pool_upload(hb_pool* p, Solve& s, const void* phi0, const void* phi1, int mem, int dtype) {
    if (dtype != HB_DTYPE_F64 && dtype != HB_DTYPE_F32) return fail(HB_E_ARG, "bad dtype");
    if (mem != HB_HOST && mem != HB_DEVICE) return fail(HB_E_ARG, "bad memory kind");
    HB_TRY(solve_clear(s, p->xfer));
    const long long cnt = (long long)s.L.nx * s.L.ny * s.L.nz;
    const size_t vb = (size_t)cnt * (dtype == HB_DTYPE_F64 ? 8 : 4);
    const size_t tb = (size_t)s.ctab_steps * 4 * sizeof(double);
    const size_t voff = (size_t)round_up((long long)tb, 256);
    const int nsrc = mem == HB_HOST ? (phi1 ? 2 : 1) : 0;
    void* h = nullptr;
    HB_TRY(p->hst.get(voff + vb * (size_t)nsrc, &h));
    std::vector<double> tab;
    try {
        fill_ctab(s.cfg, 0, s.ctab_steps, tab);
    } catch (const std::bad_alloc&) {
        return fail(HB_E_NOMEM, "coefficient table: host allocation failed");
    }
    std::memcpy(h, tab.data(), tb);
    HIP_TRY(hipMemcpyAsync(s.ctab, h, tb, hipMemcpyHostToDevice, p->xfer));
    const void* src[2] = {phi0, phi1};
    void* hi[2] = {s.f[0], s.f[2]};
    float* lo[2] = {s.lo_view(0, 0), s.lo_view(1, 0)};
    void* dst = nullptr;
    if (nsrc) HB_TRY(p->device_staging(vb * (size_t)nsrc, &dst));
    for (int k = 0; k < 2; ++k) {
        const void* d = src[k];
        if (src[k] && mem == HB_HOST) {
            char* hk = (char*)h + voff + vb * (size_t)k;
            std::memcpy(hk, src[k], vb);
            char* dk = (char*)dst + vb * (size_t)k;
            HIP_TRY(hipMemcpyAsync(dk, hk, vb, hipMemcpyHostToDevice, p->xfer));
            d = dk;
        }
        if (k == 1 && !src[1]) continue;  // psi stays zero from the clear
        HB_TRY(from_hip(launch_unpack(s.prec(), dtype, d, s.L.nx, s.L.ny, s.L.nz, s.L.sy, s.L.sz, s.L.cs,
                                      hi[k], lo[k], p->xfer),
                        "unpack"));
    }
    HB_TRY(p->hst.mark(p->xfer));
    return HB_OK;
}

}  // namespace

extern "C" {

int hb_pool_create(size_t hbm_budget, int max_slots, void* stream, hb_pool** out) {
    g_last_error.clear();
    if (!out) return fail(HB_E_ARG, "out is NULL");
    *out = nullptr;
    if (max_slots < 1 || max_slots > (1 << 20) || hbm_budget == 0)
        return fail(HB_E_ARG, "need 1 <= max_slots <= 2^20 and a budget");
    auto p = std::make_unique<hb_pool>();
    p->slots.resize(max_slots);
    p->budget = hbm_budget;
    if (stream) {
        p->stream = (hipStream_t)stream;
    } else {
        HIP_TRY(hipStreamCreateWithFlags(&p->stream, hipStreamNonBlocking));
        p->own_stream = true;
    }
    HIP_TRY(hipStreamCreateWithFlags(&p->xfer, hipStreamNonBlocking));
    p->groups[0].prec = HB_F64;
    p->groups[1].prec = HB_F32C;
    for (Group& g : p->groups) g.by = MULTI_BY;  // whole-step scheme
    *out = p.release();
    return HB_OK;
}

int hb_pool_admit(hb_pool* p, const hb_config* cfg, const void* phi0, const void* phi1, int mem,
                  int dtype, int64_t steps, int* slot) {
    if (!p || !slot) return fail(HB_E_ARG, "NULL argument");
    *slot = -1;
    HB_TRY(validate(cfg));
    if (!phi0) return fail(HB_E_ARG, "phi0 is NULL");
    if (steps < 0 || steps > MAX_STEPS) return fail(HB_E_ARG, "steps must be in [0, 2^40]");
    if (scheme_of(cfg->flags) != SCHEME_STEP)
        return fail(HB_E_ARG, "pool solves use the whole-step kernel (no HB_PAIRWISE/HB_STAGEWISE)");
    if (dtype != HB_DTYPE_F64 && dtype != HB_DTYPE_F32) return fail(HB_E_ARG, "bad dtype");
    if (mem != HB_HOST && mem != HB_DEVICE) return fail(HB_E_ARG, "bad memory kind");
    const size_t need = solve_footprint(*cfg, SCHEME_STEP, steps + 1);
    int free_slot = -1;
    for (size_t i = 0; i < p->slots.size(); ++i)
        if (!p->slots[i].busy) {
            free_slot = (int)i;
            break;
        }
    if (free_slot < 0) return fail(HB_E_BUSY, "no free slot");
    // a released solve whose field allocation and coefficient table have
    // exactly the sizes this configuration needs is taken over
    const Layout need_L = plan_layout(*cfg, SCHEME_STEP);
    const size_t need_mem = field_bytes(need_L) * (size_t)need_L.nfields;
    const long long need_cap = ctab_capacity(steps + 1, 0);
    int reuse = -1;
    for (size_t i = 0; i < p->spares.size(); ++i)
        if (p->spares[i].mem_bytes == need_mem && p->spares[i].s->ctab_steps == need_cap) {
            reuse = (int)i;
            break;
        }
    // spares count against the budget (in_use + spare_bytes <= budget):
    // without one to take over, give spares back, oldest first, until the
    // solve fits (freeing a block waits for the device)
    if (reuse < 0) {
        size_t k = 0;
        while (need + p->in_use + p->spare_bytes > p->budget && k < p->spares.size()) {
            hb_pool::Spare& sp = p->spares[k];
            if (sp.retired) {
                (void)hipEventSynchronize(sp.retired);
                (void)hipEventDestroy(sp.retired);
            }
            p->spare_bytes -= sp.bytes;
            sp.s.reset();
            p->spares.erase(p->spares.begin() + (long)k);
        }
    }
    if (p->in_use + (p->spare_bytes - (reuse >= 0 ? p->spares[reuse].bytes : 0)) + need > p->budget)
        return fail(HB_E_BUSY, "HBM budget exhausted");
    std::unique_ptr<Solve> s;
    if (reuse >= 0) {
        hb_pool::Spare sp = std::move(p->spares[reuse]);
        p->spares.erase(p->spares.begin() + reuse);
        p->spare_bytes -= sp.bytes;
        s = std::move(sp.s);
        // the copy stream rewrites the memory only after the compute stream
        // has passed every launch that could still touch it
        hipError_t e = sp.retired ? hipStreamWaitEvent(p->xfer, sp.retired, 0) : hipSuccess;
        if (sp.retired) (void)hipEventDestroy(sp.retired);
        if (e != hipSuccess) return fail(HB_E_HIP, "pool reuse wait: %s", hipGetErrorString(e));
        solve_views(*s, *cfg, SCHEME_STEP);
    } else {
        s = std::make_unique<Solve>();
        HB_TRY(dev_alloc((void**)&s->mem, need_mem, "solve state", p->xfer));
        solve_views(*s, *cfg, SCHEME_STEP);
        HB_TRY(dev_alloc((void**)&s->ctab, (size_t)need_cap * 4 * sizeof(double), "coefficient table",
                         p->xfer));
        s->ctab_steps = need_cap;
    }
    if (mem == HB_DEVICE) {
        // device inputs are read in the pool stream's order
        hb_pool::Slot& sl0 = p->slots[free_slot];
        HB_TRY(ensure_event(&sl0.ready));
        HIP_TRY(hipEventRecord(sl0.ready, p->stream));
        HIP_TRY(hipStreamWaitEvent(p->xfer, sl0.ready, 0));
    }
    HB_TRY(pool_upload(p, *s, phi0, phi1, mem, dtype));
    s->nstep = 0;
    s->target = steps;
    s->has_initial = true;
    hb_pool::Slot& sl = p->slots[free_slot];
    HB_TRY(ensure_event(&sl.ready));
    HIP_TRY(hipEventRecord(sl.ready, p->xfer));
    sl.s = std::move(s);
    sl.bytes = need;
    sl.busy = true;
    sl.done = (steps == 0);
    sl.reported = false;
    sl.joined = false;
    sl.has_fin = false;
    p->in_use += need;
    p->dirty = true;
    *slot = free_slot;
    return HB_OK;
}

static int pool_rebuild(hb_pool* p) {
    for (Group& g : p->groups) g.members.clear();
    for (auto& sl : p->slots)
        if (sl.busy && !sl.done) {
            if (!sl.joined) {
                // the compute stream waits for this solve's admission copies only
                HIP_TRY(hipStreamWaitEvent(p->stream, sl.ready, 0));
                sl.joined = true;
            }
            p->groups[sl.s->prec()].members.push_back(sl.s.get());
        }
    for (Group& g : p->groups) {
        if (g.members.empty()) {
            g.drop_graph();
            g.ntiles = 0;
            continue;
        }
        HB_TRY(group_rebuild(g, p->stream));
    }
    p->dirty = false;
    return HB_OK;
}

// mark a slot finished: its last step is behind everything enqueued so far
static int pool_finish(hb_pool* p, hb_pool::Slot& sl) {
    sl.done = true;
    HB_TRY(ensure_event(&sl.fin));
    HIP_TRY(hipEventRecord(sl.fin, p->stream));
    sl.has_fin = true;
    p->dirty = true;
    return HB_OK;
}

int hb_pool_advance(hb_pool* p, int k) {
    if (!p) return fail(HB_E_ARG, "pool is NULL");
    if (k < 0) return fail(HB_E_ARG, "k must be >= 0");
    // while the active set is the one of the previous advance, steps replay
    // the group's captured graph; a changed set is rebuilt and launched
    // directly this time
    const bool changed = p->dirty;
    if (changed) HB_TRY(pool_rebuild(p));
    for (Group& g : p->groups) HB_TRY(group_step(g, k, !changed, p->stream));
    for (auto& sl : p->slots)
        if (sl.busy && !sl.done && sl.s->nstep >= sl.s->target) HB_TRY(pool_finish(p, sl));
    return HB_OK;
}

int hb_pool_poll(hb_pool* p, int* done, int cap, int* ndone) {
    if (!p || !ndone || (cap > 0 && !done)) return fail(HB_E_ARG, "NULL argument");
    int n = 0;
    for (size_t i = 0; i < p->slots.size(); ++i) {
        auto& sl = p->slots[i];
        if (sl.busy && sl.done && !sl.reported && n < cap) {
            if (done) done[n] = (int)i;
            sl.reported = true;
            ++n;
        }
    }
    *ndone = n;
    return HB_OK;
}

int hb_pool_check(hb_pool* p, int* failed, int cap, int* nfailed) {
    if (!p || !nfailed || (cap > 0 && !failed)) return fail(HB_E_ARG, "NULL argument");
    *nfailed = 0;
    if (p->dirty) HB_TRY(pool_rebuild(p));
    // one diagnostics pass per active solve, on its group's descriptor; the
    // partials buffer is reused in stream order
    int maxparts = 0, members = 0;
    for (Group& g : p->groups)
        for (Solve* s : g.members) {
            maxparts = std::max(maxparts, diag_partials_needed(s->L.nx, s->L.ny, s->L.nz));
            ++members;
        }
    if (members == 0) return HB_OK;
    double* parts = nullptr;
    double* outs = nullptr;
    HB_TRY(dev_alloc((void**)&parts, (size_t)maxparts * DIAG_COUNT * sizeof(double), "check partials",
                     p->stream));
    int rc = dev_alloc((void**)&outs, (size_t)members * DIAG_COUNT * sizeof(double), "check results",
                       p->stream);
    std::vector<double> host((size_t)members * DIAG_COUNT);
    std::vector<Solve*> order;
    for (Group& g : p->groups)
        for (size_t i = 0; i < g.members.size() && rc == HB_OK; ++i) {
            Solve* s = g.members[i];
            rc = from_hip(launch_diagnostics(s->prec(), g.d_desc + i, (int)(s->nstep & 1), 0.0, parts,
                                             diag_partials_needed(s->L.nx, s->L.ny, s->L.nz),
                                             outs + order.size() * DIAG_COUNT, p->stream),
                          "check");
            order.push_back(s);
        }
    if (rc == HB_OK)
        rc = from_hip(hipMemcpyAsync(host.data(), outs, host.size() * sizeof(double),
                                     hipMemcpyDeviceToHost, p->stream),
                      "check copy");
    if (rc == HB_OK) rc = from_hip(hipStreamSynchronize(p->stream), "check sync");
    dev_free(parts);
    dev_free(outs);
    HB_TRY(rc);
    int n = 0;
    for (size_t m = 0; m < order.size(); ++m) {
        if (host[m * DIAG_COUNT + DIAG_NONFINITE] == 0.0) continue;
        for (size_t i = 0; i < p->slots.size(); ++i) {
            auto& sl = p->slots[i];
            if (!sl.busy || sl.s.get() != order[m]) continue;
            HB_TRY(pool_finish(p, sl));  // stops stepping; hb_pool_poll reports it
            if (n < cap) failed[n] = (int)i;
            ++n;
        }
    }
    *nfailed = std::min(n, std::max(cap, 0));
    return HB_OK;
}

int hb_pool_stats(const hb_pool* p, int* active, size_t* in_use) {
    if (!p) return fail(HB_E_ARG, "pool is NULL");
    int a = 0;
    for (auto& sl : p->slots)
        if (sl.busy && !sl.done) ++a;
    if (active) *active = a;
    if (in_use) *in_use = p->in_use;
    return HB_OK;
}

int hb_pool_read(hb_pool* p, int slot, void* phi, void* phi_t, int mem, int dtype) {
    if (!p || slot < 0 || slot >= (int)p->slots.size() || !p->slots[slot].busy)
        return fail(HB_E_ARG, "bad slot");
    auto& sl = p->slots[slot];
    if (!sl.done || !sl.has_fin) {
        // not finished by a step (still running, or admitted with 0 steps):
        // read in the compute stream's order, after the admission copies
        if (!sl.joined) {
            HIP_TRY(hipStreamWaitEvent(p->stream, sl.ready, 0));
            sl.joined = true;
        }
        return download_state(*sl.s, phi, phi_t, mem, dtype, p->stream);
    }
    if (dtype != HB_DTYPE_F64 && dtype != HB_DTYPE_F32) return fail(HB_E_ARG, "bad dtype");
    if (mem != HB_HOST && mem != HB_DEVICE) return fail(HB_E_ARG, "bad memory kind");
    // a finished solve is copied out on the copy stream, after its last step
    // and without waiting for the steps of the others enqueued since
    Solve& s = *sl.s;
    HIP_TRY(hipStreamWaitEvent(p->xfer, sl.fin, 0));
    const int par = (int)(s.nstep & 1);
    const long long cnt = (long long)s.L.nx * s.L.ny * s.L.nz;
    const size_t vb = (size_t)cnt * (dtype == HB_DTYPE_F64 ? 8 : 4);
    void* dst[2] = {phi, phi_t};
    const void* hi[2] = {s.f[0 + par], s.f[2 + par]};
    const float* lo[2] = {s.lo_view(0, par), s.lo_view(1, par)};
    if (mem == HB_DEVICE) {
        for (int k = 0; k < 2; ++k)
            if (dst[k])
                HB_TRY(from_hip(launch_pack(s.prec(), dtype, dst[k], s.L.nx, s.L.ny, s.L.nz, s.L.sy, s.L.sz,
                                            s.L.cs, hi[k], lo[k], p->xfer),
                                "pack"));
        HIP_TRY(hipStreamSynchronize(p->xfer));
        return HB_OK;
    }
    const int nout = (phi ? 1 : 0) + (phi_t ? 1 : 0);
    if (nout == 0) return HB_OK;
    void* d = nullptr;
    void* h = nullptr;
    HB_TRY(p->device_staging(vb * (size_t)nout, &d));
    HB_TRY(p->hst.get(vb * (size_t)nout, &h));
    int j = 0;
    for (int k = 0; k < 2; ++k) {
        if (!dst[k]) continue;
        char* dk = (char*)d + vb * (size_t)j;
        HB_TRY(from_hip(launch_pack(s.prec(), dtype, dk, s.L.nx, s.L.ny, s.L.nz, s.L.sy, s.L.sz, s.L.cs,
                                    hi[k], lo[k], p->xfer),
                        "pack"));
        HIP_TRY(hipMemcpyAsync((char*)h + vb * (size_t)j, dk, vb, hipMemcpyDeviceToHost, p->xfer));
        ++j;
    }
    HB_TRY(p->hst.mark(p->xfer));
    HIP_TRY(hipStreamSynchronize(p->xfer));
    j = 0;
    for (int k = 0; k < 2; ++k)
        if (dst[k]) std::memcpy(dst[k], (char*)h + vb * (size_t)j++, vb);
    return HB_OK;
}

int hb_pool_release(hb_pool* p, int slot) {
    if (!p || slot < 0 || slot >= (int)p->slots.size() || !p->slots[slot].busy)
        return fail(HB_E_ARG, "bad slot");
    auto& sl = p->slots[slot];
    const bool active = !sl.done;
    // the solve is kept for a later admission of the same footprint; it may
    // be rewritten once the compute stream has passed what is enqueued now
    hb_pool::Spare sp;
    HB_TRY(ensure_event(&sp.retired));
    HIP_TRY(hipEventRecord(sp.retired, p->stream));
    // a join that never happened still orders the compute stream after the
    // admission copies (they precede every later copy-stream use anyway)
    sp.mem_bytes = field_bytes(sl.s->L) * (size_t)sl.s->L.nfields;
    sp.s = std::move(sl.s);
    sp.bytes = sl.bytes;
    p->in_use -= sl.bytes;
    p->spare_bytes += sl.bytes;
    p->spares.push_back(std::move(sp));
    sl.busy = false;
    sl.done = false;
    sl.reported = false;
    sl.joined = false;
    sl.has_fin = false;
    sl.bytes = 0;
    if (active) p->dirty = true;
    return HB_OK;
}

int hb_pool_destroy(hb_pool* p) {
    if (!p) return HB_OK;
    delete p;
    return HB_OK;
}

}  // extern "C"

// ---- measurement: streamed-bandwidth probe -----------------------------------------

extern "C" int hb_probe_bandwidth(int kind, size_t bytes_per_array, int iters, double* gbps) {
    if (kind < 0 || kind > 2 || iters < 1 || bytes_per_array < 4096 || !gbps)
        return fail(HB_E_ARG, "bad probe arguments");
    const int nin = kind == 0 ? 1 : kind == 1 ? 2 : 5;
    const int nout = kind == 2 ? 2 : 1;
    const long long n16 = (long long)(bytes_per_array / 16);
    const size_t bytes = (size_t)n16 * 16;
    void* in[5] = {};
    void* out[2] = {};
    int rc = HB_OK;
    for (int k = 0; k < nin && rc == HB_OK; ++k)
        if (hipMalloc(&in[k], bytes) != hipSuccess) rc = fail(HB_E_NOMEM, "probe allocation");
    for (int k = 0; k < nout && rc == HB_OK; ++k)
        if (hipMalloc(&out[k], bytes) != hipSuccess) rc = fail(HB_E_NOMEM, "probe allocation");
    for (int k = 0; k < nin && rc == HB_OK; ++k)
        if (hipMemset(in[k], 0, bytes) != hipSuccess) rc = fail(HB_E_HIP, "probe memset");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (rc == HB_OK && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = fail(HB_E_HIP, "probe events");
    const long long want = (n16 + 255) / 256;
    const int blocks = (int)std::min<long long>(want, 1LL << 30);  // one element per thread
    if (rc == HB_OK) rc = from_hip(launch_probe(kind, in, out, n16, blocks, nullptr), "probe");
    if (rc == HB_OK) rc = from_hip(hipEventRecord(e0, nullptr), "event");
    for (int i = 0; i < iters && rc == HB_OK; ++i)
        rc = from_hip(launch_probe(kind, in, out, n16, blocks, nullptr), "probe");
    if (rc == HB_OK) rc = from_hip(hipEventRecord(e1, nullptr), "event");
    if (rc == HB_OK) rc = from_hip(hipEventSynchronize(e1), "event sync");
    float ms = 0;
    if (rc == HB_OK) rc = from_hip(hipEventElapsedTime(&ms, e0, e1), "event elapsed");
    if (rc == HB_OK) *gbps = (double)bytes * (nin + nout) * iters / (ms * 1e-3) / 1e9;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    for (void* p : in)
        if (p) (void)hipFree(p);
    for (void* p : out)
        if (p) (void)hipFree(p);
    return rc;
}

// ---- batched radial solves ------------------------------------------------------

namespace {

constexpr long long RADIAL_CHUNK = 1LL << 16;
// c(t) table of one launch: at most this many doubles (the launch length
// shrinks when many solves have distinct (t0, dt, inv_L2))
constexpr long long RADIAL_TABLE_DOUBLES = 4LL << 20;

// A validated radial batch: descriptors, and the distinct (t0, dt, inv_L2)
// of its solves, whose c(t) rows the launches share.
struct RadialPlan {
    std::vector<RadialDesc> descs;
    std::vector<int> key_of;                     // per solve: its (t0, dt, inv_L2)
    std::vector<std::array<double, 3>> keys;     // t0, dt, inv_L2
    std::vector<long long> key_steps;            // most steps of any solve of the key
    long long total = 0, max_steps = 0;
    int max_m = 0;
};

int radial_plan(int count, const hb_radial_config* cfgs, RadialPlan& p) {
    p.descs.assign(count, RadialDesc{});
    p.key_of.assign(count, 0);
    std::map<std::array<double, 3>, int> index;
    for (int i = 0; i < count; ++i) {
        const hb_radial_config& c = cfgs[i];
        if (c.m < 1 || c.m > HB_RADIAL_MAX_NODES)
            return fail(HB_E_ARG, "radial solve %d: m = %d outside [1, %d]", i, c.m, HB_RADIAL_MAX_NODES);
        if (!(c.dr > 0) || !(c.dt > 0) || !std::isfinite(c.dr) || !std::isfinite(c.dt) || c.steps < 0)
            return fail(HB_E_ARG, "radial solve %d: need dr > 0, dt > 0, steps >= 0", i);
        if (c.steps > MAX_STEPS) return fail(HB_E_ARG, "radial solve %d: steps beyond 2^40", i);
        if (!std::isfinite(c.mu2) || !std::isfinite(c.lambda) || !std::isfinite(c.inv_L2) ||
            !std::isfinite(c.t0) || c.inv_L2 < 0)
            return fail(HB_E_ARG, "radial solve %d: coefficients must be finite (inv_L2 >= 0)", i);
        if (!(c.flags & HB_ALLOW_UNSTABLE)) {
            const double c0 = c.inv_L2 * std::exp(-2.0 * c.t0);
            if (c.dt * std::sqrt(c0 * 16.0 / (c.dr * c.dr)) > 2.0 * std::sqrt(2.0))
                return fail(HB_E_CFL, "radial solve %d: dt = %g beyond the stability limit", i, c.dt);
        }
        RadialDesc& d = p.descs[i];
        std::memset(&d, 0, sizeof d);
        d.offset = p.total;
        d.steps = c.steps;
        d.m = c.m;
        d.dr = c.dr;
        d.mu2 = c.mu2;
        d.lambda = c.lambda;
        d.inv_L2 = c.inv_L2;
        d.t0 = c.t0;
        d.dt = c.dt;
        const std::array<double, 3> key = {c.t0, c.dt, c.inv_L2};
        auto it = index.find(key);
        if (it == index.end()) {
            it = index.emplace(key, (int)p.keys.size()).first;
            p.keys.push_back(key);
            p.key_steps.push_back(0);
        }
        p.key_of[i] = it->second;
        p.key_steps[it->second] = std::max<long long>(p.key_steps[it->second], c.steps);
        p.total += c.m;
        p.max_m = std::max(p.max_m, c.m);
        p.max_steps = std::max<long long>(p.max_steps, c.steps);
    }
    return HB_OK;
}

// steps per launch: at most RADIAL_CHUNK, and few enough that every key's
// rows fit `table_doubles` (0 if not even one step fits)
long long radial_chunk(const RadialPlan& p, long long table_doubles) {
    const long long per_step = 3 * (long long)std::max<size_t>(1, p.keys.size());
    return std::min<long long>(RADIAL_CHUNK, table_doubles / per_step);
}

// Run a planned batch on device state dphi/dpsi with the given descriptor
// array (descs.size() entries) and c(t) table (>= 3 x chunk x keys doubles).
// Each launch covers `chunk` steps of every solve; its table rows are filled
// on the host (the stage times of eq. (rhs) in FP64, as for the 3-D path) and
// copied before the launch, and the stream is drained after it, so the table
// can be refilled.  Waits for completion.
int radial_run(RadialPlan& p, long long chunk, RadialDesc* d_desc, double* d_table, double* dphi,
               double* dpsi, hipStream_t s) {
    for (size_t i = 0; i < p.descs.size(); ++i) p.descs[i].ctab = 3 * chunk * p.key_of[i];
    HIP_TRY(hipMemcpyAsync(d_desc, p.descs.data(), p.descs.size() * sizeof(RadialDesc),
                           hipMemcpyHostToDevice, s));
    std::vector<double> table;
    try {
        table.assign((size_t)(3 * chunk * (long long)p.keys.size()), 0.0);
    } catch (const std::bad_alloc&) {
        return fail(HB_E_NOMEM, "radial coefficient table: host allocation failed");
    }
    // launches of at most `chunk` steps each, so no single kernel runs for an
    // unbounded time (the state goes through memory between them)
    for (long long n0 = 0; n0 < std::max<long long>(p.max_steps, 1); n0 += chunk) {
        const long long n1 = n0 + chunk;
        for (size_t k = 0; k < p.keys.size(); ++k) {
            const double t0 = p.keys[k][0], dt = p.keys[k][1], il2 = p.keys[k][2];
            double* row = &table[(size_t)(3 * chunk * (long long)k)];
            for (long long n = n0; n < std::min(n1, p.key_steps[k]); ++n) {
                const double t = t0 + (double)n * dt;
                double* o = row + 3 * (n - n0);
                o[0] = std::exp(-2.0 * t) * il2;
                o[1] = std::exp(-2.0 * (t + dt / 2.0)) * il2;
                o[2] = std::exp(-2.0 * (t + dt)) * il2;
            }
        }
        HIP_TRY(hipMemcpyAsync(d_table, table.data(), table.size() * sizeof(double),
                               hipMemcpyHostToDevice, s));
        HB_TRY(from_hip(launch_radial(d_desc, d_table, (int)p.descs.size(), p.max_m, dphi, dpsi, n0, n1, s),
                        "radial launch"));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return HB_OK;
}

}  // namespace

extern "C" int hb_radial_solve(int count, const hb_radial_config* cfgs, double* phi, double* psi,
                               int mem, void* stream) {
    g_last_error.clear();
    if (count < 0 || (count > 0 && (!cfgs || !phi || !psi)))
        return fail(HB_E_ARG, "bad radial batch arguments");
    if (mem != HB_HOST && mem != HB_DEVICE) return fail(HB_E_ARG, "bad memory kind");
    if (count == 0) return HB_OK;
    RadialPlan plan;
    HB_TRY(radial_plan(count, cfgs, plan));
    hipStream_t s = (hipStream_t)stream;
    const size_t bytes = (size_t)plan.total * sizeof(double);
    const long long chunk = radial_chunk(plan, RADIAL_TABLE_DOUBLES);
    if (chunk < 1) return fail(HB_E_ARG, "radial batch: too many distinct (t0, dt, inv_L2)");
    const long long tab = 3 * std::min(chunk, std::max<long long>(plan.max_steps, 1)) *
                          (long long)plan.keys.size();
    RadialDesc* d_desc = nullptr;
    double* d_table = nullptr;
    double* dphi = nullptr;
    double* dpsi = nullptr;
    int rc = dev_alloc((void**)&d_desc, plan.descs.size() * sizeof(RadialDesc), "radial descriptors", s);
    if (rc == HB_OK) rc = dev_alloc((void**)&d_table, (size_t)tab * sizeof(double), "radial c(t) table", s);
    if (mem == HB_HOST) {
        if (rc == HB_OK) rc = dev_alloc((void**)&dphi, bytes, "radial state", s);
        if (rc == HB_OK) rc = dev_alloc((void**)&dpsi, bytes, "radial state", s);
    } else {
        dphi = phi;
        dpsi = psi;
    }
    if (rc == HB_OK && mem == HB_HOST) {
        rc = from_hip(hipMemcpyAsync(dphi, phi, bytes, hipMemcpyHostToDevice, s), "radial H2D");
        if (rc == HB_OK) rc = from_hip(hipMemcpyAsync(dpsi, psi, bytes, hipMemcpyHostToDevice, s), "radial H2D");
    }
    // the table holds `chunk` rows per key only when some solve runs that
    // long: shorter batches use a single launch of max_steps steps
    if (rc == HB_OK) rc = radial_run(plan, std::min(chunk, std::max<long long>(plan.max_steps, 1)), d_desc,
                                     d_table, dphi, dpsi, s);
    if (rc == HB_OK && mem == HB_HOST) {
        rc = from_hip(hipMemcpyAsync(phi, dphi, bytes, hipMemcpyDeviceToHost, s), "radial D2H");
        if (rc == HB_OK) rc = from_hip(hipMemcpyAsync(psi, dpsi, bytes, hipMemcpyDeviceToHost, s), "radial D2H");
    }
    hipError_t e = hipStreamSynchronize(s);
    if (rc == HB_OK && e != hipSuccess) rc = fail(HB_E_HIP, "radial sync: %s", hipGetErrorString(e));
    dev_free(d_desc);
    dev_free(d_table);
    if (mem == HB_HOST) {
        dev_free(dphi);
        dev_free(dpsi);
    }
    return rc;
}

// The radial batch without device allocation: the same plan and launches as
// hb_radial_solve, with descriptors and c(t) tables in the library's fixed
// device scratch (its address on this device from radial_scratch).  The
// state arrays are the caller's device memory.
extern "C" int hb_radial_solve_noalloc(int count, const hb_radial_config* cfgs, double* phi, double* psi,
                                       void* stream) {
    g_last_error.clear();
    if (count < 0 || (count > 0 && (!cfgs || !phi || !psi)))
        return fail(HB_E_ARG, "bad radial batch arguments");
    if (count == 0) return HB_OK;
    RadialPlan plan;
    HB_TRY(radial_plan(count, cfgs, plan));
    // descriptors first (256-byte aligned), then the c(t) table in the rest
    const size_t desc_bytes = (size_t)round_up((long long)(plan.descs.size() * sizeof(RadialDesc)), 256);
    if (desc_bytes >= RADIAL_SCRATCH_BYTES)
        return fail(HB_E_ARG, "radial batch of %d solves: descriptors exceed the %zu-byte scratch", count,
                    RADIAL_SCRATCH_BYTES);
    const long long chunk =
        radial_chunk(plan, (long long)((RADIAL_SCRATCH_BYTES - desc_bytes) / sizeof(double)));
    if (chunk < 1)
        return fail(HB_E_ARG, "radial batch: %zu distinct (t0, dt, inv_L2) exceed the %zu-byte scratch",
                    plan.keys.size(), RADIAL_SCRATCH_BYTES);
    void* base = nullptr;
    HB_TRY(from_hip(radial_scratch(&base), "scratch address"));
    RadialDesc* d_desc = (RadialDesc*)base;
    double* d_table = (double*)((char*)base + desc_bytes);
    return radial_run(plan, std::min(chunk, std::max<long long>(plan.max_steps, 1)), d_desc, d_table, phi,
                      psi, (hipStream_t)stream);
}
