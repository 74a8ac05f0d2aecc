/*
 * Plain FP64 CPU oracle for the Higgs boson equation in de Sitter spacetime
 * (Balogh, Banda, Yagdjian, arXiv:1803.01291).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The GPU library neither
 * links nor calls it, and this file includes nothing of the GPU library.
 *
 * It is deliberately slow and obvious: textbook classical RK4 with four
 * stage-derivative arrays, the fourth-order central second difference summed
 * axis by axis in the order the paper prints it, and a halo that is refilled
 * before every right-hand-side evaluation.  Build with
 * -O2 -ffp-contract=off -fno-fast-math (no FMA contraction, IEEE order).
 *
 * What is computed (section 2.1 of the paper):
 *   equation (higgs-boson-rescalled), first-order form eq. (rhs):
 *     phi_t = psi
 *     psi_t = -3 psi + c(t) Lap_h phi + mu2 phi - lambda phi^3
 *     c(t)  = inv_L2 * exp(-2 t)                 (inv_L2 = 1/L^2)
 *   space: the fourth-order central difference for each second partial
 *     d2u/dx2 ~ (-1/12 u[j-2] + 4/3 u[j-1] - 5/2 u[j] + 4/3 u[j+1] - 1/12 u[j+2]) / dx^2
 *     and Lap_h = d2/dx2 + d2/dy2 + d2/dz2 (13-point star)
 *   time: classical explicit RK4 with stage times t, t+dt/2, t+dt/2, t+dt
 *     k1 = f(t, v), k2 = f(t+dt/2, v+dt/2 k1), k3 = f(t+dt/2, v+dt/2 k2),
 *     k4 = f(t+dt, v+dt k3), v(t+dt) = v + (k1 + 2k2 + 2k3 + k4)/6 dt
 *   boundary: zero boundary condition, eq. (BC), taken as a 2-cell zero halo
 *     around a cell-centred interior (the stencil needs j-2 at the first
 *     interior node; the paper does not state a ghost rule).  A periodic halo
 *     exists only for tests (closed forms for Fourier modes).
 *
 * Layout: interior arrays are C-ordered [nz][ny][nx] (x fastest).
 *
 * Pins: the test-suite checks this file against polynomial exactness of the
 * stencil, the RK4 stability polynomial, Bessel closed forms, a Kronecker-sum
 * assembly of the same operator on tiny grids integrated by an independent
 * ODE solver, the radial 1-D form, and the paper's printed facts.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define HBO_OK 0
#define HBO_E_ARG (-1)
#define HBO_E_NOMEM (-3)

#define HBO_BC_ZERO 0
#define HBO_BC_PERIODIC 1

/* order flags for the rounding-noise-floor variants (tests only) */
#define HBO_ORDER_TEXTBOOK 0      /* k1..k4 kept, combined at the end          */
#define HBO_ORDER_PAPER_REUSE 1   /* paper's storage-reuse ordering (sec. 2.1) */
#define HBO_ORDER_AXES_REVERSED 2 /* Laplacian summed z, y, x                  */

typedef struct {
    int nx, ny, nz;       /* interior points per axis                          */
    int px, py, pz;       /* padded extents: n + 4                             */
} grid_t;

static size_t pidx(const grid_t* g, int i, int j, int k) {
    /* padded index of interior coordinate (i, j, k); i, j, k may be -2..n+1 */
    return ((size_t)(k + 2) * (size_t)g->py + (size_t)(j + 2)) * (size_t)g->px + (size_t)(i + 2);
}

static size_t iidx(const grid_t* g, int i, int j, int k) {
    return ((size_t)k * (size_t)g->ny + (size_t)j) * (size_t)g->nx + (size_t)i;
}

static int wrap(int a, int n) {
    int r = a % n;
    return r < 0 ? r + n : r;
}

/* Refill the 2-cell halo: zeros (eq. (BC)) or a periodic copy (tests). */
static void fill_halo(const grid_t* g, double* u, int bc) {
    int k;
#pragma omp parallel for schedule(static)
    for (k = -2; k < g->nz + 2; ++k) {
        for (int j = -2; j < g->ny + 2; ++j) {
            for (int i = -2; i < g->nx + 2; ++i) {
                int inside = (i >= 0 && i < g->nx && j >= 0 && j < g->ny && k >= 0 && k < g->nz);
                if (inside) continue;
                if (bc == HBO_BC_PERIODIC)
                    u[pidx(g, i, j, k)] = u[pidx(g, wrap(i, g->nx), wrap(j, g->ny), wrap(k, g->nz))];
                else
                    u[pidx(g, i, j, k)] = 0.0;
            }
        }
    }
}

/* Fourth-order central second difference along one axis (section 2.1):
 * (-1/12 u[-2] + 4/3 u[-1] - 5/2 u[0] + 4/3 u[+1] - 1/12 u[+2]) / d^2 */
static double d2(const double* u, size_t c, ptrdiff_t s, double d) {
    return (-1.0 / 12.0 * u[c - 2 * s] + 4.0 / 3.0 * u[c - s] - 5.0 / 2.0 * u[c]
            + 4.0 / 3.0 * u[c + s] - 1.0 / 12.0 * u[c + 2 * s]) / (d * d);
}

static double lap_at(const grid_t* g, const double* u, int i, int j, int k,
                     double hx, double hy, double hz, int order) {
    size_t c = pidx(g, i, j, k);
    ptrdiff_t sx = 1, sy = g->px, sz = (ptrdiff_t)g->px * g->py;
    if (order == HBO_ORDER_AXES_REVERSED)
        return d2(u, c, sz, hz) + d2(u, c, sy, hy) + d2(u, c, sx, hx);
    return d2(u, c, sx, hx) + d2(u, c, sy, hy) + d2(u, c, sz, hz);
}

/* Laplacian of a caller-filled padded array (halo supplied by the caller). */
int hbo_laplacian(int nx, int ny, int nz, double hx, double hy, double hz,
                  const double* upad, double* out) {
    if (nx < 1 || ny < 1 || nz < 1 || !upad || !out) return HBO_E_ARG;
    grid_t g = {nx, ny, nz, nx + 4, ny + 4, nz + 4};
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i)
                out[iidx(&g, i, j, k)] = lap_at(&g, upad, i, j, k, hx, hy, hz, HBO_ORDER_TEXTBOOK);
    return HBO_OK;
}

typedef struct {
    double hx, hy, hz, mu2, lambda, inv_L2;
    int bc, order;
} params_t;

/* f(t, v) of eq. (rhs): fphi = psi, fpsi = -3 psi + c(t) Lap phi + mu2 phi - lambda phi^3.
 * phi_pad must have its halo filled; psi/fphi/fpsi are padded arrays too
 * (only their interior is read or written). */
static void rhs(const grid_t* g, const params_t* p, double t,
                const double* phi_pad, const double* psi_pad, double* fphi, double* fpsi) {
    double c = exp(-2.0 * t) * p->inv_L2;
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->nz; ++k) {
        for (int j = 0; j < g->ny; ++j) {
            for (int i = 0; i < g->nx; ++i) {
                size_t q = pidx(g, i, j, k);
                double v1 = phi_pad[q];
                double v2 = psi_pad[q];
                double lap = lap_at(g, phi_pad, i, j, k, p->hx, p->hy, p->hz, p->order);
                fphi[q] = v2;
                fpsi[q] = -3.0 * v2 + c * lap + p->mu2 * v1 - p->lambda * v1 * v1 * v1;
            }
        }
    }
}

/* dst = a + s * b over the interior, then refill dst's halo */
static void axpy_stage(const grid_t* g, double* dst, const double* a, double s, const double* b, int bc) {
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) {
                size_t q = pidx(g, i, j, k);
                dst[q] = a[q] + s * b[q];
            }
    fill_halo(g, dst, bc);
}

static void copy_in(const grid_t* g, double* pad, const double* in) {
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) pad[pidx(g, i, j, k)] = in[iidx(g, i, j, k)];
}

static void copy_out(const grid_t* g, double* out, const double* pad) {
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < g->nz; ++k)
        for (int j = 0; j < g->ny; ++j)
            for (int i = 0; i < g->nx; ++i) out[iidx(g, i, j, k)] = pad[pidx(g, i, j, k)];
}

/* One right-hand-side evaluation on interior arrays (tests). */
int hbo_rhs(int nx, int ny, int nz, double hx, double hy, double hz, double mu2, double lambda,
            double inv_L2, double t, int bc, const double* phi, const double* psi,
            double* fphi, double* fpsi) {
    if (nx < 1 || ny < 1 || nz < 1 || !phi || !psi || !fphi || !fpsi) return HBO_E_ARG;
    grid_t g = {nx, ny, nz, nx + 4, ny + 4, nz + 4};
    size_t np = (size_t)g.px * g.py * g.pz;
    double* buf = (double*)calloc(4 * np, sizeof(double));
    if (!buf) return HBO_E_NOMEM;
    double *ph = buf, *ps = buf + np, *f1 = buf + 2 * np, *f2 = buf + 3 * np;
    copy_in(&g, ph, phi);
    copy_in(&g, ps, psi);
    fill_halo(&g, ph, bc);
    fill_halo(&g, ps, bc);
    params_t p = {hx, hy, hz, mu2, lambda, inv_L2, bc, HBO_ORDER_TEXTBOOK};
    rhs(&g, &p, t, ph, ps, f1, f2);
    copy_out(&g, fphi, f1);
    copy_out(&g, fpsi, f2);
    free(buf);
    return HBO_OK;
}

/* Classical RK4, steps n = step0 .. step0+nsteps-1 with t_n = t0 + n dt.
 * phi, psi: interior arrays, updated in place. */
int hbo_solve(int nx, int ny, int nz, double hx, double hy, double hz, double mu2, double lambda,
              double inv_L2, double t0, double dt, long long step0, long long nsteps, int bc,
              int order, double* phi, double* psi) {
    if (nx < 1 || ny < 1 || nz < 1 || !phi || !psi || nsteps < 0 || step0 < 0) return HBO_E_ARG;
    if (bc != HBO_BC_ZERO && bc != HBO_BC_PERIODIC) return HBO_E_ARG;
    grid_t g = {nx, ny, nz, nx + 4, ny + 4, nz + 4};
    size_t np = (size_t)g.px * g.py * g.pz;
    /* v (2), stage input u (2), k1..k4 (2 each) */
    double* buf = (double*)calloc(12 * np, sizeof(double));
    if (!buf) return HBO_E_NOMEM;
    double *y1 = buf, *y2 = buf + np, *u1 = buf + 2 * np, *u2 = buf + 3 * np;
    double *k1a = buf + 4 * np, *k1b = buf + 5 * np, *k2a = buf + 6 * np, *k2b = buf + 7 * np;
    double *k3a = buf + 8 * np, *k3b = buf + 9 * np, *k4a = buf + 10 * np, *k4b = buf + 11 * np;
    params_t p = {hx, hy, hz, mu2, lambda, inv_L2, bc, order};

    copy_in(&g, y1, phi);
    copy_in(&g, y2, psi);
    fill_halo(&g, y1, bc);
    fill_halo(&g, y2, bc);

    for (long long n = step0; n < step0 + nsteps; ++n) {
        double t = t0 + (double)n * dt;
        if (order == HBO_ORDER_PAPER_REUSE) {
            /* The paper's storage-reuse ordering (section 2.1): after k2 the
             * first slot holds k1 + 2 k2, k3 keeps its slot, the second slot
             * is refilled with k4, and the update is (k1+2k2) + 2 k3 + k4.
             * Algebraically identical to the textbook form; rounding differs. */
            rhs(&g, &p, t, y1, y2, k1a, k1b);
            axpy_stage(&g, u1, y1, dt / 2.0, k1a, bc);
            axpy_stage(&g, u2, y2, dt / 2.0, k1b, bc);
            rhs(&g, &p, t + dt / 2.0, u1, u2, k2a, k2b);
            int k;
#pragma omp parallel for schedule(static)
            for (k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        size_t q = pidx(&g, i, j, k);
                        k1a[q] = k1a[q] + 2.0 * k2a[q];
                        k1b[q] = k1b[q] + 2.0 * k2b[q];
                    }
            axpy_stage(&g, u1, y1, dt / 2.0, k2a, bc);
            axpy_stage(&g, u2, y2, dt / 2.0, k2b, bc);
            rhs(&g, &p, t + dt / 2.0, u1, u2, k3a, k3b);
            axpy_stage(&g, u1, y1, dt, k3a, bc);
            axpy_stage(&g, u2, y2, dt, k3b, bc);
            rhs(&g, &p, t + dt, u1, u2, k2a, k2b);
#pragma omp parallel for schedule(static)
            for (k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        size_t q = pidx(&g, i, j, k);
                        y1[q] = y1[q] + (k1a[q] + 2.0 * k3a[q] + k2a[q]) / 6.0 * dt;
                        y2[q] = y2[q] + (k1b[q] + 2.0 * k3b[q] + k2b[q]) / 6.0 * dt;
                    }
        } else {
            rhs(&g, &p, t, y1, y2, k1a, k1b);
            axpy_stage(&g, u1, y1, dt / 2.0, k1a, bc);
            axpy_stage(&g, u2, y2, dt / 2.0, k1b, bc);
            rhs(&g, &p, t + dt / 2.0, u1, u2, k2a, k2b);
            axpy_stage(&g, u1, y1, dt / 2.0, k2a, bc);
            axpy_stage(&g, u2, y2, dt / 2.0, k2b, bc);
            rhs(&g, &p, t + dt / 2.0, u1, u2, k3a, k3b);
            axpy_stage(&g, u1, y1, dt, k3a, bc);
            axpy_stage(&g, u2, y2, dt, k3b, bc);
            rhs(&g, &p, t + dt, u1, u2, k4a, k4b);
            int k;
#pragma omp parallel for schedule(static)
            for (k = 0; k < nz; ++k)
                for (int j = 0; j < ny; ++j)
                    for (int i = 0; i < nx; ++i) {
                        size_t q = pidx(&g, i, j, k);
                        y1[q] = y1[q] + dt / 6.0 * (k1a[q] + 2.0 * k2a[q] + 2.0 * k3a[q] + k4a[q]);
                        y2[q] = y2[q] + dt / 6.0 * (k1b[q] + 2.0 * k2b[q] + 2.0 * k3b[q] + k4b[q]);
                    }
        }
        fill_halo(&g, y1, bc);
        fill_halo(&g, y2, bc);
    }
    copy_out(&g, phi, y1);
    copy_out(&g, psi, y2);
    free(buf);
    return HBO_OK;
}

void hbo_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int hbo_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Bubble count (section 1: a bubble is a maximal connected set of points at
 * which the solution changes sign).  On the grid, the sign classes are the
 * node sets {phi < -eps} and {phi > eps} (eps >= 0; eps = 0 is the sign
 * itself, a positive eps ignores values of magnitude <= eps), and two nodes
 * are connected when they are face neighbours (6-connectivity); with
 * periodic boundaries the neighbour index wraps, otherwise the grid ends at
 * the boundary.  *nneg and *npos receive the number of maximal connected
 * sets of each class.  Plain breadth-first flood fill from every unvisited
 * node in index order, with an explicit queue.  NaN belongs to neither class.
 */
static int sign_class(double v, double eps) {
    if (v < -eps) return 1;
    if (v > eps) return 2;
    return 0;
}

int hbo_components(int nx, int ny, int nz, int bc, const double* phi, double eps,
                   long long* nneg, long long* npos) {
    if (nx < 1 || ny < 1 || nz < 1 || !phi || !nneg || !npos || !(eps >= 0.0)) return HBO_E_ARG;
    const grid_t g = {nx, ny, nz, nx + 4, ny + 4, nz + 4};
    const size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
    unsigned char* seen = (unsigned char*)calloc(n, 1);
    size_t* queue = (size_t*)malloc(n * sizeof(size_t));
    if (!seen || !queue) {
        free(seen);
        free(queue);
        return HBO_E_NOMEM;
    }
    long long count[3] = {0, 0, 0};
    for (size_t start = 0; start < n; ++start) {
        const int cls = sign_class(phi[start], eps);
        if (cls == 0 || seen[start]) continue;
        count[cls] += 1;
        size_t head = 0, tail = 0;
        queue[tail++] = start;
        seen[start] = 1;
        while (head < tail) {
            const size_t at = queue[head++];
            const int i = (int)(at % (size_t)nx);
            const int j = (int)((at / (size_t)nx) % (size_t)ny);
            const int k = (int)(at / ((size_t)nx * (size_t)ny));
            for (int d = 0; d < 6; ++d) {
                int a = i, b = j, c = k;
                const int step = (d & 1) ? 1 : -1;
                if (d < 2) a += step;
                else if (d < 4) b += step;
                else c += step;
                if (bc == HBO_BC_PERIODIC) {
                    a = wrap(a, nx);
                    b = wrap(b, ny);
                    c = wrap(c, nz);
                } else if (a < 0 || a >= nx || b < 0 || b >= ny || c < 0 || c >= nz) {
                    continue;
                }
                const size_t nb = iidx(&g, a, b, c);
                if (!seen[nb] && sign_class(phi[nb], eps) == cls) {
                    seen[nb] = 1;
                    queue[tail++] = nb;
                }
            }
        }
    }
    free(seen);
    free(queue);
    *nneg = count[1];
    *npos = count[2];
    return HBO_OK;
}
