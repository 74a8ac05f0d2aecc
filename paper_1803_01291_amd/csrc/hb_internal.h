// Internal layouts shared by the HIP kernels and the host runtime of libhb.
//
// Field layout in HBM (one allocation per solve, all fields alike):
//   cell (x, y, z), x in [-2, nx+2), y in [-2, ny+2), z in [-2, nz+2), holds
//   its value at element cs * (z*sz + y*sy + x) from the field's origin (the
//   interior point (0, 0, 0)).  cs = 1 for separate fields.  Whole-step
//   solves keep a cell's state in one 16-byte slot, one field per step
//   parity: (phi, psi) in FP64 (cs = 2) or (phi hi, psi hi, phi lo, psi lo)
//   in FP32c (cs = 4), so a cell's state moves in one 16-byte access; the
//   psi view is the phi view plus one element, the low parts follow at two
//   and three elements.  The row pitch
//   sy is nx+4 rounded up to a 128-byte multiple of cells and cell (0, y, z)
//   starts a 128-byte line.  The 2-cell halo (the zero boundary condition) is
//   zeroed once at creation and never written afterwards; periodic solves
//   never read it (their neighbour indices wrap into the interior).
#pragma once

#include <stdint.h>

namespace hb {

// precision of a solve
enum : int { PREC_F64 = 0, PREC_F32C = 1 };

// One solve as the stage kernels see it (device resident, 128-byte aligned).
struct SolveDesc {
    void* y_phi[2];      // state phi (FP64) or its FP32 high part, ping-pong by step parity
    void* y_psi[2];      // state psi, same (whole-step slot: y_phi[p] + one element)
    void* g[3];          // psi-forcing of stages 1..3 (G1, G2, G3; separate fields only)
    float* lo_phi;       // FP32c, separate fields: low parts of the compensated state
    float* lo_psi;       // (updated in place); whole-step solves keep them in the state slot
    const double* ctab;  // c(t) per stage: ctab[4 n + s], s = 0..3
    long long sy, sz;    // row and plane pitch in cells
    int nx, ny, nz, prec;
    int cs;              // elements per cell: 1 (separate fields), 2 or 4 (whole-step state slot)
    int periodic;        // 1: periodic boundaries (whole-step kernel and diagnostics), 0: zero halo
    double w0;           // -5/2 (1/hx^2 + 1/hy^2 + 1/hz^2)
    double w1[3];        // 4/3 / h_d^2
    double w2[3];        // -1/12 / h_d^2
    double mu2, lambda, dt, hdt, dt6;
    long long nstep;     // steps completed (advanced by the tick kernel)
    long long target;    // stepping stops when nstep reaches target
    long long pad_[2];
};

// One block of work: an x-y tile of 64 x BY columns over z in [z0, z1).
struct Tile {
    int solve;  // index into the launch group's descriptor array
    int x0, y0, z0, z1;
    int pad_[3];
};

constexpr int TILE_X = 64;

// Launchers (implemented in hb_kernels.hip).  All are asynchronous on `stream`.
int launch_stage(int prec, int stage, int by, const SolveDesc* descs, const Tile* tiles,
                 int ntiles, long long kstep, void* stream);
// Stage-pair kernels: pair 0 = stages 1+2 (writes G1, G2), pair 1 = stages 3+4
// (writes the next state).  Bitwise equal to the four per-stage launches.
int launch_pair(int prec, int pair, int by, const SolveDesc* descs, const Tile* tiles, int ntiles,
                long long kstep, void* stream);
// Whole-step kernel: one launch per RK4 step, on paired-state solves (cs = 2).
// A block's threads own an rx x ry region: its interior tile of
// (rx - 4) x (ry - 4) columns plus a 2-cell ring.  Shapes (`shape` indexes
// this table), one block per CU: 36 x 28 (1008 threads; tiles 32 columns
// wide), 64 x 16 (1024 threads; a region row is one wave), 68 x 15 (1020
// threads; tiles 64 columns wide, which cover multiples of 64 exactly and
// start on 128-byte lines) and 36 x 20 (720 threads, three waves per SIMD;
// 32 x 16 tiles, which cover a 256 x 256 plane in 128 tiles, so two z-chunks
// of a 256^3 grid fill one round of 256 CUs).  Bitwise equal to the
// stage-pair kernels.
struct StepShape {
    int rx, ry, blocks_per_cu;
};
constexpr StepShape STEP_SHAPES[4] = {{36, 28, 1}, {64, 16, 1}, {68, 15, 1}, {36, 20, 1}};
// periodic: some solve of the launch has periodic boundaries (selects the
// kernel that reads each descriptor's boundary; else the zero-halo kernel)
int launch_step(int prec, int shape, const SolveDesc* descs, const Tile* tiles, int ntiles,
                long long kstep, bool periodic, void* stream);
int launch_tick(SolveDesc* descs, int count, long long k, void* stream);
int launch_set_target(SolveDesc* descs, int index, long long target, void* stream);
int launch_set_nstep(SolveDesc* descs, int index, long long nstep, long long target, void* stream);

// Contiguous user array [nz][ny][nx] of src_dtype (0 = f64, 1 = f32) into a
// pitched field (cs elements per cell).  FP64 fields take the value; FP32c fields take
// hi = (float)v and lo = (float)(v - hi).  `src` may be NULL for zeros.
// quiet NaNs into every cell of one field (field start address, `cells`
// cells of cs elements of esz bytes) outside the interior and its 2-cell
// halo; corner = cell index of (-2, -2, -2), sz = sy * (ny + 4)
int launch_poison(void* field, long long cells, int esz, int cs, long long corner, long long sy,
                  long long sz, int nx, int nz, void* stream);
int launch_unpack(int prec, int src_dtype, const void* src, int nx, int ny, int nz, long long sy,
                  long long sz, int cs, void* hi, float* lo, void* stream);
// Pitched field into a contiguous user array of dst_dtype (FP32c: hi + lo in FP64).
int launch_pack(int prec, int dst_dtype, void* dst, int nx, int ny, int nz, long long sy,
                long long sz, int cs, const void* hi, const float* lo, void* stream);

// Diagnostics: per-block partials then one fixed-order final pass (deterministic).
enum { DIAG_SUM_PHI = 0, DIAG_SUM_PHI2, DIAG_SUM_PSI2, DIAG_MAX_PHI, DIAG_MAX_PSI, DIAG_MAX_LAP,
       DIAG_ENERGY, DIAG_NONFINITE, DIAG_NEGATIVE, DIAG_COUNT };
int diag_partials_needed(int nx, int ny, int nz);
int launch_diagnostics(int prec, const SolveDesc* desc, int parity, double c, double* partials,
                       int nparts, double* out, void* stream);

// Bubbles (section 1): the number of face-connected node sets of {phi < -eps}
// (counts[0]) and of {phi > eps} (counts[1]) over the interior (periodic
// solves wrap).  labels: `points` (< 2^32 - 1) entries of scratch; counts:
// two entries, written by the launch.
int launch_bubbles(int prec, const SolveDesc* desc, int parity, double eps, long long points,
                   unsigned* labels, unsigned long long* counts, void* stream);

// Bandwidth probe: kind 0 = copy (1 read, 1 write), 1 = add (2 reads, 1 write),
// 2 = 5 reads + 2 writes (the FP64 stage-4 stream mix).  n16 elements of 16 B.
int launch_probe(int kind, void* const* in, void* const* out, long long n16, int blocks,
                 void* stream);

// Batched radial solves (section 2.2 form): one workgroup per solve, state in
// LDS, all steps in one launch.  phi/psi hold the solves back to back.
struct RadialDesc {
    long long offset;  // first node of this solve in phi/psi
    long long steps;
    long long ctab;    // first entry of this solve's c(t) rows in the launch's table:
                       // ctab[ctab + 3 (n - n0) + {0, 1, 2}] = c at t_n, t_n + dt/2, t_n + dt
    int m;             // nodes r_i = i dr, i = 0..m-1 (phi = 0 at r = m dr)
    int pad_;
    double dr, mu2, lambda, inv_L2, t0, dt;
};
size_t radial_lds_bytes(int max_m);
// Device scratch of the entry point that allocates nothing (descriptors and
// c(t) table): its size, and its address on the current device (looked up
// once per device; 0, or a HIP error code on failure).
constexpr size_t RADIAL_SCRATCH_BYTES = (size_t)8 << 20;
int radial_scratch(void** ptr);
// steps n0 <= n < min(n1, steps) of every solve (state read from and
// written back to phi, psi); ctab holds each solve's c(t) rows for those steps
int launch_radial(const RadialDesc* descs, const double* ctab, int count, int max_m, double* phi,
                  double* psi, long long n0, long long n1, void* stream);

}  // namespace hb
