// Internal declarations of the lbm3 HIP library (not part of the C ABI).
#pragma once
#include <stddef.h>
#include <stdint.h>

namespace lbm3k {

// Everything the kernels need, passed by value as a kernel argument.
struct KParams {
    int D, Q;            // 2/9 or 3/27
    int nx, ny, nz;      // grid
    int nw;              // extent of the wall (last) axis
    int walls;           // 1: ghost layers at 0 and nw-1 of the last axis
    long long N;         // nodes
    long long PS;        // plane stride of the last axis (nx or nx*ny)
    long long QS;        // elements from one array of a block to the next (array_stride(N))
    double rho_l, rho_g, drho, chi;
    double a, b, T, C, psi0;
    double lam1, lam2, lam3;
    double krr, kpp, kx;         // gradient mixing coefficients
    double beta, inv_tau_g, Gamma;
    int wetting;                 // 0 force, 1 geometric interpolation, 2 extrapolation
    double cot[2][3];            // per wall: cot(theta21), cot(theta31), cot(theta23)
    double kw[2][2];             // per wall: kappa_rho^w, kappa_phi^w
    double alpha_eps, alpha_tol;
    int alpha_maxit;
    double detect_ratio;         // first interface-detection rule's threshold
    unsigned flags;              // 1 no-collide, 2 alpha = 2, 4 one fused kernel in 3D
};

constexpr unsigned kFlagFused3D = 4u;

// alpha statistics: blocks add into one of kCntSlots slots (by block index),
// each a 128-byte line, so a launch's atomics do not queue on one address;
// the reader sums the slots.  The small 2D fused kernel instead keeps one
// slot per block after those (small2d_block_slots of them), which the block
// owns: it reads its running counts with the fields and stores the sums at
// its end, without atomics (whose completion held the end of every launch).
constexpr int kCntSlots = 64, kCntStride = 16;
// the small 2D tile class: below kSmall2DNodes nodes, tiles of kSmall2DTX
constexpr long long kSmall2DNodes = 1LL << 20;
constexpr int kSmall2DTX = 62;
// per-block slots of the small 2D class for a D-dimensional nx x nw grid
// (nw: nodes along the wall axis), 0 for the other classes
inline long long small2d_block_slots(int D, long long nx, long long nw)
{
    return (D == 2 && nx * nw < kSmall2DNodes) ? ((nx + kSmall2DTX - 1) / kSmall2DTX) * nw : 0;
}

enum Prec { P64 = 0, P32 = 1, P16 = 2 };

// Element stride between consecutive arrays of one block (the Q populations
// of a set, the force components, the five g^eq values) and the size of each
// field array: N rounded up to 64 nodes, plus 544 when that is a multiple of
// 16384.  Arrays a large power of two apart (256^3 FP32: 127 x 512 KiB) start
// on the same memory channels, and 27 or 54 of them streamed together then
// read at 5.1 TB/s and push-copy at 3.8; 544 nodes further apart they reach
// 6.2 and 4.6, the rates of grids whose size is not such a multiple.
inline long long array_stride(long long N)
{
    long long q = (N + 63) / 64 * 64;
    if (q % 16384 == 0) q += 544;
    return q;
}

// Device buffers of one simulation, carved out of the caller's workspace.
struct Buffers {
    void *f[2], *g[2];           // populations [Q][QS], storage type by precision
    void *rho[2], *phi[2];       // fields [N], compute type
    void *fmu;                   // 3D two-kernel step: F, mu_phi [D + 1][QS], compute type
    void *gp;                    // implicit-g step: (a, phi, v) of g^eq [5][QS], compute type (FP32 with
                                 // FP16 storage), or null
    double *scratch;             // N doubles (upload / export staging)
    unsigned long long *counters;// kCntSlots (+ per-block) slots of kCntStride: newton, shortcut, fallback
    double *partials;            // reduction partials
    double *result;              // 32 doubles of reduced observables
    int n_partials;              // capacity in blocks
};

// One simulation of a batched launch (device copy written by the host).
struct SimDesc {
    KParams kp;
    void *f[2], *g[2], *rho[2], *phi[2];
    unsigned long long *counters;
    int pc, fc;               // buffer parities when the descriptors were written
    int chunk, ntiles;        // fused launch geometry of this simulation
    void *fmu;                // F, mu_phi of the 3D two-kernel step
    int fblk0, mblk0, gblk0;  // its first block in the fused (or stencil), moments and ghost launches
    int cblk0;                // and in the collide launch of the 3D two-kernel step
    void *gp;                 // implicit-g values (a, phi, v), or null
    int gimp0;                // g[pc] implicit (in gp) when the descriptors were written
    int mchunk;               // planes per block of its moments march (moments_march_chunk)
};

// Fused launch geometry of one simulation: tile class (0: 2D 62-node tiles,
// 1: 2D 254-node tiles, 2: 3D 32x16 tiles (32x4 in FP64), 3: 3D 32x8 tiles
// (32x4 in FP64) in the stencil pass of the two-kernel step), in-plane
// tiles, planes per block and blocks along the wall axis.
struct FusedGeom {
    int cls, ntiles, chunk, nchunks;
};

// Launchers (lbm3_kernels.hip).  All asynchronous on `stream`.
int launch_moments(const KParams &kp, int prec, const Buffers &b, int pc, int fc, void *stream);
// implicit-g step (b.gp set): the moments pass that rebuilds g from b.gp, and
// the kernel that writes that g out into b.g[pc]
int launch_moments_imp(const KParams &kp, int prec, const Buffers &b, int pc, int fc, void *stream);
int launch_g_materialize(const KParams &kp, int prec, const Buffers &b, int pc, int fc, void *stream);
int launch_ghost(const KParams &kp, int prec, const Buffers &b, int fdst, void *stream);
int launch_fused(const KParams &kp, int prec, const Buffers &b, int pc, int fc, void *stream);
// events (hipEvent_t, or null) the next launch_moments / launch_ghost /
// launch_fused stage records from its first kernel's start and its last
// kernel's end, and in a two-kernel stage also from the first kernel's end
// (sub_stop) and the second kernel's start (sub_start); set by the profiled
// step, cleared with nulls
void set_stage_events(void *start, void *stop, void *sub_stop, void *sub_start);
// true when the fused kernel fills the wall ghost layers itself (2D)
bool fused_fills_ghost(const KParams &kp);
// true when the step's last stage is the stencil pass plus the collide
// kernel (3D unless the one-kernel flag is set)
bool two_kernel_step(const KParams &kp);
int launch_init(const KParams &kp, int prec, const Buffers &b, void *stream);
int launch_init_field(const KParams &kp, int prec, const Buffers &b, int which, void *stream);
int launch_observe(const KParams &kp, int prec, const Buffers &b, int pc, int fc, void *stream);
int launch_export_pop(const KParams &kp, int prec, const Buffers &b, int pc, int fc, int which,
                      int i, void *stream);
int launch_export_field(const KParams &kp, int prec, const Buffers &b, int fsrc, int which,
                        void *stream);
int launch_contour(const KParams &kp, int prec, const Buffers &b, int fsrc, int comp, int wall,
                   double exclude, void *stream);
int observe_blocks(const KParams &kp);

// Batched launches over simulations of one class: blocks b = 0..nblocks-1
// belong to simulation sim[b] of the device descriptor array d.
FusedGeom fused_geometry(const KParams &kp, int prec);
long long moments_blocks(const KParams &kp, int prec);
// the batched moments launch: the march for a simulation with an
// implicit-g array (3D, tau_g = 1), else moments_blocks
long long moments_batch_blocks(const KParams &kp, int prec, bool implicit);
// planes per block of the moments march of a 3D simulation
int moments_march_chunk(const KParams &kp);
long long ghost_blocks(const KParams &kp);  // 0 when the step has no ghost launch
long long collide_blocks(const KParams &kp);  // 0 unless the step is two-kernel
// first: the first step since the descriptors were written (a simulation's
// g is then implicit if gimp0 says so, afterwards whenever gp is set)
int launch_moments_batch(int D, int prec, const SimDesc *d, const int *sim, long long nblocks, int phase,
                         bool first, void *stream);
int launch_ghost_batch(int D, int prec, const SimDesc *d, const int *sim, long long nblocks, int phase,
                       void *stream);
int launch_fused_batch(int cls, int prec, const SimDesc *d, const int *sim, long long nblocks, int phase,
                       void *stream);
// implicit: every simulation of the table has implicit g (gp set)
int launch_collide_batch(int D, int prec, bool implicit, const SimDesc *d, const int *sim, long long nblocks,
                         int phase, void *stream);

}  // namespace lbm3k
