// Device-side instance record and kernel launchers (internal).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "lee_internal.h"

namespace lee {

// One instance as the kernels see it; lives in device memory (an array of
// them forms a batch table).  Field planes point at the start of their
// allocation; node (i, j) sits at element org + j * pitch + i (always a
// non-negative 32-bit offset, frame rows included); the frame and padding
// around the domain hold 0.
struct DevInst {
    void *f[3][3];          // [register set A, B, C][p, u, v]; A holds q^n
    void *psi[3];           // ADE states per register set, ade_ns per ghost
    const int4 *iv;         // per row: fluid columns [x, y) and [z, w)
    const int *goff;        // ghost plane offsets (from the plane start)
    const int *cptr;        // cloud CSR pointers (G + 1)
    const int *coff;        // cloud plane offsets (from the plane start)
    const void *w4;         // 4 weights per cloud entry (T)
    const void *gd;         // per ghost: n_x, n_y, beta_D, beta_N (T)
    long long *step;        // first step of the current run (completed steps between runs)
    long long *stop;        // the member takes the steps below this one
    const int *pij;         // probe stencil origins
    const double *pw;       // probe weights, 16 per probe
    double *trace;          // ring of trace_cap steps x np x 3
    double *dft;            // 2 per probe: sum p exp(-i omega t)
    double *watch;          // ring of watch_cap steps x (p_BP, u_n,BP, fluid u_n) of ghost watch_g
    unsigned long long *xg; // ghost values of the current stage for fused launches: per ghost
                            // and field, sizeof(T)/4 words of (32 value bits | stage epoch << 32)
    long long watch_cap;
    int watch_g;            // -1: none
    long long trace_cap;
    long long dft_start, dft_count;
    double dft_omega;
    int np;
    int nx, ny, pitch, G;
    int org;                // element offset of node (0, 0) in a plane
    int sponge_w, has_src, ade_kind;
    int ade_ns;             // auxiliary states per ghost (2 for kinds 0-2)
    int src_ic, src_jc;     // source's nearest node
    int src_i0, src_i1, src_j0, src_j1;  // node box outside which the source underflows
    double x0, y0, h, dt;
    double ax[5];           // a_k / h (zero beyond the stencil half-width)
    float axf[5];           // the same in FP32
    float fdf[6];           // fd in FP32
    double fd[6];           // (sigma_d / dt) * (2 d_0, d_1 .. d_5): damping of D_x + D_y
    double fdw[6][6];       // per axis, a node whose filter row has half-width w < 5 (no
                            // non-fluid node of the domain within w along that axis) takes
                            // fd + fdw[w]: (sigma_d / dt) * (b_0 - d_0, b_1 - d_1, .., -d_5)
                            // with b the standard centred filter of half-width w (none for
                            // w = 0); row 5 is zero
    float fdwf[6][6];       // the same in FP32
    double alpha_dt[4];     // alpha_l dt
    double c_stage[4];      // stage time offsets c_l (in steps)
    double sponge_s;
    double sponge_inv;      // 1 / sponge_w
    double src_a, src_b, src_om, src_fx, src_fy;
    double ade[4];
    double ade_st[8][5];    // kind 3: per state a, bn, bp, f, c of
                            // dX_k = a X_k + bn X_{k+1} + bp X_{k-1} + f p_BP, u_n = sum c X_k
    int rad_w;              // radiation band width (nodes closer than rad_w to an edge; 0 = none)
    int fx;                 // the filter once per step (k_filter) instead of in the stages' RHS:
                            // the last stage writes register set C and fd, fdw hold sigma_d times the rows
    double rad_xc, rad_yc;  // its centre
    double rad_w7[7][7];    // first-derivative weights / h on a 7-node window, node at place r:
                            // r = 3 the central set a_k, else the one-sided maximal-order set
    float rad_wf[7][7];
    int stream;             // stage outputs take non-temporal stores (planes larger than the on-chip cache)
    int stream_in;          // the halo copy of a stage input other than q^n takes non-temporal loads
                            // (planes larger than the on-chip cache, the q^n planes not)
};

// Probe sampling carried by a launch: the (member, probe) pairs pw[0, np),
// for step *step + rel of each member that took that step (np = 0: none;
// member -1: an idle entry).
struct ProbePass {
    const int2 *pw;
    int np;
    int rel;
};

// Stage launches act on step *step + slot of each member (slot = the step's
// place in the current run).
hipError_t launch_sweep(int prec, int vec, bool filt, int waves, const DevInst *insts, const int4 *work,
                        int nwork, int stage, int slot, int blocks, hipStream_t s);
bool tile_shape_supported(int prec, int tx, int ty);
// The explicit filter after step `slot` of a run, one workgroup per tile
// item of the tile sweep's list (shape tx x ty): members with fx set take
// q <- q - sigma_d (F_x + F_y) q from register set C into register set A.
hipError_t launch_filter(int prec, int tx, int ty, const DevInst *insts, const int4 *work, int nwork, int slot,
                         hipStream_t s);
hipError_t launch_tile(int prec, bool filt, int tx, int ty, const DevInst *insts, const int4 *work, int nwork,
                       int stage, int slot, int blocks, hipStream_t s);
// One launch for a stage with the tile sweep: the first ceil(nwork2 / 8)
// workgroups fill 8 ghosts each, tile k runs in workgroup tile0 + k (the
// caller keeps dependent tiles out of the carrier workgroups).  Items flagged
// with TILE_DEP_BIT wait for the ghost values they read and patch them in:
// aux[k] = [begin, end) in patch, whose entries are (LDS element index in the
// tile's copy, ghost index * 3 + field).  sync[4] is the error flag raised by
// a wait that runs out of polls (zero before first use).  The probe pass
// runs in extra workgroups after the tiles.
// ninst: 1 for a single instance (the ghost fill reads its record with
// scalar loads), any other value for a table indexed by the work items.
// poles: some instance of the launch has a multi-pole wall (ADE kind 3);
// only then is the ghost fill's multi-pole code compiled in.
// Work items with instance -1 (ghost and sweep lists) are idle, so a batch
// can pad its lists to fixed capacities.
hipError_t launch_stage(int prec, bool filt, int tx, int ty, const DevInst *insts, int ninst, bool poles,
                        const int4 *work1, int nwork1, const int2 *aux, const int2 *patch, int tile0,
                        const int4 *work2, int nwork2, int stage, int slot, int *sync, int spin_limit, ProbePass pp,
                        hipStream_t s);
constexpr int TILE_DEP_BIT = 1 << 30;
// Sweep items whose read region holds a ghost node (in either launch form):
// their rows take the near-wall filter rows (fdw).
constexpr int TILE_WALL_BIT = 1 << 29;
constexpr int TILE_INST_MASK = TILE_WALL_BIT - 1;
constexpr int SYNC_INTS = 8;
constexpr int SPIN_LIMIT = 1 << 20;             // polls before a ghost wait gives up (about a second)
// The ghost fill of a stage, with the probe pass in extra workgroups (ninst,
// poles and work as for launch_stage).
hipError_t launch_ghost(int prec, const DevInst *insts, int ninst, bool poles, const int4 *work, int nwork,
                        int stage, int slot, ProbePass pp, hipStream_t s);
hipError_t launch_probe(int prec, const DevInst *insts, ProbePass pp, hipStream_t s);
// After a run of n steps: *step += n for each of the ninst table entries,
// held at *stop.
hipError_t launch_advance(const DevInst *insts, int ninst, int n, hipStream_t s);
hipError_t launch_fill(int prec, void *p, size_t n, hipStream_t s);
// sync words: dst[4] |= src[4] (the ghost-wait error flag)
hipError_t launch_merge_flag(const int *src, int *dst, hipStream_t s);
hipError_t launch_fill_bytes(void *p, size_t bytes, hipStream_t s);
hipError_t launch_init_ic(int prec, const DevInst *insts, int nx, int ny, int kind, const double *c,
                          hipStream_t s);
hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s);
hipError_t launch_sample(int prec, const DevInst *insts, const int *ij, const double *w, int np, double *out,
                         hipStream_t s);

}  // namespace lee
