// HIP kernels for gfx950 (MI355X): one Runge-Kutta stage of the 2-D LEE with
// a ghost-point immersed boundary and the two-state MSD ADE.
//
//   k_ghost     Sec. 3.2 steps 1-5: per ghost, gathers its cloud of the stage
//               input with the four composed weights (p_BP read-out, free,
//               Dirichlet, Neumann), advances the ADE derivative, and writes
//               the ghost values and the stage value of the ADE states.
//   k_tile      Sec. 3.2 step 6: DRP first derivatives (eq. DRP_s) in x and y,
//               11-point selective-filter damping, sponge, monopole source and
//               the low-storage RK stage update at every fluid node of a tile;
//               the workgroup copies the tile and its 5-node halo into LDS
//               (direct global-to-LDS loads) and computes one row of VEC nodes
//               per lane.
//   k_stage     k_ghost and k_tile in one launch: the first workgroups fill
//               the ghosts before their tiles; tiles that read ghost nodes
//               wait for them and patch their LDS copy.
//   k_sweep     the same sweep with a wave marching a strip of 64 VEC - 16
//               columns down a run of rows and keeping the 11-row window of p,
//               u, v in registers (the centre row goes through LDS for the x
//               neighbours); alternate runs march in opposite directions so
//               that vertically adjacent runs read their shared halo rows at
//               about the same time (L2 reuse).
//   probes      sampling of the 8- or 360-point probe sets and their DFT, in
//               extra workgroups of a later stage launch (k_probe at the end
//               of a run); k_advance moves the step counters.
//
// No matrix cores: the stage is a stencil over three fields, bound by memory
// traffic and, within a one-wave launch, by the vector ALU (about 110 FP32
// operations per node).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "lee_device.h"
#include <type_traits>

namespace lee {

template <typename T, int N>
struct alignas(sizeof(T) * N) VecT {
    T v[N];
};

// Pointers read from the instance record are generic; casting them to the
// global address space lets the compiler emit global (not flat) memory
// instructions and know that they never alias LDS.
#if defined(__HIP_DEVICE_COMPILE__)
#define GLOBAL __attribute__((address_space(1)))
#else
#define GLOBAL
#endif
template <typename T>
__device__ __forceinline__ GLOBAL T *gp(void *p)
{
    return (GLOBAL T *)p;
}
template <typename T>
__device__ __forceinline__ const GLOBAL T *gp(const void *p)
{
    return (const GLOBAL T *)p;
}
template <typename T, int N>
__device__ __forceinline__ VecT<T, N> vld(const GLOBAL T *p)
{
    return *(const GLOBAL VecT<T, N> *)p;
}
template <typename T, int N>
__device__ __forceinline__ void vst(GLOBAL T *p, const VecT<T, N> &v)
{
    *(GLOBAL VecT<T, N> *)p = v;
}

// An 8- or 16-byte store marked non-temporal: a stage's output is read back only by
// the next launch, so where the planes do not fit the on-chip cache it need not
// claim L2 lines that the tiles' halo reads share (measured: the 4096^2 step 5%
// shorter in FP32 and FP64; the 1024^2 FP64 step, whose planes fit, 3-10% longer;
// non-temporal loads of q^n were slower).
template <int B>
struct StreamWord;
template <>
struct StreamWord<8> {
    typedef unsigned type __attribute__((ext_vector_type(2)));
};
template <>
struct StreamWord<16> {
    typedef unsigned type __attribute__((ext_vector_type(4)));
};
template <typename T, int N>
__device__ __forceinline__ void vst_stream(GLOBAL T *p, const VecT<T, N> &v)
{
    using W = typename StreamWord<sizeof(VecT<T, N>)>::type;
    W w;
    __builtin_memcpy(&w, &v, sizeof(W));
    __builtin_nontemporal_store(w, (GLOBAL W *)p);
}

// Orders this wave's LDS writes before its following LDS reads.  Each wave owns
// its LDS rows, so no workgroup barrier is needed (and waves of one workgroup
// may march tiles of different lengths).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// stage -> buffer roles: input q^(l-1), output q^(l); q^n is buffer 0
__device__ __forceinline__ int in_buf(int stage) { return stage == 0 ? 0 : (stage == 2 ? 2 : 1); }
__device__ __forceinline__ int out_buf(int stage) { return stage == 0 ? 1 : (stage == 1 ? 2 : (stage == 2 ? 1 : 0)); }

// Steps of a run: the launches of the run's step `slot` act on step
// *I.step + slot of each member (*I.step is advanced only between runs), and
// a member takes the steps below *I.stop.
__device__ __forceinline__ long long step_at(const DevInst &I, int slot) { return *(const GLOBAL long long *)I.step + slot; }
__device__ __forceinline__ bool takes(const DevInst &I, long long s) { return s < *(const GLOBAL long long *)I.stop; }

// Monopole amplitude a sin(omega t) at stage l of step s, t = (s + c_l) dt
// (FP64).
__device__ __forceinline__ double src_amp(const DevInst &I, long long s, int stage)
{
    return I.src_a * sin(I.src_om * (((double)s + I.c_stage[stage]) * I.dt));
}

// ---------------------------------------------------------------------------
// ghost fill + ADE

// Stage epoch of an instance: the tag that marks ghost values published for
// stage `stage` of step `step` (never 0, the tag of cleared words).
__device__ __forceinline__ unsigned stage_epoch(long long step, int stage)
{
    return (unsigned)(step * 4 + stage + 1);
}

// Publishes one ghost value for the current stage: its 32-bit words, each
// with the epoch in the upper half, by relaxed agent-scope atomic stores.  A
// reader that sees the epoch sees the value stored with it (one atomic word),
// so no release fence (an L2 write-back) is needed, and the value comes from
// the previous launch's fields only, so nothing else must be ordered.
template <typename T>
__device__ __forceinline__ void xg_put(GLOBAL unsigned long long *w, T v, unsigned epoch)
{
    const unsigned long long tag = (unsigned long long)epoch << 32;
    if constexpr (sizeof(T) == 4) {
        __hip_atomic_store(w, tag | __float_as_uint(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        const unsigned long long b = (unsigned long long)__double_as_longlong(v);
        __hip_atomic_store(w, tag | (b & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(w + 1, tag | (b >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Variants of the ghost fill (flags): GV_ONE, a single instance instead of a
// table of them; GV_POLES, some wall of the launch is multi-pole (without it
// every wall is rigid or mass-spring-damper, two auxiliary states per ghost).
constexpr int GV_TABLE = 0, GV_ONE = 1, GV_POLES = 2;

// One ghost per GL-lane group (gid); sub is the lane within the group.  With
// PUB (fused launches) the ghost values also go to the exchange words I.xg.
// With GV_ONE the launch has a single instance: its record is read with
// scalar loads at once, instead of after the work item names it, which takes
// one dependent round trip off the ghost fill.  Only GV_POLES carries the
// multi-pole code, so the other variants keep their registers and schedule.
template <typename T, int GL, bool PUB = false, int GV = GV_TABLE>
__device__ __forceinline__ void ghost_item(const DevInst *__restrict__ insts, const int4 *__restrict__ work,
                                           int nwork, int gid, int sub, int stage, int slot)
{
    constexpr bool ONE = (GV & GV_ONE) != 0, MP = (GV & GV_POLES) != 0;
    if (gid >= nwork) return;                       // whole GL-lane groups leave together
    const int4 wk = work[gid];                      // instance, ghost, cloud entries [z, w)
    if (!ONE && wk.x < 0) return;                   // an idle item of a padded list
    const DevInst &I = insts[ONE ? 0 : wk.x];
    const int g = wk.y;
    const int ib = in_buf(stage), ob = out_buf(stage);
    GLOBAL T *P = gp<T>(I.f[ib][0]);
    GLOBAL T *U = gp<T>(I.f[ib][1]);
    GLOBAL T *V = gp<T>(I.f[ib][2]);
    // independent loads first (member flag, ghost data, ADE states, cloud
    // offsets and weights); the field values are the only dependent round trip
    const long long step = step_at(I, slot);
    const bool active = takes(I, step);
    const VecT<T, 4> gdv = vld<T, 4>(gp<T>(I.gd) + 4 * (size_t)g);
    // two states per ghost (kinds 0-2) as one pair each; a multi-pole wall's
    // ns states separately (then the pair at offset 0 is in bounds and unused)
    const bool two = MP ? (I.ade_kind == 1 || I.ade_kind == 2) : I.ade_kind != 0;
    const size_t po = (!MP || two) ? 2 * (size_t)g : 0;
    const VecT<T, 2> psv = vld<T, 2>(gp<T>(I.psi[ib]) + po);
    const VecT<T, 2> psn = vld<T, 2>(gp<T>(I.psi[0]) + po);
    T x[8], xn[8];
    if (MP && I.ade_kind == 3) {
        const int ns = I.ade_ns;
        const GLOBAL T *xin = gp<T>(I.psi[ib]) + (size_t)ns * g;
        const GLOBAL T *xq = gp<T>(I.psi[0]) + (size_t)ns * g;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            x[k] = k < ns ? xin[k] : (T)0;
            xn[k] = k < ns ? xq[k] : (T)0;
        }
    }
    const GLOBAL T *w4 = gp<T>(I.w4);
    const GLOBAL int *coff = gp<int>(I.coff);
    const int go = gp<int>(I.goff)[g];
    const T nx = gdv.v[0], ny = gdv.v[1];
    // The four sums follow one layout whatever GL is, so both launch forms
    // give the same bits: 32 virtual lanes, virtual lane v adding entries
    // v and v + 32 of every 64-entry pass in that order, then a butterfly
    // over the 32 virtual lanes.  A lane carries R = 32 / GL of them
    // (virtual lanes sub and sub + 16 when GL = 16).
    constexpr int VL = 32;
    constexpr int R = VL / GL;
    static_assert(GL == 16 || GL == 32, "16 or 32 lanes per ghost");
    T c0[R], cF[R], cD[R], cN[R];
#pragma unroll
    for (int r = 0; r < R; ++r) c0[r] = cF[r] = cD[r] = cN[r] = 0;
    const int e0 = wk.z, e1 = wk.w;
    for (int base = e0; base < e1; base += 2 * VL) {
        int off[R][2];
        VecT<T, 4> w[R][2];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int e = base + sub + r * GL + k * VL;
                const bool ok = e < e1;
                off[r][k] = ok ? coff[e] : -1;
                if (ok) w[r][k] = vld<T, 4>(w4 + 4 * (size_t)e);
                else w[r][k] = VecT<T, 4>{{0, 0, 0, 0}};
            }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                if (off[r][k] < 0) continue;
                const int o = off[r][k];
                const T p = P[o], u = U[o], v = V[o];
                c0[r] += w[r][k].v[0] * p;
                cN[r] += w[r][k].v[3] * p;
                cD[r] += w[r][k].v[2] * (nx * u + ny * v);
                cF[r] += w[r][k].v[1] * (-ny * u + nx * v);
            }
    }
    // the first butterfly step pairs virtual lanes v and v + 16
    T s0 = c0[0], sF = cF[0], sD = cD[0], sN = cN[0];
    if constexpr (R == 2) {
        s0 = c0[0] + c0[1];
        sF = cF[0] + cF[1];
        sD = cD[0] + cD[1];
        sN = cN[0] + cN[1];
    } else {
        s0 += __shfl_xor(s0, 16, GL);
        sF += __shfl_xor(sF, 16, GL);
        sD += __shfl_xor(sD, 16, GL);
        sN += __shfl_xor(sN, 16, GL);
    }
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1) {
        s0 += __shfl_xor(s0, m, GL);
        sF += __shfl_xor(sF, m, GL);
        sD += __shfl_xor(sD, m, GL);
        sN += __shfl_xor(sN, m, GL);
    }
    const T a0 = s0, aF = sF, aD = sD, aN = sN;
    // the watched ghost also records the fluid's own normal velocity at its
    // boundary point: the read-out of u.n at P_0 (weights w0), which the wall
    // datum does not constrain (Sec. 4.3 compares it with the ADE's); one
    // more pass over its cloud in the same lane layout, for that ghost only
    const bool rec = stage == 0 && g == I.watch_g && I.watch_cap > 0;
    T aW = 0;
    if (rec) {
        T cW[R];
#pragma unroll
        for (int r = 0; r < R; ++r) cW[r] = 0;
        for (int base = e0; base < e1; base += 2 * VL) {
#pragma unroll
            for (int r = 0; r < R; ++r)
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int e = base + sub + r * GL + k * VL;
                    if (e >= e1) continue;
                    const int o = coff[e];
                    cW[r] += w4[4 * (size_t)e] * (nx * U[o] + ny * V[o]);
                }
        }
        T sW = cW[0];
        if constexpr (R == 2) sW = cW[0] + cW[1];
        else sW += __shfl_xor(sW, 16, GL);
#pragma unroll
        for (int m = 8; m >= 1; m >>= 1) sW += __shfl_xor(sW, m, GL);
        aW = sW;
    }
    if (sub != 0 || !active) return;
    // steps 2-3: ADE derivative, wall normal velocity and its time derivative
    T d1 = 0, d2 = 0, Un = 0, Ud = 0;
    const T s1 = psv.v[0], s2 = psv.v[1];
    if (I.ade_kind == 1) {
        const T a = (T)I.ade[0], b = (T)I.ade[1], c1 = (T)I.ade[2], c2 = (T)I.ade[3];
        d1 = -a * s1 - b * s2 + a0;
        d2 = -a * s2 + b * s1;
        Un = c1 * s1 + c2 * s2;
        Ud = c1 * d1 + c2 * d2;
    } else if (I.ade_kind == 2) {
        const T l1 = (T)I.ade[0], l2 = (T)I.ade[1], c1 = (T)I.ade[2], c2 = (T)I.ade[3];
        d1 = l1 * s1 + a0;
        d2 = l2 * s2 + a0;
        Un = c1 * s1 + c2 * s2;
        Ud = c1 * d1 + c2 * d2;
    }
    // multi-pole wall (Sec. 2.3, eqs. ADEgeneral, unGeneral): each state is
    // coupled to at most its neighbours (a pair's two states)
    T dx[8];
    if (MP && I.ade_kind == 3) {
        const int ns = I.ade_ns;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const double *st = I.ade_st[k];
            T d = (T)st[0] * x[k] + (T)st[3] * a0;
            if (k + 1 < 8) d += (T)st[1] * x[k + 1];
            if (k > 0) d += (T)st[2] * x[k - 1];
            dx[k] = d;
            if (k < ns) {
                Un += (T)st[4] * x[k];
                Ud += (T)st[4] * d;
            }
        }
    }
    // steps 4-5: Neumann for p (dp/dn = +du_n/dt in the wall-to-fluid frame),
    // Dirichlet for u.n (= -u_n), free for u.t
    if (rec) {                                               // recording only
        double *wr = I.watch + 3 * (step % I.watch_cap);
        wr[0] = (double)a0;
        wr[1] = (double)Un;
        wr[2] = (double)(-aW);                               // positive into the wall, like U
    }
    const T pg = aN + gdv.v[3] * ((T)I.h * Ud);
    const T un = aD + gdv.v[2] * (-Un);
    const T ut = aF;
    const T ug = nx * un - ny * ut;
    const T vg = ny * un + nx * ut;
    P[go] = pg;
    U[go] = ug;
    V[go] = vg;
    if (PUB) {
        constexpr int NW = sizeof(T) / 4;
        const unsigned ep = stage_epoch(step, stage);
        GLOBAL unsigned long long *x = gp<unsigned long long>(I.xg) + (size_t)g * 3 * NW;
        xg_put<T>(x, pg, ep);
        xg_put<T>(x + NW, ug, ep);
        xg_put<T>(x + 2 * NW, vg, ep);
    }
    if (two) {
        GLOBAL T *psi_out = gp<T>(I.psi[ob]);
        const T adt = (T)I.alpha_dt[stage];
        psi_out[2 * g] = psn.v[0] + adt * d1;
        psi_out[2 * g + 1] = psn.v[1] + adt * d2;
    } else if (MP && I.ade_kind == 3) {
        const int ns = I.ade_ns;
        GLOBAL T *xout = gp<T>(I.psi[ob]) + (size_t)ns * g;
        const T adt = (T)I.alpha_dt[stage];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k < ns) xout[k] = xn[k] + adt * dx[k];
    }
}

// ---------------------------------------------------------------------------
// probes

// One probe per 16-lane group (pid), one stencil weight per lane: the
// bicubic value of p, u, v of q^n (Sec. 4.1 probes) at the end of the
// sampled step, into the trace ring, and the running DFT of p over the
// window [dft_start, dft_start + dft_count) (FP64).  Valid while buffer 0
// holds that step's result: in the first three stages of the next step, or
// after the step.
template <typename T>
__device__ __forceinline__ void probe_item(const DevInst *__restrict__ insts, const ProbePass &pp, int pid, int sub)
{
    if (pid >= pp.np) return;                       // whole 16-lane groups leave together
    const int2 q = pp.pw[pid];
    if (q.x < 0) return;                            // an idle item of a padded list
    const DevInst &I = insts[q.x];
    const int k = q.y;
    const long long s = step_at(I, pp.rel);
    if (s < 0 || !takes(I, s)) return;
    const int i0 = I.pij[2 * k], j0 = I.pij[2 * k + 1];
    const int a = sub & 3, b = sub >> 2;
    const double w = I.pw[16 * (size_t)k + sub];
    const long off = (long)I.org + (long)(j0 + b) * I.pitch + (i0 + a);
    double ap = w * (double)gp<T>(I.f[0][0])[off];
    double au = w * (double)gp<T>(I.f[0][1])[off];
    double av = w * (double)gp<T>(I.f[0][2])[off];
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1) {
        ap += __shfl_xor(ap, m, 16);
        au += __shfl_xor(au, m, 16);
        av += __shfl_xor(av, m, 16);
    }
    if (sub != 0) return;
    if (I.trace_cap > 0) {
        double *tr = I.trace + ((size_t)(s % I.trace_cap) * I.np + k) * 3;
        tr[0] = ap;
        tr[1] = au;
        tr[2] = av;
    }
    if (I.dft_count > 0 && s >= I.dft_start && s < I.dft_start + I.dft_count) {   // sum p exp(-i omega t)
        const double t = (double)(s + 1) * I.dt;
        I.dft[2 * k] += ap * cos(I.dft_omega * t);
        I.dft[2 * k + 1] -= ap * sin(I.dft_omega * t);
    }
}

// Ghost fill of a stage (256 / GL ghosts per workgroup), then the probe pass in
// the workgroups after them.
template <typename T, int GL, int GV>
__global__ __launch_bounds__(256) void k_ghost(const DevInst *__restrict__ insts,
                                               const int4 *__restrict__ work, int nwork, int stage, int slot,
                                               ProbePass pp)
{
    const int nbg = (nwork * GL + 255) / 256;
    const int b = (int)blockIdx.x;
    if (b < nbg)
        ghost_item<T, GL, false, GV>(insts, work, nwork, (int)((b * blockDim.x + threadIdx.x) / GL),
                                      (int)(threadIdx.x % GL), stage, slot);
    else
        probe_item<T>(insts, pp, (b - nbg) * 16 + (int)threadIdx.x / 16, (int)threadIdx.x % 16);
}

template <typename T>
__global__ __launch_bounds__(256) void k_probe(const DevInst *__restrict__ insts, ProbePass pp)
{
    probe_item<T>(insts, pp, (int)blockIdx.x * 16 + (int)threadIdx.x / 16, (int)threadIdx.x % 16);
}

// After a run of n steps: each member's first step of the next run, held at
// its stop step.
__global__ void k_advance(const DevInst *__restrict__ insts, int ninst, int n)
{
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= ninst) return;
    const DevInst &I = insts[k];
    const long long b = *I.step, e = *I.stop;
    if (b < e) *I.step = b + n < e ? b + n : e;
}

// ---------------------------------------------------------------------------
// the filter next to an immersed wall

// Fluid intervals of a row outside the domain: every column counts as open
// (the zero frame is not a wall).
__device__ __forceinline__ int4 open_row() { return make_int4(-(1 << 30), 1 << 30, 0, 0); }

__device__ __forceinline__ bool in_iv(const int4 iv, int col)
{
    return (col >= iv.x && col < iv.y) || (col >= iv.z && col < iv.w);
}

// Half-width (0..5) of the filter row along x of fluid node col of a row
// with fluid intervals iv: the nodes up to w away on either side hold no
// non-fluid node of the domain (an interval that reaches the domain edge is
// open beyond it).
__device__ __forceinline__ int x_width(const int4 iv, int col, int nx)
{
    const bool first = col >= iv.x && col < iv.y;
    const int a = first ? iv.x : iv.z, b = first ? iv.y : iv.w;
    const int lo = a == 0 ? 5 : min(col - a, 5);
    const int hi = b == nx ? 5 : min(b - 1 - col, 5);
    return min(lo, hi);
}

// The same along y for column col, with row(k) the intervals of row j + k.
template <typename R>
__device__ __forceinline__ int y_width(const R &row, int col)
{
    int w = 5;
#pragma unroll
    for (int k = 5; k >= 1; --k)
        if (!in_iv(row(-k), col) || !in_iv(row(k), col)) w = k - 1;
    return w;
}

// Non-fluid rows of one tile column as bits (bit b: LDS row b of the tile's
// copy, rows outside the domain open): wide enough for the copied rows.
template <int R>
using ColMask = typename std::conditional<(R <= 32), unsigned, unsigned long long>::type;

// Half-width (0..5) of the filter row along y at LDS row y of a column whose
// non-fluid rows are the bits of m: one less than the distance to the
// nearest non-fluid row within five, 5 when there is none (the same as
// y_width over the rows' intervals).
template <typename M>
__device__ __forceinline__ int y_width_bits(M m, int y)
{
    const unsigned win = (unsigned)(m >> (y - 5)) & 0x7ffu;  // rows y - 5 .. y + 5, bit 5 = row y
    const unsigned up = win >> 6, down = win & 0x1fu;
    const int du = up ? __builtin_ctz(up) + 1 : 6;          // nearest above
    const int dd = down ? 5 - (31 - __builtin_clz(down)) : 6;   // nearest below
    return min(du, dd) - 1;
}

// Change of one field's filter sum at a node whose rows have half-widths wx
// and wy: sum over both axes of dw[w][0] q_0 + sum_k dw[w][k] (q_k + q_-k),
// dw[w] being the half-width-w row minus the 11-point one (times sigma/dt;
// zero for w = 5).  qx(k), qy(k): the field at offset k along x, y.
template <typename T, typename QX, typename QY>
__device__ __forceinline__ T wall_filter_delta(const T (*dw)[6], int wx, int wy, const QX &qx, const QY &qy)
{
    const T q0 = qx(0);
    T d = dw[wx][0] * q0 + dw[wy][0] * q0;
#pragma unroll
    for (int k = 1; k <= 5; ++k) d += dw[wx][k] * (qx(k) + qx(-k)) + dw[wy][k] * (qy(k) + qy(-k));
    return d;
}

template <typename T>
__device__ __forceinline__ T fdw_at(const DevInst &I, int w, int k);
template <>
__device__ __forceinline__ float fdw_at<float>(const DevInst &I, int w, int k) { return I.fdwf[w][k]; }
template <>
__device__ __forceinline__ double fdw_at<double>(const DevInst &I, int w, int k) { return I.fdw[w][k]; }

// ---------------------------------------------------------------------------
// stage sweep

template <typename T, int VEC>
__device__ __forceinline__ void load_row(T (&dst)[3][VEC], const GLOBAL T *p, const GLOBAL T *u,
                                         const GLOBAL T *v, unsigned off)
{
    const VecT<T, VEC> a = vld<T, VEC>(p + off);
    const VecT<T, VEC> b = vld<T, VEC>(u + off);
    const VecT<T, VEC> c = vld<T, VEC>(v + off);
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        dst[0][e] = a.v[e];
        dst[1][e] = b.v[e];
        dst[2][e] = c.v[e];
    }
}

template <typename T, int VEC, bool FILT, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_sweep(const DevInst *__restrict__ insts,
                                                    const int4 *__restrict__ work, int nwork, int stage, int slot)
{
    constexpr int NL = 64 * VEC;                 // loaded columns per strip
    constexpr int KM = (5 + VEC - 1) / VEC;      // LDS chunks left of the lane's own
    constexpr int KP = (VEC + 4) / VEC;          // chunks right of it
    constexpr int XW = (KM + 1 + KP) * VEC;      // x window held per lane
    __shared__ T lds_all[WPB][3][NL];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    T(*lds)[NL] = lds_all[wv];

    for (int w = blockIdx.x * WPB + wv; w < nwork; w += gridDim.x * WPB) {
        const int4 wk = work[w];
        if (wk.x < 0) continue;                   // idle slot of the XCD-aware order
        const bool wall = FILT && (wk.x & TILE_WALL_BIT) != 0;
        const DevInst &I = insts[wk.x & TILE_INST_MASK];
        const long long step = step_at(I, slot);
        if (!takes(I, step)) continue;            // uniform per wave
        const int c0 = wk.y;                      // first output column
        const int r0 = wk.z;
        const int dir = wk.w < 0 ? -1 : 1;
        const int r1 = wk.w < 0 ? -wk.w : wk.w;
        const int nrows = r1 - r0;
        const int jbeg = dir > 0 ? r0 : r1 - 1;
        const int ib = in_buf(stage), ob = out_buf(stage);
        const int pitch = I.pitch;
        const int org = I.org;
        const GLOBAL T *Pi = gp<T>(I.f[ib][0]);
        const GLOBAL T *Ui = gp<T>(I.f[ib][1]);
        const GLOBAL T *Vi = gp<T>(I.f[ib][2]);
        const GLOBAL T *Pn = gp<T>(I.f[0][0]);
        const GLOBAL T *Un = gp<T>(I.f[0][1]);
        const GLOBAL T *Vn = gp<T>(I.f[0][2]);
        GLOBAL T *Po = gp<T>(I.f[ob][0]);
        GLOBAL T *Uo = gp<T>(I.f[ob][1]);
        GLOBAL T *Vo = gp<T>(I.f[ob][2]);
        const int col0 = c0 - 8 + lane * VEC;     // first column of this lane
        const bool out_lane = (col0 + VEC > c0) && (col0 < c0 + NL - 16);
        // coefficients
        T ax[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) ax[k] = (T)I.ax[k];
        T fd[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) fd[k] = (T)I.fd[k];
        const T adt = (T)I.alpha_dt[stage];
        const T ydir = (T)dir;
        const bool has_src = I.has_src && !(I.src_i1 < c0 || I.src_i0 >= c0 + NL - 16) &&
                             !(I.src_j1 < r0 || I.src_j0 >= r1);
        const T amp = has_src ? (T)src_amp(I, step, stage) : (T)0;
        const int sw = I.sponge_w;

        T q[11][3][VEC];
        // prologue: rows jbeg - 5 dir .. jbeg + 4 dir
#pragma unroll
        for (int s = 0; s < 10; ++s)
            load_row<T, VEC>(q[s], Pi, Ui, Vi, (unsigned)(org + (jbeg + (s - 5) * dir) * pitch + col0));

        for (int it = 0; it < nrows; ++it) {
            const int j = jbeg + it * dir;
            load_row<T, VEC>(q[10], Pi, Ui, Vi, (unsigned)(org + (j + 5 * dir) * pitch + col0));
            T qn[3][VEC];
            if (stage != 0) load_row<T, VEC>(qn, Pn, Un, Vn, (unsigned)(org + j * pitch + col0));
            const int4 iv = gp<int4>(I.iv)[j];
            wave_lds_sync();
            {
                VecT<T, VEC> a, b, c;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    a.v[e] = q[5][0][e];
                    b.v[e] = q[5][1][e];
                    c.v[e] = q[5][2][e];
                }
                *(VecT<T, VEC> *)&lds[0][lane * VEC] = a;
                *(VecT<T, VEC> *)&lds[1][lane * VEC] = b;
                if (FILT) *(VecT<T, VEC> *)&lds[2][lane * VEC] = c;
            }
            wave_lds_sync();
            if (out_lane) {
                // y parts and the centre term from the register window
                T rp[VEC], ru[VEC], rv[VEC];
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    T dpdy = 0, dvdy = 0;
#pragma unroll
                    for (int k = 1; k <= 5; ++k) {
                        dpdy += ax[k - 1] * (q[5 + k][0][e] - q[5 - k][0][e]);
                        dvdy += ax[k - 1] * (q[5 + k][2][e] - q[5 - k][2][e]);
                    }
                    rp[e] = -ydir * dvdy;
                    ru[e] = 0;
                    rv[e] = -ydir * dpdy;
                    if (FILT) {
                        T fp = fd[0] * q[5][0][e], fu = fd[0] * q[5][1][e], fv = fd[0] * q[5][2][e];
#pragma unroll
                        for (int k = 1; k <= 5; ++k) {
                            fp += fd[k] * (q[5 + k][0][e] + q[5 - k][0][e]);
                            fu += fd[k] * (q[5 + k][1][e] + q[5 - k][1][e]);
                            fv += fd[k] * (q[5 + k][2][e] + q[5 - k][2][e]);
                        }
                        rp[e] -= fp;
                        ru[e] -= fu;
                        rv[e] -= fv;
                    }
                }
                // x parts, one field window at a time from LDS
#pragma unroll
                for (int f = 0; f < (FILT ? 3 : 2); ++f) {
                    T xw[XW];
#pragma unroll
                    for (int k = -KM; k <= KP; ++k) {
                        const VecT<T, VEC> a = *(const VecT<T, VEC> *)&lds[f][lane * VEC + k * VEC];
#pragma unroll
                        for (int e = 0; e < VEC; ++e) xw[(k + KM) * VEC + e] = a.v[e];
                    }
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const int x = KM * VEC + e;
                        if (f < 2) {
                            T dx = 0;
#pragma unroll
                            for (int k = 1; k <= 5; ++k) dx += ax[k - 1] * (xw[x + k] - xw[x - k]);
                            if (f == 0) ru[e] -= dx;     // -dp/dx
                            else rp[e] -= dx;            // -du/dx
                        }
                        if (FILT) {
                            T fx = 0;
#pragma unroll
                            for (int k = 1; k <= 5; ++k) fx += fd[k] * (xw[x + k] + xw[x - k]);
                            if (f == 0) rp[e] -= fx;
                            else if (f == 1) ru[e] -= fx;
                            else rv[e] -= fx;
                        }
                    }
                }
                if (wall) {                      // nodes within five of the wall along an axis
                    const int ny = I.ny;
                    int4 rows[11];
#pragma unroll
                    for (int k = -5; k <= 5; ++k)
                        rows[k + 5] = j + k >= 0 && j + k < ny ? int4(gp<int4>(I.iv)[j + k]) : open_row();
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const int col = col0 + e;
                        if (!in_iv(iv, col)) continue;
                        const int wx = x_width(iv, col, I.nx);
                        const int wy = y_width([&](int k) { return rows[k + 5]; }, col);
                        if (wx == 5 && wy == 5) continue;
                        T dw[6][6];
#pragma unroll
                        for (int k = 0; k < 6; ++k) {
                            dw[0][k] = fdw_at<T>(I, wx, k);
                            dw[1][k] = fdw_at<T>(I, wy, k);
                        }
                        const T(*dwp)[6] = dw;
                        T d[3];
#pragma unroll
                        for (int f = 0; f < 3; ++f) {
                            d[f] = wall_filter_delta<T>(dwp, 0, 1, [&](int k) { return lds[f][lane * VEC + e + k]; },
                                                        [&](int k) { return q[5 + k][f][e]; });
                        }
                        rp[e] -= d[0];
                        ru[e] -= d[1];
                        rv[e] -= d[2];
                    }
                }
                T ro[3][VEC];
                bool ok[VEC];
                bool all = true;
#pragma unroll
                for (int e = 0; e < VEC; ++e) {
                    const int col = col0 + e;
                    if (sw > 0) {
                        int eg = min(min(col, j), min(I.nx - 1 - col, I.ny - 1 - j));
                        if (eg < sw) {
                            const T f = (T)(sw - eg) / (T)sw;
                            const T sg = (T)I.sponge_s * f * f;
                            rp[e] -= sg * q[5][0][e];
                            ru[e] -= sg * q[5][1][e];
                            rv[e] -= sg * q[5][2][e];
                        }
                    }
                    if (has_src) {      // offsets from the source's nearest node: no cancellation
                        const T xx = (T)(col - I.src_ic) * (T)I.h - (T)I.src_fx;
                        const T yy = (T)(j - I.src_jc) * (T)I.h - (T)I.src_fy;
                        rp[e] += amp * exp(-(T)I.src_b * (xx * xx + yy * yy));
                    }
                    const T p0 = stage != 0 ? qn[0][e] : q[5][0][e];
                    const T u0 = stage != 0 ? qn[1][e] : q[5][1][e];
                    const T v0 = stage != 0 ? qn[2][e] : q[5][2][e];
                    ro[0][e] = p0 + adt * rp[e];
                    ro[1][e] = u0 + adt * ru[e];
                    ro[2][e] = v0 + adt * rv[e];
                    ok[e] = (col >= iv.x && col < iv.y) || (col >= iv.z && col < iv.w);
                    all = all && ok[e];
                }
                const unsigned off = (unsigned)(org + j * pitch + col0);
                if (all) {
                    VecT<T, VEC> a, b, c;
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        a.v[e] = ro[0][e];
                        b.v[e] = ro[1][e];
                        c.v[e] = ro[2][e];
                    }
                    if (I.stream) {
                        __asm__ volatile("");
                        vst_stream<T, VEC>(Po + off, a);
                        vst_stream<T, VEC>(Uo + off, b);
                        vst_stream<T, VEC>(Vo + off, c);
                        __asm__ volatile("");
                    } else {
                        vst<T, VEC>(Po + off, a);
                        vst<T, VEC>(Uo + off, b);
                        vst<T, VEC>(Vo + off, c);
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        if (ok[e]) {
                            Po[off + e] = ro[0][e];
                            Uo[off + e] = ro[1][e];
                            Vo[off + e] = ro[2][e];
                        }
                }
            }
#pragma unroll
            for (int s = 0; s < 10; ++s)
#pragma unroll
                for (int f = 0; f < 3; ++f)
#pragma unroll
                    for (int e = 0; e < VEC; ++e) q[s][f][e] = q[s + 1][f][e];
        }
    }
}

// ---------------------------------------------------------------------------
// stage sweep, 2-D tile variant.  A 256-thread workgroup owns a TX x TY
// tile.  Its read region of q^(l-1) (the tile plus 5 halo rows above and
// below and 8 halo columns left and right, corners skipped) and its block of
// q^n are copied straight from global memory into LDS with 16-byte
// global_load_lds instructions (no register staging, so all of the tile's
// traffic is in flight at once).  Each thread then computes VEC consecutive
// nodes of one row at a time, reading the 11-point windows of each field from
// LDS.

#if defined(__HIP_DEVICE_COMPILE__)
#define LOCAL __attribute__((address_space(3)))
#else
#define LOCAL
#endif

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

// One aligned 16-byte LDS read.  The empty asm keeps all four words live so
// the compiler cannot split the read into narrower, bank-conflicting pieces.
// It is not volatile: a volatile asm is a scheduling barrier, which would
// wait for each read before issuing the next instead of keeping a window's
// reads in flight together.
template <typename T, int VEC>
__device__ __forceinline__ VecT<T, VEC> lds16(const T *p)
{
    u32x4_t w = *(const u32x4_t *)p;
    asm("" : "+v"(w));
    return __builtin_bit_cast(VecT<T, VEC>, w);
}

// stencil coefficients in the arithmetic precision (FP32 copies are kept in
// the record so they load straight into scalar registers)
template <typename T>
__device__ __forceinline__ void coefs(const DevInst &I, T (&ax)[5], T (&fd)[6]);
template <>
__device__ __forceinline__ void coefs<float>(const DevInst &I, float (&ax)[5], float (&fd)[6])
{
#pragma unroll
    for (int k = 0; k < 5; ++k) ax[k] = I.axf[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) fd[k] = I.fdf[k];
}
template <>
__device__ __forceinline__ void coefs<double>(const DevInst &I, double (&ax)[5], double (&fd)[6])
{
#pragma unroll
    for (int k = 0; k < 5; ++k) ax[k] = I.ax[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) fd[k] = I.fd[k];
}

// 16 bytes from src (per lane) to LDS at lds_wave_base + 16 * lane.
__device__ __forceinline__ void dma16(const void *src, void *lds_wave_base)
{
    __builtin_amdgcn_global_load_lds((const GLOBAL void *)src, (LOCAL void *)lds_wave_base, 16, 0, 0);
}
// The same with the non-temporal hint (cache policy NT).
__device__ __forceinline__ void dma16_nt(const void *src, void *lds_wave_base)
{
    __builtin_amdgcn_global_load_lds((const GLOBAL void *)src, (LOCAL void *)lds_wave_base, 16, 0, 2);
}

// One field's contribution to the right-hand sides of VEC nodes of one row
// (LDS row y, first LDS column lc): F = 0 (p): -dp/dx -> u, -dp/dy -> v;
// F = 1 (u): -du/dx -> p; F = 2 (v): -dv/dy -> p; and the selective-filter
// damping of the field itself, (2 d_0) f_0 + sum_k d_k (f_{+k} + f_{-k})
// summed over both directions (fd holds these coefficients times sigma/dt).
// The pair sums and differences of each offset are formed once and shared.
// Near-wall nodes (WALL, wall tiles): a node whose filter rows narrow (half-
// widths wx[e], wy[e] below 5) takes its filter sum with the rows wb[wx] and
// wb[wy] (the half-width-w centred rows times sigma_d / dt, k = 0..5; row 5
// the 11-point one), from the window values already in registers; every
// other node keeps the sum above, so a node's arithmetic does not depend on
// the tiling.
template <typename T, int VEC, bool FILT, int F, int LW, bool WALL = false>
__device__ __forceinline__ void row_field(const T (*lds)[LW], int y, int lc, const T (&ax)[5], const T (&fd)[6],
                                          T (&rp)[VEC], T (&ru)[VEC], T (&rv)[VEC],
                                          const T (*wb)[8] = nullptr, const int *wx = nullptr,
                                          const int *wy = nullptr)
{
    constexpr int KM = (5 + VEC - 1) / VEC;
    constexpr int KP = (VEC + 4) / VEC;
    constexpr int XW = (KM + 1 + KP) * VEC;
    static_assert(KM * VEC - 5 == VEC - 1 && KM * VEC + VEC + 4 == (KM + KP) * VEC,
                  "x +- 5 reaches one element of each outermost chunk");
    T yw[11][VEC];
#pragma unroll
    for (int k = 0; k < 11; ++k) {
        const VecT<T, VEC> a = lds16<T, VEC>(&lds[y - 5 + k][lc]);
#pragma unroll
        for (int e = 0; e < VEC; ++e) yw[k][e] = a.v[e];
    }
    T xw[XW];
    if (F != 2 || FILT) {
#pragma unroll
        for (int k = -KM; k <= KP; ++k) {
            if (k == 0) {                        // the centre chunk is the y window's
#pragma unroll
                for (int e = 0; e < VEC; ++e) xw[KM * VEC + e] = yw[5][e];
                continue;
            }
            // of the outermost chunks only the element next to the inner
            // ones is in reach (x +- 5): one LDS element instead of a chunk
            if (k == -KM) {
                xw[VEC - 1] = lds[y][lc - KM * VEC + VEC - 1];
                continue;
            }
            if (k == KP) {
                xw[(KM + KP) * VEC] = lds[y][lc + KP * VEC];
                continue;
            }
            const VecT<T, VEC> a = lds16<T, VEC>(&lds[y][lc + k * VEC]);
#pragma unroll
            for (int e = 0; e < VEC; ++e) xw[(k + KM) * VEC + e] = a.v[e];
        }
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const int x = KM * VEC + e;
        T dy = 0, dx = 0, fl = FILT ? fd[0] * yw[5][e] : (T)0;
#pragma unroll
        for (int k = 1; k <= 5; ++k) {
            const T yp = yw[5 + k][e], ym = yw[5 - k][e];
            const T xp = xw[x + k], xm = xw[x - k];
            if (F != 1) dy += ax[k - 1] * (yp - ym);
            if (F != 2) dx += ax[k - 1] * (xp - xm);
            if (FILT) fl += fd[k] * ((xp + xm) + (yp + ym));
        }
        if constexpr (FILT && WALL) {
            if (wx[e] < 5 || wy[e] < 5) {
                const T *bx = wb[wx[e]];
                const T *by = wb[wy[e]];
                T g = bx[0] * yw[5][e] + by[0] * yw[5][e];
#pragma unroll
                for (int k = 1; k <= 5; ++k)
                    g += bx[k] * (xw[x + k] + xw[x - k]) + by[k] * (yw[5 + k][e] + yw[5 - k][e]);
                fl = g;
            }
        }
        if (F == 0) {
            rv[e] -= dy;
            ru[e] -= dx;
            if (FILT) rp[e] -= fl;
        } else if (F == 1) {
            rp[e] -= dx;
            if (FILT) ru[e] -= fl;
        } else {
            rp[e] -= dy;
            if (FILT) rv[e] -= fl;
        }
    }
}

// Forces the partial sums to be materialised here and orders the following
// LDS reads after them (an empty asm statement: no instruction is emitted).
template <typename T, int VEC>
__device__ __forceinline__ void pin_sums(T (&rp)[VEC], T (&ru)[VEC], T (&rv)[VEC])
{
#pragma unroll
    for (int e = 0; e < VEC; ++e) asm volatile("" : "+v"(rp[e]), "+v"(ru[e]), "+v"(rv[e])::"memory");
}

// A tile of a fused stage whose stencils read ghost nodes: it takes each
// ghost value it reads from the exchange words once they carry this stage's
// epoch (bounded by spin_limit polls per word, then the error flag) and
// overwrites the ghost nodes in its LDS copy; patch[p0, p1) holds (LDS
// element index, ghost index * 3 + field) for each ghost node and field.
struct GhostDep {
    int *error;
    int spin_limit;
    const int2 *patch;
    int p0, p1;
};

// Shape of a cols x rows tile (TX x TY): NCX column groups of VEC nodes, RG
// rows in flight per pass of 256 lanes, an LDS read region of R rows x LW
// columns (CW 16-byte chunks per row, HC halo chunks per side; NCH chunks per
// field).
template <typename T, int VEC, int TX, int TY>
struct TileGeo {
    static constexpr int NT = 256;
    static constexpr int NCX = TX / VEC;
    static constexpr int RG = NT / NCX;
    static constexpr int R = TY + 10;
    static constexpr int LW = TX + 16;
    static constexpr int CW = LW / VEC;
    static constexpr int HC = 8 / VEC;
    static constexpr int NCH = R * CW;
    static_assert(sizeof(T) * VEC == 16, "16-byte chunks");
};

// Values that do not change during a launch, read with scalar loads (they
// then never wait for vector memory traffic in flight).
#if defined(__HIP_DEVICE_COMPILE__)
#define CONSTAS __attribute__((address_space(4)))
#else
#define CONSTAS
#endif
template <typename T>
__device__ __forceinline__ T sload(const void *p)
{
    return *(const CONSTAS T *)p;
}

// Per-tile values shared by all lanes.
template <typename T>
struct TileCtx {
    int c0, r0, r1, ib, ob;
    bool in_sponge, has_src, in_band, wall;
    T adt, sp_inv, sp_s, amp;
    T ax[5], fd[6];
};

template <typename T, int TX>
__device__ __forceinline__ TileCtx<T> tile_ctx(const DevInst &I, const int4 wk, int stage, long long step, bool wall)
{
    TileCtx<T> c;
    c.wall = wall;
    c.c0 = wk.y;
    c.r0 = wk.z;
    c.r1 = wk.w < 0 ? -wk.w : wk.w;
    c.ib = in_buf(stage);
    // with the explicit filter the last stage leaves its result in register
    // set C, from which k_filter writes q^{n+1} into A
    c.ob = stage == 3 && I.fx ? 2 : out_buf(stage);
    coefs<T>(I, c.ax, c.fd);
    c.adt = (T)I.alpha_dt[stage];
    const int sw = I.sponge_w;
    // the sponge band and the source box are tested once per tile
    c.in_sponge = sw > 0 && (c.c0 < sw || c.r0 < sw || c.c0 + TX > I.nx - sw || c.r1 > I.ny - sw);
    c.sp_inv = (T)I.sponge_inv;
    c.sp_s = (T)I.sponge_s;
    const int rw = I.rad_w;
    c.in_band = rw > 0 && (c.c0 < rw || c.r0 < rw || c.c0 + TX > I.nx - rw || c.r1 > I.ny - rw);
    c.has_src = I.has_src && !(I.src_i1 < c.c0 || I.src_i0 >= c.c0 + TX) && !(I.src_j1 < c.r0 || I.src_j0 >= c.r1);
    c.amp = c.has_src ? (T)src_amp(I, step, stage) : (T)0;
    return c;
}

// Starts the LDS copy of a tile: the read region of the stage input (rows
// r0 - 5 .. r0 + TY + 4, columns c0 - 8 .. c0 + TX + 7, the halo rows without
// their corner chunks, no row past the allocated frame) into reg, 64 chunks
// per wave instruction.  q^n is not staged in LDS: each lane reads its own
// q^n chunks into registers while its row's arithmetic runs, which keeps the
// workgroup's LDS at the read region alone (one more resident workgroup per
// CU for FP32 64x16 and 128x8 and FP64 64x8).
template <typename T, int VEC, int TX, int TY>
__device__ __forceinline__ void tile_copy(const DevInst &I, const TileCtx<T> &c, T (*reg)[TY + 10][TX + 16])
{
    using G = TileGeo<T, VEC, TX, TY>;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int pitch = I.pitch, org = I.org;
    const int rowmax = I.ny + 4;                 // last allocated frame row
    // a stage input other than q^n streams through the caches where q^n
    // is to stay in them (stream_in), except the last ten copied rows: the
    // tile below, next in its XCD's row-major run, reads them again
    const bool nt = I.stream_in && c.ib != 0;
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        const T *src = (const T *)I.f[c.ib][f];
        for (int base = wave * 64; base < G::NCH; base += G::NT) {
            const int q = base + lane;
            const int row = q / G::CW, cc = q - (q / G::CW) * G::CW;
            const int gr = c.r0 - 5 + row;
            const bool halo_row = row < 5 || row >= TY + 5;
            const bool ok = q < G::NCH && !(halo_row && (cc < G::HC || cc >= G::CW - G::HC)) && gr <= rowmax;
            if (!ok) continue;
            const T *at = src + (unsigned)(org + gr * pitch + (c.c0 - 8 + cc * VEC));
            if (nt && row < TY)
                dma16_nt(at, &reg[f][0][0] + base * VEC);
            else
                dma16(at, &reg[f][0][0] + base * VEC);
        }
    }
}

// The first two patch entries of this lane, p0 + lane and p0 + lane + 256
// (x = -1 when absent), loaded before the ghost wait.
__device__ __forceinline__ void patch_prefetch(const int2 *__restrict__ patch, int p0, int p1, int2 (&pre)[2])
{
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int e = p0 + (int)threadIdx.x + 256 * k;
        pre[k] = e < p1 ? patch[e] : make_int2(-1, 0);
    }
}

// One ghost value of the current stage from its exchange words: relaxed
// agent-scope atomic loads, repeated while a word carries another epoch (at
// most spin_limit polls, then the error flag is raised and the value is not
// valid).  A negative spin_limit (testing the error path from the host)
// waits -spin_limit polls for a tag no carrier ever publishes.
template <typename T>
__device__ __forceinline__ T xg_get(const GLOBAL unsigned long long *w, unsigned epoch, int spin_limit, int *error)
{
    constexpr int NW = sizeof(T) / 4;
    const unsigned want = spin_limit < 0 ? ~epoch : epoch;   // epochs are small: ~epoch never appears
    const int limit = spin_limit < 0 ? -spin_limit : spin_limit;
    unsigned long long b = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        unsigned long long v = __hip_atomic_load(w + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int polls = 0;
        while ((unsigned)(v >> 32) != want) {
            if (++polls > limit) {
                __hip_atomic_fetch_or(error, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
            v = __hip_atomic_load(w + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        b |= (v & 0xffffffffull) << (32 * k);
    }
    if constexpr (NW == 1)
        return __uint_as_float((unsigned)b);
    else
        return __longlong_as_double((long long)b);
}

// Overwrites the ghost nodes of a tile's LDS copy with this stage's ghost
// values: patch entries [p0, p1) are (LDS element index, ghost * 3 + field);
// pre holds this lane's first two entries.
template <typename T, int TX, int TY>
__device__ __forceinline__ void tile_patch(const DevInst &I, unsigned epoch, T (*reg)[TY + 10][TX + 16],
                                           const GhostDep &d, const int2 (&pre)[2])
{
    constexpr int NW = sizeof(T) / 4;
    T *base = &reg[0][0][0];
    constexpr int FS = (TY + 10) * (TX + 16);    // elements per field of the copy
#pragma unroll
    for (int k = 0; k < 2; ++k)
        if (pre[k].x >= 0)
            base[(pre[k].y % 3) * FS + pre[k].x] =
                xg_get<T>(gp<unsigned long long>(I.xg) + (size_t)pre[k].y * NW, epoch, d.spin_limit, d.error);
    for (int e = d.p0 + (int)threadIdx.x + 512; e < d.p1; e += 256) {
        const int2 pe = d.patch[e];
        base[(pe.y % 3) * FS + pe.x] =
            xg_get<T>(gp<unsigned long long>(I.xg) + (size_t)pe.y * NW, epoch, d.spin_limit, d.error);
    }
}

// Nodes within five of the wall along an axis (wall tiles): that axis takes
// the narrower centred row, so each field's filter sum changes by the
// difference of the rows (wfd; subtracted from rp, ru, rv).  The x
// half-widths come from the row's intervals iv, the y ones from the column
// masks wcm (a few bit operations per node).
template <typename T, int VEC, int TX, int TY>
__device__ __forceinline__ void wall_rows(const DevInst &I, const T (*reg)[TY + 10][TX + 16], const T (*wfd)[6],
                                          const ColMask<TY + 10> *wcm, int y, int lc, int gc, int tc, const int4 iv,
                                          T (&rp)[VEC], T (&ru)[VEC], T (&rv)[VEC])
{
    int wx[VEC], wy[VEC];
    bool any = false;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const int col = gc + e;
        wx[e] = wy[e] = 5;
        if (!in_iv(iv, col)) continue;
        wx[e] = x_width(iv, col, I.nx);
        wy[e] = y_width_bits(wcm[tc + e], y);
        any = any || wx[e] < 5 || wy[e] < 5;
    }
    if (!any) return;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        if (wx[e] == 5 && wy[e] == 5) continue;
        const int cx = lc + e;
        T d[3];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            const T(*L)[TX + 16] = reg[f];
            d[f] = wall_filter_delta<T>(wfd, wx[e], wy[e], [&](int k) { return L[y][cx + k]; },
                                        [&](int k) { return L[y + k][cx]; });
        }
        rp[e] -= d[0];
        ru[e] -= d[1];
        rv[e] -= d[2];
    }
}

// Right-hand side (Sec. 3.2 step 6) and RK stage update of row i of a tile
// for the VEC nodes of columns tc .. tc + VEC - 1 of the tile: reg is the LDS
// copy of the stage input, (pn, un, vn) the q^n values (unused in the first
// stage, whose input is q^n), iv the row's fluid column ranges.  Returns the
// new values and which of the nodes are fluid.
template <typename T, int VEC, bool FILT, int TX, int TY, bool WALL>
__device__ __forceinline__ void tile_row(const DevInst &I, const TileCtx<T> &c, const T (*reg)[TY + 10][TX + 16],
                                         const T (*wb)[8], const ColMask<TY + 10> *wcm,
                                         int stage, int i, int tc, const int4 iv, const VecT<T, VEC> &pn_,
                                         const VecT<T, VEC> &un_, const VecT<T, VEC> &vn_, VecT<T, VEC> &po,
                                         VecT<T, VEC> &uo, VecT<T, VEC> &vo, bool (&ok)[VEC], bool &all)
{
    const int j = c.r0 + i;
    const int y = i + 5;
    const int lc = tc + 8;
    const int gc = c.c0 + tc;
    T rp[VEC], ru[VEC], rv[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) rp[e] = ru[e] = rv[e] = 0;
    // near-wall half-widths of this lane's nodes (wall tiles): along x from
    // the row's intervals, along y from the column masks
    int wx[VEC], wy[VEC];
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        wx[e] = wy[e] = 5;
        if (FILT && WALL && in_iv(iv, gc + e)) {
            wx[e] = x_width(iv, gc + e, I.nx);
            wy[e] = y_width_bits(wcm[tc + e], y);
        }
    }
    // one field's windows live at a time: each field's sums are pinned
    // (empty asm, no instructions) before the next field's LDS reads
    row_field<T, VEC, FILT, 0, TX + 16, WALL>(reg[0], y, lc, c.ax, c.fd, rp, ru, rv, wb, wx, wy);
    pin_sums<T, VEC>(rp, ru, rv);
    row_field<T, VEC, FILT, 1, TX + 16, WALL>(reg[1], y, lc, c.ax, c.fd, rp, ru, rv, wb, wx, wy);
    pin_sums<T, VEC>(rp, ru, rv);
    row_field<T, VEC, FILT, 2, TX + 16, WALL>(reg[2], y, lc, c.ax, c.fd, rp, ru, rv, wb, wx, wy);
    const VecT<T, VEC> pc = *(const VecT<T, VEC> *)&reg[0][y][lc];
    const VecT<T, VEC> uc = *(const VecT<T, VEC> *)&reg[1][y][lc];
    const VecT<T, VEC> vc = *(const VecT<T, VEC> *)&reg[2][y][lc];
    const VecT<T, VEC> pn = stage != 0 ? pn_ : pc;
    const VecT<T, VEC> un = stage != 0 ? un_ : uc;
    const VecT<T, VEC> vn = stage != 0 ? vn_ : vc;
    all = true;
    if (c.in_sponge) {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const int col = gc + e;
            const int sw = I.sponge_w;
            const int eg = min(min(col, j), min(I.nx - 1 - col, I.ny - 1 - j));
            if (eg < sw) {
                const T fr = (T)(sw - eg) * c.sp_inv;
                const T sg = c.sp_s * fr * fr;
                rp[e] -= sg * pc.v[e];
                ru[e] -= sg * uc.v[e];
                rv[e] -= sg * vc.v[e];
            }
        }
    }
    if (c.has_src) {
        // the empty asm keeps the optimiser from evaluating the source term
        // on every tile and selecting it away (its exp costs about 25
        // instructions per node)
        __asm__ volatile("");
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const T xx = (T)(gc + e - I.src_ic) * (T)I.h - (T)I.src_fx;
            const T yy = (T)(j - I.src_jc) * (T)I.h - (T)I.src_fy;
            rp[e] += c.amp * exp(-(T)I.src_b * (xx * xx + yy * yy));
        }
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const int col = gc + e;
        po.v[e] = pn.v[e] + c.adt * rp[e];
        uo.v[e] = un.v[e] + c.adt * ru[e];
        vo.v[e] = vn.v[e] + c.adt * rv[e];
        ok[e] = (col >= iv.x && col < iv.y) || (col >= iv.z && col < iv.w);
        if (c.in_band && min(min(col, j), min(I.nx - 1 - col, I.ny - 1 - j)) < I.rad_w)
            ok[e] = false;                       // the band pass writes these
        all = all && ok[e];
    }
}

// Writes a row's new values at its fluid nodes (plane offset off of the
// first node) in register set ob.
template <typename T, int VEC>
__device__ __forceinline__ void tile_store(const DevInst &I, int ob, unsigned off, const VecT<T, VEC> &po,
                                           const VecT<T, VEC> &uo, const VecT<T, VEC> &vo, const bool (&ok)[VEC],
                                           bool all)
{
    GLOBAL T *Po = gp<T>(I.f[ob][0]);
    GLOBAL T *Uo = gp<T>(I.f[ob][1]);
    GLOBAL T *Vo = gp<T>(I.f[ob][2]);
    if (all) {
        if (I.stream) {
            // the empty asm statements keep the optimiser from merging these
            // stores with the plain ones below (which drops the hint)
            __asm__ volatile("");
            vst_stream<T, VEC>(Po + off, po);
            vst_stream<T, VEC>(Uo + off, uo);
            vst_stream<T, VEC>(Vo + off, vo);
            __asm__ volatile("");
        } else {
            vst<T, VEC>(Po + off, po);
            vst<T, VEC>(Uo + off, uo);
            vst<T, VEC>(Vo + off, vo);
        }
    } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            if (ok[e]) {
                Po[off + e] = po.v[e];
                Uo[off + e] = uo.v[e];
                Vo[off + e] = vo.v[e];
            }
    }
}

template <typename T>
__device__ __forceinline__ T rad_w(const DevInst &I, int r, int k);
template <>
__device__ __forceinline__ float rad_w<float>(const DevInst &I, int r, int k) { return I.rad_wf[r][k]; }
template <>
__device__ __forceinline__ double rad_w<double>(const DevInst &I, int r, int k) { return I.rad_w7[r][k]; }

// Place of a node in the 7-node window inside the domain along one axis
// (node i of n): 3 (central) where three nodes lie on either side, else the
// distance to the near edge, mirrored at the far one.
__device__ __forceinline__ int rad_place(int i, int n)
{
    const int hi = n - 1 - i;
    return i < 3 ? i : (hi < 3 ? 6 - hi : 3);
}

// Radiation band (the nodes closer than rad_w to an edge of the domain) in
// the row pass: for the band nodes among a row's VEC nodes, the outgoing-
// wave form of the LEE without mean flow replaces the interior right-hand
// side, dq/dt = -(cos(theta) dq/dx + sin(theta) dq/dy + q/(2r)) for q = p, u,
// v with r and theta about the instance's centre, no filter term, plus the
// sponge and source terms of the row pass.  The 7-node windows come from the
// tile's LDS copy of the stage input (x windows in the tile's own rows, y
// windows in its columns between the halo rows); a y window that leaves the
// copied rows (a one-row tile at the top edge) reads global memory.  wt holds
// the window weights.  The whole band and every node it reads are fluid
// (checked at set-up), so no ghost value is involved.
template <typename T, int VEC, int TX, int TY>
__device__ __forceinline__ void band_row(const DevInst &I, const TileCtx<T> &c, const T (*reg)[TY + 10][TX + 16],
                                         const T (*wt)[7], int stage, int i, int tc, const VecT<T, VEC> &pn,
                                         const VecT<T, VEC> &un, const VecT<T, VEC> &vn, VecT<T, VEC> &po,
                                         VecT<T, VEC> &uo, VecT<T, VEC> &vo, bool (&ok)[VEC], bool &all)
{
    const int W = I.rad_w, nx = I.nx, ny = I.ny;
    const int j = c.r0 + i;
    const int ry = rad_place(j, ny);
    const int y0 = j - ry - (c.r0 - 5);          // LDS row of the y window's first node
    const bool ylds = y0 >= 0 && y0 + 6 < TY + 10;
    all = true;
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const int col = c.c0 + tc + e;
        const int eg = min(min(col, j), min(nx - 1 - col, ny - 1 - j));
        if (col < nx && eg < W) {
            const int rx = rad_place(col, nx);
            const int lc = tc + e + 8;
            // node position about the centre: the offsets in FP64, the rest in T
            const T x = (T)(I.x0 - I.rad_xc) + (T)col * (T)I.h, y = (T)(I.y0 - I.rad_yc) + (T)j * (T)I.h;
            const T ir = (T)1 / sqrt(x * x + y * y);
            const T ct = x * ir, st = y * ir, hr = (T)0.5 * ir;
            T sg = 0;
            if (c.in_sponge && eg < I.sponge_w) {
                const T fr = (T)(I.sponge_w - eg) * c.sp_inv;
                sg = c.sp_s * fr * fr;
            }
            T wx[7], wy[7];                      // this node's weights, read once for the three fields
#pragma unroll
            for (int k = 0; k < 7; ++k) {
                wx[k] = wt[rx][k];
                wy[k] = wt[ry][k];
            }
            T out[3];
#pragma unroll 1
            for (int f = 0; f < 3; ++f) {
                const T *row = &reg[f][i + 5][0];
                T dx = 0, dy = 0;
#pragma unroll
                for (int k = 0; k < 7; ++k) dx += wx[k] * row[lc - rx + k];
                if (ylds) {
#pragma unroll
                    for (int k = 0; k < 7; ++k) dy += wy[k] * reg[f][y0 + k][lc];
                } else {
                    const GLOBAL T *q = gp<T>(I.f[c.ib][f]) + (I.org + (j - ry) * I.pitch + col);
#pragma unroll 1
                    for (int k = 0; k < 7; ++k) dy += wy[k] * q[k * I.pitch];
                }
                const T qc = row[lc];
                T rq = -(ct * dx + st * dy + hr * qc) - sg * qc;
                if (f == 0 && c.has_src) {
                    const T xx = (T)(col - I.src_ic) * (T)I.h - (T)I.src_fx;
                    const T yy = (T)(j - I.src_jc) * (T)I.h - (T)I.src_fy;
                    rq += c.amp * exp(-(T)I.src_b * (xx * xx + yy * yy));
                }
                out[f] = c.adt * rq + (stage != 0 ? (f == 0 ? pn.v[e] : (f == 1 ? un.v[e] : vn.v[e])) : qc);
            }
            po.v[e] = out[0];
            uo.v[e] = out[1];
            vo.v[e] = out[2];
            ok[e] = true;
        }
        all = all && ok[e];
    }
}

#ifndef BAND_PASS
#define BAND_PASS 1
#endif

// The radiation band nodes of a tile in a pass of their own, one (node,
// field) item per thread: the items of all the tile's band nodes in the
// three fields are spread over the workgroup's threads, so no lane works
// through a chain of band nodes while the rest of its wave waits (in a
// left or right edge tile only the lanes of the first or last columns hold
// band nodes, and the edge tiles of a launch that fills the device in one
// wave are on its critical path).  Each item is band_row's arithmetic for
// one field of one node; the stage input comes from the tile's LDS copy,
// q^n from global memory.
template <typename T, int TX, int TY>
__device__ __forceinline__ void band_pass(const DevInst &I, const TileCtx<T> &c, const T (*reg)[TY + 10][TX + 16],
                                          const T (*wt)[7], int stage)
{
    const int W = I.rad_w, nx = I.nx, ny = I.ny;
    const int ncol = min(TX, nx - c.c0);         // tile columns inside the domain
    const int nrow = c.r1 - c.r0;
    // tile rows [0, lo) and [hi, nrow) lie wholly in the band (j < W or
    // j >= ny - W); the rows between hold band nodes only in the columns
    // [0, cl) and [cr, ncol) (col < W or col >= nx - W)
    const int lo = max(0, min(nrow, W - c.r0));
    const int hi = max(lo, min(nrow, ny - W - c.r0));
    const int cl = max(0, min(ncol, W - c.c0));
    const int cr = max(cl, min(ncol, nx - W - c.c0));
    const int nbc = cl + (ncol - cr);
    const int nfull = (lo + (nrow - hi)) * ncol;
    const int items = 3 * (nfull + (hi - lo) * nbc);
    for (int it = (int)threadIdx.x; it < items; it += 256) {
        const int f = it % 3, nd = it / 3;
        int i, tc;
        if (nd < nfull) {
            const int r = nd / ncol;
            i = r < lo ? r : hi + (r - lo);
            tc = nd - r * ncol;
        } else {
            const int m = nd - nfull;
            const int r = m / nbc;
            const int k = m - r * nbc;
            i = lo + r;
            tc = k < cl ? k : cr + (k - cl);
        }
        const int j = c.r0 + i, col = c.c0 + tc;
        const unsigned off = (unsigned)(I.org + j * I.pitch + col);
        // q^n first, in flight during the arithmetic
        const T qn = stage != 0 ? gp<T>(I.f[0][f])[off] : (T)0;
        const int eg = min(min(col, j), min(nx - 1 - col, ny - 1 - j));
        const int rx = rad_place(col, nx), ry = rad_place(j, ny);
        const int lc = tc + 8;
        const int y0 = j - ry - (c.r0 - 5);      // LDS row of the y window's first node
        const bool ylds = y0 >= 0 && y0 + 6 < TY + 10;
        const T x = (T)(I.x0 - I.rad_xc) + (T)col * (T)I.h, y = (T)(I.y0 - I.rad_yc) + (T)j * (T)I.h;
        const T ir = (T)1 / sqrt(x * x + y * y);
        const T ct = x * ir, st = y * ir, hr = (T)0.5 * ir;
        T sg = 0;
        if (c.in_sponge && eg < I.sponge_w) {
            const T fr = (T)(I.sponge_w - eg) * c.sp_inv;
            sg = c.sp_s * fr * fr;
        }
        const T *row = &reg[f][i + 5][0];
        T dx = 0, dy = 0;
#pragma unroll
        for (int k = 0; k < 7; ++k) dx += wt[rx][k] * row[lc - rx + k];
        if (ylds) {
#pragma unroll
            for (int k = 0; k < 7; ++k) dy += wt[ry][k] * reg[f][y0 + k][lc];
        } else {
            const GLOBAL T *q = gp<T>(I.f[c.ib][f]) + (I.org + (j - ry) * I.pitch + col);
#pragma unroll 1
            for (int k = 0; k < 7; ++k) dy += wt[ry][k] * q[k * I.pitch];
        }
        const T qc = row[lc];
        T rq = -(ct * dx + st * dy + hr * qc) - sg * qc;
        if (f == 0 && c.has_src) {
            const T xx = (T)(col - I.src_ic) * (T)I.h - (T)I.src_fx;
            const T yy = (T)(j - I.src_jc) * (T)I.h - (T)I.src_fy;
            rq += c.amp * exp(-(T)I.src_b * (xx * xx + yy * yy));
        }
        gp<T>(I.f[c.ob][f])[off] = c.adt * rq + (stage != 0 ? qn : qc);
    }
}

// Wall tiles, while the copy flies: the near-wall filter rows into LDS and
// the fluid intervals of copied row threadIdx.x (rows outside the domain
// are open) into a register.
template <typename T, int VEC, int TX, int TY>
__device__ __forceinline__ int4 wall_prefetch(const DevInst &I, const TileCtx<T> &c, T (*wfd)[6])
{
    using G = TileGeo<T, VEC, TX, TY>;
    const int tid = threadIdx.x;
    int4 r = make_int4(0, 0, 0, 0);
    if (c.wall) {
        if (tid < 36) wfd[tid / 6][tid % 6] = fdw_at<T>(I, tid / 6, tid % 6);
        const int row = c.r0 - 5 + tid;
        if (tid < G::R) r = row >= 0 && row < I.ny ? int4(gp<int4>(I.iv)[row]) : open_row();
    }
    return r;
}

// Wall tiles: the column masks of non-fluid copied rows from the rows'
// intervals (each row's bit OR-ed into every column it is not fluid at,
// after the masks are cleared); ordered before their use by the barrier
// that follows the copy.
template <typename T, int VEC, int TX, int TY>
__device__ __forceinline__ void wall_masks(const TileCtx<T> &c, const int4 wivr, ColMask<TY + 10> *wcm)
{
    using G = TileGeo<T, VEC, TX, TY>;
    __shared__ int4 wiv[G::R];
    const int tid = threadIdx.x;
    if (tid < TX) wcm[tid] = 0;
    if (tid < G::R) wiv[tid] = wivr;
    __syncthreads();
    for (int q = tid; q < TX * G::R; q += G::NT) {
        const int b = q / TX, col = q - (q / TX) * TX;
        if (!in_iv(wiv[b], c.c0 + col)) atomicOr(&wcm[col], (ColMask<G::R>)1 << b);
    }
}

// The row passes of a tile: each lane computes VEC nodes of rows i0,
// i0 + RG, .. (the q^n values of a row in flight during its arithmetic).
template <typename T, int VEC, bool FILT, int TX, int TY, bool WALL>
__device__ __forceinline__ void tile_rows(const DevInst &I, const TileCtx<T> &c, const T (*lds)[TY + 10][TX + 16],
                                          const T (*wt)[7], const T (*wb)[8], const ColMask<TY + 10> *wcm,
                                          int stage, int i0, int tc, int4 iv)
{
    using G = TileGeo<T, VEC, TX, TY>;
#pragma unroll 1
    for (int i = i0; i < TY; i += G::RG) {
        const int j = c.r0 + i;
        if (j >= c.r1) break;
        if (c.in_band && (j < I.rad_w || j >= I.ny - I.rad_w)) continue;   // wholly band nodes
        if (i != i0) iv = gp<int4>(I.iv)[j];
        VecT<T, VEC> pn{}, un{}, vn{};
        if (stage != 0) {                        // in flight during the row's arithmetic
            const unsigned qo = (unsigned)(I.org + j * I.pitch + c.c0 + tc);
            pn = vld<T, VEC>(gp<T>(I.f[0][0]) + qo);
            un = vld<T, VEC>(gp<T>(I.f[0][1]) + qo);
            vn = vld<T, VEC>(gp<T>(I.f[0][2]) + qo);
        }
        VecT<T, VEC> po, uo, vo;
        bool ok[VEC];
        bool all;
        tile_row<T, VEC, FILT, TX, TY, WALL>(I, c, lds, wb, wcm, stage, i, tc, iv, pn, un, vn, po, uo, vo, ok,
                                             all);
        if (!BAND_PASS && c.in_band)
            band_row<T, VEC, TX, TY>(I, c, lds, wt, stage, i, tc, pn, un, vn, po, uo, vo, ok, all);
        tile_store<T, VEC>(I, c.ob, (unsigned)(I.org + j * I.pitch + c.c0 + tc), po, uo, vo, ok, all);
    }
}

// One tile: wk = {instance, first column, first row, +-(end row)}.
template <typename T, int VEC, bool FILT, int TX, int TY>
__device__ __forceinline__ void tile_body(const DevInst *__restrict__ insts, const int4 wk, int stage, int slot,
                                          const GhostDep *dep, bool wall)
{
    using G = TileGeo<T, VEC, TX, TY>;
    __shared__ alignas(16) T lds[3][G::R][G::LW];
    const DevInst &I = insts[wk.x];
    const long long step = sload<long long>(I.step) + slot;
    if (step >= sload<long long>(I.stop)) return;
    const int tid = threadIdx.x;
    const TileCtx<T> c = tile_ctx<T, TX>(I, wk, stage, step, FILT && wall);
    tile_copy<T, VEC, TX, TY>(I, c, lds);
    __shared__ T wt[7][7];                       // radiation window weights (band tiles only)
    if (c.in_band && tid < 49) wt[tid / 7][tid % 7] = rad_w<T>(I, tid / 7, tid % 7);
    // wall tiles: the near-wall filter rows and the fluid intervals of the
    // copied rows (rows outside the domain are open)
    __shared__ T wfd[6][6];
    __shared__ alignas(16) T wb[6][8];           // near-wall filter rows, half-width w = 0..5
    __shared__ ColMask<G::R> wcm[TX];            // per tile column, its non-fluid copied rows
    const int4 wivr = wall_prefetch<T, VEC, TX, TY>(I, c, wfd);
    if (c.wall && tid < 48) {
        const int w = tid / 8, k = tid % 8;
        wb[w][k] = k < 6 ? (T)((k == 0 ? 0.5 * I.fd[0] : I.fd[k]) + I.fdw[w][k]) : (T)0;
    }
    // while the copy flies: this lane's first row ranges and its first patch
    // entries
    const int i0 = tid / G::NCX;
    int4 iv = make_int4(0, 0, 0, 0);
    if (i0 < TY && c.r0 + i0 < c.r1) iv = gp<int4>(I.iv)[c.r0 + i0];
    int2 pre[2];
    if (dep) patch_prefetch(dep->patch, dep->p0, dep->p1, pre);
    if (c.wall) wall_masks<T, VEC, TX, TY>(c, wivr, wcm);
    __builtin_amdgcn_s_waitcnt(0);               // this wave's DMA has landed in LDS
    __syncthreads();                             // ... and every other wave's
    if (dep) {                                   // this stage's ghost values over the copied ones
        tile_patch<T, TX, TY>(I, stage_epoch(step, stage), lds, *dep, pre);
        __syncthreads();
    }
    const int tc = (tid % G::NCX) * VEC;
    // wall tiles run a row loop of their own, so that the near-wall code
    // takes nothing from the scheduling of the plain tiles' loop
    if (FILT && c.wall)
        tile_rows<T, VEC, FILT, TX, TY, true>(I, c, lds, wt, wb, wcm, stage, i0, tc, iv);
    else
        tile_rows<T, VEC, FILT, TX, TY, false>(I, c, lds, wt, wb, wcm, stage, i0, tc, iv);
    if (BAND_PASS && c.in_band) band_pass<T, TX, TY>(I, c, lds, wt, stage);
}

// Work items of the tile sweep: x = instance | DEP_BIT when a fused tile's
// read region holds ghost nodes | TILE_WALL_BIT when it does in either form,
// -1 for an idle slot of the XCD-aware order.
constexpr int DEP_BIT = TILE_DEP_BIT;

template <typename T, int VEC, bool FILT, int TX, int TY>
__global__ __launch_bounds__(256) void k_tile(const DevInst *__restrict__ insts, const int4 *__restrict__ work,
                                              int nwork, int stage, int slot)
{
    const int w = blockIdx.x;
    if (w >= nwork) return;
    int4 wk = work[w];
    if (wk.x < 0) return;
    const bool wall = (wk.x & TILE_WALL_BIT) != 0;
    wk.x &= TILE_INST_MASK;
    tile_body<T, VEC, FILT, TX, TY>(insts, wk, stage, slot, nullptr, wall);
}

// One stage in one launch.  The first ncar workgroups each fill 256 / GL
// ghosts (ghost fill and ADE update) before their own tile and publish each
// ghost value with this stage's epoch in the exchange words; no workgroups
// are added for the ghosts, so a launch that fills the device in one wave
// still does.  Tiles whose stencils read no ghost node run at once.  The
// others start their LDS copy and then take the ghost values they read
// (aux[k] = their range in patch) as soon as those carry the epoch.  The
// ghost shares belong to the lowest workgroup ids and no waiting tile has
// such an id (the host orders the work so), so they are dispatched no later
// than any tile that waits for them and they wait for nothing themselves;
// each wait is bounded by spin_limit polls all the same, and a wait that runs
// out raises the error flag sync[4] instead of hanging.  The probe pass, if
// any, runs in the workgroups after the tiles (tend and up).
template <typename T, int VEC, bool FILT, int TX, int TY, int GL, int GV>
__global__ __launch_bounds__(256) void k_stage(const DevInst *__restrict__ insts, const int4 *__restrict__ work1,
                                               int nwork1, const int4 *__restrict__ work2, int nwork2, int ncar,
                                               int tile0, int tend, int stage, int slot, int *sync, int spin_limit,
                                               const int2 *__restrict__ aux, const int2 *__restrict__ patch,
                                               ProbePass pp)
{
    const int tid = threadIdx.x;
    const int w = (int)blockIdx.x;
    if (w >= tend) {
        probe_item<T>(insts, pp, (w - tend) * 16 + tid / 16, tid % 16);
        return;
    }
    if (w < ncar)
        ghost_item<T, GL, true, GV>(insts, work2, nwork2, w * (256 / GL) + tid / GL, tid % GL, stage, slot);
    const int k = w - tile0;
    if (k < 0 || k >= nwork1) return;
    int4 wk = work1[k];
    if (wk.x < 0) return;
    const bool wall = (wk.x & TILE_WALL_BIT) != 0;
    if (wk.x & DEP_BIT) {
        wk.x &= TILE_INST_MASK;
        const int2 rg = aux[k];
        const GhostDep dep{&sync[4], spin_limit, patch, rg.x, rg.y};
        tile_body<T, VEC, FILT, TX, TY>(insts, wk, stage, slot, &dep, wall);
    } else {
        wk.x &= TILE_INST_MASK;
        tile_body<T, VEC, FILT, TX, TY>(insts, wk, stage, slot, nullptr, wall);
    }
}

// ---------------------------------------------------------------------------
// the filter once per step (the explicit form)

// One field's filter sum at the VEC nodes of one row of a tile's LDS copy:
// fd[0] q_0 + sum_k fd[k] ((q_{x+k} + q_{x-k}) + (q_{y+k} + q_{y-k})), the sum
// of row_field's damping term in the same order.
template <typename T, int VEC, int LW>
__device__ __forceinline__ void filt_field(const T (*lds)[LW], int y, int lc, const T (&fd)[6], T (&fl)[VEC])
{
    constexpr int KM = (5 + VEC - 1) / VEC;
    constexpr int KP = (VEC + 4) / VEC;
    constexpr int XW = (KM + 1 + KP) * VEC;
    T yw[11][VEC];
#pragma unroll
    for (int k = 0; k < 11; ++k) {
        const VecT<T, VEC> a = lds16<T, VEC>(&lds[y - 5 + k][lc]);
#pragma unroll
        for (int e = 0; e < VEC; ++e) yw[k][e] = a.v[e];
    }
    T xw[XW];
#pragma unroll
    for (int k = -KM; k <= KP; ++k) {
        if (k == 0) {
#pragma unroll
            for (int e = 0; e < VEC; ++e) xw[KM * VEC + e] = yw[5][e];
            continue;
        }
        if (k == -KM) {
            xw[VEC - 1] = lds[y][lc - KM * VEC + VEC - 1];
            continue;
        }
        if (k == KP) {
            xw[(KM + KP) * VEC] = lds[y][lc + KP * VEC];
            continue;
        }
        const VecT<T, VEC> a = lds16<T, VEC>(&lds[y][lc + k * VEC]);
#pragma unroll
        for (int e = 0; e < VEC; ++e) xw[(k + KM) * VEC + e] = a.v[e];
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        const int x = KM * VEC + e;
        T f = fd[0] * yw[5][e];
#pragma unroll
        for (int k = 1; k <= 5; ++k) f += fd[k] * ((xw[x + k] + xw[x - k]) + (yw[5 + k][e] + yw[5 - k][e]));
        fl[e] = f;
    }
}

// The explicit filter after step `slot` of a run: in this form a step's
// last stage leaves its result in register set C; each tile copies it with
// its halo into LDS and every fluid node outside the radiation band takes
// q - sigma_d (F_x + F_y) q into register set A (fd and fdw hold sigma_d
// times the rows in this form; nodes within five of the wall take the
// narrower rows as in the stages).  Other nodes of A are not written: the
// next stage fills the ghosts again.  Members without the explicit filter,
// or past their stop step, are skipped.
template <typename T, int VEC, int TX, int TY>
__global__ __launch_bounds__(256) void k_filter(const DevInst *__restrict__ insts, const int4 *__restrict__ work,
                                                int nwork, int slot)
{
    using G = TileGeo<T, VEC, TX, TY>;
    __shared__ alignas(16) T lds[3][G::R][G::LW];
    const int w = blockIdx.x;
    if (w >= nwork) return;
    int4 wk = work[w];
    if (wk.x < 0) return;
    const bool wall = (wk.x & TILE_WALL_BIT) != 0;
    wk.x &= TILE_INST_MASK;
    const DevInst &I = insts[wk.x];
    if (!I.fx) return;
    const long long step = sload<long long>(I.step) + slot;
    if (step >= sload<long long>(I.stop)) return;
    const int tid = threadIdx.x;
    TileCtx<T> c = tile_ctx<T, TX>(I, wk, 3, step, wall);
    c.ib = 2;
    c.ob = 0;
    tile_copy<T, VEC, TX, TY>(I, c, lds);
    __shared__ T wfd[6][6];
    __shared__ ColMask<G::R> wcm[TX];
    const int4 wivr = wall_prefetch<T, VEC, TX, TY>(I, c, wfd);
    const int i0 = tid / G::NCX;
    int4 iv = make_int4(0, 0, 0, 0);
    if (i0 < TY && c.r0 + i0 < c.r1) iv = gp<int4>(I.iv)[c.r0 + i0];
    if (c.wall) wall_masks<T, VEC, TX, TY>(c, wivr, wcm);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int tc = (tid % G::NCX) * VEC;
#pragma unroll 1
    for (int i = i0; i < TY; i += G::RG) {
        const int j = c.r0 + i;
        if (j >= c.r1) break;
        if (i != i0) iv = gp<int4>(I.iv)[j];
        const int y = i + 5, lc = tc + 8, gc = c.c0 + tc;
        T rp[VEC], ru[VEC], rv[VEC];
        filt_field<T, VEC, TX + 16>(lds[0], y, lc, c.fd, rp);
        filt_field<T, VEC, TX + 16>(lds[1], y, lc, c.fd, ru);
        filt_field<T, VEC, TX + 16>(lds[2], y, lc, c.fd, rv);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            rp[e] = -rp[e];
            ru[e] = -ru[e];
            rv[e] = -rv[e];
        }
        if (c.wall) wall_rows<T, VEC, TX, TY>(I, lds, wfd, wcm, y, lc, gc, tc, iv, rp, ru, rv);
        const VecT<T, VEC> pc = *(const VecT<T, VEC> *)&lds[0][y][lc];
        const VecT<T, VEC> uc = *(const VecT<T, VEC> *)&lds[1][y][lc];
        const VecT<T, VEC> vc = *(const VecT<T, VEC> *)&lds[2][y][lc];
        VecT<T, VEC> po, uo, vo;
        bool ok[VEC];
        bool all = true;
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
            const int col = gc + e;
            po.v[e] = pc.v[e] + rp[e];
            uo.v[e] = uc.v[e] + ru[e];
            vo.v[e] = vc.v[e] + rv[e];
            ok[e] = in_iv(iv, col);
            if (c.in_band && min(min(col, j), min(I.nx - 1 - col, I.ny - 1 - j)) < I.rad_w) ok[e] = false;
            all = all && ok[e];
        }
        tile_store<T, VEC>(I, 0, (unsigned)(I.org + j * I.pitch + c.c0 + tc), po, uo, vo, ok, all);
        if (c.in_band) {
            // band nodes keep the step's value: copy it from C to A
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const int col = gc + e;
                if (in_iv(iv, col) && min(min(col, j), min(I.nx - 1 - col, I.ny - 1 - j)) < I.rad_w) {
                    const unsigned off = (unsigned)(I.org + j * I.pitch + col);
                    gp<T>(I.f[0][0])[off] = pc.v[e];
                    gp<T>(I.f[0][1])[off] = uc.v[e];
                    gp<T>(I.f[0][2])[off] = vc.v[e];
                }
            }
        }
    }
}

template <typename T>
__global__ void k_fill(T *p, size_t n, T v)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// initial condition at fluid nodes of q^n (Sec. 2.1, 4.1, 4.2)
template <typename T>
__global__ void k_init_ic(const DevInst *__restrict__ insts, int ic_kind, double c0, double c1, double c2,
                          double c3, double c4, double c5, double c6)
{
    const DevInst &I = insts[0];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= I.nx || j >= I.ny) return;
    const int4 iv = I.iv[j];
    if (!((i >= iv.x && i < iv.y) || (i >= iv.z && i < iv.w))) return;
    const double x = I.x0 + (double)i * I.h, y = I.y0 + (double)j * I.h;
    double p = 0, u = 0, v = 0;
    if (ic_kind == 1) {
        const double b = 0.6931471805599453 / (c3 * c3);
        p = c2 * exp(-b * ((x - c0) * (x - c0) + (y - c1) * (y - c1)));
    } else if (ic_kind == 2) {
        const double s = (x - c0) * c2 + (y - c1) * c3;
        p = 0.5 * c4 * exp(-(c5 * c5) * s * s) * cos(6.283185307179586 * c6 * s);
        u = p * c2;
        v = p * c3;
    }
    const long off = (long)I.org + (long)j * I.pitch + i;
    ((T *)I.f[0][0])[off] = (T)p;
    ((T *)I.f[0][1])[off] = (T)u;
    ((T *)I.f[0][2])[off] = (T)v;
}

template <typename T>
__global__ void k_sample(const DevInst *__restrict__ insts, const int *__restrict__ ij, const double *__restrict__ w,
                         int np, double *out)
{
    const DevInst &I = insts[0];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= np) return;
    double acc[3] = {0, 0, 0};
    for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 4; ++a) {
            const long off = (long)I.org + (long)(ij[2 * k + 1] + b) * I.pitch + (ij[2 * k] + a);
            for (int f = 0; f < 3; ++f) acc[f] += w[16 * k + b * 4 + a] * (double)((const T *)I.f[0][f])[off];
        }
    for (int f = 0; f < 3; ++f) out[3 * k + f] = acc[f];
}

// ---------------------------------------------------------------------------
// launch wrappers

template <typename T, int VEC, bool FILT, int WPB>
static hipError_t launch_sweep_t(const DevInst *insts, const int4 *work, int nwork, int stage, int slot, int blocks,
                                 hipStream_t s)
{
    const int nb = blocks > 0 ? blocks : (nwork + WPB - 1) / WPB;
    hipLaunchKernelGGL((k_sweep<T, VEC, FILT, WPB>), dim3(nb), dim3(64 * WPB), 0, s, insts, work, nwork, stage, slot);
    return hipGetLastError();
}

template <typename T, int VEC, bool FILT>
static hipError_t launch_sweep_w(const DevInst *insts, const int4 *work, int nwork, int stage, int slot, int waves,
                                 int blocks, hipStream_t s)
{
    if (waves == 4) return launch_sweep_t<T, VEC, FILT, 4>(insts, work, nwork, stage, slot, blocks, s);
    if (waves == 2) return launch_sweep_t<T, VEC, FILT, 2>(insts, work, nwork, stage, slot, blocks, s);
    return launch_sweep_t<T, VEC, FILT, 1>(insts, work, nwork, stage, slot, blocks, s);
}

hipError_t launch_sweep(int prec, int vec, bool filt, int waves, const DevInst *insts, const int4 *work,
                        int nwork, int stage, int slot, int blocks, hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    if (prec == LEE_F32) {
        if (vec == 4) return filt ? launch_sweep_w<float, 4, true>(insts, work, nwork, stage, slot, waves, blocks, s)
                                  : launch_sweep_w<float, 4, false>(insts, work, nwork, stage, slot, waves, blocks, s);
        return filt ? launch_sweep_w<float, 2, true>(insts, work, nwork, stage, slot, waves, blocks, s)
                    : launch_sweep_w<float, 2, false>(insts, work, nwork, stage, slot, waves, blocks, s);
    }
    return filt ? launch_sweep_w<double, 2, true>(insts, work, nwork, stage, slot, waves, blocks, s)
                : launch_sweep_w<double, 2, false>(insts, work, nwork, stage, slot, waves, blocks, s);
}


// Lanes per ghost: 32 in the fused stage, whose ghost-carrying workgroups
// are on the launch's critical path (8 ghosts each, shorter per-lane load
// chains), 16 in the separate ghost launch, which batches fill with many
// ghosts (16 per workgroup, fewer idle lanes).
constexpr int GHOST_LANES_FUSED = 32;
constexpr int GHOST_LANES = 16;

// Fused launch arguments (the ghost part, the tile offset, the probe pass).
struct FuseArgs {
    const int4 *work2;
    int nwork2;
    int *sync;
    int spin_limit;
    const int2 *aux;
    const int2 *patch;
    int tile0;
    ProbePass pp;
    int gv;                                      // ghost-fill variant (GV_*)
};

template <typename T, int VEC, bool FILT, int TX, int TY>
static hipError_t launch_tile_t(const DevInst *insts, const int4 *work, int nwork, int stage, int slot,
                                const FuseArgs *fa, hipStream_t s)
{
    if (!fa) {
        hipLaunchKernelGGL((k_tile<T, VEC, FILT, TX, TY>), dim3(nwork), dim3(256), 0, s, insts, work, nwork, stage,
                           slot);
    } else {
        // the first ncar workgroups carry 256 / GHOST_LANES_FUSED ghosts each;
        // the probe pass takes 16 probes per workgroup after the tiles
        const int ncar = (fa->nwork2 * GHOST_LANES_FUSED + 255) / 256;
        const int tend = std::max(ncar, fa->tile0 + nwork);
        const int nbp = (fa->pp.np + 15) / 16;
        constexpr int GL = GHOST_LANES_FUSED;
        if (fa->gv == GV_ONE)
            hipLaunchKernelGGL((k_stage<T, VEC, FILT, TX, TY, GL, GV_ONE>), dim3(tend + nbp), dim3(256), 0, s, insts,
                               work, nwork, fa->work2, fa->nwork2, ncar, fa->tile0, tend, stage, slot, fa->sync,
                               fa->spin_limit, fa->aux, fa->patch, fa->pp);
        else if (fa->gv == (GV_ONE | GV_POLES))
            hipLaunchKernelGGL((k_stage<T, VEC, FILT, TX, TY, GL, GV_ONE | GV_POLES>), dim3(tend + nbp), dim3(256), 0,
                               s, insts, work, nwork, fa->work2, fa->nwork2, ncar, fa->tile0, tend, stage, slot,
                               fa->sync, fa->spin_limit, fa->aux, fa->patch, fa->pp);
        else if (fa->gv == GV_POLES)
            hipLaunchKernelGGL((k_stage<T, VEC, FILT, TX, TY, GL, GV_POLES>), dim3(tend + nbp), dim3(256), 0, s, insts,
                               work, nwork, fa->work2, fa->nwork2, ncar, fa->tile0, tend, stage, slot, fa->sync,
                               fa->spin_limit, fa->aux, fa->patch, fa->pp);
        else
            hipLaunchKernelGGL((k_stage<T, VEC, FILT, TX, TY, GL, GV_TABLE>), dim3(tend + nbp), dim3(256), 0, s, insts,
                               work, nwork, fa->work2, fa->nwork2, ncar, fa->tile0, tend, stage, slot, fa->sync,
                               fa->spin_limit, fa->aux, fa->patch, fa->pp);
    }
    return hipGetLastError();
}

// supported tile shapes (columns x rows)
template <typename T, int VEC, bool FILT>
static hipError_t launch_tile_v(int tx, int ty, const DevInst *insts, const int4 *work, int nwork, int stage,
                                int slot, const FuseArgs *fa, hipStream_t s)
{
    constexpr bool F4 = sizeof(T) == 4;
    if (tx == 128) {
        if (ty == 4) return launch_tile_t<T, VEC, FILT, 128, 4>(insts, work, nwork, stage, slot, fa, s);
        if (ty == 8) return launch_tile_t<T, VEC, FILT, 128, 8>(insts, work, nwork, stage, slot, fa, s);
        if (ty == 16) return launch_tile_t<T, VEC, FILT, 128, 16>(insts, work, nwork, stage, slot, fa, s);
        if (F4 && ty == 32)
            return launch_tile_t<T, VEC, FILT, 128, (F4 ? 32 : 16)>(insts, work, nwork, stage, slot, fa, s);
    } else if (tx == 256) {
        if (ty == 4) return launch_tile_t<T, VEC, FILT, 256, 4>(insts, work, nwork, stage, slot, fa, s);
        if (F4 && ty == 8)
            return launch_tile_t<T, VEC, FILT, 256, (F4 ? 8 : 4)>(insts, work, nwork, stage, slot, fa, s);
        if (F4 && ty == 16)
            return launch_tile_t<T, VEC, FILT, 256, (F4 ? 16 : 4)>(insts, work, nwork, stage, slot, fa, s);
    } else if (tx == 64) {
        if (ty == 8) return launch_tile_t<T, VEC, FILT, 64, 8>(insts, work, nwork, stage, slot, fa, s);
        if (ty == 16) return launch_tile_t<T, VEC, FILT, 64, 16>(insts, work, nwork, stage, slot, fa, s);
        if (ty == 32) return launch_tile_t<T, VEC, FILT, 64, 32>(insts, work, nwork, stage, slot, fa, s);
    }
    return hipErrorInvalidValue;
}

bool tile_shape_supported(int prec, int tx, int ty)
{
    const bool f4 = prec == LEE_F32;
    if (tx == 128) return ty == 4 || ty == 8 || ty == 16 || (f4 && ty == 32);
    if (tx == 256) return ty == 4 || (f4 && (ty == 8 || ty == 16));
    if (tx == 64) return ty == 8 || ty == 16 || ty == 32;
    return false;
}


hipError_t launch_tile(int prec, bool filt, int tx, int ty, const DevInst *insts, const int4 *work, int nwork,
                       int stage, int slot, int blocks, hipStream_t s)
{
    (void)blocks;                                // one workgroup per tile
    if (nwork <= 0) return hipSuccess;
    if (prec == LEE_F32)
        return filt ? launch_tile_v<float, 4, true>(tx, ty, insts, work, nwork, stage, slot, nullptr, s)
                    : launch_tile_v<float, 4, false>(tx, ty, insts, work, nwork, stage, slot, nullptr, s);
    return filt ? launch_tile_v<double, 2, true>(tx, ty, insts, work, nwork, stage, slot, nullptr, s)
                : launch_tile_v<double, 2, false>(tx, ty, insts, work, nwork, stage, slot, nullptr, s);
}

template <typename T, int VEC, int TX, int TY>
static hipError_t launch_filter_t(const DevInst *insts, const int4 *work, int nwork, int slot, hipStream_t s)
{
    hipLaunchKernelGGL((k_filter<T, VEC, TX, TY>), dim3(nwork), dim3(256), 0, s, insts, work, nwork, slot);
    return hipGetLastError();
}

template <typename T, int VEC>
static hipError_t launch_filter_v(int tx, int ty, const DevInst *insts, const int4 *work, int nwork, int slot,
                                  hipStream_t s)
{
    constexpr bool F4 = sizeof(T) == 4;
    if (tx == 128) {
        if (ty == 4) return launch_filter_t<T, VEC, 128, 4>(insts, work, nwork, slot, s);
        if (ty == 8) return launch_filter_t<T, VEC, 128, 8>(insts, work, nwork, slot, s);
        if (ty == 16) return launch_filter_t<T, VEC, 128, 16>(insts, work, nwork, slot, s);
        if (F4 && ty == 32) return launch_filter_t<T, VEC, 128, (F4 ? 32 : 16)>(insts, work, nwork, slot, s);
    } else if (tx == 256) {
        if (ty == 4) return launch_filter_t<T, VEC, 256, 4>(insts, work, nwork, slot, s);
        if (F4 && ty == 8) return launch_filter_t<T, VEC, 256, (F4 ? 8 : 4)>(insts, work, nwork, slot, s);
        if (F4 && ty == 16) return launch_filter_t<T, VEC, 256, (F4 ? 16 : 4)>(insts, work, nwork, slot, s);
    } else if (tx == 64) {
        if (ty == 8) return launch_filter_t<T, VEC, 64, 8>(insts, work, nwork, slot, s);
        if (ty == 16) return launch_filter_t<T, VEC, 64, 16>(insts, work, nwork, slot, s);
        if (ty == 32) return launch_filter_t<T, VEC, 64, 32>(insts, work, nwork, slot, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_filter(int prec, int tx, int ty, const DevInst *insts, const int4 *work, int nwork, int slot,
                         hipStream_t s)
{
    if (nwork <= 0) return hipSuccess;
    if (prec == LEE_F32) return launch_filter_v<float, 4>(tx, ty, insts, work, nwork, slot, s);
    return launch_filter_v<double, 2>(tx, ty, insts, work, nwork, slot, s);
}

static int ghost_variant(int ninst, bool poles) { return (ninst == 1 ? GV_ONE : GV_TABLE) | (poles ? GV_POLES : 0); }

hipError_t launch_stage(int prec, bool filt, int tx, int ty, const DevInst *insts, int ninst, bool poles,
                        const int4 *work1, int nwork1, const int2 *aux, const int2 *patch, int tile0,
                        const int4 *work2, int nwork2, int stage, int slot, int *sync, int spin_limit, ProbePass pp,
                        hipStream_t s)
{
    if (nwork2 <= 0) {                           // no ghosts: the plain sweep, then the probes
        hipError_t e = launch_tile(prec, filt, tx, ty, insts, work1, nwork1, stage, slot, 0, s);
        if (e == hipSuccess && pp.np > 0) e = launch_probe(prec, insts, pp, s);
        return e;
    }
    const FuseArgs fa{work2, nwork2, sync, spin_limit, aux, patch, tile0, pp, ghost_variant(ninst, poles)};
    if (prec == LEE_F32)
        return filt ? launch_tile_v<float, 4, true>(tx, ty, insts, work1, nwork1, stage, slot, &fa, s)
                    : launch_tile_v<float, 4, false>(tx, ty, insts, work1, nwork1, stage, slot, &fa, s);
    return filt ? launch_tile_v<double, 2, true>(tx, ty, insts, work1, nwork1, stage, slot, &fa, s)
                : launch_tile_v<double, 2, false>(tx, ty, insts, work1, nwork1, stage, slot, &fa, s);
}

template <typename T>
static void launch_ghost_t(int gv, const DevInst *insts, const int4 *work, int nwork, int stage, int slot,
                           ProbePass pp, int nb, hipStream_t s)
{
    constexpr int GL = GHOST_LANES;
    if (gv == GV_ONE)
        hipLaunchKernelGGL((k_ghost<T, GL, GV_ONE>), dim3(nb), dim3(256), 0, s, insts, work, nwork, stage, slot, pp);
    else if (gv == (GV_ONE | GV_POLES))
        hipLaunchKernelGGL((k_ghost<T, GL, GV_ONE | GV_POLES>), dim3(nb), dim3(256), 0, s, insts, work, nwork, stage,
                           slot, pp);
    else if (gv == GV_POLES)
        hipLaunchKernelGGL((k_ghost<T, GL, GV_POLES>), dim3(nb), dim3(256), 0, s, insts, work, nwork, stage, slot,
                           pp);
    else
        hipLaunchKernelGGL((k_ghost<T, GL, GV_TABLE>), dim3(nb), dim3(256), 0, s, insts, work, nwork, stage, slot,
                           pp);
}

hipError_t launch_ghost(int prec, const DevInst *insts, int ninst, bool poles, const int4 *work, int nwork,
                        int stage, int slot, ProbePass pp, hipStream_t s)
{
    const int nb = (std::max(nwork, 0) * GHOST_LANES + 255) / 256 + (pp.np + 15) / 16;
    if (nb == 0) return hipSuccess;
    if (prec == LEE_F32)
        launch_ghost_t<float>(ghost_variant(ninst, poles), insts, work, std::max(nwork, 0), stage, slot, pp, nb, s);
    else
        launch_ghost_t<double>(ghost_variant(ninst, poles), insts, work, std::max(nwork, 0), stage, slot, pp, nb, s);
    return hipGetLastError();
}

hipError_t launch_probe(int prec, const DevInst *insts, ProbePass pp, hipStream_t s)
{
    if (pp.np <= 0) return hipSuccess;
    const int nb = (pp.np + 15) / 16;
    if (prec == LEE_F32)
        hipLaunchKernelGGL((k_probe<float>), dim3(nb), dim3(256), 0, s, insts, pp);
    else
        hipLaunchKernelGGL((k_probe<double>), dim3(nb), dim3(256), 0, s, insts, pp);
    return hipGetLastError();
}

hipError_t launch_advance(const DevInst *insts, int ninst, int n, hipStream_t s)
{
    if (ninst <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_advance, dim3((ninst + 255) / 256), dim3(256), 0, s, insts, ninst, n);
    return hipGetLastError();
}

// dst[4] |= src[4]: a ghost-wait error flag raised in one set of sync words
// carried over to another
__global__ void k_merge_flag(const int *__restrict__ src, int *__restrict__ dst)
{
    if (threadIdx.x == 0 && src[4] != 0) atomicOr(&dst[4], src[4]);
}

hipError_t launch_merge_flag(const int *src, int *dst, hipStream_t s)
{
    hipLaunchKernelGGL(k_merge_flag, dim3(1), dim3(64), 0, s, src, dst);
    return hipGetLastError();
}

hipError_t launch_fill(int prec, void *p, size_t n, hipStream_t s)
{
    const int nb = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    if (n == 0) return hipSuccess;
    if (prec == LEE_F32)
        hipLaunchKernelGGL((k_fill<float>), dim3(nb), dim3(256), 0, s, (float *)p, n, 0.0f);
    else
        hipLaunchKernelGGL((k_fill<double>), dim3(nb), dim3(256), 0, s, (double *)p, n, 0.0);
    return hipGetLastError();
}

hipError_t launch_fill_bytes(void *p, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    const int nb = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    hipLaunchKernelGGL((k_fill<uint32_t>), dim3(nb), dim3(256), 0, s, (uint32_t *)p, n, 0u);
    return hipGetLastError();
}

hipError_t launch_init_ic(int prec, const DevInst *insts, int nx, int ny, int kind, const double *c, hipStream_t s)
{
    dim3 grid((nx + 255) / 256, ny);
    if (prec == LEE_F32)
        hipLaunchKernelGGL((k_init_ic<float>), grid, dim3(256), 0, s, insts, kind, c[0], c[1], c[2], c[3], c[4],
                           c[5], c[6]);
    else
        hipLaunchKernelGGL((k_init_ic<double>), grid, dim3(256), 0, s, insts, kind, c[0], c[1], c[2], c[3], c[4],
                           c[5], c[6]);
    return hipGetLastError();
}

hipError_t launch_sample(int prec, const DevInst *insts, const int *ij, const double *w, int np, double *out,
                         hipStream_t s)
{
    if (np <= 0) return hipSuccess;
    if (prec == LEE_F32)
        hipLaunchKernelGGL((k_sample<float>), dim3((np + 63) / 64), dim3(64), 0, s, insts, ij, w, np, out);
    else
        hipLaunchKernelGGL((k_sample<double>), dim3((np + 63) / 64), dim3(64), 0, s, insts, ij, w, np, out);
    return hipGetLastError();
}

}  // namespace lee

namespace lee {

// plain device copy, one 16-byte chunk per lane (a grid-stride loop over
// fewer workgroups measured 25% slower at 1 GiB): the reference kernel of
// known traffic (2 x bytes) for calibrating hardware byte counters and the
// achievable HBM rate
__global__ __launch_bounds__(256) void k_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 16;
    if (n == 0) return hipSuccess;
    const int nb = (int)std::min<size_t>((n + 255) / 256, (size_t)1 << 30);
    hipLaunchKernelGGL(k_copy, dim3(nb), dim3(256), 0, s, (const uint4 *)src, (uint4 *)dst, n);
    return hipGetLastError();
}

}  // namespace lee
