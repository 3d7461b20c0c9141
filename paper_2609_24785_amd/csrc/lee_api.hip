// C ABI of the library: instance life cycle, device memory layout, work lists,
// stage sequencing, hipGraph capture of a step, probes and timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstddef>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <mutex>
#include <string>
#include <vector>

#include "lee_device.h"

using namespace lee;

constexpr int GRAPH_STEPS_DEFAULT = 16;            // measured: amortises the gap between graph launches
constexpr int GRAPH_STEPS_MAX = 256;

// Captured steps: `many` holds `per` consecutive steps, `one` a single step
// for the remainder.  per == 0 launches every kernel eagerly.
struct StepGraphs {
    int per = GRAPH_STEPS_DEFAULT;
    int64_t captures = 0;           // graphs captured so far
    hipGraph_t gm = nullptr, g1 = nullptr;
    hipGraphExec_t em = nullptr, e1 = nullptr;
    int rest_len = 0;               // steps of the remainder graph (g1, e1)
    void drop_rest()
    {
        if (e1) hipGraphExecDestroy(e1);
        if (g1) hipGraphDestroy(g1);
        e1 = nullptr;
        g1 = nullptr;
        rest_len = 0;
    }
    void drop()
    {
        if (em) hipGraphExecDestroy(em);
        if (gm) hipGraphDestroy(gm);
        em = nullptr;
        gm = nullptr;
        drop_rest();
    }
};
struct lee_instance {
    Host host;
    lee_tiling tl{};
    // device
    bool bound = false;
    int device = -1;
    hipStream_t stream = nullptr;
    char *base = nullptr;
    size_t bytes = 0;
    DevInst dev{};
    DevInst *d_inst = nullptr;
    int4 *d_work1 = nullptr;
    size_t work1_cap = 0;
    int nwork1 = 0;
    int2 *d_aux = nullptr;          // per work slot: range of its ghost patches
    int tile0 = 0;                  // fused launch: id of the first tile workgroup
    int2 *d_patch = nullptr;        // (LDS index, plane offset) of ghost nodes read by fused tiles
    size_t patch_cap = 0;
    int4 *d_work2 = nullptr;
    int nwork2 = 0;
    int *d_sync = nullptr;          // fused-stage error flag
    int2 *d_pwork = nullptr;        // (member, probe) pairs of the probe pass
    std::vector<int2> up_pwork;
    int *d_sij = nullptr;
    double *d_sw = nullptr, *d_sout = nullptr;
    // host staging kept alive for asynchronous uploads
    std::vector<char> up_w4, up_gd;
    std::vector<int> up_goff, up_coff;
    std::vector<int4> up_work1, up_iv;
    std::vector<int2> up_aux, up_patch;
    std::vector<int4> up_work2;
    long long up_counters[2] = {0, LLONG_MAX};
    // sequencing
    StepGraphs graphs;
    int next_stage = 0;
    int64_t steps_issued = 0;
    int spin = SPIN_LIMIT;          // polls per ghost-value wait (negative: test mode)
};

namespace {

constexpr int SAMPLE_MAX = 256;

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int esize(const Host &h) { return h.d.precision == LEE_F32 ? 4 : 8; }

int pitch_of(const Host &h)
{
    int p = LPAD + h.d.nx + RPAD_MIN;
    return (p + 63) / 64 * 64;
}

size_t plane_elems(const Host &h) { return (size_t)(h.d.ny + 2 * FRAME) * pitch_of(h); }

// A ghost node lies in the stencil region of at most 4 row tiles (rows >= 4)
// and 2 column blocks (cols >= 64), with one entry per field.
// Band rows cut into one-row tiles (radiation band on) add at most 2 rw row
// ranges to a ghost's reach.
size_t band_rows(const Host &h) { return h.d.radiation ? 2 * (size_t)h.d.stencil_half : 0; }

size_t patch_capacity(const Host &h) { return (24 + 6 * band_rows(h)) * h.gidx.size() + 64; }

// Relative cost of a sweep item whose nodes take the near-wall filter rows
// (measured: about twice a plain tile's time).
constexpr int WALL_ITEM_COST = 2;

// Field planes beyond this many bytes take streaming (non-temporal) stores.
constexpr size_t STREAM_STORE_BYTES = size_t(128) << 20;

// With planes beyond STREAM_STORE_BYTES but q^n planes (read in every stage)
// within QN_RESIDENT_BYTES of the 256 MB on-chip cache, the halo copy of the
// other stage inputs takes non-temporal loads, so that they do not displace
// q^n from the cache during a step (measured at 4096^2: FP32, whose q^n
// planes take 202 MB, 3.8% shorter steps; FP64, 404 MB, 14% longer launches
// with the same loads, hence the bound).
constexpr size_t QN_RESIDENT_BYTES = size_t(224) << 20;

int stream_in_for(size_t plane_bytes, size_t qn_bytes)
{
    return plane_bytes > STREAM_STORE_BYTES && qn_bytes <= QN_RESIDENT_BYTES ? 1 : 0;
}

size_t work1_capacity(const Host &h)
{
    const int ow_min = 64;                       // narrowest strip: 64-column tiles
    const size_t strips = (h.d.nx + ow_min - 1) / ow_min;
    const size_t tiles = (h.d.ny + 3) / 4 + band_rows(h);
    // the slot order pads the list to at most WALL_ITEM_COST times the
    // items plus 24 units of up to 4 items
    return WALL_ITEM_COST * strips * tiles + 128;
}

struct Layout {
    size_t inst, planes[9], psi[3], iv, goff, cptr, coff, w4, gd, counters, pij, pw, pwork, trace, dft, watch, xg,
        work1, aux, patch, work2, sync, sij, sw, sout, total;
};

// Exchange words of the fused stage: per ghost and field, sizeof(T) / 4
// words of 8 bytes.
size_t xg_bytes(const Host &h) { return 3 * (size_t)(esize(h) / 4) * std::max<size_t>(h.gidx.size(), 1) * 8; }

Layout layout(const Host &h)
{
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t n) {
        size_t at = o;
        o = align256(o + n);
        return at;
    };
    const size_t es = esize(h);
    const size_t G = h.gidx.size(), nnz = h.cidx.size();
    L.inst = take(sizeof(DevInst));
    for (int k = 0; k < 9; ++k) L.planes[k] = take(plane_elems(h) * es);
    for (int k = 0; k < 3; ++k) L.psi[k] = take((size_t)h.ade_ns * std::max<size_t>(G, 1) * es);
    L.iv = take((size_t)h.d.ny * sizeof(int4));
    L.goff = take(std::max<size_t>(G, 1) * 4);
    L.cptr = take((G + 1) * 4);
    L.coff = take(std::max<size_t>(nnz, 1) * 4);
    L.w4 = take(4 * std::max<size_t>(nnz, 1) * es);
    L.gd = take(4 * std::max<size_t>(G, 1) * es);
    L.counters = take(2 * 8);
    L.pij = take(2 * std::max(h.np, 1) * 4);
    L.pw = take(16 * std::max(h.np, 1) * 8);
    L.pwork = take(std::max(h.np, 1) * sizeof(int2));
    L.trace = take(std::max<size_t>((size_t)h.trace_cap * h.np * 3, 1) * 8);
    L.dft = take(2 * std::max(h.np, 1) * 8);
    L.watch = take(3 * std::max<size_t>((size_t)h.watch_cap, 1) * 8);
    L.xg = take(xg_bytes(h));
    L.work1 = take(work1_capacity(h) * sizeof(int4));
    L.aux = take(work1_capacity(h) * sizeof(int2));
    L.patch = take(patch_capacity(h) * sizeof(int2));
    L.work2 = take(std::max<size_t>(G, 1) * sizeof(int4));
    L.sync = take(SYNC_INTS * sizeof(int));
    L.sij = take(2 * SAMPLE_MAX * 4);
    L.sw = take(16 * SAMPLE_MAX * 8);
    L.sout = take(3 * SAMPLE_MAX * 8);
    L.total = o;
    return L;
}

lee_status hip_fail(hipError_t e, const char *what)
{
    return fail(LEE_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #x); \
    } while (0)

// Slot order of the work list: the units (per_unit consecutive items) are cut
// into 8 contiguous runs of about equal cost, and workgroup b (which the
// hardware places on XCD b mod 8) takes unit b / 8 of run b mod 8.  Each XCD
// thus gets neighbouring tiles and shares their halos in its own L2, the XCD
// that holds the wall's tiles gets fewer of the others, and within a run the
// costlier units go first, so that none of them starts last and finishes
// after the rest of the launch.  Returns, per slot, the item index or -1 for
// an idle slot.  Every run is padded to ceil(total cost / (8 per_unit)) + 2
// units, a bound on the longest run, so the length depends on the multiset
// of items alone (a batch whose members change order keeps its list length).
std::vector<int> xcd_slots(const std::vector<int4> &items, int per_unit)
{
    const size_t n_items = items.size();
    const int units = (int)((n_items + per_unit - 1) / per_unit);
    std::vector<double> cost(units, 0.0);
    double total = 0.0;
    for (size_t k = 0; k < n_items; ++k) {
        const int x = items[k].x;
        const double c = (x >= 0 && (x & TILE_WALL_BIT)) ? WALL_ITEM_COST : 1;
        cost[k / per_unit] += c;
        total += c;
    }
    int start[9];
    start[0] = 0;
    int r = 1;
    double acc = 0.0;
    for (int u = 0; u < units && r < 8; ++u) {
        // cut before unit u once its midpoint lies past r / 8 of the total
        while (r < 8 && acc + 0.5 * cost[u] > total * r / 8.0) start[r++] = u;
        acc += cost[u];
    }
    while (r < 8) start[r++] = units;
    start[8] = units;
    // a run's units have midpoints within an eighth of the total and cost
    // per_unit at least (but the last), hence this bound
    int per = units ? (int)std::ceil(total / (8.0 * per_unit)) + 2 : 0;
    for (r = 0; r < 8; ++r) per = std::max(per, start[r + 1] - start[r]);
    std::vector<int> order(units);
    for (r = 0; r < 8; ++r) {
        int q = start[r];
        for (int u = start[r]; u < start[r + 1]; ++u)
            if (cost[u] > per_unit) order[q++] = u;
        for (int u = start[r]; u < start[r + 1]; ++u)
            if (cost[u] <= per_unit) order[q++] = u;
    }
    std::vector<int> out;
    for (int b = 0; b < 8 * per; ++b) {
        const int t = b / 8, run = b % 8;
        const int su = start[run] + t < start[run + 1] ? order[start[run] + t] : -1;
        for (int w = 0; w < per_unit; ++w) {
            const size_t k = (size_t)su * per_unit + w;
            out.push_back(su >= 0 && k < n_items ? (int)k : -1);
        }
    }
    return out;
}

// Sweep items in slot order, with each dependent tile's range of patch
// entries in aux (slot-aligned) and the entries themselves in patch.  In the
// fused form the first ncar workgroups carry the ghost fill, and dependent
// tiles wait for them, so no dependent tile may sit in a carrier slot: such
// tiles are swapped with the first later plain tile (or idle slot) of the
// same residue mod 8, which keeps them on their XCD.  If too few plain tiles
// exist, or when `dedicated` asks for it (batches: the first tile workgroup
// then depends on the ghost capacity alone and stays put across membership
// changes), the tiles start after ncar dedicated carrier workgroups instead.
// Returns the id of the first tile workgroup (0 or ncar rounded up to 8).
int order_work(const std::vector<int4> &items, const std::vector<std::vector<int2>> &patches, int per_unit,
               int ncar, bool dedicated, std::vector<int4> &out, std::vector<int2> &aux, std::vector<int2> &patch)
{
    out.clear();
    aux.clear();
    patch.clear();
    std::vector<int> slots = xcd_slots(items, per_unit);
    auto dep = [&](int k) { return k >= 0 && (items[k].x & TILE_DEP_BIT); };
    int tile0 = dedicated && ncar > 0 ? (ncar + 7) / 8 * 8 : 0;
    if (ncar > 0 && tile0 == 0) {
        int next[8];
        for (int r = 0; r < 8; ++r) next[r] = ncar + ((r - ncar % 8) + 8) % 8;   // first slot >= ncar of residue r
        for (int b = 0; b < std::min<int>(ncar, (int)slots.size()) && tile0 == 0; ++b) {
            if (!dep(slots[b])) continue;
            int &c = next[b % 8];
            while (c < (int)slots.size() && dep(slots[c])) c += 8;
            if (c >= (int)slots.size()) {
                tile0 = (ncar + 7) / 8 * 8;      // not enough plain tiles: dedicated carriers
                break;
            }
            std::swap(slots[b], slots[c]);
            c += 8;
        }
        if (tile0) slots = xcd_slots(items, per_unit);
    }
    for (int k : slots) {
        if (k < 0) {
            out.push_back(make_int4(-1, 0, 0, 1));
            aux.push_back(make_int2(0, 0));
            continue;
        }
        out.push_back(items[k]);
        const int p0 = (int)patch.size();
        if (k < (int)patches.size()) patch.insert(patch.end(), patches[k].begin(), patches[k].end());
        aux.push_back(make_int2(p0, (int)patch.size()));
    }
    return tile0;
}

// Workgroups that carry the ghost fill of a fused launch (8 ghosts each: 32
// lanes per ghost).
int carriers_for(const lee_tiling &t, size_t nwork2)
{
    return (t.kind == LEE_SWEEP_TILE && t.fused) ? (int)((nwork2 + 7) / 8) : 0;
}

bool tiling_valid(int prec, const lee_tiling &t)
{
    if (t.kind == LEE_SWEEP_TILE) return (t.fused == 0 || t.fused == 1) && tile_shape_supported(prec, t.cols, t.rows);
    if (t.kind == LEE_SWEEP_MARCH) {
        const bool f32 = prec == LEE_F32;
        if (!((f32 && (t.vec == 2 || t.vec == 4)) || (!f32 && t.vec == 2))) return false;
        return t.rows >= 4 && t.rows <= 4096 && (t.waves == 1 || t.waves == 2 || t.waves == 4);
    }
    return false;
}

// Built-in choice: the 2-D tile kernel with the shape measured fastest on
// MI355X at both 1024^2 and 4096^2 (64 columns; 16 rows FP32, 8 rows FP64),
// ghost fill and sweep in two launches.
lee_tiling default_tiling_for(int prec, int nx, int ny)
{
    (void)nx;
    (void)ny;
    lee_tiling t{};
    t.kind = LEE_SWEEP_TILE;
    t.cols = 64;
    t.vec = prec == LEE_F32 ? 4 : 2;
    t.waves = 1;
    t.rows = prec == LEE_F32 ? 16 : 8;
    t.fused = 0;                                 // measured: fused wins only for FP64 on small grids
    return t;
}

// The filter's form: 0 none, 1 the damping term of every stage's right-hand
// side, 2 once after every step (k_filter).
int filter_form(const Host &h) { return h.d.filter_sigma > 0.0 ? (h.d.filter_explicit ? 2 : 1) : 0; }

void default_tiling(lee_instance *I)
{
    I->tl = default_tiling_for(I->host.d.precision, I->host.d.nx, I->host.d.ny);
}

// Sweep work list of one instance: one item per (column block, row tile)
// holding fluid nodes, in natural order.  A march item covers 64 vec - 16
// output columns and alternates its direction between row tiles; a tile item
// covers `cols` columns.  For the fused tile sweep, patches (when given)
// receives per item the ghost nodes its stencils read, three entries per node
// (LDS element index in the tile's copy, ghost index * 3 + field), and items
// with any are flagged TILE_DEP_BIT.  The stencils of a tile read its own rows over the columns
// [c0 - 5, c0 + cols + 5) and the 5 rows above and below over [c0, c0 + cols).
// With the filter on, items whose stencils read a ghost node (in any launch
// form) are flagged TILE_WALL_BIT: only their nodes can sit closer than five
// nodes to the wall along an axis, where the filter row narrows.
void build_items(const Host &h, int inst_id, const lee_tiling &t, std::vector<int4> &items,
                 std::vector<std::vector<int2>> *patches)
{
    const int ow = t.kind == LEE_SWEEP_MARCH ? 64 * t.vec - 16 : t.cols;
    const int rows = t.rows;
    const int strips = (h.d.nx + ow - 1) / ow;
    const int tiles = (h.d.ny + rows - 1) / rows;
    const bool fused = t.kind == LEE_SWEEP_TILE && t.fused && patches;
    const bool walls = h.d.filter_sigma > 0.0 && !h.gidx.empty();
    // ghost columns by row (ascending: the ghost list is sorted by linear
    // index) and the ghost index of each
    std::vector<std::vector<int>> grow_cols, grow_g;
    if (fused || walls) {
        grow_cols.resize(h.d.ny);
        grow_g.resize(h.d.ny);
        for (size_t g = 0; g < h.gidx.size(); ++g) {
            grow_cols[h.gidx[g] / h.d.nx].push_back(h.gidx[g] % h.d.nx);
            grow_g[h.gidx[g] / h.d.nx].push_back((int)g);
        }
    }
    const int LW = ow + 16;
    // row ranges of the tiles: with the radiation band on, a tile row that
    // meets the band's top or bottom rows (wholly band nodes, computed by the
    // band pass, one item per node and field) is cut into one-row tiles there
    // and one tile for the rest, so that no edge tile works through a chain of
    // band rows while the other tiles of its launch have finished
    const int rw = h.d.radiation ? h.d.stencil_half : 0;
    std::vector<std::array<int, 3>> ranges;      // r0, r1, tile row
    for (int r = 0; r < tiles; ++r) {
        const int r0 = r * rows, r1 = std::min(r0 + rows, h.d.ny);
        const int b0 = std::min(std::max(r0, rw), r1);            // [r0, b0): top band rows
        const int b1 = std::max(std::min(r1, h.d.ny - rw), b0);   // [b1, r1): bottom band rows
        if (rw == 0 || (b0 == r0 && b1 == r1)) {
            ranges.push_back({r0, r1, r});
            continue;
        }
        for (int j = r0; j < b0; ++j) ranges.push_back({j, j + 1, r});
        if (b0 < b1) ranges.push_back({b0, b1, r});
        for (int j = b1; j < r1; ++j) ranges.push_back({j, j + 1, r});
    }
    for (const auto &rg : ranges) {
        const int r0 = rg[0], r1 = rg[1], r = rg[2];
        for (int s = 0; s < strips; ++s) {
            const int c0 = s * ow, c1 = std::min(c0 + ow, h.d.nx);
            bool any = false;
            for (int j = r0; j < r1 && !any; ++j) {
                const int *iv = &h.iv[(size_t)j * 4];
                for (int q = 0; q < 2; ++q)
                    if (iv[2 * q] < iv[2 * q + 1] && iv[2 * q] < c1 && iv[2 * q + 1] > c0) any = true;
            }
            if (!any) continue;
            std::vector<int2> pl;
            bool wall = false;
            if (fused || walls) {
                for (int j = std::max(0, r0 - 5); j < std::min(h.d.ny, r1 + 5); ++j) {
                    const bool own = j >= r0 && j < r1;
                    const int lo = own ? c0 - 5 : c0, hi = own ? c0 + ow + 5 : c0 + ow;
                    const std::vector<int> &gc = grow_cols[j];
                    for (auto it = std::lower_bound(gc.begin(), gc.end(), lo); it != gc.end() && *it < hi; ++it) {
                        wall = walls;
                        if (!fused) break;
                        const int g = grow_g[j][it - gc.begin()];
                        for (int f = 0; f < 3; ++f)
                            pl.push_back(make_int2((j - (r0 - 5)) * LW + (*it - (c0 - 8)), 3 * g + f));
                    }
                }
            }
            const int flag = (pl.empty() ? 0 : TILE_DEP_BIT) | (wall ? TILE_WALL_BIT : 0);
            items.push_back(make_int4(inst_id | flag, c0, r0, (r & 1) ? -r1 : r1));
            if (patches) patches->push_back(std::move(pl));
        }
    }
}

int per_unit_of(const lee_tiling &t) { return t.kind == LEE_SWEEP_MARCH ? t.waves : 1; }

lee_status upload_work1(lee_instance *I)
{
    std::vector<int4> items;
    std::vector<std::vector<int2>> patches;
    build_items(I->host, 0, I->tl, items, &patches);
    I->tile0 = order_work(items, patches, per_unit_of(I->tl), carriers_for(I->tl, I->host.gidx.size()), false,
                          I->up_work1, I->up_aux, I->up_patch);
    if (I->up_work1.size() > I->work1_cap) return fail(LEE_E_ARG, "tiling produces too many work items");
    if (I->up_patch.size() > I->patch_cap) return fail(LEE_E_ARG, "tiling produces too many ghost patches");
    I->nwork1 = (int)I->up_work1.size();
    HIPCHK(hipMemcpyAsync(I->d_work1, I->up_work1.data(), I->up_work1.size() * sizeof(int4),
                          hipMemcpyHostToDevice, I->stream));
    HIPCHK(hipMemcpyAsync(I->d_aux, I->up_aux.data(), I->up_aux.size() * sizeof(int2), hipMemcpyHostToDevice,
                          I->stream));
    if (!I->up_patch.empty())
        HIPCHK(hipMemcpyAsync(I->d_patch, I->up_patch.data(), I->up_patch.size() * sizeof(int2),
                              hipMemcpyHostToDevice, I->stream));
    return LEE_OK;
}

void drop_graph(lee_instance *I) { I->graphs.drop(); }

// n steps on stream s through the captured graphs (or eagerly); issue_run(k)
// enqueues one run of k steps (the launches of each step, then the run's
// tail, which samples the probes after the last step and advances the step
// counters).  Graphs hold runs of G.per steps and one run of the remainder
// n mod G.per, kept for the next call of the same remainder (with G.per = 1,
// one-step graphs).
lee_status run_steps(StepGraphs &G, hipStream_t s, int64_t n, const std::function<hipError_t(int)> &issue_run)
{
    if (s == nullptr || G.per == 0) {            // the legacy default stream cannot be captured
        for (int64_t k = 0; k < n; k += 1 << 20) HIPCHK(issue_run((int)std::min<int64_t>(n - k, 1 << 20)));
        return LEE_OK;
    }
    auto capture = [&](int steps, hipGraph_t &g, hipGraphExec_t &ex) -> lee_status {
        HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = issue_run(steps);
        hipGraph_t cg = nullptr;
        hipError_t e2 = hipStreamEndCapture(s, &cg);
        if (e != hipSuccess) {
            if (cg) hipGraphDestroy(cg);
            return hip_fail(e, "capturing steps");
        }
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
        g = cg;
        HIPCHK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
        ++G.captures;
        return LEE_OK;
    };
    const int64_t full = G.per > 1 ? n / G.per : 0;
    const int64_t rest = n - full * G.per;
    const int rlen = G.per > 1 ? (int)rest : 1;
    const int64_t rlaunch = G.per > 1 ? (rest > 0 ? 1 : 0) : rest;
    if (full > 0 && !G.em) {
        lee_status st = capture(G.per, G.gm, G.em);
        if (st != LEE_OK) return st;
    }
    if (rlaunch > 0 && (!G.e1 || G.rest_len != rlen)) {
        G.drop_rest();
        lee_status st = capture(rlen, G.g1, G.e1);
        if (st != LEE_OK) return st;
        G.rest_len = rlen;
    }
    for (int64_t k = 0; k < full; ++k) HIPCHK(hipGraphLaunch(G.em, s));
    for (int64_t k = 0; k < rlaunch; ++k) HIPCHK(hipGraphLaunch(G.e1, s));
    return LEE_OK;
}

int graph_steps_from(int32_t v) { return v == 0 ? GRAPH_STEPS_DEFAULT : (v < 0 ? 0 : v); }

hipError_t sweep(int prec, bool filt, const lee_tiling &t, const DevInst *insts, const int4 *work, int nwork,
                 int stage, int slot, int blocks, hipStream_t s)
{
    if (t.kind == LEE_SWEEP_TILE)
        return launch_tile(prec, filt, t.cols, t.rows, insts, work, nwork, stage, slot, blocks, s);
    return launch_sweep(prec, t.vec, filt, t.waves, insts, work, nwork, stage, slot, blocks, s);
}

bool fused(const lee_tiling &t) { return t.kind == LEE_SWEEP_TILE && t.fused; }

// The ghost fill and sweep of one stage: one fused launch, or two launches.
// Events, when given, bracket the ghost launch (g0, g1) and the sweep or
// fused launch (s0, s1).
hipError_t stage_launches(int prec, bool filt, const lee_tiling &t, const DevInst *insts, int ninst, bool poles,
                          const int4 *work1, int nwork1, const int2 *aux, const int2 *patch, int tile0,
                          const int4 *work2, int nwork2, int *sync, int stage, int slot, ProbePass pp, int blocks,
                          hipStream_t s, hipEvent_t *ev = nullptr, int spin = SPIN_LIMIT)
{
    hipError_t e = hipSuccess;
    if (ev) hipEventRecord(ev[0], s);
    if (!fused(t)) e = launch_ghost(prec, insts, ninst, poles, work2, nwork2, stage, slot, pp, s);
    if (ev) {
        hipEventRecord(ev[1], s);
        hipEventRecord(ev[2], s);
    }
    if (e != hipSuccess) return e;
    if (fused(t))
        e = launch_stage(prec, filt, t.cols, t.rows, insts, ninst, poles, work1, nwork1, aux, patch, tile0, work2,
                         nwork2, stage, slot, sync, spin, pp, s);
    else
        e = sweep(prec, filt, t, insts, work1, nwork1, stage, slot, blocks, s);
    if (ev) hipEventRecord(ev[3], s);
    return e;
}

// The probe pass a stage launch carries: in the second stage of every step
// of a run but the first, the probes after the previous step (buffer 0 holds
// its result through the first three stages).
ProbePass probe_pass(const int2 *pw, int np, int stage, int slot)
{
    if (stage == 1 && slot >= 1) return ProbePass{pw, np, slot - 1};
    return ProbePass{pw, 0, 0};
}

// Stage `stage` of step `slot` of the current run.
hipError_t issue_stage(lee_instance *I, int stage, int slot)
{
    const int prec = I->host.d.precision;
    return stage_launches(prec, filter_form(I->host) == 1, I->tl, I->d_inst, 1, I->host.ade_kind == 3,
                          I->d_work1, I->nwork1, I->d_aux,
                          I->d_patch, I->tile0, I->d_work2, I->nwork2, I->d_sync, stage, slot,
                          probe_pass(I->d_pwork, I->host.np, stage, slot), 0, I->stream, nullptr, I->spin);
}

// The tail of a run of n steps: the probes after its last step, then the
// step counter.
hipError_t issue_tail(lee_instance *I, int n)
{
    hipError_t e = launch_probe(I->host.d.precision, I->d_inst, ProbePass{I->d_pwork, I->host.np, n - 1}, I->stream);
    if (e == hipSuccess) e = launch_advance(I->d_inst, 1, n, I->stream);
    return e;
}

// The explicit filter after step `slot` of the run (its form only).
hipError_t issue_filter(lee_instance *I, int slot)
{
    if (filter_form(I->host) != 2) return hipSuccess;
    return launch_filter(I->host.d.precision, I->tl.cols, I->tl.rows, I->d_inst, I->d_work1, I->nwork1, slot,
                         I->stream);
}

hipError_t issue_run(lee_instance *I, int n)
{
    hipError_t e = hipSuccess;
    for (int j = 0; j < n && e == hipSuccess; ++j) {
        for (int l = 0; l < 4 && e == hipSuccess; ++l) e = issue_stage(I, l, j);
        if (e == hipSuccess) e = issue_filter(I, j);
    }
    if (e == hipSuccess) e = issue_tail(I, n);
    return e;
}

// Times each run (a sequence of asynchronous launches) with one pair of
// events on stream s; out[k] receives run k's duration in microseconds.
lee_status time_runs(hipStream_t s, std::initializer_list<std::function<hipError_t()>> runs, double *out)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    int k = 0;
    for (auto it = runs.begin(); it != runs.end() && e == hipSuccess; ++it, ++k) {
        e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = (*it)();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        out[k] = 1000.0 * ms;
    }
    hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "timing run");
    return LEE_OK;
}

// Waits for the stream and reports a fused stage whose ghost wait ran out.
lee_status check_sync(const int *d_sync, hipStream_t s)
{
    int flag = 0;
    HIPCHK(hipMemcpyAsync(&flag, d_sync + 4, sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (flag) return fail(LEE_E_DEVICE, "a fused stage stopped waiting for its ghost fill (spin limit)");
    return LEE_OK;
}

template <typename T>
void pack_lists(lee_instance *I)
{
    const Host &h = I->host;
    const int pitch = pitch_of(h);
    const size_t G = h.gidx.size(), nnz = h.cidx.size();
    I->up_w4.assign(4 * nnz * sizeof(T), 0);
    T *w = (T *)I->up_w4.data();
    for (size_t k = 0; k < 4 * nnz; ++k) w[k] = (T)h.w4[k];
    I->up_gd.assign(4 * G * sizeof(T), 0);
    T *gd = (T *)I->up_gd.data();
    for (size_t g = 0; g < G; ++g) {
        gd[4 * g + 0] = (T)h.gnx[g];
        gd[4 * g + 1] = (T)h.gny[g];
        gd[4 * g + 2] = (T)h.beta[2 * g];
        gd[4 * g + 3] = (T)h.beta[2 * g + 1];
    }
    const int org = FRAME * pitch + LPAD;
    I->up_goff.resize(G);
    for (size_t g = 0; g < G; ++g) I->up_goff[g] = org + (h.gidx[g] / h.d.nx) * pitch + h.gidx[g] % h.d.nx;
    I->up_coff.resize(nnz);
    for (size_t e = 0; e < nnz; ++e) I->up_coff[e] = org + (h.cidx[e] / h.d.nx) * pitch + h.cidx[e] % h.d.nx;
}

}  // namespace

extern "C" {

lee_status lee_setup_grid(const lee_case_desc *d, lee_instance **out)
{
    if (!out) return fail(LEE_E_ARG, "null output pointer");
    *out = nullptr;
    lee_instance *I = new (std::nothrow) lee_instance();
    if (!I) return fail(LEE_E_NOMEM, "host allocation");
    lee_status s = host_setup(d, &I->host);
    if (s != LEE_OK) {
        delete I;
        return s;
    }
    default_tiling(I);
    *out = I;
    return LEE_OK;
}

lee_status lee_build_ghosts(lee_instance *I, const lee_impedance *z, int32_t degree, lee_ghost_summary *out)
{
    if (!I) return fail(LEE_E_ARG, "null instance");
    if (I->bound) return fail(LEE_E_STATE, "lee_build_ghosts after lee_bind");
    return host_build(&I->host, z, degree, out);
}

lee_status lee_set_probes(lee_instance *I, int32_t np, const double *xy, int64_t capacity, double dft_omega,
                          int64_t dft_start, int64_t dft_count)
{
    if (!I) return fail(LEE_E_ARG, "null instance");
    if (I->bound) return fail(LEE_E_STATE, "lee_set_probes after lee_bind");
    if (np < 0 || (np > 0 && !xy) || capacity < 0 || dft_count < 0 || dft_start < 0)
        return fail(LEE_E_ARG, "probe arguments");
    Host &h = I->host;
    h.probe_ij.assign(2 * (size_t)np, 0);
    h.probe_w.assign(16 * (size_t)np, 0.0);
    for (int k = 0; k < np; ++k) {
        lee_status s = host_probe_stencil(&h, xy[2 * k], xy[2 * k + 1], &h.probe_ij[2 * k], &h.probe_ij[2 * k + 1],
                                          &h.probe_w[16 * k]);
        if (s != LEE_OK) return s;
    }
    h.np = np;
    h.trace_cap = np > 0 ? capacity : 0;
    h.dft_omega = dft_omega;
    h.dft_start = dft_start;
    h.dft_count = np > 0 ? dft_count : 0;
    return LEE_OK;
}

lee_status lee_set_watch(lee_instance *I, double x, double y, int64_t capacity, int32_t *ghost)
{
    if (!I) return fail(LEE_E_ARG, "null instance");
    if (I->bound) return fail(LEE_E_STATE, "lee_set_watch after lee_bind");
    Host &h = I->host;
    if (!h.built) return fail(LEE_E_STATE, "lee_build_ghosts first");
    if (h.gidx.empty()) return fail(LEE_E_ARG, "no ghost points to watch");
    if (capacity < 0) return fail(LEE_E_ARG, "negative capacity");
    int best = 0;
    double bd = 0.0;
    for (int g = 0; g < (int)h.gidx.size(); ++g) {
        const double dx = h.bx[g] - x, dy = h.by[g] - y;
        const double d2 = dx * dx + dy * dy;
        if (g == 0 || d2 < bd) {
            best = g;
            bd = d2;
        }
    }
    h.watch_g = capacity > 0 ? best : -1;
    h.watch_cap = capacity;
    if (ghost) *ghost = best;
    return LEE_OK;
}

lee_status lee_watch_traces(lee_instance *I, double *out, int64_t cap, int64_t *n)
{
    if (!I || !I->bound || !n) return fail(LEE_E_ARG, "instance not bound or null argument");
    const Host &h = I->host;
    *n = 0;
    if (h.watch_g < 0 || h.watch_cap == 0) return LEE_OK;
    long long done = 0;
    HIPCHK(hipMemcpyAsync(&done, I->dev.step, 8, hipMemcpyDeviceToHost, I->stream));
    std::vector<double> ring(3 * (size_t)h.watch_cap);
    HIPCHK(hipMemcpyAsync(ring.data(), I->dev.watch, ring.size() * 8, hipMemcpyDeviceToHost, I->stream));
    HIPCHK(hipStreamSynchronize(I->stream));
    int64_t m = std::min<int64_t>({(int64_t)done, (int64_t)h.watch_cap, cap});
    if (m > 0 && !out) return fail(LEE_E_ARG, "null output");
    const int64_t first = done - m;
    for (int64_t s = 0; s < m; ++s) {
        const size_t r = (size_t)((first + s) % h.watch_cap);
        for (int k = 0; k < 3; ++k) out[3 * s + k] = ring[3 * r + k];
    }
    *n = m;
    return LEE_OK;
}

lee_status lee_required_bytes(const lee_instance *I, size_t *dev_bytes)
{
    if (!I || !dev_bytes) return fail(LEE_E_ARG, "null argument");
    if (!I->host.built) return fail(LEE_E_STATE, "lee_build_ghosts first");
    *dev_bytes = layout(I->host).total;
    return LEE_OK;
}

lee_status lee_bind(lee_instance *I, void *dev_ptr, size_t bytes, void *hip_stream)
{
    if (!I || !dev_ptr) return fail(LEE_E_ARG, "null argument");
    if (I->bound) return fail(LEE_E_STATE, "already bound");
    if (!I->host.built) return fail(LEE_E_STATE, "lee_build_ghosts first");
    if (((uintptr_t)dev_ptr & 255) != 0) return fail(LEE_E_ARG, "device buffer must be 256-byte aligned");
    const Host &h = I->host;
    const Layout L = layout(h);
    if (bytes < L.total) return fail(LEE_E_NOMEM, "device buffer smaller than lee_required_bytes");
    HIPCHK(hipGetDevice(&I->device));
    I->stream = (hipStream_t)hip_stream;
    I->base = (char *)dev_ptr;
    I->bytes = bytes;
    char *b = I->base;
    const int pitch = pitch_of(h);
    const size_t es = esize(h);
    DevInst &D = I->dev;
    std::memset(&D, 0, sizeof(D));
    for (int r = 0; r < 3; ++r)
        for (int f = 0; f < 3; ++f) D.f[r][f] = b + L.planes[3 * r + f];
    D.org = FRAME * pitch + LPAD;
    for (int r = 0; r < 3; ++r) D.psi[r] = b + L.psi[r];
    D.iv = (const int4 *)(b + L.iv);
    D.goff = (const int *)(b + L.goff);
    D.cptr = (const int *)(b + L.cptr);
    D.coff = (const int *)(b + L.coff);
    D.w4 = b + L.w4;
    D.gd = b + L.gd;
    D.step = (long long *)(b + L.counters);
    D.stop = D.step + 1;
    D.pij = (const int *)(b + L.pij);
    D.pw = (const double *)(b + L.pw);
    D.trace = (double *)(b + L.trace);
    D.watch = (double *)(b + L.watch);
    D.xg = (unsigned long long *)(b + L.xg);
    D.watch_cap = h.watch_cap;
    D.watch_g = h.watch_g;
    D.dft = (double *)(b + L.dft);
    D.trace_cap = h.trace_cap;
    D.dft_start = h.dft_start;
    D.dft_count = h.dft_count;
    D.dft_omega = h.dft_omega;
    D.np = h.np;
    D.nx = h.d.nx;
    D.ny = h.d.ny;
    D.pitch = pitch;
    D.G = (int)h.gidx.size();
    D.x0 = h.d.x0;
    D.y0 = h.d.y0;
    D.h = h.d.h;
    D.dt = h.dt;
    static const double A5[5] = {0.872756993962, -0.286511173973, 0.090320001280, -0.020779405824, 0.002484594688};
    static const double A3[3] = {0.770882380518, -0.166705904415, 0.020843142770};
    static const double FD[6] = {0.215044884112, -0.187772883589, 0.123755948787, -0.059227575576, 0.018721609157,
                                 -0.002999540835};
    for (int k = 0; k < 5; ++k) {
        const double a = h.d.stencil_half == 5 ? A5[k] : (k < 3 ? A3[k] : 0.0);
        D.ax[k] = a / h.d.h;
    }
    // the damping term carries sigma_d / dt; the explicit form, applied once
    // per step, sigma_d itself
    const double sd = h.d.filter_explicit ? h.d.filter_sigma : h.d.filter_sigma / h.dt;
    D.fd[0] = sd * 2.0 * FD[0];
    for (int k = 1; k < 6; ++k) D.fd[k] = sd * FD[k];
    for (int k = 0; k < 5; ++k) D.axf[k] = (float)D.ax[k];
    for (int k = 0; k < 6; ++k) D.fdf[k] = (float)D.fd[k];
    // near an immersed wall an axis of half-width w < 5 takes the standard
    // centred filter of that half-width, whose damping function is
    // ((1 - cos k) / 2)^w: its row is the w-fold convolution of the
    // three-point row (-1/4, 1/2, -1/4); none for w = 0
    for (int w = 0; w < 5; ++w) {
        double row[11] = {0};                    // offsets -5..5
        if (w > 0) {
            row[5] = 1.0;
            for (int c = 0; c < w; ++c) {
                double nxt[11] = {0};
                for (int k = 1; k < 10; ++k) nxt[k] = 0.5 * row[k] - 0.25 * (row[k - 1] + row[k + 1]);
                std::memcpy(row, nxt, sizeof(row));
            }
        }
        for (int j = 0; j < 6; ++j) D.fdw[w][j] = sd * (row[5 + j] - FD[j]);
    }
    for (int w = 0; w < 6; ++w)
        for (int j = 0; j < 6; ++j) D.fdwf[w][j] = (float)D.fdw[w][j];
    static const double ALPHA[4] = {0.25, 1.0 / 3.0, 0.5, 1.0};
    static const double CST[4] = {0.0, 0.25, 1.0 / 3.0, 0.5};
    for (int l = 0; l < 4; ++l) {
        D.alpha_dt[l] = ALPHA[l] * h.dt;
        D.c_stage[l] = CST[l];
    }
    D.rad_w = h.d.radiation ? h.d.stencil_half : 0;
    D.fx = filter_form(h) == 2 ? 1 : 0;
    // stage outputs bypass the caches when the field planes cannot stay in
    // the 256 MB on-chip cache anyway (half of it, leaving room for the rest)
    D.stream = 9 * plane_elems(h) * esize(h) > STREAM_STORE_BYTES ? 1 : 0;
    D.stream_in = stream_in_for(9 * plane_elems(h) * esize(h), 3 * plane_elems(h) * esize(h));
    D.rad_xc = h.d.rad_xc;
    D.rad_yc = h.d.rad_yc;
    // window weights: place 3 the central 7-node set (-a3, -a2, -a1, 0, a1,
    // a2, a3); any other place m the derivative at node m of the Lagrange basis
    // on nodes 0..6, l_k'(m) = prod_{q != k, m} (m - q) / prod_{q != k} (k - q)
    // for k != m and l_m'(m) = sum_{q != m} 1 / (m - q)
    for (int m = 0; m < 7; ++m)
        for (int k = 0; k < 7; ++k) {
            double v = 0.0;
            if (m == 3) {
                v = k == 3 ? 0.0 : (k > 3 ? A3[k - 4] : -A3[2 - k]);
            } else if (k == m) {
                for (int q = 0; q < 7; ++q)
                    if (q != m) v += 1.0 / (m - q);
            } else {
                double num = 1.0, den = 1.0;
                for (int q = 0; q < 7; ++q) {
                    if (q != k) den *= (k - q);
                    if (q != k && q != m) num *= (m - q);
                }
                v = num / den;
            }
            D.rad_w7[m][k] = v / h.d.h;
            D.rad_wf[m][k] = (float)D.rad_w7[m][k];
        }
    D.sponge_w = h.d.sponge_cells;
    D.sponge_s = h.d.sponge_sigma;
    D.sponge_inv = h.d.sponge_cells > 0 ? 1.0 / h.d.sponge_cells : 0.0;
    D.has_src = h.d.src_kind == LEE_SRC_MONOPOLE ? 1 : 0;
    if (D.has_src) {
        const double xs = h.d.src[0], ys = h.d.src[1], w = h.d.src[3];
        D.src_a = h.d.src[2];
        D.src_b = 0.6931471805599453 / (w * w);
        D.src_om = h.d.src[4];
        D.src_ic = (int)std::lround((xs - h.d.x0) / h.d.h);
        D.src_jc = (int)std::lround((ys - h.d.y0) / h.d.h);
        D.src_fx = xs - (h.d.x0 + D.src_ic * h.d.h);
        D.src_fy = ys - (h.d.y0 + D.src_jc * h.d.h);
        // exp(-b r^2) < 1e-45 beyond r^2 > 104 / b
        const int rad = (int)std::ceil(std::sqrt(104.0 / D.src_b) / h.d.h) + 1;
        D.src_i0 = D.src_ic - rad;
        D.src_i1 = D.src_ic + rad;
        D.src_j0 = D.src_jc - rad;
        D.src_j1 = D.src_jc + rad;
    }
    D.ade_kind = h.ade_kind;
    for (int k = 0; k < 4; ++k) D.ade[k] = h.ade[k];
    D.ade_ns = h.ade_ns;
    std::memcpy(D.ade_st, h.ade_st, sizeof(D.ade_st));

    // uploads
    if (h.d.precision == LEE_F32)
        pack_lists<float>(I);
    else
        pack_lists<double>(I);
    I->up_iv.resize(h.d.ny);
    for (int j = 0; j < h.d.ny; ++j)
        I->up_iv[j] = make_int4(h.iv[4 * j], h.iv[4 * j + 1], h.iv[4 * j + 2], h.iv[4 * j + 3]);
    const size_t G = h.gidx.size(), nnz = h.cidx.size();
    hipStream_t s = I->stream;
    HIPCHK(hipMemcpyAsync((void *)D.iv, I->up_iv.data(), h.d.ny * sizeof(int4), hipMemcpyHostToDevice, s));
    if (G) {
        HIPCHK(hipMemcpyAsync((void *)D.goff, I->up_goff.data(), G * 4, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync((void *)D.cptr, h.cptr.data(), (G + 1) * 4, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync((void *)D.gd, I->up_gd.data(), I->up_gd.size(), hipMemcpyHostToDevice, s));
    }
    if (nnz) {
        HIPCHK(hipMemcpyAsync((void *)D.coff, I->up_coff.data(), nnz * 4, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync((void *)D.w4, I->up_w4.data(), I->up_w4.size(), hipMemcpyHostToDevice, s));
    }
    I->d_pwork = (int2 *)(b + L.pwork);
    I->up_pwork.resize(h.np);
    for (int k = 0; k < h.np; ++k) I->up_pwork[k] = make_int2(0, k);
    if (h.np) {
        HIPCHK(hipMemcpyAsync((void *)D.pij, h.probe_ij.data(), 2 * h.np * 4, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync((void *)D.pw, h.probe_w.data(), 16 * h.np * 8, hipMemcpyHostToDevice, s));
        HIPCHK(hipMemcpyAsync(I->d_pwork, I->up_pwork.data(), h.np * sizeof(int2), hipMemcpyHostToDevice, s));
    }
    I->d_inst = (DevInst *)(b + L.inst);
    HIPCHK(hipMemcpyAsync(I->d_inst, &I->dev, sizeof(DevInst), hipMemcpyHostToDevice, s));
    I->d_work1 = (int4 *)(b + L.work1);
    I->work1_cap = work1_capacity(h);
    I->d_aux = (int2 *)(b + L.aux);
    I->d_patch = (int2 *)(b + L.patch);
    I->patch_cap = patch_capacity(h);
    I->d_work2 = (int4 *)(b + L.work2);
    I->up_work2.resize(G);
    for (size_t g = 0; g < G; ++g) I->up_work2[g] = make_int4(0, (int)g, h.cptr[g], h.cptr[g + 1]);
    I->nwork2 = (int)G;
    if (G) HIPCHK(hipMemcpyAsync(I->d_work2, I->up_work2.data(), G * sizeof(int4), hipMemcpyHostToDevice, s));
    I->d_sync = (int *)(b + L.sync);
    I->d_sij = (int *)(b + L.sij);
    I->d_sw = (double *)(b + L.sw);
    I->d_sout = (double *)(b + L.sout);
    lee_status st = upload_work1(I);
    if (st != LEE_OK) return st;
    I->bound = true;
    return lee_init_fields(I);
}

lee_status lee_init_fields(lee_instance *I)
{
    if (!I || !I->bound) return fail(LEE_E_STATE, "instance not bound");
    const Host &h = I->host;
    const Layout L = layout(h);
    hipStream_t s = I->stream;
    const int prec = h.d.precision;
    for (int k = 0; k < 9; ++k) HIPCHK(launch_fill(prec, I->base + L.planes[k], plane_elems(h), s));
    for (int k = 0; k < 3; ++k)
        HIPCHK(launch_fill(prec, I->base + L.psi[k], (size_t)h.ade_ns * std::max<size_t>(h.gidx.size(), 1), s));
    HIPCHK(launch_fill_bytes(I->base + L.trace, std::max<size_t>((size_t)h.trace_cap * h.np * 3, 1) * 8, s));
    HIPCHK(launch_fill_bytes(I->base + L.dft, 2 * std::max(h.np, 1) * 8, s));
    HIPCHK(launch_fill_bytes(I->base + L.watch, 3 * std::max<size_t>((size_t)h.watch_cap, 1) * 8, s));
    HIPCHK(launch_fill_bytes(I->base + L.xg, xg_bytes(h), s));
    HIPCHK(launch_fill_bytes(I->base + L.sync, SYNC_INTS * sizeof(int), s));
    I->up_counters[0] = 0;                       // first step of the next run
    I->up_counters[1] = LLONG_MAX;               // no stop
    HIPCHK(hipMemcpyAsync(I->dev.step, I->up_counters, sizeof(I->up_counters), hipMemcpyHostToDevice, s));
    HIPCHK(launch_init_ic(prec, I->d_inst, h.d.nx, h.d.ny, h.d.ic_kind, h.d.ic, s));
    I->next_stage = 0;
    I->steps_issued = 0;
    return LEE_OK;
}

lee_status lee_rk_stage(lee_instance *I, int32_t stage)
{
    if (!I || !I->bound) return fail(LEE_E_STATE, "instance not bound");
    if (stage < 0 || stage > 3) return fail(LEE_E_ARG, "stage must be 0..3");
    if (stage != I->next_stage) return fail(LEE_E_STATE, "stages must be issued in order 0, 1, 2, 3");
    HIPCHK(issue_stage(I, stage, 0));
    if (stage == 3) HIPCHK(issue_filter(I, 0));
    if (stage == 3) HIPCHK(issue_tail(I, 1));
    I->next_stage = (stage + 1) & 3;
    if (stage == 3) ++I->steps_issued;
    return LEE_OK;
}

lee_status lee_step_n(lee_instance *I, int64_t n)
{
    if (!I || !I->bound) return fail(LEE_E_STATE, "instance not bound");
    if (n < 0) return fail(LEE_E_ARG, "n < 0");
    if (I->next_stage != 0) return fail(LEE_E_STATE, "a partial step is pending");
    if (n == 0) return LEE_OK;
    lee_status st = run_steps(I->graphs, I->stream, n, [I](int k) { return issue_run(I, k); });
    if (st != LEE_OK) return st;
    I->steps_issued += n;
    return LEE_OK;
}

lee_status lee_set_graph_steps(lee_instance *I, int32_t steps)
{
    if (!I) return fail(LEE_E_ARG, "null instance");
    if (steps > GRAPH_STEPS_MAX) return fail(LEE_E_ARG, "too many steps per graph");
    drop_graph(I);
    I->graphs.per = graph_steps_from(steps);
    return LEE_OK;
}

lee_status lee_set_ghost_wait(lee_instance *I, int32_t polls)
{
    if (!I) return fail(LEE_E_ARG, "null instance");
    drop_graph(I);
    I->spin = polls == 0 ? SPIN_LIMIT : polls;
    return LEE_OK;
}

lee_status lee_set_tiling(lee_instance *I, const lee_tiling *t)
{
    if (!I || !t) return fail(LEE_E_ARG, "null argument");
    if (!tiling_valid(I->host.d.precision, *t)) return fail(LEE_E_ARG, "unsupported tiling");
    if (t->kind == LEE_SWEEP_MARCH && I->host.d.radiation)
        return fail(LEE_E_ARG, "the march sweep has no radiation band; use a tile sweep");
    if (t->kind == LEE_SWEEP_MARCH && filter_form(I->host) == 2)
        return fail(LEE_E_ARG, "the explicit filter runs on the tile sweep's items; use a tile sweep");
    if (I->next_stage != 0) return fail(LEE_E_STATE, "a partial step is pending");
    I->tl = *t;
    drop_graph(I);
    if (I->bound) return upload_work1(I);
    return LEE_OK;
}

lee_status lee_get_tiling(const lee_instance *I, lee_tiling *t)
{
    if (!I || !t) return fail(LEE_E_ARG, "null argument");
    *t = I->tl;
    return LEE_OK;
}

lee_status lee_get_step(const lee_instance *I, int64_t *step)
{
    if (!I || !step) return fail(LEE_E_ARG, "null argument");
    *step = I->steps_issued;
    if (!I->bound) return LEE_OK;
    lee_status st = check_sync(I->d_sync, I->stream);  // also waits for the stream
    if (st != LEE_OK) return st;
    long long done = 0;                                // budgets may have idled a batch member
    HIPCHK(hipMemcpy(&done, I->dev.step, 8, hipMemcpyDeviceToHost));
    *step = done;
    return LEE_OK;
}

lee_status lee_synchronize(lee_instance *I)
{
    if (!I || !I->bound) return fail(LEE_E_STATE, "instance not bound");
    return check_sync(I->d_sync, I->stream);
}

}  // extern "C"

namespace {

template <typename T>
lee_status copy_plane_out(lee_instance *I, int reg, int f, double *out)
{
    const Host &h = I->host;
    std::vector<T> tmp((size_t)h.d.nx * h.d.ny);
    HIPCHK(hipMemcpy2DAsync(tmp.data(), h.d.nx * sizeof(T), (T *)I->dev.f[reg][f] + I->dev.org, pitch_of(h) * sizeof(T),
                            h.d.nx * sizeof(T), h.d.ny, hipMemcpyDeviceToHost, I->stream));
    HIPCHK(hipStreamSynchronize(I->stream));
    for (size_t k = 0; k < tmp.size(); ++k) out[k] = (double)tmp[k];
    return LEE_OK;
}

template <typename T>
lee_status copy_plane_in(lee_instance *I, int f, const double *in)
{
    const Host &h = I->host;
    std::vector<T> tmp((size_t)h.d.nx * h.d.ny);
    for (size_t k = 0; k < tmp.size(); ++k) tmp[k] = h.fluid[k] ? (T)in[k] : (T)0;
    HIPCHK(hipMemcpy2DAsync((T *)I->dev.f[0][f] + I->dev.org, pitch_of(h) * sizeof(T), tmp.data(), h.d.nx * sizeof(T),
                            h.d.nx * sizeof(T), h.d.ny, hipMemcpyHostToDevice, I->stream));
    HIPCHK(hipStreamSynchronize(I->stream));
    return LEE_OK;
}

}  // namespace

extern "C" {

lee_status lee_get_fields(lee_instance *I, double *p, double *u, double *v)
{
    if (!I || !I->bound) return fail(LEE_E_STATE, "instance not bound");
    if (I->next_stage != 0) return fail(LEE_E_STATE, "a partial step is pending");
    double *o[3] = {p, u, v};
    for (int f = 0; f < 3; ++f) {
        if (!o[f]) continue;
        lee_status s = I->host.d.precision == LEE_F32 ? copy_plane_out<float>(I, 0, f, o[f])
                                                      : copy_plane_out<double>(I, 0, f, o[f]);
        if (s != LEE_OK) return s;
    }
    return check_sync(I->d_sync, I->stream);
}

lee_status lee_set_fields(lee_instance *I, const double *p, const double *u, const double *v)
{
    if (!I || !I->bound) return fail(LEE_E_STATE, "instance not bound");
    if (I->next_stage != 0) return fail(LEE_E_STATE, "a partial step is pending");
    const double *in[3] = {p, u, v};
    for (int f = 0; f < 3; ++f) {
        if (!in[f]) continue;
        lee_status s = I->host.d.precision == LEE_F32 ? copy_plane_in<float>(I, f, in[f])
                                                      : copy_plane_in<double>(I, f, in[f]);
        if (s != LEE_OK) return s;
    }
    return LEE_OK;
}

lee_status lee_get_ade_states(lee_instance *I, double *out)
{
    if (!I || !I->bound || !out) return fail(LEE_E_ARG, "instance not bound or null output");
    const size_t n = (size_t)I->host.ade_ns * I->host.gidx.size();
    if (!n) return LEE_OK;
    if (I->host.d.precision == LEE_F32) {
        std::vector<float> t(n);
        HIPCHK(hipMemcpyAsync(t.data(), I->dev.psi[0], n * 4, hipMemcpyDeviceToHost, I->stream));
        HIPCHK(hipStreamSynchronize(I->stream));
        for (size_t k = 0; k < n; ++k) out[k] = t[k];
    } else {
        HIPCHK(hipMemcpyAsync(out, I->dev.psi[0], n * 8, hipMemcpyDeviceToHost, I->stream));
        HIPCHK(hipStreamSynchronize(I->stream));
    }
    return LEE_OK;
}

lee_status lee_set_ade_states(lee_instance *I, const double *in)
{
    if (!I || !I->bound || !in) return fail(LEE_E_ARG, "instance not bound or null input");
    if (I->next_stage != 0) return fail(LEE_E_STATE, "a partial step is pending");
    const size_t n = (size_t)I->host.ade_ns * I->host.gidx.size();
    if (!n) return LEE_OK;
    if (I->host.d.precision == LEE_F32) {
        std::vector<float> t(n);
        for (size_t k = 0; k < n; ++k) t[k] = (float)in[k];
        HIPCHK(hipMemcpyAsync(I->dev.psi[0], t.data(), n * 4, hipMemcpyHostToDevice, I->stream));
        HIPCHK(hipStreamSynchronize(I->stream));
    } else {
        HIPCHK(hipMemcpyAsync(I->dev.psi[0], in, n * 8, hipMemcpyHostToDevice, I->stream));
        HIPCHK(hipStreamSynchronize(I->stream));
    }
    return LEE_OK;
}

lee_status lee_rhs(lee_instance *I, double *p, double *u, double *v, double *psi)
{
    if (!I || !I->bound) return fail(LEE_E_STATE, "instance not bound");
    if (I->next_stage != 0) return fail(LEE_E_STATE, "a partial step is pending");
    const Host &h = I->host;
    const Layout L = layout(h);
    hipStream_t s = I->stream;
    // the step's first stage with an update coefficient of one writes
    // q^(1) = q^n + RHS(q^n) and Psi^(1) = Psi^n + dPsi/dt; the coefficient is
    // put back before anything else runs on the stream
    static const double one = 1.0;
    char *adt0 = (char *)I->d_inst + offsetof(DevInst, alpha_dt);
    HIPCHK(hipMemcpyAsync(adt0, &one, sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(issue_stage(I, 0, 0));
    HIPCHK(hipMemcpyAsync(adt0, &I->dev.alpha_dt[0], sizeof(double), hipMemcpyHostToDevice, s));
    // a fused launch published its ghost values with this step's first-stage
    // epoch: clear them, so that the step itself cannot take them
    HIPCHK(launch_fill_bytes(I->base + L.xg, xg_bytes(h), s));
    const size_t nn = (size_t)h.d.nx * h.d.ny;
    double *o[3] = {p, u, v};
    std::vector<double> q1(nn), qn(nn);
    for (int f = 0; f < 3; ++f) {
        if (!o[f]) continue;
        lee_status st = h.d.precision == LEE_F32 ? copy_plane_out<float>(I, 1, f, q1.data())
                                                 : copy_plane_out<double>(I, 1, f, q1.data());
        if (st == LEE_OK)
            st = h.d.precision == LEE_F32 ? copy_plane_out<float>(I, 0, f, qn.data())
                                          : copy_plane_out<double>(I, 0, f, qn.data());
        if (st != LEE_OK) return st;
        for (size_t k = 0; k < nn; ++k) o[f][k] = h.fluid[k] ? q1[k] - qn[k] : 0.0;
    }
    const size_t n = (size_t)h.ade_ns * h.gidx.size();
    if (psi && n) {
        if (h.ade_kind == 0) {
            std::fill(psi, psi + n, 0.0);
        } else if (h.d.precision == LEE_F32) {
            std::vector<float> a(n), b(n);
            HIPCHK(hipMemcpyAsync(a.data(), I->dev.psi[1], n * 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(b.data(), I->dev.psi[0], n * 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (size_t k = 0; k < n; ++k) psi[k] = (double)a[k] - (double)b[k];
        } else {
            std::vector<double> a(n), b(n);
            HIPCHK(hipMemcpyAsync(a.data(), I->dev.psi[1], n * 8, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(b.data(), I->dev.psi[0], n * 8, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (size_t k = 0; k < n; ++k) psi[k] = a[k] - b[k];
        }
    }
    return check_sync(I->d_sync, s);
}

lee_status lee_probe(lee_instance *I, int32_t np, const double *xy, double *out)
{
    if (!I || !I->bound) return fail(LEE_E_STATE, "instance not bound");
    if (np < 0 || np > SAMPLE_MAX || (np > 0 && (!xy || !out))) return fail(LEE_E_ARG, "probe arguments");
    if (I->next_stage != 0) return fail(LEE_E_STATE, "a partial step is pending");
    if (np == 0) return LEE_OK;
    std::vector<int> ij(2 * np);
    std::vector<double> w(16 * np);
    for (int k = 0; k < np; ++k) {
        lee_status s = host_probe_stencil(&I->host, xy[2 * k], xy[2 * k + 1], &ij[2 * k], &ij[2 * k + 1], &w[16 * k]);
        if (s != LEE_OK) return s;
    }
    HIPCHK(hipMemcpyAsync(I->d_sij, ij.data(), ij.size() * 4, hipMemcpyHostToDevice, I->stream));
    HIPCHK(hipMemcpyAsync(I->d_sw, w.data(), w.size() * 8, hipMemcpyHostToDevice, I->stream));
    HIPCHK(launch_sample(I->host.d.precision, I->d_inst, I->d_sij, I->d_sw, np, I->d_sout, I->stream));
    HIPCHK(hipMemcpyAsync(out, I->d_sout, 3 * np * 8, hipMemcpyDeviceToHost, I->stream));
    HIPCHK(hipStreamSynchronize(I->stream));
    return LEE_OK;
}

lee_status lee_probe_traces(lee_instance *I, double *out, int64_t cap, int64_t *n)
{
    if (!I || !I->bound || !n) return fail(LEE_E_ARG, "instance not bound or null argument");
    const Host &h = I->host;
    *n = 0;
    if (h.np == 0 || h.trace_cap == 0) return LEE_OK;
    long long done = 0;
    HIPCHK(hipMemcpyAsync(&done, I->dev.step, 8, hipMemcpyDeviceToHost, I->stream));
    std::vector<double> ring((size_t)h.trace_cap * h.np * 3);
    HIPCHK(hipMemcpyAsync(ring.data(), I->dev.trace, ring.size() * 8, hipMemcpyDeviceToHost, I->stream));
    HIPCHK(hipStreamSynchronize(I->stream));
    int64_t m = std::min<int64_t>({(int64_t)done, (int64_t)h.trace_cap, cap});
    if (m > 0 && !out) return fail(LEE_E_ARG, "null output");
    const int64_t first = done - m;
    const size_t row = (size_t)h.np * 3;
    for (int64_t s = 0; s < m; ++s)
        std::memcpy(out + s * row, ring.data() + (size_t)((first + s) % h.trace_cap) * row, row * 8);
    *n = m;
    return LEE_OK;
}

lee_status lee_probe_dft(lee_instance *I, double *out)
{
    if (!I || !I->bound || !out) return fail(LEE_E_ARG, "instance not bound or null output");
    const Host &h = I->host;
    if (h.np == 0) return LEE_OK;
    std::vector<double> acc(2 * (size_t)h.np);
    HIPCHK(hipMemcpyAsync(acc.data(), I->dev.dft, acc.size() * 8, hipMemcpyDeviceToHost, I->stream));
    HIPCHK(hipStreamSynchronize(I->stream));
    const double N = h.dft_count > 0 ? (double)h.dft_count : 1.0;
    for (int k = 0; k < h.np; ++k) {      // P = (2i/N) (Sr + i Si)
        out[2 * k] = -2.0 * acc[2 * k + 1] / N;
        out[2 * k + 1] = 2.0 * acc[2 * k] / N;
    }
    return LEE_OK;
}

lee_status lee_export_lists(const lee_instance *I, int32_t *ghost_idx, int32_t *cloud_ptr, int32_t *cloud_idx,
                            int8_t *degree, double *weights, double *beta, double *geom)
{
    if (!I) return fail(LEE_E_ARG, "null instance");
    const Host &h = I->host;
    if (!h.built) return fail(LEE_E_STATE, "lee_build_ghosts first");
    const size_t G = h.gidx.size(), nnz = h.cidx.size();
    if (ghost_idx) std::copy(h.gidx.begin(), h.gidx.end(), ghost_idx);
    if (cloud_ptr) std::copy(h.cptr.begin(), h.cptr.end(), cloud_ptr);
    if (cloud_idx) std::copy(h.cidx.begin(), h.cidx.end(), cloud_idx);
    if (degree) std::copy(h.deg.begin(), h.deg.end(), degree);
    if (weights) std::copy(h.w4.begin(), h.w4.end(), weights);
    if (beta) std::copy(h.beta.begin(), h.beta.end(), beta);
    if (geom)
        for (size_t g = 0; g < G; ++g) {
            geom[5 * g + 0] = h.bx[g];
            geom[5 * g + 1] = h.by[g];
            geom[5 * g + 2] = h.gnx[g];
            geom[5 * g + 3] = h.gny[g];
            geom[5 * g + 4] = h.r[g];
        }
    (void)nnz;
    return LEE_OK;
}

lee_status lee_time_kernels(lee_instance *I, int64_t n, double *sweep_us, double *ghost_us, double *step_us)
{
    if (!I || !I->bound) return fail(LEE_E_STATE, "instance not bound");
    if (n <= 0) return fail(LEE_E_ARG, "n must be positive");
    if (I->next_stage != 0) return fail(LEE_E_STATE, "a partial step is pending");
    const int prec = I->host.d.precision;
    const bool filt = filter_form(I->host) == 1;
    auto ghosts = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        for (int64_t k = 0; k < 4 * n && e == hipSuccess; ++k)
            e = launch_ghost(prec, I->d_inst, 1, I->host.ade_kind == 3, I->d_work2, I->nwork2, (int)(k & 3), 0,
                             ProbePass{nullptr, 0, 0},
                             I->stream);
        return e;
    };
    auto sweeps = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        for (int64_t k = 0; k < 4 * n && e == hipSuccess; ++k) {
            const int l = (int)(k & 3);
            e = fused(I->tl) ? launch_stage(prec, filt, I->tl.cols, I->tl.rows, I->d_inst, 1, I->host.ade_kind == 3,
                                            I->d_work1, I->nwork1,
                                            I->d_aux, I->d_patch, I->tile0, I->d_work2, I->nwork2, l, 0, I->d_sync,
                                            I->spin, ProbePass{nullptr, 0, 0}, I->stream)
                             : sweep(prec, filt, I->tl, I->d_inst, I->d_work1, I->nwork1, l, 0, 0, I->stream);
        }
        return e;
    };
    auto steps = [&]() -> hipError_t { return issue_run(I, (int)std::min<int64_t>(n, 1 << 20)); };
    double out[3] = {0, 0, 0};
    lee_status st = time_runs(I->stream, {ghosts, sweeps, steps}, out);
    lee_status st2 = lee_init_fields(I);
    if (st != LEE_OK) return st;
    if (st2 != LEE_OK) return st2;
    if (ghost_us) *ghost_us = out[0] / (4.0 * n);
    if (sweep_us) *sweep_us = out[1] / (4.0 * n);
    if (step_us) *step_us = out[2] / n;
    return LEE_OK;
}

lee_status lee_stream_copy(void *dst, const void *src, size_t bytes, void *hip_stream)
{
    if (!dst || !src || (bytes & 15) || (((uintptr_t)dst | (uintptr_t)src) & 15))
        return fail(LEE_E_ARG, "copy needs 16-byte aligned buffers and a multiple of 16 bytes");
    HIPCHK(launch_copy(src, dst, bytes, (hipStream_t)hip_stream));
    return LEE_OK;
}

void lee_destroy(lee_instance *I)
{
    if (!I) return;
    drop_graph(I);
    delete I;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batches: one launch per phase over the work of all members

struct lee_batch {
    std::vector<lee_instance *> members;
    int prec = LEE_F32;
    bool filt = true;                            // the stages carry the filter's damping term
    bool fx = false;                             // the filter runs once per step (k_filter)
    lee_tiling tl{};
    int pblocks = 0;
    hipStream_t stream = nullptr;
    int device = -1;
    DevInst *d_table = nullptr;
    size_t table_cap = 0;
    int4 *d_work1 = nullptr;
    size_t work1_cap = 0;
    int nwork1 = 0;
    int4 *d_work2 = nullptr;
    size_t work2_cap = 0;
    int nwork2 = 0;
    int *d_sync = nullptr;
    std::vector<DevInst> up_table;
    std::vector<int4> up_work1;
    std::vector<int2> up_aux, up_patch;
    int2 *d_aux = nullptr, *d_patch = nullptr;
    size_t aux_cap = 0, patch_cap = 0;
    int tile0 = 0;
    std::vector<int4> up_work2;
    int2 *d_pwork = nullptr;               // (member, probe) pairs of the probe pass
    size_t pwork_cap = 0;
    int npwork = 0;
    std::vector<int2> up_pwork;
    std::vector<long long> up_budget;      // stop steps being uploaded
    long long *d_idle = nullptr;           // step and stop counters of the idle table entries (0, 0)
    bool poles = false;                    // some member has a multi-pole wall
    DevInst idle{};                        // table entry past the members
    StepGraphs graphs;
};

namespace {

void batch_drop_graph(lee_batch *B) { B->graphs.drop(); }

// Frees the table and work lists (the caller has synchronised the stream).
void batch_release_lists(lee_batch *B)
{
    auto rel = [](auto *&p, size_t &cap) {
        if (p) hipFree(p);
        p = nullptr;
        cap = 0;
    };
    rel(B->d_table, B->table_cap);
    rel(B->d_work1, B->work1_cap);
    rel(B->d_work2, B->work2_cap);
    rel(B->d_aux, B->aux_cap);
    rel(B->d_patch, B->patch_cap);
    rel(B->d_pwork, B->pwork_cap);
}

// The sweep work list over all members, in XCD-aware order, with the ghost
// patches of the fused form.  The carriers are those of the padded ghost
// list (work2_cap items), which is what the launches see.
void batch_build_work1(lee_batch *B)
{
    std::vector<int4> items;
    std::vector<std::vector<int2>> patches;
    for (size_t k = 0; k < B->members.size(); ++k) build_items(B->members[k]->host, (int)k, B->tl, items, &patches);
    B->tile0 = order_work(items, patches, per_unit_of(B->tl), carriers_for(B->tl, B->work2_cap), true,
                          B->up_work1, B->up_aux, B->up_patch);
}

hipError_t batch_issue_stage(lee_batch *B, int stage, int slot)
{
    int blocks = 0;
    const int per = B->tl.kind == LEE_SWEEP_MARCH ? B->tl.waves : 1;
    if (B->pblocks > 0) blocks = std::min(B->pblocks, (B->nwork1 + per - 1) / per);
    return stage_launches(B->prec, B->filt, B->tl, B->d_table, 0, B->poles, B->d_work1, B->nwork1,
                          B->d_aux, B->d_patch,
                          B->tile0, B->d_work2, B->nwork2, B->d_sync, stage, slot,
                          probe_pass(B->d_pwork, B->npwork, stage, slot), blocks, B->stream);
}

hipError_t batch_issue_run(lee_batch *B, int n)
{
    hipError_t e = hipSuccess;
    for (int j = 0; j < n && e == hipSuccess; ++j) {
        for (int l = 0; l < 4 && e == hipSuccess; ++l) e = batch_issue_stage(B, l, j);
        if (e == hipSuccess && B->fx)
            e = launch_filter(B->prec, B->tl.cols, B->tl.rows, B->d_table, B->d_work1, B->nwork1, j, B->stream);
    }
    if (e == hipSuccess) e = launch_probe(B->prec, B->d_table, ProbePass{B->d_pwork, B->npwork, n - 1}, B->stream);
    if (e == hipSuccess) e = launch_advance(B->d_table, (int)B->table_cap, n, B->stream);
    return e;
}

// Grows a device array to hold n elements, with a quarter more room once it
// has held some (synchronising before it frees the old one, which queued
// kernels may still read).
template <typename T>
hipError_t grow(T *&p, size_t &cap, size_t n, hipStream_t s)
{
    n = std::max<size_t>(n, 1);
    if (n <= cap) return hipSuccess;
    const size_t want = cap ? std::max(n, cap + cap / 4) : n;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) return e;
    if (p) hipFree(p);
    p = nullptr;
    cap = 0;
    e = hipMalloc(&p, want * sizeof(T));
    if (e == hipSuccess) cap = want;
    return e;
}

// Instance table and work lists from the member list, uploaded on the
// batch's stream.  Every list is padded with idle entries to its device
// capacity, and the launches cover the capacities, so the captured graphs
// stay valid across membership changes: they are dropped only when a list
// outgrows its capacity (capacities grow by at least a quarter; the fused
// form's carriers follow the ghost capacity), when a sweep or ghost list
// falls below three quarters of its capacity, or when `drop` is set; then
// every capacity is trimmed to the current lists (no idle workgroups).
lee_status batch_rebuild(lee_batch *B, bool drop = false)
{
    if (drop) {
        HIPCHK(hipStreamSynchronize(B->stream));
        batch_drop_graph(B);
        batch_release_lists(B);
    }
    const size_t n = B->members.size();
    B->up_table.clear();
    B->up_work2.clear();
    B->up_pwork.clear();
    // the members' planes together decide the streaming stores: a batch
    // whose planes exceed the on-chip cache streams every member's outputs
    size_t plane_bytes = 0;
    for (const auto *I : B->members) plane_bytes += 9 * plane_elems(I->host) * esize(I->host);
    const int sin = stream_in_for(plane_bytes, plane_bytes / 3);
    for (size_t k = 0; k < n; ++k) {
        const lee_instance *I = B->members[k];
        B->up_table.push_back(I->dev);
        B->up_table.back().stream = plane_bytes > STREAM_STORE_BYTES ? 1 : 0;
        B->up_table.back().stream_in = sin;
        for (int g = 0; g < (int)I->host.gidx.size(); ++g)
            B->up_work2.push_back(make_int4((int)k, g, I->host.cptr[g], I->host.cptr[g + 1]));
        for (int p = 0; p < I->host.np; ++p) B->up_pwork.push_back(make_int2((int)k, p));
    }
    // a list that grows drops the graphs (they launch the old capacities);
    // the capacities are compared as well as the pointers, since a new
    // allocation can come back at the address of the one it replaces
    const void *before[6] = {B->d_table, B->d_work1, B->d_work2, B->d_aux, B->d_patch, B->d_pwork};
    const size_t caps_before[6] = {B->table_cap, B->work1_cap, B->work2_cap, B->aux_cap, B->patch_cap, B->pwork_cap};
    const int tile0_before = B->tile0;
    HIPCHK(grow(B->d_table, B->table_cap, n, B->stream));
    HIPCHK(grow(B->d_work2, B->work2_cap, B->up_work2.size(), B->stream));
    HIPCHK(grow(B->d_pwork, B->pwork_cap, B->up_pwork.size(), B->stream));
    batch_build_work1(B);
    // lists far below their capacities would launch many idle workgroups in
    // every stage: trim them (new graphs) instead
    auto sparse = [](size_t used, size_t cap) { return cap > 256 && 4 * used < 3 * cap; };
    if (!drop && (sparse(B->up_work1.size(), B->work1_cap) || sparse(B->up_work2.size(), B->work2_cap)))
        return batch_rebuild(B, true);
    HIPCHK(grow(B->d_work1, B->work1_cap, B->up_work1.size(), B->stream));
    HIPCHK(grow(B->d_aux, B->aux_cap, B->work1_cap, B->stream));
    HIPCHK(grow(B->d_patch, B->patch_cap, B->up_patch.size(), B->stream));
    const void *after[6] = {B->d_table, B->d_work1, B->d_work2, B->d_aux, B->d_patch, B->d_pwork};
    const size_t caps_after[6] = {B->table_cap, B->work1_cap, B->work2_cap, B->aux_cap, B->patch_cap, B->pwork_cap};
    for (int k = 0; k < 6; ++k) drop = drop || before[k] != after[k] || caps_before[k] != caps_after[k];
    bool poles = false;
    for (const auto *I : B->members) poles = poles || I->host.ade_kind == 3;
    drop = drop || poles != B->poles;               // another ghost-fill variant
    B->poles = poles;
    drop = drop || B->tile0 != tile0_before;
    if (drop) batch_drop_graph(B);             // after a trim the pointers have changed as well
    B->up_table.resize(B->table_cap, B->idle);
    B->up_work1.resize(B->work1_cap, make_int4(-1, 0, 0, 1));
    B->up_aux.resize(B->work1_cap, make_int2(0, 0));
    B->up_work2.resize(B->work2_cap, make_int4(-1, 0, 0, 0));
    B->up_pwork.resize(B->pwork_cap, make_int2(-1, 0));
    B->nwork1 = (int)B->work1_cap;
    B->nwork2 = (int)B->work2_cap;
    B->npwork = (int)B->pwork_cap;
    HIPCHK(hipMemcpyAsync(B->d_table, B->up_table.data(), B->table_cap * sizeof(DevInst), hipMemcpyHostToDevice,
                          B->stream));
    HIPCHK(hipMemcpyAsync(B->d_work1, B->up_work1.data(), B->work1_cap * sizeof(int4), hipMemcpyHostToDevice,
                          B->stream));
    HIPCHK(hipMemcpyAsync(B->d_aux, B->up_aux.data(), B->work1_cap * sizeof(int2), hipMemcpyHostToDevice,
                          B->stream));
    HIPCHK(hipMemcpyAsync(B->d_work2, B->up_work2.data(), B->work2_cap * sizeof(int4), hipMemcpyHostToDevice,
                          B->stream));
    HIPCHK(hipMemcpyAsync(B->d_pwork, B->up_pwork.data(), B->pwork_cap * sizeof(int2), hipMemcpyHostToDevice,
                          B->stream));
    if (!B->up_patch.empty())
        HIPCHK(hipMemcpyAsync(B->d_patch, B->up_patch.data(), B->up_patch.size() * sizeof(int2),
                              hipMemcpyHostToDevice, B->stream));
    HIPCHK(hipStreamSynchronize(B->stream));      // the host staging vectors change with the next rebuild
    return LEE_OK;
}

lee_status member_ok(const lee_batch *B, const lee_instance *I)
{
    if (!I || !I->bound) return fail(LEE_E_STATE, "every member must be bound");
    if (I->next_stage != 0) return fail(LEE_E_STATE, "a member has a partial step pending");
    if (I->host.d.precision != B->prec) return fail(LEE_E_ARG, "mixed precision");
    if ((filter_form(I->host) == 1) != B->filt || (filter_form(I->host) == 2) != B->fx)
        return fail(LEE_E_ARG, "mixed filter forms");
    if (I->device != B->device) return fail(LEE_E_ARG, "members on different devices");
    if (I->host.d.radiation && B->tl.kind == LEE_SWEEP_MARCH)
        return fail(LEE_E_ARG, "the march sweep has no radiation band");
    if (filter_form(I->host) == 2 && B->tl.kind == LEE_SWEEP_MARCH)
        return fail(LEE_E_ARG, "the explicit filter needs a tile sweep");
    return LEE_OK;
}

void batch_free(lee_batch *B)
{
    batch_drop_graph(B);
    batch_release_lists(B);
    if (B->d_sync) hipFree(B->d_sync);
    if (B->d_idle) hipFree(B->d_idle);
    B->d_idle = nullptr;
    B->d_sync = nullptr;
}

}  // namespace

extern "C" {

lee_status lee_batch_create(lee_instance *const *v, int32_t n, const lee_batch_opts *opts, lee_batch **out)
{
    if (!v || n <= 0 || !out) return fail(LEE_E_ARG, "batch arguments");
    *out = nullptr;
    for (int k = 0; k < n; ++k) {
        if (!v[k] || !v[k]->bound) return fail(LEE_E_STATE, "every member must be bound");
        if (v[k]->next_stage != 0) return fail(LEE_E_STATE, "a member has a partial step pending");
        if (v[k]->host.d.precision != v[0]->host.d.precision) return fail(LEE_E_ARG, "mixed precision");
        if (filter_form(v[k]->host) != filter_form(v[0]->host)) return fail(LEE_E_ARG, "mixed filter forms");
        if (v[k]->device != v[0]->device) return fail(LEE_E_ARG, "members on different devices");
    }
    lee_batch *B = new (std::nothrow) lee_batch();
    if (!B) return fail(LEE_E_NOMEM, "host allocation");
    B->members.assign(v, v + n);
    B->prec = v[0]->host.d.precision;
    B->filt = filter_form(v[0]->host) == 1;
    B->fx = filter_form(v[0]->host) == 2;
    B->stream = v[0]->stream;
    B->device = v[0]->device;
    B->tl = default_tiling_for(B->prec, 4096, 4096);
    if (opts) {
        if (opts->tiling.kind >= 0) B->tl = opts->tiling;
        B->pblocks = opts->persistent_blocks;
        if (opts->graph_steps > GRAPH_STEPS_MAX) {
            delete B;
            return fail(LEE_E_ARG, "too many steps per graph");
        }
        B->graphs.per = graph_steps_from(opts->graph_steps);
    }
    if (!tiling_valid(B->prec, B->tl) || B->pblocks < 0 || (B->fx && B->tl.kind == LEE_SWEEP_MARCH)) {
        delete B;
        return fail(LEE_E_ARG, "batch tiling options");
    }
    if (B->pblocks > 0) B->pblocks = (B->pblocks + 7) / 8 * 8;   // keep the XCD pattern
    hipError_t e = hipMalloc(&B->d_sync, SYNC_INTS * sizeof(int));
    if (e == hipSuccess) e = launch_fill_bytes(B->d_sync, SYNC_INTS * sizeof(int), B->stream);
    if (e == hipSuccess) e = hipMalloc(&B->d_idle, 2 * sizeof(long long));
    if (e == hipSuccess) e = launch_fill_bytes(B->d_idle, 2 * sizeof(long long), B->stream);
    B->idle.step = B->d_idle;
    B->idle.stop = B->d_idle ? B->d_idle + 1 : nullptr;
    if (e != hipSuccess) {
        batch_free(B);
        delete B;
        return hip_fail(e, "batch set-up");
    }
    lee_status st = batch_rebuild(B);
    if (st != LEE_OK) {
        batch_free(B);
        delete B;
        return st;
    }
    *out = B;
    return LEE_OK;
}

lee_status lee_batch_add(lee_batch *B, lee_instance *I)
{
    if (!B) return fail(LEE_E_ARG, "null batch");
    lee_status st = member_ok(B, I);
    if (st != LEE_OK) return st;
    if (std::find(B->members.begin(), B->members.end(), I) != B->members.end())
        return fail(LEE_E_ARG, "already a member");
    HIPCHK(hipStreamSynchronize(I->stream));      // its set-up ran on its own stream
    B->members.push_back(I);
    st = batch_rebuild(B);
    if (st != LEE_OK) B->members.pop_back();
    return st;
}

lee_status lee_batch_remove(lee_batch *B, lee_instance *I)
{
    if (!B || !I) return fail(LEE_E_ARG, "null argument");
    auto it = std::find(B->members.begin(), B->members.end(), I);
    if (it == B->members.end()) return fail(LEE_E_ARG, "not a member");
    HIPCHK(hipStreamSynchronize(B->stream));      // no queued step may still use it
    B->members.erase(it);
    return batch_rebuild(B);
}

lee_status lee_batch_update(lee_batch *B, lee_instance *const *add, int32_t nadd, lee_instance *const *remove,
                            int32_t nremove)
{
    if (!B || nadd < 0 || nremove < 0 || (nadd > 0 && !add) || (nremove > 0 && !remove))
        return fail(LEE_E_ARG, "batch update arguments");
    std::vector<lee_instance *> next = B->members;
    for (int32_t k = 0; k < nremove; ++k) {
        auto it = std::find(next.begin(), next.end(), remove[k]);
        if (!remove[k] || it == next.end()) return fail(LEE_E_ARG, "not a member");
        next.erase(it);
    }
    for (int32_t k = 0; k < nadd; ++k) {
        lee_status st = member_ok(B, add[k]);
        if (st != LEE_OK) return st;
        if (std::find(next.begin(), next.end(), add[k]) != next.end()) return fail(LEE_E_ARG, "already a member");
        next.push_back(add[k]);
    }
    HIPCHK(hipStreamSynchronize(B->stream));      // no queued step may still use a removed member
    for (int32_t k = 0; k < nadd; ++k) HIPCHK(hipStreamSynchronize(add[k]->stream));   // their set-up
    std::vector<lee_instance *> before = B->members;
    B->members = std::move(next);
    lee_status st = batch_rebuild(B);
    if (st != LEE_OK) B->members = std::move(before);
    return st;
}

lee_status lee_batch_graph_captures(const lee_batch *B, int64_t *n)
{
    if (!B || !n) return fail(LEE_E_ARG, "null argument");
    *n = B->graphs.captures;
    return LEE_OK;
}

lee_status lee_batch_size(const lee_batch *B, int32_t *n)
{
    if (!B || !n) return fail(LEE_E_ARG, "null argument");
    *n = (int32_t)B->members.size();
    return LEE_OK;
}

lee_status lee_batch_set_budget(lee_batch *B, const int64_t *steps)
{
    if (!B || !steps) return fail(LEE_E_ARG, "null argument");
    const size_t n = B->members.size();
    for (size_t k = 0; k < n; ++k)
        if (steps[k] < 0) return fail(LEE_E_ARG, "negative budget");
    // each member stops `steps` steps after the ones it has completed
    B->up_budget.assign(n, 0);
    HIPCHK(hipStreamSynchronize(B->stream));
    for (size_t k = 0; k < n; ++k)
        HIPCHK(hipMemcpy(&B->up_budget[k], B->members[k]->dev.step, 8, hipMemcpyDeviceToHost));
    for (size_t k = 0; k < n; ++k) {
        B->up_budget[k] += steps[k];
        HIPCHK(hipMemcpyAsync(B->members[k]->dev.stop, &B->up_budget[k], 8, hipMemcpyHostToDevice, B->stream));
    }
    HIPCHK(hipStreamSynchronize(B->stream));
    return LEE_OK;
}

lee_status lee_batch_step_n(lee_batch *B, int64_t n)
{
    if (!B) return fail(LEE_E_ARG, "null batch");
    if (n < 0) return fail(LEE_E_ARG, "n < 0");
    if (n == 0 || B->members.empty()) return LEE_OK;
    lee_status st = run_steps(B->graphs, B->stream, n, [B](int k) { return batch_issue_run(B, k); });
    if (st != LEE_OK) return st;
    for (auto *I : B->members) I->steps_issued += n;   // upper bound; budgets may idle members
    return LEE_OK;
}

lee_status lee_batch_time_kernels(lee_batch *B, int64_t n, double *sweep_us, double *ghost_us, double *step_us)
{
    if (!B) return fail(LEE_E_ARG, "null batch");
    if (B->members.empty()) return fail(LEE_E_STATE, "empty batch");
    if (n <= 0) return fail(LEE_E_ARG, "n must be positive");
    int blocks = 0;
    const int per = B->tl.kind == LEE_SWEEP_MARCH ? B->tl.waves : 1;
    if (B->pblocks > 0) blocks = std::min(B->pblocks, (B->nwork1 + per - 1) / per);
    auto ghosts = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        for (int64_t k = 0; k < 4 * n && e == hipSuccess; ++k)
            e = launch_ghost(B->prec, B->d_table, 0, B->poles, B->d_work2, B->nwork2, (int)(k & 3), 0,
                             ProbePass{nullptr, 0, 0}, B->stream);
        return e;
    };
    auto sweeps = [&]() -> hipError_t {
        hipError_t e = hipSuccess;
        for (int64_t k = 0; k < 4 * n && e == hipSuccess; ++k) {
            const int l = (int)(k & 3);
            e = fused(B->tl) ? launch_stage(B->prec, B->filt, B->tl.cols, B->tl.rows, B->d_table, 0, B->poles,
                                            B->d_work1,
                                            B->nwork1, B->d_aux, B->d_patch, B->tile0, B->d_work2, B->nwork2, l, 0,
                                            B->d_sync, SPIN_LIMIT, ProbePass{nullptr, 0, 0}, B->stream)
                             : sweep(B->prec, B->filt, B->tl, B->d_table, B->d_work1, B->nwork1, l, 0, blocks,
                                     B->stream);
        }
        return e;
    };
    auto steps = [&]() -> hipError_t { return batch_issue_run(B, (int)std::min<int64_t>(n, 1 << 20)); };
    double out[3] = {0, 0, 0};
    lee_status st = time_runs(B->stream, {ghosts, sweeps, steps}, out);
    for (auto *I : B->members) {
        lee_status s2 = lee_init_fields(I);
        if (st == LEE_OK) st = s2;
    }
    if (st != LEE_OK) return st;
    if (ghost_us) *ghost_us = out[0] / (4.0 * n);
    if (sweep_us) *sweep_us = out[1] / (4.0 * n);
    if (step_us) *step_us = out[2] / n;
    return LEE_OK;
}

lee_status lee_batch_synchronize(lee_batch *B)
{
    if (!B) return fail(LEE_E_ARG, "null batch");
    return check_sync(B->d_sync, B->stream);
}

lee_status lee_batch_set_tiling(lee_batch *B, const lee_tiling *t)
{
    if (!B || !t) return fail(LEE_E_ARG, "null argument");
    if (!tiling_valid(B->prec, *t)) return fail(LEE_E_ARG, "unsupported tiling");
    if (t->kind == LEE_SWEEP_MARCH) {
        if (B->fx) return fail(LEE_E_ARG, "the explicit filter needs a tile sweep");
        for (lee_instance *m : B->members)
            if (m->host.d.radiation) return fail(LEE_E_ARG, "the march sweep has no radiation band");
    }
    HIPCHK(hipStreamSynchronize(B->stream));     // the old lists may still be read
    B->tl = *t;
    return batch_rebuild(B, true);
}

lee_status lee_batch_get_tiling(const lee_batch *B, lee_tiling *t)
{
    if (!B || !t) return fail(LEE_E_ARG, "null argument");
    *t = B->tl;
    return LEE_OK;
}

lee_status lee_batch_set_graph_steps(lee_batch *B, int32_t steps)
{
    if (!B) return fail(LEE_E_ARG, "null batch");
    if (steps > GRAPH_STEPS_MAX) return fail(LEE_E_ARG, "too many steps per graph");
    batch_drop_graph(B);
    B->graphs.per = graph_steps_from(steps);
    return LEE_OK;
}

void lee_batch_destroy(lee_batch *B)
{
    if (!B) return;
    batch_free(B);
    delete B;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// members stepped together without allocating: the batch's instance table,
// work lists and error flag in a static device array

// In host code this name is a host-side stand-in, not a device address: only
// the address hipGetSymbolAddress returns (per device) may reach a kernel or
// a copy.
static __device__ __align__(256) unsigned char scratch[LEE_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int SCRATCH_DEVICES = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[SCRATCH_DEVICES] = {};

// The array's address on device dev, looked up once per device with that
// device current.
lee_status scratch_on(int dev, unsigned char **out)
{
    if (dev < 0 || dev >= SCRATCH_DEVICES) return fail(LEE_E_ARG, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        int cur = -1;
        HIPCHK(hipGetDevice(&cur));
        if (cur != dev) HIPCHK(hipSetDevice(dev));
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != dev) hipSetDevice(cur);
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = (unsigned char *)p;
    }
    *out = g_scratch_ptr[dev];
    return LEE_OK;
}

// Host staging of the lists, kept between calls of a thread.
struct NoAllocStaging {
    std::vector<DevInst> table;
    std::vector<int4> items, work1, work2;
    std::vector<std::vector<int2>> patches;
    std::vector<int2> aux, patch, pwork;
};
thread_local NoAllocStaging g_noalloc;

}  // namespace

extern "C" lee_status lee_step_members_noalloc(lee_instance *const *v, int32_t n, const lee_tiling *tiling,
                                               int64_t steps)
{
    if (!v || n <= 0 || n > LEE_NOALLOC_MAX_MEMBERS || steps < 0) return fail(LEE_E_ARG, "member list or steps");
    for (int k = 0; k < n; ++k) {
        if (!v[k] || !v[k]->bound) return fail(LEE_E_STATE, "every member must be bound");
        if (v[k]->next_stage != 0) return fail(LEE_E_STATE, "a member has a partial step pending");
        if (v[k]->host.d.precision != v[0]->host.d.precision) return fail(LEE_E_ARG, "mixed precision");
        if (filter_form(v[k]->host) != filter_form(v[0]->host)) return fail(LEE_E_ARG, "mixed filter forms");
        if (v[k]->device != v[0]->device) return fail(LEE_E_ARG, "members on different devices");
    }
    const int prec = v[0]->host.d.precision;
    const bool filt = filter_form(v[0]->host) == 1;
    const bool fx = filter_form(v[0]->host) == 2;
    const lee_tiling tl = tiling ? *tiling : default_tiling_for(prec, 4096, 4096);
    if (!tiling_valid(prec, tl)) return fail(LEE_E_ARG, "unsupported tiling");
    bool poles = false;
    for (int k = 0; k < n; ++k) {
        if (v[k]->host.d.radiation && tl.kind == LEE_SWEEP_MARCH)
            return fail(LEE_E_ARG, "the march sweep has no radiation band");
        if (fx && tl.kind == LEE_SWEEP_MARCH) return fail(LEE_E_ARG, "the explicit filter needs a tile sweep");
        poles = poles || v[k]->host.ade_kind == 3;
    }
    if (steps == 0) return LEE_OK;
    hipStream_t s = v[0]->stream;
    for (int k = 1; k < n; ++k)                  // their set-up ran on their own streams
        if (v[k]->stream != s) HIPCHK(hipStreamSynchronize(v[k]->stream));
    unsigned char *base = nullptr;
    lee_status st = scratch_on(v[0]->device, &base);
    if (st != LEE_OK) return st;

    // the lists of a batch of these members (as batch_rebuild and
    // batch_build_work1 make them, without padding)
    NoAllocStaging &S = g_noalloc;
    S.table.clear();
    S.work2.clear();
    S.pwork.clear();
    S.items.clear();
    S.patches.clear();
    size_t plane_bytes = 0;                      // as for batches: the members together
    for (int k = 0; k < n; ++k) plane_bytes += 9 * plane_elems(v[k]->host) * esize(v[k]->host);
    const int sin = stream_in_for(plane_bytes, plane_bytes / 3);
    for (int k = 0; k < n; ++k) {
        const lee_instance *I = v[k];
        S.table.push_back(I->dev);
        S.table.back().stream = plane_bytes > STREAM_STORE_BYTES ? 1 : 0;
        S.table.back().stream_in = sin;
        for (int g = 0; g < (int)I->host.gidx.size(); ++g)
            S.work2.push_back(make_int4(k, g, I->host.cptr[g], I->host.cptr[g + 1]));
        for (int p = 0; p < I->host.np; ++p) S.pwork.push_back(make_int2(k, p));
        build_items(I->host, k, tl, S.items, &S.patches);
    }
    const int tile0 = order_work(S.items, S.patches, per_unit_of(tl), carriers_for(tl, S.work2.size()), true,
                                 S.work1, S.aux, S.patch);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = (off + std::max<size_t>(bytes, 1) + 255) / 256 * 256;
        return o;
    };
    const size_t o_table = take(S.table.size() * sizeof(DevInst));
    const size_t o_work1 = take(S.work1.size() * sizeof(int4));
    const size_t o_aux = take(S.aux.size() * sizeof(int2));
    const size_t o_work2 = take(S.work2.size() * sizeof(int4));
    const size_t o_patch = take(S.patch.size() * sizeof(int2));
    const size_t o_pwork = take(S.pwork.size() * sizeof(int2));
    const size_t o_sync = take(SYNC_INTS * sizeof(int));
    if (off > LEE_NOALLOC_SCRATCH_BYTES)
        return fail(LEE_E_ARG, "the members' table and work lists need " + std::to_string(off) +
                                   " bytes; the no-alloc scratch holds " +
                                   std::to_string((size_t)LEE_NOALLOC_SCRATCH_BYTES));
    DevInst *d_table = (DevInst *)(base + o_table);
    int4 *d_work1 = (int4 *)(base + o_work1);
    int2 *d_aux = (int2 *)(base + o_aux);
    int4 *d_work2 = (int4 *)(base + o_work2);
    int2 *d_patch = (int2 *)(base + o_patch);
    int2 *d_pwork = (int2 *)(base + o_pwork);
    int *d_sync = (int *)(base + o_sync);
    auto up = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
        return bytes ? hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    HIPCHK(up(d_table, S.table.data(), S.table.size() * sizeof(DevInst)));
    HIPCHK(up(d_work1, S.work1.data(), S.work1.size() * sizeof(int4)));
    HIPCHK(up(d_aux, S.aux.data(), S.aux.size() * sizeof(int2)));
    HIPCHK(up(d_work2, S.work2.data(), S.work2.size() * sizeof(int4)));
    HIPCHK(up(d_patch, S.patch.data(), S.patch.size() * sizeof(int2)));
    HIPCHK(up(d_pwork, S.pwork.data(), S.pwork.size() * sizeof(int2)));
    HIPCHK(launch_fill_bytes(d_sync, SYNC_INTS * sizeof(int), s));   // a fill kernel: the flag starts clear
    HIPCHK(hipStreamSynchronize(s));             // the host staging is reused by the next call

    const int nwork1 = (int)S.work1.size(), nwork2 = (int)S.work2.size(), npwork = (int)S.pwork.size();
    for (int64_t done = 0; done < steps;) {
        const int run = (int)std::min<int64_t>(steps - done, 1 << 20);
        for (int j = 0; j < run; ++j) {
            for (int l = 0; l < 4; ++l)
                HIPCHK(stage_launches(prec, filt, tl, d_table, 0, poles, d_work1, nwork1, d_aux, d_patch, tile0,
                                      d_work2, nwork2, d_sync, l, j, probe_pass(d_pwork, npwork, l, j), 0, s));
            if (fx) HIPCHK(launch_filter(prec, tl.cols, tl.rows, d_table, d_work1, nwork1, j, s));
        }
        HIPCHK(launch_probe(prec, d_table, ProbePass{d_pwork, npwork, run - 1}, s));
        HIPCHK(launch_advance(d_table, n, run, s));
        done += run;
    }
    HIPCHK(launch_merge_flag(d_sync, v[0]->d_sync, s));
    for (int k = 0; k < n; ++k) v[k]->steps_issued += steps;
    return LEE_OK;
}
