// nb_runtime.cpp -- C ABI of libnbody (include/nbody.h): parameter checks, workspace layout,
// the segment tables that drive every launch, the step sequence and the read-backs.
#include "nbody.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <atomic>
#include <mutex>
#include <new>
#include <vector>

#include "nb_internal.h"

using namespace nbk;

namespace {

constexpr size_t ALIGN = 256;
constexpr double PI = 3.14159265358979323846;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// eq. (3): Roche-lobe radius over separation for mass ratio q.
double roche_lobe_ratio(double q)
{
    const double c = std::cbrt(q);
    return 0.49 * c * c / (0.69 * c * c + std::log(1.0 + c));
}

// L1 of two point masses 1 and q at unit separation, measured from the mass-1 star: the zero in
// (0, 1) of the axial Roche-potential gradient (1/(1+q)) / x^2 - (q/(1+q)) / (1-x)^2 - x +
// q/(1+q), which decreases strictly across the interval. Interval halving until it collapses.
double l1_from_accretor(double q)
{
    const double w1 = 1.0 / (1.0 + q), w2 = q / (1.0 + q);
    double left = 0.0, right = 1.0;
    while (true) {
        const double x = left + 0.5 * (right - left);
        if (!(x > left && x < right)) break;
        const double g = w1 / (x * x) - w2 / ((1.0 - x) * (1.0 - x)) - x + w2;
        (g > 0.0 ? left : right) = x;
    }
    return left + 0.5 * (right - left);
}

struct TileCfg {
    int ki, nsplit, iblock, jchunk, n_iblocks, n_units, n_ounits;
    int npad, p1, nalloc, ntiles;
    int sym, ch;            // symmetric kernel (Kahan and FP64 modes) and its tiles per chunk
    int rows;               // tile rows per band of the symmetric kernel (1, 2 or 4)
    size_t react_floats;    // reaction partials of the symmetric kernel (elements of the mode's type)
};

struct Override {
    int64_t lo, hi;
    int mode, law, nsplit, rows;
};

std::mutex g_cfg_mu;
std::vector<Override> g_overrides;
size_t g_budget = 0;  // workspace budget of nb_set_workspace_budget (0: none)

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct Layout;
Layout layout_for(int mode, int law, const TileCfg &c);
size_t layout_total(int mode, int law, const TileCfg &c);

// The work split fields of c for ns requested chunks and bands of `rows` tile rows.
void finish_split(TileCfg &c, int mode, int ns, int rows)
{
    c.rows = mode == NB_FP32_KAHAN ? rows : 1;  // bands of several rows: FP32 Kahan kernel only
    c.sym = 0;
    c.react_floats = 0;
    if (mode != NB_FP32_PLAIN && c.ntiles > 0) {
        // symmetric kernel: band g holds tile rows rows g .. rows g + rows - 1 and covers tiles
        // rows g .. T-1 in chunks of ch tiles; its reactions are stored for the tiles after its
        // first row. nsplit is the chunk count of the longest band.
        c.sym = 1;
        c.ch = std::max(1, (c.ntiles + std::max(ns, 1) - 1) / std::max(ns, 1));
        c.nsplit = (c.ntiles + c.ch - 1) / c.ch;
        c.jchunk = c.ch * TJ;
        int64_t units = 0, react_tiles = 0;
        for (int g = 0; g * c.rows < c.ntiles; ++g) {
            const int span = c.ntiles - g * c.rows;
            units += (span + c.ch - 1) / c.ch;
            react_tiles += span - 1;
        }
        // far beyond any device's memory the unit count no longer fits int32: n_units = -1
        // makes nb_scratch_bytes and nb_create report NB_E_NOMEM
        c.n_units = units > INT32_MAX ? -1 : (int)units;
        c.react_floats = (size_t)3 * TJ * (size_t)react_tiles;
        return;
    }
    // chunk c covers tiles [c ntiles / nsplit, (c + 1) ntiles / nsplit)
    c.nsplit = c.ntiles > 0 ? std::max(1, std::min(ns, c.ntiles)) : 1;
    c.jchunk = c.ntiles > 0 ? (c.ntiles + c.nsplit - 1) / c.nsplit * TJ : TJ;
    const int64_t units = (int64_t)c.n_iblocks * c.nsplit;
    c.n_units = units > INT32_MAX ? -1 : (int)units;
}

// Sorted layout and work split of a system; a function of (n, n1, mode, law), the overrides and
// the workspace budget only.
TileCfg tile_config(int64_t n, int64_t n1, int mode, int law)
{
    TileCfg c{};
    c.ki = 1;
    c.iblock = BT;
    c.p1 = (int)round_up(n1, TJ);
    c.npad = c.p1 + (int)round_up(n - n1, TJ);
    c.ntiles = c.npad / TJ;
    c.nalloc = (int)round_up(std::max(c.npad, 1), c.iblock);
    c.n_iblocks = c.npad > 0 ? c.nalloc / c.iblock : 0;
    c.n_ounits = (int)((n + BT - 1) / BT);
    int ns = 1, rows = 1;
    size_t budget = 0;
    if (mode != NB_FP32_PLAIN && c.ntiles > 0) {
        // built-in rule: about 65536 work units, chunks of 2..16 tiles; from 256 tiles on,
        // bands of four rows under the contact law and of two under eqs. (4)-(6) (measured
        // faster there, with a quarter or half of the reaction partials; the eqs. (4)-(6)
        // kernel spills at four), one row below
        const int64_t per = (int64_t)c.ntiles * c.n_iblocks / 65536;
        const int tpc = (int)std::min<int64_t>(16, std::max<int64_t>(2, per));
        ns = std::max(1, (c.ntiles + tpc / 2) / tpc);
        rows = c.ntiles < 256 ? 1 : (law == NB_LAW_CONTACT ? MAX_BAND : 2);
        std::lock_guard<std::mutex> g(g_cfg_mu);
        for (const Override &o : g_overrides) {
            if (o.mode == mode && o.law == law && n >= o.lo && n <= o.hi) {
                ns = o.nsplit;
                rows = o.rows;
            }
        }
        budget = g_budget;
    }
    finish_split(c, mode, ns, rows);
    // over the workspace budget: taller bands first (FP32 Kahan), then fewer, longer chunks,
    // until the layout fits or cannot shrink further
    while (budget > 0 && c.sym && c.n_units >= 0 && layout_total(mode, law, c) > budget) {
        if (mode == NB_FP32_KAHAN && c.rows < MAX_BAND) {
            finish_split(c, mode, c.nsplit, c.rows * 2);
        } else if (c.nsplit > 1) {
            finish_split(c, mode, c.nsplit / 2, c.rows);
        } else {
            break;
        }
    }
    return c;
}

struct Layout {
    size_t state, desc, diag, red, pe, log, xs, ys, zs, vxs, vys, vzs, perm, tbox, units, react,
        part, total;
};

Layout layout_for(int mode, int law, const TileCfg &c)
{
    Layout L{};
    const size_t elem = mode == NB_FP64 ? sizeof(double) : sizeof(float);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off = align_up(off + bytes, ALIGN);
        return at;
    };
    L.state = take(sizeof(DevState));
    L.desc = take(sizeof(SysDesc));
    L.diag = take(sizeof(DiagOut));
    L.red = take((size_t)std::max(c.n_ounits, 1) * RED_STRIDE * sizeof(double));
    L.pe = take((size_t)std::max(c.n_ounits, 1) * sizeof(double));
    L.log = take((size_t)L1_LOG_CAP * 4 * sizeof(int32_t));
    L.xs = take((size_t)c.nalloc * elem);
    L.ys = take((size_t)c.nalloc * elem);
    L.zs = take((size_t)c.nalloc * elem);
    // sorted velocities: only eqs. (4)-(6) read them
    L.vxs = take(law == NB_LAW_PAPER ? (size_t)c.nalloc * elem : 0);
    L.vys = take(law == NB_LAW_PAPER ? (size_t)c.nalloc * elem : 0);
    L.vzs = take(law == NB_LAW_PAPER ? (size_t)c.nalloc * elem : 0);
    L.perm = take((size_t)c.nalloc * sizeof(int32_t));
    L.tbox = take((size_t)std::max(c.ntiles, 1) * 8 * sizeof(float));
    L.units = take(c.sym ? (size_t)c.n_units * 2 * sizeof(int32_t) : 0);
    L.react = take(c.sym ? c.react_floats * elem : 0);
    L.part = off;
    if (c.nsplit > 1 || c.sym) take((size_t)c.nsplit * 3 * (size_t)c.nalloc * elem);
    L.total = off;
    return L;
}

size_t layout_total(int mode, int law, const TileCfg &c) { return layout_for(mode, law, c).total; }

// Morton order of each star's initial positions (10 bits per axis inside the star's bounding
// box, ties by index): consecutive sorted slots are close in space, so tiles have small boxes.
uint32_t spread10(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

template <typename T>
void morton_order(const T *x, const T *y, const T *z, int64_t b, int64_t e,
                  std::vector<int32_t> &out)
{
    out.clear();
    if (e <= b) return;
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = b; i < e; ++i) {
        const double p[3] = {(double)x[i], (double)y[i], (double)z[i]};
        for (int d = 0; d < 3; ++d) {
            if (std::isfinite(p[d])) {
                lo[d] = std::min(lo[d], p[d]);
                hi[d] = std::max(hi[d], p[d]);
            }
        }
    }
    std::vector<std::pair<uint32_t, int32_t>> keys((size_t)(e - b));
    for (int64_t i = b; i < e; ++i) {
        const double p[3] = {(double)x[i], (double)y[i], (double)z[i]};
        uint32_t q[3];
        for (int d = 0; d < 3; ++d) {
            const double span = hi[d] > lo[d] ? hi[d] - lo[d] : 1.0;
            double f = std::isfinite(p[d]) ? (p[d] - lo[d]) / span : 0.0;
            f = std::min(std::max(f, 0.0), 1.0);
            q[d] = (uint32_t)std::min(1023.0, f * 1024.0);
        }
        keys[(size_t)(i - b)] = {spread10(q[0]) | (spread10(q[1]) << 1) | (spread10(q[2]) << 2),
                                 (int32_t)i};
    }
    std::sort(keys.begin(), keys.end());
    out.resize(keys.size());
    for (size_t k = 0; k < keys.size(); ++k) out[k] = keys[k].second;
}

// The sorted order of the current positions (each star in Morton order, star 2 from slot p1,
// padding -1) into `perm`, uploaded to dperm on `st`. Synchronises `st` (the positions are read
// back first); `perm` must stay alive until the upload has completed.
int upload_sorted_order(const nb_params *p, const nb_buffers *b, const TileCfg &cfg,
                        int32_t *dperm, hipStream_t st, std::vector<int32_t> &perm)
{
    perm.assign((size_t)cfg.nalloc, -1);
    if (p->n > 0) {
        const size_t elem = p->mode == NB_FP64 ? sizeof(double) : sizeof(float);
        const size_t bytes = (size_t)p->n * elem;
        std::vector<char> hx(bytes), hy(bytes), hz(bytes);
        if (hipMemcpyAsync(hx.data(), b->x, bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(hy.data(), b->y, bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipMemcpyAsync(hz.data(), b->z, bytes, hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return NB_E_HIP;
        std::vector<int32_t> o1, o2;
        if (p->mode == NB_FP64) {
            const double *X = (const double *)hx.data(), *Y = (const double *)hy.data(),
                         *Z = (const double *)hz.data();
            morton_order(X, Y, Z, 0, p->n1, o1);
            morton_order(X, Y, Z, p->n1, p->n, o2);
        } else {
            const float *X = (const float *)hx.data(), *Y = (const float *)hy.data(),
                        *Z = (const float *)hz.data();
            morton_order(X, Y, Z, 0, p->n1, o1);
            morton_order(X, Y, Z, p->n1, p->n, o2);
        }
        std::copy(o1.begin(), o1.end(), perm.begin());
        std::copy(o2.begin(), o2.end(), perm.begin() + cfg.p1);
    }
    if (hipMemcpyAsync(dperm, perm.data(), perm.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                       st) != hipSuccess)
        return NB_E_HIP;
    return NB_OK;
}

bool params_ok(const nb_params *p)
{
    if (!p) return false;
    // n < 2^30 keeps every padded slot count and slot index inside int32
    if (p->n < 0 || p->n >= (int64_t(1) << 30)) return false;
    if (p->n1 < 0 || p->n1 > p->n) return false;
    if (p->mode != NB_FP32_PLAIN && p->mode != NB_FP32_KAHAN && p->mode != NB_FP64) return false;
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!std::isfinite(p->G) || p->G < 0.0) return false;
    if (!pos(p->m) || !std::isfinite(p->dt)) return false;
    if (!pos(p->D1) || !pos(p->D2) || !pos(p->q) || !pos(p->a) || !pos(p->R2_0)) return false;
    if (!std::isfinite(p->growth_rate) || p->growth_rate < 0.0) return false;
    if (p->law != NB_LAW_CONTACT && p->law != NB_LAW_PAPER) return false;
    if (p->law == NB_LAW_PAPER) {
        // the pair sums are kept per unit of G m, so the law needs G > 0; the symmetric FP32
        // kernel and the FP64 kernel implement it, the plain FP32 kernel does not
        if (p->mode == NB_FP32_PLAIN || !(p->G > 0.0)) return false;
        if (!std::isfinite(p->eps) || p->eps < 0.0) return false;
        if (!std::isfinite(p->gamma) || p->gamma < 0.0) return false;
        if (!std::isfinite(p->beta) || p->beta < 0.0 || p->beta > 1.0) return false;
        const double gc = p->gamma * PI / (12.0 * p->G * p->m * p->m);
        if (!std::isfinite(gc) || (p->mode != NB_FP64 && gc > 3.0e38)) return false;
    }
    return true;
}

// Force-kernel timing (nb_timing_*).
struct Timing {
    std::mutex mu;
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    double total_ms = 0.0;
    int64_t launches = 0;
} g_timing;

// Library-owned segment table for multi-system steps, one per device.
// Segment table of the last multi-system nb_step, one per (device, stream): work queued on one
// stream never reads a table that a call on another stream rewrites.
struct BatchTable {
    int device = -1;
    hipStream_t stream = nullptr;
    SysDesc *d = nullptr;
    SysDesc *h = nullptr;  // pinned staging
    int cap = 0;
    std::vector<SysDesc> last;
};
std::mutex g_batch_mu;
std::vector<BatchTable> g_batches;

// Force-kernel grid: 0 = one block per work unit, > 0 = persistent launch of this many blocks.
std::atomic<int> g_force_grid{0};

}  // namespace

// Segment table of nb_step_static: a fixed array in each GPU's memory, held until the process
// ends. In host code `scratch` only names the symbol; its device address on each GPU comes from
// hipGetSymbolAddress (static_table below), taken once per device with that device current.
static __device__ __align__(256) SysDesc scratch[NB_STATIC_MAX_SYS];

namespace {

constexpr int STATIC_MAX_DEVICES = 64;
std::mutex g_static_mu;
SysDesc *g_static_ptr[STATIC_MAX_DEVICES] = {};

// Device address of `scratch` on the current device `device` (looked up on first use).
int static_table(int device, SysDesc **out)
{
    if (device < 0 || device >= STATIC_MAX_DEVICES) return NB_E_INVAL;
    std::lock_guard<std::mutex> g(g_static_mu);
    if (!g_static_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return NB_E_HIP;
        }
        g_static_ptr[device] = static_cast<SysDesc *>(ptr);
    }
    *out = g_static_ptr[device];
    return NB_OK;
}

}  // namespace

struct nb_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    SysDesc *d_table = nullptr;  // the graph's own segment table
    int n_sys = 0, n_steps = 0;
};

struct nb_system {
    nb_params p;
    nb_buffers b;
    TileCfg cfg;
    Layout lay;
    SysDesc desc;  // unit_begin = ounit_begin = 0
    SysDesc *d_desc;
    DevState *d_state;
    DiagOut *d_diag;
    int device;
};

namespace {

int hip_status(hipError_t e) { return e == hipSuccess ? NB_OK : NB_E_HIP; }

#define NB_TRY(expr)                           \
    do {                                       \
        hipError_t e_ = (expr);                \
        if (e_ != hipSuccess) return NB_E_HIP; \
    } while (0)

int launch_force_timed(const Launch &L, int mode, hipStream_t st, bool need_combine,
                       bool allow_timing = true)
{
    NB_TRY(launch_gather(L, mode, st));
    hipEvent_t a = nullptr, b = nullptr;
    bool timed = false;
    if (allow_timing) {
        std::lock_guard<std::mutex> g(g_timing.mu);
        timed = g_timing.on;
    }
    if (timed) {
        // events are destroyed on every failure path, so a failed launch leaks nothing
        if (hipEventCreate(&a) != hipSuccess) return NB_E_HIP;
        if (hipEventCreate(&b) != hipSuccess || hipEventRecord(a, st) != hipSuccess) {
            (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
            return NB_E_HIP;
        }
    }
    const hipError_t e = launch_forces(L, mode, g_force_grid.load(), st);
    if (timed) {
        if (e != hipSuccess || hipEventRecord(b, st) != hipSuccess) {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            return NB_E_HIP;
        }
        std::lock_guard<std::mutex> g(g_timing.mu);
        g_timing.pending.emplace_back(a, b);
    }
    if (e != hipSuccess) return NB_E_HIP;
    if (need_combine) NB_TRY(launch_combine(L, mode, st));
    return NB_OK;
}

int run_steps(const Launch &L, int mode, int n_steps, bool need_combine, hipStream_t st,
              bool allow_timing = true)
{
    for (int k = 0; k < n_steps; ++k) {
        NB_TRY(launch_kick_drift(L, mode, st));
        int rc = launch_force_timed(L, mode, st, need_combine, allow_timing);
        if (rc != NB_OK) return rc;
        NB_TRY(launch_kick_stats(L, mode, 1, st));
        NB_TRY(launch_finalize_step(L, 1, st));
        NB_TRY(launch_l1_classify(L, mode, 0, st));
        NB_TRY(launch_finalize_l1(L, 0, st));
    }
    return NB_OK;
}

// Index of a band height in Launch::band_end.
int band_index(int rows) { return rows >= 4 ? 2 : (rows == 2 ? 1 : 0); }

Launch single_launch(const nb_system *s)
{
    Launch L{};
    L.sys = s->d_desc;
    L.n_sys = 1;
    L.law = s->p.law;
    L.total_units = s->cfg.n_units;
    L.total_ounits = s->cfg.n_ounits;
    L.total_tunits = s->cfg.ntiles;
    const int b = band_index(s->cfg.rows);
    for (int k = 0; k < 3; ++k) L.band_end[k] = k >= b ? L.total_units : 0;
    return L;
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// A system's buffers live on the device that was current at nb_create; every later call must be
// made with that device current, or its kernels would be queued on another GPU.
bool device_buffer(const void *ptr, int device)
{
    // device (or managed) memory of `device`; host memory, pinned or not, is refused, so a
    // wrong pointer is reported instead of reaching a kernel
    hipPointerAttribute_t at{};
    if (hipPointerGetAttributes(&at, ptr) != hipSuccess) {
        (void)hipGetLastError();  // the failed query must not linger as the thread's last error
        return false;
    }
    return (at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged) &&
           at.device == device;
}

bool on_own_device(const nb_system *s)
{
    int d = -1;
    return hipGetDevice(&d) == hipSuccess && d == s->device;
}

int check_system_list(nb_system *const *sys, int32_t n_sys)
{
    if (!sys || n_sys < 1) return NB_E_INVAL;
    int64_t units = 0, ounits = 0, tiles = 0;
    for (int k = 0; k < n_sys; ++k) {
        if (!sys[k] || !on_own_device(sys[k])) return NB_E_INVAL;
        if (sys[k]->p.mode != sys[0]->p.mode) return NB_E_MISMATCH;
        if (sys[k]->p.law != sys[0]->p.law) return NB_E_MISMATCH;
        for (int j = 0; j < k; ++j) {
            if (sys[j] == sys[k]) return NB_E_INVAL;
        }
        units += sys[k]->cfg.n_units;
        ounits += sys[k]->cfg.n_ounits;
        tiles += sys[k]->cfg.ntiles;
    }
    // the segment table's prefix offsets are int32
    if (units > INT32_MAX || ounits > INT32_MAX || tiles > INT32_MAX) return NB_E_NOMEM;
    return NB_OK;
}

// Table order of a multi-system launch: by band height (so each height's force units are one
// range), in the given order within a height. Writes n_sys indices into `order`. The order
// decides only which workgroup runs which unit, never a system's arithmetic.
void table_order(nb_system *const *sys, int32_t n_sys, int *order)
{
    int k = 0;
    for (int b = 0; b < 3; ++b) {
        for (int i = 0; i < n_sys; ++i) {
            if (band_index(sys[i]->cfg.rows) == b) order[k++] = i;
        }
    }
}

// Prefix offsets of table entry `pos` (system s) and the launch totals after it.
void table_append(Launch &L, const nb_system *s, int32_t &unit_begin, int32_t &ounit_begin,
                  int32_t &tunit_begin)
{
    unit_begin = L.total_units;
    ounit_begin = L.total_ounits;
    tunit_begin = L.total_tunits;
    L.total_units += s->cfg.n_units;
    L.total_ounits += s->cfg.n_ounits;
    L.total_tunits += s->cfg.ntiles;
    const int b = band_index(s->cfg.rows);
    for (int k = b; k < 3; ++k) L.band_end[k] = L.total_units;
}

// Segment table of several systems: each system's units follow the previous system's.
Launch build_table(nb_system *const *sys, int32_t n_sys, std::vector<SysDesc> &table,
                   bool &combine)
{
    table.resize(n_sys);
    std::vector<int> order((size_t)n_sys);
    table_order(sys, n_sys, order.data());
    Launch L{};
    combine = false;
    for (int k = 0; k < n_sys; ++k) {
        const nb_system *s = sys[order[k]];
        table[k] = s->desc;
        table_append(L, s, table[k].unit_begin, table[k].ounit_begin, table[k].tunit_begin);
        combine = combine || s->cfg.nsplit > 1 || s->cfg.sym;
    }
    L.n_sys = n_sys;
    L.law = sys[0]->p.law;
    return L;
}

// Segment-table entry of one system whose workspace starts at `base` (unit_begin = ounit_begin
// = tunit_begin = 0); st and diag are set by the caller.
void fill_desc(SysDesc &d, const nb_params *p, const nb_buffers *b, const TileCfg &cfg,
               const Layout &lay, char *base)
{
    std::memset(&d, 0, sizeof d);
    d.x = b->x;
    d.y = b->y;
    d.z = b->z;
    d.vx = b->vx;
    d.vy = b->vy;
    d.vz = b->vz;
    d.ax = b->ax;
    d.ay = b->ay;
    d.az = b->az;
    d.side = static_cast<int8_t *>(b->side);
    d.part = (cfg.nsplit > 1 || cfg.sym) ? base + lay.part : nullptr;
    d.units = cfg.sym ? reinterpret_cast<int32_t *>(base + lay.units) : nullptr;
    d.react = cfg.sym ? reinterpret_cast<float *>(base + lay.react) : nullptr;
    d.ch = cfg.ch;
    d.sym = cfg.sym;
    d.rows = cfg.rows;
    d.xs = base + lay.xs;
    d.ys = base + lay.ys;
    d.zs = base + lay.zs;
    const bool paper = p->law == NB_LAW_PAPER;
    d.vxs = paper ? base + lay.vxs : nullptr;
    d.vys = paper ? base + lay.vys : nullptr;
    d.vzs = paper ? base + lay.vzs : nullptr;
    d.law = p->law;
    d.perm = reinterpret_cast<int32_t *>(base + lay.perm);
    d.tbox = reinterpret_cast<float *>(base + lay.tbox);
    d.npad = cfg.npad;
    d.p1 = cfg.p1;
    d.nalloc = cfg.nalloc;
    d.ntiles = cfg.ntiles;
    d.tunit_begin = 0;
    d.red = reinterpret_cast<double *>(base + lay.red);
    d.pe_part = reinterpret_cast<double *>(base + lay.pe);
    d.l1_log = reinterpret_cast<int32_t *>(base + lay.log);
    d.n = (int32_t)p->n;
    d.n1 = (int32_t)p->n1;
    d.nsplit = cfg.nsplit;
    d.jchunk = cfg.jchunk;
    d.iblock = cfg.iblock;
    d.n_iblocks = cfg.n_iblocks;
    d.n_units = cfg.n_units;
    d.n_ounits = cfg.n_ounits;
    d.unit_begin = 0;
    d.ounit_begin = 0;
    d.n_peunits = cfg.n_ounits;
}

// Initial device state of a system: FP64 masters and the derived FP32 force constants.
void fill_state(DevState &init, const nb_params *p)
{
    std::memset(&init, 0, sizeof init);
    init.D1 = p->D1;
    init.D2 = p->D2;
    init.D2_0 = p->D2;
    init.R2_0 = p->R2_0;
    init.rL_a = roche_lobe_ratio(p->q) * p->a;
    init.growth_rate = p->growth_rate;
    init.G = p->G;
    init.m = p->m;
    init.dt = p->dt;
    init.xi_l1 = l1_from_accretor(p->q);
    const double Ds[3] = {p->D1, 0.5 * (p->D1 + p->D2), p->D2};
    for (int k = 0; k < 3; ++k) {
        init.c1d[k] = 11.0 / (Ds[k] * Ds[k] * Ds[k]);
        init.c2d[k] = 10.0 / (Ds[k] * Ds[k]);
        init.c1f[k] = (float)init.c1d[k];
        init.c2f[k] = (float)init.c2d[k];
        init.far2f[k] = (float)(Ds[k] * Ds[k] * (1.0 + (double)FAR_MARGIN));
    }
    init.gm_d = p->G * p->m;
    init.h_d = 0.5 * p->dt;
    init.gm_f = (float)init.gm_d;
    init.h_f = (float)init.h_d;
    init.dt_f = (float)p->dt;
    init.growth_on = p->growth_on ? 1 : 0;
    init.law = p->law;
    init.gamma = p->gamma;
    init.beta = p->beta;
    init.leps_d = p->eps;
    if (p->law == NB_LAW_PAPER) {
        init.lgc_d = p->gamma * PI / (12.0 * p->G * p->m * p->m);
        init.lgcb_d = p->beta * init.lgc_d;
    }
    for (int k = 0; k < 3; ++k) init.lD_f[k] = (float)Ds[k];
    init.leps_f = (float)p->eps;
    init.lgc_f = (float)init.lgc_d;
    init.lgcb_f = (float)init.lgcb_d;
}

}  // namespace

extern "C" {

int nb_version(void) { return 4; }

const char *nb_strerror(int status)
{
    switch (status) {
    case NB_OK: return "ok";
    case NB_E_INVAL: return "invalid argument";
    case NB_E_HIP: return "HIP runtime error";
    case NB_E_NOMEM: return "workspace too small, table allocation failed or system too large";
    case NB_E_NONFINITE: return "non-finite position or velocity";
    case NB_E_MISMATCH: return "systems of different modes or element laws in one call";
    case NB_E_LIMIT: return "more systems than the static segment table holds (NB_STATIC_MAX_SYS)";
    default: return "unknown status";
    }
}

int nb_tile_config(int64_t n, int64_t n1, int32_t mode, int32_t law, int32_t *ki, int32_t *nsplit,
                   int32_t *iblock, int32_t *jchunk, int32_t *rows)
{
    if (n < 0 || n >= (int64_t(1) << 30) || n1 < 0 || n1 > n) return NB_E_INVAL;
    if (mode != NB_FP32_PLAIN && mode != NB_FP32_KAHAN && mode != NB_FP64) return NB_E_INVAL;
    if (law != NB_LAW_CONTACT && law != NB_LAW_PAPER) return NB_E_INVAL;
    TileCfg c = tile_config(n, n1, mode, law);
    if (ki) *ki = c.ki;
    if (nsplit) *nsplit = c.nsplit;
    if (iblock) *iblock = c.iblock;
    if (jchunk) *jchunk = c.jchunk;
    if (rows) *rows = c.rows;
    return NB_OK;
}

int nb_set_force_grid(int32_t blocks)
{
    if (blocks < 0) return NB_E_INVAL;
    g_force_grid.store(blocks);
    return NB_OK;
}

int nb_tile_override(int64_t n_lo, int64_t n_hi, int32_t mode, int32_t law, int32_t nsplit,
                     int32_t rows)
{
    if (n_lo < 0 || n_hi < n_lo || nsplit < 0 || nsplit > 4096) return NB_E_INVAL;
    if (mode != NB_FP32_PLAIN && mode != NB_FP32_KAHAN && mode != NB_FP64) return NB_E_INVAL;
    if (law != NB_LAW_CONTACT && law != NB_LAW_PAPER) return NB_E_INVAL;
    if (nsplit > 0 && rows != 1 && rows != 2 && rows != 4) return NB_E_INVAL;
    if (nsplit > 0 && rows != 1 && mode != NB_FP32_KAHAN) return NB_E_INVAL;
    std::lock_guard<std::mutex> g(g_cfg_mu);
    g_overrides.erase(std::remove_if(g_overrides.begin(), g_overrides.end(),
                                     [&](const Override &o) {
                                         return o.mode == mode && o.law == law && o.lo == n_lo &&
                                                o.hi == n_hi;
                                     }),
                      g_overrides.end());
    if (nsplit > 0) g_overrides.push_back({n_lo, n_hi, mode, law, nsplit, rows});
    return NB_OK;
}

int nb_set_workspace_budget(size_t bytes)
{
    std::lock_guard<std::mutex> g(g_cfg_mu);
    g_budget = bytes;
    return NB_OK;
}

int nb_scratch_bytes(const nb_params *p, size_t *out)
{
    if (!params_ok(p) || !out) return NB_E_INVAL;
    TileCfg c = tile_config(p->n, p->n1, p->mode, p->law);
    if (c.n_units < 0) return NB_E_NOMEM;
    *out = layout_for(p->mode, p->law, c).total;
    return NB_OK;
}

int nb_create(const nb_params *p, const nb_buffers *b, void *stream, nb_system **out)
{
    if (!out) return NB_E_INVAL;
    *out = nullptr;
    if (!params_ok(p) || !b) return NB_E_INVAL;
    const size_t elem = p->mode == NB_FP64 ? sizeof(double) : sizeof(float);
    if (p->n > 0) {
        const void *arr[9] = {b->x, b->y, b->z, b->vx, b->vy, b->vz, b->ax, b->ay, b->az};
        for (const void *a : arr) {
            if (!a || !aligned(a, elem)) return NB_E_INVAL;
        }
        if (!b->side) return NB_E_INVAL;
    }
    if (!b->scratch || !aligned(b->scratch, ALIGN)) return NB_E_INVAL;
    TileCfg cfg = tile_config(p->n, p->n1, p->mode, p->law);
    if (cfg.n_units < 0) return NB_E_NOMEM;
    Layout lay = layout_for(p->mode, p->law, cfg);
    if (b->scratch_bytes < lay.total) return NB_E_NOMEM;
    int device = -1;
    if (hipGetDevice(&device) != hipSuccess) return NB_E_HIP;
    if (!device_buffer(b->scratch, device)) return NB_E_INVAL;
    if (p->n > 0) {
        const void *arr[10] = {b->x, b->y, b->z, b->vx, b->vy, b->vz, b->ax, b->ay, b->az, b->side};
        for (const void *a : arr) {
            if (!device_buffer(a, device)) return NB_E_INVAL;
        }
    }

    nb_system *s = new (std::nothrow) nb_system();
    if (!s) return NB_E_NOMEM;
    s->p = *p;
    s->b = *b;
    s->cfg = cfg;
    s->lay = lay;
    s->device = device;
    char *base = static_cast<char *>(b->scratch);
    s->d_state = reinterpret_cast<DevState *>(base + lay.state);
    s->d_desc = reinterpret_cast<SysDesc *>(base + lay.desc);
    s->d_diag = reinterpret_cast<DiagOut *>(base + lay.diag);

    SysDesc &d = s->desc;
    fill_desc(d, p, b, cfg, lay, base);
    d.st = s->d_state;
    d.diag = s->d_diag;
    DevState init;
    fill_state(init, p);
    const bool paper = p->law == NB_LAW_PAPER;

    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = NB_OK;
    do {
        // sorted layout: permutation from the initial positions (host-side Morton sort)
        std::vector<int32_t> perm;
        rc = upload_sorted_order(p, b, cfg, d.perm, st, perm);
        if (rc != NB_OK) break;
        std::vector<int32_t> units;
        if (cfg.sym) {
            // (band, chunk) pairs, full-length chunks first (each band's last chunk may be short)
            std::vector<std::pair<int, std::pair<int, int>>> order;
            for (int g = 0; g * cfg.rows < cfg.ntiles; ++g) {
                const int span = cfg.ntiles - g * cfg.rows;
                const int chunks = (span + cfg.ch - 1) / cfg.ch;
                for (int c = 0; c < chunks; ++c) {
                    const int len = std::min(cfg.ch, span - c * cfg.ch);
                    order.push_back({-len, {g, c}});
                }
            }
            std::stable_sort(order.begin(), order.end(),
                             [](const auto &a, const auto &b) { return a.first < b.first; });
            units.reserve(order.size() * 2);
            for (const auto &o : order) {
                units.push_back(o.second.first);
                units.push_back(o.second.second);
            }
            if ((int)order.size() != cfg.n_units) { rc = NB_E_INVAL; break; }
            if (hipMemcpyAsync(d.units, units.data(), units.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, st) != hipSuccess) { rc = NB_E_HIP; break; }
        }
        if (launch_fill_sorted(d.xs, d.ys, d.zs, cfg.nalloc, p->mode, true, st) != hipSuccess) {
            rc = NB_E_HIP;
            break;
        }
        if (paper && launch_fill_sorted(d.vxs, d.vys, d.vzs, cfg.nalloc, p->mode, false, st) !=
                         hipSuccess) {
            rc = NB_E_HIP;
            break;
        }
        if (launch_init_state(s->d_state, init, st) != hipSuccess) { rc = NB_E_HIP; break; }
        if (hipMemcpyAsync(s->d_desc, &s->desc, sizeof(SysDesc), hipMemcpyHostToDevice, st) !=
            hipSuccess) { rc = NB_E_HIP; break; }
        Launch L = single_launch(s);
        if (launch_kick_stats(L, p->mode, 0, st) != hipSuccess) { rc = NB_E_HIP; break; }
        if (launch_finalize_step(L, 0, st) != hipSuccess) { rc = NB_E_HIP; break; }
        if (launch_l1_classify(L, p->mode, 1, st) != hipSuccess) { rc = NB_E_HIP; break; }
        if (launch_finalize_l1(L, 1, st) != hipSuccess) { rc = NB_E_HIP; break; }
        if (launch_gather(L, p->mode, st) != hipSuccess) { rc = NB_E_HIP; break; }
        if (launch_forces(L, p->mode, g_force_grid.load(), st) != hipSuccess) { rc = NB_E_HIP; break; }
        if ((cfg.nsplit > 1 || cfg.sym) && launch_combine(L, p->mode, st) != hipSuccess) {
            rc = NB_E_HIP;
            break;
        }
        if (hipStreamSynchronize(st) != hipSuccess) { rc = NB_E_HIP; break; }
    } while (0);
    if (rc != NB_OK) {
        delete s;
        return rc;
    }
    *out = s;
    return NB_OK;
}

int nb_forces(nb_system *s, void *stream)
{
    if (!s || !on_own_device(s)) return NB_E_INVAL;
    return launch_force_timed(single_launch(s), s->p.mode, static_cast<hipStream_t>(stream),
                              s->cfg.nsplit > 1 || s->cfg.sym);
}

int nb_step(nb_system *const *sys, int32_t n_sys, int32_t n_steps, void *stream)
{
    if (n_steps < 0) return NB_E_INVAL;
    const int chk = check_system_list(sys, n_sys);
    if (chk != NB_OK) return chk;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int mode = sys[0]->p.mode;
    if (n_sys == 1) {
        return run_steps(single_launch(sys[0]), mode, n_steps,
                         sys[0]->cfg.nsplit > 1 || sys[0]->cfg.sym, st);
    }
    int device = 0;
    NB_TRY(hipGetDevice(&device));
    std::lock_guard<std::mutex> g(g_batch_mu);
    BatchTable *bt = nullptr;
    for (BatchTable &t : g_batches) {
        if (t.device == device && t.stream == st) bt = &t;
    }
    if (!bt) {
        g_batches.emplace_back();
        bt = &g_batches.back();
        bt->device = device;
        bt->stream = st;
    }
    std::vector<SysDesc> table;
    bool combine = false;
    Launch L = build_table(sys, n_sys, table, combine);
    const bool same = bt->last.size() == table.size() &&
                      std::memcmp(bt->last.data(), table.data(), table.size() * sizeof(SysDesc)) == 0;
    if (!same) {
        if (n_sys > bt->cap) {
            // the previous table may still be read by queued work on this stream
            if (bt->d) {
                NB_TRY(hipStreamSynchronize(st));
                NB_TRY(hipFree(bt->d));
                NB_TRY(hipHostFree(bt->h));
                bt->d = nullptr;
                bt->h = nullptr;
            }
            int cap = std::max(n_sys, 2 * bt->cap);
            if (hipMalloc(&bt->d, (size_t)cap * sizeof(SysDesc)) != hipSuccess) return NB_E_NOMEM;
            if (hipHostMalloc(&bt->h, (size_t)cap * sizeof(SysDesc), 0) != hipSuccess) {
                (void)hipFree(bt->d);
                bt->d = nullptr;
                return NB_E_NOMEM;
            }
            bt->cap = cap;
        }
        // the staging buffer may still feed an earlier queued copy
        NB_TRY(hipStreamSynchronize(st));
        std::memcpy(bt->h, table.data(), table.size() * sizeof(SysDesc));
        NB_TRY(hipMemcpyAsync(bt->d, bt->h, table.size() * sizeof(SysDesc), hipMemcpyHostToDevice,
                              st));
        bt->last = table;
    }
    L.sys = bt->d;
    return run_steps(L, mode, n_steps, combine, st);
}

int nb_step_static(nb_system *const *sys, int32_t n_sys, int32_t n_steps, void *stream)
{
    if (n_steps < 0) return NB_E_INVAL;
    if (sys && n_sys > NB_STATIC_MAX_SYS) return NB_E_LIMIT;
    const int chk = check_system_list(sys, n_sys);
    if (chk != NB_OK) return chk;
    int device = -1;
    NB_TRY(hipGetDevice(&device));
    SysDesc *table = nullptr;
    const int rc = static_table(device, &table);
    if (rc != NB_OK) return rc;
    hipStream_t st = static_cast<hipStream_t>(stream);
    // the table is rewritten on the device, ordered on `stream` before the steps that read it:
    // each entry is the system's own one-entry table with this call's prefix offsets
    Launch L{};
    L.n_sys = n_sys;
    L.law = sys[0]->p.law;
    bool combine = false;
    int order[NB_STATIC_MAX_SYS];
    table_order(sys, n_sys, order);
    TableChunk c;
    for (int first = 0; first < n_sys; first += TABLE_CHUNK) {
        std::memset(&c, 0, sizeof c);
        c.first = first;
        c.count = std::min(TABLE_CHUNK, n_sys - first);
        for (int k = 0; k < c.count; ++k) {
            const nb_system *s = sys[order[first + k]];
            c.src[k] = s->d_desc;
            table_append(L, s, c.unit_begin[k], c.ounit_begin[k], c.tunit_begin[k]);
            combine = combine || s->cfg.nsplit > 1 || s->cfg.sym;
        }
        NB_TRY(launch_copy_table(table, c, st));
    }
    L.sys = table;
    return run_steps(L, sys[0]->p.mode, n_steps, combine, st, false);
}

int nb_graph_create(nb_system *const *sys, int32_t n_sys, int32_t n_steps, void *stream,
                    nb_graph **out)
{
    if (!out) return NB_E_INVAL;
    *out = nullptr;
    if (n_steps < 1) return NB_E_INVAL;
    const int chk = check_system_list(sys, n_sys);
    if (chk != NB_OK) return chk;
    std::vector<SysDesc> table;
    bool combine = false;
    Launch L = build_table(sys, n_sys, table, combine);
    nb_graph *g = new (std::nothrow) nb_graph();
    if (!g) return NB_E_NOMEM;
    g->n_sys = n_sys;
    g->n_steps = n_steps;
    (void)stream;  // nothing is queued on the caller's stream
    hipStream_t cs = nullptr;
    int rc = NB_OK;
    do {
        if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
            cs = nullptr;
            rc = NB_E_HIP;
            break;
        }
        if (hipMalloc(&g->d_table, table.size() * sizeof(SysDesc)) != hipSuccess) {
            g->d_table = nullptr;
            rc = NB_E_NOMEM;
            break;
        }
        // the table travels on the private stream, so work already queued elsewhere keeps
        // running while the graph is built
        if (hipMemcpyAsync(g->d_table, table.data(), table.size() * sizeof(SysDesc),
                           hipMemcpyHostToDevice, cs) != hipSuccess ||
            hipStreamSynchronize(cs) != hipSuccess) { rc = NB_E_HIP; break; }
        L.sys = g->d_table;
        if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            rc = NB_E_HIP;
            break;
        }
        rc = run_steps(L, sys[0]->p.mode, n_steps, combine, cs, false);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &graph);
        g->graph = graph;
        if (rc != NB_OK) break;
        if (e != hipSuccess || !graph) { rc = NB_E_HIP; break; }
        if (hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            g->exec = nullptr;
            rc = NB_E_HIP;
            break;
        }
    } while (0);
    if (cs) (void)hipStreamDestroy(cs);
    if (rc != NB_OK) {
        nb_graph_destroy(g);
        return rc;
    }
    *out = g;
    return NB_OK;
}

int nb_graph_launch(nb_graph *g, void *stream)
{
    if (!g || !g->exec) return NB_E_INVAL;
    NB_TRY(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    return NB_OK;
}

void nb_graph_destroy(nb_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->d_table) (void)hipFree(g->d_table);
    delete g;
}

int nb_diagnostics(nb_system *s, int32_t with_pe, nb_diag *out, void *stream)
{
    if (!s || !out || !on_own_device(s)) return NB_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    NB_TRY(launch_diag(single_launch(s), s->p.mode, with_pe ? 1 : 0, st));
    DiagOut d;
    DevState ds;
    NB_TRY(hipMemcpyAsync(&d, s->d_diag, sizeof d, hipMemcpyDeviceToHost, st));
    NB_TRY(hipMemcpyAsync(&ds, s->d_state, sizeof ds, hipMemcpyDeviceToHost, st));
    NB_TRY(hipStreamSynchronize(st));
    std::memset(out, 0, sizeof *out);
    for (int k = 0; k < 3; ++k) {
        out->com[k] = d.v[k];
        out->P[k] = d.v[3 + k];
        out->L[k] = d.v[6 + k];
    }
    out->KE = d.v[9];
    out->PE = with_pe ? d.v[10] : 0.0;
    out->E = out->KE + out->PE;
    out->D2 = ds.D2;
    out->R2 = ds.R2_0 * ds.D2 / ds.D2_0;
    out->step = ds.step;
    out->n_past_L1 = ds.n_past;
    out->cross_fwd = ds.fwd;
    out->cross_bwd = ds.bwd;
    out->growth_stopped = ds.growth_stopped;
    out->nonfinite = ds.nonfinite;
    return ds.nonfinite ? NB_E_NONFINITE : NB_OK;
}

int nb_retention(nb_system *s, int32_t *n_past, int32_t *n_bound, void *stream)
{
    if (!s || !n_past || !n_bound || !on_own_device(s)) return NB_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    NB_TRY(launch_retention(single_launch(s), s->p.mode, st));
    DevState ds;
    NB_TRY(hipMemcpyAsync(&ds, s->d_state, sizeof ds, hipMemcpyDeviceToHost, st));
    NB_TRY(hipStreamSynchronize(st));
    *n_past = ds.ret_past;
    *n_bound = ds.ret_bound;
    return NB_OK;
}

int nb_nonfinite_async(nb_system *const *sys, int32_t n_sys, int32_t *out_host, void *stream)
{
    if (!out_host) return NB_E_INVAL;
    // the same checks as a step over these systems: distinct, each on its own (current) device
    if (!sys || n_sys < 1) return NB_E_INVAL;
    for (int k = 0; k < n_sys; ++k) {
        if (!sys[k] || !on_own_device(sys[k])) return NB_E_INVAL;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    for (int k = 0; k < n_sys; ++k) {
        NB_TRY(hipMemcpyAsync(out_host + k, &sys[k]->d_state->nonfinite, sizeof(int32_t),
                              hipMemcpyDeviceToHost, st));
    }
    return NB_OK;
}

int nb_l1_log(nb_system *s, int32_t *out_host, int32_t max_steps, int32_t *n_out, void *stream)
{
    if (!s || !n_out || max_steps < 0 || (max_steps > 0 && !out_host) || !on_own_device(s))
        return NB_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<int32_t> log((size_t)L1_LOG_CAP * 4);
    DevState ds;
    NB_TRY(hipMemcpyAsync(log.data(), s->desc.l1_log, log.size() * sizeof(int32_t),
                          hipMemcpyDeviceToHost, st));
    NB_TRY(hipMemcpyAsync(&ds, s->d_state, sizeof ds, hipMemcpyDeviceToHost, st));
    NB_TRY(hipStreamSynchronize(st));
    const int64_t last = ds.step;
    const int64_t avail = std::min<int64_t>(last, L1_LOG_CAP);
    const int64_t rows = std::min<int64_t>(avail, max_steps);
    for (int64_t r = 0; r < rows; ++r) {
        const int64_t step = last - rows + 1 + r;
        const int32_t *src = &log[4 * (size_t)(step % L1_LOG_CAP)];
        std::memcpy(out_host + 4 * r, src, 4 * sizeof(int32_t));
    }
    *n_out = (int32_t)rows;
    return NB_OK;
}

int nb_resort(nb_system *s, void *stream)
{
    if (!s || !on_own_device(s)) return NB_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<int32_t> perm;
    const int rc = upload_sorted_order(&s->p, &s->b, s->cfg, s->desc.perm, st, perm);
    if (rc != NB_OK) return rc;
    NB_TRY(hipStreamSynchronize(st));  // perm is read by the upload until it completes
    return NB_OK;
}

int nb_sorted_order(nb_system *s, int32_t *out_host, int64_t cap, int64_t *n_out, void *stream)
{
    if (!s || !n_out || cap < 0 || (cap > 0 && !out_host) || !on_own_device(s)) return NB_E_INVAL;
    const int64_t total = s->cfg.nalloc;
    *n_out = total;
    const int64_t k = std::min(cap, total);
    if (k == 0) return NB_OK;
    hipStream_t st = static_cast<hipStream_t>(stream);
    NB_TRY(hipMemcpyAsync(out_host, s->desc.perm, (size_t)k * sizeof(int32_t),
                          hipMemcpyDeviceToHost, st));
    NB_TRY(hipStreamSynchronize(st));
    return NB_OK;
}

int nb_valu_probe(int32_t op, int32_t blocks, int32_t iters, void *sink, void *stream,
                  double *ms, int64_t *lane_ops, double *clock_ratio)
{
    if (op < 0 || op > 8 || blocks < 1 || iters < 1 || !sink || !ms || !lane_ops || !clock_ratio)
        return NB_E_INVAL;
    int device = -1;
    NB_TRY(hipGetDevice(&device));
    if (!device_buffer(sink, device)) return NB_E_INVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess) return NB_E_HIP;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return NB_E_HIP;
    }
    int rc = NB_OK;
    float t = 0.f;
    if (hipEventRecord(a, st) != hipSuccess ||
        launch_valu_probe(op, static_cast<float *>(sink), blocks, iters, st) != hipSuccess ||
        hipEventRecord(b, st) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
        hipEventElapsedTime(&t, a, b) != hipSuccess)
        rc = NB_E_HIP;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc != NB_OK) return rc;
    *ms = t;
    uint64_t clk[2] = {0, 0};
    NB_TRY(hipMemcpy(clk, static_cast<char *>(sink) + 8, sizeof clk, hipMemcpyDeviceToHost));
    *clock_ratio = clk[1] > 0 ? (double)clk[0] / (double)clk[1] : 0.0;
    // eight chains per lane; op 3 issues three FMAs and one reciprocal square root per chain
    // step, op 8 a multiply and an add
    *lane_ops = (int64_t)blocks * 256 * (int64_t)iters * 8 * (op == 3 ? 4 : (op == 8 ? 2 : 1));
    return NB_OK;
}

int nb_timing_enable(int32_t on)
{
    std::lock_guard<std::mutex> g(g_timing.mu);
    g_timing.on = on != 0;
    return NB_OK;
}

int nb_timing_read(double *total_ms, int64_t *launches)
{
    std::lock_guard<std::mutex> g(g_timing.mu);
    int rc = NB_OK;
    for (auto &ev : g_timing.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(ev.second) != hipSuccess ||
            hipEventElapsedTime(&ms, ev.first, ev.second) != hipSuccess) {
            rc = NB_E_HIP;
        } else {
            g_timing.total_ms += ms;
            g_timing.launches += 1;
        }
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    g_timing.pending.clear();
    if (total_ms) *total_ms = g_timing.total_ms;
    if (launches) *launches = g_timing.launches;
    return rc;
}

int nb_timing_reset(void)
{
    double t;
    int64_t n;
    int rc = nb_timing_read(&t, &n);
    std::lock_guard<std::mutex> g(g_timing.mu);
    g_timing.total_ms = 0.0;
    g_timing.launches = 0;
    return rc;
}

void nb_destroy(nb_system *s) { delete s; }

}  // extern "C"
