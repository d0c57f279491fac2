// nb_runtime.cpp -- C ABI of libnbody (include/nbody.h): parameter checks, workspace layout,
// the segment tables that drive every launch, the step sequence and the read-backs.
#include "nbody.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "nb_internal.h"

using namespace nbk;

namespace {

constexpr size_t ALIGN = 256;

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
};

struct Override {
    int64_t lo, hi;
    int nsplit;
};

std::mutex g_cfg_mu;
std::vector<Override> g_overrides;

TileCfg tile_config(int64_t n, int mode)
{
    TileCfg c{};
    c.ki = mode == NB_FP64 ? KI64 : KI32;
    c.iblock = BT * c.ki;
    c.n_iblocks = (int)((n + c.iblock - 1) / c.iblock);
    c.n_ounits = (int)((n + BT - 1) / BT);
    int ns = 1;
    if (mode != NB_FP32_PLAIN && n > 0) {
        // aim at >= 2048 work units (8 blocks per CU on 256 CUs) with chunks of >= 2048 j
        const int want = (2048 + c.n_iblocks - 1) / c.n_iblocks;
        const int most = (int)std::max<int64_t>(1, n / 2048);
        ns = std::max(1, std::min(want, most));
        std::lock_guard<std::mutex> g(g_cfg_mu);
        for (const Override &o : g_overrides) {
            if (n >= o.lo && n <= o.hi) ns = std::max(1, o.nsplit);
        }
    }
    int64_t chunk = n > 0 ? (n + ns - 1) / ns : TJ;
    chunk = (chunk + TJ - 1) / TJ * TJ;
    c.jchunk = (int)chunk;
    c.nsplit = n > 0 ? (int)((n + chunk - 1) / chunk) : 1;
    c.n_units = c.n_iblocks * c.nsplit;
    return c;
}

struct Layout {
    size_t state, desc, diag, red, pe, log, part, total;
};

Layout layout_for(int64_t n, int mode, const TileCfg &c)
{
    Layout L{};
    size_t off = 0;
    L.state = off;
    off = align_up(off + sizeof(DevState), ALIGN);
    L.desc = off;
    off = align_up(off + sizeof(SysDesc), ALIGN);
    L.diag = off;
    off = align_up(off + sizeof(DiagOut), ALIGN);
    L.red = off;
    off = align_up(off + (size_t)std::max(c.n_ounits, 1) * RED_STRIDE * sizeof(double), ALIGN);
    L.pe = off;
    off = align_up(off + (size_t)std::max(c.n_ounits, 1) * sizeof(double), ALIGN);
    L.log = off;
    off = align_up(off + (size_t)L1_LOG_CAP * 4 * sizeof(int32_t), ALIGN);
    L.part = off;
    if (c.nsplit > 1) {
        const size_t elem = mode == NB_FP64 ? sizeof(double) : sizeof(float);
        off = align_up(off + (size_t)c.nsplit * 3 * (size_t)n * elem, ALIGN);
    }
    L.total = off;
    return L;
}

bool params_ok(const nb_params *p)
{
    if (!p) return false;
    if (p->n < 0 || p->n >= (int64_t(1) << 31)) return false;
    if (p->n1 < 0 || p->n1 > p->n) return false;
    if (p->mode != NB_FP32_PLAIN && p->mode != NB_FP32_KAHAN && p->mode != NB_FP64) return false;
    auto pos = [](double v) { return std::isfinite(v) && v > 0.0; };
    if (!std::isfinite(p->G) || p->G < 0.0) return false;
    if (!pos(p->m) || !std::isfinite(p->dt)) return false;
    if (!pos(p->D1) || !pos(p->D2) || !pos(p->q) || !pos(p->a) || !pos(p->R2_0)) return false;
    if (!std::isfinite(p->growth_rate) || p->growth_rate < 0.0) return false;
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
struct BatchTable {
    int device = -1;
    SysDesc *d = nullptr;
    SysDesc *h = nullptr;  // pinned staging
    int cap = 0;
    std::vector<SysDesc> last;
};
std::mutex g_batch_mu;
std::vector<BatchTable> g_batches;

}  // namespace

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

int launch_force_timed(const Launch &L, int mode, hipStream_t st, bool need_combine)
{
    hipEvent_t a = nullptr, b = nullptr;
    bool timed = false;
    {
        std::lock_guard<std::mutex> g(g_timing.mu);
        timed = g_timing.on;
    }
    if (timed) {
        NB_TRY(hipEventCreate(&a));
        NB_TRY(hipEventCreate(&b));
        NB_TRY(hipEventRecord(a, st));
    }
    NB_TRY(launch_forces(L, mode, st));
    if (timed) {
        NB_TRY(hipEventRecord(b, st));
        std::lock_guard<std::mutex> g(g_timing.mu);
        g_timing.pending.emplace_back(a, b);
    }
    if (need_combine) NB_TRY(launch_combine(L, mode, st));
    return NB_OK;
}

int run_steps(const Launch &L, int mode, int n_steps, bool need_combine, hipStream_t st)
{
    for (int k = 0; k < n_steps; ++k) {
        NB_TRY(launch_kick_drift(L, mode, st));
        int rc = launch_force_timed(L, mode, st, need_combine);
        if (rc != NB_OK) return rc;
        NB_TRY(launch_kick_stats(L, mode, 1, st));
        NB_TRY(launch_finalize_step(L, 1, st));
        NB_TRY(launch_l1_classify(L, mode, 0, st));
        NB_TRY(launch_finalize_l1(L, 0, st));
    }
    return NB_OK;
}

Launch single_launch(const nb_system *s)
{
    Launch L{};
    L.sys = s->d_desc;
    L.n_sys = 1;
    L.total_units = s->cfg.n_units;
    L.total_ounits = s->cfg.n_ounits;
    return L;
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

}  // namespace

extern "C" {

int nb_version(void) { return 1; }

const char *nb_strerror(int status)
{
    switch (status) {
    case NB_OK: return "ok";
    case NB_E_INVAL: return "invalid argument";
    case NB_E_HIP: return "HIP runtime error";
    case NB_E_NOMEM: return "workspace too small or table allocation failed";
    case NB_E_NONFINITE: return "non-finite position or velocity";
    case NB_E_MISMATCH: return "systems of different modes in one call";
    default: return "unknown status";
    }
}

int nb_tile_config(int64_t n, int32_t mode, int32_t *ki, int32_t *nsplit, int32_t *iblock,
                   int32_t *jchunk)
{
    if (n < 0 || n >= (int64_t(1) << 31)) return NB_E_INVAL;
    if (mode != NB_FP32_PLAIN && mode != NB_FP32_KAHAN && mode != NB_FP64) return NB_E_INVAL;
    TileCfg c = tile_config(n, mode);
    if (ki) *ki = c.ki;
    if (nsplit) *nsplit = c.nsplit;
    if (iblock) *iblock = c.iblock;
    if (jchunk) *jchunk = c.jchunk;
    return NB_OK;
}

int nb_tile_override(int64_t n_lo, int64_t n_hi, int32_t nsplit)
{
    if (n_lo < 0 || n_hi < n_lo || nsplit < 0 || nsplit > 4096) return NB_E_INVAL;
    std::lock_guard<std::mutex> g(g_cfg_mu);
    g_overrides.erase(std::remove_if(g_overrides.begin(), g_overrides.end(),
                                     [&](const Override &o) { return o.lo == n_lo && o.hi == n_hi; }),
                      g_overrides.end());
    if (nsplit > 0) g_overrides.push_back({n_lo, n_hi, nsplit});
    return NB_OK;
}

int nb_scratch_bytes(const nb_params *p, size_t *out)
{
    if (!params_ok(p) || !out) return NB_E_INVAL;
    TileCfg c = tile_config(p->n, p->mode);
    *out = layout_for(p->n, p->mode, c).total;
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
    TileCfg cfg = tile_config(p->n, p->mode);
    Layout lay = layout_for(p->n, p->mode, cfg);
    if (b->scratch_bytes < lay.total) return NB_E_NOMEM;

    nb_system *s = new (std::nothrow) nb_system();
    if (!s) return NB_E_NOMEM;
    s->p = *p;
    s->b = *b;
    s->cfg = cfg;
    s->lay = lay;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return NB_E_HIP;
    }
    char *base = static_cast<char *>(b->scratch);
    s->d_state = reinterpret_cast<DevState *>(base + lay.state);
    s->d_desc = reinterpret_cast<SysDesc *>(base + lay.desc);
    s->d_diag = reinterpret_cast<DiagOut *>(base + lay.diag);

    SysDesc &d = s->desc;
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
    d.st = s->d_state;
    d.part = cfg.nsplit > 1 ? base + lay.part : nullptr;
    d.red = reinterpret_cast<double *>(base + lay.red);
    d.pe_part = reinterpret_cast<double *>(base + lay.pe);
    d.l1_log = reinterpret_cast<int32_t *>(base + lay.log);
    d.diag = s->d_diag;
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

    DevState init;
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
    }
    init.gm_d = p->G * p->m;
    init.h_d = 0.5 * p->dt;
    init.gm_f = (float)init.gm_d;
    init.h_f = (float)init.h_d;
    init.dt_f = (float)p->dt;
    init.growth_on = p->growth_on ? 1 : 0;

    hipStream_t st = static_cast<hipStream_t>(stream);
    int rc = NB_OK;
    do {
        if (launch_init_state(s->d_state, init, st) != hipSuccess) { rc = NB_E_HIP; break; }
        if (hipMemcpyAsync(s->d_desc, &s->desc, sizeof(SysDesc), hipMemcpyHostToDevice, st) !=
            hipSuccess) { rc = NB_E_HIP; break; }
        Launch L = single_launch(s);
        if (launch_kick_stats(L, p->mode, 0, st) != hipSuccess) { rc = NB_E_HIP; break; }
        if (launch_finalize_step(L, 0, st) != hipSuccess) { rc = NB_E_HIP; break; }
        if (launch_l1_classify(L, p->mode, 1, st) != hipSuccess) { rc = NB_E_HIP; break; }
        if (launch_finalize_l1(L, 1, st) != hipSuccess) { rc = NB_E_HIP; break; }
        if (launch_forces(L, p->mode, st) != hipSuccess) { rc = NB_E_HIP; break; }
        if (cfg.nsplit > 1 && launch_combine(L, p->mode, st) != hipSuccess) { rc = NB_E_HIP; break; }
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
    if (!s) return NB_E_INVAL;
    return launch_force_timed(single_launch(s), s->p.mode, static_cast<hipStream_t>(stream),
                              s->cfg.nsplit > 1);
}

int nb_step(nb_system *const *sys, int32_t n_sys, int32_t n_steps, void *stream)
{
    if (!sys || n_sys < 1 || n_steps < 0) return NB_E_INVAL;
    for (int k = 0; k < n_sys; ++k) {
        if (!sys[k]) return NB_E_INVAL;
        if (sys[k]->p.mode != sys[0]->p.mode) return NB_E_MISMATCH;
        for (int j = 0; j < k; ++j) {
            if (sys[j] == sys[k]) return NB_E_INVAL;
        }
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int mode = sys[0]->p.mode;
    if (n_sys == 1) {
        return run_steps(single_launch(sys[0]), mode, n_steps, sys[0]->cfg.nsplit > 1, st);
    }
    int device = 0;
    NB_TRY(hipGetDevice(&device));
    std::lock_guard<std::mutex> g(g_batch_mu);
    BatchTable *bt = nullptr;
    for (BatchTable &t : g_batches) {
        if (t.device == device) bt = &t;
    }
    if (!bt) {
        g_batches.emplace_back();
        bt = &g_batches.back();
        bt->device = device;
    }
    std::vector<SysDesc> table(n_sys);
    int units = 0, ounits = 0;
    bool combine = false;
    for (int k = 0; k < n_sys; ++k) {
        table[k] = sys[k]->desc;
        table[k].unit_begin = units;
        table[k].ounit_begin = ounits;
        units += sys[k]->cfg.n_units;
        ounits += sys[k]->cfg.n_ounits;
        combine = combine || sys[k]->cfg.nsplit > 1;
    }
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
    Launch L{};
    L.sys = bt->d;
    L.n_sys = n_sys;
    L.total_units = units;
    L.total_ounits = ounits;
    return run_steps(L, mode, n_steps, combine, st);
}

int nb_diagnostics(nb_system *s, int32_t with_pe, nb_diag *out, void *stream)
{
    if (!s || !out) return NB_E_INVAL;
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

int nb_l1_log(nb_system *s, int32_t *out_host, int32_t max_steps, int32_t *n_out, void *stream)
{
    if (!s || !n_out || max_steps < 0 || (max_steps > 0 && !out_host)) return NB_E_INVAL;
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
