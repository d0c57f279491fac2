// nb_internal.h -- device-side data structures shared by the HIP kernels and the C++ runtime of
// libnbody. Not part of the public ABI (include/nbody.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nbk {

// Waves per SIMD asked of the compiler (its vector-register cap) for the force kernels, by kernel
// and band height (1, 2, 4 tile rows per lane): measured choices.
constexpr int PLAIN_WAVES = 8;
constexpr int SYM_WAVES[3] = {6, 5, 4};
constexpr int SYM_PAPER_WAVES[3] = {6, 5, 4};  // eqs. (4)-(6): at one row a few per-tile values
                                               // spill, none inside the pair loop; faster than 5
                                               // waves without spills

constexpr int BT = 256;          // threads per block, every kernel
constexpr int TJ = 256;          // j elements staged in LDS per tile (one per thread)
constexpr int MAX_BAND = 4;      // tallest band of the FP32 symmetric kernel (tile rows per lane)
constexpr int RED_STRIDE = 32;   // doubles per O(N)-unit partial record
constexpr int RED_STEP = 0;      // record slots [0, 16): per-step sums (COMs, flags, L1 counts)
constexpr int RED_DIAG = 16;     // record slots [16, 32): diagnostics sums
constexpr int RED_RET = 26;      // record slots [26, 31): retention sums (after the diagnostics)
constexpr int L1_LOG_CAP = 4096; // rows of the per-step L1 log
// Position of padding slots in the sorted layout. A padding element at 1e18 (FP32) or 1e150
// (FP64) gives w^3 below the type's smallest subnormal, so its contribution is exactly 0.
constexpr float SENTINEL_F32 = 1.0e18f;
constexpr double SENTINEL_F64 = 1.0e150;
constexpr float FAR_MARGIN = 2.0e-5f;  // relative margin on D^2 for the far-tile test

// Pair classes: 0 = star 1 with star 1, 1 = across the stars, 2 = star 2 with star 2.

// Per-system state that lives in device memory (first bytes of the system's workspace).
struct alignas(16) DevState {
    // FP64 masters
    double D1, D2, D2_0, R2_0, rL_a, growth_rate;
    double G, m, dt, xi_l1;
    double c1d[3], c2d[3];   // 11 / D^3 and 10 / D^2 per pair class
    double gm_d, h_d;        // G m and dt / 2
    // L1 plane of the current step
    double com1[3], com2[3], e[3], xi_cut;
    // FP32 copies used by the FP32 kernels
    float c1f[3], c2f[3];
    float far2f[3];          // (1 + FAR_MARGIN) D^2 per pair class
    float gm_f, h_f, dt_f, pad_f;
    int64_t step;
    int32_t growth_on, growth_stopped;
    int32_t n_past, fwd, bwd, nonfinite;
    int32_t plane_ok, law;
    // element law of eqs. (4)-(6), with the overlap volume written as (pi / 12) (D - r)^2
    // (r + 2D), D = 2R the pair's element diameter: gc = gamma pi / (12 G m^2) and
    // gcb = beta gc scale it for converging and separating pairs; eps softens the attraction
    double gamma, beta, leps_d, lgc_d, lgcb_d;
    float lD_f[3];           // D per pair class (follows the donor growth)
    float leps_f, lgc_f, lgcb_f, pad_l;
    // accretor-side retention (nb_retention): star 1's mean velocity and the two counts
    double v1[3];
    int32_t ret_past, ret_bound;
};

struct DiagOut {
    double v[16];  // com[3], P[3], L[3], KE, PE
};

// One entry of a launch's segment table.
//
// The force kernels work on a sorted copy of the positions: each star's elements in Morton
// order of their initial positions, star 1 in slots [0, n1), star 2 from slot p1 =
// roundup(n1, TJ), both padded with sentinels to a multiple of TJ (npad slots in all, nalloc
// allocated). Every j tile then lies inside one star, and each tile's bounding box lets the
// kernel skip the contact test for tiles that are provably farther than D.
struct SysDesc {
    void *x, *y, *z, *vx, *vy, *vz, *ax, *ay, *az;
    int8_t *side;
    DevState *st;
    void *xs, *ys, *zs;   // sorted positions, nalloc slots
    int32_t *perm;        // nalloc: element index of each sorted slot, -1 for padding
    float *tbox;          // ntiles * 8: min xyz, pad, max xyz, pad of each j tile
    void *part;         // j-split partial sums, nsplit * 3 * nalloc values (nsplit > 1 only)
    double *red;        // n_ounits * RED_STRIDE doubles
    double *pe_part;    // n_peunits doubles
    int32_t *l1_log;    // L1_LOG_CAP * 4 int32
    DiagOut *diag;
    int32_t n, n1;
    int32_t nsplit, jchunk;     // j chunks per i-block and chunk length (multiple of TJ)
    int32_t iblock, n_iblocks;  // i elements per block (BT * ki) and block count
    int32_t n_units, n_ounits;  // force units (n_iblocks * nsplit) and O(N) units (ceil(n / BT))
    int32_t unit_begin, ounit_begin;  // prefix offsets in the launch's segment table
    int32_t n_peunits, pad;
    int32_t npad, p1, nalloc, ntiles;  // sorted layout (see above)
    int32_t tunit_begin, pad2;         // prefix offset of this system's tiles in the launch
    // symmetric kernels (FP32 Kahan and FP64 modes): work units (band g, chunk c) and reaction
    // partials, per band g the tiles after its first row: 3 * TJ * sum_g (T - rows g - 1)
    int32_t *units;       // n_units pairs (g, c)
    float *react;         // (double * in the FP64 mode)
    int32_t ch, sym;      // tiles per chunk; 1 when the symmetric kernel is used
    void *vxs, *vys, *vzs;  // sorted velocities (eqs. 4-6 only; null otherwise)
    int32_t law, rows;    // element law; tile rows per band (1 in the FP64 mode)
};

// Kernel argument describing one launch over a segment table.
struct Launch {
    const SysDesc *sys;
    int32_t n_sys;
    int32_t unit_base;     // first force unit of this launch (a force launch may cover a range)
    int32_t total_units;   // force units: (i-block, j chunk) pairs; the launch ends before this
    int32_t total_ounits;  // O(N) units: 256 elements in element order
    int32_t total_tunits;  // tiles: 256 slots in sorted order
    int32_t law;           // element law of every system in the launch (NB_LAW_*)
    // FP32 Kahan mode: the table is ordered by band height; systems with bands of 1, 2 and 4 rows
    // own the force units [0, band_end[0]), [band_end[0], band_end[1]), [band_end[1], band_end[2])
    int32_t band_end[3];
};

// Segment-table entries written on the device from the systems' own one-entry tables (each
// system's SysDesc in its workspace), with this launch's prefix offsets: up to TABLE_CHUNK
// systems per kernel launch, passed by value as a kernel argument.
constexpr int TABLE_CHUNK = 64;
struct TableChunk {
    const SysDesc *src[TABLE_CHUNK];
    int32_t unit_begin[TABLE_CHUNK], ounit_begin[TABLE_CHUNK], tunit_begin[TABLE_CHUNK];
    int32_t first, count;  // entries [first, first + count) of the destination table
};

// Host-side launchers (nb_kernels.hip). All return the HIP status of the launch.
hipError_t launch_init_state(DevState *st, const DevState &init, hipStream_t s);
hipError_t launch_fill_sorted(void *xs, void *ys, void *zs, int nalloc, int mode, bool sentinel,
                              hipStream_t s);
hipError_t launch_gather(const Launch &L, int mode, hipStream_t s);
hipError_t launch_forces(const Launch &L, int mode, int max_blocks, hipStream_t s);
hipError_t launch_combine(const Launch &L, int mode, hipStream_t s);
hipError_t launch_kick_drift(const Launch &L, int mode, hipStream_t s);
hipError_t launch_kick_stats(const Launch &L, int mode, int do_kick, hipStream_t s);
hipError_t launch_finalize_step(const Launch &L, int do_growth, hipStream_t s);
hipError_t launch_l1_classify(const Launch &L, int mode, int init, hipStream_t s);
hipError_t launch_finalize_l1(const Launch &L, int init, hipStream_t s);
hipError_t launch_diag(const Launch &L, int mode, int with_pe, hipStream_t s);
hipError_t launch_retention(const Launch &L, int mode, hipStream_t s);
hipError_t launch_valu_probe(int op, float *sink, int blocks, int iters, hipStream_t s);
hipError_t launch_copy_table(SysDesc *dst, const TableChunk &c, hipStream_t s);

}  // namespace nbk
