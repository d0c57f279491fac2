/*
 * nbody.h -- C ABI of libnbody, the MI355X (gfx950) library for the gravity-centred binary-star
 * element model of Goderya et al., "N-body simulation of binary star mass transfer using NVIDIA
 * GPUs".
 *
 * The model (Methodology section): a star is a ball of N elements of one common mass and one
 * common diameter; every element's motion comes only from the sum of all pairwise
 * element-element interactions. Elements always attract; elements in contact also repel. Two
 * element laws are implemented (nb_params.law). The default is a conservative contact law
 *     f(r) = G m^2 / r^2                       r >= D
 *     f(r) = G m^2 r / D^3 - K (1 - r/D)       r <  D,   K = 10 G m^2 / D^2
 * (f > 0 attracts), with D the element diameter of the pair: D1 inside star 1, D2 inside star 2,
 * (D1 + D2)/2 across; the other is the paper's own law, eqs. (4)-(6), described at nb_params.
 * Time stepping is the leap-frog integrator (Methodology) in kick-drift-kick
 * form. The donor (star 2) expands by growing its element diameter until its radius reaches the
 * Roche-lobe radius of eq. (3); elements of the donor crossing the plane through L1 are counted
 * every step.
 *
 * Conventions shared by every entry point
 *  - Status: 0 = NB_OK; negative values are errors (nb_strerror names them). No exception or
 *    signal crosses the ABI; invalid arguments are reported, never dereferenced.
 *  - Device memory is owned by the caller (for example PyTorch tensors, passed as data
 *    pointers). The library never frees it. It keeps only host-side structs and HIP events.
 *    Multi-system steps additionally use one small library-owned device table (segment table).
 *  - Streams are `hipStream_t` values passed as `void *` (NULL = the default stream). Every call
 *    on a system is ordered on the stream it is given; calls on different systems may run
 *    concurrently on different streams.
 *  - Layout: structure of arrays. x, y, z, vx, vy, vz, ax, ay, az are n contiguous elements each
 *    (float for the FP32 modes, double for NB_FP64). Star 1 (the accretor, mass 1) owns indices
 *    [0, n1), star 2 (the donor, mass q) owns [n1, n).
 *  - A system's buffers must not be used by another system at the same time.
 *  - A system belongs to the device that is current when nb_create runs (its buffers must be on
 *    that device). Every later call naming the system must be made with that device current;
 *    otherwise the call returns NB_E_INVAL and queues nothing.
 */
#ifndef NBODY_H
#define NBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define NB_OK 0
#define NB_E_INVAL (-1)     /* bad argument: null pointer, size, mode, misaligned buffer */
#define NB_E_HIP (-2)       /* a HIP runtime call failed */
#define NB_E_NOMEM (-3)     /* scratch smaller than nb_scratch_bytes, a library table failed, or
                               the work split of a huge system would overflow int32 units */
#define NB_E_NONFINITE (-4) /* a position or velocity became NaN or infinite */
#define NB_E_MISMATCH (-5)  /* systems of different precision modes or element laws in one
                               multi-system call */
#define NB_E_LIMIT (-6)     /* more systems than nb_step_static's fixed table holds */

/* element laws */
#define NB_LAW_CONTACT 0 /* conservative contact law (default; see the header comment) */
#define NB_LAW_PAPER 1   /* eqs. (4)-(6): G m^2/(r+eps)^2 minus gamma V(r) in contact, times beta
                            while the pair does not converge (FP32 Kahan and FP64 modes only) */

/* precision modes of the force evaluation */
#define NB_FP32_PLAIN 0 /* FP32, one running sum per element over all j in order */
#define NB_FP32_KAHAN 1 /* FP32 tile partials, compensated (Kahan) sum across tiles */
#define NB_FP64 2       /* FP64 throughout (reference mode) */

typedef struct nb_system nb_system; /* opaque, host-side, owned by the library */
typedef struct nb_graph nb_graph;   /* opaque: a captured multi-step launch sequence */

/* Physical and numerical parameters of one two-star system. */
typedef struct {
    int64_t n;           /* elements, 0 <= n < 2^30 */
    int64_t n1;          /* elements of star 1, 0 <= n1 <= n */
    double G;            /* gravitational constant */
    double m;            /* common element mass */
    double dt;           /* leap-frog time step */
    double D1, D2;       /* element diameters of star 1 and star 2 at t = 0 (> 0) */
    double q;            /* mass ratio m2/m1 used by eq. (3) and for L1 (> 0) */
    double a;            /* nominal separation; the donor stops growing at r_L(q) a */
    double R2_0;         /* donor radius at t = 0; its radius is R2_0 D2 / D2(t=0) */
    double growth_rate;  /* D2 <- D2 (1 + growth_rate) per step while growing */
    int32_t growth_on;   /* 0: the donor never grows */
    int32_t mode;        /* NB_FP32_PLAIN, NB_FP32_KAHAN or NB_FP64 */
    int32_t law;         /* NB_LAW_CONTACT or NB_LAW_PAPER */
    int32_t pad;
    /* NB_LAW_PAPER only (eqs. 4-6). Pair radius R = D_ij / 2; contact means r < 2R; V(r) =
     * pi (4/3 R^3 - R^2 r + r^3/12) is the overlap volume of two spheres of radius R; the pair
     * converges when (v_j - v_i).(r_j - r_i) < 0, and the force law then reads
     *   f(r) = G m^2 / (r + eps)^2 - g V(r),  g = gamma (converging) or gamma beta (otherwise).
     * The force seen in a leap-frog step uses the half-step velocities. Requires G > 0. */
    double eps;          /* softening length (>= 0) */
    double gamma;        /* repulsion per unit overlap volume (>= 0) */
    double beta;         /* reduction factor while not converging (0 <= beta <= 1) */
} nb_params;

/* Device buffers of one system (caller-owned, see the conventions above). */
typedef struct {
    void *x, *y, *z;     /* positions (inout), n elements each */
    void *vx, *vy, *vz;  /* velocities (inout) */
    void *ax, *ay, *az;  /* accelerations (out; valid after nb_create) */
    void *side;          /* n bytes: per-element L1 side flag (library-written) */
    void *scratch;       /* workspace, 256-byte aligned, at least nb_scratch_bytes() */
    size_t scratch_bytes;
} nb_buffers;

/* FP64 diagnostics of one system, read back by nb_diagnostics. */
typedef struct {
    double com[3];       /* centre of mass */
    double P[3];         /* linear momentum, sum m v */
    double L[3];         /* angular momentum about the origin, sum m r x v */
    double KE, PE, E;    /* kinetic, potential (0 unless requested) and total energy */
    double D2, R2;       /* current donor element diameter and nominal donor radius */
    int64_t step;        /* completed leap-frog steps */
    int32_t n_past_L1;   /* donor elements past the L1 plane after the last step */
    int32_t cross_fwd;   /* donor elements that crossed toward the accretor in the last step */
    int32_t cross_bwd;   /* donor elements that crossed back in the last step */
    int32_t growth_stopped; /* 1 once the donor has reached its Roche lobe */
    int32_t nonfinite;   /* elements with a non-finite position or velocity (last step) */
    int32_t pad;
} nb_diag;

/* Bytes of device workspace (`scratch`) a system with these parameters needs. Depends on n, n1,
 * mode and law, and on the work split installed for n (nb_tile_override). Returns NB_E_INVAL for
 * invalid parameters. */
int nb_scratch_bytes(const nb_params *p, size_t *out);

/* Validates p and b (every buffer must be device or managed memory of the current device; host
 * memory, pinned or not, is NB_E_INVAL), lays out the workspace, initialises the device state (FP64 diameters and
 * growth flag, derived FP32 force constants), sets every donor element's L1 side from the
 * initial positions and evaluates the initial accelerations a(x0) into ax/ay/az, all ordered on
 * `stream`, which it synchronises before returning. On success *out owns a new handle (free with
 * nb_destroy). On error *out is NULL and nothing needs freeing. */
int nb_create(const nb_params *p, const nb_buffers *b, void *stream, nb_system **out);

/* One all-pairs evaluation (Methodology: the sum of every pairwise interaction):
 * a_i = sum_{j != i} (f(r_ij) / m) (r_j - r_i) / r_ij with the current diameters, written to
 * ax/ay/az. Asynchronous on `stream`. */
int nb_forces(nb_system *s, void *stream);

/* Advances every listed system by n_steps leap-frog steps (Methodology: leap-frog integrator):
 * v += a dt/2; x += v dt; a = F(x); v += a dt/2; then the donor growth update (diameter grows by
 * (1 + growth_rate) while R2_0 D2/D2_0 <= r_L(q) a, eq. 3; the first step that finds it larger
 * stops growth for good) and the L1 count. n_sys = 1 steps one system alone. With n_sys > 1 all
 * systems advance together: each kernel of a step is one launch over all systems' work (a
 * segment table), and each system's results are bitwise the same as when it runs alone. The
 * systems must be distinct (NB_E_INVAL) and share one mode and one element law (NB_E_MISMATCH);
 * a batch whose summed work units, elements or tiles exceed int32 returns NB_E_NOMEM.
 * The library keeps the segment table of the last multi-system call per device and stream;
 * calls on one stream are ordered, calls on different streams do not share a table.
 * Asynchronous on `stream`. */
int nb_step(nb_system *const *sys, int32_t n_sys, int32_t n_steps, void *stream);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): nb_step with the multi-system segment table kept in a fixed array of
 * NB_STATIC_MAX_SYS entries in each GPU's memory (76 KB, held by the library until the
 * process ends) instead of a table the library allocates. The same work and bitwise the same
 * results as nb_step(sys, n_sys, n_steps, stream); any n_sys from 1 to NB_STATIC_MAX_SYS.
 * Allocates no device or host memory and synchronises nothing: the table is rewritten on the
 * device by a small kernel queued on `stream` ahead of the steps, from each system's own
 * one-entry table. Every call on a GPU shares that GPU's one table, which keeps the last call's
 * contents: calls that overlap on one GPU (on different streams, or from different threads
 * without ordering) race, so order them on one stream. Force-kernel timing (nb_timing_*) does
 * not cover these calls. n_sys > NB_STATIC_MAX_SYS returns NB_E_LIMIT and queues nothing; the
 * other errors are nb_step's. */
#define NB_STATIC_MAX_SYS 256
int nb_step_static(nb_system *const *sys, int32_t n_sys, int32_t n_steps, void *stream);

/* Captures n_steps steps of the listed systems (exactly the work nb_step would queue for them)
 * into a HIP graph with its own copy of the segment table, for replay with nb_graph_launch. The
 * table upload and the capture run on a private stream: nothing executes and nothing is queued
 * on `stream` (kept for symmetry with the other calls), so work already queued anywhere keeps
 * running. The graph refers to the systems' buffers: it must be destroyed before any of them
 * is. Force-kernel timing (nb_timing_*) does not cover graph replays. */
int nb_graph_create(nb_system *const *sys, int32_t n_sys, int32_t n_steps, void *stream,
                    nb_graph **out);

/* Queues one replay (n_steps steps of every system in the graph) on `stream`. Replays and
 * nb_step calls on the same systems must be ordered on one stream. */
int nb_graph_launch(nb_graph *g, void *stream);

/* Frees the graph. No replay of it may still be queued (synchronise its stream first). */
void nb_graph_destroy(nb_graph *g);

/* FP64 diagnostics: centre of mass, momentum, angular momentum, kinetic energy, and with
 * with_pe != 0 the potential energy sum_{i<j} U(r_ij) (U continuous with dU/dr = f; O(n^2)).
 * Synchronises `stream` and fills *out. Returns NB_E_NONFINITE (after filling *out) if the last
 * step saw a non-finite element. */
int nb_diagnostics(nb_system *s, int32_t with_pe, nb_diag *out, void *stream);

/* Health of running systems (Methodology: the element state is advanced step after step; a
 * state that is no longer finite cannot be advanced further): queues on `stream` one copy per
 * listed system of its non-finite element count after its last completed step (the value
 * nb_diagnostics reports as `nonfinite`) into out_host[k] (int32, n_sys entries). Nothing is
 * synchronised: the values are valid once `stream` has passed this call (an event recorded after
 * it, or a stream synchronisation). With pinned host memory the copies are asynchronous; with
 * pageable memory HIP may wait for them. Work that steps the systems on another stream must be
 * ordered before this call by the caller (an event). NB_E_INVAL for null or foreign systems. */
int nb_nonfinite_async(nb_system *const *sys, int32_t n_sys, int32_t *out_host, void *stream);

/* Per-step L1 record of the most recent steps: up to max_steps rows of
 * {step, n_past, forward, backward}, oldest first, into out_host (int32, 4 per row). The library
 * keeps the last NB_L1_LOG_CAP steps. Synchronises `stream`. *n_out receives the row count. */
#define NB_L1_LOG_CAP 4096
int nb_l1_log(nb_system *s, int32_t *out_host, int32_t max_steps, int32_t *n_out, void *stream);

/* Accretor-side retention of the mass that crossed L1 (Methodology: transfer through L1 onto the
 * accretor; eq. 2's geometry). Of the donor elements past the L1 plane of the current state (the
 * plane the last step used), *n_past is their count and *n_bound those bound to the accretor
 * taken as a point mass n1 m at its centre of mass C1, moving with star 1's mean velocity V1:
 * |v - V1|^2 / 2 - G n1 m / |r - C1| < 0. Evaluated in FP64 from the current state (FP32 state
 * promoted in the FP32 modes). Both are 0 when either star is empty. Synchronises `stream`.
 * Returns NB_E_INVAL for null arguments. */
int nb_retention(nb_system *s, int32_t *n_past, int32_t *n_bound, void *stream);

/* Rebuilds the sorted order the force kernels work in from the current positions (each star in
 * Morton order, as nb_create does from the initial ones). Elements drift from their creation-time
 * neighbours as a run goes on and the donor grows; tiles then span more space, more of them need
 * the contact test, and the force evaluation slows. The new order changes the order of the pair
 * sums, so results agree with an unsorted run to rounding, not bitwise; a system re-sorted by a
 * rule that depends only on its own state (for example every K of its own steps) gets the same
 * bits alone and in any batch. Synchronises `stream` (the positions are read back and sorted on
 * the host); work on the system must be ordered before the call. NB_E_INVAL for a null or
 * foreign system. */
int nb_resort(nb_system *s, void *stream);

/* The sorted order the force kernels work in (a diagnostic of the layout, no part of the model):
 * slot k of the sorted copy holds element out_host[k], or -1 for a padding slot. Star 1 fills
 * slots [0, n1) in Morton order of its positions at nb_create, star 2 starts at slot
 * roundup(n1, 256), each star padded to whole tiles of 256 slots. Copies min(cap, total) entries
 * (int32) and sets *n_out to the total slot count. Synchronises `stream`. NB_E_INVAL for null
 * arguments, a negative cap or a foreign system. */
int nb_sorted_order(nb_system *s, int32_t *out_host, int64_t cap, int64_t *n_out, void *stream);

/* Force-kernel timing: while enabled, every force launch issued by nb_forces/nb_step is
 * bracketed by HIP events on its stream. nb_timing_read synchronises those events and returns
 * the summed kernel time (ms) and launch count since the last reset. */
int nb_timing_enable(int32_t on);
int nb_timing_read(double *total_ms, int64_t *launches);
int nb_timing_reset(void);

/* Work split chosen for a system of n elements (n1 in star 1) in a mode and element law: i
 * elements per lane
 * (ki), j chunks per i-block (nsplit; for the symmetric kernels of the FP32 Kahan and FP64 modes,
 * the chunk count of the longest band), i-block size, chunk length (in sorted slots) and band
 * height (rows: tile rows of 256 slots whose pairs one work unit evaluates together, 1, 2 or 4
 * in the FP32 Kahan mode, 1 otherwise; a band of k rows stores 1/k of the reaction partials of
 * single rows). The force kernels work on a copy of the positions sorted per star (Morton order
 * of the initial positions, each star padded to a multiple of 256 slots); results are returned
 * in element order. Depends only on (n, n1, mode, law) and the overrides below. Any output
 * pointer may be NULL. NB_E_INVAL for a bad size, mode or law. */
int nb_tile_config(int64_t n, int64_t n1, int32_t mode, int32_t law, int32_t *ki, int32_t *nsplit,
                   int32_t *iblock, int32_t *jchunk, int32_t *rows);

/* Overrides the split choice of one (mode, law) for systems created afterwards whose n lies in
 * [n_lo, n_hi]: nsplit chunks of the longest band and bands of `rows` tile rows (1, 2 or 4; not 1
 * only in NB_FP32_KAHAN). nsplit = 0 restores the built-in rule (one row per band). Used by the
 * autotuner. NB_E_INVAL for a bad mode, law, range, split or height. */
int nb_tile_override(int64_t n_lo, int64_t n_hi, int32_t mode, int32_t law, int32_t nsplit,
                     int32_t rows);

/* Workspace budget for systems created afterwards (and for nb_scratch_bytes and nb_tile_config):
 * when a system's split, built-in or overridden, would need more than `bytes` of workspace, the
 * split is coarsened step by step, first to taller bands (FP32 Kahan mode: 1, 2, then 4 rows),
 * then to half as many chunks, until the workspace fits or cannot shrink further (the workspace
 * also holds the sorted state, so a budget below that is never met). 0 (the default) sets no
 * budget. The split of a system, and with it the order of its sums, is fixed when it is created.
 * Always NB_OK. */
int nb_set_workspace_budget(size_t bytes);

/* Launch shape of the force kernel for calls issued afterwards (graphs keep the shape they were
 * captured with): 0 (default) launches one workgroup per work unit and lets the hardware
 * dispatcher balance them; blocks > 0 launches at most that many workgroups, each looping over
 * units blockIdx, blockIdx + blocks, ... (a persistent launch). Results are bitwise the same
 * either way: a unit's arithmetic does not depend on which workgroup runs it. */
int nb_set_force_grid(int32_t blocks);

/* Measurement aid for the force kernels' roofline (no part of the model): times one launch of an
 * issue-rate probe of the vector ALU on the current device and stream. Each of blocks x 256 lanes
 * runs iters steps of eight independent dependency chains of one instruction: op 0 v_fma_f32
 * (VOP3), op 1 v_rsq_f32, op 2 v_rcp_f32, op 3 three v_fma_f32 per v_rsq_f32, op 4 v_fmac_f32,
 * op 5 v_add_f32, op 6 v_mul_f32 (VOP2), op 7 v_sub_f32 with a DPP wave-rotation source, op 8
 * one v_mul_f32 and one v_add_f32 in turn. *lane_ops receives the lane-instructions executed, *ms
 * the kernel time (HIP events; synchronises `stream`), *clock_ratio the shader-clock cycles
 * (s_memtime) per tick of the constant-rate counter (s_memrealtime) over block 0's run: with that
 * counter at 100 MHz the shader clock held under the probe's stream is 0.1 x clock_ratio GHz.
 * `sink` is a device buffer of at least 32 bytes that the probe writes (bytes 8..23 hold the two
 * counter spans). NB_E_INVAL for a bad op, size or buffer. */
int nb_valu_probe(int32_t op, int32_t blocks, int32_t iters, void *sink, void *stream, double *ms,
                  int64_t *lane_ops, double *clock_ratio);

void nb_destroy(nb_system *s);
const char *nb_strerror(int status);
/* ABI version: 4 (band height in nb_tile_config and nb_tile_override, overrides per mode and
 * law). */
int nb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NBODY_H */
