// nb_kernels.hip -- gfx950 kernels of libnbody.
//
// The O(N^2) all-pairs force evaluation (Methodology: every element moves only under the sum of
// all pairwise element-element interactions) is the hot path. It runs on the FP32 vector ALUs:
// the pair sum is not a dense contraction, so there is no MFMA here. The kernels that evaluate it:
//   - k_force_sym<KR> / k_force_sym_paper<KR> (FP32, Kahan mode, the default): each unordered
//     pair once, bands of KR tile rows with one i element of each row per lane in registers and
//     the j sums rotating across the wave (see the section below), contact law / eqs. (4)-(6);
//   - k_force_f32 (FP32, plain mode): one-sided, one i element per lane, the block streams
//     256-element SoA j tiles through LDS (broadcast ds_read_b128), one FP32 running sum;
//   - k_force_sym64<LAW> (FP64 reference mode): the symmetric scheme in FP64, both element laws.
// All of them work on a Morton-sorted, star-by-star padded copy of the positions; the FP32 ones
// skip the contact test on tiles whose bounding boxes are at least D apart. Per pair of the
// contact law:
//   d = r_j - r_i,  r2 = d.d + eps,  w = rsqrt(r2)  (v_rsq_f32),
//   s = min(w^3, c1 - c2 w),  acc += s d,
// where c1 = 11 / D^3 and c2 = 10 / D^2 for the pair's diameter D. Dividing the contact law
// f(r) = G m^2 / r^2 (r >= D), G m^2 r / D^3 - K (1 - r/D) (r < D, K = 10 G m^2 / D^2) by
// G m^2 r gives w^3 outside and c1 - c2 w inside; with x = r/D, 11 - 10/x - 1/x^3 is increasing
// and vanishes at x = 1, so the smaller of the two expressions is always the right branch.
// The self pair has d = 0 exactly and contributes 0; eps = 1e-24 keeps its w finite. The law of
// eqs. (4)-(6) is written out at pair_s.
//
// The remaining kernels are O(N): leap-frog kicks and drift, per-star centres of mass, the
// donor growth update (eq. 3), the L1-plane count and the FP64 diagnostics. Every reduction runs
// in a fixed order (butterfly within a wave, waves in index order, units in index order), so
// results do not depend on scheduling or on which other systems share a launch.
#include "nb_internal.h"

#include <math.h>

#include <algorithm>

namespace nbk {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ int find_sys(const Launch &L, int u, bool ounit)
{
    int lo = 0, hi = L.n_sys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        int b = ounit ? L.sys[mid].ounit_begin : L.sys[mid].unit_begin;
        if (b <= u) {
            lo = mid;
        } else {
            hi = mid - 1;
        }
    }
    return lo;
}

// Fixed-order block sum of NV doubles per thread; the result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*lds)[BT / 64])
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off, 64);
        v[k] = x;
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k][wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double t = lds[k][0];
#pragma unroll
            for (int w = 1; w < BT / 64; ++w) t += lds[k][w];
            v[k] = t;
        }
    }
    __syncthreads();
}

__device__ __forceinline__ void kahan_add(float &sum, float &comp, float v)
{
    float y = v - comp;
    float t = sum + y;
    comp = (t - sum) - y;
    sum = t;
}

__device__ __forceinline__ int pair_class(int istar, int jstar) { return istar + jstar; }

constexpr double PI_D = 3.14159265358979323846;

// ------------------------------------------------------------------ sorted layout

__device__ __forceinline__ int find_tile_sys(const Launch &L, int u)
{
    int lo = 0, hi = L.n_sys - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (L.sys[mid].tunit_begin <= u) {
            lo = mid;
        } else {
            hi = mid - 1;
        }
    }
    return lo;
}

__device__ __forceinline__ float wave_min(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

template <typename T>
__global__ __launch_bounds__(BT) void k_fill_sorted(T *xs, T *ys, T *zs, int nalloc, T value)
{
    const int k = blockIdx.x * BT + threadIdx.x;
    if (k < nalloc) {
        xs[k] = value;
        ys[k] = value;
        zs[k] = value;
    }
}

// Pulls the current positions (and, under eqs. (4)-(6), velocities) into sorted order and records
// each tile's bounding box (padding slots keep their fill values and are left out of the box).
template <typename T>
__global__ __launch_bounds__(BT) void k_gather(Launch L)
{
    __shared__ float lds[6][BT / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int u = blockIdx.x; u < L.total_tunits; u += gridDim.x) {
        const SysDesc &S = L.sys[find_tile_sys(L, u)];
        const int tile = u - S.tunit_begin;
        const int slot = tile * TJ + threadIdx.x;
        const int idx = S.perm[slot];
        float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
        if (idx >= 0) {
            const T x = static_cast<const T *>(S.x)[idx];
            const T y = static_cast<const T *>(S.y)[idx];
            const T z = static_cast<const T *>(S.z)[idx];
            static_cast<T *>(S.xs)[slot] = x;
            static_cast<T *>(S.ys)[slot] = y;
            static_cast<T *>(S.zs)[slot] = z;
            if (S.vxs) {
                static_cast<T *>(S.vxs)[slot] = static_cast<const T *>(S.vx)[idx];
                static_cast<T *>(S.vys)[slot] = static_cast<const T *>(S.vy)[idx];
                static_cast<T *>(S.vzs)[slot] = static_cast<const T *>(S.vz)[idx];
            }
            v[0] = v[3] = (float)x;
            v[1] = v[4] = (float)y;
            v[2] = v[5] = (float)z;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            v[k] = wave_min(v[k]);
            v[3 + k] = wave_max(v[3 + k]);
        }
        if (lane == 0) {
#pragma unroll
            for (int k = 0; k < 6; ++k) lds[k][wave] = v[k];
        }
        __syncthreads();
        if (threadIdx.x < 8) {
            const int k = threadIdx.x;
            float r = 0.0f;
            if (k < 3 || (k >= 4 && k < 7)) {
                const int q = k < 3 ? k : k - 1;
                r = lds[q][0];
                for (int w = 1; w < BT / 64; ++w) r = q < 3 ? fminf(r, lds[q][w]) : fmaxf(r, lds[q][w]);
            }
            S.tbox[(size_t)tile * 8 + k] = r;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ FP32 one-sided force kernel

// Near tiles: the contact law s = min(w^3, c1 - c2 w) for every pair; far tiles (every pair at
// r >= D, proven from bounding boxes): s = w^3, the value the contact law's minimum selects there.
template <bool FAR>
__device__ __forceinline__ void interact4_f32(const float4 &X, const float4 &Y, const float4 &Z,
                                              float xi, float yi, float zi, float &ax, float &ay,
                                              float &az, float c1, float nc2)
{
    const float eps = 1.0e-24f;
    const float xs[4] = {X.x, X.y, X.z, X.w};
    const float ys[4] = {Y.x, Y.y, Y.z, Y.w};
    const float zs[4] = {Z.x, Z.y, Z.z, Z.w};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float dx = xs[q] - xi;
        const float dy = ys[q] - yi;
        const float dz = zs[q] - zi;
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps)));
        const float w = __builtin_amdgcn_rsqf(r2);
        const float w3 = (w * w) * w;
        const float s = FAR ? w3 : fminf(w3, fmaf(nc2, w, c1));
        ax = fmaf(s, dx, ax);
        ay = fmaf(s, dy, ay);
        az = fmaf(s, dz, az);
    }
}

__device__ __forceinline__ float4 lds4(const float *p) { return *reinterpret_cast<const float4 *>(p); }

// One force unit of the plain mode: i-block `ib` (256 sorted slots, one per lane) against j
// chunk `c` (a run of whole tiles), one running FP32 sum per element in tile order.
__device__ __forceinline__ void force_unit_f32(const SysDesc &S, int ib, int c,
                                               float (*sh)[3][TJ])
{
    const int tid = threadIdx.x;
    const float *__restrict__ XS = static_cast<const float *>(S.xs);
    const float *__restrict__ YS = static_cast<const float *>(S.ys);
    const float *__restrict__ ZS = static_cast<const float *>(S.zs);
    const DevState *st = S.st;

    const int slot = ib * BT + tid;
    const float xi = XS[slot], yi = YS[slot], zi = ZS[slot];
    float ax = 0.0f, ay = 0.0f, az = 0.0f;
    const bool real = S.perm[slot] >= 0;
    float lo[3], hi[3];
    lo[0] = wave_min(real ? xi : INFINITY);
    lo[1] = wave_min(real ? yi : INFINITY);
    lo[2] = wave_min(real ? zi : INFINITY);
    hi[0] = wave_max(real ? xi : -INFINITY);
    hi[1] = wave_max(real ? yi : -INFINITY);
    hi[2] = wave_max(real ? zi : -INFINITY);
    // the block's slots lie in one star (p1 is a multiple of TJ)
    const int istar = ib * BT >= S.p1 ? 1 : 0;
    const float c1a = st->c1f[istar], nc2a = -st->c2f[istar], far2a = st->far2f[istar];
    const float c1b = st->c1f[istar + 1], nc2b = -st->c2f[istar + 1], far2b = st->far2f[istar + 1];

    // chunk c covers tiles [c ntiles / nsplit, (c + 1) ntiles / nsplit): sizes differ by <= 1
    const int t0 = (int)(((int64_t)c * S.ntiles) / S.nsplit);
    const int t1 = (int)(((int64_t)(c + 1) * S.ntiles) / S.nsplit);
    float px = 0.f, py = 0.f, pz = 0.f;
    if (t0 < t1) {
        px = XS[t0 * TJ + tid];
        py = YS[t0 * TJ + tid];
        pz = ZS[t0 * TJ + tid];
    }
    for (int t = t0; t < t1; ++t) {
        const int buf = (t - t0) & 1;
        sh[buf][0][tid] = px;
        sh[buf][1][tid] = py;
        sh[buf][2][tid] = pz;
        __syncthreads();
        if (t + 1 < t1) {
            px = XS[(t + 1) * TJ + tid];
            py = YS[(t + 1) * TJ + tid];
            pz = ZS[(t + 1) * TJ + tid];
        }
        const bool jstar = t * TJ >= S.p1;
        const float *bx = S.tbox + (size_t)t * 8;
        const float gx = fmaxf(0.0f, fmaxf(bx[0] - hi[0], lo[0] - bx[4]));
        const float gy = fmaxf(0.0f, fmaxf(bx[1] - hi[1], lo[1] - bx[5]));
        const float gz = fmaxf(0.0f, fmaxf(bx[2] - hi[2], lo[2] - bx[6]));
        const float gap2 = gx * gx + gy * gy + gz * gz;
        const int far = __builtin_amdgcn_readfirstlane(gap2 >= (jstar ? far2b : far2a) ? 1 : 0);
        const float *sx = sh[buf][0], *sy = sh[buf][1], *sz = sh[buf][2];
        if (far) {
#pragma unroll 2
            for (int jj = 0; jj < TJ; jj += 4)
                interact4_f32<true>(lds4(sx + jj), lds4(sy + jj), lds4(sz + jj), xi, yi, zi, ax,
                                    ay, az, 0.f, 0.f);
        } else {
            const float c1 = jstar ? c1b : c1a, nc2 = jstar ? nc2b : nc2a;
#pragma unroll 2
            for (int jj = 0; jj < TJ; jj += 4)
                interact4_f32<false>(lds4(sx + jj), lds4(sy + jj), lds4(sz + jj), xi, yi, zi, ax,
                                     ay, az, c1, nc2);
        }
    }
    __syncthreads();  // the next unit of this block reuses both LDS buffers

    const int idx = S.perm[slot];
    if (idx < 0) return;
    if (S.nsplit == 1) {
        const float gm = st->gm_f;
        static_cast<float *>(S.ax)[idx] = gm * ax;
        static_cast<float *>(S.ay)[idx] = gm * ay;
        static_cast<float *>(S.az)[idx] = gm * az;
    } else {
        float *P = static_cast<float *>(S.part);
        const size_t na = S.nalloc;
        const size_t b = (size_t)c * 3 * na + slot;
        P[b] = ax;
        P[b + na] = ay;
        P[b + 2 * na] = az;
    }
}

__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(PLAIN_WAVES)))
void k_force_f32(Launch L)
{
    __shared__ __attribute__((aligned(16))) float sh[2][3][TJ];
    for (int u = L.unit_base + blockIdx.x; u < L.total_units; u += gridDim.x) {
        const int s = find_sys(L, u, false);
        const SysDesc &S = L.sys[s];
        const int local = u - S.unit_begin;
        const int ib = local / S.nsplit;
        const int c = local - ib * S.nsplit;
        force_unit_f32(S, ib, c, sh);
    }
}

// ------------------------------------------------------------------ FP32 symmetric force kernel
//
// Newton's third law halves the pair work: the pair (i, j) with i in tile I and j in a later
// tile J > I is evaluated once. The tile rows are taken in groups ("row bands") of KR consecutive
// rows (KR = 1, 2 or 4, chosen per system size): a work unit is group g, rows I = KR g .. KR g +
// KR - 1, against chunk c of its tiles, a run of `ch` tiles starting at KR g + c ch. Each lane of
// the block's four waves keeps one i element of every row of the band, at the same position in
// each row. A tile's 256 j elements are taken as four groups of 64. At step s (0..63) lane l
// meets element (l - s) mod 64 of each group: its position is read from LDS once at that
// rotating offset and paired with the lane's KR i elements, and the j accumulator travels with
// it, one lane per step: in short bands by a DPP wave rotation fused into the first row's update
// a_j <- rotate(a_j) - s (r_j - r_i), in tall ones through the LDS crossbar after the group's
// last row (see sym_tile); the rows add their terms in row order. After 64 steps and the last
// move every lane holds the summed reaction of the wave's 64 KR i elements on its own j. The
// waves' sums are added in wave order and stored once per (group, tile): a band of KR rows
// stores 1/KR of the reaction blocks of single rows. Tiles inside the band are split by row:
// tile KR g + k is one-sided for row k, full for the rows before it and skipped by the rows
// after it. k_combine_sym adds, per element, its own row's chunk partials and then the reactions
// of every group with a row before the element's tile, in group order, with Kahan compensation.
// The order of every sum is fixed by the system's own size, so results do not depend on
// scheduling or on the other systems of a launch.

constexpr int DPP_WAVE_ROR1 = 0x13C;  // lane l receives lane l - 1 (mod 64)

__device__ __forceinline__ float wave_ror1(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), DPP_WAVE_ROR1, 0xf, 0xf, true));
}

// The same move through the LDS crossbar (ds_bpermute, no LDS storage): addr = 4 ((l - 1) mod 64)
// in lane l.
__device__ __forceinline__ float xbar_ror1(float v, int addr)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}

// A value that is the same in every lane, moved to a scalar register.
__device__ __forceinline__ float wave_uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// Constants of one pair class for the FP32 kernels.
struct LawF {
    float c1, nc2;            // contact law: 11 / D^3 and -10 / D^2
    float D, twoD, eps, gc, gcb;  // eqs. (4)-(6): see DevState
};

__device__ __forceinline__ LawF law_uniform(LawF K)
{
    K.c1 = wave_uniform(K.c1);
    K.nc2 = wave_uniform(K.nc2);
    K.D = wave_uniform(K.D);
    K.twoD = wave_uniform(K.twoD);
    K.eps = wave_uniform(K.eps);
    K.gc = wave_uniform(K.gc);
    K.gcb = wave_uniform(K.gcb);
    return K;
}

__device__ __forceinline__ LawF law_f(const DevState *st, int cls)
{
    LawF K;
    K.c1 = st->c1f[cls];
    K.nc2 = -st->c2f[cls];
    K.D = st->lD_f[cls];
    K.twoD = 2.0f * st->lD_f[cls];
    K.eps = st->leps_f;
    K.gc = st->lgc_f;
    K.gcb = st->lgcb_f;
    return K;
}

// Pair scalar s = f / (G m^2 r) of one pair from r2 = |d|^2; the caller adds s d to the i sum.
//   contact law:  w = rsqrt(r2); min(w^3, c1 - c2 w) near, w^3 far.
//   eqs. (4)-(6): r = sqrt(r2), t = r + eps; s = 1 / (t^2 r) - g (D - r)_+^2 (1 + 2 D w) with
//                 w = 1 / r = t^2 s_att, g = gc for a converging pair ((v_j - v_i).(r_j - r_i)
//                 < 0) and gcb otherwise; the overlap term is left out on far tiles, where every
//                 pair has r >= D. (pi / 12) (D - r)^2 (r + 2D) is the overlap volume of eq. (5)
//                 in factored form, so it has no cancellation near D. The square root form takes
//                 one multiply fewer per far pair than r = r2 rsqrt(r2) (measured 2.5 % faster).
//                 A padding slot (r near 1.7e18) gives t^2 r = inf, s = 0 and w = 0.
// On a far tile the near form gives the same bits (the contact law's minimum picks w^3 by a margin
// far above rounding once r^2 >= (1 + FAR_MARGIN) D^2; the overlap term is exactly 0 for r >= D),
// so the near/far choice changes speed only.
template <int LAW, bool NEAR>
__device__ __forceinline__ float pair_s(float r2, float dx, float dy, float dz, const float4 &vj,
                                        const float4 &vi, const LawF &K)
{
#pragma clang fp contract(off)
    if constexpr (LAW == 0) {
        const float w = __builtin_amdgcn_rsqf(r2);
        const float w3 = (w * w) * w;
        return NEAR ? fminf(w3, fmaf(K.nc2, w, K.c1)) : w3;
    } else {
        const float r = __builtin_amdgcn_sqrtf(r2);
        const float t = r + K.eps;
        const float t2 = t * t;
        float s = __builtin_amdgcn_rcpf(t2 * r);
        if constexpr (NEAR) {
            const float w = t2 * s;
            const float dot = fmaf(vj.x - vi.x, dx, fmaf(vj.y - vi.y, dy, (vj.z - vi.z) * dz));
            const float g = dot < 0.0f ? K.gc : K.gcb;
            const float u = fmaxf(K.D - r, 0.0f);
            s = s - ((g * u) * u) * fmaf(K.twoD, w, 1.0f);
        }
        return s;
    }
}

// The i side of a band: one element of each of KR tile rows per lane.
template <int KR>
struct Band {
    float x[KR], y[KR], z[KR];     // positions
    float ax[KR], ay[KR], az[KR];  // sums over the current tile
    float4 v[KR];                  // half-step velocities (eqs. 4-6 only)
};

// One-sided diagonal tile of one row from an AoS LDS tile (x, y, z, unused). The self pair has
// d = 0; under eqs. (4)-(6) it is also masked, since its overlap term is of order 1/eps.
template <int LAW>
__device__ __forceinline__ void diag_tile(const float4 *__restrict__ sj,
                                          const float4 *__restrict__ sv, float xi, float yi,
                                          float zi, const float4 &vi, const LawF &K, float &ax,
                                          float &ay, float &az)
{
    const float eps = 1.0e-24f;
    const int self = threadIdx.x;
#pragma unroll 4
    for (int jj = 0; jj < TJ; ++jj) {
        const float4 P = sj[jj];
        const float dx = P.x - xi;
        const float dy = P.y - yi;
        const float dz = P.z - zi;
        const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps)));
        float s;
        if constexpr (LAW == 0) {
            s = pair_s<0, true>(r2, dx, dy, dz, vi, vi, K);
        } else {
            s = pair_s<LAW, true>(r2, dx, dy, dz, sv[jj], vi, K);
            s = jj == self ? 0.0f : s;
        }
        ax = fmaf(s, dx, ax);
        ay = fmaf(s, dy, ay);
        az = fmaf(s, dz, az);
    }
}

// A full tile against the band's rows 0 .. nact - 1 (all KR rows unless MASKED; nact >= 1), with
// the reactions on the tile's 256 j left in the wave's rw slice.
template <bool NEAR, int LAW, int KR, bool MASKED>
__device__ __forceinline__ void sym_tile(const float4 *__restrict__ sj,
                                         const float4 *__restrict__ sv, Band<KR> &B,
                                         const LawF (&K)[KR], float *rwx, float *rwy, float *rwz,
                                         int lane, int nact)
{
    // The j sums move one lane per step (lane l takes lane l - 1's sums). With one row per band
    // the move folds into row 0's update, a_j <- rotate(a_j) - p with p = s d kept as an operand
    // of its own (a VOP2 subtraction with a DPP source; a fused multiply-add cannot take one).
    // The other rows add s d to both sums with fused multiply-adds: two instructions per
    // component instead of three. In taller bands (four rows under the contact law, two or more
    // under eqs. (4)-(6)) the sums of each j group move through the LDS crossbar (ds_bpermute)
    // after the group's last row instead, off the vector ALU, and row 0 takes the FMA form too
    // (measured 6 % faster at four rows under the contact law, 7.5 % at two under eqs. 4-6).
    // Under the contact law at two rows the DPP form measured 0.5 % faster (its pair code is
    // the shorter), and at one row three crossbar moves per pair saturate the LDS (half speed).
#pragma clang fp contract(off)
    constexpr bool XBAR = LAW == 0 ? KR >= 4 : KR >= 2;
    const float eps = 1.0e-24f;
    float ajx[4] = {0.f, 0.f, 0.f, 0.f}, ajy[4] = {0.f, 0.f, 0.f, 0.f};
    float ajz[4] = {0.f, 0.f, 0.f, 0.f};
    const int rot_addr = ((lane + 63) & 63) << 2;  // byte address of lane l - 1 (mod 64)
    for (int st = 0; st < 64; ++st) {
        const int e = (lane - st) & 63;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const float4 P = sj[g * 64 + e];
            float4 Vj = make_float4(0.f, 0.f, 0.f, 0.f);
            if constexpr (LAW != 0 && NEAR) Vj = sv[g * 64 + e];
#pragma unroll
            for (int r = 0; r < KR; ++r) {
                if (MASKED && r >= nact) continue;  // wave-uniform
                const float dx = P.x - B.x[r];
                const float dy = P.y - B.y[r];
                const float dz = P.z - B.z[r];
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps)));
                const float s = pair_s<LAW, NEAR>(r2, dx, dy, dz, Vj, B.v[r], K[r]);
                if (!XBAR && r == 0) {
                    const float px = s * dx, py = s * dy, pz = s * dz;
                    B.ax[r] += px;
                    B.ay[r] += py;
                    B.az[r] += pz;
                    ajx[g] = wave_ror1(ajx[g]) - px;
                    ajy[g] = wave_ror1(ajy[g]) - py;
                    ajz[g] = wave_ror1(ajz[g]) - pz;
                } else {
                    B.ax[r] = fmaf(s, dx, B.ax[r]);
                    B.ay[r] = fmaf(s, dy, B.ay[r]);
                    B.az[r] = fmaf(s, dz, B.az[r]);
                    ajx[g] = fmaf(-s, dx, ajx[g]);
                    ajy[g] = fmaf(-s, dy, ajy[g]);
                    ajz[g] = fmaf(-s, dz, ajz[g]);
                }
                // contact law: keep each pair's instructions together. Left free, the scheduler
                // gathers the twelve rotated updates of a step at its end, and back-to-back DPP
                // subtractions issue at about a third of the rate of plain ones (measured 11 %
                // slower at one row per band; with the crossbar form at four rows 1.5 % slower).
                // The eqs. (4)-(6) loop measured 3.5 % faster without the barrier.
                if constexpr (LAW == 0) __builtin_amdgcn_sched_barrier(0);
            }
            if constexpr (XBAR) {
                ajx[g] = xbar_ror1(ajx[g], rot_addr);
                ajy[g] = xbar_ror1(ajy[g], rot_addr);
                ajz[g] = xbar_ror1(ajz[g], rot_addr);
            }
        }
    }
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        // element l's sum back in lane l: one more rotation after the last step (the crossbar
        // form did it already)
        rwx[g * 64 + lane] = XBAR ? ajx[g] : wave_ror1(ajx[g]);
        rwy[g * 64 + lane] = XBAR ? ajy[g] : wave_ror1(ajy[g]);
        rwz[g * 64 + lane] = XBAR ? ajz[g] : wave_ror1(ajz[g]);
    }
}

// Reactions are stored per group g (tile rows KR g .. KR g + KR - 1) for the tiles t after the
// group's first row, t = KR g + 1 .. T - 1: three components one after the other, each
// (T - KR g - 1) TJ values. Group g starts after
// sum_{g' < g} 3 TJ (T - KR g' - 1) = 3 TJ (g (T - 1) - KR g (g - 1) / 2) values.
__device__ __forceinline__ size_t react_group_offset(int g, int ntiles, int kr)
{
    return (size_t)3 * TJ *
           ((size_t)g * (ntiles - 1) - (size_t)kr * (size_t)g * (size_t)(g - 1) / 2);
}

// Whether a tile lies at least D from every i of the wave (its bounding box against the wave's),
// for the larger of the band's thresholds.
__device__ __forceinline__ bool far_tile(const float *bx, const float (&lo)[3],
                                         const float (&hi)[3], float far2)
{
    const float gx = fmaxf(0.0f, fmaxf(bx[0] - hi[0], lo[0] - bx[4]));
    const float gy = fmaxf(0.0f, fmaxf(bx[1] - hi[1], lo[1] - bx[5]));
    const float gz = fmaxf(0.0f, fmaxf(bx[2] - hi[2], lo[2] - bx[6]));
    const float gap2 = gx * gx + gy * gy + gz * gz;
    return __builtin_amdgcn_readfirstlane(gap2 >= far2 ? 1 : 0) != 0;
}

// One work unit of the symmetric kernel: band `grp` against chunk c of its tiles (see above).
template <int LAW, int KR>
__device__ void force_unit_sym(const SysDesc &S, int grp, int c, float4 *sj, float4 *sv,
                               float (*rw)[3][TJ])
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const float *__restrict__ XS = static_cast<const float *>(S.xs);
    const float *__restrict__ YS = static_cast<const float *>(S.ys);
    const float *__restrict__ ZS = static_cast<const float *>(S.zs);
    const float *__restrict__ VXS = static_cast<const float *>(S.vxs);
    const float *__restrict__ VYS = static_cast<const float *>(S.vys);
    const float *__restrict__ VZS = static_cast<const float *>(S.vzs);
    const DevState *st = S.st;
    const int T = S.ntiles;
    const int g0 = KR * grp;               // first tile row of the band
    const int nv = min(KR, T - g0);        // rows of the band inside the system (the last is short)
    Band<KR> B;
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    LawF Ka[KR], Kb[KR];
    float far2a = 0.0f, far2b = 0.0f;
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        const int row = r < nv ? g0 + r : g0;  // a missing row mirrors row 0 and stays unused
        const int slot = row * TJ + tid;
        B.x[r] = XS[slot];
        B.y[r] = YS[slot];
        B.z[r] = ZS[slot];
        B.ax[r] = B.ay[r] = B.az[r] = 0.0f;
        B.v[r] = make_float4(0.f, 0.f, 0.f, 0.f);
        if constexpr (LAW != 0) B.v[r] = make_float4(VXS[slot], VYS[slot], VZS[slot], 0.0f);
        if (r < nv && S.perm[slot] >= 0) {
            lo[0] = fminf(lo[0], B.x[r]);
            lo[1] = fminf(lo[1], B.y[r]);
            lo[2] = fminf(lo[2], B.z[r]);
            hi[0] = fmaxf(hi[0], B.x[r]);
            hi[1] = fmaxf(hi[1], B.y[r]);
            hi[2] = fmaxf(hi[2], B.z[r]);
        }
        const int istar = row * TJ >= S.p1 ? 1 : 0;
        Ka[r] = law_uniform(law_f(st, istar));
        Kb[r] = law_uniform(law_f(st, istar + 1));
        far2a = fmaxf(far2a, st->far2f[istar]);
        far2b = fmaxf(far2b, st->far2f[istar + 1]);
    }
    // the box and the constants are the same in every lane; held in scalar registers they leave
    // the vector registers to the pair loop
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[d] = wave_uniform(wave_min(lo[d]));
        hi[d] = wave_uniform(wave_max(hi[d]));
    }
    far2a = wave_uniform(far2a);
    far2b = wave_uniform(far2b);

    float sumx[KR], sumy[KR], sumz[KR], cx[KR], cy[KR], cz[KR];
#pragma unroll
    for (int r = 0; r < KR; ++r) sumx[r] = sumy[r] = sumz[r] = cx[r] = cy[r] = cz[r] = 0.0f;
    const int t0 = g0 + c * S.ch;
    const int t1 = min(T, t0 + S.ch);
    float *R = S.react;
    const size_t roff = react_group_offset(grp, T, KR);
    const size_t rlen = (size_t)(T - g0 - 1) * TJ;
    float px = 0.f, py = 0.f, pz = 0.f, qx = 0.f, qy = 0.f, qz = 0.f;
    if (t0 < t1) {
        px = XS[t0 * TJ + tid];
        py = YS[t0 * TJ + tid];
        pz = ZS[t0 * TJ + tid];
        if constexpr (LAW != 0) {
            qx = VXS[t0 * TJ + tid];
            qy = VYS[t0 * TJ + tid];
            qz = VZS[t0 * TJ + tid];
        }
    }
    for (int t = t0; t < t1; ++t) {
        sj[tid] = make_float4(px, py, pz, 0.0f);
        if constexpr (LAW != 0) sv[tid] = make_float4(qx, qy, qz, 0.0f);
        __syncthreads();
        if (t + 1 < t1) {
            px = XS[(t + 1) * TJ + tid];
            py = YS[(t + 1) * TJ + tid];
            pz = ZS[(t + 1) * TJ + tid];
            if constexpr (LAW != 0) {
                qx = VXS[(t + 1) * TJ + tid];
                qy = VYS[(t + 1) * TJ + tid];
                qz = VZS[(t + 1) * TJ + tid];
            }
        }
        const bool jstar = t * TJ >= S.p1;
        LawF K[KR];
#pragma unroll
        for (int r = 0; r < KR; ++r) K[r] = jstar ? Kb[r] : Ka[r];
        const float far2 = jstar ? far2b : far2a;
        const int k = t - g0;  // tile t is row k of the band when k < KR
        if (k >= KR) {
            if (far_tile(S.tbox + (size_t)t * 8, lo, hi, far2)) {
                sym_tile<false, LAW, KR, false>(sj, sv, B, K, rw[wave][0], rw[wave][1],
                                                rw[wave][2], lane, KR);
            } else {
                sym_tile<true, LAW, KR, false>(sj, sv, B, K, rw[wave][0], rw[wave][1],
                                               rw[wave][2], lane, KR);
            }
        } else {
            if (k > 0) {
                // rows 0 .. k - 1 lie before tile t: full pairs with reactions
                sym_tile<true, LAW, KR, true>(sj, sv, B, K, rw[wave][0], rw[wave][1], rw[wave][2],
                                              lane, k);
            }
#pragma unroll
            for (int r = 0; r < KR; ++r) {
                if (r == k) {
                    diag_tile<LAW>(sj, sv, B.x[r], B.y[r], B.z[r], B.v[r], K[r], B.ax[r], B.ay[r],
                                   B.az[r]);
                }
            }
        }
        if (t > g0) {
            // tile t lies after the band's first row, so at least one row left reactions
            __syncthreads();
            const size_t at = roff + (size_t)(t - g0 - 1) * TJ + tid;
#pragma unroll
            for (int d = 0; d < 3; ++d)
                R[at + d * rlen] = ((rw[0][d][tid] + rw[1][d][tid]) + rw[2][d][tid]) + rw[3][d][tid];
        }
#pragma unroll
        for (int r = 0; r < KR; ++r) {
            kahan_add(sumx[r], cx[r], B.ax[r]);
            kahan_add(sumy[r], cy[r], B.ay[r]);
            kahan_add(sumz[r], cz[r], B.az[r]);
            B.ax[r] = B.ay[r] = B.az[r] = 0.0f;
        }
        __syncthreads();  // sj, sv and rw are rewritten by the next tile
    }
    float *P = static_cast<float *>(S.part);
    const size_t na = S.nalloc;
#pragma unroll
    for (int r = 0; r < KR; ++r) {
        if (r >= nv) continue;
        const int slot = (g0 + r) * TJ + tid;
        if (S.perm[slot] < 0) continue;
        const size_t b = (size_t)c * 3 * na + slot;
        P[b] = sumx[r] - cx[r];
        P[b + na] = sumy[r] - cy[r];
        P[b + 2 * na] = sumz[r] - cz[r];
    }
}

template <int LAW, int KR>
__device__ __forceinline__ void force_sym_units(const Launch &L, float4 *sj, float4 *sv,
                                                float (*rw)[3][TJ])
{
    for (int u = L.unit_base + blockIdx.x; u < L.total_units; u += gridDim.x) {
        const SysDesc &S = L.sys[find_sys(L, u, false)];
        const int2 gc = reinterpret_cast<const int2 *>(S.units)[u - S.unit_begin];
        force_unit_sym<LAW, KR>(S, gc.x, gc.y, sj, sv, rw);
    }
}

// Contact law; the launch covers the units [unit_base, total_units) of systems with KR rows per
// band (the runtime orders a segment table by band height, so each height is one range).
template <int KR>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(SYM_WAVES[KR / 2])))
void k_force_sym(Launch L)
{
    __shared__ float4 sj[TJ];
    __shared__ __attribute__((aligned(16))) float rw[4][3][TJ];
    force_sym_units<0, KR>(L, sj, nullptr, rw);
}

// The same under eqs. (4)-(6): each tile also stages the sorted half-step velocities.
template <int KR>
__global__ __launch_bounds__(BT) __attribute__((amdgpu_waves_per_eu(SYM_PAPER_WAVES[KR / 2])))
void k_force_sym_paper(Launch L)
{
    __shared__ float4 sj[TJ];
    __shared__ float4 sv[TJ];
    __shared__ __attribute__((aligned(16))) float rw[4][3][TJ];
    force_sym_units<1, KR>(L, sj, sv, rw);
}

// a = G m (sum of the element's own chunk partials, then the reactions of every band with a
// row before the element's tile, in band order), scattered to the element's own index. KR is the
// system's band height. The element's terms (its cj chunk partials, then its ng band reactions)
// are cut into COMBINE_SEGS contiguous runs, one thread each; a run is a Kahan sum per component
// in term order, with the three components' loads issued together, eight terms at a time. The
// runs' results are then added in run order with Kahan compensation by the element's first
// thread. The order of every addition depends on the system's size alone.
constexpr int COMBINE_SEGS = 4;

template <int KR>
__device__ __forceinline__ void combine_tile(const SysDesc &S, int J, int e, int k,
                                             float (*part)[COMBINE_SEGS][TJ])
{
    const int T = S.ntiles;
    const int slot = J * TJ + e;
    const int idx = S.perm[slot];
    const float *P = static_cast<const float *>(S.part);
    const float *R = S.react;
    const size_t na = S.nalloc;
    const int own = J / KR;                           // the element's own band
    const int cj = (T - KR * own + S.ch - 1) / S.ch;  // its chunk count
    const int ng = (J + KR - 1) / KR;                 // bands with a row before J
    const int M = cj + ng;                            // terms
    const int t0 = (int)(((int64_t)M * k) / COMBINE_SEGS);
    const int t1 = (int)(((int64_t)M * (k + 1)) / COMBINE_SEGS);
    float sum[3] = {0.f, 0.f, 0.f}, comp[3] = {0.f, 0.f, 0.f};
    if (idx >= 0) {
        int t = t0;
        // chunk partials
        for (; t < min(t1, cj); ++t) {
            const size_t at = (size_t)t * 3 * na + slot;
            const float vx = P[at], vy = P[at + na], vz = P[at + 2 * na];
            kahan_add(sum[0], comp[0], vx);
            kahan_add(sum[1], comp[1], vy);
            kahan_add(sum[2], comp[2], vz);
        }
        // band reactions: band g's block starts at 3 TJ (g (T - 1) - KR g (g - 1) / 2) and holds
        // three components of (T - KR g - 1) TJ values; the element's value sits at slot -
        // TJ (KR g + 1) inside each
        int g = t - cj;
        const int g1 = t1 - cj;
        if (g < g1) {
            size_t off = react_group_offset(g, T, KR);
            size_t len = (size_t)(T - KR * g - 1) * TJ;
            for (; g + 8 <= g1; g += 8) {
                float v[8][3];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const size_t at = off + slot - (size_t)TJ * (KR * (g + q) + 1);
                    v[q][0] = R[at];
                    v[q][1] = R[at + len];
                    v[q][2] = R[at + 2 * len];
                    off += 3 * len;
                    len -= (size_t)KR * TJ;
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    kahan_add(sum[0], comp[0], v[q][0]);
                    kahan_add(sum[1], comp[1], v[q][1]);
                    kahan_add(sum[2], comp[2], v[q][2]);
                }
            }
            for (; g < g1; ++g) {
                const size_t at = off + slot - (size_t)TJ * (KR * g + 1);
                kahan_add(sum[0], comp[0], R[at]);
                kahan_add(sum[1], comp[1], R[at + len]);
                kahan_add(sum[2], comp[2], R[at + 2 * len]);
                off += 3 * len;
                len -= (size_t)KR * TJ;
            }
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) part[d][k][e] = sum[d] - comp[d];
    __syncthreads();
    if (k == 0 && idx >= 0) {
        float out[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            float s = part[d][0][e], c = 0.f;
#pragma unroll
            for (int q = 1; q < COMBINE_SEGS; ++q) kahan_add(s, c, part[d][q][e]);
            out[d] = s - c;
        }
        const float gm = S.st->gm_f;
        static_cast<float *>(S.ax)[idx] = gm * out[0];
        static_cast<float *>(S.ay)[idx] = gm * out[1];
        static_cast<float *>(S.az)[idx] = gm * out[2];
    }
    __syncthreads();  // part is rewritten by the block's next tile
}

__global__ __launch_bounds__(BT * COMBINE_SEGS) void k_combine_sym(Launch L)
{
    __shared__ float part[3][COMBINE_SEGS][TJ];
    const int e = threadIdx.x % TJ, k = threadIdx.x / TJ;
    for (int u = blockIdx.x; u < L.total_tunits; u += gridDim.x) {
        const SysDesc &S = L.sys[find_tile_sys(L, u)];
        const int J = u - S.tunit_begin;
        switch (S.rows) {
        case 1: combine_tile<1>(S, J, e, k, part); break;
        case 2: combine_tile<2>(S, J, e, k, part); break;
        default: combine_tile<4>(S, J, e, k, part); break;
        }
    }
}

// ------------------------------------------------------------------ FP64 force kernel

// FP64 reciprocal square root and reciprocal from the hardware estimates, each refined by one
// correction of higher order instead of two Newton steps. With e the estimate's residual,
// 1 / sqrt(x) = y (1 - e)^(-1/2) = y (1 + e/2 + 3 e^2/8 + ...) and 1 / b = y (1 - e)^(-1) =
// y (1 + e + e^2 + ...); the estimates' relative error measures below 2^-24 on this part, so
// the truncated terms are below 2^-70 and the results lie within an ulp of the exact values
// (measured over 1.7e7 arguments from 1e-200 to 1e300: at most 0.99 ulp for the square root,
// 0.50 for the reciprocal, tighter than two Newton steps' 1.75 and 0.50). Every argument the
// kernels pass is normal, with a normal result.
__device__ __forceinline__ double rsqrt_f64(double r2)
{
    const double y = __builtin_amdgcn_rsq(r2);
    const double e = fma(-r2 * y, y, 1.0);  // 1 - r2 y^2
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

__device__ __forceinline__ double rcp_f64(double b)
{
    const double y = __builtin_amdgcn_rcp(b);
    const double e = fma(-b, y, 1.0);  // 1 - b y
    return fma(y, fma(e, e, e), y);
}

// Per-tile constants of the FP64 pair code, read once per tile: the pair class's element diameter
// and contact-law coefficients, and the eqs. (4)-(6) softening and overlap scales.
struct LawD {
    double D, c1, c2, eps, gc, gcb;
};

__device__ __forceinline__ LawD law_d(const DevState *st, int cls)
{
    LawD K;
    K.D = cls == 0 ? st->D1 : (cls == 2 ? st->D2 : 0.5 * (st->D1 + st->D2));
    K.c1 = st->c1d[cls];
    K.c2 = st->c2d[cls];
    K.eps = st->leps_d;
    K.gc = st->lgc_d;
    K.gcb = st->lgcb_d;
    return K;
}

// Pair scalar s = f / (G m^2 r) in FP64 (see pair_s); w = 1 / r. Under eqs. (4)-(6) the
// attraction w / t^2 takes the refined reciprocal of t^2 (rcp_f64) instead of an IEEE division
// (measured 12 % faster; the division's scaling and fix-up steps cost more than the reciprocal
// itself). Coincident elements (d = 0, r^2 = 1e-200 after the floor added in pair_s64_at) get a
// large but finite s under both laws (w = 1e100, s at most about 1e300 with eps = 0), so their
// term s d is exactly 0, the oracle's r = 0 rule.
template <int LAW>
__device__ __forceinline__ double pair_s64(double r2, double w, double dx, double dy, double dz,
                                           double dvx, double dvy, double dvz, const LawD &K)
{
    if constexpr (LAW == 0) {
        const double w3 = w * w * w;
        return fmin(w3, K.c1 - K.c2 * w);
    } else {
        const double r = r2 * w;
        const double t = r + K.eps;
        double s = w * rcp_f64(t * t);
        if (r < K.D) {
            const double dot = dvx * dx + dvy * dy + dvz * dz;
            const double g = dot < 0.0 ? K.gc : K.gcb;
            const double u = K.D - r;
            s -= g * u * u * (1.0 + 2.0 * K.D * w);
        }
        return s;
    }
}

// ------------------------------------------------------------------ FP64 symmetric force kernel
//
// The FP64 reference mode with the work split of k_force_sym (one tile row per block): each
// unordered pair once, i in registers, the j sums rotating across the wave (a double moves as its
// two 32-bit halves, one DPP move each), the diagonal tile one-sided, reactions stored per (tile
// row, later tile) and added by k_combine_sym64 after the element's own chunk partials, rows in
// order. Every sum is plain FP64 in a fixed order. There is no far-tile path: the tile boxes are
// FP32, and every pair takes the full law.

__device__ __forceinline__ double wave_ror1_d(double v)
{
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), DPP_WAVE_ROR1, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), DPP_WAVE_ROR1, 0xf, 0xf, true);
    return __hiloint2double(hi, lo);
}

struct I64 {
    double x, y, z, vx, vy, vz;
};

template <int LAW>
__device__ __forceinline__ double pair_s64_at(const double (*sj)[TJ], const double (*sv)[TJ], int j,
                                              const I64 &I, const LawD &K, double &dx, double &dy,
                                              double &dz)
{
    dx = sj[0][j] - I.x;
    dy = sj[1][j] - I.y;
    dz = sj[2][j] - I.z;
    // the 1e-200 floor changes no r^2 above about 1e-184 and keeps the pair code free of a
    // branch for d = 0 (measured 4 % faster for the contact law, 7 % under eqs. 4-6)
    const double r2 = fma(dx, dx, fma(dy, dy, fma(dz, dz, 1.0e-200)));
    const double w = rsqrt_f64(r2);
    if constexpr (LAW == 0) {
        return pair_s64<0>(r2, w, dx, dy, dz, 0.0, 0.0, 0.0, K);
    } else {
        return pair_s64<LAW>(r2, w, dx, dy, dz, sv[0][j] - I.vx, sv[1][j] - I.vy, sv[2][j] - I.vz,
                             K);
    }
}

template <int LAW>
__device__ void force_unit_sym64(const SysDesc &S, int I, int c, double (*sj)[TJ],
                                 double (*sv)[TJ], double (*rw)[3][TJ])
{
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const double *__restrict__ XS = static_cast<const double *>(S.xs);
    const double *__restrict__ YS = static_cast<const double *>(S.ys);
    const double *__restrict__ ZS = static_cast<const double *>(S.zs);
    const double *__restrict__ VXS = static_cast<const double *>(S.vxs);
    const double *__restrict__ VYS = static_cast<const double *>(S.vys);
    const double *__restrict__ VZS = static_cast<const double *>(S.vzs);
    const DevState *st = S.st;
    const int T = S.ntiles;
    const int slot = I * TJ + tid;
    I64 Ist{XS[slot], YS[slot], ZS[slot], 0.0, 0.0, 0.0};
    if constexpr (LAW != 0) {
        Ist.vx = VXS[slot];
        Ist.vy = VYS[slot];
        Ist.vz = VZS[slot];
    }
    const int istar = I * TJ >= S.p1 ? 1 : 0;
    double ax = 0.0, ay = 0.0, az = 0.0;
    const int t0 = I + c * S.ch;
    const int t1 = min(T, t0 + S.ch);
    double *R = reinterpret_cast<double *>(S.react);
    const size_t roff = react_group_offset(I, T, 1);
    const size_t rlen = (size_t)(T - I - 1) * TJ;
    for (int t = t0; t < t1; ++t) {
        sj[0][tid] = XS[t * TJ + tid];
        sj[1][tid] = YS[t * TJ + tid];
        sj[2][tid] = ZS[t * TJ + tid];
        if constexpr (LAW != 0) {
            sv[0][tid] = VXS[t * TJ + tid];
            sv[1][tid] = VYS[t * TJ + tid];
            sv[2][tid] = VZS[t * TJ + tid];
        }
        __syncthreads();
        const int cls = pair_class(istar, t * TJ >= S.p1 ? 1 : 0);
        const LawD K = law_d(st, cls);
        if (t == I) {
            // the self pair (d = 0) adds s d = 0 under both laws
            for (int jj = 0; jj < TJ; ++jj) {
                double dx, dy, dz;
                const double s = pair_s64_at<LAW>(sj, sv, jj, Ist, K, dx, dy, dz);
                ax = fma(s, dx, ax);
                ay = fma(s, dy, ay);
                az = fma(s, dz, az);
            }
        } else {
            double ajx[4] = {0.0, 0.0, 0.0, 0.0}, ajy[4] = {0.0, 0.0, 0.0, 0.0};
            double ajz[4] = {0.0, 0.0, 0.0, 0.0};
            for (int step = 0; step < 64; ++step) {
                const int e = (lane - step) & 63;
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    double dx, dy, dz;
                    const double s = pair_s64_at<LAW>(sj, sv, g * 64 + e, Ist, K, dx, dy, dz);
                    const double px = s * dx, py = s * dy, pz = s * dz;
                    ax += px;
                    ay += py;
                    az += pz;
                    ajx[g] = wave_ror1_d(ajx[g]) - px;
                    ajy[g] = wave_ror1_d(ajy[g]) - py;
                    ajz[g] = wave_ror1_d(ajz[g]) - pz;
                }
            }
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                // one more rotation brings element l's sum back to lane l
                rw[wave][0][g * 64 + lane] = wave_ror1_d(ajx[g]);
                rw[wave][1][g * 64 + lane] = wave_ror1_d(ajy[g]);
                rw[wave][2][g * 64 + lane] = wave_ror1_d(ajz[g]);
            }
            __syncthreads();
            const size_t at = roff + (size_t)(t - I - 1) * TJ + tid;
#pragma unroll
            for (int d = 0; d < 3; ++d)
                R[at + d * rlen] = ((rw[0][d][tid] + rw[1][d][tid]) + rw[2][d][tid]) + rw[3][d][tid];
        }
        __syncthreads();  // sj, sv and rw are rewritten by the next tile
    }
    if (S.perm[slot] >= 0) {
        double *P = static_cast<double *>(S.part);
        const size_t na = S.nalloc;
        const size_t b = (size_t)c * 3 * na + slot;
        P[b] = ax;
        P[b + na] = ay;
        P[b + 2 * na] = az;
    }
}

template <int LAW>
__global__ __launch_bounds__(BT) void k_force_sym64(Launch L)
{
    __shared__ double sj[3][TJ];
    __shared__ double sv[LAW == 0 ? 1 : 3][TJ];
    __shared__ double rw[4][3][TJ];
    for (int u = L.unit_base + blockIdx.x; u < L.total_units; u += gridDim.x) {
        const SysDesc &S = L.sys[find_sys(L, u, false)];
        const int2 ic = reinterpret_cast<const int2 *>(S.units)[u - S.unit_begin];
        force_unit_sym64<LAW>(S, ic.x, ic.y, sj, sv, rw);
    }
}

// a = G m (sum of the element's own chunk partials, then the reactions of every earlier tile row
// in row order), plain FP64, scattered to the element's own index.
__global__ __launch_bounds__(BT) void k_combine_sym64(Launch L)
{
    const int e = threadIdx.x;
    for (int u = blockIdx.x; u < L.total_tunits; u += gridDim.x) {
        const SysDesc &S = L.sys[find_tile_sys(L, u)];
        const int J = u - S.tunit_begin;
        const int T = S.ntiles;
        const int slot = J * TJ + e;
        const int idx = S.perm[slot];
        if (idx < 0) continue;
        const double *P = static_cast<const double *>(S.part);
        const double *R = reinterpret_cast<const double *>(S.react);
        const size_t na = S.nalloc;
        const int cj = (T - J + S.ch - 1) / S.ch;  // the chunk count of the element's own row
        double out[3];
        for (int d = 0; d < 3; ++d) {
            double sum = 0.0;
            for (int c = 0; c < cj; ++c) sum += P[(size_t)c * 3 * na + d * na + slot];
            // rows are read eight at a time (independent loads in flight), then added in row
            // order; the arithmetic is the same as one row at a time
            size_t off = 0, len = (size_t)(T - 1) * TJ;
            int g = 0;
            for (; g + 8 <= J; g += 8) {
                double v[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    v[q] = R[off + d * len + slot - (size_t)TJ * (g + q + 1)];
                    off += 3 * len;
                    len -= TJ;
                }
#pragma unroll
                for (int q = 0; q < 8; ++q) sum += v[q];
            }
            for (; g < J; ++g) {
                sum += R[off + d * len + slot - (size_t)TJ * (g + 1)];
                off += 3 * len;
                len -= TJ;
            }
            out[d] = sum;
        }
        const double gm = S.st->gm_d;
        static_cast<double *>(S.ax)[idx] = gm * out[0];
        static_cast<double *>(S.ay)[idx] = gm * out[1];
        static_cast<double *>(S.az)[idx] = gm * out[2];
    }
}

// ------------------------------------------------------------------ j-split combine

// Plain mode: sums the chunk partials of each sorted slot in chunk order (plain FP32) and
// scatters a = G m sum to the element's own index.
__global__ __launch_bounds__(BT) void k_combine_f32(Launch L)
{
    for (int u = blockIdx.x; u < L.total_tunits; u += gridDim.x) {
        const SysDesc &S = L.sys[find_tile_sys(L, u)];
        if (S.nsplit == 1) continue;
        const int slot = (u - S.tunit_begin) * TJ + threadIdx.x;
        const int idx = S.perm[slot];
        if (idx < 0) continue;
        const float *P = static_cast<const float *>(S.part);
        const size_t na = S.nalloc;
        float out[3];
        for (int d = 0; d < 3; ++d) {
            float sum = 0.0f;
            for (int c = 0; c < S.nsplit; ++c) sum += P[(size_t)c * 3 * na + d * na + slot];
            out[d] = sum;
        }
        const float gm = S.st->gm_f;
        static_cast<float *>(S.ax)[idx] = gm * out[0];
        static_cast<float *>(S.ay)[idx] = gm * out[1];
        static_cast<float *>(S.az)[idx] = gm * out[2];
    }
}

// ------------------------------------------------------------------ leap-frog and L1 plane

template <typename T>
__device__ __forceinline__ T h_of(const DevState *st);
template <>
__device__ __forceinline__ float h_of<float>(const DevState *st) { return st->h_f; }
template <>
__device__ __forceinline__ double h_of<double>(const DevState *st) { return st->h_d; }
template <typename T>
__device__ __forceinline__ T dt_of(const DevState *st);
template <>
__device__ __forceinline__ float dt_of<float>(const DevState *st) { return st->dt_f; }
template <>
__device__ __forceinline__ double dt_of<double>(const DevState *st) { return st->dt; }

// v += a dt/2; x += v dt
template <typename T>
__global__ __launch_bounds__(BT) void k_kick_drift(Launch L)
{
    for (int u = blockIdx.x; u < L.total_ounits; u += gridDim.x) {
        const SysDesc &S = L.sys[find_sys(L, u, true)];
        const int i = (u - S.ounit_begin) * BT + threadIdx.x;
        if (i >= S.n) continue;
        const T h = h_of<T>(S.st), dt = dt_of<T>(S.st);
        T *x = static_cast<T *>(S.x), *y = static_cast<T *>(S.y), *z = static_cast<T *>(S.z);
        T *vx = static_cast<T *>(S.vx), *vy = static_cast<T *>(S.vy), *vz = static_cast<T *>(S.vz);
        const T *ax = static_cast<const T *>(S.ax), *ay = static_cast<const T *>(S.ay),
                *az = static_cast<const T *>(S.az);
        const T nvx = vx[i] + h * ax[i], nvy = vy[i] + h * ay[i], nvz = vz[i] + h * az[i];
        vx[i] = nvx;
        vy[i] = nvy;
        vz[i] = nvz;
        x[i] = x[i] + dt * nvx;
        y[i] = y[i] + dt * nvy;
        z[i] = z[i] + dt * nvz;
    }
}

// Optional second kick v += a dt/2, then per-unit FP64 sums of each star's positions and the
// count of non-finite elements.
template <typename T>
__global__ __launch_bounds__(BT) void k_kick_stats(Launch L, int do_kick)
{
    __shared__ double lds[7][BT / 64];
    for (int u = blockIdx.x; u < L.total_ounits; u += gridDim.x) {
        const SysDesc &S = L.sys[find_sys(L, u, true)];
        const int local = u - S.ounit_begin;
        const int i = local * BT + threadIdx.x;
        double v[7] = {0, 0, 0, 0, 0, 0, 0};
        if (i < S.n) {
            T *vx = static_cast<T *>(S.vx), *vy = static_cast<T *>(S.vy),
              *vz = static_cast<T *>(S.vz);
            T wx = vx[i], wy = vy[i], wz = vz[i];
            if (do_kick) {
                const T h = h_of<T>(S.st);
                wx = wx + h * static_cast<const T *>(S.ax)[i];
                wy = wy + h * static_cast<const T *>(S.ay)[i];
                wz = wz + h * static_cast<const T *>(S.az)[i];
                vx[i] = wx;
                vy[i] = wy;
                vz[i] = wz;
            }
            const double px = static_cast<const T *>(S.x)[i];
            const double py = static_cast<const T *>(S.y)[i];
            const double pz = static_cast<const T *>(S.z)[i];
            const int o = i >= S.n1 ? 3 : 0;
            v[o + 0] = px;
            v[o + 1] = py;
            v[o + 2] = pz;
            const bool fin = isfinite(px) && isfinite(py) && isfinite(pz) &&
                             isfinite((double)wx) && isfinite((double)wy) && isfinite((double)wz);
            v[6] = fin ? 0.0 : 1.0;
        }
        block_sum<7>(v, lds);
        if (threadIdx.x == 0) {
            double *r = S.red + (size_t)local * RED_STRIDE + RED_STEP;
            for (int k = 0; k < 7; ++k) r[k] = v[k];
        }
    }
}

// One block per system: star centres, L1 plane, non-finite flag and (optionally) the donor
// growth update with the derived force constants.
__global__ __launch_bounds__(BT) void k_finalize_step(Launch L, int do_growth)
{
    __shared__ double lds[7][BT / 64];
    for (int s = blockIdx.x; s < L.n_sys; s += gridDim.x) {
        const SysDesc &S = L.sys[s];
        double v[7] = {0, 0, 0, 0, 0, 0, 0};
        for (int u = threadIdx.x; u < S.n_ounits; u += BT) {
            const double *r = S.red + (size_t)u * RED_STRIDE + RED_STEP;
            for (int k = 0; k < 7; ++k) v[k] += r[k];
        }
        block_sum<7>(v, lds);
        if (threadIdx.x == 0) {
            DevState *st = S.st;
            const int n1 = S.n1, n2 = S.n - S.n1;
            double c1[3], c2[3], e[3];
            for (int d = 0; d < 3; ++d) {
                c1[d] = n1 > 0 ? v[d] / (double)n1 : 0.0;
                c2[d] = n2 > 0 ? v[3 + d] / (double)n2 : 0.0;
                e[d] = c2[d] - c1[d];
                st->com1[d] = c1[d];
                st->com2[d] = c2[d];
            }
            const double dist = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
            const int ok = (n1 > 0 && n2 > 0 && dist > 0.0) ? 1 : 0;
            for (int d = 0; d < 3; ++d) st->e[d] = ok ? e[d] / dist : 0.0;
            st->xi_cut = st->xi_l1 * dist;
            st->plane_ok = ok;
            st->nonfinite = (int32_t)v[6];
            if (do_growth && st->growth_on && !st->growth_stopped) {
                const double R2 = st->R2_0 * st->D2 / st->D2_0;
                if (R2 <= st->rL_a) {
                    st->D2 = st->D2 * (1.0 + st->growth_rate);
                    const double Ds[3] = {st->D1, 0.5 * (st->D1 + st->D2), st->D2};
                    for (int k = 0; k < 3; ++k) {
                        const double D = Ds[k];
                        st->c1d[k] = 11.0 / (D * D * D);
                        st->c2d[k] = 10.0 / (D * D);
                        st->c1f[k] = (float)st->c1d[k];
                        st->c2f[k] = (float)st->c2d[k];
                        st->far2f[k] = (float)(D * D * (1.0 + (double)FAR_MARGIN));
                        st->lD_f[k] = (float)D;
                    }
                } else {
                    st->growth_stopped = 1;
                }
            }
        }
        __syncthreads();
    }
}

// Donor elements: side of the L1 plane, crossings since the previous call.
template <typename T>
__global__ __launch_bounds__(BT) void k_l1_classify(Launch L, int init)
{
    __shared__ double lds[3][BT / 64];
    for (int u = blockIdx.x; u < L.total_ounits; u += gridDim.x) {
        const SysDesc &S = L.sys[find_sys(L, u, true)];
        const int local = u - S.ounit_begin;
        const int i = local * BT + threadIdx.x;
        double v[3] = {0, 0, 0};
        const DevState *st = S.st;
        if (i < S.n && i >= S.n1) {
            const double px = static_cast<const T *>(S.x)[i];
            const double py = static_cast<const T *>(S.y)[i];
            const double pz = static_cast<const T *>(S.z)[i];
            const double xi = (px - st->com1[0]) * st->e[0] + (py - st->com1[1]) * st->e[1] +
                              (pz - st->com1[2]) * st->e[2];
            const int past = (st->plane_ok && xi < st->xi_cut) ? 1 : 0;
            const int prev = S.side[i];
            v[0] = past;
            if (!init) {
                v[1] = (past && !prev) ? 1.0 : 0.0;
                v[2] = (!past && prev) ? 1.0 : 0.0;
            }
            S.side[i] = (int8_t)past;
        }
        block_sum<3>(v, lds);
        if (threadIdx.x == 0) {
            double *r = S.red + (size_t)local * RED_STRIDE + RED_STEP + 8;
            for (int k = 0; k < 3; ++k) r[k] = v[k];
        }
    }
}

__global__ __launch_bounds__(BT) void k_finalize_l1(Launch L, int init)
{
    __shared__ double lds[3][BT / 64];
    for (int s = blockIdx.x; s < L.n_sys; s += gridDim.x) {
        const SysDesc &S = L.sys[s];
        double v[3] = {0, 0, 0};
        for (int u = threadIdx.x; u < S.n_ounits; u += BT) {
            const double *r = S.red + (size_t)u * RED_STRIDE + RED_STEP + 8;
            for (int k = 0; k < 3; ++k) v[k] += r[k];
        }
        block_sum<3>(v, lds);
        if (threadIdx.x == 0) {
            DevState *st = S.st;
            st->n_past = (int32_t)v[0];
            st->fwd = (int32_t)v[1];
            st->bwd = (int32_t)v[2];
            if (!init) {
                const int64_t step = st->step + 1;
                st->step = step;
                int32_t *row = S.l1_log + 4 * (size_t)(step % L1_LOG_CAP);
                row[0] = (int32_t)step;
                row[1] = st->n_past;
                row[2] = st->fwd;
                row[3] = st->bwd;
            }
        }
        __syncthreads();
    }
}

__global__ void k_init_state(DevState *st, DevState init)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *st = init;
}

// ------------------------------------------------------------------ FP64 diagnostics

template <typename T>
__global__ __launch_bounds__(BT) void k_diag_partials(Launch L)
{
    __shared__ double lds[10][BT / 64];
    for (int u = blockIdx.x; u < L.total_ounits; u += gridDim.x) {
        const SysDesc &S = L.sys[find_sys(L, u, true)];
        const int local = u - S.ounit_begin;
        const int i = local * BT + threadIdx.x;
        double v[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (i < S.n) {
            const double m = S.st->m;
            const double x = static_cast<const T *>(S.x)[i], y = static_cast<const T *>(S.y)[i],
                         z = static_cast<const T *>(S.z)[i];
            const double vx = static_cast<const T *>(S.vx)[i],
                         vy = static_cast<const T *>(S.vy)[i],
                         vz = static_cast<const T *>(S.vz)[i];
            v[0] = m * x;
            v[1] = m * y;
            v[2] = m * z;
            v[3] = m * vx;
            v[4] = m * vy;
            v[5] = m * vz;
            v[6] = m * (y * vz - z * vy);
            v[7] = m * (z * vx - x * vz);
            v[8] = m * (x * vy - y * vx);
            v[9] = 0.5 * m * (vx * vx + vy * vy + vz * vz);
        }
        block_sum<10>(v, lds);
        if (threadIdx.x == 0) {
            double *r = S.red + (size_t)local * RED_STRIDE + RED_DIAG;
            for (int k = 0; k < 10; ++k) r[k] = v[k];
        }
    }
}

// Potential energy: each i sums U(r_ij) over all j != i; the total is halved at the end.
// Contact law: U = -A / r for r >= D and A (11 r^2 - 20 D r + 7 D^2) / (2 D^3) inside, A = G m^2,
// the primitive of the law that is continuous at D.
template <typename T>
__global__ __launch_bounds__(BT) void k_pe(Launch L)
{
    __shared__ double sh[3][TJ];
    __shared__ double lds[1][BT / 64];
    for (int u = blockIdx.x; u < L.total_ounits; u += gridDim.x) {
        const SysDesc &S = L.sys[find_sys(L, u, true)];
        const int local = u - S.ounit_begin;
        const int n = S.n, n1 = S.n1;
        const int i = local * BT + threadIdx.x;
        const int ic = min(i, n - 1);
        const T *X = static_cast<const T *>(S.x), *Y = static_cast<const T *>(S.y),
                *Z = static_cast<const T *>(S.z);
        const double xi = X[ic], yi = Y[ic], zi = Z[ic];
        const int si = ic >= n1 ? 1 : 0;
        const DevState *st = S.st;
        const double A = st->G * st->m * st->m;
        double Ds[2];
        for (int js = 0; js < 2; ++js) {
            const int cls = pair_class(si, js);
            Ds[js] = cls == 0 ? st->D1 : (cls == 2 ? st->D2 : 0.5 * (st->D1 + st->D2));
        }
        double acc = 0.0;
        for (int t0 = 0; t0 < n; t0 += TJ) {
            const int j = t0 + threadIdx.x;
            const int jc = min(j, n - 1);
            sh[0][threadIdx.x] = X[jc];
            sh[1][threadIdx.x] = Y[jc];
            sh[2][threadIdx.x] = Z[jc];
            __syncthreads();
            const int jend = min(TJ, n - t0);
            for (int jj = 0; jj < jend; ++jj) {
                const int jg = t0 + jj;
                const double dx = sh[0][jj] - xi, dy = sh[1][jj] - yi, dz = sh[2][jj] - zi;
                const double r = sqrt(dx * dx + dy * dy + dz * dz);
                const double D = Ds[jg >= n1 ? 1 : 0];
                double U;
                if (L.law == 0) {
                    if (r >= D) {
                        U = -A / r;
                    } else {
                        U = A * (11.0 * r * r - 20.0 * D * r + 7.0 * D * D) / (2.0 * D * D * D);
                    }
                } else {
                    // eqs. (4)-(6), converging branch: -A / (r + eps) plus the overlap energy
                    // gamma pi (D - r)^3 (r + 3D) / 48 inside D
                    U = -A / (r + st->leps_d);
                    if (r < D) {
                        const double u = D - r;
                        U += st->gamma * PI_D / 48.0 * u * u * u * (r + 3.0 * D);
                    }
                }
                if (jg != ic && r > 0.0) acc += U;
            }
            __syncthreads();
        }
        double v[1] = {i < n ? acc : 0.0};
        block_sum<1>(v, lds);
        if (threadIdx.x == 0) S.pe_part[local] = 0.5 * v[0];
    }
}

__global__ __launch_bounds__(BT) void k_finalize_diag(Launch L, int with_pe)
{
    __shared__ double lds[11][BT / 64];
    for (int s = blockIdx.x; s < L.n_sys; s += gridDim.x) {
        const SysDesc &S = L.sys[s];
        double v[11] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int u = threadIdx.x; u < S.n_ounits; u += BT) {
            const double *r = S.red + (size_t)u * RED_STRIDE + RED_DIAG;
            for (int k = 0; k < 10; ++k) v[k] += r[k];
            if (with_pe) v[10] += S.pe_part[u];
        }
        block_sum<11>(v, lds);
        if (threadIdx.x == 0) {
            const double M = S.st->m * (double)S.n;
            DiagOut *o = S.diag;
            for (int d = 0; d < 3; ++d) o->v[d] = M > 0.0 ? v[d] / M : 0.0;
            for (int k = 3; k < 11; ++k) o->v[k] = v[k];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ accretor-side retention

// Pass 1: per-unit sums of star 1's velocities.
template <typename T>
__global__ __launch_bounds__(BT) void k_ret_vsum(Launch L)
{
    __shared__ double lds[3][BT / 64];
    for (int u = blockIdx.x; u < L.total_ounits; u += gridDim.x) {
        const SysDesc &S = L.sys[find_sys(L, u, true)];
        const int local = u - S.ounit_begin;
        const int i = local * BT + threadIdx.x;
        double v[3] = {0, 0, 0};
        if (i < S.n1) {
            v[0] = static_cast<const T *>(S.vx)[i];
            v[1] = static_cast<const T *>(S.vy)[i];
            v[2] = static_cast<const T *>(S.vz)[i];
        }
        block_sum<3>(v, lds);
        if (threadIdx.x == 0) {
            double *r = S.red + (size_t)local * RED_STRIDE + RED_RET;
            for (int k = 0; k < 3; ++k) r[k] = v[k];
        }
    }
}

// One block per system: star 1's mean velocity.
__global__ __launch_bounds__(BT) void k_ret_mean(Launch L)
{
    __shared__ double lds[3][BT / 64];
    for (int s = blockIdx.x; s < L.n_sys; s += gridDim.x) {
        const SysDesc &S = L.sys[s];
        double v[3] = {0, 0, 0};
        for (int u = threadIdx.x; u < S.n_ounits; u += BT) {
            const double *r = S.red + (size_t)u * RED_STRIDE + RED_RET;
            for (int k = 0; k < 3; ++k) v[k] += r[k];
        }
        block_sum<3>(v, lds);
        if (threadIdx.x == 0) {
            for (int k = 0; k < 3; ++k) S.st->v1[k] = S.n1 > 0 ? v[k] / (double)S.n1 : 0.0;
        }
        __syncthreads();
    }
}

// Pass 2: donor elements past the L1 plane of the last step, and those of them bound to the
// accretor as a point mass n1 m at its centre, moving with its mean velocity:
// |v - V1|^2 / 2 - G n1 m / |r - C1| < 0, in FP64.
template <typename T>
__global__ __launch_bounds__(BT) void k_ret_count(Launch L)
{
    __shared__ double lds[2][BT / 64];
    for (int u = blockIdx.x; u < L.total_ounits; u += gridDim.x) {
        const SysDesc &S = L.sys[find_sys(L, u, true)];
        const int local = u - S.ounit_begin;
        const int i = local * BT + threadIdx.x;
        const DevState *st = S.st;
        double v[2] = {0, 0};
        if (i < S.n && i >= S.n1 && S.n1 > 0 && st->plane_ok) {
            const double rx = (double)static_cast<const T *>(S.x)[i] - st->com1[0];
            const double ry = (double)static_cast<const T *>(S.y)[i] - st->com1[1];
            const double rz = (double)static_cast<const T *>(S.z)[i] - st->com1[2];
            if (rx * st->e[0] + ry * st->e[1] + rz * st->e[2] < st->xi_cut) {
                v[0] = 1.0;
                const double ux = (double)static_cast<const T *>(S.vx)[i] - st->v1[0];
                const double uy = (double)static_cast<const T *>(S.vy)[i] - st->v1[1];
                const double uz = (double)static_cast<const T *>(S.vz)[i] - st->v1[2];
                const double r = sqrt(rx * rx + ry * ry + rz * rz);
                const double gm1 = st->G * st->m * (double)S.n1;
                const double energy = 0.5 * (ux * ux + uy * uy + uz * uz) - gm1 / r;
                v[1] = energy < 0.0 ? 1.0 : 0.0;
            }
        }
        block_sum<2>(v, lds);
        if (threadIdx.x == 0) {
            double *r = S.red + (size_t)local * RED_STRIDE + RED_RET + 3;
            r[0] = v[0];
            r[1] = v[1];
        }
    }
}

__global__ __launch_bounds__(BT) void k_ret_total(Launch L)
{
    __shared__ double lds[2][BT / 64];
    for (int s = blockIdx.x; s < L.n_sys; s += gridDim.x) {
        const SysDesc &S = L.sys[s];
        double v[2] = {0, 0};
        for (int u = threadIdx.x; u < S.n_ounits; u += BT) {
            const double *r = S.red + (size_t)u * RED_STRIDE + RED_RET + 3;
            v[0] += r[0];
            v[1] += r[1];
        }
        block_sum<2>(v, lds);
        if (threadIdx.x == 0) {
            S.st->ret_past = (int32_t)v[0];
            S.st->ret_bound = (int32_t)v[1];
        }
        __syncthreads();
    }
}

// Copies entry k of the chunk: the system's own SysDesc word by word, with the launch's prefix
// offsets in place of its zero ones. One block per entry.
__global__ __launch_bounds__(64) void k_copy_table(SysDesc *dst, TableChunk c)
{
    static_assert(sizeof(SysDesc) % 4 == 0, "SysDesc is copied in 32-bit words");
    constexpr int W = (int)(sizeof(SysDesc) / 4);
    constexpr int WU = (int)(offsetof(SysDesc, unit_begin) / 4);
    constexpr int WO = (int)(offsetof(SysDesc, ounit_begin) / 4);
    constexpr int WT = (int)(offsetof(SysDesc, tunit_begin) / 4);
    const int k = blockIdx.x;
    const uint32_t *src = reinterpret_cast<const uint32_t *>(c.src[k]);
    uint32_t *out = reinterpret_cast<uint32_t *>(dst + c.first + k);
    for (int w = threadIdx.x; w < W; w += blockDim.x) {
        uint32_t v = src[w];
        if (w == WU) v = (uint32_t)c.unit_begin[k];
        if (w == WO) v = (uint32_t)c.ounit_begin[k];
        if (w == WT) v = (uint32_t)c.tunit_begin[k];
        out[w] = v;
    }
}

// ------------------------------------------------------------------ launchers

static inline int grid_for(int units)
{
    return units < 1 ? 1 : units;
}

hipError_t launch_copy_table(SysDesc *dst, const TableChunk &c, hipStream_t s)
{
    if (c.count < 1 || c.count > TABLE_CHUNK) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_copy_table, dim3(c.count), dim3(64), 0, s, dst, c);
    return hipGetLastError();
}

hipError_t launch_init_state(DevState *st, const DevState &init, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, st, init);
    return hipGetLastError();
}

// sentinel: fill with the padding position; otherwise with zeros (sorted velocities)
hipError_t launch_fill_sorted(void *xs, void *ys, void *zs, int nalloc, int mode, bool sentinel,
                              hipStream_t s)
{
    if (nalloc <= 0) return hipSuccess;
    const dim3 g((nalloc + BT - 1) / BT), b(BT);
    if (mode == 2) {
        hipLaunchKernelGGL(k_fill_sorted<double>, g, b, 0, s, static_cast<double *>(xs),
                           static_cast<double *>(ys), static_cast<double *>(zs), nalloc,
                           sentinel ? SENTINEL_F64 : 0.0);
    } else {
        hipLaunchKernelGGL(k_fill_sorted<float>, g, b, 0, s, static_cast<float *>(xs),
                           static_cast<float *>(ys), static_cast<float *>(zs), nalloc,
                           sentinel ? SENTINEL_F32 : 0.0f);
    }
    return hipGetLastError();
}

hipError_t launch_gather(const Launch &L, int mode, hipStream_t s)
{
    if (L.total_tunits == 0) return hipSuccess;
    const dim3 g(grid_for(L.total_tunits)), b(BT);
    if (mode == 2) {
        hipLaunchKernelGGL(k_gather<double>, g, b, 0, s, L);
    } else {
        hipLaunchKernelGGL(k_gather<float>, g, b, 0, s, L);
    }
    return hipGetLastError();
}

hipError_t launch_forces(const Launch &L, int mode, int max_blocks, hipStream_t s)
{
    if (L.total_units == 0) return hipSuccess;
    if (L.law != 0 && L.law != 1) return hipErrorInvalidValue;
    // max_blocks > 0: persistent launch, each block loops over units u, u + grid, ...
    auto grid = [&](int units) {
        return dim3(grid_for(max_blocks > 0 ? std::min(units, max_blocks) : units));
    };
    Launch R = L;
    R.unit_base = 0;
    if (mode == 0) {
        if (L.law != 0) return hipErrorInvalidValue;  // eqs. (4)-(6) have no plain FP32 kernel
        hipLaunchKernelGGL(k_force_f32, grid(L.total_units), dim3(BT), 0, s, R);
        return hipGetLastError();
    }
    if (mode == 2) {
        if (L.law == 0) {
            hipLaunchKernelGGL(k_force_sym64<0>, grid(L.total_units), dim3(BT), 0, s, R);
        } else {
            hipLaunchKernelGGL(k_force_sym64<1>, grid(L.total_units), dim3(BT), 0, s, R);
        }
        return hipGetLastError();
    }
    // FP32 Kahan: one launch per band height present in the table
    int begin = 0;
    for (int b = 0; b < 3; ++b) {
        const int end = L.band_end[b];
        if (end <= begin) continue;
        R.unit_base = begin;
        R.total_units = end;
        const dim3 g = grid(end - begin), blk(BT);
        switch (b * 2 + L.law) {
        case 0: hipLaunchKernelGGL(k_force_sym<1>, g, blk, 0, s, R); break;
        case 1: hipLaunchKernelGGL(k_force_sym_paper<1>, g, blk, 0, s, R); break;
        case 2: hipLaunchKernelGGL(k_force_sym<2>, g, blk, 0, s, R); break;
        case 3: hipLaunchKernelGGL(k_force_sym_paper<2>, g, blk, 0, s, R); break;
        case 4: hipLaunchKernelGGL(k_force_sym<4>, g, blk, 0, s, R); break;
        default: hipLaunchKernelGGL(k_force_sym_paper<4>, g, blk, 0, s, R); break;
        }
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        begin = end;
    }
    return begin == L.total_units ? hipSuccess : hipErrorInvalidValue;
}

hipError_t launch_combine(const Launch &L, int mode, hipStream_t s)
{
    if (L.total_tunits == 0) return hipSuccess;
    const dim3 g(grid_for(L.total_tunits)), b(BT);
    if (mode == 0) {
        hipLaunchKernelGGL(k_combine_f32, g, b, 0, s, L);
    } else if (mode == 1) {
        hipLaunchKernelGGL(k_combine_sym, g, dim3(BT * COMBINE_SEGS), 0, s, L);
    } else {
        hipLaunchKernelGGL(k_combine_sym64, g, b, 0, s, L);
    }
    return hipGetLastError();
}

hipError_t launch_kick_drift(const Launch &L, int mode, hipStream_t s)
{
    if (L.total_ounits == 0) return hipSuccess;
    const dim3 g(grid_for(L.total_ounits)), b(BT);
    if (mode == 2) {
        hipLaunchKernelGGL(k_kick_drift<double>, g, b, 0, s, L);
    } else {
        hipLaunchKernelGGL(k_kick_drift<float>, g, b, 0, s, L);
    }
    return hipGetLastError();
}

hipError_t launch_kick_stats(const Launch &L, int mode, int do_kick, hipStream_t s)
{
    if (L.total_ounits == 0) return hipSuccess;
    const dim3 g(grid_for(L.total_ounits)), b(BT);
    if (mode == 2) {
        hipLaunchKernelGGL(k_kick_stats<double>, g, b, 0, s, L, do_kick);
    } else {
        hipLaunchKernelGGL(k_kick_stats<float>, g, b, 0, s, L, do_kick);
    }
    return hipGetLastError();
}

hipError_t launch_finalize_step(const Launch &L, int do_growth, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_step, dim3(grid_for(L.n_sys)), dim3(BT), 0, s, L, do_growth);
    return hipGetLastError();
}

hipError_t launch_l1_classify(const Launch &L, int mode, int init, hipStream_t s)
{
    if (L.total_ounits == 0) return hipSuccess;
    const dim3 g(grid_for(L.total_ounits)), b(BT);
    if (mode == 2) {
        hipLaunchKernelGGL(k_l1_classify<double>, g, b, 0, s, L, init);
    } else {
        hipLaunchKernelGGL(k_l1_classify<float>, g, b, 0, s, L, init);
    }
    return hipGetLastError();
}

hipError_t launch_finalize_l1(const Launch &L, int init, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_l1, dim3(grid_for(L.n_sys)), dim3(BT), 0, s, L, init);
    return hipGetLastError();
}

hipError_t launch_diag(const Launch &L, int mode, int with_pe, hipStream_t s)
{
    if (L.total_ounits > 0) {
        const dim3 g(grid_for(L.total_ounits)), b(BT);
        if (mode == 2) {
            hipLaunchKernelGGL(k_diag_partials<double>, g, b, 0, s, L);
            if (with_pe) hipLaunchKernelGGL(k_pe<double>, g, b, 0, s, L);
        } else {
            hipLaunchKernelGGL(k_diag_partials<float>, g, b, 0, s, L);
            if (with_pe) hipLaunchKernelGGL(k_pe<float>, g, b, 0, s, L);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_finalize_diag, dim3(grid_for(L.n_sys)), dim3(BT), 0, s, L, with_pe);
    return hipGetLastError();
}

hipError_t launch_retention(const Launch &L, int mode, hipStream_t s)
{
    if (L.total_ounits > 0) {
        const dim3 g(grid_for(L.total_ounits)), b(BT);
        if (mode == 2) {
            hipLaunchKernelGGL(k_ret_vsum<double>, g, b, 0, s, L);
        } else {
            hipLaunchKernelGGL(k_ret_vsum<float>, g, b, 0, s, L);
        }
    }
    hipLaunchKernelGGL(k_ret_mean, dim3(grid_for(L.n_sys)), dim3(BT), 0, s, L);
    if (L.total_ounits > 0) {
        const dim3 g(grid_for(L.total_ounits)), b(BT);
        if (mode == 2) {
            hipLaunchKernelGGL(k_ret_count<double>, g, b, 0, s, L);
        } else {
            hipLaunchKernelGGL(k_ret_count<float>, g, b, 0, s, L);
        }
    }
    hipLaunchKernelGGL(k_ret_total, dim3(grid_for(L.n_sys)), dim3(BT), 0, s, L);
    return hipGetLastError();
}

}  // namespace nbk
