// nb_kernels.hip -- gfx950 kernels of libnbody.
//
// The O(N^2) all-pairs force evaluation (Methodology: every element moves only under the sum of
// all pairwise element-element interactions) is the hot path. It runs on the FP32 vector ALUs:
// the pair sum is not a dense contraction, so there is no MFMA here. Each lane keeps KI i
// elements in registers, the block streams j elements through LDS in 256-element SoA tiles
// (coalesced global loads, double-buffered, one barrier per tile) and each wave reads a tile
// back with broadcast ds_read_b128. Per pair:
//   d = r_j - r_i,  r2 = d.d + eps,  w = rsqrt(r2)  (v_rsq_f32),
//   s = min(w^3, c1 - c2 w),  acc += s d,
// where c1 = 11 / D^3 and c2 = 10 / D^2 for the pair's diameter D. Dividing the contact law
// f(r) = G m^2 / r^2 (r >= D), G m^2 r / D^3 - K (1 - r/D) (r < D, K = 10 G m^2 / D^2) by
// G m^2 r gives w^3 outside and c1 - c2 w inside; with x = r/D, 11 - 10/x - 1/x^3 is increasing
// and vanishes at x = 1, so the smaller of the two expressions is always the right branch.
// The self pair has d = 0 exactly and contributes 0; eps = 1e-24 keeps its w finite.
//
// The remaining kernels are O(N): leap-frog kicks and drift, per-star centres of mass, the
// donor growth update (eq. 3), the L1-plane count and the FP64 diagnostics. Every reduction runs
// in a fixed order (butterfly within a wave, waves in index order, units in index order), so
// results do not depend on scheduling or on which other systems share a launch.
#include "nb_internal.h"

#include <math.h>

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

// ------------------------------------------------------------------ FP32 force kernel

template <int KI>
struct IState {
    float x[KI], y[KI], z[KI];
    float ax[KI], ay[KI], az[KI];
};

template <int KI>
__device__ __forceinline__ void interact_tile_f32(const float *__restrict__ sx,
                                                  const float *__restrict__ sy,
                                                  const float *__restrict__ sz, IState<KI> &I,
                                                  const float (&c1)[KI], const float (&nc2)[KI])
{
    const float eps = 1.0e-24f;
#pragma unroll 2
    for (int jj = 0; jj < TJ; jj += 4) {
        const float4 X = *reinterpret_cast<const float4 *>(sx + jj);
        const float4 Y = *reinterpret_cast<const float4 *>(sy + jj);
        const float4 Z = *reinterpret_cast<const float4 *>(sz + jj);
        const float xs[4] = {X.x, X.y, X.z, X.w};
        const float ys[4] = {Y.x, Y.y, Y.z, Y.w};
        const float zs[4] = {Z.x, Z.y, Z.z, Z.w};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int k = 0; k < KI; ++k) {
                const float dx = xs[q] - I.x[k];
                const float dy = ys[q] - I.y[k];
                const float dz = zs[q] - I.z[k];
                const float r2 = fmaf(dx, dx, fmaf(dy, dy, fmaf(dz, dz, eps)));
                const float w = __builtin_amdgcn_rsqf(r2);
                const float w3 = (w * w) * w;
                const float s = fminf(w3, fmaf(nc2[k], w, c1[k]));
                I.ax[k] = fmaf(s, dx, I.ax[k]);
                I.ay[k] = fmaf(s, dy, I.ay[k]);
                I.az[k] = fmaf(s, dz, I.az[k]);
            }
        }
    }
}

// One force unit: the i-block `ib` of system S against j chunk `c`.
template <int KI, bool KAHAN>
__device__ __forceinline__ void force_unit_f32(const SysDesc &S, int ib, int c,
                                               float (*sh)[3][TJ])
{
    const int tid = threadIdx.x;
    const int n = S.n, n1 = S.n1;
    const float *__restrict__ X = static_cast<const float *>(S.x);
    const float *__restrict__ Y = static_cast<const float *>(S.y);
    const float *__restrict__ Z = static_cast<const float *>(S.z);
    const DevState *st = S.st;

    IState<KI> I;
    float c1a[KI], nc2a[KI], c1b[KI], nc2b[KI];
    const int i0 = ib * (BT * KI);
#pragma unroll
    for (int k = 0; k < KI; ++k) {
        const int i = min(i0 + k * BT + tid, n - 1);
        I.x[k] = X[i];
        I.y[k] = Y[i];
        I.z[k] = Z[i];
        I.ax[k] = I.ay[k] = I.az[k] = 0.0f;
        const int si = i >= n1 ? 1 : 0;
        c1a[k] = st->c1f[pair_class(si, 0)];
        nc2a[k] = -st->c2f[pair_class(si, 0)];
        c1b[k] = st->c1f[pair_class(si, 1)];
        nc2b[k] = -st->c2f[pair_class(si, 1)];
    }
    float sumx[KI], sumy[KI], sumz[KI], cx[KI], cy[KI], cz[KI];
#pragma unroll
    for (int k = 0; k < KI; ++k) sumx[k] = sumy[k] = sumz[k] = cx[k] = cy[k] = cz[k] = 0.0f;

    // j range of this chunk, split at n1 into a star-1 and a star-2 segment
    const int j0 = c * S.jchunk;
    const int j1 = min(n, j0 + S.jchunk);
    const int a0 = j0, a1 = min(j1, n1);
    const int b0 = max(j0, n1), b1 = j1;
    const int ta = a1 > a0 ? (a1 - a0 + TJ - 1) / TJ : 0;
    const int tb = b1 > b0 ? (b1 - b0 + TJ - 1) / TJ : 0;
    const int nt = ta + tb;

    auto fetch = [&](int t, float &px, float &py, float &pz) {
        int start, end;
        if (t < ta) {
            start = a0 + t * TJ;
            end = a1;
        } else {
            start = b0 + (t - ta) * TJ;
            end = b1;
        }
        const int j = start + tid;
        if (j < end) {
            px = X[j];
            py = Y[j];
            pz = Z[j];
        } else {
            px = py = pz = SENTINEL_F32;
        }
    };

    float px = 0.f, py = 0.f, pz = 0.f;
    if (nt > 0) fetch(0, px, py, pz);
    for (int t = 0; t < nt; ++t) {
        const int buf = t & 1;
        sh[buf][0][tid] = px;
        sh[buf][1][tid] = py;
        sh[buf][2][tid] = pz;
        __syncthreads();
        if (t + 1 < nt) fetch(t + 1, px, py, pz);
        if (t < ta) {
            interact_tile_f32<KI>(sh[buf][0], sh[buf][1], sh[buf][2], I, c1a, nc2a);
        } else {
            interact_tile_f32<KI>(sh[buf][0], sh[buf][1], sh[buf][2], I, c1b, nc2b);
        }
        if (KAHAN) {
#pragma unroll
            for (int k = 0; k < KI; ++k) {
                kahan_add(sumx[k], cx[k], I.ax[k]);
                kahan_add(sumy[k], cy[k], I.ay[k]);
                kahan_add(sumz[k], cz[k], I.az[k]);
                I.ax[k] = I.ay[k] = I.az[k] = 0.0f;
            }
        }
    }
    __syncthreads();  // the next unit of this block reuses both LDS buffers

    const float gm = st->gm_f;
#pragma unroll
    for (int k = 0; k < KI; ++k) {
        const int i = i0 + k * BT + tid;
        if (i >= n) continue;
        float vx, vy, vz;
        if (KAHAN) {
            vx = sumx[k] - cx[k];
            vy = sumy[k] - cy[k];
            vz = sumz[k] - cz[k];
        } else {
            vx = I.ax[k];
            vy = I.ay[k];
            vz = I.az[k];
        }
        if (S.nsplit == 1) {
            static_cast<float *>(S.ax)[i] = gm * vx;
            static_cast<float *>(S.ay)[i] = gm * vy;
            static_cast<float *>(S.az)[i] = gm * vz;
        } else {
            float *P = static_cast<float *>(S.part);
            const size_t base = (size_t)c * 3 * n;
            P[base + i] = vx;
            P[base + n + i] = vy;
            P[base + 2 * (size_t)n + i] = vz;
        }
    }
}

template <int KI, bool KAHAN>
__global__ __launch_bounds__(BT) void k_force_f32(Launch L)
{
    __shared__ __attribute__((aligned(16))) float sh[2][3][TJ];
    for (int u = blockIdx.x; u < L.total_units; u += gridDim.x) {
        const int s = find_sys(L, u, false);
        const SysDesc &S = L.sys[s];
        const int local = u - S.unit_begin;
        const int ib = local / S.nsplit;
        const int c = local - ib * S.nsplit;
        force_unit_f32<KI, KAHAN>(S, ib, c, sh);
    }
}

// ------------------------------------------------------------------ FP64 force kernel

__device__ __forceinline__ double rsqrt_f64(double r2)
{
    // hardware estimate refined by two Newton steps y <- y (3 - r2 y^2) / 2
    double y = __builtin_amdgcn_rsq(r2);
    const double h = 0.5 * r2;
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

__device__ void force_unit_f64(const SysDesc &S, int ib, int c, double (*sh)[4][TJ])
{
    const int tid = threadIdx.x;
    const int n = S.n, n1 = S.n1;
    const double *__restrict__ X = static_cast<const double *>(S.x);
    const double *__restrict__ Y = static_cast<const double *>(S.y);
    const double *__restrict__ Z = static_cast<const double *>(S.z);
    const DevState *st = S.st;
    const int i = ib * BT + tid;
    const int ic = min(i, n - 1);
    const double xi = X[ic], yi = Y[ic], zi = Z[ic];
    const int si = ic >= n1 ? 1 : 0;
    double ax = 0.0, ay = 0.0, az = 0.0;

    const int j0 = c * S.jchunk;
    const int j1 = min(n, j0 + S.jchunk);
    const int a0 = j0, a1 = min(j1, n1);
    const int b0 = max(j0, n1), b1 = j1;
    const int ta = a1 > a0 ? (a1 - a0 + TJ - 1) / TJ : 0;
    const int tb = b1 > b0 ? (b1 - b0 + TJ - 1) / TJ : 0;
    const int nt = ta + tb;
    for (int t = 0; t < nt; ++t) {
        int start, end, js;
        if (t < ta) {
            start = a0 + t * TJ;
            end = a1;
            js = 0;
        } else {
            start = b0 + (t - ta) * TJ;
            end = b1;
            js = 1;
        }
        const int j = start + tid;
        const bool ok = j < end;
        sh[0][0][tid] = ok ? X[j] : 0.0;
        sh[0][1][tid] = ok ? Y[j] : 0.0;
        sh[0][2][tid] = ok ? Z[j] : 0.0;
        sh[0][3][tid] = ok ? 1.0 : 0.0;
        __syncthreads();
        const int cls = pair_class(si, js);
        const double c1 = st->c1d[cls], c2 = st->c2d[cls];
        for (int jj = 0; jj < TJ; ++jj) {
            const double dx = sh[0][0][jj] - xi;
            const double dy = sh[0][1][jj] - yi;
            const double dz = sh[0][2][jj] - zi;
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            const double w = r2 > 0.0 ? rsqrt_f64(r2) : 0.0;
            const double w3 = w * w * w;
            const double s = fmin(w3, c1 - c2 * w) * sh[0][3][jj];
            ax = fma(s, dx, ax);
            ay = fma(s, dy, ay);
            az = fma(s, dz, az);
        }
        __syncthreads();
    }
    if (i < n) {
        if (S.nsplit == 1) {
            const double gm = st->gm_d;
            static_cast<double *>(S.ax)[i] = gm * ax;
            static_cast<double *>(S.ay)[i] = gm * ay;
            static_cast<double *>(S.az)[i] = gm * az;
        } else {
            double *P = static_cast<double *>(S.part);
            const size_t base = (size_t)c * 3 * n;
            P[base + i] = ax;
            P[base + n + i] = ay;
            P[base + 2 * (size_t)n + i] = az;
        }
    }
}

__global__ __launch_bounds__(BT) void k_force_f64(Launch L)
{
    __shared__ double sh[1][4][TJ];
    for (int u = blockIdx.x; u < L.total_units; u += gridDim.x) {
        const int s = find_sys(L, u, false);
        const SysDesc &S = L.sys[s];
        const int local = u - S.unit_begin;
        const int ib = local / S.nsplit;
        const int c = local - ib * S.nsplit;
        force_unit_f64(S, ib, c, sh);
    }
}

// ------------------------------------------------------------------ j-split combine

template <typename T, bool KAHAN>
__global__ __launch_bounds__(BT) void k_combine(Launch L)
{
    for (int u = blockIdx.x; u < L.total_ounits; u += gridDim.x) {
        const SysDesc &S = L.sys[find_sys(L, u, true)];
        if (S.nsplit == 1) continue;
        const int i = (u - S.ounit_begin) * BT + threadIdx.x;
        if (i >= S.n) continue;
        const T *P = static_cast<const T *>(S.part);
        const size_t n = S.n;
        T out[3];
        for (int d = 0; d < 3; ++d) {
            T sum = 0, comp = 0;
            for (int c = 0; c < S.nsplit; ++c) {
                const T v = P[(size_t)c * 3 * n + d * n + i];
                if (KAHAN) {
                    const T y = v - comp;
                    const T t = sum + y;
                    comp = (t - sum) - y;
                    sum = t;
                } else {
                    sum += v;
                }
            }
            out[d] = KAHAN ? sum - comp : sum;
        }
        T gm;
        if constexpr (sizeof(T) == 4) {
            gm = S.st->gm_f;
        } else {
            gm = S.st->gm_d;
        }
        static_cast<T *>(S.ax)[i] = gm * out[0];
        static_cast<T *>(S.ay)[i] = gm * out[1];
        static_cast<T *>(S.az)[i] = gm * out[2];
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
// U = -A / r for r >= D and A (11 r^2 - 20 D r + 7 D^2) / (2 D^3) inside, A = G m^2: the
// primitive of the contact law that is continuous at D.
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
                if (r >= D) {
                    U = -A / r;
                } else {
                    U = A * (11.0 * r * r - 20.0 * D * r + 7.0 * D * D) / (2.0 * D * D * D);
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

// ------------------------------------------------------------------ launchers

static inline int grid_for(int units)
{
    return units < 1 ? 1 : units;
}

hipError_t launch_init_state(DevState *st, const DevState &init, hipStream_t s)
{
    hipLaunchKernelGGL(k_init_state, dim3(1), dim3(64), 0, s, st, init);
    return hipGetLastError();
}

hipError_t launch_forces(const Launch &L, int mode, hipStream_t s)
{
    if (L.total_units == 0) return hipSuccess;
    const dim3 g(grid_for(L.total_units)), b(BT);
    if (mode == 0) {
        hipLaunchKernelGGL((k_force_f32<KI32, false>), g, b, 0, s, L);
    } else if (mode == 1) {
        hipLaunchKernelGGL((k_force_f32<KI32, true>), g, b, 0, s, L);
    } else {
        hipLaunchKernelGGL(k_force_f64, g, b, 0, s, L);
    }
    return hipGetLastError();
}

hipError_t launch_combine(const Launch &L, int mode, hipStream_t s)
{
    if (L.total_ounits == 0) return hipSuccess;
    const dim3 g(grid_for(L.total_ounits)), b(BT);
    if (mode == 0) {
        hipLaunchKernelGGL((k_combine<float, false>), g, b, 0, s, L);
    } else if (mode == 1) {
        hipLaunchKernelGGL((k_combine<float, true>), g, b, 0, s, L);
    } else {
        hipLaunchKernelGGL((k_combine<double, false>), g, b, 0, s, L);
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

}  // namespace nbk
