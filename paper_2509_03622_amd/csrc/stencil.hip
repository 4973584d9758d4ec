// Global 5-point FDFD operator with UPML stretching (Eq. 1, E_z form):
//   (A u)[x,y] = cxm[x] u[x-1,y] + cxp[x] u[x+1,y] + cym[y] u[x,y-1] + cyp[y] u[x,y+1]
//              + (-(cxm[x]+cxp[x]+cym[y]+cyp[y]) - k0^2 eps[x,y]) u[x,y]
// with cxp[x] = -1/(s_x(x+1/2) s_x(x) h^2), cxm[x] = -1/(s_x(x-1/2) s_x(x) h^2)
// (same in y) and zero field outside the grid.  y = A x, or y = b - A x.
//
// HBM-bound: per cell and RHS it reads x (8 B), optionally b (8 B), eps (4 B,
// shared by every RHS) and writes y (8 B).  A wave owns 64 consecutive cells
// of a row (aligned stores); the x-neighbours inside the wave arrive by DPP
// wave shifts, and the two outside it come from one extra load per row
// (lane 0 fetches the cell on the left, lane 1 the cell on the right) read
// back with readlane.  Each thread walks ST_ROWS rows of its column with all
// loads issued before the first use; the per-row y coefficients are
// wave-uniform scalar loads.
#include "common.h"

namespace nosdd {

constexpr int ST_WAVES = 4;
constexpr int ST_ROWS = 8;

// Whole-wave lane shifts (DPP): from lane i - 1, and from lane i + 1.
constexpr int DPP_WAVE_SHR1 = 0x138;
constexpr int DPP_WAVE_SHL1 = 0x130;
template <int CTRL>
__device__ __forceinline__ float lane_shift(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double lane_shift(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(u & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(u >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL> __device__ __forceinline__ float2 lane_shift(float2 v) {
    return make_float2(lane_shift<CTRL>(v.x), lane_shift<CTRL>(v.y));
}
template <int CTRL> __device__ __forceinline__ double2 lane_shift(double2 v) {
    return make_double2(lane_shift<CTRL>(v.x), lane_shift<CTRL>(v.y));
}
__device__ __forceinline__ float read_lane1(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 1));
}
__device__ __forceinline__ double read_lane1(double v) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), 1);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), 1);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float2 read_lane1(float2 v) { return make_float2(read_lane1(v.x), read_lane1(v.y)); }
__device__ __forceinline__ double2 read_lane1(double2 v) { return make_double2(read_lane1(v.x), read_lane1(v.y)); }
__device__ __forceinline__ double2 wide(float2 v) { return make_double2(v.x, v.y); }
__device__ __forceinline__ double2 wide(double2 v) { return v; }
template <typename T> __device__ __forceinline__ T zero_of();
template <> __device__ __forceinline__ float2 zero_of<float2>() { return make_float2(0.f, 0.f); }
template <> __device__ __forceinline__ double2 zero_of<double2>() { return make_double2(0.0, 0.0); }

// The products and sums are formed in FP64 from FP64 coefficients and rounded
// once: FGMRES relies on w = A z for the exact operator, and with a good
// preconditioner |A| |z| exceeds |A z| by one to two orders of magnitude, so
// FP32 coefficients or FP32 accumulation would put errors above the 1e-6
// tolerance into the Arnoldi relation.  The kernel stays HBM-bound.
//
// XT is the type of x: float2, or double2 for the residual of the FP64 outer
// iterate.  HAS_B: y = b - A x, else y = A x.  NT: streaming (non-temporal)
// stores, for outputs too large to stay in the last-level cache.
template <typename XT, bool HAS_B, bool NT>
__global__ __launch_bounds__(64 * ST_WAVES) void stencil_kernel(const XT *__restrict__ x,
                                                                const XT *__restrict__ b,
                                                                float2 *__restrict__ y,
                                                                const float *__restrict__ eps,
                                                                const double2 *__restrict__ coef,
                                                                const double *__restrict__ k0v, int nx, int ny,
                                                                int n_src, const int *__restrict__ active) {
    const int rhs = blockIdx.x;
    if (active && !active[rhs]) return;
    const int wl = rhs / n_src;
    const long long N = (long long)nx * ny;
    const XT *xr = x + rhs * N;
    float2 *yr = y + rhs * N;
    const XT *br = HAS_B ? b + rhs * N : nullptr;
    const double2 *cf = coef + wl * coef_stride(nx, ny);
    const double2 *cxm = cf, *cxp = cf + nx, *cym = cf + 2 * nx, *cyp = cf + 2 * nx + ny;
    const double kk = k0v[wl] * k0v[wl];

    const int lane = threadIdx.x;
    const int ix0 = blockIdx.y * 64;
    const int ix = ix0 + lane;
    const int iy0 = __builtin_amdgcn_readfirstlane((blockIdx.z * ST_WAVES + threadIdx.y) * ST_ROWS);
    if (iy0 >= ny) return;
    const bool inx = ix < nx;
    const int ixc = min(ix, nx - 1);
    // lane 0: the cell left of the wave, lane 1: the cell right of it
    const int hx = lane == 0 ? ix0 - 1 : ix0 + 64;
    const bool hin = hx >= 0 && hx < nx;
    const int hxc = min(max(hx, 0), nx - 1);
    const XT zero = zero_of<XT>();

    XT xv[ST_ROWS + 2], xh[ST_ROWS];
    float ev[ST_ROWS];
    XT bv[ST_ROWS] = {};
#pragma unroll
    for (int i = 0; i < ST_ROWS + 2; ++i) {
        const int iyc = min(max(iy0 - 1 + i, 0), ny - 1);
        xv[i] = xr[(long long)iyc * nx + ixc];
    }
#pragma unroll
    for (int i = 0; i < ST_ROWS; ++i) {
        const long long row = (long long)min(iy0 + i, ny - 1) * nx;
        xh[i] = xr[row + hxc];
        ev[i] = eps[row + ixc];
        if (HAS_B) bv[i] = br[row + ixc];
    }
    const double2 am = cxm[ixc], ap = cxp[ixc];
    const double sx = am.x + ap.x;
    // Outside the PML every coupling is real (the stretch is exactly 1 there):
    // the real-coefficient form below then gives the same products with half
    // the FP64 work.  Decided per wave (x) and per row (y).
    const bool xreal = __all(am.y == 0.0 && ap.y == 0.0);
    // zero field outside the grid
#pragma unroll
    for (int i = 0; i < ST_ROWS + 2; ++i) {
        const int iy = iy0 - 1 + i;
        if (!inx || iy < 0 || iy >= ny) xv[i] = zero;
    }
#pragma unroll
    for (int i = 0; i < ST_ROWS; ++i) {
        const int iy = iy0 + i;
        if (iy >= ny) break;
        if (!hin) xh[i] = zero;
        XT left = lane_shift<DPP_WAVE_SHR1>(xv[i + 1]);
        XT right = lane_shift<DPP_WAVE_SHL1>(xv[i + 1]);
        const XT rh = read_lane1(xh[i]);
        if (lane == 0) left = xh[i];
        if (lane == 63) right = rh;
        const double2 bm = cym[iy], bp = cyp[iy];
        const double dr = -((sx + bm.x) + bp.x) - kk * (double)ev[i];
        const double2 xc = wide(xv[i + 1]), xl = wide(left), xr_ = wide(right), xb = wide(xv[i]), xt = wide(xv[i + 2]);
        double2 acc;
        if (xreal && bm.y == 0.0 && bp.y == 0.0) {
            acc.x = dr * xc.x;
            acc.y = dr * xc.y;
            acc.x = fma(am.x, xl.x, acc.x);
            acc.y = fma(am.x, xl.y, acc.y);
            acc.x = fma(ap.x, xr_.x, acc.x);
            acc.y = fma(ap.x, xr_.y, acc.y);
            acc.x = fma(bm.x, xb.x, acc.x);
            acc.y = fma(bm.x, xb.y, acc.y);
            acc.x = fma(bp.x, xt.x, acc.x);
            acc.y = fma(bp.x, xt.y, acc.y);
        } else {
            const double2 d = make_double2(dr, -(am.y + ap.y + bm.y + bp.y));
            acc = zmul(d, xc);
            acc = zadd(acc, zmul(am, xl));
            acc = zadd(acc, zmul(ap, xr_));
            acc = zadd(acc, zmul(bm, xb));
            acc = zadd(acc, zmul(bp, xt));
        }
        if (HAS_B) acc = zsub(wide(bv[i]), acc);
        if (inx) {
            float2 *dst = yr + (long long)iy * nx + ix;
            if (NT) {
                typedef float f32x2 __attribute__((ext_vector_type(2)));
                const f32x2 v = {(float)acc.x, (float)acc.y};
                __builtin_nontemporal_store(v, reinterpret_cast<f32x2 *>(dst));
            } else {
                *dst = make_float2((float)acc.x, (float)acc.y);
            }
        }
    }
}

static dim3 stencil_grid(int nx, int ny, int n_rhs) {
    // RHS fastest: the blocks of one grid patch run together and share eps in L2
    return dim3(n_rhs, (nx + 63) / 64, (ny + ST_WAVES * ST_ROWS - 1) / (ST_WAVES * ST_ROWS));
}

// Outputs above this size cannot stay in the 256 MB last-level cache for the
// next kernel, so they are written with streaming stores.
constexpr long long ST_STREAM_BYTES = 256LL << 20;

template <typename XT, bool HAS_B>
static void stencil_launch(hipStream_t s, const XT *x, const XT *b, float2 *y, const float *eps,
                           const double2 *coef, const double *k0, int nx, int ny, int n_rhs, int n_src,
                           const int *active) {
    const bool nt = (long long)nx * ny * n_rhs * (long long)sizeof(float2) > ST_STREAM_BYTES;
    if (nt)
        hipLaunchKernelGGL((stencil_kernel<XT, HAS_B, true>), stencil_grid(nx, ny, n_rhs), dim3(64, ST_WAVES), 0, s,
                           x, b, y, eps, coef, k0, nx, ny, n_src, active);
    else
        hipLaunchKernelGGL((stencil_kernel<XT, HAS_B, false>), stencil_grid(nx, ny, n_rhs), dim3(64, ST_WAVES), 0, s,
                           x, b, y, eps, coef, k0, nx, ny, n_src, active);
}

void launch_stencil(hipStream_t s, const float2 *x, const float2 *b, float2 *y, const float *eps,
                    const double2 *coef, const double *k0, int nx, int ny, int n_rhs, int n_src,
                    const int *active) {
    if (b)
        stencil_launch<float2, true>(s, x, b, y, eps, coef, k0, nx, ny, n_rhs, n_src, active);
    else
        stencil_launch<float2, false>(s, x, b, y, eps, coef, k0, nx, ny, n_rhs, n_src, active);
}

// r = b - A x with the iterate x and the right-hand side b kept in FP64
// (mixed-precision refinement of the outer iteration): the residual is formed
// in FP64 and rounded once.
void launch_residual64(hipStream_t s, const double2 *x, const double2 *b, float2 *r, const float *eps,
                       const double2 *coef, const double *k0, int nx, int ny, int n_rhs, int n_src) {
    stencil_launch<double2, true>(s, x, b, r, eps, coef, k0, nx, ny, n_rhs, n_src, nullptr);
}

// Robin traces g_p = (x_q - x_p)/h + i kappa_p (x_q + x_p)/2 at interface-ring
// entries; entries[e] = (p, q, unused, unused) as linear cell indices.
__global__ void robin_trace_kernel(const int4 *__restrict__ ent, int n_e, const float *__restrict__ eps,
                                   const float *__restrict__ k0, float h, long long N,
                                   const float2 *__restrict__ x, float2 *__restrict__ g, int vec_per_wl) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    const int v = blockIdx.y;
    if (e >= n_e) return;
    const int wl = v / vec_per_wl;
    const int4 pq = ent[e];
    const float2 up = x[v * N + pq.x], uq = x[v * N + pq.y];
    const float kap = k0[wl] * sqrtf(eps[pq.x]);
    float2 r;
    r.x = (uq.x - up.x) / h - 0.5f * kap * (uq.y + up.y);
    r.y = (uq.y - up.y) / h + 0.5f * kap * (uq.x + up.x);
    g[(long long)v * n_e + e] = r;
}

void launch_robin_trace(hipStream_t s, const int4 *entries, int n_entries, const float *eps, const float *k0,
                        float h, int nx, int ny, const float2 *x, float2 *g, int n_vec, int vec_per_wl) {
    if (n_entries == 0) return;
    dim3 grid((n_entries + 255) / 256, n_vec);
    hipLaunchKernelGGL(robin_trace_kernel, grid, dim3(256), 0, s, entries, n_entries, eps, k0, h,
                       (long long)nx * ny, x, g, vec_per_wl);
}

}  // namespace nosdd
