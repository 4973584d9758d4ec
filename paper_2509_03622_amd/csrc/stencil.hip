// Global 5-point FDFD operator with UPML stretching (Eq. 1, E_z form):
//   (A u)[x,y] = cxm[x] u[x-1,y] + cxp[x] u[x+1,y] + cym[y] u[x,y-1] + cyp[y] u[x,y+1]
//              + (-(cxm[x]+cxp[x]+cym[y]+cyp[y]) - k0^2 eps[x,y]) u[x,y]
// with cxp[x] = -1/(s_x(x+1/2) s_x(x) h^2), cxm[x] = -1/(s_x(x-1/2) s_x(x) h^2)
// (same in y) and zero field outside the grid.  y = A x, or y = b - A x.
//
// HBM-bound: per cell and RHS it reads x (8 B), optionally b (8 B), eps (4 B,
// shared by every RHS) and writes y (8 B).  One thread owns one column x of a
// 64 x ROWS strip and marches up the strip, so every x value comes from HBM
// once: the row below and the current row stay in registers, the row above is
// the one new load, and the x-neighbours of the current row are the adjacent
// lanes' values (L1 hits of the same cache lines).
#include "common.h"

namespace nosdd {

constexpr int ST_BX = 64;
constexpr int ST_BY = 4;
constexpr int ST_ROWS = 8;

// The products and sums are formed in FP64 from FP64 coefficients and rounded
// once: FGMRES relies on w = A z for the exact operator, and with a good
// preconditioner |A| |z| exceeds |A z| by one to two orders of magnitude, so
// FP32 coefficients or FP32 accumulation would put errors above the 1e-6
// tolerance into the Arnoldi relation.  The kernel stays HBM-bound.
__global__ __launch_bounds__(ST_BX *ST_BY) void stencil_kernel(const float2 *__restrict__ x,
                                                               const float2 *__restrict__ b,
                                                               float2 *__restrict__ y,
                                                               const float *__restrict__ eps,
                                                               const double2 *__restrict__ coef,
                                                               const double *__restrict__ k0v, int nx, int ny,
                                                               int n_src, const int *__restrict__ active) {
    const int rhs = blockIdx.z;
    if (active && !active[rhs]) return;
    const int wl = rhs / n_src;
    const long long N = (long long)nx * ny;
    const float2 *xr = x + rhs * N;
    float2 *yr = y + rhs * N;
    const float2 *br = b ? b + rhs * N : nullptr;
    const double2 *cf = coef + wl * coef_stride(nx, ny);
    const double2 *cxm = cf, *cxp = cf + nx, *cym = cf + 2 * nx, *cyp = cf + 2 * nx + ny;
    const double kk = k0v[wl] * k0v[wl];

    const int ix = blockIdx.x * ST_BX + threadIdx.x;
    const int iy0 = (blockIdx.y * ST_BY + threadIdx.y) * ST_ROWS;
    if (ix >= nx || iy0 >= ny) return;
    const int iy1 = min(iy0 + ST_ROWS, ny);
    const double2 am = cxm[ix], ap = cxp[ix];
    const float2 zero = make_float2(0.f, 0.f);
    auto wide = [](float2 v) { return make_double2(v.x, v.y); };

    float2 below = iy0 > 0 ? xr[(long long)(iy0 - 1) * nx + ix] : zero;
    float2 cur = xr[(long long)iy0 * nx + ix];
    for (int iy = iy0; iy < iy1; ++iy) {
        const long long row = (long long)iy * nx;
        const float2 above = iy + 1 < ny ? xr[row + nx + ix] : zero;
        const float2 left = ix > 0 ? xr[row + ix - 1] : zero;
        const float2 right = ix + 1 < nx ? xr[row + ix + 1] : zero;
        const double2 bm = cym[iy], bp = cyp[iy];
        const double2 d = make_double2(-(am.x + ap.x + bm.x + bp.x) - kk * (double)eps[row + ix],
                                       -(am.y + ap.y + bm.y + bp.y));
        double2 acc = zmul(d, wide(cur));
        acc = zadd(acc, zmul(am, wide(left)));
        acc = zadd(acc, zmul(ap, wide(right)));
        acc = zadd(acc, zmul(bm, wide(below)));
        acc = zadd(acc, zmul(bp, wide(above)));
        if (br) acc = zsub(wide(br[row + ix]), acc);
        yr[row + ix] = make_float2((float)acc.x, (float)acc.y);
        below = cur;
        cur = above;
    }
}

void launch_stencil(hipStream_t s, const float2 *x, const float2 *b, float2 *y, const float *eps,
                    const double2 *coef, const double *k0, int nx, int ny, int n_rhs, int n_src,
                    const int *active) {
    dim3 block(ST_BX, ST_BY);
    dim3 grid((nx + ST_BX - 1) / ST_BX, (ny + ST_BY * ST_ROWS - 1) / (ST_BY * ST_ROWS), n_rhs);
    hipLaunchKernelGGL(stencil_kernel, grid, block, 0, s, x, b, y, eps, coef, k0, nx, ny, n_src, active);
}

// r = b - A x with the iterate x kept in FP64 (mixed-precision refinement of
// the outer iteration): the residual is formed in FP64 and rounded once.
__global__ __launch_bounds__(ST_BX *ST_BY) void residual64_kernel(const double2 *__restrict__ x,
                                                                  const float2 *__restrict__ b,
                                                                  float2 *__restrict__ r,
                                                                  const float *__restrict__ eps,
                                                                  const double2 *__restrict__ coef,
                                                                  const double *__restrict__ k0v, int nx, int ny,
                                                                  int n_src) {
    const int rhs = blockIdx.z;
    const int wl = rhs / n_src;
    const long long N = (long long)nx * ny;
    const double2 *xr = x + rhs * N;
    const double2 *cf = coef + wl * coef_stride(nx, ny);
    const double2 *cxm = cf, *cxp = cf + nx, *cym = cf + 2 * nx, *cyp = cf + 2 * nx + ny;
    const double kk = k0v[wl] * k0v[wl];
    const int ix = blockIdx.x * ST_BX + threadIdx.x;
    const int iy0 = (blockIdx.y * ST_BY + threadIdx.y) * ST_ROWS;
    if (ix >= nx || iy0 >= ny) return;
    const int iy1 = min(iy0 + ST_ROWS, ny);
    const double2 am = cxm[ix], ap = cxp[ix];
    const double2 zero = make_double2(0.0, 0.0);
    double2 below = iy0 > 0 ? xr[(long long)(iy0 - 1) * nx + ix] : zero;
    double2 cur = xr[(long long)iy0 * nx + ix];
    for (int iy = iy0; iy < iy1; ++iy) {
        const long long row = (long long)iy * nx;
        const double2 above = iy + 1 < ny ? xr[row + nx + ix] : zero;
        const double2 left = ix > 0 ? xr[row + ix - 1] : zero;
        const double2 right = ix + 1 < nx ? xr[row + ix + 1] : zero;
        const double2 bm = cym[iy], bp = cyp[iy];
        double2 d = make_double2(-(am.x + ap.x + bm.x + bp.x) - kk * (double)eps[row + ix], -(am.y + ap.y + bm.y + bp.y));
        double2 acc = zmul(d, cur);
        acc = zadd(acc, zmul(am, left));
        acc = zadd(acc, zmul(ap, right));
        acc = zadd(acc, zmul(bm, below));
        acc = zadd(acc, zmul(bp, above));
        const float2 bv = b[rhs * N + row + ix];
        r[rhs * N + row + ix] = make_float2((float)((double)bv.x - acc.x), (float)((double)bv.y - acc.y));
        below = cur;
        cur = above;
    }
}

void launch_residual64(hipStream_t s, const double2 *x, const float2 *b, float2 *r, const float *eps,
                       const double2 *coef, const double *k0, int nx, int ny, int n_rhs, int n_src) {
    dim3 block(ST_BX, ST_BY);
    dim3 grid((nx + ST_BX - 1) / ST_BX, (ny + ST_BY * ST_ROWS - 1) / (ST_BY * ST_ROWS), n_rhs);
    hipLaunchKernelGGL(residual64_kernel, grid, block, 0, s, x, b, r, eps, coef, k0, nx, ny, n_src);
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
