// Exact subdomain solves u = B_i^-1 v for the local Robin matrices B_i (Eq. 2
// boundary condition eliminated into the diagonal of the interface nodes).
//
// B_i is block-tridiagonal: nb blocks (grid rows or columns of the tile) of
// size b; within a block the couplings are the 1D stencil (tridiagonal),
// between consecutive blocks they are a scalar times the identity
// (c_lo(k) to block k-1, c_hi(k) to block k+1).  Block LU ("block Thomas"):
//   D_0 = A_00,  D_k = A_kk - c_lo(k) c_hi(k-1) D_{k-1}^-1,
//   forward   w_k = D_k^-1 (v_k - c_lo(k) w_{k-1}),
//   backward  u_{nb-1} = w_{nb-1},  u_k = w_k - c_hi(k) D_k^-1 u_{k+1}.
//
// bt_factor_kernel (set-up, once per tile and wavelength): builds D_k in LDS
// in FP64 and inverts it by Gauss-Jordan elimination with partial pivoting;
// D_k^-1 is stored as complex64, column-major per block ([c][r]).
//
// bt_solve_kernel (hot path): one workgroup per (tile, RHS) streams the
// 2 nb - 1 blocks D_k^-1 from HBM, each once, and keeps the sequential
// recurrence in LDS.  The D blocks do not depend on the data, so each thread
// holds the blocks of the next two steps in registers while it multiplies the
// current one (~80 KB per CU in flight with one workgroup per CU).  The gather of R_i v (input restricted to the
// extended tile, which carries the neighbours' Robin traces by the Robin
// identity) and the core-only scatter (restricted additive Schwarz
// prolongation) are fused into the same kernel.
#include "common.h"

namespace nosdd {

// ------------------------------------------------------------------ geometry
struct BlockMap {
    int x0, y0, lx, tr;
    __device__ __forceinline__ int cx(int k, int m) const { return tr ? x0 + k : x0 + m; }
    __device__ __forceinline__ int cy(int k, int m) const { return tr ? y0 + m : y0 + k; }
    __device__ __forceinline__ int lidx(int k, int m) const {
        return tr ? m * lx + k : k * lx + m;
    }
};

// ------------------------------------------------------------------ factor
constexpr int BT_FACT_THREADS = 256;

template <int BMAX>
__global__ __launch_bounds__(BT_FACT_THREADS) void bt_factor_kernel(const TileDesc *__restrict__ tiles,
                                                                    const float *__restrict__ eps,
                                                                    const double2 *__restrict__ coef,
                                                                    const double *__restrict__ k0v, double h,
                                                                    int nx, int ny, float2 *__restrict__ dinv,
                                                                    long long wl_stride) {
    __shared__ double2 M[BMAX * BMAX];
    __shared__ double2 fcol[BMAX], prow[BMAX];
    __shared__ int piv[BMAX];
    __shared__ int pivrow;
    const TileDesc t = tiles[blockIdx.x];
    const int wl = blockIdx.y;
    const int b = t.b, nb = t.nb, tid = threadIdx.x;
    const double2 *cd = coef + wl * coef_stride(nx, ny);
    const double2 *cxm = cd, *cxp = cd + nx, *cym = cd + 2 * nx, *cyp = cd + 2 * nx + ny;
    const double k0 = k0v[wl];
    float2 *outw = dinv + wl * wl_stride + t.dinv_off;
    const BlockMap bm{t.x0, t.y0, t.x1 - t.x0, t.tr};

    for (int k = 0; k < nb; ++k) {
        double2 alpha = make_double2(0.0, 0.0);
        if (k > 0) {
            double2 clo = t.tr ? cxm[t.x0 + k] : cym[t.y0 + k];
            double2 chi = t.tr ? cxp[t.x0 + k - 1] : cyp[t.y0 + k - 1];
            alpha = zmul(clo, chi);
        }
        // D_k = A_kk - alpha * D_{k-1}^-1 (the inverse is in M, row-major)
        for (int e = tid; e < b * b; e += BT_FACT_THREADS) {
            const int r = e / b, c = e - r * b;
            double2 v = make_double2(0.0, 0.0);
            if (k > 0) {
                double2 prev = M[e];
                v = make_double2(-(alpha.x * prev.x - alpha.y * prev.y), -(alpha.x * prev.y + alpha.y * prev.x));
            }
            const int x = bm.cx(k, r), y = bm.cy(k, r);
            if (c == r) {
                double2 d;
                d.x = -(cxm[x].x + cxp[x].x + cym[y].x + cyp[y].x) - k0 * k0 * (double)eps[(long long)y * nx + x];
                d.y = -(cxm[x].y + cxp[x].y + cym[y].y + cyp[y].y);
                // Robin closure on interface sides: ghost u_q = rho u_p + tau g
                const double kap = k0 * sqrt((double)eps[(long long)y * nx + x]);
                const double2 rho = zdiv(make_double2(1.0, -0.5 * kap * h), make_double2(1.0, 0.5 * kap * h));
                if ((t.iface & SIDE_LEFT) && x == t.x0) d = zadd(d, zmul(cxm[x], rho));
                if ((t.iface & SIDE_RIGHT) && x == t.x1 - 1) d = zadd(d, zmul(cxp[x], rho));
                if ((t.iface & SIDE_BOTTOM) && y == t.y0) d = zadd(d, zmul(cym[y], rho));
                if ((t.iface & SIDE_TOP) && y == t.y1 - 1) d = zadd(d, zmul(cyp[y], rho));
                v = zadd(v, d);
            } else if (c == r + 1) {
                v = zadd(v, t.tr ? cyp[y] : cxp[x]);
            } else if (c == r - 1) {
                v = zadd(v, t.tr ? cym[y] : cxm[x]);
            }
            M[e] = v;
        }
        __syncthreads();
        // Gauss-Jordan inversion in place, partial pivoting
        for (int col = 0; col < b; ++col) {
            if (tid < 64) {
                double best = -1.0;
                int bi = col;
                for (int i = col + tid; i < b; i += 64) {
                    double a = zabs2(M[i * b + col]);
                    if (a > best) { best = a; bi = i; }
                }
                for (int off = 32; off > 0; off >>= 1) {
                    double ob = __shfl_down(best, off, 64);
                    int oi = __shfl_down(bi, off, 64);
                    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
                }
                if (tid == 0) { pivrow = bi; piv[col] = bi; }
            }
            __syncthreads();
            const int p = pivrow;
            if (p != col) {
                for (int j = tid; j < b; j += BT_FACT_THREADS) {
                    double2 a = M[p * b + j];
                    M[p * b + j] = M[col * b + j];
                    M[col * b + j] = a;
                }
                __syncthreads();
            }
            const double2 inv = zdiv(make_double2(1.0, 0.0), M[col * b + col]);
            for (int i = tid; i < b; i += BT_FACT_THREADS) {
                fcol[i] = M[i * b + col];
                prow[i] = zmul(M[col * b + i], inv);
            }
            __syncthreads();
            for (int e = tid; e < b * b; e += BT_FACT_THREADS) {
                const int i = e / b, j = e - i * b;
                double2 v;
                if (i == col) {
                    v = (j == col) ? inv : prow[j];
                } else if (j == col) {
                    double2 f = zmul(fcol[i], inv);
                    v = make_double2(-f.x, -f.y);
                } else {
                    v = zfms(M[e], fcol[i], prow[j]);
                }
                M[e] = v;
            }
            __syncthreads();
        }
        for (int col = b - 1; col >= 0; --col) {
            const int p = piv[col];
            if (p != col) {
                for (int i = tid; i < b; i += BT_FACT_THREADS) {
                    double2 a = M[i * b + p];
                    M[i * b + p] = M[i * b + col];
                    M[i * b + col] = a;
                }
                __syncthreads();
            }
        }
        // store D_k^-1 column-major: element (r, c) at c*b + r
        float2 *dk = outw + (long long)k * b * b;
        for (int e = tid; e < b * b; e += BT_FACT_THREADS) {
            const int c = e / b, r = e - c * b;
            const double2 v = M[r * b + c];
            dk[e] = make_float2((float)v.x, (float)v.y);
        }
        __syncthreads();
    }
}

void launch_bt_factor(hipStream_t s, const TileDesc *tiles, int n_tiles, int n_wl, const float *eps,
                      const float2 *coef_f, const double *coef_d, const double *k0, double h, int nx, int ny,
                      float2 *dinv, long long dinv_wl_stride, int bmax) {
    (void)coef_f;
    dim3 grid(n_tiles, n_wl);
    // the caller guarantees bmax <= 72 (FP64 block of 72 x 72 = 81 KB of LDS)
    (void)bmax;
    hipLaunchKernelGGL(bt_factor_kernel<72>, grid, dim3(BT_FACT_THREADS), 0, s, tiles, eps,
                       (const double2 *)coef_d, k0, h, nx, ny, dinv, dinv_wl_stride);
}

// ------------------------------------------------------------------ solve
// Thread layout per (subdomain, RHS) workgroup: lane group rp (8 lanes) owns
// rows 2rp, 2rp+1 of every block; lane cg of the group covers the columns
// c = cg + 8 j.  Each lane loads one float4 (the two rows' entries of one
// column) per column, the 8 lanes' partial sums are combined with three xor
// shuffles inside the wave, and lane 0 of the group runs the recurrence for
// its two rows.  One barrier per block step.
constexpr int BT_BMAX = 128;
constexpr int BT_GROUP = 8;

template <int MAXJ>
__device__ __forceinline__ void bt_load(float4 (&slot)[MAXJ], const float2 *__restrict__ Dk, int b, int half, int rp,
                                        int cg, bool on) {
    const float4 *D4 = reinterpret_cast<const float4 *>(Dk);
#pragma unroll
    for (int j = 0; j < MAXJ; ++j) {
        const int c = cg + BT_GROUP * j;
        slot[j] = (on && c < b) ? D4[c * half + rp] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
}

template <int MAXJ>
__global__ __launch_bounds__(512) void bt_solve_kernel(const TileDesc *__restrict__ tiles, int n_src, const float2 *__restrict__ dinv,
                                long long dinv_wl_stride, const float2 *__restrict__ coef, int nx, int ny,
                                const float2 *__restrict__ vin, long long vin_stride, float2 *__restrict__ out,
                                long long out_stride, float2 *__restrict__ hist, long long hist_stride,
                                const int *__restrict__ active, int mode) {
    __shared__ float2 ysh[BT_BMAX];
    const int tile = blockIdx.x, rhs = blockIdx.y;
    if (active && !active[rhs]) return;
    const int wl = rhs / n_src;
    const TileDesc t = tiles[tile];
    const int b = t.b, nb = t.nb, half = b >> 1;
    const int tid = threadIdx.x;
    const int rp = tid / BT_GROUP, cg = tid - rp * BT_GROUP;
    const bool on = rp < half;
    const bool lead = on && cg == 0;
    const float2 *D = dinv + wl * dinv_wl_stride + t.dinv_off;
    const long long bb = (long long)b * b;
    const BlockMap bm{t.x0, t.y0, t.x1 - t.x0, t.tr};
    const float2 *cf = coef + wl * coef_stride(nx, ny);
    const float2 *clo_a = t.tr ? cf : cf + 2 * nx;               // cxm or cym
    const float2 *chi_a = t.tr ? cf + nx : cf + 2 * nx + ny;      // cxp or cyp
    const int base = t.tr ? t.x0 : t.y0;
    const bool local_in = mode & 1, local_out = mode & 2;
    const float2 *vr = vin + rhs * vin_stride + (local_in ? t.loc_off : 0);
    float2 *orr = out + rhs * out_stride + (local_out ? t.loc_off : 0);
    float4 *hr = reinterpret_cast<float4 *>(hist + rhs * hist_stride + t.loc_off);
    const int r0 = 2 * rp;

    auto vload = [&](int k, int r) -> float2 {
        const int idx = local_in ? bm.lidx(k, r) : bm.cy(k, r) * nx + bm.cx(k, r);
        return vr[idx];
    };
    auto emit = [&](int k, int r, float2 u) {
        const int x = bm.cx(k, r), y = bm.cy(k, r);
        if (local_out) {
            orr[bm.lidx(k, r)] = u;
        } else if (x >= t.cx0 && x < t.cx1 && y >= t.cy0 && y < t.cy1) {
            orr[(long long)y * nx + x] = u;
        }
    };
    const int nsteps = 2 * nb - 1;
    auto blk = [&](int s) { return s < nb ? s : 2 * nb - 2 - s; };

    if (lead) {
        ysh[r0] = vload(0, r0);
        ysh[r0 + 1] = vload(0, r0 + 1);
    }
    __syncthreads();

    float4 pa[MAXJ], pb[MAXJ], pc[MAXJ];
    bt_load<MAXJ>(pa, D + blk(0) * bb, b, half, rp, cg, on);
    if (nsteps > 1) bt_load<MAXJ>(pb, D + blk(1) * bb, b, half, rp, cg, on);

    auto step = [&](int s, const float4(&slot)[MAXJ]) {
        const int k = blk(s);
        const bool fwd = s < nb;
        float4 pre = make_float4(0.f, 0.f, 0.f, 0.f);
        if (lead) {
            if (fwd) {
                if (k + 1 < nb) {
                    const float2 a = vload(k + 1, r0), c = vload(k + 1, r0 + 1);
                    pre = make_float4(a.x, a.y, c.x, c.y);
                }
            } else {
                pre = hr[(k * b + r0) >> 1];
            }
        }
        float2 a0 = make_float2(0.f, 0.f), a1 = make_float2(0.f, 0.f);
#pragma unroll
        for (int j = 0; j < MAXJ; ++j) {
            const int c = cg + BT_GROUP * j;
            if (c < b) {
                const float2 yc = ysh[c];
                a0 = cfma(a0, make_float2(slot[j].x, slot[j].y), yc);
                a1 = cfma(a1, make_float2(slot[j].z, slot[j].w), yc);
            }
        }
#pragma unroll
        for (int o = 1; o < BT_GROUP; o <<= 1) {
            a0.x += __shfl_xor(a0.x, o, 64);
            a0.y += __shfl_xor(a0.y, o, 64);
            a1.x += __shfl_xor(a1.x, o, 64);
            a1.y += __shfl_xor(a1.y, o, 64);
        }
        __syncthreads();     // every lane has read ysh for this step
        if (lead) {
            if (fwd) {
                hr[(k * b + r0) >> 1] = make_float4(a0.x, a0.y, a1.x, a1.y);     // w_k
                if (k + 1 < nb) {
                    const float2 cl = clo_a[base + k + 1];
                    ysh[r0] = cfms(make_float2(pre.x, pre.y), cl, a0);          // y_{k+1}
                    ysh[r0 + 1] = cfms(make_float2(pre.z, pre.w), cl, a1);
                } else {
                    emit(k, r0, a0);                                            // u_{nb-1} = w_{nb-1}
                    emit(k, r0 + 1, a1);
                    ysh[r0] = a0;
                    ysh[r0 + 1] = a1;
                }
            } else {
                const float2 ch = chi_a[base + k];
                const float2 u0 = cfms(make_float2(pre.x, pre.y), ch, a0);     // u_k
                const float2 u1 = cfms(make_float2(pre.z, pre.w), ch, a1);
                emit(k, r0, u0);
                emit(k, r0 + 1, u1);
                ysh[r0] = u0;
                ysh[r0 + 1] = u1;
            }
        }
        __syncthreads();
    };

    for (int s = 0; s < nsteps; s += 3) {
        if (s + 2 < nsteps) bt_load<MAXJ>(pc, D + blk(s + 2) * bb, b, half, rp, cg, on);
        step(s, pa);
        if (s + 1 < nsteps) {
            if (s + 3 < nsteps) bt_load<MAXJ>(pa, D + blk(s + 3) * bb, b, half, rp, cg, on);
            step(s + 1, pb);
        }
        if (s + 2 < nsteps) {
            if (s + 4 < nsteps) bt_load<MAXJ>(pb, D + blk(s + 4) * bb, b, half, rp, cg, on);
            step(s + 2, pc);
        }
    }
}

void launch_bt_solve(hipStream_t s, const TileDesc *tiles, int n_tiles, int n_rhs, int n_src, const float2 *dinv,
                     long long dinv_wl_stride, const float2 *coef, int nx, int ny, const float2 *vin,
                     long long vin_stride, float2 *out, long long out_stride, float2 *hist, long long hist_stride,
                     const int *active, int mode, int bmax) {
    dim3 grid(n_tiles, n_rhs);
    const int threads = ((bmax / 2) * BT_GROUP + 63) / 64 * 64;
    const int maxj = (bmax + BT_GROUP - 1) / BT_GROUP;
    if (maxj <= 9) {
        hipLaunchKernelGGL(bt_solve_kernel<9>, grid, dim3(threads), 0, s, tiles, n_src, dinv, dinv_wl_stride, coef, nx,
                           ny, vin, vin_stride, out, out_stride, hist, hist_stride, active, mode);
    } else if (maxj <= 13) {
        hipLaunchKernelGGL(bt_solve_kernel<13>, grid, dim3(threads), 0, s, tiles, n_src, dinv, dinv_wl_stride, coef,
                           nx, ny, vin, vin_stride, out, out_stride, hist, hist_stride, active, mode);
    } else {
        hipLaunchKernelGGL(bt_solve_kernel<16>, grid, dim3(threads), 0, s, tiles, n_src, dinv, dinv_wl_stride, coef,
                           nx, ny, vin, vin_stride, out, out_stride, hist, hist_stride, active, mode);
    }
}

}  // namespace nosdd
