// Coarse-space correction of the two-level preconditioner (volume form of the
// paper's coarse normal equations, Methods two-level subsection):
//   t = v - A z1,  d = W^H t,  c = G^-1 d,  z = z1 + Phi c,  A z = A z1 + W c,
// with Phi the basis fields (each supported on one subdomain core), W = A Phi
// (supported on the core grown by one cell, the "box") and G = W^H W.
// d and c are accumulated / solved in FP64 (G^-1 is applied as a dense FP64
// product: G is small, n_sub * k_coarse, and its explicit inverse is formed at
// set-up from a Cholesky factorisation in FP64).
#include "common.h"

namespace nosdd {

// d[r][col] = sum_box conj(W[wl][col]) (v - w1), one workgroup per (col, rhs), FP64 sums
// (a box of about 66 x 66 cells: 1024 threads keep the per-thread loop short).
constexpr int CD_THREADS = 1024;
__global__ __launch_bounds__(CD_THREADS) void coarse_dot_kernel(const TileDesc *__restrict__ tiles, int kc,
                                                         const float2 *__restrict__ Wbox, long long wl_stride,
                                                         const float2 *__restrict__ v, const float2 *__restrict__ w1,
                                                         int nx, long long N, int n_src, int n_c,
                                                         const int *__restrict__ active, double2 *__restrict__ d) {
    __shared__ double2 red[CD_THREADS / 64];
    const int col = blockIdx.x, r = blockIdx.y;
    if (active && !active[r]) return;
    const int wl = r / n_src;
    const TileDesc t = tiles[col / kc];
    const int l = col - (col / kc) * kc;
    const float2 *Wc = Wbox + wl * wl_stride + t.box_off + (long long)l * t.bw * t.bh;
    const float2 *vr = v + r * N, *wr = w1 + r * N;
    double sx = 0.0, sy = 0.0;
    const int nbox = t.bw * t.bh;
    for (int e = threadIdx.x; e < nbox; e += CD_THREADS) {
        const int by = e / t.bw, bx = e - by * t.bw;
        const long long g = (long long)(t.by0 + by) * nx + (t.bx0 + bx);
        const float2 tv = csub(vr[g], wr[g]);
        const float2 wv = Wc[e];
        sx += (double)wv.x * tv.x + (double)wv.y * tv.y;
        sy += (double)wv.x * tv.y - (double)wv.y * tv.x;
    }
    for (int off = 32; off > 0; off >>= 1) {
        sx += __shfl_down(sx, off, 64);
        sy += __shfl_down(sy, off, 64);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_double2(sx, sy);
    __syncthreads();
    if (threadIdx.x == 0) {
        double2 s = red[0];
        for (int i = 1; i < CD_THREADS / 64; ++i) s = zadd(s, red[i]);
        d[(long long)r * n_c + col] = s;
    }
}

void launch_coarse_dot(hipStream_t s, const TileDesc *tiles, int n_c, int kc, const float2 *Wbox,
                       long long box_wl_stride, const float2 *v, const float2 *w1, int nx, long long N, int n_rhs,
                       int n_src, const int *active, double2 *d) {
    hipLaunchKernelGGL(coarse_dot_kernel, dim3(n_c, n_rhs), dim3(CD_THREADS), 0, s, tiles, kc, Wbox, box_wl_stride, v, w1,
                       nx, N, n_src, n_c, active, d);
}

// c[r] = G^-1 d[r] in FP64; G^-1 stored transposed (GinvT[wl][j][i] = Ginv[i][j])
// so that consecutive outputs read contiguous entries.  A workgroup owns 64
// outputs; its four waves take interleaved quarters of the sum over j, with
// several independent loads in flight per lane, and are combined in LDS in a
// fixed order.
constexpr int CS_OUT = 64, CS_SLICES = 4;
__global__ __launch_bounds__(CS_OUT *CS_SLICES) void coarse_solve_kernel(const double2 *__restrict__ GinvT, int n_c,
                                                                         const double2 *__restrict__ d,
                                                                         float2 *__restrict__ c, int n_src,
                                                                         const int *__restrict__ active) {
    __shared__ double2 part[CS_SLICES][CS_OUT];
    const int r = blockIdx.y;
    if (active && !active[r]) return;
    const int wl = r / n_src;
    const double2 *dr = d + (long long)r * n_c;
    const int lane = threadIdx.x % CS_OUT, sl = threadIdx.x / CS_OUT;
    const int i = blockIdx.x * CS_OUT + lane;
    const int ic = i < n_c ? i : n_c - 1;
    const double2 *G = GinvT + (long long)wl * n_c * n_c + ic;
    double ax[2] = {0.0, 0.0}, ay[2] = {0.0, 0.0};
    int j = sl;
#pragma unroll 4
    for (; j < n_c; j += CS_SLICES) {
        const double2 g = G[(long long)j * n_c];
        const double2 dv = dr[j];
        const int u = (j / CS_SLICES) & 1;
        ax[u] += g.x * dv.x - g.y * dv.y;
        ay[u] += g.x * dv.y + g.y * dv.x;
    }
    part[sl][lane] = make_double2(ax[0] + ax[1], ay[0] + ay[1]);
    __syncthreads();
    if (sl == 0 && i < n_c) {
        double2 s = part[0][lane];
        for (int q = 1; q < CS_SLICES; ++q) s = make_double2(s.x + part[q][lane].x, s.y + part[q][lane].y);
        c[(long long)r * n_c + i] = make_float2((float)s.x, (float)s.y);
    }
}

void launch_coarse_solve(hipStream_t s, const double2 *GinvT, int n_c, const double2 *d, float2 *c, int n_rhs,
                         int n_src, const int *active) {
    hipLaunchKernelGGL(coarse_solve_kernel, dim3((n_c + CS_OUT - 1) / CS_OUT, n_rhs), dim3(CS_OUT * CS_SLICES), 0, s,
                       GinvT, n_c, d, c, n_src, active);
}

__device__ __forceinline__ float2 box_sum(const TileDesc &t, const float2 *base, int kc, const float2 *cc, int x,
                                          int y) {
    const int e = (y - t.by0) * t.bw + (x - t.bx0);
    const long long colstride = (long long)t.bw * t.bh;
    float2 s = make_float2(0.f, 0.f);
    for (int l = 0; l < kc; ++l) s = cfma(s, cc[l], base[t.box_off + l * colstride + e]);
    return s;
}

// z += Phi c (owner core), w += W c (owner box and the boxes of the cores
// across each side of the cell: W = A Phi vanishes on a box's corner cells,
// so only the owners of the four side neighbours can contribute, and they
// are distinct from each other and from the cell's own core).  owner[y][x]
// is the index of the core holding (x, y), for any arrangement of cores.
__global__ __launch_bounds__(256) void coarse_update_kernel(const TileDesc *__restrict__ tiles,
                                                            const int *__restrict__ owner, int kc,
                                                            const float2 *__restrict__ Phibox,
                                                            const float2 *__restrict__ Wbox, long long wl_stride,
                                                            const float2 *__restrict__ c, int n_c, float2 *__restrict__ z,
                                                            float2 *__restrict__ w, int nx, int ny, int n_src,
                                                            const int *__restrict__ active) {
    const int r = blockIdx.z;
    if (active && !active[r]) return;
    const int wl = r / n_src;
    const int x = blockIdx.x * 64 + threadIdx.x;
    const int y = blockIdx.y * 4 + threadIdx.y;
    if (x >= nx || y >= ny) return;
    const long long cell = (long long)y * nx + x;
    const int own = owner[cell];
    const TileDesc t = tiles[own];
    const float2 *cr = c + (long long)r * n_c;
    const float2 *Pb = Phibox + wl * wl_stride;
    const float2 *Wb = Wbox + wl * wl_stride;
    const long long g = (long long)r * nx * ny + cell;
    if (z) z[g] = cadd(z[g], box_sum(t, Pb, kc, cr + own * kc, x, y));     // null: Phi c deferred to the cycle end
    float2 acc = box_sum(t, Wb, kc, cr + own * kc, x, y);
    if (x == t.cx0 && x > 0) {
        const int nb = owner[cell - 1];
        acc = cadd(acc, box_sum(tiles[nb], Wb, kc, cr + nb * kc, x, y));
    }
    if (x == t.cx1 - 1 && x + 1 < nx) {
        const int nb = owner[cell + 1];
        acc = cadd(acc, box_sum(tiles[nb], Wb, kc, cr + nb * kc, x, y));
    }
    if (y == t.cy0 && y > 0) {
        const int nb = owner[cell - nx];
        acc = cadd(acc, box_sum(tiles[nb], Wb, kc, cr + nb * kc, x, y));
    }
    if (y == t.cy1 - 1 && y + 1 < ny) {
        const int nb = owner[cell + nx];
        acc = cadd(acc, box_sum(tiles[nb], Wb, kc, cr + nb * kc, x, y));
    }
    w[g] = cadd(w[g], acc);
}

void launch_coarse_update(hipStream_t s, const TileDesc *tiles, const int *owner, int kc, const float2 *Phibox,
                          const float2 *Wbox, long long box_wl_stride, const float2 *c, int n_c, float2 *z, float2 *w,
                          int nx, int ny, int n_rhs, int n_src, const int *active) {
    dim3 grid((nx + 63) / 64, (ny + 3) / 4, n_rhs);
    hipLaunchKernelGGL(coarse_update_kernel, grid, dim3(64, 4), 0, s, tiles, owner, kc, Phibox, Wbox, box_wl_stride,
                       c, n_c, z, w, nx, ny, n_src, active);
}

// Deferred coarse part of the preconditioned directions: within a restart
// cycle z_j = z1_j + Phi c_j keeps only z1_j and stores c_j, and the cycle's
// update x += sum_j y_j z_j takes the coarse part as x += Phi (sum_j y_j c_j).
// cy[r][col] = sum_{j < kcyc[r]} y[r][j] c_j[r][col] (FP64), then x += Phi cy
// on every core.
__global__ __launch_bounds__(256) void coarse_cy_kernel(const float2 *__restrict__ C, long long cstride,
                                                        const float2 *__restrict__ y, int m,
                                                        const int *__restrict__ kcyc, int n_c,
                                                        double2 *__restrict__ cy) {
    const int r = blockIdx.y, col = blockIdx.x * 256 + threadIdx.x;
    if (col >= n_c) return;
    const int k = kcyc[r];
    double sx = 0.0, sy = 0.0;
    for (int j = 0; j < k; ++j) {
        const float2 a = y[r * m + j], c = C[j * cstride + (long long)r * n_c + col];
        sx += (double)a.x * c.x - (double)a.y * c.y;
        sy += (double)a.x * c.y + (double)a.y * c.x;
    }
    cy[(long long)r * n_c + col] = make_double2(sx, sy);
}

__global__ __launch_bounds__(256) void coarse_x_kernel(double2 *__restrict__ x, const TileDesc *__restrict__ tiles,
                                                       const int *__restrict__ owner, int kc,
                                                       const float2 *__restrict__ Phibox, long long wl_stride,
                                                       const double2 *__restrict__ cy, int n_c, int nx, int ny,
                                                       int n_src, const int *__restrict__ kcyc) {
    const int r = blockIdx.z;
    if (kcyc[r] == 0) return;
    const int xx = blockIdx.x * 64 + threadIdx.x, yy = blockIdx.y * 4 + threadIdx.y;
    if (xx >= nx || yy >= ny) return;
    const long long cell = (long long)yy * nx + xx;
    const int own = owner[cell];
    const TileDesc t = tiles[own];
    const float2 *Pb = Phibox + (r / n_src) * wl_stride + t.box_off;
    const int e = (yy - t.by0) * t.bw + (xx - t.bx0);
    const long long colstride = (long long)t.bw * t.bh;
    const double2 *c = cy + (long long)r * n_c + (long long)own * kc;
    double sx = 0.0, sy = 0.0;
    for (int l = 0; l < kc; ++l) {
        const float2 ph = Pb[l * colstride + e];
        sx += (double)ph.x * c[l].x - (double)ph.y * c[l].y;
        sy += (double)ph.x * c[l].y + (double)ph.y * c[l].x;
    }
    double2 &xv = x[(long long)r * nx * ny + cell];
    xv = make_double2(xv.x + sx, xv.y + sy);
}

void launch_coarse_cycle_end(hipStream_t s, double2 *x, const TileDesc *tiles, const int *owner, int kc,
                             const float2 *Phibox, long long box_wl_stride, const float2 *C, const float2 *y, int m,
                             const int *kcyc, int n_c, double2 *cy, int nx, int ny, int n_rhs, int n_src) {
    hipLaunchKernelGGL(coarse_cy_kernel, dim3((n_c + 255) / 256, n_rhs), dim3(256), 0, s, C, (long long)n_rhs * n_c, y,
                       m, kcyc, n_c, cy);
    hipLaunchKernelGGL(coarse_x_kernel, dim3((nx + 63) / 64, (ny + 3) / 4, n_rhs), dim3(64, 4), 0, s, x, tiles, owner,
                       kc, Phibox, box_wl_stride, cy, n_c, nx, ny, n_src, kcyc);
}

}  // namespace nosdd
