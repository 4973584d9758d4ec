// The paper's own outer loop (Algorithm 3): stationary sweeps over the Robin
// data g of every subdomain's interface entries, with momentum, and the
// coarse correction in Robin-data space.
//
//   sweep      u_i = B_i^-1 (R_i b + inj(g_i)),  x = sum_i Rt_i^T u_i,  g_new = traces(x)
//   mismatch   e = g_new - g   (residual of the fixed-point equation (I - T) g = c)
//   coarse     z = ((I-T)Q)^H (I-T)Q)^-1 ((I-T)Q)^H e   (normal equations, FP64)
//   update     g <- m g + (1 - m) g_new + (m Q + (1 - m) T Q) z
//
// Q holds the rotated probe data of each subdomain's coarse columns on its own
// entries, T Q the traces of the corresponding basis fields on the
// neighbours' entries; both are stored sparse, by entry (update) and by column
// (dots).  The local solves reuse the block-Thomas kernel (packed local input,
// core-only scatter) and the traces the Robin-trace kernel.
#include "common.h"

namespace nosdd {

// rhs[r] (packed local) = R_i b[r] + inj(g[r]);  inj(g)_p = injc_e g_e summed
// over the entries e of node p (one per interface side; a corner node has two,
// consecutive in the entry order, and the first one's thread adds both).
__global__ __launch_bounds__(256) void robin_rhs_kernel(const TileDesc *__restrict__ tiles,
                                                        const int4 *__restrict__ ent,
                                                        const float2 *__restrict__ injc, int ne,
                                                        const float2 *__restrict__ b, const float2 *__restrict__ g,
                                                        float2 *__restrict__ rhs, long long N, long long LT, int nx,
                                                        int n_src, const int *__restrict__ active) {
    const int tile = blockIdx.x, r = blockIdx.y;
    if (!active[r]) return;
    const int wl = r / n_src;
    const TileDesc t = tiles[tile];
    const int lx = t.x1 - t.x0, ly = t.y1 - t.y0;
    const float2 *br = b + r * N;
    float2 *out = rhs + r * LT + t.loc_off;
    for (int e = threadIdx.x; e < lx * ly; e += blockDim.x) {
        const int yy = e / lx, xx = e - yy * lx;
        out[e] = br[(long long)(t.y0 + yy) * nx + (t.x0 + xx)];
    }
    __syncthreads();
    const float2 *ic = injc + (long long)wl * ne;
    const float2 *gr = g + (long long)r * ne;
    for (int e = threadIdx.x; e < t.n_tr; e += blockDim.x) {
        const int E = t.tr_off + e;
        const int pc = ent[E].x;
        if (e > 0 && ent[E - 1].x == pc) continue;
        float2 v = cmul(ic[E], gr[E]);
        if (e + 1 < t.n_tr && ent[E + 1].x == pc) v = cadd(v, cmul(ic[E + 1], gr[E + 1]));
        const int px = pc % nx, py = pc / nx;
        const int li = (py - t.y0) * lx + (px - t.x0);
        out[li] = cadd(out[li], v);
    }
}

void launch_robin_rhs(hipStream_t s, const TileDesc *tiles, int n_tiles, const int4 *ent, const float2 *injc, int ne,
                      const float2 *b, const float2 *g, float2 *rhs, long long N, long long LT, int nx, int n_rhs,
                      int n_src, const int *active) {
    hipLaunchKernelGGL(robin_rhs_kernel, dim3(n_tiles, n_rhs), dim3(256), 0, s, tiles, ent, injc, ne, b, g, rhs, N, LT,
                       nx, n_src, active);
}

// d[r][c] = sum_k conj(M[k]) (g_new - g)[entry k] over column c's support, FP64, fixed order
constexpr int RC_THREADS = 256;
__global__ __launch_bounds__(RC_THREADS) void rc_dot_kernel(const int *__restrict__ col_ptr,
                                                            const int *__restrict__ col_ent,
                                                            const float2 *__restrict__ col_val, int nnz, int nc,
                                                            int ne, const float2 *__restrict__ g,
                                                            const float2 *__restrict__ gn, double2 *__restrict__ d,
                                                            int n_src, const int *__restrict__ active) {
    __shared__ double2 red[RC_THREADS / 64];
    const int c = blockIdx.x, r = blockIdx.y;
    if (!active[r]) return;
    const int wl = r / n_src;
    const float2 *mv = col_val + (long long)wl * nnz;
    const float2 *gr = g + (long long)r * ne, *gnr = gn + (long long)r * ne;
    double sx = 0.0, sy = 0.0;
    for (int k = col_ptr[c] + threadIdx.x; k < col_ptr[c + 1]; k += RC_THREADS) {
        const int e = col_ent[k];
        const float2 m = mv[k];
        const float2 df = csub(gnr[e], gr[e]);
        sx += (double)m.x * df.x + (double)m.y * df.y;
        sy += (double)m.x * df.y - (double)m.y * df.x;
    }
    for (int off = 32; off > 0; off >>= 1) {
        sx += __shfl_down(sx, off, 64);
        sy += __shfl_down(sy, off, 64);
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = make_double2(sx, sy);
    __syncthreads();
    if (threadIdx.x == 0) {
        double2 s = red[0];
        for (int i = 1; i < RC_THREADS / 64; ++i) s = zadd(s, red[i]);
        d[(long long)r * nc + c] = s;
    }
}

void launch_rc_dot(hipStream_t s, const int *col_ptr, const int *col_ent, const float2 *col_val, int nnz, int nc,
                   int ne, const float2 *g, const float2 *gn, double2 *d, int n_rhs, int n_src, const int *active) {
    hipLaunchKernelGGL(rc_dot_kernel, dim3(nc, n_rhs), dim3(RC_THREADS), 0, s, col_ptr, col_ent, col_val, nnz, nc, ne, g,
                       gn, d, n_src, active);
}

// g <- m g + (1 - m) g_new (+ sum over the entry's columns of (m q + (1 - m) tq) z)
__global__ __launch_bounds__(256) void rc_update_kernel(const int *__restrict__ row_ptr,
                                                        const int *__restrict__ row_col,
                                                        const float2 *__restrict__ row_q,
                                                        const float2 *__restrict__ row_tq, int nnz, int ne, int nc,
                                                        float2 *__restrict__ g, const float2 *__restrict__ gn,
                                                        const float2 *__restrict__ z, float m, int coarse, int n_src,
                                                        const int *__restrict__ active) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
    if (e >= ne || !active[r]) return;
    const long long ge = (long long)r * ne + e;
    float2 v = make_float2(m * g[ge].x + (1.f - m) * gn[ge].x, m * g[ge].y + (1.f - m) * gn[ge].y);
    if (coarse) {
        const int wl = r / n_src;
        const float2 *q = row_q + (long long)wl * nnz, *tq = row_tq + (long long)wl * nnz;
        const float2 *zr = z + (long long)r * nc;
        for (int k = row_ptr[e]; k < row_ptr[e + 1]; ++k) {
            const float2 a = make_float2(m * q[k].x + (1.f - m) * tq[k].x, m * q[k].y + (1.f - m) * tq[k].y);
            v = cfma(v, a, zr[row_col[k]]);
        }
    }
    g[ge] = v;
}

void launch_rc_update(hipStream_t s, const int *row_ptr, const int *row_col, const float2 *row_q,
                      const float2 *row_tq, int nnz, int ne, int nc, float2 *g, const float2 *gn, const float2 *z,
                      float m, int coarse, int n_rhs, int n_src, const int *active) {
    if (ne == 0) return;
    hipLaunchKernelGGL(rc_update_kernel, dim3((ne + 255) / 256, n_rhs), dim3(256), 0, s, row_ptr, row_col, row_q,
                       row_tq, nnz, ne, nc, g, gn, z, m, coarse, n_src, active);
}

// ||v_r||^2 in FP64: per-workgroup partials, then one fixed-order sum per RHS
constexpr int NRM_BLOCKS = 256;
__global__ __launch_bounds__(256) void norm2_partial_kernel(const float2 *__restrict__ v, long long N,
                                                            double *__restrict__ part) {
    __shared__ double red[4];
    const int r = blockIdx.y;
    const float2 *vr = v + r * N;
    double s = 0.0;
    for (long long n = (long long)blockIdx.x * 256 + threadIdx.x; n < N; n += (long long)gridDim.x * 256)
        s += (double)vr[n].x * vr[n].x + (double)vr[n].y * vr[n].y;
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[(long long)r * gridDim.x + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void norm2_final_kernel(const double *__restrict__ part, int nblk, double *__restrict__ out) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int i = 0; i < nblk; ++i) s += part[(long long)blockIdx.x * nblk + i];
    out[blockIdx.x] = s;
}

void launch_norm2(hipStream_t s, const float2 *v, long long N, int n_rhs, double *part, double *out) {
    hipLaunchKernelGGL(norm2_partial_kernel, dim3(NRM_BLOCKS, n_rhs), dim3(256), 0, s, v, N, part);
    hipLaunchKernelGGL(norm2_final_kernel, dim3(n_rhs), dim3(64), 0, s, part, NRM_BLOCKS, out);
}
int norm2_partials() { return NRM_BLOCKS; }

}  // namespace nosdd
