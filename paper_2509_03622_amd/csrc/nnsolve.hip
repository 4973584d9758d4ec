// Per-subdomain flexible GMRES preconditioned by the neural operator
// (Algorithm 1, inference branch), batched over every (subdomain, RHS)
// sample of a Schwarz sweep:
//   x0 = 0, r0 = b_i = R_i v, v_1 = r0 / beta;
//   for k = 1..N: z_k = NN(v_k); w = B_i z_k; Gram-Schmidt (two passes) against
//   v_1..v_k; v_{k+1} = w / h_{k+1,k}; Givens; stop when |gamma_{k+1}| / beta
//   <= th_sub (relative threshold) or k = N;
//   u_i = Z_k y_k, and the core of u_i is written to the global vector.
// The network always sees a unit-norm residual (its input scaling and output
// scaling follow from the rms of a unit vector over the subdomain).
// A sample whose recurrence meets a non-finite value, or whose final residual
// estimate |gamma_k| / beta is not below NN_FALLBACK_RATIO, writes nothing and
// is queued for the exact LU solve of its subdomain (the factors exist for
// every subdomain), which the caller launches right after.
#include <cmath>

#include "common.h"

namespace nosdd {

constexpr int NN_MAXK = 8;

__device__ __forceinline__ double bsum(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    return s;
}

// vloc[s][c] = v[rhs][global cell of c]   (s = rhs * n_tiles + tile), or a
// plain copy when v is already subdomain-local (local != 0).
__global__ void loc_gather_kernel(const TileDesc *__restrict__ tiles, int n_tiles, const float2 *__restrict__ v,
                                  long long N, int nx, long long loc_total, float2 *__restrict__ vloc,
                                  const int *__restrict__ active, int local) {
    const int s = blockIdx.y;
    const int rhs = s / n_tiles, t = s - rhs * n_tiles;
    if (active && !active[rhs]) return;
    const TileDesc T = tiles[t];
    const int lx = T.x1 - T.x0, n = lx * (T.y1 - T.y0);
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const long long dst = rhs * loc_total + T.loc_off + c;
    if (local) {
        vloc[dst] = v[dst];
        return;
    }
    const int y = c / lx, x = c - y * lx;
    vloc[dst] = v[rhs * N + (long long)(T.y0 + y) * nx + (T.x0 + x)];
}

// beta = ||b_i||; v_1 = b_i / beta; network scalings; sample flags.
__global__ __launch_bounds__(256) void loc_start_kernel(const TileDesc *__restrict__ tiles, int n_tiles,
                                                        long long loc_total, float2 *__restrict__ vloc,
                                                        const int *__restrict__ active, float *__restrict__ beta,
                                                        float *__restrict__ vscale, float *__restrict__ oscale,
                                                        int *__restrict__ sact, int *__restrict__ kstep,
                                                        float2 *__restrict__ gam, int maxk, int *__restrict__ fb) {
    __shared__ double red[4];
    const int s = blockIdx.x;
    const int rhs = s / n_tiles, t = s - rhs * n_tiles;
    const TileDesc T = tiles[t];
    const int n = (T.x1 - T.x0) * (T.y1 - T.y0);
    float2 *vs = vloc + rhs * loc_total + T.loc_off;
    const bool on = !active || active[rhs];
    double a = 0.0;
    if (on)
        for (int c = threadIdx.x; c < n; c += 256) a += (double)cabs2(vs[c]);
    const double b2 = bsum(a, red);
    const double b = sqrt(b2);
    const float inv = b > 0 ? (float)(1.0 / b) : 0.f;
    if (on && b > 0)
        for (int c = threadIdx.x; c < n; c += 256) vs[c] = cscale(vs[c], inv);
    if (threadIdx.x == 0) {
        beta[s] = (float)b;
        vscale[s] = sqrtf((float)n);          // unit vector -> rms 1
        oscale[s] = 1.f / sqrtf((float)n);
        sact[s] = (on && b > 0) ? 1 : 0;
        kstep[s] = 0;
        fb[s] = 0;
        for (int i = 0; i <= maxk; ++i) gam[s * (maxk + 1) + i] = make_float2(0.f, 0.f);
        gam[s * (maxk + 1)] = make_float2((float)b, 0.f);
    }
}

// w = B_i z for each active sample (5-point UPML stencil, zero outside the
// subdomain, Robin closure on the interface sides; FP64 arithmetic).
__global__ void loc_stencil_kernel(const TileDesc *__restrict__ tiles, int n_tiles, int n_src, long long loc_total,
                                   const float2 *__restrict__ z, float2 *__restrict__ w, const float *__restrict__ eps,
                                   const double2 *__restrict__ coef, const double *__restrict__ k0v, double h, int nx,
                                   int ny, const int *__restrict__ sact) {
    const int s = blockIdx.y;
    if (!sact[s]) return;
    const int rhs = s / n_tiles, t = s - rhs * n_tiles;
    const TileDesc T = tiles[t];
    const int lx = T.x1 - T.x0, ly = T.y1 - T.y0, n = lx * ly;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int wl = rhs / n_src;
    const double2 *cf = coef + wl * coef_stride(nx, ny);
    const int ly_ = c / lx, lx_ = c - ly_ * lx;
    const int x = T.x0 + lx_, y = T.y0 + ly_;
    const double2 am = cf[x], ap = cf[nx + x], bm = cf[2 * nx + y], bp = cf[2 * nx + ny + y];
    const double k0 = k0v[wl];
    const double e = (double)eps[(long long)y * nx + x];
    double2 d = make_double2(-(am.x + ap.x + bm.x + bp.x) - k0 * k0 * e, -(am.y + ap.y + bm.y + bp.y));
    const double kap = k0 * sqrt(e);
    const double2 rho = zdiv(make_double2(1.0, -0.5 * kap * h), make_double2(1.0, 0.5 * kap * h));
    if ((T.iface & SIDE_LEFT) && lx_ == 0) d = zadd(d, zmul(am, rho));
    if ((T.iface & SIDE_RIGHT) && lx_ == lx - 1) d = zadd(d, zmul(ap, rho));
    if ((T.iface & SIDE_BOTTOM) && ly_ == 0) d = zadd(d, zmul(bm, rho));
    if ((T.iface & SIDE_TOP) && ly_ == ly - 1) d = zadd(d, zmul(bp, rho));
    const float2 *zs = z + rhs * loc_total + T.loc_off;
    auto wide = [](float2 v) { return make_double2(v.x, v.y); };
    double2 acc = zmul(d, wide(zs[c]));
    if (lx_ > 0) acc = zadd(acc, zmul(am, wide(zs[c - 1])));
    if (lx_ < lx - 1) acc = zadd(acc, zmul(ap, wide(zs[c + 1])));
    if (ly_ > 0) acc = zadd(acc, zmul(bm, wide(zs[c - lx])));
    if (ly_ < ly - 1) acc = zadd(acc, zmul(bp, wide(zs[c + lx])));
    w[rhs * loc_total + T.loc_off + c] = make_float2((float)acc.x, (float)acc.y);
}

// One Arnoldi step k for each active sample: two classical Gram-Schmidt
// passes of w against v_0..v_k, v_{k+1} = w / ||w||, Givens on column k.
__global__ __launch_bounds__(256) void loc_arnoldi_kernel(const TileDesc *__restrict__ tiles, int n_tiles,
                                                          long long loc_total, long long vstride, float2 *__restrict__ Vin,
                                                          float2 *__restrict__ w, int k, int maxk, float tol,
                                                          float2 *__restrict__ H, float *__restrict__ cs,
                                                          float2 *__restrict__ sn, float2 *__restrict__ gam,
                                                          const float *__restrict__ beta, int *__restrict__ sact,
                                                          int *__restrict__ kstep, int *__restrict__ fb) {
    __shared__ double red[4];
    __shared__ double2 hs[NN_MAXK + 1];
    const int s = blockIdx.x;
    if (!sact[s]) return;
    const int rhs = s / n_tiles, t = s - rhs * n_tiles;
    const TileDesc T = tiles[t];
    const int n = (T.x1 - T.x0) * (T.y1 - T.y0);
    const long long off = rhs * loc_total + T.loc_off;
    float2 *ws = w + off;
    float2 *Hs = H + (long long)s * (maxk + 1) * maxk;
    if (threadIdx.x <= k) Hs[threadIdx.x * maxk + k] = make_float2(0.f, 0.f);
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i <= k; ++i) {
            const float2 *vi = Vin + i * vstride + off;
            double ax = 0.0, ay = 0.0;
            for (int c = threadIdx.x; c < n; c += 256) {
                const float2 a = vi[c], b = ws[c];
                ax += (double)a.x * b.x + (double)a.y * b.y;
                ay += (double)a.x * b.y - (double)a.y * b.x;
            }
            const double hx = bsum(ax, red);
            const double hy = bsum(ay, red);
            if (threadIdx.x == 0) hs[i] = make_double2(hx, hy);
        }
        __syncthreads();
        for (int c = threadIdx.x; c < n; c += 256) {
            float2 v = ws[c];
            for (int i = 0; i <= k; ++i) {
                const float2 hh = make_float2((float)hs[i].x, (float)hs[i].y);
                v = cfms(v, hh, Vin[i * vstride + off + c]);
            }
            ws[c] = v;
        }
        if (threadIdx.x <= k) {
            float2 &e = Hs[threadIdx.x * maxk + k];
            e = make_float2(e.x + (float)hs[threadIdx.x].x, e.y + (float)hs[threadIdx.x].y);
        }
        __syncthreads();
    }
    double a = 0.0;
    for (int c = threadIdx.x; c < n; c += 256) a += (double)cabs2(ws[c]);
    const double hn = sqrt(bsum(a, red));
    const float inv = hn > 0 ? (float)(1.0 / hn) : 0.f;
    float2 *vn = Vin + (k + 1) * vstride + off;
    for (int c = threadIdx.x; c < n; c += 256) vn[c] = cscale(ws[c], inv);
    if (threadIdx.x != 0) return;
    // Givens on column k
    float *css = cs + s * maxk;
    float2 *sns = sn + s * maxk;
    Hs[(k + 1) * maxk + k] = make_float2((float)hn, 0.f);
    for (int i = 0; i < k; ++i) {
        const float2 hi = Hs[i * maxk + k], hi1 = Hs[(i + 1) * maxk + k];
        const float c = css[i];
        const float2 sv = sns[i];
        Hs[i * maxk + k] = make_float2(c * hi.x + sv.x * hi1.x - sv.y * hi1.y, c * hi.y + sv.x * hi1.y + sv.y * hi1.x);
        Hs[(i + 1) * maxk + k] =
            make_float2(-(sv.x * hi.x + sv.y * hi.y) + c * hi1.x, -(sv.x * hi.y - sv.y * hi.x) + c * hi1.y);
    }
    const float2 av = Hs[k * maxk + k], bv = Hs[(k + 1) * maxk + k];
    const float aa = sqrtf(cabs2(av));
    float c;
    float2 sv;
    if (aa == 0.f) {
        c = 0.f;
        sv = make_float2(1.f, 0.f);
    } else {
        const float rho = sqrtf(cabs2(av) + cabs2(bv));
        c = aa / rho;
        const float2 ph = make_float2(av.x / aa, av.y / aa);
        sv = make_float2((ph.x * bv.x + ph.y * bv.y) / rho, (ph.y * bv.x - ph.x * bv.y) / rho);
    }
    css[k] = c;
    sns[k] = sv;
    Hs[k * maxk + k] = make_float2(c * av.x + sv.x * bv.x - sv.y * bv.y, c * av.y + sv.x * bv.y + sv.y * bv.x);
    Hs[(k + 1) * maxk + k] = make_float2(0.f, 0.f);
    float2 *g = gam + s * (maxk + 1);
    const float2 gj = g[k];
    g[k + 1] = make_float2(-(sv.x * gj.x + sv.y * gj.y), -(sv.x * gj.y - sv.y * gj.x));
    g[k] = make_float2(c * gj.x, c * gj.y);
    kstep[s] = k + 1;
    const float res = sqrtf(cabs2(g[k + 1])) / beta[s];
    if (!(res <= 3.0e38f)) {              // NaN or Inf: stop and hand the sample to the exact solve
        sact[s] = 0;
        fb[s] = 1;
    } else if (res <= tol || hn == 0.0) {
        sact[s] = 0;
    }
}

// u_i = Z y (y = R^-1 gamma over kstep columns); core cells -> global z, or
// every cell -> the subdomain-local z (local != 0).
__global__ __launch_bounds__(256) void loc_finish_kernel(const TileDesc *__restrict__ tiles, int n_tiles,
                                                         long long loc_total, long long vstride,
                                                         const float2 *__restrict__ Zin, int maxk,
                                                         const float2 *__restrict__ H, const float2 *__restrict__ gam,
                                                         const int *__restrict__ kstep, const int *__restrict__ active,
                                                         float2 *__restrict__ zout, long long N, int nx, int local,
                                                         const float *__restrict__ beta, const int *__restrict__ fb,
                                                         int2 *__restrict__ fb_order, unsigned *__restrict__ fb_count) {
    __shared__ float2 y[NN_MAXK];
    __shared__ int failed;
    const int s = blockIdx.x;
    const int rhs = s / n_tiles, t = s - rhs * n_tiles;
    if (active && !active[rhs]) {
        if (threadIdx.x == 0) fb_order[s] = make_int2(-1, -1);
        return;
    }
    const TileDesc T = tiles[t];
    const int lx = T.x1 - T.x0, n = lx * (T.y1 - T.y0);
    const int k = kstep[s];
    if (threadIdx.x == 0) {
        const float2 *Hs = H + (long long)s * (maxk + 1) * maxk;
        const float2 *g = gam + s * (maxk + 1);
        // no reduction of the subdomain residual, or a non-finite value: exact solve instead
        const float fin = k > 0 ? sqrtf(cabs2(g[k])) / beta[s] : 0.f;
        const int bad = fb[s] || !(fin < NN_FALLBACK_RATIO);
        failed = bad;
        fb_order[s] = bad ? make_int2(t, rhs) : make_int2(-1, -1);
        if (bad) atomicAdd(fb_count, 1u);
        for (int i = k - 1; i >= 0; --i) {
            float2 acc = g[i];
            for (int l = i + 1; l < k; ++l) acc = cfms(acc, Hs[i * maxk + l], y[l]);
            const float2 d = Hs[i * maxk + i];
            const float dd = cabs2(d);
            y[i] = dd > 0.f ? make_float2((acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd)
                            : make_float2(0.f, 0.f);
        }
    }
    __syncthreads();
    if (failed) return;
    const long long off = rhs * loc_total + T.loc_off;
    for (int c = threadIdx.x; c < n; c += 256) {
        const int yy = c / lx, xx = c - yy * lx;
        const int gx = T.x0 + xx, gy = T.y0 + yy;
        if (!local && (gx < T.cx0 || gx >= T.cx1 || gy < T.cy0 || gy >= T.cy1)) continue;
        float2 u = make_float2(0.f, 0.f);
        for (int i = 0; i < k; ++i) u = cfma(u, y[i], Zin[i * vstride + off + c]);
        if (local)
            zout[off + c] = u;
        else
            zout[rhs * N + (long long)gy * nx + gx] = u;
    }
}

void nn_precond(hipStream_t st, const NnWork &nw, const TileDesc *tiles, int n_tiles, int n_rhs, int n_src,
                long long loc_total, int max_cells, const float2 *v, float2 *z, const int *active, const float *eps,
                const double2 *coef, const double *k0, double h, int nx, int ny, int local) {
    const long long N = (long long)nx * ny;
    const int S = n_rhs * n_tiles;
    const long long vstride = (long long)n_rhs * loc_total;
    const int cblk = (max_cells + 255) / 256;
    hipLaunchKernelGGL(loc_gather_kernel, dim3(cblk, S), dim3(256), 0, st, tiles, n_tiles, v, N, nx, loc_total, nw.Vin,
                       active, local);
    hipLaunchKernelGGL(loc_start_kernel, dim3(S), dim3(256), 0, st, tiles, n_tiles, loc_total, nw.Vin, active, nw.beta,
                       nw.vscale, nw.oscale, nw.sact, nw.kstep, nw.gam, nw.maxk, nw.fb);
    for (int k = 0; k < nw.steps; ++k) {
        fno_forward(st, *nw.net, nw.smp, nw.sact, S, max_cells, nw.Vin + k * vstride, nw.vscale, nw.oscale, nw.aux,
                    loc_total, nw.act0, nw.act1, nw.spec, nw.X, nw.Y, nw.Zin + k * vstride);
        hipLaunchKernelGGL(loc_stencil_kernel, dim3(cblk, S), dim3(256), 0, st, tiles, n_tiles, n_src, loc_total,
                           nw.Zin + k * vstride, nw.w, eps, coef, k0, h, nx, ny, nw.sact);
        hipLaunchKernelGGL(loc_arnoldi_kernel, dim3(S), dim3(256), 0, st, tiles, n_tiles, loc_total, vstride, nw.Vin,
                           nw.w, k, nw.maxk, nw.tol, nw.H, nw.cs, nw.sn, nw.gam, nw.beta, nw.sact, nw.kstep, nw.fb);
    }
    hipLaunchKernelGGL(loc_finish_kernel, dim3(S), dim3(256), 0, st, tiles, n_tiles, loc_total, vstride, nw.Zin,
                       nw.maxk, nw.H, nw.gam, nw.kstep, active, z, N, nx, local, nw.beta, nw.fb, nw.fb_order,
                       nw.fb_count);
}

// vscale = 1/rms(v_s), oscale = rms(v_s) per sample (rms over the subdomain's cells)
__global__ __launch_bounds__(256) void nn_rms_kernel(const FnoSample *__restrict__ smp, const float2 *__restrict__ v,
                                                     float *__restrict__ vscale, float *__restrict__ oscale) {
    __shared__ double red[4];
    const int s = blockIdx.x;
    const FnoSample S = smp[s];
    const int n = S.lx * S.ly;
    double a = 0.0;
    for (int c = threadIdx.x; c < n; c += 256) a += (double)cabs2(v[S.cell_off + c]);
    const double ms = bsum(a, red) / n;
    if (threadIdx.x == 0) {
        const double r = sqrt(ms);
        vscale[s] = r > 0 ? (float)(1.0 / r) : 0.f;
        oscale[s] = (float)r;
    }
}

void nn_rms_scales(hipStream_t st, const FnoSample *smp, int S, const float2 *v, float *vscale, float *oscale) {
    hipLaunchKernelGGL(nn_rms_kernel, dim3(S), dim3(256), 0, st, smp, v, vscale, oscale);
}

}  // namespace nosdd
