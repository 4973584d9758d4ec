// Flexible GMRES building blocks (Algorithm 1 recurrence, batched over RHS).
//
// Orthogonalisation is classical Gram-Schmidt with one selective second pass
// (Daniel-Gragg-Kaufman-Stewart test ||w'|| < 0.7 ||w||): with j basis vectors
// a pass reads j+1 vectors for the dots and j+1 for the update and writes one,
// so the Arnoldi traffic per step is about 8 (2 j + 5) bytes per cell.
// Reductions are two-stage and fixed-order (no atomics): per-workgroup
// partials in FP64, then one workgroup per RHS sums them, so results are
// bit-reproducible run to run.
//
// Givens rotations (complex, FP32) follow
//   rho = sqrt(|a|^2 + |b|^2), c = |a|/rho, s = (a/|a|) conj(b)/rho  (c=0, s=1 if a=0),
//   gamma_{j+1} = -conj(s) gamma_j,  gamma_j <- c gamma_j.
#include "common.h"

namespace nosdd {

constexpr int KR_THREADS = 256;
constexpr int KR_MAXV = 32;       // basis vectors handled per pass (restart <= 31)
constexpr int KR_SLOTS = KR_MAXV + 1;

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// Block-level sum of NV complex values held per thread (slots i < nv and the
// last slot); result valid in thread 0.  red holds (KR_THREADS/64) * NV double2.
template <int NV>
__device__ __forceinline__ void block_sum(double2 (&acc)[NV], int nv, double2 *red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if (i < nv || i == NV - 1) {
            double rx = wave_sum(acc[i].x), ry = wave_sum(acc[i].y);
            if (lane == 0) red[wid * NV + i] = make_double2(rx, ry);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            if (i < nv || i == NV - 1) {
                double2 s = red[i];
                for (int w = 1; w < KR_THREADS / 64; ++w) s = zadd(s, red[w * NV + i]);
                acc[i] = s;
            }
        }
    }
}

// partial[r][blk][i] = sum conj(V_i) w over this block's cells (i < nv);
// partial[r][blk][KR_MAXV].x = sum |w|^2.  Each thread accumulates its few
// cells in FP32, the workgroup sum is formed in FP64.
__global__ __launch_bounds__(KR_THREADS) void dots_kernel(const float2 *__restrict__ V, long long vstride, int nv,
                                                           const float2 *__restrict__ w, long long N,
                                                           const int *__restrict__ active,
                                                           double2 *__restrict__ partial, int nblk) {
    __shared__ double2 red[(KR_THREADS / 64) * KR_SLOTS];
    const int r = blockIdx.y;
    if (active && !active[r]) return;
    const float2 *wr = w + r * N;
    const float2 *Vr = V + r * N;
    float2 facc[KR_MAXV];
    float fn = 0.f;
#pragma unroll
    for (int i = 0; i < KR_MAXV; ++i) facc[i] = make_float2(0.f, 0.f);
    const long long stride = (long long)gridDim.x * KR_THREADS;
    for (long long n = (long long)blockIdx.x * KR_THREADS + threadIdx.x; n < N; n += stride) {
        const float2 wv = wr[n];
        fn += cabs2(wv);
#pragma unroll
        for (int i = 0; i < KR_MAXV; ++i)
            if (i < nv) facc[i] = cfma_conj(facc[i], Vr[i * vstride + n], wv);
    }
    // per-wave FP64 sums, then one thread per value sums the waves
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < KR_MAXV; ++i) {
        if (i < nv) {
            const double rx = wave_sum((double)facc[i].x), ry = wave_sum((double)facc[i].y);
            if (lane == 0) red[wid * KR_SLOTS + i] = make_double2(rx, ry);
        }
    }
    {
        const double rn = wave_sum((double)fn);
        if (lane == 0) red[wid * KR_SLOTS + KR_MAXV] = make_double2(rn, 0.0);
    }
    __syncthreads();
    const int i = threadIdx.x;
    if (i < nv || i == KR_MAXV) {
        double2 s = red[i];
        for (int wv = 1; wv < KR_THREADS / 64; ++wv) s = zadd(s, red[wv * KR_SLOTS + i]);
        partial[((long long)r * nblk + blockIdx.x) * KR_SLOTS + i] = s;
    }
}

void launch_dots(hipStream_t s, const float2 *V, long long vstride, int nv, const float2 *w, long long N, int n_rhs,
                 const int *active, double2 *partial, int nblk) {
    hipLaunchKernelGGL(dots_kernel, dim3(nblk, n_rhs), dim3(KR_THREADS), 0, s, V, vstride, nv, w, N, active,
                       partial, nblk);
}

// Sum partials (fixed order).  Writes H[r][i][col] (i < nv) as FP32 (added to
// the existing entries when accumulate), and norm2_out[r] = ||w||^2.
__global__ __launch_bounds__(KR_THREADS) void reduce_dots_kernel(const double2 *__restrict__ partial, int nblk,
                                                                  int nv, const int *__restrict__ active,
                                                                  float2 *__restrict__ H, int m, int col,
                                                                  int accumulate, double *__restrict__ norm2_out) {
    __shared__ double2 red[KR_THREADS];
    const int r = blockIdx.x;
    if (active && !active[r]) return;
    const double2 *pr = partial + (long long)r * nblk * KR_SLOTS;
    for (int i = 0; i <= nv; ++i) {
        const int slot = i < nv ? i : KR_MAXV;
        double2 s = make_double2(0.0, 0.0);
        for (int bk = threadIdx.x; bk < nblk; bk += KR_THREADS) s = zadd(s, pr[(long long)bk * KR_SLOTS + slot]);
        red[threadIdx.x] = s;
        __syncthreads();
        for (int o = KR_THREADS / 2; o > 0; o >>= 1) {
            if (threadIdx.x < o) red[threadIdx.x] = zadd(red[threadIdx.x], red[threadIdx.x + o]);
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            const double2 v = red[0];
            if (i < nv) {
                float2 *h = H + ((long long)r * (m + 1) + i) * m + col;
                if (accumulate) *h = make_float2(h->x + (float)v.x, h->y + (float)v.y);
                else *h = make_float2((float)v.x, (float)v.y);
            } else if (norm2_out) {
                norm2_out[r] = v.x;
            }
        }
        __syncthreads();
    }
}

void launch_reduce_dots(hipStream_t s, const double2 *partial, int nblk, int nv, int n_rhs, const int *active,
                        float2 *H, int ldh, int m, int col, int accumulate, double *norm2_out) {
    (void)ldh;
    hipLaunchKernelGGL(reduce_dots_kernel, dim3(n_rhs), dim3(KR_THREADS), 0, s, partial, nblk, nv, active, H, m, col,
                       accumulate, norm2_out);
}

// dst = w - sum_{i<nv} coef_i V_i with coef_i = H[r][i][col] (or the second-pass
// correction stored in the same layout when gate is given); partial norm of dst.
// When gate is non-null and gate[r] == 0 the RHS is skipped.
__global__ __launch_bounds__(KR_THREADS) void update_kernel(const float2 *__restrict__ V, long long vstride, int nv,
                                                             const float2 *w, float2 *dst, long long N,
                                                             const int *__restrict__ active,
                                                             const float2 *__restrict__ Hc, int m, int col,
                                                             const int *__restrict__ gate,
                                                             double2 *__restrict__ partial, int nblk) {
    __shared__ double2 red[(KR_THREADS / 64) * 1];
    __shared__ float2 hs[KR_MAXV];
    const int r = blockIdx.y;
    if (active && !active[r]) return;
    if (gate && !gate[r]) return;
    if (threadIdx.x < nv) hs[threadIdx.x] = Hc[((long long)r * (m + 1) + threadIdx.x) * m + col];
    __syncthreads();
    float2 hreg[KR_MAXV];
#pragma unroll
    for (int i = 0; i < KR_MAXV; ++i) hreg[i] = i < nv ? hs[i] : make_float2(0.f, 0.f);
    const float2 *wr = w + r * N;
    float2 *dr = dst + r * N;
    const float2 *Vr = V + r * N;
    double nrm = 0.0;
    float fn = 0.f;
    int cnt = 0;
    const long long stride = (long long)gridDim.x * KR_THREADS;
    for (long long n = (long long)blockIdx.x * KR_THREADS + threadIdx.x; n < N; n += stride) {
        float2 v = wr[n];
#pragma unroll
        for (int i = 0; i < KR_MAXV; ++i)
            if (i < nv) v = cfms(v, hreg[i], Vr[i * vstride + n]);
        dr[n] = v;
        fn += cabs2(v);
        if (++cnt == 16) { nrm += fn; fn = 0.f; cnt = 0; }
    }
    nrm += fn;
    double2 acc[1] = {make_double2(nrm, 0.0)};
    block_sum<1>(acc, 0, red);
    if (threadIdx.x == 0) partial[((long long)r * nblk + blockIdx.x) * KR_SLOTS + KR_MAXV] = acc[0];
}

void launch_update(hipStream_t s, const float2 *V, long long vstride, int nv, const float2 *w, float2 *dst, long long N,
                   int n_rhs, const int *active, const float2 *H, int ldh, int m, int col, const int *gate,
                   double2 *partial, int nblk) {
    (void)ldh;
    hipLaunchKernelGGL(update_kernel, dim3(nblk, n_rhs), dim3(KR_THREADS), 0, s, V, vstride, nv, w, dst, N, active,
                       H, m, col, gate, partial, nblk);
}

__global__ __launch_bounds__(KR_THREADS) void reduce_norm_kernel(const double2 *__restrict__ partial, int nblk,
                                                                  const int *__restrict__ active,
                                                                  const int *__restrict__ gate,
                                                                  double *__restrict__ out) {
    __shared__ double red[KR_THREADS];
    const int r = blockIdx.x;
    if (active && !active[r]) return;
    if (gate && !gate[r]) return;
    double s = 0.0;
    for (int bk = threadIdx.x; bk < nblk; bk += KR_THREADS) s += partial[((long long)r * nblk + bk) * KR_SLOTS + KR_MAXV].x;
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = KR_THREADS / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[r] = red[0];
}

void launch_reduce_norm(hipStream_t s, const double2 *partial, int nblk, int n_rhs, const int *active, double *out) {
    hipLaunchKernelGGL(reduce_norm_kernel, dim3(n_rhs), dim3(KR_THREADS), 0, s, partial, nblk, active,
                       (const int *)nullptr, out);
}

void launch_reduce_norm_gated(hipStream_t s, const double2 *partial, int nblk, int n_rhs, const int *active,
                              const int *gate, double *out) {
    hipLaunchKernelGGL(reduce_norm_kernel, dim3(n_rhs), dim3(KR_THREADS), 0, s, partial, nblk, active, gate, out);
}

// DGKS: ask for a second Gram-Schmidt pass when ||w'|| < 0.7 ||w||.
__global__ void dgks_kernel(const double *nw_pre, const double *nw_post, int *reorth, const int *active, int n_rhs) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rhs) return;
    reorth[r] = (active[r] && nw_post[r] < 0.49 * nw_pre[r]) ? 1 : 0;
}

void launch_dgks(hipStream_t s, const double *nw_pre, const double *nw_post, int *reorth, const int *active,
                 int n_rhs) {
    hipLaunchKernelGGL(dgks_kernel, dim3((n_rhs + 63) / 64), dim3(64), 0, s, nw_pre, nw_post, reorth, active, n_rhs);
}

// One Givens step per active RHS (column j of H already holds h_{0..j,j};
// h_{j+1,j} = ||w'|| comes from nw_post, or nw_reorth after a second pass).
__global__ void givens_kernel(GivensArgs a, int j, int n_rhs) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rhs || !a.active[r]) return;
    const int m = a.m;
    float2 *Hr = a.H + (long long)r * (m + 1) * m;
    const double nw = (a.reorth && a.reorth[r]) ? a.nw_reorth[r] : a.nw_post[r];
    const float hn = (float)sqrt(nw);
    Hr[(j + 1) * m + j] = make_float2(hn, 0.f);
    float *cs = a.cs + r * m;
    float2 *sn = a.sn + r * m;
    for (int i = 0; i < j; ++i) {
        const float2 hi = Hr[i * m + j], hi1 = Hr[(i + 1) * m + j];
        const float c = cs[i];
        const float2 s = sn[i];
        // t = c*hi + s*hi1 ; hi1' = -conj(s)*hi + c*hi1
        float2 t = make_float2(c * hi.x + s.x * hi1.x - s.y * hi1.y, c * hi.y + s.x * hi1.y + s.y * hi1.x);
        float2 u = make_float2(-(s.x * hi.x + s.y * hi.y) + c * hi1.x, -(s.x * hi.y - s.y * hi.x) + c * hi1.y);
        Hr[i * m + j] = t;
        Hr[(i + 1) * m + j] = u;
    }
    const float2 av = Hr[j * m + j], bv = Hr[(j + 1) * m + j];
    const float aa = sqrtf(cabs2(av));
    float c;
    float2 s;
    if (aa == 0.f) {
        c = 0.f;
        s = make_float2(1.f, 0.f);
    } else {
        const float rho = sqrtf(cabs2(av) + cabs2(bv));
        c = aa / rho;
        const float2 ph = make_float2(av.x / aa, av.y / aa);
        // s = ph * conj(bv) / rho
        s = make_float2((ph.x * bv.x + ph.y * bv.y) / rho, (ph.y * bv.x - ph.x * bv.y) / rho);
    }
    cs[j] = c;
    sn[j] = s;
    Hr[j * m + j] = make_float2(c * av.x + s.x * bv.x - s.y * bv.y, c * av.y + s.x * bv.y + s.y * bv.x);
    Hr[(j + 1) * m + j] = make_float2(0.f, 0.f);
    float2 *g = a.gam + r * (m + 1);
    const float2 gj = g[j];
    g[j + 1] = make_float2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
    g[j] = make_float2(c * gj.x, c * gj.y);
    const float res = sqrtf(cabs2(g[j + 1])) / a.bnorm[r];
    const int it = a.iters[r];
    if (it < a.hist_ld) a.hist[(long long)r * a.hist_ld + it] = res;
    a.iters[r] = it + 1;
    a.kcyc[r] = j + 1;
    const double nwpre = a.nw_pre[r];
    const bool breakdown = nw <= 1e-12 * nwpre;        // ||w'|| <= 1e-6 ||w|| in FP32
    int fl = 0;
    if (res <= a.tol) fl |= 1;
    if (breakdown) fl |= 2;
    if (it + 1 >= a.max_iters) fl |= 4;
    a.flags[r] = fl;
    a.inv_h[r] = hn > 0.f ? 1.f / hn : 0.f;
    if (fl) a.active[r] = 0;
}

void launch_givens(hipStream_t s, const GivensArgs &a, int j, int n_rhs) {
    hipLaunchKernelGGL(givens_kernel, dim3((n_rhs + 63) / 64), dim3(64), 0, s, a, j, n_rhs);
}

// v *= sc[r]
__global__ void scale_kernel(float2 *v, long long N, const int *active, const float *sc) {
    const int r = blockIdx.y;
    if (active && !active[r]) return;
    const float f = sc[r];
    float2 *vr = v + r * N;
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x)
        vr[n] = cscale(vr[n], f);
}

void launch_scale(hipStream_t s, float2 *v, long long N, int n_rhs, const int *active, const float *sc) {
    const int nb = (int)(((N + 255) / 256) < 1024 ? (N + 255) / 256 : 1024);
    hipLaunchKernelGGL(scale_kernel, dim3(nb, n_rhs), dim3(256), 0, s, v, N, active, sc);
}

// y = R^-1 gamma for the first kcyc[r] columns (R upper triangular in H).
__global__ void backsolve_kernel(const float2 *H, int m, const float2 *gam, const int *kcyc, float2 *y, int n_rhs) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rhs) return;
    const int k = kcyc[r];
    const float2 *Hr = H + (long long)r * (m + 1) * m;
    const float2 *g = gam + r * (m + 1);
    float2 *yr = y + r * m;
    for (int i = k - 1; i >= 0; --i) {
        float2 s = g[i];
        for (int l = i + 1; l < k; ++l) s = cfms(s, Hr[i * m + l], yr[l]);
        const float2 d = Hr[i * m + i];
        const float dd = cabs2(d);
        yr[i] = make_float2((s.x * d.x + s.y * d.y) / dd, (s.y * d.x - s.x * d.y) / dd);
    }
}

void launch_backsolve(hipStream_t s, const float2 *H, int ldh, int m, const float2 *gam, const int *kcyc, float2 *y,
                      int n_rhs) {
    (void)ldh;
    hipLaunchKernelGGL(backsolve_kernel, dim3((n_rhs + 63) / 64), dim3(64), 0, s, H, m, gam, kcyc, y, n_rhs);
}

// x += sum_{i < kcyc[r]} y_i Z_i  (x in FP64; the FP32 products are accumulated in FP64)
__global__ __launch_bounds__(256) void xupdate_kernel(double2 *x, const float2 *Z, long long zstride, const float2 *y,
                                                      int m, const int *kcyc, long long N) {
    __shared__ float2 ys[KR_MAXV];
    const int r = blockIdx.y;
    const int k = kcyc[r];
    if (k == 0) return;
    if (threadIdx.x < k) ys[threadIdx.x] = y[r * m + threadIdx.x];
    __syncthreads();
    double2 *xr = x + r * N;
    const float2 *Zr = Z + r * N;
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
        double2 v = xr[n];
        for (int i = 0; i < k; ++i) {
            const float2 zz = Zr[i * zstride + n];
            const float2 yy = ys[i];
            v.x += (double)yy.x * zz.x - (double)yy.y * zz.y;
            v.y += (double)yy.x * zz.y + (double)yy.y * zz.x;
        }
        xr[n] = v;
    }
}

void launch_xupdate(hipStream_t s, double2 *x, const float2 *Z, long long zstride, const float2 *y, int m,
                    const int *kcyc, long long N, int n_rhs) {
    const int nb = (int)(((N + 255) / 256) < 1024 ? (N + 255) / 256 : 1024);
    hipLaunchKernelGGL(xupdate_kernel, dim3(nb, n_rhs), dim3(256), 0, s, x, Z, zstride, y, m, kcyc, N);
}

// Begin a cycle for RHS with want[r]: V0 = r/beta, gamma = beta e1, kcyc = 0, active = 1.
__global__ void start_cycle_kernel(float2 *V0, const float2 *res, const double *beta2, float2 *gam, int m, int *kcyc,
                                   int *active, const int *want, long long N) {
    const int r = blockIdx.y;
    if (!want[r]) return;
    const double beta = sqrt(beta2[r]);
    const float inv = beta > 0 ? (float)(1.0 / beta) : 0.f;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int i = 0; i <= m; ++i) gam[r * (m + 1) + i] = make_float2(0.f, 0.f);
        gam[r * (m + 1)] = make_float2((float)beta, 0.f);
        kcyc[r] = 0;
        active[r] = 1;
    }
    const float2 *rr = res + r * N;
    float2 *vr = V0 + r * N;
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x)
        vr[n] = cscale(rr[n], inv);
}

void launch_start_cycle(hipStream_t s, float2 *V0, const float2 *r, const double *beta2, const float *bnorm,
                        float2 *gam, int m, int *kcyc, int *active, const int *want, long long N, int n_rhs) {
    (void)bnorm;
    const int nb = (int)(((N + 255) / 256) < 1024 ? (N + 255) / 256 : 1024);
    hipLaunchKernelGGL(start_cycle_kernel, dim3(nb, n_rhs), dim3(256), 0, s, V0, r, beta2, gam, m, kcyc, active, want,
                       N);
}

// H[r][i][col] += H2[r][i][col] for i < nv (second Gram-Schmidt pass), gated.
__global__ void hadd_kernel(float2 *H, const float2 *H2, int m, int col, int nv, const int *gate, int n_rhs) {
    const int r = blockIdx.x;
    const int i = threadIdx.x;
    if (r >= n_rhs || !gate[r] || i >= nv) return;
    const long long o = ((long long)r * (m + 1) + i) * m + col;
    H[o] = cadd(H[o], H2[o]);
}

void launch_hadd(hipStream_t s, float2 *H, const float2 *H2, int m, int col, int nv, const int *gate, int n_rhs) {
    hipLaunchKernelGGL(hadd_kernel, dim3(n_rhs), dim3(64), 0, s, H, H2, m, col, nv, gate, n_rhs);
}

}  // namespace nosdd
