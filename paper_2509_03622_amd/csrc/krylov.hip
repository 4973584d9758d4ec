// Flexible GMRES building blocks (Algorithm 1 recurrence, batched over RHS).
//
// Orthogonalisation is classical Gram-Schmidt applied twice.  Default
// (stored-basis) form: the dots of pass one, then pass one's update fused with
// pass two's dots; the second pass's correction and the normalisation are kept
// in an upper-triangular FP64 map T from the stored vectors to the orthonormal
// basis (dots against the basis are T^H times dots against the stored
// vectors), so no third pass rewrites the new vector and a step moves about
// 8 (2 j + 5) bytes per cell with j basis vectors.  Alternative form: the
// second pass runs where the Daniel-Gragg-Kaufman-Stewart test
// ||w'|| < 0.7 ||w|| asks for it, and a third pass writes the normalised
// vector (about 8 (3 j + 8) bytes per cell).
// Reductions are two-stage and fixed-order (no atomics): per-workgroup
// partials in FP64, then one workgroup per RHS sums them, so results are
// bit-reproducible run to run.
//
// Givens rotations (complex, FP32) follow
//   rho = sqrt(|a|^2 + |b|^2), c = |a|/rho, s = (a/|a|) conj(b)/rho  (c=0, s=1 if a=0),
//   gamma_{j+1} = -conj(s) gamma_j,  gamma_j <- c gamma_j.
#include <algorithm>

#include "common.h"

namespace nosdd {

constexpr int KR_THREADS = 256;
constexpr int KR_MAXV = 32;       // basis vectors handled per pass (restart <= 31)
constexpr int KR_SLOTS = KR_MAXV + 1;

// FP32 butterfly over the 64 lanes (result in every lane); the per-lane
// inputs are sums of a few FP32 products, so FP32 is ample at this level and
// the xor pattern maps onto cross-lane data movement without LDS round trips.
__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

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

// One Givens step for RHS r (column j of H holds h_{0..j,j}; ||w'||^2 = nw).
// The column and the earlier rotations are read through `col`, `csr`, `snr`
// (global memory, or LDS copies made by the calling workgroup), and the
// rotated column is written to H.
template <typename HC, typename CS, typename SN>
__device__ void givens_core(const GivensArgs &a, int r, int j, double nw, HC col, CS csr, SN snr) {
    const int m = a.m;
    float2 *Hr = a.H + (long long)r * (m + 1) * m;
    const float hn = (float)sqrt(nw);
    col(j + 1) = make_float2(hn, 0.f);
    float *cs = a.cs + r * m;
    float2 *sn = a.sn + r * m;
    for (int i = 0; i < j; ++i) {
        const float2 hi = col(i), hi1 = col(i + 1);
        const float c = csr(i);
        const float2 s = snr(i);
        // t = c hi + s hi1 ; hi1' = -conj(s) hi + c hi1
        const float2 t = make_float2(c * hi.x + s.x * hi1.x - s.y * hi1.y, c * hi.y + s.x * hi1.y + s.y * hi1.x);
        const float2 u = make_float2(-(s.x * hi.x + s.y * hi.y) + c * hi1.x, -(s.x * hi.y - s.y * hi.x) + c * hi1.y);
        col(i) = t;
        col(i + 1) = u;
    }
    const float2 av = col(j), bv = col(j + 1);
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
        s = make_float2((ph.x * bv.x + ph.y * bv.y) / rho, (ph.y * bv.x - ph.x * bv.y) / rho);   // ph conj(b) / rho
    }
    cs[j] = c;
    sn[j] = s;
    col(j) = make_float2(c * av.x + s.x * bv.x - s.y * bv.y, c * av.y + s.x * bv.y + s.y * bv.x);
    col(j + 1) = make_float2(0.f, 0.f);
    for (int i = 0; i <= j + 1; ++i) Hr[i * m + j] = col(i);
    float2 *g = a.gam + r * (m + 1);
    const float2 gj = g[j];
    g[j + 1] = make_float2(-(s.x * gj.x + s.y * gj.y), -(s.x * gj.y - s.y * gj.x));
    g[j] = make_float2(c * gj.x, c * gj.y);
    const float res = sqrtf(cabs2(g[j + 1])) / a.bnorm[r];
    const int it = a.iters[r];
    if (it < a.hist_ld) a.hist[(long long)r * a.hist_ld + it] = res;
    a.iters[r] = it + 1;
    a.kcyc[r] = j + 1;
    const bool breakdown = nw <= 1e-12 * a.nw_pre[r];   // ||w'|| <= 1e-6 ||w||
    int fl = 0;
    if (res <= a.tol) fl |= 1;
    if (breakdown) fl |= 2;
    if (it + 1 >= a.max_iters) fl |= 4;
    a.flags[r] = fl;
    a.inv_h[r] = hn > 0.f ? 1.f / hn : 0.f;
    if (fl) a.active[r] = 0;
}

__device__ void givens_step(const GivensArgs &a, int r, int j, double nw) {
    float2 *Hr = a.H + (long long)r * (a.m + 1) * a.m;
    const float *cs = a.cs + r * a.m;
    const float2 *sn = a.sn + r * a.m;
    const int m = a.m;
    givens_core(a, r, j, nw, [&](int i) -> float2 & { return Hr[i * m + j]; }, [&](int i) { return cs[i]; },
                [&](int i) { return sn[i]; });
}

// Gram-Schmidt dots pass: per-workgroup partials of h_i = V_i^H w (i < NV) and
// ||w||^2 (slot KR_MAXV), summed by cgs_reduce_kernel.  Software-pipelined:
// the NV + 1 loads of a thread's next cell are issued before the products of
// the current one, so every wave keeps a cell's worth of loads in flight
// through its arithmetic.  Byte offsets within a vector are 32-bit (grids
// have fewer than 2^29 cells), so the loads take the vector bases as scalars.
template <int NV>
__global__ __launch_bounds__(KR_THREADS) void cgs_dots_kernel(const float2 *__restrict__ V, long long vstride,
                                                              const float2 *__restrict__ w, long long N,
                                                              const int *__restrict__ gate,
                                                              double2 *__restrict__ partial, int nblk) {
    __shared__ double2 red[(KR_THREADS / 64) * KR_SLOTS];
    constexpr int NA = NV > 0 ? NV : 1;
    const int r = blockIdx.y;
    if (!gate[r]) return;
    const char *wb = reinterpret_cast<const char *>(w + r * N);
    const char *vb = reinterpret_cast<const char *>(V + r * N);
    float2 facc[NA];
#pragma unroll
    for (int i = 0; i < NV; ++i) facc[i] = make_float2(0.f, 0.f);
    float fn = 0.f;
    // cells past the end load as zeros, which add nothing
    auto load = [&](float2 &wv, float2 (&vv)[NA], long long n) {
        if (n < N) {
            const unsigned off = (unsigned)n * 8u;
            wv = *reinterpret_cast<const float2 *>(wb + off);
#pragma unroll
            for (int i = 0; i < NV; ++i) vv[i] = *reinterpret_cast<const float2 *>(vb + i * vstride * 8 + off);
        } else {
            wv = make_float2(0.f, 0.f);
#pragma unroll
            for (int i = 0; i < NV; ++i) vv[i] = make_float2(0.f, 0.f);
        }
    };
    auto use = [&](const float2 &wv, const float2 (&vv)[NA]) {
        fn += cabs2(wv);
#pragma unroll
        for (int i = 0; i < NV; ++i) facc[i] = cfma_conj(facc[i], vv[i], wv);
    };
    const long long stride = (long long)gridDim.x * KR_THREADS;
    long long n = (long long)blockIdx.x * KR_THREADS + threadIdx.x;
    float2 wa, va[NA], wn, vn[NA];
    load(wa, va, n);
    for (; n < N; n += 2 * stride) {
        load(wn, vn, n + stride);
        use(wa, va);
        load(wa, va, n + 2 * stride);
        use(wn, vn);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const float rx = wave_sum_f(facc[i].x), ry = wave_sum_f(facc[i].y);
        if (lane == 0) red[wid * KR_SLOTS + i] = make_double2(rx, ry);
    }
    {
        const float rn = wave_sum_f(fn);
        if (lane == 0) red[wid * KR_SLOTS + KR_MAXV] = make_double2(rn, 0.0);
    }
    __syncthreads();
    double2 *pr = partial + (long long)r * nblk * KR_SLOTS;
    const int i = threadIdx.x;
    if (i < NV || i == KR_MAXV) {
        double2 s = red[i];
        for (int wv = 1; wv < KR_THREADS / 64; ++wv) s = zadd(s, red[wv * KR_SLOTS + i]);
        pr[(long long)i * nblk + blockIdx.x] = s;            // slot-major: the reduction reads rows
    }
}

// First-pass update fused with the second pass's dots: dst = w - sum_i Hc_i V_i,
// and, from the same loads of V, per-workgroup partials of V_i^H dst (slots
// i < NV) and of ||dst||^2 (slot KR_MAXV).  The second pass then needs one
// more read of V (its update) instead of two.  Laid out like the dots kernel:
// the coefficients are uniform per workgroup (scalar registers), the vector
// bases are scalars with 32-bit byte offsets, and the next cell's loads are
// issued before the current cell's arithmetic.
template <int NV>
__global__ __launch_bounds__(KR_THREADS) void cgs_update_dots_kernel(const float2 *__restrict__ V, long long vstride,
                                                                     const float2 *w, float2 *dst, long long N,
                                                                     const int *__restrict__ gate,
                                                                     const float2 *__restrict__ Hc, int m, int col,
                                                                     double2 *__restrict__ partial, int nblk,
                                                                     const float *__restrict__ scale) {
    __shared__ double2 red[(KR_THREADS / 64) * KR_SLOTS];
    constexpr int NA = NV > 0 ? NV : 1;
    const int r = blockIdx.y;
    if (!gate[r]) return;
    const float sf = scale ? scale[r] : 1.f;
    float2 h[NA];
#pragma unroll
    for (int i = 0; i < NV; ++i) h[i] = Hc[((long long)r * (m + 1) + i) * m + col];
    const char *wb = reinterpret_cast<const char *>(w + r * N);
    char *db = reinterpret_cast<char *>(dst + r * N);
    const char *vb = reinterpret_cast<const char *>(V + r * N);
    float2 facc[NA];
#pragma unroll
    for (int i = 0; i < NV; ++i) facc[i] = make_float2(0.f, 0.f);
    float fn = 0.f;
    // cells past the end load as zeros and store nothing
    auto load = [&](float2 &wv, float2 (&vv)[NA], long long n) {
        if (n < N) {
            const unsigned off = (unsigned)n * 8u;
            wv = *reinterpret_cast<const float2 *>(wb + off);
#pragma unroll
            for (int i = 0; i < NV; ++i) vv[i] = *reinterpret_cast<const float2 *>(vb + i * vstride * 8 + off);
        } else {
            wv = make_float2(0.f, 0.f);
#pragma unroll
            for (int i = 0; i < NV; ++i) vv[i] = make_float2(0.f, 0.f);
        }
    };
    auto use = [&](const float2 &wv, const float2 (&vv)[NA], long long n) {
        float2 v = wv;
#pragma unroll
        for (int i = 0; i < NV; ++i) v = cfms(v, h[i], vv[i]);
        v = cscale(v, sf);
        if (n < N) {
            // the new basis vector (one per step, far larger than the last-level
            // cache) goes out with streaming stores
            typedef float f32x2 __attribute__((ext_vector_type(2)));
            const f32x2 t = {v.x, v.y};
            __builtin_nontemporal_store(t, reinterpret_cast<f32x2 *>(db + (unsigned)n * 8u));
        }
        fn += cabs2(v);
#pragma unroll
        for (int i = 0; i < NV; ++i) facc[i] = cfma_conj(facc[i], vv[i], v);
    };
    const long long stride = (long long)gridDim.x * KR_THREADS;
    long long n = (long long)blockIdx.x * KR_THREADS + threadIdx.x;
    float2 wa, va[NA], wn, vn[NA];
    load(wa, va, n);
    for (; n < N; n += 2 * stride) {
        load(wn, vn, n + stride);
        use(wa, va, n);
        load(wa, va, n + 2 * stride);
        use(wn, vn, n + stride);
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        const float rx = wave_sum_f(facc[i].x), ry = wave_sum_f(facc[i].y);
        if (lane == 0) red[wid * KR_SLOTS + i] = make_double2(rx, ry);
    }
    {
        const float rn = wave_sum_f(fn);
        if (lane == 0) red[wid * KR_SLOTS + KR_MAXV] = make_double2(rn, 0.0);
    }
    __syncthreads();
    double2 *pr = partial + (long long)r * nblk * KR_SLOTS;
    const int i = threadIdx.x;
    if (i < NV || i == KR_MAXV) {
        double2 s = red[i];
        for (int q = 1; q < KR_THREADS / 64; ++q) s = zadd(s, red[q * KR_SLOTS + i]);
        pr[(long long)i * nblk + blockIdx.x] = s;            // slot-major: the reduction reads rows
    }
}

// Sum the partials of each RHS (fixed order; waves split the slots, lanes the
// workgroups) and take the scalar step of the Arnoldi recurrence:
//   mode 0  norm only: ||.||^2 -> norm_out (||b||, restart residuals);
//   mode 1  first-pass dots: h -> H[:, col], ||w||^2 -> nw_pre;
//   mode 2  first-pass norm: ||w'||^2; DGKS (||w'|| < 0.7 ||w|| asks for a
//           second pass: reorth = 1), else the Givens step;
//   mode 3  second-pass dots: h2 -> H2[:, col], H[:, col] += h2;
//   mode 4  norm ||.||^2 and the Givens step;
//   mode 5  fused first-pass norm and second-pass dots: the DGKS test of mode 2,
//           and where a second pass is due, the h2 bookkeeping of mode 3 and the
//           Givens step with ||w''||^2 = ||w'||^2 - ||h2||^2 (w'' = w' - V h2 and
//           V^H w'' = 0 to working precision, so the norm is known before the
//           second update runs; that update then writes v_{j+1} directly);
//   modes 6, 7  the two passes on the stored basis (stored_basis_step).
constexpr int RED_THREADS = 1024;
static_assert(KR_MAXV * KR_MAXV <= RED_THREADS && KR_MAXV <= 64, "one thread per entry of T, one wave for ||h||^2");

// Two-pass classical Gram-Schmidt on the stored basis (modes 6 and 7).  The
// orthonormal basis is V = Vs T (Vs the stored vectors, T upper triangular,
// FP64), so dots against V are T^H times dots against Vs, and an update by V h
// is an update by Vs (T h).  Step j, with w = A z_j:
//   mode 6  d = Vs^H w, ||w||^2:  h1 = T^H d -> H[:, j];  coefficients T h1 on
//           the stored vectors -> G1[:, j];  the first-pass update will store
//           s (w - V h1) with s = 1/sqrt(max(||w||^2 - ||h1||^2, 1e-20 ||w||^2))
//           (any scale is exact, T records it; this one keeps the stored
//           vectors near unit norm);
//   mode 7  d = Vs^H s w', ||s w'||^2:  h2 = T^H d / s (the second pass),
//           H[:, j] += h2, h^2 = ||w'||^2 - ||h2||^2 (V^H w'' = 0), and
//           v_{j+1} = (w' - V h2)/h enters T as its column j+1:
//           T[k][j+1] = -(T h2)_k / h (k <= j), T[j+1][j+1] = 1/(s h);
//           then the Givens step with h^2.
// The second pass thus costs no pass over the vectors: the stored vector is
// never rewritten, and the preconditioner of the next step is applied to it
// (flexible GMRES takes any direction z; the relation A Z = V H holds with V
// the orthonormal basis above).
// The operands of the step that do not depend on this step's dots (entry e =
// threadIdx.x of the leading nv x nv block of T, and for mode 7 the earlier
// rotations and the first-pass column of H), loaded before the partial sums
// so that their latency overlaps that of the reduction.
struct StepOperands {
    double2 t;
    float cs;
    float2 sn, hc;
};
__device__ __forceinline__ StepOperands stored_basis_operands(int nv, int col, int mode, int r, const GivensArgs &ga) {
    const int m = ga.m, ld = m + 1, t = threadIdx.x;
    StepOperands o = {make_double2(0.0, 0.0), 1.f, make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
    if (t < nv * nv) {
        const int k = t / nv, i = t - k * nv;
        o.t = (mode == 6 && col == 0) ? make_double2(1.0, 0.0)            // v_0 is stored normalised
              : (k <= i ? ga.T[(long long)r * ld * ld + k * ld + i] : make_double2(0.0, 0.0));
    }
    if (mode == 7) {
        if (t < col) {
            o.cs = ga.cs[r * m + t];
            o.sn = ga.sn[r * m + t];
        }
        if (t < nv) o.hc = ga.H[(long long)r * (m + 1) * m + t * m + col];
    }
    return o;
}

__device__ void stored_basis_step(const double2 *vals, int nv, int col, int mode, int r, const GivensArgs &ga,
                                  const StepOperands &op) {
    __shared__ double2 hv[KR_SLOTS];
    __shared__ double2 Ts[KR_MAXV][KR_MAXV];       // the leading nv x nv block of T (upper triangle)
    __shared__ double sh_s, sh_h;
    const int m = ga.m, ld = m + 1;
    double2 *Tr = ga.T + (long long)r * ld * ld;
    float2 *Hr = ga.H + (long long)r * (m + 1) * m;
    const int t = threadIdx.x;
    // T staged in LDS (the triangular products below walk its columns)
    if (t < nv * nv) Ts[t / nv][t % nv] = op.t;
    if (mode == 6 && col == 0 && t == 0) Tr[0] = make_double2(1.0, 0.0);
    __syncthreads();
    const double inv_s = mode == 7 ? 1.0 / (double)ga.scale[r] : 1.0;
    // h = T^H d (column i of T has entries k <= i)
    if (t < nv) {
        double sx = 0.0, sy = 0.0;
        for (int k = 0; k <= t; ++k) {
            const double2 a = Ts[k][t], d = vals[k];
            sx += a.x * d.x + a.y * d.y;
            sy += a.x * d.y - a.y * d.x;
        }
        hv[t] = make_double2(sx * inv_s, sy * inv_s);
    }
    __syncthreads();
    if (t < 64) {                                     // nv <= KR_MAXV <= 64: one wave sums ||h||^2
        const double hn = wave_sum(t < nv ? hv[t].x * hv[t].x + hv[t].y * hv[t].y : 0.0);
        if (t == 0 && mode == 6) {
            const double n2 = vals[KR_MAXV].x;
            ga.nw_pre_w[r] = n2;
            const double e = n2 - hn;
            // clamped so that a vanishing w (a breakdown, stopped by the Givens step) cannot overflow FP32
            ga.scale[r] = n2 > 0.0 ? (float)fmin(1.0 / sqrt(e > 1e-20 * n2 ? e : 1e-20 * n2), 1e30) : 1.f;
        } else if (t == 0) {
            const double n2 = vals[KR_MAXV].x * inv_s * inv_s;
            const double e = n2 > hn ? n2 - hn : 0.0;
            sh_h = e;
            sh_s = (double)ga.scale[r];
        }
    }
    __syncthreads();
    if (mode == 6) {
        if (t < nv) Hr[t * m + col] = make_float2((float)hv[t].x, (float)hv[t].y);
        // coefficients on the stored vectors: g_k = sum_{i >= k} T[k][i] h1_i
        if (t < nv) {
            double gx = 0.0, gy = 0.0;
            for (int i = t; i < nv; ++i) {
                const double2 a = Ts[t][i], h = hv[i];
                gx += a.x * h.x - a.y * h.y;
                gy += a.x * h.y + a.y * h.x;
            }
            ga.G1[((long long)r * (m + 1) + t) * m + col] = make_float2((float)gx, (float)gy);
        }
        return;
    }
    const double hsq = sh_h, h = sqrt(hsq), sc = sh_s;
    // the Givens step runs on LDS copies of the column and of the earlier
    // rotations (one dependent LDS access per rotation instead of a global round trip)
    __shared__ float2 hcol[KR_SLOTS], snl[KR_MAXV];
    __shared__ float csl[KR_MAXV];
    if (t < col) {
        csl[t] = op.cs;
        snl[t] = op.sn;
    }
    if (t < nv) {
        hcol[t] = cadd(op.hc, make_float2((float)hv[t].x, (float)hv[t].y));
        double gx = 0.0, gy = 0.0;
        for (int i = t; i < nv; ++i) {
            const double2 a = Ts[t][i], q = hv[i];
            gx += a.x * q.x - a.y * q.y;
            gy += a.x * q.y + a.y * q.x;
        }
        Tr[t * ld + col + 1] = h > 0.0 ? make_double2(-gx / h, -gy / h) : make_double2(0.0, 0.0);
    }
    if (t == 0) Tr[(col + 1) * ld + col + 1] = h > 0.0 ? make_double2(1.0 / (sc * h), 0.0) : make_double2(0.0, 0.0);
    __syncthreads();
    if (t == 0) {
        givens_core(ga, r, col, hsq, [&](int i) -> float2 & { return hcol[i]; }, [&](int i) { return csl[i]; },
                    [&](int i) { return snl[i]; });
        if (ga.host_flags) ga.host_flags[r] = ga.active[r];     // read by the host once the step has completed
    }
}

__global__ __launch_bounds__(RED_THREADS) void cgs_reduce_kernel(const double2 *__restrict__ partial, int nblk, int nv,
                                                                 const int *__restrict__ gate, int col, int mode,
                                                                 double *__restrict__ norm_out, GivensArgs ga) {
    __shared__ double2 vals[KR_SLOTS];
    const int r = blockIdx.x;
    if ((mode == 2 || mode == 5) && !ga.active[r]) {       // keep the second-pass flag of idle RHS cleared
        if (threadIdx.x == 0) ga.reorth[r] = 0;
        return;
    }
    if (gate && !gate[r]) {
        if (mode == 7 && ga.host_flags && threadIdx.x == 0) ga.host_flags[r] = 0;
        return;
    }
    const int ns = (mode == 1 || mode == 3 || mode == 5 || mode == 6 || mode == 7) ? nv : 0;
    const bool sb = mode == 6 || mode == 7;
    StepOperands op;
    if (sb) op = stored_basis_operands(nv, col, mode, r, ga);
    const double2 *pr = partial + (long long)r * nblk * KR_SLOTS;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int v = wid; v <= ns; v += RED_THREADS / 64) {
        const int slot = v < ns ? v : KR_MAXV;
        double sx = 0.0, sy = 0.0;
        for (int bk = lane; bk < nblk; bk += 64) {
            const double2 q = pr[(long long)slot * nblk + bk];
            sx += q.x;
            sy += q.y;
        }
        sx = wave_sum(sx);
        sy = wave_sum(sy);
        if (lane == 0) vals[slot] = make_double2(sx, sy);
    }
    __syncthreads();
    if (sb) {
        stored_basis_step(vals, nv, col, mode, r, ga, op);
        return;
    }
    if (threadIdx.x != 0) return;
    const double n2 = vals[KR_MAXV].x;
    const int m = ga.m;
    float2 *Hr = ga.H + (long long)r * (m + 1) * m;
    switch (mode) {
        case 0:
            norm_out[r] = n2;
            break;
        case 1:
            for (int i = 0; i < nv; ++i) Hr[i * m + col] = make_float2((float)vals[i].x, (float)vals[i].y);
            ga.nw_pre_w[r] = n2;
            break;
        case 2:
            if (n2 < 0.49 * ga.nw_pre[r]) {
                ga.reorth[r] = 1;
            } else {
                ga.reorth[r] = 0;
                givens_step(ga, r, col, n2);
            }
            break;
        case 5: {
            if (n2 >= 0.49 * ga.nw_pre[r]) {
                ga.reorth[r] = 0;
                givens_step(ga, r, col, n2);
                break;
            }
            ga.reorth[r] = 1;
            double h2n = 0.0;
            for (int i = 0; i < nv; ++i) {
                const float2 h = make_float2((float)vals[i].x, (float)vals[i].y);
                ga.H2[((long long)r * (m + 1) + i) * m + col] = h;
                Hr[i * m + col] = cadd(Hr[i * m + col], h);
                h2n += vals[i].x * vals[i].x + vals[i].y * vals[i].y;
            }
            givens_step(ga, r, col, n2 > h2n ? n2 - h2n : 0.0);
            break;
        }
        case 3:
            for (int i = 0; i < nv; ++i) {
                const float2 h = make_float2((float)vals[i].x, (float)vals[i].y);
                ga.H2[((long long)r * (m + 1) + i) * m + col] = h;
                Hr[i * m + col] = cadd(Hr[i * m + col], h);
            }
            break;
        default:
            givens_step(ga, r, col, n2);
            break;
    }
}

int nblk_for_update(long long N, int n_rhs) {
    long long nb = (N + 2047) / 2048;
    nb = std::max<long long>(nb, std::min<long long>((N + 255) / 256, (512 + n_rhs - 1) / n_rhs));
    return (int)std::max<long long>(1, std::min<long long>(1024, nb));
}

#define NOSDD_NV_CASES(X) \
    X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) \
    X(17) X(18) X(19) X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)

void launch_cgs_dots(hipStream_t s, const float2 *V, long long vstride, int nv, const float2 *w, long long N,
                     int n_rhs, const int *gate, double2 *partial, int nblk) {
    dim3 grid(nblk, n_rhs);
    switch (nv) {
#define CASE(K)                                                                                                  \
    case K:                                                                                                      \
        hipLaunchKernelGGL((cgs_dots_kernel<K>), grid, dim3(KR_THREADS), 0, s, V, vstride, w, N, gate, partial,    \
                           nblk);                                                                                \
        break;
        NOSDD_NV_CASES(CASE)
#undef CASE
        default: break;
    }
}

void launch_cgs_update_dots(hipStream_t s, const float2 *V, long long vstride, int nv, const float2 *w, float2 *dst,
                            long long N, int n_rhs, const int *gate, const float2 *Hc, int m, int col,
                            double2 *partial, int nblk, const float *scale) {
    dim3 grid(nblk, n_rhs);
    switch (nv) {
#define CASE(K)                                                                                                     \
    case K:                                                                                                         \
        hipLaunchKernelGGL((cgs_update_dots_kernel<K>), grid, dim3(KR_THREADS), 0, s, V, vstride, w, dst, N, gate,  \
                           Hc, m, col, partial, nblk, scale);                                                       \
        break;
        NOSDD_NV_CASES(CASE)
#undef CASE
        default: break;
    }
}

void launch_cgs_reduce(hipStream_t s, const double2 *partial, int nblk, int nv, int n_rhs, const int *gate, int col,
                       int mode, double *norm_out, const GivensArgs &ga) {
    hipLaunchKernelGGL(cgs_reduce_kernel, dim3(n_rhs), dim3(RED_THREADS), 0, s, partial, nblk, nv, gate, col, mode,
                       norm_out, ga);
}

// Second Gram-Schmidt pass fused with the normalisation:
//   dst = (w - sum_{i<NV} Hc[r][i][col] V_i) * inv_h[r]   where reorth[r],
//   dst = w * inv_h[r]                                    otherwise,
// for the RHS still active (their h_{j+1,j} is already known, mode 5).
template <int NV, int U>
__global__ __launch_bounds__(KR_THREADS) void cgs_update_scale_kernel(const float2 *__restrict__ V, long long vstride,
                                                                      const float2 *w, float2 *dst, long long N,
                                                                      const int *__restrict__ active,
                                                                      const int *__restrict__ reorth,
                                                                      const float2 *__restrict__ Hc, int m, int col,
                                                                      const float *__restrict__ inv_h) {
    __shared__ float2 hs[NV > 0 ? NV : 1];
    const int r = blockIdx.y;
    if (!active[r]) return;
    const float f = inv_h[r];
    const float2 *wr = w + r * N;
    float2 *dr = dst + r * N;
    const long long stride = (long long)gridDim.x * KR_THREADS * U;
    if (!reorth[r]) {
        for (long long n = (long long)blockIdx.x * KR_THREADS + threadIdx.x; n < N;
             n += (long long)gridDim.x * KR_THREADS)
            dr[n] = cscale(wr[n], f);
        return;
    }
    if (threadIdx.x < NV) hs[threadIdx.x] = Hc[((long long)r * (m + 1) + threadIdx.x) * m + col];
    __syncthreads();
    float2 hreg[NV > 0 ? NV : 1];
#pragma unroll
    for (int i = 0; i < NV; ++i) hreg[i] = hs[i];
    const float2 *Vr = V + r * N;
    for (long long n0 = (long long)blockIdx.x * KR_THREADS * U + threadIdx.x; n0 < N; n0 += stride) {
        float2 wv[U], vv[U][NV > 0 ? NV : 1];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const long long n = n0 + (long long)u * KR_THREADS;
            const bool in = n < N;
            wv[u] = in ? wr[n] : make_float2(0.f, 0.f);
#pragma unroll
            for (int i = 0; i < NV; ++i) vv[u][i] = in ? Vr[i * vstride + n] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            float2 v = wv[u];
#pragma unroll
            for (int i = 0; i < NV; ++i) v = cfms(v, hreg[i], vv[u][i]);
            const long long n = n0 + (long long)u * KR_THREADS;
            if (n < N) dr[n] = cscale(v, f);
        }
    }
}

void launch_cgs_update_scale(hipStream_t s, const float2 *V, long long vstride, int nv, const float2 *w, float2 *dst,
                             long long N, int n_rhs, const int *active, const int *reorth, const float2 *Hc, int m,
                             int col, const float *inv_h, int nblk) {
    dim3 grid(nblk, n_rhs);
    switch (nv) {
#define CASE(K)                                                                                                  \
    case K:                                                                                                      \
        hipLaunchKernelGGL((cgs_update_scale_kernel<K, (K > 16 ? 2 : 1)>), grid, dim3(KR_THREADS), 0, s, V,      \
                           vstride, w, dst, N, active, reorth, Hc, m, col, inv_h);                               \
        break;
        NOSDD_NV_CASES(CASE)
#undef CASE
        default: break;
    }
}

// y = R^-1 gamma for the k x k upper triangle of the rotated H, one workgroup
// per RHS: the triangle and gamma are staged in LDS, then one thread runs the
// substitution in the usual order (no dependent global round trips).
__global__ __launch_bounds__(64) void backsolve_kernel(const float2 *H, int m, const float2 *gam, const int *kcyc,
                                                       float2 *y) {
    __shared__ float2 Hs[KR_MAXV][KR_MAXV + 1];
    __shared__ float2 gs[KR_MAXV], ys[KR_MAXV];
    const int r = blockIdx.x;
    const int k = kcyc[r];
    const float2 *Hr = H + (long long)r * (m + 1) * m;
    for (int e = threadIdx.x; e < k * k; e += blockDim.x) {
        const int i = e / k, l = e - i * k;
        if (l >= i) Hs[i][l] = Hr[i * m + l];
    }
    if (threadIdx.x < k) gs[threadIdx.x] = gam[r * (m + 1) + threadIdx.x];
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = k - 1; i >= 0; --i) {
            float2 s = gs[i];
            for (int l = i + 1; l < k; ++l) s = cfms(s, Hs[i][l], ys[l]);
            const float2 d = Hs[i][i];
            const float dd = cabs2(d);
            ys[i] = make_float2((s.x * d.x + s.y * d.y) / dd, (s.y * d.x - s.x * d.y) / dd);
        }
    }
    __syncthreads();
    if (threadIdx.x < k) y[r * m + threadIdx.x] = ys[threadIdx.x];
}

void launch_backsolve(hipStream_t s, const float2 *H, int ldh, int m, const float2 *gam, const int *kcyc, float2 *y,
                      int n_rhs) {
    (void)ldh;
    hipLaunchKernelGGL(backsolve_kernel, dim3(n_rhs), dim3(64), 0, s, H, m, gam, kcyc, y);
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

}  // namespace nosdd
