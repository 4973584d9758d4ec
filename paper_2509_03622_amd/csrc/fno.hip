// Subdomain Fourier neural operator, batched inference on gfx950.
//
// Network (Fig. 2 architecture, plain spectral form): 9 input channels
// [Re v/s, Im v/s, (eps-1)/11, k0 h sqrt(eps), Re/Im 1/s_x, Re/Im 1/s_y,
// interface-ring mask] (s = rms of v over the subdomain), lift to C = 64,
// L blocks u <- act(W u + b + F^-1(R . F u)) on the kept modes kx in
// {0..15} U {Lx-16..Lx-1}, ky in {0..15} (512 modes), leaky ReLU 0.01
// (identity after the last block), projection 64 -> 128 (leaky) -> 2,
// output (o0 + i o1) s.
//
// A "sample" is one (subdomain, RHS) pair; all samples of a sweep run in one
// launch per stage.  Activations are FP32 [sample][C][cells] with the
// subdomain's own (lx, ly).  The dense channel contractions -- the 1x1 mix W
// and the per-mode complex mix R -- run on MFMA in BF16 with FP32
// accumulation (v_mfma_f32_32x32x8_bf16): R is applied as the real 128 x 128
// form of the complex 64 x 64 mix to (Re X_c, Im X_c) interleaved per
// channel.  The truncated DFTs are separable FP32 sums in LDS with twiddle
// tables precomputed per subdomain side.
#include "common.h"

namespace nosdd {

constexpr int FC = 64;          // channels
constexpr int FM = 16;          // modes per axis (kx: 2*FM, ky: FM)
constexpr int FMODES = 2 * FM * FM;
constexpr int FH = 128;         // projection width
constexpr int FIN = 9;
constexpr float LEAK = 0.01f;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ unsigned short f2bf(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);        // round to nearest even
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float leaky(float x) { return x >= 0.f ? x : LEAK * x; }

// ------------------------------------------------------------------ lift
// u[s][o][c] = sum_i lift_w[o][i] x_i + lift_b[o]; x from v (scaled) and aux.
__global__ __launch_bounds__(256) void fno_lift_kernel(const FnoSample *__restrict__ smp, const int *__restrict__ sact,
                                                       const float2 *__restrict__ v, const float *__restrict__ vscale,
                                                       const float *__restrict__ aux, long long aux_ch_stride,
                                                       const float *__restrict__ lw, const float *__restrict__ lb,
                                                       float *__restrict__ act) {
    __shared__ float w[FC * FIN + FC];
    const int s = blockIdx.y;
    if (sact && !sact[s]) return;
    for (int i = threadIdx.x; i < FC * FIN; i += 256) w[i] = lw[i];
    for (int i = threadIdx.x; i < FC; i += 256) w[FC * FIN + i] = lb[i];
    __syncthreads();
    const FnoSample S = smp[s];
    const int n = S.lx * S.ly;
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= n) return;
    const float sc = vscale[s];
    const float2 vv = v[S.cell_off + c];
    float x[FIN];
    x[0] = vv.x * sc;
    x[1] = vv.y * sc;
#pragma unroll
    for (int k = 0; k < 7; ++k) x[2 + k] = aux[S.aux_off + k * aux_ch_stride + c];
    float *out = act + S.cell_off * FC + c;
#pragma unroll 4
    for (int o = 0; o < FC; ++o) {
        float a = w[FC * FIN + o];
#pragma unroll
        for (int k = 0; k < FIN; ++k) a += w[o * FIN + k] * x[k];
        out[(long long)o * n] = a;
    }
}

// ------------------------------------------------------------------ forward DFT
// X[mode][s][2c], X[mode][s][2c+1] = Re, Im of the kept mode of channel c,
// mode = q * FM + ky.
__global__ __launch_bounds__(256) void fno_dft_fwd_kernel(const FnoSample *__restrict__ smp, const int *__restrict__ sact,
                                                          const float *__restrict__ act, float *__restrict__ X, int S_tot,
                                                          const float2 *__restrict__ tw) {
    __shared__ float u[72 * 72];
    __shared__ float2 T[72 * 2 * FM];
    __shared__ float2 Ex[72 * 2 * FM];
    __shared__ float2 Ey[72 * FM];
    const int ch = blockIdx.x, s = blockIdx.y;
    if (sact && !sact[s]) return;
    const FnoSample S = smp[s];
    const int lx = S.lx, ly = S.ly, n = lx * ly;
    const float *src = act + S.cell_off * FC + (long long)ch * n;
    for (int i = threadIdx.x; i < n; i += 256) u[i] = src[i];
    {
        const float2 *twx = tw + (long long)FNO_TW_UNIT * lx * (lx - 1) / 2;
        const float2 *twy = tw + (long long)FNO_TW_UNIT * ly * (ly - 1) / 2 + FNO_TW_FWD_Y * ly;
        for (int i = threadIdx.x; i < lx * 2 * FM; i += 256) Ex[i] = twx[i];
        for (int i = threadIdx.x; i < ly * FM; i += 256) Ey[i] = twy[i];
    }
    __syncthreads();
    // along x: T[y][q] = sum_x u[y][x] Ex[x][q]; a thread owns one q and FWD_RY
    // rows, so each twiddle load (consecutive q across lanes) feeds FWD_RY
    // products and the u loads are broadcasts
    constexpr int FWD_RY = 4;
    for (int e = threadIdx.x; e < ((ly + FWD_RY - 1) / FWD_RY) * 2 * FM; e += 256) {
        const int yb = (e / (2 * FM)) * FWD_RY, q = e - (e / (2 * FM)) * (2 * FM);
        float re[FWD_RY], im[FWD_RY];
#pragma unroll
        for (int i = 0; i < FWD_RY; ++i) re[i] = im[i] = 0.f;
        for (int x = 0; x < lx; ++x) {
            const float2 t = Ex[x * 2 * FM + q];
#pragma unroll
            for (int i = 0; i < FWD_RY; ++i) {
                const float a = u[min(yb + i, ly - 1) * lx + x];
                re[i] += a * t.x;
                im[i] += a * t.y;
            }
        }
#pragma unroll
        for (int i = 0; i < FWD_RY; ++i)
            if (yb + i < ly) T[(yb + i) * 2 * FM + q] = make_float2(re[i], im[i]);
    }
    __syncthreads();
    // along y: X[q][ky] = sum_y T[y][q] Ey[y][ky]
    for (int e = threadIdx.x; e < FMODES; e += 256) {
        const int q = e / FM, ky = e - q * FM;
        float re = 0.f, im = 0.f;
        for (int y = 0; y < ly; ++y) {
            const float2 t = T[y * 2 * FM + q], w = Ey[y * FM + ky];
            re += t.x * w.x - t.y * w.y;
            im += t.x * w.y + t.y * w.x;
        }
        reinterpret_cast<float2 *>(X)[((long long)e * S_tot + s) * FC + ch] = make_float2(re, im);
    }
}

// ------------------------------------------------------------------ MFMA helpers
// Wave-level 32x32 tile product with K in steps of 8 on BF16 operands in LDS.
// A is [32][K] row-major (lda), B is [K][32] row-major (ldb); both unsigned short (bf16 bits).
// Lane l holds A[l%32][4(l/32)..+3], B[4(l/32)..+3][l%32]; the result lane l holds
// D[8(i/4) + 4(l/32) + i%4][l%32] in acc[i].
__device__ __forceinline__ void mfma_tile(const unsigned short *A, int lda, const unsigned short *B, int ldb, int K,
                                          f32x16 &acc) {
    const int lane = threadIdx.x & 63;
    const int row = lane & 31, kq = (lane >> 5) * 4;
    for (int k0 = 0; k0 < K; k0 += 8) {
        bf16x4 a, b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] = (short)A[row * lda + k0 + kq + j];
            b[j] = (short)B[(k0 + kq + j) * ldb + row];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
}

__device__ __forceinline__ int mfma_row(int i) { return 8 * (i >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (i & 3); }

// ------------------------------------------------------------------ spectral mix (MFMA)
// Y[mode][s][:] = X[mode][s][:] (1 x 128, Re/Im interleaved per channel) . Rb[mode] (128 x 128),
// 64 samples per workgroup.
__global__ __launch_bounds__(256) void fno_spectral_kernel(const float *__restrict__ X,
                                                           const unsigned short *__restrict__ Rb,
                                                           float *__restrict__ Y, int S_tot) {
    __shared__ unsigned short As[64 * 128];
    __shared__ unsigned short Bs[128 * 128];
    const int mode = blockIdx.x, s0 = blockIdx.y * 64;
    const float *Xm = X + (long long)mode * S_tot * 128;
    for (int i = threadIdx.x; i < 64 * 128; i += 256) {
        const int r = i >> 7, k = i & 127;
        As[i] = (s0 + r < S_tot) ? f2bf(Xm[(long long)(s0 + r) * 128 + k]) : (unsigned short)0;
    }
    const unsigned short *Rm = Rb + (long long)mode * 128 * 128;
    for (int i = threadIdx.x; i < 128 * 128; i += 256) Bs[i] = Rm[i];
    __syncthreads();
    const int wv = threadIdx.x >> 6;          // 4 waves: rows (wv & 1) * 32, columns (wv >> 1) * 64
    const int rb = (wv & 1) * 32, cb = (wv >> 1) * 64;
    float *Ym = Y + (long long)mode * S_tot * 128;
    for (int t = 0; t < 2; ++t) {
        f32x16 acc;
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.f;
        mfma_tile(As + rb * 128, 128, Bs + cb + 32 * t, 128, 128, acc);
        const int col = cb + 32 * t + (threadIdx.x & 31);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = s0 + rb + mfma_row(i);
            if (r < S_tot) Ym[(long long)r * 128 + col] = acc[i];
        }
    }
}

// ------------------------------------------------------------------ inverse DFT
// spec[s][c][y][x] = 1/(lx ly) sum_q sum_ky c_ky Re(Y[q][ky] exp(+2 pi i (kx x/lx + ky y/ly)))
// with c_0 = 1, c_ky = 2 (Hermitian completion of the real signal along y).
__global__ __launch_bounds__(256) void fno_dft_inv_kernel(const FnoSample *__restrict__ smp, const int *__restrict__ sact,
                                                          const float *__restrict__ Y, float *__restrict__ spec,
                                                          int S_tot, const float2 *__restrict__ tw) {
    __shared__ float2 Ys[FMODES];
    __shared__ float2 P[72 * 2 * FM];
    __shared__ float2 ExT[2 * FM * 72];     // [q][x]: consecutive x in consecutive banks
    __shared__ float2 Ey[72 * FM];
    const int ch = blockIdx.x, s = blockIdx.y;
    if (sact && !sact[s]) return;
    const FnoSample S = smp[s];
    const int lx = S.lx, ly = S.ly, n = lx * ly;
    for (int e = threadIdx.x; e < FMODES; e += 256) {
        const float2 v = reinterpret_cast<const float2 *>(Y)[((long long)e * S_tot + s) * FC + ch];
        const float c = (e % FM) == 0 ? 1.f : 2.f;
        Ys[e] = make_float2(c * v.x, c * v.y);
    }
    {
        const float2 *twx = tw + (long long)FNO_TW_UNIT * lx * (lx - 1) / 2 + FNO_TW_INV_X * lx;
        const float2 *twy = tw + (long long)FNO_TW_UNIT * ly * (ly - 1) / 2 + FNO_TW_INV_Y * ly;
        for (int i = threadIdx.x; i < lx * 2 * FM; i += 256) ExT[i] = twx[i];
        for (int i = threadIdx.x; i < ly * FM; i += 256) Ey[i] = twy[i];
    }
    __syncthreads();
    // along y: P[y][q] = sum_ky Ys[q][ky] Ey[y][ky]
    for (int e = threadIdx.x; e < ly * 2 * FM; e += 256) {
        const int y = e / (2 * FM), q = e - y * (2 * FM);
        float re = 0.f, im = 0.f;
        for (int ky = 0; ky < FM; ++ky) {
            const float2 t = Ys[q * FM + ky], w = Ey[y * FM + ky];
            re += t.x * w.x - t.y * w.y;
            im += t.x * w.y + t.y * w.x;
        }
        P[y * 2 * FM + q] = make_float2(re, im);
    }
    __syncthreads();
    // along x: out[y][x] = Re sum_q P[y][q] Ex[x][q]; a thread owns one x and
    // INV_RY rows: one conflict-free twiddle load per q feeds INV_RY products,
    // the P loads are broadcasts
    constexpr int INV_RY = 8;
    const float norm = 1.f / (float)(lx * ly);
    float *dst = spec + S.cell_off * FC + (long long)ch * n;
    for (int e = threadIdx.x; e < ((ly + INV_RY - 1) / INV_RY) * lx; e += 256) {
        const int yb = (e / lx) * INV_RY, x = e - (e / lx) * lx;
        float re[INV_RY];
#pragma unroll
        for (int i = 0; i < INV_RY; ++i) re[i] = 0.f;
        for (int q = 0; q < 2 * FM; ++q) {
            const float2 w = ExT[q * lx + x];
#pragma unroll
            for (int i = 0; i < INV_RY; ++i) {
                const float2 t = P[min(yb + i, ly - 1) * 2 * FM + q];
                re[i] += t.x * w.x - t.y * w.y;
            }
        }
#pragma unroll
        for (int i = 0; i < INV_RY; ++i)
            if (yb + i < ly) dst[(yb + i) * lx + x] = re[i] * norm;
    }
}

// ------------------------------------------------------------------ pointwise (MFMA)
// out[s][o][c] = act(sum_i W[o][i] u[s][i][c] + b[o] + spec[s][o][c]) on 64-cell tiles.
__global__ __launch_bounds__(256) void fno_pointwise_kernel(const FnoSample *__restrict__ smp,
                                                            const int *__restrict__ sact, const float *__restrict__ u,
                                                            const float *__restrict__ spec,
                                                            const unsigned short *__restrict__ Wb,
                                                            const float *__restrict__ bias, float *__restrict__ out,
                                                            int apply_act) {
    __shared__ unsigned short As[FC * FC];
    __shared__ unsigned short Bs[FC * 64];
    const int s = blockIdx.y;
    if (sact && !sact[s]) return;
    const FnoSample S = smp[s];
    const int n = S.lx * S.ly;
    const int c0 = blockIdx.x * 64;
    if (c0 >= n) return;
    for (int i = threadIdx.x; i < FC * FC; i += 256) As[i] = Wb[i];
    const float *us = u + S.cell_off * FC;
    for (int i = threadIdx.x; i < FC * 64; i += 256) {
        const int k = i >> 6, c = i & 63;
        Bs[i] = (c0 + c < n) ? f2bf(us[(long long)k * n + c0 + c]) : (unsigned short)0;
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6;
    const int rb = (wv & 1) * 32, cb = (wv >> 1) * 32;
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.f;
    mfma_tile(As + rb * FC, FC, Bs + cb, 64, FC, acc);
    const int c = c0 + cb + (threadIdx.x & 31);
    if (c >= n) return;
    const float *sp = spec + S.cell_off * FC;
    float *os = out + S.cell_off * FC;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int o = rb + mfma_row(i);
        float v = acc[i] + bias[o] + sp[(long long)o * n + c];
        os[(long long)o * n + c] = apply_act ? leaky(v) : v;
    }
}

// ------------------------------------------------------------------ projection
// p = leaky(P1 u + b1) (MFMA, 128 x 64), o = P2 p + b2 (FP32), e = (o0 + i o1) * oscale.
__global__ __launch_bounds__(256) void fno_project_kernel(const FnoSample *__restrict__ smp, const int *__restrict__ sact,
                                                          const float *__restrict__ u,
                                                          const unsigned short *__restrict__ P1b,
                                                          const float *__restrict__ b1, const float *__restrict__ P2,
                                                          const float *__restrict__ b2,
                                                          const float *__restrict__ oscale, float2 *__restrict__ e) {
    __shared__ unsigned short As[FH * FC];
    __shared__ unsigned short Bs[FC * 64];
    __shared__ float Ps[FH * 64];
    const int s = blockIdx.y;
    if (sact && !sact[s]) return;
    const FnoSample S = smp[s];
    const int n = S.lx * S.ly;
    const int c0 = blockIdx.x * 64;
    if (c0 >= n) return;
    for (int i = threadIdx.x; i < FH * FC; i += 256) As[i] = P1b[i];
    const float *us = u + S.cell_off * FC;
    for (int i = threadIdx.x; i < FC * 64; i += 256) {
        const int k = i >> 6, c = i & 63;
        Bs[i] = (c0 + c < n) ? f2bf(us[(long long)k * n + c0 + c]) : (unsigned short)0;
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6;          // wave wv: rows 32 wv, both column halves
    for (int t = 0; t < 2; ++t) {
        f32x16 acc;
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.f;
        mfma_tile(As + 32 * wv * FC, FC, Bs + 32 * t, 64, FC, acc);
        const int c = 32 * t + (threadIdx.x & 31);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int o = 32 * wv + mfma_row(i);
            Ps[o * 64 + c] = leaky(acc[i] + b1[o]);
        }
    }
    __syncthreads();
    if (threadIdx.x >= 128) return;
    const int c = threadIdx.x & 63, which = threadIdx.x >> 6;
    if (c0 + c >= n) return;
    float a = b2[which];
    for (int k = 0; k < FH; ++k) a += P2[which * FH + k] * Ps[k * 64 + c];
    // two threads per cell write re / im
    float *eo = reinterpret_cast<float *>(e + S.cell_off + c0 + c);
    eo[which] = a * oscale[s];
}

// ------------------------------------------------------------------ host side
void fno_forward(hipStream_t st, const FnoDevice &net, const FnoSample *smp, const int *sact, int S_tot, int max_cells,
                 const float2 *v, const float *vscale, const float *oscale, const float *aux, long long aux_ch_stride,
                 float *act0, float *act1, float *spec, float *X, float *Y, float2 *e) {
    const int cblk = (max_cells + 255) / 256;
    const int tblk = (max_cells + 63) / 64;
    hipLaunchKernelGGL(fno_lift_kernel, dim3(cblk, S_tot), dim3(256), 0, st, smp, sact, v, vscale, aux, aux_ch_stride,
                       net.lift_w, net.lift_b, act0);
    float *cur = act0, *nxt = act1;
    for (int l = 0; l < net.layers; ++l) {
        hipLaunchKernelGGL(fno_dft_fwd_kernel, dim3(FC, S_tot), dim3(256), 0, st, smp, sact, cur, X, S_tot, net.tw);
        hipLaunchKernelGGL(fno_spectral_kernel, dim3(FMODES, (S_tot + 63) / 64), dim3(256), 0, st, X,
                           net.R + (long long)l * FMODES * 128 * 128, Y, S_tot);
        hipLaunchKernelGGL(fno_dft_inv_kernel, dim3(FC, S_tot), dim3(256), 0, st, smp, sact, Y, spec, S_tot, net.tw);
        hipLaunchKernelGGL(fno_pointwise_kernel, dim3(tblk, S_tot), dim3(256), 0, st, smp, sact, cur, spec,
                           net.W + (long long)l * FC * FC, net.b + (long long)l * FC, nxt,
                           l < net.layers - 1 ? 1 : 0);
        float *t = cur;
        cur = nxt;
        nxt = t;
    }
    hipLaunchKernelGGL(fno_project_kernel, dim3(tblk, S_tot), dim3(256), 0, st, smp, sact, cur, net.p1w, net.p1b,
                       net.p2w, net.p2b, oscale, e);
}

}  // namespace nosdd
