// Subdomain Fourier neural operator, batched inference on gfx950.
//
// Network (Fig. 2 architecture): 9 input channels
// [Re v/s, Im v/s, (eps-1)/11, k0 h sqrt(eps), Re/Im 1/s_x, Re/Im 1/s_y,
// interface-ring mask] (s = rms of v over the subdomain), lift to C = 64,
// L blocks u <- act(W u + b + F^-1(R . F u)) on the kept modes kx in
// {0..15} U {Lx-16..Lx-1}, ky in {0..15} (512 modes), leaky ReLU 0.01
// (identity after the last block), projection 64 -> 128 (leaky) -> 2,
// output (o0 + i o1) s.  The modulated low-rank form of Fig. 2 runs the same
// kernels: its R = A B is expanded once when the weights are loaded, and its
// per-mode modulation (a function of the auxiliary channels only) is formed
// once per (subdomain, wavelength) at set-up and multiplies the spectral
// product in fno_spectral_kernel.
//
// A "sample" is one (subdomain, RHS) pair; all samples of a sweep run in one
// launch per stage.  Activations are stored in BF16 [sample][C][cells] with
// the subdomain's own (lx, ly) (every block reads its input rounded to BF16,
// the operand of both the forward transform and the channel mix); the
// transforms' intermediates are split into BF16 high and low parts in LDS,
// their spectra are FP32, and the inverse-transform term handed to the
// pointwise stage is stored in BF16.  The dense channel contractions -- the 1x1 mix W
// and the per-mode complex mix R -- run on MFMA in BF16 with FP32
// accumulation (v_mfma_f32_32x32x8_bf16): R is applied as the real 128 x 128
// form of the complex 64 x 64 mix to (Re X_c, Im X_c) interleaved per
// channel.  The truncated DFTs are four batched MFMA contractions against
// twiddle tables built on the host in FP64 per subdomain side: the
// y-transform first (it keeps 16 of the ly frequencies), then the x-transform
// of those 16 rows, and the inverse in the reverse order with the Hermitian
// weights of the real inverse folded into its last table.  Both pairs run
// in BF16 (v_mfma_f32_32x32x16_bf16) on FP32 operands split into high and
// low BF16 parts, which keeps them close to FP32 accuracy.
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
__device__ __forceinline__ float bf2f(unsigned short b) { return __uint_as_float((unsigned)b << 16); }
__device__ __forceinline__ float leaky(float x) { return x >= 0.f ? x : LEAK * x; }

// ------------------------------------------------------------------ lift
// u[s][o][c] = sum_i lift_w[o][i] x_i + lift_b[o]; x from v (scaled) and aux.
__global__ __launch_bounds__(256) void fno_lift_kernel(const FnoSample *__restrict__ smp, const int *__restrict__ sact,
                                                       const float2 *__restrict__ v, const float *__restrict__ vscale,
                                                       const float *__restrict__ aux, long long aux_ch_stride,
                                                       const float *__restrict__ lw, const float *__restrict__ lb,
                                                       unsigned short *__restrict__ act) {
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
    unsigned short *out = act + S.cell_off * FC + c;
#pragma unroll 4
    for (int o = 0; o < FC; ++o) {
        float a = w[FC * FIN + o];
#pragma unroll
        for (int k = 0; k < FIN; ++k) a += w[o * FIN + k] * x[k];
        out[(long long)o * n] = f2bf(a);
    }
}

// ------------------------------------------------------------------ truncated DFTs on MFMA
// The truncated transforms of one subdomain are small dense contractions over
// a few channels at once, computed as BF16 MFMA GEMMs:
//   forward  A: T1[c][x][ky]   = sum_y u[c][y][x] e^{-2pi i ky y/Ly}
//            B: X[kx][ky][c]   = sum_x T1[c][x][ky] e^{-2pi i kx x/Lx}
//   inverse  C: P[c][ky][x]    = sum_kx Y[kx][ky][c] e^{+2pi i kx x/Lx}
//            D: s[c][y][x]     = Re sum_ky w_ky P[c][ky][x] e^{+2pi i ky y/Ly} / (Lx Ly)
// with w_0 = 1, w_ky = 2 (Hermitian completion along y).  Complex products
// use the real 2 x 2 form of each complex entry (Re/Im interleaved in K and
// N).  A and B run in one kernel that keeps T1 in LDS, C and D in one that
// keeps P in LDS.
typedef float f32x16v __attribute__((ext_vector_type(16)));
__device__ __forceinline__ const float2 *tw_side(const float2 *tw, int L) {
    return tw + (long long)FNO_TW_UNIT * L * (L - 1) / 2;
}

// C+D: both inverse transforms of FI_CB channels of one sample in one
// workgroup, the x-transform's result kept in LDS:
//   P[c][ky][x]  = sum_kx Y[kx][ky][c] e^{+2pi i kx x/Lx}             rows (c, ky), K = (kx, ri), N = (x, ri)
//   s[c][y][x]   = Re sum_ky w_ky P[c][ky][x] e^{+2pi i ky y/Ly} / (Lx Ly)   rows y, K = (ky, ri), N = (c, x)
// (w_0 = 1, w_ky = 2: Hermitian completion along y).  Both run as BF16 MFMA
// contractions (v_mfma_f32_32x32x16_bf16) with every FP32 operand split into
// BF16 high and low parts, v = h + l with |v - h - l| <= 2^-16 |v|, and three
// products per k step (h h, h l, l h; the l l term is below FP32 rounding of
// the sum), so the transforms keep close to FP32 accuracy at the BF16 rate.
// The x-transform's B operand is the host-built table twb (high and low parts
// of the FP64 twiddles); its result goes to LDS already split, as the
// y-transform's B operand.  A lane's eight k values of an operand are one
// 16-byte load; the A and B operands use the same lane-to-k assignment, so the
// contraction does not depend on the order of k inside a lane group.
// Grid (64 / FI_CB, S), FI_THREADS threads, FI_LDS bytes of dynamic LDS (BF16):
//   Ya [2][FI_CB 16][FI_KA]   the block's spectrum, rows (c, ky), k = (kx, ri)
//   Pb [2][FI_CB 72][FI_KP]   P, rows n = (c, x), k = (ky, ri)
//   Wa [2][96][FI_KP]         the inverse y weights, rows y, k = (ky, ri)
constexpr int FI_CB = 4, FI_THREADS = 512;
constexpr int FI_KA = 4 * FM + 8, FI_KP = 2 * FM + 8, FI_NP = FI_CB * FNO_MAXL, FI_YR = 96;
constexpr size_t FI_LDS = 2 * ((size_t)2 * FI_CB * FM * FI_KA + (size_t)2 * FI_NP * FI_KP + (size_t)2 * FI_YR * FI_KP);
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
__device__ __forceinline__ bf16x8v ld_bf8(const unsigned short *p) {
    return __builtin_bit_cast(bf16x8v, *reinterpret_cast<const uint4 *>(p));
}
__device__ __forceinline__ void split_bf(float v, unsigned short &h, unsigned short &l) {
    h = f2bf(v);
    l = f2bf(v - bf2f(h));
}
__device__ __forceinline__ f32x16v mfma_hl(bf16x8v ah, bf16x8v al, bf16x8v bh, bf16x8v bl, f32x16v acc) {
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
    return acc;
}
__global__ __launch_bounds__(FI_THREADS) void fno_dft_inv_kernel(const FnoSample *__restrict__ smp,
                                                                 const int *__restrict__ sact,
                                                                 const float *__restrict__ Y,
                                                                 unsigned short *__restrict__ spec, int S_tot,
                                                                 const float2 *__restrict__ tw,
                                                                 const unsigned short *__restrict__ twb) {
    extern __shared__ __align__(16) unsigned short fb[];
    const int s = blockIdx.y;
    if (sact && !sact[s]) return;
    const FnoSample S = smp[s];
    const int lx = S.lx, ly = S.ly, n = lx * ly;
    const int c0 = blockIdx.x * FI_CB;
    unsigned short *Ya = fb;                                   // [hi, lo][FI_CB * FM][FI_KA]
    unsigned short *Pb = Ya + 2 * FI_CB * FM * FI_KA;          // [hi, lo][FI_NP][FI_KP]
    unsigned short *Wa = Pb + 2 * FI_NP * FI_KP;               // [hi, lo][FI_YR][FI_KP]
    constexpr int YA_LO = FI_CB * FM * FI_KA, PB_LO = FI_NP * FI_KP, WA_LO = FI_YR * FI_KP;
    // the block's modes: FI_CB channels x (Re, Im) per mode, as float4 pairs of channels
    const long long mstride = (long long)S_tot * (2 * FC);
    for (int i = threadIdx.x; i < FMODES * (FI_CB / 2); i += FI_THREADS) {
        const int mode = i / (FI_CB / 2), h = i % (FI_CB / 2);
        const float4 v = *reinterpret_cast<const float4 *>(Y + mode * mstride + (long long)s * (2 * FC) + 2 * c0 + 4 * h);
        const int kx = mode / FM, ky = mode % FM;
        unsigned short *ra = Ya + ((2 * h) * FM + ky) * FI_KA + 2 * kx, *rb = ra + FM * FI_KA;
        split_bf(v.x, ra[0], ra[YA_LO]);
        split_bf(v.y, ra[1], ra[YA_LO + 1]);
        split_bf(v.z, rb[0], rb[YA_LO]);
        split_bf(v.w, rb[1], rb[YA_LO + 1]);
    }
    // inverse y weights (rows y >= ly are zero), and P's rows beyond the block's cells
    const float2 *ey = tw_side(tw, ly) + FNO_TW_INV_Y * ly;     // [y][ky]
    const float norm = 1.f / (float)n;
    for (int i = threadIdx.x; i < FI_YR * FM; i += FI_THREADS) {
        const int y = i / FM, ky = i % FM;
        float wr = 0.f, wi = 0.f;
        if (y < ly) {
            const float2 e = ey[y * FM + ky];
            const float w = (ky == 0 ? 1.f : 2.f) * norm;
            wr = w * e.x;
            wi = -w * e.y;
        }
        unsigned short *wa = Wa + y * FI_KP + 2 * ky;
        split_bf(wr, wa[0], wa[WA_LO]);
        split_bf(wi, wa[1], wa[WA_LO + 1]);
    }
    for (int i = threadIdx.x; i < (FI_NP - FI_CB * lx) * 2 * FM; i += FI_THREADS) {
        const int r = FI_CB * lx + i / (2 * FM), k = i % (2 * FM);
        Pb[r * FI_KP + k] = 0;
        Pb[PB_LO + r * FI_KP + k] = 0;
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 31, lk = 8 * (lane >> 5);
    constexpr int NW = FI_THREADS / 64;
    // x-transform: rows (c, ky) in FI_CB / 2 tiles of 32, N = (x, ri) in tiles of 32, K = 64;
    // a wave takes one column tile for every row tile, so its B fragments are loaded once
    {
        const int N = 2 * lx, nct = (N + 31) / 32;
        const unsigned short *tb = twb + (size_t)128 * lx * (lx - 1), *tbl = tb + (size_t)2 * lx * 64;
        for (int ct = wv; ct < nct; ct += NW) {
            const int nn = ct * 32 + lr, nr = min(nn, N - 1);
            f32x16v acc[FI_CB / 2];
#pragma unroll
            for (int rt = 0; rt < FI_CB / 2; ++rt)
#pragma unroll
                for (int i = 0; i < 16; ++i) acc[rt][i] = 0.f;
#pragma unroll
            for (int k0 = 0; k0 < 4 * FM; k0 += 16) {
                const bf16x8v bh = ld_bf8(tb + nr * 64 + k0 + lk), bl = ld_bf8(tbl + nr * 64 + k0 + lk);
#pragma unroll
                for (int rt = 0; rt < FI_CB / 2; ++rt) {
                    const unsigned short *ar = Ya + (rt * 32 + lr) * FI_KA + k0 + lk;
                    acc[rt] = mfma_hl(ld_bf8(ar), ld_bf8(ar + YA_LO), bh, bl, acc[rt]);
                }
            }
            if (nn < N) {
                const int x = nn >> 1, ro = nn & 1;
#pragma unroll
                for (int rt = 0; rt < FI_CB / 2; ++rt)
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        const int row = rt * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
                        const int c = row / FM, ky = row % FM;
                        unsigned short *pb = Pb + (c * lx + x) * FI_KP + 2 * ky + ro;
                        split_bf(acc[rt][i], pb[0], pb[PB_LO]);
                    }
            }
        }
    }
    __syncthreads();
    // y-transform: rows y (3 tiles of 32), N = (c, x) (FI_CB Lx) in tiles of 32, K = 32
    {
        const int N = FI_CB * lx, nrt = (ly + 31) / 32, nct = (N + 31) / 32, ntile = nrt * nct;
        unsigned short *sp = spec + S.cell_off * FC + (long long)c0 * n;
        for (int t = wv; t < ntile; t += NW) {
            const int rt = t / nct, ct = t % nct;
            const int nn = ct * 32 + lr;
            const unsigned short *ar = Wa + (rt * 32 + lr) * FI_KP + lk, *br = Pb + nn * FI_KP + lk;
            f32x16v acc;
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[i] = 0.f;
#pragma unroll
            for (int k0 = 0; k0 < 2 * FM; k0 += 16)
                acc = mfma_hl(ld_bf8(ar + k0), ld_bf8(ar + WA_LO + k0), ld_bf8(br + k0), ld_bf8(br + PB_LO + k0), acc);
            if (nn < N) {
                const int c = nn / lx, x = nn % lx;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int yy = rt * 32 + 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);
                    if (yy < ly) sp[(long long)c * n + yy * lx + x] = f2bf(acc[i]);
                }
            }
        }
    }
}

// A+B: both forward transforms of FF_CB channels of one sample in one
// workgroup, the y-transform's result kept in LDS (no T1 round trip):
//   T1[c][x][ky] = sum_y u[c][y][x] e^{-2pi i ky y/Ly}       rows (ky, ri), K = y, N = (c, x)
//   X[kx][ky][c] = sum_x T1[c][x][ky] e^{-2pi i kx x/Lx}     rows (c, ky), K = (x, ri), N = (kx, ri)
// on BF16 MFMA (v_mfma_f32_32x32x16_bf16).  The activations are BF16 values
// already, so the y-transform needs two products per k step (twiddle high and
// low parts); T1 goes to LDS split into high and low parts and the
// x-transform takes three (against the host-built table twf).
// Grid (64 / FF_CB, S), FF_THREADS threads, FF_LDS bytes of dynamic LDS (BF16):
//   Bu [FF_NU][FF_KY]          activations, rows n = (c, x), k = y (zero for y >= ly)
//   Ey [2][32][FF_KY]          forward y twiddles, rows (ky, ri), k = y
//   A2 [2][FF_CB 16][FF_K2]    T1, rows (c, ky), k = (x, ri) (zero for x >= lx)
//   Xs (aliases Bu) [512][2 FF_CB] f32: the block's modes, for 16-byte stores
constexpr int FF_CB = 2, FF_THREADS = 512;
constexpr int FF_LPT = (FF_CB * FNO_MAXL * FNO_MAXL + FF_THREADS - 1) / FF_THREADS;   // activation loads per thread
constexpr int FF_KY = 88, FF_NU = 5 * 32, FF_K2 = 2 * FNO_MAXL + 8;
constexpr size_t FF_LDS = 2 * ((size_t)FF_NU * FF_KY + (size_t)2 * 32 * FF_KY + (size_t)2 * FF_CB * FM * FF_K2);
static_assert(FF_CB * FNO_MAXL <= FF_NU && FNO_MAXL <= 80 && FNO_TWF_K % 16 == 0, "one sample's rows and k fit the buffers");
static_assert(sizeof(float) * FMODES * 2 * FF_CB <= 2 * (size_t)FF_NU * FF_KY, "Xs fits in Bu");
__global__ __launch_bounds__(FF_THREADS) void fno_dft_fwd_kernel(const FnoSample *__restrict__ smp,
                                                                 const int *__restrict__ sact,
                                                                 const unsigned short *__restrict__ act,
                                                                 float *__restrict__ X, int S_tot,
                                                                 const float2 *__restrict__ tw,
                                                                 const unsigned short *__restrict__ twf) {
    extern __shared__ __align__(16) unsigned short fb[];
    const int s = blockIdx.y;
    if (sact && !sact[s]) return;
    const FnoSample S = smp[s];
    const int lx = S.lx, ly = S.ly, n = lx * ly;
    const int c0 = blockIdx.x * FF_CB;
    unsigned short *Bu = fb;                                   // [FF_NU][FF_KY]
    unsigned short *Ey = Bu + FF_NU * FF_KY;                   // [hi, lo][32][FF_KY]
    unsigned short *A2 = Ey + 2 * 32 * FF_KY;                  // [hi, lo][FF_CB * FM][FF_K2]
    constexpr int EY_LO = 32 * FF_KY, A2_LO = FF_CB * FM * FF_K2;
    // activations, transposed to rows (c, x) with y contiguous: every load of the
    // thread is issued before the first store, and the (c, y, x) of its elements
    // advance by the thread stride without divisions.  The k padding y >= ly of
    // those rows is zeroed (the twiddles are zero there too, but 0 x NaN is not
    // zero); rows beyond FF_CB lx only feed output columns that are dropped.
    const unsigned short *u = act + S.cell_off * FC + (long long)c0 * n;
    {
        unsigned short uv[FF_LPT];
#pragma unroll
        for (int j = 0; j < FF_LPT; ++j) {
            const int i = threadIdx.x + j * FF_THREADS;
            uv[j] = i < FF_CB * n ? u[i] : (unsigned short)0;
        }
        const int dy = FF_THREADS / lx, dx = FF_THREADS % lx;
        int c = threadIdx.x / n, y = (threadIdx.x % n) / lx, x = threadIdx.x % lx;
#pragma unroll
        for (int j = 0; j < FF_LPT; ++j) {
            if (c < FF_CB) Bu[(c * lx + x) * FF_KY + y] = uv[j];
            x += dx;
            y += dy;
            if (x >= lx) {
                x -= lx;
                ++y;
            }
            while (y >= ly) {
                y -= ly;
                ++c;
            }
        }
        const int npad = 80 - ly;
        for (int i = threadIdx.x; i < FF_CB * lx * npad; i += FF_THREADS)
            Bu[(i / npad) * FF_KY + ly + i % npad] = 0;
    }
    // forward y twiddles (FP32 table) split into high and low parts; k >= ly zero
    const float2 *ey = tw_side(tw, ly) + FNO_TW_FWD_Y * ly;     // [y][ky]
    for (int i = threadIdx.x; i < FM * FF_KY; i += FF_THREADS) {
        const int ky = i / FF_KY, y = i % FF_KY;
        const float2 e = y < ly ? ey[y * FM + ky] : make_float2(0.f, 0.f);
        unsigned short *er = Ey + (2 * ky) * FF_KY + y;
        split_bf(e.x, er[0], er[EY_LO]);
        split_bf(e.y, er[FF_KY], er[EY_LO + FF_KY]);
    }
    // T1's k >= 2 lx (x beyond the sample) zero
    for (int i = threadIdx.x; i < FF_CB * FM * (FF_K2 - 2 * lx); i += FF_THREADS) {
        const int r = i / (FF_K2 - 2 * lx), k = 2 * lx + i % (FF_K2 - 2 * lx);
        A2[r * FF_K2 + k] = 0;
        A2[A2_LO + r * FF_K2 + k] = 0;
    }
    __syncthreads();
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane & 31, lk = 8 * (lane >> 5);
    constexpr int NW = FF_THREADS / 64;
    // y-transform: one row tile (ky, ri), N = (c, x) in tiles of 32, K = y (5 steps of 16)
    {
        const int N = FF_CB * lx, nct = (N + 31) / 32;
        const unsigned short *ar = Ey + lr * FF_KY + lk;
        for (int ct = wv; ct < nct; ct += NW) {
            const int nn = ct * 32 + lr;
            const unsigned short *br = Bu + nn * FF_KY + lk;
            f32x16v acc;
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[i] = 0.f;
#pragma unroll
            for (int k0 = 0; k0 < 80; k0 += 16) {
                const bf16x8v b = ld_bf8(br + k0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ld_bf8(ar + k0), b, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ld_bf8(ar + EY_LO + k0), b, acc, 0, 0, 0);
            }
            if (nn < N) {
                const int c = nn / lx, x = nn % lx;
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int row = 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);     // (ky, ri)
                    unsigned short *a2 = A2 + (c * FM + (row >> 1)) * FF_K2 + 2 * x + (row & 1);
                    split_bf(acc[i], a2[0], a2[A2_LO]);
                }
            }
        }
    }
    __syncthreads();
    // x-transform: one row tile (c, ky), N = (kx, ri) in 2 tiles, K = (x, ri) in steps of 16
    float *Xs = reinterpret_cast<float *>(Bu);                 // [mode][2 FF_CB]
    {
        // all FNO_TWF_K / 16 steps: the table and T1 are zero for k >= 2 lx, and the
        // fixed count lets every twiddle load be issued ahead of the products
        const unsigned short *tf = twf + (size_t)2 * 64 * FNO_TWF_K * (lx - 1), *tfl = tf + (size_t)64 * FNO_TWF_K;
        const unsigned short *ar = A2 + lr * FF_K2 + lk;
        for (int ct = wv; ct < 2; ct += NW) {
            const int nn = ct * 32 + lr;
            const unsigned short *bh = tf + nn * FNO_TWF_K + lk, *bl = tfl + nn * FNO_TWF_K + lk;
            f32x16v acc;
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[i] = 0.f;
#pragma unroll
            for (int ks = 0; ks < FNO_TWF_K / 16; ++ks)
                acc = mfma_hl(ld_bf8(ar + 16 * ks), ld_bf8(ar + A2_LO + 16 * ks), ld_bf8(bh + 16 * ks),
                              ld_bf8(bl + 16 * ks), acc);
            const int q = nn >> 1, ro = nn & 1;
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int row = 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3);         // (c, ky)
                Xs[(q * FM + (row % FM)) * (2 * FF_CB) + 2 * (row / FM) + ro] = acc[i];
            }
        }
    }
    __syncthreads();
    for (int mode = threadIdx.x; mode < FMODES; mode += FF_THREADS) {
        const float4 v = *reinterpret_cast<const float4 *>(Xs + mode * (2 * FF_CB));
        *reinterpret_cast<float4 *>(X + ((long long)mode * S_tot + s) * (2 * FC) + 2 * c0) = v;
    }
}

// ------------------------------------------------------------------ MFMA helpers
// Wave-level 32x32 tile product with K in steps of 8 on BF16 operands in LDS.
// A is [32][K] (row stride lda) and Bt is B transposed, [32][K] (row stride
// ldb), both k-contiguous (unsigned short, bf16 bits), so lane l reads its
// A[l%32][4(l/32)..+3] and B[4(l/32)..+3][l%32] as one 8-byte LDS load each.
// Row strides of K + 4 elements put consecutive rows two banks apart, so a
// wave's loads are conflict-free (a stride of K elements would put all 32
// rows in one bank).  The result lane l holds D[8(i/4) + 4(l/32) + i%4][l%32]
// in acc[i].
constexpr int LDS_PAD = 4;
__device__ __forceinline__ void mfma_tile(const unsigned short *A, int lda, const unsigned short *Bt, int ldb, int K,
                                          f32x16 &acc) {
    const int lane = threadIdx.x & 63;
    const int row = lane & 31, kq = (lane >> 5) * 4;
    const unsigned short *ap = A + row * lda + kq, *bp = Bt + row * ldb + kq;
    for (int k0 = 0; k0 < K; k0 += 8) {
        const bf16x4 a = *reinterpret_cast<const bf16x4 *>(ap + k0);
        const bf16x4 b = *reinterpret_cast<const bf16x4 *>(bp + k0);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc, 0, 0, 0);
    }
}

// Stage a [K][64] block of BF16 values from global memory (element (k, c) at
// src[k * stride + c], c < valid, zero beyond) into LDS transposed, Bt[c][k]
// with row stride K + LDS_PAD: each thread gathers four consecutive k of one
// c (coalesced over c across the wave) and stores them as one 8-byte word.
template <int K>
__device__ __forceinline__ void stage_transposed(unsigned short *Bt, const unsigned short *src, long long stride,
                                                 int valid) {
    for (int i = threadIdx.x; i < 64 * (K / 4); i += 256) {
        const int c = i & 63, k4 = (i >> 6) * 4;
        bf16x4 v;
#pragma unroll
        for (int j = 0; j < 4; ++j) v[j] = (short)(c < valid ? src[(long long)(k4 + j) * stride + c] : 0);
        *reinterpret_cast<bf16x4 *>(Bt + c * (K + LDS_PAD) + k4) = v;
    }
}

__device__ __forceinline__ int mfma_row(int i) { return 8 * (i >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (i & 3); }

// ------------------------------------------------------------------ spectral mix (MFMA)
// Y[mode][s][:] = X[mode][s][:] (1 x 128, Re/Im interleaved per channel) . Rb[mode] (128 x 128),
// 64 samples per workgroup.
// With mod (modulated network), output (o, Re/Im) pairs of sample s are
// multiplied by mod[smp[s].mod_idx][layer][mode] (complex); the pair sits in
// two adjacent lanes.
__global__ __launch_bounds__(256) void fno_spectral_kernel(const float *__restrict__ X,
                                                           const unsigned short *__restrict__ Rb,
                                                           float *__restrict__ Y, int S_tot,
                                                           const FnoSample *__restrict__ smp,
                                                           const float2 *__restrict__ mod, int layer, int n_layers) {
    constexpr int LD = 128 + LDS_PAD;
    __shared__ __align__(16) unsigned short As[64 * LD];
    __shared__ __align__(16) unsigned short Bt[128 * LD];      // R of this mode, transposed: [out][in]
    const int mode = blockIdx.x, s0 = blockIdx.y * 64;
    const float *Xm = X + (long long)mode * S_tot * 128;
    for (int i = threadIdx.x; i < 64 * 64; i += 256) {
        const int r = i >> 6, k = 2 * (i & 63);
        float2 x = make_float2(0.f, 0.f);
        if (s0 + r < S_tot) x = *reinterpret_cast<const float2 *>(Xm + (long long)(s0 + r) * 128 + k);
        *reinterpret_cast<unsigned *>(As + r * LD + k) = (unsigned)f2bf(x.x) | ((unsigned)f2bf(x.y) << 16);
    }
    const unsigned short *Rm = Rb + (long long)mode * 128 * 128;
    stage_transposed<128>(Bt, Rm, 128, 64);
    stage_transposed<128>(Bt + 64 * LD, Rm + 64, 128, 64);
    __syncthreads();
    const int wv = threadIdx.x >> 6;          // 4 waves: rows (wv & 1) * 32, columns (wv >> 1) * 64
    const int rb = (wv & 1) * 32, cb = (wv >> 1) * 64;
    float *Ym = Y + (long long)mode * S_tot * 128;
    for (int t = 0; t < 2; ++t) {
        f32x16 acc;
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.f;
        mfma_tile(As + rb * LD, LD, Bt + (cb + 32 * t) * LD, LD, 128, acc);
        const int col = cb + 32 * t + (threadIdx.x & 31);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int r = s0 + rb + mfma_row(i);
            float v = acc[i];
            if (mod) {                                       // uniform branch: every lane shuffles
                const float partner = __shfl_xor(v, 1, 64);
                const float2 md = mod[((long long)smp[r < S_tot ? r : S_tot - 1].mod_idx * n_layers + layer) *
                                          FMODES + mode];
                const float re = (col & 1) ? partner : v, im = (col & 1) ? v : partner;
                v = (col & 1) ? md.x * im + md.y * re : md.x * re - md.y * im;
            }
            if (r < S_tot) Ym[(long long)r * 128 + col] = v;
        }
    }
}

// ------------------------------------------------------------------ pointwise (MFMA)
// out[s][o][c] = act(sum_i W[o][i] u[s][i][c] + b[o] + spec[s][o][c]) on 64-cell
// tiles, FNO_PW_TILES tiles per workgroup (W is staged in LDS once for all;
// one tile per workgroup measured fastest: more workgroups in flight).
constexpr int FNO_PW_TILES = 1, FNO_PROJ_TILES = 4;
__global__ __launch_bounds__(256) void fno_pointwise_kernel(const FnoSample *__restrict__ smp,
                                                            const int *__restrict__ sact,
                                                            const unsigned short *__restrict__ u,
                                                            const unsigned short *__restrict__ spec,
                                                            const unsigned short *__restrict__ Wb,
                                                            const float *__restrict__ bias, unsigned short *__restrict__ out,
                                                            int apply_act) {
    constexpr int LD = FC + LDS_PAD;
    __shared__ __align__(16) unsigned short As[FC * LD];       // W [o][i]
    __shared__ __align__(16) unsigned short Bt[64 * LD];       // u of the tile, transposed: [cell][i]
    __shared__ float bs[FC];
    const int s = blockIdx.y;
    if (sact && !sact[s]) return;
    const FnoSample S = smp[s];
    const int n = S.lx * S.ly;
    const int cbase = blockIdx.x * 64 * FNO_PW_TILES;
    if (cbase >= n) return;
    for (int i = threadIdx.x; i < FC * FC; i += 256) As[(i / FC) * LD + i % FC] = Wb[i];
    if (threadIdx.x < FC) bs[threadIdx.x] = bias[threadIdx.x];
    const unsigned short *us = u + S.cell_off * FC;
    const unsigned short *sp = spec + S.cell_off * FC;
    unsigned short *os = out + S.cell_off * FC;
    const int wv = threadIdx.x >> 6;
    const int rb = (wv & 1) * 32, cb = (wv >> 1) * 32;
    for (int t = 0; t < FNO_PW_TILES; ++t) {
        const int c0 = cbase + 64 * t;
        if (c0 >= n) break;
        __syncthreads();                              // previous tile's operands consumed
        stage_transposed<FC>(Bt, us + c0, n, n - c0);
        __syncthreads();
        f32x16 acc;
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[i] = 0.f;
        mfma_tile(As + rb * LD, LD, Bt + cb * LD, LD, FC, acc);
        const int c = c0 + cb + (threadIdx.x & 31);
        if (c < n) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int o = rb + mfma_row(i);
                const float v = acc[i] + bs[o] + bf2f(sp[(long long)o * n + c]);
                os[(long long)o * n + c] = f2bf(apply_act ? leaky(v) : v);
            }
        }
    }
}

// ------------------------------------------------------------------ projection
// p = leaky(P1 u + b1) (MFMA, 128 x 64), o = P2 p + b2 (FP32), e = (o0 + i o1) * oscale,
// FNO_PROJ_TILES 64-cell tiles per workgroup; the 128-term sums of the last
// projection are split in two halves over all 256 threads.
__global__ __launch_bounds__(256) void fno_project_kernel(const FnoSample *__restrict__ smp, const int *__restrict__ sact,
                                                          const unsigned short *__restrict__ u,
                                                          const unsigned short *__restrict__ P1b,
                                                          const float *__restrict__ b1, const float *__restrict__ P2,
                                                          const float *__restrict__ b2,
                                                          const float *__restrict__ oscale, float2 *__restrict__ e) {
    constexpr int LD = FC + LDS_PAD;
    __shared__ __align__(16) unsigned short As[FH * LD];       // P1 [h][c]
    __shared__ __align__(16) unsigned short Bt[64 * LD];       // u of the tile, transposed: [cell][c]
    __shared__ float Ps[FH * 64];
    __shared__ float p2s[2 * FH], b1s[FH], red[2][2][64];
    const int s = blockIdx.y;
    if (sact && !sact[s]) return;
    const FnoSample S = smp[s];
    const int n = S.lx * S.ly;
    const int cbase = blockIdx.x * 64 * FNO_PROJ_TILES;
    if (cbase >= n) return;
    for (int i = threadIdx.x; i < FH * FC; i += 256) As[(i / FC) * LD + i % FC] = P1b[i];
    for (int i = threadIdx.x; i < 2 * FH; i += 256) p2s[i] = P2[i];
    for (int i = threadIdx.x; i < FH; i += 256) b1s[i] = b1[i];
    const unsigned short *us = u + S.cell_off * FC;
    const float osc = oscale[s];
    const int wv = threadIdx.x >> 6;          // wave wv: rows 32 wv, both column halves
    const int tc = threadIdx.x & 63, which = (threadIdx.x >> 6) & 1, half = threadIdx.x >> 7;
    for (int tt = 0; tt < FNO_PROJ_TILES; ++tt) {
        const int c0 = cbase + 64 * tt;
        if (c0 >= n) break;
        __syncthreads();                              // previous tile's Bt, Ps and red consumed
        stage_transposed<FC>(Bt, us + c0, n, n - c0);
        __syncthreads();
        for (int t = 0; t < 2; ++t) {
            f32x16 acc;
#pragma unroll
            for (int i = 0; i < 16; ++i) acc[i] = 0.f;
            mfma_tile(As + 32 * wv * LD, LD, Bt + 32 * t * LD, LD, FC, acc);
            const int c = 32 * t + (threadIdx.x & 31);
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int o = 32 * wv + mfma_row(i);
                Ps[o * 64 + c] = leaky(acc[i] + b1s[o]);
            }
        }
        __syncthreads();
        float a = 0.f;
#pragma unroll 8
        for (int k = half * (FH / 2); k < (half + 1) * (FH / 2); ++k) a += p2s[which * FH + k] * Ps[k * 64 + tc];
        red[half][which][tc] = a;
        __syncthreads();
        if (threadIdx.x < 128 && c0 + tc < n) {
            // two threads per cell write re / im
            float *eo = reinterpret_cast<float *>(e + S.cell_off + c0 + tc);
            eo[which] = (b2[which] + red[0][which][tc] + red[1][which][tc]) * osc;
        }
    }
}

// ------------------------------------------------------------------ host side
void fno_prepare() {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&fno_dft_inv_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)FI_LDS);
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&fno_dft_fwd_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)FF_LDS);
}

void fno_forward(hipStream_t st, const FnoDevice &net, const FnoSample *smp, const int *sact, int S_tot, int max_cells,
                 const float2 *v, const float *vscale, const float *oscale, const float *aux, long long aux_ch_stride,
                 float *act0, float *act1, float *spec, float *X, float *Y, float2 *e) {
    const int cblk = (max_cells + 255) / 256;
    const int tblk = (max_cells + 64 * FNO_PW_TILES - 1) / (64 * FNO_PW_TILES);
    const int pblk = (max_cells + 64 * FNO_PROJ_TILES - 1) / (64 * FNO_PROJ_TILES);
    // activations are stored in BF16 [sample][channel][cell] between kernels
    auto bf = [](float *p) { return reinterpret_cast<unsigned short *>(p); };
    hipLaunchKernelGGL(fno_lift_kernel, dim3(cblk, S_tot), dim3(256), 0, st, smp, sact, v, vscale, aux, aux_ch_stride,
                       net.lift_w, net.lift_b, bf(act0));
    float *cur = act0, *nxt = act1;
    for (int l = 0; l < net.layers; ++l) {
        hipLaunchKernelGGL(fno_dft_fwd_kernel, dim3(FC / FF_CB, S_tot), dim3(FF_THREADS), FF_LDS, st, smp, sact,
                           bf(cur), X, S_tot, net.tw, net.twf);
        hipLaunchKernelGGL(fno_spectral_kernel, dim3(FMODES, (S_tot + 63) / 64), dim3(256), 0, st, X,
                           net.R + (long long)l * FMODES * 128 * 128, Y, S_tot, smp, net.mod, l, net.layers);
        hipLaunchKernelGGL(fno_dft_inv_kernel, dim3(FC / FI_CB, S_tot), dim3(FI_THREADS), FI_LDS, st, smp, sact, Y,
                           bf(spec), S_tot, net.tw, net.twb);
        hipLaunchKernelGGL(fno_pointwise_kernel, dim3(tblk, S_tot), dim3(256), 0, st, smp, sact, bf(cur), bf(spec),
                           net.W + (long long)l * FC * FC, net.b + (long long)l * FC, bf(nxt),
                           l < net.layers - 1 ? 1 : 0);
        float *t = cur;
        cur = nxt;
        nxt = t;
    }
    hipLaunchKernelGGL(fno_project_kernel, dim3(pblk, S_tot), dim3(256), 0, st, smp, sact, bf(cur), net.p1w, net.p1b,
                       net.p2w, net.p2b, oscale, e);
}

}  // namespace nosdd
