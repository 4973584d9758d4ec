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
// The UPML operator is S^-1 times a complex-symmetric matrix (S = s_x s_y at
// cell centres) and the Robin closure only changes the diagonal, so with
// S_k the stretches of block k, S_k D_k is the Schur complement of the
// symmetric matrix S B_i and M_k = D_k^-1 S_k^-1 is complex symmetric:
// D_k^-1 y = M_k (S_k y), and half of M_k suffices (layout in common.h).
//
// bt_factor_*_kernel (set-up, once per tile and wavelength): builds D_k in
// FP64 and inverts it by Gauss-Jordan elimination with partial pivoting, then
// stores the upper triangle of M_k as complex64 sub-blocks.
//
// bt_solve_kernel (hot path): one workgroup per (tile, RHS) streams the
// 2 nb - 1 blocks M_k from HBM, each once, and keeps the sequential
// recurrence in LDS.  The M blocks do not depend on the data, so each thread
// holds the blocks of the next steps in registers while it multiplies the
// current one.  The gather of R_i v (input restricted to the extended tile,
// which carries the neighbours' Robin traces by the Robin identity) and the
// core-only scatter (restricted additive Schwarz prolongation) are fused into
// the same kernel.
#include <algorithm>

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
constexpr int BT_FACT_LDS_B = 72;        // FP64 block of 72 x 72 = 81 KB of LDS
constexpr int BT_FACT_MAX_B = 128;       // larger blocks work in a global FP64 scratch

// Block-Thomas factorisation of one (tile, wavelength): D_k^-1 for every block
// k, with the b x b FP64 working matrix M (row-major) in LDS or in global
// scratch private to the workgroup.
template <int BMAX>
__device__ __forceinline__ void bt_factor_body(double2 *M, double2 *fcol, double2 *prow, int *piv, int *pivrow,
                                               const TileDesc &t, int wl, const float *__restrict__ eps,
                                               const double2 *__restrict__ coef, const double *__restrict__ k0v,
                                               double h, int nx, int ny, const float2 *__restrict__ sc,
                                               float2 *__restrict__ dinv, long long wl_stride) {
    const int b = t.b, nb = t.nb, tid = threadIdx.x;
    const int P = b / 2;
    const long long blk = bt_sym_block(b);
    // centre stretches along the block (s_in, per row r) and across blocks (s_out, per block k)
    const float2 *scw = sc + (long long)wl * (nx + ny);
    const float2 *s_in = t.tr ? scw + nx + t.y0 : scw + t.x0;
    const float2 *s_out = t.tr ? scw + t.x0 : scw + nx + t.y0;
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
                if (tid == 0) { *pivrow = bi; piv[col] = bi; }
            }
            __syncthreads();
            const int p = *pivrow;
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
        // store the upper triangle of M_k = D_k^-1 S_k^-1 (symmetric), 2 x 2 sub-blocks
        float2 *dk = outw + (long long)k * blk;
        const float2 so = s_out[k];
        const int nsub = (int)(blk >> 2);
        for (int e = tid; e < (int)blk; e += BT_FACT_THREADS) {
            // e: half (first / second columns), sub-block, row within the pair
            const int half = e >= 2 * nsub, sub = (e - half * 2 * nsub) >> 1, comp = (e & 1) | (half << 1);
            int bp, bq;
            bt_sym_pq(P, sub, bp, bq);
            const int r = 2 * bp + (comp & 1), c = 2 * bq + (comp >> 1);
            const float2 si = s_in[c];
            const double2 sk = make_double2((double)si.x * so.x - (double)si.y * so.y,
                                            (double)si.x * so.y + (double)si.y * so.x);
            const double2 v = zdiv(M[r * b + c], sk);
            dk[e] = make_float2((float)v.x, (float)v.y);
        }
        __syncthreads();
    }
}

// Tiles whose short side fits the LDS matrix (others return at once).
__global__ __launch_bounds__(BT_FACT_THREADS) void bt_factor_lds_kernel(const TileDesc *__restrict__ tiles,
                                                                        const float *__restrict__ eps,
                                                                        const double2 *__restrict__ coef,
                                                                        const double *__restrict__ k0v, double h,
                                                                        int nx, int ny, const float2 *__restrict__ sc,
                                                                        float2 *__restrict__ dinv,
                                                                        long long wl_stride) {
    __shared__ double2 M[BT_FACT_LDS_B * BT_FACT_LDS_B];
    __shared__ double2 fcol[BT_FACT_LDS_B], prow[BT_FACT_LDS_B];
    __shared__ int piv[BT_FACT_LDS_B];
    __shared__ int pivrow;
    const TileDesc t = tiles[blockIdx.x];
    if (t.b > BT_FACT_LDS_B) return;
    bt_factor_body<BT_FACT_LDS_B>(M, fcol, prow, piv, &pivrow, t, blockIdx.y, eps, coef, k0v, h, nx, ny, sc, dinv,
                                  wl_stride);
}

// Tiles listed in `big` (short side above the LDS limit): the working matrix
// lives in scratch[(blockIdx.y * n_big + blockIdx.x) * BT_FACT_MAX_B^2].
__global__ __launch_bounds__(BT_FACT_THREADS) void bt_factor_global_kernel(const TileDesc *__restrict__ tiles,
                                                                           const int *__restrict__ big, int n_big,
                                                                           const float *__restrict__ eps,
                                                                           const double2 *__restrict__ coef,
                                                                           const double *__restrict__ k0v, double h,
                                                                           int nx, int ny,
                                                                           const float2 *__restrict__ sc,
                                                                           float2 *__restrict__ dinv,
                                                                           long long wl_stride,
                                                                           double2 *__restrict__ scratch) {
    __shared__ double2 fcol[BT_FACT_MAX_B], prow[BT_FACT_MAX_B];
    __shared__ int piv[BT_FACT_MAX_B];
    __shared__ int pivrow;
    const TileDesc t = tiles[big[blockIdx.x]];
    double2 *M = scratch + ((long long)blockIdx.y * n_big + blockIdx.x) * BT_FACT_MAX_B * BT_FACT_MAX_B;
    bt_factor_body<BT_FACT_MAX_B>(M, fcol, prow, piv, &pivrow, t, blockIdx.y, eps, coef, k0v, h, nx, ny, sc, dinv,
                                  wl_stride);
}

void launch_bt_factor(hipStream_t s, const TileDesc *tiles, int n_tiles, int n_wl, const float *eps,
                      const double *coef_d, const double *k0, double h, int nx, int ny, const float2 *sc,
                      float2 *dinv, long long dinv_wl_stride, const int *big, int n_big, double2 *scratch) {
    hipLaunchKernelGGL(bt_factor_lds_kernel, dim3(n_tiles, n_wl), dim3(BT_FACT_THREADS), 0, s, tiles, eps,
                       (const double2 *)coef_d, k0, h, nx, ny, sc, dinv, dinv_wl_stride);
    if (n_big > 0)
        hipLaunchKernelGGL(bt_factor_global_kernel, dim3(n_big, n_wl), dim3(BT_FACT_THREADS), 0, s, tiles, big,
                           n_big, eps, (const double2 *)coef_d, k0, h, nx, ny, sc, dinv, dinv_wl_stride, scratch);
}

// ------------------------------------------------------------------ solve
// Thread layout per (subdomain, RHS) workgroup: lane group rp (8 lanes) owns
// rows 2rp, 2rp+1 of every block; lane cg of the group takes the column pairs
// q = (rp + d) mod P for the offsets d = cg + 8 j.  For each it takes one 2 x 2
// sub-block of M_k (two float4), directly (q >= rp) or as the transpose of the
// stored sub-block (q, rp), so every off-diagonal sub-block is used by two
// groups in the same step.  Blocks up to 80 cells are copied once per step
// into LDS by the whole workgroup and the lanes read their sub-blocks there
// (staged form); wider blocks are loaded by each lane from global memory, a
// sub-block then coming once from HBM and once from cache.  For a fixed d the
// groups of a wave read consecutive entries of one storage row, so the loads
// coalesce.  The 8 lanes' partial sums are combined with three DPP
// steps and lanes 0 and 1 of the group run the recurrence for rows 2rp and
// 2rp + 1.  A workgroup of more than four waves puts two waves on one SIMD;
// when its last wave would be at most half full (P mod 8 <= 4), that wave
// takes its row pairs with 16 lanes each (offsets d = cg + 16 j, one more
// DPP step), so that the SIMD it shares carries fewer offset slots.
//
// Only the M stream touches HBM inside the recurrence: the subdomain RHS is
// gathered into LDS up front (block-major, [k][r]), w_k overwrites v_k in
// place during the forward sweep and is read back by the backward sweep, and
// the inter-block couplings and the stretches sit in LDS too.  The operand
// vector (already multiplied by S_k) is double-buffered, so each block step
// ends with a single barrier; M blocks are prefetched NS - 1 steps ahead into
// a register ring.
constexpr int BT_BMAX = 128;
constexpr int BT_GROUP = 8;
// offset slots per lane of the 16-lane tail wave: ceil(P / 16) for the
// widest block of each offset-slot instance (80, 112 and 128 cells)
constexpr int bt_tail_nj(int nj) { return nj <= 5 ? 3 : 4; }

// Unconditional loads: lanes without a sub-block (offset d >= P, or no row
// pair) read a valid entry instead and their products are zeroed at use.
// Keeping every load unpredicated lets the compiler wait only for the oldest
// slot of the ring.
// The loads go through a buffer resource over the tile's factors: the
// per-lane offset stays in a 32-bit register and the block offset in a
// scalar register, so no address arithmetic runs per load.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t bt_rsrc(const void *base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
template <int NJ>
__device__ __forceinline__ void bt_load(float4 (&slot)[2 * NJ], __amdgpu_buffer_rsrc_t rs, unsigned blkoff,
                                        const unsigned (&off)[NJ], unsigned half) {
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        slot[2 * j] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, off[j], blkoff, 0));
        slot[2 * j + 1] =
            __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, off[j], blkoff + half, 0));
    }
}

// Cross-lane moves inside groups of 8 lanes (DPP): swap neighbours, swap
// pairs, mirror the half-row of 8 lanes.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
constexpr int DPP_QUAD_XOR1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int DPP_HALF_MIRROR = 0x141;    // row_half_mirror (lane i <-> 7 - i)

constexpr int DPP_ROW_MIRROR = 0x140;     // row_mirror (lane i <-> 15 - i)

// Sums of the two rows' partial products over the G = 8 or 16 lanes of a
// group, with two values per lane instead of four: each lane keeps one row
// and sends the other to its neighbour, then the kept sums are combined.
// Lanes 4..7 keep the opposite rows to lanes 0..3 so that the half-row mirror
// pairs equal rows; the pattern is symmetric under i <-> 7 - i, so with 16
// lanes the row mirror pairs equal rows too.  Lane 0 ends with row 2rp,
// lane 1 with row 2rp + 1.
template <int G>
__device__ __forceinline__ float2 pair_sum(float2 a0, float2 a1, bool keep1) {
    float2 keep = keep1 ? a1 : a0;
    const float2 send = keep1 ? a0 : a1;
    keep.x += dpp<DPP_QUAD_XOR1>(send.x);
    keep.y += dpp<DPP_QUAD_XOR1>(send.y);
    keep.x += dpp<DPP_QUAD_XOR2>(keep.x);
    keep.y += dpp<DPP_QUAD_XOR2>(keep.y);
    keep.x += dpp<DPP_HALF_MIRROR>(keep.x);
    keep.y += dpp<DPP_HALF_MIRROR>(keep.y);
    if (G == 16) {
        keep.x += dpp<DPP_ROW_MIRROR>(keep.x);
        keep.y += dpp<DPP_ROW_MIRROR>(keep.y);
    }
    return keep;
}

// One lane's share of M_k x: the sub-blocks of its offset slots (loaded in
// `slot`, used directly or transposed) times the operand pairs in LDS;
// returns the group's sums for rows 2rp (lane 0) and 2rp + 1 (lane 1).
template <int NJ, int G>
__device__ __forceinline__ float2 bt_matvec(const float4 (&slot)[2 * NJ], const float2 *__restrict__ ysrc,
                                            const int (&qj)[NJ], unsigned direct_mask, bool keep1) {
    // even and odd slots accumulate separately: half the dependent chain length
    float2 a0[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
    float2 a1[2] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        // unused slots hold a clamped load of sub-block 0 and multiply the zero pair
        const float4 x = *reinterpret_cast<const float4 *>(ysrc + 2 * qj[j]);
        const float2 x0 = make_float2(x.x, x.y), x1 = make_float2(x.z, x.w);
        const float2 A = make_float2(slot[2 * j].x, slot[2 * j].y);           // M[2p'][2q']
        const float2 B = make_float2(slot[2 * j].z, slot[2 * j].w);           // M[2p'+1][2q']
        const float2 C = make_float2(slot[2 * j + 1].x, slot[2 * j + 1].y);   // M[2p'][2q'+1]
        const float2 Dd = make_float2(slot[2 * j + 1].z, slot[2 * j + 1].w);  // M[2p'+1][2q'+1]
        const bool dir = (direct_mask >> j) & 1;
        const float2 E = dir ? C : B, F = dir ? B : C;
        a0[j & 1] = cfma(a0[j & 1], A, x0);
        a0[j & 1] = cfma(a0[j & 1], E, x1);
        a1[j & 1] = cfma(a1[j & 1], F, x0);
        a1[j & 1] = cfma(a1[j & 1], Dd, x1);
    }
    return pair_sum<G>(make_float2(a0[0].x + a0[1].x, a0[0].y + a0[1].y),
                       make_float2(a1[0].x + a1[1].x, a1[0].y + a1[1].y), keep1);
}

// The recurrence of one wave: G lanes per row pair, NJ offset slots per lane,
// the factor blocks prefetched NS - 1 steps ahead.  Every wave of the
// workgroup runs the same steps and barriers; only the lane mapping differs.
// U = 0: each lane loads its own sub-blocks into a register ring (every
// off-diagonal sub-block is then fetched by two groups).  U > 0: the
// workgroup copies each block once, U 16-byte chunks per thread, through a
// register ring into one of two LDS stages behind vl, and the lanes read
// their sub-blocks from there (half the vector-memory instructions).
template <int NJ, int NS, int G, int U>
__device__ __forceinline__ void bt_run(const TileDesc &t, int rp, int cg, int tid, const float2 *__restrict__ D,
                                       long long bbytes, int nx, bool local_out, float2 *__restrict__ orr,
                                       float2 *__restrict__ vl, float2 (*ysh)[BT_BMAX + 2],
                                       const float2 *__restrict__ cl_s, const float2 *__restrict__ ch_s,
                                       const float2 *__restrict__ so_s, const float2 *__restrict__ si_s) {
    const int b = t.b, nb = t.nb, P = b >> 1;
    const int lx = t.x1 - t.x0;
    const bool on = rp < P;
    const int nsteps = 2 * nb - 1;
    auto blk = [&](int s) { return s < nb ? s : 2 * nb - 2 - s; };
    // per offset: storage entry (byte offset within a block), transposed flag, operand pair
    unsigned off[NJ];
    int qj[NJ];
    unsigned direct_mask = 0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int d = cg + G * j;
        const bool valid = on && d < P;          // blocks narrower than the widest tile leave slots unused
        bool direct = true;
        const int sub = valid ? bt_sym_index(P, rp, d, direct) : 0;
        off[j] = (unsigned)sub * 16u;
        qj[j] = valid ? (rp + d) % P : BT_BMAX / 2;
        if (direct) direct_mask |= 1u << j;
    }
    const __amdgpu_buffer_rsrc_t rs = bt_rsrc(D, (unsigned)(nb * bbytes));
    const unsigned half = (unsigned)(bbytes >> 1);         // second columns of the sub-blocks
    constexpr int RW = U > 0 ? U : 2 * NJ;                 // ring entries per thread and block
    float4 ring[NS][RW];
    // staged form: chunk tid + u * nthr of the block (clamped: surplus threads
    // re-read the last chunk and store nothing)
    const int nthr = blockDim.x, nchunk = (int)(bbytes >> 4), SZ = (nchunk + 63) & ~63;
    float4 *stg = reinterpret_cast<float4 *>(vl + nb * b);
    unsigned coff[U > 0 ? U : 1];
#pragma unroll
    for (int u = 0; u < (U > 0 ? U : 1); ++u) coff[u] = (unsigned)min(tid + u * nthr, nchunk - 1) * 16u;
    auto load = [&](float4 (&rr)[RW], int s) {
        const unsigned bo = (unsigned)(blk(min(s, nsteps - 1)) * bbytes);
        if constexpr (U > 0) {
#pragma unroll
            for (int u = 0; u < U; ++u)
                rr[u] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, coff[u], bo, 0));
        } else {
            bt_load<NJ>(rr, rs, bo, off, half);
        }
    };
    auto stage = [&](const float4 (&rr)[RW], int st) {
        if constexpr (U > 0) {
            float4 *dst = stg + st * SZ;
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (tid + u * nthr < nchunk) dst[tid + u * nthr] = rr[u];
        }
    };
#pragma unroll
    for (int i = 0; i < NS - 1; ++i) load(ring[i], i);

    // lanes 0 and 1 of each group carry the recurrence for rows 2rp and 2rp + 1
    const int myr = 2 * rp + (cg & 1);
    const bool wr = on && cg < 2;
    // output index of row myr in block k: obase + k * kstride; the block index
    // range [kc0, kc1) and okr select the core rows (all rows for local output)
    long long obase;
    int kstride, kc0, kc1;
    bool okr;
    if (local_out) {
        obase = t.tr ? (long long)myr * lx : myr;
        kstride = t.tr ? 1 : lx;
        kc0 = 0;
        kc1 = nb;
        okr = true;
    } else if (t.tr) {
        obase = (long long)(t.y0 + myr) * nx + t.x0;
        kstride = 1;
        kc0 = t.cx0 - t.x0;
        kc1 = t.cx1 - t.x0;
        okr = t.y0 + myr >= t.cy0 && t.y0 + myr < t.cy1;
    } else {
        obase = (long long)t.y0 * nx + t.x0 + myr;
        kstride = nx;
        kc0 = t.cy0 - t.y0;
        kc1 = t.cy1 - t.y0;
        okr = t.x0 + myr >= t.cx0 && t.x0 + myr < t.cx1;
    }
    const bool emit_lane = wr && okr;
    stage(ring[0], 0);
    __syncthreads();
    const float2 si = wr ? si_s[myr] : make_float2(0.f, 0.f);
    if (wr) ysh[0][myr] = cmul(cmul(si, so_s[0]), vl[myr]);      // S_0 v_0
    if (tid < 4) ysh[tid >> 1][BT_BMAX + (tid & 1)] = make_float2(0.f, 0.f);
    __syncthreads();

    const bool keep1 = (((cg & 7) ^ ((cg & 7) >> 2)) & 1) != 0;
    auto step = [&](int s, const float4(&regs)[RW]) {
        float4 slot[2 * NJ];
        if constexpr (U > 0) {
            const float4 *sb = stg + (s & 1) * SZ;
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                slot[2 * j] = sb[off[j] >> 4];
                slot[2 * j + 1] = sb[(off[j] + half) >> 4];
            }
        } else {
#pragma unroll
            for (int q = 0; q < 2 * NJ; ++q) slot[q] = regs[q];
        }
        const int k = blk(s);
        const int p = s & 1;
        const bool fwd = s < nb;
        const bool turn = s == nb - 1;                // u_{nb-1} = w_{nb-1}
        const int knext = fwd && !turn ? k + 1 : k - 1;
        // everything the recurrence needs besides the product, read first:
        // v_{k+1} (forward) or w_k (backward), the coupling, S_knext
        float2 pre = make_float2(0.f, 0.f), cc = make_float2(0.f, 0.f), skn = make_float2(0.f, 0.f);
        if (wr) {
            pre = vl[min(fwd ? k + 1 : k, nb - 1) * b + myr];
            cc = fwd ? cl_s[min(k + 1, nb - 1)] : ch_s[k];
            skn = cmul(si, so_s[max(knext, 0)]);
        }
        const float2 a = bt_matvec<NJ, G>(slot, ysh[p], qj, direct_mask, keep1);
        if (wr) {
            if (fwd) vl[k * b + myr] = a;                                   // w_k
            const float2 y = turn ? a : cfms(pre, cc, a);                   // y_{k+1} or u_k
            if ((!fwd || turn) && emit_lane && k >= kc0 && k < kc1) orr[obase + (long long)k * kstride] = y;
            ysh[p ^ 1][myr] = knext >= 0 ? cmul(skn, y) : y;                // operand of the next step
        }
        __syncthreads();
    };

    // steady state: step s refills the ring entry of step s - 1 with the block
    // of step s + NS - 1 (clamped at the end: a re-read); the register form
    // then uses ring[s % NS], the staged form first stores block s + 1 (loaded
    // NS - 2 steps ago) into LDS stage (s + 1) & 1 and reads block s from stage
    // s & 1, the step's closing barrier publishing the new stage
    int s0 = 0;
    for (; s0 + NS <= nsteps; s0 += NS) {
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            load(ring[(i + NS - 1) % NS], s0 + i + NS - 1);
            stage(ring[(i + 1) % NS], (s0 + i + 1) & 1);
            step(s0 + i, ring[i]);
        }
    }
    // tail: fewer than NS steps left, their blocks are already in the ring
#pragma unroll
    for (int i = 0; i < NS - 1; ++i)
        if (s0 + i < nsteps) {
            stage(ring[(i + 1) % NS], (s0 + i + 1) & 1);
            step(s0 + i, ring[i]);
        }
}

template <int NJ, int NS, int NJT, int U>
__global__ __launch_bounds__(512) void bt_solve_kernel(const TileDesc *__restrict__ tiles, int n_src,
                                                       const float2 *__restrict__ dinv, long long dinv_wl_stride,
                                                       const float2 *__restrict__ coef,
                                                       const float2 *__restrict__ sc, int nx, int ny,
                                                       const float2 *__restrict__ vin, long long vin_stride,
                                                       float2 *__restrict__ out, long long out_stride,
                                                       const int *__restrict__ active, int mode,
                                                       const int2 *__restrict__ order) {
    extern __shared__ float2 vl[];                    // [nb][b]: v_k, then w_k
    __shared__ __align__(16) float2 ysh[2][BT_BMAX + 2];   // + a zero pair read by unused offset slots
    __shared__ float2 cl_s[BT_NBMAX], ch_s[BT_NBMAX], so_s[BT_NBMAX], si_s[BT_BMAX];
    const int2 job = order[blockIdx.x];               // (tile, rhs); tile < 0 pads the queue
    const int tile = job.x, rhs = job.y;
    if (tile < 0 || (active && !active[rhs])) return;
    const int wl = rhs / n_src;
    const TileDesc t = tiles[tile];
    const int b = t.b, nb = t.nb, P = b >> 1;
    const int tid = threadIdx.x;
    const float2 *D = dinv + wl * dinv_wl_stride + t.dinv_off;
    const long long bbytes = bt_sym_block(b) * (long long)sizeof(float2);
    const int lx = t.x1 - t.x0, ly = t.y1 - t.y0;
    const float2 *cf = coef + wl * coef_stride(nx, ny);
    const float2 *clo_a = t.tr ? cf : cf + 2 * nx;               // cxm or cym
    const float2 *chi_a = t.tr ? cf + nx : cf + 2 * nx + ny;      // cxp or cyp
    const float2 *scw = sc + (long long)wl * (nx + ny);
    const float2 *s_in = t.tr ? scw + nx + t.y0 : scw + t.x0;     // along the block
    const float2 *s_out = t.tr ? scw + t.x0 : scw + nx + t.y0;    // across blocks
    const int base = t.tr ? t.x0 : t.y0;
    const bool local_in = mode & 1, local_out = mode & 2;
    const float2 *vr = vin + rhs * vin_stride + (local_in ? t.loc_off : 0);
    float2 *orr = out + rhs * out_stride + (local_out ? t.loc_off : 0);

    // gather R_i v (row-major over the tile, coalesced) into block-major LDS
    for (int e = tid; e < lx * ly; e += blockDim.x) {
        const int yy = e / lx, xx = e - yy * lx;
        const float2 val = local_in ? vr[e] : vr[(long long)(t.y0 + yy) * nx + (t.x0 + xx)];
        vl[t.tr ? xx * b + yy : e] = val;
    }
    for (int k = tid; k < nb; k += blockDim.x) {
        cl_s[k] = clo_a[base + k];
        ch_s[k] = chi_a[base + k];
        so_s[k] = s_out[k];
    }
    // the in-block scaling goes through LDS as well: a global load left in
    // flight past the prefetch below would make every step's first use of it
    // wait for the whole register ring
    for (int k = tid; k < b; k += blockDim.x) si_s[k] = s_in[k];
    // waves of 8-lane groups; when the last wave holds at most four row pairs
    // (it is then at most half full), it takes them with 16-lane groups
    // instead, so that it carries fewer offset slots per lane than the full
    // waves (the SIMD that runs it runs two waves)
    const int full = P >> 3, rest = P & 7;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (NJT > 0 && rest > 0 && rest <= 4 && wave == full) {
        const int l = tid - 64 * full;
        bt_run<(NJT > 0 ? NJT : 1), NS, 16, U>(t, 8 * full + (l >> 4), l & 15, tid, D, bbytes, nx, local_out, orr, vl,
                                          ysh, cl_s, ch_s, so_s, si_s);
    } else {
        bt_run<NJ, NS, 8, U>(t, tid >> 3, tid & 7, tid, D, bbytes, nx, local_out, orr, vl, ysh, cl_s, ch_s, so_s, si_s);
    }
}

template <int NJ, int NS, int U>
static void bt_solve_launch(hipStream_t s, dim3 grid, int threads, size_t lds, const TileDesc *tiles, int n_src,
                            const float2 *dinv, long long dinv_wl_stride, const float2 *coef, const float2 *sc,
                            int nx, int ny, const float2 *vin, long long vin_stride, float2 *out,
                            long long out_stride, const int *active, int mode, const int2 *order) {
    hipLaunchKernelGGL((bt_solve_kernel<NJ, NS, bt_tail_nj(NJ), U>), grid, dim3(threads), lds, s, tiles, n_src, dinv,
                       dinv_wl_stride, coef, sc, nx, ny, vin, vin_stride, out, out_stride, active, mode, order);
}

static int bt_nj(int bmax) { return ((bmax / 2) + BT_GROUP - 1) / BT_GROUP; }
static int bt_threads(int bmax) { return ((bmax / 2) * BT_GROUP + 63) / 64 * 64; }

// Dynamic LDS of the solve: the gathered subdomain (max_cells complex values)
// and, in the staged form, two stages of the widest block's 16-byte chunks.
static size_t bt_lds_bytes(int bmax, int max_cells, bool staged) {
    size_t l = (size_t)max_cells * sizeof(float2);
    if (staged) l += 2 * (size_t)(((bmax * (bmax + 2) / 4) + 63) & ~63) * 16;
    return l;
}
constexpr size_t BT_DYN_LDS_MAX = 150 * 1024;     // 160 KB per CU, less the static arrays

// Chunks per thread of the staged form (4, 5 or 6), or 0 for the register
// form: blocks up to 80 cells whose two stages fit in LDS beside the subdomain.
static int bt_stage_u(int bmax, int max_cells) {
    if (bt_nj(bmax) > 5) return 0;
    const int nthr = bt_threads(bmax);
    const int u = (bmax * (bmax + 2) / 4 + nthr - 1) / nthr;
    if (u > 6 || bt_lds_bytes(bmax, max_cells, true) > BT_DYN_LDS_MAX) return 0;
    return u < 4 ? 4 : u;
}

// Kernels that need more than 64 KB of dynamic LDS must say so once per
// process, before any launch (and outside graph capture).
void bt_solve_prepare(int bmax, int max_cells) {
    const int u = bt_stage_u(bmax, max_cells);
    const size_t lds = bt_lds_bytes(bmax, max_cells, u > 0);
    if (lds <= 65536) return;
    const int nj = bt_nj(bmax);
    const void *fs[3];
    int nf = 0;
    if (u == 4) {
        fs[nf++] = reinterpret_cast<const void *>(&bt_solve_kernel<5, 4, bt_tail_nj(5), 4>);
    } else if (u == 5) {
        fs[nf++] = reinterpret_cast<const void *>(&bt_solve_kernel<5, 4, bt_tail_nj(5), 5>);
    } else if (u == 6) {
        fs[nf++] = reinterpret_cast<const void *>(&bt_solve_kernel<5, 4, bt_tail_nj(5), 6>);
    } else if (nj <= 5) {
        fs[nf++] = reinterpret_cast<const void *>(&bt_solve_kernel<5, 3, bt_tail_nj(5), 0>);
        fs[nf++] = reinterpret_cast<const void *>(&bt_solve_kernel<5, 4, bt_tail_nj(5), 0>);
        fs[nf++] = reinterpret_cast<const void *>(&bt_solve_kernel<5, 5, bt_tail_nj(5), 0>);
    } else if (nj <= 7) {
        fs[nf++] = reinterpret_cast<const void *>(&bt_solve_kernel<7, 3, bt_tail_nj(7), 0>);
    } else {
        fs[nf++] = reinterpret_cast<const void *>(&bt_solve_kernel<8, 3, bt_tail_nj(8), 0>);
    }
    for (int i = 0; i < nf; ++i) (void)hipFuncSetAttribute(fs[i], hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

// Prefetch depths available for a block size (the register ring holds NS - 1
// blocks ahead); the first is the default.  The staged form always runs depth 4.
int bt_solve_depths(int bmax, int *depths) {
    if (bt_nj(bmax) <= 5) {
        depths[0] = 4;
        depths[1] = 3;
        depths[2] = 5;
        return 3;
    }
    depths[0] = 3;
    return 1;
}

void launch_bt_solve(hipStream_t s, const TileDesc *tiles, const int2 *order, int n_jobs, int n_src,
                     const float2 *dinv, long long dinv_wl_stride, const float2 *coef, const float2 *sc, int nx,
                     int ny, const float2 *vin, long long vin_stride, float2 *out, long long out_stride,
                     const int *active, int mode, int bmax, int max_cells, int depth) {
    dim3 grid(n_jobs);
    const int threads = bt_threads(bmax);
    const int nj = bt_nj(bmax);
    const int u = bt_stage_u(bmax, max_cells);
    const size_t lds = bt_lds_bytes(bmax, max_cells, u > 0);
#define BT_ARGS s, grid, threads, lds, tiles, n_src, dinv, dinv_wl_stride, coef, sc, nx, ny, vin, vin_stride, out, \
                out_stride, active, mode, order
    if (u == 4) {
        bt_solve_launch<5, 4, 4>(BT_ARGS);
    } else if (u == 5) {
        bt_solve_launch<5, 4, 5>(BT_ARGS);
    } else if (u == 6) {
        bt_solve_launch<5, 4, 6>(BT_ARGS);
    } else if (nj <= 5) {
        if (depth == 3)
            bt_solve_launch<5, 3, 0>(BT_ARGS);
        else if (depth == 5)
            bt_solve_launch<5, 5, 0>(BT_ARGS);
        else
            bt_solve_launch<5, 4, 0>(BT_ARGS);
    } else if (nj <= 7) {
        bt_solve_launch<7, 3, 0>(BT_ARGS);
    } else {
        bt_solve_launch<8, 3, 0>(BT_ARGS);
    }
#undef BT_ARGS
}

// ----------------------------------------------------------- many sources
// Sources that share a wavelength share every factor block, so a workgroup
// takes one (subdomain, wavelength) and a group of sources: each block M_k is
// read from HBM once, expanded in LDS into its real and imaginary b x b parts
// (both triangles), and the step's products for all sources, M_k (S_k Y) with
// Y the b x NCOL operand, run as FP32 MFMA contractions (16 x 16 x 4):
//   Re = M_r Y_r + M_i (-Y_i),  Im = M_r Y_i + M_i Y_r.
// The recurrence then runs elementwise over (row, source): the forward sweep
// reads each block of the right-hand sides straight from the global vector
// (the gather R_i v), keeps w_k block-major in a packed workspace
// (loc[rhs][tile cells]) for the backward sweep, and the backward sweep
// writes the core cells of u_k straight to the global output (the RAS scatter).
// The group width follows the tile: 32 sources for blocks up to 80 cells,
// 16 above (LDS), so one launch serves mixed tile sizes and the common
// 72-wide tiles stream each factor block once per wavelength.
// Every global load of the step loop is unpredicated (clamped addresses), so
// the compiler counts them exactly: factor blocks are fetched two steps ahead
// into a two-slot register ring and the recurrence operands one step ahead,
// and a step waits only for the loads it consumes.
typedef float f32x4v __attribute__((ext_vector_type(4)));
constexpr int BM_THREADS = 1024;
typedef unsigned bm_u32x2 __attribute__((ext_vector_type(2)));
constexpr int BM_NARROW = 80;                  // widest block of the 32-source form

// LDS layout (b the tile's block size, padded to BP = 16 * ceil(b / 16) in rows and in k):
//   M  [BP][BP + 2] float2 (re, im): the expanded block, row-major, k contiguous;
//   X  3 x [NCOL][BP + 4] float: Re, Im and -Im of the operand S_k Y, source-major, k contiguous;
//   C  2 x [BP][NCOL + 1] float: Re and Im of the products.
// The MFMA lane groups (lane / 16) take contiguous quarters of k, so each lane
// reads four k at once (16-byte LDS loads) for four consecutive MFMAs.
__host__ __device__ __forceinline__ int bm_pad(int b) { return (b + 15) & ~15; }
__host__ __device__ __forceinline__ int bm_cols(int b) { return b <= BM_NARROW ? 32 : 16; }
int bt_multi_cols(int b) { return bm_cols(b); }
static size_t bm_lds_class(int b, int ncol) {
    const int BP = bm_pad(b);
    return sizeof(float) * ((size_t)2 * BP * (BP + 2) + (size_t)3 * ncol * (BP + 4) + (size_t)2 * BP * (ncol + 1));
}
// dynamic LDS of a launch whose widest block is bmax (either group form may run)
static size_t bm_lds_bytes(int bmax);

template <int NCOL, int EMAX, int RMAX>
__device__ __forceinline__ void bm_solve(const TileDesc &t, int wl, int s0, int ns, int n_src,
                                         const float2 *__restrict__ dinv, long long dinv_wl_stride,
                                         const float2 *__restrict__ coef, const float2 *__restrict__ sc, int nx, int ny,
                                         const float2 *__restrict__ vin, long long vin_stride, float2 *__restrict__ out,
                                         long long out_stride, const int *__restrict__ active, float2 *__restrict__ loc,
                                         long long LT, float *lds, float2 *cl_s, float2 *ch_s, float2 *so_s,
                                         float2 *si_s, int *colr) {
    const int b = t.b, nb = t.nb, P = b >> 1, tid = threadIdx.x;
    const int BP = bm_pad(b), LDM = BP + 2, LDK = BP + 4, LDC = NCOL + 1;
    float2 *M = reinterpret_cast<float2 *>(lds);
    float *Xr = lds + 2 * BP * LDM, *Xi = Xr + NCOL * LDK, *Xn = Xi + NCOL * LDK;
    float *Cr = Xn + NCOL * LDK, *Ci = Cr + BP * LDC;
    const int rfirst = wl * n_src + s0;               // a valid right-hand side of this job (clamped loads)
    if (tid < NCOL) {
        const int r = rfirst + tid;
        colr[tid] = (tid < ns && (!active || active[r])) ? r : -1;
    }
    
    const float2 *cf = coef + wl * coef_stride(nx, ny);
    const float2 *clo_a = t.tr ? cf : cf + 2 * nx;
    const float2 *chi_a = t.tr ? cf + nx : cf + 2 * nx + ny;
    const float2 *scw = sc + (long long)wl * (nx + ny);
    const float2 *s_in = t.tr ? scw + nx + t.y0 : scw + t.x0;
    const float2 *s_out = t.tr ? scw + t.x0 : scw + nx + t.y0;
    const int base = t.tr ? t.x0 : t.y0;
    for (int k = tid; k < nb; k += BM_THREADS) {
        cl_s[k] = clo_a[base + k];
        ch_s[k] = chi_a[base + k];
        so_s[k] = s_out[k];
    }
    for (int i = tid; i < b; i += BM_THREADS) si_s[i] = s_in[i];
    // zero the padding of the MFMA operands once (rows and k >= b)
    for (int e = tid; e < BP * LDM; e += BM_THREADS) M[e] = make_float2(0.f, 0.f);
    for (int e = tid; e < 3 * NCOL * LDK; e += BM_THREADS) Xr[e] = 0.f;
    __syncthreads();
    // this thread's elements of a packed block: a clamped (always valid) load
    // index and the two LDS positions of the element, packed in 16 bits each
    // (0xffff: nothing to store).  The per-thread state of this kernel is kept
    // compact on purpose: at 1024 threads a wave has 128 registers, and a
    // spill reloaded inside the step loop would make the compiler wait for
    // every outstanding load there (vmcnt(0)), prefetched factor blocks included.
    const long long blk = bt_sym_block(b);
    const int nsub = (int)(blk >> 2);
    const float2 *D = dinv + wl * dinv_wl_stride + t.dinv_off;
    // every global access goes through a buffer resource: the per-lane byte
    // offset stays in one 32-bit register and the block step's offset in a
    // scalar one, so no 64-bit address is formed per access (the host keeps
    // each range below 2^31 bytes)
    const __amdgpu_buffer_rsrc_t rsD = bt_rsrc(D, (unsigned)(nb * blk * (long long)sizeof(float2)));
    const __amdgpu_buffer_rsrc_t rsV =
        bt_rsrc(vin + (long long)rfirst * vin_stride, (unsigned)((long long)ns * vin_stride * sizeof(float2)));
    const __amdgpu_buffer_rsrc_t rsL =
        bt_rsrc(loc + (long long)rfirst * LT, (unsigned)((long long)ns * LT * sizeof(float2)));
    const __amdgpu_buffer_rsrc_t rsO =
        bt_rsrc(out + (long long)rfirst * out_stride, (unsigned)((long long)ns * out_stride * sizeof(float2)));
    auto ld = [](__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
        return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0));
    };
    auto st = [](__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, float2 v) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bm_u32x2, v), rs, (int)voff, (int)soff, 0);
    };
    unsigned gi[EMAX];
    unsigned opos[EMAX];
#pragma unroll
    for (int j = 0; j < EMAX; ++j) {
        const int e = tid + j * BM_THREADS;
        gi[j] = (unsigned)(e < (int)blk ? e : (int)blk - 1) * (unsigned)sizeof(float2);
        opos[j] = 0xffffffffu;
        if (e < (int)blk) {
            const int half = e >= 2 * nsub, sub = (e - half * 2 * nsub) >> 1, comp = (e & 1) | (half << 1);
            int bp, bq;
            bt_sym_pq(P, sub, bp, bq);
            const int rr = 2 * bp + (comp & 1), cc = 2 * bq + (comp >> 1);
            opos[j] = (unsigned)(rr * LDM + cc) | ((unsigned)(cc * LDM + rr) << 16);
        }
    }
    // this thread's (row, source) elements of the recurrence, fixed for all
    // steps: row and column packed (-1 when idle), and the byte offsets of
    // their workspace row and of their cells in the global input and output,
    // relative to the group's first source (clamped to it when idle).  Cell
    // (block k, row i) is (x0 + i, y0 + k) for row blocks and (x0 + k, y0 + i)
    // for column blocks.
    int rcx[RMAX];
    unsigned poff[RMAX], voff[RMAX], ooff[RMAX];
    const unsigned kstep = (t.tr ? 1u : (unsigned)nx) * (unsigned)sizeof(float2);   // bytes per block step
#pragma unroll
    for (int j = 0; j < RMAX; ++j) {
        const int e = tid + j * BM_THREADS;
        const bool valid = e < b * NCOL;
        const int i = valid ? e % b : 0, c = valid ? e / b : 0;
        rcx[j] = valid ? (i | (c << 16)) : -1;
        const int r = colr[c], rl = r >= 0 ? r - rfirst : 0;
        const long long cell0 = t.tr ? (long long)(t.y0 + i) * nx + t.x0 : (long long)t.y0 * nx + t.x0 + i;
        poff[j] = (unsigned)(((long long)rl * LT + t.loc_off + i) * (long long)sizeof(float2));
        voff[j] = (unsigned)(((long long)rl * vin_stride + cell0) * (long long)sizeof(float2));
        ooff[j] = (unsigned)(((long long)rl * out_stride + cell0) * (long long)sizeof(float2));
    }
    const unsigned bstep = (unsigned)b * (unsigned)sizeof(float2);                   // workspace bytes per block
    // core rows of the block direction and core range of the in-block index
    const int kc0 = t.tr ? t.cx0 - t.x0 : t.cy0 - t.y0, kc1 = t.tr ? t.cx1 - t.x0 : t.cy1 - t.y0;
    const int ic0 = t.tr ? t.cy0 - t.y0 : t.cx0 - t.x0, ic1 = t.tr ? t.cy1 - t.y0 : t.cx1 - t.x0;
    const int nsteps = 2 * nb - 1;
    auto blk_of = [&](int s) { return s < nb ? s : 2 * nb - 2 - s; };
    auto fetch = [&](int s, float2(&dst)[EMAX]) {
        const unsigned bo = (unsigned)(blk_of(s < nsteps ? s : nsteps - 1) * blk * (long long)sizeof(float2));
#pragma unroll
        for (int j = 0; j < EMAX; ++j) dst[j] = ld(rsD, gi[j], bo);
    };
    auto expand = [&](const float2(&src)[EMAX]) {
#pragma unroll
        for (int j = 0; j < EMAX; ++j)
            if (opos[j] != 0xffffffffu) {
                M[opos[j] & 0xffffu] = src[j];
                M[opos[j] >> 16] = src[j];
            }
    };
    // v_{k+1} from the global input (forward) or w_k from the workspace (backward) for step s
    auto load_pre = [&](int s, float2(&dst)[RMAX]) {
        const int sc_ = s < nsteps ? s : nsteps - 1;
        const int k = blk_of(sc_);
        if (sc_ < nb) {
            const int kk = k + 1 < nb ? k + 1 : nb - 1;
#pragma unroll
            for (int j = 0; j < RMAX; ++j) dst[j] = ld(rsV, voff[j], (unsigned)kk * kstep);
        } else {
#pragma unroll
            for (int j = 0; j < RMAX; ++j) dst[j] = ld(rsL, poff[j], (unsigned)k * bstep);
        }
    };
    float2 ra[EMAX], rb[EMAX], pre_c[RMAX], pre_n[RMAX];
    fetch(0, ra);
    fetch(1, rb);
    load_pre(0, pre_c);
    // operand of the first step: S_0 v_0
    for (int e = tid; e < b * NCOL; e += BM_THREADS) {
        const int i = e % b, c = e / b, r = colr[c];
        float2 z = make_float2(0.f, 0.f);
        if (r >= 0)
            z = cmul(cmul(si_s[i], so_s[0]),
                     vin[(long long)r * vin_stride + (t.tr ? (long long)(t.y0 + i) * nx + t.x0 : (long long)t.y0 * nx + t.x0 + i)]);
        Xr[c * LDK + i] = z.x;
        Xi[c * LDK + i] = z.y;
        Xn[c * LDK + i] = -z.y;
    }
    expand(ra);
    const int wave = tid >> 6, lane = tid & 63;
    const int RT = BP / 16, nT = RT * (NCOL / 16), KQ = BP / 4;
    // one block step: block s is expanded in M (it came from cur), block s + 1 waits in nxt
    auto step = [&](int s, float2(&cur)[EMAX], float2(&nxt)[EMAX]) {
        const int k = blk_of(s);
        const bool fwd = s < nb, turn = s == nb - 1;
        fetch(s + 2, cur);
        load_pre(s + 1, pre_n);
        __syncthreads();                              // M_k and the operand are in LDS
        for (int q = wave; q < nT; q += BM_THREADS / 64) {
            const int rt = q % RT, ct = q / RT;
            f32x4v accR = {0.f, 0.f, 0.f, 0.f}, accI = {0.f, 0.f, 0.f, 0.f};
            const int bcol = ct * 16 + (lane & 15), k0 = (lane >> 4) * KQ;
            const float2 *arow = M + (rt * 16 + (lane & 15)) * LDM + k0;
            const float *xr = Xr + bcol * LDK + k0, *xi = Xi + bcol * LDK + k0, *xn = Xn + bcol * LDK + k0;
            for (int kk = 0; kk < KQ; kk += 4) {
                const float4 a01 = *reinterpret_cast<const float4 *>(arow + kk);
                const float4 a23 = *reinterpret_cast<const float4 *>(arow + kk + 2);
                const float4 yr = *reinterpret_cast<const float4 *>(xr + kk);
                const float4 yi = *reinterpret_cast<const float4 *>(xi + kk);
                const float4 yn = *reinterpret_cast<const float4 *>(xn + kk);
                const float ar[4] = {a01.x, a01.z, a23.x, a23.z}, ai[4] = {a01.y, a01.w, a23.y, a23.w};
                const float vr[4] = {yr.x, yr.y, yr.z, yr.w}, vi[4] = {yi.x, yi.y, yi.z, yi.w};
                const float vn[4] = {yn.x, yn.y, yn.z, yn.w};
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    accR = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[u], vr[u], accR, 0, 0, 0);
                    accR = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[u], vn[u], accR, 0, 0, 0);
                    accI = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[u], vi[u], accI, 0, 0, 0);
                    accI = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[u], vr[u], accI, 0, 0, 0);
                }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = rt * 16 + 4 * (lane >> 4) + i;
                Cr[row * LDC + bcol] = accR[i];
                Ci[row * LDC + bcol] = accI[i];
            }
        }
        __syncthreads();                              // products in LDS; M_k and the operand consumed
        const int knext = fwd && !turn ? k + 1 : k - 1;
        const float2 cc = fwd ? cl_s[min(k + 1, nb - 1)] : ch_s[k];
#pragma unroll
        for (int j = 0; j < RMAX; ++j) {
            if (rcx[j] < 0) break;
            const int i = rcx[j] & 0xffff, c = rcx[j] >> 16, r = colr[c];
            float2 z = make_float2(0.f, 0.f);
            if (r >= 0) {
                const float2 a = make_float2(Cr[i * LDC + c], Ci[i * LDC + c]);
                float2 y;
                if (fwd) {
                    if (!turn) st(rsL, poff[j], (unsigned)k * bstep, a);           // w_k
                    y = turn ? a : cfms(pre_c[j], cc, a);                           // y_{k+1} or u_{nb-1}
                } else {
                    y = cfms(pre_c[j], cc, a);                                      // u_k
                }
                // u_k (and u_{nb-1} at the turn): core cells to the output
                if ((!fwd || turn) && k >= kc0 && k < kc1 && i >= ic0 && i < ic1)
                    st(rsO, ooff[j], (unsigned)k * kstep, y);
                if (knext >= 0) z = cmul(cmul(si_s[i], so_s[knext]), y);
            }
            Xr[c * LDK + i] = z.x;
            Xi[c * LDK + i] = z.y;
            Xn[c * LDK + i] = -z.y;
        }
#pragma unroll
        for (int j = 0; j < RMAX; ++j) pre_c[j] = pre_n[j];
        if (s + 1 < nsteps) expand(nxt);
    };
    for (int s = 0; s < nsteps; s += 2) {
        step(s, ra, rb);
        if (s + 1 < nsteps) step(s + 1, rb, ra);
    }
}

// The 32-source form (blocks up to 80 cells), synchronised per step through LDS
// counters instead of workgroup barriers (see the step below).
// M_k is complex symmetric, so the step's products are formed transposed,
// C^T = Y^T M_k (rows: sources, columns: block rows), and the wave that forms
// an output tile runs the recurrence of its 16 x 16 (source, row) elements
// straight from its accumulators: each lane holds 4 sources of one block row,
// so its global loads and stores are row-contiguous across lanes.  The waves
// without a tile meanwhile expand the next factor block into the second of
// two LDS buffers, and the operand of the next step goes to the second of two
// operand buffers, so a step needs no product buffer.
// Re C^T = Yr Mr - Yi Mi is accumulated as two sums (the operand is kept as
// Re and Im only), Im C^T = Yr Mi + Yi Mr as one.
constexpr int B32_EMAX = 9;                           // expand elements per lane: ceil(3280 / (6 * 64))
__host__ __device__ __forceinline__ size_t b32_lds_bytes(int b) {
    const int BP = bm_pad(b);
    return sizeof(float) * ((size_t)2 * 2 * BP * (BP + 2) + (size_t)2 * 2 * 32 * (BP + 4));
}
__device__ __forceinline__ void bm_solve32(const TileDesc &t, int wl, int s0, int ns, int n_src,
                                           const float2 *__restrict__ dinv, long long dinv_wl_stride,
                                           const float2 *__restrict__ coef, const float2 *__restrict__ sc, int nx,
                                           int ny, const float2 *__restrict__ vin, long long vin_stride,
                                           float2 *__restrict__ out, long long out_stride,
                                           const int *__restrict__ active, float2 *__restrict__ loc, long long LT,
                                           float *lds, float2 *cl_s, float2 *ch_s, float2 *so_s, float2 *si_s,
                                           int *colr, int *sync) {
    constexpr int NCOL = 32;
    const int b = t.b, nb = t.nb, P = b >> 1, tid = threadIdx.x;
    const int BP = bm_pad(b), LDM = BP + 2, LDK = BP + 4;
    // buffers are addressed arithmetically (an array of pointers indexed at run
    // time would live in scratch memory and lose the LDS address space)
    auto MB = [&](int buf) { return reinterpret_cast<float2 *>(lds) + buf * BP * LDM; };
    float *Xb = lds + 2 * 2 * BP * LDM;               // [buffer][Re, Im][NCOL][LDK]
    auto XR = [&](int buf) { return Xb + (2 * buf) * NCOL * LDK; };
    auto XI = [&](int buf) { return Xb + (2 * buf + 1) * NCOL * LDK; };
    const int rfirst = wl * n_src + s0;
    if (tid < NCOL) {
        const int r = rfirst + tid;
        colr[tid] = (tid < ns && (!active || active[r])) ? r : -1;
    }
    const float2 *cf = coef + wl * coef_stride(nx, ny);
    const float2 *clo_a = t.tr ? cf : cf + 2 * nx;
    const float2 *chi_a = t.tr ? cf + nx : cf + 2 * nx + ny;
    const float2 *scw = sc + (long long)wl * (nx + ny);
    const float2 *s_in = t.tr ? scw + nx + t.y0 : scw + t.x0;
    const float2 *s_out = t.tr ? scw + t.x0 : scw + nx + t.y0;
    const int base = t.tr ? t.x0 : t.y0;
    for (int k = tid; k < nb; k += BM_THREADS) {
        cl_s[k] = clo_a[base + k];
        ch_s[k] = chi_a[base + k];
        so_s[k] = s_out[k];
    }
    for (int i = tid; i < b; i += BM_THREADS) si_s[i] = s_in[i];
    // zero both factor buffers and both operand buffers (padding rows and k >= b stay zero)
    for (int e = tid; e < 2 * BP * LDM; e += BM_THREADS) MB(0)[e] = make_float2(0.f, 0.f);
    for (int e = tid; e < 2 * 2 * NCOL * LDK; e += BM_THREADS) Xb[e] = 0.f;
    if (tid < 5) sync[tid] = 0;
    __syncthreads();
    const long long blk = bt_sym_block(b);
    const int nsub = (int)(blk >> 2);
    const float2 *D = dinv + wl * dinv_wl_stride + t.dinv_off;
    const __amdgpu_buffer_rsrc_t rsD = bt_rsrc(D, (unsigned)(nb * blk * (long long)sizeof(float2)));
    const __amdgpu_buffer_rsrc_t rsV =
        bt_rsrc(vin + (long long)rfirst * vin_stride, (unsigned)((long long)ns * vin_stride * sizeof(float2)));
    const __amdgpu_buffer_rsrc_t rsL =
        bt_rsrc(loc + (long long)rfirst * LT, (unsigned)((long long)ns * LT * sizeof(float2)));
    const __amdgpu_buffer_rsrc_t rsO =
        bt_rsrc(out + (long long)rfirst * out_stride, (unsigned)((long long)ns * out_stride * sizeof(float2)));
    auto ld = [](__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff) {
        return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0));
    };
    auto st = [](__amdgpu_buffer_rsrc_t rs, unsigned voff, unsigned soff, float2 v) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(bm_u32x2, v), rs, (int)voff, (int)soff, 0);
    };
    const int wave = tid >> 6, lane = tid & 63;
    const int RT = BP / 16, nT = 2 * RT;                  // output tiles: 2 source tiles x RT row tiles
    const int KG = 2 * ((b + 7) >> 3);                    // k per MFMA lane group: 4 KG >= b, 4 KG <= BP
    const bool prod = wave < nT;                           // wave-uniform role
    const int nsteps = 2 * nb - 1;
    auto blk_of = [&](int s) { return s < nb ? s : 2 * nb - 2 - s; };
    // ---- expand waves: element e of the packed block goes to lane e mod (their
    // lane count); its two LDS positions (both triangles, 16 bits each) are
    // formed once, since the index arithmetic of every step would compete for
    // issue with the product waves on the same SIMDs; one register slot holds
    // the next block: it is expanded at the start of a step and refilled at once
    const int ne_lanes = (BM_THREADS / 64 - nT) * 64, el = tid - nT * 64;
    unsigned epos[B32_EMAX];
#pragma unroll
    for (int j = 0; j < B32_EMAX; ++j) {
        const int e = el + j * ne_lanes;
        epos[j] = 0xffffffffu;
        if (!prod && e < (int)blk) {
            const int half = e >= 2 * nsub, sub = (e - half * 2 * nsub) >> 1, comp = (e & 1) | (half << 1);
            int bp, bq;
            bt_sym_pq(P, sub, bp, bq);
            const int rr = 2 * bp + (comp & 1), cc = 2 * bq + (comp >> 1);
            epos[j] = (unsigned)(rr * LDM + cc) | ((unsigned)(cc * LDM + rr) << 16);
        }
    }
    auto fetch = [&](int s, float2(&dst)[B32_EMAX]) {
        const unsigned bo = (unsigned)(blk_of(s < nsteps ? s : nsteps - 1) * blk * (long long)sizeof(float2));
#pragma unroll
        for (int j = 0; j < B32_EMAX; ++j) {
            const int e = min(el + j * ne_lanes, (int)blk - 1);
            dst[j] = ld(rsD, (unsigned)e * (unsigned)sizeof(float2), bo);
        }
    };
    auto expand = [&](const float2(&src)[B32_EMAX], float2 *M) {
#pragma unroll
        for (int j = 0; j < B32_EMAX; ++j) {
            if (epos[j] != 0xffffffffu) {
                M[epos[j] & 0xffffu] = src[j];
                M[epos[j] >> 16] = src[j];
            }
        }
    };
    // ---- product waves: tile (source tile st, row tile it); lane: row i, sources c_q
    const int tile = prod ? wave : 0, st_ = tile / RT, it = tile % RT;
    const int i = it * 16 + (lane & 15);
    const int cq0 = st_ * 16 + 4 * (lane >> 4);
    const bool irow = prod && i < b;
    const int ic = i < b ? i : 0;                          // clamped row for addresses
    const long long cell0 = t.tr ? (long long)(t.y0 + ic) * nx + t.x0 : (long long)t.y0 * nx + t.x0 + ic;
    const unsigned kstep = (t.tr ? 1u : (unsigned)nx) * (unsigned)sizeof(float2);
    const unsigned bstep = (unsigned)b * (unsigned)sizeof(float2);
    // byte offsets of element q: its source's vector (rl_q, packed 8 bits each)
    // times a scalar stride plus the row's base, formed at each use
    int live = 0;                                          // bit q: (c_q, i) is a live element
    unsigned rlpk = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int c = cq0 + q, r = colr[c], rl = r >= 0 ? r - rfirst : 0;
        if (irow && r >= 0) live |= 1 << q;
        rlpk |= (unsigned)rl << (8 * q);
    }
    const unsigned lbase = (unsigned)((t.loc_off + ic) * (long long)sizeof(float2));
    const unsigned cbase = (unsigned)(cell0 * (long long)sizeof(float2));
    const unsigned LT8 = (unsigned)(LT * (long long)sizeof(float2));
    const unsigned VS8 = (unsigned)(vin_stride * (long long)sizeof(float2));
    const unsigned OS8 = (unsigned)(out_stride * (long long)sizeof(float2));
    auto rl_of = [&](int q) { return (rlpk >> (8 * q)) & 0xffu; };
    auto poff = [&](int q) { return rl_of(q) * LT8 + lbase; };
    auto voff = [&](int q) { return rl_of(q) * VS8 + cbase; };
    auto ooff = [&](int q) { return rl_of(q) * OS8 + cbase; };
    const int kc0 = t.tr ? t.cx0 - t.x0 : t.cy0 - t.y0, kc1 = t.tr ? t.cx1 - t.x0 : t.cy1 - t.y0;
    const int ic0 = t.tr ? t.cy0 - t.y0 : t.cx0 - t.x0, ic1 = t.tr ? t.cy1 - t.y0 : t.cx1 - t.x0;
    const bool icore = i >= ic0 && i < ic1;
    // v_{k+1} from the global input (forward) or w_k from the workspace (backward) for step s
    auto load_pre = [&](int s, float2(&dst)[4]) {
        const int sc_ = s < nsteps ? s : nsteps - 1;
        const int k = blk_of(sc_);
        if (sc_ < nb) {
            const unsigned so = (unsigned)(k + 1 < nb ? k + 1 : nb - 1) * kstep;
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[q] = ld(rsV, voff(q), so);
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[q] = ld(rsL, poff(q), (unsigned)k * bstep);
        }
    };
    float2 slot[B32_EMAX], pre[4];
    if (prod) {
        // operand of the first step: S_0 v_0, and v_1 for the first recurrence
        float2 v0[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) v0[q] = ld(rsV, voff(q), 0u);
        load_pre(0, pre);
        if (irow) {
            const float2 f = cmul(si_s[i], so_s[0]);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const float2 z = (live >> q) & 1 ? cmul(f, v0[q]) : make_float2(0.f, 0.f);
                XR(0)[(cq0 + q) * LDK + i] = z.x;
                XI(0)[(cq0 + q) * LDK + i] = z.y;
            }
        }
    } else {
        fetch(0, slot);
        expand(slot, MB(0));
        fetch(1, slot);
    }
    __syncthreads();
    // one block step s on buffers cur = s & 1; the expand waves expand block s + 1
    // (waiting in the slot) into the other buffer and refill the slot with block s + 2
    // The two source tiles (halves) are independent recurrences that share only
    // the factor block, so instead of a workgroup barrier per step the waves
    // synchronise through LDS counters, and one half's recurrence can overlap the
    // other half's products:
    //   sync[h]      product phases of half h done (its reads of M finished): RT per step
    //   sync[2]      expansions done: NE per step (block s + 1 during step s)
    //   sync[3 + h]  recurrences of half h done (its next operand written): RT per step
    // Products of step s wait for block s (sync[2] >= NE s) and for their half's
    // operand (sync[3 + h] >= RT s); the expansion of block s + 1 into the buffer
    // that step s - 1 read waits for the other expansion waves' previous block
    // (sync[2] >= NE s) and for both halves' products of step s - 1 (sync[h] >= RT s).
    // A count reaches k per wave only when every wave of its group has finished
    // step k - 1: no wave of a group starts step k before its whole group has
    // finished step k - 1, which each wait above ensures.  No wait depends on a
    // later one, so the halves drift at most a step apart, which the double
    // buffers cover.  Every wait is bounded (2^18 short sleeps, milliseconds,
    // where a block step takes a few microseconds), so a wave always finishes; a wave
    // whose wait ran out writes NaN instead of its values, which the outer
    // solver reports as a non-finite result rather than a wrong one.
    const int NE = BM_THREADS / 64 - nT, half = prod ? tile / RT : 0;
    auto wait_ge = [&](int idx, int target) {
        for (int spin = 0; spin < (1 << 18); ++spin) {
            if (__hip_atomic_load(&sync[idx], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP) >= target) return true;
            __builtin_amdgcn_s_sleep(1);
        }
        return false;
    };
    const float qnan = __builtin_nanf("");
    auto signal = [&](int idx) {
        if (lane == 0) __hip_atomic_fetch_add(&sync[idx], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    auto step = [&](int s) {
        const int cur = s & 1, k = blk_of(s);
        const bool fwd = s < nb, turn = s == nb - 1;
        if (prod) {
            const bool ok = wait_ge(2, NE * s) & wait_ge(3 + half, RT * s);
            // the first half contracts at raised issue priority, so the halves fall out
            // of step and one half's recurrence runs beside the other's products
            if (half == 0) __builtin_amdgcn_s_setprio(2);
            // three real products per complex one (Gauss): T1 = Yr Mr, T2 = Yi Mi,
            // T3 = (Yr + Yi)(Mr + Mi); Re = T1 - T2, Im = T3 - T1 - T2
            f32x4v accA = {0.f, 0.f, 0.f, 0.f}, accB = {0.f, 0.f, 0.f, 0.f}, accS = {0.f, 0.f, 0.f, 0.f};
            const int k0 = (lane >> 4) * KG;
            const float2 *mrow = MB(cur) + (it * 16 + (lane & 15)) * LDM + k0;
            const float *xr = XR(cur) + (st_ * 16 + (lane & 15)) * LDK + k0;
            const float *xi = XI(cur) + (st_ * 16 + (lane & 15)) * LDK + k0;
#pragma unroll 3
            for (int kk = 0; kk < KG; kk += 2) {
                const float4 m = *reinterpret_cast<const float4 *>(mrow + kk);
                const float2 yr = *reinterpret_cast<const float2 *>(xr + kk);
                const float2 yi = *reinterpret_cast<const float2 *>(xi + kk);
                const float mr[2] = {m.x, m.z}, mi[2] = {m.y, m.w}, vr[2] = {yr.x, yr.y}, vi[2] = {yi.x, yi.y};
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    accA = __builtin_amdgcn_mfma_f32_16x16x4f32(vr[u], mr[u], accA, 0, 0, 0);
                    accB = __builtin_amdgcn_mfma_f32_16x16x4f32(vi[u], mi[u], accB, 0, 0, 0);
                    accS = __builtin_amdgcn_mfma_f32_16x16x4f32(vr[u] + vi[u], mr[u] + mi[u], accS, 0, 0, 0);
                }
            }
            __builtin_amdgcn_s_setprio(0);
            signal(half);                                 // this step's reads of M and X done
            // recurrence of this lane's 4 (source, row) elements, straight from the accumulators.
            // Wait for every outstanding memory operation first: the counter retires in
            // issue order, so once this step's stores are issued, the wait for the operand
            // loaded in the previous step would also wait for those stores to complete.
            __builtin_amdgcn_s_waitcnt(0x0F70);           // vmcnt(0); expcnt, lgkmcnt unconstrained
            const int knext = fwd && !turn ? k + 1 : k - 1;
            const float2 cc = fwd ? cl_s[min(k + 1, nb - 1)] : ch_s[k];
            const float2 f = knext >= 0 && irow ? cmul(si_s[i], so_s[knext]) : make_float2(0.f, 0.f);
            const bool kcore = k >= kc0 && k < kc1;
            float *xrn = XR(cur ^ 1), *xin = XI(cur ^ 1);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                float2 z = make_float2(0.f, 0.f);
                if ((live >> q) & 1) {
                    const float2 a = ok ? make_float2(accA[q] - accB[q], accS[q] - accA[q] - accB[q])
                                        : make_float2(qnan, qnan);
                    float2 y;
                    if (fwd) {
                        if (!turn) st(rsL, poff(q), (unsigned)k * bstep, a);          // w_k
                        y = turn ? a : cfms(pre[q], cc, a);                            // y_{k+1} or u_{nb-1}
                    } else {
                        y = cfms(pre[q], cc, a);                                       // u_k
                    }
                    if ((!fwd || turn) && kcore && icore) st(rsO, ooff(q), (unsigned)k * kstep, y);
                    z = cmul(f, y);
                }
                if (irow) {
                    xrn[(cq0 + q) * LDK + i] = z.x;
                    xin[(cq0 + q) * LDK + i] = z.y;
                }
            }
            signal(3 + half);                             // the half's next operand written
            // the next step's v_{k+1} or w_k: in flight over the next products
            load_pre(s + 1, pre);
        } else if (s + 1 < nsteps) {
            // every expansion of block s done; step s - 1 no longer reads MB(cur ^ 1)
            const bool ok = wait_ge(2, NE * s) & wait_ge(0, RT * s) & wait_ge(1, RT * s);
            if (!ok)
#pragma unroll
                for (int j = 0; j < B32_EMAX; ++j) slot[j] = make_float2(qnan, qnan);
            expand(slot, MB(cur ^ 1));
            signal(2);
            fetch(s + 2, slot);
        }
    };
    for (int s = 0; s < nsteps; ++s) step(s);
}

// dynamic LDS of a launch whose widest block is bmax (either group form may run)
static size_t bm_lds_bytes(int bmax) {
    if (bmax <= BM_NARROW) return b32_lds_bytes(bmax);
    return std::max(b32_lds_bytes(BM_NARROW), bm_lds_class(bmax, 16));
}

// jobs[j] = (tile, wavelength, first source, sources), at most bm_cols(b) sources
__global__ __launch_bounds__(BM_THREADS) void bt_solve_multi_kernel(
    const TileDesc *__restrict__ tiles, const int4 *__restrict__ jobs, int n_src, const float2 *__restrict__ dinv,
    long long dinv_wl_stride, const float2 *__restrict__ coef, const float2 *__restrict__ sc, int nx, int ny,
    const float2 *__restrict__ vin, long long vin_stride, float2 *__restrict__ out, long long out_stride,
    const int *__restrict__ active, float2 *__restrict__ loc, long long LT) {
    extern __shared__ __align__(16) float lds[];
    __shared__ float2 cl_s[BT_NBMAX], ch_s[BT_NBMAX], so_s[BT_NBMAX], si_s[BT_BMAX];
    __shared__ int colr[32];                          // RHS index of each column, -1 when idle
    __shared__ int sync[5];                           // step counters of the 32-source form
    const int4 job = jobs[blockIdx.x];
    if (job.x < 0) return;
    const TileDesc t = tiles[job.x];
    if (t.b <= BM_NARROW)
        bm_solve32(t, job.y, job.z, job.w, n_src, dinv, dinv_wl_stride, coef, sc, nx, ny, vin, vin_stride, out,
                   out_stride, active, loc, LT, lds, cl_s, ch_s, so_s, si_s, colr, sync);
    else
        bm_solve<16, 7, 2>(t, job.y, job.z, job.w, n_src, dinv, dinv_wl_stride, coef, sc, nx, ny, vin, vin_stride,
                           out, out_stride, active, loc, LT, lds, cl_s, ch_s, so_s, si_s, colr);
}

void launch_bt_solve_multi(hipStream_t s, const TileDesc *tiles, const int4 *jobs, int n_jobs, int n_src,
                           const float2 *dinv, long long dinv_wl_stride, const float2 *coef, const float2 *sc, int nx,
                           int ny, const float2 *vin, long long vin_stride, float2 *out, long long out_stride,
                           const int *active, float2 *loc, long long LT, int bmax) {
    hipLaunchKernelGGL(bt_solve_multi_kernel, dim3(n_jobs), dim3(BM_THREADS), bm_lds_bytes(bmax), s, tiles, jobs,
                       n_src, dinv, dinv_wl_stride, coef, sc, nx, ny, vin, vin_stride, out, out_stride, active, loc,
                       LT);
}

void bt_solve_multi_prepare(int bmax) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void *>(&bt_solve_multi_kernel),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)bm_lds_bytes(bmax));
}

}  // namespace nosdd
