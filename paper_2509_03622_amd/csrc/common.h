// Internal declarations shared by the HIP translation units of libnosdd.
// Complex values are float2 / double2 with (x, y) = (re, im).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nosdd {

// ------------------------------------------------------------ complex helpers
__host__ __device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a + b*c
__host__ __device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c) {
    return make_float2(a.x + b.x * c.x - b.y * c.y, a.y + b.x * c.y + b.y * c.x);
}
// a - b*c
__host__ __device__ __forceinline__ float2 cfms(float2 a, float2 b, float2 c) {
    return make_float2(a.x - b.x * c.x + b.y * c.y, a.y - b.x * c.y - b.y * c.x);
}
// a + conj(b)*c
__host__ __device__ __forceinline__ float2 cfma_conj(float2 a, float2 b, float2 c) {
    return make_float2(a.x + b.x * c.x + b.y * c.y, a.y + b.x * c.y - b.y * c.x);
}
__host__ __device__ __forceinline__ float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }
__host__ __device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

__host__ __device__ __forceinline__ double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__host__ __device__ __forceinline__ double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__host__ __device__ __forceinline__ double2 zmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ __forceinline__ double2 zfms(double2 a, double2 b, double2 c) {
    return make_double2(a.x - b.x * c.x + b.y * c.y, a.y - b.x * c.y - b.y * c.x);
}
__host__ __device__ __forceinline__ double2 zdiv(double2 a, double2 b) {
    double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__host__ __device__ __forceinline__ double zabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// ------------------------------------------------------------ problem geometry
// Interface-side bits of a tile.
enum { SIDE_BOTTOM = 1, SIDE_RIGHT = 2, SIDE_TOP = 4, SIDE_LEFT = 8 };

// One extended subdomain, as seen by the kernels.  The tile is factorised as
// block-tridiagonal with nb blocks of size b: blocks are grid rows (tr = 0,
// block k <-> y = y0 + k, position m <-> x = x0 + m) or grid columns (tr = 1,
// block k <-> x = x0 + k, m <-> y = y0 + m), whichever makes b the smaller side.
struct TileDesc {
    int x0, x1, y0, y1;       // extended box [x0,x1) x [y0,y1)
    int cx0, cx1, cy0, cy1;   // core
    int tr, b, nb, iface;
    long long loc_off;        // cell offset in a packed local vector (one RHS)
    long long dinv_off;       // float2 offset of this tile's D_k^-1 blocks (one wavelength)
    int tr_off, n_tr;         // trace entries
    int box_off;              // float2 offset of this tile's coarse box (one column)
    int bw, bh;               // coarse box (core grown by one cell, clipped)
    int bx0, by0;
};

// Per-wavelength stencil coefficient layout inside a float2 array:
// [cxm(nx) | cxp(nx) | cym(ny) | cyp(ny)], stride 2*(nx+ny) per wavelength.
__host__ __device__ __forceinline__ long long coef_stride(int nx, int ny) { return 2LL * (nx + ny); }

// ------------------------------------------------------------ launchers
// All launches go on `s`; vectors are [rhs][ny][nx] float2 with rhs = wl*n_src + src.
void launch_stencil(hipStream_t s, const float2 *x, const float2 *b, float2 *y, const float *eps,
                    const double2 *coef, const double *k0, int nx, int ny, int n_rhs, int n_src,
                    const int *active);

void launch_residual64(hipStream_t s, const double2 *x, const double2 *b, float2 *r, const float *eps,
                       const double2 *coef, const double *k0, int nx, int ny, int n_rhs, int n_src);

// Symmetric storage of the subdomain factors.  With S_k = diag of the centre
// stretches s_x s_y on block k, M_k = D_k^-1 S_k^-1 = (S_k D_k)^-1 is complex
// symmetric, and D_k^-1 y = M_k (S_k y).  Only the upper triangle is kept, as
// 2 x 2 sub-blocks (rows 2p, 2p+1; columns 2q, 2q+1; q >= p).  A block holds
// n = P (P + 1) / 2 sub-blocks in two halves: first the first columns
// (M[2p][2q], M[2p+1][2q]) of every sub-block, 16 bytes each, then their
// second columns (M[2p][2q+1], M[2p+1][2q+1]), so that one 16-byte load per
// lane over consecutive sub-blocks reads whole cache lines.  With
// P = b/2 the sub-blocks are laid out in rows D = 0 .. P/2 of P entries (the
// last one, D = P/2 for even P, has P/2): row 0 is the diagonal, row D > 0
// holds diagonal D at entries 0..P-D-1 and diagonal P-D at entries P-D..P-1,
// so the row-pair p and the offset d = 0..P-1 (column pair (p + d) mod P)
// always find their sub-block at entry bt_sym_index.
__host__ __device__ __forceinline__ long long bt_sym_block(int b) { return (long long)b * (b + 2) / 2; }  // complex
// sub-block (row of the storage D, entry i) -> (p, q) with q >= p
__host__ __device__ __forceinline__ void bt_sym_pq(int P, int sub, int &p, int &q) {
    if (sub < P) {
        p = q = sub;
        return;
    }
    const int D = sub / P, i = sub - D * P;
    if (i < P - D) {
        p = i;
        q = i + D;
    } else {
        p = i - (P - D);
        q = i;
    }
}
// row pair p, offset d in [0, P): storage sub-block index and whether the
// sub-block is (p, q) as stored (true) or its transpose (false)
__host__ __device__ __forceinline__ int bt_sym_index(int P, int p, int d, bool &direct) {
    direct = p + d < P;
    if (d == 0) return p;
    if (2 * d == P) return d * P + (p < d ? p : p - d);
    if (2 * d < P) return d * P + p;
    const int D = P - d, idx = p + d < P ? p + d : p + d - P;
    return D * P + idx;
}

// Factorisation of every (tile, wavelength); tiles whose short side exceeds
// 72 (listed in big[n_big]) use scratch[n_wl * n_big * 128 * 128] (FP64 complex).
void launch_bt_factor(hipStream_t s, const TileDesc *tiles, int n_tiles, int n_wl, const float *eps,
                      const double *coef_d, const double *k0, double h, int nx, int ny, const float2 *sc,
                      float2 *dinv, long long dinv_wl_stride, const int *big, int n_big, double2 *scratch);
constexpr int BT_FACT_SCRATCH_B = 128;

// mode bit 0: input is a packed local vector (else gathered from a global vector)
// mode bit 1: output is a packed local vector (else core cells scattered to a global vector)
// Subdomain LU solves; the tile's RHS lives in max_cells * 8 bytes of LDS.
constexpr int BT_NBMAX = 256;                                // longest tile side
constexpr int BT_LDS_MAX_CELLS = 15360;                      // 120 KB of LDS
// One workgroup per job: order[n_jobs] = (tile, rhs), tile < 0 for padding.
// depth: prefetch depth of the factor-block ring (one of bt_solve_depths, 0 = default).
void launch_bt_solve(hipStream_t s, const TileDesc *tiles, const int2 *order, int n_jobs, int n_src,
                     const float2 *dinv, long long dinv_wl_stride, const float2 *coef, const float2 *sc, int nx,
                     int ny, const float2 *vin, long long vin_stride, float2 *out, long long out_stride,
                     const int *active, int mode, int bmax, int max_cells, int depth = 0);
void bt_solve_prepare(int bmax, int max_cells);
// Many sources per wavelength: one workgroup per jobs[j] = (tile, wavelength,
// first source, sources), bt_multi_cols(tile block size) sources at most; the gathered
// right-hand sides and intermediate blocks go through loc[n_rhs][LT] (packed
// local layout, block-major within a tile).  Global input and core output.
int bt_multi_cols(int b);
void launch_bt_solve_multi(hipStream_t s, const TileDesc *tiles, const int4 *jobs, int n_jobs, int n_src,
                           const float2 *dinv, long long dinv_wl_stride, const float2 *coef, const float2 *sc, int nx,
                           int ny, const float2 *vin, long long vin_stride, float2 *out, long long out_stride,
                           const int *active, float2 *loc, long long LT, int bmax);
void bt_solve_multi_prepare(int bmax);
int bt_solve_depths(int bmax, int *depths);

// Algorithm 3 loop (paperloop.hip)
void launch_robin_rhs(hipStream_t s, const TileDesc *tiles, int n_tiles, const int4 *ent, const float2 *injc, int ne,
                      const float2 *b, const float2 *g, float2 *rhs, long long N, long long LT, int nx, int n_rhs,
                      int n_src, const int *active);
void launch_rc_dot(hipStream_t s, const int *col_ptr, const int *col_ent, const float2 *col_val, int nnz, int nc,
                   int ne, const float2 *g, const float2 *gn, double2 *d, int n_rhs, int n_src, const int *active);
void launch_rc_update(hipStream_t s, const int *row_ptr, const int *row_col, const float2 *row_q,
                      const float2 *row_tq, int nnz, int ne, int nc, float2 *g, const float2 *gn, const float2 *z,
                      float m, int coarse, int n_rhs, int n_src, const int *active);
void launch_norm2(hipStream_t s, const float2 *v, long long N, int n_rhs, double *part, double *out);
int norm2_partials();

void launch_robin_trace(hipStream_t s, const int4 *entries, int n_entries, const float *eps,
                        const float *k0, float h, int nx, int ny, const float2 *x, float2 *g,
                        int n_vec, int vec_per_wl);

// Krylov helpers.  V is the basis: vector i of rhs r at V + i*vstride + r*N.

struct GivensArgs {
    float2 *H; int ldh; int m;        // H[r][i][j] at H + (r*(m+1) + i)*m + j
    float2 *H2;                       // second-pass coefficients, same layout
    float *cs; float2 *sn; float2 *gam;
    const double *nw_pre;             // ||w||^2 before orthogonalisation (read by the Givens step)
    double *nw_pre_w;                 // the same buffer, written by the first reduction
    int *reorth;                      // per-rhs gate set here (DGKS test)
    const float *bnorm; float tol;
    int *active; int *iters; int *kcyc; int max_iters;
    float *hist; int hist_ld;
    float *inv_h; int *flags;         // flags bit 0 converged, bit 1 breakdown, bit 2 budget
    // stored-basis form of the two-pass Gram-Schmidt (modes 6 and 7): the
    // orthonormal basis is V = Vs T with Vs the stored vectors and T upper
    // triangular, T[r][k][i] at T + (r*(m+1) + k)*(m+1) + i (FP64); G1 holds the
    // first-pass coefficients on the stored vectors (layout of H); scale the
    // factor the first-pass update applies to the vector it stores
    double2 *T; float2 *G1; float *scale;
    int *host_flags;                  // nullable: pinned host copy of active[] written by the last reduction of a step
};
void launch_cgs_dots(hipStream_t s, const float2 *V, long long vstride, int nv, const float2 *w, long long N,
                     int n_rhs, const int *gate, double2 *partial, int nblk);
// second pass and normalisation in one: v_{j+1} = (w - V h2) / h (reorth) or w / h
void launch_cgs_update_scale(hipStream_t s, const float2 *V, long long vstride, int nv, const float2 *w, float2 *dst,
                             long long N, int n_rhs, const int *active, const int *reorth, const float2 *Hc, int m,
                             int col, const float *inv_h, int nblk);
void launch_cgs_update_dots(hipStream_t s, const float2 *V, long long vstride, int nv, const float2 *w, float2 *dst,
                            long long N, int n_rhs, const int *gate, const float2 *Hc, int m, int col,
                            double2 *partial, int nblk, const float *scale = nullptr);
void launch_cgs_reduce(hipStream_t s, const double2 *partial, int nblk, int nv, int n_rhs, const int *gate, int col,
                       int mode, double *norm_out, const GivensArgs &ga);
int nblk_for_update(long long N, int n_rhs);
void launch_backsolve(hipStream_t s, const float2 *H, int ldh, int m, const float2 *gam, const int *kcyc,
                      float2 *y, int n_rhs);
void launch_xupdate(hipStream_t s, double2 *x, const float2 *Z, long long zstride, const float2 *y, int m,
                    const int *kcyc, long long N, int n_rhs);
void launch_start_cycle(hipStream_t s, float2 *V0, const float2 *r, const double *beta2, const float *bnorm,
                        float2 *gam, int m, int *kcyc, int *active, const int *want, long long N, int n_rhs);

// Coarse space
void launch_coarse_dot(hipStream_t s, const TileDesc *tiles, int n_c, int kc, const float2 *Wbox,
                       long long box_wl_stride, const float2 *v, const float2 *w1, int nx, long long N, int n_rhs,
                       int n_src, const int *active, double2 *d);
void launch_coarse_solve(hipStream_t s, const double2 *GinvT, int n_c, const double2 *d, float2 *c, int n_rhs,
                         int n_src, const int *active);
void launch_coarse_update(hipStream_t s, const TileDesc *tiles, const int *owner, int kc, const float2 *Phibox,
                          const float2 *Wbox, long long box_wl_stride, const float2 *c, int n_c, float2 *z, float2 *w,
                          int nx, int ny, int n_rhs, int n_src, const int *active);
void launch_coarse_cycle_end(hipStream_t s, double2 *x, const TileDesc *tiles, const int *owner, int kc,
                             const float2 *Phibox, long long box_wl_stride, const float2 *C, const float2 *y, int m,
                             const int *kcyc, int n_c, double2 *cy, int nx, int ny, int n_rhs, int n_src);

// ------------------------------------------------------------ neural subdomain solver
// One sample = one (subdomain, RHS) pair: tile geometry and where its vectors live.
struct FnoSample {
    int lx, ly;
    long long cell_off;     // offset of the sample's cells in a sample-packed cell array
    long long aux_off;      // offset (cells) of its aux channels in [wl][7][loc_total]
    int mod_idx;            // (wavelength, subdomain) index of its modulation tensors
    int pad_;
};

// Network parameters on the device (C = 64, 16 modes, projection width 128).
struct FnoDevice {
    int layers = 0;
    float *lift_w = nullptr, *lift_b = nullptr;   // [64][9], [64]
    unsigned short *R = nullptr;                  // [layer][512][128][128] bf16: real form of the complex mix,
                                                  // rows (Re, Im) of input channel i at 2i, 2i+1, columns likewise
    unsigned short *W = nullptr;                  // [layer][64][64] bf16
    float *b = nullptr;                           // [layer][64]
    unsigned short *p1w = nullptr;                // [128][64] bf16
    float *p1b = nullptr, *p2w = nullptr, *p2b = nullptr;   // [128], [2][128], [2]
    float2 *tw = nullptr;                         // twiddle tables, FNO_TW_UNIT * L float2 per side L
    // inverse x-transform as the B operand of BF16 MFMA: per side L, at
    // twb + 128 L (L-1), the real 2 x 2 form [n = (x, Re/Im out)][k = (kx, Re/Im in)]
    // (2L x 64) as BF16 high parts, then the same as BF16 low parts (value - high)
    unsigned short *twb = nullptr;
    // forward x-transform as the B operand of BF16 MFMA: per side L, at
    // twf + 2 * 64 * FNO_TWF_K * (L - 1), [n = (kx, Re/Im out)][k = (x, Re/Im in)]
    // (64 x FNO_TWF_K, zero for k >= 2L) as BF16 high parts, then as low parts
    unsigned short *twf = nullptr;
    // modulated network: mod[mod_idx][layer][mode] (complex) multiplies the
    // spectral product of every block mode by mode; null for the plain network
    const float2 *mod = nullptr;
};
// Twiddle tables of the truncated DFTs for side L, at tw + FNO_TW_UNIT L (L-1)/2:
// forward kx [x][q] (L x 32), inverse kx [q][x] at FNO_TW_INV_X L, forward ky
// [y][ky] (L x 16) at FNO_TW_FWD_Y L, inverse ky at FNO_TW_INV_Y L.
constexpr int FNO_MAXL = 72;
constexpr int FNO_MODES_TOTAL = 512;                          // 32 kx x 16 ky kept modes
constexpr int FNO_TW_INV_X = 32, FNO_TW_FWD_Y = 64, FNO_TW_INV_Y = 80, FNO_TW_UNIT = 96;
constexpr int FNO_TWF_K = 2 * FNO_MAXL;                       // row length of the twf tables

// Workspace of the batched inner NN-FGMRES (device pointers).
struct NnWork {
    const FnoDevice *net = nullptr;
    const FnoSample *smp = nullptr;
    int steps = 0, maxk = 0;
    float tol = 0.f;
    float2 *Vin = nullptr, *Zin = nullptr, *w = nullptr;     // [k][rhs][loc_total]
    float *beta = nullptr, *vscale = nullptr, *oscale = nullptr, *cs = nullptr;
    int *sact = nullptr, *kstep = nullptr;
    float2 *gam = nullptr, *H = nullptr, *sn = nullptr;
    const float *aux = nullptr;                               // [wl][7][loc_total]
    float *act0 = nullptr, *act1 = nullptr, *spec = nullptr, *X = nullptr, *Y = nullptr;
    // exact-LU fallback: per-sample failure flag, the fallback job queue
    // (tile, rhs) per sample ((-1, -1) where the inner solve is kept) and a
    // running count of fallen-back samples
    int *fb = nullptr;
    int2 *fb_order = nullptr;
    unsigned *fb_count = nullptr;
};

// Fixed per-device scratch of the entry point that allocates nothing (noalloc.hip):
// init looks the array's device address up on `device` (once; done at context
// creation), noalloc_scratch returns it (nullptr before init).
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(16) << 20;
hipError_t noalloc_scratch_init(int device);
void *noalloc_scratch(int device);
void launch_noalloc_queue(hipStream_t s, int2 *order, int n_tiles, int n_rhs);

// An inner solve whose final residual estimate is not below this fraction of
// its right-hand side's norm, or that meets a non-finite value, is replaced
// by the exact subdomain LU solve in the same sweep.
constexpr float NN_FALLBACK_RATIO = 0.99f;

// Inverse-design gradient (adjoint.hip).  sc: per wavelength [s_x(nx) | s_y(ny)]
// centre stretches; focal: (ix, iy) cells.
void launch_adjoint_rhs(hipStream_t s, const float2 *E, long long N, int nx, int ny, const int2 *focal, int n_focal,
                        const float2 *sc, const float *k0f, int n_rhs, int n_src, float2 *Jadj, double *fomv);
void launch_adjoint_grad(hipStream_t s, const float2 *E, const float2 *mu, long long N, int nx, int ny, int n_rhs,
                         int n_src, const float2 *sc, const float *k0f, float *grad);

// Inner NN-FGMRES on every (tile, RHS) sample.  local == 0: v and z are
// global [n_rhs][N] vectors (gather over the extended subdomain, core-only
// scatter); local != 0: v and z are subdomain-local [n_rhs][loc_total].
// Samples that fail (see NN_FALLBACK_RATIO) leave z untouched and are listed
// in nw.fb_order for an exact block-Thomas solve (launch_bt_solve over
// n_rhs * n_tiles jobs) that the caller issues next.
void nn_precond(hipStream_t st, const NnWork &nw, const TileDesc *tiles, int n_tiles, int n_rhs, int n_src,
                long long loc_total, int max_cells, const float2 *v, float2 *z, const int *active, const float *eps,
                const double2 *coef, const double *k0, double h, int nx, int ny, int local);
// per-sample rms scalings for a plain network application on arbitrary vectors
void nn_rms_scales(hipStream_t st, const FnoSample *smp, int S, const float2 *v, float *vscale, float *oscale);

// e = NN(v) for every active sample; v, e: sample-packed complex cells.
// raises the dynamic-LDS limit of the network kernels that need more than 64 KB
void fno_prepare();
void fno_forward(hipStream_t st, const FnoDevice &net, const FnoSample *smp, const int *sact, int S_tot, int max_cells,
                 const float2 *v, const float *vscale, const float *oscale, const float *aux, long long aux_ch_stride,
                 float *act0, float *act1, float *spec, float *X, float *Y, float2 *e);

}  // namespace nosdd
