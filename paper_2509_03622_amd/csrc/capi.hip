// libnosdd host runtime and C ABI (declared in include/nosdd.h).
//
// Owns the device memory plan of a problem (permittivity, per-wavelength
// stencil coefficients, subdomain factors, coarse basis, Krylov workspace) and
// drives right-preconditioned flexible GMRES(restart) on the global FDFD
// system, one Schwarz sweep (all subdomains x all RHS in one launch) per
// preconditioner application.  The host only reads back one small status
// array per outer iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <map>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/nosdd.h"
#include "common.h"
#include "hostla.h"

using namespace nosdd;
using cd = std::complex<double>;

struct nosdd_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    hipStream_t cap_stream = nullptr;     // private stream for graph capture (created on first use)
    std::string err;
};

namespace {

// Bumped on every device (re)allocation: captured graphs bake buffer addresses
// into their kernel arguments and are rebuilt when this changes.
std::atomic<long long> g_alloc_gen{0};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    hipError_t ensure(size_t n) {
        if (n <= bytes && p) return hipSuccess;
        release();
        ++g_alloc_gen;
        hipError_t e = hipMalloc(&p, n ? n : 16);
        if (e == hipSuccess) bytes = n;
        return e;
    }
    template <class T>
    T *as() const { return static_cast<T *>(p); }
};

struct Workspace {
    int n_rhs = 0, m = 0, max_iters = 0, nblk = 0;
    // Gram-Schmidt workgroups per RHS by basis size (bucket of j + 1: <= 8, 16, 24, 32),
    // chosen by the autotuner; nblk_max bounds the partials buffer
    int nblk_b[4] = {0, 0, 0, 0}, nblk_max = 0;
    bool tuned = false;
    long long N = 0;
    DevBuf T, G1, scale;                           // stored-basis Gram-Schmidt (T: FP64 [rhs][m+1][m+1])
    DevBuf cstep, cy;                              // coarse coefficients per step [m][rhs][n_c], their y-sum
    DevBuf x, b, b64, V, Z, w, partial, H, H2, cs, sn, gam, y, nw_pre, nw_post, bnorm2, bnorm, beta2,
        iters, kcyc, active, want, ones, reorth, inv_h, flags, hist, cd_, cc_;
    DevBuf loc;                                    // packed local vectors of the many-source solve
};

}  // namespace

struct nosdd_problem {
    nosdd_ctx *ctx = nullptr;
    int nx = 0, ny = 0, npml = 0, pml_m = 2;
    double h = 0.05, lnR = -30.0;
    std::vector<float> eps;
    std::vector<double> wl;
    int overlap = 0, ext = 0;
    std::vector<TileDesc> tiles;
    std::vector<int> owner;                          // [ny][nx]: index of the core holding the cell
    std::vector<std::vector<int>> nbrs;              // per tile: tiles whose ring reaches into it
    std::vector<std::vector<int4>> tile_entries;     // (p, q, side, 0) linear cell indices
    long long loc_total = 0, dinv_wl_stride = 0;
    int bmax = 0;
    std::vector<std::vector<cd>> coefd;             // per wl: cxm|cxp|cym|cyp
    DevBuf d_eps, d_coef, d_coefd, d_k0sq, d_k0f, d_k0, d_tiles, d_dinv, d_entries, d_owner;
    DevBuf d_sc;                                   // per wl: centre stretches s_x(nx) | s_y(ny)
    DevBuf adj_E, adj_mu, adj_J, adj_focal, adj_fom; // inverse-design gradient buffers
    int n_entries = 0;
    // coarse space
    int kc = 0, ktrial = 8, n_c = 0;
    long long box_wl_stride = 0;
    DevBuf d_phi, d_W, d_GinvT;
    // Robin-data injection coefficients -a_pq tau_p per (wl, entry), and the
    // Robin-space coarse space of the Algorithm 3 loop: (I - T) Q sparse by
    // entry (Q, T Q values) and by column (M = Q - T Q), per wavelength, and
    // the FP64 inverse (transposed) of M^H M
    DevBuf d_injc;
    int rc_nnz = 0;
    DevBuf d_rc_rowptr, d_rc_rowcol, d_rc_q, d_rc_tq, d_rc_colptr, d_rc_colent, d_rc_colval, d_rc_GinvT;
    bool setup_done = false;
    int sub_solver = 0;
    Workspace ws;
    // neural subdomain solver
    FnoDevice net;
    DevBuf d_net, d_aux, d_smp, d_mod;
    // modulation path of the modulated network (host copy, FP32 values of the
    // BF16 weights): conv 3x3 7 -> mod_ch, pool to mod_pool^2, FC -> mod_hidden, FC -> layers x 512 x 2
    int mod_ch = 0, mod_pool = 0, mod_hidden = 0;
    std::vector<float> mod_cw, mod_cb, mod_f1w, mod_f1b, mod_f2w, mod_f2b;
    int nn_steps = 2, max_cells = 0;
    float nn_tol = 0.1f;
    int smp_rhs = 0;                              // samples built for this many RHS
    DevBuf nn_Vin, nn_Zin, nn_w, nn_beta, nn_vs, nn_os, nn_cs, nn_sact, nn_kstep, nn_gam, nn_H, nn_sn, nn_act0, nn_act1,
        nn_spec, nn_X, nn_Y;
    DevBuf nn_fb, nn_fborder, nn_fbcount;          // exact-LU fallback of failed inner solves
    NnWork nw;
    double setup_ms = 0.0, solve_ms = 0.0;
    int last_iters = 0;
    // optional per-class kernel timing (events on the context stream)
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<std::pair<int, std::pair<int, int>>> ev_pending;   // class, (start, stop) pool index
    int ev_next = 0;
    double prof_ms[4] = {0, 0, 0, 0};
    long long prof_launch[4] = {0, 0, 0, 0}, prof_units[4] = {0, 0, 0, 0};
    // launch queues of the subdomain solve, per (n_rhs, n_src)
    struct OrderBuf {
        DevBuf buf;
        int n_jobs = 0;
        DevBuf mbuf;                                 // many-source jobs (tile, wavelength, first source, sources)
        int n_mjobs = 0;
    };
    std::map<std::pair<int, int>, OrderBuf> orders;
    // autotuned launch parameters (subdomain-solve prefetch depth; the Gram-Schmidt
    // grid lives in the workspace)
    bool use_autotune = true;
    bool use_multi = true;                        // many-source solve (use_multi())
    bool stored_basis = true;                     // Gram-Schmidt second pass in coefficient space
    int bt_depth = 0;
    bool bt_tuned = false;
    // one captured graph per Arnoldi step j of a restart cycle (replayed every cycle)
    bool use_graphs = true;
    std::vector<hipGraphExec_t> gexec;
    std::vector<long long> gkey;
    int *h_flags = nullptr;                       // pinned: active flags of steps of either parity
    int *d_flags = nullptr;                       // the same memory as seen from the device
    int h_flags_n = 0;
    hipEvent_t gev[2] = {nullptr, nullptr};
    void drop_graphs() {
        for (hipGraphExec_t g : gexec) (void)hipGraphExecDestroy(g);
        gexec.clear();
        gkey.clear();
    }
    ~nosdd_problem() {
        for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
        drop_graphs();
        for (hipEvent_t e : gev)
            if (e) (void)hipEventDestroy(e);
        if (h_flags) (void)hipHostFree(h_flags);
    }
};

namespace {

#define HIPCHK(ctx, expr)                                                                    \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            (ctx)->err = std::string("HIP error: ") + hipGetErrorString(e_) + " at " #expr;   \
            return e_ == hipErrorOutOfMemory ? NOSDD_ENOMEM : NOSDD_EHIP;                    \
        }                                                                                    \
    } while (0)

nosdd_status fail(nosdd_ctx *ctx, nosdd_status s, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return s;
}

// Timing events and pinned host memory of one call, released on every return path.
struct CallResources {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int *h_pinned = nullptr;
    ~CallResources() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (h_pinned) (void)hipHostFree(h_pinned);
    }
};

// ---------------------------------------------------------------- PML / stencil
// s(q) = 1 - i sigma_hat d(q)^m,  sigma_hat = (m+1)(-lnR) / (2 k0 npml h),
// d(q) = clip(max(npml - 1/2 - q, q - (n - npml - 1/2)) / npml, 0, 1).
cd stretch(double q, int n, int npml, int m, double sh) {
    if (npml == 0) return cd(1.0, 0.0);
    double d = std::max(npml - 0.5 - q, q - (n - npml - 0.5)) / npml;
    d = std::min(1.0, std::max(0.0, d));
    return cd(1.0, -sh * std::pow(d, m));
}

std::vector<cd> axis_coefs(int n, int npml, int m, double lnR, double k0, double h) {
    const double sh = npml ? (m + 1) * (-lnR) / (2.0 * k0 * npml * h) : 0.0;
    std::vector<cd> out(2 * n);
    for (int i = 0; i < n; ++i) {
        const cd sc = stretch(i, n, npml, m, sh);
        const cd sm = stretch(i - 0.5, n, npml, m, sh);
        const cd sp = stretch(i + 0.5, n, npml, m, sh);
        out[i] = -1.0 / (sm * sc * h * h);        // coupling to i-1
        out[n + i] = -1.0 / (sp * sc * h * h);    // coupling to i+1
    }
    return out;
}

// ---------------------------------------------------------------- small dense FP64 linear algebra
// Hermitian eigen-decomposition by cyclic Jacobi rotations (n <= 64).
void herm_eig(int n, std::vector<cd> A, std::vector<double> &w, std::vector<cd> &V) {
    V.assign((size_t)n * n, cd(0, 0));
    for (int i = 0; i < n; ++i) V[(size_t)i * n + i] = 1.0;
    double nrm = 0;
    for (auto &a : A) nrm += std::norm(a);
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off += std::norm(A[(size_t)p * n + q]);
        if (off <= 1e-30 * nrm) break;
        for (int p = 0; p < n; ++p) {
            for (int q = p + 1; q < n; ++q) {
                const cd apq = A[(size_t)p * n + q];
                const double a = std::abs(apq);
                if (a == 0.0) continue;
                const cd ph = apq / a;                      // e^{i phi}
                const double al = A[(size_t)p * n + p].real(), be = A[(size_t)q * n + q].real();
                const double th = 0.5 * std::atan2(2.0 * a, be - al);
                const double c = std::cos(th), s = std::sin(th);
                const cd em = std::conj(ph);                // e^{-i phi}
                // A <- A J (columns p, q)
                for (int i = 0; i < n; ++i) {
                    const cd xp = A[(size_t)i * n + p], xq = A[(size_t)i * n + q];
                    A[(size_t)i * n + p] = c * xp - s * em * xq;
                    A[(size_t)i * n + q] = s * xp + c * em * xq;
                    const cd vp = V[(size_t)i * n + p], vq = V[(size_t)i * n + q];
                    V[(size_t)i * n + p] = c * vp - s * em * vq;
                    V[(size_t)i * n + q] = s * vp + c * em * vq;
                }
                // A <- J^H A (rows p, q)
                for (int j = 0; j < n; ++j) {
                    const cd xp = A[(size_t)p * n + j], xq = A[(size_t)q * n + j];
                    A[(size_t)p * n + j] = c * xp - s * ph * xq;
                    A[(size_t)q * n + j] = s * xp + c * ph * xq;
                }
            }
        }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = A[(size_t)i * n + i].real();
}

// Explicit inverse of a Hermitian positive-definite matrix through its
// profile Cholesky factor (the coarse matrices are block-sparse: only
// neighbouring subdomains couple), column solves spread over host threads.
bool hpd_inverse(int n, const std::vector<cd> &G, std::vector<cd> &Ginv) {
    return hpd_inverse_profile(n, G, Ginv);
}

// ---------------------------------------------------------------- geometry helpers
void ring_nodes(const TileDesc &t, std::vector<std::pair<int, int>> &nodes) {
    nodes.clear();
    for (int x = t.x0; x < t.x1; ++x) nodes.push_back({x, t.y0});
    for (int y = t.y0 + 1; y < t.y1; ++y) nodes.push_back({t.x1 - 1, y});
    for (int x = t.x1 - 2; x >= t.x0; --x) nodes.push_back({x, t.y1 - 1});
    for (int y = t.y1 - 2; y > t.y0; --y) nodes.push_back({t.x0, y});
}

// trace entries of a tile (p, q linear; z = side bit; w = ring node index)
void trace_entries(const TileDesc &t, int nx, std::vector<int4> &out) {
    std::vector<std::pair<int, int>> nodes;
    ring_nodes(t, nodes);
    out.clear();
    for (int r = 0; r < (int)nodes.size(); ++r) {
        const int x = nodes[r].first, y = nodes[r].second;
        const int p = y * nx + x;
        if ((t.iface & SIDE_BOTTOM) && y == t.y0) out.push_back(make_int4(p, p - nx, SIDE_BOTTOM, r));
        if ((t.iface & SIDE_RIGHT) && x == t.x1 - 1) out.push_back(make_int4(p, p + 1, SIDE_RIGHT, r));
        if ((t.iface & SIDE_TOP) && y == t.y1 - 1) out.push_back(make_int4(p, p + nx, SIDE_TOP, r));
        if ((t.iface & SIDE_LEFT) && x == t.x0) out.push_back(make_int4(p, p - 1, SIDE_LEFT, r));
    }
}

// b = -i omega J for every RHS; J is [n_src][N] (shared by the wavelengths),
// or [n_rhs][N] when per_rhs is set.
__global__ void make_rhs_kernel(const float2 *J, float2 *b, const float *k0, long long N, int n_src, int per_rhs) {
    const int r = blockIdx.y;
    const int wl = r / n_src, s = r - wl * n_src;
    const float om = k0[wl];
    const float2 *Jr = J + (per_rhs ? r : s) * N;
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
        const float2 j = Jr[n];
        b[r * N + n] = make_float2(om * j.y, -om * j.x);    // -i omega J
    }
}

// The same right-hand side in FP64 (-i omega J with omega in FP64), for the
// residuals of the FP64 outer iterate.
__global__ void make_rhs64_kernel(const float2 *J, double2 *b, const double *k0, long long N, int n_src,
                                  int per_rhs) {
    const int r = blockIdx.y;
    const int wl = r / n_src, s = r - wl * n_src;
    const double om = k0[wl];
    const float2 *Jr = J + (per_rhs ? r : s) * N;
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
        const float2 j = Jr[n];
        b[r * N + n] = make_double2(om * j.y, -om * j.x);
    }
}

__global__ void fill_f32_kernel(float *p, long long n, float v) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// x (FP64) = x0 (FP32), or 0 when x0 is null
__global__ void widen_kernel(const float2 *x0, double2 *x, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        x[i] = x0 ? make_double2(x0[i].x, x0[i].y) : make_double2(0.0, 0.0);
}

__global__ void narrow_kernel(const double2 *x, float2 *e, long long n) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        e[i] = make_float2((float)x[i].x, (float)x[i].y);
}

long long grid_blocks(long long N) { return std::min<long long>(1024, (N + 255) / 256); }

// Profiling marks: begin/end a launch group of class c on the context stream.
int prof_mark(nosdd_problem *p) {
    if (p->ev_next == (int)p->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return -1;
        p->ev_pool.push_back(e);
    }
    const int i = p->ev_next++;
    (void)hipEventRecord(p->ev_pool[i], p->ctx->stream);
    return i;
}

struct ProfScope {
    nosdd_problem *p;
    int cls, start;
    ProfScope(nosdd_problem *p_, int c, long long units) : p(p_), cls(c), start(-1) {
        if (p->prof) {
            start = prof_mark(p);
            p->prof_launch[c] += 1;
            p->prof_units[c] += units;
        }
    }
    ~ProfScope() {
        if (p->prof && start >= 0) {
            const int stop = prof_mark(p);
            if (stop >= 0) p->ev_pending.push_back({cls, {start, stop}});
        }
    }
};

// Fold recorded event pairs into the per-class totals (the stream must be idle).
void prof_flush(nosdd_problem *p) {
    for (auto &pe : p->ev_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p->ev_pool[pe.second.first], p->ev_pool[pe.second.second]) == hipSuccess)
            p->prof_ms[pe.first] += ms;
    }
    p->ev_pending.clear();
    p->ev_next = 0;
}

nosdd_status ensure_ws(nosdd_problem *p, int n_rhs, int m, int max_iters) {
    Workspace &w = p->ws;
    nosdd_ctx *ctx = p->ctx;
    const long long N = (long long)p->nx * p->ny;
    // about 8 cells per thread and at least ~512 workgroups in all, at most 1024 per RHS
    long long nb = (N + 2047) / 2048;
    nb = std::max<long long>(nb, std::min<long long>((N + 255) / 256, (512 + n_rhs - 1) / n_rhs));
    const int nblk = (int)std::max<long long>(1, std::min<long long>(1024, nb));
    if (w.n_rhs != n_rhs || w.N != N || w.m != m) w.tuned = false;
    w.n_rhs = n_rhs;
    w.m = m;
    w.max_iters = max_iters;
    w.N = N;
    w.nblk = nblk;
    w.nblk_max = std::min(1024, 2 * nblk);
    if (!w.tuned)
        for (int &v : w.nblk_b) v = nblk;
    const size_t vec = (size_t)n_rhs * N * sizeof(float2);
    HIPCHK(ctx, w.x.ensure(vec * 2));        // FP64 iterate
    HIPCHK(ctx, w.b.ensure(vec));
    HIPCHK(ctx, w.b64.ensure(vec * 2));      // FP64 right-hand side of the restart residuals
    HIPCHK(ctx, w.w.ensure(vec));
    HIPCHK(ctx, w.V.ensure(vec * (m + 1)));
    HIPCHK(ctx, w.Z.ensure(vec * m));
    HIPCHK(ctx, w.partial.ensure((size_t)n_rhs * w.nblk_max * 33 * sizeof(double2)));
    const size_t hsz = (size_t)n_rhs * (m + 1) * m * sizeof(float2);
    HIPCHK(ctx, w.H.ensure(hsz));
    HIPCHK(ctx, w.H2.ensure(hsz));
    HIPCHK(ctx, w.G1.ensure(hsz));
    HIPCHK(ctx, w.T.ensure((size_t)n_rhs * (m + 1) * (m + 1) * sizeof(double2)));
    HIPCHK(ctx, w.scale.ensure((size_t)n_rhs * sizeof(float)));
    HIPCHK(ctx, w.cs.ensure((size_t)n_rhs * m * sizeof(float)));
    HIPCHK(ctx, w.sn.ensure((size_t)n_rhs * m * sizeof(float2)));
    HIPCHK(ctx, w.gam.ensure((size_t)n_rhs * (m + 1) * sizeof(float2)));
    HIPCHK(ctx, w.y.ensure((size_t)n_rhs * m * sizeof(float2)));
    for (DevBuf *d : {&w.nw_pre, &w.nw_post, &w.bnorm2, &w.beta2})
        HIPCHK(ctx, d->ensure((size_t)n_rhs * sizeof(double)));
    for (DevBuf *d : {&w.bnorm, &w.inv_h}) HIPCHK(ctx, d->ensure((size_t)n_rhs * sizeof(float)));
    for (DevBuf *d : {&w.iters, &w.kcyc, &w.active, &w.want, &w.reorth, &w.flags})
        HIPCHK(ctx, d->ensure((size_t)n_rhs * sizeof(int)));
    {
        const bool fresh = w.ones.bytes < (size_t)n_rhs * sizeof(int);
        HIPCHK(ctx, w.ones.ensure((size_t)n_rhs * sizeof(int)));
        if (fresh) {
            std::vector<int> one(n_rhs, 1);
            HIPCHK(ctx, hipMemcpy(w.ones.p, one.data(), n_rhs * sizeof(int), hipMemcpyHostToDevice));
        }
    }
    HIPCHK(ctx, w.hist.ensure((size_t)n_rhs * std::max(1, max_iters) * sizeof(float)));
    HIPCHK(ctx, w.loc.ensure((size_t)n_rhs * p->loc_total * sizeof(float2)));
    const int nc = std::max(1, p->n_c);
    HIPCHK(ctx, w.cd_.ensure((size_t)n_rhs * nc * sizeof(double2)));
    HIPCHK(ctx, w.cc_.ensure((size_t)n_rhs * nc * sizeof(float2)));
    HIPCHK(ctx, w.cstep.ensure((size_t)m * n_rhs * nc * sizeof(float2)));
    HIPCHK(ctx, w.cy.ensure((size_t)n_rhs * nc * sizeof(double2)));
    return NOSDD_OK;
}

// ---------------------------------------------------------------- neural subdomain solver
uint16_t bf16_of(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
float f32_of_bf16(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// Read the weights file ("NOSDDFNO", int32 header, bfloat16 tensors) into device
// buffers; R is expanded to the real 128 x 128 block form used by the MFMA mix.
nosdd_status load_network(nosdd_problem *p, const char *path) {
    nosdd_ctx *ctx = p->ctx;
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(ctx, NOSDD_ENOWEIGHTS, std::string("cannot open weights file ") + path);
    char magic[8];
    int32_t hdr[7], hdr2[4] = {0, 0, 0, 0};
    if (std::fread(magic, 1, 8, f) != 8 || std::memcmp(magic, "NOSDDFNO", 8) != 0 || std::fread(hdr, 4, 7, f) != 7 ||
        (hdr[0] == 2 && std::fread(hdr2, 4, 4, f) != 4)) {
        std::fclose(f);
        return fail(ctx, NOSDD_ENOWEIGHTS, "not a network weights file");
    }
    const int C = hdr[1], m = hdr[2], L = hdr[3], in_ch = hdr[4], hid = hdr[5];
    const int ver = hdr[0], rank = hdr2[0], mch = hdr2[1], mpool = hdr2[2], mhid = hdr2[3];
    if ((ver != 1 && ver != 2) || hdr[6] != 1 || C != 64 || m != 16 || in_ch != 9 || hid != 128 || L < 1 || L > 16 ||
        (ver == 2 && (rank < 1 || rank > 256 || mch < 1 || mch > 64 || mpool < 1 || mpool > 16 || mhid < 1 ||
                      mhid > 1024))) {
        std::fclose(f);
        return fail(ctx, NOSDD_ENOWEIGHTS, "weights file must hold a bf16 network of width 64, 16 modes, 9 inputs, "
                                           "projection 128 (version 1 plain, version 2 modulated low-rank)");
    }
    const size_t spec_per_layer = ver == 1 ? 2ull * (2 * m) * m * C * C
                                           : 2ull * (2 * m) * m * rank + 2ull * rank * C * C;
    const size_t per_layer = spec_per_layer + (size_t)C * C + C;
    const size_t mod_total = ver == 1 ? 0
                                      : (size_t)mch * 7 * 9 + mch + (size_t)mhid * mch * mpool * mpool + mhid +
                                            (size_t)L * 2 * m * m * 2 * mhid + (size_t)L * 2 * m * m * 2;
    const size_t total = (size_t)C * in_ch + C + L * per_layer + (size_t)hid * C + hid + 2ull * hid + 2 + mod_total;
    std::vector<uint16_t> w(total);
    const size_t got = std::fread(w.data(), 2, total, f);
    const bool extra = std::fgetc(f) != EOF;
    std::fclose(f);
    if (got != total || extra) return fail(ctx, NOSDD_ENOWEIGHTS, "weights file size does not match its header");
    size_t pos = 0;
    auto f32s = [&](size_t n) {
        std::vector<float> v(n);
        for (size_t i = 0; i < n; ++i) v[i] = f32_of_bf16(w[pos + i]);
        pos += n;
        return v;
    };
    std::vector<float> lift_w = f32s((size_t)C * in_ch), lift_b = f32s(C);
    const int nmodes = 2 * m * m;
    std::vector<uint16_t> R((size_t)L * nmodes * 128 * 128), Wb((size_t)L * C * C);
    std::vector<float> bias((size_t)L * C);
    std::vector<uint16_t> lr_expanded;                    // version 2: R = A B per layer, rounded to bf16
    for (int l = 0; l < L; ++l) {
        if (ver == 2) {
            // R[k][i][o] = sum_r A[k][r] B[r][i][o] (complex), in FP64, then rounded
            std::vector<double> Ar(nmodes * (size_t)rank), Ai(nmodes * (size_t)rank), Br((size_t)rank * C * C),
                Bi((size_t)rank * C * C);
            for (size_t i = 0; i < Ar.size(); ++i) Ar[i] = f32_of_bf16(w[pos + i]);
            pos += Ar.size();
            for (size_t i = 0; i < Ai.size(); ++i) Ai[i] = f32_of_bf16(w[pos + i]);
            pos += Ai.size();
            for (size_t i = 0; i < Br.size(); ++i) Br[i] = f32_of_bf16(w[pos + i]);
            pos += Br.size();
            for (size_t i = 0; i < Bi.size(); ++i) Bi[i] = f32_of_bf16(w[pos + i]);
            pos += Bi.size();
            lr_expanded.assign(2ull * nmodes * C * C, 0);
            std::vector<double> re((size_t)C * C), im((size_t)C * C);
            for (int md = 0; md < nmodes; ++md) {
                std::fill(re.begin(), re.end(), 0.0);
                std::fill(im.begin(), im.end(), 0.0);
                for (int r = 0; r < rank; ++r) {
                    const double a = Ar[(size_t)md * rank + r], b = Ai[(size_t)md * rank + r];
                    const double *br = &Br[(size_t)r * C * C], *bi = &Bi[(size_t)r * C * C];
                    for (int e = 0; e < C * C; ++e) {
                        re[e] += a * br[e] - b * bi[e];
                        im[e] += a * bi[e] + b * br[e];
                    }
                }
                for (int e = 0; e < C * C; ++e) {
                    lr_expanded[(size_t)md * C * C + e] = bf16_of((float)re[e]);
                    lr_expanded[(size_t)nmodes * C * C + (size_t)md * C * C + e] = bf16_of((float)im[e]);
                }
            }
        }
        const uint16_t *rr = ver == 2 ? lr_expanded.data() : &w[pos];
        const uint16_t *ri = rr + (size_t)nmodes * C * C;
        for (int md = 0; md < nmodes; ++md) {
            uint16_t *dst = &R[((size_t)l * nmodes + md) * 128 * 128];
            for (int i = 0; i < C; ++i)
                for (int o = 0; o < C; ++o) {
                    const uint16_t a = rr[((size_t)md * C + i) * C + o], b = ri[((size_t)md * C + i) * C + o];
                    // real form of the complex mix, rows (Re X_i, Im X_i) interleaved as
                    // 2i, 2i+1 and columns (Re Y_o, Im Y_o) as 2o, 2o+1
                    dst[(2 * i) * 128 + 2 * o] = a;
                    dst[(2 * i) * 128 + 2 * o + 1] = b;
                    dst[(2 * i + 1) * 128 + 2 * o] = (uint16_t)(b ^ 0x8000u);     // -Im R
                    dst[(2 * i + 1) * 128 + 2 * o + 1] = a;
                }
        }
        if (ver == 1) pos += 2ull * nmodes * C * C;
        std::memcpy(&Wb[(size_t)l * C * C], &w[pos], (size_t)C * C * 2);
        pos += (size_t)C * C;
        for (int o = 0; o < C; ++o) bias[(size_t)l * C + o] = f32_of_bf16(w[pos + o]);
        pos += C;
    }
    std::vector<uint16_t> p1w(w.begin() + pos, w.begin() + pos + (size_t)hid * C);
    pos += (size_t)hid * C;
    std::vector<float> p1b = f32s(hid), p2w = f32s(2ull * hid), p2b = f32s(2);
    p->mod_ch = p->mod_pool = p->mod_hidden = 0;
    if (ver == 2) {
        p->mod_ch = mch;
        p->mod_pool = mpool;
        p->mod_hidden = mhid;
        p->mod_cw = f32s((size_t)mch * 7 * 9);
        p->mod_cb = f32s(mch);
        p->mod_f1w = f32s((size_t)mhid * mch * mpool * mpool);
        p->mod_f1b = f32s(mhid);
        p->mod_f2w = f32s((size_t)L * nmodes * 2 * mhid);
        p->mod_f2b = f32s((size_t)L * nmodes * 2);
    }
    // truncated-DFT twiddle tables for every subdomain side L <= 72 (FP64 on the host)
    std::vector<float2> tw((size_t)FNO_TW_UNIT * FNO_MAXL * (FNO_MAXL + 1) / 2);
    for (int L = 1; L <= FNO_MAXL; ++L) {
        float2 *base = &tw[(size_t)FNO_TW_UNIT * L * (L - 1) / 2];
        auto kx = [&](int q) { return q < m ? q : L - 2 * m + q; };
        auto ph = [&](long long k, int i, double sign) {
            const double a = sign * 2.0 * M_PI * (double)((k * i) % L) / (double)L;
            return make_float2((float)std::cos(a), (float)std::sin(a));
        };
        for (int i = 0; i < L; ++i)
            for (int q = 0; q < 2 * m; ++q) {
                base[i * 2 * m + q] = ph(kx(q), i, -1.0);                   // forward, [x][q]
                base[FNO_TW_INV_X * L + q * L + i] = ph(kx(q), i, 1.0);     // inverse, [q][x]
            }
        for (int i = 0; i < L; ++i)
            for (int q = 0; q < m; ++q) {
                base[FNO_TW_FWD_Y * L + i * m + q] = ph(q, i, -1.0);       // forward, [y][ky]
                base[FNO_TW_INV_Y * L + i * m + q] = ph(q, i, 1.0);        // inverse, [y][ky]
            }
    }
    // the x-transforms' real 2 x 2 forms split into BF16 high and low parts
    // (from the FP64 values), the B operands of their BF16 MFMA contractions
    std::vector<unsigned short> twb((size_t)128 * FNO_MAXL * (FNO_MAXL + 1));
    std::vector<unsigned short> twf((size_t)2 * 64 * FNO_TWF_K * FNO_MAXL, 0);
    {
        auto bf = [](double v) {
            const float f = (float)v;
            unsigned u;
            std::memcpy(&u, &f, 4);
            u += 0x7FFFu + ((u >> 16) & 1u);       // round to nearest even
            return (unsigned short)(u >> 16);
        };
        auto val = [](unsigned short b) {
            const unsigned u = (unsigned)b << 16;
            float f;
            std::memcpy(&f, &u, 4);
            return (double)f;
        };
        for (int L = 1; L <= FNO_MAXL; ++L) {
            // forward x: [n = (q, ro)][k = (x, ri)], e^{-2 pi i kx x / L}
            unsigned short *fh = &twf[(size_t)2 * 64 * FNO_TWF_K * (L - 1)], *fl = fh + (size_t)64 * FNO_TWF_K;
            for (int x = 0; x < L; ++x)
                for (int q = 0; q < 2 * m; ++q) {
                    const int k = q < m ? q : L - 2 * m + q;
                    const double a = -2.0 * M_PI * (double)(((long long)k * x) % L) / (double)L;
                    const double c = std::cos(a), sn = std::sin(a);
                    const double e[2][2] = {{c, sn}, {-sn, c}};              // [Re/Im in][Re/Im out]
                    for (int ri = 0; ri < 2; ++ri)
                        for (int ro = 0; ro < 2; ++ro) {
                            const size_t i = (size_t)(2 * q + ro) * FNO_TWF_K + 2 * x + ri;
                            fh[i] = bf(e[ri][ro]);
                            fl[i] = bf(e[ri][ro] - val(fh[i]));
                        }
                }
            // inverse x: [n = (x, ro)][k = (q, ri)], e^{+2 pi i kx x / L}
            unsigned short *hi = &twb[(size_t)128 * L * (L - 1)], *lo = hi + (size_t)2 * L * 64;
            for (int x = 0; x < L; ++x)
                for (int q = 0; q < 2 * m; ++q) {
                    const int k = q < m ? q : L - 2 * m + q;
                    const double a = 2.0 * M_PI * (double)(((long long)k * x) % L) / (double)L;
                    const double c = std::cos(a), sn = std::sin(a);
                    const double e[2][2] = {{c, sn}, {-sn, c}};              // [Re/Im in][Re/Im out]
                    for (int ri = 0; ri < 2; ++ri)
                        for (int ro = 0; ro < 2; ++ro) {
                            const size_t i = (size_t)(2 * x + ro) * 64 + 2 * q + ri;
                            hi[i] = bf(e[ri][ro]);
                            lo[i] = bf(e[ri][ro] - val(hi[i]));
                        }
                }
        }
    }
    // one device buffer, carved
    const size_t bytes = (lift_w.size() + lift_b.size() + bias.size() + p1b.size() + p2w.size() + p2b.size()) * 4 +
                         (R.size() + Wb.size() + p1w.size()) * 2 + tw.size() * sizeof(float2) + twb.size() * 2 +
                         twf.size() * 2 + 11 * 256;
    HIPCHK(ctx, p->d_net.ensure(bytes));
    char *base = p->d_net.as<char>();
    size_t off = 0;
    hipStream_t st = ctx->stream;
    auto put = [&](const void *src, size_t nb) -> void * {
        void *dst = base + off;
        off += (nb + 255) / 256 * 256;
        (void)hipMemcpyAsync(dst, src, nb, hipMemcpyHostToDevice, st);
        return dst;
    };
    FnoDevice &n = p->net;
    n.layers = L;
    n.lift_w = (float *)put(lift_w.data(), lift_w.size() * 4);
    n.lift_b = (float *)put(lift_b.data(), lift_b.size() * 4);
    n.R = (unsigned short *)put(R.data(), R.size() * 2);
    n.W = (unsigned short *)put(Wb.data(), Wb.size() * 2);
    n.b = (float *)put(bias.data(), bias.size() * 4);
    n.p1w = (unsigned short *)put(p1w.data(), p1w.size() * 2);
    n.p1b = (float *)put(p1b.data(), p1b.size() * 4);
    n.p2w = (float *)put(p2w.data(), p2w.size() * 4);
    n.p2b = (float *)put(p2b.data(), p2b.size() * 4);
    n.tw = (float2 *)put(tw.data(), tw.size() * sizeof(float2));
    n.twb = (unsigned short *)put(twb.data(), twb.size() * 2);
    n.twf = (unsigned short *)put(twf.data(), twf.size() * 2);
    HIPCHK(ctx, hipStreamSynchronize(st));
    return NOSDD_OK;
}

// Constant network inputs per (wavelength, subdomain): (eps-1)/11, k0 h sqrt(eps),
// Re/Im 1/s_x, Re/Im 1/s_y (cell-centre stretches of the global PML), ring mask.
nosdd_status build_aux(nosdd_problem *p) {
    nosdd_ctx *ctx = p->ctx;
    const int nwl = (int)p->wl.size(), nx = p->nx, ny = p->ny;
    const long long LT = p->loc_total;
    std::vector<float> aux((size_t)nwl * 7 * LT, 0.f);
    for (int wi = 0; wi < nwl; ++wi) {
        const double k0 = 2.0 * M_PI / p->wl[wi];
        const double sh = p->npml ? (p->pml_m + 1) * (-p->lnR) / (2.0 * k0 * p->npml * p->h) : 0.0;
        for (auto &t : p->tiles) {
            const int lx = t.x1 - t.x0, ly = t.y1 - t.y0;
            for (int yy = 0; yy < ly; ++yy)
                for (int xx = 0; xx < lx; ++xx) {
                    const int x = t.x0 + xx, y = t.y0 + yy;
                    const double e = p->eps[(size_t)y * nx + x];
                    const cd isx = 1.0 / stretch(x, nx, p->npml, p->pml_m, sh);
                    const cd isy = 1.0 / stretch(y, ny, p->npml, p->pml_m, sh);
                    const bool ring = ((t.iface & SIDE_LEFT) && xx == 0) || ((t.iface & SIDE_RIGHT) && xx == lx - 1) ||
                                      ((t.iface & SIDE_BOTTOM) && yy == 0) || ((t.iface & SIDE_TOP) && yy == ly - 1);
                    const float v[7] = {(float)((e - 1.0) / 11.0), (float)(k0 * p->h * std::sqrt(e)),
                                        (float)isx.real(), (float)isx.imag(), (float)isy.real(), (float)isy.imag(),
                                        ring ? 1.f : 0.f};
                    const long long c = t.loc_off + (long long)yy * lx + xx;
                    for (int k = 0; k < 7; ++k) aux[((size_t)wi * 7 + k) * LT + c] = v[k];
                }
        }
    }
    HIPCHK(ctx, p->d_aux.ensure(aux.size() * 4));
    HIPCHK(ctx, hipMemcpyAsync(p->d_aux.p, aux.data(), aux.size() * 4, hipMemcpyHostToDevice, ctx->stream));
    p->net.mod = nullptr;
    if (p->mod_ch > 0) {
        // modulation tensors of the modulated network, one set per (wavelength,
        // subdomain): they depend on the auxiliary channels only (Fig. 2
        // modulation path), so they are formed once here, in FP64
        const int nt = (int)p->tiles.size(), L = p->net.layers, mc = p->mod_ch, P = p->mod_pool, mh = p->mod_hidden;
        const int nout = L * FNO_MODES_TOTAL * 2;
        std::vector<float2> mod((size_t)nwl * nt * L * FNO_MODES_TOTAL);
        std::vector<double> h, pool((size_t)mc * P * P), fh(mh);
        for (int wi = 0; wi < nwl; ++wi)
            for (int ti = 0; ti < nt; ++ti) {
                const TileDesc &t = p->tiles[ti];
                const int lx = t.x1 - t.x0, ly = t.y1 - t.y0;
                auto a = [&](int k, int y, int x) -> double {
                    if (x < 0 || x >= lx || y < 0 || y >= ly) return 0.0;
                    return aux[((size_t)wi * 7 + k) * LT + t.loc_off + (long long)y * lx + x];
                };
                h.assign((size_t)mc * ly * lx, 0.0);
                for (int c = 0; c < mc; ++c)
                    for (int y = 0; y < ly; ++y)
                        for (int x = 0; x < lx; ++x) {
                            double acc = p->mod_cb[c];
                            for (int k = 0; k < 7; ++k)
                                for (int dy = 0; dy < 3; ++dy)
                                    for (int dx = 0; dx < 3; ++dx)
                                        acc += (double)p->mod_cw[((c * 7 + k) * 3 + dy) * 3 + dx] * a(k, y + dy - 1, x + dx - 1);
                            h[((size_t)c * ly + y) * lx + x] = acc >= 0 ? acc : 0.01 * acc;
                        }
                for (int c = 0; c < mc; ++c)
                    for (int py = 0; py < P; ++py)
                        for (int px = 0; px < P; ++px) {
                            const int y0 = py * ly / P, y1 = (py + 1) * ly / P, x0 = px * lx / P, x1 = (px + 1) * lx / P;
                            double acc = 0.0;
                            for (int y = y0; y < y1; ++y)
                                for (int x = x0; x < x1; ++x) acc += h[((size_t)c * ly + y) * lx + x];
                            pool[((size_t)c * P + py) * P + px] = acc / ((double)(y1 - y0) * (x1 - x0));
                        }
                for (int j = 0; j < mh; ++j) {
                    double acc = p->mod_f1b[j];
                    for (int k = 0; k < mc * P * P; ++k) acc += (double)p->mod_f1w[(size_t)j * mc * P * P + k] * pool[k];
                    fh[j] = acc >= 0 ? acc : 0.01 * acc;
                }
                float2 *out = &mod[((size_t)wi * nt + ti) * L * FNO_MODES_TOTAL];
                for (int n = 0; n < nout / 2; ++n) {
                    double re = p->mod_f2b[2 * n], im = p->mod_f2b[2 * n + 1];
                    for (int j = 0; j < mh; ++j) {
                        re += (double)p->mod_f2w[(size_t)(2 * n) * mh + j] * fh[j];
                        im += (double)p->mod_f2w[(size_t)(2 * n + 1) * mh + j] * fh[j];
                    }
                    out[n] = make_float2((float)(1.0 + re), (float)im);      // n = (layer, kx, ky)
                }
            }
        HIPCHK(ctx, p->d_mod.ensure(mod.size() * sizeof(float2)));
        HIPCHK(ctx, hipMemcpyAsync(p->d_mod.p, mod.data(), mod.size() * sizeof(float2), hipMemcpyHostToDevice,
                                   ctx->stream));
        p->net.mod = p->d_mod.as<float2>();
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return NOSDD_OK;
}

// Sample descriptors and inner-solver workspace for n_rhs right-hand sides.
nosdd_status ensure_nn(nosdd_problem *p, int n_rhs, int n_src) {
    nosdd_ctx *ctx = p->ctx;
    const int nt = (int)p->tiles.size();
    const int S = n_rhs * nt;
    const long long LT = p->loc_total;
    if (p->smp_rhs != n_rhs) {
        std::vector<FnoSample> smp(S);
        for (int r = 0; r < n_rhs; ++r)
            for (int t = 0; t < nt; ++t) {
                const TileDesc &T = p->tiles[t];
                FnoSample &q = smp[(size_t)r * nt + t];
                q.lx = T.x1 - T.x0;
                q.ly = T.y1 - T.y0;
                q.cell_off = (long long)r * LT + T.loc_off;
                q.aux_off = (long long)(r / n_src) * 7 * LT + T.loc_off;
                q.mod_idx = (r / n_src) * nt + t;
                q.pad_ = 0;
            }
        HIPCHK(ctx, p->d_smp.ensure(smp.size() * sizeof(FnoSample)));
        HIPCHK(ctx, hipMemcpy(p->d_smp.p, smp.data(), smp.size() * sizeof(FnoSample), hipMemcpyHostToDevice));
        p->smp_rhs = n_rhs;
    }
    const int K = p->nn_steps;
    const size_t vec = (size_t)n_rhs * LT * sizeof(float2);
    HIPCHK(ctx, p->nn_Vin.ensure(vec * (K + 1)));
    HIPCHK(ctx, p->nn_Zin.ensure(vec * K));
    HIPCHK(ctx, p->nn_w.ensure(vec));
    for (DevBuf *d : {&p->nn_beta, &p->nn_vs, &p->nn_os}) HIPCHK(ctx, d->ensure((size_t)S * 4));
    for (DevBuf *d : {&p->nn_sact, &p->nn_kstep}) HIPCHK(ctx, d->ensure((size_t)S * 4));
    HIPCHK(ctx, p->nn_cs.ensure((size_t)S * K * 4));
    HIPCHK(ctx, p->nn_sn.ensure((size_t)S * K * 8));
    HIPCHK(ctx, p->nn_gam.ensure((size_t)S * (K + 1) * 8));
    HIPCHK(ctx, p->nn_H.ensure((size_t)S * (K + 1) * K * 8));
    const size_t actb = (size_t)n_rhs * LT * 64 * 4;
    HIPCHK(ctx, p->nn_act0.ensure(actb));
    HIPCHK(ctx, p->nn_act1.ensure(actb));
    HIPCHK(ctx, p->nn_spec.ensure(actb));
    HIPCHK(ctx, p->nn_X.ensure((size_t)512 * S * 128 * 4));
    HIPCHK(ctx, p->nn_Y.ensure((size_t)512 * S * 128 * 4));
    HIPCHK(ctx, p->nn_fb.ensure((size_t)S * sizeof(int)));
    HIPCHK(ctx, p->nn_fborder.ensure((size_t)S * sizeof(int2)));
    if (!p->nn_fbcount.p) {
        HIPCHK(ctx, p->nn_fbcount.ensure(sizeof(unsigned)));
        HIPCHK(ctx, hipMemset(p->nn_fbcount.p, 0, sizeof(unsigned)));
    }
    NnWork &nw = p->nw;
    nw.net = &p->net;
    nw.smp = p->d_smp.as<FnoSample>();
    nw.steps = K;
    nw.maxk = K;
    nw.tol = p->nn_tol;
    nw.Vin = p->nn_Vin.as<float2>();
    nw.Zin = p->nn_Zin.as<float2>();
    nw.w = p->nn_w.as<float2>();
    nw.beta = p->nn_beta.as<float>();
    nw.vscale = p->nn_vs.as<float>();
    nw.oscale = p->nn_os.as<float>();
    nw.cs = p->nn_cs.as<float>();
    nw.sact = p->nn_sact.as<int>();
    nw.kstep = p->nn_kstep.as<int>();
    nw.gam = p->nn_gam.as<float2>();
    nw.H = p->nn_H.as<float2>();
    nw.sn = p->nn_sn.as<float2>();
    nw.aux = p->d_aux.as<float>();
    nw.act0 = p->nn_act0.as<float>();
    nw.act1 = p->nn_act1.as<float>();
    nw.spec = p->nn_spec.as<float>();
    nw.X = p->nn_X.as<float>();
    nw.Y = p->nn_Y.as<float>();
    nw.fb = p->nn_fb.as<int>();
    nw.fb_order = p->nn_fborder.as<int2>();
    nw.fb_count = p->nn_fbcount.as<unsigned>();
    return NOSDD_OK;
}

// Inner NN-FGMRES on every (tile, RHS) sample, then the exact block-Thomas
// solve of the samples it queued as failed (global or subdomain-local vectors
// as in nn_precond; n_rhs * n_tiles fallback jobs, most of them empty).
void nn_sweep(nosdd_problem *p, hipStream_t s, const float2 *v, float2 *z, int n_rhs, int n_src, const int *active,
              int local) {
    const long long N = (long long)p->nx * p->ny;
    const int nt = (int)p->tiles.size();
    nn_precond(s, p->nw, p->d_tiles.as<TileDesc>(), nt, n_rhs, n_src, p->loc_total, p->max_cells, v, z, active,
               p->d_eps.as<float>(), p->d_coefd.as<double2>(), p->d_k0.as<double>(), p->h, p->nx, p->ny, local);
    const long long stride = local ? p->loc_total : N;
    launch_bt_solve(s, p->d_tiles.as<TileDesc>(), p->nw.fb_order, n_rhs * nt, n_src, p->d_dinv.as<float2>(),
                    p->dinv_wl_stride, p->d_coef.as<float2>(), p->d_sc.as<float2>(), p->nx, p->ny, v, stride, z, stride,
                    active, local ? 3 : 0, p->bmax, p->max_cells, p->bt_depth);
}

// Launch queue of the batched subdomain solve.  Jobs (tile, rhs) are grouped by
// the factorisation they stream (tile, wavelength), groups ordered largest
// tile first and dealt round-robin to eight queues, one per XCD: workgroup i
// of a launch is placed on XCD i mod 8, so the right-hand sides that share a
// factorisation run on one XCD and share its L2.  Queues are padded with
// (-1, -1) to equal length.  Built once per (n_rhs, n_src), outside any
// graph capture.
// Sources that share a wavelength are solved together (one factor stream,
// MFMA products) from 4 sources per wavelength on, for blocks up to 112 wide
// (LDS of the expanded block and operands).
// The many-source kernel addresses the vectors of one group of sources (at
// most 32) through buffer resources with 32-bit byte offsets: each group's
// range must stay below 2^31 bytes (grids and workspaces up to 2^23 cells).
bool use_multi(const nosdd_problem *p, int n_src) {
    const long long span = 32LL * std::max((long long)p->nx * p->ny, (long long)p->loc_total) * 8;
    return n_src >= 4 && p->bmax <= 112 && p->use_multi && span < (1LL << 31);
}

nosdd_status solve_order(nosdd_problem *p, int n_rhs, int n_src, const int2 **order, int *n_jobs) {
    auto key = std::make_pair(n_rhs, n_src);
    auto it = p->orders.find(key);
    if (it == p->orders.end()) {
        const int nt = (int)p->tiles.size(), nwl = n_rhs / n_src;
        std::vector<std::pair<int, int>> groups;              // (tile, wavelength)
        for (int w = 0; w < nwl; ++w)
            for (int t = 0; t < nt; ++t) groups.push_back({t, w});
        auto cells = [&](int t) { return (p->tiles[t].x1 - p->tiles[t].x0) * (p->tiles[t].y1 - p->tiles[t].y0); };
        std::stable_sort(groups.begin(), groups.end(),
                         [&](const std::pair<int, int> &a, const std::pair<int, int> &b) { return cells(a.first) > cells(b.first); });
        constexpr int NXCD = 8;
        std::vector<std::vector<int2>> q(NXCD);
        for (size_t g = 0; g < groups.size(); ++g)
            for (int sidx = 0; sidx < n_src; ++sidx)
                q[g % NXCD].push_back(make_int2(groups[g].first, groups[g].second * n_src + sidx));
        size_t len = 0;
        for (auto &v : q) len = std::max(len, v.size());
        std::vector<int2> ord(len * NXCD, make_int2(-1, -1));
        for (size_t slot = 0; slot < len; ++slot)
            for (int x = 0; x < NXCD; ++x)
                if (slot < q[x].size()) ord[slot * NXCD + x] = q[x][slot];
        auto &ob = p->orders[key];
        HIPCHK(p->ctx, ob.buf.ensure(ord.size() * sizeof(int2)));
        HIPCHK(p->ctx, hipMemcpy(ob.buf.p, ord.data(), ord.size() * sizeof(int2), hipMemcpyHostToDevice));
        ob.n_jobs = (int)ord.size();
        if (use_multi(p, n_src)) {
            // one job per (tile, wavelength, group of sources), largest tiles first;
            // the group width follows the tile's block size
            std::vector<int4> mj;
            for (const auto &g : groups) {
                const int ncol = bt_multi_cols(p->tiles[g.first].b);
                for (int s0 = 0; s0 < n_src; s0 += ncol) mj.push_back(make_int4(g.first, g.second, s0, std::min(ncol, n_src - s0)));
            }
            HIPCHK(p->ctx, ob.mbuf.ensure(mj.size() * sizeof(int4)));
            HIPCHK(p->ctx, hipMemcpy(ob.mbuf.p, mj.data(), mj.size() * sizeof(int4), hipMemcpyHostToDevice));
            ob.n_mjobs = (int)mj.size();
        }
        it = p->orders.find(key);
    }
    *order = it->second.buf.as<int2>();
    *n_jobs = it->second.n_jobs;
    return NOSDD_OK;
}

// z = sum_i Rt_i^T B_i^-1 R_i v (exact local solves, global in and out) for
// n_rhs vectors, n_src per wavelength; the launch queue must exist
// (solve_order) and, for grouped sources, the workspace's packed local buffer.
void local_sweep(nosdd_problem *p, hipStream_t s, const float2 *v, float2 *z, int n_rhs, int n_src,
                 const int *active) {
    const long long N = (long long)p->nx * p->ny;
    const auto &ob = p->orders.at(std::make_pair(n_rhs, n_src));
    if (ob.n_mjobs > 0)
        launch_bt_solve_multi(s, p->d_tiles.as<TileDesc>(), ob.mbuf.as<int4>(), ob.n_mjobs, n_src,
                              p->d_dinv.as<float2>(), p->dinv_wl_stride, p->d_coef.as<float2>(), p->d_sc.as<float2>(),
                              p->nx, p->ny, v, N, z, N, active, p->ws.loc.as<float2>(), p->loc_total, p->bmax);
    else
        launch_bt_solve(s, p->d_tiles.as<TileDesc>(), ob.buf.as<int2>(), ob.n_jobs, n_src, p->d_dinv.as<float2>(),
                        p->dinv_wl_stride, p->d_coef.as<float2>(), p->d_sc.as<float2>(), p->nx, p->ny, v, N, z, N,
                        active, 0, p->bmax, p->max_cells, p->bt_depth);
}

// z = M^-1 v (two-level), wout = A z.  v, z, wout: [n_rhs][N].  With c_store
// the coarse coefficients go there and z keeps only the one-level part (the
// caller adds Phi c later); wout is the full A z either way.
void precond(nosdd_problem *p, hipStream_t s, const float2 *v, float2 *z, float2 *wout, int n_src, int n_rhs,
             const int *active, int n_live, float2 *c_store = nullptr) {
    Workspace &w = p->ws;
    const long long N = (long long)p->nx * p->ny;
    {
    ProfScope ps(p, 0, (long long)n_live * (long long)p->tiles.size());
    if (p->sub_solver == 1) {
        nn_sweep(p, s, v, z, n_rhs, n_src, active, 0);
    } else
    local_sweep(p, s, v, z, n_rhs, n_src, active);
    }
    if (wout == nullptr) return;
    {
        ProfScope ps(p, 1, n_live);
        launch_stencil(s, z, nullptr, wout, p->d_eps.as<float>(), p->d_coefd.as<double2>(), p->d_k0.as<double>(),
                       p->nx, p->ny, n_rhs, n_src, active);
    }
    if (p->n_c > 0) {
        ProfScope ps(p, 3, n_live);
        launch_coarse_dot(s, p->d_tiles.as<TileDesc>(), p->n_c, p->kc, p->d_W.as<float2>(), p->box_wl_stride, v,
                          wout, p->nx, N, n_rhs, n_src, active, w.cd_.as<double2>());
        float2 *cc = c_store ? c_store : w.cc_.as<float2>();
        launch_coarse_solve(s, p->d_GinvT.as<double2>(), p->n_c, w.cd_.as<double2>(), cc, n_rhs, n_src, active);
        launch_coarse_update(s, p->d_tiles.as<TileDesc>(), p->d_owner.as<int>(), p->kc, p->d_phi.as<float2>(),
                             p->d_W.as<float2>(), p->box_wl_stride, cc, p->n_c, c_store ? nullptr : z, wout, p->nx, p->ny,
                             n_rhs, n_src, active);
    }
}

// ---------------------------------------------------------------- coarse set-up
// Pseudo-plane-wave probe Robin data of one tile (ne x K, row-major), made
// orthonormal by modified Gram-Schmidt; *n_kept independent columns come first,
// the rest are zero.  The phase is accumulated along the
// counter-clockwise boundary ring with the local wavenumber k0 sqrt(eps).
std::vector<cd> build_probes(const TileDesc &t, const std::vector<int4> &ent, const float *eps, int nx, double k0,
                             double h, int K, int *n_kept) {
    const int ne = (int)ent.size();
    std::vector<std::pair<int, int>> nodes;
    ring_nodes(t, nodes);
    std::vector<double> kap(nodes.size());
    for (size_t r = 0; r < nodes.size(); ++r)
        kap[r] = k0 * std::sqrt((double)eps[(size_t)nodes[r].second * nx + nodes[r].first]);
    std::vector<cd> Xe((size_t)ne * K);
    for (int l = 0; l < K; ++l) {
        const double th = 2.0 * M_PI * l / K;
        const double dx = std::cos(th), dy = std::sin(th);
        std::vector<double> phi(nodes.size(), 0.0);
        for (size_t r = 0; r + 1 < nodes.size(); ++r) {
            const double sx = nodes[r + 1].first - nodes[r].first, sy = nodes[r + 1].second - nodes[r].second;
            phi[r + 1] = phi[r] + h * 0.5 * (kap[r] + kap[r + 1]) * (dx * sx + dy * sy);
        }
        for (int e = 0; e < ne; ++e) Xe[(size_t)e * K + l] = std::exp(cd(0.0, -phi[ent[e].w]));
    }
    // modified Gram-Schmidt; a probe whose residual falls below 1e-8 of its
    // norm is dependent and removed, the kept ones are packed first
    std::vector<cd> Q((size_t)ne * K, cd(0, 0));
    int kept = 0;
    for (int l = 0; l < K; ++l) {
        std::vector<cd> v(ne);
        double n0 = 0;
        for (int e = 0; e < ne; ++e) {
            v[e] = Xe[(size_t)e * K + l];
            n0 += std::norm(v[e]);
        }
        for (int q = 0; q < kept; ++q) {
            cd dot = 0;
            for (int e = 0; e < ne; ++e) dot += std::conj(Q[(size_t)e * K + q]) * v[e];
            for (int e = 0; e < ne; ++e) v[e] -= dot * Q[(size_t)e * K + q];
        }
        double nr = 0;
        for (int e = 0; e < ne; ++e) nr += std::norm(v[e]);
        if (!(std::sqrt(nr) > 1e-8 * std::sqrt(n0))) continue;
        nr = std::sqrt(nr);
        for (int e = 0; e < ne; ++e) Q[(size_t)e * K + kept] = v[e] / nr;
        ++kept;
    }
    *n_kept = kept;
    Xe.swap(Q);
    return Xe;
}

nosdd_status coarse_setup(nosdd_problem *p) {
    nosdd_ctx *ctx = p->ctx;
    hipStream_t s = ctx->stream;
    const int nt = (int)p->tiles.size();
    const int K = std::max(p->ktrial, p->kc);
    const int kc = p->kc;
    const int nwl = (int)p->wl.size();
    const int nx = p->nx, ny = p->ny;
    const double h = p->h;
    p->n_c = nt * kc;
    // box geometry
    long long box_total = 0;
    for (auto &t : p->tiles) {
        t.bx0 = std::max(t.cx0 - 1, 0);
        t.by0 = std::max(t.cy0 - 1, 0);
        t.bw = std::min(t.cx1 + 1, nx) - t.bx0;
        t.bh = std::min(t.cy1 + 1, ny) - t.by0;
        t.box_off = (int)box_total;
        box_total += (long long)kc * t.bw * t.bh;
    }
    p->box_wl_stride = box_total;
    HIPCHK(ctx, hipMemcpyAsync(p->d_tiles.p, p->tiles.data(), p->tiles.size() * sizeof(TileDesc),
                               hipMemcpyHostToDevice, s));
    // probe Robin data per (wl, probe), injected into packed local vectors
    const long long LT = p->loc_total;
    std::vector<std::vector<cd>> Xt((size_t)nwl * nt);
    std::vector<int> Kt((size_t)nwl * nt, 0);
    std::vector<float2> rhs((size_t)nwl * K * LT, make_float2(0.f, 0.f));
    for (int wi = 0; wi < nwl; ++wi) {
        const double k0 = 2.0 * M_PI / p->wl[wi];
        const auto &cf = p->coefd[wi];
        for (int ti = 0; ti < nt; ++ti) {
            const TileDesc &t = p->tiles[ti];
            const auto &ent = p->tile_entries[ti];
            const int ne = (int)ent.size();
            int kept = 0;
            std::vector<cd> Xe = build_probes(t, ent, p->eps.data(), nx, k0, h, K, &kept);
            Kt[(size_t)wi * nt + ti] = kept;
            // inj(g)_p = -a_pq tau_p g_p
            for (int e = 0; e < ne; ++e) {
                const int pc = ent[e].x, px = pc % nx, py = pc / nx;
                cd apq;
                switch (ent[e].z) {
                    case SIDE_LEFT: apq = cf[px]; break;
                    case SIDE_RIGHT: apq = cf[nx + px]; break;
                    case SIDE_BOTTOM: apq = cf[2 * nx + py]; break;
                    default: apq = cf[2 * nx + ny + py]; break;
                }
                const double kp = k0 * std::sqrt((double)p->eps[pc]);
                const cd tau = h / cd(1.0, 0.5 * kp * h);
                const long long li = t.loc_off + (long long)(py - t.y0) * (t.x1 - t.x0) + (px - t.x0);
                for (int l = 0; l < K; ++l) {
                    const cd v = -apq * tau * Xe[(size_t)e * K + l];
                    float2 &dst = rhs[((size_t)wi * K + l) * LT + li];
                    dst.x += (float)v.real();
                    dst.y += (float)v.imag();
                }
            }
            Xt[(size_t)wi * nt + ti] = std::move(Xe);
        }
    }
    // batched homogeneous probe solves on the GPU: F = B^-1 inj(X)
    DevBuf d_rhs, d_F;
    const size_t bytes = rhs.size() * sizeof(float2);
    HIPCHK(ctx, d_rhs.ensure(bytes));
    HIPCHK(ctx, d_F.ensure(bytes));
    HIPCHK(ctx, hipMemcpyAsync(d_rhs.p, rhs.data(), bytes, hipMemcpyHostToDevice, s));
    {
        const int2 *ord = nullptr;
        int nj = 0;
        nosdd_status so = solve_order(p, nwl * K, K, &ord, &nj);
        if (so != NOSDD_OK) return so;
        launch_bt_solve(s, p->d_tiles.as<TileDesc>(), ord, nj, K, p->d_dinv.as<float2>(), p->dinv_wl_stride,
                        p->d_coef.as<float2>(), p->d_sc.as<float2>(), nx, ny, d_rhs.as<float2>(), LT, d_F.as<float2>(), LT, nullptr, 3,
                        p->bmax, p->max_cells);
    }
    std::vector<float2> F(rhs.size());
    HIPCHK(ctx, hipMemcpyAsync(F.data(), d_F.p, bytes, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));

    // per tile: neighbour traces, SVD (through Y^H Y), basis fields, W = A Phi
    std::vector<float2> phi_h((size_t)nwl * box_total), W_h((size_t)nwl * box_total);
    std::vector<std::vector<cd>> Wd((size_t)nwl * nt);   // FP64 W boxes for G
    const int nc = p->n_c;
    std::vector<double2> ginv_dev((size_t)nwl * nc * nc);
    // Robin-space coarse space (Algorithm 3 loop): per wavelength, the nonzeros
    // (entry, column, Q value, T Q value) in column order
    struct RcNz {
        int e, col;
        cd q, tq;
    };
    std::vector<std::vector<RcNz>> rcnz((size_t)nwl);
    for (int wi = 0; wi < nwl; ++wi) {
        const double k0 = 2.0 * M_PI / p->wl[wi];
        const auto &cf = p->coefd[wi];
        const cd *cxm = cf.data(), *cxp = cf.data() + nx, *cym = cf.data() + 2 * nx, *cyp = cf.data() + 2 * nx + ny;
        for (int ti = 0; ti < nt; ++ti) {
            const TileDesc &t = p->tiles[ti];
            const int lx = t.x1 - t.x0;
            auto Fv = [&](int l, int x, int y) -> cd {
                const float2 f = F[((size_t)wi * K + l) * LT + t.loc_off + (long long)(y - t.y0) * lx + (x - t.x0)];
                return cd(f.x, f.y);
            };
            // rows of Y: traces on neighbours' ring entries lying inside this tile
            const int Kk = Kt[(size_t)wi * nt + ti];
            std::vector<cd> Y;
            int nrows = 0;
            for (const int tj : p->nbrs[ti])
                for (const int4 &e : p->tile_entries[tj]) {
                    const int px = e.x % nx, py = e.x / nx, qx = e.y % nx, qy = e.y / nx;
                    if (px < t.x0 || px >= t.x1 || py < t.y0 || py >= t.y1) continue;
                    if (qx < t.x0 || qx >= t.x1 || qy < t.y0 || qy >= t.y1) continue;
                    const double kp = k0 * std::sqrt((double)p->eps[e.x]);
                    for (int l = 0; l < Kk; ++l) {
                        const cd up = Fv(l, px, py), uq = Fv(l, qx, qy);
                        Y.push_back((uq - up) / h + cd(0.0, 0.5 * kp) * (uq + up));
                    }
                    ++nrows;
                }
            // right singular vectors of Y = eigenvectors of Y^H Y, by decreasing eigenvalue
            std::vector<cd> YhY((size_t)Kk * Kk, cd(0, 0));
            for (int rr = 0; rr < nrows; ++rr)
                for (int a = 0; a < Kk; ++a)
                    for (int bb = 0; bb < Kk; ++bb)
                        YhY[(size_t)a * Kk + bb] += std::conj(Y[(size_t)rr * Kk + a]) * Y[(size_t)rr * Kk + bb];
            std::vector<double> ev;
            std::vector<cd> Vv;
            herm_eig(Kk, YhY, ev, Vv);
            std::vector<int> order(Kk);
            for (int i = 0; i < Kk; ++i) order[i] = i;
            std::stable_sort(order.begin(), order.end(), [&](int a, int bb) { return ev[a] > ev[bb]; });
            // basis fields on the core, stored on the box (core grown by one cell)
            const int bw = t.bw, bh = t.bh;
            std::vector<cd> phib((size_t)kc * bw * bh, cd(0, 0)), wb((size_t)kc * bw * bh, cd(0, 0));
            for (int l = 0; l < std::min(kc, Kk); ++l) {     // columns beyond Kk stay zero
                const int col = order[l];
                for (int y = t.cy0; y < t.cy1; ++y)
                    for (int x = t.cx0; x < t.cx1; ++x) {
                        cd v = 0;
                        for (int q = 0; q < Kk; ++q) v += Fv(q, x, y) * Vv[(size_t)q * Kk + col];
                        phib[(size_t)l * bw * bh + (size_t)(y - t.by0) * bw + (x - t.bx0)] = v;
                    }
                auto ph = [&](int x, int y) -> cd {
                    if (x < t.cx0 || x >= t.cx1 || y < t.cy0 || y >= t.cy1) return cd(0, 0);
                    return phib[(size_t)l * bw * bh + (size_t)(y - t.by0) * bw + (x - t.bx0)];
                };
                for (int y = t.by0; y < t.by0 + bh; ++y)
                    for (int x = t.bx0; x < t.bx0 + bw; ++x) {
                        const cd dg = -(cxm[x] + cxp[x] + cym[y] + cyp[y]) - k0 * k0 * (double)p->eps[(size_t)y * nx + x];
                        cd v = dg * ph(x, y);
                        if (x > 0) v += cxm[x] * ph(x - 1, y);
                        if (x + 1 < nx) v += cxp[x] * ph(x + 1, y);
                        if (y > 0) v += cym[y] * ph(x, y - 1);
                        if (y + 1 < ny) v += cyp[y] * ph(x, y + 1);
                        wb[(size_t)l * bw * bh + (size_t)(y - t.by0) * bw + (x - t.bx0)] = v;
                    }
            }
            for (size_t e = 0; e < phib.size(); ++e) {
                phi_h[(size_t)wi * box_total + t.box_off + e] = make_float2((float)phib[e].real(), (float)phib[e].imag());
                W_h[(size_t)wi * box_total + t.box_off + e] = make_float2((float)wb[e].real(), (float)wb[e].imag());
            }
            // Q: the rotated probe data on this tile's own entries; T Q: the Robin
            // traces of the basis fields (core-only) on the neighbours' entries
            // that touch this core
            {
                const auto &Xe = Xt[(size_t)wi * nt + ti];
                const auto &own = p->tile_entries[ti];
                for (int l = 0; l < kc; ++l) {
                    const int col = ti * kc + l;
                    const bool valid = l < std::min(kc, Kk);
                    for (int e = 0; e < (int)own.size(); ++e) {
                        cd u = 0;
                        if (valid)
                            for (int q = 0; q < Kk; ++q) u += Xe[(size_t)e * K + q] * Vv[(size_t)q * Kk + order[l]];
                        rcnz[wi].push_back({t.tr_off + e, col, u, cd(0, 0)});
                    }
                    auto phv = [&](int x, int y) -> cd {
                        if (!valid || x < t.cx0 || x >= t.cx1 || y < t.cy0 || y >= t.cy1) return cd(0, 0);
                        return phib[(size_t)l * t.bw * t.bh + (size_t)(y - t.by0) * t.bw + (x - t.bx0)];
                    };
                    for (const int tj : p->nbrs[ti]) {
                        const TileDesc &u = p->tiles[tj];
                        const auto &ent = p->tile_entries[tj];
                        for (int e = 0; e < (int)ent.size(); ++e) {
                            const int px = ent[e].x % nx, py = ent[e].x / nx, qx = ent[e].y % nx, qy = ent[e].y / nx;
                            const bool inp = px >= t.cx0 && px < t.cx1 && py >= t.cy0 && py < t.cy1;
                            const bool inq = qx >= t.cx0 && qx < t.cx1 && qy >= t.cy0 && qy < t.cy1;
                            if (!inp && !inq) continue;
                            const cd up = phv(px, py), uq = phv(qx, qy);
                            const double kp = k0 * std::sqrt((double)p->eps[ent[e].x]);
                            rcnz[wi].push_back({u.tr_off + e, col, cd(0, 0),
                                                (uq - up) / h + cd(0.0, 0.5 * kp) * (uq + up)});
                        }
                    }
                }
            }
            Wd[(size_t)wi * nt + ti] = std::move(wb);
        }
        // G = W^H W over overlapping boxes (neighbouring tiles only)
        std::vector<cd> G((size_t)nc * nc, cd(0, 0));
        for (int ti = 0; ti < nt; ++ti) {
            const TileDesc &a = p->tiles[ti];
            std::vector<int> cand = p->nbrs[ti];
            cand.push_back(ti);
            for (const int tj : cand) {
                const TileDesc &bt = p->tiles[tj];
                const int x0 = std::max(a.bx0, bt.bx0), x1 = std::min(a.bx0 + a.bw, bt.bx0 + bt.bw);
                const int y0 = std::max(a.by0, bt.by0), y1 = std::min(a.by0 + a.bh, bt.by0 + bt.bh);
                if (x0 >= x1 || y0 >= y1) continue;
                const auto &wa = Wd[(size_t)wi * nt + ti], &wbb = Wd[(size_t)wi * nt + tj];
                for (int la = 0; la < kc; ++la)
                    for (int lb = 0; lb < kc; ++lb) {
                        cd s = 0;
                        for (int y = y0; y < y1; ++y)
                            for (int x = x0; x < x1; ++x)
                                s += std::conj(wa[(size_t)la * a.bw * a.bh + (size_t)(y - a.by0) * a.bw + (x - a.bx0)]) *
                                     wbb[(size_t)lb * bt.bw * bt.bh + (size_t)(y - bt.by0) * bt.bw + (x - bt.bx0)];
                        G[(size_t)(ti * kc + la) * nc + (tj * kc + lb)] = s;
                    }
            }
        }
        // zero basis columns (tiles with fewer independent probes) get a unit
        // diagonal entry, which pins their coefficient to 0
        for (int ti = 0; ti < nt; ++ti)
            for (int l = Kt[(size_t)wi * nt + ti]; l < kc; ++l)
                G[(size_t)(ti * kc + l) * nc + (ti * kc + l)] = 1.0;
        std::vector<cd> Gi;
        if (!hpd_inverse(nc, G, Gi)) return fail(ctx, NOSDD_EBREAKDOWN, "coarse matrix G = W^H W is not positive definite");
        for (int j = 0; j < nc; ++j)
            for (int i = 0; i < nc; ++i) {
                const cd g = Gi[(size_t)i * nc + j];
                ginv_dev[(size_t)wi * nc * nc + (size_t)j * nc + i] = make_double2(g.real(), g.imag());
            }
    }
    {
        // structure (identical for every wavelength: it is geometric) by entry and by column
        const int ne = p->n_entries;
        const auto &z0 = rcnz[0];
        const int nnz = (int)z0.size();
        p->rc_nnz = nnz;
        std::vector<int> colptr(nc + 1, 0), rowptr(ne + 1, 0), colent(nnz), rowcol(nnz), perm(nnz);
        for (int k = 0; k < nnz; ++k) {
            colptr[z0[k].col + 1]++;
            rowptr[z0[k].e + 1]++;
            colent[k] = z0[k].e;
        }
        for (int c = 0; c < nc; ++c) colptr[c + 1] += colptr[c];
        for (int e = 0; e < ne; ++e) rowptr[e + 1] += rowptr[e];
        {
            std::vector<int> fill(rowptr.begin(), rowptr.end() - 1);
            for (int k = 0; k < nnz; ++k) perm[fill[z0[k].e]++] = k;      // row position -> column-order index
        }
        for (int k = 0; k < nnz; ++k) rowcol[k] = z0[perm[k]].col;
        std::vector<float2> rq((size_t)nwl * nnz), rtq((size_t)nwl * nnz), cval((size_t)nwl * nnz);
        std::vector<double2> rginv((size_t)nwl * nc * nc);
        for (int wi = 0; wi < nwl; ++wi) {
            const auto &zz = rcnz[wi];
            for (int k = 0; k < nnz; ++k) {
                const cd mv = zz[k].q - zz[k].tq;
                cval[(size_t)wi * nnz + k] = make_float2((float)mv.real(), (float)mv.imag());
                const RcNz &r = zz[perm[k]];
                rq[(size_t)wi * nnz + k] = make_float2((float)r.q.real(), (float)r.q.imag());
                rtq[(size_t)wi * nnz + k] = make_float2((float)r.tq.real(), (float)r.tq.imag());
            }
            // M^H M from the entries' nonzeros (M = Q - T Q), FP64
            std::vector<cd> G((size_t)nc * nc, cd(0, 0));
            for (int e = 0; e < ne; ++e)
                for (int a = rowptr[e]; a < rowptr[e + 1]; ++a) {
                    const RcNz &za = zz[perm[a]];
                    const cd ma = std::conj(za.q - za.tq);
                    for (int bb = rowptr[e]; bb < rowptr[e + 1]; ++bb) {
                        const RcNz &zb = zz[perm[bb]];
                        G[(size_t)za.col * nc + zb.col] += ma * (zb.q - zb.tq);
                    }
                }
            for (int c = 0; c < nc; ++c)
                if (std::abs(G[(size_t)c * nc + c]) == 0.0) G[(size_t)c * nc + c] = 1.0;   // zero column: z_c = 0
            std::vector<cd> Gi;
            if (!hpd_inverse(nc, G, Gi))
                return fail(ctx, NOSDD_EBREAKDOWN, "Robin-space coarse matrix is not positive definite");
            for (int j = 0; j < nc; ++j)
                for (int i = 0; i < nc; ++i) {
                    const cd g = Gi[(size_t)i * nc + j];
                    rginv[(size_t)wi * nc * nc + (size_t)j * nc + i] = make_double2(g.real(), g.imag());
                }
        }
        auto up = [&](DevBuf &d, const void *src, size_t bytes) -> hipError_t {
            hipError_t er = d.ensure(std::max<size_t>(bytes, 16));
            if (er != hipSuccess) return er;
            return bytes ? hipMemcpyAsync(d.p, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
        };
        HIPCHK(ctx, up(p->d_rc_rowptr, rowptr.data(), rowptr.size() * sizeof(int)));
        HIPCHK(ctx, up(p->d_rc_rowcol, rowcol.data(), rowcol.size() * sizeof(int)));
        HIPCHK(ctx, up(p->d_rc_colptr, colptr.data(), colptr.size() * sizeof(int)));
        HIPCHK(ctx, up(p->d_rc_colent, colent.data(), colent.size() * sizeof(int)));
        HIPCHK(ctx, up(p->d_rc_q, rq.data(), rq.size() * sizeof(float2)));
        HIPCHK(ctx, up(p->d_rc_tq, rtq.data(), rtq.size() * sizeof(float2)));
        HIPCHK(ctx, up(p->d_rc_colval, cval.data(), cval.size() * sizeof(float2)));
        HIPCHK(ctx, up(p->d_rc_GinvT, rginv.data(), rginv.size() * sizeof(double2)));
        HIPCHK(ctx, hipStreamSynchronize(s));
    }
    HIPCHK(ctx, p->d_phi.ensure(phi_h.size() * sizeof(float2)));
    HIPCHK(ctx, p->d_W.ensure(W_h.size() * sizeof(float2)));
    HIPCHK(ctx, p->d_GinvT.ensure(ginv_dev.size() * sizeof(double2)));
    HIPCHK(ctx, hipMemcpyAsync(p->d_phi.p, phi_h.data(), phi_h.size() * sizeof(float2), hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipMemcpyAsync(p->d_W.p, W_h.data(), W_h.size() * sizeof(float2), hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipMemcpyAsync(p->d_GinvT.p, ginv_dev.data(), ginv_dev.size() * sizeof(double2), hipMemcpyHostToDevice,
                               s));
    HIPCHK(ctx, p->d_owner.ensure(p->owner.size() * sizeof(int)));
    HIPCHK(ctx, hipMemcpyAsync(p->d_owner.p, p->owner.data(), p->owner.size() * sizeof(int), hipMemcpyHostToDevice, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return NOSDD_OK;
}

int cgs_bucket(int nv) { return nv <= 8 ? 0 : nv <= 16 ? 1 : nv <= 24 ? 2 : 3; }

// Launch-parameter autotuning on the problem's own buffers, once per
// workspace shape (and, for the subdomain solve, once per set-up), before any
// graph capture.  Every candidate computes the same result (the Gram-Schmidt
// reductions are fixed-order for a given grid, and the prefetch depth does
// not change the arithmetic), so only time decides:
//   * Gram-Schmidt workgroups per RHS: {nblk/2, nblk, 2 nblk} around the
//     bandwidth heuristic, per basis-size bucket, timing one dots, fused
//     update-dots and update pass at the bucket's middle size;
//   * subdomain-solve prefetch depth among those the block size allows.
// Each candidate is timed as the median of three runs with HIP events.
nosdd_status autotune(nosdd_problem *p, int n_rhs, int n_src, int m, const GivensArgs &ga) {
    (void)ga;
    nosdd_ctx *ctx = p->ctx;
    Workspace &w = p->ws;
    hipStream_t s = ctx->stream;
    const long long N = w.N;
    const long long vstride = (long long)n_rhs * N;
    float2 *V = w.V.as<float2>(), *wv = w.w.as<float2>(), *Z = w.Z.as<float2>();
    CallResources res;
    HIPCHK(ctx, hipEventCreate(&res.e0));
    HIPCHK(ctx, hipEventCreate(&res.e1));
    hipEvent_t e0 = res.e0, e1 = res.e1;
    auto time_ms = [&](auto &&launch) -> float {
        float t[3];
        launch();                                      // warm
        for (int r = 0; r < 3; ++r) {
            (void)hipEventRecord(e0, s);
            launch();
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            (void)hipEventElapsedTime(&t[r], e0, e1);
        }
        std::sort(t, t + 3);
        return t[1];
    };
    if (!w.tuned) {
        std::vector<int> cand;
        for (int c : {w.nblk, std::max(1, w.nblk / 2), std::min(w.nblk_max, 2 * w.nblk)})
            if (std::find(cand.begin(), cand.end(), c) == cand.end()) cand.push_back(c);
        const int probe_nv[4] = {6, 14, 22, 30};
        double2 *part = w.partial.as<double2>();
        const int *ones = w.ones.as<int>();
        for (int bk = 0; bk < 4; ++bk) {
            const int nv = std::min(probe_nv[bk], m);        // the update writes basis slot nv <= m
            if (nv < 1) continue;
            float best = 1e30f;
            int pick = w.nblk;
            for (int c : cand) {
                const float ms = time_ms([&] {
                    launch_cgs_dots(s, V, vstride, nv, wv, N, n_rhs, ones, part, c);
                    launch_cgs_update_dots(s, V, vstride, nv, wv, V + nv * vstride, N, n_rhs, ones,
                                           w.H.as<float2>(), m, nv - 1, part, c);
                    if (!p->stored_basis)
                        launch_cgs_update_scale(s, V, vstride, nv, V + nv * vstride, V + nv * vstride, N, n_rhs,
                                                ones, ones, w.H2.as<float2>(), m, nv - 1, w.inv_h.as<float>(), c);
                });
                if (ms < best) {
                    best = ms;
                    pick = c;
                }
            }
            w.nblk_b[bk] = pick;
        }
        w.tuned = true;
    }
    // the prefetch depth belongs to the one-source kernel: nothing to tune when
    // the sources of a wavelength are solved together
    if (!p->bt_tuned && p->sub_solver == 0 && !use_multi(p, n_src)) {
        int depths[4];
        const int nd = bt_solve_depths(p->bmax, depths);
        const int2 *ord = nullptr;
        int nj = 0;
        nosdd_status so = solve_order(p, n_rhs, n_src, &ord, &nj);
        if (so != NOSDD_OK) return so;
        float best = 1e30f;
        int pick = 0;
        for (int i = 0; i < nd; ++i) {
            const float ms = time_ms([&] {
                launch_bt_solve(s, p->d_tiles.as<TileDesc>(), ord, nj, n_src, p->d_dinv.as<float2>(),
                                p->dinv_wl_stride, p->d_coef.as<float2>(), p->d_sc.as<float2>(), p->nx, p->ny, V, N, Z, N,
                                w.ones.as<int>(), 0, p->bmax, p->max_cells, depths[i]);
            });
            if (ms < best) {
                best = ms;
                pick = depths[i];
            }
        }
        p->bt_depth = pick;
        p->bt_tuned = true;
    }
    HIPCHK(ctx, hipGetLastError());
    return NOSDD_OK;
}

// Capture (or reuse) one graph per Arnoldi step j of a restart cycle.  The
// graphs bake in buffer addresses, sizes and the solve options, so they are
// keyed on those and on the allocation generation.  Each graph ends with a
// copy of the active flags into pinned host memory (one buffer per parity of
// j), which the host reads two steps later.  Only kernels and that copy are
// captured: no memsets.
template <class Step>
nosdd_status ensure_graphs(nosdd_problem *p, int n_rhs, int n_src, int m, const nosdd_solve_opts *o, Step &step) {
    nosdd_ctx *ctx = p->ctx;
    Workspace &w = p->ws;
    if (p->h_flags_n < n_rhs) {
        if (p->h_flags) (void)hipHostFree(p->h_flags);
        p->h_flags = nullptr;
        p->h_flags_n = 0;
        HIPCHK(ctx, hipHostMalloc((void **)&p->h_flags, 2 * (size_t)n_rhs * sizeof(int), hipHostMallocDefault));
        HIPCHK(ctx, hipHostGetDevicePointer((void **)&p->d_flags, p->h_flags, 0));
        p->h_flags_n = n_rhs;
        ++g_alloc_gen;
    }
    for (hipEvent_t &e : p->gev)
        if (!e) HIPCHK(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    long long tolbits = 0;
    std::memcpy(&tolbits, &o->tol, sizeof(double));
    const std::vector<long long> key = {g_alloc_gen.load(), n_rhs, n_src, m, o->max_iters, tolbits,
                                        (long long)(intptr_t)p->h_flags, p->bt_depth, w.nblk_b[0], w.nblk_b[1],
                                        w.nblk_b[2], w.nblk_b[3]};
    if (key == p->gkey && (int)p->gexec.size() == m) return NOSDD_OK;
    p->drop_graphs();
    if (!ctx->cap_stream) HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = ctx->cap_stream;
    for (int j = 0; j < m; ++j) {
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        HIPCHK(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
        // the host reads the step's active flags from pinned memory: written by
        // the step's last reduction in the stored-basis form, copied otherwise
        step(cs, j, n_rhs, p->stored_basis ? p->d_flags + (j & 1) * n_rhs : nullptr);
        hipError_t e = p->stored_basis ? hipSuccess
                                       : hipMemcpyAsync(p->h_flags + (j & 1) * n_rhs, w.active.p, n_rhs * sizeof(int),
                                                        hipMemcpyDeviceToHost, cs);
        hipError_t e2 = hipStreamEndCapture(cs, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            p->drop_graphs();
            return fail(ctx, NOSDD_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e));
        }
        p->gexec.push_back(ge);
    }
    p->gkey = key;
    return NOSDD_OK;
}

nosdd_status solve_impl(nosdd_problem *p, const float2 *J_dev, int n_src, const nosdd_solve_opts *o, const float2 *x0_dev,
                        float2 *E_dev, float *resid_hist, int *iters_out, float *final_out, bool j_per_rhs = false,
                        double2 *E64_dev = nullptr) {
    nosdd_ctx *ctx = p->ctx;
    hipStream_t s = ctx->stream;
    const int nwl = (int)p->wl.size();
    const int n_rhs = nwl * n_src;
    const int m = o->restart;
    const long long N = (long long)p->nx * p->ny;
    nosdd_status st = ensure_ws(p, n_rhs, m, o->max_iters);
    if (st != NOSDD_OK) return st;
    if (p->sub_solver == 1) {
        st = ensure_nn(p, n_rhs, n_src);
        if (st != NOSDD_OK) return st;
    }
    Workspace &w = p->ws;
    GivensArgs ga;
    ga.H = w.H.as<float2>();
    ga.ldh = m;
    ga.m = m;
    ga.cs = w.cs.as<float>();
    ga.sn = w.sn.as<float2>();
    ga.gam = w.gam.as<float2>();
    ga.nw_pre = w.nw_pre.as<double>();
    ga.nw_pre_w = w.nw_pre.as<double>();
    ga.H2 = w.H2.as<float2>();
    ga.reorth = w.reorth.as<int>();
    ga.bnorm = w.bnorm.as<float>();
    ga.tol = (float)o->tol;
    ga.active = w.active.as<int>();
    ga.iters = w.iters.as<int>();
    ga.kcyc = w.kcyc.as<int>();
    ga.max_iters = o->max_iters;
    ga.hist = w.hist.as<float>();
    ga.hist_ld = std::max(1, o->max_iters);
    ga.inv_h = w.inv_h.as<float>();
    ga.flags = w.flags.as<int>();
    ga.host_flags = nullptr;
    ga.T = w.T.as<double2>();
    ga.G1 = w.G1.as<float2>();
    ga.scale = w.scale.as<float>();
    CallResources res;
    HIPCHK(ctx, hipEventCreate(&res.e0));
    HIPCHK(ctx, hipEventCreate(&res.e1));
    HIPCHK(ctx, hipEventRecord(res.e0, s));

    double2 *x = w.x.as<double2>();
    float2 *b = w.b.as<float2>(), *V = w.V.as<float2>(), *Z = w.Z.as<float2>(),
           *wv = w.w.as<float2>();
    const long long vstride = (long long)n_rhs * N;
    hipLaunchKernelGGL(make_rhs_kernel, dim3((unsigned)grid_blocks(N), n_rhs), dim3(256), 0, s, J_dev, b,
                       p->d_k0f.as<float>(), N, n_src, j_per_rhs ? 1 : 0);
    hipLaunchKernelGGL(make_rhs64_kernel, dim3((unsigned)grid_blocks(N), n_rhs), dim3(256), 0, s, J_dev,
                       w.b64.as<double2>(), p->d_k0.as<double>(), N, n_src, j_per_rhs ? 1 : 0);
    hipLaunchKernelGGL(widen_kernel, dim3((unsigned)grid_blocks(vstride)), dim3(256), 0, s, x0_dev, x, vstride);
    HIPCHK(ctx, hipMemsetAsync(w.iters.p, 0, n_rhs * sizeof(int), s));
    if (p->nn_fbcount.p) HIPCHK(ctx, hipMemsetAsync(p->nn_fbcount.p, 0, sizeof(unsigned), s));
    {
        const long long nh = (long long)n_rhs * std::max(1, o->max_iters);
        hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)grid_blocks(nh)), dim3(256), 0, s, w.hist.as<float>(), nh,
                           -1.0f);
    }
    // ||b||
    launch_cgs_dots(s, V, vstride, 0, b, N, n_rhs, w.ones.as<int>(), w.partial.as<double2>(), w.nblk_b[0]);
    launch_cgs_reduce(s, w.partial.as<double2>(), w.nblk_b[0], 0, n_rhs, nullptr, 0, 0, w.bnorm2.as<double>(), ga);
    std::vector<double> bn2(n_rhs), beta2(n_rhs);
    HIPCHK(ctx, hipMemcpyAsync(bn2.data(), w.bnorm2.p, n_rhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    std::vector<float> bnorm(n_rhs);
    for (int r = 0; r < n_rhs; ++r) bnorm[r] = (float)std::sqrt(bn2[r]);
    HIPCHK(ctx, hipMemcpyAsync(w.bnorm.p, bnorm.data(), n_rhs * sizeof(float), hipMemcpyHostToDevice, s));


    std::vector<int> iters(n_rhs, 0), want(n_rhs), act(n_rhs);
    std::vector<double> final_res(n_rhs, 0.0);
    // stagnation: a right-hand side whose explicit residual did not decrease
    // over a whole restart cycle is stopped (status NOT_CONVERGED)
    std::vector<double> prev_res(n_rhs, 0.0);
    std::vector<char> ran(n_rhs, 0), stalled(n_rhs, 0);
    int n_stalled = 0;
    HIPCHK(ctx, hipHostMalloc((void **)&res.h_pinned, n_rhs * sizeof(int) * 2, hipHostMallocDefault));
    int *h_act = res.h_pinned;
    nosdd_status result = NOSDD_OK;
    int total_outer = 0;
    const int *active = w.active.as<int>();
    // One Arnoldi step j: z_j = M^-1 v_j, w = A z_j, two passes of classical
    // Gram-Schmidt against the basis, Givens rotation and residual estimate.
    // Stored-basis form (default): the first pass's dots, then its update fused
    // with the second pass's dots; the second pass's correction and the
    // normalisation enter the triangular map T from stored vectors to the
    // orthonormal basis instead of a third pass over the vectors.  The other
    // form runs the second pass where the DGKS test asks for it and writes
    // v_{j+1} = (w' - V h2) / h_{j+1,j} with a third pass.  Every argument is
    // fixed for the solve, so the step can be captured in a graph.
    const bool stored_basis = p->stored_basis;
    auto step = [&](hipStream_t st, int j, int n_live_, int *host_flags = nullptr) {
        float2 *Vj = V + j * vstride, *Vn = V + (j + 1) * vstride, *Zj = Z + j * vstride;
        precond(p, st, Vj, Zj, wv, n_src, n_rhs, active, n_live_,
                p->n_c > 0 ? w.cstep.as<float2>() + (size_t)j * n_rhs * p->n_c : nullptr);
        ProfScope arn(p, 2, n_live_);
        double2 *part = w.partial.as<double2>();
        const int *ro = w.reorth.as<int>();
        const float *ih = w.inv_h.as<float>();
        const int nb = w.nblk_b[cgs_bucket(j + 1)];
        launch_cgs_dots(st, V, vstride, j + 1, wv, N, n_rhs, active, part, nb);
        if (stored_basis) {
            launch_cgs_reduce(st, part, nb, j + 1, n_rhs, active, j, 6, nullptr, ga);
            launch_cgs_update_dots(st, V, vstride, j + 1, wv, Vn, N, n_rhs, active, w.G1.as<float2>(), m, j, part,
                                   nb, w.scale.as<float>());
            GivensArgs g7 = ga;
            g7.host_flags = host_flags;
            launch_cgs_reduce(st, part, nb, j + 1, n_rhs, active, j, 7, nullptr, g7);
            return;
        }
        launch_cgs_reduce(st, part, nb, j + 1, n_rhs, active, j, 1, nullptr, ga);
        // first-pass update with the second pass's dots taken from the same loads
        launch_cgs_update_dots(st, V, vstride, j + 1, wv, Vn, N, n_rhs, active, w.H.as<float2>(), m, j, part, nb);
        launch_cgs_reduce(st, part, nb, j + 1, n_rhs, nullptr, j, 5, nullptr, ga);
        launch_cgs_update_scale(st, V, vstride, j + 1, Vn, Vn, N, n_rhs, active, ro, w.H2.as<float2>(), m, j, ih,
                                nb);
    };
    {
        const int2 *ord = nullptr;
        int nj = 0;
        nosdd_status so = solve_order(p, n_rhs, n_src, &ord, &nj);
        if (so != NOSDD_OK) return so;
    }
    if (p->use_autotune) {
        nosdd_status ts = autotune(p, n_rhs, n_src, m, ga);
        if (ts != NOSDD_OK) return ts;
    }
    const bool graphs = p->use_graphs && !p->prof;
    if (graphs) {
        nosdd_status gs = ensure_graphs(p, n_rhs, n_src, m, o, step);
        if (gs != NOSDD_OK) return gs;
    }
    for (;;) {
        // explicit residual r = b - A x (FP64) into w, beta^2
        {
        ProfScope ps(p, 1, n_rhs);
        launch_residual64(s, x, w.b64.as<double2>(), wv, p->d_eps.as<float>(), p->d_coefd.as<double2>(), p->d_k0.as<double>(), p->nx,
                          p->ny, n_rhs, n_src);
        }
        launch_cgs_dots(s, V, vstride, 0, wv, N, n_rhs, w.ones.as<int>(), w.partial.as<double2>(), w.nblk_b[0]);
        launch_cgs_reduce(s, w.partial.as<double2>(), w.nblk_b[0], 0, n_rhs, nullptr, 0, 0, w.beta2.as<double>(), ga);
        HIPCHK(ctx, hipMemcpyAsync(beta2.data(), w.beta2.p, n_rhs * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipMemcpyAsync(iters.data(), w.iters.p, n_rhs * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        int any = 0;
        for (int r = 0; r < n_rhs; ++r) {
            const double rel = bn2[r] > 0 ? std::sqrt(beta2[r] / bn2[r]) : 0.0;
            final_res[r] = rel;
            if (!std::isfinite(rel)) return fail(ctx, NOSDD_ENONFINITE, "non-finite residual");
            if (ran[r] && !stalled[r] && rel > o->tol && rel >= prev_res[r]) {
                stalled[r] = 1;
                ++n_stalled;
            }
            want[r] = (!stalled[r] && rel > o->tol && iters[r] < o->max_iters && bn2[r] > 0) ? 1 : 0;
            ran[r] = (char)want[r];
            prev_res[r] = rel;
            any |= want[r];
        }
        if (!any) break;
        HIPCHK(ctx, hipMemcpyAsync(w.want.p, want.data(), n_rhs * sizeof(int), hipMemcpyHostToDevice, s));
        HIPCHK(ctx, hipMemsetAsync(w.kcyc.p, 0, n_rhs * sizeof(int), s));
        HIPCHK(ctx, hipMemsetAsync(w.active.p, 0, n_rhs * sizeof(int), s));
        HIPCHK(ctx, hipMemsetAsync(w.reorth.p, 0, n_rhs * sizeof(int), s));
        HIPCHK(ctx, hipMemsetAsync(w.H.p, 0, (size_t)n_rhs * (m + 1) * m * sizeof(float2), s));
        launch_start_cycle(s, V, wv, w.beta2.as<double>(), w.bnorm.as<float>(), w.gam.as<float2>(), m,
                           w.kcyc.as<int>(), w.active.as<int>(), w.want.as<int>(), N, n_rhs);
        int n_live = 0;
        for (int r = 0; r < n_rhs; ++r) n_live += want[r];
        if (graphs) {
            // Replay the captured steps; the host stays at most two steps ahead
            // and stops once a completed step reports no active right-hand side
            // (steps launched after that are masked out on the device).
            for (int j = 0; j < m; ++j) {
                if (j >= 2) {
                    HIPCHK(ctx, hipEventSynchronize(p->gev[j & 1]));
                    const int *f = p->h_flags + (j & 1) * n_rhs;
                    n_live = 0;
                    for (int r = 0; r < n_rhs; ++r) n_live += f[r] ? 1 : 0;
                    if (!n_live) break;
                }
                HIPCHK(ctx, hipGraphLaunch(p->gexec[j], s));
                HIPCHK(ctx, hipEventRecord(p->gev[j & 1], s));
                ++total_outer;
            }
        } else {
            for (int j = 0; j < m; ++j) {
                step(s, j, n_live);
                ++total_outer;
                HIPCHK(ctx, hipMemcpyAsync(h_act, w.active.p, n_rhs * sizeof(int), hipMemcpyDeviceToHost, s));
                HIPCHK(ctx, hipStreamSynchronize(s));
                n_live = 0;
                for (int r = 0; r < n_rhs; ++r) n_live += h_act[r] ? 1 : 0;
                if (!n_live) break;
            }
        }
        launch_backsolve(s, w.H.as<float2>(), m, m, w.gam.as<float2>(), w.kcyc.as<int>(), w.y.as<float2>(), n_rhs);
        launch_xupdate(s, x, Z, vstride, w.y.as<float2>(), m, w.kcyc.as<int>(), N, n_rhs);
        if (p->n_c > 0)
            launch_coarse_cycle_end(s, x, p->d_tiles.as<TileDesc>(), p->d_owner.as<int>(), p->kc,
                                    p->d_phi.as<float2>(), p->box_wl_stride, w.cstep.as<float2>(), w.y.as<float2>(), m,
                                    w.kcyc.as<int>(), p->n_c, w.cy.as<double2>(), p->nx, p->ny, n_rhs, n_src);
    }
    HIPCHK(ctx, hipGetLastError());
    if (E_dev)
        hipLaunchKernelGGL(narrow_kernel, dim3((unsigned)grid_blocks(vstride)), dim3(256), 0, s, x, E_dev, vstride);
    if (E64_dev) HIPCHK(ctx, hipMemcpyAsync(E64_dev, x, (size_t)vstride * sizeof(double2), hipMemcpyDeviceToDevice, s));
    HIPCHK(ctx, hipEventRecord(res.e1, s));
    HIPCHK(ctx, hipMemcpyAsync(iters.data(), w.iters.p, n_rhs * sizeof(int), hipMemcpyDeviceToHost, s));
    if (resid_hist && o->max_iters > 0)
        HIPCHK(ctx, hipMemcpyAsync(resid_hist, w.hist.p, (size_t)n_rhs * std::max(1, o->max_iters) * sizeof(float),
                                   hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, res.e0, res.e1);
    if (p->prof) prof_flush(p);
    p->solve_ms = ms;
    p->last_iters = total_outer;
    for (int r = 0; r < n_rhs; ++r) {
        if (iters_out) iters_out[r] = iters[r];
        if (final_out) final_out[r] = (float)final_res[r];
        if (final_res[r] > o->tol) result = NOSDD_NOT_CONVERGED;
    }
    if (n_stalled > 0)
        ctx->err = std::to_string(n_stalled) + " right-hand side(s) stopped early: the explicit residual did not "
                                                "decrease over a whole restart cycle";
    return result;
}

nosdd_status check_problem(nosdd_problem *p, bool need_setup) {
    if (!p) return NOSDD_EINVAL;
    if (need_setup && !p->setup_done) return fail(p->ctx, NOSDD_ESTATE, "nosdd_problem_setup has not been called");
    if (hipSetDevice(p->ctx->device) != hipSuccess) return fail(p->ctx, NOSDD_EHIP, "hipSetDevice failed");
    (void)hipGetLastError();    // errors left by unrelated earlier runtime calls are not ours
    return NOSDD_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

nosdd_status nosdd_ctx_create(int hip_device, void *hip_stream, nosdd_ctx **out) {
    if (!out) return NOSDD_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device < 0 || hip_device >= n) return NOSDD_EINVAL;
    if (hipSetDevice(hip_device) != hipSuccess) return NOSDD_EHIP;
    // device address of this GPU's fixed scratch (nosdd_precond_apply_noalloc)
    if (noalloc_scratch_init(hip_device) != hipSuccess) return NOSDD_EHIP;
    nosdd_ctx *c = new nosdd_ctx();
    c->device = hip_device;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreate(&c->stream) != hipSuccess) {
            delete c;
            return NOSDD_EHIP;
        }
        c->own_stream = true;
    }
    *out = c;
    return NOSDD_OK;
}

void nosdd_ctx_destroy(nosdd_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->own_stream && ctx->stream) (void)hipStreamDestroy(ctx->stream);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
}

const char *nosdd_last_error(const nosdd_ctx *ctx) {
    if (!ctx) return "null context";
    return ctx->err.c_str();
}

// Problem over an explicit list of cores (cx0, cx1, cy0, cy1), half-open,
// that covers every cell once: each core is extended by overlap/2 across every
// side that is not on the global boundary.  Shared by the tensor-product
// partition and the general (e.g. quad-tree) one.
static nosdd_status problem_create_impl(nosdd_ctx *ctx, const nosdd_grid *g, const float *eps,
                                        const std::vector<int4> &cores, int overlap, const double *wavelengths,
                                        int n_wl, nosdd_problem **out) {
    if (g->nx < 4 || g->ny < 4 || !(g->h > 0) || g->npml < 0 || 2 * g->npml >= std::min(g->nx, g->ny) || g->pml_m < 0)
        return fail(ctx, NOSDD_EINVAL, "invalid grid");
    if ((long long)g->nx * g->ny >= (1LL << 29))          // byte offsets within a vector stay 32-bit
        return fail(ctx, NOSDD_EINVAL, "grid too large: at most 2^29 - 1 cells");
    for (int i = 0; i < n_wl; ++i)
        if (!(wavelengths[i] > 0)) return fail(ctx, NOSDD_EINVAL, "wavelengths must be positive");
    if (cores.empty()) return fail(ctx, NOSDD_EPARTITION, "empty partition");
    if (overlap < 2 || overlap % 2) return fail(ctx, NOSDD_EPARTITION, "overlap must be even and >= 2");
    const int ext = overlap / 2;
    const int gnx = g->nx, gny = g->ny;
    std::vector<int> owner((size_t)gnx * gny, -1);
    int minc = 1 << 30;
    for (int k = 0; k < (int)cores.size(); ++k) {
        const int4 c = cores[k];
        if (!(0 <= c.x && c.x < c.y && c.y <= gnx && 0 <= c.z && c.z < c.w && c.w <= gny))
            return fail(ctx, NOSDD_EPARTITION, "a core is empty or leaves the grid");
        for (int y = c.z; y < c.w; ++y)
            for (int x = c.x; x < c.y; ++x) {
                int &o = owner[(size_t)y * gnx + x];
                if (o >= 0) return fail(ctx, NOSDD_EPARTITION, "cores overlap");
                o = k;
            }
        minc = std::min(minc, std::min(c.y - c.x, c.w - c.z));
    }
    for (const int o : owner)
        if (o < 0) return fail(ctx, NOSDD_EPARTITION, "cores do not cover the grid");
    if (cores.size() > 1 && ext + 1 > minc) return fail(ctx, NOSDD_EPARTITION, "overlap/2 + 1 exceeds a core");
    // the Robin wavenumber kappa = k0 sqrt(eps) is real only for eps > 0
    for (int i = 0; i < gnx * gny; ++i)
        if (!(std::isfinite(eps[i]) && eps[i] > 0.f)) return fail(ctx, NOSDD_EINVAL, "eps must be finite and positive");

    nosdd_problem *p = new nosdd_problem();
    p->ctx = ctx;
    p->nx = gnx;
    p->ny = gny;
    p->h = g->h;
    p->npml = g->npml;
    p->pml_m = g->pml_m;
    p->lnR = g->pml_lnR;
    p->eps.assign(eps, eps + (size_t)gnx * gny);
    p->wl.assign(wavelengths, wavelengths + n_wl);
    p->overlap = overlap;
    p->ext = ext;
    p->owner = std::move(owner);
    // tiles
    long long loc = 0, dinv = 0;
    for (const int4 &c : cores) {
        TileDesc t{};
        t.cx0 = c.x;
        t.cx1 = c.y;
        t.cy0 = c.z;
        t.cy1 = c.w;
        t.iface = (t.cy0 > 0 ? SIDE_BOTTOM : 0) | (t.cx1 < gnx ? SIDE_RIGHT : 0) | (t.cy1 < gny ? SIDE_TOP : 0) |
                  (t.cx0 > 0 ? SIDE_LEFT : 0);
        t.x0 = (t.iface & SIDE_LEFT) ? t.cx0 - ext : t.cx0;
        t.x1 = (t.iface & SIDE_RIGHT) ? t.cx1 + ext : t.cx1;
        t.y0 = (t.iface & SIDE_BOTTOM) ? t.cy0 - ext : t.cy0;
        t.y1 = (t.iface & SIDE_TOP) ? t.cy1 + ext : t.cy1;
        const int n = p->npml;
        auto bad_x = [&](int xb) { return xb < n || xb > p->nx - n - 1; };
        auto bad_y = [&](int yb) { return yb < n || yb > p->ny - n - 1; };
        if (((t.iface & SIDE_LEFT) && bad_x(t.x0)) || ((t.iface & SIDE_RIGHT) && bad_x(t.x1 - 1)) ||
            ((t.iface & SIDE_BOTTOM) && bad_y(t.y0)) || ((t.iface & SIDE_TOP) && bad_y(t.y1 - 1))) {
            delete p;
            return fail(ctx, NOSDD_EPARTITION, "a subdomain interface lies inside the PML of its normal direction");
        }
        const int lx = t.x1 - t.x0, ly = t.y1 - t.y0;
        t.tr = lx > ly ? 1 : 0;
        t.b = std::min(lx, ly);
        t.nb = std::max(lx, ly);
        if (t.b % 2 || t.b > BT_FACT_SCRATCH_B) {
            delete p;
            return fail(ctx, NOSDD_EPARTITION, "extended subdomains need an even short side of at most 128 cells");
        }
        if (t.nb > BT_NBMAX || lx * ly > BT_LDS_MAX_CELLS) {
            delete p;
            return fail(ctx, NOSDD_EPARTITION, "an extended subdomain is too large for an LDS-resident solve");
        }
        p->max_cells = std::max(p->max_cells, lx * ly);
        t.loc_off = loc;
        loc += (long long)lx * ly;
        t.dinv_off = dinv;
        dinv += (long long)t.nb * bt_sym_block(t.b);
        p->bmax = std::max(p->bmax, t.b);
        p->tiles.push_back(t);
    }
    // neighbours: tiles whose extended rectangle grown by one cell (the ghost
    // nodes of its ring) meets this tile's, in index order; every interface
    // entry that touches a tile belongs to one of them
    // (candidates: the owners of the cells within ext + 1 of the extended
    // tile, since a neighbour's extended tile grown by one lies within ext + 1
    // of its core; linear in the grid, whatever the number of cores)
    const int nt = (int)p->tiles.size();
    p->nbrs.assign(nt, {});
    std::vector<int> seen(nt, -1);
    for (int i = 0; i < nt; ++i) {
        const TileDesc &t = p->tiles[i];
        const int gx0 = std::max(t.x0 - ext - 1, 0), gx1 = std::min(t.x1 + ext + 1, gnx);
        const int gy0 = std::max(t.y0 - ext - 1, 0), gy1 = std::min(t.y1 + ext + 1, gny);
        std::vector<int> cand;
        for (int y = gy0; y < gy1; ++y)
            for (int x = gx0; x < gx1; ++x) {
                const int j = p->owner[(size_t)y * gnx + x];
                if (j != i && seen[j] != i) {
                    seen[j] = i;
                    cand.push_back(j);
                }
            }
        std::sort(cand.begin(), cand.end());
        for (const int j : cand) {
            const TileDesc &u = p->tiles[j];
            if (u.x0 - 1 < t.x1 && t.x0 < u.x1 + 1 && u.y0 - 1 < t.y1 && t.y0 < u.y1 + 1) p->nbrs[i].push_back(j);
        }
    }
    p->loc_total = loc;
    p->dinv_wl_stride = dinv;
    for (auto &t : p->tiles) {
        std::vector<int4> e;
        trace_entries(t, p->nx, e);
        t.tr_off = p->n_entries;
        t.n_tr = (int)e.size();
        p->n_entries += t.n_tr;
        p->tile_entries.push_back(e);
    }
    // coefficients
    const int nx = p->nx, ny = p->ny;
    std::vector<float2> cf((size_t)n_wl * 2 * (nx + ny));
    std::vector<float2> scv;
    std::vector<double2> cdv((size_t)n_wl * 2 * (nx + ny));
    std::vector<float> k0sq(n_wl), k0f(n_wl);
    std::vector<double> k0d(n_wl);
    for (int w = 0; w < n_wl; ++w) {
        const double k0 = 2.0 * M_PI / p->wl[w];
        k0d[w] = k0;
        k0f[w] = (float)k0;
        k0sq[w] = (float)(k0 * k0);
        auto ax = axis_coefs(nx, p->npml, p->pml_m, p->lnR, k0, p->h);
        auto ay = axis_coefs(ny, p->npml, p->pml_m, p->lnR, k0, p->h);
        std::vector<cd> all(2 * (nx + ny));
        for (int i = 0; i < 2 * nx; ++i) all[i] = ax[i];
        for (int i = 0; i < 2 * ny; ++i) all[2 * nx + i] = ay[i];
        for (size_t i = 0; i < all.size(); ++i) {
            cf[(size_t)w * all.size() + i] = make_float2((float)all[i].real(), (float)all[i].imag());
            cdv[(size_t)w * all.size() + i] = make_double2(all[i].real(), all[i].imag());
        }
        p->coefd.push_back(all);
        // centre stretches s_x(ix), s_y(iy) (inverse-design gradient)
        const double sh = p->npml ? (p->pml_m + 1) * (-p->lnR) / (2.0 * k0 * p->npml * p->h) : 0.0;
        for (int i = 0; i < nx; ++i) {
            const cd v = stretch((double)i, nx, p->npml, p->pml_m, sh);
            scv.push_back(make_float2((float)v.real(), (float)v.imag()));
        }
        for (int i = 0; i < ny; ++i) {
            const cd v = stretch((double)i, ny, p->npml, p->pml_m, sh);
            scv.push_back(make_float2((float)v.real(), (float)v.imag()));
        }
    }
    std::vector<int4> ents;
    for (auto &e : p->tile_entries) ents.insert(ents.end(), e.begin(), e.end());
    hipStream_t s = ctx->stream;
    auto up = [&](DevBuf &d, const void *src, size_t bytes) -> hipError_t {
        hipError_t e = d.ensure(bytes);
        if (e != hipSuccess) return e;
        return bytes ? hipMemcpyAsync(d.p, src, bytes, hipMemcpyHostToDevice, s) : hipSuccess;
    };
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = up(p->d_eps, p->eps.data(), p->eps.size() * sizeof(float));
    if (e == hipSuccess) e = up(p->d_coef, cf.data(), cf.size() * sizeof(float2));
    if (e == hipSuccess) e = up(p->d_coefd, cdv.data(), cdv.size() * sizeof(double2));
    if (e == hipSuccess) e = up(p->d_k0sq, k0sq.data(), k0sq.size() * sizeof(float));
    if (e == hipSuccess) e = up(p->d_k0f, k0f.data(), k0f.size() * sizeof(float));
    if (e == hipSuccess) e = up(p->d_k0, k0d.data(), k0d.size() * sizeof(double));
    if (e == hipSuccess) e = up(p->d_tiles, p->tiles.data(), p->tiles.size() * sizeof(TileDesc));
    if (e == hipSuccess) e = up(p->d_entries, ents.data(), ents.size() * sizeof(int4));
    if (e == hipSuccess) e = up(p->d_sc, scv.data(), scv.size() * sizeof(float2));
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        ctx->err = std::string("HIP error during problem_create: ") + hipGetErrorString(e);
        delete p;
        return e == hipErrorOutOfMemory ? NOSDD_ENOMEM : NOSDD_EHIP;
    }
    *out = p;
    return NOSDD_OK;
}

nosdd_status nosdd_problem_create(nosdd_ctx *ctx, const nosdd_grid *g, const float *eps, const nosdd_partition *part,
                                  const double *wavelengths, int n_wl, nosdd_problem **out) {
    if (!ctx) return NOSDD_EINVAL;
    if (!out || !g || !eps || !part || !wavelengths || n_wl <= 0) return fail(ctx, NOSDD_EINVAL, "null argument or n_wl <= 0");
    *out = nullptr;
    if (!part->core_x || !part->core_y || part->ncx <= 0 || part->ncy <= 0)
        return fail(ctx, NOSDD_EPARTITION, "empty partition");
    long long sx = 0, sy = 0;
    for (int i = 0; i < part->ncx; ++i) {
        if (part->core_x[i] <= 0) return fail(ctx, NOSDD_EPARTITION, "core sizes must be positive");
        sx += part->core_x[i];
    }
    for (int i = 0; i < part->ncy; ++i) {
        if (part->core_y[i] <= 0) return fail(ctx, NOSDD_EPARTITION, "core sizes must be positive");
        sy += part->core_y[i];
    }
    if (sx != g->nx || sy != g->ny) return fail(ctx, NOSDD_EPARTITION, "core sizes must sum to the grid size");
    std::vector<int4> cores;
    for (int ty = 0, cy = 0; ty < part->ncy; cy += part->core_y[ty++])
        for (int tx = 0, cx = 0; tx < part->ncx; cx += part->core_x[tx++])
            cores.push_back(make_int4(cx, cx + part->core_x[tx], cy, cy + part->core_y[ty]));
    return problem_create_impl(ctx, g, eps, cores, part->overlap, wavelengths, n_wl, out);
}

nosdd_status nosdd_problem_create_cores(nosdd_ctx *ctx, const nosdd_grid *g, const float *eps, const int *cores,
                                        int n_cores, int overlap, const double *wavelengths, int n_wl,
                                        nosdd_problem **out) {
    if (!ctx) return NOSDD_EINVAL;
    if (!out || !g || !eps || !cores || !wavelengths || n_wl <= 0 || n_cores <= 0)
        return fail(ctx, NOSDD_EINVAL, "null argument, n_cores <= 0 or n_wl <= 0");
    *out = nullptr;
    std::vector<int4> cv((size_t)n_cores);
    for (int k = 0; k < n_cores; ++k) cv[k] = make_int4(cores[4 * k], cores[4 * k + 1], cores[4 * k + 2], cores[4 * k + 3]);
    return problem_create_impl(ctx, g, eps, cv, overlap, wavelengths, n_wl, out);
}

nosdd_status nosdd_problem_setup(nosdd_problem *p, const nosdd_setup_opts *o) {
    nosdd_status st = check_problem(p, false);
    if (st) return st;
    nosdd_ctx *ctx = p->ctx;
    if (!o) return fail(ctx, NOSDD_EINVAL, "null options");
    if (o->sub_solver != 0 && o->sub_solver != 1) return fail(ctx, NOSDD_EINVAL, "sub_solver must be 0 or 1");
    if (o->k_coarse < 0 || o->k_trial < 0) return fail(ctx, NOSDD_EINVAL, "negative coarse size");
    if (o->sub_solver == 1 && (!o->nn_weights || !o->nn_weights[0]))
        return fail(ctx, NOSDD_ENOWEIGHTS, "neural subdomain solver requested without a weights file");
    if (o->sub_solver == 1 && (o->inner_max < 1 || o->inner_max > 8 || !(o->inner_tol >= 0.f)))
        return fail(ctx, NOSDD_EINVAL, "inner_max must be in [1, 8] and inner_tol >= 0");
    hipStream_t s = ctx->stream;
    CallResources res;
    HIPCHK(ctx, hipEventCreate(&res.e0));
    HIPCHK(ctx, hipEventCreate(&res.e1));
    HIPCHK(ctx, hipEventRecord(res.e0, s));
    const int nwl = (int)p->wl.size();
    HIPCHK(ctx, p->d_dinv.ensure((size_t)nwl * p->dinv_wl_stride * sizeof(float2)));
    {
        // tiles whose short side exceeds the LDS factorisation limit work in global scratch
        std::vector<int> big;
        for (int t = 0; t < (int)p->tiles.size(); ++t)
            if (p->tiles[t].b > 72) big.push_back(t);
        DevBuf d_big, d_scr;
        if (!big.empty()) {
            HIPCHK(ctx, d_big.ensure(big.size() * sizeof(int)));
            HIPCHK(ctx, hipMemcpy(d_big.p, big.data(), big.size() * sizeof(int), hipMemcpyHostToDevice));
            HIPCHK(ctx, d_scr.ensure((size_t)nwl * big.size() * BT_FACT_SCRATCH_B * BT_FACT_SCRATCH_B *
                                     sizeof(double2)));
        }
        launch_bt_factor(s, p->d_tiles.as<TileDesc>(), (int)p->tiles.size(), nwl, p->d_eps.as<float>(),
                         p->d_coefd.as<double>(), p->d_k0.as<double>(), p->h, p->nx, p->ny, p->d_sc.as<float2>(),
                         p->d_dinv.as<float2>(),
                         p->dinv_wl_stride, d_big.as<int>(), (int)big.size(), d_scr.as<double2>());
        HIPCHK(ctx, hipGetLastError());
        HIPCHK(ctx, hipStreamSynchronize(s));
    }
    bt_solve_prepare(p->bmax, p->max_cells);
    if (p->bmax <= 112) bt_solve_multi_prepare(p->bmax);
    fno_prepare();
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(s));
    {
        // Robin-data injection inj(g)_p = -a_pq tau_p g_p per (wavelength, entry)
        const int ne = p->n_entries;
        std::vector<float2> ic((size_t)nwl * std::max(ne, 1), make_float2(0.f, 0.f));
        for (int wi = 0; wi < nwl; ++wi) {
            const double k0 = 2.0 * M_PI / p->wl[wi];
            const auto &cf = p->coefd[wi];
            for (int ti = 0; ti < (int)p->tiles.size(); ++ti) {
                const auto &ent = p->tile_entries[ti];
                for (int e = 0; e < (int)ent.size(); ++e) {
                    const int pc = ent[e].x, px = pc % p->nx, py = pc / p->nx;
                    cd apq;
                    switch (ent[e].z) {
                        case SIDE_LEFT: apq = cf[px]; break;
                        case SIDE_RIGHT: apq = cf[p->nx + px]; break;
                        case SIDE_BOTTOM: apq = cf[2 * p->nx + py]; break;
                        default: apq = cf[2 * p->nx + p->ny + py]; break;
                    }
                    const double kp = k0 * std::sqrt((double)p->eps[pc]);
                    const cd v = -apq * (p->h / cd(1.0, 0.5 * kp * p->h));
                    ic[(size_t)wi * ne + p->tiles[ti].tr_off + e] = make_float2((float)v.real(), (float)v.imag());
                }
            }
        }
        HIPCHK(ctx, p->d_injc.ensure(ic.size() * sizeof(float2)));
        HIPCHK(ctx, hipMemcpy(p->d_injc.p, ic.data(), ic.size() * sizeof(float2), hipMemcpyHostToDevice));
    }
    if (o->sub_solver == 1) {
        for (auto &t : p->tiles)
            if (t.x1 - t.x0 > 72 || t.y1 - t.y0 > 72 || t.x1 - t.x0 < 32 || t.y1 - t.y0 < 32)
                return fail(ctx, NOSDD_EPARTITION,
                            "the neural subdomain solver takes subdomains of 32 x 32 to 72 x 72 cells");
        st = load_network(p, o->nn_weights);
        if (st) return st;
        st = build_aux(p);
        if (st) return st;
        p->nn_steps = o->inner_max;
        p->nn_tol = o->inner_tol;
        p->smp_rhs = 0;
    }
    p->sub_solver = 0;          // the coarse probes below use the exact subdomain solves
    p->kc = (p->tiles.size() > 1) ? o->k_coarse : 0;
    p->ktrial = o->k_trial > 0 ? o->k_trial : 8;
    p->n_c = 0;
    if (p->kc > 0) {
        if (p->kc > std::max(p->ktrial, p->kc) || std::max(p->ktrial, p->kc) > 64)
            return fail(ctx, NOSDD_EINVAL, "k_trial must be at most 64");
        st = coarse_setup(p);
        if (st) return st;
    }
    HIPCHK(ctx, hipEventRecord(res.e1, s));
    HIPCHK(ctx, hipEventSynchronize(res.e1));
    float ms = 0;
    (void)hipEventElapsedTime(&ms, res.e0, res.e1);
    p->setup_ms = ms;
    p->sub_solver = o->sub_solver;
    p->setup_done = true;
    p->drop_graphs();
    p->bt_tuned = false;
    p->bt_depth = 0;
    return NOSDD_OK;
}

void nosdd_problem_destroy(nosdd_problem *p) {
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    (void)hipStreamSynchronize(p->ctx->stream);
    delete p;
}

static nosdd_status validate_solve(nosdd_problem *p, const void *J, int n_src, const nosdd_solve_opts *o, const void *E) {
    nosdd_status st = check_problem(p, true);
    if (st) return st;
    if (!J || !o || !E || n_src <= 0) return fail(p->ctx, NOSDD_EINVAL, "null argument or n_src <= 0");
    if (o->restart < 1 || o->restart > 31) return fail(p->ctx, NOSDD_EINVAL, "restart must be in [1, 31]");
    if (o->max_iters < 0 || !(o->tol > 0)) return fail(p->ctx, NOSDD_EINVAL, "invalid tolerance or max_iters");
    return NOSDD_OK;
}

nosdd_status nosdd_solve_device(nosdd_problem *p, const nosdd_c32 *J_dev, int n_src, const nosdd_solve_opts *o,
                                nosdd_c32 *E_dev, float *resid_hist, int *iters, float *final_resid) {
    nosdd_status st = validate_solve(p, J_dev, n_src, o, E_dev);
    if (st) return st;
    return solve_impl(p, (const float2 *)J_dev, n_src, o, (const float2 *)o->x0, (float2 *)E_dev, resid_hist, iters,
                      final_resid);
}

nosdd_status nosdd_solve_device_c64(nosdd_problem *p, const nosdd_c32 *J_dev, int n_src, const nosdd_solve_opts *o,
                                    nosdd_c64 *E64_dev, float *resid_hist, int *iters, float *final_resid) {
    nosdd_status st = validate_solve(p, J_dev, n_src, o, E64_dev);
    if (st) return st;
    return solve_impl(p, (const float2 *)J_dev, n_src, o, (const float2 *)o->x0, nullptr, resid_hist, iters,
                      final_resid, false, (double2 *)E64_dev);
}

nosdd_status nosdd_solve_paper_device(nosdd_problem *p, const nosdd_c32 *J_dev, int n_src, const nosdd_paper_opts *o,
                                      nosdd_c32 *E_dev, float *resid_hist, int *iters, float *final_resid) {
    nosdd_status st = check_problem(p, true);
    if (st) return st;
    nosdd_ctx *ctx = p->ctx;
    if (!J_dev || !o || !E_dev || n_src <= 0) return fail(ctx, NOSDD_EINVAL, "null argument or n_src <= 0");
    if (!(o->momentum >= 0.0 && o->momentum < 1.0)) return fail(ctx, NOSDD_EINVAL, "momentum must be in [0, 1)");
    if (o->max_iters < 1 || !(o->tol > 0)) return fail(ctx, NOSDD_EINVAL, "invalid tolerance or max_iters");
    if (p->sub_solver != 0) return fail(ctx, NOSDD_EINVAL, "the Algorithm 3 loop takes exact subdomain solves");
    if (o->coarse && p->n_c == 0) return fail(ctx, NOSDD_EINVAL, "coarse correction requested without a coarse space");
    hipStream_t s = ctx->stream;
    const int n_wl = (int)p->wl.size(), n_rhs = n_wl * n_src, nt = (int)p->tiles.size();
    const long long N = (long long)p->nx * p->ny, LT = p->loc_total;
    const int ne = p->n_entries, nc = p->n_c;
    DevBuf b, r, rhs, g, gn, d, z, part, nrm, act;
    HIPCHK(ctx, b.ensure((size_t)n_rhs * N * sizeof(float2)));
    HIPCHK(ctx, r.ensure((size_t)n_rhs * N * sizeof(float2)));
    HIPCHK(ctx, rhs.ensure((size_t)n_rhs * LT * sizeof(float2)));
    HIPCHK(ctx, g.ensure((size_t)n_rhs * std::max(ne, 1) * sizeof(float2)));
    HIPCHK(ctx, gn.ensure((size_t)n_rhs * std::max(ne, 1) * sizeof(float2)));
    HIPCHK(ctx, d.ensure((size_t)n_rhs * std::max(nc, 1) * sizeof(double2)));
    HIPCHK(ctx, z.ensure((size_t)n_rhs * std::max(nc, 1) * sizeof(float2)));
    HIPCHK(ctx, part.ensure((size_t)n_rhs * norm2_partials() * sizeof(double)));
    HIPCHK(ctx, nrm.ensure((size_t)n_rhs * sizeof(double)));
    HIPCHK(ctx, act.ensure((size_t)n_rhs * sizeof(int)));
    const int2 *ord = nullptr;
    int nj = 0;
    st = solve_order(p, n_rhs, n_src, &ord, &nj);
    if (st != NOSDD_OK) return st;
    hipLaunchKernelGGL(make_rhs_kernel, dim3((unsigned)grid_blocks(N), n_rhs), dim3(256), 0, s, (const float2 *)J_dev,
                       b.as<float2>(), p->d_k0f.as<float>(), N, n_src, 0);
    HIPCHK(ctx, hipMemsetAsync(g.p, 0, (size_t)n_rhs * std::max(ne, 1) * sizeof(float2), s));
    std::vector<double> n2(n_rhs), bn(n_rhs);
    launch_norm2(s, b.as<float2>(), N, n_rhs, part.as<double>(), nrm.as<double>());
    HIPCHK(ctx, hipMemcpyAsync(n2.data(), nrm.p, n_rhs * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    std::vector<int> active(n_rhs), it(n_rhs, 0);
    std::vector<float> last(n_rhs, 0.f);
    for (int q = 0; q < n_rhs; ++q) {
        bn[q] = std::sqrt(n2[q]);
        active[q] = bn[q] > 0.0 ? 1 : 0;
    }
    if (resid_hist)
        for (size_t q = 0; q < (size_t)n_rhs * o->max_iters; ++q) resid_hist[q] = -1.f;
    // zero sources: zero field, no sweeps
    hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)grid_blocks(2LL * n_rhs * N)), dim3(256), 0, s, (float *)E_dev,
                       2LL * n_rhs * N, 0.0f);
    const float m = (float)o->momentum;
    for (int k = 0; k < o->max_iters; ++k) {
        int n_act = 0;
        for (int q = 0; q < n_rhs; ++q) n_act += active[q];
        if (!n_act) break;
        HIPCHK(ctx, hipMemcpyAsync(act.p, active.data(), n_rhs * sizeof(int), hipMemcpyHostToDevice, s));
        // sweep: local right-hand sides, subdomain solves, core-only assembly
        launch_robin_rhs(s, p->d_tiles.as<TileDesc>(), nt, p->d_entries.as<int4>(), p->d_injc.as<float2>(), ne,
                         b.as<float2>(), g.as<float2>(), rhs.as<float2>(), N, LT, p->nx, n_rhs, n_src, act.as<int>());
        launch_bt_solve(s, p->d_tiles.as<TileDesc>(), ord, nj, n_src, p->d_dinv.as<float2>(), p->dinv_wl_stride,
                        p->d_coef.as<float2>(), p->d_sc.as<float2>(), p->nx, p->ny, rhs.as<float2>(), LT,
                        (float2 *)E_dev, N, act.as<int>(), 1, p->bmax, p->max_cells, p->bt_depth);
        // ||b - A x|| after the sweep
        launch_stencil(s, (const float2 *)E_dev, b.as<float2>(), r.as<float2>(), p->d_eps.as<float>(),
                       p->d_coefd.as<double2>(), p->d_k0.as<double>(), p->nx, p->ny, n_rhs, n_src, act.as<int>());
        launch_norm2(s, r.as<float2>(), N, n_rhs, part.as<double>(), nrm.as<double>());
        // data of the next sweep (used only by the RHS that stay active)
        launch_robin_trace(s, p->d_entries.as<int4>(), ne, p->d_eps.as<float>(), p->d_k0f.as<float>(), (float)p->h,
                           p->nx, p->ny, (const float2 *)E_dev, gn.as<float2>(), n_rhs, n_src);
        if (o->coarse) {
            launch_rc_dot(s, p->d_rc_colptr.as<int>(), p->d_rc_colent.as<int>(), p->d_rc_colval.as<float2>(),
                          p->rc_nnz, nc, ne, g.as<float2>(), gn.as<float2>(), d.as<double2>(), n_rhs, n_src,
                          act.as<int>());
            launch_coarse_solve(s, p->d_rc_GinvT.as<double2>(), nc, d.as<double2>(), z.as<float2>(), n_rhs, n_src,
                                act.as<int>());
        }
        launch_rc_update(s, p->d_rc_rowptr.as<int>(), p->d_rc_rowcol.as<int>(), p->d_rc_q.as<float2>(),
                         p->d_rc_tq.as<float2>(), p->rc_nnz, ne, nc, g.as<float2>(), gn.as<float2>(), z.as<float2>(),
                         m, o->coarse ? 1 : 0, n_rhs, n_src, act.as<int>());
        HIPCHK(ctx, hipGetLastError());
        HIPCHK(ctx, hipMemcpyAsync(n2.data(), nrm.p, n_rhs * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        for (int q = 0; q < n_rhs; ++q) {
            if (!active[q]) continue;
            const float res = (float)(std::sqrt(n2[q]) / bn[q]);
            if (resid_hist) resid_hist[(size_t)q * o->max_iters + k] = res;
            it[q] = k + 1;
            last[q] = res;
            if (res <= o->tol) active[q] = 0;              // a NaN residual keeps iterating
        }
    }
    bool all = true;
    for (int q = 0; q < n_rhs; ++q) {
        if (iters) iters[q] = it[q];
        if (final_resid) final_resid[q] = last[q];
        if (active[q]) all = false;
    }
    return all ? NOSDD_OK : NOSDD_NOT_CONVERGED;
}

nosdd_status nosdd_fom_gradient_device(nosdd_problem *p, const nosdd_c32 *J_dev, int n_src, const int *focal,
                                       int n_focal, const nosdd_solve_opts *o, double *fom, float *grad_dev,
                                       int *iters) {
    nosdd_status st = validate_solve(p, J_dev, n_src, o, grad_dev);
    if (st) return st;
    nosdd_ctx *ctx = p->ctx;
    if (!focal || n_focal <= 0) return fail(ctx, NOSDD_EINVAL, "no focal cells");
    for (int f = 0; f < n_focal; ++f)
        if (focal[2 * f] < 0 || focal[2 * f] >= p->nx || focal[2 * f + 1] < 0 || focal[2 * f + 1] >= p->ny)
            return fail(ctx, NOSDD_EINVAL, "focal cell outside the grid");
    hipStream_t s = ctx->stream;
    const int n_rhs = (int)p->wl.size() * n_src;
    const long long N = (long long)p->nx * p->ny;
    const size_t vec = (size_t)n_rhs * N * sizeof(float2);
    HIPCHK(ctx, p->adj_E.ensure(vec));
    HIPCHK(ctx, p->adj_mu.ensure(vec));
    HIPCHK(ctx, p->adj_J.ensure(vec));
    HIPCHK(ctx, p->adj_focal.ensure((size_t)n_focal * sizeof(int2)));
    HIPCHK(ctx, p->adj_fom.ensure((size_t)n_rhs * n_focal * sizeof(double)));
    HIPCHK(ctx, hipMemcpyAsync(p->adj_focal.p, focal, (size_t)n_focal * sizeof(int2), hipMemcpyHostToDevice, s));
    nosdd_solve_opts fo = *o;
    fo.x0 = nullptr;
    std::vector<int> it_f(n_rhs, 0), it_a(n_rhs, 0);
    // forward fields
    nosdd_status sf = solve_impl(p, (const float2 *)J_dev, n_src, &fo, nullptr, p->adj_E.as<float2>(), nullptr,
                                 it_f.data(), nullptr);
    if (sf < 0) return sf;
    // |E(r_f)|^2 and the adjoint current at the focal cells
    hipLaunchKernelGGL(fill_f32_kernel, dim3((unsigned)grid_blocks(2LL * n_rhs * N)), dim3(256), 0, s,
                       p->adj_J.as<float>(), 2LL * n_rhs * N, 0.0f);
    launch_adjoint_rhs(s, p->adj_E.as<float2>(), N, p->nx, p->ny, p->adj_focal.as<int2>(), n_focal,
                       p->d_sc.as<float2>(), p->d_k0f.as<float>(), n_rhs, n_src, p->adj_J.as<float2>(),
                       p->adj_fom.as<double>());
    HIPCHK(ctx, hipGetLastError());
    // adjoint fields mu (A mu = S^-1 P conj(E)), then the gradient
    nosdd_status sa = solve_impl(p, p->adj_J.as<float2>(), n_src, &fo, nullptr, p->adj_mu.as<float2>(), nullptr,
                                 it_a.data(), nullptr, true);
    if (sa < 0) return sa;
    launch_adjoint_grad(s, p->adj_E.as<float2>(), p->adj_mu.as<float2>(), N, p->nx, p->ny, n_rhs, n_src,
                        p->d_sc.as<float2>(), p->d_k0f.as<float>(), (float *)grad_dev);
    HIPCHK(ctx, hipGetLastError());
    std::vector<double> fv((size_t)n_rhs * n_focal);
    HIPCHK(ctx, hipMemcpyAsync(fv.data(), p->adj_fom.p, fv.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (fom) {
        double t = 0.0;
        for (double v : fv) t += v;
        *fom = t;
    }
    if (iters)
        for (int r = 0; r < n_rhs; ++r) {
            iters[r] = it_f[r];
            iters[n_rhs + r] = it_a[r];
        }
    return (sf == NOSDD_NOT_CONVERGED || sa == NOSDD_NOT_CONVERGED) ? NOSDD_NOT_CONVERGED : NOSDD_OK;
}

nosdd_status nosdd_solve(nosdd_problem *p, const nosdd_c32 *J, int n_src, const nosdd_solve_opts *o, nosdd_c32 *E_out,
                         float *resid_hist, int *iters, float *final_resid) {
    nosdd_status st = validate_solve(p, J, n_src, o, E_out);
    if (st) return st;
    nosdd_ctx *ctx = p->ctx;
    hipStream_t s = ctx->stream;
    const long long N = (long long)p->nx * p->ny;
    const int n_rhs = (int)p->wl.size() * n_src;
    DevBuf dJ, dE, dx0;
    HIPCHK(ctx, dJ.ensure((size_t)n_src * N * sizeof(float2)));
    HIPCHK(ctx, dE.ensure((size_t)n_rhs * N * sizeof(float2)));
    HIPCHK(ctx, hipMemcpyAsync(dJ.p, J, (size_t)n_src * N * sizeof(float2), hipMemcpyHostToDevice, s));
    nosdd_solve_opts od = *o;
    if (o->x0) {
        HIPCHK(ctx, dx0.ensure((size_t)n_rhs * N * sizeof(float2)));
        HIPCHK(ctx, hipMemcpyAsync(dx0.p, o->x0, (size_t)n_rhs * N * sizeof(float2), hipMemcpyHostToDevice, s));
        od.x0 = (const nosdd_c32 *)dx0.p;
    }
    st = solve_impl(p, dJ.as<float2>(), n_src, &od, (const float2 *)od.x0, dE.as<float2>(), resid_hist, iters,
                    final_resid);
    if (st < 0) return st;
    HIPCHK(ctx, hipMemcpyAsync(E_out, dE.p, (size_t)n_rhs * N * sizeof(float2), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return st;
}

nosdd_status nosdd_apply_operator(nosdd_problem *p, const nosdd_c32 *x, const nosdd_c32 *b, nosdd_c32 *y, int n_src) {
    nosdd_status st = check_problem(p, false);
    if (st) return st;
    if (!x || !y || n_src <= 0) return fail(p->ctx, NOSDD_EINVAL, "null argument or n_src <= 0");
    launch_stencil(p->ctx->stream, (const float2 *)x, (const float2 *)b, (float2 *)y, p->d_eps.as<float>(),
                   p->d_coefd.as<double2>(), p->d_k0.as<double>(), p->nx, p->ny, (int)p->wl.size() * n_src, n_src,
                   nullptr);
    HIPCHK(p->ctx, hipGetLastError());
    return NOSDD_OK;
}

nosdd_status nosdd_schwarz_sweep(nosdd_problem *p, const nosdd_c32 *v, nosdd_c32 *z, int n_src) {
    nosdd_status st = check_problem(p, true);
    if (st) return st;
    if (!v || !z || n_src <= 0) return fail(p->ctx, NOSDD_EINVAL, "null argument or n_src <= 0");
    const int n_rhs = (int)p->wl.size() * n_src;
    const long long N = (long long)p->nx * p->ny;
    const int2 *ord = nullptr;
    int nj = 0;
    st = solve_order(p, n_rhs, n_src, &ord, &nj);
    if (st) return st;
    (void)N;
    HIPCHK(p->ctx, p->ws.loc.ensure((size_t)n_rhs * p->loc_total * sizeof(float2)));
    local_sweep(p, p->ctx->stream, (const float2 *)v, (float2 *)z, n_rhs, n_src, nullptr);
    HIPCHK(p->ctx, hipGetLastError());
    HIPCHK(p->ctx, hipStreamSynchronize(p->ctx->stream));
    return NOSDD_OK;
}

nosdd_status nosdd_precond_apply(nosdd_problem *p, const nosdd_c32 *v, nosdd_c32 *z, nosdd_c32 *Az, int n_src) {
    nosdd_status st = check_problem(p, true);
    if (st) return st;
    if (!v || !z || n_src <= 0) return fail(p->ctx, NOSDD_EINVAL, "null argument or n_src <= 0");
    const int n_rhs = (int)p->wl.size() * n_src;
    st = ensure_ws(p, n_rhs, std::max(1, p->ws.m), std::max(1, p->ws.max_iters));
    if (st) return st;
    if (p->sub_solver == 1) {
        st = ensure_nn(p, n_rhs, n_src);
        if (st) return st;
    }
    {
        const int2 *ord = nullptr;
        int nj = 0;
        st = solve_order(p, n_rhs, n_src, &ord, &nj);
        if (st) return st;
    }
    const long long N = (long long)p->nx * p->ny;
    DevBuf tmp;
    float2 *w = (float2 *)Az;
    if (!w) {
        HIPCHK(p->ctx, tmp.ensure((size_t)n_rhs * N * sizeof(float2)));
        w = tmp.as<float2>();
    }
    precond(p, p->ctx->stream, (const float2 *)v, (float2 *)z, w, n_src, n_rhs, nullptr, n_rhs);
    HIPCHK(p->ctx, hipGetLastError());
    HIPCHK(p->ctx, hipStreamSynchronize(p->ctx->stream));
    return NOSDD_OK;
}

nosdd_status nosdd_precond_apply_noalloc(nosdd_problem *p, const nosdd_c32 *v, nosdd_c32 *z, nosdd_c32 *Az,
                                         int n_src) {
    static_assert(NOALLOC_SCRATCH_BYTES == NOSDD_NOALLOC_SCRATCH_BYTES, "scratch size differs from the header");
    nosdd_status st = check_problem(p, true);
    if (st) return st;
    if (!v || !z || !Az || n_src <= 0) return fail(p->ctx, NOSDD_EINVAL, "null argument or n_src <= 0");
    if (p->sub_solver != 0)
        return fail(p->ctx, NOSDD_ESTATE, "the allocation-free sweep takes exact subdomain solves (sub_solver 0)");
    const long long nt = (long long)p->tiles.size(), n_rhs = (long long)p->wl.size() * n_src;
    const long long nc = p->n_c;
    auto up = [](long long b) { return (b + 255) / 256 * 256; };
    const long long q_bytes = up(nt * n_rhs * (long long)sizeof(int2));
    const long long d_bytes = up(n_rhs * nc * (long long)sizeof(double2));
    const long long c_bytes = up(n_rhs * nc * (long long)sizeof(float2));
    if (n_rhs > (1 << 20) || q_bytes + d_bytes + c_bytes > (long long)NOALLOC_SCRATCH_BYTES)
        return fail(p->ctx, NOSDD_EINVAL,
                    "batch too large for the fixed scratch: needs " + std::to_string(q_bytes + d_bytes + c_bytes) +
                        " bytes, at most " + std::to_string((long long)NOALLOC_SCRATCH_BYTES));
    char *scr = static_cast<char *>(noalloc_scratch(p->ctx->device));
    if (!scr) return fail(p->ctx, NOSDD_ESTATE, "no scratch address for this device");
    int2 *order = reinterpret_cast<int2 *>(scr);
    double2 *cd = reinterpret_cast<double2 *>(scr + q_bytes);
    float2 *cc = reinterpret_cast<float2 *>(scr + q_bytes + d_bytes);
    hipStream_t s = p->ctx->stream;
    const long long N = (long long)p->nx * p->ny;
    // every entry of the queue, d and c is written before it is read: nothing to clear
    launch_noalloc_queue(s, order, (int)nt, (int)n_rhs);
    launch_bt_solve(s, p->d_tiles.as<TileDesc>(), order, (int)(nt * n_rhs), n_src, p->d_dinv.as<float2>(),
                    p->dinv_wl_stride, p->d_coef.as<float2>(), p->d_sc.as<float2>(), p->nx, p->ny, (const float2 *)v, N,
                    (float2 *)z, N, nullptr, 0, p->bmax, p->max_cells, p->bt_depth);
    launch_stencil(s, (const float2 *)z, nullptr, (float2 *)Az, p->d_eps.as<float>(), p->d_coefd.as<double2>(),
                   p->d_k0.as<double>(), p->nx, p->ny, (int)n_rhs, n_src, nullptr);
    if (nc > 0) {
        launch_coarse_dot(s, p->d_tiles.as<TileDesc>(), p->n_c, p->kc, p->d_W.as<float2>(), p->box_wl_stride,
                          (const float2 *)v, (const float2 *)Az, p->nx, N, (int)n_rhs, n_src, nullptr, cd);
        launch_coarse_solve(s, p->d_GinvT.as<double2>(), p->n_c, cd, cc, (int)n_rhs, n_src, nullptr);
        launch_coarse_update(s, p->d_tiles.as<TileDesc>(), p->d_owner.as<int>(), p->kc, p->d_phi.as<float2>(),
                             p->d_W.as<float2>(), p->box_wl_stride, cc, p->n_c, (float2 *)z, (float2 *)Az, p->nx, p->ny,
                             (int)n_rhs, n_src, nullptr);
    }
    HIPCHK(p->ctx, hipGetLastError());
    return NOSDD_OK;
}

nosdd_status nosdd_local_solve(nosdd_problem *p, const nosdd_c32 *rhs, nosdd_c32 *u) {
    nosdd_status st = check_problem(p, true);
    if (st) return st;
    if (!rhs || !u) return fail(p->ctx, NOSDD_EINVAL, "null argument");
    const int nwl = (int)p->wl.size();
    if (p->sub_solver == 1) {
        st = ensure_nn(p, nwl, 1);
        if (st) return st;
        nn_sweep(p, p->ctx->stream, (const float2 *)rhs, (float2 *)u, nwl, 1, nullptr, 1);
        HIPCHK(p->ctx, hipGetLastError());
        HIPCHK(p->ctx, hipStreamSynchronize(p->ctx->stream));
        return NOSDD_OK;
    }
    const int2 *ord = nullptr;
    int nj = 0;
    st = solve_order(p, nwl, 1, &ord, &nj);
    if (st) return st;
    launch_bt_solve(p->ctx->stream, p->d_tiles.as<TileDesc>(), ord, nj, 1, p->d_dinv.as<float2>(), p->dinv_wl_stride,
                    p->d_coef.as<float2>(), p->d_sc.as<float2>(), p->nx, p->ny, (const float2 *)rhs, p->loc_total, (float2 *)u,
                    p->loc_total, nullptr, 3, p->bmax, p->max_cells);
    HIPCHK(p->ctx, hipGetLastError());
    HIPCHK(p->ctx, hipStreamSynchronize(p->ctx->stream));
    return NOSDD_OK;
}

nosdd_status nosdd_nn_apply(nosdd_problem *p, const nosdd_c32 *v, nosdd_c32 *e) {
    nosdd_status st = check_problem(p, true);
    if (st) return st;
    if (!v || !e) return fail(p->ctx, NOSDD_EINVAL, "null argument");
    if (p->sub_solver != 1) return fail(p->ctx, NOSDD_ESTATE, "the problem was not set up with the neural solver");
    const int nwl = (int)p->wl.size();
    st = ensure_nn(p, nwl, 1);
    if (st) return st;
    hipStream_t s = p->ctx->stream;
    const int S = nwl * (int)p->tiles.size();
    nn_rms_scales(s, p->nw.smp, S, (const float2 *)v, p->nw.vscale, p->nw.oscale);
    fno_forward(s, p->net, p->nw.smp, nullptr, S, p->max_cells, (const float2 *)v, p->nw.vscale, p->nw.oscale,
                p->nw.aux, p->loc_total, p->nw.act0, p->nw.act1, p->nw.spec, p->nw.X, p->nw.Y, (float2 *)e);
    HIPCHK(p->ctx, hipGetLastError());
    HIPCHK(p->ctx, hipStreamSynchronize(s));
    return NOSDD_OK;
}

nosdd_status nosdd_robin_trace(nosdd_problem *p, const nosdd_c32 *x, nosdd_c32 *g) {
    nosdd_status st = check_problem(p, false);
    if (st) return st;
    if (!x || !g) return fail(p->ctx, NOSDD_EINVAL, "null argument");
    launch_robin_trace(p->ctx->stream, p->d_entries.as<int4>(), p->n_entries, p->d_eps.as<float>(), p->d_k0f.as<float>(),
                       (float)p->h, p->nx, p->ny, (const float2 *)x, (float2 *)g, (int)p->wl.size(), 1);
    HIPCHK(p->ctx, hipGetLastError());
    return NOSDD_OK;
}

nosdd_status nosdd_tile_info(const nosdd_problem *p, int tile, long long info[10]) {
    if (!p || !info || tile < 0 || tile >= (int)p->tiles.size()) return NOSDD_EINVAL;
    const TileDesc &t = p->tiles[tile];
    const long long v[10] = {t.x0, t.x1, t.y0, t.y1, t.cx0, t.cx1, t.cy0, t.cy1, t.loc_off, t.tr_off};
    for (int i = 0; i < 10; ++i) info[i] = v[i];
    return NOSDD_OK;
}

nosdd_status nosdd_sizes(const nosdd_problem *p, int *n_tiles, long long *local_cells, long long *trace_entries,
                         int *n_coarse) {
    if (!p) return NOSDD_EINVAL;
    if (n_tiles) *n_tiles = (int)p->tiles.size();
    if (local_cells) *local_cells = p->loc_total;
    if (trace_entries) *trace_entries = p->n_entries;
    if (n_coarse) *n_coarse = p->n_c;
    return NOSDD_OK;
}

nosdd_status nosdd_coarse_basis(const nosdd_problem *p, int wl, nosdd_c32 *phi, long long *box) {
    if (!p || wl < 0 || wl >= (int)p->wl.size()) return NOSDD_EINVAL;
    if (box)
        for (size_t t = 0; t < p->tiles.size(); ++t) {
            box[4 * t] = p->tiles[t].bx0;
            box[4 * t + 1] = p->tiles[t].by0;
            box[4 * t + 2] = p->tiles[t].bw;
            box[4 * t + 3] = p->tiles[t].bh;
        }
    if (phi && p->n_c > 0) {
        if (hipSetDevice(p->ctx->device) != hipSuccess) return NOSDD_EHIP;
        if (hipMemcpy(phi, p->d_phi.as<float2>() + wl * p->box_wl_stride, p->box_wl_stride * sizeof(float2),
                      hipMemcpyDeviceToHost) != hipSuccess)
            return NOSDD_EHIP;
    }
    return NOSDD_OK;
}

nosdd_status nosdd_profile(nosdd_problem *p, int enable) {
    if (!p) return NOSDD_EINVAL;
    if (enable) {
        for (int i = 0; i < 4; ++i) {
            p->prof_ms[i] = 0;
            p->prof_launch[i] = p->prof_units[i] = 0;
        }
        p->ev_pending.clear();
        p->ev_next = 0;
    }
    p->prof = enable != 0;
    return NOSDD_OK;
}

nosdd_status nosdd_autotune(nosdd_problem *p, int enable) {
    if (!p) return NOSDD_EINVAL;
    p->use_autotune = enable != 0;
    if (!p->use_autotune) {
        p->ws.tuned = false;
        for (int &v : p->ws.nblk_b) v = p->ws.nblk;
        p->bt_tuned = false;
        p->bt_depth = 0;
        p->drop_graphs();
    }
    return NOSDD_OK;
}

nosdd_status nosdd_tuning(const nosdd_problem *p, int out[6]) {
    if (!p || !out) return NOSDD_EINVAL;
    out[0] = p->bt_depth;
    for (int i = 0; i < 4; ++i) out[1 + i] = p->ws.nblk_b[i];
    out[5] = (p->ws.tuned ? 1 : 0) | (p->bt_tuned ? 2 : 0);
    return NOSDD_OK;
}

nosdd_status nosdd_graphs(nosdd_problem *p, int enable) {
    if (!p) return NOSDD_EINVAL;
    p->use_graphs = enable != 0;
    if (!p->use_graphs) p->drop_graphs();
    return NOSDD_OK;
}

nosdd_status nosdd_multi_source(nosdd_problem *p, int enable) {
    if (!p) return NOSDD_EINVAL;
    p->use_multi = enable != 0;
    p->orders.clear();                            // launch queues are rebuilt with or without the grouped jobs
    p->drop_graphs();
    return NOSDD_OK;
}

nosdd_status nosdd_stored_basis(nosdd_problem *p, int enable) {
    if (!p) return NOSDD_EINVAL;
    p->stored_basis = enable != 0;
    p->drop_graphs();                             // the captured steps launch different kernels
    p->ws.tuned = false;                          // and the Gram-Schmidt grid is timed on those kernels
    return NOSDD_OK;
}

nosdd_status nosdd_kernel_times(const nosdd_problem *p, double ms[4], long long launches[4], long long units[4]) {
    if (!p) return NOSDD_EINVAL;
    for (int i = 0; i < 4; ++i) {
        if (ms) ms[i] = p->prof_ms[i];
        if (launches) launches[i] = p->prof_launch[i];
        if (units) units[i] = p->prof_units[i];
    }
    return NOSDD_OK;
}

nosdd_status nosdd_fallback_count(const nosdd_problem *p, long long *count) {
    if (!p || !count) return NOSDD_EINVAL;
    *count = 0;
    if (!p->nn_fbcount.p) return NOSDD_OK;
    unsigned c = 0;
    HIPCHK(p->ctx, hipMemcpyAsync(&c, p->nn_fbcount.p, sizeof(unsigned), hipMemcpyDeviceToHost, p->ctx->stream));
    HIPCHK(p->ctx, hipStreamSynchronize(p->ctx->stream));
    *count = c;
    return NOSDD_OK;
}

nosdd_status nosdd_last_timing(const nosdd_problem *p, double *setup_ms, double *solve_ms, int *outer_iters) {
    if (!p) return NOSDD_EINVAL;
    if (setup_ms) *setup_ms = p->setup_ms;
    if (solve_ms) *solve_ms = p->solve_ms;
    if (outer_iters) *outer_iters = p->last_iters;
    return NOSDD_OK;
}

}  // extern "C"
