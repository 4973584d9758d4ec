// Adjoint-variables gradient of the inverse-design figure of merit
//   FoM = sum over wavelengths, sources and focal cells f of |E(r_f)|^2,
//   dFoM/deps_p = 2 k0^2 Re(E_p lam_p),   A^T lam = P conj(E),
// (dA/deps_p = -k0^2 e_p e_p^T).  With S = diag(s_x s_y) at cell centres the
// stretched operator S A is complex symmetric, so A^T = S A S^-1 and
// lam = S mu with A mu = S^-1 P conj(E): the adjoint field comes from the
// forward solver with another right-hand side.
#include "common.h"

namespace nosdd {

// One thread per RHS r: fomv[r][f] = |E_r(r_f)|^2 and the adjoint current at
// the focal cells, J_adj[r] = (i / k0) S^-1 conj(E_r) there (so that the
// solver's b = -i k0 J_adj is S^-1 P conj(E_r)); J_adj must be zero elsewhere.
__global__ void adjoint_rhs_kernel(const float2 *__restrict__ E, long long N, int nx, int ny,
                                   const int2 *__restrict__ focal, int n_focal, const float2 *__restrict__ sc,
                                   const float *__restrict__ k0f, int n_rhs, int n_src, float2 *__restrict__ Jadj,
                                   double *__restrict__ fomv) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n_rhs) return;
    const int wl = r / n_src;
    const float2 *sx = sc + (long long)wl * (nx + ny), *sy = sx + nx;
    const float ik0 = 1.f / k0f[wl];
    for (int f = 0; f < n_focal; ++f) {
        const int2 c = focal[f];
        const long long idx = (long long)c.y * nx + c.x;
        const float2 e = E[r * N + idx];
        fomv[(long long)r * n_focal + f] = (double)e.x * e.x + (double)e.y * e.y;
        const float2 S = cmul(sx[c.x], sy[c.y]);
        const float ss = cabs2(S);
        // conj(e) / S = conj(e) conj(S) / |S|^2
        const float2 g = make_float2((e.x * S.x - e.y * S.y) / ss, (-e.y * S.x - e.x * S.y) / ss);
        float2 &j = Jadj[r * N + idx];
        j = make_float2(j.x - g.y * ik0, j.y + g.x * ik0);      // += i g / k0
    }
}

// grad[cell] = sum_r 2 k0(r)^2 Re(E_r[cell] S_r(cell) mu_r[cell]), summed in FP64.
__global__ void adjoint_grad_kernel(const float2 *__restrict__ E, const float2 *__restrict__ mu, long long N, int nx,
                                    int ny, int n_rhs, int n_src, const float2 *__restrict__ sc,
                                    const float *__restrict__ k0f, float *__restrict__ grad) {
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N; n += (long long)gridDim.x * blockDim.x) {
        const int iy = (int)(n / nx), ix = (int)(n - (long long)iy * nx);
        double acc = 0.0;
        for (int r = 0; r < n_rhs; ++r) {
            const int wl = r / n_src;
            const float2 *sx = sc + (long long)wl * (nx + ny), *sy = sx + nx;
            const float2 lam = cmul(cmul(sx[ix], sy[iy]), mu[r * N + n]);
            const float2 e = E[r * N + n];
            const double k0 = k0f[wl];
            acc += 2.0 * k0 * k0 * ((double)e.x * lam.x - (double)e.y * lam.y);
        }
        grad[n] = (float)acc;
    }
}

void launch_adjoint_rhs(hipStream_t s, const float2 *E, long long N, int nx, int ny, const int2 *focal, int n_focal,
                        const float2 *sc, const float *k0f, int n_rhs, int n_src, float2 *Jadj, double *fomv) {
    hipLaunchKernelGGL(adjoint_rhs_kernel, dim3((n_rhs + 63) / 64), dim3(64), 0, s, E, N, nx, ny, focal, n_focal, sc,
                       k0f, n_rhs, n_src, Jadj, fomv);
}

void launch_adjoint_grad(hipStream_t s, const float2 *E, const float2 *mu, long long N, int nx, int ny, int n_rhs,
                         int n_src, const float2 *sc, const float *k0f, float *grad) {
    const long long nb = (N + 255) / 256;
    hipLaunchKernelGGL(adjoint_grad_kernel, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, s, E, mu, N, nx, ny,
                       n_rhs, n_src, sc, k0f, grad);
}

}  // namespace nosdd
