// Adjoint-state ingredients of the discrete elastic Helmholtz system.
//
// The matrix A of eq. (14) is complex symmetric (A^T = A), so its adjoint is the
// conjugate matrix and the adjoint system A^H y = g is solved as A conj(y) = conj(g)
// (k_conj applies the conjugations).  For a real misfit L(x) with A x = b, the
// derivative with respect to a cell medium value is dL/dm = -Re y^H (dA/dm) x
// (the full-waveform inversion setting that motivates the solver, section 1).
// k_media_gradient evaluates that contraction for lambda, mu and rho at every
// cell, matrix-free, from the derivative of each term of the discretisation of
// section 2.1 (eqs. (4), (5) and (14)):
//   * the pressure row -1/(lambda + mu):         d/dlambda = d/dmu = +1/(lambda + mu)^2;
//   * the Laplacian grad^T A_e(mu) grad: a normal derivative of u_k at a cell
//     carries mu of that cell, a tangential derivative at a node (2D) or edge
//     (3D) carries the mean of mu over the existing cells around it -- the
//     mean beside the face along k (1/2 each) times the mean over the cells
//     along the derivative axis that exist (1 or 2);
//   * the mass -w^2 A_f(rho (1 - i gamma)): each interior face averages its two
//     cells, so d/drho_c = -w^2 (1 - i gamma_c) / 2 on the faces of cell c.
// Units: the operator is in the nondimensional scaling (lambda/mu_bar, mu/mu_bar,
// rho/rho_bar at fixed mu_bar, rho_bar); the kernel divides by mu_bar or rho_bar to
// give derivatives per Pa and per kg/m^3.
#include "internal.hpp"

namespace ehh {
namespace {

inline unsigned nblocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

__global__ void k_conj(const double* __restrict__ x, double* __restrict__ y, int64_t N, int nrhs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * N * nrhs) return;
    const double v = x[t];
    y[t] = (t % (2 * N)) < N ? v : -v;
}

// u_k at face position p (a zero beyond the walls and on the wall faces).
template <int D>
__device__ inline cx<double> face_at(const Geo& g, const double* __restrict__ v, int k, const int* p) {
    if (!face_ok<D>(g, k, p)) return mk(0.0, 0.0);
    const int64_t i = g.off[k] + face_idx<D>(g, k, p);
    return mk(v[i], v[g.N + i]);
}

// Re(conj(a) b)
__device__ inline double re_cdot(cx<double> a, cx<double> b) { return a.re * b.re + a.im * b.im; }
// conj(a) b
__device__ inline cx<double> cdot(cx<double> a, cx<double> b) {
    return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}

// One thread per cell; the right-hand sides are summed in registers, so every
// output is written once (deterministic, no atomics).
template <int D>
__global__ void __launch_bounds__(256) k_media_gradient(Geo g, const double* __restrict__ fine, double om2,
                                                        const double* __restrict__ y, const double* __restrict__ x,
                                                        int nrhs, double inv_mu_bar, double inv_rho_bar,
                                                        double* __restrict__ gl, double* __restrict__ gm,
                                                        double* __restrict__ gr, int accumulate) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.ncell) return;
    int c[3];
    cell_pos<D>(g, t, c);
    double s_p = 0.0;     // Re sum conj(y_p) x_p
    double s_lap = 0.0;   // Re sum of the Laplacian terms of d/dmu
    cx<double> s_m = mk(0.0, 0.0);   // sum conj(y_u) x_u over the faces of the cell
    for (int r = 0; r < nrhs; ++r) {
        const double* yr = y + (int64_t)r * 2 * g.N;
        const double* xr = x + (int64_t)r * 2 * g.N;
        const int64_t ip = g.off[3] + t;
        s_p += re_cdot(mk(yr[ip], yr[g.N + ip]), mk(xr[ip], xr[g.N + ip]));
        for (int k = 0; k < D; ++k) {
            int p[3] = {c[0], c[1], c[2]};
            // the two faces of the cell along k: positions c_k and c_k + 1
            const cx<double> ylo = face_at<D>(g, yr, k, p), xlo = face_at<D>(g, xr, k, p);
            p[k] = c[k] + 1;
            const cx<double> yhi = face_at<D>(g, yr, k, p), xhi = face_at<D>(g, xr, k, p);
            s_m = s_m + cdot(ylo, xlo) + cdot(yhi, xhi);
            s_lap += re_cdot(yhi - ylo, xhi - xlo);
            // tangential derivatives along a != k at nodes/edges m in {c_a, c_a + 1}
            for (int a = 0; a < D; ++a) {
                if (a == k) continue;
                for (int df = 0; df < 2; ++df) {
                    const int f = c[k] + df;
                    if (f < 1 || f > g.n[k] - 1) continue;
                    for (int dm = 0; dm < 2; ++dm) {
                        const int m = c[a] + dm;
                        const int cnt = (m >= 1) + (m <= g.n[a] - 1);
                        int q[3] = {c[0], c[1], c[2]};
                        q[k] = f;
                        q[a] = m;
                        const cx<double> yh = face_at<D>(g, yr, k, q), xh = face_at<D>(g, xr, k, q);
                        q[a] = m - 1;
                        const cx<double> yl = face_at<D>(g, yr, k, q), xl = face_at<D>(g, xr, k, q);
                        s_lap += (0.5 / (double)cnt) * re_cdot(yh - yl, xh - xl);
                    }
                }
            }
        }
    }
    const double dinv = fine[g.ncell + t];
    const double gam = fine[3 * g.ncell + t];
    const double d_lam = -(dinv * dinv * s_p) * inv_mu_bar;
    const double d_mu = -(dinv * dinv * s_p + s_lap) * inv_mu_bar;
    // Re[-w^2 (1 - i gam) / 2 * s_m] = -w^2 (s_m.re + gam s_m.im) / 2, negated for dL/drho
    const double d_rho = 0.5 * om2 * (s_m.re + gam * s_m.im) * inv_rho_bar;
    if (accumulate) {
        gl[t] += d_lam;
        gm[t] += d_mu;
        gr[t] += d_rho;
    } else {
        gl[t] = d_lam;
        gm[t] = d_mu;
        gr[t] = d_rho;
    }
}

}  // namespace

hipError_t launch_conj(const double* x, double* y, int64_t N, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL(k_conj, nblocks(2 * N * nrhs), 256, 0, s, x, y, N, nrhs);
    return hipGetLastError();
}

hipError_t launch_media_gradient(const Geo& g, const double* fine, double om2, const double* y, const double* x,
                                 int nrhs, double mu_bar, double rho_bar, double* gl, double* gm, double* gr,
                                 int accumulate, hipStream_t s) {
    if (g.dim == 2)
        hipLaunchKernelGGL(k_media_gradient<2>, nblocks(g.ncell), 256, 0, s, g, fine, om2, y, x, nrhs,
                           1.0 / mu_bar, 1.0 / rho_bar, gl, gm, gr, accumulate);
    else
        hipLaunchKernelGGL(k_media_gradient<3>, nblocks(g.ncell), 256, 0, s, g, fine, om2, y, x, nrhs,
                           1.0 / mu_bar, 1.0 / rho_bar, gl, gm, gr, accumulate);
    return hipGetLastError();
}

}  // namespace ehh
