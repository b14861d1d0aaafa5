// Setup kernels: media check and nondimensional coefficients with the absorbing
// layers, the stencil form of the finest shifted operator, Galerkin coarsening
// (eq. (9)), dense assembly and inversion of the coarsest operator and its
// application in every cycle.
#include <math.h>

#include "internal.hpp"
#include "ops.hpp"

namespace ehh {

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------------------ media check
int media_check_blocks(int64_t ncell) {
    int64_t b = (ncell + 1023) / 1024;
    return (int)(b < 1024 ? (b < 1 ? 1 : b) : 1024);
}

__global__ __launch_bounds__(256) void k_media_partial(const double* __restrict__ lam, const double* __restrict__ mu,
                                                       const double* __restrict__ rho, const double* __restrict__ gam,
                                                       int64_t n, double* __restrict__ partial) {
    __shared__ double sm[3][256];
    double smu = 0, srho = 0, bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double l = lam[i], m = mu[i], r = rho[i];
        const double gg = gam ? gam[i] : 0.0;
        const bool ok = isfinite(l) && isfinite(m) && isfinite(r) && isfinite(gg) && r > 0.0 && m >= 0.0 &&
                        (l + m) > 0.0 && gg >= 0.0;
        if (!ok) bad += 1.0;
        smu += m;
        srho += r;
    }
    sm[0][threadIdx.x] = smu;
    sm[1][threadIdx.x] = srho;
    sm[2][threadIdx.x] = bad;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int j = 0; j < 3; ++j) sm[j][threadIdx.x] += sm[j][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int j = 0; j < 3; ++j) partial[(int64_t)j * gridDim.x + blockIdx.x] = sm[j][0];
}

__global__ void k_media_final(const double* __restrict__ partial, int nb, const double* lam, const double* mu,
                              int64_t n, double* __restrict__ out) {
    if (threadIdx.x != 0) return;
    double s[3] = {0, 0, 0};
    for (int j = 0; j < 3; ++j)
        for (int b = 0; b < nb; ++b) s[j] += partial[(int64_t)j * nb + b];
    out[0] = s[0];
    out[1] = s[1];
    out[2] = s[2];
    // fallback stiffness scale when mu vanishes everywhere: mean(lambda + 2 mu)
    if (s[0] <= 0.0) {
        double t = 0;
        for (int64_t i = 0; i < n; ++i) t += lam[i] + 2.0 * mu[i];
        out[3] = t;
    } else {
        out[3] = 0.0;
    }
}

hipError_t launch_media_check(const double* lam, const double* mu, const double* rho, const double* gam,
                              int64_t ncell, double* partial, int nb, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_media_partial, nb, 256, 0, s, lam, mu, rho, gam, ncell, partial);
    hipLaunchKernelGGL(k_media_final, 1, 64, 0, s, partial, nb, lam, mu, ncell, out);
    return hipGetLastError();
}

// ------------------------------------------------------------ level-0 coefficients
// Quadratic absorbing ramp t^2 (section 2.1) towards both ends of an axis of n
// cells with a layer of L cells; 0 when L <= 0.
EHH_DEV double ramp(int i, int n, int L_lo, int L_hi) {
    const double x = i + 0.5;
    double t = 0.0;
    if (L_lo > 0) t = fmax(t, (L_lo - x) / L_lo);
    if (L_hi > 0) t = fmax(t, (x - (n - L_hi)) / L_hi);
    return t * t;
}

__global__ __launch_bounds__(256) void k_fine_coef(FineCoefParams p, const double* __restrict__ lam,
                                                   const double* __restrict__ mu, const double* __restrict__ rho,
                                                   const double* __restrict__ gph, double* __restrict__ out) {
    const int64_t nl = (int64_t)p.n_loc[0] * p.n_loc[1] * (p.dim == 3 ? p.n_loc[2] : 1);
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nl) return;
    int c[3];
    c[0] = (int)(t % p.n_loc[0]);
    c[1] = (int)((t / p.n_loc[0]) % p.n_loc[1]);
    c[2] = p.dim == 3 ? (int)(t / ((int64_t)p.n_loc[0] * p.n_loc[1])) : 0;
    int gpos[3];
    double gam = p.gam0;
    for (int a = 0; a < p.dim; ++a) {
        int gc = c[a] + p.origin[a];
        gc = gc < 0 ? 0 : (gc >= p.n_glob[a] ? p.n_glob[a] - 1 : gc);
        gpos[a] = gc;
        gam += p.abl_max * ramp(gc, p.n_glob[a], p.abl[a], p.abl[a]);
        gam += p.abl_max * ramp(c[a], p.n_loc[a], p.pad_lo[a], p.pad_hi[a]);
    }
    const int64_t gi = p.dim == 3 ? ((int64_t)gpos[2] * p.n_glob[1] + gpos[1]) * p.n_glob[0] + gpos[0]
                                  : (int64_t)gpos[1] * p.n_glob[0] + gpos[0];
    if (gph) gam += gph[gi] * p.inv_omega;
    const double m = mu[gi] / p.mu_bar;
    const double l = lam[gi] / p.mu_bar;
    out[t] = m;
    out[nl + t] = 1.0 / (l + m);
    out[2 * nl + t] = rho[gi] / p.rho_bar;
    out[3 * nl + t] = gam;
}

hipError_t launch_fine_coef(const FineCoefParams& p, const double* lam, const double* mu, const double* rho,
                            const double* gam_phys, double* out, hipStream_t s) {
    const int64_t nl = (int64_t)p.n_loc[0] * p.n_loc[1] * (p.dim == 3 ? p.n_loc[2] : 1);
    hipLaunchKernelGGL(k_fine_coef, nblk(nl), 256, 0, s, p, lam, mu, rho, gam_phys, out);
    return hipGetLastError();
}

// ------------------------------------------------------------- stencil of level 0
template <int D>
__global__ __launch_bounds__(256) void k_materialise(Geo g, FineCoef<double> c, double* __restrict__ st) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const StCoef<double> sv = stencil_view<D, double>(g, (const double*)st);
    if (t < g.ncell) {
        const int64_t off = sv.pp - (const double*)st;
        st[off + t] = -c.dinv[t];
    }
    if (t >= g.off[3]) return;
    int k = 0;
    while (k < D - 1 && t >= g.off[k + 1]) ++k;
    const int64_t fi = t - g.off[k];
    int p[3];
    face_pos<D>(g, k, fi, p);
    FineOp<D, double> op{g, c};
    double* uu = st + (sv.uu[k] - (const double*)st);
    double* up = st + (sv.up[k] - (const double*)st);
    const int64_t cnt = g.cnt[k];
    constexpr int CF = St<D>::CF;
    for (int s = 0; s < St<D>::NUU; ++s) {
        uu[(2 * s) * cnt + fi] = 0.0;
        uu[(2 * s + 1) * cnt + fi] = 0.0;
    }
    const cx<double> dg = op.diag_u(k, p);
    uu[fi] = dg.re;
    uu[cnt + fi] = dg.im;
    if (p[k] + 1 <= g.n[k] - 1) uu[2 * 1 * cnt + fi] = -op.mu_c(p);   // dn = +1
    for (int tt = 0; tt < D - 1; ++tt) {
        const int tax = tt == 0 ? tang1<D>(k) : tang2<D>(k);
        if (p[tax] + 1 < g.n[tax]) {
            const int F = tt == 0 ? full_index<D>(0, 1, 0) : full_index<D>(0, 0, 1);
            uu[2 * (F - CF) * cnt + fi] = -op.mu_edge(k, p, tax, p[tax] + 1);
        }
    }
    for (int q = 0; q < St<D>::NUP; ++q) up[q * cnt + fi] = 0.0;
    up[up_index<D>(0, 0, 0) * cnt + fi] = -1.0;
    up[up_index<D>(1, 0, 0) * cnt + fi] = 1.0;
}

hipError_t launch_materialise(const Geo& g, const FineCoef<double>& c, double* st, hipStream_t s) {
    const int64_t n = g.N > g.ncell ? g.N : g.ncell;
    if (g.dim == 2)
        hipLaunchKernelGGL((k_materialise<2>), nblk(n), 256, 0, s, g, c, st);
    else
        hipLaunchKernelGGL((k_materialise<3>), nblk(n), 256, 0, s, g, c, st);
    return hipGetLastError();
}

// ---------------------------------------------------------------------- Galerkin
EHH_DEV double wn_(int d) { return d == 0 ? 1.0 : ((d == 1 || d == -1) ? 0.5 : 0.0); }
EHH_DEV double wt_(int d) { return (d == 0 || d == 1) ? 0.75 : ((d == -1 || d == 2) ? 0.25 : 0.0); }

// Entry A(f, f + offset F) of a stencil-format level (0 if the neighbour is absent).
template <int D>
EHH_DEV cx<double> st_entry(const StOp<D, double>& op, int k, const int* f, int64_t fi, int F, int* gpos,
                            bool& ok) {
    int dn, d1, d2;
    full_offset<D>(F, dn, d1, d2);
    const int t1 = tang1<D>(k), t2 = tang2<D>(k);
    gpos[0] = f[0];
    gpos[1] = f[1];
    gpos[2] = f[2];
    gpos[k] += dn;
    gpos[t1] += d1;
    if (D == 3) gpos[t2] += d2;
    ok = face_ok<D>(op.g, k, gpos);
    if (!ok) return mk(0.0, 0.0);
    constexpr int CF = St<D>::CF;
    return F >= CF ? op.uu(k, fi, F - CF) : op.uu(k, face_idx<D>(op.g, k, gpos), CF - F);
}

// One thread per (coarse face X of component k, stored offset s).
template <int D>
__global__ __launch_bounds__(256) void k_galerkin_uu(Geo gf, StCoef<double> cf, Geo gc, double* __restrict__ stc) {
    constexpr int NUU = St<D>::NUU, CF = St<D>::CF, NF = St<D>::NF;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nu = gc.off[3];
    if (t >= nu * NUU) return;
    const int s = (int)(t / nu);
    const int64_t u = t - (int64_t)s * nu;
    int k = 0;
    while (k < D - 1 && u >= gc.off[k + 1]) ++k;
    const int64_t Xi = u - gc.off[k];
    int X[3], Y[3];
    face_pos<D>(gc, k, Xi, X);
    const int t1 = tang1<D>(k), t2 = tang2<D>(k);
    int dn, d1, d2;
    full_offset<D>(s + CF, dn, d1, d2);
    Y[0] = X[0];
    Y[1] = X[1];
    Y[2] = X[2];
    Y[k] += dn;
    Y[t1] += d1;
    if (D == 3) Y[t2] += d2;
    StCoef<double> cc = stencil_view<D, double>(gc, (const double*)stc);
    double* outp = stc + (cc.uu[k] - (const double*)stc);
    double sre = 0.0, sim = 0.0;
    if (face_ok<D>(gc, k, Y)) {
        const StOp<D, double> op{gf, cf};
        const int nb2 = D == 3 ? 4 : 1;
        for (int a = -1; a <= 1; ++a)
            for (int b1 = -1; b1 <= 2; ++b1)
                for (int b2i = 0; b2i < nb2; ++b2i) {
                    const int b2 = D == 3 ? b2i - 1 : 0;
                    int f[3];
                    f[k] = 2 * X[k] + a;
                    f[t1] = 2 * X[t1] + b1;
                    if (D == 3) f[t2] = 2 * X[t2] + b2;
                    else f[2] = 0;
                    if (!face_ok<D>(gf, k, f)) continue;
                    const double wX = wn_(a) * wt_(b1) * (D == 3 ? wt_(b2) : 1.0);
                    const int64_t fi = face_idx<D>(gf, k, f);
                    for (int F = 0; F < NF; ++F) {
                        int gp[3];
                        int fdn, fd1, fd2;
                        full_offset<D>(F, fdn, fd1, fd2);
                        gp[k] = f[k] + fdn;
                        gp[t1] = f[t1] + fd1;
                        gp[t2] = D == 3 ? f[t2] + fd2 : 0;
                        const double wY = wn_(gp[k] - 2 * Y[k]) * wt_(gp[t1] - 2 * Y[t1]) *
                                          (D == 3 ? wt_(gp[t2] - 2 * Y[t2]) : 1.0);
                        if (wY == 0.0) continue;
                        bool ok;
                        int gq[3];
                        const cx<double> a_ = st_entry<D>(op, k, f, fi, F, gq, ok);
                        if (!ok) continue;
                        sre += wX * wY * a_.re;
                        sim += wX * wY * a_.im;
                    }
                }
    }
    outp[(int64_t)(2 * s) * gc.cnt[k] + Xi] = sre;
    outp[(int64_t)(2 * s + 1) * gc.cnt[k] + Xi] = sim;
}

// One thread per (coarse face X of component k, u-p entry q).
template <int D>
__global__ __launch_bounds__(256) void k_galerkin_up(Geo gf, StCoef<double> cf, Geo gc, double* __restrict__ stc) {
    constexpr int NUP = St<D>::NUP;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nu = gc.off[3];
    if (t >= nu * NUP) return;
    const int q = (int)(t / nu);
    const int64_t u = t - (int64_t)q * nu;
    int k = 0;
    while (k < D - 1 && u >= gc.off[k + 1]) ++k;
    const int64_t Xi = u - gc.off[k];
    int X[3];
    face_pos<D>(gc, k, Xi, X);
    const int t1 = tang1<D>(k), t2 = tang2<D>(k);
    int side, e1, e2;
    up_decode<D>(q, side, e1, e2);
    int C[3] = {X[0], X[1], X[2]};
    C[k] += side - 1;
    C[t1] += e1;
    if (D == 3) C[t2] += e2;
    StCoef<double> cc = stencil_view<D, double>(gc, (const double*)stc);
    double* outp = stc + (cc.up[k] - (const double*)stc);
    double sum = 0.0;
    if (cell_ok<D>(gc, C)) {
        const StOp<D, double> op{gf, cf};
        const int nb2 = D == 3 ? 4 : 1;
        for (int a = -1; a <= 1; ++a)
            for (int b1 = -1; b1 <= 2; ++b1)
                for (int b2i = 0; b2i < nb2; ++b2i) {
                    const int b2 = D == 3 ? b2i - 1 : 0;
                    int f[3];
                    f[k] = 2 * X[k] + a;
                    f[t1] = 2 * X[t1] + b1;
                    if (D == 3) f[t2] = 2 * X[t2] + b2;
                    else f[2] = 0;
                    if (!face_ok<D>(gf, k, f)) continue;
                    const double wX = wn_(a) * wt_(b1) * (D == 3 ? wt_(b2) : 1.0);
                    const int64_t fi = face_idx<D>(gf, k, f);
                    for (int qq = 0; qq < NUP; ++qq) {
                        int sd, f1, f2;
                        up_decode<D>(qq, sd, f1, f2);
                        int cfp[3] = {f[0], f[1], f[2]};
                        cfp[k] += sd - 1;
                        cfp[t1] += f1;
                        if (D == 3) cfp[t2] += f2;
                        if (!cell_ok<D>(gf, cfp)) continue;
                        if ((cfp[0] >> 1) != C[0] || (cfp[1] >> 1) != C[1] || (D == 3 && (cfp[2] >> 1) != C[2]))
                            continue;
                        sum += wX * op.up(k, fi, qq);
                    }
                }
    }
    outp[(int64_t)q * gc.cnt[k] + Xi] = sum;
}

template <int D>
__global__ __launch_bounds__(256) void k_galerkin_pp(Geo gf, StCoef<double> cf, Geo gc, double* __restrict__ stc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= gc.ncell) return;
    int C[3];
    cell_pos<D>(gc, t, C);
    double s = 0.0;
    for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                int f[3] = {2 * C[0] + dx, 2 * C[1] + dy, D == 3 ? 2 * C[2] + dz : 0};
                s += cf.pp[cell_idx<D>(gf, f)];
            }
    StCoef<double> cc = stencil_view<D, double>(gc, (const double*)stc);
    stc[(cc.pp - (const double*)stc) + t] = s;
}

hipError_t launch_galerkin(const Geo& gf, const double* stf, const Geo& gc, double* stc, hipStream_t s) {
    const int64_t nu = gc.off[3];
    if (gf.dim == 2) {
        const StCoef<double> cf = stencil_view<2, double>(gf, stf);
        hipLaunchKernelGGL((k_galerkin_uu<2>), nblk(nu * St<2>::NUU), 256, 0, s, gf, cf, gc, stc);
        hipLaunchKernelGGL((k_galerkin_up<2>), nblk(nu * St<2>::NUP), 256, 0, s, gf, cf, gc, stc);
        hipLaunchKernelGGL((k_galerkin_pp<2>), nblk(gc.ncell), 256, 0, s, gf, cf, gc, stc);
    } else {
        const StCoef<double> cf = stencil_view<3, double>(gf, stf);
        hipLaunchKernelGGL((k_galerkin_uu<3>), nblk(nu * St<3>::NUU), 256, 0, s, gf, cf, gc, stc);
        hipLaunchKernelGGL((k_galerkin_up<3>), nblk(nu * St<3>::NUP), 256, 0, s, gf, cf, gc, stc);
        hipLaunchKernelGGL((k_galerkin_pp<3>), nblk(gc.ncell), 256, 0, s, gf, cf, gc, stc);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ dense coarsest
// One thread per row (unknown) of the level: scatter its stencil into the
// row-major complex matrix (zeroed beforehand).
template <int D>
__global__ __launch_bounds__(256) void k_dense_assemble(Geo g, StCoef<double> c, double* __restrict__ A) {
    const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= g.N) return;
    const StOp<D, double> op{g, c};
    const int64_t n = g.N;
    double* R = A + 2 * row * n;
    int k = 0;
    while (k < 3 && row >= g.off[k + 1]) ++k;
    if (k >= D) k = 3;
    const int64_t li = row - g.off[k];
    if (k == 3) {
        int cc[3];
        cell_pos<D>(g, li, cc);
        R[2 * row] = c.pp[li];
        for (int kk = 0; kk < D; ++kk) {
            const int t1 = tang1<D>(kk), t2 = tang2<D>(kk);
            for (int qq = 0; qq < St<D>::NUP; ++qq) {
                int side, e1, e2;
                up_decode<D>(qq, side, e1, e2);
                int q[3] = {cc[0], cc[1], cc[2]};
                q[kk] += 1 - side;
                q[t1] -= e1;
                if (D == 3) q[t2] -= e2;
                if (!face_ok<D>(g, kk, q)) continue;
                const int64_t qi = face_idx<D>(g, kk, q);
                R[2 * (g.off[kk] + qi)] += op.up(kk, qi, qq);
            }
        }
        return;
    }
    int p[3];
    face_pos<D>(g, k, li, p);
    const int t1 = tang1<D>(k), t2 = tang2<D>(k);
    for (int F = 0; F < St<D>::NF; ++F) {
        bool ok;
        int q[3];
        const cx<double> a = st_entry<D>(op, k, p, li, F, q, ok);
        if (!ok) continue;
        const int64_t col = g.off[k] + face_idx<D>(g, k, q);
        R[2 * col] += a.re;
        R[2 * col + 1] += a.im;
    }
    for (int qq = 0; qq < St<D>::NUP; ++qq) {
        int side, e1, e2;
        up_decode<D>(qq, side, e1, e2);
        int q[3] = {p[0], p[1], p[2]};
        q[k] += side - 1;
        q[t1] += e1;
        if (D == 3) q[t2] += e2;
        if (!cell_ok<D>(g, q)) continue;
        R[2 * (g.off[3] + cell_idx<D>(g, q))] += op.up(k, li, qq);
    }
}

hipError_t launch_dense_assemble(const Geo& g, const double* st, double* dense, hipStream_t s) {
    hipError_t e = hipMemsetAsync(dense, 0, sizeof(double) * 2 * g.N * g.N, s);
    if (e != hipSuccess) return e;
    if (g.dim == 2)
        hipLaunchKernelGGL((k_dense_assemble<2>), nblk(g.N), 256, 0, s, g, stencil_view<2, double>(g, st), dense);
    else
        hipLaunchKernelGGL((k_dense_assemble<3>), nblk(g.N), 256, 0, s, g, stencil_view<3, double>(g, st), dense);
    return hipGetLastError();
}

// Gauss-Jordan step k, part 1 (one block per matrix): choose the pivot row of
// column k among rows >= k, swap it into row k, scale row k by 1/pivot with the
// pivot position replaced by 1 first (so that column k accumulates the inverse),
// and save column k (the elimination factors) before zeroing it.
__global__ __launch_bounds__(1024) void k_gj_pivot(double* __restrict__ Ab, int64_t n, int64_t k,
                                                   double* __restrict__ workb, int* __restrict__ pivb) {
    double* A = Ab + (int64_t)blockIdx.y * 2 * n * n;
    double* f = workb + (int64_t)blockIdx.y * 2 * n;
    int* piv = pivb + (int64_t)blockIdx.y * n;
    __shared__ double bv[1024];
    __shared__ int bi[1024];
    double best = -1.0;
    int bidx = (int)k;
    for (int64_t i = k + threadIdx.x; i < n; i += blockDim.x) {
        const double re = A[2 * (i * n + k)], im = A[2 * (i * n + k) + 1];
        const double m = re * re + im * im;
        if (m > best) {
            best = m;
            bidx = (int)i;
        }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = bidx;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double o = bv[threadIdx.x + w];
            const int oi = bi[threadIdx.x + w];
            if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
                bv[threadIdx.x] = o;
                bi[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    const int p = bi[0];
    if (threadIdx.x == 0) piv[k] = p;
    if (p != k) {
        for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
            const double ar = A[2 * (k * n + j)], ai = A[2 * (k * n + j) + 1];
            A[2 * (k * n + j)] = A[2 * (p * n + j)];
            A[2 * (k * n + j) + 1] = A[2 * (p * n + j) + 1];
            A[2 * (p * n + j)] = ar;
            A[2 * (p * n + j) + 1] = ai;
        }
    }
    __syncthreads();
    const double pr = A[2 * (k * n + k)], pi = A[2 * (k * n + k) + 1];
    const double dd = pr * pr + pi * pi;
    const double ir = pr / dd, ii = -pi / dd;
    __syncthreads();
    if (threadIdx.x == 0) {
        A[2 * (k * n + k)] = 1.0;
        A[2 * (k * n + k) + 1] = 0.0;
    }
    __syncthreads();
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
        const double ar = A[2 * (k * n + j)], ai = A[2 * (k * n + j) + 1];
        A[2 * (k * n + j)] = ar * ir - ai * ii;
        A[2 * (k * n + j) + 1] = ar * ii + ai * ir;
    }
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        if (i == k) {
            f[2 * i] = 0.0;
            f[2 * i + 1] = 0.0;
            continue;
        }
        f[2 * i] = A[2 * (i * n + k)];
        f[2 * i + 1] = A[2 * (i * n + k) + 1];
        A[2 * (i * n + k)] = 0.0;
        A[2 * (i * n + k) + 1] = 0.0;
    }
}

// Part 2: A[i][j] -= f[i] * A[k][j] for i != k (column k included: it receives
// -f[i]/pivot).
__global__ __launch_bounds__(256) void k_gj_elim(double* __restrict__ Ab, int64_t n, int64_t k,
                                                 const double* __restrict__ workb) {
    double* A = Ab + (int64_t)blockIdx.z * 2 * n * n;
    const double* f = workb + (int64_t)blockIdx.z * 2 * n;
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i0 = (int64_t)blockIdx.y * 16;
    if (j >= n) return;
    const double kr = A[2 * (k * n + j)], ki = A[2 * (k * n + j) + 1];
    for (int64_t i = i0; i < i0 + 16 && i < n; ++i) {
        if (i == k) continue;
        const double fr = f[2 * i], fi = f[2 * i + 1];
        A[2 * (i * n + j)] -= fr * kr - fi * ki;
        A[2 * (i * n + j) + 1] -= fr * ki + fi * kr;
    }
}

// Undo the row interchanges as column interchanges, last step first.
__global__ __launch_bounds__(256) void k_gj_unpivot(double* __restrict__ Ab, int64_t n, const int* __restrict__ pivb) {
    double* A = Ab + (int64_t)blockIdx.y * 2 * n * n;
    const int* piv = pivb + (int64_t)blockIdx.y * n;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int64_t k = n - 1; k >= 0; --k) {
        const int64_t p = piv[k];
        if (p == k) continue;
        const double ar = A[2 * (i * n + k)], ai = A[2 * (i * n + k) + 1];
        A[2 * (i * n + k)] = A[2 * (i * n + p)];
        A[2 * (i * n + k) + 1] = A[2 * (i * n + p) + 1];
        A[2 * (i * n + p)] = ar;
        A[2 * (i * n + p) + 1] = ai;
    }
}

hipError_t launch_dense_invert(double* dense, int64_t n, int batch, double* work, int* piv, hipStream_t s) {
    for (int64_t k = 0; k < n; ++k) {
        hipLaunchKernelGGL(k_gj_pivot, dim3(1, batch), 1024, 0, s, dense, n, k, work, piv);
        hipLaunchKernelGGL(k_gj_elim, dim3(nblk(n), (unsigned)((n + 15) / 16), batch), 256, 0, s, dense, n, k, work);
    }
    hipLaunchKernelGGL(k_gj_unpivot, dim3(nblk(n), batch), 256, 0, s, dense, n, piv);
    return hipGetLastError();
}

// ------------------------------------------------------------------ coarse apply
// One 64-wide wavefront per (row, group of up to 4 right-hand sides): lanes stride
// over the columns with FP64 accumulation and a butterfly reduction.  The grid
// spans rows x right-hand-side groups so that a batch fills the chip.
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_apply(const double* __restrict__ inv, int64_t n, const T* __restrict__ r,
                                                      T* __restrict__ e, int nrhs) {
    constexpr int RG = 4;
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (row >= n) return;
    const int r0 = blockIdx.y * RG;
    const int nr = nrhs - r0 < RG ? nrhs - r0 : RG;
    const double* R = inv + 2 * row * n;
    double ar[RG], ai[RG];
#pragma unroll
    for (int q = 0; q < RG; ++q) ar[q] = ai[q] = 0.0;
    for (int64_t j = lane; j < n; j += 64) {
        const double mr = R[2 * j], mi = R[2 * j + 1];
#pragma unroll
        for (int q = 0; q < RG; ++q) {
            if (q < nr) {
                const T* rv = r + (int64_t)(r0 + q) * 2 * n;
                const double vr = (double)rv[j], vi = (double)rv[n + j];
                ar[q] += mr * vr - mi * vi;
                ai[q] += mr * vi + mi * vr;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < RG; ++q) {
        double sr = ar[q], si = ai[q];
        for (int o = 32; o > 0; o >>= 1) {
            sr += __shfl_xor(sr, o, 64);
            si += __shfl_xor(si, o, 64);
        }
        if (lane == 0 && q < nr) {
            T* ev = e + (int64_t)(r0 + q) * 2 * n;
            ev[row] = (T)sr;
            ev[n + row] = (T)si;
        }
    }
}

template <typename T>
hipError_t launch_coarse_apply(const double* inv, int64_t n, const T* r, T* e, int nrhs, hipStream_t s) {
    hipLaunchKernelGGL((k_coarse_apply<T>), dim3(nblk(n * 64), (nrhs + 3) / 4), 256, 0, s, inv, n, r, e, nrhs);
    return hipGetLastError();
}
template hipError_t launch_coarse_apply<float>(const double*, int64_t, const float*, float*, int, hipStream_t);
template hipError_t launch_coarse_apply<double>(const double*, int64_t, const double*, double*, int, hipStream_t);

__global__ void k_zero_words(uint32_t* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}
// Zero fill by a kernel (not a memset node, so it may sit inside a captured graph).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 4);
    hipLaunchKernelGGL(k_zero_words, nblk(n), 256, 0, s, (uint32_t*)p, n);
    return hipGetLastError();
}

__global__ void k_cast_d2f(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}
__global__ void k_cast_f2d(const float* __restrict__ in, double* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}
hipError_t launch_cast_d2f(const double* in, float* out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_cast_d2f, nblk(n), 256, 0, s, in, out, n);
    return hipGetLastError();
}
hipError_t launch_cast_f2d(const float* in, double* out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_cast_f2d, nblk(n), 256, 0, s, in, out, n);
    return hipGetLastError();
}

}  // namespace ehh
