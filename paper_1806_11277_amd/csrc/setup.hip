// Setup kernels: media check and nondimensional coefficients with the absorbing
// layers, the stencil form of the finest shifted operator, Galerkin coarsening
// (eq. (9)), dense assembly and inversion of the coarsest operator and its
// application in every cycle.
#include <math.h>

#include <cstdlib>

#include <mutex>

#include "internal.hpp"
#include "launchlog.hpp"
#include "batch.hpp"
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
    EHH_LAUNCH(k_media_partial, nb, 256, 0, s, lam, mu, rho, gam, ncell, partial);
    EHH_LAUNCH(k_media_final, 1, 64, 0, s, partial, nb, lam, mu, ncell, out);
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
    EHH_LAUNCH(k_fine_coef, nblk(nl), 256, 0, s, p, lam, mu, rho, gam_phys, out);
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
        EHH_LAUNCH((k_materialise<2>), nblk(n), 256, 0, s, g, c, st);
    else
        EHH_LAUNCH((k_materialise<3>), nblk(n), 256, 0, s, g, c, st);
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
    constexpr int NUU = St<D>::NUU, CF = St<D>::CF;
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
                    // only the stencil offsets whose target lies in the support of
                    // the prolongation at Y (|normal| <= 1 and tangential in -1..2
                    // around 2 Y), walked in increasing term index F, so that the
                    // sum takes the same terms in the same order as a walk over all
                    // NF terms that skips the zero weights
                    const int nlo = max(-1, 2 * Y[k] - 1 - f[k]), nhi = min(1, 2 * Y[k] + 1 - f[k]);
                    const int alo = max(-2, 2 * Y[t1] - 1 - f[t1]), ahi = min(2, 2 * Y[t1] + 2 - f[t1]);
                    const int blo = D == 3 ? max(-2, 2 * Y[t2] - 1 - f[t2]) : 0;
                    const int bhi = D == 3 ? min(2, 2 * Y[t2] + 2 - f[t2]) : 0;
                    for (int e2 = blo; e2 <= bhi; ++e2)
                        for (int e1 = alo; e1 <= ahi; ++e1)
                            for (int en = nlo; en <= nhi; ++en) {
                                const int F = (en + 1) + 3 * (e1 + 2) + (D == 3 ? 15 * (e2 + 2) : 0);
                                const double wY = wn_(f[k] + en - 2 * Y[k]) * wt_(f[t1] + e1 - 2 * Y[t1]) *
                                                  (D == 3 ? wt_(f[t2] + e2 - 2 * Y[t2]) : 1.0);
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
        EHH_LAUNCH((k_galerkin_uu<2>), nblk(nu * St<2>::NUU), 256, 0, s, gf, cf, gc, stc);
        EHH_LAUNCH((k_galerkin_up<2>), nblk(nu * St<2>::NUP), 256, 0, s, gf, cf, gc, stc);
        EHH_LAUNCH((k_galerkin_pp<2>), nblk(gc.ncell), 256, 0, s, gf, cf, gc, stc);
    } else {
        const StCoef<double> cf = stencil_view<3, double>(gf, stf);
        EHH_LAUNCH((k_galerkin_uu<3>), nblk(nu * St<3>::NUU), 256, 0, s, gf, cf, gc, stc);
        EHH_LAUNCH((k_galerkin_up<3>), nblk(nu * St<3>::NUP), 256, 0, s, gf, cf, gc, stc);
        EHH_LAUNCH((k_galerkin_pp<3>), nblk(gc.ncell), 256, 0, s, gf, cf, gc, stc);
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
        EHH_LAUNCH((k_dense_assemble<2>), nblk(g.N), 256, 0, s, g, stencil_view<2, double>(g, st), dense);
    else
        EHH_LAUNCH((k_dense_assemble<3>), nblk(g.N), 256, 0, s, g, stencil_view<3, double>(g, st), dense);
    return hipGetLastError();
}

// ------------------------------------------------------------------ dense inverse
// Blocked Gauss-Jordan inversion of an n x n complex matrix (row-major, re/im
// interleaved), in place, for the exact coarsest solve of the multigrid cycle.
// Panels of GJ_NB indices K are swept in turn: W = A[K,K]^{-1} by Gauss-Jordan
// with partial pivoting inside the block (one workgroup, in LDS), the block's
// row interchanges applied to the rest of those rows, then
//      A[K,J] <- W A[K,J],  A[I,J] <- A[I,J] - A[I,K] A[K,J],
//      A[I,K] <- -A[I,K] W,  A[K,K] <- W   (I, J outside K),
// the block form of the scalar Gauss-Jordan step, as 64 x 64 output tiles with
// 16-deep k chunks staged in LDS.  Pivot rows are sought inside the diagonal
// block only: for the shifted Galerkin operators every leading principal
// submatrix in the [u; p] ordering is nonsingular (the displacement block has
// a positive-definite imaginary part, omega^2 (gamma + alpha) times a mass
// matrix, and the pressure Schur complement stays definite), so elimination in
// this order needs no interchange for existence; the in-block search guards
// against small pivots.  The result is (Pi A)^{-1} for the accumulated row
// interchanges Pi; the caller undoes Pi as a column permutation
// (launch_permute_columns).
constexpr int GJ_NB = 64;

__device__ inline void cmul_acc(double& cr, double& ci, double ar, double ai, double br, double bi) {
    cr = fma(ar, br, fma(-ai, bi, cr));
    ci = fma(ar, bi, fma(ai, br, ci));
}

// Apply the block's row interchanges (in order) to the columns outside K (the
// block itself already holds the inverse of its interchanged rows).
__global__ __launch_bounds__(256) void k_swap_rows(double* __restrict__ A, int64_t n, int64_t k0, int kb,
                                                   const int* __restrict__ piv) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n || (j >= k0 && j < k0 + kb)) return;
    for (int c = 0; c < kb; ++c) {
        const int64_t p = piv[k0 + c];
        const int64_t k = k0 + c;
        if (p == k) continue;
        const double ar = A[2 * (k * n + j)], ai = A[2 * (k * n + j) + 1];
        A[2 * (k * n + j)] = A[2 * (p * n + j)];
        A[2 * (k * n + j) + 1] = A[2 * (p * n + j) + 1];
        A[2 * (p * n + j)] = ar;
        A[2 * (p * n + j) + 1] = ai;
    }
}

// A[K,K] <- (Pi_K A[K,K])^{-1} by Gauss-Jordan with partial pivoting inside the
// block; piv[k0 + k] = row swapped with k0 + k.  One workgroup of GJ_THREADS
// threads holds the block in registers: lane i of a wavefront owns row i, and
// wavefront w the columns w + 16 q (sixteen wavefronts of 4 entries).  Rows are
// then exchanged inside a wavefront (the pivot row and row k of every column
// are broadcast from their lanes, wave-uniform indices), and a column lives in
// one wavefront, which picks the next pivot itself (a butterfly maximum over a
// 64-bit key: the modulus's bits above the lowest six, then 63 - row, i.e. the
// largest modulus, ties within 2^-46 relative going to the lowest row) and
// publishes that column and the pivot in LDS (double-buffered): one barrier per
// step.  (The transposed layout with the rows exchanged through LDS and the
// pivot taken by an LDS atomic needed two barriers per step: 137 against 128 us
// per 64 x 64 block under rocprofv3.  Four wavefronts of 16 entries took 263 us,
// one wavefront per SIMD leaving the latencies of a step exposed.)
__device__ inline unsigned long long gj_key(double m, int row) {
    return (__double_as_longlong(m) & ~0x3FULL) | (unsigned long long)(63 - row);
}
__device__ inline double gj_lane(double x, int lane) {   // x of a lane (wave-uniform index)
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), lane);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), lane);
    return __hiloint2double(hi, lo);
}

constexpr int GJ_THREADS = 1024;
__global__ __launch_bounds__(GJ_THREADS) void k_diag_inverse(double* __restrict__ A, int64_t n, int64_t k0, int kb,
                                                             int* __restrict__ piv, int* __restrict__ flag) {
    constexpr int NW = GJ_THREADS / 64;   // wavefronts
    constexpr int Q = GJ_NB / NW;         // columns per wavefront
    static_assert(GJ_NB == 64 && Q * NW == GJ_NB, "one row per lane, whole columns per wavefront");
    __shared__ double colk[2][GJ_NB][2];  // the step's column k before the interchange
    __shared__ int pk[2];                 // the step's pivot row
    __shared__ int pivs[GJ_NB];
    const int t = threadIdx.x, i = t & 63, wv = t >> 6;
    const bool iok = i < kb;
    double ar[Q], ai[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = wv + NW * q;
        ar[q] = ai[q] = 0.0;
        if (iok && j < kb) {
            ar[q] = A[2 * ((k0 + i) * n + k0 + j)];
            ai[q] = A[2 * ((k0 + i) * n + k0 + j) + 1];
        }
    }
    // column c's owner: the pivot among rows c .. kb-1, then column c and the
    // pivot row in LDS buffer c & 1 (no global store inside the step loop: a
    // barrier waits for the workgroup's outstanding stores)
    auto publish = [&](int c) {
        const int qc = c / NW;
        double vr = 0.0, vi = 0.0;
#pragma unroll
        for (int q = 0; q < Q; ++q)
            if (q == qc) {
                vr = ar[q];
                vi = ai[q];
            }
        unsigned long long key = (i >= c && iok) ? gj_key(vr * vr + vi * vi, i) : 0ULL;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const unsigned lo = (unsigned)__shfl_xor((int)(unsigned)key, o, 64);
            const unsigned hi = (unsigned)__shfl_xor((int)(unsigned)(key >> 32), o, 64);
            const unsigned long long other = ((unsigned long long)hi << 32) | lo;
            key = other > key ? other : key;
        }
        colk[c & 1][i][0] = vr;
        colk[c & 1][i][1] = vi;
        if (i == 0) pk[c & 1] = 63 - (int)(key & 0x3FULL);
    };
    if (wv == 0) publish(0);
    __syncthreads();
    bool singular = false;
    for (int k = 0; k < kb; ++k) {
        const int b = k & 1;
        const int p = __builtin_amdgcn_readfirstlane(pk[b]);
        // V = the block with rows k and p interchanged; pivot V(k, k) = A(p, k)
        const double pr = colk[b][p][0], pi = colk[b][p][1];
        const double dd = pr * pr + pi * pi;
        singular = singular || !(dd > 0.0);
        const double rdd = 1.0 / dd;
        const double ir = pr * rdd, ii = -pi * rdd;
        // this row's multiplier V(i, k)
        const int si = i == p ? k : i;
        const double fr = colk[b][si][0], fi = colk[b][si][1];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const int j = wv + NW * q;
            // V(k, j) = A(p, j), and V(p, j) = A(k, j), from their lanes
            const double apr = gj_lane(ar[q], p), api = gj_lane(ai[q], p);
            const double akr = gj_lane(ar[q], k), aki = gj_lane(ai[q], k);
            if (iok && j < kb) {
                // row k of the result: V(k, j) / pivot, and 1 / pivot at j = k
                double rkr = ir, rki = ii;
                if (j != k) {
                    rkr = apr * ir - api * ii;
                    rki = apr * ii + api * ir;
                }
                if (i == k) {
                    ar[q] = rkr;
                    ai[q] = rki;
                } else if (j == k) {
                    ar[q] = -(fr * ir - fi * ii);
                    ai[q] = -(fr * ii + fi * ir);
                } else {
                    const double vr = i == p ? akr : ar[q], vi = i == p ? aki : ai[q];
                    ar[q] = vr - (fr * rkr - fi * rki);
                    ai[q] = vi - (fr * rki + fi * rkr);
                }
            }
        }
        if (t == 0) pivs[k] = p;
        if (k + 1 < kb && wv == (k + 1) % NW) publish(k + 1);
        __syncthreads();
    }
    if (t < kb) piv[k0 + t] = (int)(k0 + pivs[t]);
    if (t == 0 && singular) *flag = 1;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const int j = wv + NW * q;
        if (iok && j < kb) {
            A[2 * ((k0 + i) * n + k0 + j)] = ar[q];
            A[2 * ((k0 + i) * n + k0 + j) + 1] = ai[q];
        }
    }
}

// C[i][j] = (beta_one ? C[i][j] : 0) + alpha sum_k A[i][k] B[k][j] on one 64 x 64
// output tile (complex, interleaved, row-major; leading dimensions in complex
// elements).  Rows in [rh_lo, rh_hi) and columns in [ch_lo, ch_hi) of C are left
// untouched, and so is the output tile at (skip_r0, skip_c0) (-1: none).  All
// reads of a tile's operands finish before its writes, so C may alias the
// operand that only this tile reads.
__global__ __launch_bounds__(256) void k_zgemm_tile(double* C, int64_t ldc, const double* A, int64_t lda,
                                                    const double* B, int64_t ldb, int64_t m, int64_t ncol, int kdim,
                                                    double alpha, int beta_one, int64_t rh_lo, int64_t rh_hi,
                                                    int64_t ch_lo, int64_t ch_hi, int64_t skip_r0, int64_t skip_c0) {
    const int64_t row0 = (int64_t)blockIdx.y * 64, col0 = (int64_t)blockIdx.x * 64;
    if ((row0 >= rh_lo && row0 + 64 <= rh_hi) || (col0 >= ch_lo && col0 + 64 <= ch_hi)) return;
    if (row0 == skip_r0 && col0 == skip_c0) return;
    __shared__ double As[16][65 * 2];
    __shared__ double Bs[16][64 * 2];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double cr[4][4], ci[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) cr[i][j] = ci[i][j] = 0.0;
    // the operands of a 16-wide chunk of k: four entries of A and of B per thread,
    // loaded into registers one chunk ahead of the arithmetic, so that the loads
    // of chunk c + 1 are in flight while chunk c is summed
    double par[4], pai[4], pbr[4], pbi[4];
    auto load_chunk = [&](int k0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + 256 * q;
            const int r = e >> 4, kk = e & 15;
            const int64_t gr = row0 + r;
            const int gk = k0 + kk;
            par[q] = pai[q] = 0.0;
            if (gr < m && gk < kdim) {
                par[q] = A[2 * (gr * lda + gk)];
                pai[q] = A[2 * (gr * lda + gk) + 1];
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + 256 * q;
            const int kk = e >> 6, cc = e & 63;
            const int gk = k0 + kk;
            const int64_t gc = col0 + cc;
            pbr[q] = pbi[q] = 0.0;
            if (gk < kdim && gc < ncol) {
                pbr[q] = B[2 * ((int64_t)gk * ldb + gc)];
                pbi[q] = B[2 * ((int64_t)gk * ldb + gc) + 1];
            }
        }
    };
    load_chunk(0);
    for (int k0 = 0; k0 < kdim; k0 += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = threadIdx.x + 256 * q;
            As[e & 15][2 * (e >> 4)] = par[q];
            As[e & 15][2 * (e >> 4) + 1] = pai[q];
            Bs[e >> 6][2 * (e & 63)] = pbr[q];
            Bs[e >> 6][2 * (e & 63) + 1] = pbi[q];
        }
        __syncthreads();
        if (k0 + 16 < kdim) load_chunk(k0 + 16);
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
            double ar[4], ai[4], br[4], bi[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                ar[i] = As[kk][2 * (ty + 16 * i)];
                ai[i] = As[kk][2 * (ty + 16 * i) + 1];
                br[i] = Bs[kk][2 * (tx + 16 * i)];
                bi[i] = Bs[kk][2 * (tx + 16 * i) + 1];
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) cmul_acc(cr[i][j], ci[i][j], ar[i], ai[i], br[j], bi[j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t r = row0 + ty + 16 * i;
        if (r >= m || (r >= rh_lo && r < rh_hi)) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t cidx = col0 + tx + 16 * j;
            if (cidx >= ncol || (cidx >= ch_lo && cidx < ch_hi)) continue;
            double* o = C + 2 * (r * ldc + cidx);
            const double o0 = beta_one ? o[0] : 0.0, o1 = beta_one ? o[1] : 0.0;
            o[0] = o0 + alpha * cr[i][j];
            o[1] = o1 + alpha * ci[i][j];
        }
    }
}

// out[i][j] = X[i][qinv[j]] (the column permutation that turns (Pi A)^{-1} into A^{-1}).
__global__ __launch_bounds__(256) void k_permute_columns(const double* __restrict__ X, double* __restrict__ out,
                                                         int64_t n, const int* __restrict__ qinv) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = blockIdx.y;
    if (j >= n) return;
    const int64_t src = qinv[j];
    out[2 * (i * n + j)] = X[2 * (i * n + src)];
    out[2 * (i * n + j) + 1] = X[2 * (i * n + src) + 1];
}

// The next panel's diagonal block depends only on its own tile of the trailing
// update, so a second stream updates that tile and inverts it while the first
// runs the rest of the update (the inversion is one workgroup and would
// otherwise leave the device idle for its whole duration).
hipError_t launch_dense_invert(double* A, int64_t n, int* piv, int* flag, hipStream_t s) {
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int), s);
    if (e != hipSuccess) return e;
    hipStream_t s2 = nullptr;
    hipEvent_t ev_row = nullptr, ev_tile = nullptr, ev_diag = nullptr;
    auto cleanup = [&]() {
        if (ev_row) (void)hipEventDestroy(ev_row);
        if (ev_tile) (void)hipEventDestroy(ev_tile);
        if (ev_diag) (void)hipEventDestroy(ev_diag);
        if (s2) (void)hipStreamDestroy(s2);
    };
    if (n > GJ_NB) {
        if ((e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&ev_row, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&ev_tile, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&ev_diag, hipEventDisableTiming)) != hipSuccess) {
            cleanup();
            return e;
        }
    }
    const unsigned tiles = (unsigned)((n + 63) / 64);
    for (int64_t k0 = 0; k0 < n; k0 += GJ_NB) {
        const int kb = (int)std::min<int64_t>(GJ_NB, n - k0);
        const int64_t k1 = k0 + kb;   // first index of the next panel
        if (k0 == 0)
            EHH_LAUNCH(k_diag_inverse, 1, GJ_THREADS, 0, s, A, n, k0, kb, piv, flag);
        else if ((e = hipStreamWaitEvent(s, ev_diag, 0)) != hipSuccess)
            break;
        EHH_LAUNCH(k_swap_rows, nblk(n), 256, 0, s, A, n, k0, kb, piv);
        double* AK = A + 2 * k0 * n;           // rows K
        double* AKK = AK + 2 * k0;             // the inverted block W
        double* ACK = A + 2 * k0;              // columns K
        // A[K,J] <- W A[K,J]
        EHH_LAUNCH(k_zgemm_tile, dim3(tiles, 1), 256, 0, s, AK, n, AKK, n, AK, n, (int64_t)kb, n, kb, 1.0, 0,
                           (int64_t)0, (int64_t)0, k0, k1, (int64_t)-1, (int64_t)-1);
        int64_t skip = -1;
        if (k1 < n) {
            // the next diagonal tile: A[K1,K1] -= A[K1,K] A[K,K1] (A[K1,K] before
            // its scaling below), then its inverse, on the second stream
            const int kb1 = (int)std::min<int64_t>(GJ_NB, n - k1);
            if ((e = hipEventRecord(ev_row, s)) != hipSuccess || (e = hipStreamWaitEvent(s2, ev_row, 0)) != hipSuccess)
                break;
            EHH_LAUNCH(k_zgemm_tile, dim3(1, 1), 256, 0, s2, A + 2 * (k1 * n + k1), n, A + 2 * (k1 * n + k0),
                               n, A + 2 * (k0 * n + k1), n, (int64_t)kb1, (int64_t)kb1, kb, -1.0, 1, (int64_t)0,
                               (int64_t)0, (int64_t)0, (int64_t)0, (int64_t)-1, (int64_t)-1);
            if ((e = hipEventRecord(ev_tile, s2)) != hipSuccess) break;
            EHH_LAUNCH(k_diag_inverse, 1, GJ_THREADS, 0, s2, A, n, k1, kb1, piv, flag);
            if ((e = hipEventRecord(ev_diag, s2)) != hipSuccess) break;
            skip = k1;
        }
        // A[I,J] <- A[I,J] - A[I,K] A[K,J] (but the next diagonal tile), after
        // that tile: its inversion is then queued before the update fills the
        // device, and A[K1,K] has been read before it is scaled below
        if (k1 < n && (e = hipStreamWaitEvent(s, ev_tile, 0)) != hipSuccess) break;
        EHH_LAUNCH(k_zgemm_tile, dim3(tiles, tiles), 256, 0, s, A, n, ACK, n, AK, n, n, n, kb, -1.0, 1, k0,
                           k1, k0, k1, skip, skip);
        // A[I,K] <- -A[I,K] W
        EHH_LAUNCH(k_zgemm_tile, dim3(1, tiles), 256, 0, s, ACK, n, ACK, n, AKK, n, n, (int64_t)kb, kb, -1.0,
                           0, k0, k1, (int64_t)0, (int64_t)0, (int64_t)-1, (int64_t)-1);
    }
    if (e == hipSuccess) e = hipGetLastError();
    cleanup();
    return e;
}

hipError_t launch_permute_columns(const double* X, double* out, int64_t n, const int* qinv, hipStream_t s) {
    EHH_LAUNCH(k_permute_columns, dim3(nblk(n), (unsigned)n), 256, 0, s, X, out, n, qinv);
    return hipGetLastError();
}

// ------------------------------------------------------------------ coarse apply
// One 64-wide wavefront per (row, group of up to 4 right-hand sides): lanes stride
// over the columns with FP64 accumulation and a butterfly reduction.  The grid
// spans rows x right-hand-side groups so that a batch fills the chip.
template <typename T>
EHH_DEV void k_coarse_apply_body(VB ehh_vb, const double* __restrict__ inv, int64_t n, const T* __restrict__ r, T* __restrict__ e, int nrhs) {
    constexpr int RG = 4;
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)ehh_vb.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
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
__global__ __launch_bounds__(256) void k_coarse_apply(const double* __restrict__ inv, int64_t n, const T* __restrict__ r,
                                                      T* __restrict__ e, int nrhs) {
    k_coarse_apply_body<T>(single_block<false>(), inv, n, r, e, nrhs);
}
template <class PK, typename T>
__global__ __launch_bounds__(256) void k_coarse_apply_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_coarse_apply_body<T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// Many right-hand sides: a workgroup owns 512/W rows and W right-hand sides and
// walks the columns in chunks of 64, staging the rows' chunk of the inverse and
// the vectors' chunk (as FP64) in LDS, so that the matrix is read from HBM once
// per W right-hand sides instead of once per 4.  Thread: one right-hand side,
// two rows; the row values are LDS broadcasts within a wavefront.
template <typename T, int W>
EHH_DEV void k_coarse_apply_multi_body(VB ehh_vb, const double* __restrict__ inv, int64_t n, const T* __restrict__ r, T* __restrict__ e, int nrhs, int64_t kseg, double* __restrict__ part) {
    constexpr int ROWS = 512 / W;
    constexpr int KC = 64;
    __shared__ double Ms[ROWS][KC * 2];
    __shared__ double Xs[KC][W * 2];
    const int t = threadIdx.x;
    const int q = t % W, rg = t / W;
    const int64_t i0 = (int64_t)ehh_vb.x * ROWS;
    const int q0 = blockIdx.y * W;
    const int64_t jb = (int64_t)blockIdx.z * kseg;
    const int64_t je = jb + kseg < n ? jb + kseg : n;
    double a0r = 0.0, a0i = 0.0, a1r = 0.0, a1i = 0.0;
    for (int64_t j0 = jb; j0 < je; j0 += KC) {
        for (int el = t; el < ROWS * KC; el += 256) {
            const int rr = el / KC, cc = el % KC;
            const int64_t gi = i0 + rr, gj = j0 + cc;
            double vr = 0.0, vi = 0.0;
            if (gi < n && gj < je) {
                vr = inv[2 * (gi * n + gj)];
                vi = inv[2 * (gi * n + gj) + 1];
            }
            Ms[rr][2 * cc] = vr;
            Ms[rr][2 * cc + 1] = vi;
        }
        for (int el = t; el < KC * W; el += 256) {
            const int kk = el % KC, qq = el / KC;
            const int64_t gj = j0 + kk;
            double vr = 0.0, vi = 0.0;
            if (gj < je && q0 + qq < nrhs) {
                const T* rv = r + (int64_t)(q0 + qq) * 2 * n;
                vr = (double)rv[gj];
                vi = (double)rv[n + gj];
            }
            Xs[kk][2 * qq] = vr;
            Xs[kk][2 * qq + 1] = vi;
        }
        __syncthreads();
#pragma unroll 8
        for (int kk = 0; kk < KC; ++kk) {
            const double xr = Xs[kk][2 * q], xi = Xs[kk][2 * q + 1];
            const double m0r = Ms[2 * rg][2 * kk], m0i = Ms[2 * rg][2 * kk + 1];
            const double m1r = Ms[2 * rg + 1][2 * kk], m1i = Ms[2 * rg + 1][2 * kk + 1];
            a0r = fma(m0r, xr, fma(-m0i, xi, a0r));
            a0i = fma(m0r, xi, fma(m0i, xr, a0i));
            a1r = fma(m1r, xr, fma(-m1i, xi, a1r));
            a1i = fma(m1r, xi, fma(m1i, xr, a1i));
        }
        __syncthreads();
    }
    if (q0 + q >= nrhs) return;
    const int64_t g0 = i0 + 2 * rg;
    if (part) {   // partial sum of column segment blockIdx.z, reduced by k_coarse_reduce
        double* pv = part + ((int64_t)blockIdx.z * nrhs + q0 + q) * 2 * n;
        if (g0 < n) {
            pv[g0] = a0r;
            pv[n + g0] = a0i;
        }
        if (g0 + 1 < n) {
            pv[g0 + 1] = a1r;
            pv[n + g0 + 1] = a1i;
        }
        return;
    }
    T* ev = e + (int64_t)(q0 + q) * 2 * n;
    if (g0 < n) {
        ev[g0] = (T)a0r;
        ev[n + g0] = (T)a0i;
    }
    if (g0 + 1 < n) {
        ev[g0 + 1] = (T)a1r;
        ev[n + g0 + 1] = (T)a1i;
    }
}
template <typename T, int W>
__global__ __launch_bounds__(256) void k_coarse_apply_multi(const double* __restrict__ inv, int64_t n,
                                                            const T* __restrict__ r, T* __restrict__ e, int nrhs,
                                                            int64_t kseg, double* __restrict__ part) {
    k_coarse_apply_multi_body<T, W>(single_block<false>(), inv, n, r, e, nrhs, kseg, part);
}
template <class PK, typename T, int W>
__global__ __launch_bounds__(256) void k_coarse_apply_multi_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_coarse_apply_multi_body<T, W>(ehh_vb, a...); }, b.arg[ehh_s]);
}


// Matrix-core variant (FP64 MFMA 16x16x4) for groups of up to 32 right-hand
// sides: a workgroup owns 64 rows x 32 right-hand sides of one column segment and
// stages 32-column chunks of the inverse and of the vectors in LDS (the next
// chunk is loaded into registers during the products of the current); wave w keeps
// the 16 x 16 output blocks of rows 16 w .. 16 w + 15 and both 16-source halves.
// A complex product takes four real MFMAs (re*re - im*im, re*im + im*re).
// Operand layout of v_mfma_f64_16x16x4 (checked on MI355X): lane l holds
// A[l % 16][l / 16] and B[l / 16][l % 16]; register r of lane l holds the result
// D[l / 16 + 4 r][l % 16].
typedef double ehh_d4 __attribute__((ext_vector_type(4)));
template <typename T>
EHH_DEV void k_coarse_apply_mfma_body(VB ehh_vb, const double* __restrict__ inv, int64_t n, const T* __restrict__ r, T* __restrict__ e, int nrhs, int64_t kseg, double* __restrict__ part) {
    constexpr int ROWS = 64, W = 32, KC = 32, MS = KC + 1;   // MS: padded row of the staged chunk
    constexpr int NM = ROWS * KC / 256, NX = KC * W / 256;   // staged values per thread
    __shared__ double Ms[ROWS * MS * 2];
    __shared__ double Xs[KC * W * 2];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t i0 = (int64_t)ehh_vb.x * ROWS;
    const int q0 = blockIdx.y * W;
    const int64_t jb = (int64_t)blockIdx.z * kseg;
    const int64_t je = jb + kseg < n ? jb + kseg : n;
    ehh_d4 dre[2], dim[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) dre[h] = dim[h] = ehh_d4{0.0, 0.0, 0.0, 0.0};
    const int li = lane & 15, lk = lane >> 4;
    // the next chunk is read into registers while the current one is multiplied
    double pmr[NM], pmi[NM], pxr[NX], pxi[NX];
    auto fetch = [&](int64_t j0) {
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            const int el = t + 256 * m;
            const int64_t gi = i0 + el / KC, gj = j0 + el % KC;
            const bool ok = gi < n && gj < je;
            pmr[m] = ok ? inv[2 * (gi * n + gj)] : 0.0;
            pmi[m] = ok ? inv[2 * (gi * n + gj) + 1] : 0.0;
        }
#pragma unroll
        for (int m = 0; m < NX; ++m) {
            const int el = t + 256 * m;
            const int kk = el % KC, qq = el / KC;
            const int64_t gj = j0 + kk;
            const bool ok = gj < je && q0 + qq < nrhs;
            const T* rv = r + (int64_t)(ok ? q0 + qq : 0) * 2 * n;
            pxr[m] = ok ? (double)rv[gj] : 0.0;
            pxi[m] = ok ? (double)rv[n + gj] : 0.0;
        }
    };
    if (jb < je) fetch(jb);
    for (int64_t j0 = jb; j0 < je; j0 += KC) {
#pragma unroll
        for (int m = 0; m < NM; ++m) {
            const int el = t + 256 * m;
            const int rr = el / KC, cc = el % KC;
            Ms[2 * (rr * MS + cc)] = pmr[m];
            Ms[2 * (rr * MS + cc) + 1] = pmi[m];
        }
#pragma unroll
        for (int m = 0; m < NX; ++m) {
            const int el = t + 256 * m;
            const int kk = el % KC, qq = el / KC;
            Xs[2 * (kk * W + qq)] = pxr[m];
            Xs[2 * (kk * W + qq) + 1] = pxi[m];
        }
        __syncthreads();
        if (j0 + KC < je) fetch(j0 + KC);
#pragma unroll
        for (int kb = 0; kb < KC; kb += 4) {
            const int row = 16 * w + li, col = kb + lk;
            const double ar = Ms[2 * (row * MS + col)], ai = Ms[2 * (row * MS + col) + 1];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int q = 16 * h + li;
                const double xr = Xs[2 * (col * W + q)], xi = Xs[2 * (col * W + q) + 1];
                dre[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, xr, dre[h], 0, 0, 0);
                dre[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai, xi, dre[h], 0, 0, 0);
                dim[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar, xi, dim[h], 0, 0, 0);
                dim[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai, xr, dim[h], 0, 0, 0);
            }
        }
        lds_barrier();
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = q0 + 16 * h + li;
        if (q >= nrhs) continue;
#pragma unroll
        for (int rg = 0; rg < 4; ++rg) {
            const int64_t g = i0 + 16 * w + lk + 4 * rg;
            if (g >= n) continue;
            if (part) {
                double* pv = part + ((int64_t)blockIdx.z * nrhs + q) * 2 * n;
                pv[g] = dre[h][rg];
                pv[n + g] = dim[h][rg];
            } else {
                T* ev = e + (int64_t)q * 2 * n;
                ev[g] = (T)dre[h][rg];
                ev[n + g] = (T)dim[h][rg];
            }
        }
    }
}
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_apply_mfma(const double* __restrict__ inv, int64_t n,
                                                           const T* __restrict__ r, T* __restrict__ e, int nrhs,
                                                           int64_t kseg, double* __restrict__ part) {
    k_coarse_apply_mfma_body<T>(single_block<false>(), inv, n, r, e, nrhs, kseg, part);
}
template <class PK, typename T>
__global__ __launch_bounds__(256) void k_coarse_apply_mfma_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_coarse_apply_mfma_body<T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// e = sum over the column segments of the partial products, in segment order.
template <typename T>
EHH_DEV void k_coarse_reduce_body(VB ehh_vb, const double* __restrict__ part, int ks, int64_t n, int nrhs, T* __restrict__ e) {
    const int64_t t = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (t >= 2 * n * nrhs) return;
    double s = 0.0;
    for (int z = 0; z < ks; ++z) s += part[(int64_t)z * 2 * n * nrhs + t];
    e[t] = (T)s;
}
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_reduce(const double* __restrict__ part, int ks, int64_t n, int nrhs,
                                                       T* __restrict__ e) {
    k_coarse_reduce_body<T>(single_block<false>(), part, ks, n, nrhs, e);
}
template <class PK, typename T>
__global__ __launch_bounds__(256) void k_coarse_reduce_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_coarse_reduce_body<T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// ------------------------------------------------ symmetric coarse apply
// The coarsest operator is complex symmetric (a Galerkin product P^T A P of the
// complex symmetric operator of eq. (14)), hence so is its inverse: only the
// 64 x 64 tiles (I, J) with I >= J are kept, tile after tile (row-major inside a
// tile, diagonal tiles whole, entries beyond n zero); tile (I, J) sits at
// I (I + 1) / 2 + J.  A tile below the diagonal then serves both y_I += A_IJ x_J
// and y_J += A_IJ^T x_I, so a solve streams half the inverse.
constexpr int SY = 64;

static inline __device__ void sym_tile_of(int64_t b, int& I, int& J) {
    int i = (int)((sqrt(8.0 * (double)b + 1.0) - 1.0) * 0.5);
    while ((int64_t)(i + 1) * (i + 2) / 2 <= b) ++i;
    while ((int64_t)i * (i + 1) / 2 > b) --i;
    I = i;
    J = (int)(b - (int64_t)i * (i + 1) / 2);
}

__global__ __launch_bounds__(256) void k_pack_sym(const double* __restrict__ inv, int64_t n,
                                                  double* __restrict__ sym, int64_t total) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    int I, J;
    sym_tile_of(e / (SY * SY), I, J);
    const int w = (int)(e % (SY * SY));
    const int64_t gi = (int64_t)I * SY + w / SY, gj = (int64_t)J * SY + w % SY;
    double vr = 0.0, vi = 0.0;
    if (gi < n && gj < n) {
        vr = inv[2 * (gi * n + gj)];
        vi = inv[2 * (gi * n + gj) + 1];
    }
    sym[2 * e] = vr;
    sym[2 * e + 1] = vi;
}

// One step of a recursive-halving sum over lanes: lanes with bit M set keep the
// upper HALF of their values, the others the lower half, each adding its
// partner's copy (all exchanges issued before the sums).
template <int HALF, int M>
__device__ inline void halve_step(double* vr, double* vi, int lane) {
    const bool up = (lane & M) != 0;
    double gr[HALF], gi[HALF];
#pragma unroll
    for (int rr = 0; rr < HALF; ++rr) {
        gr[rr] = __shfl_xor(up ? vr[rr] : vr[rr + HALF], M, 64);
        gi[rr] = __shfl_xor(up ? vi[rr] : vi[rr + HALF], M, 64);
    }
#pragma unroll
    for (int rr = 0; rr < HALF; ++rr) {
        vr[rr] = (up ? vr[rr + HALF] : vr[rr]) + gr[rr];
        vi[rr] = (up ? vi[rr + HALF] : vi[rr]) + gi[rr];
    }
}

// One workgroup per stored tile and group of up to 4 right-hand sides; wave w
// takes rows 16 w .. 16 w + 15 of the tile, lane = column.  The row products are
// summed over the lanes by recursive halving (16 partial sums per lane folded
// into one per lane in four exchange steps, then two more), the column products
// over the rows of a wave in registers and over the four waves in LDS.  Partial
// results go to ws[q][X_out][J_src][64] and are summed by k_sym_reduce (a
// separate launch: a device-wide fence, which a last-workgroup-sums scheme would
// need, writes back the L2 of each XCD and costs more than the launch).
template <typename T>
EHH_DEV void k_coarse_apply_sym_body(VB ehh_vb, const double* __restrict__ sym, int64_t n, int nb, const T* __restrict__ r, int nrhs, double* __restrict__ ws) {
    constexpr int RG = 4;
    __shared__ double xs[2][RG][SY][2];
    __shared__ double cs[4][RG][SY][2];
    int I, J;
    sym_tile_of(ehh_vb.x, I, J);
    const int r0 = blockIdx.y * RG;
    const int nr = nrhs - r0 < RG ? nrhs - r0 : RG;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // x_I (side 0) and x_J (side 1) of the group's right-hand sides
    for (int e2 = threadIdx.x; e2 < 2 * RG * SY; e2 += blockDim.x) {
        const int side = e2 / (RG * SY), q = (e2 / SY) % RG, i = e2 % SY;
        const int64_t gi = (int64_t)(side == 0 ? I : J) * SY + i;
        double vr = 0.0, vi = 0.0;
        if (q < nr && gi < n) {
            const T* rv = r + (int64_t)(r0 + q) * 2 * n;
            vr = (double)rv[gi];
            vi = (double)rv[n + gi];
        }
        xs[side][q][i][0] = vr;
        xs[side][q][i][1] = vi;
    }
    __syncthreads();
    const double* tile = sym + (size_t)ehh_vb.x * SY * SY * 2;
    double ar[16], ai[16];
#pragma unroll
    for (int rr = 0; rr < 16; ++rr) {
        const int i = 16 * w + rr;
        ar[rr] = tile[2 * (i * SY + lane)];
        ai[rr] = tile[2 * (i * SY + lane) + 1];
    }
    const bool offdiag = I != J;
#pragma unroll 1
    for (int q = 0; q < nr; ++q) {
        const double xjr = xs[1][q][lane][0], xji = xs[1][q][lane][1];
        double vr[16], vi[16];
        double cr = 0.0, ci = 0.0;
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
            vr[rr] = ar[rr] * xjr - ai[rr] * xji;
            vi[rr] = ar[rr] * xji + ai[rr] * xjr;
            const double xir = xs[0][q][16 * w + rr][0], xii = xs[0][q][16 * w + rr][1];
            cr += ar[rr] * xir - ai[rr] * xii;
            ci += ar[rr] * xii + ai[rr] * xir;
        }
        // recursive halving over lane bits 5..2; afterwards lane l holds row l >> 2
        halve_step<8, 32>(vr, vi, lane);
        halve_step<4, 16>(vr, vi, lane);
        halve_step<2, 8>(vr, vi, lane);
        halve_step<1, 4>(vr, vi, lane);
        double tr = vr[0], ti = vi[0];
        tr += __shfl_xor(tr, 2, 64);
        ti += __shfl_xor(ti, 2, 64);
        tr += __shfl_xor(tr, 1, 64);
        ti += __shfl_xor(ti, 1, 64);
        if ((lane & 3) == 0) {
            double* o = ws + 2 * ((((int64_t)(r0 + q) * nb + I) * nb + J) * SY + 16 * w + (lane >> 2));
            o[0] = tr;
            o[1] = ti;
        }
        cs[w][q][lane][0] = cr;
        cs[w][q][lane][1] = ci;
    }
    lds_barrier();
    if (offdiag) {
        for (int e2 = threadIdx.x; e2 < nr * SY; e2 += blockDim.x) {
            const int q = e2 / SY, j = e2 % SY;
            double sr = 0.0, si = 0.0;
#pragma unroll
            for (int ww = 0; ww < 4; ++ww) {
                sr += cs[ww][q][j][0];
                si += cs[ww][q][j][1];
            }
            double* o = ws + 2 * ((((int64_t)(r0 + q) * nb + J) * nb + I) * SY + j);
            o[0] = sr;
            o[1] = si;
        }
    }
}
template <typename T>
__global__ __launch_bounds__(256) void k_coarse_apply_sym(const double* __restrict__ sym, int64_t n, int nb,
                                                          const T* __restrict__ r, int nrhs,
                                                          double* __restrict__ ws) {
    k_coarse_apply_sym_body<T>(single_block<false>(), sym, n, nb, r, nrhs, ws);
}
template <class PK, typename T>
__global__ __launch_bounds__(256) void k_coarse_apply_sym_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_coarse_apply_sym_body<T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// e[q][X * 64 + i] = sum over the source blocks J of ws[q][X][J][i], four lanes
// per output (each a fixed quarter of the sources, then a fixed pairwise sum).
template <typename T>
EHH_DEV void k_sym_reduce_body(VB ehh_vb, const double* __restrict__ ws, int64_t n, int nb, int nrhs, T* __restrict__ e) {
    const int64_t t = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    const int part = (int)(t & 3);
    const int64_t o = t >> 2;
    const bool live = o < n * nrhs;
    const int64_t q = live ? o / n : 0, gi = live ? o % n : 0;
    const int64_t X = gi / SY, i = gi % SY;
    const double* p = ws + 2 * (((q * nb + X) * nb) * SY + i);
    const int per = (nb + 3) / 4;
    const int j0 = part * per, j1 = j0 + per < nb ? j0 + per : nb;
    double sr = 0.0, si = 0.0;
    if (live) {
        int Jb = j0;
        for (; Jb + 4 <= j1; Jb += 4) {
            double vr[4], vi[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                vr[u] = p[2 * (int64_t)(Jb + u) * SY];
                vi[u] = p[2 * (int64_t)(Jb + u) * SY + 1];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                sr += vr[u];
                si += vi[u];
            }
        }
        for (; Jb < j1; ++Jb) {
            sr += p[2 * (int64_t)Jb * SY];
            si += p[2 * (int64_t)Jb * SY + 1];
        }
    }
    sr += __shfl_xor(sr, 1, 64);
    si += __shfl_xor(si, 1, 64);
    sr += __shfl_xor(sr, 2, 64);
    si += __shfl_xor(si, 2, 64);
    if (live && part == 0) {
        T* ev = e + q * 2 * n;
        ev[gi] = (T)sr;
        ev[n + gi] = (T)si;
    }
}
template <typename T>
__global__ __launch_bounds__(256) void k_sym_reduce(const double* __restrict__ ws, int64_t n, int nb, int nrhs,
                                                    T* __restrict__ e) {
    k_sym_reduce_body<T>(single_block<false>(), ws, n, nb, nrhs, e);
}
template <class PK, typename T>
__global__ __launch_bounds__(256) void k_sym_reduce_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_sym_reduce_body<T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

int64_t sym_tiles(int64_t n) {
    const int64_t nb = (n + SY - 1) / SY;
    return nb * (nb + 1) / 2;
}
hipError_t launch_pack_sym(const double* inv, int64_t n, double* sym, hipStream_t s) {
    const int64_t total = sym_tiles(n) * SY * SY;
    EHH_LAUNCH(k_pack_sym, nblk(total), 256, 0, s, inv, n, sym, total);
    return hipGetLastError();
}
// Workspace of the symmetric apply (partial results; rewritten by every call).
static size_t sym_ws_doubles(int64_t n, int nrhs) {
    const int64_t nb = (n + SY - 1) / SY;
    return (size_t)2 * SY * nb * nb * nrhs;
}


// Column segments of the multi-right-hand-side coarse apply: enough workgroups to
// fill the chip (about 1024), segments of at least 256 columns.
static int coarse_width(int nrhs) { return nrhs <= 4 ? 0 : nrhs <= 8 ? 8 : nrhs <= 16 ? 16 : 32; }
int coarse_ksplit(int64_t n, int nrhs) {
    const int W = coarse_width(nrhs);
    if (W == 0) return 1;
    const int rows = W == 32 ? 64 : 512 / W;   // rows per workgroup
    const int64_t blocks = ((n + rows - 1) / rows) * ((nrhs + W - 1) / W);
    int64_t ks = (1024 + blocks - 1) / blocks;
    const int64_t kmax = n / 256 > 1 ? n / 256 : 1;
    ks = ks < 1 ? 1 : (ks > kmax ? kmax : ks);
    return (int)ks;
}
size_t coarse_ws_doubles(int64_t n, int nrhs) {
    if (coarse_width(nrhs) == 0) return sym_ws_doubles(n, nrhs);
    const int ks = coarse_ksplit(n, nrhs);
    return ks > 1 ? (size_t)ks * 2 * n * nrhs : 0;
}

// A few right-hand sides: the packed symmetric inverse (half the bytes) where it
// is given with a workspace, else one wavefront per row of the full inverse.
template <typename T>
hipError_t launch_coarse_apply(const double* inv, const double* sym, int64_t n, const T* r, T* e, int nrhs,
                               double* ws, hipStream_t s) {
    const int W = coarse_width(nrhs);
    // algorithmic bytes: the inverse (packed half or whole) once, r read, e written
    const double vec = nrhs * 2.0 * sizeof(T) * (double)n;
    const LaunchBytes lb_sym{(double)sym_tiles(n) * SY * SY * 16.0 + vec, 16.0 * n * n + vec};
    const LaunchBytes lb_full{16.0 * n * n + vec, 16.0 * n * n + vec};
    const LaunchBytes lb_red{vec, vec};
    if (W == 0 && sym && ws) {   // W == 0: one group of at most 4 right-hand sides
        const int nb = (int)((n + SY - 1) / SY);
        EHH_LAUNCHK(lb_sym, k_coarse_apply_sym, (T), dim3((unsigned)sym_tiles(n), 1), 256, 0, s, sym, n, nb, r, nrhs,
                           ws);
        EHH_LAUNCHK(lb_red, k_sym_reduce, (T), nblk(4 * n * nrhs), 256, 0, s, ws, n, nb, nrhs, e);
        return hipGetLastError();
    }
    if (W == 0) {
        EHH_LAUNCHK(lb_full, k_coarse_apply, (T), dim3(nblk(n * 64), (nrhs + 3) / 4), 256, 0, s, inv, n, r, e, nrhs);
        return hipGetLastError();
    }
    int ks = coarse_ksplit(n, nrhs);
    if (ks > 1 && !ws) ks = 1;
    const int64_t kseg = ((n + ks - 1) / ks + 63) / 64 * 64;
    ks = (int)((n + kseg - 1) / kseg);
    double* part = ks > 1 ? ws : nullptr;
    if (W == 32) {   // the FP64 matrix cores (groups of 32 right-hand sides)
        const dim3 grid_rb((unsigned)((n + 63) / 64), (unsigned)((nrhs + 31) / 32), (unsigned)ks);
        EHH_LAUNCHK(lb_full, k_coarse_apply_mfma, (T), grid_rb, 256, 0, s, inv, n, r, e, nrhs, kseg, part);
        if (part) EHH_LAUNCHK(lb_red, k_coarse_reduce, (T), nblk(2 * n * nrhs), 256, 0, s, part, ks, n, nrhs, e);
        return hipGetLastError();
    }
    const unsigned rows = (unsigned)((n + 512 / W - 1) / (512 / W));
    const dim3 grid(rows, (unsigned)((nrhs + W - 1) / W), (unsigned)ks);
    if (W == 8)
        EHH_LAUNCHK(lb_full, k_coarse_apply_multi, (T, 8), grid, 256, 0, s, inv, n, r, e, nrhs, kseg, part);
    else
        EHH_LAUNCHK(lb_full, k_coarse_apply_multi, (T, 16), grid, 256, 0, s, inv, n, r, e, nrhs, kseg, part);
    if (part) EHH_LAUNCHK(lb_red, k_coarse_reduce, (T), nblk(2 * n * nrhs), 256, 0, s, part, ks, n, nrhs, e);
    return hipGetLastError();
}
// Scratch of the coarsest solve for callers that cannot allocate
// (ehh_coarse_solve_noalloc): the column-segment partial sums live in this
// library-wide array, one copy per device, held until the process ends.  In
// host code the name stands for a host-side symbol, never a device address:
// the address of each device's copy comes from hipGetSymbolAddress, taken once
// per device with that device current, and only that address is used.
static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace {
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> l(g_scratch_mutex);
    if (g_scratch_ptr[dev]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev) return hipErrorInvalidDevice;   // the caller makes dev current
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (double*)p;
    return hipSuccess;
}

double* noalloc_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> l(g_scratch_mutex);
    return g_scratch_ptr[dev];
}

template hipError_t launch_coarse_apply<float>(const double*, const double*, int64_t, const float*, float*, int,
                                               double*, hipStream_t);
template hipError_t launch_coarse_apply<double>(const double*, const double*, int64_t, const double*, double*, int,
                                                double*, hipStream_t);

template <int Z = 0>
EHH_DEV void k_zero_words_body(VB ehh_vb, uint32_t* __restrict__ p, int64_t n) {
    const int64_t i = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}
template <int Z = 0>
__global__ void k_zero_words(uint32_t* __restrict__ p, int64_t n) {
    k_zero_words_body<Z>(single_block<false>(), p, n);
}
template <class PK, int Z = 0>
__global__ __launch_bounds__(256) void k_zero_words_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_zero_words_body<Z>(ehh_vb, a...); }, b.arg[ehh_s]);
}
// Zero fill by a kernel (not a memset node, so it may sit inside a captured graph).
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    const int64_t n = (int64_t)(bytes / 4);
    EHH_LAUNCHK(bytes_plain((double)bytes), k_zero_words, (0), nblk(n), 256, 0, s, (uint32_t*)p, n);
    return hipGetLastError();
}

template <int Z = 0>
EHH_DEV void k_cast_d2f_body(VB ehh_vb, const double* __restrict__ in, float* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}
template <int Z = 0>
__global__ void k_cast_d2f(const double* __restrict__ in, float* __restrict__ out, int64_t n) {
    k_cast_d2f_body<Z>(single_block<false>(), in, out, n);
}
template <class PK, int Z = 0>
__global__ __launch_bounds__(256) void k_cast_d2f_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_cast_d2f_body<Z>(ehh_vb, a...); }, b.arg[ehh_s]);
}
template <int Z = 0>
EHH_DEV void k_cast_f2d_body(VB ehh_vb, const float* __restrict__ in, double* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (double)in[i];
}
template <int Z = 0>
__global__ void k_cast_f2d(const float* __restrict__ in, double* __restrict__ out, int64_t n) {
    k_cast_f2d_body<Z>(single_block<false>(), in, out, n);
}
template <class PK, int Z = 0>
__global__ __launch_bounds__(256) void k_cast_f2d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_cast_f2d_body<Z>(ehh_vb, a...); }, b.arg[ehh_s]);
}
hipError_t launch_cast_d2f(const double* in, float* out, int64_t n, hipStream_t s) {
    EHH_LAUNCHK(bytes_plain(12.0 * n), k_cast_d2f, (0), nblk(n), 256, 0, s, in, out, n);
    return hipGetLastError();
}
hipError_t launch_cast_f2d(const float* in, double* out, int64_t n, hipStream_t s) {
    EHH_LAUNCHK(bytes_plain(12.0 * n), k_cast_f2d, (0), nblk(n), 256, 0, s, in, out, n);
    return hipGetLastError();
}

}  // namespace ehh
