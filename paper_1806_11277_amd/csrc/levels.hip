// Multigrid level kernels: operator application / residual, damped red-black
// cell-wise Vanka half-sweep, restriction P^T and prolongation-correction.
//
// Every kernel loops over the right-hand sides inside the thread so that the
// operator coefficients (and the Vanka block factorisation) are read and
// formed once per cell for the whole batch.
#include "internal.hpp"
#include "ops.hpp"

namespace ehh {

// --------------------------------------------------------------- y = A x, r = b - A x
// One thread per cell; the cell owns its low face of every component (if that
// face is interior) and its pressure.
template <int D, typename T, class Op>
__global__ __launch_bounds__(256) void k_apply(Op op, const T* __restrict__ x, const T* __restrict__ b,
                                               T* __restrict__ y, int nrhs, int64_t stride) {
    const Geo& g = op.g;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.ncell) return;
    int c[3];
    cell_pos<D>(g, t, c);
    for (int r = 0; r < nrhs; ++r) {
        const CVec<T> xv{x + r * stride, g.N};
        const Vec<T> yv{y + r * stride, g.N};
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (c[k] < 1) continue;
            const int64_t i = g.off[k] + face_idx<D>(g, k, c);
            cx<T> v = op.row_u(k, c, xv);
            if (b) {
                const CVec<T> bv{b + r * stride, g.N};
                v = bv.ld(i) - v;
            }
            yv.st(i, v);
        }
        const int64_t ip = g.off[3] + cell_idx<D>(g, c);
        cx<T> v = op.row_p(c, xv);
        if (b) {
            const CVec<T> bv{b + r * stride, g.N};
            v = bv.ld(ip) - v;
        }
        yv.st(ip, v);
    }
}

// ------------------------------------------------------------ red-black Vanka half-sweep
// One thread per pair of cells along x: the cell of the swept colour is relaxed
// (its 2D+1 unknowns: both faces of every component and the pressure), the other
// cell only has its pressure carried over.  Every face belongs to exactly one cell
// of each colour, so the pairs together write each unknown once.  The residual of
// the cell's unknowns is taken from e_in (the state at the start of the
// half-sweep); the update e_out = e_in + w B_K^{-1} r_K uses the closed form of
// the block: one 2x2 complex system per displacement component (diagonal only in
// the economic variant) and the scalar Schur complement on the pressure.
template <int D, typename T, class Op>
__global__ __launch_bounds__(256) void k_relax(Op op, int colour, T w, int econ,
                                               const T* __restrict__ b, const T* __restrict__ ein,
                                               T* __restrict__ eout, int nrhs, int64_t stride) {
    const Geo& g = op.g;
    const int hp = g.n[0] >> 1;
    const int64_t npair = (int64_t)hp * g.n[1] * g.n[2];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npair) return;
    const int px = (int)(t % hp);
    const int64_t rest = t / hp;
    const int yy = (int)(rest % g.n[1]);
    const int zz = (int)(rest / g.n[1]);
    const int par = (colour + yy + zz) & 1;
    int cr[3] = {2 * px + par, yy, zz};
    int cb[3] = {2 * px + 1 - par, yy, zz};

    cx<T> i00[D], i01[D], i11[D], zlo[D], zhi[D];
    T glo[D], ghi[D];
    bool lok[D], hok[D];
    int64_t ilo[D], ihi[D];
    cx<T> S = mk<T>(op.pdiag(cr), T(0));
#pragma unroll
    for (int k = 0; k < D; ++k) {
        lok[k] = cr[k] >= 1;
        hok[k] = cr[k] + 1 <= g.n[k] - 1;
        cx<T> all, ahh, alh;
        op.block(cr, k, all, ahh, alh, glo[k], ghi[k], lok[k], hok[k]);
        if (econ) alh = mk<T>(T(0), T(0));
        const cx<T> idet = cinv(all * ahh - alh * alh);
        i00[k] = ahh * idet;
        i11[k] = all * idet;
        i01[k] = mk<T>(T(0), T(0)) - alh * idet;
        zlo[k] = glo[k] * i00[k] + ghi[k] * i01[k];
        zhi[k] = glo[k] * i01[k] + ghi[k] * i11[k];
        S = S - (glo[k] * zlo[k] + ghi[k] * zhi[k]);
        int q[3] = {cr[0], cr[1], cr[2]};
        ilo[k] = lok[k] ? g.off[k] + face_idx<D>(g, k, q) : 0;
        q[k] += 1;
        ihi[k] = hok[k] ? g.off[k] + face_idx<D>(g, k, q) : 0;
    }
    const cx<T> iS = cinv(S);
    const int64_t ipr = g.off[3] + cell_idx<D>(g, cr);
    const int64_t ipb = g.off[3] + cell_idx<D>(g, cb);
    const cx<T> zero = mk<T>(T(0), T(0));

    for (int r = 0; r < nrhs; ++r) {
        const CVec<T> bv{b + r * stride, g.N};
        const Vec<T> ov{eout + r * stride, g.N};
        const CVec<T> ev{ein ? ein + r * stride : nullptr, g.N};
        cx<T> rlo[D], rhi[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            int q[3] = {cr[0], cr[1], cr[2]};
            rlo[k] = zero;
            rhi[k] = zero;
            if (lok[k]) rlo[k] = ein ? bv.ld(ilo[k]) - op.row_u(k, q, ev) : bv.ld(ilo[k]);
            q[k] += 1;
            if (hok[k]) rhi[k] = ein ? bv.ld(ihi[k]) - op.row_u(k, q, ev) : bv.ld(ihi[k]);
        }
        const cx<T> rp = ein ? bv.ld(ipr) - op.row_p(cr, ev) : bv.ld(ipr);
        cx<T> ylo[D], yhi[D];
        cx<T> acc = rp;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            ylo[k] = i00[k] * rlo[k] + i01[k] * rhi[k];
            yhi[k] = i01[k] * rlo[k] + i11[k] * rhi[k];
            acc = acc - (glo[k] * ylo[k] + ghi[k] * yhi[k]);
        }
        const cx<T> dp = acc * iS;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (lok[k]) {
                const cx<T> d = ylo[k] - zlo[k] * dp;
                ov.st(ilo[k], (ein ? ev.ld(ilo[k]) : zero) + w * d);
            }
            if (hok[k]) {
                const cx<T> d = yhi[k] - zhi[k] * dp;
                ov.st(ihi[k], (ein ? ev.ld(ihi[k]) : zero) + w * d);
            }
        }
        ov.st(ipr, (ein ? ev.ld(ipr) : zero) + w * dp);
        ov.st(ipb, ein ? ev.ld(ipb) : zero);
    }
}

// --------------------------------------------------------------------- transfers
// Staggered bilinear transfer: u_k linear along its normal (weights 1 / (1/2, 1/2)),
// linear along each tangential axis (3/4 nearer coarse row, 1/4 the other, zero
// beyond the wall); pressure piecewise constant.  Restriction is P^T.
EHH_DEV float w_tang(int d) { return (d == 0 || d == 1) ? 0.75f : ((d == -1 || d == 2) ? 0.25f : 0.f); }

template <int D, typename T>
__global__ __launch_bounds__(256) void k_restrict(Geo gf, Geo gc, const T* __restrict__ rf,
                                                  T* __restrict__ rc, int nrhs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= gc.N) return;
    int k = 0;
    while (k < 3 && t >= gc.off[k + 1]) ++k;
    if (k >= D) k = 3;
    const int64_t li = t - gc.off[k];
    const int64_t sf = 2 * gf.N, sc = 2 * gc.N;
    if (k == 3) {
        int C[3];
        cell_pos<D>(gc, li, C);
        int64_t idx[8];
        int m = 0;
        for (int dz = 0; dz < (D == 3 ? 2 : 1); ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    int f[3] = {2 * C[0] + dx, 2 * C[1] + dy, D == 3 ? 2 * C[2] + dz : 0};
                    idx[m++] = gf.off[3] + cell_idx<D>(gf, f);
                }
        for (int r = 0; r < nrhs; ++r) {
            const CVec<T> fv{rf + r * sf, gf.N};
            cx<T> s = mk<T>(T(0), T(0));
            for (int j = 0; j < m; ++j) s = s + fv.ld(idx[j]);
            Vec<T>{rc + r * sc, gc.N}.st(t, s);
        }
        return;
    }
    int P[3];
    face_pos<D>(gc, k, li, P);
    const int t1 = tang1<D>(k), t2 = tang2<D>(k);
    const int nn2 = D == 3 ? 4 : 1;
    for (int r = 0; r < nrhs; ++r) {
        const CVec<T> fv{rf + r * sf, gf.N};
        cx<T> s = mk<T>(T(0), T(0));
        for (int a = -1; a <= 1; ++a) {
            const T wn = a == 0 ? T(1) : T(0.5);
            for (int b1 = -1; b1 <= 2; ++b1) {
                const int f1 = 2 * P[t1] + b1;
                if (f1 < 0 || f1 >= gf.n[t1]) continue;
                for (int b2i = 0; b2i < nn2; ++b2i) {
                    const int b2 = D == 3 ? b2i - 1 : 0;
                    int f[3];
                    f[k] = 2 * P[k] + a;
                    f[t1] = f1;
                    if (D == 3) {
                        f[t2] = 2 * P[t2] + b2;
                        if (f[t2] < 0 || f[t2] >= gf.n[t2]) continue;
                    } else {
                        f[2] = 0;
                    }
                    T wgt = wn * T(w_tang(b1));
                    if (D == 3) wgt *= T(w_tang(b2));
                    s = s + wgt * fv.ld(gf.off[k] + face_idx<D>(gf, k, f));
                }
            }
        }
        Vec<T>{rc + r * sc, gc.N}.st(t, s);
    }
}

template <int D, typename T>
__global__ __launch_bounds__(256) void k_prolong(Geo gf, Geo gc, const T* __restrict__ ec,
                                                 T* __restrict__ ef, int nrhs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= gf.N) return;
    int k = 0;
    while (k < 3 && t >= gf.off[k + 1]) ++k;
    if (k >= D) k = 3;
    const int64_t li = t - gf.off[k];
    const int64_t sf = 2 * gf.N, sc = 2 * gc.N;
    if (k == 3) {
        int c[3];
        cell_pos<D>(gf, li, c);
        int C[3] = {c[0] >> 1, c[1] >> 1, c[2] >> 1};
        const int64_t ci = gc.off[3] + cell_idx<D>(gc, C);
        for (int r = 0; r < nrhs; ++r) {
            const Vec<T> fv{ef + r * sf, gf.N};
            fv.st(t, fv.ld(t) + CVec<T>{ec + r * sc, gc.N}.ld(ci));
        }
        return;
    }
    int p[3];
    face_pos<D>(gf, k, li, p);
    const int t1 = tang1<D>(k), t2 = tang2<D>(k);
    // normal contributions
    int xn[2];
    T wn[2];
    int nn = 0;
    if ((p[k] & 1) == 0) {
        xn[nn] = p[k] >> 1;
        wn[nn++] = T(1);
    } else {
        xn[nn] = (p[k] - 1) >> 1;
        wn[nn++] = T(0.5);
        xn[nn] = (p[k] + 1) >> 1;
        wn[nn++] = T(0.5);
    }
    int x1[2], x2[2];
    T w1[2], w2[2];
    int n1 = 0, n2 = 0;
    {
        const int C = p[t1] >> 1, o = (p[t1] & 1) ? C + 1 : C - 1;
        x1[n1] = C;
        w1[n1++] = T(0.75);
        if (o >= 0 && o < gc.n[t1]) {
            x1[n1] = o;
            w1[n1++] = T(0.25);
        }
    }
    if (D == 3) {
        const int C = p[t2] >> 1, o = (p[t2] & 1) ? C + 1 : C - 1;
        x2[n2] = C;
        w2[n2++] = T(0.75);
        if (o >= 0 && o < gc.n[t2]) {
            x2[n2] = o;
            w2[n2++] = T(0.25);
        }
    } else {
        x2[0] = 0;
        w2[0] = T(1);
        n2 = 1;
    }
    int64_t idx[8];
    T wt[8];
    int m = 0;
    for (int a = 0; a < nn; ++a) {
        if (xn[a] < 1 || xn[a] > gc.n[k] - 1) continue;
        for (int i1 = 0; i1 < n1; ++i1)
            for (int i2 = 0; i2 < n2; ++i2) {
                int P[3];
                P[k] = xn[a];
                P[t1] = x1[i1];
                if (D == 3) P[t2] = x2[i2];
                else P[2] = 0;
                idx[m] = gc.off[k] + face_idx<D>(gc, k, P);
                wt[m++] = wn[a] * w1[i1] * w2[i2];
            }
    }
    for (int r = 0; r < nrhs; ++r) {
        const CVec<T> cv{ec + r * sc, gc.N};
        const Vec<T> fv{ef + r * sf, gf.N};
        cx<T> s = fv.ld(t);
        for (int j = 0; j < m; ++j) s = s + wt[j] * cv.ld(idx[j]);
        fv.st(t, s);
    }
}

// ------------------------------------------------------------------------ launchers
static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

template <typename T>
hipError_t launch_apply(const LevelDesc<T>& L, const T* x, const T* b, T* y, int nrhs, hipStream_t s) {
    const int64_t stride = 2 * L.g.N;
    const unsigned gb = nblk(L.g.ncell);
    if (L.g.dim == 2) {
        if (L.fine)
            hipLaunchKernelGGL((k_apply<2, T, FineOp<2, T>>), gb, 256, 0, s, FineOp<2, T>{L.g, L.f}, x, b, y, nrhs, stride);
        else
            hipLaunchKernelGGL((k_apply<2, T, StOp<2, T>>), gb, 256, 0, s, StOp<2, T>{L.g, L.s}, x, b, y, nrhs, stride);
    } else {
        if (L.fine)
            hipLaunchKernelGGL((k_apply<3, T, FineOp<3, T>>), gb, 256, 0, s, FineOp<3, T>{L.g, L.f}, x, b, y, nrhs, stride);
        else
            hipLaunchKernelGGL((k_apply<3, T, StOp<3, T>>), gb, 256, 0, s, StOp<3, T>{L.g, L.s}, x, b, y, nrhs, stride);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_relax(const LevelDesc<T>& L, int colour, double w, int econ, const T* b, const T* ein,
                        T* eout, int nrhs, hipStream_t s) {
    const int64_t stride = 2 * L.g.N;
    const int64_t npair = (int64_t)(L.g.n[0] / 2) * L.g.n[1] * L.g.n[2];
    const unsigned gb = nblk(npair);
    const T tw = (T)w;
    if (L.g.dim == 2) {
        if (L.fine)
            hipLaunchKernelGGL((k_relax<2, T, FineOp<2, T>>), gb, 256, 0, s, FineOp<2, T>{L.g, L.f}, colour, tw, econ, b, ein, eout, nrhs, stride);
        else
            hipLaunchKernelGGL((k_relax<2, T, StOp<2, T>>), gb, 256, 0, s, StOp<2, T>{L.g, L.s}, colour, tw, econ, b, ein, eout, nrhs, stride);
    } else {
        if (L.fine)
            hipLaunchKernelGGL((k_relax<3, T, FineOp<3, T>>), gb, 256, 0, s, FineOp<3, T>{L.g, L.f}, colour, tw, econ, b, ein, eout, nrhs, stride);
        else
            hipLaunchKernelGGL((k_relax<3, T, StOp<3, T>>), gb, 256, 0, s, StOp<3, T>{L.g, L.s}, colour, tw, econ, b, ein, eout, nrhs, stride);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict(const Geo& gf, const Geo& gc, const T* rf, T* rc, int nrhs, hipStream_t s) {
    if (gf.dim == 2)
        hipLaunchKernelGGL((k_restrict<2, T>), nblk(gc.N), 256, 0, s, gf, gc, rf, rc, nrhs);
    else
        hipLaunchKernelGGL((k_restrict<3, T>), nblk(gc.N), 256, 0, s, gf, gc, rf, rc, nrhs);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(const Geo& gf, const Geo& gc, const T* ec, T* ef, int nrhs, hipStream_t s) {
    if (gf.dim == 2)
        hipLaunchKernelGGL((k_prolong<2, T>), nblk(gf.N), 256, 0, s, gf, gc, ec, ef, nrhs);
    else
        hipLaunchKernelGGL((k_prolong<3, T>), nblk(gf.N), 256, 0, s, gf, gc, ec, ef, nrhs);
    return hipGetLastError();
}

#define EHH_INST(T)                                                                                       \
    template hipError_t launch_apply<T>(const LevelDesc<T>&, const T*, const T*, T*, int, hipStream_t);  \
    template hipError_t launch_relax<T>(const LevelDesc<T>&, int, double, int, const T*, const T*, T*,    \
                                        int, hipStream_t);                                               \
    template hipError_t launch_restrict<T>(const Geo&, const Geo&, const T*, T*, int, hipStream_t);      \
    template hipError_t launch_prolong<T>(const Geo&, const Geo&, const T*, T*, int, hipStream_t);
EHH_INST(float)
EHH_INST(double)

}  // namespace ehh
