// Row evaluation of the level operators and the cell-wise Vanka block.
//
// FineOp: the matrix-free staggered operator of eq. (14) on the finest level,
//   u_k rows: grad^T A_e(mu) grad (weighted vector Laplacian of eq. (4), normal
//   derivative weights mu at cells, tangential weights mu averaged over the
//   existing cells adjacent to the edge/node), - w^2 A_f(rho (1 - i (gamma + alpha)))
//   (eq. (5), eq. (10)), + grad_h p; p rows: grad_h^T u - p / (lambda + mu).
// StOp: the Galerkin operators of the coarse levels (eq. (9)) held as stencils:
//   3 x 5 (x 5) u_k-u_k entries (upper half stored, the rest read transposed from
//   the neighbour, the matrices being complex symmetric), 2 x 3 (x 3) real u_k-p
//   entries and a real p-p diagonal.
#pragma once

#include "common.hpp"

namespace ehh {

template <int D, typename T> struct FineOp {
    Geo g;
    FineCoef<T> c;

    EHH_DEV T mu_c(const int* q) const { return c.mu[cell_idx<D>(g, q)]; }

    // Mean of mu over the existing cells touching the edge of component k that
    // lies at node position m along tangential axis t.
    EHH_DEV T mu_edge(int k, const int* p, int t, int m) const {
        int q[3] = {p[0], p[1], p[2]};
        T s = T(0);
        int cntc = 0;
#pragma unroll
        for (int dk = -1; dk <= 0; ++dk) {
#pragma unroll
            for (int dt = -1; dt <= 0; ++dt) {
                q[k] = p[k] + dk;
                q[t] = m + dt;
                if (q[t] >= 0 && q[t] < g.n[t]) {
                    s += mu_c(q);
                    ++cntc;
                }
            }
        }
        return s / T(cntc);
    }

    EHH_DEV cx<T> diag_u(int k, const int* p) const {
        int ql[3] = {p[0], p[1], p[2]};
        ql[k] -= 1;
        const int64_t il = cell_idx<D>(g, ql), ih = cell_idx<D>(g, p);
        T w = c.mu[il] + c.mu[ih];
        const int t1 = tang1<D>(k);
        w += mu_edge(k, p, t1, p[t1]) + mu_edge(k, p, t1, p[t1] + 1);
        if (D == 3) {
            const int t2 = tang2<D>(k);
            w += mu_edge(k, p, t2, p[t2]) + mu_edge(k, p, t2, p[t2] + 1);
        }
        const T rl = c.rho[il], rh = c.rho[ih];
        const T mre = T(0.5) * (rl + rh);
        const T mim = -T(0.5) * (rl * (c.gam[il] + c.alpha) + rh * (c.gam[ih] + c.alpha));
        return mk<T>(w - c.om2 * mre, -c.om2 * mim);
    }

    // (A e) at the face p of component k.
    EHH_DEV cx<T> row_u(int k, const int* p, const CVec<T>& e) const {
        cx<T> acc = diag_u(k, p) * e.ld(g.off[k] + face_idx<D>(g, k, p));
        int q[3] = {p[0], p[1], p[2]};
        // normal neighbours couple through the cells above/below the face
        if (p[k] + 1 <= g.n[k] - 1) {
            q[k] = p[k] + 1;
            acc = acc - mu_c(p) * e.ld(g.off[k] + face_idx<D>(g, k, q));
        }
        if (p[k] - 1 >= 1) {
            q[k] = p[k] - 1;
            int ql[3] = {p[0], p[1], p[2]};
            ql[k] -= 1;
            acc = acc - mu_c(ql) * e.ld(g.off[k] + face_idx<D>(g, k, q));
        }
        q[k] = p[k];
#pragma unroll
        for (int tt = 0; tt < D - 1; ++tt) {
            const int t = tt == 0 ? tang1<D>(k) : tang2<D>(k);
            if (p[t] + 1 < g.n[t]) {
                q[t] = p[t] + 1;
                acc = acc - mu_edge(k, p, t, p[t] + 1) * e.ld(g.off[k] + face_idx<D>(g, k, q));
            }
            if (p[t] - 1 >= 0) {
                q[t] = p[t] - 1;
                acc = acc - mu_edge(k, p, t, p[t]) * e.ld(g.off[k] + face_idx<D>(g, k, q));
            }
            q[t] = p[t];
        }
        int ql[3] = {p[0], p[1], p[2]};
        ql[k] -= 1;
        acc = acc + e.ld(g.off[3] + cell_idx<D>(g, p)) - e.ld(g.off[3] + cell_idx<D>(g, ql));
        return acc;
    }

    // (A e) at the pressure of cell cc.
    EHH_DEV cx<T> row_p(const int* cc, const CVec<T>& e) const {
        const int64_t ic = cell_idx<D>(g, cc);
        cx<T> acc = (-c.dinv[ic]) * e.ld(g.off[3] + ic);
        int q[3] = {cc[0], cc[1], cc[2]};
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (cc[k] + 1 <= g.n[k] - 1) {
                q[k] = cc[k] + 1;
                acc = acc - e.ld(g.off[k] + face_idx<D>(g, k, q));
            }
            if (cc[k] >= 1) {
                q[k] = cc[k];
                acc = acc + e.ld(g.off[k] + face_idx<D>(g, k, q));
            }
            q[k] = cc[k];
        }
        return acc;
    }

    // Block entries of the cell: u_k low/high diagonals, their coupling, the
    // couplings to the cell pressure and the pressure diagonal.
    EHH_DEV void block(const int* cc, int k, cx<T>& all, cx<T>& ahh, cx<T>& alh, T& glo, T& ghi,
                       bool lo_ok, bool hi_ok) const {
        int q[3] = {cc[0], cc[1], cc[2]};
        all = lo_ok ? diag_u(k, q) : mk<T>(T(1), T(0));
        q[k] = cc[k] + 1;
        ahh = hi_ok ? diag_u(k, q) : mk<T>(T(1), T(0));
        alh = (lo_ok && hi_ok) ? mk<T>(-mu_c(cc), T(0)) : mk<T>(T(0), T(0));
        glo = lo_ok ? T(1) : T(0);
        ghi = hi_ok ? T(-1) : T(0);
    }
    EHH_DEV T pdiag(const int* cc) const { return -c.dinv[cell_idx<D>(g, cc)]; }
};

template <int D, typename T> struct StOp {
    Geo g;
    StCoef<T> c;

    EHH_DEV cx<T> uu(int k, int64_t fidx, int s) const {
        const T* b = c.uu[k] + (int64_t)(2 * s) * g.cnt[k] + fidx;
        return mk<T>(b[0], b[g.cnt[k]]);
    }
    EHH_DEV T up(int k, int64_t fidx, int q) const { return c.up[k][(int64_t)q * g.cnt[k] + fidx]; }

    EHH_DEV cx<T> row_u(int k, const int* p, const CVec<T>& e) const {
        constexpr int CF = St<D>::CF;
        const int t1 = tang1<D>(k), t2 = tang2<D>(k);
        const int64_t fi = face_idx<D>(g, k, p);
        cx<T> acc = mk<T>(T(0), T(0));
        int q[3];
#pragma unroll
        for (int F = 0; F < St<D>::NF; ++F) {
            int dn, d1, d2;
            full_offset<D>(F, dn, d1, d2);
            q[0] = p[0];
            q[1] = p[1];
            q[2] = p[2];
            q[k] += dn;
            q[t1] += d1;
            if (D == 3) q[t2] += d2;
            if (!face_ok<D>(g, k, q)) continue;
            const int64_t qi = face_idx<D>(g, k, q);
            const cx<T> a = F >= CF ? uu(k, fi, F - CF) : uu(k, qi, CF - F);
            acc = acc + a * e.ld(g.off[k] + qi);
        }
#pragma unroll
        for (int qq = 0; qq < St<D>::NUP; ++qq) {
            int side, e1, e2;
            up_decode<D>(qq, side, e1, e2);
            q[0] = p[0];
            q[1] = p[1];
            q[2] = p[2];
            q[k] += side - 1;
            q[t1] += e1;
            if (D == 3) q[t2] += e2;
            if (!cell_ok<D>(g, q)) continue;
            acc = acc + up(k, fi, qq) * e.ld(g.off[3] + cell_idx<D>(g, q));
        }
        return acc;
    }

    EHH_DEV cx<T> row_p(const int* cc, const CVec<T>& e) const {
        const int64_t ic = cell_idx<D>(g, cc);
        cx<T> acc = c.pp[ic] * e.ld(g.off[3] + ic);
        int q[3];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int t1 = tang1<D>(k), t2 = tang2<D>(k);
#pragma unroll
            for (int qq = 0; qq < St<D>::NUP; ++qq) {
                int side, e1, e2;
                up_decode<D>(qq, side, e1, e2);
                q[0] = cc[0];
                q[1] = cc[1];
                q[2] = cc[2];
                q[k] += 1 - side;
                q[t1] -= e1;
                if (D == 3) q[t2] -= e2;
                if (!face_ok<D>(g, k, q)) continue;
                const int64_t qi = face_idx<D>(g, k, q);
                acc = acc + up(k, qi, qq) * e.ld(g.off[k] + qi);
            }
        }
        return acc;
    }

    EHH_DEV void block(const int* cc, int k, cx<T>& all, cx<T>& ahh, cx<T>& alh, T& glo, T& ghi,
                       bool lo_ok, bool hi_ok) const {
        int q[3] = {cc[0], cc[1], cc[2]};
        const int64_t il = lo_ok ? face_idx<D>(g, k, q) : 0;
        q[k] = cc[k] + 1;
        const int64_t ih = hi_ok ? face_idx<D>(g, k, q) : 0;
        all = lo_ok ? uu(k, il, 0) : mk<T>(T(1), T(0));
        ahh = hi_ok ? uu(k, ih, 0) : mk<T>(T(1), T(0));
        alh = (lo_ok && hi_ok) ? uu(k, il, 1) : mk<T>(T(0), T(0));
        glo = lo_ok ? up(k, il, up_index<D>(1, 0, 0)) : T(0);
        ghi = hi_ok ? up(k, ih, up_index<D>(0, 0, 0)) : T(0);
    }
    EHH_DEV T pdiag(const int* cc) const { return c.pp[cell_idx<D>(g, cc)]; }
};

}  // namespace ehh
