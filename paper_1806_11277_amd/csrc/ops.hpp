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

// Workgroup barrier that orders LDS accesses only.  __syncthreads() also waits
// for the workgroup's outstanding global stores (its fence covers all memory),
// which costs a memory round trip per barrier in loops that store results.
EHH_DEV void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// A matrix row as (index, coefficient) terms, built once per row and then
// applied to every right-hand side: terms beyond the row's support point at a
// valid index with a zero coefficient.
// Raw buffer access: a scalar resource descriptor (base, size in bytes) plus a
// 32-bit byte offset per lane, so that a kernel keeps one VGPR per address.
// Reads past the descriptor's size return zero.
typedef uint32_t ehh_u2 __attribute__((ext_vector_type(2)));
template <typename T> struct Buf;
template <> struct Buf<float> {
    __amdgpu_buffer_rsrc_t r;
    EHH_DEV Buf() {}
    EHH_DEV Buf(const void* p, uint32_t bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000)) {}
    EHH_DEV float ld(uint32_t off) const { return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0)); }
    // per-lane offset plus a wave-uniform one (kept in a scalar register)
    EHH_DEV float ld(uint32_t off, uint32_t soff) const {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
    }
    EHH_DEV void st(uint32_t off, float v) const {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 0);
    }
};
template <> struct Buf<double> {
    __amdgpu_buffer_rsrc_t r;
    EHH_DEV Buf() {}
    EHH_DEV Buf(const void* p, uint32_t bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000)) {}
    EHH_DEV double ld(uint32_t off) const {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    }
    EHH_DEV double ld(uint32_t off, uint32_t soff) const {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
    }
    EHH_DEV void st(uint32_t off, double v) const {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(ehh_u2, v), r, off, 0, 0);
    }
};

// FP16 storage (stored rows of the 3D Galerkin levels in the complex64 cycle when
// asked for): loads only, widened by the caller.
template <> struct Buf<_Float16> {
    __amdgpu_buffer_rsrc_t r;
    EHH_DEV Buf() {}
    EHH_DEV Buf(const void* p, uint32_t bytes)
        : r(__builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000)) {}
    EHH_DEV _Float16 ld(uint32_t off) const {
        return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, off, 0, 0));
    }
    EHH_DEV _Float16 ld(uint32_t off, uint32_t soff) const {
        return __builtin_bit_cast(_Float16, __builtin_amdgcn_raw_buffer_load_b16(r, off, soff, 0));
    }
};

template <typename T, int NT> struct Plan {
    int32_t ix[NT];
    T re[NT], im[NT];
    EHH_DEV void set(int j, int64_t i, T a, T b) {
        ix[j] = (int32_t)i;
        re[j] = a;
        im[j] = b;
    }
    EHH_DEV cx<T> dot(const CVec<T>& e) const {
        T ar = T(0), ai = T(0);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const cx<T> v = e.ld(ix[j]);
            ar += re[j] * v.re - im[j] * v.im;
            ai += re[j] * v.im + im[j] * v.re;
        }
        return mk<T>(ar, ai);
    }
};

template <int D, typename T> struct FineOp {
    Geo g;
    FineCoef<T> c;

    EHH_DEV T mu_c(const int* q) const { return c.mu[cell_idx<D>(g, q)]; }

    // Mean of mu over the existing cells touching the edge of component k that
    // lies at node position m along tangential axis t (rows m-1 and m along t;
    // a row beyond the wall is read clamped and left out of the mean).
    EHH_DEV T mu_edge(int k, const int* p, int t, int m) const {
        int q[3] = {p[0], p[1], p[2]};
        const bool lo = m - 1 >= 0, hi = m < g.n[t];
        T s = T(0);
#pragma unroll
        for (int dk = -1; dk <= 0; ++dk) {
            q[k] = p[k] + dk;
            q[t] = lo ? m - 1 : m;
            const T a = mu_c(q);
            q[t] = hi ? m : m - 1;
            const T b = mu_c(q);
            s += (lo ? a : T(0)) + (hi ? b : T(0));
        }
        return s / T(2 * ((int)lo + (int)hi));
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

    // (A e) at the face p of component k (branch-free: absent neighbours are read
    // at the face itself and weighted by zero).
    EHH_DEV cx<T> row_u(int k, const int* p, const CVec<T>& e) const {
        const int64_t self = g.off[k] + face_idx<D>(g, k, p);
        cx<T> acc = diag_u(k, p) * e.ld(self);
        int ql[3] = {p[0], p[1], p[2]};
        ql[k] -= 1;
        {
            int q[3] = {p[0], p[1], p[2]};
            const bool okh = p[k] + 1 <= g.n[k] - 1, okl = p[k] - 1 >= 1;
            q[k] = p[k] + 1;
            const int64_t ih = okh ? g.off[k] + face_idx<D>(g, k, q) : self;
            q[k] = p[k] - 1;
            const int64_t il = okl ? g.off[k] + face_idx<D>(g, k, q) : self;
            const T wh = okh ? mu_c(p) : T(0), wl = okl ? mu_c(ql) : T(0);
            acc = acc - wh * e.ld(ih) - wl * e.ld(il);
        }
#pragma unroll
        for (int tt = 0; tt < D - 1; ++tt) {
            const int t = tt == 0 ? tang1<D>(k) : tang2<D>(k);
            int q[3] = {p[0], p[1], p[2]};
            const bool okh = p[t] + 1 < g.n[t], okl = p[t] - 1 >= 0;
            q[t] = p[t] + 1;
            const int64_t ih = okh ? g.off[k] + face_idx<D>(g, k, q) : self;
            q[t] = p[t] - 1;
            const int64_t il = okl ? g.off[k] + face_idx<D>(g, k, q) : self;
            const T wh = okh ? mu_edge(k, p, t, p[t] + 1) : T(0);
            const T wl = okl ? mu_edge(k, p, t, p[t]) : T(0);
            acc = acc - wh * e.ld(ih) - wl * e.ld(il);
        }
        acc = acc + e.ld(g.off[3] + cell_idx<D>(g, p)) - e.ld(g.off[3] + cell_idx<D>(g, ql));
        return acc;
    }

    // (A e) at the pressure of cell cc.
    EHH_DEV cx<T> row_p(const int* cc, const CVec<T>& e) const {
        const int64_t ic = cell_idx<D>(g, cc);
        cx<T> acc = (-c.dinv[ic]) * e.ld(g.off[3] + ic);
#pragma unroll
        for (int k = 0; k < D; ++k) {
            int q[3] = {cc[0], cc[1], cc[2]};
            const bool okh = cc[k] + 1 <= g.n[k] - 1, okl = cc[k] >= 1;
            q[k] = cc[k] + 1;
            const int64_t ih = g.off[k] + (okh ? face_idx<D>(g, k, q) : 0);
            q[k] = cc[k];
            const int64_t il = g.off[k] + (okl ? face_idx<D>(g, k, q) : 0);
            const cx<T> vh = e.ld(ih), vl = e.ld(il);
            acc = acc - (okh ? T(1) : T(0)) * vh + (okl ? T(1) : T(0)) * vl;
        }
        return acc;
    }


    // Row plans: u row = self, normal high/low, tangential high/low per axis,
    // then the pressures of the cells above and below the face.
    static constexpr int NT = 2 * D + 3;
    static constexpr int T_SELF = 0, T_NHI = 1, T_PHI = NT - 2, T_PLO = NT - 1;
    EHH_DEV void plan_u(int k, const int* p, Plan<T, NT>& P) const {
        const int64_t self = g.off[k] + face_idx<D>(g, k, p);
        const cx<T> dg = diag_u(k, p);
        P.set(0, self, dg.re, dg.im);
        int ql[3] = {p[0], p[1], p[2]};
        ql[k] -= 1;
        {
            int q[3] = {p[0], p[1], p[2]};
            const bool okh = p[k] + 1 <= g.n[k] - 1, okl = p[k] - 1 >= 1;
            q[k] = p[k] + 1;
            P.set(1, okh ? g.off[k] + face_idx<D>(g, k, q) : self, okh ? -mu_c(p) : T(0), T(0));
            q[k] = p[k] - 1;
            P.set(2, okl ? g.off[k] + face_idx<D>(g, k, q) : self, okl ? -mu_c(ql) : T(0), T(0));
        }
#pragma unroll
        for (int tt = 0; tt < D - 1; ++tt) {
            const int t = tt == 0 ? tang1<D>(k) : tang2<D>(k);
            int q[3] = {p[0], p[1], p[2]};
            const bool okh = p[t] + 1 < g.n[t], okl = p[t] - 1 >= 0;
            q[t] = p[t] + 1;
            P.set(3 + 2 * tt, okh ? g.off[k] + face_idx<D>(g, k, q) : self, okh ? -mu_edge(k, p, t, p[t] + 1) : T(0), T(0));
            q[t] = p[t] - 1;
            P.set(4 + 2 * tt, okl ? g.off[k] + face_idx<D>(g, k, q) : self, okl ? -mu_edge(k, p, t, p[t]) : T(0), T(0));
        }
        P.set(T_PHI, g.off[3] + cell_idx<D>(g, p), T(1), T(0));
        P.set(T_PLO, g.off[3] + cell_idx<D>(g, ql), T(-1), T(0));
    }
    EHH_DEV void plan_p(const int* cc, Plan<T, NT>& P) const {
        const int64_t self = g.off[3] + cell_idx<D>(g, cc);
        P.set(0, self, -c.dinv[cell_idx<D>(g, cc)], T(0));
#pragma unroll
        for (int k = 0; k < D; ++k) {
            int q[3] = {cc[0], cc[1], cc[2]};
            const bool okh = cc[k] + 1 <= g.n[k] - 1, okl = cc[k] >= 1;
            q[k] = cc[k] + 1;
            P.set(1 + 2 * k, okh ? g.off[k] + face_idx<D>(g, k, q) : self, okh ? T(-1) : T(0), T(0));
            q[k] = cc[k];
            P.set(2 + 2 * k, okl ? g.off[k] + face_idx<D>(g, k, q) : self, okl ? T(1) : T(0), T(0));
        }
#pragma unroll
        for (int j = 2 * D + 1; j < NT; ++j) P.set(j, self, T(0), T(0));
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

    // Branch-free evaluation: absent neighbours are read at a clamped (valid)
    // address and weighted by zero, so every load of the row can be in flight
    // at once instead of one guarded load after another.
    EHH_DEV cx<T> row_u(int k, const int* p, const CVec<T>& e) const {
        constexpr int CF = St<D>::CF;
        const int t1 = tang1<D>(k), t2 = tang2<D>(k);
        const int64_t fi = face_idx<D>(g, k, p);
        T are = T(0), aim = T(0);
#pragma unroll
        for (int F = 0; F < St<D>::NF; ++F) {
            int dn, d1, d2;
            full_offset<D>(F, dn, d1, d2);
            int q[3] = {p[0], p[1], p[2]};
            q[k] += dn;
            q[t1] += d1;
            if (D == 3) q[t2] += d2;
            const bool ok = face_ok<D>(g, k, q);
            const int64_t qi = ok ? face_idx<D>(g, k, q) : fi;
            const cx<T> a = F >= CF ? uu(k, fi, F - CF) : uu(k, qi, CF - F);
            const cx<T> v = e.ld(g.off[k] + qi);
            const T sre = ok ? a.re : T(0), sim = ok ? a.im : T(0);
            are += sre * v.re - sim * v.im;
            aim += sre * v.im + sim * v.re;
        }
        const int64_t pc = g.off[3] + cell_idx<D>(g, p);
#pragma unroll
        for (int qq = 0; qq < St<D>::NUP; ++qq) {
            int side, e1, e2;
            up_decode<D>(qq, side, e1, e2);
            int q[3] = {p[0], p[1], p[2]};
            q[k] += side - 1;
            q[t1] += e1;
            if (D == 3) q[t2] += e2;
            const bool ok = cell_ok<D>(g, q);
            const int64_t ci = ok ? g.off[3] + cell_idx<D>(g, q) : pc;
            const T c = ok ? up(k, fi, qq) : T(0);
            const cx<T> v = e.ld(ci);
            are += c * v.re;
            aim += c * v.im;
        }
        return mk<T>(are, aim);
    }

    EHH_DEV cx<T> row_p(const int* cc, const CVec<T>& e) const {
        const int64_t ic = cell_idx<D>(g, cc);
        const cx<T> vp = e.ld(g.off[3] + ic);
        const T d = c.pp[ic];
        T are = d * vp.re, aim = d * vp.im;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int t1 = tang1<D>(k), t2 = tang2<D>(k);
#pragma unroll
            for (int qq = 0; qq < St<D>::NUP; ++qq) {
                int side, e1, e2;
                up_decode<D>(qq, side, e1, e2);
                int q[3] = {cc[0], cc[1], cc[2]};
                q[k] += 1 - side;
                q[t1] -= e1;
                if (D == 3) q[t2] -= e2;
                const bool ok = face_ok<D>(g, k, q);
                const int64_t qi = ok ? face_idx<D>(g, k, q) : 0;
                const T cf = ok ? up(k, qi, qq) : T(0);
                const cx<T> v = e.ld(g.off[k] + qi);
                are += cf * v.re;
                aim += cf * v.im;
            }
        }
        return mk<T>(are, aim);
    }


    // Rows for a block of RB right-hand sides: each coefficient is read once and
    // applied to all RB vectors (used where a whole row plan does not fit in
    // registers, i.e. the 3D Galerkin levels).
    template <int RB>
    EHH_DEV void row_u_rb(int k, const int* p, const CVec<T>* ev, cx<T>* out) const {
        constexpr int CF = St<D>::CF;
        const int t1 = tang1<D>(k), t2 = tang2<D>(k);
        const int64_t fi = face_idx<D>(g, k, p);
#pragma unroll
        for (int q = 0; q < RB; ++q) out[q] = mk<T>(T(0), T(0));
        for (int F = 0; F < St<D>::NF; ++F) {
            int dn, d1, d2;
            full_offset<D>(F, dn, d1, d2);
            int q3[3] = {p[0], p[1], p[2]};
            q3[k] += dn;
            q3[t1] += d1;
            if (D == 3) q3[t2] += d2;
            const bool ok = face_ok<D>(g, k, q3);
            const int64_t qi = ok ? face_idx<D>(g, k, q3) : fi;
            const cx<T> a0 = F >= CF ? uu(k, fi, F - CF) : uu(k, qi, CF - F);
            const cx<T> a = ok ? a0 : mk<T>(T(0), T(0));
            const int64_t ix = g.off[k] + qi;
#pragma unroll
            for (int q = 0; q < RB; ++q) out[q] = out[q] + a * ev[q].ld(ix);
        }
        const int64_t pc = g.off[3] + cell_idx<D>(g, p);
        for (int qq = 0; qq < St<D>::NUP; ++qq) {
            int side, e1, e2;
            up_decode<D>(qq, side, e1, e2);
            int q3[3] = {p[0], p[1], p[2]};
            q3[k] += side - 1;
            q3[t1] += e1;
            if (D == 3) q3[t2] += e2;
            const bool ok = cell_ok<D>(g, q3);
            const int64_t ci = ok ? g.off[3] + cell_idx<D>(g, q3) : pc;
            const T c0 = ok ? up(k, fi, qq) : T(0);
#pragma unroll
            for (int q = 0; q < RB; ++q) out[q] = out[q] + c0 * ev[q].ld(ci);
        }
    }
    template <int RB>
    EHH_DEV void row_p_rb(const int* cc, const CVec<T>* ev, cx<T>* out) const {
        const int64_t ic = cell_idx<D>(g, cc);
        const T d = c.pp[ic];
#pragma unroll
        for (int q = 0; q < RB; ++q) out[q] = d * ev[q].ld(g.off[3] + ic);
        for (int k = 0; k < D; ++k) {
            const int t1 = tang1<D>(k), t2 = tang2<D>(k);
            for (int qq = 0; qq < St<D>::NUP; ++qq) {
                int side, e1, e2;
                up_decode<D>(qq, side, e1, e2);
                int q3[3] = {cc[0], cc[1], cc[2]};
                q3[k] += 1 - side;
                q3[t1] -= e1;
                if (D == 3) q3[t2] -= e2;
                const bool ok = face_ok<D>(g, k, q3);
                const int64_t qi = ok ? face_idx<D>(g, k, q3) : 0;
                const T cf = ok ? up(k, qi, qq) : T(0);
#pragma unroll
                for (int q = 0; q < RB; ++q) out[q] = out[q] + cf * ev[q].ld(g.off[k] + qi);
            }
        }
    }

    // Row plans (used for D == 2, where a whole row fits in registers): u row =
    // the NF u-u offsets in full-offset order, then the NUP u-p entries; p row =
    // the pressure itself, then the u-p entries of the faces around the cell.
    static constexpr int NT = St<D>::NF + St<D>::NUP;
    static constexpr int T_SELF = St<D>::CF, T_NHI = St<D>::CF + 1;
    static constexpr int T_PHI = St<D>::NF + (D == 2 ? 1 + 2 : 1 + 2 * 4), T_PLO = St<D>::NF + (D == 2 ? 2 : 2 * 4);
    EHH_DEV void plan_u(int k, const int* p, Plan<T, NT>& P) const {
        constexpr int CF = St<D>::CF;
        const int t1 = tang1<D>(k), t2 = tang2<D>(k);
        const int64_t fi = face_idx<D>(g, k, p);
        const int64_t self = g.off[k] + fi;
#pragma unroll
        for (int F = 0; F < St<D>::NF; ++F) {
            int dn, d1, d2;
            full_offset<D>(F, dn, d1, d2);
            int q[3] = {p[0], p[1], p[2]};
            q[k] += dn;
            q[t1] += d1;
            if (D == 3) q[t2] += d2;
            const bool ok = face_ok<D>(g, k, q);
            const int64_t qi = ok ? face_idx<D>(g, k, q) : fi;
            const cx<T> a = F >= CF ? uu(k, fi, F - CF) : uu(k, qi, CF - F);
            P.set(F, g.off[k] + qi, ok ? a.re : T(0), ok ? a.im : T(0));
        }
        const int64_t pc = g.off[3] + cell_idx<D>(g, p);
#pragma unroll
        for (int qq = 0; qq < St<D>::NUP; ++qq) {
            int side, e1, e2;
            up_decode<D>(qq, side, e1, e2);
            int q[3] = {p[0], p[1], p[2]};
            q[k] += side - 1;
            q[t1] += e1;
            if (D == 3) q[t2] += e2;
            const bool ok = cell_ok<D>(g, q);
            P.set(St<D>::NF + qq, ok ? g.off[3] + cell_idx<D>(g, q) : pc, ok ? up(k, fi, qq) : T(0), T(0));
        }
    }
    EHH_DEV void plan_p(const int* cc, Plan<T, NT>& P) const {
        const int64_t ic = cell_idx<D>(g, cc);
        const int64_t self = g.off[3] + ic;
        P.set(0, self, c.pp[ic], T(0));
        int j = 1;
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int t1 = tang1<D>(k), t2 = tang2<D>(k);
#pragma unroll
            for (int qq = 0; qq < St<D>::NUP; ++qq) {
                int side, e1, e2;
                up_decode<D>(qq, side, e1, e2);
                int q[3] = {cc[0], cc[1], cc[2]};
                q[k] += 1 - side;
                q[t1] -= e1;
                if (D == 3) q[t2] -= e2;
                const bool ok = face_ok<D>(g, k, q);
                const int64_t qi = ok ? face_idx<D>(g, k, q) : 0;
                P.set(j++, ok ? g.off[k] + qi : self, ok ? up(k, qi, qq) : T(0), T(0));
            }
        }
#pragma unroll
        for (int jj = 1 + D * St<D>::NUP; jj < NT; ++jj) P.set(jj, self, T(0), T(0));
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
