// Multigrid level kernels: operator application / residual, damped red-black
// cell-wise Vanka half-sweep, restriction P^T and prolongation-correction.
//
// Every kernel loops over the right-hand sides inside the thread so that the
// operator coefficients (and the Vanka block factorisation) are read and
// formed once per cell for the whole batch.
#include <cstdlib>

#include "internal.hpp"
#include "launchlog.hpp"
#include "batch.hpp"
#include "ops.hpp"

namespace ehh {

// --------------------------------------------------------------- y = A x, r = b - A x
// One thread per unknown (row): short independent load chains, so that small
// coarse levels are not bound by the latency of one long serial row loop.
template <int D, typename T, class Op, int RB>
EHH_DEV void k_apply_body(VB ehh_vb, const Op& op, const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ y, int nrhs, int64_t stride, int rpb) {
    // right-hand sides [blockIdx.y * rpb, ...) of this grid row
    {
        const int rb0 = blockIdx.y * rpb;
        x += rb0 * stride;
        if (b) b += rb0 * stride;
        y += rb0 * stride;
        nrhs = nrhs - rb0 < rpb ? nrhs - rb0 : rpb;
    }
    const Geo& g = op.g;
    const int64_t t = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (t >= g.N) return;
    int k = 0;
    while (k < 3 && t >= g.off[k + 1]) ++k;
    const int64_t li = t - g.off[k];
    int p[3];
    if (k == 3) cell_pos<D>(g, li, p);
    else face_pos<D>(g, k, li, p);
    for (int r0 = 0; r0 < nrhs; r0 += RB) {
        CVec<T> xv[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) xv[q] = CVec<T>{x + (r0 + q < nrhs ? r0 + q : r0) * stride, g.N};
        cx<T> v[RB];
        if (k == 3) op.template row_p_rb<RB>(p, xv, v);
        else op.template row_u_rb<RB>(k, p, xv, v);
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = r0 + q;
            if (r >= nrhs) break;
            cx<T> o = v[q];
            if (b) o = CVec<T>{b + r * stride, g.N}.ld(t) - o;
            Vec<T>{y + r * stride, g.N}.st(t, o);
        }
    }
}
template <int D, typename T, class Op, int RB>
__global__ __launch_bounds__(256) void k_apply(Op op, const T* __restrict__ x, const T* __restrict__ b,
                                               T* __restrict__ y, int nrhs, int64_t stride, int rpb) {
    k_apply_body<D, T, Op, RB>(single_block<false>(), op, x, b, y, nrhs, stride, rpb);
}
template <class PK, int D, typename T, class Op, int RB>
__global__ __launch_bounds__(256) void k_apply_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_apply_body<D, T, Op, RB>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// ------------------------------------------------------------ red-black Vanka half-sweep
// Eight lanes of a wavefront per relaxed cell: lane j < 2D+1 evaluates row j of
// the cell block (row 2k / 2k+1 = low / high face of component k, row 2D = the
// pressure), the lane of row 0 gathers the residuals with wave shuffles, solves
// the block in closed form (one 2x2 complex system per displacement component,
// diagonal only in the economic variant, and the scalar Schur complement on the
// pressure) and hands each lane its correction; lane 2D+1 carries the pressure
// of the other cell of the pair over.  Cells of one colour share no unknown and
// every face belongs to exactly one of them, so e_out is written once per
// unknown; the residual is taken from e_in (the state at the start of the
// half-sweep).
template <int D, typename T, class Op, int RB>
EHH_DEV void k_relax_body(VB ehh_vb, const Op& op, int colour, T w, T wp, int econ, const T* __restrict__ b, const T* __restrict__ ein, T* __restrict__ eout, int nrhs, int64_t stride, int rpb) {
    {
        const int rb0 = blockIdx.y * rpb;
        b += rb0 * stride;
        if (ein) ein += rb0 * stride;
        eout += rb0 * stride;
        nrhs = nrhs - rb0 < rpb ? nrhs - rb0 : rpb;
    }
    constexpr int R = 2 * D + 1;
    const Geo& g = op.g;
    const int hp = g.n[0] >> 1;
    const int64_t npair = (int64_t)hp * g.n[1] * g.n[2];
    // lane = 8 * row + cell: the eight cells of a wavefront are consecutive, so a
    // load of one row term by the eight lanes of a row touches neighbouring cells
    const int lane = threadIdx.x & 63;
    const int row = lane >> 3;
    const int cig = lane & 7;
    const int64_t t = (((int64_t)ehh_vb.x * blockDim.x + threadIdx.x) >> 6) * 8 + cig;
    const int base = cig;   // lane of row 0 of this cell
    const bool live = t < npair;
    const int64_t tt = live ? t : 0;
    const int px = (int)(tt % hp);
    const int64_t rest = tt / hp;
    const int yy = (int)(rest % g.n[1]);
    const int zz = (int)(rest / g.n[1]);
    const int par = (colour + yy + zz) & 1;
    const int cr[3] = {2 * px + par, yy, zz};
    const int cb[3] = {2 * px + 1 - par, yy, zz};
    // the unknown of this lane's row
    const int k = row < 2 * D ? (row >> 1) : 3;
    int p[3] = {cr[0], cr[1], cr[2]};
    bool ok = live && row < R;
    if (k < 3) {
        p[k] += row & 1;
        ok = ok && p[k] >= 1 && p[k] <= g.n[k] - 1;
    }
    const int64_t idx = !ok ? 0 : (k == 3 ? g.off[3] + cell_idx<D>(g, p) : g.off[k] + face_idx<D>(g, k, p));
    const bool carry = live && row == R;
    const int64_t ipb = g.off[3] + cell_idx<D>(g, cb);

    // block factorisation (lane of row 0)
    cx<T> i00[D], i01[D], i11[D], zlo[D], zhi[D];
    T glo[D], ghi[D];
    cx<T> iS = mk<T>(T(0), T(0));
    if (row == 0 && live) {
        cx<T> S = mk<T>(op.pdiag(cr), T(0));
#pragma unroll
        for (int kk = 0; kk < D; ++kk) {
            const bool lok = cr[kk] >= 1, hok = cr[kk] + 1 <= g.n[kk] - 1;
            cx<T> all, ahh, alh;
            op.block(cr, kk, all, ahh, alh, glo[kk], ghi[kk], lok, hok);
            if (econ) alh = mk<T>(T(0), T(0));
            const cx<T> idet = cinv(all * ahh - alh * alh);
            i00[kk] = ahh * idet;
            i11[kk] = all * idet;
            i01[kk] = mk<T>(T(0), T(0)) - alh * idet;
            zlo[kk] = glo[kk] * i00[kk] + ghi[kk] * i01[kk];
            zhi[kk] = glo[kk] * i01[kk] + ghi[kk] * i11[kk];
            S = S - (glo[kk] * zlo[kk] + ghi[kk] * zhi[kk]);
        }
        iS = cinv(S);
    }

    for (int r0 = 0; r0 < nrhs; r0 += RB) {
    cx<T> resb[RB];
    {
        CVec<T> evb[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q)
            evb[q] = CVec<T>{ein ? ein + (r0 + q < nrhs ? r0 + q : r0) * stride : nullptr, g.N};
#pragma unroll
        for (int q = 0; q < RB; ++q) resb[q] = mk<T>(T(0), T(0));
        if (ok && ein) {
            if (k == 3) op.template row_p_rb<RB>(p, evb, resb);
            else op.template row_u_rb<RB>(k, p, evb, resb);
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = r0 + q < nrhs ? r0 + q : r0;
            resb[q] = ok ? CVec<T>{b + r * stride, g.N}.ld(idx) - resb[q] : mk<T>(T(0), T(0));
        }
    }
#pragma unroll
    for (int q = 0; q < RB; ++q) {
        const int r = r0 + q;
        if (r >= nrhs) break;
        const CVec<T> ev{ein ? ein + r * stride : nullptr, g.N};
        const Vec<T> ov{eout + r * stride, g.N};
        const cx<T> res = resb[q];
        // gather the block residual in the lane of row 0
        cx<T> rr[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            rr[j].re = __shfl(res.re, base + 8 * j, 64);
            rr[j].im = __shfl(res.im, base + 8 * j, 64);
        }
        cx<T> d[R];
        if (row == 0) {
            cx<T> acc = rr[2 * D];
            cx<T> ylo[D], yhi[D];
#pragma unroll
            for (int kk = 0; kk < D; ++kk) {
                ylo[kk] = i00[kk] * rr[2 * kk] + i01[kk] * rr[2 * kk + 1];
                yhi[kk] = i01[kk] * rr[2 * kk] + i11[kk] * rr[2 * kk + 1];
                acc = acc - (glo[kk] * ylo[kk] + ghi[kk] * yhi[kk]);
            }
            const cx<T> dp = acc * iS;
#pragma unroll
            for (int kk = 0; kk < D; ++kk) {
                d[2 * kk] = ylo[kk] - zlo[kk] * dp;
                d[2 * kk + 1] = yhi[kk] - zhi[kk] * dp;
            }
            d[2 * D] = dp;
        }
        // hand every lane its correction
        cx<T> mine = mk<T>(T(0), T(0));
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const T vr = __shfl(d[j].re, base, 64);
            const T vi = __shfl(d[j].im, base, 64);
            if (row == j) mine = mk<T>(vr, vi);
        }
        if (ok) ov.st(idx, (ein ? ev.ld(idx) : mk<T>(T(0), T(0))) + (row == 2 * D ? wp : w) * mine);
        if (carry) ov.st(ipb, ein ? ev.ld(ipb) : mk<T>(T(0), T(0)));
    }
    }
}
template <int D, typename T, class Op, int RB>
__global__ __launch_bounds__(256) void k_relax(Op op, int colour, T w, T wp, int econ,
                                               const T* __restrict__ b, const T* __restrict__ ein,
                                               T* __restrict__ eout, int nrhs, int64_t stride, int rpb) {
    k_relax_body<D, T, Op, RB>(single_block<false>(), op, colour, w, wp, econ, b, ein, eout, nrhs, stride, rpb);
}
template <class PK, int D, typename T, class Op, int RB>
__global__ __launch_bounds__(256) void k_relax_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_relax_body<D, T, Op, RB>(ehh_vb, a...); }, b.arg[ehh_s]);
}



// A per-lane offset past the end of every 2D stored-row buffer (their sizes stay
// below 2 GiB, and the term offsets, also below 2 GiB, go in a scalar register, so
// the sum cannot wrap): such a load returns zero and reads no memory.  The
// pressure rows use it for their imaginary parts and their unused terms, which
// are stored as zeros, so that a cache line holding only such slots is never
// fetched.
constexpr uint32_t OOB_OFF = 0x80000000u;


// ------------------------------------------------ plan-based apply and half-sweep
// The row plan (indices and coefficients) is built once per row and reused for
// every right-hand side, so a batch streams only the vectors.
template <int D, typename T, class Op, int RB>
EHH_DEV void k_apply_plan_body(VB ehh_vb, const Op& op, const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ y, int nrhs, int64_t stride, int rpb) {
    // right-hand sides [blockIdx.y * rpb, ...) of this grid row
    {
        const int rb0 = blockIdx.y * rpb;
        x += rb0 * stride;
        if (b) b += rb0 * stride;
        y += rb0 * stride;
        nrhs = nrhs - rb0 < rpb ? nrhs - rb0 : rpb;
    }
    const Geo& g = op.g;
    const int64_t t = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (t >= g.N) return;
    int k = 0;
    while (k < 3 && t >= g.off[k + 1]) ++k;
    const int64_t li = t - g.off[k];
    int p[3];
    Plan<T, Op::NT> P;
    if (k == 3) {
        cell_pos<D>(g, li, p);
        op.plan_p(p, P);
    } else {
        face_pos<D>(g, k, li, p);
        op.plan_u(k, p, P);
    }
    // blocks of RB right-hand sides keep RB independent load streams in flight
    int r = 0;
    for (; r + RB <= nrhs; r += RB) {
        cx<T> v[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) v[q] = P.dot(CVec<T>{x + (r + q) * stride, g.N});
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            if (b) v[q] = CVec<T>{b + (r + q) * stride, g.N}.ld(t) - v[q];
            Vec<T>{y + (r + q) * stride, g.N}.st(t, v[q]);
        }
    }
    for (; r < nrhs; ++r) {
        cx<T> v = P.dot(CVec<T>{x + r * stride, g.N});
        if (b) v = CVec<T>{b + r * stride, g.N}.ld(t) - v;
        Vec<T>{y + r * stride, g.N}.st(t, v);
    }
}
template <int D, typename T, class Op, int RB>
__global__ __launch_bounds__(256) void k_apply_plan(Op op, const T* __restrict__ x, const T* __restrict__ b,
                                                    T* __restrict__ y, int nrhs, int64_t stride, int rpb) {
    k_apply_plan_body<D, T, Op, RB>(single_block<false>(), op, x, b, y, nrhs, stride, rpb);
}
template <class PK, int D, typename T, class Op, int RB>
__global__ __launch_bounds__(256) void k_apply_plan_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_apply_plan_body<D, T, Op, RB>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// Vanka block of one cell spread over the eight lanes of its rows (lane base + 8 j
// holds row j: the low and high face of each component, then the pressure).
// factor() gathers the block entries from those lanes (diagonal dre + i dim, the
// coupling of a component's two faces cre + i cim given by the low row, zero in
// the economic variant, and the real coupling gg of each face to the cell
// pressure) and factorises the block in the lane of row 0: a 2 x 2 inverse per
// component and the scalar Schur complement of the pressure.  solve() turns the
// rows' residuals into this lane's correction.
template <int D, typename T> struct VankaBlock {
    static constexpr int R = 2 * D + 1;
    cx<T> i00[D], i01[D], i11[D], zlo[D], zhi[D];
    T glo[D], ghi[D];
    cx<T> iS;

    EHH_DEV void factor(T dre, T dim, T cre, T cim, T gg, int base, int row) {
        const T pd = __shfl(dre, base + 8 * (2 * D), 64);
        cx<T> S = mk<T>(pd, T(0));
#pragma unroll
        for (int kk = 0; kk < D; ++kk) {
            const cx<T> all = mk<T>(__shfl(dre, base + 8 * (2 * kk), 64), __shfl(dim, base + 8 * (2 * kk), 64));
            const cx<T> ahh = mk<T>(__shfl(dre, base + 8 * (2 * kk + 1), 64), __shfl(dim, base + 8 * (2 * kk + 1), 64));
            const cx<T> alh = mk<T>(__shfl(cre, base + 8 * (2 * kk), 64), __shfl(cim, base + 8 * (2 * kk), 64));
            glo[kk] = __shfl(gg, base + 8 * (2 * kk), 64);
            ghi[kk] = __shfl(gg, base + 8 * (2 * kk + 1), 64);
            if (row == 0) {
                const cx<T> idet = cinv(all * ahh - alh * alh);
                i00[kk] = ahh * idet;
                i11[kk] = all * idet;
                i01[kk] = mk<T>(T(0), T(0)) - alh * idet;
                zlo[kk] = glo[kk] * i00[kk] + ghi[kk] * i01[kk];
                zhi[kk] = glo[kk] * i01[kk] + ghi[kk] * i11[kk];
                S = S - (glo[kk] * zlo[kk] + ghi[kk] * zhi[kk]);
            }
        }
        iS = row == 0 ? cinv(S) : mk<T>(T(0), T(0));
    }

    EHH_DEV cx<T> solve(cx<T> res, int base, int row) const {
        cx<T> rr[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            rr[j].re = __shfl(res.re, base + 8 * j, 64);
            rr[j].im = __shfl(res.im, base + 8 * j, 64);
        }
        cx<T> d[R];
        if (row == 0) {
            cx<T> acc = rr[2 * D];
            cx<T> ylo[D], yhi[D];
#pragma unroll
            for (int kk = 0; kk < D; ++kk) {
                ylo[kk] = i00[kk] * rr[2 * kk] + i01[kk] * rr[2 * kk + 1];
                yhi[kk] = i01[kk] * rr[2 * kk] + i11[kk] * rr[2 * kk + 1];
                acc = acc - (glo[kk] * ylo[kk] + ghi[kk] * yhi[kk]);
            }
            const cx<T> dp = acc * iS;
#pragma unroll
            for (int kk = 0; kk < D; ++kk) {
                d[2 * kk] = ylo[kk] - zlo[kk] * dp;
                d[2 * kk + 1] = yhi[kk] - zhi[kk] * dp;
            }
            d[2 * D] = dp;
        }
        cx<T> mine = mk<T>(T(0), T(0));
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const T vr = __shfl(d[j].re, base, 64);
            const T vi = __shfl(d[j].im, base, 64);
            if (row == j) mine = mk<T>(vr, vi);
        }
        return mine;
    }
};

// Eight lanes per relaxed cell as in k_relax, each lane holding the plan of its
// block row, built in the kernel; the block itself (diagonals, the coupling of
// the two faces of a component, the couplings to the cell pressure) is read off
// the lanes' plans.
template <int D, typename T, class Op, int RB>
EHH_DEV void k_relax_plan_body(VB ehh_vb, const Op& op, int colour, T w, T wp, int econ, const T* __restrict__ b, const T* __restrict__ ein, T* __restrict__ eout, int nrhs, int64_t stride, int rpb) {
    {
        const int rb0 = blockIdx.y * rpb;
        b += rb0 * stride;
        if (ein) ein += rb0 * stride;
        eout += rb0 * stride;
        nrhs = nrhs - rb0 < rpb ? nrhs - rb0 : rpb;
    }
    constexpr int R = 2 * D + 1;
    const Geo& g = op.g;
    const int hp = g.n[0] >> 1;
    const int64_t npair = (int64_t)hp * g.n[1] * g.n[2];
    // lane = 8 * row + cell: the eight cells of a wavefront are consecutive, so a
    // load of one row term by the eight lanes of a row touches neighbouring cells
    const int lane = threadIdx.x & 63;
    const int row = lane >> 3;
    const int cig = lane & 7;
    const int64_t t = (((int64_t)ehh_vb.x * blockDim.x + threadIdx.x) >> 6) * 8 + cig;
    const int base = cig;   // lane of row 0 of this cell
    const bool live = t < npair;
    const int64_t tt = live ? t : 0;
    const int px = (int)(tt % hp);
    const int64_t rest = tt / hp;
    const int yy = (int)(rest % g.n[1]);
    const int zz = (int)(rest / g.n[1]);
    const int par = (colour + yy + zz) & 1;
    const int cr[3] = {2 * px + par, yy, zz};
    const int cb[3] = {2 * px + 1 - par, yy, zz};
    const int k = row < 2 * D ? (row >> 1) : 3;
    int p[3] = {cr[0], cr[1], cr[2]};
    bool ok = live && row < R;
    if (k < 3) {
        p[k] += row & 1;
        ok = ok && p[k] >= 1 && p[k] <= g.n[k] - 1;
    }
    Plan<T, Op::NT> P;
    int64_t idx = 0;
    if (ok) {
        if (k == 3) {
            op.plan_p(p, P);
            idx = g.off[3] + cell_idx<D>(g, p);
        } else {
            op.plan_u(k, p, P);
            idx = g.off[k] + face_idx<D>(g, k, p);
        }
    } else {
#pragma unroll
        for (int j = 0; j < Op::NT; ++j) P.set(j, 0, T(0), T(0));
    }
    const bool carry = live && row == R;
    const int64_t ipb = g.off[3] + cell_idx<D>(g, cb);
    // this row's block entries: the diagonal sits at T_SELF in a u row and at
    // term 0 in the pressure row
    const bool lowrow = row < 2 * D && (row & 1) == 0;
    VankaBlock<D, T> V;
    V.factor(ok ? (k == 3 ? P.re[0] : P.re[Op::T_SELF]) : T(1), ok ? (k == 3 ? P.im[0] : P.im[Op::T_SELF]) : T(0),
             (ok && lowrow && !econ) ? P.re[Op::T_NHI] : T(0), (ok && lowrow && !econ) ? P.im[Op::T_NHI] : T(0),
             (ok && row < 2 * D) ? (lowrow ? P.re[Op::T_PHI] : P.re[Op::T_PLO]) : T(0), base, row);

    for (int r0 = 0; r0 < nrhs; r0 += RB) {
        // residual rows of a block of right-hand sides (independent load streams)
        cx<T> resb[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            resb[q] = mk<T>(T(0), T(0));
            const int r = r0 + q;
            if (ok && r < nrhs) {
                resb[q] = CVec<T>{b + r * stride, g.N}.ld(idx);
                if (ein) resb[q] = resb[q] - P.dot(CVec<T>{ein + r * stride, g.N});
            }
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = r0 + q;
            if (r >= nrhs) break;
            const CVec<T> ev{ein ? ein + r * stride : nullptr, g.N};
            const Vec<T> ov{eout + r * stride, g.N};
            const cx<T> mine = V.solve(resb[q], base, row);
            if (ok) ov.st(idx, (ein ? ev.ld(idx) : mk<T>(T(0), T(0))) + (row == 2 * D ? wp : w) * mine);
            if (carry) ov.st(ipb, ein ? ev.ld(ipb) : mk<T>(T(0), T(0)));
        }
    }
}
template <int D, typename T, class Op, int RB>
__global__ __launch_bounds__(256) void k_relax_plan(Op op, int colour, T w, T wp, int econ,
                                                    const T* __restrict__ b, const T* __restrict__ ein,
                                                    T* __restrict__ eout, int nrhs, int64_t stride, int rpb) {
    k_relax_plan_body<D, T, Op, RB>(single_block<false>(), op, colour, w, wp, econ, b, ein, eout, nrhs, stride, rpb);
}
template <class PK, int D, typename T, class Op, int RB>
__global__ __launch_bounds__(256) void k_relax_plan_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_relax_plan_body<D, T, Op, RB>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// Staggered bilinear transfer weights along a tangential axis: 3/4 for the two
// fine rows nearer the coarse row, 1/4 for the next ones, zero beyond.
EHH_DEV float w_tang(int d) { return (d == 0 || d == 1) ? 0.75f : ((d == -1 || d == 2) ? 0.25f : 0.f); }

// (P^T r_f) at the coarse 2D unknown of component k (0, 1, or 3 for the
// pressure) at position (X, Y): twelve fine faces (weights 1 or 1/2 along the
// normal, 3/4 or 1/4 along the tangential axis) or the four fine cells; every
// load is issued before the sum, terms outside the grid read a clamped index
// with weight zero.  rf: one right-hand side's fine vector (real plane, then
// imaginary plane).
template <typename T>
EHH_DEV cx<T> restrict_at2d(const Geo& gf, const T* __restrict__ rf, int k, int X, int Y) {
    const int Nf = (int)gf.N, nfx = gf.n[0], nfy = gf.n[1];
    // 32-bit byte offsets into a buffer descriptor (the callers keep a vector
    // below 4 GiB), the imaginary plane through the scalar offset
    const Buf<T> rv(rf, 2u * (uint32_t)Nf * (uint32_t)sizeof(T));
    const uint32_t NB = (uint32_t)Nf * (uint32_t)sizeof(T);
    constexpr uint32_t E = (uint32_t)sizeof(T);
    T sr = T(0), si = T(0);
    if (k == 3) {
        const int b = (int)gf.off[3] + 2 * Y * nfx + 2 * X;
        const int ix[4] = {b, b + 1, b + nfx, b + nfx + 1};
        T vr[4], vi[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            vr[j] = rv.ld(E * (uint32_t)ix[j], 0);
            vi[j] = rv.ld(E * (uint32_t)ix[j], NB);
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            sr += vr[j];
            si += vi[j];
        }
        return mk<T>(sr, si);
    }
    const bool k0 = k == 0;
    // the weights are constants of (a, b1); only the tangential rows outside
    // the grid (b1 = -1 at the low wall, b1 = 2 at the high wall) drop out, so
    // the weights are applied as constants with a select on those two cases
    const int fn0 = 2 * (k0 ? X : Y), ft0 = 2 * (k0 ? Y : X), nt = k0 ? nfy : nfx;
    const bool lo_ok = ft0 - 1 >= 0, hi_ok = ft0 + 2 < nt;
    int ix[12];
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
        for (int b1 = -1; b1 <= 2; ++b1) {
            const int j = (a + 1) * 4 + b1 + 1;
            const int fn = fn0 + a, ft = ft0 + b1;
            const int fc = ft < 0 ? 0 : (ft >= nt ? nt - 1 : ft);
            ix[j] = k0 ? (int)gf.off[0] + fc * (nfx - 1) + fn - 1 : (int)gf.off[1] + (fn - 1) * nfx + fc;
        }
    T vr[12], vi[12];
#pragma unroll
    for (int j = 0; j < 12; ++j) {
        vr[j] = rv.ld(E * (uint32_t)ix[j], 0);
        vi[j] = rv.ld(E * (uint32_t)ix[j], NB);
    }
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
        for (int b1 = -1; b1 <= 2; ++b1) {
            const int j = (a + 1) * 4 + b1 + 1;
            const T wc = (a == 0 ? T(1) : T(0.5)) * T(w_tang(b1));
            const T wt = b1 == -1 ? (lo_ok ? wc : T(0)) : (b1 == 2 ? (hi_ok ? wc : T(0)) : wc);
            sr += wt * vr[j];
            si += wt * vi[j];
        }
    return mk<T>(sr, si);
}

// ------------------------------------ stored Galerkin rows with computed columns (2D)
// The 2D Galerkin levels keep their rows' coefficients, built once at setup, in
// the order the kernels read them: term j of lane (or row) i at [j * lanes + i],
// imaginary parts for the NF u-u terms only (the u-p and p-p couplings are
// real).  The column of a term is the row's own position plus the term's fixed
// stencil offset; a term that leaves the grid holds a zero coefficient and reads
// a clamped column.  So the vector loads depend on no loaded index and are in
// flight together with the coefficient loads.
struct Cols2 {
    int self;        // global index of the row
    int sn, st;      // u row: strides of its face grid along the normal / tangential axis
    int pc, cn, ct;  // u row: global index of the cell above the face, cell strides
    int f0, f1;      // p row: global index of the cell's low face in u_0 / u_1
    int nx, last;    // cells along x, N - 1
    bool isp;
};

EHH_DEV inline Cols2 cols2(const Geo& g, int k, const int* p) {
    Cols2 c;
    const int nx = g.n[0];
    c.nx = nx;
    c.last = (int)g.N - 1;
    c.isp = k == 3;
    const int ci = (int)g.off[3] + p[1] * nx + p[0];   // cell at p (for a face: the cell above it)
    c.pc = ci;
    c.f0 = (int)g.off[0] + p[1] * (nx - 1) + p[0] - 1;
    c.f1 = (int)g.off[1] + (p[1] - 1) * nx + p[0];
    if (k == 0) {
        c.self = c.f0;
        c.sn = 1;
        c.st = nx - 1;
        c.cn = 1;
        c.ct = nx;
    } else if (k == 1) {
        c.self = c.f1;
        c.sn = nx;
        c.st = 1;
        c.cn = nx;
        c.ct = 1;
    } else {
        c.self = ci;
        c.sn = c.st = c.cn = c.ct = 0;
    }
    return c;
}

// Column of term j (a compile-time constant after unrolling) of the row: u rows
// follow the order of StOp::plan_u (full u-u offsets, then the u-p entries), the
// pressure row that of StOp::plan_p (itself, then the u-p entries of u_0's and
// u_1's faces).
EHH_DEV inline int col2(const Cols2& c, int j) {
    constexpr int NF = St<2>::NF, NUP = St<2>::NUP;
    int iu;
    if (j < NF) {
        const int dn = j % 3 - 1, d1 = (j / 3) % 5 - 2;
        iu = c.self + dn * c.sn + d1 * c.st;
    } else {
        const int qq = j - NF, side = qq & 1, e1 = (qq >> 1) % 3 - 1;
        iu = c.pc + (side - 1) * c.cn + e1 * c.ct;
    }
    int ip = c.self;
    if (j >= 1 && j <= 2 * NUP) {
        const int kk = (j - 1) / NUP, qq = (j - 1) % NUP, side = qq & 1, e1 = (qq >> 1) % 3 - 1;
        ip = kk == 0 ? c.f0 + (1 - side) - e1 * (c.nx - 1) : c.f1 + (1 - side) * c.nx - e1;
    }
    const int i = c.isp ? ip : iu;
    return i < 0 ? 0 : (i > c.last ? c.last : i);
}

// Half-sweep over stored rows: the lane layout of k_relax_plan (eight lanes per
// cell, lane 8 j + cell holds row j), blocks renumbered per XCD.  KEEP holds a
// lane's coefficients in registers for the whole batch (FP32); otherwise (FP64)
// they are re-read per right-hand side in three parts of the row (measured on
// MI355X: three parts of 7 terms, 3 wavefronts per SIMD, beat two of 11 at 2 per
// SIMD on a 256^2 level, and one batch of all 21 terms at 1 per SIMD even on the
// 128^2 and 64^2 levels, where no SIMD holds more than one wavefront), and the
// block is re-factorised per right-hand side.
//
// RST (first half-sweep of a visit, from zero): the right-hand side is formed
// here as P^T of the finer level's residual rf (geometry gf) and written to bw,
// one unknown per lane (the carry lane forms the other cell's pressure), which
// saves the restriction's own launch.
template <typename T, bool KEEP, bool RST, typename C = T>
EHH_DEV void k_relax_st2d_body(VB ehh_vb, const Geo& g, int colour, T w, T wp, int econ, const T* __restrict__ b, const T* __restrict__ ein, T* __restrict__ eout, int nrhs, int64_t stride, int rpb, const C* __restrict__ cre, const C* __restrict__ cim, int64_t lanes, const Geo& gf, const T* __restrict__ rf, T* __restrict__ bw, T csc) {
    constexpr int D = 2, R = 2 * D + 1, NF = St<2>::NF, NUP = St<2>::NUP, NT = NF + NUP, H = 7;
    constexpr int T_SELF = St<2>::CF, T_NHI = St<2>::CF + 1, T_PLO = NF + 2, T_PHI = NF + 3;
    const int64_t sf = 2 * gf.N;
    {
        const int rb0 = blockIdx.y * rpb;
        b += rb0 * stride;
        if (ein) ein += rb0 * stride;
        eout += rb0 * stride;
        if (RST) {
            rf += rb0 * sf;
            bw += rb0 * stride;
        }
        nrhs = nrhs - rb0 < rpb ? nrhs - rb0 : rpb;
    }
    const int hp = g.n[0] >> 1;
    const int npair = hp * g.n[1];
    const int lane = threadIdx.x & 63;
    const int row = lane >> 3;
    const int cig = lane & 7;
    const int64_t gl = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    const int t = (int)(gl >> 6) * 8 + cig;
    const int base = cig;
    const bool live = t < npair;
    const int tt = live ? t : 0;
    const int px = tt % hp;
    const int yy = tt / hp;
    const int par = (colour + yy) & 1;
    const int k = row < 2 * D ? (row >> 1) : 3;
    int p[3] = {2 * px + par, yy, 0};
    bool ok = live && row < R;
    if (k < 3) {
        p[k] += row & 1;
        ok = ok && p[k] >= 1 && p[k] <= g.n[k] - 1;
    }
    const Cols2 cc = cols2(g, k, p);
    const int idx = cc.self;
    const bool carry = live && row == R;
    const int ipb = (int)g.off[3] + yy * g.n[0] + 2 * px + 1 - par;
    // coefficient loads: lane offset in a VGPR, term offset in a scalar register;
    // absent rows and the unused terms of the pressure row are stored as zeros.
    // C = FP16: the rows hold the coefficients divided by csc (a power of two).
    const Buf<C> cR(cre, (uint32_t)(NT * lanes * sizeof(C))), cI(cim, (uint32_t)(NF * lanes * sizeof(C)));
    const uint32_t lo = (uint32_t)gl * (uint32_t)sizeof(C), ls = (uint32_t)lanes * (uint32_t)sizeof(C);
    const uint32_t vb = 2 * (uint32_t)g.N * (uint32_t)sizeof(T), nb = (uint32_t)g.N * (uint32_t)sizeof(T);
    const auto cv = [csc](C v) -> T {
        if constexpr (std::is_same<C, T>::value) return v;
        else return csc * (T)v;
    };
    // this row's block entries: the diagonal sits at T_SELF in a u row and at
    // term 0 in the pressure row
    const bool lowrow = row < 2 * D && (row & 1) == 0;
    T dre = T(1), dim = T(0), ore = T(0), oim = T(0), gg = T(0);
    if (ok) {
        const uint32_t js = (uint32_t)(k == 3 ? 0 : T_SELF) * ls;
        dre = cv(cR.ld(lo + js));
        if (k < 3) {
            dim = cv(cI.ld(lo + js));
            gg = cv(cR.ld(lo + (uint32_t)(lowrow ? T_PHI : T_PLO) * ls));
            if (lowrow && !econ) {
                ore = cv(cR.ld(lo + (uint32_t)T_NHI * ls));
                oim = cv(cI.ld(lo + (uint32_t)T_NHI * ls));
            }
        }
    }
    // pressure rows (and the lanes past the rows) skip the slots stored as zeros
    const uint32_t lq = k == 3 ? OOB_OFF : lo;
    T are[KEEP ? NT : 1], aim[KEEP ? NF : 1];
    if (KEEP) {
        const uint32_t lr = row < R ? lo : OOB_OFF;
#pragma unroll
        for (int j = 0; j < (KEEP ? NT : 0); ++j) are[j] = cv(cR.ld(j > 2 * NUP ? lq : lr, j * ls));
#pragma unroll
        for (int j = 0; j < (KEEP ? NF : 0); ++j) aim[j] = cv(cI.ld(lq, j * ls));
    }

    VankaBlock<D, T> V;
    bool factored = false;
    for (int r = 0; r < nrhs; ++r) {
        const CVec<T> bv{b + r * stride, g.N};
        cx<T> res = mk<T>(T(0), T(0));
        cx<T> eown = mk<T>(T(0), T(0));
        // the other colour's pressure, loaded before the row's terms so that its
        // latency is not added after the block solve
        cx<T> ecarry = mk<T>(T(0), T(0));
        if (carry && ein) ecarry = CVec<T>{ein + r * stride, g.N}.ld(ipb);
        if (RST) {
            const Vec<T> bo{bw + r * stride, g.N};
            if (ok) {
                res = restrict_at2d<T>(gf, rf + r * sf, k, p[0], p[1]);
                bo.st(idx, res);
            }
            if (carry) bo.st(ipb, restrict_at2d<T>(gf, rf + r * sf, 3, 2 * px + 1 - par, yy));
        } else if (ok) {
            res = bv.ld(idx);
            if (ein) {
                // every term's load first (columns are clamped into the vector),
                // then the sums
                const Buf<T> ev(ein + r * stride, vb);
                T ar = T(0), ai = T(0);
                const uint32_t o = (uint32_t)idx * (uint32_t)sizeof(T);
                eown = mk<T>(ev.ld(o, 0), ev.ld(o, nb));
                if (KEEP) {
                    T vr[NT], vi[NT];
#pragma unroll
                    for (int j = 0; j < NT; ++j) {
                        const uint32_t oj = (uint32_t)col2(cc, j) * (uint32_t)sizeof(T);
                        vr[j] = ev.ld(oj, 0);
                        vi[j] = ev.ld(oj, nb);
                    }
                    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                    for (int j = 0; j < NT; ++j) {
                        ar = fma(are[KEEP ? j : 0], vr[j], ar);
                        ai = fma(are[KEEP ? j : 0], vi[j], ai);
                        if (j < NF) {
                            ar = fma(-aim[KEEP ? j : 0], vi[j], ar);
                            ai = fma(aim[KEEP ? j : 0], vr[j], ai);
                        }
                    }
                } else {
                    // The columns are recomputed per right-hand side, and the
                    // second half's addresses are made to depend on the first
                    // half's sums (empty asm statements), so that the halves'
                    // loads are not merged into one batch of registers.
                    Cols2 cl = cc;
                    uint32_t lh = lo, lhq = lq;
                    asm volatile("" : "+v"(cl.self), "+v"(cl.pc), "+v"(cl.f0), "+v"(cl.f1), "+v"(lh), "+v"(lhq),
                                 "+v"(cl.sn), "+v"(cl.st), "+v"(cl.cn), "+v"(cl.ct), "+v"(cl.nx));
#pragma unroll
                    for (int h = 0; h < NT; h += H) {
                        if (h > 0)
                            asm volatile("" : "+v"(cl.self), "+v"(cl.pc), "+v"(cl.f0), "+v"(cl.f1), "+v"(lh),
                                         "+v"(lhq)
                                         : "v"(ar), "v"(ai));
                        T cr_[H], ci_[H], vr[H], vi[H];
#pragma unroll
                        for (int jj = 0; jj < H; ++jj) {
                            const int j = h + jj;
                            if (j < NT) {
                                cr_[jj] = cv(cR.ld(j > 2 * NUP ? lhq : lh, j * ls));
                                ci_[jj] = j < NF ? cv(cI.ld(lhq, j * ls)) : T(0);
                                const uint32_t oj = (uint32_t)col2(cl, j) * (uint32_t)sizeof(T);
                                vr[jj] = ev.ld(oj, 0);
                                vi[jj] = ev.ld(oj, nb);
                            }
                        }
                        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                        for (int jj = 0; jj < H; ++jj) {
                            if (h + jj < NT) {
                                ar = fma(cr_[jj], vr[jj], ar);
                                ai = fma(cr_[jj], vi[jj], ai);
                                if (h + jj < NF) {
                                    ar = fma(-ci_[jj], vi[jj], ar);
                                    ai = fma(ci_[jj], vr[jj], ai);
                                }
                            }
                        }
                    }
                }
                res = res - mk<T>(ar, ai);
            }
        }
        if (!KEEP || !factored) {   // after the residual, so that its loads go first
            V.factor(dre, dim, ore, oim, gg, base, row);
            factored = true;
        }
        const cx<T> mine = V.solve(res, base, row);
        const Vec<T> ov{eout + r * stride, g.N};
        if (ok) ov.st(idx, eown + (row == 4 ? wp : w) * mine);
        if (carry) ov.st(ipb, ecarry);
    }
}
template <typename T, bool KEEP, bool RST, typename C = T>
__global__ __launch_bounds__(256) void k_relax_st2d(Geo g, int colour, T w, T wp, int econ, const T* __restrict__ b,
                                                    const T* __restrict__ ein, T* __restrict__ eout, int nrhs,
                                                    int64_t stride, int rpb, const C* __restrict__ cre,
                                                    const C* __restrict__ cim, int64_t lanes, Geo gf,
                                                    const T* __restrict__ rf, T* __restrict__ bw, T csc) {
    k_relax_st2d_body<T, KEEP, RST, C>(single_block<true>(), g, colour, w, wp, econ, b, ein, eout, nrhs, stride, rpb, cre, cim, lanes, gf, rf, bw, csc);
}
template <class PK, typename T, bool KEEP, bool RST, typename C = T>
__global__ __launch_bounds__(256) void k_relax_st2d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<true>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_relax_st2d_body<T, KEEP, RST, C>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// FP64 half-sweep over stored rows with each row split over two wavefronts: the
// lane layout and stored-row slots of k_relax_st2d (eight cells per wavefront,
// lane 8 j + cell), but a pair of wavefronts per group of eight cells, the odd
// one summing terms 11..20 of every row and handing its partial sums over in
// LDS, the even one terms 0..10, then the block solve.  Each row's loads then go
// out in one batch (the single-wavefront FP64 kernel needs three to stay within
// its registers), which pays on small levels where a launch is one wave of
// wavefronts deep.  Only for half-sweeps that start from e_in.
template <typename T>
EHH_DEV void k_relax_st2d_split_body(VB ehh_vb, const Geo& g, int colour, T w, T wp, int econ, const T* __restrict__ b, const T* __restrict__ ein, T* __restrict__ eout, int nrhs, int64_t stride, int rpb, const T* __restrict__ cre, const T* __restrict__ cim, int64_t lanes) {
    constexpr int D = 2, R = 2 * D + 1, NF = St<2>::NF, NUP = St<2>::NUP, NT = NF + NUP, HT = 11;
    constexpr int T_SELF = St<2>::CF, T_NHI = St<2>::CF + 1, T_PLO = NF + 2, T_PHI = NF + 3;
    __shared__ T part[2][2][2][64];   // [r parity][cell group of the block][re, im][lane]
    {
        const int rb0 = blockIdx.y * rpb;
        b += rb0 * stride;
        ein += rb0 * stride;
        eout += rb0 * stride;
        nrhs = nrhs - rb0 < rpb ? nrhs - rb0 : rpb;
    }
    const int hp = g.n[0] >> 1;
    const int npair = hp * g.n[1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int half = wv & 1, grp = wv >> 1;
    const int row = lane >> 3, cig = lane & 7;
    const int64_t group = (int64_t)ehh_vb.x * 2 + grp;   // cell group of eight cells
    const int64_t gl = group * 64 + lane;                                  // stored-row slot
    const int t = (int)group * 8 + cig;
    const int base = cig;
    const bool live = t < npair;
    const int tt = live ? t : 0;
    const int px = tt % hp;
    const int yy = tt / hp;
    const int par = (colour + yy) & 1;
    const int k = row < 2 * D ? (row >> 1) : 3;
    int p[3] = {2 * px + par, yy, 0};
    bool ok = live && row < R;
    if (k < 3) {
        p[k] += row & 1;
        ok = ok && p[k] >= 1 && p[k] <= g.n[k] - 1;
    }
    const Cols2 cc = cols2(g, k, p);
    const int idx = cc.self;
    const bool carry = live && row == R;
    const int ipb = (int)g.off[3] + yy * g.n[0] + 2 * px + 1 - par;
    const bool slot_ok = gl < lanes;
    const Buf<T> cR(cre, (uint32_t)(NT * lanes * sizeof(T))), cI(cim, (uint32_t)(NF * lanes * sizeof(T)));
    const uint32_t lo = (uint32_t)(slot_ok ? gl : 0) * (uint32_t)sizeof(T), ls = (uint32_t)lanes * (uint32_t)sizeof(T);
    const uint32_t lq = k == 3 ? OOB_OFF : lo;   // pressure rows: skip the slots stored as zeros
    const uint32_t vb = 2 * (uint32_t)g.N * (uint32_t)sizeof(T), nb = (uint32_t)g.N * (uint32_t)sizeof(T);
    const bool lowrow = row < 2 * D && (row & 1) == 0;
    VankaBlock<D, T> V;
    for (int r = 0; r < nrhs; ++r) {
        const Buf<T> ev(ein + r * stride, vb);
        T ar = T(0), ai = T(0);
        cx<T> res = mk<T>(T(0), T(0)), eown = mk<T>(T(0), T(0));
        if (half == 1) {
            if (row < R && slot_ok) {
                T cr_[NT - HT], ci_[NT - HT], vr[NT - HT], vi[NT - HT];
#pragma unroll
                for (int jj = 0; jj < NT - HT; ++jj) {
                    const int j = HT + jj;
                    cr_[jj] = cR.ld(j > 2 * NUP ? lq : lo, j * ls);
                    ci_[jj] = j < NF ? cI.ld(lq, j * ls) : T(0);
                    const uint32_t o = (uint32_t)col2(cc, j) * (uint32_t)sizeof(T);
                    vr[jj] = ev.ld(o, 0);
                    vi[jj] = ev.ld(o, nb);
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int jj = 0; jj < NT - HT; ++jj) {
                    ar = fma(cr_[jj], vr[jj], ar);
                    ai = fma(cr_[jj], vi[jj], ai);
                    if (HT + jj < NF) {
                        ar = fma(-ci_[jj], vi[jj], ar);
                        ai = fma(ci_[jj], vr[jj], ai);
                    }
                }
            }
            part[r & 1][grp][0][lane] = ar;
            part[r & 1][grp][1][lane] = ai;
        } else {
            T dre = T(1), dim = T(0), ore = T(0), oim = T(0), gg = T(0);
            cx<T> bo = mk<T>(T(0), T(0));
            cx<T> ecarry = mk<T>(T(0), T(0));
            if (carry) ecarry = CVec<T>{ein + r * stride, g.N}.ld(ipb);
            if (row < R && slot_ok) {
                T cr_[HT], ci_[HT], vr[HT], vi[HT];
#pragma unroll
                for (int jj = 0; jj < HT; ++jj) {
                    cr_[jj] = cR.ld(lo, jj * ls);
                    ci_[jj] = cI.ld(lq, jj * ls);
                    const uint32_t o = (uint32_t)col2(cc, jj) * (uint32_t)sizeof(T);
                    vr[jj] = ev.ld(o, 0);
                    vi[jj] = ev.ld(o, nb);
                }
                const uint32_t o = (uint32_t)idx * (uint32_t)sizeof(T);
                eown = mk<T>(ev.ld(o, 0), ev.ld(o, nb));
                if (ok) bo = CVec<T>{b + r * stride, g.N}.ld(idx);
                if (ok) {
                    const uint32_t js = (uint32_t)(k == 3 ? 0 : T_SELF) * ls;
                    dre = cR.ld(lo + js);
                    if (k < 3) {
                        dim = cI.ld(lo + js);
                        gg = cR.ld(lo + (uint32_t)(lowrow ? T_PHI : T_PLO) * ls);
                        if (lowrow && !econ) {
                            ore = cR.ld(lo + (uint32_t)T_NHI * ls);
                            oim = cI.ld(lo + (uint32_t)T_NHI * ls);
                        }
                    }
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int jj = 0; jj < HT; ++jj) {
                    ar = fma(cr_[jj], vr[jj], ar);
                    ai = fma(cr_[jj], vi[jj], ai);
                    if (jj < NF) {
                        ar = fma(-ci_[jj], vi[jj], ar);
                        ai = fma(ci_[jj], vr[jj], ai);
                    }
                }
            }
            V.factor(dre, dim, ore, oim, gg, base, row);
            lds_barrier();   // the odd wavefront's partial sums are in LDS
            if (ok) res = bo - mk<T>(ar + part[r & 1][grp][0][lane], ai + part[r & 1][grp][1][lane]);
            const cx<T> mine = V.solve(res, base, row);
            const Vec<T> ov{eout + r * stride, g.N};
            if (ok) ov.st(idx, eown + (row == 4 ? wp : w) * mine);
            if (carry) ov.st(ipb, ecarry);
            continue;
        }
        lds_barrier();
    }
}
template <typename T>
__global__ __launch_bounds__(256) void k_relax_st2d_split(Geo g, int colour, T w, T wp, int econ, const T* __restrict__ b,
                                                          const T* __restrict__ ein, T* __restrict__ eout, int nrhs,
                                                          int64_t stride, int rpb, const T* __restrict__ cre,
                                                          const T* __restrict__ cim, int64_t lanes) {
    k_relax_st2d_split_body<T>(single_block<true>(), g, colour, w, wp, econ, b, ein, eout, nrhs, stride, rpb, cre, cim, lanes);
}
template <class PK, typename T>
__global__ __launch_bounds__(256) void k_relax_st2d_split_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<true>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_relax_st2d_split_body<T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// y = A x or r = b - A x over stored rows (term j of row t at [j * N + t]).
// (C, csc: storage of the rows and their scale, as in k_relax_st2d.)
template <typename T, typename C = T>
EHH_DEV void k_apply_st2d_body(VB ehh_vb, const Geo& g, const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ y, int nrhs, int64_t stride, int rpb, const C* __restrict__ cre, const C* __restrict__ cim, T csc) {
    constexpr int NF = St<2>::NF, NUP = St<2>::NUP, NT = NF + NUP;
    {
        const int rb0 = blockIdx.y * rpb;
        x += rb0 * stride;
        if (b) b += rb0 * stride;
        y += rb0 * stride;
        nrhs = nrhs - rb0 < rpb ? nrhs - rb0 : rpb;
    }
    const int N = (int)g.N;
    const int t = (int)(int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    int k = 0;
    while (k < 3 && t >= g.off[k + 1]) ++k;
    const int li = t - (int)g.off[k];
    const int d0 = g.n[0] - (k == 0);
    int p[3] = {li % d0, li / d0, 0};
    if (k == 0) p[0] += 1;
    if (k == 1) p[1] += 1;
    const Cols2 cc = cols2(g, k, p);
    const Buf<C> cR(cre, (uint32_t)(NT * N * sizeof(C))), cI(cim, (uint32_t)(NF * N * sizeof(C)));
    const uint32_t lo = (uint32_t)t * (uint32_t)sizeof(C), cs = (uint32_t)N * (uint32_t)sizeof(C);
    const auto cv = [csc](C v) -> T {
        if constexpr (std::is_same<C, T>::value) return v;
        else return csc * (T)v;
    };
    // unused terms of the pressure rows are stored as zeros, and not read
    const uint32_t lq = k == 3 ? OOB_OFF : lo;
    T are[NT], aim[NF];
#pragma unroll
    for (int j = 0; j < NT; ++j) are[j] = cv(cR.ld(j > 2 * NUP ? lq : lo, j * cs));
#pragma unroll
    for (int j = 0; j < NF; ++j) aim[j] = cv(cI.ld(lq, j * cs));
    const uint32_t ls = (uint32_t)N * (uint32_t)sizeof(T), vb = 2 * ls;
    for (int r = 0; r < nrhs; ++r) {
        const Buf<T> xv(x + r * stride, vb);
        T vr[NT], vi[NT];
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const uint32_t o = (uint32_t)col2(cc, j) * (uint32_t)sizeof(T);
            vr[j] = xv.ld(o, 0);
            vi[j] = xv.ld(o, ls);
        }
        __builtin_amdgcn_sched_barrier(0);
        T ar = T(0), ai = T(0);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            ar = fma(are[j], vr[j], ar);
            ai = fma(are[j], vi[j], ai);
            if (j < NF) {
                ar = fma(-aim[j], vi[j], ar);
                ai = fma(aim[j], vr[j], ai);
            }
        }
        cx<T> o = mk<T>(ar, ai);
        if (b) o = CVec<T>{b + r * stride, g.N}.ld(t) - o;
        Vec<T>{y + r * stride, g.N}.st(t, o);
    }
}
template <typename T, typename C = T>
__global__ __launch_bounds__(256) void k_apply_st2d(Geo g, const T* __restrict__ x, const T* __restrict__ b,
                                                    T* __restrict__ y, int nrhs, int64_t stride, int rpb,
                                                    const C* __restrict__ cre, const C* __restrict__ cim, T csc) {
    k_apply_st2d_body<T, C>(single_block<true>(), g, x, b, y, nrhs, stride, rpb, cre, cim, csc);
}
template <class PK, typename T, typename C = T>
__global__ __launch_bounds__(256) void k_apply_st2d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<true>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_apply_st2d_body<T, C>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// rc = P^T (b - A e) from a 2D level with stored rows in one launch: sixteen
// lanes per coarse unknown, lane j forming the fine residual of the j-th fine
// unknown the coarse one gathers (twelve faces of the restriction's stencil,
// the weights of restrict_at2d, or the four cells of a pressure) from the
// stored rows as k_apply_st2d does, scaled by its weight; the sixteen products
// are summed by a butterfly over the lanes.  A fine residual shared by
// neighbouring coarse unknowns is formed once for each (the level is small
// and in the caches), which saves writing the fine residual and the
// restriction's own launch.
template <typename T>
EHH_DEV void k_residual_restrict2d_body(VB ehh_vb, const Geo& gf, const Geo& gc, const T* __restrict__ e, const T* __restrict__ b, T* __restrict__ rc, int nrhs, const T* __restrict__ cre, const T* __restrict__ cim) {
    constexpr int NF = St<2>::NF, NUP = St<2>::NUP, NT = NF + NUP;
    const int gl = (int)(ehh_vb.x * blockDim.x + threadIdx.x);
    const int Nc = (int)gc.N, N = (int)gf.N;
    const int tc0 = gl >> 4, j = gl & 15;
    const bool live = tc0 < Nc;
    const int tc = live ? tc0 : 0;
    const int ncx = gc.n[0], nfx = gf.n[0], nfy = gf.n[1];
    int k, X, Y;
    if (tc >= (int)gc.off[3]) {
        const int li = tc - (int)gc.off[3];
        k = 3;
        X = li % ncx;
        Y = li / ncx;
    } else if (tc < (int)gc.off[1]) {
        const int li = tc - (int)gc.off[0];
        k = 0;
        X = li % (ncx - 1) + 1;
        Y = li / (ncx - 1);
    } else {
        const int li = tc - (int)gc.off[1];
        k = 1;
        X = li % ncx;
        Y = li / ncx + 1;
    }
    // this lane's fine unknown (row position p, index ix) and weight
    int p[3] = {0, 0, 0};
    int ix = 0;
    T wt = T(0);
    if (k == 3) {
        p[0] = 2 * X + (j & 1);
        p[1] = 2 * Y + ((j >> 1) & 1);
        ix = (int)gf.off[3] + p[1] * nfx + p[0];
        wt = j < 4 ? T(1) : T(0);
    } else {
        const bool k0 = k == 0;
        const int a = (j >> 2) - 1, b1 = (j & 3) - 1;
        const int fn = 2 * (k0 ? X : Y) + a, ft = 2 * (k0 ? Y : X) + b1, nt = k0 ? nfy : nfx;
        const bool ok = j < 12 && ft >= 0 && ft < nt;
        const int fc = ft < 0 ? 0 : (ft >= nt ? nt - 1 : ft);
        // (lanes 12..15, a = 2, carry no weight; their face is clamped into the grid)
        const int nn = k0 ? nfx : nfy;
        const int fnc = fn < 1 ? 1 : (fn > nn - 1 ? nn - 1 : fn);
        p[0] = k0 ? fnc : fc;
        p[1] = k0 ? fc : fnc;
        ix = k0 ? (int)gf.off[0] + fc * (nfx - 1) + fnc - 1 : (int)gf.off[1] + (fnc - 1) * nfx + fc;
        wt = ok ? (a == 0 ? T(1) : T(0.5)) * T(w_tang(b1)) : T(0);
    }
    const bool act = live && wt != T(0);
    if (!act) ix = 0;
    const Cols2 cc = cols2(gf, k, p);
    const Buf<T> cR(cre, (uint32_t)(NT * N * sizeof(T))), cI(cim, (uint32_t)(NF * N * sizeof(T)));
    const uint32_t lo = (uint32_t)ix * (uint32_t)sizeof(T), ls = (uint32_t)N * (uint32_t)sizeof(T);
    // pressure rows: unused terms and imaginary parts are stored as zeros, and
    // inactive lanes read nothing
    const uint32_t lr = act ? lo : OOB_OFF, lq = (act && k != 3) ? lo : OOB_OFF;
    T are[NT], aim[NF];
#pragma unroll
    for (int jj = 0; jj < NT; ++jj) are[jj] = cR.ld(jj > 2 * NUP ? lq : lr, jj * ls);
#pragma unroll
    for (int jj = 0; jj < NF; ++jj) aim[jj] = cI.ld(lq, jj * ls);
    const uint32_t vb = 2 * ls;
    for (int r = 0; r < nrhs; ++r) {
        const Buf<T> xv(e + (int64_t)r * 2 * N, vb);
        T vr[NT], vi[NT];
#pragma unroll
        for (int jj = 0; jj < NT; ++jj) {
            const uint32_t o = (uint32_t)col2(cc, jj) * (uint32_t)sizeof(T);
            vr[jj] = xv.ld(o, 0);
            vi[jj] = xv.ld(o, ls);
        }
        const Buf<T> bv(b + (int64_t)r * 2 * N, vb);
        const T br = bv.ld(lo, 0), bi = bv.ld(lo, ls);
        __builtin_amdgcn_sched_barrier(0);
        T ar = T(0), ai = T(0);
#pragma unroll
        for (int jj = 0; jj < NT; ++jj) {
            ar = fma(are[jj], vr[jj], ar);
            ai = fma(are[jj], vi[jj], ai);
            if (jj < NF) {
                ar = fma(-aim[jj], vi[jj], ar);
                ai = fma(aim[jj], vr[jj], ai);
            }
        }
        T sr = act ? wt * (br - ar) : T(0), si = act ? wt * (bi - ai) : T(0);
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
            sr += __shfl_xor(sr, o, 16);
            si += __shfl_xor(si, o, 16);
        }
        if (live && j == 0) {
            rc[(int64_t)r * 2 * Nc + tc] = sr;
            rc[(int64_t)r * 2 * Nc + Nc + tc] = si;
        }
    }
}
template <typename T>
__global__ __launch_bounds__(256) void k_residual_restrict2d(Geo gf, Geo gc, const T* __restrict__ e,
                                                             const T* __restrict__ b, T* __restrict__ rc,
                                                             int nrhs, const T* __restrict__ cre,
                                                             const T* __restrict__ cim) {
    k_residual_restrict2d_body<T>(single_block<false>(), gf, gc, e, b, rc, nrhs, cre, cim);
}
template <class PK, typename T>
__global__ __launch_bounds__(256) void k_residual_restrict2d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_residual_restrict2d_body<T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// ------------------------------------ stored Galerkin rows with computed columns (3D)
// As in 2D: a 3D Galerkin level keeps its rows' coefficients in the order the
// kernels read them (93 real parts, 75 u-u imaginary parts per row), and a term's
// column is the row's own position plus the term's stencil offset.  The rows are
// long (75 u-u and 18 u-p terms), so a lane reads each coefficient once per block
// of RB right-hand sides and applies it to all of them, walking the row in
// chunks of terms.
struct Cols3 {
    int self;            // global index of the row
    int sn, s1, s2;      // u row: face-grid strides of its component along normal, t1, t2
    int pc, cn, c1, c2;  // u row: index of the cell above the face, cell strides along normal, t1, t2
    int f[3];            // p row: index of the cell's low face in u_0, u_1, u_2
    int fs[3][3];        // face-grid strides of component k along axis a
    int last;
    bool isp;
};

EHH_DEV inline Cols3 cols3(const Geo& g, int k, const int* p) {
    Cols3 c;
    const int n0 = g.n[0], n1 = g.n[1];
    c.last = (int)g.N - 1;
    c.isp = k == 3;
    const int cs[3] = {1, n0, n0 * n1};
#pragma unroll
    for (int kk = 0; kk < 3; ++kk) {
        const int d0 = n0 - (kk == 0), d1 = n1 - (kk == 1);
        c.fs[kk][0] = 1;
        c.fs[kk][1] = d0;
        c.fs[kk][2] = d0 * d1;
        const int q0 = p[0] - (kk == 0), q1 = p[1] - (kk == 1), q2 = p[2] - (kk == 2);
        c.f[kk] = (int)g.off[kk] + (q2 * d1 + q1) * d0 + q0;
    }
    c.pc = (int)g.off[3] + (p[2] * n1 + p[1]) * n0 + p[0];
    // the lane's component selects its strides (selects, not indexing, so that
    // nothing lands in scratch): normal k, tangential t1 = (k == 0 ? 1 : 0),
    // t2 = (k == 2 ? 1 : 2)
    const int d00 = n0 - 1, d10 = n0, d11 = n1 - 1, d20 = n0;
    c.self = k == 0 ? c.f[0] : (k == 1 ? c.f[1] : (k == 2 ? c.f[2] : c.pc));
    c.sn = k == 0 ? 1 : (k == 1 ? d10 : d20 * n1);
    c.s1 = k == 0 ? d00 : 1;
    c.s2 = k == 0 ? d00 * n1 : (k == 1 ? d10 * d11 : d20);
    c.cn = k == 0 ? cs[0] : (k == 1 ? cs[1] : cs[2]);
    c.c1 = k == 0 ? cs[1] : cs[0];
    c.c2 = k == 2 ? cs[1] : cs[2];
    return c;
}

// Column of term j (compile-time after unrolling): u rows in the order of
// StOp::plan_u, the pressure row in that of StOp::plan_p.
EHH_DEV inline int col3(const Cols3& c, int j) {
    constexpr int NF = St<3>::NF, NUP = St<3>::NUP;
    int iu;
    if (j < NF) {
        int dn, d1, d2;
        full_offset<3>(j, dn, d1, d2);
        iu = c.self + dn * c.sn + d1 * c.s1 + d2 * c.s2;
    } else {
        int side, e1, e2;
        up_decode<3>(j - NF, side, e1, e2);
        iu = c.pc + (side - 1) * c.cn + e1 * c.c1 + e2 * c.c2;
    }
    int ip = c.self;
    if (j >= 1 && j <= 3 * NUP) {
        const int kk = (j - 1) / NUP;
        int side, e1, e2;
        up_decode<3>((j - 1) % NUP, side, e1, e2);
        const int t1 = kk == 0 ? 1 : 0, t2 = kk == 2 ? 1 : 2;
        ip = c.f[kk] + (1 - side) * c.fs[kk][kk] - e1 * c.fs[kk][t1] - e2 * c.fs[kk][t2];
    }
    const int i = c.isp ? ip : iu;
    return i < 0 ? 0 : (i > c.last ? c.last : i);
}

// Residual terms of a row for a block of RB right-hand sides: coefficient j read
// once (lane offset lo, term stride ls, both in bytes) and applied to every
// vector; terms in chunks of CH, each chunk's loads issued before its sums and
// the next chunk's addresses tied to them (empty asm), so that the registers
// hold one chunk at a time.  nt (wave-uniform) ends the walk after the chunk
// holding term nt - 1: a wavefront of pressure rows only passes 1 + 3 NUP, its
// row's last nonzero term plus one (the pressure row is stored as zeros beyond).
template <typename T, int RB, int CH, typename C = T>
EHH_DEV void rows3_rb(const Buf<C>& cR, const Buf<C>& cI, uint32_t lo, uint32_t ls, const Cols3& cc,
                      const T* const* ev, uint32_t vb, uint32_t nb, T* ar, T* ai, int nt) {
    constexpr int NF = St<3>::NF, NT = NF + St<3>::NUP;
#pragma unroll
    for (int q = 0; q < RB; ++q) ar[q] = ai[q] = T(0);
    Cols3 cl = cc;
    uint32_t lh = lo;
    Buf<T> eb[RB] = {};
#pragma unroll
    for (int q = 0; q < RB; ++q) eb[q] = Buf<T>(ev[q], vb);
#pragma unroll
    for (int h = 0; h < NT; h += CH) {
        const bool walk = h < nt;
#pragma unroll
        for (int q = 0; q < RB; ++q) asm volatile("" ::"v"(ar[q]), "v"(ai[q]));
        asm volatile("" : "+v"(cl.self), "+v"(cl.pc), "+v"(cl.f[0]), "+v"(cl.f[1]), "+v"(cl.f[2]), "+v"(lh));
        // the strides too, so that no column offset is formed ahead of its chunk
        asm volatile("" : "+v"(cl.sn), "+v"(cl.s1), "+v"(cl.s2), "+v"(cl.cn), "+v"(cl.c1), "+v"(cl.c2));
        asm volatile("" : "+v"(cl.fs[0][1]), "+v"(cl.fs[0][2]), "+v"(cl.fs[1][1]), "+v"(cl.fs[1][2]),
                     "+v"(cl.fs[2][1]), "+v"(cl.fs[2][2]), "+v"(cl.last));
        T cr[CH], ci[CH], vr[CH][RB], vi[CH][RB];
#pragma unroll
        for (int jj = 0; jj < CH; ++jj) {
            const int j = h + jj;
            if (j < NT && walk) {
                cr[jj] = (T)cR.ld(lh, j * ls);
                ci[jj] = j < NF ? (T)cI.ld(lh, j * ls) : T(0);
                const uint32_t o = (uint32_t)col3(cl, j) * (uint32_t)sizeof(T);
#pragma unroll
                for (int q = 0; q < RB; ++q) {
                    vr[jj][q] = eb[q].ld(o, 0);
                    vi[jj][q] = eb[q].ld(o, nb);
                }
            }
        }
#pragma unroll
        for (int jj = 0; jj < CH; ++jj) {
            if (h + jj < NT && walk) {
#pragma unroll
                for (int q = 0; q < RB; ++q) {
                    ar[q] = fma(cr[jj], vr[jj][q], ar[q]);
                    ar[q] = fma(-ci[jj], vi[jj][q], ar[q]);
                    ai[q] = fma(cr[jj], vi[jj][q], ai[q]);
                    ai[q] = fma(ci[jj], vr[jj][q], ai[q]);
                }
            }
        }
    }
}

// Half-sweep over stored rows on a 3D Galerkin level.  A workgroup of 256 lanes
// relaxes 32 cells of the colour; lanes 32 j .. 32 j + 31 hold block row j of
// those cells (the low and high face of u_0, u_1, u_2, then the pressure; row 7
// carries the other cell's pressure), so one wavefront holds the two faces of
// one component for 32 neighbouring cells and a term's loads hit interleaved
// faces of the same cache lines (with one cell's eight rows in a wavefront,
// they spread over eight index families).  The Vanka blocks go through LDS:
// every lane factorises its cell's block from the rows' entries, then for each
// group of RB sources the rows' residuals are exchanged, lane (j, c) solves
// source j of the group for cell c, and each row lane applies its correction.
//
// C: storage type of the rows (T, or FP16 holding the coefficients divided by
// the level's power-of-two scale csc, which the sums and the block entries are
// multiplied by again; csc = 1 otherwise).
template <typename T, int RB, int CH, typename C = T>
EHH_DEV void k_relax_st3d_body(VB ehh_vb, const Geo& g, int colour, T w, T wp, int econ, const T* __restrict__ b, const T* __restrict__ ein, T* __restrict__ eout, int nrhs, int64_t stride, int rpb, const C* __restrict__ cre, const C* __restrict__ cim, int64_t lanes, T csc) {
    constexpr int D = 3, R = 2 * D + 1, NF = St<3>::NF, NT = NF + St<3>::NUP, CW = 32;
    constexpr int T_SELF = St<3>::CF, T_NHI = St<3>::CF + 1, T_PLO = NF + 8, T_PHI = NF + 9;
    static_assert(RB <= 8, "one source of a group per block row");
    __shared__ T ent[5][R][CW];          // block entries of the rows: dre, dim, ore, oim, gg
    __shared__ T rs[RB][R][CW][2];       // the rows' residuals, then the corrections
    {
        const int rb0 = blockIdx.y * rpb;
        b += rb0 * stride;
        if (ein) ein += rb0 * stride;
        eout += rb0 * stride;
        nrhs = nrhs - rb0 < rpb ? nrhs - rb0 : rpb;
    }
    const int hp = g.n[0] >> 1;
    const int npair = hp * g.n[1] * g.n[2];
    const int row = (int)(threadIdx.x >> 5) & 7;
    const int c = (int)threadIdx.x & (CW - 1);
    const int64_t gl = (int64_t)ehh_vb.x * 256 + threadIdx.x;
    const int t = (int)ehh_vb.x * CW + c;
    const bool live = t < npair;
    const int tt = live ? t : 0;
    const int px = tt % hp;
    const int rest = tt / hp;
    const int yy = rest % g.n[1], zz = rest / g.n[1];
    const int par = (colour + yy + zz) & 1;
    const int k = row < 2 * D ? (row >> 1) : 3;
    int p[3] = {2 * px + par, yy, zz};
    bool ok = live && row < R;
    if (k < 3) {
        p[k] += row & 1;
        ok = ok && p[k] >= 1 && p[k] <= g.n[k] - 1;
    }
    const Cols3 cc = cols3(g, k, p);
    const int idx = cc.self;
    const bool carry = live && row == R;
    const int ipb = (int)g.off[3] + (zz * g.n[1] + yy) * g.n[0] + 2 * px + 1 - par;
    const Buf<C> cR(cre, (uint32_t)(NT * lanes * sizeof(C))), cI(cim, (uint32_t)(NF * lanes * sizeof(C)));
    const uint32_t lo = (uint32_t)gl * (uint32_t)sizeof(C), ls = (uint32_t)lanes * (uint32_t)sizeof(C);
    const uint32_t vb = 2 * (uint32_t)g.N * (uint32_t)sizeof(T), nb = (uint32_t)g.N * (uint32_t)sizeof(T);
    // this row's block entries (the diagonal sits at T_SELF in a u row, at term 0
    // in the pressure row); rows outside the grid keep an identity entry
    {
        const bool lowrow = row < 2 * D && (row & 1) == 0;
        T dre = T(1), dim = T(0), ore = T(0), oim = T(0), gg = T(0);
        if (ok) {
            const uint32_t js = (uint32_t)(k == 3 ? 0 : T_SELF) * ls;
            dre = csc * (T)cR.ld(lo + js);
            if (k < 3) {
                dim = csc * (T)cI.ld(lo + js);
                gg = csc * (T)cR.ld(lo + (uint32_t)(lowrow ? T_PHI : T_PLO) * ls);
                if (lowrow && !econ) {
                    ore = csc * (T)cR.ld(lo + (uint32_t)T_NHI * ls);
                    oim = csc * (T)cI.ld(lo + (uint32_t)T_NHI * ls);
                }
            }
        }
        if (row < R) {
            ent[0][row][c] = dre;
            ent[1][row][c] = dim;
            ent[2][row][c] = ore;
            ent[3][row][c] = oim;
            ent[4][row][c] = gg;
        }
    }
    __syncthreads();
    // cell c's block, factorised in every lane: a 2 x 2 inverse per component and
    // the Schur complement of the pressure
    cx<T> i00[D], i01[D], i11[D], zlo[D], zhi[D];
    T glo[D], ghi[D];
    cx<T> iS;
    {
        cx<T> S = mk<T>(ent[0][2 * D][c], T(0));
#pragma unroll
        for (int kk = 0; kk < D; ++kk) {
            const cx<T> all = mk<T>(ent[0][2 * kk][c], ent[1][2 * kk][c]);
            const cx<T> ahh = mk<T>(ent[0][2 * kk + 1][c], ent[1][2 * kk + 1][c]);
            const cx<T> alh = mk<T>(ent[2][2 * kk][c], ent[3][2 * kk][c]);
            glo[kk] = ent[4][2 * kk][c];
            ghi[kk] = ent[4][2 * kk + 1][c];
            const cx<T> idet = cinv(all * ahh - alh * alh);
            i00[kk] = ahh * idet;
            i11[kk] = all * idet;
            i01[kk] = mk<T>(T(0), T(0)) - alh * idet;
            zlo[kk] = glo[kk] * i00[kk] + ghi[kk] * i01[kk];
            zhi[kk] = glo[kk] * i01[kk] + ghi[kk] * i11[kk];
            S = S - (glo[kk] * zlo[kk] + ghi[kk] * zhi[kk]);
        }
        iS = cinv(S);
    }

    // wavefront 3 holds the pressure row (and the carry lanes)
    const int nt_wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)) == D ? 1 + D * St<3>::NUP : NT;
    for (int r0 = 0; r0 < nrhs; r0 += RB) {
        T ar[RB], ai[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) ar[q] = ai[q] = T(0);
        if (ein && row < R) {
            const T* ev[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) ev[q] = ein + (r0 + q < nrhs ? r0 + q : r0) * stride;
            rows3_rb<T, RB, CH, C>(cR, cI, lo, ls, cc, ev, vb, nb, ar, ai, nt_wave);
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                ar[q] *= csc;
                ai[q] *= csc;
            }
        }
        // the row's own unknown and the carried pressure as 32-bit byte offsets
        // into buffer descriptors (wave-uniform bases), formed here so that no
        // per-source address is kept across the row walk
        uint32_t oi = (uint32_t)idx * (uint32_t)sizeof(T), ob = (uint32_t)ipb * (uint32_t)sizeof(T);
        asm volatile("" : "+v"(oi), "+v"(ob));
        __syncthreads();   // the previous group's corrections have been read
        if (row < R) {
#pragma unroll
            for (int q = 0; q < RB; ++q) {
                const int r = r0 + q;
                if (r >= nrhs) break;
                T xr = T(0), xi = T(0);
                if (ok) {
                    const Buf<T> bq(b + r * stride, vb);
                    xr = bq.ld(oi, 0) - ar[q];
                    xi = bq.ld(oi, nb) - ai[q];
                }
                rs[q][row][c][0] = xr;
                rs[q][row][c][1] = xi;
            }
        }
        __syncthreads();
        // lane (row, c) solves source `row` of the group for cell c
        if (row < RB && r0 + row < nrhs) {
            cx<T> rr[R];
#pragma unroll
            for (int j = 0; j < R; ++j) rr[j] = mk<T>(rs[row][j][c][0], rs[row][j][c][1]);
            cx<T> acc = rr[2 * D];
            cx<T> ylo[D], yhi[D];
#pragma unroll
            for (int kk = 0; kk < D; ++kk) {
                ylo[kk] = i00[kk] * rr[2 * kk] + i01[kk] * rr[2 * kk + 1];
                yhi[kk] = i01[kk] * rr[2 * kk] + i11[kk] * rr[2 * kk + 1];
                acc = acc - (glo[kk] * ylo[kk] + ghi[kk] * yhi[kk]);
            }
            const cx<T> dp = acc * iS;
#pragma unroll
            for (int kk = 0; kk < D; ++kk) {
                const cx<T> dl = ylo[kk] - zlo[kk] * dp, dh = yhi[kk] - zhi[kk] * dp;
                rs[row][2 * kk][c][0] = dl.re;
                rs[row][2 * kk][c][1] = dl.im;
                rs[row][2 * kk + 1][c][0] = dh.re;
                rs[row][2 * kk + 1][c][1] = dh.im;
            }
            rs[row][2 * D][c][0] = dp.re;
            rs[row][2 * D][c][1] = dp.im;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = r0 + q;
            if (r >= nrhs) break;
            const Buf<T> oq(eout + r * stride, vb);
            if (ok) {
                cx<T> eown = mk<T>(T(0), T(0));
                if (ein) {
                    const Buf<T> eq(ein + r * stride, vb);
                    eown = mk<T>(eq.ld(oi, 0), eq.ld(oi, nb));
                }
                const T ww = row == 2 * D ? wp : w;
                oq.st(oi, eown.re + ww * rs[q][row][c][0]);
                oq.st(oi + nb, eown.im + ww * rs[q][row][c][1]);
            }
            if (carry) {
                T vr = T(0), vi = T(0);
                if (ein) {
                    const Buf<T> eq(ein + r * stride, vb);
                    vr = eq.ld(ob, 0);
                    vi = eq.ld(ob, nb);
                }
                oq.st(ob, vr);
                oq.st(ob + nb, vi);
            }
        }
    }
}
template <typename T, int RB, int CH, typename C = T>
__global__ __launch_bounds__(256) void k_relax_st3d(Geo g, int colour, T w, T wp, int econ, const T* __restrict__ b,
                                                    const T* __restrict__ ein, T* __restrict__ eout, int nrhs,
                                                    int64_t stride, int rpb, const C* __restrict__ cre,
                                                    const C* __restrict__ cim, int64_t lanes, T csc) {
    k_relax_st3d_body<T, RB, CH, C>(single_block<true>(), g, colour, w, wp, econ, b, ein, eout, nrhs, stride, rpb, cre, cim, lanes, csc);
}
template <class PK, typename T, int RB, int CH, typename C = T>
__global__ __launch_bounds__(256) void k_relax_st3d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<true>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_relax_st3d_body<T, RB, CH, C>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// y = A x or r = b - A x over stored rows on a 3D Galerkin level (term j of row t
// at [j * N + t]).
// (C, csc: storage of the rows and their scale, as in k_relax_st3d.)
template <typename T, int RB, int CH, typename C = T>
EHH_DEV void k_apply_st3d_body(VB ehh_vb, const Geo& g, const T* __restrict__ x, const T* __restrict__ b, T* __restrict__ y, int nrhs, int64_t stride, int rpb, const C* __restrict__ cre, const C* __restrict__ cim, T csc) {
    constexpr int NF = St<3>::NF, NT = NF + St<3>::NUP;
    {
        const int rb0 = blockIdx.y * rpb;
        x += rb0 * stride;
        if (b) b += rb0 * stride;
        y += rb0 * stride;
        nrhs = nrhs - rb0 < rpb ? nrhs - rb0 : rpb;
    }
    const int N = (int)g.N;
    const int t = (int)(int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (t >= N) return;
    int k = 0;
    while (k < 3 && t >= g.off[k + 1]) ++k;
    const int li = t - (int)g.off[k];
    const int d0 = g.n[0] - (k == 0), d1 = g.n[1] - (k == 1);
    int p[3] = {li % d0, (li / d0) % d1, li / (d0 * d1)};
    if (k < 3) p[k] += 1;
    const Cols3 cc = cols3(g, k, p);
    const Buf<C> cR(cre, (uint32_t)(NT * N * sizeof(C))), cI(cim, (uint32_t)(NF * N * sizeof(C)));
    const uint32_t lc = (uint32_t)t * (uint32_t)sizeof(C), lsc = (uint32_t)N * (uint32_t)sizeof(C);
    const uint32_t lo = (uint32_t)t * (uint32_t)sizeof(T), ls = (uint32_t)N * (uint32_t)sizeof(T);
    const uint32_t vb = 2 * ls;
    // every row walks all NT terms: ending pressure-row wavefronts early (as the
    // half-sweep does) costs this kernel a wavefront per SIMD of occupancy, and
    // measured slower (101 -> 109 us on a 72^3 level with 16 sources)
    for (int r0 = 0; r0 < nrhs; r0 += RB) {
        const T* xv[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) xv[q] = x + (r0 + q < nrhs ? r0 + q : r0) * stride;
        T ar[RB], ai[RB];
        rows3_rb<T, RB, CH, C>(cR, cI, lc, lsc, cc, xv, vb, ls, ar, ai, NT);
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            ar[q] *= csc;
            ai[q] *= csc;
        }
        // per-source buffer descriptors (wave-uniform bases) and the row's byte
        // offset formed here, so that no per-source address is kept across the row
        uint32_t ot = lo;
        asm volatile("" : "+v"(ot));
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = r0 + q;
            if (r >= nrhs) break;
            cx<T> o = mk<T>(ar[q], ai[q]);
            if (b) {
                const Buf<T> bq(b + r * stride, vb);
                o = mk<T>(bq.ld(ot, 0), bq.ld(ot, ls)) - o;
            }
            const Buf<T> yq(y + r * stride, vb);
            yq.st(ot, o.re);
            yq.st(ot + ls, o.im);
        }
    }
}
template <typename T, int RB, int CH, typename C = T>
__global__ __launch_bounds__(256) void k_apply_st3d(Geo g, const T* __restrict__ x, const T* __restrict__ b,
                                                    T* __restrict__ y, int nrhs, int64_t stride, int rpb,
                                                    const C* __restrict__ cre, const C* __restrict__ cim, T csc) {
    k_apply_st3d_body<T, RB, CH, C>(single_block<true>(), g, x, b, y, nrhs, stride, rpb, cre, cim, csc);
}
template <class PK, typename T, int RB, int CH, typename C = T>
__global__ __launch_bounds__(256) void k_apply_st3d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<true>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_apply_st3d_body<T, RB, CH, C>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// Builders of the 3D stored rows: coefficient of term j of the u_k row at face
// p (k < 3) or of the pressure row at cell p (k == 3), in the order of
// StOp::plan_u / plan_p, zero for terms outside the grid.
template <typename T>
EHH_DEV void term3(const StOp<3, T>& op, int k, const int* p, int j, T& re, T& im) {
    constexpr int D = 3, NF = St<3>::NF, NUP = St<3>::NUP, CF = St<3>::CF;
    const Geo& g = op.g;
    re = im = T(0);
    if (k < 3) {
        const int t1 = tang1<D>(k), t2 = tang2<D>(k);
        const int64_t fi = face_idx<D>(g, k, p);
        if (j < NF) {
            int dn, d1, d2;
            full_offset<D>(j, dn, d1, d2);
            int q[3] = {p[0], p[1], p[2]};
            q[k] += dn;
            q[t1] += d1;
            q[t2] += d2;
            if (!face_ok<D>(g, k, q)) return;
            const cx<T> a = j >= CF ? op.uu(k, fi, j - CF) : op.uu(k, face_idx<D>(g, k, q), CF - j);
            re = a.re;
            im = a.im;
        } else {
            int side, e1, e2;
            up_decode<D>(j - NF, side, e1, e2);
            int q[3] = {p[0], p[1], p[2]};
            q[k] += side - 1;
            q[t1] += e1;
            q[t2] += e2;
            if (!cell_ok<D>(g, q)) return;
            re = op.up(k, fi, j - NF);
        }
    } else {
        if (j == 0) {
            re = op.c.pp[cell_idx<D>(g, p)];
            return;
        }
        if (j > 3 * NUP) return;
        const int kk = (j - 1) / NUP, qq = (j - 1) % NUP;
        const int t1 = tang1<D>(kk), t2 = tang2<D>(kk);
        int side, e1, e2;
        up_decode<D>(qq, side, e1, e2);
        int q[3] = {p[0], p[1], p[2]};
        q[kk] += 1 - side;
        q[t1] -= e1;
        q[t2] -= e2;
        if (!face_ok<D>(g, kk, q)) return;
        re = op.up(kk, face_idx<D>(g, kk, q), qq);
    }
}

// one thread per (lane, term): the lane order of k_relax_st3d
template <typename T>
__global__ __launch_bounds__(256) void k_build_rows3d(StOp<3, T> op, int colour, T* __restrict__ re,
                                                      T* __restrict__ im, int64_t lanes) {
    constexpr int D = 3, R = 2 * D + 1, NF = St<3>::NF, NT = NF + St<3>::NUP;
    const Geo& g = op.g;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= lanes * NT) return;
    const int j = (int)(e / lanes);
    const int64_t gl = e % lanes;
    const int hp = g.n[0] >> 1;
    const int64_t npair = (int64_t)hp * g.n[1] * g.n[2];
    // the lane order of k_relax_st3d: 32 cells per 256 lanes, row j in lanes 32 j ..
    const int row = (int)((gl & 255) >> 5);
    const int64_t t = (gl >> 8) * 32 + (gl & 31);
    const bool live = t < npair;
    const int64_t tt = live ? t : 0;
    const int px = (int)(tt % hp);
    const int64_t rest = tt / hp;
    const int yy = (int)(rest % g.n[1]), zz = (int)(rest / g.n[1]);
    const int par = (colour + yy + zz) & 1;
    const int k = row < 2 * D ? (row >> 1) : 3;
    int p[3] = {2 * px + par, yy, zz};
    bool ok = live && row < R;
    if (k < 3) {
        p[k] += row & 1;
        ok = ok && p[k] >= 1 && p[k] <= g.n[k] - 1;
    }
    T a = T(0), bi = T(0);
    if (ok) term3<T>(op, k, p, j, a, bi);
    re[e] = a;
    if (j < NF) im[e] = bi;
}

// one thread per (row, term): row order for k_apply_st3d
template <typename T>
__global__ __launch_bounds__(256) void k_build_row_rows3d(StOp<3, T> op, T* __restrict__ re, T* __restrict__ im) {
    constexpr int NF = St<3>::NF, NT = NF + St<3>::NUP;
    const Geo& g = op.g;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= g.N * NT) return;
    const int j = (int)(e / g.N);
    const int64_t t = e % g.N;
    int k = 0;
    while (k < 3 && t >= g.off[k + 1]) ++k;
    const int64_t li = t - g.off[k];
    int p[3];
    if (k == 3) cell_pos<3>(g, li, p);
    else face_pos<3>(g, k, li, p);
    T a, bi;
    term3<T>(op, k, p, j, a, bi);
    re[e] = a;
    if (j < NF) im[e] = bi;
}

// ------------------------------------------- one thread per cell (2D finest level)
// The finest level's rows have few terms (self, two normal and two tangential
// neighbours, two pressures; the off-diagonal weights are real), so one thread
// owns one cell of the colour: it builds the cell's 5 x 5 block inverse once
// (per component a 2 x 2 inverse, then the Schur complement on the pressure) and
// then, for each of its right-hand sides, loads the 21 values of e_in its five
// rows touch plus b, and writes the corrected unknowns.  Consecutive threads own
// consecutive cells of the colour along x, so every load of a wavefront covers
// 128 consecutive cells and the other colour's half of each line is used by the
// neighbour loads of the same wavefront.  The thread also copies the pressure
// of the other cell of its x-pair (not relaxed in this half-sweep).
// TO: type of e_out (double lets the last half-sweep of a complex64 cycle write
// the FP64 result directly).
template <typename T, typename TO = T>
EHH_DEV void k_relax_cell2d_body(VB ehh_vb, const FineOp<2, T>& op, int colour, T w, T wp, int econ, const T* __restrict__ b, const T* __restrict__ ein, TO* __restrict__ eout, int nrhs, int64_t stride, int rpb) {
    const Geo& g = op.g;
    const int n0 = g.n[0], n1 = g.n[1];
    const int hp = n0 >> 1;
    const int64_t t = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)hp * n1) return;
    const int r_begin = blockIdx.y * rpb;
    const int r_end = r_begin + rpb < nrhs ? r_begin + rpb : nrhs;
    const int px = (int)(t % hp), y = (int)(t / hp);
    const int par = (colour + y) & 1;
    const int x = 2 * px + par;          // the relaxed cell
    const int xo = 2 * px + 1 - par;     // the other cell of the pair
    // unknown indices (clamped to a valid unknown where a neighbour is absent)
    const int64_t o0 = g.off[0], o1 = g.off[1], op3 = g.off[3];
    const int d0 = n0 - 1;                // u_0 faces per row
    auto iu0 = [&](int fx, int yy) { return o0 + (int64_t)yy * d0 + (fx - 1); };
    auto iu1 = [&](int xx, int fy) { return o1 + (int64_t)(fy - 1) * n0 + xx; };
    auto ip = [&](int xx, int yy) { return op3 + (int64_t)yy * n0 + xx; };
    // the four faces of the cell and their existence
    const bool vl = x >= 1, vr = x + 1 <= n0 - 1, vb = y >= 1, vt = y + 1 <= n1 - 1;
    const int pl[3] = {x, y, 0}, pr[3] = {x + 1, y, 0}, pb[3] = {x, y, 0}, pt[3] = {x, y + 1, 0};
    // row coefficients: diagonal (complex) and the real neighbour weights (0 when absent)
    const cx<T> one = mk<T>(T(1), T(0));
    const cx<T> dl = vl ? op.diag_u(0, pl) : one, dr = vr ? op.diag_u(0, pr) : one;
    const cx<T> db = vb ? op.diag_u(1, pb) : one, dt = vt ? op.diag_u(1, pt) : one;
    const int cc[3] = {x, y, 0};
    const T mu_k = op.mu_c(cc);
    // left face u0(x): normal lo u0(x-1) [cell x-1], tangential u0(x, y +- 1)
    const bool l_nlo = vl && x - 1 >= 1;
    int cq[3] = {x - 1, y, 0};
    const T wl_nlo = l_nlo ? -op.mu_c(cq) : T(0);
    const T wl_thi = (vl && y + 1 < n1) ? -op.mu_edge(0, pl, 1, y + 1) : T(0);
    const T wl_tlo = (vl && y - 1 >= 0) ? -op.mu_edge(0, pl, 1, y) : T(0);
    // right face u0(x+1): normal hi u0(x+2) [cell x+1], tangential u0(x+1, y +- 1)
    const bool r_nhi = vr && x + 2 <= n0 - 1;
    cq[0] = x + 1;
    const T wr_nhi = r_nhi ? -op.mu_c(cq) : T(0);
    const T wr_thi = (vr && y + 1 < n1) ? -op.mu_edge(0, pr, 1, y + 1) : T(0);
    const T wr_tlo = (vr && y - 1 >= 0) ? -op.mu_edge(0, pr, 1, y) : T(0);
    // bottom face u1(y): normal lo u1(y-1) [cell y-1], tangential u1(x +- 1, y)
    const bool b_nlo = vb && y - 1 >= 1;
    cq[0] = x;
    cq[1] = y - 1;
    const T wb_nlo = b_nlo ? -op.mu_c(cq) : T(0);
    const T wb_thi = (vb && x + 1 < n0) ? -op.mu_edge(1, pb, 0, x + 1) : T(0);
    const T wb_tlo = (vb && x - 1 >= 0) ? -op.mu_edge(1, pb, 0, x) : T(0);
    // top face u1(y+1): normal hi u1(y+2) [cell y+1], tangential u1(x +- 1, y+1)
    const bool t_nhi = vt && y + 2 <= n1 - 1;
    cq[1] = y + 1;
    const T wt_nhi = t_nhi ? -op.mu_c(cq) : T(0);
    const T wt_thi = (vt && x + 1 < n0) ? -op.mu_edge(1, pt, 0, x + 1) : T(0);
    const T wt_tlo = (vt && x - 1 >= 0) ? -op.mu_edge(1, pt, 0, x) : T(0);
    // in-block coupling of the two faces of a component (through mu of the cell)
    const T c0 = (vl && vr) ? -mu_k : T(0), c1 = (vb && vt) ? -mu_k : T(0);
    const T pdiag = -op.c.dinv[cell_idx<2>(g, cc)];
    // block inverse: per component [[d_lo, c], [c, d_hi]]^{-1}; g = (+1, -1) on present faces
    const T gl0 = vl ? T(1) : T(0), gh0 = vr ? T(-1) : T(0), gl1 = vb ? T(1) : T(0), gh1 = vt ? T(-1) : T(0);
    const T cu0 = econ ? T(0) : c0, cu1 = econ ? T(0) : c1;
    const cx<T> id0 = cinv(dl * dr - mk<T>(cu0 * cu0, T(0)));
    const cx<T> id1 = cinv(db * dt - mk<T>(cu1 * cu1, T(0)));
    const cx<T> a00 = dr * id0, a11 = dl * id0, a01 = (-cu0) * id0;   // inverse of component 0
    const cx<T> b00 = dt * id1, b11 = db * id1, b01 = (-cu1) * id1;   // inverse of component 1
    const cx<T> z0l = gl0 * a00 + gh0 * a01, z0h = gl0 * a01 + gh0 * a11;
    const cx<T> z1l = gl1 * b00 + gh1 * b01, z1h = gl1 * b01 + gh1 * b11;
    const cx<T> iS = cinv(mk<T>(pdiag, T(0)) - (gl0 * z0l + gh0 * z0h + gl1 * z1l + gh1 * z1h));
    // 32-bit byte offsets within one right-hand side's vector for buffer access
    // (the launcher checks that a vector stays below 4 GiB); absent neighbours
    // are read at the face itself (their weight is zero)
    using U = uint32_t;
    constexpr U E = (U)sizeof(T);
    const U kl = E * (U)iu0(vl ? x : 1, y), kr = E * (U)iu0(vr ? x + 1 : 1, y);
    const U kb = E * (U)iu1(x, vb ? y : 1), kt = E * (U)iu1(x, vt ? y + 1 : 1);
    const U kp = E * (U)ip(x, y), kpo = E * (U)ip(xo, y);
    const U ud0 = E * (U)d0, un0 = E * (U)n0;
    // which neighbours exist, one bit each; the offsets are formed from these bits
    // inside the loop over sources, so that they hold no registers across it
    const U nzm = (l_nlo ? 1u : 0u) | (r_nhi ? 2u : 0u) | (wl_thi != T(0) ? 4u : 0u) | (wl_tlo != T(0) ? 8u : 0u) |
                  (wr_thi != T(0) ? 16u : 0u) | (wr_tlo != T(0) ? 32u : 0u) | (b_nlo ? 64u : 0u) |
                  (t_nhi ? 128u : 0u) | (wb_thi != T(0) ? 256u : 0u) | (wb_tlo != T(0) ? 512u : 0u) |
                  (wt_thi != T(0) ? 1024u : 0u) | (wt_tlo != T(0) ? 2048u : 0u) | (vl ? 4096u : 0u) |
                  (vr ? 8192u : 0u) | (vb ? 16384u : 0u) | (vt ? 32768u : 0u);
    const U NB = E * (U)g.N;   // bytes of one plane (real or imaginary parts)
    const U VB = 2 * NB;       // bytes of one right-hand side's vector
    for (int r = r_begin; r < r_end; ++r) {
        const Buf<T> bb(b + (int64_t)r * stride, VB);
        constexpr U SO = (U)(sizeof(TO) / sizeof(T));   // output offsets scale
        const Buf<TO> eo(eout + (int64_t)r * stride, VB * SO);
        auto ldb = [&](U i) { return mk<T>(bb.ld(i), bb.ld(NB + i)); };
        cx<T> rl = vl ? ldb(kl) : mk<T>(T(0), T(0)), rr = vr ? ldb(kr) : mk<T>(T(0), T(0));
        cx<T> rb_ = vb ? ldb(kb) : mk<T>(T(0), T(0)), rt = vt ? ldb(kt) : mk<T>(T(0), T(0));
        cx<T> rp = ldb(kp);
        cx<T> el = mk<T>(T(0), T(0)), ere = el, eb = el, et = el, ep = el, epo = el;
        if (ein) {
            const Buf<T> ei(ein + (int64_t)r * stride, VB);
            auto ld = [&](U i) { return mk<T>(ei.ld(i), ei.ld(NB + i)); };
            U nz = nzm;
            asm volatile("" : "+v"(nz));
            // offset s where bit b of nz is set, else 0
            auto on = [&](int b, U s) { return (0u - ((nz >> b) & 1u)) & s; };
            const U sl_n = on(0, 0u - E), sr_n = on(1, E), sl_th = on(2, ud0), sl_tl = on(3, 0u - ud0);
            const U sr_th = on(4, ud0), sr_tl = on(5, 0u - ud0), sb_n = on(6, 0u - un0), st_n = on(7, un0);
            const U sb_th = on(8, E), sb_tl = on(9, 0u - E), st_th = on(10, E), st_tl = on(11, 0u - E);
            const U sp_l = on(12, 0u - E), sp_r = on(13, E), sp_b = on(14, 0u - un0), sp_t = on(15, un0);
            // every load of the iteration is issued before the arithmetic
            el = ld(kl);
            ere = ld(kr);
            eb = ld(kb);
            et = ld(kt);
            ep = ld(kp);
            epo = ld(kpo);
            const cx<T> pl_ = ld(kp + sp_l), pr_ = ld(kp + sp_r), pb_ = ld(kp + sp_b), pt_ = ld(kp + sp_t);
            const cx<T> l_n = ld(kl + sl_n), l_th = ld(kl + sl_th), l_tl = ld(kl + sl_tl);
            const cx<T> r_n = ld(kr + sr_n), r_th = ld(kr + sr_th), r_tl = ld(kr + sr_tl);
            const cx<T> b_n = ld(kb + sb_n), b_th = ld(kb + sb_th), b_tl = ld(kb + sb_tl);
            const cx<T> t_n = ld(kt + st_n), t_th = ld(kt + st_th), t_tl = ld(kt + st_tl);
            __builtin_amdgcn_sched_barrier(0);
            // residuals of the five rows: r = b - A e
            rl = rl - (dl * el + c0 * ere + wl_nlo * l_n + wl_thi * l_th + wl_tlo * l_tl + gl0 * (ep - pl_));
            rr = rr - (dr * ere + c0 * el + wr_nhi * r_n + wr_thi * r_th + wr_tlo * r_tl + (-gh0) * (pr_ - ep));
            rb_ = rb_ - (db * eb + c1 * et + wb_nlo * b_n + wb_thi * b_th + wb_tlo * b_tl + gl1 * (ep - pb_));
            rt = rt - (dt * et + c1 * eb + wt_nhi * t_n + wt_thi * t_th + wt_tlo * t_tl + (-gh1) * (pt_ - ep));
            rp = rp - (pdiag * ep + gh0 * ere + gl0 * el + gh1 * et + gl1 * eb);
        }
        // closed-form block solve
        const cx<T> y0l = a00 * rl + a01 * rr, y0h = a01 * rl + a11 * rr;
        const cx<T> y1l = b00 * rb_ + b01 * rt, y1h = b01 * rb_ + b11 * rt;
        const cx<T> dp = (rp - (gl0 * y0l + gh0 * y0h + gl1 * y1l + gh1 * y1h)) * iS;
        auto st = [&](U i, cx<T> v) {
            eo.st(SO * i, (TO)v.re);
            eo.st(SO * (NB + i), (TO)v.im);
        };
        if (vl) st(kl, el + w * (y0l - z0l * dp));
        if (vr) st(kr, ere + w * (y0h - z0h * dp));
        if (vb) st(kb, eb + w * (y1l - z1l * dp));
        if (vt) st(kt, et + w * (y1h - z1h * dp));
        st(kp, ep + wp * dp);
        st(kpo, epo);
    }
}
template <typename T, typename TO = T>
__global__ __launch_bounds__(256) void k_relax_cell2d(FineOp<2, T> op, int colour, T w, T wp, int econ,
                                                      const T* __restrict__ b, const T* __restrict__ ein,
                                                      TO* __restrict__ eout, int nrhs, int64_t stride, int rpb) {
    k_relax_cell2d_body<T, TO>(single_block<true>(), op, colour, w, wp, econ, b, ein, eout, nrhs, stride, rpb);
}
template <class PK, typename T, typename TO = T>
__global__ __launch_bounds__(256) void k_relax_cell2d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<true>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_relax_cell2d_body<T, TO>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// y = A x (or b - A x) on the finest 2D level, one thread per cell: the cell
// owns its left u_0 face, its bottom u_1 face and its pressure (the faces on the
// walls are not unknowns), so every unknown is written once; the three rows
// need thirteen values of x.
template <typename T, typename TX = T>
EHH_DEV void k_apply_cell2d_body(VB ehh_vb, const FineOp<2, T>& op, const TX* __restrict__ x, const T* __restrict__ b, T* __restrict__ y, int nrhs, int64_t stride, int rpb) {
    const Geo& g = op.g;
    const int n0 = g.n[0], n1 = g.n[1];
    const int64_t t = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)n0 * n1) return;
    const int r_begin = blockIdx.y * rpb;
    const int r_end = r_begin + rpb < nrhs ? r_begin + rpb : nrhs;
    const int cx_ = (int)(t % n0), cy = (int)(t / n0);
    const bool vu = cx_ >= 1, vv = cy >= 1;           // the owned faces exist
    const int pu[3] = {cx_, cy, 0}, pv[3] = {cx_, cy, 0};
    using U = uint32_t;
    constexpr U E = (U)sizeof(T);
    const int d0 = n0 - 1;
    // owned unknowns (clamped to a valid unknown when absent; not written then)
    const U ku = E * (U)(g.off[0] + (int64_t)cy * d0 + (vu ? cx_ - 1 : 0));
    const U kv = E * (U)(g.off[1] + (int64_t)(vv ? cy - 1 : 0) * n0 + cx_);
    const U kp = E * (U)(g.off[3] + (int64_t)cy * n0 + cx_);
    // u_0 row at face (cx, cy)
    cx<T> du = mk<T>(T(0), T(0));
    T wu_nh = T(0), wu_nl = T(0), wu_th = T(0), wu_tl = T(0);
    if (vu) {
        du = op.diag_u(0, pu);
        int q[3] = {cx_, cy, 0};
        if (cx_ + 1 <= n0 - 1) wu_nh = -op.mu_c(q);
        q[0] = cx_ - 1;
        if (cx_ - 1 >= 1) wu_nl = -op.mu_c(q);
        if (cy + 1 < n1) wu_th = -op.mu_edge(0, pu, 1, cy + 1);
        if (cy - 1 >= 0) wu_tl = -op.mu_edge(0, pu, 1, cy);
    }
    // u_1 row at face (cx, cy)
    cx<T> dv = mk<T>(T(0), T(0));
    T wv_nh = T(0), wv_nl = T(0), wv_th = T(0), wv_tl = T(0);
    if (vv) {
        dv = op.diag_u(1, pv);
        int q[3] = {cx_, cy, 0};
        if (cy + 1 <= n1 - 1) wv_nh = -op.mu_c(q);
        q[1] = cy - 1;
        if (cy - 1 >= 1) wv_nl = -op.mu_c(q);
        if (cx_ + 1 < n0) wv_th = -op.mu_edge(1, pv, 0, cx_ + 1);
        if (cx_ - 1 >= 0) wv_tl = -op.mu_edge(1, pv, 0, cx_);
    }
    const int cc[3] = {cx_, cy, 0};
    const T pdiag = -op.c.dinv[cell_idx<2>(g, cc)];
    // neighbour offsets relative to the owned unknowns (0 where the weight is 0)
    // and the p row's faces right (u_0 at cx+1) and top (u_1 at cy+1) when
    // interior: one bit each, the offsets and signs formed inside the loop over
    // sources, so that they hold no registers across it
    const U ud0 = E * (U)d0, un0 = E * (U)n0;
    const bool pl = cx_ >= 1, pb = cy >= 1;           // cells left and below exist
    const bool fr = cx_ + 1 <= n0 - 1, ft = cy + 1 <= n1 - 1;
    const U nzm = (wu_nh != T(0) ? 1u : 0u) | (wu_nl != T(0) ? 2u : 0u) | (wu_th != T(0) ? 4u : 0u) |
                  (wu_tl != T(0) ? 8u : 0u) | (wv_nh != T(0) ? 16u : 0u) | (wv_nl != T(0) ? 32u : 0u) |
                  (wv_th != T(0) ? 64u : 0u) | (wv_tl != T(0) ? 128u : 0u) | (pl ? 256u : 0u) | (pb ? 512u : 0u) |
                  (fr ? 1024u : 0u) | (ft ? 2048u : 0u) | (vu ? 4096u : 0u) | (vv ? 8192u : 0u) |
                  (fr && vu ? 16384u : 0u) | (ft && vv ? 32768u : 0u);
    const U NB = E * (U)g.N, VB = 2 * NB;
    for (int r = r_begin; r < r_end; ++r) {
        // x may be FP32 (the complex64 cycle's output read by the FP64 matrix-vector
        // product): its byte offsets are the FP64 ones halved
        constexpr U XS = sizeof(T) == 2 * sizeof(TX) ? 1u : 0u;
        const Buf<TX> xb(x + (int64_t)r * stride, VB >> XS);
        const Buf<T> yb(y + (int64_t)r * stride, VB);
        auto ld = [&](U i) { return mk<T>((T)xb.ld(i >> XS), (T)xb.ld((NB + i) >> XS)); };
        U nz = nzm;
        asm volatile("" : "+v"(nz));
        auto bit = [&](int b_) { return ((nz >> b_) & 1u) != 0u; };
        auto on = [&](int b_, U s_) { return (0u - ((nz >> b_) & 1u)) & s_; };
        const U su_nh = on(0, E), su_nl = on(1, 0u - E), su_th = on(2, ud0), su_tl = on(3, 0u - ud0);
        const U sv_nh = on(4, un0), sv_nl = on(5, 0u - un0), sv_th = on(6, E), sv_tl = on(7, 0u - E);
        const U sp_l = on(8, 0u - E), sp_b = on(9, 0u - un0);
        const U kur = ku + on(14, E), kvt = kv + on(15, un0);   // the faces right and top
        auto keep = [&](int b_, cx<T> v) { return bit(b_) ? v : mk<T>(T(0), T(0)); };
        // every load of the iteration is issued before the arithmetic (the
        // scheduler would otherwise wait on each load in turn)
        const cx<T> xu = ld(ku), xv = ld(kv), xp = ld(kp);
        const cx<T> xpl = ld(kp + sp_l), xpb = ld(kp + sp_b);
        const cx<T> u_nh = ld(ku + su_nh), u_nl = ld(ku + su_nl), u_th = ld(ku + su_th), u_tl = ld(ku + su_tl);
        const cx<T> v_nh = ld(kv + sv_nh), v_nl = ld(kv + sv_nl), v_th = ld(kv + sv_th), v_tl = ld(kv + sv_tl);
        const cx<T> x_r = ld(kur), x_t = ld(kvt);
        cx<T> b_u = mk<T>(T(0), T(0)), b_v = b_u, b_p = b_u;
        if (b) {
            const Buf<T> bb(b + (int64_t)r * stride, VB);
            b_u = mk<T>(bb.ld(ku), bb.ld(NB + ku));
            b_v = mk<T>(bb.ld(kv), bb.ld(NB + kv));
            b_p = mk<T>(bb.ld(kp), bb.ld(NB + kp));
        }
        __builtin_amdgcn_sched_barrier(0);
        cx<T> au = du * xu + wu_nh * u_nh + wu_nl * u_nl + wu_th * u_th + wu_tl * u_tl + (xp - xpl);
        cx<T> av = dv * xv + wv_nh * v_nh + wv_nl * v_nl + wv_th * v_th + wv_tl * v_tl + (xp - xpb);
        cx<T> ap = pdiag * xp - keep(10, x_r) + keep(12, xu) - keep(11, x_t) + keep(13, xv);
        if (b) {
            au = b_u - au;
            av = b_v - av;
            ap = b_p - ap;
        }
        if (vu) {
            yb.st(ku, au.re);
            yb.st(NB + ku, au.im);
        }
        if (vv) {
            yb.st(kv, av.re);
            yb.st(NB + kv, av.im);
        }
        yb.st(kp, ap.re);
        yb.st(NB + kp, ap.im);
    }
}
template <typename T, typename TX = T>
__global__ __launch_bounds__(256) void k_apply_cell2d(FineOp<2, T> op, const TX* __restrict__ x,
                                                      const T* __restrict__ b, T* __restrict__ y, int nrhs,
                                                      int64_t stride, int rpb) {
    k_apply_cell2d_body<T, TX>(single_block<true>(), op, x, b, y, nrhs, stride, rpb);
}
template <class PK, typename T>
__global__ __launch_bounds__(256) void k_apply_cell2d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<true>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_apply_cell2d_body<T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// ------------------------------------------- one thread per cell (3D finest level)
// The 3D form of k_relax_cell2d: the cell's 7 x 7 block (a 2 x 2 block per
// displacement component, the pressure coupled to all six faces) is inverted in
// closed form once per thread; each source then needs 43 values of e_in (per
// component the two faces, their outer normal neighbours and four tangential
// neighbours each; the pressure and its six neighbours) and b at 7 unknowns.
template <typename T>
EHH_DEV void k_relax_cell3d_body(VB ehh_vb, const FineOp<3, T>& op, int colour, T w, T wp, int econ, const T* __restrict__ b, const T* __restrict__ ein, T* __restrict__ eout, int nrhs, int64_t stride, int rpb) {
    const Geo& g = op.g;
    const int n[3] = {g.n[0], g.n[1], g.n[2]};
    const int hp = n[0] >> 1;
    const int64_t t = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)hp * n[1] * n[2]) return;
    const int r_begin = blockIdx.y * rpb;
    const int r_end = r_begin + rpb < nrhs ? r_begin + rpb : nrhs;
    const int px = (int)(t % hp);
    const int yz = (int)(t / hp);
    const int y = yz % n[1], z = yz / n[1];
    const int par = (colour + y + z) & 1;
    const int c[3] = {2 * px + par, y, z};
    const int xo = 2 * px + 1 - par;
    using U = uint32_t;
    constexpr U E = (U)sizeof(T);
    const cx<T> one = mk<T>(T(1), T(0));
    // per component k: faces lo (p[k] = c[k]) and hi (p[k] = c[k] + 1)
    bool vlo[3], vhi[3];
    cx<T> dlo[3], dhi[3];
    T cpl[3];                      // in-block coupling -mu(c) (0 if a face is absent)
    T wn_lo[3], wn_hi[3];          // outer normal neighbours
    T wt_lo[3][4], wt_hi[3][4];    // tangential neighbours: (t1+, t1-, t2+, t2-)
    U klo[3], khi[3];
    // which neighbours exist, 12 bits per component (outer normal lo / hi,
    // tangential lo 0..3, tangential hi 0..3, pressure lo / hi): the neighbour
    // offsets are formed from these bits inside the loop over sources, so that
    // they hold no registers across it
    U nzm[3];
    const T mu_k = op.mu_c(c);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int t1 = tang1<3>(k), t2 = tang2<3>(k);
        int pl[3] = {c[0], c[1], c[2]}, ph[3] = {c[0], c[1], c[2]};
        ph[k] += 1;
        vlo[k] = c[k] >= 1;
        vhi[k] = c[k] + 1 <= n[k] - 1;
        dlo[k] = vlo[k] ? op.diag_u(k, pl) : one;
        dhi[k] = vhi[k] ? op.diag_u(k, ph) : one;
        cpl[k] = (vlo[k] && vhi[k]) ? -mu_k : T(0);
        int q[3] = {c[0], c[1], c[2]};
        q[k] = c[k] - 1;
        const bool nl = vlo[k] && c[k] - 1 >= 1;
        wn_lo[k] = nl ? -op.mu_c(q) : T(0);
        q[k] = c[k] + 1;
        const bool nh = vhi[k] && c[k] + 2 <= n[k] - 1;
        wn_hi[k] = nh ? -op.mu_c(q) : T(0);
        int pcl[3] = {c[0], c[1], c[2]};
        if (!vlo[k]) pcl[k] = 1;
        int pch[3] = {c[0], c[1], c[2]};
        pch[k] = vhi[k] ? c[k] + 1 : 1;
        klo[k] = E * (U)(g.off[k]) + E * (U)face_idx<3>(g, k, pcl);
        khi[k] = E * (U)(g.off[k]) + E * (U)face_idx<3>(g, k, pch);
        U m = (nl ? 1u : 0u) | (nh ? 2u : 0u) | (vlo[k] ? 1u << 10 : 0u) | (vhi[k] ? 1u << 11 : 0u);
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int ta = j == 0 ? t1 : t2;
            const bool up_ok = c[ta] + 1 < n[ta], dn_ok = c[ta] - 1 >= 0;
            wt_lo[k][2 * j] = (vlo[k] && up_ok) ? -op.mu_edge(k, pl, ta, c[ta] + 1) : T(0);
            wt_lo[k][2 * j + 1] = (vlo[k] && dn_ok) ? -op.mu_edge(k, pl, ta, c[ta]) : T(0);
            wt_hi[k][2 * j] = (vhi[k] && up_ok) ? -op.mu_edge(k, ph, ta, c[ta] + 1) : T(0);
            wt_hi[k][2 * j + 1] = (vhi[k] && dn_ok) ? -op.mu_edge(k, ph, ta, c[ta]) : T(0);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                m |= (wt_lo[k][2 * j + h] != T(0) ? 1u : 0u) << (2 + 2 * j + h);
                m |= (wt_hi[k][2 * j + h] != T(0) ? 1u : 0u) << (6 + 2 * j + h);
            }
        }
        nzm[k] = m;
    }
    const T pdiag = -op.c.dinv[cell_idx<3>(g, c)];
    // block inverse: per component [[d_lo, c], [c, d_hi]]^{-1}; g = (+1, -1) on present faces
    cx<T> a00[3], a01[3], a11[3], zl[3], zh[3];
    T gl[3], gh[3];
    cx<T> S = mk<T>(pdiag, T(0));
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        gl[k] = vlo[k] ? T(1) : T(0);
        gh[k] = vhi[k] ? T(-1) : T(0);
        const T cu = econ ? T(0) : cpl[k];
        const cx<T> id = cinv(dlo[k] * dhi[k] - mk<T>(cu * cu, T(0)));
        a00[k] = dhi[k] * id;
        a11[k] = dlo[k] * id;
        a01[k] = (-cu) * id;
        zl[k] = gl[k] * a00[k] + gh[k] * a01[k];
        zh[k] = gl[k] * a01[k] + gh[k] * a11[k];
        S = S - (gl[k] * zl[k] + gh[k] * zh[k]);
    }
    const cx<T> iS = cinv(S);
    const U kp = E * (U)(g.off[3] + cell_idx<3>(g, c));
    int co[3] = {xo, y, z};
    const U kpo = E * (U)(g.off[3] + cell_idx<3>(g, co));
    const U pstride[3] = {E, E * (U)n[0], E * (U)n[0] * (U)n[1]};
    // byte strides of component k's faces along each axis
    U fst[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const U d0 = (U)(n[0] - (k == 0)), d1 = (U)(n[1] - (k == 1));
        fst[k][0] = E;
        fst[k][1] = E * d0;
        fst[k][2] = E * d0 * d1;
    }
    const U NB = E * (U)g.N, VB = 2 * NB;
    for (int r = r_begin; r < r_end; ++r) {
        const Buf<T> bb(b + (int64_t)r * stride, VB);
        const Buf<T> eo(eout + (int64_t)r * stride, VB);
        auto ldb = [&](U i) { return mk<T>(bb.ld(i), bb.ld(NB + i)); };
        cx<T> rlo[3], rhi[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            rlo[k] = vlo[k] ? ldb(klo[k]) : mk<T>(T(0), T(0));
            rhi[k] = vhi[k] ? ldb(khi[k]) : mk<T>(T(0), T(0));
        }
        cx<T> rp = ldb(kp);
        cx<T> elo[3], ehi[3], ep = mk<T>(T(0), T(0)), epo = ep;
#pragma unroll
        for (int k = 0; k < 3; ++k) elo[k] = ehi[k] = mk<T>(T(0), T(0));
        if (ein) {
            const Buf<T> ei(ein + (int64_t)r * stride, VB);
            auto ld = [&](U i) { return mk<T>(ei.ld(i), ei.ld(NB + i)); };
            cx<T> nlo[3], nhi[3], tlo[3][4], thi[3][4], plo[3], phi[3];
            U nz[3] = {nzm[0], nzm[1], nzm[2]};
            asm volatile("" : "+v"(nz[0]), "+v"(nz[1]), "+v"(nz[2]));
            // offset +s or -s where bit b of nz[k] is set, else 0
            auto pos = [&](int k, int b, U s) { return (0u - ((nz[k] >> b) & 1u)) & s; };
            auto neg = [&](int k, int b, U s) { return (0u - ((nz[k] >> b) & 1u)) & (0u - s); };
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const int t1 = tang1<3>(k), t2 = tang2<3>(k);
                elo[k] = ld(klo[k]);
                ehi[k] = ld(khi[k]);
                nlo[k] = ld(klo[k] + neg(k, 0, fst[k][k]));
                nhi[k] = ld(khi[k] + pos(k, 1, fst[k][k]));
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const U sa = fst[k][j == 0 ? t1 : t2];
                    tlo[k][2 * j] = ld(klo[k] + pos(k, 2 + 2 * j, sa));
                    tlo[k][2 * j + 1] = ld(klo[k] + neg(k, 3 + 2 * j, sa));
                    thi[k][2 * j] = ld(khi[k] + pos(k, 6 + 2 * j, sa));
                    thi[k][2 * j + 1] = ld(khi[k] + neg(k, 7 + 2 * j, sa));
                }
                plo[k] = ld(kp + neg(k, 10, pstride[k]));
                phi[k] = ld(kp + pos(k, 11, pstride[k]));
            }
            ep = ld(kp);
            epo = ld(kpo);
            __builtin_amdgcn_sched_barrier(0);
            // residuals r = b - A e of the seven rows
            cx<T> ap = pdiag * ep;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                cx<T> al = dlo[k] * elo[k] + cpl[k] * ehi[k] + wn_lo[k] * nlo[k] + gl[k] * (ep - plo[k]);
                cx<T> ah = dhi[k] * ehi[k] + cpl[k] * elo[k] + wn_hi[k] * nhi[k] + (-gh[k]) * (phi[k] - ep);
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    al = al + wt_lo[k][j] * tlo[k][j];
                    ah = ah + wt_hi[k][j] * thi[k][j];
                }
                rlo[k] = rlo[k] - al;
                rhi[k] = rhi[k] - ah;
                ap = ap + gh[k] * ehi[k] + gl[k] * elo[k];
            }
            rp = rp - ap;
        }
        // closed-form block solve
        cx<T> ylo[3], yhi[3];
        cx<T> acc = rp;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ylo[k] = a00[k] * rlo[k] + a01[k] * rhi[k];
            yhi[k] = a01[k] * rlo[k] + a11[k] * rhi[k];
            acc = acc - (gl[k] * ylo[k] + gh[k] * yhi[k]);
        }
        const cx<T> dp = acc * iS;
        auto st = [&](U i, cx<T> v) {
            eo.st(i, v.re);
            eo.st(NB + i, v.im);
        };
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (vlo[k]) st(klo[k], elo[k] + w * (ylo[k] - zl[k] * dp));
            if (vhi[k]) st(khi[k], ehi[k] + w * (yhi[k] - zh[k] * dp));
        }
        st(kp, ep + wp * dp);
        st(kpo, epo);
    }
}
template <typename T>
__global__ __launch_bounds__(256) void k_relax_cell3d(FineOp<3, T> op, int colour, T w, T wp, int econ,
                                                      const T* __restrict__ b, const T* __restrict__ ein,
                                                      T* __restrict__ eout, int nrhs, int64_t stride, int rpb) {
    k_relax_cell3d_body<T>(single_block<true>(), op, colour, w, wp, econ, b, ein, eout, nrhs, stride, rpb);
}
template <class PK, typename T>
__global__ __launch_bounds__(256) void k_relax_cell3d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<true>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_relax_cell3d_body<T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// y = A x (or b - A x) on the finest 3D level, one thread per cell owning its
// three lower faces (those on the walls are not unknowns) and its pressure.
template <typename T, typename TX = T>
EHH_DEV void k_apply_cell3d_body(VB ehh_vb, const FineOp<3, T>& op, const TX* __restrict__ x, const T* __restrict__ b, T* __restrict__ y, int nrhs, int64_t stride, int rpb) {
    const Geo& g = op.g;
    const int n[3] = {g.n[0], g.n[1], g.n[2]};
    const int64_t t = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (t >= g.ncell) return;
    const int r_begin = blockIdx.y * rpb;
    const int r_end = r_begin + rpb < nrhs ? r_begin + rpb : nrhs;
    int c[3];
    cell_pos<3>(g, t, c);
    using U = uint32_t;
    constexpr U E = (U)sizeof(T);
    bool v[3];
    cx<T> dg[3];
    T wnh[3], wnl[3], wt[3][4];
    U ku[3], fst[3][3];
    // which neighbours exist, 10 bits per component (normal hi / lo, tangential
    // 0..3, pressure below, upper face interior, and the two combined for the
    // upper face's offset): the offsets are formed inside the loop over sources,
    // so that they hold no registers across it
    U nzm[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int d0 = n[0] - (k == 0), d1 = n[1] - (k == 1);
        fst[k][0] = E;
        fst[k][1] = E * (U)d0;
        fst[k][2] = E * (U)d0 * (U)d1;
        const int t1 = tang1<3>(k), t2 = tang2<3>(k);
        v[k] = c[k] >= 1;
        int pc[3] = {c[0], c[1], c[2]};
        if (!v[k]) pc[k] = 1;
        ku[k] = E * (U)(g.off[k] + face_idx<3>(g, k, pc));
        dg[k] = mk<T>(T(0), T(0));
        wnh[k] = wnl[k] = T(0);
#pragma unroll
        for (int j = 0; j < 4; ++j) wt[k][j] = T(0);
        if (v[k]) {
            dg[k] = op.diag_u(k, c);
            int q[3] = {c[0], c[1], c[2]};
            if (c[k] + 1 <= n[k] - 1) wnh[k] = -op.mu_c(q);
            q[k] = c[k] - 1;
            if (c[k] - 1 >= 1) wnl[k] = -op.mu_c(q);
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int ta = j == 0 ? t1 : t2;
                if (c[ta] + 1 < n[ta]) wt[k][2 * j] = -op.mu_edge(k, c, ta, c[ta] + 1);
                if (c[ta] - 1 >= 0) wt[k][2 * j + 1] = -op.mu_edge(k, c, ta, c[ta]);
            }
        }
        // the p row's upper face of component k (face c[k] + 1), when interior:
        // the next face along axis k, or the owned face itself when that is
        // absent (then c[k] = 0 and the clamped owned face is face 1)
        const bool fh = c[k] + 1 <= n[k] - 1;
        U m = (wnh[k] != T(0) ? 1u : 0u) | (wnl[k] != T(0) ? 2u : 0u) | (v[k] ? 64u : 0u) | (fh ? 128u : 0u) |
              (fh && v[k] ? 256u : 0u);
#pragma unroll
        for (int j = 0; j < 4; ++j) m |= (wt[k][j] != T(0) ? 1u : 0u) << (2 + j);
        nzm[k] = m;
    }
    const T pdiag = -op.c.dinv[t];
    const U kp = E * (U)(g.off[3] + t);
    const U pstr[3] = {E, E * (U)n[0], E * (U)n[0] * (U)n[1]};
    const U NB = E * (U)g.N, VB = 2 * NB;
    for (int r = r_begin; r < r_end; ++r) {
        // x may be FP32 (the complex64 cycle's output read by the FP64 matrix-vector
        // product): its byte offsets are the FP64 ones halved
        constexpr U XS = sizeof(T) == 2 * sizeof(TX) ? 1u : 0u;
        const Buf<TX> xb(x + (int64_t)r * stride, VB >> XS);
        const Buf<T> yb(y + (int64_t)r * stride, VB);
        auto ld = [&](U i) { return mk<T>((T)xb.ld(i >> XS), (T)xb.ld((NB + i) >> XS)); };
        U nz[3] = {nzm[0], nzm[1], nzm[2]};
        asm volatile("" : "+v"(nz[0]), "+v"(nz[1]), "+v"(nz[2]));
        auto on = [&](int k, int b_, U s_) { return (0u - ((nz[k] >> b_) & 1u)) & s_; };
        auto keep = [&](int k, int b_, cx<T> val) { return ((nz[k] >> b_) & 1u) ? val : mk<T>(T(0), T(0)); };
        cx<T> xu[3], xnh[3], xnl[3], xt[3][4], xpl[3], xh[3], bu[3];
        const cx<T> xp = ld(kp);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int t1 = tang1<3>(k), t2 = tang2<3>(k);
            xu[k] = ld(ku[k]);
            xnh[k] = ld(ku[k] + on(k, 0, fst[k][k]));
            xnl[k] = ld(ku[k] + on(k, 1, 0u - fst[k][k]));
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const U sa = fst[k][j == 0 ? t1 : t2];
                xt[k][2 * j] = ld(ku[k] + on(k, 2 + 2 * j, sa));
                xt[k][2 * j + 1] = ld(ku[k] + on(k, 3 + 2 * j, 0u - sa));
            }
            xpl[k] = ld(kp + on(k, 6, 0u - pstr[k]));
            xh[k] = ld(ku[k] + on(k, 8, fst[k][k]));
        }
        cx<T> bp = mk<T>(T(0), T(0));
#pragma unroll
        for (int k = 0; k < 3; ++k) bu[k] = bp;
        if (b) {
            const Buf<T> bb(b + (int64_t)r * stride, VB);
#pragma unroll
            for (int k = 0; k < 3; ++k) bu[k] = mk<T>(bb.ld(ku[k]), bb.ld(NB + ku[k]));
            bp = mk<T>(bb.ld(kp), bb.ld(NB + kp));
        }
        __builtin_amdgcn_sched_barrier(0);
        cx<T> ap = pdiag * xp;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            cx<T> au = dg[k] * xu[k] + wnh[k] * xnh[k] + wnl[k] * xnl[k] + (xp - xpl[k]);
#pragma unroll
            for (int j = 0; j < 4; ++j) au = au + wt[k][j] * xt[k][j];
            if (b) au = bu[k] - au;
            if (v[k]) {
                yb.st(ku[k], au.re);
                yb.st(NB + ku[k], au.im);
            }
            ap = ap - keep(k, 7, xh[k]) + keep(k, 6, xu[k]);
        }
        if (b) ap = bp - ap;
        yb.st(kp, ap.re);
        yb.st(NB + kp, ap.im);
    }
}
template <typename T, typename TX = T>
__global__ __launch_bounds__(256) void k_apply_cell3d(FineOp<3, T> op, const TX* __restrict__ x,
                                                      const T* __restrict__ b, T* __restrict__ y, int nrhs,
                                                      int64_t stride, int rpb) {
    k_apply_cell3d_body<T, TX>(single_block<true>(), op, x, b, y, nrhs, stride, rpb);
}
template <class PK, typename T>
__global__ __launch_bounds__(256) void k_apply_cell3d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<true>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_apply_cell3d_body<T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// Builds the stored rows of one colour's half-sweep in the lane order of
// k_relax_st2d (same lane -> cell/row mapping, absent rows all zero): real parts
// of all NT terms, imaginary parts of the NF u-u terms.
template <typename T>
__global__ __launch_bounds__(256) void k_build_plans(StOp<2, T> op, int colour, T* __restrict__ re,
                                                     T* __restrict__ im, int64_t lanes) {
    constexpr int D = 2;
    constexpr int R = 2 * D + 1;
    using Op = StOp<2, T>;
    const Geo& g = op.g;
    const int64_t gl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gl >= lanes) return;
    const int hp = g.n[0] >> 1;
    const int64_t npair = (int64_t)hp * g.n[1] * g.n[2];
    const int lane = (int)(gl & 63);
    const int row = lane >> 3;
    const int cig = lane & 7;
    const int64_t t = (gl >> 6) * 8 + cig;
    const bool live = t < npair;
    const int64_t tt = live ? t : 0;
    const int px = (int)(tt % hp);
    const int64_t rest = tt / hp;
    const int yy = (int)(rest % g.n[1]);
    const int zz = (int)(rest / g.n[1]);
    const int par = (colour + yy + zz) & 1;
    const int k = row < 2 * D ? (row >> 1) : 3;
    int p[3] = {2 * px + par, yy, zz};
    bool ok = live && row < R;
    if (k < 3) {
        p[k] += row & 1;
        ok = ok && p[k] >= 1 && p[k] <= g.n[k] - 1;
    }
    Plan<T, Op::NT> P;
    if (ok) {
        if (k == 3)
            op.plan_p(p, P);
        else
            op.plan_u(k, p, P);
    } else {
#pragma unroll
        for (int j = 0; j < Op::NT; ++j) P.set(j, 0, T(0), T(0));
    }
#pragma unroll
    for (int j = 0; j < Op::NT; ++j) re[j * lanes + gl] = P.re[j];
#pragma unroll
    for (int j = 0; j < St<2>::NF; ++j) im[j * lanes + gl] = P.im[j];
}

// Stored rows of y = A x in row order (term j of row t at [j * N + t]; as above,
// imaginary parts of the u-u terms only).
template <typename T>
__global__ __launch_bounds__(256) void k_build_row_plans(StOp<2, T> op, T* __restrict__ re, T* __restrict__ im) {
    using Op = StOp<2, T>;
    const Geo& g = op.g;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= g.N) return;
    int k = 0;
    while (k < 3 && t >= g.off[k + 1]) ++k;
    const int64_t li = t - g.off[k];
    int p[3];
    Plan<T, Op::NT> P;
    if (k == 3) {
        cell_pos<2>(g, li, p);
        op.plan_p(p, P);
    } else {
        face_pos<2>(g, k, li, p);
        op.plan_u(k, p, P);
    }
#pragma unroll
    for (int j = 0; j < Op::NT; ++j) re[j * g.N + t] = P.re[j];
#pragma unroll
    for (int j = 0; j < St<2>::NF; ++j) im[j * g.N + t] = P.im[j];
}

// ---------------------------------------------------- LDS-staged half-sweep (2D)
// A block relaxes the red cells of a 16 x 8 tile (64 cells, eight lanes each as in
// k_relax_plan).  For every right-hand side the vectors the tile's rows touch
// (tile plus a halo of one face along the normal and `ht` cells along the
// tangential axis of each component, one cell for the pressure) are loaded once,
// coalesced, into LDS; the rows are then evaluated from LDS instead of
// re-reading neighbours through the caches (a Galerkin row has 21 terms).
static constexpr int LT_X = 16, LT_Y = 8;

template <typename T, class Op>
EHH_DEV void k_relax_lds2d_body(VB ehh_vb, const Op& op, int colour, T w, T wp, int econ, const T* __restrict__ b, const T* __restrict__ ein, T* __restrict__ eout, int nrhs, int64_t stride, int rpb, int ht) {
    constexpr int D = 2, R = 5;
    __shared__ T sre[(LT_X + 3) * (LT_Y + 4) + (LT_X + 4) * (LT_Y + 3) + (LT_X + 2) * (LT_Y + 2)];
    __shared__ T sim[(LT_X + 3) * (LT_Y + 4) + (LT_X + 4) * (LT_Y + 3) + (LT_X + 2) * (LT_Y + 2)];
    {
        const int rb0 = blockIdx.y * rpb;
        b += rb0 * stride;
        if (ein) ein += rb0 * stride;
        eout += rb0 * stride;
        nrhs = nrhs - rb0 < rpb ? nrhs - rb0 : rpb;
    }
    const Geo& g = op.g;
    const int tiles_x = (g.n[0] + LT_X - 1) / LT_X;
    const int x0 = (ehh_vb.x % tiles_x) * LT_X, y0 = (ehh_vb.x / tiles_x) * LT_Y;
    const int lane = threadIdx.x & 63, row = lane >> 3, cig = lane & 7;
    const int yl = threadIdx.x >> 6;   // one tile row per wavefront
    const int yy = y0 + yl;
    const int par = (colour + yy) & 1;
    const int cr[3] = {x0 + 2 * cig + par, yy, 0};
    const int cb[3] = {x0 + 2 * cig + 1 - par, yy, 0};
    const bool live = yy < g.n[1] && x0 + 2 * cig < g.n[0];
    const int base = cig;
    // region geometry: component 0 (x faces), 1 (y faces), pressure
    const int w0x = LT_X + 3, w0y = LT_Y + 2 * ht, o0x = x0 - 1, o0y = y0 - ht;
    const int w1x = LT_X + 2 * ht, w1y = LT_Y + 3, o1x = x0 - ht, o1y = y0 - 1;
    const int wpx = LT_X + 2, wpy = LT_Y + 2, opx = x0 - 1, opy = y0 - 1;
    const int b1 = w0x * w0y, bp = b1 + w1x * w1y, nreg = bp + wpx * wpy;

    const int k = row < 2 * D ? (row >> 1) : 3;
    int p[3] = {cr[0], cr[1], 0};
    bool ok = live && row < R;
    if (k < 3) {
        p[k] += row & 1;
        ok = ok && p[k] >= 1 && p[k] <= g.n[k] - 1;
    }
    Plan<T, Op::NT> P;
    int64_t idx = 0;
    int own = 0;
    if (ok) {
        if (k == 3) {
            op.plan_p(p, P);
            idx = g.off[3] + cell_idx<D>(g, p);
        } else {
            op.plan_u(k, p, P);
            idx = g.off[k] + face_idx<D>(g, k, p);
        }
    } else {
#pragma unroll
        for (int j = 0; j < Op::NT; ++j) P.set(j, 0, T(0), T(0));
    }
    // block entries (before the plan indices are turned into LDS offsets)
    const T dre = ok ? (k == 3 ? P.re[0] : P.re[Op::T_SELF]) : T(1);
    const T dim = ok ? (k == 3 ? P.im[0] : P.im[Op::T_SELF]) : T(0);
    const bool lowrow = row < 2 * D && (row & 1) == 0;
    const T cre = (ok && lowrow && !econ) ? P.re[Op::T_NHI] : T(0);
    const T cim = (ok && lowrow && !econ) ? P.im[Op::T_NHI] : T(0);
    const T gg = (ok && row < 2 * D) ? (lowrow ? P.re[Op::T_PHI] : P.re[Op::T_PLO]) : T(0);
    // global index -> LDS offset (clamped to 0 outside the region; such terms
    // carry a zero coefficient)
    auto to_lds = [&](int64_t gi) -> int {
        int kk = gi < g.off[1] ? 0 : (gi < g.off[3] ? 1 : 3);
        const int li = (int)(gi - g.off[kk]);
        int q0, q1, o;
        if (kk == 0) {
            const int d0 = g.n[0] - 1;
            q0 = li % d0 + 1;
            q1 = li / d0;
            q0 -= o0x;
            q1 -= o0y;
            o = (q0 >= 0 && q0 < w0x && q1 >= 0 && q1 < w0y) ? q0 + w0x * q1 : -1;
        } else if (kk == 1) {
            const int d0 = g.n[0];
            q0 = li % d0;
            q1 = li / d0 + 1;
            q0 -= o1x;
            q1 -= o1y;
            o = (q0 >= 0 && q0 < w1x && q1 >= 0 && q1 < w1y) ? b1 + q0 + w1x * q1 : -1;
        } else {
            const int d0 = g.n[0];
            q0 = li % d0 - opx;
            q1 = li / d0 - opy;
            o = (q0 >= 0 && q0 < wpx && q1 >= 0 && q1 < wpy) ? bp + q0 + wpx * q1 : -1;
        }
        return o < 0 ? 0 : o;
    };
    // LDS offsets (below 2^16) packed two to a register
    uint32_t pk[(Op::NT + 1) / 2];
#pragma unroll
    for (int j = 0; j < (Op::NT + 1) / 2; ++j) {
        const uint32_t lo = (uint32_t)to_lds(P.ix[2 * j]);
        const uint32_t hi = 2 * j + 1 < Op::NT ? (uint32_t)to_lds(P.ix[2 * j + 1]) : 0u;
        pk[j] = lo | (hi << 16);
    }
    own = ok ? to_lds(idx) : 0;
    const bool carry = live && row == R;
    const int64_t ipb = g.off[3] + cell_idx<D>(g, cb);
    const int ownb = carry ? to_lds(ipb) : 0;

    cx<T> i00[D], i01[D], i11[D], zlo[D], zhi[D];
    T glo[D], ghi[D];
    cx<T> S;
    {
        const T pd = __shfl(dre, base + 8 * (2 * D), 64);
        S = mk<T>(pd, T(0));
#pragma unroll
        for (int kk = 0; kk < D; ++kk) {
            const cx<T> all = mk<T>(__shfl(dre, base + 8 * (2 * kk), 64), __shfl(dim, base + 8 * (2 * kk), 64));
            const cx<T> ahh = mk<T>(__shfl(dre, base + 8 * (2 * kk + 1), 64), __shfl(dim, base + 8 * (2 * kk + 1), 64));
            const cx<T> alh = mk<T>(__shfl(cre, base + 8 * (2 * kk), 64), __shfl(cim, base + 8 * (2 * kk), 64));
            glo[kk] = __shfl(gg, base + 8 * (2 * kk), 64);
            ghi[kk] = __shfl(gg, base + 8 * (2 * kk + 1), 64);
            if (row == 0) {
                const cx<T> idet = cinv(all * ahh - alh * alh);
                i00[kk] = ahh * idet;
                i11[kk] = all * idet;
                i01[kk] = mk<T>(T(0), T(0)) - alh * idet;
                zlo[kk] = glo[kk] * i00[kk] + ghi[kk] * i01[kk];
                zhi[kk] = glo[kk] * i01[kk] + ghi[kk] * i11[kk];
                S = S - (glo[kk] * zlo[kk] + ghi[kk] * zhi[kk]);
            }
        }
    }
    const cx<T> iS = row == 0 ? cinv(S) : mk<T>(T(0), T(0));

    // Byte offset of each tile entry this thread stages (OOB_OFF outside the grid:
    // the buffer load returns zero), computed once for all right-hand sides.
    constexpr int NREG = (LT_X + 3) * (LT_Y + 4) + (LT_X + 4) * (LT_Y + 3) + (LT_X + 2) * (LT_Y + 2);
    constexpr int NST = (NREG + 511) / 512;
    uint32_t vo[NST];
#pragma unroll
    for (int i = 0; i < NST; ++i) {
        const int e = threadIdx.x + i * 512;
        vo[i] = OOB_OFF;
        if (e < nreg) {
            int kk, q0, q1;
            if (e < b1) {
                kk = 0;
                q0 = e % w0x + o0x;
                q1 = e / w0x + o0y;
            } else if (e < bp) {
                kk = 1;
                q0 = (e - b1) % w1x + o1x;
                q1 = (e - b1) / w1x + o1y;
            } else {
                kk = 3;
                q0 = (e - bp) % wpx + opx;
                q1 = (e - bp) / wpx + opy;
            }
            const int q[3] = {q0, q1, 0};
            const bool in = kk == 3 ? cell_ok<D>(g, q) : face_ok<D>(g, kk, q);
            if (in)
                vo[i] = (uint32_t)(kk == 3 ? g.off[3] + cell_idx<D>(g, q) : g.off[kk] + face_idx<D>(g, kk, q)) * sizeof(T);
        }
    }
    // The buffers span this block's right-hand sides (under 2 GiB, checked at
    // launch); the source is selected by a wave-uniform offset.
    const uint32_t span = (uint32_t)(nrhs * stride * (int64_t)sizeof(T));
    const uint32_t imo = (uint32_t)(g.N * sizeof(T));
    const Buf<T> eb(ein, ein ? span : 0u), bb(b, span);
    const uint32_t bo = ok ? (uint32_t)idx * sizeof(T) : OOB_OFF;
    cx<T> nst[NST], nb;
    auto fetch = [&](int r) {
        const uint32_t so = (uint32_t)(r * stride * (int64_t)sizeof(T));
        if (ein) {
#pragma unroll
            for (int i = 0; i < NST; ++i) nst[i] = mk<T>(eb.ld(vo[i], so), eb.ld(vo[i], so + imo));
        }
        nb = mk<T>(bb.ld(bo, so), bb.ld(bo, so + imo));
    };
    for (int r = 0; r < nrhs; ++r) {
        // keeps the unpacking of the LDS indices inside the loop (hoisted, it
        // would take a register per term again)
#pragma unroll
        for (int j = 0; j < (Op::NT + 1) / 2; ++j) asm volatile("" : "+v"(pk[j]));
        fetch(r);
        const Vec<T> ov{eout + r * stride, g.N};
        const cx<T> bcur = nb;
        cx<T> res = mk<T>(T(0), T(0));
        cx<T> eown = mk<T>(T(0), T(0)), ecarry = mk<T>(T(0), T(0));
        if (ein) {
            lds_barrier();   // the previous right-hand side is done with the tile
#pragma unroll
            for (int i = 0; i < NST; ++i) {
                const int e = threadIdx.x + i * 512;
                if (e < nreg) {
                    sre[e] = nst[i].re;
                    sim[e] = nst[i].im;
                }
            }
            lds_barrier();
            if (ok) {
                // one fused multiply-add per real product; the u-p and p-u terms
                // (from St<2>::NF on) are real
                T ar = T(0), ai = T(0);
#pragma unroll
                for (int j = 0; j < Op::NT; ++j) {
                    const uint32_t o = (j & 1) ? (pk[j >> 1] >> 16) : (pk[j >> 1] & 0xffffu);
                    const T vr = sre[o], vi = sim[o];
                    ar = fma(P.re[j], vr, ar);
                    ai = fma(P.re[j], vi, ai);
                    if (j < St<2>::NF) {
                        ar = fma(-P.im[j], vi, ar);
                        ai = fma(P.im[j], vr, ai);
                    }
                }
                res = bcur - mk<T>(ar, ai);
                eown = mk<T>(sre[own], sim[own]);
            }
            if (carry) ecarry = mk<T>(sre[ownb], sim[ownb]);
        } else if (ok) {
            res = bcur;
        }
        cx<T> rr[R];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            rr[j].re = __shfl(res.re, base + 8 * j, 64);
            rr[j].im = __shfl(res.im, base + 8 * j, 64);
        }
        cx<T> d[R];
        if (row == 0) {
            cx<T> acc = rr[2 * D];
            cx<T> ylo[D], yhi[D];
#pragma unroll
            for (int kk = 0; kk < D; ++kk) {
                ylo[kk] = i00[kk] * rr[2 * kk] + i01[kk] * rr[2 * kk + 1];
                yhi[kk] = i01[kk] * rr[2 * kk] + i11[kk] * rr[2 * kk + 1];
                acc = acc - (glo[kk] * ylo[kk] + ghi[kk] * yhi[kk]);
            }
            const cx<T> dp = acc * iS;
#pragma unroll
            for (int kk = 0; kk < D; ++kk) {
                d[2 * kk] = ylo[kk] - zlo[kk] * dp;
                d[2 * kk + 1] = yhi[kk] - zhi[kk] * dp;
            }
            d[2 * D] = dp;
        }
        cx<T> mine = mk<T>(T(0), T(0));
#pragma unroll
        for (int j = 0; j < R; ++j) {
            const T vr = __shfl(d[j].re, base, 64);
            const T vi = __shfl(d[j].im, base, 64);
            if (row == j) mine = mk<T>(vr, vi);
        }
        if (ok) ov.st(idx, eown + (row == 4 ? wp : w) * mine);
        if (carry) ov.st(ipb, ecarry);
    }
}
// Tiles are numbered per XCD, so that neighbouring tiles, which stage the same
// halo rows, share an L2 (256^2 with 32 sources: 100.6 -> 97.4 us).  Loading the
// next source's tile while the current one is computed gave nothing (97.6 us).
template <typename T, class Op>
__global__ __launch_bounds__(512) void k_relax_lds2d(Op op, int colour, T w, T wp, int econ, const T* __restrict__ b,
                                                     const T* __restrict__ ein, T* __restrict__ eout, int nrhs,
                                                     int64_t stride, int rpb, int ht) {
    k_relax_lds2d_body<T, Op>(single_block<true>(), op, colour, w, wp, econ, b, ein, eout, nrhs, stride, rpb, ht);
}
template <class PK, typename T, class Op>
__global__ __launch_bounds__(512) void k_relax_lds2d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<true>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_relax_lds2d_body<T, Op>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// --------------------------------------------------------------------- transfers
// Staggered bilinear transfer: u_k linear along its normal (weights 1 / (1/2, 1/2)),
// linear along each tangential axis (3/4 nearer coarse row, 1/4 the other, zero
// beyond the wall); pressure piecewise constant.  Restriction is P^T.

template <int D, typename T>
EHH_DEV void k_restrict_body(VB ehh_vb, const Geo& gf, const Geo& gc, const T* __restrict__ rf, T* __restrict__ rc, int nrhs) {
    const int64_t t = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (t >= gc.N) return;
    int k = 0;
    while (k < 3 && t >= gc.off[k + 1]) ++k;
    if (k >= D) k = 3;
    const int64_t li = t - gc.off[k];
    const int64_t sf = 2 * gf.N, sc = 2 * gc.N;
    const int r0 = blockIdx.y;   // one right-hand side per grid row
    rf += r0 * sf;
    rc += r0 * sc;
    nrhs = 1;
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
__global__ __launch_bounds__(256) void k_restrict(Geo gf, Geo gc, const T* __restrict__ rf,
                                                  T* __restrict__ rc, int nrhs) {
    k_restrict_body<D, T>(single_block<false>(), gf, gc, rf, rc, nrhs);
}
template <class PK, int D, typename T>
__global__ __launch_bounds__(256) void k_restrict_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_restrict_body<D, T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

template <int D, typename T>
EHH_DEV void k_prolong_body(VB ehh_vb, const Geo& gf, const Geo& gc, const T* __restrict__ ec, T* __restrict__ ef, int nrhs) {
    const int64_t t = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (t >= gf.N) return;
    int k = 0;
    while (k < 3 && t >= gf.off[k + 1]) ++k;
    if (k >= D) k = 3;
    const int64_t li = t - gf.off[k];
    const int64_t sf = 2 * gf.N, sc = 2 * gc.N;
    const int r0 = blockIdx.y;   // one right-hand side per grid row
    ef += r0 * sf;
    ec += r0 * sc;
    nrhs = 1;
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
template <int D, typename T>
__global__ __launch_bounds__(256) void k_prolong(Geo gf, Geo gc, const T* __restrict__ ec,
                                                 T* __restrict__ ef, int nrhs) {
    k_prolong_body<D, T>(single_block<false>(), gf, gc, ec, ef, nrhs);
}
template <class PK, int D, typename T>
__global__ __launch_bounds__(256) void k_prolong_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_prolong_body<D, T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// 2D transfers with 32-bit indices and every load issued before the sums, in the
// same term order as k_restrict / k_prolong (a term outside the grid reads a
// clamped index with weight zero).  One right-hand side per grid row.
template <typename T>
EHH_DEV void k_restrict2d_body(VB ehh_vb, const Geo& gf, const Geo& gc, const T* __restrict__ rf, T* __restrict__ rc) {
    const int t = (int)(ehh_vb.x * blockDim.x + threadIdx.x);
    const int Nc = (int)gc.N;
    if (t >= Nc) return;
    rf += (int64_t)blockIdx.y * 2 * gf.N;
    rc += (int64_t)blockIdx.y * 2 * gc.N;
    const int ncx = gc.n[0];
    int k, X, Y;
    if (t >= (int)gc.off[3]) {
        const int li = t - (int)gc.off[3];
        k = 3;
        X = li % ncx;
        Y = li / ncx;
    } else if (t < (int)gc.off[1]) {
        const int li = t - (int)gc.off[0];
        k = 0;
        X = li % (ncx - 1) + 1;
        Y = li / (ncx - 1);
    } else {
        const int li = t - (int)gc.off[1];
        k = 1;
        X = li % ncx;
        Y = li / ncx + 1;
    }
    const cx<T> v = restrict_at2d<T>(gf, rf, k, X, Y);
    rc[t] = v.re;
    rc[Nc + t] = v.im;
}
template <typename T>
__global__ __launch_bounds__(256) void k_restrict2d(Geo gf, Geo gc, const T* __restrict__ rf, T* __restrict__ rc) {
    k_restrict2d_body<T>(single_block<false>(), gf, gc, rf, rc);
}
template <class PK, typename T>
__global__ __launch_bounds__(256) void k_restrict2d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_restrict2d_body<T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

template <typename T>
EHH_DEV void k_prolong2d_body(VB ehh_vb, const Geo& gf, const Geo& gc, const T* __restrict__ ec, T* __restrict__ ef) {
    const int t = (int)(ehh_vb.x * blockDim.x + threadIdx.x);
    const int Nc = (int)gc.N, Nf = (int)gf.N;
    if (t >= Nf) return;
    ec += (int64_t)blockIdx.y * 2 * gc.N;
    ef += (int64_t)blockIdx.y * 2 * gf.N;
    const int ncx = gc.n[0], ncy = gc.n[1], nfx = gf.n[0];
    if (t >= (int)gf.off[3]) {   // pressure: piecewise constant
        const int li = t - (int)gf.off[3];
        const int x = li % nfx, y = li / nfx;
        const int ci = (int)gc.off[3] + (y >> 1) * ncx + (x >> 1);
        const T cr = ec[ci], cim = ec[Nc + ci];
        const T fr = ef[t], fi = ef[Nf + t];
        ef[t] = fr + cr;
        ef[Nf + t] = fi + cim;
        return;
    }
    const bool k0 = t < (int)gf.off[1];
    int pn, pt;   // fine position along the normal and the tangential axis
    if (k0) {
        const int li = t - (int)gf.off[0];
        pn = li % (nfx - 1) + 1;
        pt = li / (nfx - 1);
    } else {
        const int li = t - (int)gf.off[1];
        pt = li % nfx;
        pn = li / nfx + 1;
    }
    const int ncn = k0 ? ncx : ncy, nct = k0 ? ncy : ncx;
    // normal: the coincident coarse face (weight 1) or the two around it (1/2 each)
    const int xn0 = (pn & 1) ? (pn - 1) >> 1 : pn >> 1, xn1 = (pn + 1) >> 1;
    const T wn0 = (pn & 1) ? T(0.5) : T(1), wn1 = (pn & 1) ? T(0.5) : T(0);
    // tangential: the nearer coarse row (3/4) and the other one (1/4) inside the grid
    const int C = pt >> 1, o = (pt & 1) ? C + 1 : C - 1;
    const bool ook = o >= 0 && o < nct;
    const int xs[2] = {xn0, xn1};
    const T ws[2] = {wn0, wn1};
    const int ts[2] = {C, ook ? o : C};
    const T wts[2] = {T(0.75), ook ? T(0.25) : T(0)};
    int ix[4];
    T wt[4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int i1 = 0; i1 < 2; ++i1) {
            const int X = xs[a];
            const bool ok = X >= 1 && X <= ncn - 1;
            const int Xc = ok ? X : 1;
            ix[2 * a + i1] = k0 ? (int)gc.off[0] + ts[i1] * (ncx - 1) + Xc - 1 : (int)gc.off[1] + (Xc - 1) * ncx + ts[i1];
            wt[2 * a + i1] = ok ? ws[a] * wts[i1] : T(0);
        }
    T vr[4], vi[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        vr[j] = ec[ix[j]];
        vi[j] = ec[Nc + ix[j]];
    }
    T sr = ef[t], si = ef[Nf + t];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        sr += wt[j] * vr[j];
        si += wt[j] * vi[j];
    }
    ef[t] = sr;
    ef[Nf + t] = si;
}
template <typename T>
__global__ __launch_bounds__(256) void k_prolong2d(Geo gf, Geo gc, const T* __restrict__ ec, T* __restrict__ ef) {
    k_prolong2d_body<T>(single_block<false>(), gf, gc, ec, ef);
}
template <class PK, typename T>
__global__ __launch_bounds__(256) void k_prolong2d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_prolong2d_body<T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// 3D transfers in the same style: positions along the normal and the two
// tangential axes of the row's component, strides chosen by selects, all loads
// issued before the sums (term order of k_restrict / k_prolong).
struct FaceAxes3 {
    int n, t1, t2;        // position along normal, t1, t2
    int sn, st1, st2;     // strides of the component's face grid along them
    int dn, dt1, dt2;     // cells along normal, t1, t2
};
EHH_DEV inline FaceAxes3 face_axes3(int k, const int* p, int nx, int ny, int nz) {
    FaceAxes3 a;
    const int d0 = nx - (k == 0), d1 = ny - (k == 1);
    a.n = k == 0 ? p[0] : (k == 1 ? p[1] : p[2]);
    a.t1 = k == 0 ? p[1] : p[0];
    a.t2 = k == 2 ? p[1] : p[2];
    a.sn = k == 0 ? 1 : (k == 1 ? d0 : d0 * d1);
    a.st1 = k == 0 ? d0 : 1;
    a.st2 = k == 2 ? d0 : d0 * d1;
    a.dn = k == 0 ? nx : (k == 1 ? ny : nz);
    a.dt1 = k == 0 ? ny : nx;
    a.dt2 = k == 2 ? ny : nz;
    return a;
}
// decode a face (k < 3) or cell (k == 3) index into its position
EHH_DEV inline void pos3(int k, int li, int nx, int ny, int* p) {
    const int d0 = nx - (k == 0), d1 = ny - (k == 1);
    p[0] = li % d0;
    p[1] = (li / d0) % d1;
    p[2] = li / (d0 * d1);
    if (k == 0) p[0] += 1;
    if (k == 1) p[1] += 1;
    if (k == 2) p[2] += 1;
}

template <typename T>
EHH_DEV void k_restrict3d_body(VB ehh_vb, const Geo& gf, const Geo& gc, const T* __restrict__ rf, T* __restrict__ rc) {
    const int t = (int)(ehh_vb.x * blockDim.x + threadIdx.x);
    const int Nc = (int)gc.N, Nf = (int)gf.N;
    if (t >= Nc) return;
    rf += (int64_t)blockIdx.y * 2 * gf.N;
    rc += (int64_t)blockIdx.y * 2 * gc.N;
    const int fx = gf.n[0], fy = gf.n[1], fz = gf.n[2];
    int k = 0;
    while (k < 3 && t >= (int)gc.off[k + 1]) ++k;
    const int li = t - (int)gc.off[k];
    int P[3];
    pos3(k, li, gc.n[0], gc.n[1], P);
    T sr = T(0), si = T(0);
    if (k == 3) {   // pressure: the eight fine cells
        const int b = (int)gf.off[3] + ((2 * P[2]) * fy + 2 * P[1]) * fx + 2 * P[0];
        T vr[8], vi[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int ix = b + ((j >> 2) * fy + ((j >> 1) & 1)) * fx + (j & 1);
            vr[j] = rf[ix];
            vi[j] = rf[Nf + ix];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            sr += vr[j];
            si += vi[j];
        }
    } else {
        // fine face grid of component k, addressed from the coarse position
        const int Pf[3] = {2 * P[0], 2 * P[1], 2 * P[2]};
        const FaceAxes3 A = face_axes3(k, Pf, fx, fy, fz);
        const int base = (int)gf.off[k] + (A.n - 1) * A.sn + A.t1 * A.st1 + A.t2 * A.st2;
        T vr[48], vi[48], wt[48];
#pragma unroll
        for (int a = -1; a <= 1; ++a)
#pragma unroll
            for (int b1 = -1; b1 <= 2; ++b1)
#pragma unroll
                for (int b2 = -1; b2 <= 2; ++b2) {
                    const int j = ((a + 1) * 4 + b1 + 1) * 4 + b2 + 1;
                    const int f1 = A.t1 + b1, f2 = A.t2 + b2;
                    const bool ok = f1 >= 0 && f1 < A.dt1 && f2 >= 0 && f2 < A.dt2;
                    const int c1 = f1 < 0 ? 0 : (f1 >= A.dt1 ? A.dt1 - 1 : f1);
                    const int c2 = f2 < 0 ? 0 : (f2 >= A.dt2 ? A.dt2 - 1 : f2);
                    const int ix = base + a * A.sn + (c1 - A.t1) * A.st1 + (c2 - A.t2) * A.st2;
                    wt[j] = ok ? (a == 0 ? T(1) : T(0.5)) * T(w_tang(b1)) * T(w_tang(b2)) : T(0);
                    vr[j] = rf[ix];
                    vi[j] = rf[Nf + ix];
                }
#pragma unroll
        for (int j = 0; j < 48; ++j) {
            sr += wt[j] * vr[j];
            si += wt[j] * vi[j];
        }
    }
    rc[t] = sr;
    rc[Nc + t] = si;
}
template <typename T>
__global__ __launch_bounds__(256) void k_restrict3d(Geo gf, Geo gc, const T* __restrict__ rf, T* __restrict__ rc) {
    k_restrict3d_body<T>(single_block<false>(), gf, gc, rf, rc);
}
template <class PK, typename T>
__global__ __launch_bounds__(256) void k_restrict3d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_restrict3d_body<T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

template <typename T>
EHH_DEV void k_prolong3d_body(VB ehh_vb, const Geo& gf, const Geo& gc, const T* __restrict__ ec, T* __restrict__ ef) {
    const int t = (int)(ehh_vb.x * blockDim.x + threadIdx.x);
    const int Nc = (int)gc.N, Nf = (int)gf.N;
    if (t >= Nf) return;
    ec += (int64_t)blockIdx.y * 2 * gc.N;
    ef += (int64_t)blockIdx.y * 2 * gf.N;
    const int cx_ = gc.n[0], cy = gc.n[1], cz = gc.n[2];
    int k = 0;
    while (k < 3 && t >= (int)gf.off[k + 1]) ++k;
    const int li = t - (int)gf.off[k];
    int p[3];
    pos3(k, li, gf.n[0], gf.n[1], p);
    if (k == 3) {   // pressure: piecewise constant
        const int ci = (int)gc.off[3] + ((p[2] >> 1) * cy + (p[1] >> 1)) * cx_ + (p[0] >> 1);
        const T cr = ec[ci], cim = ec[Nc + ci];
        const T fr = ef[t], fi = ef[Nf + t];
        ef[t] = fr + cr;
        ef[Nf + t] = fi + cim;
        return;
    }
    const FaceAxes3 F = face_axes3(k, p, gf.n[0], gf.n[1], gf.n[2]);
    int pc[3] = {0, 0, 0};
    const FaceAxes3 C = face_axes3(k, pc, cx_, cy, cz);   // coarse strides and sizes
    // normal: the coincident coarse face (weight 1) or the two around it (1/2 each)
    const int xn0 = (F.n & 1) ? (F.n - 1) >> 1 : F.n >> 1, xn1 = (F.n + 1) >> 1;
    const T wn0 = (F.n & 1) ? T(0.5) : T(1), wn1 = (F.n & 1) ? T(0.5) : T(0);
    // tangential: the nearer coarse row (3/4) and the other one (1/4) inside the grid
    const int C1 = F.t1 >> 1, o1 = (F.t1 & 1) ? C1 + 1 : C1 - 1;
    const int C2 = F.t2 >> 1, o2 = (F.t2 & 1) ? C2 + 1 : C2 - 1;
    const bool ok1 = o1 >= 0 && o1 < C.dt1, ok2 = o2 >= 0 && o2 < C.dt2;
    const int xs[2] = {xn0, xn1}, y1s[2] = {C1, ok1 ? o1 : C1}, y2s[2] = {C2, ok2 ? o2 : C2};
    const T wns[2] = {wn0, wn1}, w1s[2] = {T(0.75), ok1 ? T(0.25) : T(0)}, w2s[2] = {T(0.75), ok2 ? T(0.25) : T(0)};
    T vr[8], vi[8], wt[8];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int i1 = 0; i1 < 2; ++i1)
#pragma unroll
            for (int i2 = 0; i2 < 2; ++i2) {
                const int j = (a * 2 + i1) * 2 + i2;
                const int X = xs[a];
                const bool ok = X >= 1 && X <= C.dn - 1;
                const int Xc = ok ? X : 1;
                const int ix = (int)gc.off[k] + (Xc - 1) * C.sn + y1s[i1] * C.st1 + y2s[i2] * C.st2;
                wt[j] = ok ? wns[a] * w1s[i1] * w2s[i2] : T(0);
                vr[j] = ec[ix];
                vi[j] = ec[Nc + ix];
            }
    T sr = ef[t], si = ef[Nf + t];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        sr += wt[j] * vr[j];
        si += wt[j] * vi[j];
    }
    ef[t] = sr;
    ef[Nf + t] = si;
}
template <typename T>
__global__ __launch_bounds__(256) void k_prolong3d(Geo gf, Geo gc, const T* __restrict__ ec, T* __restrict__ ef) {
    k_prolong3d_body<T>(single_block<false>(), gf, gc, ec, ef);
}
template <class PK, typename T>
__global__ __launch_bounds__(256) void k_prolong3d_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_prolong3d_body<T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// ------------------------------------------------------------------------ launchers
static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Right-hand sides per grid row: a level whose rows fill fewer than a target
// number of wavefronts (2048; 4096 for the one-thread-per-cell finest-level
// kernels, 2048 in 3D) gets its batch split over grid rows (the coefficients of
// a small level stay in cache, so re-reading them per group costs little).
static constexpr int64_t kWaves = 2048, kCellWaves = 4096, kCell3dWaves = 2048;
static inline int rhs_per_block(int64_t waves, int nrhs, int rb, int64_t target = kWaves) {
    int64_t groups = waves >= target ? 1 : (target + waves - 1) / waves;
    const int64_t maxg = (nrhs + rb - 1) / rb;
    if (groups > maxg) groups = maxg;
    if (groups < 1) groups = 1;
    int rpb = (int)((nrhs + groups - 1) / groups);
    rpb = ((rpb + rb - 1) / rb) * rb;
    return rpb < 1 ? 1 : rpb;
}
// Sources per grid row of the one-thread-per-cell kernels (groups of whole sources).
static inline int rhs_per_cells(int64_t cells, int nrhs, int64_t target) {
    int64_t groups = (target + (cells + 63) / 64 - 1) / ((cells + 63) / 64);
    groups = groups < 1 ? 1 : (groups > nrhs ? nrhs : groups);
    return (int)((nrhs + groups - 1) / groups);
}
// The autotuner's choice for a launch (tune = source groups per launch, 0: keep
// the heuristic value dflt), as sources per grid row in multiples of rb.
static inline int tuned(int tune, int nrhs, int rb, int dflt) {
    if (tune <= 0) return dflt;
    const int g = tune < nrhs ? tune : nrhs;
    int r = (nrhs + g - 1) / g;
    r = (r + rb - 1) / rb * rb;
    return r < 1 ? 1 : r;
}
// Right-hand sides evaluated together per row by the row-plan kernels (the
// fallbacks where no stored rows or one-thread-per-cell kernel serve a level):
// one per row (measured on MI355X: fewer registers, more wavefronts in flight
// outweigh the extra independent loads); the 3D Galerkin rows (93 terms) share
// each coefficient load across a block of right-hand sides.
template <typename T> static inline int rhs_block() { return 1; }
template <typename T> static inline int rhs_block_3d_stencil() { return sizeof(T) == 4 ? 4 : 2; }


#define EHH_RB_DISPATCH(RBV, CALL) \
    do {                           \
        if ((RBV) == 1) {          \
            constexpr int RB = 1;  \
            CALL;                  \
        } else if ((RBV) == 2) {   \
            constexpr int RB = 2;  \
            CALL;                  \
        } else {                   \
            constexpr int RB = 4;  \
            CALL;                  \
        }                          \
    } while (0)

template <typename T>
hipError_t launch_apply(const LevelDesc<T>& L, const T* x, const T* b, T* y, int nrhs, hipStream_t s) {
    const int64_t stride = 2 * L.g.N;
#define TUNE(V, RBV) tuned(L.tune_apply, nrhs, (RBV), (V))
    const int rb = rhs_block<T>();
    const int rpb = TUNE(rhs_per_block((L.g.N + 63) / 64, nrhs, rb), rb);
    const dim3 gb(nblk(L.g.N), (nrhs + rpb - 1) / rpb);
    const int rb3 = rhs_block_3d_stencil<T>();
    const int rpb3 = TUNE(rhs_per_block((L.g.N + 63) / 64, nrhs, rb3), rb3);
    const dim3 gb3(nblk(L.g.N), (nrhs + rpb3 - 1) / rpb3);
    const double coef_es = L.fine ? (double)sizeof(T) : (L.sp.half ? 2.0 : (double)sizeof(T));
    const LaunchBytes lb = bytes_apply(L.g, L.fine, nrhs, b != nullptr, (int)sizeof(T), coef_es);
    if (L.g.dim == 2 && L.fine && 2 * L.g.N * (int64_t)sizeof(T) < (int64_t(1) << 32)) {
        const int64_t cells = L.g.ncell;
        const int rpc = TUNE(rhs_per_cells(cells, nrhs, kCellWaves), 1);
        const dim3 gc(nblk(cells), (nrhs + rpc - 1) / rpc);
        EHH_LAUNCHK(lb, k_apply_cell2d, (T), gc, 256, 0, s, FineOp<2, T>{L.g, L.f}, x, b, y, nrhs, stride, rpc);
    } else if (L.g.dim == 2) {
        if (L.fine)
            EHH_RB_DISPATCH(rb, EHH_LAUNCHK(lb, k_apply_plan, (2, T, FineOp<2, T>, RB), gb, 256, 0, s, FineOp<2, T>{L.g, L.f}, x, b, y, nrhs, stride, rpb));
        else if (L.sp.rre) {
            if constexpr (sizeof(T) == 4)
                if (L.sp.half) {
                    EHH_LAUNCHK(lb, k_apply_st2d, (T, _Float16), gb, 256, 0, s, L.g, x, b, y, nrhs, stride, rpb,
                                (const _Float16*)L.sp.rre, (const _Float16*)L.sp.rim, (T)L.sp.scale);
                    return hipGetLastError();
                }
            EHH_LAUNCHK(lb, k_apply_st2d, (T, T), gb, 256, 0, s, L.g, x, b, y, nrhs, stride, rpb, L.sp.rre, L.sp.rim, T(1));
        }
        else
            EHH_RB_DISPATCH(rb, EHH_LAUNCHK(lb, k_apply_plan, (2, T, StOp<2, T>, RB), gb, 256, 0, s, StOp<2, T>{L.g, L.s}, x, b, y, nrhs, stride, rpb));
    } else if (L.g.dim == 3 && L.fine && 2 * L.g.N * (int64_t)sizeof(T) < (int64_t(1) << 32)) {
        const int64_t cells = L.g.ncell;
        const int rpc = TUNE(rhs_per_cells(cells, nrhs, kCellWaves), 1);
        const dim3 gc(nblk(cells), (nrhs + rpc - 1) / rpc);
        EHH_LAUNCHK(lb, k_apply_cell3d, (T), gc, 256, 0, s, FineOp<3, T>{L.g, L.f}, x, b, y, nrhs, stride, rpc);
    } else {
        if (L.fine)
            EHH_RB_DISPATCH(rb, EHH_LAUNCHK(lb, k_apply_plan, (3, T, FineOp<3, T>, RB), gb, 256, 0, s, FineOp<3, T>{L.g, L.f}, x, b, y, nrhs, stride, rpb));
        else if (L.sp.rre) {
#define EHH_APPLY_ST3D(RB, CH, C)                                                                                \
    {                                                                                                            \
        const int rpbs = TUNE(rhs_per_block((L.g.N + 63) / 64, nrhs, RB), RB);                                   \
        EHH_LAUNCHK(lb, k_apply_st3d, (T, RB, CH, C), dim3(nblk(L.g.N), (nrhs + rpbs - 1) / rpbs), 256, 0, s,   \
                           L.g, x, b, y, nrhs, stride, rpbs, (const C*)L.sp.rre, (const C*)L.sp.rim,             \
                           (T)L.sp.scale);                                                                       \
    }
            if constexpr (sizeof(T) == 8) EHH_APPLY_ST3D(2, 4, T)
            else if (L.sp.half) EHH_APPLY_ST3D(8, 4, _Float16)
            else EHH_APPLY_ST3D(8, 4, T)
#undef EHH_APPLY_ST3D
        } else
            EHH_RB_DISPATCH(rb3, EHH_LAUNCHK(lb, k_apply, (3, T, StOp<3, T>, RB), gb3, 256, 0, s, StOp<3, T>{L.g, L.s}, x, b, y, nrhs, stride, rpb3));
    }
#undef TUNE
    return hipGetLastError();
}

template <typename T>
hipError_t launch_relax(const LevelDesc<T>& L, int colour, Damp w, int econ, const T* b, const T* ein,
                        T* eout, int nrhs, hipStream_t s) {
    const int64_t stride = 2 * L.g.N;
#define TUNE(V, RBV) tuned(L.tune_relax, nrhs, (RBV), (V))
    const int64_t npair = (int64_t)(L.g.n[0] / 2) * L.g.n[1] * L.g.n[2];
    const int rb = rhs_block<T>();
    const int rpb = TUNE(rhs_per_block((npair * 8 + 63) / 64, nrhs, rb), rb);
    const dim3 gb(nblk(npair * 8), (nrhs + rpb - 1) / rpb);
    const int rb3 = rhs_block_3d_stencil<T>();
    const int rpb3 = TUNE(rhs_per_block((npair * 8 + 63) / 64, nrhs, rb3), rb3);
    const dim3 gb3(nblk(npair * 8), (nrhs + rpb3 - 1) / rpb3);
    const T tw = (T)w.u, twp = (T)w.p;
    const double coef_es = L.fine ? (double)sizeof(T) : (L.sp.half ? 2.0 : (double)sizeof(T));
    const LaunchBytes lb = bytes_relax(L.g, L.fine, nrhs, ein != nullptr, (int)sizeof(T), (int)sizeof(T), coef_es);
    // LDS staging pays on the 21-term Galerkin rows of large levels with many
    // sources (measured on 256^2 with 32 sources: 123 us, against 178 us with
    // stored row plans and 217 us with plans built in the kernel); with a few
    // sources the stored plans win (one FP64 source: 30 us against 53 us), and at
    // 128^2 and below the block-wide synchronisation costs more than it saves.
    const bool big_batch = !(L.sp.re[colour] && nrhs <= 8);
    const int lds_tiles = ((L.g.n[0] + LT_X - 1) / LT_X) * ((L.g.n[1] + LT_Y - 1) / LT_Y);
    const int rpl = TUNE(rhs_per_block((int64_t)lds_tiles * 8, nrhs, 1), 1);
    if (L.g.dim == 2 && !L.fine && L.g.ncell >= 65536 && rpl * stride * (int64_t)sizeof(T) < (int64_t(1) << 31) &&
        big_batch) {
        const int tiles = lds_tiles;
        const dim3 gl(tiles, (nrhs + rpl - 1) / rpl);
        EHH_LAUNCHK(lb, k_relax_lds2d, (T, StOp<2, T>), gl, 512, 0, s, StOp<2, T>{L.g, L.s}, colour, tw, twp, econ, b, ein, eout, nrhs, stride, rpl, 2);
    } else if (L.g.dim == 2 && L.fine && 2 * L.g.N * (int64_t)sizeof(T) < (int64_t(1) << 32)) {
        const int64_t cells = npair;
        const int rpc = TUNE(rhs_per_cells(cells, nrhs, kCellWaves), 1);
        const dim3 gc(nblk(cells), (nrhs + rpc - 1) / rpc);
        EHH_LAUNCHK(lb, k_relax_cell2d, (T), gc, 256, 0, s, FineOp<2, T>{L.g, L.f}, colour, tw, twp, econ, b, ein, eout, nrhs, stride, rpc);
    } else if (L.g.dim == 2) {
        if (L.fine)
            EHH_RB_DISPATCH(rb, EHH_LAUNCHK(lb, k_relax_plan, (2, T, FineOp<2, T>, RB), gb, 256, 0, s, FineOp<2, T>{L.g, L.f}, colour, tw, twp, econ, b, ein, eout, nrhs, stride, rpb));
        else if (L.sp.re[colour])
        {
            // the smallest FP64 levels (one wavefront per CU): rows split over two
            // wavefronts, one batch of loads per row instead of three (measured on
            // MI355X: 64^2 5.4 -> 4.8 us; no gain at 128^2)
            const int64_t groups = L.sp.lanes / 64;
            if (sizeof(T) == 8 && ein && groups <= 256)
                EHH_LAUNCHK(lb, k_relax_st2d_split, (T), dim3((unsigned)((groups + 1) / 2), gb.y), 256, 0, s, L.g, colour, tw, twp, econ, b, ein, eout, nrhs, stride, rpb, L.sp.re[colour], L.sp.im[colour], L.sp.lanes);
            else {
                bool half = false;
                if constexpr (sizeof(T) == 4)
                    if (L.sp.half) {
                        EHH_LAUNCHK(lb, k_relax_st2d, (T, true, false, _Float16), gb, 256, 0, s, L.g, colour, tw, twp, econ, b, ein, eout, nrhs, stride, rpb, (const _Float16*)L.sp.re[colour], (const _Float16*)L.sp.im[colour], L.sp.lanes, L.g, (const T*)nullptr, (T*)nullptr, (T)L.sp.scale);
                        half = true;
                    }
                if (!half)
                    EHH_LAUNCHK(lb, k_relax_st2d, (T, sizeof(T) == 4, false, T), gb, 256, 0, s, L.g, colour, tw, twp, econ, b, ein, eout, nrhs, stride, rpb, L.sp.re[colour], L.sp.im[colour], L.sp.lanes, L.g, (const T*)nullptr, (T*)nullptr, T(1));
            }
        }
        else
            EHH_RB_DISPATCH(rb, EHH_LAUNCHK(lb, k_relax_plan, (2, T, StOp<2, T>, RB), gb, 256, 0, s, StOp<2, T>{L.g, L.s}, colour, tw, twp, econ, b, ein, eout, nrhs, stride, rpb));
    } else if (L.fine && 2 * L.g.N * (int64_t)sizeof(T) < (int64_t(1) << 32)) {
        const int64_t cells = npair;
        // one source group (16 sources per thread) beat two on the 72^3 subdomains:
        // the 7 x 7 block inverse is then formed once per cell (c4 solve 8.60 -> 8.51 s)
        const int rpc = TUNE(rhs_per_cells(cells, nrhs, kCell3dWaves), 1);
        const dim3 gc(nblk(cells), (nrhs + rpc - 1) / rpc);
        EHH_LAUNCHK(lb, k_relax_cell3d, (T), gc, 256, 0, s, FineOp<3, T>{L.g, L.f}, colour, tw, twp, econ, b, ein, eout, nrhs, stride, rpc);
    } else {
        if (L.fine)
            EHH_RB_DISPATCH(rb, EHH_LAUNCHK(lb, k_relax_plan, (3, T, FineOp<3, T>, RB), gb, 256, 0, s, FineOp<3, T>{L.g, L.f}, colour, tw, twp, econ, b, ein, eout, nrhs, stride, rpb));
        else if (L.sp.re[colour]) {
#define EHH_RELAX_ST3D(RB, CH, C)                                                                                 \
    {                                                                                                             \
        const int rpbs = TUNE(rhs_per_block((npair * 8 + 63) / 64, nrhs, RB, 4096), RB);                          \
        EHH_LAUNCHK(lb, k_relax_st3d, (T, RB, CH, C), dim3(nblk(npair * 8), (nrhs + rpbs - 1) / rpbs), 256, 0,  \
                           s, L.g, colour, tw, twp, econ, b, ein, eout, nrhs, stride, rpbs, (const C*)L.sp.re[colour], \
                           (const C*)L.sp.im[colour], L.sp.lanes, (T)L.sp.scale);                                 \
    }
            // measured on MI355X (36^3 level, 16 FP32 sources): 8 sources per
            // coefficient load in chunks of 8 terms 284 us, of 4 terms 299 us;
            // source groups sized for 4096 wavefronts (two groups of 8 there)
            // 273 us against 284 us for 2048 (one group of 16)
            // (both two wavefronts per SIMD); with the row-loop addresses held
            // across the loop (one wavefront per SIMD) 8 x 4 took 331 us, 8 x 2
            // 335 us, 4 x 4 358 us, 16 x 2 322 us but 2x slower on 18^3
            if constexpr (sizeof(T) == 8) EHH_RELAX_ST3D(2, 4, T)
            else if (L.sp.half) EHH_RELAX_ST3D(8, 8, _Float16)
            else EHH_RELAX_ST3D(8, 8, T)
#undef EHH_RELAX_ST3D
        } else
            EHH_RB_DISPATCH(rb3, EHH_LAUNCHK(lb, k_relax, (3, T, StOp<3, T>, RB), gb3, 256, 0, s, StOp<3, T>{L.g, L.s}, colour, tw, twp, econ, b, ein, eout, nrhs, stride, rpb3));
    }
#undef TUNE
    return hipGetLastError();
}

// Colour-1 half-sweep of the finest 2D level writing e_out in FP64 (the last
// half-sweep of a complex64 cycle); false where that level is not served by the
// one-thread-per-cell kernel.
hipError_t launch_relax_to64(const LevelDesc<float>& L, Damp w, int econ, const float* b, const float* ein,
                             double* eout, int nrhs, hipStream_t s, bool* done) {
    *done = false;
    if (!(L.g.dim == 2 && L.fine && 2 * L.g.N * (int64_t)sizeof(double) < (int64_t(1) << 32)))
        return hipSuccess;
    const int64_t stride = 2 * L.g.N;
    const int64_t cells = (int64_t)(L.g.n[0] / 2) * L.g.n[1];
    const int rpc = tuned(L.tune_relax, nrhs, 1, rhs_per_cells(cells, nrhs, kCellWaves));
    const dim3 gc(nblk(cells), (nrhs + rpc - 1) / rpc);
    EHH_LAUNCHK(bytes_relax(L.g, true, nrhs, true, 4, 8, 4.0), k_relax_cell2d, (float, double), gc, 256, 0, s,
                 FineOp<2, float>{L.g, L.f}, 1, (float)w.u, (float)w.p, econ, b, ein, eout, nrhs, stride, rpc);
    *done = true;
    return hipGetLastError();
}

template <typename T>
bool relax_restrict_supported(const LevelDesc<T>& L, const Geo& gf, int nrhs) {
    if (L.g.dim != 2 || L.fine || !L.sp.re[0]) return false;
    // the finer level's residual is read through a buffer descriptor
    if (2 * gf.N * (int64_t)sizeof(T) >= (int64_t(1) << 32)) return false;
    // same routing as launch_relax: the LDS kernel serves large levels with many sources
    return !(L.g.ncell >= 65536 && nrhs > 8);
}
template <typename T>
hipError_t launch_relax_restrict(const LevelDesc<T>& L, Damp w, int econ, const Geo& gf, const T* rf, T* b,
                                 T* eout, int nrhs, hipStream_t s) {
    const int64_t stride = 2 * L.g.N;
    const int64_t npair = (int64_t)(L.g.n[0] / 2) * L.g.n[1] * L.g.n[2];
    const int rpb = tuned(L.tune_relax, nrhs, 1, rhs_per_block((npair * 8 + 63) / 64, nrhs, 1));
    const dim3 gb(nblk(npair * 8), (nrhs + rpb - 1) / rpb);
    LaunchBytes lb = bytes_relax(L.g, false, nrhs, false, (int)sizeof(T), (int)sizeof(T), L.sp.half ? 2.0 : (double)sizeof(T));
    lb.mine += nrhs * 2.0 * sizeof(T) * (double)(gf.N + L.g.N);              // rf read, b written
    lb.model += nrhs * 2.0 * sizeof(T) * (gf.dim + 1) * (double)(gf.ncell + L.g.ncell);
    if constexpr (sizeof(T) == 4)
        if (L.sp.half) {
            EHH_LAUNCHK(lb, k_relax_st2d, (T, true, true, _Float16), gb, 256, 0, s, L.g, 0, (T)w.u, (T)w.p, econ,
                        (const T*)b, (const T*)nullptr, eout, nrhs, stride, rpb, (const _Float16*)L.sp.re[0],
                        (const _Float16*)L.sp.im[0], L.sp.lanes, gf, rf, b, (T)L.sp.scale);
            return hipGetLastError();
        }
    EHH_LAUNCHK(lb, k_relax_st2d, (T, sizeof(T) == 4, true, T), gb, 256, 0, s, L.g, 0, (T)w.u, (T)w.p, econ,
                (const T*)b, (const T*)nullptr, eout, nrhs, stride, rpb, L.sp.re[0], L.sp.im[0], L.sp.lanes, gf, rf,
                b, T(1));
    return hipGetLastError();
}
template bool relax_restrict_supported<float>(const LevelDesc<float>&, const Geo&, int);
template bool relax_restrict_supported<double>(const LevelDesc<double>&, const Geo&, int);
template hipError_t launch_relax_restrict<float>(const LevelDesc<float>&, Damp, int, const Geo&, const float*,
                                                 float*, float*, int, hipStream_t);
template hipError_t launch_relax_restrict<double>(const LevelDesc<double>&, Damp, int, const Geo&, const double*,
                                                  double*, double*, int, hipStream_t);

int64_t stored_plan_lanes(const Geo& g) {
    const int64_t npair = (int64_t)(g.n[0] / 2) * g.n[1] * g.n[2];
    return (int64_t)nblk(npair * 8) * 256;
}
// Every Galerkin level keeps its rows (the large 2D ones use them for small
// batches, see launch_relax).
bool stored_plan_wanted(const Geo& g, bool fine) {
    // the kernels address the stored rows and the vectors with 32-bit byte offsets
    // (2D: below 2 GiB, which keeps the pressure rows' skipped slots out of range)
    const int64_t NT = g.dim == 2 ? St<2>::NF + St<2>::NUP : St<3>::NF + St<3>::NUP;
    const int64_t lim = g.dim == 2 ? int64_t(1) << 31 : int64_t(1) << 32;
    return !fine && NT * stored_plan_lanes(g) * 8 < lim && NT * g.N * 8 < lim &&
           16 * g.N < lim;
}
int stored_terms(int dim) { return dim == 2 ? St<2>::NF + St<2>::NUP : St<3>::NF + St<3>::NUP; }
int stored_imag_terms(int dim) { return dim == 2 ? St<2>::NF : St<3>::NF; }
template <typename T>
hipError_t launch_build_plans(const LevelDesc<T>& L, int colour, T* re, T* im, hipStream_t s) {
    const int64_t lanes = stored_plan_lanes(L.g);
    if (L.g.dim == 2)
        EHH_LAUNCH((k_build_plans<T>), nblk(lanes), 256, 0, s, StOp<2, T>{L.g, L.s}, colour, re, im, lanes);
    else
        EHH_LAUNCH((k_build_rows3d<T>), nblk(lanes * stored_terms(3)), 256, 0, s, StOp<3, T>{L.g, L.s},
                           colour, re, im, lanes);
    return hipGetLastError();
}
template <typename T>
hipError_t launch_build_row_plans(const LevelDesc<T>& L, T* re, T* im, hipStream_t s) {
    if (L.g.dim == 2)
        EHH_LAUNCH((k_build_row_plans<T>), nblk(L.g.N), 256, 0, s, StOp<2, T>{L.g, L.s}, re, im);
    else
        EHH_LAUNCH((k_build_row_rows3d<T>), nblk(L.g.N * stored_terms(3)), 256, 0, s, StOp<3, T>{L.g, L.s},
                           re, im);
    return hipGetLastError();
}
template hipError_t launch_build_row_plans<float>(const LevelDesc<float>&, float*, float*, hipStream_t);
template hipError_t launch_build_row_plans<double>(const LevelDesc<double>&, double*, double*, hipStream_t);
template hipError_t launch_build_plans<float>(const LevelDesc<float>&, int, float*, float*, hipStream_t);
template hipError_t launch_build_plans<double>(const LevelDesc<double>&, int, double*, double*, hipStream_t);

template <typename T>
hipError_t launch_restrict(const Geo& gf, const Geo& gc, const T* rf, T* rc, int nrhs, hipStream_t s) {
    // (k_restrict2d reads the fine vector through a buffer descriptor: below 4 GiB)
    if (gf.dim == 2 && 2 * gf.N * (int64_t)sizeof(T) < (int64_t(1) << 32))
        EHH_LAUNCHK(bytes_transfer(gf, gc, nrhs, false, (int)sizeof(T)), k_restrict2d, (T), dim3(nblk(gc.N), nrhs), 256, 0, s, gf, gc, rf, rc);
    else if (gf.dim == 2)
        EHH_LAUNCHK(bytes_transfer(gf, gc, nrhs, false, (int)sizeof(T)), k_restrict, (2, T), dim3(nblk(gc.N), nrhs), 256, 0, s, gf, gc, rf, rc, nrhs);
    else if (2 * gf.N < (int64_t(1) << 31))
        EHH_LAUNCHK(bytes_transfer(gf, gc, nrhs, false, (int)sizeof(T)), k_restrict3d, (T), dim3(nblk(gc.N), nrhs), 256, 0, s, gf, gc, rf, rc);
    else
        EHH_LAUNCHK(bytes_transfer(gf, gc, nrhs, false, (int)sizeof(T)), k_restrict, (3, T), dim3(nblk(gc.N), nrhs), 256, 0, s, gf, gc, rf, rc, nrhs);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(const Geo& gf, const Geo& gc, const T* ec, T* ef, int nrhs, hipStream_t s) {
    if (gf.dim == 2 && 2 * gf.N < (int64_t(1) << 31))
        EHH_LAUNCHK(bytes_transfer(gf, gc, nrhs, true, (int)sizeof(T)), k_prolong2d, (T), dim3(nblk(gf.N), nrhs), 256, 0, s, gf, gc, ec, ef);
    else if (gf.dim == 2)
        EHH_LAUNCHK(bytes_transfer(gf, gc, nrhs, true, (int)sizeof(T)), k_prolong, (2, T), dim3(nblk(gf.N), nrhs), 256, 0, s, gf, gc, ec, ef, nrhs);
    else if (2 * gf.N < (int64_t(1) << 31))
        EHH_LAUNCHK(bytes_transfer(gf, gc, nrhs, true, (int)sizeof(T)), k_prolong3d, (T), dim3(nblk(gf.N), nrhs), 256, 0, s, gf, gc, ec, ef);
    else
        EHH_LAUNCHK(bytes_transfer(gf, gc, nrhs, true, (int)sizeof(T)), k_prolong, (3, T), dim3(nblk(gf.N), nrhs), 256, 0, s, gf, gc, ec, ef, nrhs);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_residual_restrict(const LevelDesc<T>& L, const Geo& gc, const T* e, const T* b, T* rc, int nrhs,
                                    hipStream_t s, bool* done) {
    *done = false;
    // one launch pays with few sources (c2, one FP64 source: 114.6 -> 113.1 ms per
    // solve); a lane walks its sources in turn, so with 32 sources the separate
    // residual and restriction, which spread them over more lanes, are faster
    if (L.g.dim != 2 || L.fine || !L.sp.rre || L.sp.half || nrhs > 4) return hipSuccess;
    LaunchBytes lb = bytes_apply(L.g, false, nrhs, true, (int)sizeof(T), (double)sizeof(T));
    const LaunchBytes rb = bytes_transfer(L.g, gc, nrhs, false, (int)sizeof(T));
    lb.mine += nrhs * 2.0 * sizeof(T) * ((double)gc.N - (double)L.g.N);   // rc written, r never written
    lb.model += rb.model - nrhs * 2.0 * sizeof(T) * (L.g.dim + 1) * 2.0 * (double)L.g.ncell;
    EHH_LAUNCHK(lb, k_residual_restrict2d, (T), nblk((int64_t)gc.N * 16), 256, 0, s, L.g, gc, e, b, rc, nrhs,
                 L.sp.rre, L.sp.rim);
    *done = true;
    return hipGetLastError();
}
template hipError_t launch_residual_restrict<float>(const LevelDesc<float>&, const Geo&, const float*, const float*,
                                                    float*, int, hipStream_t, bool*);
template hipError_t launch_residual_restrict<double>(const LevelDesc<double>&, const Geo&, const double*,
                                                     const double*, double*, int, hipStream_t, bool*);

// FP16 copies of stored rows: max |x| over the rows (the bit patterns of
// non-negative floats order as integers, so an integer maximum is exact), then
// x / scale rounded to FP16, scale = a power of two that brings the largest
// modulus to about 2^14 (FP16 overflows at 65504).
__global__ __launch_bounds__(256) void k_absmax_bits(const float* __restrict__ x, int64_t n,
                                                     unsigned* __restrict__ out) {
    unsigned m = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned v = __float_as_uint(fabsf(x[i]));
        m = v > m ? v : m;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned v = __shfl_xor(m, o, 64);
        m = v > m ? v : m;
    }
    if ((threadIdx.x & 63) == 0 && m) atomicMax(out, m);
}
__global__ __launch_bounds__(256) void k_to_half(const float* __restrict__ x, _Float16* __restrict__ y, int64_t n,
                                                 float inv_scale) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (_Float16)(x[i] * inv_scale);
}
hipError_t launch_absmax_bits(const float* x, int64_t n, unsigned* out, hipStream_t s) {
    const int64_t nb = std::min<int64_t>(1024, (n + 255) / 256);
    EHH_LAUNCH(k_absmax_bits, (unsigned)(nb < 1 ? 1 : nb), 256, 0, s, x, n, out);
    return hipGetLastError();
}
hipError_t launch_to_half(const float* x, void* y, int64_t n, float inv_scale, hipStream_t s) {
    EHH_LAUNCH(k_to_half, nblk(n), 256, 0, s, x, (_Float16*)y, n, inv_scale);
    return hipGetLastError();
}

// y = A x on a finest level with x in FP32 and A, y in FP64 (the FGMRES product
// of the complex64 cycle's output, kept in FP32; each x entry is exact in FP64).
bool apply_x32_supported(const LevelDesc<double>& L) {
    return L.fine && (L.g.dim == 2 || L.g.dim == 3) && 2 * L.g.N * (int64_t)sizeof(double) < (int64_t(1) << 32);
}
hipError_t launch_apply_x32(const LevelDesc<double>& L, const float* x, double* y, int nrhs, hipStream_t s) {
    if (!apply_x32_supported(L)) return hipErrorInvalidValue;
    const int64_t stride = 2 * L.g.N;
    const int64_t cells = L.g.ncell;
    const int rpc = tuned(L.tune_apply, nrhs, 1, rhs_per_cells(cells, nrhs, kCellWaves));
    const dim3 gc(nblk(cells), (nrhs + rpc - 1) / rpc);
    LaunchBytes lb = bytes_apply(L.g, true, nrhs, false, (int)sizeof(double), (double)sizeof(double));
    lb.mine -= nrhs * L.g.N * 2.0 * (sizeof(double) - sizeof(float));   // x in FP32
    lb.model -= nrhs * (double)L.g.ncell * (L.g.dim + 1) * 2.0 * (sizeof(double) - sizeof(float));
    if (L.g.dim == 2)
        EHH_LAUNCH_B(lb, (k_apply_cell2d<double, float>), gc, 256, 0, s, FineOp<2, double>{L.g, L.f}, x,
                     (const double*)nullptr, y, nrhs, stride, rpc);
    else
        EHH_LAUNCH_B(lb, (k_apply_cell3d<double, float>), gc, 256, 0, s, FineOp<3, double>{L.g, L.f}, x,
                     (const double*)nullptr, y, nrhs, stride, rpc);
    return hipGetLastError();
}

#define EHH_INST(T)                                                                                       \
    template hipError_t launch_apply<T>(const LevelDesc<T>&, const T*, const T*, T*, int, hipStream_t);  \
    template hipError_t launch_relax<T>(const LevelDesc<T>&, int, Damp, int, const T*, const T*, T*,      \
                                        int, hipStream_t);                                               \
    template hipError_t launch_restrict<T>(const Geo&, const Geo&, const T*, T*, int, hipStream_t);      \
    template hipError_t launch_prolong<T>(const Geo&, const Geo&, const T*, T*, int, hipStream_t);
EHH_INST(float)
EHH_INST(double)

}  // namespace ehh
