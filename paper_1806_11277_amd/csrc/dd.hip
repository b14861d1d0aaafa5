// Domain-decomposition transfers between the global FP64 vectors of the outer
// Krylov method and the padded local vectors of the subdomain cycles (section
// 2.3, section 4): restriction of the residual to a subdomain (zero in its
// absorbing padding, cast to the cycle precision) and extension of the local
// correction back to the global vector, either averaged over the subdomains
// that own an unknown (one colour) or added unweighted (Algorithm 2).
#include "internal.hpp"
#include "launchlog.hpp"
#include "batch.hpp"
#include "ops.hpp"

namespace ehh {

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

// Global index of the local unknown t (component k, local position), or -1 when
// it lies outside the subdomain's extent [lo, hi).  A face belongs to the
// extent when both adjacent cells do.  *w receives the owner count product.
template <int D>
EHH_DEV int64_t local_to_global(const Geo& gg, const Geo& gl, const SubMap& m, int64_t t, int& k, int* cnt) {
    k = 0;
    while (k < 3 && t >= gl.off[k + 1]) ++k;
    if (k >= D) k = 3;
    const int64_t li = t - gl.off[k];
    int p[3];
    if (k == 3) cell_pos<D>(gl, li, p);
    else face_pos<D>(gl, k, li, p);
    int c = 1;
    for (int a = 0; a < D; ++a) {
        const int gp = p[a] + m.origin[a];
        if (a == k) {
            if (!(gp > m.lo[a] && gp < m.hi[a])) return -1;
            c *= m.cnt_face[a][gp];
        } else {
            if (!(gp >= m.lo[a] && gp < m.hi[a])) return -1;
            c *= m.cnt_cell[a][gp];
        }
        p[a] = gp;
    }
    *cnt = c;
    return k == 3 ? gg.off[3] + cell_idx<D>(gg, p) : gg.off[k] + face_idx<D>(gg, k, p);
}

template <int D, typename T>
EHH_DEV void k_dd_gather_body(VB ehh_vb, const Geo& gg, const Geo& gl, const SubMap& m, const double* __restrict__ v, T* __restrict__ out, int nrhs) {
    const int64_t t = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (t >= gl.N) return;
    int k, cnt;
    const int64_t gi = local_to_global<D>(gg, gl, m, t, k, &cnt);
    for (int r = 0; r < nrhs; ++r) {
        T* o = out + (int64_t)r * 2 * gl.N;
        const double* vv = v + (int64_t)r * 2 * gg.N;
        o[t] = gi >= 0 ? (T)vv[gi] : T(0);
        o[gl.N + t] = gi >= 0 ? (T)vv[gg.N + gi] : T(0);
    }
}
template <int D, typename T>
__global__ __launch_bounds__(256) void k_dd_gather(Geo gg, Geo gl, SubMap m, const double* __restrict__ v,
                                                   T* __restrict__ out, int nrhs) {
    k_dd_gather_body<D, T>(single_block<false>(), gg, gl, m, v, out, nrhs);
}
template <class PK, int D, typename T>
__global__ __launch_bounds__(256) void k_dd_gather_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_dd_gather_body<D, T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

template <int D, typename T>
EHH_DEV void k_dd_scatter_body(VB ehh_vb, const Geo& gg, const Geo& gl, const SubMap& m, const T* __restrict__ e, double* __restrict__ z, int nrhs, int weighted) {
    const int64_t t = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (t >= gl.N) return;
    int k, cnt;
    const int64_t gi = local_to_global<D>(gg, gl, m, t, k, &cnt);
    if (gi < 0) return;
    const double w = weighted ? 1.0 / cnt : 1.0;
    for (int r = 0; r < nrhs; ++r) {
        const T* ee = e + (int64_t)r * 2 * gl.N;
        double* zz = z + (int64_t)r * 2 * gg.N;
        zz[gi] += w * (double)ee[t];
        zz[gg.N + gi] += w * (double)ee[gl.N + t];
    }
}
template <int D, typename T>
__global__ __launch_bounds__(256) void k_dd_scatter(Geo gg, Geo gl, SubMap m, const T* __restrict__ e,
                                                    double* __restrict__ z, int nrhs, int weighted) {
    k_dd_scatter_body<D, T>(single_block<false>(), gg, gl, m, e, z, nrhs, weighted);
}
template <class PK, int D, typename T>
__global__ __launch_bounds__(256) void k_dd_scatter_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_dd_scatter_body<D, T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

template <typename T>
hipError_t launch_dd_gather(const Geo& gg, const Geo& gl, const SubMap& m, const double* v, T* out, int nrhs,
                            hipStream_t s) {
    if (gg.dim == 2)
        EHH_LAUNCHK(bytes_plain(nrhs * (double)gl.N * (16.0 + 2.0 * sizeof(T))), k_dd_gather, (2, T), nblk(gl.N), 256, 0, s, gg, gl, m, v, out, nrhs);
    else
        EHH_LAUNCHK(bytes_plain(nrhs * (double)gl.N * (16.0 + 2.0 * sizeof(T))), k_dd_gather, (3, T), nblk(gl.N), 256, 0, s, gg, gl, m, v, out, nrhs);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dd_scatter(const Geo& gg, const Geo& gl, const SubMap& m, const T* e, double* z, int nrhs,
                             int weighted, hipStream_t s) {
    if (gg.dim == 2)
        EHH_LAUNCHK(bytes_plain(nrhs * (double)gl.N * (32.0 + 2.0 * sizeof(T))), k_dd_scatter, (2, T), nblk(gl.N), 256, 0, s, gg, gl, m, e, z, nrhs, weighted);
    else
        EHH_LAUNCHK(bytes_plain(nrhs * (double)gl.N * (32.0 + 2.0 * sizeof(T))), k_dd_scatter, (3, T), nblk(gl.N), 256, 0, s, gg, gl, m, e, z, nrhs, weighted);
    return hipGetLastError();
}

template hipError_t launch_dd_gather<float>(const Geo&, const Geo&, const SubMap&, const double*, float*, int,
                                            hipStream_t);
template hipError_t launch_dd_gather<double>(const Geo&, const Geo&, const SubMap&, const double*, double*, int,
                                             hipStream_t);
template hipError_t launch_dd_scatter<float>(const Geo&, const Geo&, const SubMap&, const float*, double*, int, int,
                                             hipStream_t);
template hipError_t launch_dd_scatter<double>(const Geo&, const Geo&, const SubMap&, const double*, double*, int,
                                              int, hipStream_t);

// Algorithm 2, step 1: the local residual r_i = q_i - (A u)_{Omega_i} of the
// global (unshifted) operator, evaluated only at the unknowns of the
// subdomain's extent and written straight into its padded local vector.
// Blocks are renumbered per XCD: a row's stencil reads the global rows of its
// neighbouring blocks, which then sit in the same L2 (on 72^3 subdomains with 16
// sources 427 -> 407 us; the plain gather, the scatter and the 3D transfers
// measured slower with the renumbering and keep the hardware order).
template <int D, typename T>
EHH_DEV void k_dd_gather_res_body(VB ehh_vb, const Geo& gg, const Geo& gl, const SubMap& m, const FineCoef<double>& A, const double* __restrict__ v, const double* __restrict__ z, T* __restrict__ out, int nrhs) {
    const int64_t t = (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (t >= gl.N) return;
    int k, cnt;
    const int64_t gi = local_to_global<D>(gg, gl, m, t, k, &cnt);
    int p[3] = {0, 0, 0};
    if (gi >= 0) {
        if (k == 3) cell_pos<D>(gg, gi - gg.off[3], p);
        else face_pos<D>(gg, k, gi - gg.off[k], p);
    }
    const FineOp<D, double> op{gg, A};
    // the row (its few terms and weights) is built once and applied to every
    // right-hand side, four at a time so that their loads are in flight together
    using Op = FineOp<D, double>;
    Plan<double, Op::NT> P;
    if (gi >= 0) {
        // one call per component with a constant index, so that the row's local
        // position arrays stay in registers (a runtime index puts them in scratch)
        if (k == 0) op.plan_u(0, p, P);
        else if (k == 1) op.plan_u(1, p, P);
        else if (D == 3 && k == 2) op.plan_u(2, p, P);
        else op.plan_p(p, P);
    }
    // 32-bit byte offsets into per-source buffer descriptors (a global vector
    // stays below 4 GiB, checked by the launcher) instead of a 64-bit address
    // per term and source
    uint32_t zo[Op::NT];
#pragma unroll
    for (int j = 0; j < Op::NT; ++j) zo[j] = (uint32_t)P.ix[j] * 8u;
    const uint32_t vo = gi >= 0 ? (uint32_t)gi * 8u : 0u;
    const uint32_t NB = (uint32_t)gg.N * 8u, VB = 2u * NB;
    constexpr int RB = 4;
    for (int r0 = 0; r0 < nrhs; r0 += RB) {
        cx<double> az[RB], vz[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            const int r = r0 + q < nrhs ? r0 + q : r0;
            az[q] = vz[q] = mk<double>(0.0, 0.0);
            if (gi >= 0) {
                const Buf<double> zb(z + (int64_t)r * 2 * gg.N, VB), vb(v + (int64_t)r * 2 * gg.N, VB);
                double ar = 0.0, ai = 0.0;   // the sum of Plan::dot, in its order
#pragma unroll
                for (int j = 0; j < Op::NT; ++j) {
                    const double er = zb.ld(zo[j], 0), ei = zb.ld(zo[j], NB);
                    ar += P.re[j] * er - P.im[j] * ei;
                    ai += P.re[j] * ei + P.im[j] * er;
                }
                az[q] = mk<double>(ar, ai);
                vz[q] = mk<double>(vb.ld(vo, 0), vb.ld(vo, NB));
            }
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            if (r0 + q >= nrhs) break;
            T* o = out + (int64_t)(r0 + q) * 2 * gl.N;
            o[t] = (T)(vz[q].re - az[q].re);
            o[gl.N + t] = (T)(vz[q].im - az[q].im);
        }
    }
}
template <int D, typename T>
__global__ __launch_bounds__(256) void k_dd_gather_res(Geo gg, Geo gl, SubMap m, FineCoef<double> A,
                                                       const double* __restrict__ v, const double* __restrict__ z,
                                                       T* __restrict__ out, int nrhs) {
    k_dd_gather_res_body<D, T>(single_block<true>(), gg, gl, m, A, v, z, out, nrhs);
}
template <class PK, int D, typename T>
__global__ __launch_bounds__(256) void k_dd_gather_res_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<true>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_dd_gather_res_body<D, T>(ehh_vb, a...); }, b.arg[ehh_s]);
}

template <typename T>
hipError_t launch_dd_gather_res(const Geo& gg, const Geo& gl, const SubMap& m, const FineCoef<double>& A,
                                const double* v, const double* z, T* out, int nrhs, hipStream_t s) {
    if (16 * gg.N >= (int64_t(1) << 32)) return hipErrorInvalidValue;   // 32-bit byte offsets per source
    if (gg.dim == 2)
        EHH_LAUNCHK(bytes_plain(nrhs * (double)gl.N * (32.0 + 2.0 * sizeof(T)) + 32.0 * gl.ncell), k_dd_gather_res, (2, T), nblk(gl.N), 256, 0, s, gg, gl, m, A, v, z, out, nrhs);
    else
        EHH_LAUNCHK(bytes_plain(nrhs * (double)gl.N * (32.0 + 2.0 * sizeof(T)) + 32.0 * gl.ncell), k_dd_gather_res, (3, T), nblk(gl.N), 256, 0, s, gg, gl, m, A, v, z, out, nrhs);
    return hipGetLastError();
}
template hipError_t launch_dd_gather_res<float>(const Geo&, const Geo&, const SubMap&, const FineCoef<double>&,
                                                const double*, const double*, float*, int, hipStream_t);
template hipError_t launch_dd_gather_res<double>(const Geo&, const Geo&, const SubMap&, const FineCoef<double>&,
                                                 const double*, const double*, double*, int, hipStream_t);

}  // namespace ehh

// ------------------------------------------------ DD as the coarsest-grid solver
// The subdomains ("boxes") of the coarsest level of one hierarchy have their
// unknowns numbered one box after the other; local unknown j of box b (starting
// at bbase[b], bn[b] unknowns) is the coarsest unknown map[j].  A box's local
// vectors are stored like any level vector of its own grid: for source r the
// real plane then the imaginary plane, at loc + 2 nrhs bbase[b] + 2 bn[b] r.

namespace ehh {

// Copy the coarsest stencil of every face and cell of a box (cells [lo, hi) of
// grid gc) into the stencil arrays of the box's own grid gb.  Couplings of the
// copied rows that leave the box are simply not reached from the box's grid,
// which restricts the operator to the box.
template <int D>
__global__ __launch_bounds__(256) void k_box_stencil(Geo gc, StCoef<double> sc, Geo gb, StCoef<double> sb, int lo0,
                                                     int lo1, int lo2) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= gb.N) return;
    const int lo[3] = {lo0, lo1, lo2};
    int k = 0;
    while (k < 3 && t >= gb.off[k + 1]) ++k;
    if (k >= D) k = 3;
    const int64_t li = t - gb.off[k];
    int p[3];
    if (k == 3) {
        cell_pos<D>(gb, li, p);
        for (int a = 0; a < D; ++a) p[a] += lo[a];
        ((double*)sb.pp)[li] = sc.pp[cell_idx<D>(gc, p)];
        return;
    }
    face_pos<D>(gb, k, li, p);
    for (int a = 0; a < D; ++a) p[a] += lo[a];
    const int64_t gi = face_idx<D>(gc, k, p);
    for (int q = 0; q < 2 * St<D>::NUU; ++q)
        ((double*)sb.uu[k])[(int64_t)q * gb.cnt[k] + li] = sc.uu[k][(int64_t)q * gc.cnt[k] + gi];
    for (int q = 0; q < St<D>::NUP; ++q)
        ((double*)sb.up[k])[(int64_t)q * gb.cnt[k] + li] = sc.up[k][(int64_t)q * gc.cnt[k] + gi];
}

hipError_t launch_box_stencil(const Geo& gc, const double* stc, const Geo& gb, double* stb, const int* lo,
                              hipStream_t s) {
    if (gc.dim == 2)
        EHH_LAUNCH((k_box_stencil<2>), nblk(gb.N), 256, 0, s, gc, stencil_view<2, double>(gc, stc), gb,
                   stencil_view<2, double>(gb, (const double*)stb), lo[0], lo[1], lo[2]);
    else
        EHH_LAUNCH((k_box_stencil<3>), nblk(gb.N), 256, 0, s, gc, stencil_view<3, double>(gc, stc), gb,
                   stencil_view<3, double>(gb, (const double*)stb), lo[0], lo[1], lo[2]);
    return hipGetLastError();
}

// loc(box) <- src restricted to the box, for the local unknowns [j0, j1)
template <int Z = 0>
EHH_DEV void k_box_gather_body(VB ehh_vb, const int* __restrict__ map, const int* __restrict__ bsub, const int64_t* __restrict__ bbase, const int* __restrict__ bn, int64_t j0, int64_t j1, const double* __restrict__ src, int64_t Nc, double* __restrict__ loc, int nrhs) {
    const int64_t j = j0 + (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (j >= j1) return;
    const int b = bsub[j];
    const int64_t base = bbase[b], n = bn[b], li = j - base, g = map[j];
    double* o = loc + 2 * (int64_t)nrhs * base + li;
    for (int r = 0; r < nrhs; ++r) {
        o[2 * n * r] = src[2 * Nc * r + g];
        o[2 * n * r + n] = src[2 * Nc * r + Nc + g];
    }
}
template <int Z = 0>
__global__ __launch_bounds__(256) void k_box_gather(const int* __restrict__ map, const int* __restrict__ bsub,
                                                    const int64_t* __restrict__ bbase, const int* __restrict__ bn,
                                                    int64_t j0, int64_t j1, const double* __restrict__ src,
                                                    int64_t Nc, double* __restrict__ loc, int nrhs) {
    k_box_gather_body<Z>(single_block<false>(), map, bsub, bbase, bn, j0, j1, src, Nc, loc, nrhs);
}
template <class PK, int Z = 0>
__global__ __launch_bounds__(256) void k_box_gather_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_box_gather_body<Z>(ehh_vb, a...); }, b.arg[ehh_s]);
}

// z += w loc(box) for the local unknowns [j0, j1) (boxes of the range disjoint);
// w = wgt[g] (the inverse owner count) when wgt is given, else 1
template <int Z = 0>
EHH_DEV void k_box_scatter_body(VB ehh_vb, const int* __restrict__ map, const int* __restrict__ bsub, const int64_t* __restrict__ bbase, const int* __restrict__ bn, int64_t j0, int64_t j1, const double* __restrict__ loc, const double* __restrict__ wgt, int64_t Nc, double* __restrict__ z, int nrhs) {
    const int64_t j = j0 + (int64_t)ehh_vb.x * blockDim.x + threadIdx.x;
    if (j >= j1) return;
    const int b = bsub[j];
    const int64_t base = bbase[b], n = bn[b], li = j - base, g = map[j];
    const double w = wgt ? wgt[g] : 1.0;
    const double* o = loc + 2 * (int64_t)nrhs * base + li;
    for (int r = 0; r < nrhs; ++r) {
        z[2 * Nc * r + g] += w * o[2 * n * r];
        z[2 * Nc * r + Nc + g] += w * o[2 * n * r + n];
    }
}
template <int Z = 0>
__global__ __launch_bounds__(256) void k_box_scatter(const int* __restrict__ map, const int* __restrict__ bsub,
                                                     const int64_t* __restrict__ bbase, const int* __restrict__ bn,
                                                     int64_t j0, int64_t j1, const double* __restrict__ loc,
                                                     const double* __restrict__ wgt, int64_t Nc,
                                                     double* __restrict__ z, int nrhs) {
    k_box_scatter_body<Z>(single_block<false>(), map, bsub, bbase, bn, j0, j1, loc, wgt, Nc, z, nrhs);
}
template <class PK, int Z = 0>
__global__ __launch_bounds__(256) void k_box_scatter_batch(Batch<PK> b) {
    VB ehh_vb;
    int ehh_s;
    if (!batch_block<false>(b, ehh_vb, ehh_s)) return;
    call_pack([&](auto&&... a) { k_box_scatter_body<Z>(ehh_vb, a...); }, b.arg[ehh_s]);
}

hipError_t launch_box_gather(const BoxMap& m, int64_t j0, int64_t j1, const double* src, int64_t Nc, double* loc,
                             int nrhs, hipStream_t s) {
    if (j1 <= j0) return hipSuccess;
    EHH_LAUNCHK(bytes_plain(nrhs * 32.0 * (double)(j1 - j0)), k_box_gather, (0), nblk(j1 - j0), 256, 0, s, m.map, m.bsub,
                 m.bbase, m.bn, j0, j1, src, Nc, loc, nrhs);
    return hipGetLastError();
}
hipError_t launch_box_scatter(const BoxMap& m, int64_t j0, int64_t j1, const double* loc, const double* wgt,
                              int64_t Nc, double* z, int nrhs, hipStream_t s) {
    if (j1 <= j0) return hipSuccess;
    EHH_LAUNCHK(bytes_plain(nrhs * 48.0 * (double)(j1 - j0)), k_box_scatter, (0), nblk(j1 - j0), 256, 0, s, m.map,
                 m.bsub, m.bbase, m.bn, j0, j1, loc, wgt, Nc, z, nrhs);
    return hipGetLastError();
}

}  // namespace ehh
