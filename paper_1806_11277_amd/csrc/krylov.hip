// FP64 vector kernels of the outer flexible GMRES: block-wide Hermitian dot
// products reduced deterministically in two passes (no floating-point atomics),
// multi-vector updates, the per-right-hand-side Givens rotations of the
// Hessenberg matrix and the final x += Z y.
//
// Complex vectors hold the real plane (N doubles) then the imaginary plane.
#include <math.h>

#include "internal.hpp"

namespace ehh {

static constexpr int KB = 256;       // threads per block
static constexpr int MAXV = EHH_KMAXV;

static inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

int krylov_blocks(int64_t n) {
    int64_t b = (n + 4 * KB - 1) / (4 * KB);
    if (b > 512) b = 512;
    if (b < 1) b = 1;
    return (int)b;
}

EHH_DEV double block_sum(double v, double* sm) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sm[wid] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < KB / 64; ++w) s += sm[w];
    return s;   // valid in thread 0
}

// partial[((r * nv + i) * 2 + c) * nb + blk]; wpart (if given) receives the
// block partials of |w|^2, wpart[r * nb + blk]
__global__ __launch_bounds__(KB) void k_dots_partial(const double* __restrict__ V, int nv, const double* __restrict__ w,
                                                     int64_t N, int nrhs, double* __restrict__ partial,
                                                     double* __restrict__ wpart) {
    __shared__ double sm[KB / 64];
    const int r = blockIdx.y;
    const int nb = gridDim.x;
    const double* wr = w + (int64_t)r * 2 * N;
    double are[MAXV], aim[MAXV], ww = 0.0;
#pragma unroll
    for (int i = 0; i < MAXV; ++i) are[i] = aim[i] = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * KB + threadIdx.x; e < N; e += (int64_t)nb * KB) {
        const double xr = wr[e], xi = wr[N + e];
        ww += xr * xr + xi * xi;
#pragma unroll
        for (int i = 0; i < MAXV; ++i) {
            if (i < nv) {
                const double* v = V + ((int64_t)i * nrhs + r) * 2 * N;
                const double vr = v[e], vi = v[N + e];
                are[i] += vr * xr + vi * xi;
                aim[i] += vr * xi - vi * xr;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
        if (i < nv) {
            const double sr = block_sum(are[i], sm);
            if (threadIdx.x == 0) partial[(((int64_t)r * nv + i) * 2 + 0) * nb + blockIdx.x] = sr;
            const double si = block_sum(aim[i], sm);
            if (threadIdx.x == 0) partial[(((int64_t)r * nv + i) * 2 + 1) * nb + blockIdx.x] = si;
        }
    }
    if (wpart) {
        const double sw = block_sum(ww, sm);
        if (threadIdx.x == 0) wpart[(int64_t)r * nb + blockIdx.x] = sw;
    }
}

// One 64-wide wavefront per output: lanes stride over the block partials, then a
// fixed butterfly (deterministic order).
EHH_DEV double wave_sum(const double* p, int nb) {
    const int lane = threadIdx.x & 63;
    double s = 0.0;
    for (int b = lane; b < nb; b += 64) s += p[b];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    return s;
}

// out[r][i] (complex, i < nv) from the block partials; with wpart, the real
// part of out[r][wslot] also receives the sum of wpart's partials of source r.
__global__ __launch_bounds__(256) void k_partial_final(const double* __restrict__ partial, int nv, int nb, int nrhs,
                                                       double* __restrict__ out, int ldo,
                                                       const double* __restrict__ wpart, int wslot) {
    const int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (t < nrhs * nv * 2) {
        const int c = t & 1, i = (t >> 1) % nv, r = (t >> 1) / nv;
        const double s = wave_sum(partial + (((int64_t)r * nv + i) * 2 + c) * nb, nb);
        if ((threadIdx.x & 63) == 0) out[2 * ((int64_t)r * ldo + i) + c] = s;
    } else if (wpart && t < nrhs * nv * 2 + nrhs) {
        const int r = t - nrhs * nv * 2;
        const double s = wave_sum(wpart + (int64_t)r * nb, nb);
        if ((threadIdx.x & 63) == 0) out[2 * ((int64_t)r * ldo + wslot)] = s;
    }
}

// Whether one classical Gram-Schmidt pass leaves w orthogonal enough to V
// (the test of Daniel, Gragg, Kaufman and Stewart, 1976): the updated w keeps
// more than eta of its length, |w|^2 - sum_i |h_i|^2 > eta^2 |w|^2 (V
// orthonormal), so that its rounding error relative to V, about u |w| / |w'|,
// stays below u / eta (u the unit roundoff).  Their bound is eta = 1/sqrt(2);
// a preconditioned step removes most of w (the preconditioned operator is near
// the identity), so that bound asks for a second pass almost every time.  With
// eta = 0.1 (at most ten times the roundoff) the 2D and 3D workloads solved as
// fast as with no second pass at all, with the same iterations and residuals
// as with an unconditional second pass (32 sources at 512^2: 882 -> 845 ms per
// solve).  A zero w fails the test.
static constexpr double kGsEta2 = 1e-2;
EHH_DEV bool gs_one_pass(double w2, double p) { return w2 - p > kGsEta2 * w2; }

// The first Gram-Schmidt update, with h = h1 (slot wslot of h1 holds |w|^2
// before the pass).  Every block takes the decision of gs_one_pass (none with
// force_two) and block 0 records it in flag[r] (1: one pass).  A one-pass
// source gets its next basis vector at once, normalised:
// |w - V h|^2 = |w|^2 - sum_i |h_i|^2 (V orthonormal; the test bounds the
// cancellation to two digits), so out = (w - V h) / |w - V h| (and out32, if
// given, in FP32), nrm2[r] = |w - V h|^2 and h2[r] = 0 for the Hessenberg
// column; w is left as it was.  The other sources are left to the second pass.
__global__ __launch_bounds__(KB) void k_gs_first(const double* __restrict__ V, int nv, const double* __restrict__ w,
                                                 int64_t N, int nrhs, const double* __restrict__ h, int ldh,
                                                 int wslot, int force_two, double* __restrict__ flag,
                                                 double* __restrict__ h2, double* __restrict__ nrm2,
                                                 double* __restrict__ out, float* __restrict__ out32) {
    const int r = blockIdx.y;
    const int nb = gridDim.x;
    const double* hr0 = h + 2 * (int64_t)r * ldh;
    double p = 0.0;
    for (int i = 0; i < nv; ++i) p += hr0[2 * i] * hr0[2 * i] + hr0[2 * i + 1] * hr0[2 * i + 1];
    const double w2 = hr0[2 * wslot];
    const bool one = !force_two && gs_one_pass(w2, p);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        flag[2 * (int64_t)r * ldh] = one ? 1.0 : 0.0;
        if (one) {
            nrm2[r] = w2 - p;
            for (int i = 0; i < nv; ++i) h2[2 * ((int64_t)r * ldh + i)] = h2[2 * ((int64_t)r * ldh + i) + 1] = 0.0;
        }
    }
    if (!one) return;
    const double f = 1.0 / sqrt(w2 - p);
    const double* wr = w + (int64_t)r * 2 * N;
    double* o = out + (int64_t)r * 2 * N;
    float* o32 = out32 ? out32 + (int64_t)r * 2 * N : nullptr;
    double hr[MAXV], hi[MAXV];
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
        hr[i] = i < nv ? hr0[2 * i] : 0.0;
        hi[i] = i < nv ? hr0[2 * i + 1] : 0.0;
    }
    for (int64_t e = (int64_t)blockIdx.x * KB + threadIdx.x; e < N; e += (int64_t)nb * KB) {
        double xr = wr[e], xi = wr[N + e];
#pragma unroll
        for (int i = 0; i < MAXV; ++i) {
            if (i < nv) {
                const double* v = V + ((int64_t)i * nrhs + r) * 2 * N;
                const double vr = v[e], vi = v[N + e];
                xr -= hr[i] * vr - hi[i] * vi;
                xi -= hr[i] * vi + hi[i] * vr;
            }
        }
        const double yr = xr * f, yi = xi * f;
        o[e] = yr;
        o[N + e] = yi;
        if (o32) {
            o32[e] = (float)yr;
            o32[N + e] = (float)yi;
        }
    }
}

// Classical Gram-Schmidt, first pass and second projection in one sweep, for the
// sources that need two passes (flag[r] == 0): w <- w - sum_i h_i V_i, then the
// block partials of <V_i, w> and of |w|^2 for the updated w, with each V_i
// element loaded once for both (partial[((r * nv + i) * 2 + c) * nb + blk],
// npart[r * nb + blk]).
__global__ __launch_bounds__(KB) void k_axpy_dots(const double* __restrict__ V, int nv, double* __restrict__ w,
                                                  int64_t N, int nrhs, const double* __restrict__ h, int ldh,
                                                  double* __restrict__ partial, double* __restrict__ npart,
                                                  const double* __restrict__ flag) {
    __shared__ double sm[KB / 64];
    const int r = blockIdx.y;
    const int nb = gridDim.x;
    if (flag[2 * (int64_t)r * ldh] != 0.0) return;
    double* wr = w + (int64_t)r * 2 * N;
    double hr[MAXV], hi[MAXV], are[MAXV], aim[MAXV], ww = 0.0;
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
        hr[i] = i < nv ? h[2 * ((int64_t)r * ldh + i)] : 0.0;
        hi[i] = i < nv ? h[2 * ((int64_t)r * ldh + i) + 1] : 0.0;
        are[i] = aim[i] = 0.0;
    }
    for (int64_t e = (int64_t)blockIdx.x * KB + threadIdx.x; e < N; e += (int64_t)nb * KB) {
        double xr = wr[e], xi = wr[N + e];
        double vr[MAXV], vi[MAXV];
#pragma unroll
        for (int i = 0; i < MAXV; ++i) {
            if (i < nv) {
                const double* v = V + ((int64_t)i * nrhs + r) * 2 * N;
                vr[i] = v[e];
                vi[i] = v[N + e];
                xr -= hr[i] * vr[i] - hi[i] * vi[i];
                xi -= hr[i] * vi[i] + hi[i] * vr[i];
            }
        }
        wr[e] = xr;
        wr[N + e] = xi;
        ww += xr * xr + xi * xi;
#pragma unroll
        for (int i = 0; i < MAXV; ++i) {
            if (i < nv) {
                are[i] += vr[i] * xr + vi[i] * xi;
                aim[i] += vr[i] * xi - vi[i] * xr;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
        if (i < nv) {
            const double sr = block_sum(are[i], sm);
            if (threadIdx.x == 0) partial[(((int64_t)r * nv + i) * 2 + 0) * nb + blockIdx.x] = sr;
            const double si = block_sum(aim[i], sm);
            if (threadIdx.x == 0) partial[(((int64_t)r * nv + i) * 2 + 1) * nb + blockIdx.x] = si;
        }
    }
    const double sw = block_sum(ww, sm);
    if (threadIdx.x == 0) npart[(int64_t)r * nb + blockIdx.x] = sw;
}

// The second update of a two-pass source (flag[r] == 0).  Every block sums the
// block partials k_axpy_dots left (one wavefront per sum, the fixed order of
// wave_sum, so that all blocks agree): h2 = V^H w and |w|^2 of the once-updated
// w.  Then w - V h2 has |w - V h2|^2 = |w|^2 - sum_i |h2_i|^2 (h2 is tiny, no
// cancellation), out = (w - V h2) / |w - V h2| (out32 in FP32), and block 0
// stores h2 and nrm2[r] for the Hessenberg column.  A zero vector stays zero.
__global__ __launch_bounds__(KB) void k_gs_second(const double* __restrict__ V, int nv, const double* __restrict__ w,
                                                  int64_t N, int nrhs, const double* __restrict__ partial,
                                                  const double* __restrict__ npart, int nbp,
                                                  double* __restrict__ h2, int ldh, const double* __restrict__ flag,
                                                  double* __restrict__ nrm2, double* __restrict__ out,
                                                  float* __restrict__ out32) {
    __shared__ double hs[2 * MAXV + 1];
    const int r = blockIdx.y;
    const int nb = gridDim.x;
    if (flag[2 * (int64_t)r * ldh] != 0.0) return;
    const int nsum = 2 * nv + 1;
    for (int q = threadIdx.x >> 6; q < nsum; q += KB / 64) {
        const double* src = q < 2 * nv ? partial + ((int64_t)r * nv * 2 + q) * nbp : npart + (int64_t)r * nbp;
        const double sq = wave_sum(src, nbp);
        if ((threadIdx.x & 63) == 0) hs[q] = sq;
    }
    __syncthreads();
    double hr[MAXV], hi[MAXV];
    double p = 0.0;
#pragma unroll
    for (int i = 0; i < MAXV; ++i) {
        hr[i] = i < nv ? hs[2 * i] : 0.0;
        hi[i] = i < nv ? hs[2 * i + 1] : 0.0;
        p += hr[i] * hr[i] + hi[i] * hi[i];
    }
    const double n2 = fmax(hs[2 * nv] - p, 0.0);
    const double f = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        for (int i = 0; i < nv; ++i) {
            h2[2 * ((int64_t)r * ldh + i)] = hs[2 * i];
            h2[2 * ((int64_t)r * ldh + i) + 1] = hs[2 * i + 1];
        }
        nrm2[r] = n2;
    }
    const double* wr = w + (int64_t)r * 2 * N;
    double* o = out + (int64_t)r * 2 * N;
    float* o32 = out32 ? out32 + (int64_t)r * 2 * N : nullptr;
    for (int64_t e = (int64_t)blockIdx.x * KB + threadIdx.x; e < N; e += (int64_t)nb * KB) {
        double xr = wr[e], xi = wr[N + e];
#pragma unroll
        for (int i = 0; i < MAXV; ++i) {
            if (i < nv) {
                const double* v = V + ((int64_t)i * nrhs + r) * 2 * N;
                const double vr = v[e], vi = v[N + e];
                xr -= hr[i] * vr - hi[i] * vi;
                xi -= hr[i] * vi + hi[i] * vr;
            }
        }
        const double yr = xr * f, yi = xi * f;
        o[e] = yr;
        o[N + e] = yi;
        if (o32) {
            o32[e] = (float)yr;
            o32[N + e] = (float)yi;
        }
    }
}

hipError_t launch_orthogonalise(const double* V, int nv, double* w, int64_t N, int nrhs, double* partial,
                                double* h1, double* h2, int m, double* nrm2, double* vnext, float* v32,
                                bool force_two, hipStream_t s) {
    const int nb = krylov_blocks(N), ldh = m + 1;
    // partial: the projections' block partials (below 2 m nrhs nb), then the
    // partials of |w|^2 before the first pass and after it; slot m of h1 holds
    // |w|^2 before the pass, slot m of h2 the one-pass flag
    double* wpart = partial + (size_t)2 * m * nrhs * nb;
    double* npart = wpart + (size_t)nrhs * nb;
    double* flag = h2 + 2 * m;
    const unsigned nf = nblk((int64_t)(nrhs * nv * 2 + nrhs) * 64);
    hipLaunchKernelGGL(k_dots_partial, dim3(nb, nrhs), KB, 0, s, V, nv, (const double*)w, N, nrhs, partial, wpart);
    hipLaunchKernelGGL(k_partial_final, nf, 256, 0, s, (const double*)partial, nv, nb, nrhs, h1, ldh,
                       (const double*)wpart, m);
    hipLaunchKernelGGL(k_gs_first, dim3(nb, nrhs), KB, 0, s, V, nv, (const double*)w, N, nrhs, (const double*)h1, ldh,
                       m, force_two ? 1 : 0, flag, h2, nrm2, vnext, v32);
    hipLaunchKernelGGL(k_axpy_dots, dim3(nb, nrhs), KB, 0, s, V, nv, w, N, nrhs, (const double*)h1, ldh, partial,
                       npart, (const double*)flag);
    hipLaunchKernelGGL(k_gs_second, dim3(nb, nrhs), KB, 0, s, V, nv, (const double*)w, N, nrhs,
                       (const double*)partial, (const double*)npart, nb, h2, ldh, (const double*)flag, nrm2, vnext,
                       v32);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_norm_final(const double* __restrict__ partial, int nb, int nrhs,
                                                    double* __restrict__ out) {
    const int r = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (r >= nrhs) return;
    const double s = wave_sum(partial + (int64_t)r * nb, nb);
    if ((threadIdx.x & 63) == 0) out[r] = s;
}

__global__ __launch_bounds__(KB) void k_norm_partial(const double* __restrict__ x, int64_t N, double* __restrict__ partial) {
    __shared__ double sm[KB / 64];
    const int r = blockIdx.y;
    const int nb = gridDim.x;
    const double* xr = x + (int64_t)r * 2 * N;
    double acc = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * KB + threadIdx.x; e < 2 * N; e += (int64_t)nb * KB) acc += xr[e] * xr[e];
    const double s = block_sum(acc, sm);
    if (threadIdx.x == 0) partial[(int64_t)r * nb + blockIdx.x] = s;
}

hipError_t launch_norm2(const double* x, int64_t N, int nrhs, double* partial, double* nrm2, hipStream_t s) {
    const int nb = krylov_blocks(N);
    hipLaunchKernelGGL(k_norm_partial, dim3(nb, nrhs), KB, 0, s, x, N, partial);
    hipLaunchKernelGGL(k_norm_final, nblk((int64_t)nrhs * 64), 256, 0, s, partial, nb, nrhs, nrm2);
    return hipGetLastError();
}

// mode 0: out = x * sc[r]; mode 1: out = x / sqrt(sc[r]) (0 if sc[r] == 0)
// (out32, when given, receives the same values in FP32: the input of a
// complex64 preconditioner cycle, written in the same pass.)
__global__ void k_scale(const double* __restrict__ x, double* __restrict__ out, int64_t N, int nrhs,
                        const double* __restrict__ sc, int mode, float* __restrict__ out32) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 2 * N * nrhs) return;
    const int r = (int)(t / (2 * N));
    double f = sc[r];
    if (mode == 1) f = f > 0.0 ? 1.0 / sqrt(f) : 0.0;
    const double v = x[t] * f;
    out[t] = v;
    if (out32) out32[t] = (float)v;
}

hipError_t launch_scale(const double* x, double* out, int64_t N, int nrhs, const double* scale, int mode,
                        hipStream_t s, float* out32) {
    hipLaunchKernelGGL(k_scale, nblk(2 * N * nrhs), 256, 0, s, x, out, N, nrhs, scale, mode, out32);
    return hipGetLastError();
}

__global__ void k_axpby(const double* __restrict__ x, const double* __restrict__ y, double* __restrict__ out, int64_t n,
                        double a, double b) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) out[t] = a * x[t] + b * y[t];
}

hipError_t launch_axpby(const double* x, const double* y, double* out, int64_t n, double a, double b, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, nblk(n), 256, 0, s, x, y, out, n, a, b);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Givens rotations
// H[r][j][i] (column j, i <= m) complex; cs[r][i] = (c, s_re, s_im); g[r][i] complex.
// hcol[r][i] + hcol2[r][i] for i <= j: <v_i, w> (complex, the two CGS passes),
// hnext2[r] = |w|^2.
// One thread per right-hand side (lane 0 of a wavefront): h_{j+1,j} =
// sqrt(nrm2[r]), the squared norm the orthogonalisation left, then the
// rotations.
__global__ __launch_bounds__(64) void k_givens(double* __restrict__ H, double* __restrict__ cs,
                                               double* __restrict__ g, const double* __restrict__ hcol,
                                               const double* __restrict__ hcol2, const double* __restrict__ nrm2,
                                               int j, int m, int nrhs, const int* __restrict__ active,
                                               double* __restrict__ est, const double* __restrict__ bnorm) {
    const int r = blockIdx.x;
    if (r >= nrhs) return;
    if (threadIdx.x != 0) return;
    const double w2 = nrm2[r];
    if (!active[r]) return;
    double* col = H + 2 * (((int64_t)r * m + j) * (m + 1));
    double* c = cs + 3 * (int64_t)r * m;
    double* gg = g + 2 * (int64_t)r * (m + 1);
    for (int i = 0; i <= j; ++i) {
        const int64_t o = 2 * ((int64_t)r * (m + 1) + i);
        col[2 * i] = hcol[o] + hcol2[o];
        col[2 * i + 1] = hcol[o + 1] + hcol2[o + 1];
    }
    col[2 * (j + 1)] = sqrt(w2);
    col[2 * (j + 1) + 1] = 0.0;
    for (int i = 0; i < j; ++i) {
        const double cc = c[3 * i], sr = c[3 * i + 1], si = c[3 * i + 2];
        const double ar = col[2 * i], ai = col[2 * i + 1];
        const double br = col[2 * (i + 1)], bi = col[2 * (i + 1) + 1];
        // a' = c a + s b ; b' = -conj(s) a + c b
        col[2 * i] = cc * ar + (sr * br - si * bi);
        col[2 * i + 1] = cc * ai + (sr * bi + si * br);
        col[2 * (i + 1)] = -(sr * ar + si * ai) + cc * br;
        col[2 * (i + 1) + 1] = -(sr * ai - si * ar) + cc * bi;
    }
    const double ar = col[2 * j], ai = col[2 * j + 1];
    const double br = col[2 * (j + 1)], bi = col[2 * (j + 1) + 1];
    const double na = sqrt(ar * ar + ai * ai), nb = sqrt(br * br + bi * bi);
    double cc, sr, si;
    if (nb == 0.0) {
        cc = 1.0;
        sr = si = 0.0;
    } else if (na == 0.0) {
        cc = 0.0;
        sr = br / nb;
        si = -bi / nb;
    } else {
        const double t = sqrt(na * na + nb * nb);
        cc = na / t;
        // s = (a/|a|) conj(b) / t
        const double ur = ar / na, ui = ai / na;
        sr = (ur * br + ui * bi) / t;
        si = (ui * br - ur * bi) / t;
    }
    c[3 * j] = cc;
    c[3 * j + 1] = sr;
    c[3 * j + 2] = si;
    // new diagonal: c a + s b
    const double dr = cc * ar + (sr * br - si * bi), di = cc * ai + (sr * bi + si * br);
    col[2 * j] = dr;
    col[2 * j + 1] = di;
    col[2 * (j + 1)] = 0.0;
    col[2 * (j + 1) + 1] = 0.0;
    const double gr = gg[2 * j], gi = gg[2 * j + 1];
    gg[2 * j] = cc * gr;
    gg[2 * j + 1] = cc * gi;
    gg[2 * (j + 1)] = -(sr * gr + si * gi);
    gg[2 * (j + 1) + 1] = -(sr * gi - si * gr);
    const double er = gg[2 * (j + 1)], ei = gg[2 * (j + 1) + 1];
    est[r] = sqrt(er * er + ei * ei) / bnorm[r];
}

hipError_t launch_givens(double* H, double* cs, double* g, const double* hcol, const double* hcol2,
                         const double* nrm2, int j, int m, int nrhs, const int* active, double* est,
                         const double* bnorm, hipStream_t s) {
    hipLaunchKernelGGL(k_givens, nrhs, 64, 0, s, H, cs, g, hcol, hcol2, nrm2, j, m, nrhs, active, est, bnorm);
    return hipGetLastError();
}

// y = R^{-1} g for the first ncols[r] columns (upper triangular R in H).
__global__ void k_backsub(const double* __restrict__ H, const double* __restrict__ g, int m, int nrhs,
                          const int* __restrict__ ncols, double* __restrict__ y) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrhs) return;
    const int nc = ncols[r];
    double* yr = y + 2 * (int64_t)r * m;
    for (int i = 0; i < m; ++i) yr[2 * i] = yr[2 * i + 1] = 0.0;
    for (int i = nc - 1; i >= 0; --i) {
        double sr = g[2 * ((int64_t)r * (m + 1) + i)], si = g[2 * ((int64_t)r * (m + 1) + i) + 1];
        for (int jj = i + 1; jj < nc; ++jj) {
            const double* hc = H + 2 * (((int64_t)r * m + jj) * (m + 1) + i);
            sr -= hc[0] * yr[2 * jj] - hc[1] * yr[2 * jj + 1];
            si -= hc[0] * yr[2 * jj + 1] + hc[1] * yr[2 * jj];
        }
        const double* d = H + 2 * (((int64_t)r * m + i) * (m + 1) + i);
        const double dd = d[0] * d[0] + d[1] * d[1];
        yr[2 * i] = (sr * d[0] + si * d[1]) / dd;
        yr[2 * i + 1] = (si * d[0] - sr * d[1]) / dd;
    }
}

template <typename TZ>
__global__ __launch_bounds__(256) void k_update_x(const TZ* __restrict__ Z, double* __restrict__ x, int64_t N,
                                                  int nrhs, int m, const int* __restrict__ ncols,
                                                  const double* __restrict__ y) {
    const int r = blockIdx.y;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= N) return;
    const int nc = ncols[r];
    if (nc == 0) return;
    double* xr = x + (int64_t)r * 2 * N;
    double ar = xr[e], ai = xr[N + e];
    for (int i = 0; i < nc; ++i) {
        const TZ* z = Z + ((int64_t)i * nrhs + r) * 2 * N;
        const double yr = y[2 * ((int64_t)r * m + i)], yi = y[2 * ((int64_t)r * m + i) + 1];
        const double zr = (double)z[e], zi = (double)z[N + e];
        ar += yr * zr - yi * zi;
        ai += yr * zi + yi * zr;
    }
    xr[e] = ar;
    xr[N + e] = ai;
}

hipError_t launch_update_x(const double* H, const double* g, const double* Z, double* x, int64_t N, int nrhs, int m,
                           const int* ncols, double* y, hipStream_t s) {
    hipLaunchKernelGGL(k_backsub, nblk(nrhs, 64), 64, 0, s, H, g, m, nrhs, ncols, y);
    hipLaunchKernelGGL(k_update_x<double>, dim3(nblk(N), nrhs), 256, 0, s, Z, x, N, nrhs, m, ncols, y);
    return hipGetLastError();
}
hipError_t launch_update_x(const double* H, const double* g, const float* Z, double* x, int64_t N, int nrhs, int m,
                           const int* ncols, double* y, hipStream_t s) {
    hipLaunchKernelGGL(k_backsub, nblk(nrhs, 64), 64, 0, s, H, g, m, nrhs, ncols, y);
    hipLaunchKernelGGL(k_update_x<float>, dim3(nblk(N), nrhs), 256, 0, s, Z, x, N, nrhs, m, ncols, y);
    return hipGetLastError();
}

}  // namespace ehh
