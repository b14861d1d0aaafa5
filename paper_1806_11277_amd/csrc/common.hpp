// Shared device/host definitions of the elastic Helmholtz HIP library.
//
// Dimension-generic (D = 2 or 3) description of one grid level of the
// staggered mixed discretisation (section 2.1 of the paper): cells n[0] x n[1]
// (x n[2]); component k < D is the displacement on the interior faces normal to
// axis k, component D is the cell-centred pressure of eq. (13).  A complex
// vector of one right-hand side is stored as the real plane of all unknowns
// followed by the imaginary plane (structure of arrays).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define EHH_DEV __device__ __forceinline__
#define EHH_HD __host__ __device__ __forceinline__

namespace ehh {

struct Geo {
    int dim;
    int n[3];           // cells per axis (n[2] == 1 in 2D)
    int64_t cnt[4];     // unknowns of u_0, u_1, u_2, p (cnt[2] == 0 in 2D)
    int64_t off[4];     // start of each component in a plane
    int64_t N;          // unknowns of one right-hand side
    int64_t ncell;
};

inline Geo make_geo(int dim, const int* n) {
    Geo g{};
    g.dim = dim;
    g.n[0] = n[0];
    g.n[1] = n[1];
    g.n[2] = dim == 3 ? n[2] : 1;
    g.ncell = (int64_t)g.n[0] * g.n[1] * g.n[2];
    for (int k = 0; k < 3; ++k) {
        if (k < dim) {
            int64_t c = 1;
            for (int a = 0; a < 3; ++a) c *= (a == k) ? (g.n[a] - 1) : g.n[a];
            g.cnt[k] = c;
        } else {
            g.cnt[k] = 0;
        }
    }
    g.cnt[3] = g.ncell;
    int64_t o = 0;
    for (int k = 0; k < 4; ++k) {
        g.off[k] = o;
        o += g.cnt[k];
    }
    g.N = o;
    return g;
}

// Tangential axes of component k (increasing order, axis 2 only in 3D).
template <int D> EHH_HD int tang1(int k) { return k == 0 ? 1 : 0; }
template <int D> EHH_HD int tang2(int k) { return k == 2 ? 1 : 2; }

// Number of stored (upper-half) and full u-u stencil entries, u-p entries.
template <int D> struct St;
template <> struct St<2> {
    static constexpr int NF = 15, CF = 7, NUU = 8, NUP = 6;
};
template <> struct St<3> {
    static constexpr int NF = 75, CF = 37, NUU = 38, NUP = 18;
};

// Full u-u offset index: dn along the normal in {-1,0,1}, dt1/dt2 along the
// tangential axes in {-2..2}.  The entry of offset F is stored at the face itself
// when F >= CF, otherwise (transposed) at the neighbour with index 2CF - F.
template <int D> EHH_HD int full_index(int dn, int dt1, int dt2) {
    return D == 2 ? (dt1 + 2) * 3 + (dn + 1) : ((dt2 + 2) * 5 + (dt1 + 2)) * 3 + (dn + 1);
}
template <int D> EHH_HD void full_offset(int F, int& dn, int& dt1, int& dt2) {
    dn = F % 3 - 1;
    dt1 = (F / 3) % 5 - 2;
    dt2 = D == 2 ? 0 : F / 15 - 2;
}
// u-p entry index: side 0 = cell below the face along the normal, 1 = above;
// e1/e2 cell offsets along the tangential axes in {-1,0,1}.
template <int D> EHH_HD int up_index(int side, int e1, int e2) {
    return D == 2 ? side + 2 * (e1 + 1) : side + 2 * ((e1 + 1) + 3 * (e2 + 1));
}
template <int D> EHH_HD void up_decode(int q, int& side, int& e1, int& e2) {
    side = q & 1;
    e1 = (q >> 1) % 3 - 1;
    e2 = D == 2 ? 0 : (q >> 1) / 3 - 1;
}

// ------------------------------------------------------------------- indexing
template <int D> EHH_HD bool face_ok(const Geo& g, int k, const int* p) {
    if (p[k] < 1 || p[k] > g.n[k] - 1) return false;
    for (int a = 0; a < D; ++a)
        if (a != k && (p[a] < 0 || p[a] >= g.n[a])) return false;
    return true;
}
template <int D> EHH_HD int64_t face_idx(const Geo& g, int k, const int* p) {
    const int d0 = g.n[0] - (k == 0), d1 = g.n[1] - (k == 1);
    const int c0 = p[0] - (k == 0), c1 = p[1] - (k == 1);
    if (D == 2) return (int64_t)c1 * d0 + c0;
    const int c2 = p[2] - (k == 2);
    return ((int64_t)c2 * d1 + c1) * d0 + c0;
}
template <int D> EHH_HD bool cell_ok(const Geo& g, const int* c) {
    for (int a = 0; a < D; ++a)
        if (c[a] < 0 || c[a] >= g.n[a]) return false;
    return true;
}
template <int D> EHH_HD int64_t cell_idx(const Geo& g, const int* c) {
    if (D == 2) return (int64_t)c[1] * g.n[0] + c[0];
    return ((int64_t)c[2] * g.n[1] + c[1]) * g.n[0] + c[0];
}
// Decode a face index of component k into its position.
template <int D> EHH_HD void face_pos(const Geo& g, int k, int64_t idx, int* p) {
    const int d0 = g.n[0] - (k == 0), d1 = g.n[1] - (k == 1);
    p[0] = (int)(idx % d0);
    int64_t r = idx / d0;
    if (D == 2) {
        p[1] = (int)r;
        p[2] = 0;
    } else {
        p[1] = (int)(r % d1);
        p[2] = (int)(r / d1);
    }
    p[k] += 1;
}
template <int D> EHH_HD void cell_pos(const Geo& g, int64_t idx, int* c) {
    c[0] = (int)(idx % g.n[0]);
    int64_t r = idx / g.n[0];
    if (D == 2) {
        c[1] = (int)r;
        c[2] = 0;
    } else {
        c[1] = (int)(r % g.n[1]);
        c[2] = (int)(r / g.n[1]);
    }
}

// ------------------------------------------------------------------- complex
template <typename T> struct cx {
    T re, im;
};
template <typename T> EHH_HD cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <typename T> EHH_HD cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> EHH_HD cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> EHH_HD cx<T> operator*(cx<T> a, cx<T> b) {
    return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> EHH_HD cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> EHH_HD cx<T> cinv(cx<T> a) {
    T d = a.re * a.re + a.im * a.im;
    return {a.re / d, -a.im / d};
}
template <typename T> EHH_HD cx<T> cdiv(cx<T> a, cx<T> b) { return a * cinv(b); }

// Access to component c of one right-hand side (base points at its real plane).
template <typename T> struct Vec {
    T* base;
    int64_t N;
    EHH_DEV cx<T> ld(int64_t i) const { return {base[i], base[N + i]}; }
    EHH_DEV void st(int64_t i, cx<T> v) const {
        base[i] = v.re;
        base[N + i] = v.im;
    }
};
template <typename T> struct CVec {
    const T* base;
    int64_t N;
    EHH_DEV cx<T> ld(int64_t i) const { return {base[i], base[N + i]}; }
};

// ------------------------------------------------------------- coefficients
// Level 0 (matrix free): nondimensional cell arrays; the shifted/unshifted
// operator differ only in alpha.
template <typename T> struct FineCoef {
    const T* mu;
    const T* dinv;   // 1 / (lambda + mu)
    const T* rho;
    const T* gam;    // gamma / omega (layer + constant + physical)
    T om2;           // omega^2
    T alpha;         // shift (0 for the unshifted operator)
};

// Levels >= 1 (Galerkin): per component k, NUU complex planes (re, im) and NUP
// real planes over the faces of k; one real plane over the cells.
template <typename T> struct StCoef {
    const T* uu[3];
    const T* up[3];
    const T* pp;
};

template <int D> inline int64_t stencil_reals(const Geo& g) {
    int64_t s = 0;
    for (int k = 0; k < D; ++k) s += g.cnt[k] * (2 * St<D>::NUU + St<D>::NUP);
    return s + g.ncell;
}

template <int D, typename T, typename P> EHH_HD StCoef<T> stencil_view(const Geo& g, P base) {
    StCoef<T> s{};
    int64_t o = 0;
    for (int k = 0; k < D; ++k) {
        s.uu[k] = base + o;
        o += 2 * St<D>::NUU * g.cnt[k];
    }
    for (int k = 0; k < D; ++k) {
        s.up[k] = base + o;
        o += St<D>::NUP * g.cnt[k];
    }
    s.pp = base + o;
    return s;
}

}  // namespace ehh
